/*
 * Plain, slow, FP64 CPU oracle for the direct Hartree-Fock J/K build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * What it computes (paper: "Theoretical Background"):
 *   - contracted Cartesian Gaussians (eqs. cgf, prim), each Cartesian
 *     component normalised to unit self-overlap (the paper leaves n_a
 *     unspecified; this is the reading taken);
 *   - ERIs (ab|cd) as the sum over primitive quartets (contracted-ERI
 *     definition) with two independent recurrence schemes:
 *       * McMurchie-Davidson Hermite expansion (eq. MD def1, eqs. EabP
 *         def1-3, R recursion of the MMD section) -- primary;
 *       * Obara-Saika vertical recurrences (eqs. vrr1, vrr2) contracted on
 *         the fly, then horizontal recurrences (eq. hrr) -- cross-check;
 *     The printed fundamental-integral prefactors are garbled; both schemes
 *     use [00|00]^(m) = U_P U_Q (2 theta/sqrt(pi)) F_m(T) and
 *     R_{0,m} = U_P U_Q (2 theta/sqrt(pi)) (-2 theta^2)^m F_m(T).  In eq. vrr2
 *     the PQ term is taken as +zeta/(zeta+eta) (P-Q) (W - Q), which is what
 *     the MMD/OS agreement test pins.
 *   - the Boys function F_m(T) of eq. boys-fn-def by its power series
 *     (T <= 35) and by erf plus upward recursion (T > 35);
 *   - J and K of the Hartree-Fock section (J_uv = sum (uv|ls) D_ls,
 *     K_uv = sum (ul|vs) D_ls), by adding every distinct permutation of each
 *     unique shell quartet literally (no degeneracy factors), unscreened;
 *   - one-electron integrals S, T, V (needed for h), MMD/Hermite form.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 3
#define OR_MAXL4 (4 * OR_MAXL)

/* ------------------------------------------------------------- Boys ---- */
void oracle_boys(int mmax, double T, double *F)
{
    if (T <= 35.0) {
        double e = exp(-T);
        for (int m = 0; m <= mmax; ++m) {
            double term = 1.0 / (2 * m + 1), sum = term;
            for (int k = 1; k < 2000; ++k) {
                term *= 2.0 * T / (2 * m + 2 * k + 1);
                sum += term;
                if (term < 1e-17 * sum) break;
            }
            F[m] = e * sum;
        }
    } else {
        double e = exp(-T);
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0 * T);
    }
}

/* ------------------------------------------------------- Cartesians ---- */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int ncum(int l) { return l * (l + 1) * (l + 2) / 6; } /* # comps with total < l */

/* component k of shell l in the order x^l, x^(l-1)y, x^(l-1)z, ... z^l */
static void cart(int l, int k, int *lx, int *ly, int *lz)
{
    int c = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (c == k) { *lx = x; *ly = y; *lz = l - x - y; return; }
            ++c;
        }
}
static int cart_index(int x, int y, int z) /* global index over all totals */
{
    int l = x + y + z;
    return ncum(l) + (l - x) * (l - x + 1) / 2 + z;
}

/* ------------------------------------------------------------ basis ---- */
typedef struct {
    int nshell, natom, nbf;
    const int *Z;
    const double *xyz;
    const int *sh_atom, *sh_l, *sh_nprim;
    int *prim_off, *bf_off;
    double *exps;   /* copy */
    double *coef;   /* d_i * N(alpha_i, l), then contraction-normalised */
    double *cscale; /* per basis function: 1/sqrt(self overlap) */
} obasis;

static double dfact(int n) /* (n)!! with (-1)!! = 1 */
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

/* 1-D Hermite expansion coefficients E[i][j][t] of x_A^i x_B^j about P
 * (eqs. EabP def1-3; E^{00}_0 = 1, the Gaussian product factor lives in U_P). */
#define EDIM (OR_MAXL + 3)
static void hermite_E(int la, int lb, double zeta, double PA, double PB,
                      double E[EDIM][EDIM][2 * EDIM])
{
    memset(E, 0, sizeof(double) * EDIM * EDIM * 2 * EDIM);
    double oo2z = 0.5 / zeta;
    E[0][0][0] = 1.0;
    for (int i = 0; i < la; ++i)
        for (int t = 0; t <= i + 1; ++t) {
            double v = PA * E[i][0][t];
            if (t > 0) v += oo2z * E[i][0][t - 1];
            if (t + 1 <= i) v += (t + 1) * E[i][0][t + 1];
            E[i + 1][0][t] = v;
        }
    for (int j = 0; j < lb; ++j)
        for (int i = 0; i <= la; ++i)
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = PB * E[i][j][t];
                if (t > 0) v += oo2z * E[i][j][t - 1];
                if (t + 1 <= i + j) v += (t + 1) * E[i][j][t + 1];
                E[i][j + 1][t] = v;
            }
}

/* overlap of two primitive Cartesian Gaussians with unit coefficients */
static double prim_overlap(const int *a, const int *b, double al, double be,
                           const double *A, const double *B)
{
    double zeta = al + be, res = pow(M_PI / zeta, 1.5);
    double mu = al * be / zeta, r2 = 0;
    for (int k = 0; k < 3; ++k) {
        double P = (al * A[k] + be * B[k]) / zeta;
        double E[EDIM][EDIM][2 * EDIM];
        hermite_E(a[k], b[k], zeta, P - A[k], P - B[k], E);
        res *= E[a[k]][b[k]][0];
        r2 += (A[k] - B[k]) * (A[k] - B[k]);
    }
    return res * exp(-mu * r2);
}

static int ob_init(obasis *ob, int natom, const int *Z, const double *xyz, int nshell,
                   const int *sh_atom, const int *sh_l, const int *sh_nprim,
                   const double *exps, const double *coefs)
{
    ob->natom = natom; ob->Z = Z; ob->xyz = xyz; ob->nshell = nshell;
    ob->sh_atom = sh_atom; ob->sh_l = sh_l; ob->sh_nprim = sh_nprim;
    ob->prim_off = malloc(sizeof(int) * (nshell + 1));
    ob->bf_off = malloc(sizeof(int) * (nshell + 1));
    ob->prim_off[0] = 0; ob->bf_off[0] = 0;
    for (int s = 0; s < nshell; ++s) {
        if (sh_l[s] < 0 || sh_l[s] > OR_MAXL || sh_nprim[s] < 1) return -1;
        ob->prim_off[s + 1] = ob->prim_off[s] + sh_nprim[s];
        ob->bf_off[s + 1] = ob->bf_off[s] + ncart(sh_l[s]);
    }
    ob->nbf = ob->bf_off[nshell];
    int np = ob->prim_off[nshell];
    ob->exps = malloc(sizeof(double) * np);
    ob->coef = malloc(sizeof(double) * np);
    ob->cscale = malloc(sizeof(double) * ob->nbf);
    memcpy(ob->exps, exps, sizeof(double) * np);
    for (int s = 0; s < nshell; ++s) {
        int l = sh_l[s];
        for (int p = ob->prim_off[s]; p < ob->prim_off[s + 1]; ++p) {
            double a = exps[p];
            ob->coef[p] = coefs[p] * pow(2 * a / M_PI, 0.75) * pow(4 * a, 0.5 * l) / sqrt(dfact(2 * l - 1));
        }
        /* unit self-overlap of every Cartesian component (computed literally) */
        const double *A = xyz + 3 * sh_atom[s];
        for (int k = 0; k < ncart(l); ++k) {
            int c[3];
            cart(l, k, &c[0], &c[1], &c[2]);
            double S = 0;
            for (int p = ob->prim_off[s]; p < ob->prim_off[s + 1]; ++p)
                for (int q = ob->prim_off[s]; q < ob->prim_off[s + 1]; ++q)
                    S += ob->coef[p] * ob->coef[q] * prim_overlap(c, c, ob->exps[p], ob->exps[q], A, A);
            ob->cscale[ob->bf_off[s] + k] = 1.0 / sqrt(S);
        }
    }
    return 0;
}

static void ob_free(obasis *ob)
{
    free(ob->prim_off); free(ob->bf_off); free(ob->exps); free(ob->coef); free(ob->cscale);
}

/* -------------------------------------------------- MMD primitive ERI -- */
/* R^{(0)}_{tuv} for t+u+v <= L (MMD section R recursion), scaled so that
 * R^{(n)}_{000} = (-2 rho)^n F_n(rho |PQ|^2).  R is [L+1]^3. */
#define RD (OR_MAXL4 + 1)
static void hermite_R(int L, double rho, const double *PQ, double *R /* RD^3 */)
{
    double F[RD + 1];
    double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
    oracle_boys(L, T, F);
    /* Rn[n][t][u][v] */
    static __thread double *Rn = NULL;
    if (!Rn) Rn = malloc(sizeof(double) * RD * RD * RD * RD);
#define RN(n, t, u, v) Rn[(((n) * RD + (t)) * RD + (u)) * RD + (v)]
    double f = 1.0;
    for (int n = 0; n <= L; ++n) { RN(n, 0, 0, 0) = f * F[n]; f *= -2.0 * rho; }
    for (int s = 1; s <= L; ++s)
        for (int t = 0; t <= s; ++t)
            for (int u = 0; u <= s - t; ++u) {
                int v = s - t - u;
                for (int n = 0; n <= L - s; ++n) {
                    double val;
                    if (t > 0) {
                        val = PQ[0] * RN(n + 1, t - 1, u, v);
                        if (t > 1) val += (t - 1) * RN(n + 1, t - 2, u, v);
                    } else if (u > 0) {
                        val = PQ[1] * RN(n + 1, t, u - 1, v);
                        if (u > 1) val += (u - 1) * RN(n + 1, t, u - 2, v);
                    } else {
                        val = PQ[2] * RN(n + 1, t, u, v - 1);
                        if (v > 1) val += (v - 1) * RN(n + 1, t, u, v - 2);
                    }
                    RN(n, t, u, v) = val;
                }
            }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) R[(t * RD + u) * RD + v] = RN(0, t, u, v);
#undef RN
}

/* contracted shell quartet by MMD; out[na][nb][nc][nd], unscaled components */
static void eri_mmd(const obasis *ob, int sa, int sb, int sc, int sd, double *out)
{
    int l[4] = {ob->sh_l[sa], ob->sh_l[sb], ob->sh_l[sc], ob->sh_l[sd]};
    int sh[4] = {sa, sb, sc, sd};
    int n[4];
    for (int i = 0; i < 4; ++i) n[i] = ncart(l[i]);
    int L = l[0] + l[1] + l[2] + l[3];
    const double *A = ob->xyz + 3 * ob->sh_atom[sa], *B = ob->xyz + 3 * ob->sh_atom[sb];
    const double *C = ob->xyz + 3 * ob->sh_atom[sc], *D = ob->xyz + 3 * ob->sh_atom[sd];
    int comp[4][10][3];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < n[i]; ++k) cart(l[i], k, &comp[i][k][0], &comp[i][k][1], &comp[i][k][2]);
    int ntot = n[0] * n[1] * n[2] * n[3];
    memset(out, 0, sizeof(double) * ntot);
    double *R = malloc(sizeof(double) * RD * RD * RD);
    int Lab = l[0] + l[1];
    double *W = malloc(sizeof(double) * (Lab + 1) * (Lab + 1) * (Lab + 1));
    double AB2 = 0, CD2 = 0;
    for (int k = 0; k < 3; ++k) { AB2 += (A[k] - B[k]) * (A[k] - B[k]); CD2 += (C[k] - D[k]) * (C[k] - D[k]); }
    for (int i = ob->prim_off[sa]; i < ob->prim_off[sa + 1]; ++i)
    for (int j = ob->prim_off[sb]; j < ob->prim_off[sb + 1]; ++j) {
        double ai = ob->exps[i], aj = ob->exps[j], zeta = ai + aj;
        double P[3], Eab[3][EDIM][EDIM][2 * EDIM];
        for (int k = 0; k < 3; ++k) {
            P[k] = (ai * A[k] + aj * B[k]) / zeta;
            hermite_E(l[0], l[1], zeta, P[k] - A[k], P[k] - B[k], Eab[k]);
        }
        double UP = ob->coef[i] * ob->coef[j] * pow(M_PI / zeta, 1.5) * exp(-ai * aj / zeta * AB2);
        for (int kk = ob->prim_off[sc]; kk < ob->prim_off[sc + 1]; ++kk)
        for (int ll = ob->prim_off[sd]; ll < ob->prim_off[sd + 1]; ++ll) {
            double ak = ob->exps[kk], al = ob->exps[ll], eta = ak + al;
            double Q[3], PQ[3], Ecd[3][EDIM][EDIM][2 * EDIM];
            for (int k = 0; k < 3; ++k) {
                Q[k] = (ak * C[k] + al * D[k]) / eta;
                PQ[k] = P[k] - Q[k];
                hermite_E(l[2], l[3], eta, Q[k] - C[k], Q[k] - D[k], Ecd[k]);
            }
            double UQ = ob->coef[kk] * ob->coef[ll] * pow(M_PI / eta, 1.5) * exp(-ak * al / eta * CD2);
            double rho = zeta * eta / (zeta + eta);
            double pref = UP * UQ * 2.0 * sqrt(rho) / sqrt(M_PI);
            hermite_R(L, rho, PQ, R);
            for (int c = 0; c < n[2]; ++c)
            for (int d = 0; d < n[3]; ++d) {
                const int *cc = comp[2][c], *dd = comp[3][d];
                /* W_tuv = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi} */
                for (int t = 0; t <= Lab; ++t)
                for (int u = 0; u <= Lab - t; ++u)
                for (int v = 0; v <= Lab - t - u; ++v) {
                    double s = 0;
                    for (int ta = 0; ta <= cc[0] + dd[0]; ++ta)
                    for (int nu = 0; nu <= cc[1] + dd[1]; ++nu)
                    for (int ph = 0; ph <= cc[2] + dd[2]; ++ph) {
                        double e = Ecd[0][cc[0]][dd[0]][ta] * Ecd[1][cc[1]][dd[1]][nu] * Ecd[2][cc[2]][dd[2]][ph];
                        if ((ta + nu + ph) & 1) e = -e;
                        s += e * R[((t + ta) * RD + (u + nu)) * RD + (v + ph)];
                    }
                    W[(t * (Lab + 1) + u) * (Lab + 1) + v] = s;
                }
                for (int a = 0; a < n[0]; ++a)
                for (int b = 0; b < n[1]; ++b) {
                    const int *aa = comp[0][a], *bb = comp[1][b];
                    double s = 0;
                    for (int t = 0; t <= aa[0] + bb[0]; ++t)
                    for (int u = 0; u <= aa[1] + bb[1]; ++u)
                    for (int v = 0; v <= aa[2] + bb[2]; ++v)
                        s += Eab[0][aa[0]][bb[0]][t] * Eab[1][aa[1]][bb[1]][u] * Eab[2][aa[2]][bb[2]][v]
                             * W[(t * (Lab + 1) + u) * (Lab + 1) + v];
                    out[((a * n[1] + b) * n[2] + c) * n[3] + d] += pref * s;
                }
            }
        }
    }
    free(R); free(W);
    (void)sh;
}

/* ----------------------------------------------- Obara-Saika / HGP ---- */
#define NCG(L) (((L) + 1) * ((L) + 2) * ((L) + 3) / 6) /* comps with total <= L */

static void eri_os(const obasis *ob, int sa, int sb, int sc, int sd, double *out)
{
    int la = ob->sh_l[sa], lb = ob->sh_l[sb], lc = ob->sh_l[sc], ld = ob->sh_l[sd];
    int Le = la + lb, Lf = lc + ld, L = Le + Lf;
    int ne = NCG(Le), nf = NCG(Lf), nm = L + 1;
    const double *A = ob->xyz + 3 * ob->sh_atom[sa], *B = ob->xyz + 3 * ob->sh_atom[sb];
    const double *C = ob->xyz + 3 * ob->sh_atom[sc], *D = ob->xyz + 3 * ob->sh_atom[sd];
    /* enumerate Cartesian tuples of every total */
    int ecomp[NCG(2 * OR_MAXL)][3];
    for (int l = 0; l <= 2 * OR_MAXL; ++l)
        for (int k = 0; k < ncart(l); ++k) {
            int x, y, z;
            cart(l, k, &x, &y, &z);
            int g = cart_index(x, y, z);
            ecomp[g][0] = x; ecomp[g][1] = y; ecomp[g][2] = z;
        }
    double *V = malloc(sizeof(double) * ne * nf * nm);
    double *Cn = calloc((size_t)ne * nf, sizeof(double)); /* contracted (e0|f0) */
#define VV(e, f, m) V[((size_t)(e) * nf + (f)) * nm + (m)]
    double AB2 = 0, CD2 = 0;
    for (int k = 0; k < 3; ++k) { AB2 += (A[k] - B[k]) * (A[k] - B[k]); CD2 += (C[k] - D[k]) * (C[k] - D[k]); }
    for (int i = ob->prim_off[sa]; i < ob->prim_off[sa + 1]; ++i)
    for (int j = ob->prim_off[sb]; j < ob->prim_off[sb + 1]; ++j)
    for (int kk = ob->prim_off[sc]; kk < ob->prim_off[sc + 1]; ++kk)
    for (int ll = ob->prim_off[sd]; ll < ob->prim_off[sd + 1]; ++ll) {
        double ai = ob->exps[i], aj = ob->exps[j], ak = ob->exps[kk], al = ob->exps[ll];
        double zeta = ai + aj, eta = ak + al, zpe = zeta + eta, rho = zeta * eta / zpe;
        double P[3], Q[3], PA[3], QC[3], WP[3], WQ[3], PQ2 = 0;
        for (int k = 0; k < 3; ++k) {
            P[k] = (ai * A[k] + aj * B[k]) / zeta;
            Q[k] = (ak * C[k] + al * D[k]) / eta;
            PA[k] = P[k] - A[k];
            QC[k] = Q[k] - C[k];
            double pq = P[k] - Q[k];
            WP[k] = -eta / zpe * pq;  /* W - P */
            WQ[k] = zeta / zpe * pq;  /* W - Q */
            PQ2 += pq * pq;
        }
        double UP = ob->coef[i] * ob->coef[j] * pow(M_PI / zeta, 1.5) * exp(-ai * aj / zeta * AB2);
        double UQ = ob->coef[kk] * ob->coef[ll] * pow(M_PI / eta, 1.5) * exp(-ak * al / eta * CD2);
        double F[OR_MAXL4 + 1];
        oracle_boys(L, rho * PQ2, F);
        double pref = UP * UQ * 2.0 * sqrt(rho) / sqrt(M_PI);
        for (int m = 0; m <= L; ++m) VV(0, 0, m) = pref * F[m];
        /* vrr1: build e on the bra with f = 0 */
        for (int e = 1; e < ne; ++e) {
            const int *ev = ecomp[e];
            int le = ev[0] + ev[1] + ev[2];
            int d = ev[0] ? 0 : (ev[1] ? 1 : 2);
            int e1[3] = {ev[0], ev[1], ev[2]};
            e1[d] -= 1;
            int g1 = cart_index(e1[0], e1[1], e1[2]);
            int has2 = e1[d] > 0, g2 = 0;
            if (has2) { int e2[3] = {e1[0], e1[1], e1[2]}; e2[d] -= 1; g2 = cart_index(e2[0], e2[1], e2[2]); }
            for (int m = 0; m <= L - le; ++m) {
                double v = PA[d] * VV(g1, 0, m) + WP[d] * VV(g1, 0, m + 1);
                if (has2) v += e1[d] / (2 * zeta) * (VV(g2, 0, m) - rho / zeta * VV(g2, 0, m + 1));
                VV(e, 0, m) = v;
            }
        }
        /* vrr2: build f on the ket, for every e */
        for (int f = 1; f < nf; ++f) {
            const int *fv = ecomp[f];
            int lf = fv[0] + fv[1] + fv[2];
            int d = fv[0] ? 0 : (fv[1] ? 1 : 2);
            int f1[3] = {fv[0], fv[1], fv[2]};
            f1[d] -= 1;
            int h1 = cart_index(f1[0], f1[1], f1[2]);
            int has2 = f1[d] > 0, h2 = 0;
            if (has2) { int f2[3] = {f1[0], f1[1], f1[2]}; f2[d] -= 1; h2 = cart_index(f2[0], f2[1], f2[2]); }
            for (int e = 0; e < ne; ++e) {
                const int *ev = ecomp[e];
                int le = ev[0] + ev[1] + ev[2];
                int hase = ev[d] > 0, ge = 0;
                if (hase) { int em[3] = {ev[0], ev[1], ev[2]}; em[d] -= 1; ge = cart_index(em[0], em[1], em[2]); }
                for (int m = 0; m <= L - le - lf; ++m) {
                    double v = QC[d] * VV(e, h1, m) + WQ[d] * VV(e, h1, m + 1);
                    if (has2) v += f1[d] / (2 * eta) * (VV(e, h2, m) - rho / eta * VV(e, h2, m + 1));
                    if (hase) v += ev[d] / (2 * zpe) * VV(ge, h1, m + 1);
                    VV(e, f, m) = v;
                }
            }
        }
        for (int e = 0; e < ne; ++e)
            for (int f = 0; f < nf; ++f) Cn[(size_t)e * nf + f] += VV(e, f, 0);
    }
#undef VV
    /* hrr on the bra: (a b+1_i| = (a+1_i b| + AB_i (a b|  for every f */
    int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    /* H[a_g][b_g][f] with a over totals <= Le, b over totals <= lb */
    int nbg = NCG(lb);
    double *H = calloc((size_t)ne * nbg * nf, sizeof(double));
#define HH(a, b, f) H[((size_t)(a) * nbg + (b)) * nf + (f)]
    for (int a = 0; a < ne; ++a)
        for (int f = 0; f < nf; ++f) HH(a, 0, f) = Cn[(size_t)a * nf + f];
    for (int lbb = 1; lbb <= lb; ++lbb)
        for (int kb = 0; kb < ncart(lbb); ++kb) {
            int bv[3];
            cart(lbb, kb, &bv[0], &bv[1], &bv[2]);
            int d = bv[0] ? 0 : (bv[1] ? 1 : 2);
            int b1[3] = {bv[0], bv[1], bv[2]};
            b1[d] -= 1;
            int gb = cart_index(bv[0], bv[1], bv[2]), gb1 = cart_index(b1[0], b1[1], b1[2]);
            for (int a = 0; a < NCG(Le - lbb); ++a) {
                int av[3] = {ecomp[a][0], ecomp[a][1], ecomp[a][2]};
                int ap[3] = {av[0], av[1], av[2]};
                ap[d] += 1;
                int ga1 = cart_index(ap[0], ap[1], ap[2]);
                for (int f = 0; f < nf; ++f)
                    HH(a, gb, f) = HH(ga1, gb1, f) + (A[d] - B[d]) * HH(a, gb1, f);
            }
        }
    /* hrr on the ket for every target (a,b) */
    int ndg = NCG(ld);
    double *K2 = malloc(sizeof(double) * nf * ndg);
#define KK(c, dd) K2[(size_t)(c) * ndg + (dd)]
    for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < nb; ++ib) {
        int av[3], bv[3];
        cart(la, ia, &av[0], &av[1], &av[2]);
        cart(lb, ib, &bv[0], &bv[1], &bv[2]);
        int ga = cart_index(av[0], av[1], av[2]), gb = cart_index(bv[0], bv[1], bv[2]);
        for (int c = 0; c < nf; ++c) KK(c, 0) = HH(ga, gb, c);
        for (int ldd = 1; ldd <= ld; ++ldd)
            for (int kd = 0; kd < ncart(ldd); ++kd) {
                int dv[3];
                cart(ldd, kd, &dv[0], &dv[1], &dv[2]);
                int d = dv[0] ? 0 : (dv[1] ? 1 : 2);
                int d1[3] = {dv[0], dv[1], dv[2]};
                d1[d] -= 1;
                int gd = cart_index(dv[0], dv[1], dv[2]), gd1 = cart_index(d1[0], d1[1], d1[2]);
                for (int c = 0; c < NCG(Lf - ldd); ++c) {
                    int cp[3] = {ecomp[c][0], ecomp[c][1], ecomp[c][2]};
                    cp[d] += 1;
                    int gc1 = cart_index(cp[0], cp[1], cp[2]);
                    KK(c, gd) = KK(gc1, gd1) + (C[d] - D[d]) * KK(c, gd1);
                }
            }
        for (int ic = 0; ic < nc; ++ic)
        for (int id = 0; id < nd; ++id) {
            int cv[3], dv[3];
            cart(lc, ic, &cv[0], &cv[1], &cv[2]);
            cart(ld, id, &dv[0], &dv[1], &dv[2]);
            out[((ia * nb + ib) * nc + ic) * nd + id] =
                KK(cart_index(cv[0], cv[1], cv[2]), cart_index(dv[0], dv[1], dv[2]));
        }
    }
#undef KK
#undef HH
    free(K2); free(H); free(V); free(Cn);
}

static void eri_scaled(const obasis *ob, int method, int sa, int sb, int sc, int sd, double *out)
{
    if (method == 1) eri_os(ob, sa, sb, sc, sd, out);
    else eri_mmd(ob, sa, sb, sc, sd, out);
    int n[4] = {ncart(ob->sh_l[sa]), ncart(ob->sh_l[sb]), ncart(ob->sh_l[sc]), ncart(ob->sh_l[sd])};
    const double *s0 = ob->cscale + ob->bf_off[sa], *s1 = ob->cscale + ob->bf_off[sb];
    const double *s2 = ob->cscale + ob->bf_off[sc], *s3 = ob->cscale + ob->bf_off[sd];
    for (int a = 0; a < n[0]; ++a)
    for (int b = 0; b < n[1]; ++b)
    for (int c = 0; c < n[2]; ++c)
    for (int d = 0; d < n[3]; ++d)
        out[((a * n[1] + b) * n[2] + c) * n[3] + d] *= s0[a] * s1[b] * s2[c] * s3[d];
}

/* ---------------------------------------------------------- exports ---- */
#define OB_ARGS int natom, const int *Z, const double *xyz, int nshell, const int *sh_atom, \
                const int *sh_l, const int *sh_nprim, const double *exps, const double *coefs
#define OB_PASS natom, Z, xyz, nshell, sh_atom, sh_l, sh_nprim, exps, coefs

int oracle_nbf(OB_ARGS)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    int n = ob.nbf;
    ob_free(&ob);
    return n;
}

/* one contracted, normalised shell quartet; method 0 = MMD, 1 = OS/HGP */
int oracle_eri_quartet(OB_ARGS, int sa, int sb, int sc, int sd, int method, double *out)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    eri_scaled(&ob, method, sa, sb, sc, sd, out);
    ob_free(&ob);
    return 0;
}

/* nq listed shell quartets q[4k..4k+3], each evaluated as oracle_eri_quartet
 * does (MMD), OpenMP over the list; the sum of |(ab|cd)| over every integral is
 * returned in *sink.  Used to time the oracle on a sample of a workload's
 * quartets; adds no arithmetic of its own. */
int oracle_eri_list(OB_ARGS, int nq, const int *q, int nthreads, double *sink)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    double total = 0.0;
#pragma omp parallel reduction(+ : total)
    {
        double *buf = malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 4)
        for (int k = 0; k < nq; ++k) {
            const int *t = q + 4 * k;
            eri_scaled(&ob, 0, t[0], t[1], t[2], t[3], buf);
            const int n = ncart(sh_l[t[0]]) * ncart(sh_l[t[1]]) * ncart(sh_l[t[2]]) * ncart(sh_l[t[3]]);
            for (int i = 0; i < n; ++i) total += fabs(buf[i]);
        }
        free(buf);
    }
    *sink = total;
    ob_free(&ob);
    return 0;
}

/* full N^4 tensor (tiny systems only) */
int oracle_eri_full(OB_ARGS, double *out)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    int N = ob.nbf;
    double *buf = malloc(sizeof(double) * 10000);
    for (int a = 0; a < nshell; ++a)
    for (int b = 0; b < nshell; ++b)
    for (int c = 0; c < nshell; ++c)
    for (int d = 0; d < nshell; ++d) {
        eri_scaled(&ob, 0, a, b, c, d, buf);
        int n1 = ncart(sh_l[b]), n2 = ncart(sh_l[c]), n3 = ncart(sh_l[d]);
        for (int i = 0; i < ncart(sh_l[a]); ++i)
        for (int j = 0; j < n1; ++j)
        for (int k = 0; k < n2; ++k)
        for (int l = 0; l < n3; ++l) {
            size_t p = ob.bf_off[a] + i, q = ob.bf_off[b] + j, r = ob.bf_off[c] + k, s = ob.bf_off[d] + l;
            out[((p * N + q) * N + r) * N + s] = buf[((i * n1 + j) * n2 + k) * n3 + l];
        }
    }
    free(buf);
    ob_free(&ob);
    return 0;
}

/* J and K over all shell quartets: each unique shell quartet (a>=b, c>=d,
 * ab>=cd) is computed once; every DISTINCT ordered shell quartet in its
 * permutation orbit then adds its integrals literally to J and K. */
int oracle_jk(OB_ARGS, const double *Dm, double *J, double *K, int nthreads)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    int N = ob.nbf;
    int npair = nshell * (nshell + 1) / 2;
    int *pa = malloc(sizeof(int) * npair), *pb = malloc(sizeof(int) * npair);
    for (int a = 0, p = 0; a < nshell; ++a)
        for (int b = 0; b <= a; ++b, ++p) { pa[p] = a; pb[p] = b; }
    memset(J, 0, sizeof(double) * N * N);
    memset(K, 0, sizeof(double) * N * N);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *Jt = calloc((size_t)N * N, sizeof(double));
        double *Kt = calloc((size_t)N * N, sizeof(double));
        double *v = malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npair; ++p)
            for (int q = 0; q <= p; ++q) {
                int s[4] = {pa[p], pb[p], pa[q], pb[q]};
                eri_scaled(&ob, 0, s[0], s[1], s[2], s[3], v);
                int n[4];
                for (int i = 0; i < 4; ++i) n[i] = ncart(sh_l[s[i]]);
                /* the 8 index permutations as position maps */
                static const int perms[8][4] = {{0,1,2,3},{1,0,2,3},{0,1,3,2},{1,0,3,2},
                                                {2,3,0,1},{3,2,0,1},{2,3,1,0},{3,2,1,0}};
                int seen[8][4], nseen = 0;
                for (int pi = 0; pi < 8; ++pi) {
                    int t[4];
                    for (int k = 0; k < 4; ++k) t[k] = s[perms[pi][k]];
                    int dup = 0;
                    for (int u = 0; u < nseen; ++u)
                        if (!memcmp(seen[u], t, sizeof t)) { dup = 1; break; }
                    if (dup) continue;
                    memcpy(seen[nseen++], t, sizeof t);
                    const int *src = perms[pi];
                    int m[4];
                    for (int k = 0; k < 4; ++k) m[k] = n[src[k]];
                    int idx[4];
                    for (idx[0] = 0; idx[0] < m[0]; ++idx[0])
                    for (idx[1] = 0; idx[1] < m[1]; ++idx[1])
                    for (idx[2] = 0; idx[2] < m[2]; ++idx[2])
                    for (idx[3] = 0; idx[3] < m[3]; ++idx[3]) {
                        int ci[4];
                        for (int k = 0; k < 4; ++k) ci[src[k]] = idx[k];
                        double val = v[((ci[0] * n[1] + ci[1]) * n[2] + ci[2]) * n[3] + ci[3]];
                        int P0 = ob.bf_off[t[0]] + idx[0], P1 = ob.bf_off[t[1]] + idx[1];
                        int P2 = ob.bf_off[t[2]] + idx[2], P3 = ob.bf_off[t[3]] + idx[3];
                        Jt[(size_t)P0 * N + P1] += val * Dm[(size_t)P2 * N + P3];
                        Kt[(size_t)P0 * N + P2] += val * Dm[(size_t)P1 * N + P3];
                    }
                }
            }
#pragma omp critical
        {
            for (size_t i = 0; i < (size_t)N * N; ++i) { J[i] += Jt[i]; K[i] += Kt[i]; }
        }
        free(Jt); free(Kt); free(v);
    }
    free(pa); free(pb);
    ob_free(&ob);
    return 0;
}

/* Selected shell blocks of J and K by the literal unsymmetrised sums:
 *   J[A,B] block = sum over ALL ordered shells (C,D) of (AB|CD) D_CD
 *   K[A,C] block = sum over ALL ordered shells (B,D) of (AB|CD) D_BD
 * Jout/Kout hold the blocks one after the other, row-major. */
int oracle_jk_blocks(OB_ARGS, const double *Dm, int nJ, const int *Jsh, double *Jout,
                     int nK, const int *Ksh, double *Kout, int nthreads)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    int N = ob.nbf;
    int *Joff = malloc(sizeof(int) * (nJ + 1)), *Koff = malloc(sizeof(int) * (nK + 1));
    Joff[0] = 0; Koff[0] = 0;
    for (int i = 0; i < nJ; ++i) Joff[i + 1] = Joff[i] + ncart(sh_l[Jsh[2 * i]]) * ncart(sh_l[Jsh[2 * i + 1]]);
    for (int i = 0; i < nK; ++i) Koff[i + 1] = Koff[i] + ncart(sh_l[Ksh[2 * i]]) * ncart(sh_l[Ksh[2 * i + 1]]);
    memset(Jout, 0, sizeof(double) * Joff[nJ]);
    memset(Kout, 0, sizeof(double) * Koff[nK]);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int ntask = (nJ + nK) * nshell;
#pragma omp parallel
    {
        double *v = malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 1)
        for (int task = 0; task < ntask; ++task) {
            int blk = task / nshell, x = task % nshell;
            if (blk < nJ) {
                int A = Jsh[2 * blk], B = Jsh[2 * blk + 1], Cs = x;
                int na = ncart(sh_l[A]), nb = ncart(sh_l[B]), nc = ncart(sh_l[Cs]);
                double *acc = calloc(na * nb, sizeof(double));
                for (int Ds = 0; Ds < nshell; ++Ds) {
                    int nd = ncart(sh_l[Ds]);
                    eri_scaled(&ob, 0, A, B, Cs, Ds, v);
                    for (int a = 0; a < na; ++a) for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c) for (int d = 0; d < nd; ++d)
                        acc[a * nb + b] += v[((a * nb + b) * nc + c) * nd + d]
                                           * Dm[(size_t)(ob.bf_off[Cs] + c) * N + ob.bf_off[Ds] + d];
                }
#pragma omp critical
                for (int i = 0; i < na * nb; ++i) Jout[Joff[blk] + i] += acc[i];
                free(acc);
            } else {
                int kb = blk - nJ;
                int A = Ksh[2 * kb], Cs = Ksh[2 * kb + 1], B = x;
                int na = ncart(sh_l[A]), nb = ncart(sh_l[B]), nc = ncart(sh_l[Cs]);
                double *acc = calloc(na * nc, sizeof(double));
                for (int Ds = 0; Ds < nshell; ++Ds) {
                    int nd = ncart(sh_l[Ds]);
                    eri_scaled(&ob, 0, A, B, Cs, Ds, v);
                    for (int a = 0; a < na; ++a) for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c) for (int d = 0; d < nd; ++d)
                        acc[a * nc + c] += v[((a * nb + b) * nc + c) * nd + d]
                                           * Dm[(size_t)(ob.bf_off[B] + b) * N + ob.bf_off[Ds] + d];
                }
#pragma omp critical
                for (int i = 0; i < na * nc; ++i) Kout[Koff[kb] + i] += acc[i];
                free(acc);
            }
        }
        free(v);
    }
    free(Joff); free(Koff);
    ob_free(&ob);
    return 0;
}

/* One-electron integrals S, T (kinetic), V (nuclear attraction), Hermite form. */
int oracle_oneel(OB_ARGS, double *S, double *T, double *V)
{
    obasis ob;
    if (ob_init(&ob, OB_PASS)) return -1;
    int N = ob.nbf;
    for (int sa = 0; sa < nshell; ++sa)
    for (int sb = 0; sb < nshell; ++sb) {
        int la = sh_l[sa], lb = sh_l[sb];
        const double *A = xyz + 3 * sh_atom[sa], *B = xyz + 3 * sh_atom[sb];
        double AB2 = 0;
        for (int k = 0; k < 3; ++k) AB2 += (A[k] - B[k]) * (A[k] - B[k]);
        for (int ia = 0; ia < ncart(la); ++ia)
        for (int ib = 0; ib < ncart(lb); ++ib) {
            int a[3], b[3];
            cart(la, ia, &a[0], &a[1], &a[2]);
            cart(lb, ib, &b[0], &b[1], &b[2]);
            double s = 0, t = 0, v = 0;
            for (int i = ob.prim_off[sa]; i < ob.prim_off[sa + 1]; ++i)
            for (int j = ob.prim_off[sb]; j < ob.prim_off[sb + 1]; ++j) {
                double al = ob.exps[i], be = ob.exps[j], p = al + be;
                double P[3], E[3][EDIM][EDIM][2 * EDIM];
                for (int k = 0; k < 3; ++k) {
                    P[k] = (al * A[k] + be * B[k]) / p;
                    hermite_E(la, lb + 2, p, P[k] - A[k], P[k] - B[k], E[k]);
                }
                double Kab = exp(-al * be / p * AB2), cc = ob.coef[i] * ob.coef[j];
                double s1[3], t1[3];
                for (int k = 0; k < 3; ++k) {
                    double sq = sqrt(M_PI / p);
                    s1[k] = E[k][a[k]][b[k]][0] * sq;
                    double tk = -2 * be * be * E[k][a[k]][b[k] + 2][0] * sq + be * (2 * b[k] + 1) * s1[k];
                    if (b[k] >= 2) tk -= 0.5 * b[k] * (b[k] - 1) * E[k][a[k]][b[k] - 2][0] * sq;
                    t1[k] = tk;
                }
                s += cc * Kab * s1[0] * s1[1] * s1[2];
                t += cc * Kab * (t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2] + s1[0] * s1[1] * t1[2]);
                /* nuclear attraction: -Z_C (2 pi/p) sum_tuv E_t E_u E_v R_tuv(p, P-C) */
                int Lt = la + lb;
                double R[RD * RD * RD];
                for (int c = 0; c < natom; ++c) {
                    double PC[3] = {P[0] - xyz[3 * c], P[1] - xyz[3 * c + 1], P[2] - xyz[3 * c + 2]};
                    hermite_R(Lt, p, PC, R);
                    double acc = 0;
                    for (int tt = 0; tt <= a[0] + b[0]; ++tt)
                    for (int uu = 0; uu <= a[1] + b[1]; ++uu)
                    for (int vv = 0; vv <= a[2] + b[2]; ++vv)
                        acc += E[0][a[0]][b[0]][tt] * E[1][a[1]][b[1]][uu] * E[2][a[2]][b[2]][vv]
                               * R[(tt * RD + uu) * RD + vv];
                    v += -Z[c] * 2 * M_PI / p * Kab * cc * acc;
                }
            }
            double sc = ob.cscale[ob.bf_off[sa] + ia] * ob.cscale[ob.bf_off[sb] + ib];
            size_t idx = (size_t)(ob.bf_off[sa] + ia) * N + ob.bf_off[sb] + ib;
            S[idx] = s * sc; T[idx] = t * sc; V[idx] = v * sc;
        }
    }
    ob_free(&ob);
    return 0;
}

double oracle_enuc(int natom, const int *Z, const double *xyz)
{
    double e = 0;
    for (int a = 0; a < natom; ++a)
        for (int b = 0; b < a; ++b) {
            double r2 = 0;
            for (int k = 0; k < 3; ++k) r2 += (xyz[3 * a + k] - xyz[3 * b + k]) * (xyz[3 * a + k] - xyz[3 * b + k]);
            e += Z[a] * Z[b] / sqrt(r2);
        }
    return e;
}

/* Count of nonzero Hermite coefficients E^{ab}_{tuv} over all component pairs
 * of a shell pair (la, lb), out of the dense count ncart(la) ncart(lb)
 * (la+lb+1)(la+lb+2)(la+lb+3)/6 (MMD section, E-tensor size remark). */
void oracle_hermite_nnz(int la, int lb, double zeta, const double *PA, const double *PB,
                        int *dense, int *nnz)
{
    double E[3][EDIM][EDIM][2 * EDIM];
    for (int k = 0; k < 3; ++k) hermite_E(la, lb, zeta, PA[k], PB[k], E[k]);
    int L = la + lb, cnt = 0, tot = 0;
    for (int ia = 0; ia < ncart(la); ++ia)
    for (int ib = 0; ib < ncart(lb); ++ib) {
        int a[3], b[3];
        cart(la, ia, &a[0], &a[1], &a[2]);
        cart(lb, ib, &b[0], &b[1], &b[2]);
        for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
        for (int v = 0; v <= L - t - u; ++v) {
            ++tot;
            double e = (t <= a[0] + b[0] ? E[0][a[0]][b[0]][t] : 0.0)
                     * (u <= a[1] + b[1] ? E[1][a[1]][b[1]][u] : 0.0)
                     * (v <= a[2] + b[2] ? E[2][a[2]][b[2]][v] : 0.0);
            if (e != 0.0) ++cnt;
        }
    }
    *dense = tot; *nnz = cnt;
}
