// Rys-quadrature electron repulsion integrals of contracted Cartesian shells.
//
// The contracted integral (ab|cd) is the sum over primitive quartets
// [ab|cd]_ijkl (paper, "Notation", definition of contracted ERIs).  For one
// primitive quartet with exponents zeta = a_i + a_j, eta = a_k + a_l, centres
// P, Q (eq. zeta) and prefactors U_P, U_Q:
//
//   [ab|cd] = U_P U_Q (2/sqrt(pi)) sqrt(rho) sum_r w_r Ix_r Iy_r Iz_r,
//   rho = zeta eta / (zeta + eta),  T = rho |P - Q|^2,
//
// where (u_r, w_r) is the n-point Rys rule of T (n = floor(L/2) + 1) and the
// factors I_r are 1-D integrals built by the vertical recurrences of eqs.
// vrr1/vrr2 with the ratio [.]^(m+1)/[.]^(m) replaced by the root u_r:
//
//   I(e+1,f) = C00 I(e,f) + e B10 I(e-1,f) + f B00 I(e,f-1)
//   I(e,f+1) = C00' I(e,f) + f B01 I(e,f-1) + e B00 I(e-1,f)
//   C00  = PA - eta/(zeta+eta) (P-Q) u,   C00' = QC + zeta/(zeta+eta) (P-Q) u,
//   B10  = (1 - eta u/(zeta+eta))/(2 zeta),  B01 = (1 - zeta u/(zeta+eta))/(2 eta),
//   B00  = u / (2 (zeta+eta)),
//
// followed by the horizontal recurrences of eq. hrr applied per axis,
// I(a,b+1) = I(a+1,b) + AB I(a,b) and I(.., c,d+1) = I(.., c+1,d) + CD I(.., c,d),
// which need no primitive data.  (The printed eq. vrr2 carries a minus sign on
// its PQ term; with PQ = P - Q the consistent sign is plus, since W - Q =
// zeta (P-Q)/(zeta+eta).)
//
// All loops have compile-time trip counts so that every array lives in
// registers after unrolling.
#pragma once

#include "fk_rys.h"

namespace fk {

constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian exponents of component k of a shell of total l, ordered
// x^l, x^(l-1)y, x^(l-1)z, ..., z^l.
struct CartTab {
    int x[4][10], y[4][10], z[4][10];
};
constexpr CartTab make_cart() {
    CartTab t{};
    for (int l = 0; l < 4; ++l) {
        int k = 0;
        for (int a = l; a >= 0; --a)
            for (int b = l - a; b >= 0; --b) {
                t.x[l][k] = a; t.y[l][k] = b; t.z[l][k] = l - a - b;
                ++k;
            }
    }
    return t;
}
constexpr CartTab kCart = make_cart();

template <int LA, int LB, int LC, int LD>
struct QClass {
    static constexpr int L = LA + LB + LC + LD;
    static constexpr int NR = L / 2 + 1;
    static constexpr int LAB = LA + LB, LCD = LC + LD;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NOUT = NA * NB * NC * ND;
};

// Primitive-pair data as consumed by the integral code.
struct PrimPair {
    double zeta;   // exponent sum
    double oo2z;   // 1 / (2 zeta)
    double P[3];   // Gaussian product centre
    double PA[3];  // P - A (A = centre of the pair's first shell)
    double K;      // c_i c_j (pi/zeta)^(3/2) exp(-a_i a_j/zeta |AB|^2) (2/sqrt(pi))^(1/2) sqrt(zeta)
};

// 2-D recurrences of one axis for one root followed by both horizontal
// recurrences; I[a][b][c][d] for a <= LA, b <= LB, c <= LC, d <= LD.
template <int LA, int LB, int LC, int LD, typename R = double>
FK_HD void vrr_hrr_axis(R C00, R C00p, R B00, R B10, R B01, R AB, R CD, R g00,
                        R (&I)[LA + 1][LB + 1][LC + 1][LD + 1])
{
    constexpr int LAB = LA + LB, LCD = LC + LD;
    R G[LAB + 1][LCD + 1];
    G[0][0] = g00;
    if constexpr (LAB > 0) {
        G[1][0] = C00 * g00;
#pragma unroll
        for (int e = 1; e < LAB; ++e) G[e + 1][0] = C00 * G[e][0] + (R)e * B10 * G[e - 1][0];
    }
    if constexpr (LCD > 0) {
        G[0][1] = C00p * g00;
#pragma unroll
        for (int e = 1; e <= LAB; ++e) G[e][1] = C00p * G[e][0] + (R)e * B00 * G[e - 1][0];
#pragma unroll
        for (int f = 1; f < LCD; ++f) {
            G[0][f + 1] = C00p * G[0][f] + (R)f * B01 * G[0][f - 1];
#pragma unroll
            for (int e = 1; e <= LAB; ++e)
                G[e][f + 1] = C00p * G[e][f] + (R)f * B01 * G[e][f - 1] + (R)e * B00 * G[e - 1][f];
        }
    }
    // bra HRR: H[a][b][f], valid for a <= LAB - b
    R H[LAB + 1][LB + 1][LCD + 1];
#pragma unroll
    for (int e = 0; e <= LAB; ++e)
#pragma unroll
        for (int f = 0; f <= LCD; ++f) H[e][0][f] = G[e][f];
#pragma unroll
    for (int b = 0; b < LB; ++b)
#pragma unroll
        for (int a = 0; a < LAB - b; ++a)
#pragma unroll
            for (int f = 0; f <= LCD; ++f) H[a][b + 1][f] = H[a + 1][b][f] + AB * H[a][b][f];
    // ket HRR for every (a, b)
#pragma unroll
    for (int a = 0; a <= LA; ++a)
#pragma unroll
        for (int b = 0; b <= LB; ++b) {
            R Kt[LCD + 1][LD + 1];
#pragma unroll
            for (int c = 0; c <= LCD; ++c) Kt[c][0] = H[a][b][c];
#pragma unroll
            for (int d = 0; d < LD; ++d)
#pragma unroll
                for (int c = 0; c < LCD - d; ++c) Kt[c][d + 1] = Kt[c + 1][d] + CD * Kt[c][d];
#pragma unroll
            for (int c = 0; c <= LC; ++c)
#pragma unroll
                for (int d = 0; d <= LD; ++d) I[a][b][c][d] = Kt[c][d];
        }
}

// Shared per-primitive-quartet set-up.
struct QuartetSetup {
    double inv, ez, zz, pref, T;
    double PQ[3];
};

// 1/sqrt(x) for x > 0: on the device the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2)/2 (each doubles the correct bits); on the
// host the library functions.
FK_HD double fk_rsqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
#else
    return 1.0 / sqrt(x);
#endif
}

// One reciprocal square root serves the quartet: with r = (zeta + eta)^(-1/2),
// 1/(zeta + eta) = r^2 and, since each pair's K carries sqrt(zeta),
// K_P K_Q r = K_P K_Q sqrt(zeta eta / (zeta + eta)) (the sqrt(rho) of the
// fundamental integral).
FK_HD QuartetSetup quartet_setup(const PrimPair &p, const PrimPair &q)
{
    QuartetSetup s;
    const double r = fk_rsqrt(p.zeta + q.zeta);
    s.inv = r * r;
    s.PQ[0] = p.P[0] - q.P[0];
    s.PQ[1] = p.P[1] - q.P[1];
    s.PQ[2] = p.P[2] - q.P[2];
    s.T = (p.zeta * q.zeta * s.inv) * (s.PQ[0] * s.PQ[0] + s.PQ[1] * s.PQ[1] + s.PQ[2] * s.PQ[2]);
    s.pref = p.K * q.K * r;
    s.ez = q.zeta * s.inv;
    s.zz = p.zeta * s.inv;
    return s;
}

// Adds the primitive quartet [ab|cd] to acc[NA][NB][NC][ND] (all components).
// Adds the primitive quartet [ab|cd] to acc[NA][NB][NC][ND] (all components).
// The set-up (T, prefactor) and the roots and weights are FP64; the 2-D
// recurrences, transfers and products run in R (double, or float for the
// quartets the precision split assigns to FP32).
template <int LA, int LB, int LC, int LD, typename R = double, bool BRANCHLESS = false>
FK_HD void rys_prim_all(const double *__restrict tab, const PrimPair &p, const PrimPair &q,
                        const double AB[3], const double CD[3], R *__restrict acc)
{
    using Q = QClass<LA, LB, LC, LD>;
    QuartetSetup s = quartet_setup(p, q);
    double u[Q::NR], w[Q::NR];
    rys_roots<Q::NR, (Q::L > 0), BRANCHLESS>(s.T, tab, u, w);
    if constexpr (Q::L == 0) {
        acc[0] += (R)(w[0] * s.pref);
        return;
    } else {
        R ezPQ[3], zzPQ[3], PA[3], QC[3], ab[3], cd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ezPQ[k] = (R)(s.ez * s.PQ[k]);
            zzPQ[k] = (R)(s.zz * s.PQ[k]);
            PA[k] = (R)p.PA[k];
            QC[k] = (R)q.PA[k];
            ab[k] = (R)AB[k];
            cd[k] = (R)CD[k];
        }
        const R hinv = (R)(0.5 * s.inv), ez = (R)s.ez, zz = (R)s.zz, po = (R)p.oo2z, qo = (R)q.oo2z;
#pragma unroll
        for (int r = 0; r < Q::NR; ++r) {
            const R ur = (R)u[r];
            const R B00 = hinv * ur;
            const R B10 = po * ((R)1 - ez * ur);
            const R B01 = qo * ((R)1 - zz * ur);
            R I[3][LA + 1][LB + 1][LC + 1][LD + 1];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                vrr_hrr_axis<LA, LB, LC, LD, R>(PA[k] - ezPQ[k] * ur, QC[k] + zzPQ[k] * ur, B00, B10, B01, ab[k], cd[k],
                                                k == 2 ? (R)(w[r] * s.pref) : (R)1, I[k]);
#pragma unroll
            for (int ia = 0; ia < Q::NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < Q::NB; ++ib)
#pragma unroll
                    for (int ic = 0; ic < Q::NC; ++ic)
#pragma unroll
                        for (int id = 0; id < Q::ND; ++id) {
                            const int o = ((ia * Q::NB + ib) * Q::NC + ic) * Q::ND + id;
                            acc[o] += I[0][kCart.x[LA][ia]][kCart.x[LB][ib]][kCart.x[LC][ic]][kCart.x[LD][id]]
                                    * I[1][kCart.y[LA][ia]][kCart.y[LB][ib]][kCart.y[LC][ic]][kCart.y[LD][id]]
                                    * I[2][kCart.z[LA][ia]][kCart.z[LB][ib]][kCart.z[LC][ic]][kCart.z[LD][id]];
                        }
        }
    }
}

// Binomial coefficients for the closed form of the horizontal recurrence
// (x - B)^b = sum_k C(b,k) (A - B)^(b-k) (x - A)^k.
FK_HD constexpr double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// One bra component (ax, bx per axis given at run time) of a primitive
// quartet: adds w * prod over axes of I(a,b; c,d) for every ket component
// (c, d) to acc[NC][ND].  Used when the full output block of a class is too
// large for one lane: each lane then owns some bra components.
template <int LA, int LB, int LC, int LD>
FK_HD void rys_prim_bra_comp(const double *__restrict tab, const PrimPair &p, const PrimPair &q,
                             const double AB[3], const double CD[3], const int a[3], const int b[3],
                             double *__restrict acc)
{
    using Q = QClass<LA, LB, LC, LD>;
    constexpr int LAB = Q::LAB, LCD = Q::LCD;
    QuartetSetup s = quartet_setup(p, q);
    double u[Q::NR], w[Q::NR];
    rys_roots<Q::NR, true>(s.T, tab, u, w);
#pragma unroll
    for (int r = 0; r < Q::NR; ++r) {
        const double ur = u[r];
        const double B00 = 0.5 * s.inv * ur;
        const double B10 = p.oo2z * (1.0 - s.ez * ur);
        const double B01 = q.oo2z * (1.0 - s.zz * ur);
        double I[3][LC + 1][LD + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double C00 = p.PA[k] - s.ez * s.PQ[k] * ur;
            const double C00p = q.PA[k] + s.zz * s.PQ[k] * ur;
            double G[LAB + 1][LCD + 1];
            G[0][0] = (k == 2) ? w[r] * s.pref : 1.0;
            if constexpr (LAB > 0) {
                G[1][0] = C00 * G[0][0];
#pragma unroll
                for (int e = 1; e < LAB; ++e) G[e + 1][0] = C00 * G[e][0] + (double)e * B10 * G[e - 1][0];
            }
            if constexpr (LCD > 0) {
                G[0][1] = C00p * G[0][0];
#pragma unroll
                for (int e = 1; e <= LAB; ++e) G[e][1] = C00p * G[e][0] + (double)e * B00 * G[e - 1][0];
#pragma unroll
                for (int f = 1; f < LCD; ++f) {
                    G[0][f + 1] = C00p * G[0][f] + (double)f * B01 * G[0][f - 1];
#pragma unroll
                    for (int e = 1; e <= LAB; ++e)
                        G[e][f + 1] = C00p * G[e][f] + (double)f * B01 * G[e][f - 1] + (double)e * B00 * G[e - 1][f];
                }
            }
            // bra transfer for this lane's (a_k, b_k): h[f] = sum_j C(b,j) AB^(b-j) G[a+j][f]
            double h[LCD + 1];
#pragma unroll
            for (int f = 0; f <= LCD; ++f) h[f] = 0.0;
            double abp = 1.0;
            const int ak = a[k], bk = b[k];
#pragma unroll
            for (int j = LB; j >= 0; --j) {
                // term j contributes when j <= bk: coefficient C(bk, j) AB^(bk-j)
                if (j <= bk) {
                    const double cf = binom(bk, j) * abp;
#pragma unroll
                    for (int e = 0; e <= LA; ++e)
                        if (e == ak) {
#pragma unroll
                            for (int f = 0; f <= LCD; ++f) h[f] += cf * G[e + j][f];
                        }
                    abp *= AB[k];
                }
            }
            // ket HRR on h
            double Kt[LCD + 1][LD + 1];
#pragma unroll
            for (int c = 0; c <= LCD; ++c) Kt[c][0] = h[c];
#pragma unroll
            for (int d = 0; d < LD; ++d)
#pragma unroll
                for (int c = 0; c < LCD - d; ++c) Kt[c][d + 1] = Kt[c + 1][d] + CD[k] * Kt[c][d];
#pragma unroll
            for (int c = 0; c <= LC; ++c)
#pragma unroll
                for (int d = 0; d <= LD; ++d) I[k][c][d] = Kt[c][d];
        }
#pragma unroll
        for (int ic = 0; ic < Q::NC; ++ic)
#pragma unroll
            for (int id = 0; id < Q::ND; ++id)
                acc[ic * Q::ND + id] += I[0][kCart.x[LC][ic]][kCart.x[LD][id]]
                                      * I[1][kCart.y[LC][ic]][kCart.y[LD][id]]
                                      * I[2][kCart.z[LC][ic]][kCart.z[LD][id]];
    }
}

// Team form: the lane owns bra component a (exponents a[3], run-time) and,
// for MODE 1, every b component (NB*NC*ND outputs), for MODE 2 the single b
// component b[3] (NC*ND outputs).  The 2-D recurrences are evaluated per lane;
// the bra transfer uses the closed form I(a,b) = sum_j C(b,j) AB^(b-j) G(a+j).
template <int LA, int LB, int LC, int LD, int MODE, typename R = double>
FK_HD void rys_prim_team(const double *__restrict tab, const PrimPair &p, const PrimPair &q, const double AB[3],
                         const double CD[3], const int a[3], const int b[3], R *__restrict acc)
{
    using Q = QClass<LA, LB, LC, LD>;
    constexpr int LAB = Q::LAB, LCD = Q::LCD;
    constexpr int NBL = (MODE == 1) ? Q::NB : 1;
    QuartetSetup s = quartet_setup(p, q);
    double u[Q::NR], w[Q::NR];
    rys_roots<Q::NR, (Q::L > 0)>(s.T, tab, u, w);
#pragma unroll
    for (int r = 0; r < Q::NR; ++r) {
        const R ur = (Q::L > 0) ? (R)u[r] : (R)0;
        const R B00 = (R)(0.5 * s.inv) * ur;
        const R B10 = (R)p.oo2z * ((R)1 - (R)s.ez * ur);
        const R B01 = (R)q.oo2z * ((R)1 - (R)s.zz * ur);
        R I[3][NBL][LC + 1][LD + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const R C00 = (R)p.PA[k] - (R)(s.ez * s.PQ[k]) * ur;
            const R C00p = (R)q.PA[k] + (R)(s.zz * s.PQ[k]) * ur;
            R G[LAB + 1][LCD + 1];
            G[0][0] = (k == 2) ? (R)(w[r] * s.pref) : (R)1;
            if constexpr (LAB > 0) {
                G[1][0] = C00 * G[0][0];
#pragma unroll
                for (int e = 1; e < LAB; ++e) G[e + 1][0] = C00 * G[e][0] + (R)e * B10 * G[e - 1][0];
            }
            if constexpr (LCD > 0) {
                G[0][1] = C00p * G[0][0];
#pragma unroll
                for (int e = 1; e <= LAB; ++e) G[e][1] = C00p * G[e][0] + (R)e * B00 * G[e - 1][0];
#pragma unroll
                for (int f = 1; f < LCD; ++f) {
                    G[0][f + 1] = C00p * G[0][f] + (R)f * B01 * G[0][f - 1];
#pragma unroll
                    for (int e = 1; e <= LAB; ++e)
                        G[e][f + 1] = C00p * G[e][f] + (R)f * B01 * G[e][f - 1] + (R)e * B00 * G[e - 1][f];
                }
            }
            // rows a_k .. a_k + LB of G for this lane's run-time a_k
            const int ak = a[k];
            R Gs[LB + 1][LCD + 1];
#pragma unroll
            for (int j = 0; j <= LB; ++j)
#pragma unroll
                for (int f = 0; f <= LCD; ++f) {
                    R v = G[j][f];
#pragma unroll
                    for (int e = 1; e <= LA; ++e) v = (ak == e) ? G[e + j][f] : v;
                    Gs[j][f] = v;
                }
            R abp[LB + 1];
            abp[0] = (R)1;
#pragma unroll
            for (int j = 1; j <= LB; ++j) abp[j] = abp[j - 1] * (R)AB[k];
#pragma unroll
            for (int ib = 0; ib < NBL; ++ib) {
                R h[LCD + 1];
                if constexpr (MODE == 1) {
                    constexpr int dummy = 0;
                    (void)dummy;
                    // b exponent of component ib along axis k is a compile-time constant
                    const int bk = (k == 0) ? kCart.x[LB][ib] : (k == 1 ? kCart.y[LB][ib] : kCart.z[LB][ib]);
#pragma unroll
                    for (int f = 0; f <= LCD; ++f) {
                        R v = (R)0;
#pragma unroll
                        for (int j = 0; j <= LB; ++j)
                            if (j <= bk) v += (R)binom(bk, j) * abp[bk - j] * Gs[j][f];
                        h[f] = v;
                    }
                } else {
                    const int bk = b[k];
                    R cf[LB + 1];
#pragma unroll
                    for (int j = 0; j <= LB; ++j) {
                        R c = (R)0;
#pragma unroll
                        for (int bb = 0; bb <= LB; ++bb)
                            if (j <= bb) c = (bk == bb) ? (R)binom(bb, j) * abp[bb - j] : c;
                        cf[j] = c;
                    }
#pragma unroll
                    for (int f = 0; f <= LCD; ++f) {
                        R v = (R)0;
#pragma unroll
                        for (int j = 0; j <= LB; ++j) v += cf[j] * Gs[j][f];
                        h[f] = v;
                    }
                }
                R Kt[LCD + 1][LD + 1];
#pragma unroll
                for (int c = 0; c <= LCD; ++c) Kt[c][0] = h[c];
#pragma unroll
                for (int d = 0; d < LD; ++d)
#pragma unroll
                    for (int c = 0; c < LCD - d; ++c) Kt[c][d + 1] = Kt[c + 1][d] + (R)CD[k] * Kt[c][d];
#pragma unroll
                for (int c = 0; c <= LC; ++c)
#pragma unroll
                    for (int d = 0; d <= LD; ++d) I[k][ib][c][d] = Kt[c][d];
            }
        }
#pragma unroll
        for (int ib = 0; ib < NBL; ++ib)
#pragma unroll
            for (int ic = 0; ic < Q::NC; ++ic)
#pragma unroll
                for (int id = 0; id < Q::ND; ++id)
                    acc[(ib * Q::NC + ic) * Q::ND + id] += I[0][ib][kCart.x[LC][ic]][kCart.x[LD][id]]
                                                         * I[1][ib][kCart.y[LC][ic]][kCart.y[LD][id]]
                                                         * I[2][ib][kCart.z[LC][ic]][kCart.z[LD][id]];
    }
}

// Algorithmic flop count of one primitive quartet of class (LA LB|LC LD) for
// the all-components path (rys_prim_all): FMA = 2, add/mul/sub = 1,
// divide/sqrt = 1 each; root evaluation counted as its Horner steps.
constexpr double flops_prim(int LA, int LB, int LC, int LD)
{
    const int L = LA + LB + LC + LD, NR = L / 2 + 1, LAB = LA + LB, LCD = LC + LD;
    const int NOUT = ncart(LA) * ncart(LB) * ncart(LC) * ncart(LD);
    double f = 0;
    f += 1 + 1 + 1 + 3 + 5 + 3 + 2 + 2;            // zpe, rsqrt, inv, PQ, |PQ|^2, T, pref, ez and zz
    const int nfun = (L > 0) ? 2 * NR : NR;
    f += nfun * RYS_DEG * 2.0 + 4;                 // Horner + interval arithmetic
    if (L == 0) return f + 2;
    f += 6;                                        // ezPQ, zzPQ
    double per_root = 2 + 3 + 3;                   // B00, B10, B01
    for (int k = 0; k < 3; ++k) {
        double v = 4;                              // C00, C00p
        // vertical recurrences (number of grid points built, 2-3 fma-ish ops each)
        if (LAB > 0) v += 1 + (LAB - 1) * 3.0;
        if (LCD > 0) {
            v += 1 + LAB * 3.0;
            v += (LCD - 1) * (3.0 + LAB * 5.0);
        }
        // bra HRR
        for (int b = 0; b < LB; ++b) v += (LAB - b) * (LCD + 1) * 2.0;
        // ket HRR
        double kh = 0;
        for (int d = 0; d < LD; ++d) kh += (LCD - d) * 2.0;
        v += (LA + 1) * (LB + 1) * kh;
        per_root += v;
    }
    per_root += 1 + NOUT * 3.0;                    // weight*pref, assembly (mul + fma)
    return f + NR * per_root;
}

// Digestion flops per contracted quartet: 6 blocks, one FMA per integral each,
// plus the degeneracy scaling.
constexpr double flops_digest(int LA, int LB, int LC, int LD)
{
    const int NOUT = ncart(LA) * ncart(LB) * ncart(LC) * ncart(LD);
    return NOUT * (6 * 2.0 + 1.0);
}

}  // namespace fk
