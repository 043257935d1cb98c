// McMurchie-Davidson pieces of the J engine (paper, "MMD Recursive Scheme"
// and "J matrix implementation").
//
// A primitive pair's product of Cartesian Gaussians is expanded in Hermite
// Gaussians of the pair (eqs. EabP def1-3): per axis
//
//   E^{i+1,j}_t = E^{ij}_{t-1} / (2 zeta) + PA E^{ij}_t + (t+1) E^{ij}_{t+1},
//   E^{i,j+1}_t = E^{ij}_{t-1} / (2 zeta) + PB E^{ij}_t + (t+1) E^{ij}_{t+1},
//   E^{00}_0 = 1,
//
// (the Gaussian product factor exp(-mu AB^2) sits in the pair prefactor U_P),
// and E^{ab}_{tuv} = E^{ax bx}_t E^{ay by}_u E^{az bz}_v.  A primitive
// integral is then
//
//   [ab|cd] = sum_{tuv} sum_{t'u'v'} E^{ab}_{tuv} (-1)^{t'+u'+v'} R_{t+t',u+u',v+v'} E^{cd}_{t'u'v'}
//
// with the Hermite integrals R_{tuv} = d^t/dX^t d^u/dY^u d^v/dZ^v of
// U_P U_Q (2/sqrt(pi)) sqrt(rho) F_0(rho |PQ|^2), X, Y, Z the components of
// PQ = P - Q (the paper's R recursion with R_{0,m} as read in the Rys
// header).  Here they come from the same n-point Rys rule the Rys engine uses
// (n = floor(L/2) + 1): F_0(T) = int_0^1 exp(-T t^2) dt and the t-derivatives
// of exp(-a X^2), a = rho u, u = t^2, are g_t(X) exp(-a X^2) with
//
//   g_0 = 1,  g_1 = -2 a X,  g_{t+1} = -2 a (X g_t + t g_{t-1}),
//
// so R_{tuv} = U_P U_Q (2/sqrt(pi)) sqrt(rho) sum_r w_r g_t(X) g_u(Y) g_v(Z)
// at a = rho u_r: each product is a polynomial of degree t+u+v <= L in u,
// which the rule integrates exactly (degree < 2n).
#pragma once

#include "fk_eri.h"
#include "fk_hgp.h"

namespace fk {

// Hermite functions with total order up to L: index cidx(t, u, v).
constexpr int nherm(int L) { return ncum(L + 1); }

// 1-D expansion coefficients E[i][j][t], i <= I, j <= J, t <= i + j, of one axis.
template <int I, int J>
FK_HD void mmd_e1(double oo2z, double PA, double PB, double (&E)[I + 1][J + 1][I + J + 1])
{
#pragma unroll
    for (int i = 0; i <= I; ++i)
#pragma unroll
        for (int j = 0; j <= J; ++j)
#pragma unroll
            for (int t = 0; t <= I + J; ++t) E[i][j][t] = 0.0;
    E[0][0][0] = 1.0;
#pragma unroll
    for (int i = 0; i < I; ++i)
#pragma unroll
        for (int t = 0; t <= i + 1; ++t) {
            double v = PA * E[i][0][t];
            if (t > 0) v += oo2z * E[i][0][t - 1];
            if (t + 1 <= i) v += (t + 1) * E[i][0][t + 1];
            E[i + 1][0][t] = v;
        }
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int i = 0; i <= I; ++i)
#pragma unroll
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = PB * E[i][j][t];
                if (t > 0) v += oo2z * E[i][j][t - 1];
                if (t + 1 <= i + j) v += (t + 1) * E[i][j][t + 1];
                E[i][j + 1][t] = v;
            }
}

// Hermite integrals R[cidx(t, u, v)], t + u + v <= L, of one primitive quartet.
template <int L>
FK_HD void mmd_r(const double *__restrict tab, const QuartetSetup &s, double rho, double *__restrict R)
{
    constexpr int NR = L / 2 + 1;
    double u[NR], w[NR];
    rys_roots<NR, (L > 0)>(s.T, tab, u, w);
#pragma unroll
    for (int k = 0; k < nherm(L); ++k) R[k] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const double wk = s.pref * w[r];
        if constexpr (L == 0) {
            R[0] += wk;
        } else {
            const double a2 = -2.0 * rho * u[r];
            double g[3][L + 1];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                g[k][0] = 1.0;
                g[k][1] = a2 * s.PQ[k];
#pragma unroll
                for (int t = 1; t < L; ++t) g[k][t + 1] = a2 * (s.PQ[k] * g[k][t] + t * g[k][t - 1]);
            }
#pragma unroll
            for (int k = 0; k < nherm(L); ++k) R[k] += wk * g[0][kComp.x[k]] * g[1][kComp.y[k]] * g[2][kComp.z[k]];
        }
    }
}

// All Cartesian components of the primitive quartet [ab|cd] by the Hermite
// expansion, added to acc[((ia NB + ib) NC + ic) ND + id] (host checks of the
// E and R pieces against the oracle; the J engine never forms integrals).
template <int LA, int LB, int LC, int LD>
FK_HD void mmd_prim_all(const double *__restrict tab, const PrimPair &p, const PrimPair &q, const double AB[3],
                        const double CD[3], double *__restrict acc)
{
    constexpr int L = LA + LB + LC + LD, LP = LA + LB, LQ = LC + LD;
    const QuartetSetup s = quartet_setup(p, q);
    double R[nherm(L)];
    mmd_r<L>(tab, s, p.zeta * q.zeta * s.inv, R);
    double Eb[3][LA + 1][LB + 1][LP + 1], Ek[3][LC + 1][LD + 1][LQ + 1];
    for (int k = 0; k < 3; ++k) {
        mmd_e1<LA, LB>(p.oo2z, p.PA[k], p.PA[k] + AB[k], Eb[k]);
        mmd_e1<LC, LD>(q.oo2z, q.PA[k], q.PA[k] + CD[k], Ek[k]);
    }
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    for (int ia = 0; ia < NA; ++ia)
        for (int ib = 0; ib < NB; ++ib)
            for (int ic = 0; ic < NC; ++ic)
                for (int id = 0; id < ND; ++id) {
                    const int ax[3] = {kCart.x[LA][ia], kCart.y[LA][ia], kCart.z[LA][ia]};
                    const int bx[3] = {kCart.x[LB][ib], kCart.y[LB][ib], kCart.z[LB][ib]};
                    const int cx[3] = {kCart.x[LC][ic], kCart.y[LC][ic], kCart.z[LC][ic]};
                    const int dx[3] = {kCart.x[LD][id], kCart.y[LD][id], kCart.z[LD][id]};
                    double v = 0.0;
                    for (int t = 0; t <= ax[0] + bx[0]; ++t)
                        for (int uu = 0; uu <= ax[1] + bx[1]; ++uu)
                            for (int vv = 0; vv <= ax[2] + bx[2]; ++vv) {
                                const double eb = Eb[0][ax[0]][bx[0]][t] * Eb[1][ax[1]][bx[1]][uu] * Eb[2][ax[2]][bx[2]][vv];
                                for (int t2 = 0; t2 <= cx[0] + dx[0]; ++t2)
                                    for (int u2 = 0; u2 <= cx[1] + dx[1]; ++u2)
                                        for (int v2 = 0; v2 <= cx[2] + dx[2]; ++v2) {
                                            const double ek = Ek[0][cx[0]][dx[0]][t2] * Ek[1][cx[1]][dx[1]][u2] *
                                                              Ek[2][cx[2]][dx[2]][v2];
                                            const double sg = ((t2 + u2 + v2) & 1) ? -1.0 : 1.0;
                                            v += eb * ek * sg * R[cidx(t + t2, uu + u2, vv + v2)];
                                        }
                            }
                    acc[((ia * NB + ib) * NC + ic) * ND + id] += v;
                }
}

}  // namespace fk
