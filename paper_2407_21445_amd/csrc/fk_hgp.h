// Head-Gordon-Pople evaluation of contracted Cartesian ERIs with early
// contraction (paper, "HGP Recursive Scheme": eqs. vrr1 and vrr2 for the
// vertical recurrences, eq. hrr for the horizontal one; "Integral Class
// Timings" for why highly contracted low-L classes favour it).
//
// Per primitive quartet the vertical recurrences build [e0|f0]^(0) for every
// Cartesian e with la <= |e| <= la+lb and f with lc <= |f| <= lc+ld from the
// auxiliary integrals [00|00]^(m) = U_P U_Q (2/sqrt(pi)) sqrt(rho) F_m(T)
// (reading of the garbled fundamental integral, see the Rys header):
//
//   [e+1_i,0|00]^(m) = PA_i [e|00]^(m) + WP_i [e|00]^(m+1)
//                      + e_i/(2 zeta) ([e-1_i|00]^(m) - rho/zeta [e-1_i|00]^(m+1))
//   [e0|f+1_i,0]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
//                      + f_i/(2 eta) ([e|f-1_i]^(m) - rho/eta [e|f-1_i]^(m+1))
//                      + e_i/(2(zeta+eta)) [e-1_i|f]^(m+1)
//
// with WP = W - P = -eta/(zeta+eta) (P - Q) and WQ = W - Q = +zeta/(zeta+eta)
// (P - Q) (the printed vrr2 has the opposite sign on its PQ term; with
// PQ = P - Q the consistent sign is +).  These are summed over the primitive
// quartets of the contracted quartet ("early contraction"), and only then the
// horizontal recurrences (a,b+1| = (a+1,b| + AB (a,b| and likewise for the ket
// (with CD) turn them into the (ab|cd) block.
//
// F_m(T), m <= L, comes from the n-point Rys rule of the same table the Rys
// engine uses (n = floor(L/2)+1): F_m(T) = sum_i w_i u_i^m holds exactly for
// m < 2n, the defining property of the rule.
#pragma once

#include "fk_eri.h"

namespace fk {

// Cartesian component with exponents (x, y, z), l = x + y + z: its index among
// all components of momentum < l followed by the shell order x^l, x^(l-1)y, ...
constexpr int ncum(int l) { return l * (l + 1) * (l + 2) / 6; }
constexpr int cidx(int x, int y, int z)
{
    const int l = x + y + z;
    return ncum(l) + (l - x) * (l - x + 1) / 2 + (l - x - y);
}

// Exponents of the component with global index g (g < ncum(LMAX + 1)).
struct CompTab {
    int x[165], y[165], z[165];  // momenta 0..8
};
constexpr CompTab make_comp()
{
    CompTab t{};
    int g = 0;
    for (int l = 0; l <= 8; ++l)
        for (int a = l; a >= 0; --a)
            for (int b = l - a; b >= 0; --b) {
                t.x[g] = a; t.y[g] = b; t.z[g] = l - a - b;
                ++g;
            }
    return t;
}
constexpr CompTab kComp = make_comp();

constexpr int comp_e(int g, int k) { return k == 0 ? kComp.x[g] : (k == 1 ? kComp.y[g] : kComp.z[g]); }
// the axis a recurrence lowers for component g (the first with a positive exponent)
constexpr int comp_axis(int g) { return kComp.x[g] > 0 ? 0 : (kComp.y[g] > 0 ? 1 : 2); }
// index of component g lowered by n along axis k (-1 if the exponent is below n)
constexpr int comp_lower(int g, int k, int n)
{
    const int x = kComp.x[g] - (k == 0 ? n : 0), y = kComp.y[g] - (k == 1 ? n : 0), z = kComp.z[g] - (k == 2 ? n : 0);
    return (x < 0 || y < 0 || z < 0) ? -1 : cidx(x, y, z);
}
constexpr int comp_raise(int g, int k)
{
    return cidx(kComp.x[g] + (k == 0), kComp.y[g] + (k == 1), kComp.z[g] + (k == 2));
}

template <int LA, int LB, int LC, int LD>
struct HgpClass {
    static constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD, NR = L / 2 + 1;
    static constexpr int E0 = ncum(LA), E1 = ncum(LAB + 1);   // accumulated e: [E0, E1)
    static constexpr int F0 = ncum(LC), F1 = ncum(LCD + 1);   // accumulated f: [F0, F1)
    static constexpr int NE = E1 - E0, NF = F1 - F0, NACC = NE * NF;
};

// Adds pref-scaled [e0|f0]^(0) of one primitive quartet to acc[(e - E0) NF + f - F0].
template <int LA, int LB, int LC, int LD, typename R = double>
FK_HD void hgp_prim(const double *__restrict tab, const PrimPair &p, const PrimPair &q, R *__restrict acc)
{
    using H = HgpClass<LA, LB, LC, LD>;
    constexpr int L = H::L, LAB = H::LAB, LCD = H::LCD, M = L + 1;
    const QuartetSetup s = quartet_setup(p, q);
    double u[H::NR], w[H::NR];
    rys_roots<H::NR, (L > 0)>(s.T, tab, u, w);
    // [00|00]^(m) = pref F_m(T), F_m = sum_i w_i u_i^m
    R V[ncum(LAB + 1)][ncum(LCD + 1)][M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double f = 0.0;
#pragma unroll
        for (int i = 0; i < H::NR; ++i) {
            double um = 1.0;
#pragma unroll
            for (int k = 0; k < m; ++k) um *= u[i];
            f += w[i] * um;
        }
        V[0][0][m] = (R)(s.pref * f);
    }
    if constexpr (L > 0) {
        R PA[3], WP[3], QC[3], WQ[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            PA[k] = (R)p.PA[k];
            QC[k] = (R)q.PA[k];
            WP[k] = (R)(-s.ez * s.PQ[k]);
            WQ[k] = (R)(s.zz * s.PQ[k]);
        }
        const R o2z = (R)p.oo2z, o2e = (R)q.oo2z, o2ze = (R)(0.5 * s.inv), rz = (R)s.ez, re = (R)s.zz;
        // bra: [e0|00]^(m), |e| = 1..LAB, m <= L - |e|
#pragma unroll
        for (int g = 1; g < ncum(LAB + 1); ++g) {
            const int k = comp_axis(g), g1 = comp_lower(g, k, 1), g2 = comp_lower(g, k, 2);
            const int le = kComp.x[g] + kComp.y[g] + kComp.z[g];
            const R ek = (R)(comp_e(g, k) - 1);
#pragma unroll
            for (int m = 0; m <= L - le; ++m) {
                R v = PA[k] * V[g1][0][m] + WP[k] * V[g1][0][m + 1];
                if (g2 >= 0) v += ek * o2z * (V[g2][0][m] - rz * V[g2][0][m + 1]);
                V[g][0][m] = v;
            }
        }
        // ket: [e0|f0]^(m), |f| = 1..LCD, every |e| <= LAB, m <= L - |e| - |f|
#pragma unroll
        for (int h = 1; h < ncum(LCD + 1); ++h) {
            const int k = comp_axis(h), h1 = comp_lower(h, k, 1), h2 = comp_lower(h, k, 2);
            const int lf = kComp.x[h] + kComp.y[h] + kComp.z[h];
            const R fk_ = (R)(comp_e(h, k) - 1);
#pragma unroll
            for (int g = 0; g < ncum(LAB + 1); ++g) {
                const int le = kComp.x[g] + kComp.y[g] + kComp.z[g];
                const int gl = comp_lower(g, k, 1);
                const R ek = (R)comp_e(g, k);
#pragma unroll
                for (int m = 0; m <= L - le - lf; ++m) {
                    R v = QC[k] * V[g][h1][m] + WQ[k] * V[g][h1][m + 1];
                    if (h2 >= 0) v += fk_ * o2e * (V[g][h2][m] - re * V[g][h2][m + 1]);
                    if (gl >= 0) v += ek * o2ze * V[gl][h1][m + 1];
                    V[g][h][m] = v;
                }
            }
        }
    }
#pragma unroll
    for (int g = H::E0; g < H::E1; ++g)
#pragma unroll
        for (int h = H::F0; h < H::F1; ++h) acc[(g - H::E0) * H::NF + (h - H::F0)] += V[g][h][0];
}

// Horizontal recurrences on the contracted [e0|f0] block: (ab|cd) into
// out[((ia NB + ib) NC + ic) ND + id] in the shells' component order.
template <int LA, int LB, int LC, int LD, typename R = double>
FK_HD void hgp_hrr(const R *__restrict acc, const double AB[3], const double CD[3], R *__restrict out)
{
    using H = HgpClass<LA, LB, LC, LD>;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NE = H::NE, NF = H::NF;
    // bra: X[a][b][f] for |a| = LA.. , |b| = 0..LB; start (e,0|
    // level j holds (a, b) with |b| = j and LA <= |a| <= LAB - j
    R X[ncum(H::LAB + 1)][ncum(LB + 1)][NF];
#pragma unroll
    for (int g = H::E0; g < H::E1; ++g)
#pragma unroll
        for (int f = 0; f < NF; ++f) X[g][0][f] = acc[(g - H::E0) * NF + f];
#pragma unroll
    for (int b = 1; b < ncum(LB + 1); ++b) {
        const int k = comp_axis(b), b1 = comp_lower(b, k, 1);
        const int lb = kComp.x[b] + kComp.y[b] + kComp.z[b];
#pragma unroll
        for (int a = ncum(LA); a < ncum(H::LAB + 1 - lb); ++a) {
            const int a1 = comp_raise(a, k);
#pragma unroll
            for (int f = 0; f < NF; ++f) X[a][b][f] = X[a1][b1][f] + (R)AB[k] * X[a][b1][f];
        }
    }
    // ket, for every (a, b) of the shells
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            const int a = ncum(LA) + ia, b = ncum(LB) + ib;
            R Y[ncum(H::LCD + 1)][ncum(LD + 1)];
#pragma unroll
            for (int f = H::F0; f < H::F1; ++f) Y[f][0] = X[a][b][f - H::F0];
#pragma unroll
            for (int d = 1; d < ncum(LD + 1); ++d) {
                const int k = comp_axis(d), d1 = comp_lower(d, k, 1);
                const int ld = kComp.x[d] + kComp.y[d] + kComp.z[d];
#pragma unroll
                for (int c = ncum(LC); c < ncum(H::LCD + 1 - ld); ++c) {
                    const int c1 = comp_raise(c, k);
                    Y[c][d] = Y[c1][d1] + (R)CD[k] * Y[c][d1];
                }
            }
#pragma unroll
            for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                for (int id = 0; id < ND; ++id)
                    out[((ia * NB + ib) * NC + ic) * ND + id] = Y[ncum(LC) + ic][ncum(LD) + id];
        }
}

// Algorithmic flops of hgp_prim for one primitive quartet (FMA = 2): set-up
// and roots as for the Rys engine, the moments F_m, the recurrences as
// written above and the accumulation.
constexpr double hgp_flops_prim(int LA, int LB, int LC, int LD)
{
    const int L = LA + LB + LC + LD, NR = L / 2 + 1, LAB = LA + LB, LCD = LC + LD;
    double f = 1 + 1 + 1 + 3 + 5 + 3 + 2 + 2;           // set-up as quartet_setup
    const int nfun = (L > 0) ? 2 * NR : NR;
    f += nfun * RYS_DEG * 2.0 + 4;                       // roots and weights
    for (int m = 0; m <= L; ++m) f += NR * (m + 2) + 1;  // F_m and pref F_m
    if (L == 0) return f + 1;
    f += 6;                                              // WP, WQ
    for (int g = 1; g < ncum(LAB + 1); ++g) {
        const int le = kComp.x[g] + kComp.y[g] + kComp.z[g];
        const int k = comp_axis(g);
        const bool two = comp_lower(g, k, 2) >= 0;
        f += (L - le + 1) * (two ? 7.0 : 3.0);
    }
    for (int h = 1; h < ncum(LCD + 1); ++h) {
        const int lf = kComp.x[h] + kComp.y[h] + kComp.z[h];
        const int k = comp_axis(h);
        const bool two = comp_lower(h, k, 2) >= 0;
        for (int g = 0; g < ncum(LAB + 1); ++g) {
            const int le = kComp.x[g] + kComp.y[g] + kComp.z[g];
            if (L - le - lf < 0) continue;
            const bool lo = comp_lower(g, k, 1) >= 0;
            f += (L - le - lf + 1) * (3.0 + (two ? 4.0 : 0.0) + (lo ? 3.0 : 0.0));
        }
    }
    return f + (ncum(LAB + 1) - ncum(LA)) * (ncum(LCD + 1) - ncum(LC));
}

// Flops of hgp_hrr per contracted quartet.
constexpr double hgp_flops_hrr(int LA, int LB, int LC, int LD)
{
    const int LAB = LA + LB, LCD = LC + LD;
    const int NF = ncum(LCD + 1) - ncum(LC);
    double f = 0;
    for (int b = 1; b < ncum(LB + 1); ++b) {
        const int lb = kComp.x[b] + kComp.y[b] + kComp.z[b];
        f += 2.0 * NF * (ncum(LAB + 1 - lb) - ncum(LA));
    }
    double fk = 0;
    for (int d = 1; d < ncum(LD + 1); ++d) {
        const int ld = kComp.x[d] + kComp.y[d] + kComp.z[d];
        fk += 2.0 * (ncum(LCD + 1 - ld) - ncum(LC));
    }
    return f + ncart(LA) * ncart(LB) * fk;
}

}  // namespace fk
