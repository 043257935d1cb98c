// HIP kernels of the J/K build for gfx950 (CDNA4, wave64).
//
// Hot path (per Fock build):
//   k_prep_*   density preprocessing: component-scaled D and the shell-block
//              maxima D_sh used by the per-quartet density screen;
//   k_jk_lpq   lane-per-quartet Rys ERI + fused 8-fold digestion for classes
//              whose whole output block fits in registers;
//   k_jk_wpq   wave-per-quartet variant for large classes: lanes own bra
//              Cartesian components;
//   k_finalize J = X_J + X_J^T, K = X_K + X_K^T with component scaling.
//
// Digestion (paper: six Fock blocks per quartet, atomics after partial
// pre-digestion; the degeneracy factors are not printed and are derived from
// J and K's definitions): with v = (ab|cd) and s = 1/2 per coincidence among
// a = b, c = d, ab = cd (shell level),
//   X_J[a,b] += 2 s v D_cd,  X_J[c,d] += 2 s v D_ab,
//   X_K[a,c] += s v D_bd,    X_K[a,d] += s v D_bc,
//   X_K[b,c] += s v D_ad,    X_K[b,d] += s v D_ac,
// and J = X_J + X_J^T, K = X_K + X_K^T.
#include <hip/hip_runtime.h>

#include "fk_internal.h"
#include "fk_eri.h"
#include "fk_hgp.h"
#include "fk_mmd.h"

#ifndef FK_BUILD_MAXL
#define FK_BUILD_MAXL 3
#endif
// lane-per-quartet classes have at most this many integrals per lane.  Above
// it a team of lanes shares a quartet: (pp|pp) with 81 integrals spilled 292
// bytes per lane as a lane class and runs in less than half the time with
// three lanes per quartet; (fs|ds) and (fd|ss) with 60 held one wave per SIMD
// and run 4.4 and 1.4 times faster with ten lanes per quartet (two waves)
#define FK_LPQ_MAX_NOUT 54
// team classes keep at most this many integrals per lane (MODE 1: NB NC ND,
// MODE 2: NC ND); larger ones take a whole wave per quartet
#define FK_TEAM_MAX_NOUT 80
// lane-per-quartet classes with at least this many integrals (and a bra shell
// of three or more components) also have a team-per-quartet kernel, one lane
// per component of the first bra shell, which the schedule may choose
#define FK_ALT_MIN_NOUT 18
// lane-per-quartet classes up to this many integrals sum K[a,c], K[a,d] and
// J[c,d] over a block of bras in registers; larger ones take one bra per tile
#define FK_LPQ_BLOCK_NOUT 54
// lane-per-quartet classes up to this many integrals evaluate two primitive
// quartets per step of the bra-primitive loop
#define FK_LPQ_PAIR_NOUT 9
#define FK_BLOCK 256
#define FK_WAVES (FK_BLOCK / 64)

namespace {

constexpr int pair_la(int P) { return P == 0 ? 0 : (P <= 2 ? 1 : (P <= 5 ? 2 : 3)); }
constexpr int pair_lb(int P) { return P - pair_la(P) * (pair_la(P) + 1) / 2; }

// Kernel kind per class: 0 lane per quartet, 1 team over bra a components,
// 2 team over bra (a, b) component pairs, 3 wave per quartet.
template <int LA, int LB, int LC, int LD>
constexpr int kernel_kind()
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    if (Q::NOUT <= FK_LPQ_MAX_NOUT) return 0;
    if (Q::NB * Q::NC * Q::ND <= FK_TEAM_MAX_NOUT) return 1;
    if (Q::NA * Q::NB <= 64 && Q::NC * Q::ND <= FK_TEAM_MAX_NOUT) return 2;
    return 3;
}

__device__ __forceinline__ fk::PrimPair load_pp(const double *__restrict pp, int idx)
{
    const double *r = pp + (size_t)idx * FK_NPP_REC;
    fk::PrimPair p;
    p.zeta = r[0];
    p.oo2z = r[1];
    p.P[0] = r[2]; p.P[1] = r[3]; p.P[2] = r[4];
    p.PA[0] = r[5]; p.PA[1] = r[6]; p.PA[2] = r[7];
    p.K = r[8];
    return p;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void lds_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// FP64 atomic adds to device memory are served one 32-byte sector request per
// lane unless lanes of the same instruction address the same sector (measured
// on MI355X: 2.4e10 scattered adds/s, 9.4e10 when four lanes share a sector).
// flush_block therefore issues a lane's R x C block of values, which lies in
// rows row..row+R-1 and the C consecutive columns col..col+C-1 of X (stride n),
// with G = C rounded up to a power of two consecutive lanes adding the C
// doubles of one row of one lane: 64/G lanes' rows per instruction instead of
// one double per lane.  The values pass through the wave's LDS stage
// ([R C][64] doubles); zeros (inactive lanes, absent contributions) are not
// added.  All 64 lanes must call it (wave-uniform control flow).
template <int R, int C>
__device__ __forceinline__ void flush_block(double *X, int n, int row, int col, const double *v, double *stage,
                                            int lane)
{
    if constexpr (C == 1) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v[r] != 0.0) atomic_add(&X[(size_t)(row + r) * n + col], v[r]);
    } else {
        constexpr int G = C <= 2 ? 2 : (C <= 4 ? 4 : (C <= 8 ? 8 : 16));
        constexpr int OWN = 64 / G;
        wave_sync_lds();
#pragma unroll
        for (int x = 0; x < R * C; ++x) stage[x * 64 + lane] = v[x];
        wave_sync_lds();
        const int q = lane % G, sub = lane / G;
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int k = t * OWN + sub;
            const int rk = __shfl(row, k, 64), ck = __shfl(col, k, 64);
            if (q < C) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double val = stage[(r * C + q) * 64 + k];
                    if (val != 0.0) atomic_add(&X[(size_t)(rk + r) * n + ck + q], val);
                }
            }
        }
    }
}

// Adds the block B[i][j] (i < NI components of shell row_i, j < NJ of shell
// col_j, per lane) to X[oi + i][oj + j], or -- when the accumulator is later
// symmetrised and NI > NJ -- to X[oj + j][oi + i], whichever puts the larger
// component count in the contiguous dimension.
template <int NI, int NJ>
__device__ __forceinline__ void flush_sym(double *X, int n, int oi, int oj, const double *B, double *stage, int lane)
{
    if constexpr (NJ >= NI) {
        flush_block<NI, NJ>(X, n, oi, oj, B, stage, lane);
    } else {
        double T[NI * NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) T[j * NI + i] = B[i * NJ + j];
        flush_block<NJ, NI>(X, n, oj, oi, T, stage, lane);
    }
}

template <int NR>
__device__ __forceinline__ void load_table(double *s_tab, const double *__restrict g)
{
    constexpr int TABN = rys_lds_size(NR);
    for (int i = threadIdx.x; i < TABN; i += blockDim.x) s_tab[i] = g[i];
    __syncthreads();
}

// Density factor of the quartet screen: the largest |D| over the shell blocks
// the quartet's contributions are multiplied by -- ab and cd for J, ac, ad, bc,
// bd for K, all six when both are built (want: bit 0 J, bit 1 K).
__device__ __forceinline__ double dmax_want(const double *__restrict Dsh, int ns, int sa, int sb, int sc, int sd,
                                            int want)
{
    double m = 0.0;
    if (want & FK_WANT_J) m = fmax(Dsh[sa * ns + sb], Dsh[sc * ns + sd]);
    if (want & FK_WANT_K) {
        const double m2 = fmax(Dsh[sa * ns + sc], Dsh[sa * ns + sd]);
        const double m3 = fmax(Dsh[sb * ns + sc], Dsh[sb * ns + sd]);
        m = fmax(m, fmax(m2, m3));
    }
    return m;
}

// K-block skip (paper, "K matrix implementation"): with |D_cd| <= H
// exp(-Lambda |CD|), R_x the largest distance from shell x to a partner of a
// Schwarz-significant pair and G_x its largest pair factor, every contribution
// to block K_xy is at most H exp(-Lambda max(0, |XY| - R_x - R_y)) G_x G_y.
__device__ __forceinline__ bool kblock_live(const FkJKArgs &a, int x, int y)
{
    const double *X = a.ks_shell + 5 * x, *Y = a.ks_shell + 5 * y;
    const double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
    const double d = fmax(0.0, sqrt(dx * dx + dy * dy + dz * dz) - X[3] - Y[3]);
    return a.ks_fit[0] * exp(-a.ks_fit[1] * d) * X[4] * Y[4] > a.ks_tau;
}

// Density factor of a K-only launch with the block skip: the density block of
// each K target counts only while that target block is live (K_ac takes D_bd,
// K_ad D_bc, K_bc D_ad, K_bd D_ac).  A quartet none of whose blocks is live
// gets factor 0.
__device__ __forceinline__ double dmax_kskip(const FkJKArgs &a, const double *__restrict Dsh, int ns, int sa, int sb,
                                             int sc, int sd)
{
    double m = 0.0;
    if (kblock_live(a, sa, sc)) m = fmax(m, Dsh[sb * ns + sd]);
    if (kblock_live(a, sa, sd)) m = fmax(m, Dsh[sb * ns + sc]);
    if (kblock_live(a, sb, sc)) m = fmax(m, Dsh[sa * ns + sd]);
    if (kblock_live(a, sb, sd)) m = fmax(m, Dsh[sa * ns + sc]);
    return m;
}

__device__ __forceinline__ double dmax_args(const FkJKArgs &a, const double *__restrict Dsh, int ns, int sa, int sb,
                                            int sc, int sd)
{
    if (a.ks_shell && a.want == FK_WANT_K) return dmax_kskip(a, Dsh, ns, sa, sb, sc, sd);
    return dmax_want(Dsh, ns, sa, sb, sc, sd, a.want);
}

// Screening of the (bra, ket) combinations of a wave and the precision split.
// A lane's quartet survives the Schwarz bound, the same-class triangle and the
// density screen G_ab G_cd D_max >= tau.  With the split (tau_fp32 > 0) the
// wave's surviving quartets of this bra go to the FP32 launch when every one
// has G_ab G_cd D_max < tau_fp32, else to the FP64 launch: both launches reach
// the same decision, so each quartet is computed once.  Returns the lanes this
// launch computes.
template <typename R>
__device__ __forceinline__ bool screen_lane(const FkJKArgs &a, bool cand, double gg, const double *__restrict Dsh,
                                            int ns, int sa, int sb, int sc, int sd)
{
    bool active = cand && (a.tau <= 0 || gg >= a.tau);
    double dm = 0.0;
    if (a.dscreen || a.tau_fp32 > 0) dm = dmax_args(a, Dsh, ns, sa, sb, sc, sd);
    if (a.dscreen) active = active && gg * dm >= a.tau;
    if (a.tau_fp32 > 0) {
        const bool need64 = __ballot(active && gg * dm >= a.tau_fp32) != 0ull;
        const bool mine = (sizeof(R) == sizeof(double)) ? need64 : !need64;
        active = active && mine;
    }
    return active;
}

// Ket pair data at a list position (consecutive lanes: consecutive positions).
struct KetInfo {
    int sc, sd;
    double CD[3], G;
};
__device__ __forceinline__ KetInfo load_ket(const FkJKArgs &a, int pos)
{
    KetInfo k;
    k.sc = a.lst_sa[pos];
    k.sd = a.lst_sb[pos];
    k.CD[0] = a.lst_CD[pos];
    k.CD[1] = a.lst_CD[a.nlist + pos];
    k.CD[2] = a.lst_CD[2 * a.nlist + pos];
    k.G = a.lst_G[pos];
    return k;
}

// Primitive pair j of the ket at position r of a group (transposed records).
__device__ __forceinline__ fk::PrimPair load_ket_pp(const double *__restrict ppT, const FkGroup &g, int j, int r)
{
    const double *q = ppT + g.base + (size_t)j * FK_NFLD * g.len + r;
    const int L = g.len;
    fk::PrimPair p;
    p.zeta = q[0];
    p.oo2z = q[L];
    p.P[0] = q[2 * L]; p.P[1] = q[3 * L]; p.P[2] = q[4 * L];
    p.PA[0] = q[5 * L]; p.PA[1] = q[6 * L]; p.PA[2] = q[7 * L];
    p.K = q[8 * L];
    return p;
}

struct BraInfo {
    int sa, sb, ppo, npp;
    double AB[3], G;
};
__device__ __forceinline__ BraInfo load_bra(const FkJKArgs &a, int bra)
{
    BraInfo b;
    b.sa = a.pair_sa[bra];
    b.sb = a.pair_sb[bra];
    b.ppo = a.pair_ppoff[bra];
    b.npp = a.pair_npp[bra];
    b.AB[0] = a.pair_AB[3 * bra];
    b.AB[1] = a.pair_AB[3 * bra + 1];
    b.AB[2] = a.pair_AB[3 * bra + 2];
    b.G = a.pair_G[bra];
    return b;
}

// The bra's primitive records are the same for every lane of the wave: they
// are read through the constant address space, which the compiler serves with
// scalar loads into SGPRs (no LDS traffic and no VGPRs for them; the records
// are not written while the kernels run).  `idx` must be wave-uniform.
typedef const __attribute__((address_space(4))) double *fk_const_ptr;
__device__ __forceinline__ fk::PrimPair sload_pp(const double *__restrict pp, int idx)
{
    const fk_const_ptr r = (fk_const_ptr)(pp + (size_t)idx * FK_NPP_REC);
    fk::PrimPair p;
    p.zeta = r[0];
    p.oo2z = r[1];
    p.P[0] = r[2]; p.P[1] = r[3]; p.P[2] = r[4];
    p.PA[0] = r[5]; p.PA[1] = r[6]; p.PA[2] = r[7];
    p.K = r[8];
    return p;
}

// position of the n-th set bit of m (n = 0 is the lowest), or -1
__device__ __forceinline__ int nth_bit(unsigned long long m, int n)
{
    for (int k = 0; k < n && m; ++k) m &= m - 1;
    return m ? __ffsll((long long)m) - 1 : -1;
}


// Digestion of one bra's contracted quartets with the lane's ket (paper,
// "Optimised GPU Implementation": the six Fock blocks of a quartet): scales the
// integrals by the coincidence factors, forms X_J[a, b] (reduced over the wave
// and added here) and the per-bra X_K[b, c], X_K[b, d] (flushed here), and adds
// to the block sums X_K[a, c], X_K[a, d], X_J[c, d] of the caller.  Every lane
// of the wave calls it (the flushes and the reduction are wave operations);
// `active` marks the lanes whose quartet is computed.  With kr_b (block
// tasks) the per-bra sums go to the workgroup's LDS rows instead of memory:
// X_K[b, x] to kr_b[ib * ncol + x] (x = colc + ic for c, cold + id for d) and
// the wave's X_J[a, b] to kr_jab.
template <int LA, int LB, int LC, int LD, typename R>
__device__ __forceinline__ void lpq_digest(R *acc, bool active, bool diag, int sa, int sb, int sc, int sd, int oa,
                                           int ob, int oc, int od, int n, const double *__restrict Ds,
                                           const double *dcd, double *kac, double *kad, double *jcd, double *XJ,
                                           double *XK, double *s_stage, int lane, bool wj, bool wk, bool &any,
                                           double *kr_b = nullptr, int ncol = 0, int colc = 0, int cold = 0,
                                           double *kr_jab = nullptr)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    constexpr int NA = Q::NA, NB = Q::NB, NC = Q::NC, ND = Q::ND, NOUT = Q::NOUT;
    const double fac = (sa == sb ? 0.5 : 1.0) * (sc == sd ? 0.5 : 1.0) * (diag ? 0.5 : 1.0);
    double jab[NA * NB];
#pragma unroll
    for (int o = 0; o < NA * NB; ++o) jab[o] = 0.0;
    if (active) {
        any = true;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) acc[o] *= (R)fac;
    }
    if (active && wj) {
        double dab[NA * NB];
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) dab[ia * NB + ib] = Ds[(size_t)(oa + ia) * n + ob + ib];
        // X_J[a, b] partial (reduced over the wave below); X_J[c, d] block sum
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab)
#pragma unroll
            for (int cd = 0; cd < NC * ND; ++cd) {
                jab[ab] += acc[ab * NC * ND + cd] * dcd[cd];
                jcd[cd] += acc[ab * NC * ND + cd] * dab[ab];
            }
    }
    double kbc[NB * NC], kbd[NB * ND];
#pragma unroll
    for (int o = 0; o < NB * NC; ++o) kbc[o] = 0.0;
#pragma unroll
    for (int o = 0; o < NB * ND; ++o) kbd[o] = 0.0;
    if (active && wk) {
        double dbc[NB * NC], dbd[NB * ND];
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) dbc[ib * NC + ic] = Ds[(size_t)(ob + ib) * n + oc + ic];
#pragma unroll
            for (int id = 0; id < ND; ++id) dbd[ib * ND + id] = Ds[(size_t)(ob + ib) * n + od + id];
        }
        // X_K[a, c] += v D_bd and X_K[a, d] += v D_bc (block sums)
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                    for (int id = 0; id < ND; ++id) {
                        const double v = acc[((ia * NB + ib) * NC + ic) * ND + id];
                        kac[ia * NC + ic] += v * dbd[ib * ND + id];
                        kad[ia * ND + id] += v * dbc[ib * NC + ic];
                    }
        // X_K[b, c] += v D_ad and X_K[b, d] += v D_ac (per bra)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) {
                double s = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int id = 0; id < ND; ++id)
                        s += acc[((ia * NB + ib) * NC + ic) * ND + id] * Ds[(size_t)(oa + ia) * n + od + id];
                kbc[ib * NC + ic] = s;
            }
#pragma unroll
            for (int id = 0; id < ND; ++id) {
                double s = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic)
                        s += acc[((ia * NB + ib) * NC + ic) * ND + id] * Ds[(size_t)(oa + ia) * n + oc + ic];
                kbd[ib * ND + id] = s;
            }
        }
    }
    if (wk) {
        if (kr_b) {
            if (active) {
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic) lds_add(&kr_b[ib * ncol + colc + ic], kbc[ib * NC + ic]);
#pragma unroll
                    for (int id = 0; id < ND; ++id) lds_add(&kr_b[ib * ncol + cold + id], kbd[ib * ND + id]);
                }
            }
        } else {
            flush_sym<NB, NC>(XK, n, ob, oc, kbc, s_stage, lane);
            flush_sym<NB, ND>(XK, n, ob, od, kbd, s_stage, lane);
        }
    }
    // all lanes (active or not) take part in the wave reduction of X_J[a, b]
    if (wj) {
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) {
            const double s = wave_sum(jab[ab]);
            if (lane == 0) {
                if (kr_jab) lds_add(&kr_jab[ab], 2.0 * s);
                else atomic_add(&XJ[(size_t)(oa + ab / NB) * n + ob + ab % NB], 2.0 * s);
            }
        }
    }
}

// ---------------------------------------------------------------- lpq ----
// One wave per tile: a block of bras (a, b_j) sharing the first shell a, and up
// to 64 kets.  Lane i holds ket i and computes the contracted quartets
// (a b_j | c_i d_i) for every bra of the block in turn: ket primitives outer
// (one coalesced load per primitive), bra primitives inner (LDS broadcast).
// Digestion: X_J[a, b_j] is reduced over the wave per bra; X_K[b_j, c],
// X_K[b_j, d] go to memory per bra; X_K[a, c], X_K[a, d] and X_J[c, d] do not
// depend on b_j and are summed in registers over the whole block first.
// Waves per SIMD the compiler must fit in registers (one workgroup of four
// waves places one per SIMD).  Five lane-per-quartet classes run faster at two
// waves per SIMD with some bytes spilled per lane than at one wave without
// spills (their register demand is just above half of the file); the others
// keep the compiler's own choice (measured: C20H42, (fs|ss) on the organic
// batch).  (ps|ss) at three waves
// spilled 124 bytes per lane, doubled its HBM traffic and gained nothing.
template <int LA, int LB, int LC, int LD>
struct LpqMinBlocks {
    static constexpr int value = 1;
};
template <>
struct LpqMinBlocks<0, 0, 0, 0> {
    static constexpr int value = 4;
};
template <>
struct LpqMinBlocks<2, 0, 0, 0> {
    static constexpr int value = 2;
};
template <>
struct LpqMinBlocks<1, 0, 1, 0> {
    static constexpr int value = 2;
};
template <>
struct LpqMinBlocks<2, 0, 1, 0> {
    static constexpr int value = 2;
};
template <>
struct LpqMinBlocks<1, 1, 1, 0> {
    static constexpr int value = 2;
};
template <>
struct LpqMinBlocks<2, 1, 0, 0> {
    static constexpr int value = 2;
};
template <>
struct LpqMinBlocks<3, 0, 0, 0> {
    static constexpr int value = 2;
};

// Bra block of the ket-outer loop order (0: bra-outer).  With the bras of a
// tile outer, each bra re-reads the tile's ket primitive records; the 64 kets'
// records of a wave (up to ~90 KB) do not survive in L2 while hundreds of
// waves per XCD stream theirs, so every bra fetches them again from memory.
// Ket-outer, each ket primitive record is read once per tile and applied to
// every bra of the block, whose contracted integrals stay in registers (NBK x
// NOUT accumulators per lane).  Measured on (H2O)64 cc-pVDZ-type: (ps|ss)
// 47.0 -> 41.7 ms with blocks of 8 (its registers also drop to three waves per
// SIMD); 16 bras cost (ps|ss) a wave per SIMD (51.8 ms); (ps|ps) and (pp|ss)
// lose with any block (32.8 -> 36.3 ms at 4 bras, 47.4 ms at 2).  With block
// tasks (the K rows of a block summed in LDS) four bras win: (ps|ss) takes
// 37.4 ms at 4 (163 VGPRs, three waves per SIMD) against 46.6 ms at 8 (188
// VGPRs, two waves; 49.1 and 45.2 ms without block tasks); (ss|ss) (HGP)
// 19.7 ms at 4 with block tasks (four workgroups per CU fit their LDS)
// against 23.2 ms at 8, where the rows would halve the workgroups per CU.
template <int LA, int LB, int LC, int LD>
struct LpqKetOuter {
    static constexpr int value = 0;
};
template <>
struct LpqKetOuter<0, 0, 0, 0> {
    static constexpr int value = 4;
};
template <>
struct LpqKetOuter<1, 0, 0, 0> {
    static constexpr int value = 4;
};

// Doubles per wave of the lane kernel's LDS stage for flush_block: the largest
// block a lane flushes (K[b,c], K[b,d], K[a,c], K[a,d], J[c,d]) times 64.
template <int LA, int LB, int LC, int LD>
struct LpqStage {
    using Q = fk::QClass<LA, LB, LC, LD>;
    static constexpr int m1 = Q::NB * Q::NC > Q::NB * Q::ND ? Q::NB * Q::NC : Q::NB * Q::ND;
    static constexpr int m2 = Q::NA * Q::NC > Q::NA * Q::ND ? Q::NA * Q::NC : Q::NA * Q::ND;
    static constexpr int m3 = m1 > m2 ? m1 : m2;
    static constexpr int value = 64 * (m3 > Q::NC * Q::ND ? m3 : Q::NC * Q::ND);
};

// Doubles per wave of the stage with block tasks, where the K sums go to the
// LDS rows and only X_J[c, d] passes through the stage (flush_sym<NC, ND>
// uses it for blocks wider than one element)
template <int LA, int LB, int LC, int LD>
struct LpqStageTask {
    using Q = fk::QClass<LA, LB, LC, LD>;
    static constexpr int value = (Q::NC > 1 || Q::ND > 1) ? 64 * Q::NC * Q::ND : 0;
};

// Bra-outer lane classes built also with workgroups of eight waves: one Rys
// table (2 or 3 roots: 34-50 KB of LDS) then serves eight waves, which leaves
// room for the K rows of block tasks at the occupancy the registers allow
// (two waves per SIMD: one workgroup of eight waves per CU)
template <int LA, int LB, int LC, int LD>
struct LpqWide {
    static constexpr bool value = false;
};
template <> struct LpqWide<1, 0, 1, 0> { static constexpr bool value = true; };
template <> struct LpqWide<1, 1, 0, 0> { static constexpr bool value = true; };
template <> struct LpqWide<1, 1, 1, 0> { static constexpr bool value = true; };
template <> struct LpqWide<2, 0, 0, 0> { static constexpr bool value = true; };
template <> struct LpqWide<2, 0, 1, 0> { static constexpr bool value = true; };
template <> struct LpqWide<2, 1, 0, 0> { static constexpr bool value = true; };
template <> struct LpqWide<2, 1, 1, 0> { static constexpr bool value = true; };

// workgroups per CU the launch bounds ask for with NW waves per workgroup (the
// same waves per SIMD as LpqMinBlocks workgroups of four waves)
template <int LA, int LB, int LC, int LD, int NW>
struct LpqBounds {
    static constexpr int value = (LpqMinBlocks<LA, LB, LC, LD>::value * FK_WAVES + NW - 1) / NW;
};

// ENG: the integral engine, 0 Rys quadrature, 1 HGP with early contraction;
// NW: waves per workgroup
template <int LA, int LB, int LC, int LD, typename R = double, int ENG = 0, int NW = FK_WAVES>
__global__ void __launch_bounds__(64 * NW, (LpqBounds<LA, LB, LC, LD, NW>::value)) k_jk_lpq(FkJKArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    constexpr int NA = Q::NA, NB = Q::NB, NC = Q::NC, ND = Q::ND, NOUT = Q::NOUT;
    static_assert(NOUT <= FK_LPQ_BLOCK_NOUT, "lane-per-quartet classes sum their bra blocks in registers");
    const bool wj = (a.want & FK_WANT_J) != 0, wk = (a.want & FK_WANT_K) != 0;
    FK_DYN_LDS(s_dyn);
    double *s_tab = s_dyn;
    load_table<Q::NR>(s_tab, a.rys_tab);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the stage of each wave: its full size, or the X_J[c, d] part with block tasks
    const int stg = a.ntask > 0 ? LpqStageTask<LA, LB, LC, LD>::value : LpqStage<LA, LB, LC, LD>::value;
    double *s_stage = s_dyn + rys_lds_size(Q::NR) + wave * stg;
    unsigned long long cq = 0, cp = 0;

    constexpr int NBK = LpqKetOuter<LA, LB, LC, LD>::value;
    // instantiations that take block tasks: the ket-outer ones and the wide ones
    constexpr bool TASKS = NBK > 0 || NW > FK_WAVES;
    // bras per block of the block tasks' rows (the class's bra block)
    const int nbk = a.krow_nbk;
    // one tile (t) for this wave; kr: the workgroup's K rows of a block task, or null
    auto do_tile = [&](int t, double *kr) {
        if constexpr (!TASKS) kr = nullptr;
        const FkTile tile = a.tiles[t];
        const bool same = (tile.grp & FK_TILE_SAME) != 0;
        const FkGroup g = a.groups[tile.grp & ~FK_TILE_SAME];
        // the tile's molecule: its blocks of D, D_sh, X_J, X_K and shells
        const int mol = g.mol;
        const int n = a.mol_nbf[mol], ns = a.mol_nsh[mol];
        const int *__restrict shbf = a.sh_bf + a.mol_sh0[mol];
        const double *__restrict Ds = a.Ds + a.mol_base[mol];
        const double *__restrict Dsh = a.Dsh + a.mol_shbase[mol];
        const long long xoff = (long long)(blockIdx.x % FK_XCD_COPIES) * a.xcopy + a.mol_base[mol];
        double *XJ = a.XJ + xoff;
        double *XK = a.XK + xoff;
        const FkBraBlock blk = a.blocks[tile.blk];
        const bool inrange = lane < tile.ket_count;
        const int pos = tile.ket_begin + (inrange ? lane : 0);
        const int r = pos - g.begin;
        const KetInfo Kt = load_ket(a, pos);
        const int sc = Kt.sc, sd = Kt.sd;
        const int oc = shbf[sc], od = shbf[sd];
        const int sa = a.pair_sa[a.blk_bra[blk.first]];
        const int oa = shbf[sa];
        int colc = 0, cold = 0;
        if (kr) {
            const int *kcol = a.krow_col + a.mol_sh0[mol];
            colc = kcol[sc];
            cold = kcol[sd] + (LC != LD ? a.krow_cnt[4 * mol + LC] : 0);
        }
        // D_cd is used with every bra of the block
        double dcd[NC * ND];
#pragma unroll
        for (int ic = 0; ic < NC; ++ic)
#pragma unroll
            for (int id = 0; id < ND; ++id) dcd[ic * ND + id] = wj ? Ds[(size_t)(oc + ic) * n + od + id] : 0.0;
        // block sums: X_K[a, c], X_K[a, d], X_J[c, d]
        double kac[NA * NC], kad[NA * ND], jcd[NC * ND];
#pragma unroll
        for (int o = 0; o < NA * NC; ++o) kac[o] = 0.0;
#pragma unroll
        for (int o = 0; o < NA * ND; ++o) kad[o] = 0.0;
#pragma unroll
        for (int o = 0; o < NC * ND; ++o) jcd[o] = 0.0;
        bool any = false;

        if constexpr (NBK > 0) {
            // ket-outer: screen every bra of the block first, then one pass over
            // the ket's primitives for all of them, then the digestion per bra
            using H = fk::HgpClass<LA, LB, LC, LD>;
            constexpr int NACC = ENG == 0 ? NOUT : H::NACC;
            const int nb = blk.count;  // at most NBK: the class reports it as its largest bra block
            unsigned act = 0u;
            int ppo[NBK], bnpp[NBK];
            R acck[NBK][NACC];
#pragma unroll
            for (int jb = 0; jb < NBK; ++jb) {
#pragma unroll
                for (int o = 0; o < NACC; ++o) acck[jb][o] = (R)0;
                ppo[jb] = 0;
                bnpp[jb] = 0;
                if (jb < nb) {
                    const int bra = a.blk_bra[blk.first + jb];
                    const int bpos = a.blk_pos[blk.first + jb];
                    const bool active = screen_lane<R>(a, inrange && (!same || pos <= bpos), a.pair_G[bra] * Kt.G,
                                                       Dsh, ns, sa, a.pair_sb[bra], sc, sd);
                    ppo[jb] = __builtin_amdgcn_readfirstlane(a.pair_ppoff[bra]);
                    bnpp[jb] = __builtin_amdgcn_readfirstlane(a.pair_npp[bra]);
                    const int nact = __popcll(__ballot(active));
                    cq += nact;
                    cp += (unsigned long long)nact * bnpp[jb] * g.npp;
                    if (active) act |= 1u << jb;
                }
            }
            if (act) {
                fk::PrimPair qn = load_ket_pp(a.ppT, g, 0, r);
                for (int j = 0; j < g.npp; ++j) {
                    const fk::PrimPair q = qn;
                    if (j + 1 < g.npp) qn = load_ket_pp(a.ppT, g, j + 1, r);
#pragma unroll
                    for (int jb = 0; jb < NBK; ++jb) {
                        if (jb < nb && ((act >> jb) & 1u)) {
                            const fk_const_ptr ab = (fk_const_ptr)(a.pair_AB + 3 * a.blk_bra[blk.first + jb]);
                            const double AB[3] = {ab[0], ab[1], ab[2]};
                            if constexpr (ENG == 0) {
                                constexpr bool PAIR = NOUT <= FK_LPQ_PAIR_NOUT;
                                int i = 0;
                                if constexpr (PAIR)
                                    for (; i + 1 < bnpp[jb]; i += 2) {
                                        const fk::PrimPair p0 = sload_pp(a.pp, ppo[jb] + i);
                                        const fk::PrimPair p1 = sload_pp(a.pp, ppo[jb] + i + 1);
                                        fk::rys_prim_all<LA, LB, LC, LD, R, true>(s_tab, p0, q, AB, Kt.CD, acck[jb]);
                                        fk::rys_prim_all<LA, LB, LC, LD, R, true>(s_tab, p1, q, AB, Kt.CD, acck[jb]);
                                    }
                                for (; i < bnpp[jb]; ++i)
                                    fk::rys_prim_all<LA, LB, LC, LD, R, PAIR>(s_tab, sload_pp(a.pp, ppo[jb] + i), q,
                                                                              AB, Kt.CD, acck[jb]);
                            } else {
                                for (int i = 0; i < bnpp[jb]; ++i)
                                    fk::hgp_prim<LA, LB, LC, LD, R>(s_tab, sload_pp(a.pp, ppo[jb] + i), q, acck[jb]);
                            }
                        }
                    }
                }
            }
            // digestion, one bra at a time: the block's accumulators move down
            // one slot per bra, so the loop body reads slot 0 only
            for (int jb = 0; jb < nb; ++jb) {
                const int bra = a.blk_bra[blk.first + jb];
                const int bpos = a.blk_pos[blk.first + jb];
                const int sb = a.pair_sb[bra];
                const bool active = ((act >> jb) & 1u) != 0u;
                R acc[NOUT];
                if constexpr (ENG == 0) {
#pragma unroll
                    for (int o = 0; o < NOUT; ++o) acc[o] = acck[0][o];
                } else {
#pragma unroll
                    for (int o = 0; o < NOUT; ++o) acc[o] = (R)0;
                    if (active) {
                        const double AB[3] = {a.pair_AB[3 * bra], a.pair_AB[3 * bra + 1], a.pair_AB[3 * bra + 2]};
                        fk::hgp_hrr<LA, LB, LC, LD, R>(acck[0], AB, Kt.CD, acc);
                    }
                }
#pragma unroll
                for (int k = 0; k + 1 < NBK; ++k)
#pragma unroll
                    for (int o = 0; o < NACC; ++o) acck[k][o] = acck[k + 1][o];
                if (__ballot(active) == 0ull) continue;
                lpq_digest<LA, LB, LC, LD, R>(acc, active, same && pos == bpos, sa, sb, sc, sd, oa, shbf[sb], oc,
                                              od, n, Ds, dcd, kac, kad, jcd, XJ, XK, s_stage, lane, wj, wk, any,
                                              kr ? kr + jb * NB * a.krow_ncol : nullptr, a.krow_ncol, colc, cold,
                                              kr ? kr + (nbk * NB + NA) * a.krow_ncol + jb * NA * NB : nullptr);
            }
        } else
        for (int jb = 0; jb < blk.count; ++jb) {
            const int bra = a.blk_bra[blk.first + jb];
            const int bpos = a.blk_pos[blk.first + jb];
            const BraInfo B = load_bra(a, bra);
            const int sb = B.sb;
            // Schwarz bound, same-class triangle (ket position <= bra position)
            // and density screen for this (bra, ket)
            const bool active = screen_lane<R>(a, inrange && (!same || pos <= bpos), B.G * Kt.G, Dsh, ns, sa, sb, sc, sd);
            const unsigned long long mask = __ballot(active);
            if (mask == 0ull) continue;
            const int nact = __popcll(mask);
            cq += nact;
            cp += (unsigned long long)nact * B.npp * g.npp;

            const int ppo = __builtin_amdgcn_readfirstlane(B.ppo);
            const int bnpp = __builtin_amdgcn_readfirstlane(B.npp);
            R acc[NOUT];
#pragma unroll
            for (int o = 0; o < NOUT; ++o) acc[o] = (R)0;
            if constexpr (ENG == 0) {
                if (active) {
                    fk::PrimPair qn = load_ket_pp(a.ppT, g, 0, r);
                    for (int j = 0; j < g.npp; ++j) {
                        const fk::PrimPair q = qn;
                        if (j + 1 < g.npp) qn = load_ket_pp(a.ppT, g, j + 1, r);
                        // two bra primitives per step for the small classes: their
                        // quartets are independent straight-line code the compiler
                        // interleaves (larger classes would spill)
                        constexpr bool PAIR = NOUT <= FK_LPQ_PAIR_NOUT;
                        int i = 0;
                        if constexpr (PAIR)
                            for (; i + 1 < bnpp; i += 2) {
                                const fk::PrimPair p0 = sload_pp(a.pp, ppo + i), p1 = sload_pp(a.pp, ppo + i + 1);
                                fk::rys_prim_all<LA, LB, LC, LD, R, true>(s_tab, p0, q, B.AB, Kt.CD, acc);
                                fk::rys_prim_all<LA, LB, LC, LD, R, true>(s_tab, p1, q, B.AB, Kt.CD, acc);
                            }
                        for (; i < bnpp; ++i)
                            fk::rys_prim_all<LA, LB, LC, LD, R, PAIR>(s_tab, sload_pp(a.pp, ppo + i), q, B.AB, Kt.CD,
                                                                      acc);
                    }
                }
            } else {
                // HGP engine: [e0|f0] summed over the primitives, then the
                // horizontal recurrences once per contracted quartet
                using H = fk::HgpClass<LA, LB, LC, LD>;
                R acce[H::NACC];
#pragma unroll
                for (int o = 0; o < H::NACC; ++o) acce[o] = (R)0;
                if (active) {
                    fk::PrimPair qn = load_ket_pp(a.ppT, g, 0, r);
                    for (int j = 0; j < g.npp; ++j) {
                        const fk::PrimPair q = qn;
                        if (j + 1 < g.npp) qn = load_ket_pp(a.ppT, g, j + 1, r);
                        for (int i = 0; i < bnpp; ++i)
                            fk::hgp_prim<LA, LB, LC, LD, R>(s_tab, sload_pp(a.pp, ppo + i), q, acce);
                    }
                    fk::hgp_hrr<LA, LB, LC, LD, R>(acce, B.AB, Kt.CD, acc);
                }
            }
            const bool diag = same && pos == bpos;
            lpq_digest<LA, LB, LC, LD, R>(acc, active, diag, sa, sb, sc, sd, oa, shbf[sb], oc, od, n, Ds, dcd, kac,
                                          kad, jcd, XJ, XK, s_stage, lane, wj, wk, any,
                                          kr ? kr + jb * NB * a.krow_ncol : nullptr, a.krow_ncol, colc, cold,
                                          kr ? kr + (nbk * NB + NA) * a.krow_ncol + jb * NA * NB : nullptr);
        }
        // block sums: a lane without work holds zeros, which are not added
        if (__ballot(any) != 0ull) {
            if (wk && kr) {
                // X_K[a, c], X_K[a, d] into the block's a rows
                double *kra = kr + nbk * NB * a.krow_ncol;
#pragma unroll
                for (int o = 0; o < NA * NC; ++o)
                    if (kac[o] != 0.0) lds_add(&kra[(o / NC) * a.krow_ncol + colc + o % NC], kac[o]);
#pragma unroll
                for (int o = 0; o < NA * ND; ++o)
                    if (kad[o] != 0.0) lds_add(&kra[(o / ND) * a.krow_ncol + cold + o % ND], kad[o]);
            } else if (wk) {
                flush_sym<NA, NC>(XK, n, oa, oc, kac, s_stage, lane);
                flush_sym<NA, ND>(XK, n, oa, od, kad, s_stage, lane);
            }
            if (wj) {
#pragma unroll
                for (int o = 0; o < NC * ND; ++o) jcd[o] *= 2.0;
                flush_sym<NC, ND>(XJ, n, oc, od, jcd, s_stage, lane);
            }
        }
    };
    if (TASKS && a.ntask > 0) {
        // block tasks: the K rows follow the table and the waves' stages
        double *kr = s_dyn + rys_lds_size(Q::NR) + NW * stg;
        const int ncol = a.krow_ncol;
        const int nkr = (nbk * NB + NA) * ncol + nbk * NA * NB;
        for (int task = blockIdx.x; task < a.ntask; task += gridDim.x) {
            const int2 tk = a.tasks[task];
            for (int i = threadIdx.x; i < nkr; i += 64 * NW) kr[i] = 0.0;
            __syncthreads();
            for (int t = tk.x + wave; t < tk.x + tk.y; t += NW) do_tile(t, kr);
            __syncthreads();
            // the block's rows to memory: nonzero entries, consecutive threads
            // on consecutive columns of a row
            const FkTile t0 = a.tiles[tk.x];
            const int mol = a.groups[t0.grp & ~FK_TILE_SAME].mol;
            const int n = a.mol_nbf[mol];
            const int *__restrict shbf = a.sh_bf + a.mol_sh0[mol];
            const long long xoff = (long long)(blockIdx.x % FK_XCD_COPIES) * a.xcopy + a.mol_base[mol];
            const FkBraBlock blk = a.blocks[t0.blk];
            const int oa = shbf[a.pair_sa[a.blk_bra[blk.first]]];
            const int cc = a.krow_cnt[4 * mol + LC];
            const int ncm = cc + (LC != LD ? a.krow_cnt[4 * mol + LD] : 0);
            const int *fnc = a.krow_fn + a.krow_off[4 * mol + LC];
            const int *fnd = a.krow_fn + a.krow_off[4 * mol + LD];
            if (wk) {
                double *XK = a.XK + xoff;
                const int nrow = blk.count * NB + NA;
                for (int e = threadIdx.x; e < nrow * ncm; e += 64 * NW) {
                    const int r = e / ncm, x = e - r * ncm;
                    const int rr = r < blk.count * NB ? r : nbk * NB + (r - blk.count * NB);
                    const double v = kr[rr * ncol + x];
                    if (v == 0.0) continue;
                    const int row = r < blk.count * NB ? shbf[a.pair_sb[a.blk_bra[blk.first + r / NB]]] + r % NB
                                                       : oa + (r - blk.count * NB);
                    const int fn = x < cc ? fnc[x] : fnd[x - cc];
                    atomic_add(&XK[(size_t)row * n + fn], v);
                }
            }
            if (wj) {
                double *XJ = a.XJ + xoff;
                const double *kj = kr + (nbk * NB + NA) * ncol;
                for (int e = threadIdx.x; e < blk.count * NA * NB; e += 64 * NW) {
                    const double v = kj[e];
                    if (v == 0.0) continue;
                    const int jb = e / (NA * NB), ab = e % (NA * NB);
                    const int ob = shbf[a.pair_sb[a.blk_bra[blk.first + jb]]];
                    atomic_add(&XJ[(size_t)(oa + ab / NB) * n + ob + ab % NB], v);
                }
            }
            __syncthreads();
        }
    } else {
        const int nwt = gridDim.x * NW;
        for (int t = blockIdx.x * NW + wave; t < a.ntiles; t += nwt) do_tile(t, nullptr);
    }
    if (lane == 0 && cq) {
        atomicAdd(&a.counters[0], cq);
        atomicAdd(&a.counters[1], cp);
    }
}

// ---------------------------------------------------------------- tpq ----
// Team per quartet: a team of TS lanes computes one contracted quartet, lane
// `comp` of the team owning bra component a (MODE 1, TS = NA, all b) or the
// bra component pair (a, b) (MODE 2, TS = NA NB); a wave holds 64/TS teams,
// which take consecutive kets of the tile.  A tile holds a block of bras that
// share their first shell a; each team keeps its ket for every bra of the
// block.  Sums that span the lanes of a team (X_K[b, c], X_K[b, d] per bra and
// X_J[c, d] per block) or the whole wave (X_J[a, b] per bra, over all kets of
// the tile) are formed with LDS atomics and reach memory once; X_K[a, c] and
// X_K[a, d] stay in the lane's registers over the block.
#define FK_TEAM_MAX_BLOCK 8

template <int LA, int LB, int LC, int LD, int MODE>
struct TeamShape {
    using Q = fk::QClass<LA, LB, LC, LD>;
    static constexpr int TS = (MODE == 1) ? Q::NA : Q::NA * Q::NB;
    static constexpr int QPW = 64 / TS;
    static constexpr int NVB = Q::NB * (Q::NC + Q::ND);   // team sums per bra
    static constexpr int NV = NVB > Q::NC * Q::ND ? NVB : Q::NC * Q::ND;
    // per-wave LDS for the reductions (doubles), after the staged bra records
    static constexpr int RED = QPW * NV + FK_TEAM_MAX_BLOCK * Q::NA * Q::NB;
};


// Waves per SIMD the compiler must fit in registers (as for the lane-per-quartet
// kernels): team classes whose demand is just above half of the file run
// faster at two waves with some bytes spilled (measured: the d classes on
// C20H42, the f classes on the organic batch).
template <int LA, int LB, int LC, int LD>
struct TpqMinBlocks {
    static constexpr int value = 1;
};
template <>
struct TpqMinBlocks<2, 1, 2, 0> {
    static constexpr int value = 2;
};
template <>
struct TpqMinBlocks<2, 2, 1, 0> {
    static constexpr int value = 2;
};
template <>
struct TpqMinBlocks<3, 2, 1, 0> {
    static constexpr int value = 2;
};
template <>
struct TpqMinBlocks<3, 0, 1, 1> {
    static constexpr int value = 2;
};
template <>
struct TpqMinBlocks<3, 1, 2, 0> {
    static constexpr int value = 2;
};
template <>
struct TpqMinBlocks<3, 0, 3, 0> {
    static constexpr int value = 2;
};

template <int LA, int LB, int LC, int LD, int MODE, typename R = double>
__global__ void __launch_bounds__(FK_BLOCK, (TpqMinBlocks<LA, LB, LC, LD>::value)) k_jk_tpq(FkJKArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    using TSh = TeamShape<LA, LB, LC, LD, MODE>;
    constexpr int NA = Q::NA, NB = Q::NB, NC = Q::NC, ND = Q::ND;
    constexpr int TS = TSh::TS, QPW = TSh::QPW, NV = TSh::NV;
    constexpr int NBL = (MODE == 1) ? NB : 1;
    constexpr int NOL = NBL * NC * ND;
    static_assert(QPW >= 1, "team larger than a wave");
    const bool wj = (a.want & FK_WANT_J) != 0, wk = (a.want & FK_WANT_K) != 0;
    FK_DYN_LDS(s_dyn);
    double *s_tab = s_dyn;
    load_table<Q::NR>(s_tab, a.rys_tab);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *s_team = s_dyn + rys_lds_size(Q::NR) + wave * TSh::RED;  // [QPW][NV] team sums
    double *s_jab = s_team + QPW * NV;       // [block bra][NA * NB] wave sums of X_J[a, b]
    const int nwt = gridDim.x * FK_WAVES;
    const int slot = lane / TS, comp = lane % TS;
    const bool lane_ok = slot < QPW;
    const int ia = (MODE == 1) ? comp : comp / NB;
    const int ib0 = (MODE == 1) ? 0 : comp % NB;
    const int ax[3] = {fk::kCart.x[LA][ia], fk::kCart.y[LA][ia], fk::kCart.z[LA][ia]};
    const int bx[3] = {fk::kCart.x[LB][ib0], fk::kCart.y[LB][ib0], fk::kCart.z[LB][ib0]};
    double *tsum = s_team + (lane_ok ? slot : 0) * NV;
    unsigned long long cq = 0, cp = 0;

    for (int t = blockIdx.x * FK_WAVES + wave; t < a.ntiles; t += nwt) {
        const FkTile tile = a.tiles[t];
        const bool same = (tile.grp & FK_TILE_SAME) != 0;
        const FkGroup g = a.groups[tile.grp & ~FK_TILE_SAME];
        // the tile's molecule: its blocks of D, D_sh, X_J, X_K and shells
        const int mol = g.mol;
        const int n = a.mol_nbf[mol], ns = a.mol_nsh[mol];
        const int *__restrict shbf = a.sh_bf + a.mol_sh0[mol];
        const double *__restrict Ds = a.Ds + a.mol_base[mol];
        const double *__restrict Dsh = a.Dsh + a.mol_shbase[mol];
        const long long xoff = (long long)(blockIdx.x % FK_XCD_COPIES) * a.xcopy + a.mol_base[mol];
        double *XJ = a.XJ + xoff;
        double *XK = a.XK + xoff;
        const FkBraBlock blk = a.blocks[tile.blk];
        const int sa = a.pair_sa[a.blk_bra[blk.first]];
        const int oa = shbf[sa];
        const size_t ra = (size_t)(oa + ia) * n;
        wave_sync_lds();
        for (int x = lane; x < blk.count * NA * NB; x += 64) s_jab[x] = 0.0;

        // rounds of QPW kets, one per team
        for (int k0 = 0; k0 < tile.ket_count; k0 += QPW) {
            const bool tin = lane_ok && k0 + slot < tile.ket_count;
            const int pos = tile.ket_begin + (tin ? k0 + slot : 0);
            const int r = pos - g.begin;
            const KetInfo Kt = load_ket(a, pos);
            const int sc = Kt.sc, sd = Kt.sd;
            const int oc = shbf[sc], od = shbf[sd];
            double kac[NC], kad[ND], jcd[NC * ND];
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) kac[ic] = 0.0;
#pragma unroll
            for (int id = 0; id < ND; ++id) kad[id] = 0.0;
#pragma unroll
            for (int o = 0; o < NC * ND; ++o) jcd[o] = 0.0;
            bool any = false;

            for (int jb = 0; jb < blk.count; ++jb) {
                const int bra = a.blk_bra[blk.first + jb];
                const int bpos = a.blk_pos[blk.first + jb];
                const BraInfo B = load_bra(a, bra);
                const int sb = B.sb;
                const bool active = screen_lane<R>(a, tin && (!same || pos <= bpos), B.G * Kt.G, Dsh, ns, sa, sb, sc, sd);
                const unsigned long long mask = __ballot(active);
                if (mask == 0ull) continue;
                const int nact = __popcll(mask) / TS;
                cq += nact;
                cp += (unsigned long long)nact * B.npp * g.npp;
                const int ppo = __builtin_amdgcn_readfirstlane(B.ppo);
                const int bnpp = __builtin_amdgcn_readfirstlane(B.npp);
                R acc[NOL];
#pragma unroll
                for (int o = 0; o < NOL; ++o) acc[o] = (R)0;
                if (active) {
                    fk::PrimPair qn = load_ket_pp(a.ppT, g, 0, r);
                    for (int j = 0; j < g.npp; ++j) {
                        const fk::PrimPair q = qn;
                        if (j + 1 < g.npp) qn = load_ket_pp(a.ppT, g, j + 1, r);
                        for (int i = 0; i < bnpp; ++i)
                            fk::rys_prim_team<LA, LB, LC, LD, MODE, R>(s_tab, sload_pp(a.pp, ppo + i), q, B.AB, Kt.CD,
                                                                      ax, bx, acc);
                    }
                }
                const bool diag = same && pos == bpos;
                const double fac = (sa == sb ? 0.5 : 1.0) * (sc == sd ? 0.5 : 1.0) * (diag ? 0.5 : 1.0);
                const int ob = shbf[sb];
                // team sums of X_K[b, c] and X_K[b, d] for this bra
                if (lane_ok)
                    for (int v = comp; v < NV; v += TS) tsum[v] = 0.0;
                wave_sync_lds();
                if (active) {
                    any = true;
#pragma unroll
                    for (int jj = 0; jj < NBL; ++jj) {
                        const int ib = (MODE == 1) ? jj : ib0;
                        const size_t rb = (size_t)(ob + ib) * n;
                        if (wj) {
                            const double dab = Ds[ra + ob + ib];
                            double sj = 0.0;
#pragma unroll
                            for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                                for (int id = 0; id < ND; ++id) {
                                    const double v = fac * acc[(jj * NC + ic) * ND + id];
                                    sj += v * Ds[(size_t)(oc + ic) * n + od + id];
                                    jcd[ic * ND + id] += v * dab;
                                }
                            lds_add(&s_jab[jb * NA * NB + ia * NB + ib], sj);
                        }
                        if (wk) {
#pragma unroll
                            for (int ic = 0; ic < NC; ++ic) {
                                double kbc = 0.0;
#pragma unroll
                                for (int id = 0; id < ND; ++id) {
                                    const double v = fac * acc[(jj * NC + ic) * ND + id];
                                    kac[ic] += v * Ds[rb + od + id];
                                    kad[id] += v * Ds[rb + oc + ic];
                                    kbc += v * Ds[ra + od + id];
                                }
                                lds_add(&tsum[ib * NC + ic], kbc);
                            }
#pragma unroll
                            for (int id = 0; id < ND; ++id) {
                                double kbd = 0.0;
#pragma unroll
                                for (int ic = 0; ic < NC; ++ic)
                                    kbd += fac * acc[(jj * NC + ic) * ND + id] * Ds[ra + oc + ic];
                                lds_add(&tsum[NB * NC + ib * ND + id], kbd);
                            }
                        }
                    }
                }
                wave_sync_lds();
                if (active && wk)
                    for (int v = comp; v < TSh::NVB; v += TS) {
                        size_t dst;
                        if (v < NB * NC) dst = (size_t)(ob + v / NC) * n + oc + v % NC;
                        else dst = (size_t)(ob + (v - NB * NC) / ND) * n + od + (v - NB * NC) % ND;
                        atomic_add(&XK[dst], tsum[v]);
                    }
                wave_sync_lds();
            }
            // end of the block for this round's kets: X_K[a, c], X_K[a, d] from
            // the lanes, X_J[c, d] as a team sum
            if (lane_ok)
                for (int v = comp; v < NV; v += TS) tsum[v] = 0.0;
            wave_sync_lds();
            if (any && wk) {
#pragma unroll
                for (int ic = 0; ic < NC; ++ic) atomic_add(&XK[ra + oc + ic], kac[ic]);
#pragma unroll
                for (int id = 0; id < ND; ++id) atomic_add(&XK[ra + od + id], kad[id]);
            }
            if (any && wj) {
#pragma unroll
                for (int o = 0; o < NC * ND; ++o) lds_add(&tsum[o], jcd[o]);
            }
            wave_sync_lds();
            if (any && wj)
                for (int v = comp; v < NC * ND; v += TS)
                    atomic_add(&XJ[(size_t)(oc + v / ND) * n + od + v % ND], 2.0 * tsum[v]);
            wave_sync_lds();
        }
        // X_J[a, b] of every bra of the block, summed over the tile's kets
        for (int x = lane; x < blk.count * NA * NB; x += 64) {
            const int jb = x / (NA * NB), ab = x % (NA * NB);
            const int ob = shbf[a.pair_sb[a.blk_bra[blk.first + jb]]];
            const double v = s_jab[x];
            if (v != 0.0) atomic_add(&XJ[(size_t)(oa + ab / NB) * n + ob + ab % NB], 2.0 * v);
        }
    }
    if (lane == 0 && cq) {
        atomicAdd(&a.counters[0], cq);
        atomicAdd(&a.counters[1], cp);
    }
}

// ---------------------------------------------------------------- wpq ----
// SPLIT consecutive waves per contracted quartet (f-f bras, whose bra
// component pairs exceed a wave): wave h of the group owns the bra component
// pairs h CPW .. (h + 1) CPW - 1, CPW = ceil(NA NB / SPLIT), lane i of it pairs
// i, i + 64, ... of that range (each with every ket component).  The waves of a
// group repeat the quartet's set-up and each adds its own part of every
// Fock block; two waves of 50 pairs instead of one wave of 64 + 36 hold half
// the accumulators per lane.
template <int LA, int LB, int LC, int LD>
struct WpqSplit {
    static constexpr int value = fk::QClass<LA, LB, LC, LD>::NA * fk::QClass<LA, LB, LC, LD>::NB > 64 ? 2 : 1;
};

template <int LA, int LB, int LC, int LD>
__global__ void __launch_bounds__(FK_BLOCK) k_jk_wpq(FkJKArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    constexpr int NB = Q::NB, NC = Q::NC, ND = Q::ND;
    constexpr int NAB = Q::NA * Q::NB, NCD = NC * ND;
    constexpr int SPLIT = WpqSplit<LA, LB, LC, LD>::value;
    static_assert(FK_WAVES % SPLIT == 0, "a wave group lies within a workgroup");
    constexpr int CPW = (NAB + SPLIT - 1) / SPLIT;
    constexpr int ITEMS = (CPW + 63) / 64;
    const bool wj = (a.want & FK_WANT_J) != 0, wk = (a.want & FK_WANT_K) != 0;
    FK_DYN_LDS(s_dyn);
    double *s_tab = s_dyn;
    load_table<Q::NR>(s_tab, a.rys_tab);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = wave % SPLIT;                  // this wave's part of the group
    const int nwt = gridDim.x * (FK_WAVES / SPLIT); // wave groups of the grid
    unsigned long long cq = 0, cp = 0;

    int iax[ITEMS][3], ibx[ITEMS][3], iab[ITEMS];
    bool ival[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int it = half * CPW + lane + 64 * k;
        ival[k] = lane + 64 * k < CPW && it < NAB;
        const int ia = ival[k] ? it / NB : 0, ib = ival[k] ? it % NB : 0;
        iab[k] = ia * NB + ib;
        iax[k][0] = fk::kCart.x[LA][ia]; iax[k][1] = fk::kCart.y[LA][ia]; iax[k][2] = fk::kCart.z[LA][ia];
        ibx[k][0] = fk::kCart.x[LB][ib]; ibx[k][1] = fk::kCart.y[LB][ib]; ibx[k][2] = fk::kCart.z[LB][ib];
    }

    for (int t = blockIdx.x * (FK_WAVES / SPLIT) + wave / SPLIT; t < a.ntiles; t += nwt) {
        const FkTile tile = a.tiles[t];
        // team and wave kernels get blocks of one bra: the tile's kets are
        // exactly that bra's Schwarz prefix (and same-class triangle)
        const int bra = a.blk_bra[a.blocks[tile.blk].first];
        const bool same = (tile.grp & FK_TILE_SAME) != 0;
        const FkGroup g = a.groups[tile.grp & ~FK_TILE_SAME];
        // the tile's molecule: its blocks of D, D_sh, X_J, X_K and shells
        const int mol = g.mol;
        const int n = a.mol_nbf[mol], ns = a.mol_nsh[mol];
        const int *__restrict shbf = a.sh_bf + a.mol_sh0[mol];
        const double *__restrict Ds = a.Ds + a.mol_base[mol];
        const double *__restrict Dsh = a.Dsh + a.mol_shbase[mol];
        const long long xoff = (long long)(blockIdx.x % FK_XCD_COPIES) * a.xcopy + a.mol_base[mol];
        double *XJ = a.XJ + xoff;
        double *XK = a.XK + xoff;
        const BraInfo B = load_bra(a, bra);
        const int sa = B.sa, sb = B.sb;
        const int oa = shbf[sa], ob = shbf[sb];
        unsigned long long live;
        {
            const bool in = lane < tile.ket_count;
            const KetInfo K0 = load_ket(a, tile.ket_begin + (in ? lane : 0));
            bool ok = in;
            if (a.dscreen) ok = ok && (B.G * K0.G * dmax_args(a, Dsh, ns, sa, sb, K0.sc, K0.sd) >= a.tau);
            live = __ballot(ok);
        }
        if (live == 0ull) continue;
        const int ppo = __builtin_amdgcn_readfirstlane(B.ppo);
        const int bnpp = __builtin_amdgcn_readfirstlane(B.npp);
        while (live) {
            const int k = __ffsll((long long)live) - 1;
            live &= live - 1;
            const int pos = tile.ket_begin + k;
            const KetInfo Kt = load_ket(a, pos);
            const int sc = Kt.sc, sd = Kt.sd;
            const int r = pos - g.begin;
            if (half == 0) {
                cq += 1;
                cp += (unsigned long long)B.npp * g.npp;
            }
            double acc[ITEMS][NCD];
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
#pragma unroll
                for (int o = 0; o < NCD; ++o) acc[it][o] = 0.0;
            for (int j = 0; j < g.npp; ++j) {
                const fk::PrimPair q = load_ket_pp(a.ppT, g, j, r);
                for (int i = 0; i < bnpp; ++i) {
                    const fk::PrimPair p = sload_pp(a.pp, ppo + i);
#pragma unroll
                    for (int it = 0; it < ITEMS; ++it)
                        if (ival[it]) fk::rys_prim_bra_comp<LA, LB, LC, LD>(s_tab, p, q, B.AB, Kt.CD, iax[it], ibx[it], acc[it]);
                }
            }
            const bool diag = same && a.ket_list[pos] == bra;
            const double fac = (sa == sb ? 0.5 : 1.0) * (sc == sd ? 0.5 : 1.0) * (diag ? 0.5 : 1.0);
            const int oc = shbf[sc], od = shbf[sd];
            double jcd[NCD];
#pragma unroll
            for (int o = 0; o < NCD; ++o) jcd[o] = 0.0;
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                if (!ival[it]) continue;
                const int ia = iab[it] / NB, ib = iab[it] % NB;
                double *v = acc[it];
#pragma unroll
                for (int o = 0; o < NCD; ++o) v[o] *= fac;
                if (wj) {
                    const double dab = Ds[(size_t)(oa + ia) * n + ob + ib];
                    double sj = 0.0;
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                        for (int id = 0; id < ND; ++id) {
                            sj += v[ic * ND + id] * Ds[(size_t)(oc + ic) * n + od + id];
                            jcd[ic * ND + id] += v[ic * ND + id] * dab;
                        }
                    atomic_add(&XJ[(size_t)(oa + ia) * n + ob + ib], 2.0 * sj);
                }
                if (!wk) continue;
#pragma unroll
                for (int ic = 0; ic < NC; ++ic) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int id = 0; id < ND; ++id) {
                        s1 += v[ic * ND + id] * Ds[(size_t)(ob + ib) * n + od + id];
                        s2 += v[ic * ND + id] * Ds[(size_t)(oa + ia) * n + od + id];
                    }
                    atomic_add(&XK[(size_t)(oa + ia) * n + oc + ic], s1);
                    atomic_add(&XK[(size_t)(ob + ib) * n + oc + ic], s2);
                }
#pragma unroll
                for (int id = 0; id < ND; ++id) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic) {
                        s1 += v[ic * ND + id] * Ds[(size_t)(ob + ib) * n + oc + ic];
                        s2 += v[ic * ND + id] * Ds[(size_t)(oa + ia) * n + oc + ic];
                    }
                    atomic_add(&XK[(size_t)(oa + ia) * n + od + id], s1);
                    atomic_add(&XK[(size_t)(ob + ib) * n + od + id], s2);
                }
            }
            if (wj) {
#pragma unroll
                for (int o = 0; o < NCD; ++o) {
                    const double s = wave_sum(jcd[o]);
                    if (lane == 0) atomic_add(&XJ[(size_t)(oc + o / ND) * n + od + o % ND], 2.0 * s);
                }
            }
        }
    }
    if (lane == 0 && cq) {
        atomicAdd(&a.counters[0], cq);
        atomicAdd(&a.counters[1], cp);
    }
}

// -------------------------------------------------------------- debug ----
// Raw contracted integrals of listed quartets (canonical orientation), one
// lane per quartet (small classes) or one wave per quartet (large classes).
template <int LA, int LB, int LC, int LD>
__global__ void __launch_bounds__(FK_BLOCK) k_debug_lpq(FkDebugArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    __shared__ double s_tab[rys_lds_size(Q::NR)];
    load_table<Q::NR>(s_tab, a.rys_tab);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int bra = a.quartets[q].x, ket = a.quartets[q].y;
    const double AB[3] = {a.pair_AB[3 * bra], a.pair_AB[3 * bra + 1], a.pair_AB[3 * bra + 2]};
    const double CD[3] = {a.pair_AB[3 * ket], a.pair_AB[3 * ket + 1], a.pair_AB[3 * ket + 2]};
    double acc[Q::NOUT];
#pragma unroll
    for (int o = 0; o < Q::NOUT; ++o) acc[o] = 0.0;
    for (int i = 0; i < a.pair_npp[bra]; ++i) {
        const fk::PrimPair p = load_pp(a.pp, a.pair_ppoff[bra] + i);
        for (int j = 0; j < a.pair_npp[ket]; ++j)
            fk::rys_prim_all<LA, LB, LC, LD>(s_tab, p, load_pp(a.pp, a.pair_ppoff[ket] + j), AB, CD, acc);
    }
#pragma unroll
    for (int o = 0; o < Q::NOUT; ++o) a.out[(size_t)q * Q::NOUT + o] = acc[o];
}

template <int LA, int LB, int LC, int LD>
__global__ void __launch_bounds__(FK_BLOCK) k_debug_wpq(FkDebugArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    constexpr int NB = Q::NB, NAB = Q::NA * Q::NB, NCD = Q::NC * Q::ND;
    __shared__ double s_tab[rys_lds_size(Q::NR)];
    load_table<Q::NR>(s_tab, a.rys_tab);
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * FK_WAVES + (threadIdx.x >> 6);
    if (q >= a.nq) return;
    const int bra = a.quartets[q].x, ket = a.quartets[q].y;
    const double AB[3] = {a.pair_AB[3 * bra], a.pair_AB[3 * bra + 1], a.pair_AB[3 * bra + 2]};
    const double CD[3] = {a.pair_AB[3 * ket], a.pair_AB[3 * ket + 1], a.pair_AB[3 * ket + 2]};
    for (int it = lane; it < NAB; it += 64) {
        const int ia = it / NB, ib = it % NB;
        const int ax[3] = {fk::kCart.x[LA][ia], fk::kCart.y[LA][ia], fk::kCart.z[LA][ia]};
        const int bx[3] = {fk::kCart.x[LB][ib], fk::kCart.y[LB][ib], fk::kCart.z[LB][ib]};
        double acc[NCD];
#pragma unroll
        for (int o = 0; o < NCD; ++o) acc[o] = 0.0;
        for (int i = 0; i < a.pair_npp[bra]; ++i) {
            const fk::PrimPair p = load_pp(a.pp, a.pair_ppoff[bra] + i);
            for (int j = 0; j < a.pair_npp[ket]; ++j)
                fk::rys_prim_bra_comp<LA, LB, LC, LD>(s_tab, p, load_pp(a.pp, a.pair_ppoff[ket] + j), AB, CD, ax, bx,
                                                      acc);
        }
#pragma unroll
        for (int o = 0; o < NCD; ++o) a.out[(size_t)q * Q::NOUT + it * NCD + o] = acc[o];
    }
}

template <int LA, int LB, int LC, int LD, int MODE>
__global__ void __launch_bounds__(FK_BLOCK) k_debug_tpq(FkDebugArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    constexpr int NB = Q::NB, NC = Q::NC, ND = Q::ND;
    constexpr int TS = (MODE == 1) ? Q::NA : Q::NA * Q::NB;
    constexpr int QPW = 64 / TS;
    constexpr int NBL = (MODE == 1) ? NB : 1;
    __shared__ double s_tab[rys_lds_size(Q::NR)];
    load_table<Q::NR>(s_tab, a.rys_tab);
    const int lane = threadIdx.x & 63;
    const int slot = lane / TS, comp = lane % TS;
    const int q = (blockIdx.x * FK_WAVES + (threadIdx.x >> 6)) * QPW + slot;
    if (slot >= QPW || q >= a.nq) return;
    const int ia = (MODE == 1) ? comp : comp / NB;
    const int ib0 = (MODE == 1) ? 0 : comp % NB;
    const int ax[3] = {fk::kCart.x[LA][ia], fk::kCart.y[LA][ia], fk::kCart.z[LA][ia]};
    const int bx[3] = {fk::kCart.x[LB][ib0], fk::kCart.y[LB][ib0], fk::kCart.z[LB][ib0]};
    const int bra = a.quartets[q].x, ket = a.quartets[q].y;
    const double AB[3] = {a.pair_AB[3 * bra], a.pair_AB[3 * bra + 1], a.pair_AB[3 * bra + 2]};
    const double CD[3] = {a.pair_AB[3 * ket], a.pair_AB[3 * ket + 1], a.pair_AB[3 * ket + 2]};
    double acc[NBL * NC * ND];
#pragma unroll
    for (int o = 0; o < NBL * NC * ND; ++o) acc[o] = 0.0;
    for (int i = 0; i < a.pair_npp[bra]; ++i) {
        const fk::PrimPair p = load_pp(a.pp, a.pair_ppoff[bra] + i);
        for (int j = 0; j < a.pair_npp[ket]; ++j)
            fk::rys_prim_team<LA, LB, LC, LD, MODE>(s_tab, p, load_pp(a.pp, a.pair_ppoff[ket] + j), AB, CD, ax, bx, acc);
    }
#pragma unroll
    for (int jb = 0; jb < NBL; ++jb) {
        const int ib = (MODE == 1) ? jb : ib0;
#pragma unroll
        for (int o = 0; o < NC * ND; ++o)
            a.out[(size_t)q * Q::NOUT + (ia * NB + ib) * NC * ND + o] = acc[jb * NC * ND + o];
    }
}

// Raw contracted integrals by the HGP engine, one lane per quartet.
template <int LA, int LB, int LC, int LD>
__global__ void __launch_bounds__(FK_BLOCK) k_debug_hgp(FkDebugArgs a)
{
    using Q = fk::QClass<LA, LB, LC, LD>;
    using H = fk::HgpClass<LA, LB, LC, LD>;
    __shared__ double s_tab[rys_lds_size(Q::NR)];
    load_table<Q::NR>(s_tab, a.rys_tab);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int bra = a.quartets[q].x, ket = a.quartets[q].y;
    const double AB[3] = {a.pair_AB[3 * bra], a.pair_AB[3 * bra + 1], a.pair_AB[3 * bra + 2]};
    const double CD[3] = {a.pair_AB[3 * ket], a.pair_AB[3 * ket + 1], a.pair_AB[3 * ket + 2]};
    double acce[H::NACC];
#pragma unroll
    for (int o = 0; o < H::NACC; ++o) acce[o] = 0.0;
    for (int i = 0; i < a.pair_npp[bra]; ++i) {
        const fk::PrimPair p = load_pp(a.pp, a.pair_ppoff[bra] + i);
        for (int j = 0; j < a.pair_npp[ket]; ++j)
            fk::hgp_prim<LA, LB, LC, LD>(s_tab, p, load_pp(a.pp, a.pair_ppoff[ket] + j), acce);
    }
    double out[Q::NOUT];
    fk::hgp_hrr<LA, LB, LC, LD>(acce, AB, CD, out);
#pragma unroll
    for (int o = 0; o < Q::NOUT; ++o) a.out[(size_t)q * Q::NOUT + o] = out[o];
}

// --------------------------------------------------------- dispatch ------
template <int P, int Q>
struct Disp {
    static constexpr int LA = pair_la(P), LB = pair_lb(P), LC = pair_la(Q), LD = pair_lb(Q);
    static constexpr bool BUILT = LA <= FK_BUILD_MAXL;
    static constexpr int KIND = kernel_kind<LA, LB, LC, LD>();
    static constexpr bool WPQ = KIND == 3;
    // classes the HGP engine is built for: lane-per-quartet kernels up to L = 4
    static constexpr bool HGP = KIND == 0 && LA + LB + LC + LD <= FK_HGP_MAX_L;
    // lane classes with a team-per-quartet alternative (MODE 1: a lane per a component)
    static constexpr bool ALT = KIND == 0 && fk::QClass<LA, LB, LC, LD>::NOUT >= FK_ALT_MIN_NOUT &&
                                fk::QClass<LA, LB, LC, LD>::NA >= 3;
    // lane classes also built with workgroups of eight waves (Rys engine)
    static constexpr bool WIDE = KIND == 0 && LpqWide<LA, LB, LC, LD>::value;
    static void info(FkClassInfo *i)
    {
        using C = fk::QClass<LA, LB, LC, LD>;
        i->la = LA; i->lb = LB; i->lc = LC; i->ld = LD;
        i->nroot = C::NR; i->nout = C::NOUT;
        i->wave_per_quartet = KIND;
        // largest bra block the kernel takes (1: one bra per tile)
        constexpr int NBK = KIND == 0 ? LpqKetOuter<LA, LB, LC, LD>::value : 0;
        i->bra_block = NBK > 0 ? NBK
                       : (KIND == 0 && C::NOUT <= FK_LPQ_BLOCK_NOUT) ? FK_MAX_BRA_BLOCK
                       : ((KIND == 1 || KIND == 2) ? FK_TEAM_MAX_BLOCK : 1);
        i->team_size = KIND == 0 ? 1 : (KIND == 1 ? C::NA : (KIND == 2 ? C::NA * C::NB : 64 * WpqSplit<LA, LB, LC, LD>::value));
        i->ket_outer = NBK;
        i->alt_team = ALT ? C::NA : 0;
        i->alt_bra_block = ALT ? FK_TEAM_MAX_BLOCK : 0;
        i->wide = WIDE ? 2 * FK_WAVES : 0;
        i->flops_prim = fk::flops_prim(LA, LB, LC, LD);
        i->flops_quartet = fk::flops_digest(LA, LB, LC, LD);
        i->hgp = HGP ? 1 : 0;
        i->flops_prim_hgp = HGP ? fk::hgp_flops_prim(LA, LB, LC, LD) : 0.0;
        i->flops_quartet_hgp = HGP ? fk::hgp_flops_hrr(LA, LB, LC, LD) + fk::flops_digest(LA, LB, LC, LD) : 0.0;
    }
    static const void *jk_kernel(bool low = false, int eng = 0, int kind = KIND, int nw = FK_WAVES)
    {
        if constexpr (!BUILT) return nullptr;
        else if constexpr (WIDE) {
            if (nw == 2 * FK_WAVES && kind == 0 && eng == 0)
                return low ? (const void *)&k_jk_lpq<LA, LB, LC, LD, float, 0, 2 * FK_WAVES>
                           : (const void *)&k_jk_lpq<LA, LB, LC, LD, double, 0, 2 * FK_WAVES>;
        }
        if constexpr (!BUILT) return nullptr;
        else if constexpr (ALT) {
            if (kind == 1)
                return low ? (const void *)&k_jk_tpq<LA, LB, LC, LD, 1, float>
                           : (const void *)&k_jk_tpq<LA, LB, LC, LD, 1, double>;
        }
        if constexpr (!BUILT) return nullptr;
        else if constexpr (HGP) {
            if (eng == 1)
                return low ? (const void *)&k_jk_lpq<LA, LB, LC, LD, float, 1>
                           : (const void *)&k_jk_lpq<LA, LB, LC, LD, double, 1>;
            return low ? (const void *)&k_jk_lpq<LA, LB, LC, LD, float> : (const void *)&k_jk_lpq<LA, LB, LC, LD, double>;
        } else if constexpr (KIND == 0)
            return low ? (const void *)&k_jk_lpq<LA, LB, LC, LD, float> : (const void *)&k_jk_lpq<LA, LB, LC, LD, double>;
        else if constexpr (KIND == 1 || KIND == 2)
            return low ? (const void *)&k_jk_tpq<LA, LB, LC, LD, KIND, float>
                       : (const void *)&k_jk_tpq<LA, LB, LC, LD, KIND, double>;
        else return (const void *)&k_jk_wpq<LA, LB, LC, LD>;
    }
    static int lds_bytes(int bra_slot, int krow_ncol, int kind = KIND, int nbk = 0, int nw = FK_WAVES)
    {
        if constexpr (ALT) {
            if (kind == 1)
                return (int)sizeof(double) *
                       (rys_lds_size(fk::QClass<LA, LB, LC, LD>::NR) + FK_WAVES * TeamShape<LA, LB, LC, LD, 1>::RED);
        }
        // the Rys segment, and per wave the team reductions (bra records are
        // read from memory by scalar loads: bra_slot needs no LDS); block
        // tasks add the block's K rows and X_J[a, b_j]
        (void)bra_slot;
        using C = fk::QClass<LA, LB, LC, LD>;
        int extra = 0, rows = 0;
        if constexpr (KIND == 0)
            extra = krow_ncol > 0 ? LpqStageTask<LA, LB, LC, LD>::value : LpqStage<LA, LB, LC, LD>::value;
        if constexpr (KIND == 1 || KIND == 2) extra = TeamShape<LA, LB, LC, LD, KIND>::RED;
        if constexpr (KIND == 0) {
            if (krow_ncol > 0) rows = (nbk * C::NB + C::NA) * krow_ncol + nbk * C::NA * C::NB;
        }
        return (int)sizeof(double) * (rys_lds_size(C::NR) + nw * extra + rows);
    }
    static int launch_jk(const FkJKArgs *a, int grid, hipStream_t st)
    {
        if constexpr (!BUILT) return -2;
        else {
            const int lds = lds_bytes(a->bra_slot, a->ntask > 0 ? a->krow_ncol : 0, a->kind, a->krow_nbk, a->nw);
            const bool low = a->prec == 1;
            const int eng = a->engine;
            if (a->kind != KIND && !(ALT && a->kind == 1)) return -2;
            if (a->nw != FK_WAVES && !(WIDE && a->nw == 2 * FK_WAVES && a->kind == 0 && eng == 0)) return -2;
            if constexpr (WIDE) {
                if (a->nw == 2 * FK_WAVES) {
                    const void *kw = jk_kernel(low, 0, 0, a->nw);
                    static int raised_w[2] = {0, 0};
                    if (lds > 65536 && lds > raised_w[low]) {
                        if (hipFuncSetAttribute(kw, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -3;
                        raised_w[low] = lds;
                    }
                    if (low)
                        hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, float, 0, 2 * FK_WAVES>), dim3(grid),
                                           dim3(128 * FK_WAVES), lds, st, *a);
                    else
                        hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, double, 0, 2 * FK_WAVES>), dim3(grid),
                                           dim3(128 * FK_WAVES), lds, st, *a);
                    return hipGetLastError() == hipSuccess ? 0 : -3;
                }
            }
            if constexpr (ALT) {
                if (a->kind == 1) {
                    if (eng != 0) return -2;
                    const void *kt = jk_kernel(low, 0, 1);
                    static int raised_t[2] = {0, 0};
                    if (lds > 65536 && lds > raised_t[low]) {
                        if (hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -3;
                        raised_t[low] = lds;
                    }
                    if (low) hipLaunchKernelGGL((k_jk_tpq<LA, LB, LC, LD, 1, float>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                    else hipLaunchKernelGGL((k_jk_tpq<LA, LB, LC, LD, 1, double>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                    return hipGetLastError() == hipSuccess ? 0 : -3;
                }
            }
            if (low && KIND == 3) return -2;  // f-f bras: FP64 only
            if (eng != 0 && !HGP) return -2;  // HGP only for the classes it is built for
            const void *k = jk_kernel(low, eng);
            static int raised[2][2] = {{0, 0}, {0, 0}};
            if (lds > 65536 && lds > raised[low][eng]) {
                if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -3;
                raised[low][eng] = lds;
            }
            if constexpr (HGP) {
                if (eng == 1) {
                    if (low) hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, float, 1>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                    else hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, double, 1>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                    return hipGetLastError() == hipSuccess ? 0 : -3;
                }
            }
            if constexpr (KIND == 0) {
                if (low) hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, float>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                else hipLaunchKernelGGL((k_jk_lpq<LA, LB, LC, LD, double>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
            } else if constexpr (KIND == 1 || KIND == 2) {
                if (low) hipLaunchKernelGGL((k_jk_tpq<LA, LB, LC, LD, KIND, float>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
                else hipLaunchKernelGGL((k_jk_tpq<LA, LB, LC, LD, KIND, double>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
            } else {
                hipLaunchKernelGGL((k_jk_wpq<LA, LB, LC, LD>), dim3(grid), dim3(FK_BLOCK), lds, st, *a);
            }
            return hipGetLastError() == hipSuccess ? 0 : -3;
        }
    }
    static int launch_debug(const FkDebugArgs *a, hipStream_t st)
    {
        if constexpr (!BUILT) return -2;
        else {
            if (a->nq <= 0) return 0;
            if (a->engine != 0) {
                if constexpr (HGP) {
                    const int grid = (a->nq + FK_BLOCK - 1) / FK_BLOCK;
                    hipLaunchKernelGGL((k_debug_hgp<LA, LB, LC, LD>), dim3(grid), dim3(FK_BLOCK), 0, st, *a);
                    return hipGetLastError() == hipSuccess ? 0 : -3;
                } else {
                    return -2;
                }
            }
            if constexpr (KIND == 3) {
                const int grid = (a->nq + FK_WAVES - 1) / FK_WAVES;
                hipLaunchKernelGGL((k_debug_wpq<LA, LB, LC, LD>), dim3(grid), dim3(FK_BLOCK), 0, st, *a);
            } else if constexpr (KIND == 1 || KIND == 2) {
                using C = fk::QClass<LA, LB, LC, LD>;
                constexpr int TS = (KIND == 1) ? C::NA : C::NA * C::NB;
                constexpr int QPB = (64 / TS) * FK_WAVES;
                const int grid = (a->nq + QPB - 1) / QPB;
                hipLaunchKernelGGL((k_debug_tpq<LA, LB, LC, LD, KIND>), dim3(grid), dim3(FK_BLOCK), 0, st, *a);
            } else {
                const int grid = (a->nq + FK_BLOCK - 1) / FK_BLOCK;
                hipLaunchKernelGGL((k_debug_lpq<LA, LB, LC, LD>), dim3(grid), dim3(FK_BLOCK), 0, st, *a);
            }
            return hipGetLastError() == hipSuccess ? 0 : -3;
        }
    }
    static int debug_host(const int *ppoff, const int *npp, const double *AB, const double *pp, const int *qs,
                          int nq, double *out, int eng)
    {
        if constexpr (!BUILT) return -2;
        else {
        using C = fk::QClass<LA, LB, LC, LD>;
        const double *tab = rys_staged_host() + rys_staged_offset(C::NR);
        auto ld = [&](int idx) {
            const double *r = pp + (size_t)idx * FK_NPP_REC;
            fk::PrimPair p;
            p.zeta = r[0]; p.oo2z = r[1];
            for (int k = 0; k < 3; ++k) { p.P[k] = r[2 + k]; p.PA[k] = r[5 + k]; }
            p.K = r[8];
            return p;
        };
        if (eng == 2) {
            // the McMurchie-Davidson pieces of the J engine (E and R), host only
            if constexpr (LA + LB + LC + LD <= 8) {
                for (int q = 0; q < nq; ++q) {
                    const int bra = qs[2 * q], ket = qs[2 * q + 1];
                    double *o = out + (size_t)q * C::NOUT;
                    for (int k = 0; k < C::NOUT; ++k) o[k] = 0.0;
                    for (int i = 0; i < npp[bra]; ++i)
                        for (int j = 0; j < npp[ket]; ++j)
                            fk::mmd_prim_all<LA, LB, LC, LD>(tab, ld(ppoff[bra] + i), ld(ppoff[ket] + j), AB + 3 * bra,
                                                             AB + 3 * ket, o);
                }
                return 0;
            } else {
                return -2;
            }
        }
        if (eng != 0) {
            if constexpr (HGP) {
                using H = fk::HgpClass<LA, LB, LC, LD>;
                for (int q = 0; q < nq; ++q) {
                    const int bra = qs[2 * q], ket = qs[2 * q + 1];
                    double acce[H::NACC] = {};
                    for (int i = 0; i < npp[bra]; ++i)
                        for (int j = 0; j < npp[ket]; ++j)
                            fk::hgp_prim<LA, LB, LC, LD>(tab, ld(ppoff[bra] + i), ld(ppoff[ket] + j), acce);
                    fk::hgp_hrr<LA, LB, LC, LD>(acce, AB + 3 * bra, AB + 3 * ket, out + (size_t)q * C::NOUT);
                }
                return 0;
            } else {
                return -2;
            }
        }
        for (int q = 0; q < nq; ++q) {
            const int bra = qs[2 * q], ket = qs[2 * q + 1];
            double *o = out + (size_t)q * C::NOUT;
            for (int x = 0; x < C::NOUT; ++x) o[x] = 0.0;
            for (int i = 0; i < npp[bra]; ++i)
                for (int j = 0; j < npp[ket]; ++j) {
                    const fk::PrimPair p = ld(ppoff[bra] + i), qq = ld(ppoff[ket] + j);
                    if constexpr (KIND == 1 || KIND == 2) {
                        constexpr int TS = (KIND == 1) ? C::NA : C::NA * C::NB;
                        constexpr int NBL = (KIND == 1) ? C::NB : 1;
                        for (int comp = 0; comp < TS; ++comp) {
                            const int ia = (KIND == 1) ? comp : comp / C::NB;
                            const int ib0 = (KIND == 1) ? 0 : comp % C::NB;
                            const int ax[3] = {fk::kCart.x[LA][ia], fk::kCart.y[LA][ia], fk::kCart.z[LA][ia]};
                            const int bx[3] = {fk::kCart.x[LB][ib0], fk::kCart.y[LB][ib0], fk::kCart.z[LB][ib0]};
                            double tmp[NBL * C::NC * C::ND] = {};
                            fk::rys_prim_team<LA, LB, LC, LD, KIND>(tab, p, qq, AB + 3 * bra, AB + 3 * ket, ax, bx, tmp);
                            for (int jb = 0; jb < NBL; ++jb) {
                                const int ib = (KIND == 1) ? jb : ib0;
                                for (int x = 0; x < C::NC * C::ND; ++x)
                                    o[(ia * C::NB + ib) * C::NC * C::ND + x] += tmp[jb * C::NC * C::ND + x];
                            }
                        }
                    } else if constexpr (WPQ) {
                        for (int it = 0; it < C::NA * C::NB; ++it) {
                            const int ia = it / C::NB, ib = it % C::NB;
                            const int ax[3] = {fk::kCart.x[LA][ia], fk::kCart.y[LA][ia], fk::kCart.z[LA][ia]};
                            const int bx[3] = {fk::kCart.x[LB][ib], fk::kCart.y[LB][ib], fk::kCart.z[LB][ib]};
                            fk::rys_prim_bra_comp<LA, LB, LC, LD>(tab, p, qq, AB + 3 * bra, AB + 3 * ket, ax, bx,
                                                                  o + it * C::NC * C::ND);
                        }
                    } else {
                        fk::rys_prim_all<LA, LB, LC, LD>(tab, p, qq, AB + 3 * bra, AB + 3 * ket, o);
                    }
                }
        }
        return 0;
        }
    }
};


#define FK_CAT2(a, b, c) a##b##c
#define FK_CAT(a, b, c) FK_CAT2(a, b, c)

template <int P, int Q = 0>
int info_q(int q, FkClassInfo *i)
{
    if constexpr (Q > P) return -1;
    else {
        if (q == Q) { Disp<P, Q>::info(i); return Disp<P, Q>::BUILT ? 0 : -2; }
        return info_q<P, Q + 1>(q, i);
    }
}
template <int P, int Q = 0>
int jk_q(int q, const FkJKArgs *a, int grid, hipStream_t st)
{
    if constexpr (Q > P) return -1;
    else return q == Q ? Disp<P, Q>::launch_jk(a, grid, st) : jk_q<P, Q + 1>(q, a, grid, st);
}
template <int P, int Q = 0>
int dbg_q(int q, const FkDebugArgs *a, hipStream_t st)
{
    if constexpr (Q > P) return -1;
    else return q == Q ? Disp<P, Q>::launch_debug(a, st) : dbg_q<P, Q + 1>(q, a, st);
}
template <int P, int Q = 0>
int host_q(int q, const int *o, const int *n, const double *ab, const double *pp, const int *qs, int nq, double *out,
           int eng)
{
    if constexpr (Q > P) return -1;
    else
        return q == Q ? Disp<P, Q>::debug_host(o, n, ab, pp, qs, nq, out, eng)
                      : host_q<P, Q + 1>(q, o, n, ab, pp, qs, nq, out, eng);
}
template <int P, int Q = 0>
int lds_q(int q, int slot, int ncol, int kind, int nbk, int nw)
{
    if constexpr (Q > P) return -1;
    else
        return q == Q ? Disp<P, Q>::lds_bytes(slot, ncol, kind, nbk, nw)
                      : lds_q<P, Q + 1>(q, slot, ncol, kind, nbk, nw);
}
template <int P, int Q = 0>
const void *kern_q(int q, int eng, int kind, int nw)
{
    if constexpr (Q > P) return nullptr;
    else {
        if (q == Q) {
            if (eng != 0 && !Disp<P, Q>::HGP) return nullptr;
            if (kind != Disp<P, Q>::KIND && !(Disp<P, Q>::ALT && kind == 1)) return nullptr;
            if (nw != FK_WAVES && !(Disp<P, Q>::WIDE && nw == 2 * FK_WAVES && kind == 0 && eng == 0)) return nullptr;
            return Disp<P, Q>::jk_kernel(false, eng, kind, nw);
        }
        return kern_q<P, Q + 1>(q, eng, kind, nw);
    }
}

}  // namespace

#if FK_ONLY_P == -2
// ---- J engine translation unit (paper, "J matrix implementation") ----
// Per build: D_q = sum_cd E^{cd}_q D_cd per ket primitive pair (k_jeng_dq),
// J_p = sum_q [p|q] D_q per bra primitive pair over the Schwarz- and
// density-screened kets (k_jeng_jp), J_ab = sum_p E^{ab}_p J_p contracted over
// the bra primitives (k_jeng_jab).  Bra-ket symmetry is not used (every bra
// takes all its kets, as the paper's J kernels do), so no J_cd digestion.
namespace {

// D_q of every primitive pair of one ket class: one thread per list position.
template <int LC, int LD>
__global__ void __launch_bounds__(256) k_jeng_dq(FkJengDqArgs a)
{
    constexpr int LQ = LC + LD, NHQ = fk::nherm(LQ), NC = fk::ncart(LC), ND = fk::ncart(LD);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.npos) return;
    const int pos = a.pos0 + idx;
    const FkGroup g = a.groups[a.pos_grp[pos]];
    const int r = pos - g.begin;
    const int sc = a.lst_sa[pos], sd = a.lst_sb[pos];
    const int oc = a.sh_bf[sc], od = a.sh_bf[sd];
    const double CD[3] = {a.lst_CD[pos], a.lst_CD[a.nlist + pos], a.lst_CD[2 * a.nlist + pos]};
    // both orders (c, d) and (d, c) of a pair of distinct shells contribute
    const double fac = sc == sd ? 1.0 : 2.0;
    double dcd[NC * ND];
#pragma unroll
    for (int ic = 0; ic < NC; ++ic)
#pragma unroll
        for (int id = 0; id < ND; ++id) dcd[ic * ND + id] = fac * a.Ds[(size_t)(oc + ic) * a.n + od + id];
    double *out = a.dq + a.dq_base[a.pos_grp[pos]] + r;
    for (int j = 0; j < g.npp; ++j) {
        const fk::PrimPair q = load_ket_pp(a.ppT, g, j, r);
        double E[3][LC + 1][LD + 1][LQ + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) fk::mmd_e1<LC, LD>(q.oo2z, q.PA[k], q.PA[k] + CD[k], E[k]);
#pragma unroll
        for (int h = 0; h < NHQ; ++h) {
            const int t = fk::kComp.x[h], u = fk::kComp.y[h], v = fk::kComp.z[h];
            double s = 0.0;
#pragma unroll
            for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                for (int id = 0; id < ND; ++id) {
                    const int cx = fk::kCart.x[LC][ic], cy = fk::kCart.y[LC][ic], cz = fk::kCart.z[LC][ic];
                    const int dx = fk::kCart.x[LD][id], dy = fk::kCart.y[LD][id], dz = fk::kCart.z[LD][id];
                    if (t > cx + dx || u > cy + dy || v > cz + dz) continue;
                    s += E[0][cx][dx][t] * E[1][cy][dy][u] * E[2][cz][dz][v] * dcd[ic * ND + id];
                }
            out[((size_t)j * NHQ + h) * g.len] = s;
        }
    }
}

// J_p of the bra primitive pairs: one wave per tile (bra, <= 64 kets), lane =
// ket; per bra primitive the lanes' sums over their kets' primitives are
// reduced over the wave and added to J_p.
template <int LP, int LQ>
__global__ void __launch_bounds__(FK_BLOCK) k_jeng_jp(FkJengArgs a)
{
    constexpr int L = LP + LQ, NR = L / 2 + 1;
    constexpr int NHP = fk::nherm(LP), NHQ = fk::nherm(LQ), NHR = fk::nherm(L);
    __shared__ double s_tab[rys_lds_size(NR)];
    load_table<NR>(s_tab, a.rys_tab);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long nwt = (long long)gridDim.x * FK_WAVES;
    for (long long t = (long long)blockIdx.x * FK_WAVES + wave; t < a.ntiles; t += nwt) {
        const FkJengTile tile = a.tiles[t];
        const FkGroup g = a.groups[tile.grp];
        const bool inrange = lane < tile.ket_count;
        const int pos = tile.ket_begin + (inrange ? lane : 0);
        const int r = pos - g.begin;
        const double gg = a.pair_G[tile.bra] * a.lst_G[pos];
        bool active = inrange && (a.tau <= 0 || gg >= a.tau);
        if (a.dscreen) active = active && gg * a.Dsh[a.lst_sa[pos] * a.ns + a.lst_sb[pos]] >= a.tau;
        if (__ballot(active) == 0ull) continue;
        const int ppo = __builtin_amdgcn_readfirstlane(a.pair_ppoff[tile.bra]);
        const int bnpp = __builtin_amdgcn_readfirstlane(a.pair_npp[tile.bra]);
        const long long jo = a.jp_off[tile.bra];
        const double *__restrict dqp = a.dq + a.dq_base[tile.grp] + r;
        for (int i = 0; i < bnpp; ++i) {
            const fk::PrimPair p = sload_pp(a.pp, ppo + i);
            double jp[NHP];
#pragma unroll
            for (int h = 0; h < NHP; ++h) jp[h] = 0.0;
            if (active) {
                for (int j = 0; j < g.npp; ++j) {
                    const fk::PrimPair q = load_ket_pp(a.ppT, g, j, r);
                    double dq[NHQ];
#pragma unroll
                    for (int h = 0; h < NHQ; ++h) dq[h] = dqp[((size_t)j * NHQ + h) * g.len];
                    const fk::QuartetSetup s = fk::quartet_setup(p, q);
                    double R[NHR];
                    fk::mmd_r<L>(s_tab, s, p.zeta * q.zeta * s.inv, R);
#pragma unroll
                    for (int hp = 0; hp < NHP; ++hp)
#pragma unroll
                        for (int hq = 0; hq < NHQ; ++hq) {
                            const int tx = fk::kComp.x[hp] + fk::kComp.x[hq];
                            const int ty = fk::kComp.y[hp] + fk::kComp.y[hq];
                            const int tz = fk::kComp.z[hp] + fk::kComp.z[hq];
                            const double v = R[fk::cidx(tx, ty, tz)] * dq[hq];
                            // [p|q] = (-1)^{|q|} R_{p+q}
                            if ((fk::kComp.x[hq] + fk::kComp.y[hq] + fk::kComp.z[hq]) & 1) jp[hp] -= v;
                            else jp[hp] += v;
                        }
                }
            }
#pragma unroll
            for (int h = 0; h < NHP; ++h) {
                const double sum = wave_sum(jp[h]);
                if (lane == 0 && sum != 0.0) atomic_add(&a.jp[jo + (long long)i * NHP + h], sum);
            }
        }
    }
}

// J_ab of every pair of one bra class: one thread per pair, its block of X_J
// (a full block for two distinct shells, half a block for a shell with itself:
// J = X_J + X_J^T then restores both).
template <int LA, int LB>
__global__ void __launch_bounds__(256) k_jeng_jab(FkJengJabArgs a)
{
    constexpr int LP = LA + LB, NHP = fk::nherm(LP), NA = fk::ncart(LA), NB = fk::ncart(LB);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.npairs) return;
    const int pr = a.pairs[idx];
    const int sa = a.pair_sa[pr], sb = a.pair_sb[pr];
    const int oa = a.sh_bf[sa], ob = a.sh_bf[sb];
    const double AB[3] = {a.pair_AB[3 * pr], a.pair_AB[3 * pr + 1], a.pair_AB[3 * pr + 2]};
    const long long jo = a.jp_off[pr];
    double acc[NA * NB];
#pragma unroll
    for (int o = 0; o < NA * NB; ++o) acc[o] = 0.0;
    for (int i = 0; i < a.pair_npp[pr]; ++i) {
        const fk::PrimPair p = load_pp(a.pp, a.pair_ppoff[pr] + i);
        double E[3][LA + 1][LB + 1][LP + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) fk::mmd_e1<LA, LB>(p.oo2z, p.PA[k], p.PA[k] + AB[k], E[k]);
        double jv[NHP];
#pragma unroll
        for (int h = 0; h < NHP; ++h) jv[h] = a.jp[jo + (long long)i * NHP + h];
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                const int ax = fk::kCart.x[LA][ia], ay = fk::kCart.y[LA][ia], az = fk::kCart.z[LA][ia];
                const int bx = fk::kCart.x[LB][ib], by = fk::kCart.y[LB][ib], bz = fk::kCart.z[LB][ib];
                double s = 0.0;
#pragma unroll
                for (int h = 0; h < NHP; ++h) {
                    const int t = fk::kComp.x[h], u = fk::kComp.y[h], v = fk::kComp.z[h];
                    if (t > ax + bx || u > ay + by || v > az + bz) continue;
                    s += E[0][ax][bx][t] * E[1][ay][by][u] * E[2][az][bz][v] * jv[h];
                }
                acc[ia * NB + ib] += s;
            }
    }
    const double fac = sa == sb ? 0.5 : 1.0;
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) a.XJ[(size_t)(oa + ia) * a.n + ob + ib] = fac * acc[ia * NB + ib];
}

template <int LC, int LD>
int launch_dq(const FkJengDqArgs *a, hipStream_t st)
{
    if (a->npos <= 0) return 0;
    hipLaunchKernelGGL((k_jeng_dq<LC, LD>), dim3((a->npos + 255) / 256), dim3(256), 0, st, *a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
template <int LP, int LQ>
int launch_jp(const FkJengArgs *a, int grid, hipStream_t st)
{
    if (a->ntiles <= 0) return 0;
    hipLaunchKernelGGL((k_jeng_jp<LP, LQ>), dim3(grid), dim3(FK_BLOCK), 0, st, *a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
template <int LA, int LB>
int launch_jab(const FkJengJabArgs *a, hipStream_t st)
{
    if (a->npairs <= 0) return 0;
    hipLaunchKernelGGL((k_jeng_jab<LA, LB>), dim3((a->npairs + 255) / 256), dim3(256), 0, st, *a);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
template <int LP, int LQ = 0>
int jp_q(int lq, const FkJengArgs *a, int grid, hipStream_t st)
{
    if constexpr (LQ > FK_JENG_MAX_LP) return -2;
    else return lq == LQ ? launch_jp<LP, LQ>(a, grid, st) : jp_q<LP, LQ + 1>(lq, a, grid, st);
}

}  // namespace

extern "C" {
// pair classes (l1 >= l2) up to d
int fk_jeng_launch_dq(int lc, int ld, const FkJengDqArgs *a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (lc * 3 + ld) {
    case 0: return launch_dq<0, 0>(a, st);
    case 3: return launch_dq<1, 0>(a, st);
    case 4: return launch_dq<1, 1>(a, st);
    case 6: return launch_dq<2, 0>(a, st);
    case 7: return launch_dq<2, 1>(a, st);
    case 8: return launch_dq<2, 2>(a, st);
    default: return -2;
    }
}
int fk_jeng_launch_jab(int la, int lb, const FkJengJabArgs *a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (la * 3 + lb) {
    case 0: return launch_jab<0, 0>(a, st);
    case 3: return launch_jab<1, 0>(a, st);
    case 4: return launch_jab<1, 1>(a, st);
    case 6: return launch_jab<2, 0>(a, st);
    case 7: return launch_jab<2, 1>(a, st);
    case 8: return launch_jab<2, 2>(a, st);
    default: return -2;
    }
}
int fk_jeng_launch_jp(int LP, int LQ, const FkJengArgs *a, int grid, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (LP) {
    case 0: return jp_q<0>(LQ, a, grid, st);
    case 1: return jp_q<1>(LQ, a, grid, st);
    case 2: return jp_q<2>(LQ, a, grid, st);
    case 3: return jp_q<3>(LQ, a, grid, st);
    case 4: return jp_q<4>(LQ, a, grid, st);
    default: return -2;
    }
}
}
#elif FK_ONLY_P >= 0
// ---- per bra-class translation unit ----
extern "C" {
int FK_CAT(fk_kp, FK_ONLY_P, _info)(int Q, FkClassInfo *i) { return info_q<FK_ONLY_P>(Q, i); }
int FK_CAT(fk_kp, FK_ONLY_P, _jk)(int Q, const FkJKArgs *a, int grid, void *st)
{
    return jk_q<FK_ONLY_P>(Q, a, grid, (hipStream_t)st);
}
int FK_CAT(fk_kp, FK_ONLY_P, _dbg)(int Q, const FkDebugArgs *a, void *st) { return dbg_q<FK_ONLY_P>(Q, a, (hipStream_t)st); }
int FK_CAT(fk_kp, FK_ONLY_P, _host)(int Q, const int *o, const int *n, const double *ab, const double *pp,
                                      const int *qs, int nq, double *out, int eng)
{
    return host_q<FK_ONLY_P>(Q, o, n, ab, pp, qs, nq, out, eng);
}
const void *FK_CAT(fk_kp, FK_ONLY_P, _kern)(int Q, int eng, int kind, int nw)
{
    return kern_q<FK_ONLY_P>(Q, eng, kind, nw);
}
int FK_CAT(fk_kp, FK_ONLY_P, _lds)(int Q, int slot, int ncol, int kind, int nbk, int nw)
{
    return lds_q<FK_ONLY_P>(Q, slot, ncol, kind, nbk, nw);
}
}
#else
// ---- common translation unit: small kernels and the dispatch tables ----
namespace {
// ------------------------------------------------------ small kernels ----
__global__ void k_fill(double *p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// molecule m with base[m] <= i < base[m + 1] (base has nmol + 1 entries)
__device__ __forceinline__ int find_mol(const long long *__restrict base, int nmol, long long i)
{
    int lo = 0, hi = nmol;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Ds = s_r s_c D over every molecule's block
__global__ void k_prep_ds(const double *__restrict D, const double *__restrict s, FkMolArgs m, double *__restrict Ds)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.nmat) return;
    const int k = find_mol(m.mol_base, m.nmol, i);
    const long long loc = i - m.mol_base[k];
    const int n = m.mol_nbf[k], f0 = m.mol_bf0[k];
    const int r = (int)(loc / n), c = (int)(loc % n);
    Ds[i] = s[f0 + r] * s[f0 + c] * D[i];
}

// D_sh[A, B] = max |D| over the shell block, per molecule
__global__ void k_prep_dsh(const double *__restrict D, FkMolArgs m, double *__restrict Dsh)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.nshmat) return;
    const int k = find_mol(m.mol_shbase, m.nmol, i);
    const long long loc = i - m.mol_shbase[k];
    const int ns = m.mol_nsh[k], n = m.mol_nbf[k];
    const int A = m.mol_sh0[k] + (int)(loc / ns), B = m.mol_sh0[k] + (int)(loc % ns);
    const double *Dm = D + m.mol_base[k];
    double v = 0.0;
    for (int r = m.sh_lbf[A]; r < m.sh_lend[A]; ++r)
        for (int c = m.sh_lbf[B]; c < m.sh_lend[B]; ++c) v = fmax(v, fabs(Dm[(size_t)r * n + c]));
    Dsh[i] = v;
}

// Density-decay fit (paper, "K matrix implementation"): the largest |D_ij|
// per bin of the distance between the functions' atoms, atoms differing
// (same-atom elements are never screened and would skew the decay); bins of
// width dr, the last one open-ended.  Non-negative doubles order like their
// bit patterns, so the maximum is an integer atomic.
__global__ void k_dfit_bins(const double *__restrict D, int n, const int *__restrict bf_atom,
                            const double *__restrict xyz, double dr, unsigned long long *__restrict bins)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    const int r = (int)(i / n), c = (int)(i % n);
    const int A = bf_atom[r], B = bf_atom[c];
    if (A == B) return;
    const double dx = xyz[3 * A] - xyz[3 * B], dy = xyz[3 * A + 1] - xyz[3 * B + 1], dz = xyz[3 * A + 2] - xyz[3 * B + 2];
    const int b = min(FK_DFIT_BINS - 1, (int)(sqrt(dx * dx + dy * dy + dz * dz) / dr));
    const double v = fabs(D[i]);
    if (v > 0) atomicMax(&bins[b], (unsigned long long)__double_as_longlong(v));
}

// Least-squares line ln max|D| = ln H - Lambda r through the non-empty bins
// (r at the bin centre), then ln H raised until the line lies on or above
// every bin's maximum at the bin's far edge (the line's lowest point over the
// bin), so that it bounds every element.  Lambda >= 0.  One thread.
__global__ void k_dfit_solve(const unsigned long long *__restrict bins, double dr, double *__restrict fit)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int m = 0;
    for (int b = 0; b < FK_DFIT_BINS; ++b) {
        const double v = __longlong_as_double((long long)bins[b]);
        if (!(v > 1e-300)) continue;
        const double x = (b + 0.5) * dr, y = log(v);
        sx += x; sy += y; sxx += x * x; sxy += x * y;
        ++m;
    }
    double lam = 0.0, lnh = 0.0;
    if (m >= 2) {
        const double den = m * sxx - sx * sx;
        lam = den > 0 ? -(m * sxy - sx * sy) / den : 0.0;
        lam = fmax(lam, 0.0);
    }
    if (m >= 1) lnh = (sy + lam * sx) / m;
    double shift = -1e300;
    for (int b = 0; b < FK_DFIT_BINS; ++b) {
        const double v = __longlong_as_double((long long)bins[b]);
        if (!(v > 1e-300)) continue;
        shift = fmax(shift, log(v) - (lnh - lam * ((b + 1) * dr)));
    }
    if (m >= 1) lnh += fmax(shift, 0.0);
    fit[0] = m >= 1 ? exp(lnh) : 0.0;
    fit[1] = lam;
}

// J = s_r s_c (X_J + X_J^T), K likewise, within each molecule's block
__global__ void k_finalize(const double *__restrict XJ, const double *__restrict XK, long long xcopy, int ncopy,
                           const double *__restrict s, FkMolArgs m, double *__restrict J, double *__restrict K)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.nmat) return;
    const int k = find_mol(m.mol_base, m.nmol, i);
    const long long loc = i - m.mol_base[k];
    const int n = m.mol_nbf[k], f0 = m.mol_bf0[k];
    const int r = (int)(loc / n), c = (int)(loc % n);
    const long long t = m.mol_base[k] + (long long)c * n + r;
    const double f = s[f0 + r] * s[f0 + c];
    // a build of one matrix passes a null pointer for the other
    if (J) {
        double sj = 0.0;
#pragma unroll
        for (int x = 0; x < ncopy; ++x) {
            const long long o = (long long)x * xcopy;
            sj += XJ[o + i] + XJ[o + t];
        }
        J[i] = f * sj;
    }
    if (K) {
        double sk = 0.0;
#pragma unroll
        for (int x = 0; x < ncopy; ++x) {
            const long long o = (long long)x * xcopy;
            sk += XK[o + i] + XK[o + t];
        }
        K[i] = f * sk;
    }
}


}  // namespace

#define FK_DECL_P(P)                                                                                         \
    int fk_kp##P##_info(int, FkClassInfo *);                                                                 \
    int fk_kp##P##_jk(int, const FkJKArgs *, int, void *);                                                   \
    int fk_kp##P##_dbg(int, const FkDebugArgs *, void *);                                                    \
    int fk_kp##P##_host(int, const int *, const int *, const double *, const double *, const int *, int,    \
                        double *, int);                                                                      \
    const void *fk_kp##P##_kern(int, int, int, int);                                                         \
    int fk_kp##P##_lds(int, int, int, int, int, int);
extern "C" {
FK_DECL_P(0) FK_DECL_P(1) FK_DECL_P(2) FK_DECL_P(3) FK_DECL_P(4)
FK_DECL_P(5) FK_DECL_P(6) FK_DECL_P(7) FK_DECL_P(8) FK_DECL_P(9)
}
#define FK_SWITCH_P(P, call)                                                                            \
    switch (P) {                                                                                        \
    case 0: return fk_kp0_##call; case 1: return fk_kp1_##call; case 2: return fk_kp2_##call;        \
    case 3: return fk_kp3_##call; case 4: return fk_kp4_##call; case 5: return fk_kp5_##call;        \
    case 6: return fk_kp6_##call; case 7: return fk_kp7_##call; case 8: return fk_kp8_##call;        \
    case 9: return fk_kp9_##call; default: break;                                                       \
    }

extern "C" {

int fk_kernels_class_info(int P, int Q, FkClassInfo *info)
{
    FK_SWITCH_P(P, info(Q, info))
    return -1;
}

int fk_kernels_launch_jk(int P, int Q, const FkJKArgs *args, int grid, void *stream)
{
    FK_SWITCH_P(P, jk(Q, args, grid, stream))
    return -1;
}

int fk_kernels_launch_debug(int P, int Q, const FkDebugArgs *args, void *stream)
{
    FK_SWITCH_P(P, dbg(Q, args, stream))
    return -1;
}

int fk_kernels_debug_host(int P, int Q, const int *pair_ppoff, const int *pair_npp, const double *pair_AB,
                          const double *pp, const int *quartets, int nq, double *out, int engine)
{
    FK_SWITCH_P(P, host(Q, pair_ppoff, pair_npp, pair_AB, pp, quartets, nq, out, engine))
    return -1;
}

static const void *kern_of(int P, int Q, int engine, int kind, int nw)
{
    FK_SWITCH_P(P, kern(Q, engine, kind, nw))
    return nullptr;
}

int fk_kernels_jk_lds_bytes(int P, int Q, int bra_slot, int krow_ncol, int kind, int nbk, int nw)
{
    FK_SWITCH_P(P, lds(Q, bra_slot, krow_ncol, kind, nbk, nw))
    return -1;
}

int fk_kernels_max_blocks(int P, int Q, int dyn_lds_bytes, int engine, int kind, int nw, int *blocks_per_cu)
{
    const void *k = kern_of(P, Q, engine, kind, nw);
    if (!k) return -2;
    int nb = 0;
    if (dyn_lds_bytes > 65536 &&
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds_bytes) != hipSuccess)
        return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * nw, dyn_lds_bytes) != hipSuccess) return -3;
    *blocks_per_cu = nb;
    return 0;
}

int fk_kernels_launch_prep(const double *D, const double *bf_scale, const FkMolArgs *m, double *Ds, double *Dsh,
                           void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (m->nmat > 0)
        hipLaunchKernelGGL(k_prep_ds, dim3((unsigned)((m->nmat + 255) / 256)), dim3(256), 0, st, D, bf_scale, *m, Ds);
    if (m->nshmat > 0)
        hipLaunchKernelGGL(k_prep_dsh, dim3((unsigned)((m->nshmat + 255) / 256)), dim3(256), 0, st, D, *m, Dsh);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int fk_kernels_launch_finalize(const double *XJ, const double *XK, long long xcopy, int ncopy, const double *bf_scale,
                               const FkMolArgs *m, double *J, double *K, void *stream)
{
    if (m->nmat > 0)
        hipLaunchKernelGGL(k_finalize, dim3((unsigned)((m->nmat + 255) / 256)), dim3(256), 0, (hipStream_t)stream, XJ,
                           XK, xcopy, ncopy, bf_scale, *m, J, K);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int fk_kernels_launch_dfit(const double *D, int n, const int *bf_atom, const double *atom_xyz, double dr,
                           unsigned long long *bins, double *fit, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(FK_DFIT_BINS), 0, st, (double *)bins, (long long)FK_DFIT_BINS);
    const long long nn = (long long)n * n;
    if (nn > 0)
        hipLaunchKernelGGL(k_dfit_bins, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, D, n, bf_atom, atom_xyz,
                           dr, bins);
    hipLaunchKernelGGL(k_dfit_solve, dim3(1), dim3(64), 0, st, bins, dr, fit);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int fk_kernels_launch_fill(double *p, long long n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
#endif
