// Host side of libfockjk: context, basis normalisation, shell pairs, Schwarz
// factors, class sort, work tiles and the C-ABI entry points declared in
// include/fockjk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unordered_map>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "fockjk.h"
#include "fk_internal.h"
#include "fk_guess.h"
#include "fk_scf_batch.h"
#include "fk_rys.h"

namespace {

constexpr int NPC = 10;  // pair classes (la >= lb, la <= 3)

constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// block tasks run where the launch needs at most this much dynamic LDS (two
// workgroups per CU)
constexpr int kKrowLdsMax = 65536;
// and with workgroups of eight waves (one workgroup per CU)
constexpr int kKrowLdsMaxWide = 160 * 1024;
// streams besides the caller's for the class launches of fk_build_jk
// (measured: three streams in all gave C20H42 7.83 ms per build against 9.06 on
// one, (H2O)64 238.6 against 244.2; four were slower on (H2O)64)
constexpr int kAuxStreams = 2;
inline int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }
// Hermite functions of total order up to L
inline int nherm_host(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

double dfact(int n)
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
};

struct QuartetClass {
    int P, Q;
    FkClassInfo info;
    int64_t tile_off, ntile;
    int64_t nquartet, nprim;  // Schwarz-surviving counts
    int64_t prim_slots;       // primitive-quartet slots the waves step through
    int blocks_per_cu;
    double grid_frac = 1.0;   // share of the resident-workgroup grid launched
    int bra_block = 1, kets_per_tile = 64;  // the schedule in effect
    int bra_slot;             // doubles per wave of staged bra primitive records
    int prec;                 // 0: FP64 launch, 1: FP32 launch of the precision split
    int engine = 0;           // 0: Rys quadrature, 1: HGP (classes with info.hgp only)
    int64_t task_off = 0, ntask = 0;  // block tasks (0: none)
    int krow_ncol = 0;        // LDS row length of the block tasks
    int nw = 4;               // waves per workgroup of the launch
    int krow_nbk = 0;         // bras per block of the block tasks' rows
    double flops_prim() const { return engine ? info.flops_prim_hgp : info.flops_prim; }
    double flops_quartet() const { return engine ? info.flops_quartet_hgp : info.flops_quartet; }
};

}  // namespace

struct fk_ctx {
    int device = -1;
    std::string err;
    int ncu = 0;
    std::string arch = "host";  // device architecture without feature suffixes (e.g. gfx950); "host" without one
    // geometry
    int natom = 0, charge = 0, nelec = 0;
    std::vector<int> Z;
    std::vector<double> xyz;
    bool have_geom = false, have_basis = false, have_quartets = false;
    // basis
    int nshell = 0, nbf = 0;
    std::vector<int> sh_atom, sh_l, sh_nprim, sh_poff, sh_bf;   // sh_bf: flat offsets over all molecules
    // molecules of a batch (one molecule unless fk_set_molecules split the atoms):
    // shells, functions and matrix blocks are numbered within each molecule
    int nmol = 1;
    std::vector<int> atom_mol;                   // molecule of each atom
    std::vector<int> sh_mol, sh_loc, sh_lbf, sh_lend;  // per shell: molecule, local index, local first/end function
    std::vector<int> mol_sh0, mol_nsh, mol_bf0, mol_nbf;
    std::vector<long long> mol_base, mol_shbase;  // [nmol + 1] offsets of the nbf^2 and nshell^2 blocks
    std::vector<int> pr_sa_loc, pr_sb_loc, lst_sa_loc, lst_sb_loc;
    std::vector<double> exps, coef;  // coef: normalised for the axis component
    std::vector<double> bf_scale;    // component scale factors
    // pairs
    fk_screen_opts opts{};
    std::vector<int> pr_sa, pr_sb, pr_ppoff, pr_npp, pr_cls;
    std::vector<double> pr_AB, pr_G, pp;
    std::vector<int> cls_list[NPC];              // sorted pair indices per class
    std::vector<std::pair<int, int>> cls_groups[NPC];  // [begin, end) of equal npp
    std::vector<int> ket_list_all;               // concatenated class lists
    int ket_off[NPC + 1] = {0};
    std::vector<int> lst_sa, lst_sb;
    std::vector<double> lst_CD, lst_G, ppT;
    std::vector<FkGroup> groups;
    std::vector<int> cls_group0;                 // first global group of each class
    std::vector<FkTile> tiles;
    std::vector<int2> tasks;                     // block tasks (first tile, count) per class
    // columns of the block tasks' LDS rows: per shell its first column among the
    // shells of its type in its molecule; per (molecule, type) the column count,
    // the offset of its function list and the functions (local numbering)
    std::vector<int> krow_col, krow_cnt, krow_off, krow_fn;
    std::vector<FkBraBlock> blocks;
    std::vector<int> blk_bra, blk_pos;
    std::vector<int64_t> blk_nppsum;             // sum of the bras' primitive-pair counts
    std::vector<QuartetClass> qclasses;
    double flops_schwarz = 0;
    int64_t nq_schwarz = 0;
    int npair_kept = 0;
    // device buffers
    DevBuf<int> d_sh_bf, d_pr_sa, d_pr_sb, d_pr_ppoff, d_pr_npp, d_ket, d_lst_sa, d_lst_sb;
    DevBuf<int> d_sh_lend, d_mol_sh0, d_mol_nsh, d_mol_bf0, d_mol_nbf;
    DevBuf<long long> d_mol_base, d_mol_shbase;
    DevBuf<double> d_bf_scale, d_pr_AB, d_pr_G, d_pp, d_rys, d_Ds, d_Dsh, d_X, d_Din, d_Jout, d_Kout;
    DevBuf<double> d_lst_CD, d_lst_G, d_ppT;
    DevBuf<FkGroup> d_groups;
    DevBuf<FkTile> d_tiles;
    DevBuf<int2> d_tasks;
    DevBuf<int> d_krow_col, d_krow_cnt, d_krow_off, d_krow_fn;
    DevBuf<FkBraBlock> d_blocks;
    DevBuf<int> d_blk_bra, d_blk_pos;
    DevBuf<unsigned long long> d_cnt;
    // J engine (built on first use after fk_build_quartets)
    bool jeng_valid = false;
    std::vector<int64_t> jeng_toff;               // tiles of bucket LP * (FK_JENG_MAX_LP + 1) + LQ
    DevBuf<FkJengTile> d_jeng_tiles;
    DevBuf<long long> d_jp_off, d_dq_base;
    DevBuf<int> d_pos_grp;
    DevBuf<double> d_jp, d_dq;
    size_t jp_n = 0;
    // density-decay fit and K-block skip (per shell: x, y, z, R, G)
    DevBuf<int> d_bf_atom;
    DevBuf<double> d_atom_xyz, d_ks_shell, d_dfit;
    DevBuf<unsigned long long> d_dfit_bins;
    double dfit_dr = 1.0;
    // last build
    bool stats_pending = false;
    bool timed = false;
    std::vector<hipEvent_t> ev;  // 2 per quartet class
    // more streams for the class launches of fk_build_jk (the device's, shared
    // by its contexts), with this context's events that fork them from and
    // join them to the caller's stream (set up with the lists, outside any
    // stream capture)
    std::vector<hipStream_t> aux;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    // per quartet class schedule (key P * NPC + Q), from fk_set_class_schedule or fk_autotune
    // bt: block tasks 1 on, 0 off, -1 the class's default (on for the ket-outer
    // classes, off for the others); alt: a lane class runs its team-per-quartet kernel
    struct ClassSched { int bb = 0, kt = 0; double gf = 1.0; int eng = 0; int bt = -1; int alt = 0; };
    std::map<int, ClassSched> sched;
    std::vector<double> oe_S, oe_T, oe_V;          // one-electron matrices of the current geometry and basis
    double dscreen_scale = 1.0;                   // per-quartet threshold = tau * this (builds from density changes)
    unsigned long long *cnt_last = nullptr;       // counters of the last build (context's or scratch)
    double *scratch = nullptr;                    // device address of this device's scratch array
    // initial guesses
    std::vector<double> coef_in;                  // contraction coefficients as given
    std::map<std::vector<double>, std::vector<double>> sad_cache; // atomic density per (element, shells)
    bool have_model = false;
    fk_mlp g_model{};                             // device copy of the guess network
    DevBuf<float> g_W[FK_MLP_MAX_LAYERS], g_b[FK_MLP_MAX_LAYERS], g_X, g_Y, g_work;
    DevBuf<FkGuessPair> g_pairs;
    DevBuf<double> g_rot, g_D;
};

namespace {

int fail(fk_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(ctx, FK_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dev_upload(fk_ctx *c, DevBuf<T> &b, const T *src, size_t n)
{
    if (b.n < n || !b.p) {
        if (b.p) hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
        if (hipMalloc((void **)&b.p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
            return fail(c, FK_ERR_OOM, "hipMalloc of %zu bytes failed", n * sizeof(T));
        b.n = std::max<size_t>(n, 1);
    }
    if (src && n) HIPCHK(c, hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice));
    return FK_OK;
}

template <class T>
void dev_free(DevBuf<T> &b)
{
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

// Contraction coefficients for the axis-aligned component, normalised so the
// contracted function has unit self-overlap; primitives use
// N(a,l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!).
void normalise_shell(int l, const double *e, const double *d, int np, double *out)
{
    for (int i = 0; i < np; ++i)
        out[i] = d[i] * std::pow(2 * e[i] / M_PI, 0.75) * std::pow(4 * e[i], 0.5 * l) / std::sqrt(dfact(2 * l - 1));
    double s = 0;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            const double p = e[i] + e[j];
            s += out[i] * out[j] * std::pow(M_PI / p, 1.5) * dfact(2 * l - 1) / std::pow(2 * p, l);
        }
    const double f = 1.0 / std::sqrt(s);
    for (int i = 0; i < np; ++i) out[i] *= f;
}

void cart_exps(int l, int k, int &x, int &y, int &z)
{
    int c = 0;
    for (int a = l; a >= 0; --a)
        for (int b = l - a; b >= 0; --b) {
            if (c == k) { x = a; y = b; z = l - a - b; return; }
            ++c;
        }
}

void free_device(fk_ctx *c)
{
    dev_free(c->d_sh_lend); dev_free(c->d_mol_sh0); dev_free(c->d_mol_nsh); dev_free(c->d_mol_bf0);
    dev_free(c->d_mol_nbf); dev_free(c->d_mol_base); dev_free(c->d_mol_shbase);
    dev_free(c->d_sh_bf); dev_free(c->d_pr_sa); dev_free(c->d_pr_sb); dev_free(c->d_pr_ppoff);
    dev_free(c->d_pr_npp); dev_free(c->d_ket); dev_free(c->d_bf_scale); dev_free(c->d_pr_AB);
    dev_free(c->d_pr_G); dev_free(c->d_pp); dev_free(c->d_rys); dev_free(c->d_Ds); dev_free(c->d_Dsh);
    dev_free(c->d_X); dev_free(c->d_Din); dev_free(c->d_Jout); dev_free(c->d_Kout); dev_free(c->d_tiles);
    dev_free(c->d_cnt); dev_free(c->d_blocks); dev_free(c->d_blk_bra); dev_free(c->d_blk_pos); dev_free(c->d_lst_sa); dev_free(c->d_lst_sb); dev_free(c->d_lst_CD);
    dev_free(c->d_lst_G); dev_free(c->d_ppT); dev_free(c->d_groups);
    dev_free(c->d_tasks); dev_free(c->d_krow_col); dev_free(c->d_krow_cnt); dev_free(c->d_krow_off); dev_free(c->d_krow_fn);
    dev_free(c->d_jeng_tiles); dev_free(c->d_jp_off); dev_free(c->d_dq_base); dev_free(c->d_pos_grp);
    dev_free(c->d_jp); dev_free(c->d_dq);
    dev_free(c->d_bf_atom); dev_free(c->d_atom_xyz); dev_free(c->d_ks_shell); dev_free(c->d_dfit); dev_free(c->d_dfit_bins);
    for (int k = 0; k < FK_MLP_MAX_LAYERS; ++k) { dev_free(c->g_W[k]); dev_free(c->g_b[k]); }
    dev_free(c->g_X); dev_free(c->g_Y); dev_free(c->g_work); dev_free(c->g_pairs); dev_free(c->g_rot); dev_free(c->g_D);
}

// canonical orientation of a shell pair: first shell has the higher l
void orient(const fk_ctx *c, int a, int b, int &sa, int &sb)
{
    if (c->sh_l[a] > c->sh_l[b] || (c->sh_l[a] == c->sh_l[b] && a >= b)) { sa = a; sb = b; }
    else { sa = b; sb = a; }
}

void make_pair(fk_ctx *c, int sa, int sb)
{
    const double *A = &c->xyz[3 * c->sh_atom[sa]], *B = &c->xyz[3 * c->sh_atom[sb]];
    double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
    const double ab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
    c->pr_sa.push_back(sa);
    c->pr_sb.push_back(sb);
    c->pr_cls.push_back(pair_class(c->sh_l[sa], c->sh_l[sb]));
    c->pr_ppoff.push_back((int)(c->pp.size() / FK_NPP_REC));
    for (int k = 0; k < 3; ++k) c->pr_AB.push_back(AB[k]);
    const double kfac = std::sqrt(2.0 / std::sqrt(M_PI));
    int np = 0;
    for (int i = c->sh_poff[sa]; i < c->sh_poff[sa + 1]; ++i)
        for (int j = c->sh_poff[sb]; j < c->sh_poff[sb + 1]; ++j) {
            const double ai = c->exps[i], aj = c->exps[j], z = ai + aj;
            double rec[FK_NPP_REC];
            rec[0] = z;
            rec[1] = 0.5 / z;
            for (int k = 0; k < 3; ++k) {
                rec[2 + k] = (ai * A[k] + aj * B[k]) / z;
                rec[5 + k] = rec[2 + k] - A[k];
            }
            rec[8] = c->coef[i] * c->coef[j] * std::pow(M_PI / z, 1.5) * std::exp(-ai * aj / z * ab2) * kfac * std::sqrt(z);
            rec[9] = 0.0;
            c->pp.insert(c->pp.end(), rec, rec + FK_NPP_REC);
            ++np;
        }
    c->pr_npp.push_back(np);
    c->pr_G.push_back(0.0);
}

// Raw contracted integrals for quartets given as (bra pair, ket pair) of one
// class pair (P = class of bra >= Q = class of ket), on device or host.
// A pair table as read by the integral code: primitive offsets/counts and
// A - B per pair, primitive records in c->pp.
struct PairTab {
    const int *ppoff, *npp;
    const double *AB;
    const int *d_ppoff, *d_npp;  // device copies (device evaluation only)
    const double *d_AB;
};

int eval_quartets_tab(fk_ctx *c, const PairTab &t, int P, int Q, const std::vector<int> &qs,
                      std::vector<double> &out, bool on_device, int engine = 0)
{
    FkClassInfo ci;
    int rc = fk_kernels_class_info(P, Q, &ci);
    if (rc) return fail(c, FK_ERR_UNSUPPORTED, "class (%d,%d) not built", P, Q);
    if (engine == 1 && !ci.hgp)
        return fail(c, FK_ERR_UNSUPPORTED, "the HGP engine is not built for class (%d%d|%d%d)", ci.la, ci.lb, ci.lc, ci.ld);
    if (engine == 2 && (on_device || ci.la + ci.lb + ci.lc + ci.ld > 8))
        return fail(c, FK_ERR_UNSUPPORTED, "McMurchie-Davidson integrals: host only, L <= 8");
    const int nq = (int)qs.size() / 2;
    out.assign((size_t)nq * ci.nout, 0.0);
    if (nq == 0) return FK_OK;
    if (!on_device) {
        rc = fk_kernels_debug_host(P, Q, t.ppoff, t.npp, t.AB, c->pp.data(), qs.data(), nq, out.data(), engine);
        return rc ? fail(c, FK_ERR_UNSUPPORTED, "host evaluation failed") : FK_OK;
    }
    DevBuf<int> dq;
    DevBuf<double> dout;
    if ((rc = dev_upload(c, dq, qs.data(), qs.size()))) return rc;
    if ((rc = dev_upload<double>(c, dout, nullptr, out.size()))) { dev_free(dq); return rc; }
    FkDebugArgs a;
    a.pair_ppoff = t.d_ppoff;
    a.pair_npp = t.d_npp;
    a.pair_AB = t.d_AB;
    a.pp = c->d_pp.p;
    a.quartets = (const int2 *)dq.p;
    a.nq = nq;
    a.out = dout.p;
    a.rys_tab = c->d_rys.p + rys_staged_offset(ci.nroot);
    a.engine = engine;
    rc = fk_kernels_launch_debug(P, Q, &a, nullptr);
    hipError_t e = hipDeviceSynchronize();
    if (rc == 0 && e == hipSuccess) e = hipMemcpy(out.data(), dout.p, out.size() * sizeof(double), hipMemcpyDeviceToHost);
    dev_free(dq);
    dev_free(dout);
    if (rc) return fail(c, FK_ERR_HIP, "debug kernel launch failed for class (%d,%d)", P, Q);
    if (e != hipSuccess) return fail(c, FK_ERR_HIP, "debug kernel: %s", hipGetErrorString(e));
    return FK_OK;
}

int eval_quartets(fk_ctx *c, int P, int Q, const std::vector<int> &qs, std::vector<double> &out, bool on_device,
                  int engine = 0)
{
    PairTab t{c->pr_ppoff.data(), c->pr_npp.data(), c->pr_AB.data(), c->d_pr_ppoff.p, c->d_pr_npp.p, c->d_pr_AB.p};
    return eval_quartets_tab(c, t, P, Q, qs, out, on_device, engine);
}

// Largest Cartesian diagonal of (ab|ab) over the components, true normalisation.
double diag_max(const fk_ctx *c, const double *v, int sa, int sb)
{
    const int na = ncart(c->sh_l[sa]), nb = ncart(c->sh_l[sb]);
    const double *fa = &c->bf_scale[c->sh_bf[sa]], *fb = &c->bf_scale[c->sh_bf[sb]];
    double g = 0;
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            const double x = v[((ia * nb + ib) * na + ia) * nb + ib] * fa[ia] * fa[ia] * fb[ib] * fb[ib];
            g = std::max(g, std::sqrt(std::fabs(x)));
        }
    return g;
}

// Primitive Cauchy-Schwarz factors G_[ab] (eq. cauchy-schwarz2) of every
// primitive pair, from the diagonal primitive quartets [ab|ab] evaluated by the
// same integral code, stored in field 9 of the primitive records.
int prim_schwarz(fk_ctx *c, bool dev)
{
    const int np = (int)(c->pp.size() / FK_NPP_REC);
    const int npair = (int)c->pr_sa.size();
    std::vector<int> owner(np), one(np, 1), self(np);
    std::vector<double> ab(3 * (size_t)np);
    for (int p = 0; p < npair; ++p)
        for (int j = 0; j < c->pr_npp[p]; ++j) {
            const int k = c->pr_ppoff[p] + j;
            owner[k] = p;
            for (int x = 0; x < 3; ++x) ab[3 * k + x] = c->pr_AB[3 * p + x];
        }
    std::iota(self.begin(), self.end(), 0);
    DevBuf<int> d_self, d_one;
    DevBuf<double> d_ab;
    int rc;
    if (dev) {
        if ((rc = dev_upload(c, d_self, self.data(), self.size())) || (rc = dev_upload(c, d_one, one.data(), one.size())) ||
            (rc = dev_upload(c, d_ab, ab.data(), ab.size()))) {
            dev_free(d_self); dev_free(d_one); dev_free(d_ab);
            return rc;
        }
    }
    PairTab t{self.data(), one.data(), ab.data(), d_self.p, d_one.p, d_ab.p};
    rc = FK_OK;
    for (int P = 0; P < NPC && rc == FK_OK; ++P) {
        std::vector<int> qs, ks;
        for (int k = 0; k < np; ++k)
            if (c->pr_cls[owner[k]] == P) { qs.push_back(k); qs.push_back(k); ks.push_back(k); }
        if (ks.empty()) continue;
        std::vector<double> out;
        if ((rc = eval_quartets_tab(c, t, P, P, qs, out, dev))) break;
        const size_t nout = out.size() / ks.size();
        for (size_t q = 0; q < ks.size(); ++q) {
            const int p = owner[ks[q]];
            const double g = diag_max(c, out.data() + q * nout, c->pr_sa[p], c->pr_sb[p]);
            if (!std::isfinite(g)) { rc = fail(c, FK_ERR_ARG, "non-finite primitive Schwarz factor"); break; }
            c->pp[(size_t)ks[q] * FK_NPP_REC + 9] = g;
        }
    }
    dev_free(d_self); dev_free(d_one); dev_free(d_ab);
    return rc;
}

// Orders each pair's primitive pairs by G_[ab] (largest first) and, when
// tau_prim > 0, deletes those with G_[ab] * max G_[cd] < tau_prim: every
// primitive quartet they belong to is then bounded by tau_prim times the
// density.  The largest primitive pair of a shell pair is always kept.
void prune_primitives(fk_ctx *c, double tau_prim)
{
    const int npair = (int)c->pr_sa.size();
    double gmax = 0;
    for (size_t k = 0; k < c->pp.size() / FK_NPP_REC; ++k) gmax = std::max(gmax, c->pp[k * FK_NPP_REC + 9]);
    std::vector<double> npp_new;
    npp_new.reserve(c->pp.size());
    for (int p = 0; p < npair; ++p) {
        std::vector<int> idx(c->pr_npp[p]);
        std::iota(idx.begin(), idx.end(), c->pr_ppoff[p]);
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
            return c->pp[(size_t)x * FK_NPP_REC + 9] > c->pp[(size_t)y * FK_NPP_REC + 9];
        });
        const int off = (int)(npp_new.size() / FK_NPP_REC);
        int kept = 0;
        for (size_t r = 0; r < idx.size(); ++r) {
            const double g = c->pp[(size_t)idx[r] * FK_NPP_REC + 9];
            if (r > 0 && tau_prim > 0 && g * gmax < tau_prim) break;
            npp_new.insert(npp_new.end(), c->pp.begin() + (size_t)idx[r] * FK_NPP_REC,
                           c->pp.begin() + (size_t)(idx[r] + 1) * FK_NPP_REC);
            ++kept;
        }
        c->pr_ppoff[p] = off;
        c->pr_npp[p] = kept;
    }
    c->pp.swap(npp_new);
}

// Every index a J/K kernel dereferences, checked on the host before upload:
// tiles -> pairs, groups and list positions; groups -> transposed records;
// pairs -> shells and primitive records; shells -> basis-function offsets.
// XCD-aware order of a lane-per-quartet class's work.  Workgroup g runs on
// XCD g mod 8, whose L2 (4 MB) serves only that XCD.  The class's bra blocks
// are cut into eight regions of equal cost by recursive bisection of the
// first bra shell's position, and the work items (tiles, or block tasks) are
// placed so that the workgroups of XCD x take region x: the density blocks
// its digestion reads (D_ac, D_ad, D_bc, D_bd) then come from one region's
// rows.  The order within a region stays cost-descending.  Used where the
// density is larger than one L2 (n > 724: n^2 doubles above 4 MB) and the
// context holds one molecule; smaller systems keep the cost order, which
// balances better.
void order_for_xcds(fk_ctx *c, const QuartetClass &q)
{
    constexpr int NX = 8;
    if (c->nmol != 1 || (int64_t)c->nbf * c->nbf * 8 <= (4 << 20) || q.info.wave_per_quartet != 0 ||
        q.ntile < 64 * NX)
        return;
    const bool tasks = q.ntask > 0;
    const int64_t nitem = tasks ? q.ntask : q.ntile;
    const int64_t wgs = tasks ? q.ntask : (q.ntile + 3) / 4;
    const int64_t cap = std::max<int64_t>(1, (int64_t)(q.grid_frac * std::max(8, q.blocks_per_cu) * std::max(c->ncu, 1)));
    const int64_t G = std::max<int64_t>(1, std::min(wgs, cap));
    if (G < NX) return;
    const int NWT = q.nw;  // waves per workgroup of the strided tile loop
    auto item_blk = [&](int64_t i) {
        return tasks ? c->tiles[q.tile_off + c->tasks[q.task_off + i].x].blk : c->tiles[q.tile_off + i].blk;
    };
    auto item_cost = [&](int64_t i) {
        auto tc = [&](const FkTile &t) {
            return (double)c->blk_nppsum[t.blk] * c->groups[t.grp & ~FK_TILE_SAME].npp * t.ket_count;
        };
        if (!tasks) return tc(c->tiles[q.tile_off + i]);
        const int2 tk = c->tasks[q.task_off + i];
        double s = 0;
        for (int k = tk.x; k < tk.x + tk.y; ++k) s += tc(c->tiles[q.tile_off + k]);
        return s;
    };
    // cost and position of every bra block of the class
    std::unordered_map<int, double> bcost;
    for (int64_t i = 0; i < nitem; ++i) bcost[item_blk(i)] += item_cost(i);
    std::vector<int> blks;
    for (const auto &kv : bcost) blks.push_back(kv.first);
    std::sort(blks.begin(), blks.end());
    auto centre = [&](int b, int k) {
        const int sa = c->pr_sa[c->blk_bra[c->blocks[b].first]];
        return c->xyz[3 * c->sh_atom[sa] + k];
    };
    std::unordered_map<int, int> region;
    std::function<void(std::vector<int> &, int, int)> cut = [&](std::vector<int> &v, int r0, int nr) {
        if (nr == 1 || v.size() <= 1) {
            for (int b : v) region[b] = r0;
            return;
        }
        int ax = 0;
        double best = -1;
        for (int k = 0; k < 3; ++k) {
            double lo = 1e300, hi = -1e300;
            for (int b : v) { lo = std::min(lo, centre(b, k)); hi = std::max(hi, centre(b, k)); }
            if (hi - lo > best) { best = hi - lo; ax = k; }
        }
        std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return centre(x, ax) < centre(y, ax); });
        double tot = 0, acc = 0;
        for (int b : v) tot += bcost[b];
        size_t m = 0;
        while (m < v.size() && acc + 0.5 * bcost[v[m]] < 0.5 * tot) acc += bcost[v[m++]];
        std::vector<int> lo(v.begin(), v.begin() + m), hi(v.begin() + m, v.end());
        cut(lo, r0, nr / 2);
        cut(hi, r0 + nr / 2, nr - nr / 2);
    };
    cut(blks, 0, NX);
    // queues per region, in the present (cost-descending) order
    std::vector<std::vector<int64_t>> qu(NX);
    for (int64_t i = 0; i < nitem; ++i) qu[region[item_blk(i)]].push_back(i);
    std::vector<size_t> head(NX, 0);
    std::vector<int64_t> order(nitem);
    for (int64_t p = 0; p < nitem; ++p) {
        const int64_t g = tasks ? p % G : (p % (G * NWT)) / NWT;
        int x = (int)(g % NX);
        if (head[x] == qu[x].size()) {
            size_t most = 0;
            for (int y = 0; y < NX; ++y)
                if (qu[y].size() - head[y] > most) { most = qu[y].size() - head[y]; x = y; }
        }
        order[p] = qu[x][head[x]++];
    }
    if (tasks) {
        // tasks keep partitioning the tiles in order: their tiles move with them
        std::vector<int2> tk(c->tasks.begin() + q.task_off, c->tasks.begin() + q.task_off + nitem);
        std::vector<FkTile> tl(c->tiles.begin() + q.tile_off, c->tiles.begin() + q.tile_off + q.ntile);
        int x = 0;
        for (int64_t p = 0; p < nitem; ++p) {
            const int2 t = tk[order[p]];
            std::copy(tl.begin() + t.x, tl.begin() + t.x + t.y, c->tiles.begin() + q.tile_off + x);
            c->tasks[q.task_off + p] = int2{x, t.y};
            x += t.y;
        }
    } else {
        std::vector<FkTile> tl(c->tiles.begin() + q.tile_off, c->tiles.begin() + q.tile_off + nitem);
        for (int64_t p = 0; p < nitem; ++p) c->tiles[q.tile_off + p] = tl[order[p]];
    }
}

int validate_lists(fk_ctx *c)
{
    const int npair = (int)c->pr_sa.size();
    const long long npp_tot = (long long)(c->pp.size() / FK_NPP_REC);
    const int nl = (int)c->ket_list_all.size();
    for (int p = 0; p < npair; ++p) {
        if (c->pr_sa[p] < 0 || c->pr_sa[p] >= c->nshell || c->pr_sb[p] < 0 || c->pr_sb[p] >= c->nshell ||
            c->pr_ppoff[p] < 0 || c->pr_npp[p] < 1 || c->pr_npp[p] > FK_MAX_K * FK_MAX_K ||
            (long long)c->pr_ppoff[p] + c->pr_npp[p] > npp_tot || !std::isfinite(c->pr_G[p]) || c->pr_G[p] < 0)
            return fail(c, FK_ERR_STATE, "internal: shell pair %d is inconsistent", p);
    }
    for (int q = 0; q < nl; ++q)
        if (c->ket_list_all[q] < 0 || c->ket_list_all[q] >= npair)
            return fail(c, FK_ERR_STATE, "internal: list position %d holds pair %d", q, c->ket_list_all[q]);
    for (size_t g = 0; g < c->groups.size(); ++g) {
        const FkGroup &G = c->groups[g];
        if (G.begin < 0 || G.len < 1 || G.begin + G.len > nl || G.npp < 1 ||
            G.base < 0 || G.base + (long long)G.npp * FK_NFLD * G.len > (long long)c->ppT.size())
            return fail(c, FK_ERR_STATE, "internal: group %zu is inconsistent", g);
        for (int r = 0; r < G.len; ++r)
            if (c->pr_npp[c->ket_list_all[G.begin + r]] != G.npp)
                return fail(c, FK_ERR_STATE, "internal: group %zu mixes primitive counts", g);
    }
    if (c->blk_pos.size() != c->blk_bra.size()) return fail(c, FK_ERR_STATE, "internal: bra block arrays differ in size");
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        const FkBraBlock &B = c->blocks[b];
        if (B.first < 0 || B.count < 1 || B.count > FK_MAX_BRA_BLOCK || (size_t)B.first + B.count > c->blk_bra.size())
            return fail(c, FK_ERR_STATE, "internal: bra block %zu is inconsistent", b);
        for (int j = 0; j < B.count; ++j) {
            const int p = c->blk_bra[B.first + j], q = c->blk_pos[B.first + j];
            if (p < 0 || p >= npair || q < 0 || q >= nl || c->ket_list_all[q] != p ||
                c->pr_sa[p] != c->pr_sa[c->blk_bra[B.first]] || c->pr_cls[p] != c->pr_cls[c->blk_bra[B.first]])
                return fail(c, FK_ERR_STATE, "internal: bra block %zu member %d is inconsistent", b, j);
        }
    }
    for (const QuartetClass &qc : c->qclasses) {
        for (int64_t t = qc.tile_off; t < qc.tile_off + qc.ntile; ++t) {
            const FkTile &T = c->tiles[t];
            const int gid = T.grp & ~FK_TILE_SAME;
            if (T.blk < 0 || T.blk >= (int)c->blocks.size() || gid < 0 || gid >= (int)c->groups.size() ||
                T.ket_count < 1 || T.ket_count > 64)
                return fail(c, FK_ERR_STATE, "internal: tile %lld is inconsistent", (long long)t);
            const FkBraBlock &B = c->blocks[T.blk];
            if (B.count > qc.info.bra_block)
                return fail(c, FK_ERR_STATE, "internal: tile %lld has %d bras, its class kernel takes %d",
                            (long long)t, B.count, qc.info.bra_block);
            for (int j = 0; j < B.count; ++j)
                if (c->pr_npp[c->blk_bra[B.first + j]] * FK_NFLD > qc.bra_slot || c->pr_cls[c->blk_bra[B.first + j]] != qc.P)
                    return fail(c, FK_ERR_STATE, "internal: tile %lld bra %d does not fit its class", (long long)t, j);
            const FkGroup &G = c->groups[gid];
            if (T.ket_begin < G.begin || T.ket_begin + T.ket_count > G.begin + G.len)
                return fail(c, FK_ERR_STATE, "internal: tile %lld leaves its group", (long long)t);
        }
    }
    for (const QuartetClass &qc : c->qclasses) {
        if (qc.ntask == 0) continue;
        // tasks partition the class's tiles in order; each holds tiles of one
        // bra block; every ket's columns lie inside the LDS rows
        if (qc.task_off < 0 || qc.task_off + qc.ntask > (int64_t)c->tasks.size() || qc.krow_ncol < 1 || qc.krow_nbk < 1)
            return fail(c, FK_ERR_STATE, "internal: block tasks of class (%d|%d)", qc.P, qc.Q);
        int64_t next = 0;
        const int lc = qc.info.lc, ld = qc.info.ld, nc = (lc + 1) * (lc + 2) / 2, nd = (ld + 1) * (ld + 2) / 2;
        for (int64_t k = qc.task_off; k < qc.task_off + qc.ntask; ++k) {
            const int2 T = c->tasks[k];
            if (T.x != next || T.y < 1 || T.x + T.y > qc.ntile)
                return fail(c, FK_ERR_STATE, "internal: block task %lld is inconsistent", (long long)k);
            next = T.x + T.y;
            const int blk = c->tiles[qc.tile_off + T.x].blk;
            if (c->blocks[blk].count > qc.krow_nbk)
                return fail(c, FK_ERR_STATE, "internal: block task %lld has more bras than its rows", (long long)k);
            for (int i = T.x; i < T.x + T.y; ++i) {
                const FkTile &tt = c->tiles[qc.tile_off + i];
                if (tt.blk != blk) return fail(c, FK_ERR_STATE, "internal: block task %lld mixes bra blocks", (long long)k);
                const int m = c->groups[tt.grp & ~FK_TILE_SAME].mol;
                const int cc = c->krow_cnt[4 * m + lc];
                const int ncm = cc + (lc != ld ? c->krow_cnt[4 * m + ld] : 0);
                if (ncm > qc.krow_ncol) return fail(c, FK_ERR_STATE, "internal: block task columns exceed the rows");
                for (int q = tt.ket_begin; q < tt.ket_begin + tt.ket_count; ++q) {
                    const int sc = c->lst_sa[q], sd = c->lst_sb[q];
                    const int xc = c->krow_col[sc], xd = c->krow_col[sd] + (lc != ld ? cc : 0);
                    if (c->sh_l[sc] != lc || c->sh_l[sd] != ld || c->sh_mol[sc] != m || c->sh_mol[sd] != m ||
                        xc < 0 || xc + nc > cc || xd < (lc != ld ? cc : 0) || xd + nd > ncm)
                        return fail(c, FK_ERR_STATE, "internal: list position %d has columns outside the rows", q);
                }
            }
        }
        if (next != qc.ntile) return fail(c, FK_ERR_STATE, "internal: block tasks do not cover class (%d|%d)", qc.P, qc.Q);
    }
    for (int s = 0; s <= c->nshell; ++s)
        if (c->sh_bf[s] < 0 || c->sh_bf[s] > c->nbf) return fail(c, FK_ERR_STATE, "internal: shell offsets");
    return FK_OK;
}

// Per-molecule numbering of shells and functions and the offsets of each
// molecule's matrix blocks in the concatenated D, J, K and shell-maximum arrays.
int layout_molecules(fk_ctx *c)
{
    const int ns = c->nshell;
    if ((int)c->atom_mol.size() != c->natom) c->atom_mol.assign(c->natom, 0);
    c->nmol = 1;
    for (int m : c->atom_mol) c->nmol = std::max(c->nmol, m + 1);
    const int nm = c->nmol;
    c->sh_mol.assign(ns, 0); c->sh_loc.assign(ns, 0); c->sh_lbf.assign(ns, 0); c->sh_lend.assign(ns, 0);
    c->mol_sh0.assign(nm, -1); c->mol_nsh.assign(nm, 0); c->mol_bf0.assign(nm, 0); c->mol_nbf.assign(nm, 0);
    for (int s = 0; s < ns; ++s) {
        const int m = c->atom_mol[c->sh_atom[s]];
        if (s > 0 && m < c->sh_mol[s - 1])
            return fail(c, FK_ERR_ARG, "fk_set_molecules: shells of a molecule must be contiguous (atoms in molecule order)");
        c->sh_mol[s] = m;
        if (c->mol_sh0[m] < 0) { c->mol_sh0[m] = s; c->mol_bf0[m] = c->sh_bf[s]; }
        c->sh_loc[s] = s - c->mol_sh0[m];
        c->sh_lbf[s] = c->sh_bf[s] - c->mol_bf0[m];
        c->sh_lend[s] = c->sh_bf[s + 1] - c->mol_bf0[m];
        c->mol_nsh[m] += 1;
        c->mol_nbf[m] += ncart(c->sh_l[s]);
    }
    c->mol_base.assign(nm + 1, 0);
    c->mol_shbase.assign(nm + 1, 0);
    for (int m = 0; m < nm; ++m) {
        if (c->mol_nsh[m] == 0) return fail(c, FK_ERR_ARG, "fk_set_molecules: molecule %d has no shells", m);
        c->mol_base[m + 1] = c->mol_base[m] + (long long)c->mol_nbf[m] * c->mol_nbf[m];
        c->mol_shbase[m + 1] = c->mol_shbase[m] + (long long)c->mol_nsh[m] * c->mol_nsh[m];
    }
    if (c->device >= 0) {
        int rc;
        if ((rc = dev_upload(c, c->d_sh_bf, c->sh_lbf.data(), c->sh_lbf.size())) ||
            (rc = dev_upload(c, c->d_sh_lend, c->sh_lend.data(), c->sh_lend.size())) ||
            (rc = dev_upload(c, c->d_mol_sh0, c->mol_sh0.data(), c->mol_sh0.size())) ||
            (rc = dev_upload(c, c->d_mol_nsh, c->mol_nsh.data(), c->mol_nsh.size())) ||
            (rc = dev_upload(c, c->d_mol_bf0, c->mol_bf0.data(), c->mol_bf0.size())) ||
            (rc = dev_upload(c, c->d_mol_nbf, c->mol_nbf.data(), c->mol_nbf.size())) ||
            (rc = dev_upload(c, c->d_mol_base, c->mol_base.data(), c->mol_base.size())) ||
            (rc = dev_upload(c, c->d_mol_shbase, c->mol_shbase.data(), c->mol_shbase.size())))
            return rc;
    }
    return FK_OK;
}

int upload_pairs(fk_ctx *c)
{
    int rc;
    // the kernels see shells by their index within the molecule
    c->pr_sa_loc.resize(c->pr_sa.size());
    c->pr_sb_loc.resize(c->pr_sb.size());
    for (size_t p = 0; p < c->pr_sa.size(); ++p) {
        c->pr_sa_loc[p] = c->sh_loc[c->pr_sa[p]];
        c->pr_sb_loc[p] = c->sh_loc[c->pr_sb[p]];
    }
    if ((rc = dev_upload(c, c->d_pr_sa, c->pr_sa_loc.data(), c->pr_sa_loc.size()))) return rc;
    if ((rc = dev_upload(c, c->d_pr_sb, c->pr_sb_loc.data(), c->pr_sb_loc.size()))) return rc;
    if ((rc = dev_upload(c, c->d_pr_ppoff, c->pr_ppoff.data(), c->pr_ppoff.size()))) return rc;
    if ((rc = dev_upload(c, c->d_pr_npp, c->pr_npp.data(), c->pr_npp.size()))) return rc;
    if ((rc = dev_upload(c, c->d_pr_AB, c->pr_AB.data(), c->pr_AB.size()))) return rc;
    if ((rc = dev_upload(c, c->d_pp, c->pp.data(), c->pp.size()))) return rc;
    return FK_OK;
}

}  // namespace

// ---------------------------------------------------- build without allocation
// The working buffers of fk_build_jk_noalloc: one file-scope device array, of
// which each GPU holds its own copy for the life of the process.  Host code
// never passes `scratch` itself to a kernel (in host code the name denotes a
// host-side stand-in); it uses the device address hipGetSymbolAddress returns,
// taken once per device, with that device current, when the first context on
// it is created, and kept per device (contexts copy it to fk_ctx::scratch).
// Layout: D scaled [NMAT], X_J and X_K [2 NMAT], D_sh [NSHMAT], counters
// [2 FK_MAX_QCLASS] (64-bit, the size of a double).
#define FK_SCRATCH_DOUBLES (3 * (size_t)FK_NOALLOC_MAX_NMAT + (size_t)FK_NOALLOC_MAX_NSHMAT + 2 * FK_MAX_QCLASS)
static __device__ __align__(256) double scratch[FK_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

// The class-launch streams of fk_build_jk, per device: created once, on the
// device's first list build, and shared by every context on it for the life
// of the process (a few streams, not a few per context: the hardware queues
// they map to are few, and streams of one build that share a queue
// serialise).
std::vector<hipStream_t> g_aux[kMaxDevices];
std::mutex g_aux_mutex;

int aux_streams(fk_ctx *c, std::vector<hipStream_t> &out)
{
    if (c->device >= kMaxDevices) return fail(c, FK_ERR_UNSUPPORTED, "device ordinal %d too large", c->device);
    std::lock_guard<std::mutex> lock(g_aux_mutex);
    std::vector<hipStream_t> &v = g_aux[c->device];
    while ((int)v.size() < kAuxStreams) {
        hipStream_t x;
        const hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(c, FK_ERR_HIP, "stream creation failed (%s)", hipGetErrorString(e));
        v.push_back(x);
    }
    out = v;
    return FK_OK;
}

// device address of the calling thread's current device's copy of `scratch`
int scratch_address(fk_ctx *c)
{
    if (c->device >= kMaxDevices) return fail(c, FK_ERR_UNSUPPORTED, "device ordinal %d too large", c->device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[c->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, FK_ERR_HIP, "scratch array: hipGetSymbolAddress failed (%s)", hipGetErrorString(e));
        g_scratch[c->device] = (double *)p;
    }
    c->scratch = g_scratch[c->device];
    return FK_OK;
}
}  // namespace

extern "C" {

// failure message of the last fk_create on this thread (there is no context yet)
static thread_local std::string g_create_err;

int fk_create(fk_ctx **out, int device)
{
    if (!out) return FK_ERR_ARG;
    *out = nullptr;
    g_create_err.clear();
    fk_ctx *c = new fk_ctx();
    c->device = device;
    if (device >= 0) {
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e == hipSuccess && device >= ndev) {
            g_create_err = "fk_create: device " + std::to_string(device) + " of " + std::to_string(ndev);
            delete c;
            return FK_ERR_ARG;
        }
        const char *what = "hipGetDeviceCount";
        if (e == hipSuccess) { what = "hipSetDevice"; e = hipSetDevice(device); }
        hipDeviceProp_t prop;
        if (e == hipSuccess) { what = "hipGetDeviceProperties"; e = hipGetDeviceProperties(&prop, device); }
        if (e != hipSuccess) {
            g_create_err = std::string("fk_create: ") + what + ": " + hipGetErrorString(e);
            delete c;
            return FK_ERR_HIP;
        }
        c->ncu = prop.multiProcessorCount;
        c->arch = prop.gcnArchName;
        c->arch = c->arch.substr(0, c->arch.find(':'));
        if (dev_upload(c, c->d_rys, rys_staged_host(), (size_t)rys_staged_total())) {
            g_create_err = c->err;
            delete c;
            return FK_ERR_OOM;
        }
        if (scratch_address(c)) {
            g_create_err = c->err;
            free_device(c);
            delete c;
            return FK_ERR_HIP;
        }
    }
    *out = c;
    return FK_OK;
}

void fk_destroy(fk_ctx *c)
{
    if (!c) return;
    if (c->device >= 0) {
        hipSetDevice(c->device);
        free_device(c);
        for (auto e : c->ev) (void)hipEventDestroy(e);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        for (auto e : c->ev_join) (void)hipEventDestroy(e);  // the streams are the device's, kept
    }
    delete c;
}

const char *fk_last_error(const fk_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int fk_set_geometry(fk_ctx *c, int natom, const int *Z, const double *xyz, int charge)
{
    if (!c) return FK_ERR_ARG;
    if (natom <= 0 || !Z || !xyz) return fail(c, FK_ERR_ARG, "fk_set_geometry: natom must be > 0 and arrays non-null");
    long long zs = 0;
    for (int i = 0; i < natom; ++i) {
        if (Z[i] < 0 || Z[i] > 118) return fail(c, FK_ERR_ARG, "fk_set_geometry: Z[%d] = %d out of range", i, Z[i]);
        zs += Z[i];
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(xyz[3 * i + k])) return fail(c, FK_ERR_ARG, "fk_set_geometry: non-finite coordinate");
    }
    const long long ne = zs - charge;
    if (ne < 0 || (ne & 1)) return fail(c, FK_ERR_ARG, "fk_set_geometry: %lld electrons (closed shell needs an even count)", ne);
    c->natom = natom;
    c->Z.assign(Z, Z + natom);
    c->xyz.assign(xyz, xyz + 3 * natom);
    c->charge = charge;
    c->nelec = (int)ne;
    c->atom_mol.assign(natom, 0);
    c->sad_cache.clear();
    c->sched.clear();
    c->oe_S.clear(); c->oe_T.clear(); c->oe_V.clear();
    c->have_geom = true;
    c->have_basis = false;
    c->have_quartets = false;
    return FK_OK;
}

int fk_set_basis(fk_ctx *c, int nshell, const int *shell_atom, const int *shell_l, const int *shell_nprim,
                 const double *exps, const double *coefs)
{
    if (!c) return FK_ERR_ARG;
    if (!c->have_geom) return fail(c, FK_ERR_STATE, "fk_set_basis: call fk_set_geometry first");
    if (nshell <= 0 || !shell_atom || !shell_l || !shell_nprim || !exps || !coefs)
        return fail(c, FK_ERR_ARG, "fk_set_basis: nshell must be > 0 and arrays non-null");
    int np = 0;
    for (int s = 0; s < nshell; ++s) {
        if (shell_atom[s] < 0 || shell_atom[s] >= c->natom)
            return fail(c, FK_ERR_ARG, "fk_set_basis: shell %d on atom %d of %d", s, shell_atom[s], c->natom);
        if (shell_l[s] < 0 || shell_l[s] > FK_MAX_L)
            return fail(c, FK_ERR_UNSUPPORTED, "fk_set_basis: shell %d has l = %d (max %d)", s, shell_l[s], FK_MAX_L);
        if (shell_nprim[s] < 1 || shell_nprim[s] > FK_MAX_K)
            return fail(c, FK_ERR_UNSUPPORTED, "fk_set_basis: shell %d has %d primitives (1..%d)", s, shell_nprim[s],
                        FK_MAX_K);
        np += shell_nprim[s];
    }
    for (int i = 0; i < np; ++i) {
        if (!(exps[i] > 0) || !std::isfinite(exps[i]))
            return fail(c, FK_ERR_ARG, "fk_set_basis: exponent %d is %g (must be > 0)", i, exps[i]);
        if (!std::isfinite(coefs[i])) return fail(c, FK_ERR_ARG, "fk_set_basis: coefficient %d not finite", i);
    }
    c->nshell = nshell;
    c->sh_atom.assign(shell_atom, shell_atom + nshell);
    c->sh_l.assign(shell_l, shell_l + nshell);
    c->sh_nprim.assign(shell_nprim, shell_nprim + nshell);
    c->sh_poff.assign(nshell + 1, 0);
    c->sh_bf.assign(nshell + 1, 0);
    for (int s = 0; s < nshell; ++s) {
        c->sh_poff[s + 1] = c->sh_poff[s] + shell_nprim[s];
        c->sh_bf[s + 1] = c->sh_bf[s] + ncart(shell_l[s]);
    }
    c->nbf = c->sh_bf[nshell];
    c->exps.assign(exps, exps + np);
    c->coef_in.assign(coefs, coefs + np);
    c->sad_cache.clear();
    c->sched.clear();
    c->oe_S.clear(); c->oe_T.clear(); c->oe_V.clear();
    c->coef.assign(np, 0.0);
    c->bf_scale.assign(c->nbf, 1.0);
    for (int s = 0; s < nshell; ++s) {
        const int l = shell_l[s];
        normalise_shell(l, &c->exps[c->sh_poff[s]], coefs + c->sh_poff[s], shell_nprim[s], &c->coef[c->sh_poff[s]]);
        for (int k = 0; k < ncart(l); ++k) {
            int x, y, z;
            cart_exps(l, k, x, y, z);
            c->bf_scale[c->sh_bf[s] + k] = std::sqrt(dfact(2 * l - 1) / (dfact(2 * x - 1) * dfact(2 * y - 1) * dfact(2 * z - 1)));
        }
    }
    c->have_basis = true;
    c->have_quartets = false;
    int rc;
    if (c->device >= 0) {
        hipSetDevice(c->device);
        if ((rc = dev_upload(c, c->d_bf_scale, c->bf_scale.data(), c->bf_scale.size()))) return rc;
    }
    if ((rc = layout_molecules(c))) { c->have_basis = false; return rc; }
    return FK_OK;
}

int fk_set_molecules(fk_ctx *c, int nmol, const int *atom_mol)
{
    if (!c) return FK_ERR_ARG;
    if (!c->have_geom) return fail(c, FK_ERR_STATE, "fk_set_molecules: geometry not set");
    if (nmol < 1 || !atom_mol) return fail(c, FK_ERR_ARG, "fk_set_molecules: nmol must be >= 1 and atom_mol non-null");
    for (int a = 0; a < c->natom; ++a) {
        if (atom_mol[a] < 0 || atom_mol[a] >= nmol || (a > 0 && atom_mol[a] < atom_mol[a - 1]))
            return fail(c, FK_ERR_ARG, "fk_set_molecules: atom %d: molecule indices must be 0..nmol-1, non-decreasing", a);
    }
    for (int m = 0; m < nmol; ++m)
        if (std::find(atom_mol, atom_mol + c->natom, m) == atom_mol + c->natom)
            return fail(c, FK_ERR_ARG, "fk_set_molecules: molecule %d has no atoms", m);
    c->atom_mol.assign(atom_mol, atom_mol + c->natom);
    c->sched.clear();
    c->have_quartets = false;
    if (c->have_basis) {
        int rc;
        if ((rc = layout_molecules(c))) { c->have_basis = false; return rc; }
    }
    return FK_OK;
}

int fk_build_quartets(fk_ctx *c, const fk_screen_opts *o)
{
    if (!c) return FK_ERR_ARG;
    if (!c->have_basis) return fail(c, FK_ERR_STATE, "fk_build_quartets: basis not set");
    fk_screen_opts opts = {1e-10, 0.0, 1, 0, 0.0, 0.0};
    if (o) opts = *o;
    if (!(opts.tau >= 0) || !(opts.tau_prim >= 0)) return fail(c, FK_ERR_ARG, "fk_build_quartets: negative threshold");
    if (!(opts.tau_fp32 >= 0)) return fail(c, FK_ERR_ARG, "fk_build_quartets: negative tau_fp32");
    if (!(opts.tau_k >= 0)) return fail(c, FK_ERR_ARG, "fk_build_quartets: negative tau_k");
    if (opts.block_tasks != 0 && opts.block_tasks != -1)
        return fail(c, FK_ERR_ARG, "fk_build_quartets: block_tasks must be 0 or -1");
    if (opts.bra_block < 0 || opts.bra_block > FK_MAX_BRA_BLOCK)
        return fail(c, FK_ERR_ARG, "fk_build_quartets: bra_block must be 0..%d", FK_MAX_BRA_BLOCK);
    c->opts = opts;
    const bool dev = c->device >= 0;
    if (dev) hipSetDevice(c->device);
    // 1. all unique shell pairs with their primitive pairs
    c->pr_sa.clear(); c->pr_sb.clear(); c->pr_ppoff.clear(); c->pr_npp.clear(); c->pr_cls.clear();
    c->pr_AB.clear(); c->pr_G.clear(); c->pp.clear();
    for (int a = 0; a < c->nshell; ++a)
        for (int b = 0; b <= a; ++b) {
            if (c->sh_mol[a] != c->sh_mol[b]) continue;  // molecules of a batch do not interact
            int sa, sb;
            orient(c, a, b, sa, sb);
            make_pair(c, sa, sb);
        }
    const int npair = (int)c->pr_sa.size();
    int rc;
    if (dev && (rc = upload_pairs(c))) return rc;
    // 2a. primitive Schwarz factors, primitive order and pruning
    if ((rc = prim_schwarz(c, dev))) return rc;
    prune_primitives(c, opts.tau_prim);
    if (dev && (rc = upload_pairs(c))) return rc;
    // 2b. Schwarz factors from the diagonal quartets (ab|ab)
    for (int P = 0; P < NPC; ++P) {
        std::vector<int> idx, qs;
        for (int p = 0; p < npair; ++p)
            if (c->pr_cls[p] == P) { idx.push_back(p); qs.push_back(p); qs.push_back(p); }
        if (idx.empty()) continue;
        std::vector<double> out;
        if ((rc = eval_quartets(c, P, P, qs, out, dev))) return rc;
        const int la = c->sh_l[c->pr_sa[idx[0]]], lb = c->sh_l[c->pr_sb[idx[0]]];
        const int na = ncart(la), nb = ncart(lb), nout = na * nb * na * nb;
        for (size_t q = 0; q < idx.size(); ++q) {
            const int p = idx[q];
            const double *sa = &c->bf_scale[c->sh_bf[c->pr_sa[p]]], *sb = &c->bf_scale[c->sh_bf[c->pr_sb[p]]];
            double g = 0;
            for (int ia = 0; ia < na; ++ia)
                for (int ib = 0; ib < nb; ++ib) {
                    const double v = out[q * nout + ((ia * nb + ib) * na + ia) * nb + ib] * sa[ia] * sa[ia] * sb[ib] * sb[ib];
                    g = std::max(g, std::sqrt(std::fabs(v)));
                }
            if (!std::isfinite(g)) return fail(c, FK_ERR_ARG, "non-finite Schwarz factor for shell pair %d", p);
            c->pr_G[p] = g;
        }
    }
    const double gmax = npair ? *std::max_element(c->pr_G.begin(), c->pr_G.end()) : 0.0;
    // 3. class lists sorted by (primitive-pair count, G descending)
    c->npair_kept = 0;
    for (int P = 0; P < NPC; ++P) { c->cls_list[P].clear(); c->cls_groups[P].clear(); }
    for (int p = 0; p < npair; ++p) {
        if (opts.tau > 0 && c->pr_G[p] * gmax < opts.tau) continue;
        c->cls_list[c->pr_cls[p]].push_back(p);
        ++c->npair_kept;
    }
    c->ket_list_all.clear();
    for (int P = 0; P < NPC; ++P) {
        auto &L = c->cls_list[P];
        std::stable_sort(L.begin(), L.end(), [&](int x, int y) {
            const int mx = c->sh_mol[c->pr_sa[x]], my = c->sh_mol[c->pr_sa[y]];
            if (mx != my) return mx < my;
            if (c->pr_npp[x] != c->pr_npp[y]) return c->pr_npp[x] > c->pr_npp[y];
            return c->pr_G[x] > c->pr_G[y];
        });
        // groups: runs of one molecule and one primitive-pair count
        for (size_t i = 0; i < L.size();) {
            size_t j = i;
            const int mi = c->sh_mol[c->pr_sa[L[i]]];
            while (j < L.size() && c->pr_npp[L[j]] == c->pr_npp[L[i]] && c->sh_mol[c->pr_sa[L[j]]] == mi) ++j;
            c->cls_groups[P].push_back({(int)i, (int)j});
            i = j;
        }
        c->ket_off[P] = (int)c->ket_list_all.size();
        c->ket_list_all.insert(c->ket_list_all.end(), L.begin(), L.end());
    }
    c->ket_off[NPC] = (int)c->ket_list_all.size();
    {
        const size_t nl = c->ket_list_all.size();
        c->lst_sa.assign(nl, 0); c->lst_sb.assign(nl, 0);
        c->lst_sa_loc.assign(nl, 0); c->lst_sb_loc.assign(nl, 0);
        c->lst_CD.assign(3 * std::max<size_t>(nl, 1), 0.0); c->lst_G.assign(nl, 0.0);
        for (size_t q = 0; q < nl; ++q) {
            const int p = c->ket_list_all[q];
            c->lst_sa[q] = c->pr_sa[p];
            c->lst_sb[q] = c->pr_sb[p];
            c->lst_sa_loc[q] = c->sh_loc[c->pr_sa[p]];
            c->lst_sb_loc[q] = c->sh_loc[c->pr_sb[p]];
            for (int k = 0; k < 3; ++k) c->lst_CD[k * nl + q] = c->pr_AB[3 * p + k];
            c->lst_G[q] = c->pr_G[p];
        }
        c->groups.clear();
        c->cls_group0.assign(NPC + 1, 0);
        c->ppT.clear();
        for (int P = 0; P < NPC; ++P) {
            c->cls_group0[P] = (int)c->groups.size();
            for (const auto &g : c->cls_groups[P]) {
                FkGroup G;
                G.begin = c->ket_off[P] + g.first;
                G.len = g.second - g.first;
                G.npp = c->pr_npp[c->cls_list[P][g.first]];
                G.mol = c->sh_mol[c->pr_sa[c->cls_list[P][g.first]]];
                G.base = (long long)c->ppT.size();
                c->ppT.resize(c->ppT.size() + (size_t)G.npp * FK_NFLD * G.len);
                for (int r = 0; r < G.len; ++r) {
                    const int p = c->ket_list_all[G.begin + r];
                    for (int j = 0; j < G.npp; ++j)
                        for (int f = 0; f < FK_NFLD; ++f)
                            c->ppT[G.base + ((size_t)j * FK_NFLD + f) * G.len + r] =
                                c->pp[((size_t)c->pr_ppoff[p] + j) * FK_NPP_REC + f];
                }
                c->groups.push_back(G);
            }
        }
        c->cls_group0[NPC] = (int)c->groups.size();
    }
    // columns of the block tasks' K rows: the functions of each shell type,
    // per molecule in shell order
    {
        const int nm = c->nmol;
        c->krow_col.assign(c->nshell, 0);
        c->krow_cnt.assign(4 * nm, 0);
        c->krow_off.assign(4 * nm, 0);
        for (int s = 0; s < c->nshell; ++s) {
            const int l = std::min(c->sh_l[s], 3);
            c->krow_col[s] = c->krow_cnt[4 * c->sh_mol[s] + l];
            c->krow_cnt[4 * c->sh_mol[s] + l] += c->sh_lend[s] - c->sh_lbf[s];
        }
        int tot = 0;
        for (int k = 0; k < 4 * nm; ++k) { c->krow_off[k] = tot; tot += c->krow_cnt[k]; }
        c->krow_fn.assign(std::max(tot, 1), 0);
        std::vector<int> fill(4 * nm, 0);
        for (int s = 0; s < c->nshell; ++s) {
            const int k = 4 * c->sh_mol[s] + std::min(c->sh_l[s], 3);
            for (int f = c->sh_lbf[s]; f < c->sh_lend[s]; ++f) c->krow_fn[c->krow_off[k] + fill[k]++] = f;
        }
    }
    c->tasks.clear();
    // 4. tiles per quartet class (P >= Q): bra blocks from class P, kets from class Q
    const int bra_block = opts.bra_block > 0 ? std::min(opts.bra_block, FK_MAX_BRA_BLOCK) : 8;
    c->tiles.clear();
    c->blocks.clear();
    c->blk_bra.clear();
    c->blk_pos.clear();
    c->blk_nppsum.clear();
    c->qclasses.clear();
    c->flops_schwarz = 0;
    c->nq_schwarz = 0;
    for (int P = 0; P < NPC; ++P)
        for (int Q = 0; Q <= P; ++Q) {
            const auto &LP = c->cls_list[P], &LQ = c->cls_list[Q];
            if (LP.empty() || LQ.empty()) continue;
            QuartetClass qc;
            qc.P = P; qc.Q = Q;
            if (fk_kernels_class_info(P, Q, &qc.info))
                return fail(c, FK_ERR_UNSUPPORTED, "quartet class (%d|%d) is not built into this library", P, Q);
            const auto sit = c->sched.find(P * NPC + Q);
            const fk_ctx::ClassSched sch = sit == c->sched.end() ? fk_ctx::ClassSched{} : sit->second;
            if (sch.alt && qc.info.alt_team > 0) {
                // the class's team-per-quartet kernel: a lane per component of a
                qc.info.wave_per_quartet = 1;
                qc.info.team_size = qc.info.alt_team;
                qc.info.bra_block = qc.info.alt_bra_block;
                qc.info.ket_outer = 0;
                qc.info.hgp = 0;
            }
            // precision split: the class gets a second, FP32 launch over the same
            // tiles (not for the f-f bra kernels, which are FP64 only); per bra
            // and tile the kernels send the work to exactly one of the two
            const bool split = opts.tau_fp32 > 0 && qc.info.wave_per_quartet != 3;
            // kets per tile: a full wave of kets for lane-per-quartet kernels, two
            // rounds of teams for team kernels, two kets for wave-per-quartet
            const int ts = std::max(1, qc.info.team_size);
            int tile_kets = qc.info.wave_per_quartet == 0 ? 64 : std::max(1, 2 * (64 / ts));
            if (qc.info.wave_per_quartet != 0 && sch.kt > 0) tile_kets = std::min(64, sch.kt);
            qc.grid_frac = sch.gf;
            qc.engine = (sch.eng != 0 && qc.info.hgp) ? sch.eng : 0;
            const int qpw = qc.info.wave_per_quartet == 0 ? 64 : (qc.info.wave_per_quartet == 3 ? 1 : 64 / ts);
            int max_bra_npp = 1;
            for (int p : LP) max_bra_npp = std::max(max_bra_npp, c->pr_npp[p]);
            qc.bra_slot = max_bra_npp * FK_NFLD;
            qc.prec = 0;
            qc.nquartet = 0; qc.nprim = 0; qc.prim_slots = 0;
            std::vector<FkTile> tl;
            // bra blocks: the class's pairs ordered by (first shell, G descending),
            // cut into runs of at most bmax pairs with the same first shell
            int bmax = std::max(1, std::min(sch.bb > 0 ? std::min(sch.bb, FK_MAX_BRA_BLOCK) : bra_block, qc.info.bra_block));
            // block tasks (fk_screen_opts.block_tasks): the lane classes whose K rows
            // fit the LDS without costing waves per CU -- the ket-outer ones with
            // their four-wave workgroups, the others with workgroups of eight
            // waves (one Rys table for eight waves) and as many bras per block as
            // fit; decided here, since it may lower the bra block
            qc.krow_ncol = 0;
            qc.nw = 4;
            if (qc.info.wave_per_quartet == 0 && (qc.info.ket_outer > 0 || qc.info.wide > 0) &&
                opts.block_tasks == 0 && (sch.bt < 0 ? qc.info.ket_outer > 0 : sch.bt != 0)) {
                int ncol = 0;
                for (int m = 0; m < c->nmol; ++m)
                    ncol = std::max(ncol, c->krow_cnt[4 * m + qc.info.lc] +
                                              (qc.info.lc != qc.info.ld ? c->krow_cnt[4 * m + qc.info.ld] : 0));
                // waves per CU of a launch (0: the LDS does not fit); without a
                // device the LDS bound alone decides
                auto waves_cu = [&](int nw, int nbk, int nc) {
                    const int lds = fk_kernels_jk_lds_bytes(P, Q, qc.bra_slot, nc, 0, nbk, nw);
                    if (lds < 0 || lds > (nw == 4 ? kKrowLdsMax : kKrowLdsMaxWide)) return 0;
                    if (!dev) return nw;
                    int nb = 0;
                    if (fk_kernels_max_blocks(P, Q, lds, qc.engine, 0, nw, &nb) != 0) return 0;
                    return nb * nw;
                };
                const int w0 = dev ? waves_cu(4, bmax, 0) : 1;
                if (ncol > 0 && w0 > 0) {
                    if (qc.info.ket_outer > 0) {
                        if (waves_cu(4, bmax, ncol) >= w0) qc.krow_ncol = ncol;
                    } else if (qc.engine == 0) {
                        for (int b = bmax; b >= 1; b = b / 2)
                            if (waves_cu(qc.info.wide, b, ncol) >= w0) {
                                qc.krow_ncol = ncol;
                                qc.nw = qc.info.wide;
                                bmax = b;
                                break;
                            }
                    }
                }
            }
            qc.krow_nbk = qc.krow_ncol > 0 ? bmax : 0;
            qc.bra_block = bmax;
            qc.kets_per_tile = tile_kets;
            std::vector<int> ord(LP.size());
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
                if (c->pr_sa[LP[x]] != c->pr_sa[LP[y]]) return c->pr_sa[LP[x]] < c->pr_sa[LP[y]];
                return c->pr_G[LP[x]] > c->pr_G[LP[y]];
            });
            // length of the prefix of [first, last) (G descending) with G_bra G_ket >= thr:
            // the same product the kernels test
            auto prefix = [&](int first, int last, double gb, double thr) {
                int lo = first, hi = last;
                while (lo < hi) {
                    const int mid = (lo + hi) / 2;
                    if (gb * c->pr_G[LQ[mid]] >= thr) lo = mid + 1; else hi = mid;
                }
                return lo - first;
            };
            for (size_t i0 = 0; i0 < ord.size();) {
                size_t i1 = i0;
                const int sa0 = c->pr_sa[LP[ord[i0]]];
                while (i1 < ord.size() && (int)(i1 - i0) < bmax && c->pr_sa[LP[ord[i1]]] == sa0) ++i1;
                const int blk = (int)c->blocks.size();
                c->blocks.push_back(FkBraBlock{(int)c->blk_bra.size(), (int)(i1 - i0)});
                int64_t nppsum = 0;
                for (size_t x = i0; x < i1; ++x) {
                    c->blk_bra.push_back(LP[ord[x]]);
                    c->blk_pos.push_back(c->ket_off[P] + ord[x]);
                    nppsum += c->pr_npp[LP[ord[x]]];
                }
                c->blk_nppsum.push_back(nppsum);
                const int bmol = c->sh_mol[sa0];
                for (size_t gi = 0; gi < c->cls_groups[Q].size(); ++gi) {
                    const auto &g = c->cls_groups[Q][gi];
                    if (c->sh_mol[c->pr_sa[LQ[g.first]]] != bmol) continue;  // kets of the bra's molecule only
                    const int gnpp = c->pr_npp[LQ[g.first]];
                    // ket range [0, hi) of the group: the union of the bras' prefixes
                    int hi = 0;
                    for (size_t x = i0; x < i1; ++x) {
                        const int pb = ord[x], bra = LP[pb];
                        const double gb = c->pr_G[bra];
                        int cnt = opts.tau > 0 ? prefix(g.first, g.second, gb, opts.tau) : g.second - g.first;
                        if (P == Q) cnt = std::min(cnt, std::max(0, pb + 1 - g.first));
                        if (cnt <= 0) continue;
                        hi = std::max(hi, cnt);
                        qc.nquartet += cnt;
                        qc.nprim += (int64_t)cnt * c->pr_npp[bra] * gnpp;
                    }
                    for (int kk = 0; kk < hi; kk += tile_kets) {
                        FkTile t;
                        t.blk = blk;
                        t.ket_begin = c->ket_off[Q] + g.first + kk;
                        t.ket_count = std::min(tile_kets, hi - kk);
                        t.grp = (c->cls_group0[Q] + (int)gi) | ((P == Q) ? FK_TILE_SAME : 0);
                        tl.push_back(t);
                        // lane slots of the tile's primitive loops: rounds of
                        // (quartets per wave) kets, 64 lanes each (a group of
                        // waves per quartet for the wave kernels), for every bra
                        const int64_t rounds = (t.ket_count + qpw - 1) / qpw;
                        const int64_t lanes = qc.info.wave_per_quartet == 3 ? std::max(64, qc.info.team_size) : 64;
                        qc.prim_slots += rounds * lanes * nppsum * gnpp;
                    }
                }
                i0 = i1;
            }
            if (tl.empty()) continue;
            // most expensive tiles first (bra primitives x ket primitives x kets)
            auto cost = [&](const FkTile &t) {
                const FkGroup &gg = c->groups[t.grp & ~FK_TILE_SAME];
                return c->blk_nppsum[t.blk] * gg.npp * t.ket_count;
            };
            std::stable_sort(tl.begin(), tl.end(), [&](const FkTile &x, const FkTile &y) { return cost(x) > cost(y); });
            // block tasks: the tiles of one bra block, cut into chunks that share
            // the block's tiles round-robin (each a similar mix of costs),
            // largest chunks first; the class's tiles are stored in task order
            qc.ntask = 0;
            if (qc.krow_ncol > 0) {
                std::stable_sort(tl.begin(), tl.end(), [](const FkTile &x, const FkTile &y) { return x.blk < y.blk; });
                const int64_t ch = std::max<int64_t>(16, std::min<int64_t>(256, (int64_t)tl.size() / 4096));
                std::vector<std::vector<FkTile>> chunks;
                std::vector<double> ccost;
                for (size_t i = 0; i < tl.size();) {
                    size_t j = i;
                    while (j < tl.size() && tl[j].blk == tl[i].blk) ++j;
                    const int64_t len = (int64_t)(j - i), nch = (len + ch - 1) / ch;
                    const size_t c0 = chunks.size();
                    chunks.resize(c0 + nch);
                    ccost.resize(c0 + nch, 0.0);
                    for (int64_t k = 0; k < len; ++k) {
                        chunks[c0 + k % nch].push_back(tl[i + k]);
                        ccost[c0 + k % nch] += (double)cost(tl[i + k]);
                    }
                    i = j;
                }
                std::vector<int> ord_c(chunks.size());
                std::iota(ord_c.begin(), ord_c.end(), 0);
                std::stable_sort(ord_c.begin(), ord_c.end(), [&](int x, int y) { return ccost[x] > ccost[y]; });
                qc.task_off = (int64_t)c->tasks.size();
                tl.clear();
                for (int k : ord_c) {
                    c->tasks.push_back(int2{(int)tl.size(), (int)chunks[k].size()});
                    tl.insert(tl.end(), chunks[k].begin(), chunks[k].end());
                }
                qc.ntask = (int64_t)chunks.size();
            }
            qc.tile_off = (int64_t)c->tiles.size();
            qc.ntile = (int64_t)tl.size();
            c->tiles.insert(c->tiles.end(), tl.begin(), tl.end());
            c->flops_schwarz += qc.nprim * qc.flops_prim() + qc.nquartet * qc.flops_quartet();
            c->nq_schwarz += qc.nquartet;
            for (int k = 0; k < (split ? 2 : 1); ++k) {
                QuartetClass q = qc;
                q.prec = k;
                if (k == 1) {
                    // the FP32 launch shares the tiles; the Schwarz counts and the
                    // lane slots belong to the class once (the FP64 entry)
                    q.nquartet = 0; q.nprim = 0; q.prim_slots = 0;
                }
                q.blocks_per_cu = 1;
                if (dev) {
                    int nb = 0;
                    const int lds = fk_kernels_jk_lds_bytes(P, Q, q.bra_slot, q.ntask > 0 ? q.krow_ncol : 0,
                                                            q.info.wave_per_quartet, q.krow_nbk, q.nw);
                    if (fk_kernels_max_blocks(P, Q, lds, q.engine, q.info.wave_per_quartet, q.nw, &nb) == 0 && nb > 0)
                        q.blocks_per_cu = nb;
                }
                if ((int)c->qclasses.size() >= FK_MAX_QCLASS)
                    return fail(c, FK_ERR_STATE, "internal: more class launches than FK_MAX_QCLASS");
                c->qclasses.push_back(q);
            }
            order_for_xcds(c, c->qclasses.back());
        }
    if ((rc = validate_lists(c))) return rc;
    if (dev) {
        if (!c->ev_fork) HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        if (c->aux.empty()) {
            if ((rc = aux_streams(c, c->aux))) return rc;
            for (size_t k = 0; k < c->aux.size(); ++k) {
                hipEvent_t e;
                HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
                c->ev_join.push_back(e);
            }
        }
        if ((rc = dev_upload(c, c->d_pr_G, c->pr_G.data(), c->pr_G.size()))) return rc;
        if ((rc = dev_upload(c, c->d_ket, c->ket_list_all.data(), c->ket_list_all.size()))) return rc;
        if ((rc = dev_upload(c, c->d_lst_sa, c->lst_sa_loc.data(), c->lst_sa_loc.size()))) return rc;
        if ((rc = dev_upload(c, c->d_lst_sb, c->lst_sb_loc.data(), c->lst_sb_loc.size()))) return rc;
        if ((rc = dev_upload(c, c->d_lst_CD, c->lst_CD.data(), c->lst_CD.size()))) return rc;
        if ((rc = dev_upload(c, c->d_lst_G, c->lst_G.data(), c->lst_G.size()))) return rc;
        if ((rc = dev_upload(c, c->d_ppT, c->ppT.data(), c->ppT.size()))) return rc;
        if ((rc = dev_upload(c, c->d_groups, c->groups.data(), c->groups.size()))) return rc;
        if ((rc = dev_upload(c, c->d_tiles, c->tiles.data(), c->tiles.size()))) return rc;
        if ((rc = dev_upload(c, c->d_tasks, c->tasks.data(), c->tasks.size()))) return rc;
        if ((rc = dev_upload(c, c->d_krow_col, c->krow_col.data(), c->krow_col.size()))) return rc;
        if ((rc = dev_upload(c, c->d_krow_cnt, c->krow_cnt.data(), c->krow_cnt.size()))) return rc;
        if ((rc = dev_upload(c, c->d_krow_off, c->krow_off.data(), c->krow_off.size()))) return rc;
        if ((rc = dev_upload(c, c->d_krow_fn, c->krow_fn.data(), c->krow_fn.size()))) return rc;
        const size_t nn = (size_t)c->mol_base[c->nmol];
        if ((rc = dev_upload<double>(c, c->d_Ds, nullptr, nn))) return rc;
        if ((rc = dev_upload<double>(c, c->d_Dsh, nullptr, (size_t)c->mol_shbase[c->nmol]))) return rc;
        if ((rc = dev_upload<double>(c, c->d_X, nullptr, 2 * nn * FK_XCD_COPIES))) return rc;
        if ((rc = dev_upload<unsigned long long>(c, c->d_cnt, nullptr, 2 * FK_MAX_QCLASS))) return rc;
        if ((rc = dev_upload(c, c->d_blocks, c->blocks.data(), c->blocks.size()))) return rc;
        if ((rc = dev_upload(c, c->d_blk_bra, c->blk_bra.data(), c->blk_bra.size()))) return rc;
        if ((rc = dev_upload(c, c->d_blk_pos, c->blk_pos.data(), c->blk_pos.size()))) return rc;
    }
    c->have_quartets = true;
    c->jeng_valid = false;
    c->stats_pending = false;
    return FK_OK;
}

int fk_info(const fk_ctx *c, fk_info_t *info)
{
    if (!c || !info) return FK_ERR_ARG;
    std::memset(info, 0, sizeof *info);
    info->nbf = c->nbf;
    info->nshell = c->nshell;
    info->natom = c->natom;
    info->nelec = c->nelec;
    info->npair = (int)c->pr_sa.size();
    info->npair_kept = c->npair_kept;
    int ncls = 0;
    for (int P = 0; P < NPC; ++P) ncls += !c->cls_list[P].empty();
    info->nclass_pair = ncls;
    info->nquartet_class = (int)c->qclasses.size();
    info->nprim_pair = (int64_t)(c->pp.size() / FK_NPP_REC);
    info->nquartet_schwarz = c->nq_schwarz;
    info->ntile = (int64_t)c->tiles.size();
    info->flops_schwarz = c->flops_schwarz;
    info->nmol = c->nmol;
    info->nmat = c->mol_base.empty() ? 0 : c->mol_base[c->nmol];
    return FK_OK;
}

int fk_molecule_layout(const fk_ctx *c, int *nbf, int64_t *offset)
{
    if (!c || !nbf || !offset) return FK_ERR_ARG;
    if (!c->have_basis) return FK_ERR_STATE;
    for (int m = 0; m < c->nmol; ++m) nbf[m] = c->mol_nbf[m];
    for (int m = 0; m <= c->nmol; ++m) offset[m] = c->mol_base[m];
    return FK_OK;
}

}  // extern "C"

namespace {

// Device buffers one J/K build works in: the component-scaled density, the
// shell-block maxima, ncopy copies of (X_J, X_K) xcopy doubles apart, and the
// per-launch counters.
struct JKBufs {
    double *Ds, *Dsh, *X;
    long long xcopy;
    int ncopy;
    unsigned long long *cnt;
};

constexpr int kJengNB = FK_JENG_MAX_LP + 1;

int ensure_dfit(fk_ctx *c);  // density-bound data, below

// Lists and buffers of the J engine for the current quartet lists: per pair
// the offset of its J_p block, per ket group the offset of its D_q block, and
// the work tiles (bra pair, <= 64 kets of one group) of every bra class
// against every ket class, bucketed by (la + lb, lc + ld), each bucket
// ordered by cost (bra x ket primitives x kets), most expensive first.
int ensure_jeng(fk_ctx *c)
{
    if (c->jeng_valid) return FK_OK;
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "FK_J_ENGINE: one molecule per context");
    for (int s = 0; s < c->nshell; ++s)
        if (c->sh_l[s] > 2) return fail(c, FK_ERR_UNSUPPORTED, "FK_J_ENGINE: built for s, p and d shells");
    const int npair = (int)c->pr_sa.size();
    std::vector<long long> jp_off(npair);
    long long njp = 0;
    for (int p = 0; p < npair; ++p) {
        jp_off[p] = njp;
        njp += (long long)c->pr_npp[p] * nherm_host(c->sh_l[c->pr_sa[p]] + c->sh_l[c->pr_sb[p]]);
    }
    const int ng = (int)c->groups.size();
    std::vector<long long> dq_base(ng, 0);
    std::vector<int> pos_grp(c->ket_list_all.size(), 0);
    long long ndq = 0;
    for (int Q = 0; Q < NPC; ++Q)
        for (size_t gi = 0; gi < c->cls_groups[Q].size(); ++gi) {
            const int g = c->cls_group0[Q] + (int)gi;
            const FkGroup &G = c->groups[g];
            const int lq = c->sh_l[c->lst_sa[G.begin]] + c->sh_l[c->lst_sb[G.begin]];
            dq_base[g] = ndq;
            ndq += (long long)G.npp * nherm_host(lq) * G.len;
            for (int r = 0; r < G.len; ++r) pos_grp[G.begin + r] = g;
        }
    std::vector<std::vector<FkJengTile>> bucket(kJengNB * kJengNB);
    const double tau = c->opts.tau;
    for (int P = 0; P < NPC; ++P) {
        const auto &LP_ = c->cls_list[P];
        if (LP_.empty()) continue;
        const int lp = c->sh_l[c->pr_sa[LP_[0]]] + c->sh_l[c->pr_sb[LP_[0]]];
        for (int Q = 0; Q < NPC; ++Q) {
            const auto &LQ_ = c->cls_list[Q];
            if (LQ_.empty()) continue;
            const int lq = c->sh_l[c->pr_sa[LQ_[0]]] + c->sh_l[c->pr_sb[LQ_[0]]];
            auto &tl = bucket[lp * kJengNB + lq];
            for (int bra : LP_) {
                const double gb = c->pr_G[bra];
                for (size_t gi = 0; gi < c->cls_groups[Q].size(); ++gi) {
                    const auto &g = c->cls_groups[Q][gi];
                    int cnt = g.second - g.first;
                    if (tau > 0) {  // prefix with G_bra G_ket >= tau (G descending in a group)
                        int lo = g.first, hi = g.second;
                        while (lo < hi) {
                            const int mid = (lo + hi) / 2;
                            if (gb * c->pr_G[LQ_[mid]] >= tau) lo = mid + 1; else hi = mid;
                        }
                        cnt = lo - g.first;
                    }
                    for (int kk = 0; kk < cnt; kk += 64)
                        tl.push_back(FkJengTile{bra, c->ket_off[Q] + g.first + kk, std::min(64, cnt - kk),
                                                c->cls_group0[Q] + (int)gi});
                }
            }
            (void)lq;
        }
    }
    std::vector<FkJengTile> all;
    c->jeng_toff.assign(kJengNB * kJengNB + 1, 0);
    for (int k = 0; k < kJengNB * kJengNB; ++k) {
        auto &tl = bucket[k];
        auto cost = [&](const FkJengTile &t) {
            return (long long)c->pr_npp[t.bra] * c->groups[t.grp].npp * t.ket_count;
        };
        std::stable_sort(tl.begin(), tl.end(), [&](const FkJengTile &x, const FkJengTile &y) { return cost(x) > cost(y); });
        c->jeng_toff[k] = (int64_t)all.size();
        all.insert(all.end(), tl.begin(), tl.end());
    }
    c->jeng_toff[kJengNB * kJengNB] = (int64_t)all.size();
    int rc;
    if ((rc = dev_upload(c, c->d_jeng_tiles, all.data(), all.size())) || (rc = dev_upload(c, c->d_jp_off, jp_off.data(), jp_off.size())) ||
        (rc = dev_upload(c, c->d_dq_base, dq_base.data(), dq_base.size())) ||
        (rc = dev_upload(c, c->d_pos_grp, pos_grp.data(), pos_grp.size())) ||
        (rc = dev_upload<double>(c, c->d_jp, nullptr, (size_t)std::max<long long>(njp, 1))) ||
        (rc = dev_upload<double>(c, c->d_dq, nullptr, (size_t)std::max<long long>(ndq, 1))))
        return rc;
    c->jp_n = (size_t)njp;
    if ((rc = ensure_dfit(c))) return rc;
    c->jeng_valid = true;
    return FK_OK;
}

// Device data of the density-decay fit for one molecule: the atom of every
// function, the atoms' positions, the bin width (the largest interatomic
// distance over FK_DFIT_BINS - 1 bins), and per shell its centre, R (largest
// distance to the partner shell of a pair with G >= tau) and G (largest pair
// factor).
int ensure_dfit(fk_ctx *c)
{
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "density bound: one molecule per context");
    std::vector<int> bfa(c->nbf);
    for (int s = 0; s < c->nshell; ++s)
        for (int k = c->sh_bf[s]; k < c->sh_bf[s] + ncart(c->sh_l[s]); ++k) bfa[k] = c->sh_atom[s];
    double rmax = 0;
    for (int a = 0; a < c->natom; ++a)
        for (int b = 0; b < a; ++b) {
            double r2 = 0;
            for (int k = 0; k < 3; ++k) r2 += (c->xyz[3 * a + k] - c->xyz[3 * b + k]) * (c->xyz[3 * a + k] - c->xyz[3 * b + k]);
            rmax = std::max(rmax, std::sqrt(r2));
        }
    c->dfit_dr = std::max(rmax, 1.0) / (FK_DFIT_BINS - 1);
    std::vector<double> ks(5 * (size_t)c->nshell, 0.0);
    for (int s = 0; s < c->nshell; ++s)
        for (int k = 0; k < 3; ++k) ks[5 * s + k] = c->xyz[3 * c->sh_atom[s] + k];
    for (size_t p = 0; p < c->pr_sa.size(); ++p) {
        const int x = c->pr_sa[p], y = c->pr_sb[p];
        const double g = c->pr_G[p];
        double r2 = 0;
        for (int k = 0; k < 3; ++k) r2 += (ks[5 * x + k] - ks[5 * y + k]) * (ks[5 * x + k] - ks[5 * y + k]);
        for (int z : {x, y}) {
            ks[5 * z + 4] = std::max(ks[5 * z + 4], g);
            if (g >= c->opts.tau) ks[5 * z + 3] = std::max(ks[5 * z + 3], std::sqrt(r2));
        }
    }
    int rc;
    if ((rc = dev_upload(c, c->d_bf_atom, bfa.data(), bfa.size())) || (rc = dev_upload(c, c->d_atom_xyz, c->xyz.data(), c->xyz.size())) ||
        (rc = dev_upload(c, c->d_ks_shell, ks.data(), ks.size())) || (rc = dev_upload<double>(c, c->d_dfit, nullptr, 2)) ||
        (rc = dev_upload<unsigned long long>(c, c->d_dfit_bins, nullptr, FK_DFIT_BINS)))
        return rc;
    return FK_OK;
}

// J by the J engine into X_J (block per bra pair; see k_jeng_jab).
int jeng_build(fk_ctx *c, const JKBufs &b, hipStream_t st)
{
    if (fk_kernels_launch_fill(c->d_jp.p, (long long)c->jp_n, st)) return fail(c, FK_ERR_HIP, "fill kernel launch failed");
    const int nlist = (int)c->ket_list_all.size();
    for (int Q = 0; Q < NPC; ++Q) {
        if (c->cls_list[Q].empty()) continue;
        FkJengDqArgs a;
        a.groups = c->d_groups.p; a.pos_grp = c->d_pos_grp.p;
        a.pos0 = c->ket_off[Q]; a.npos = (int)c->cls_list[Q].size();
        a.lst_sa = c->d_lst_sa.p; a.lst_sb = c->d_lst_sb.p; a.lst_CD = c->d_lst_CD.p; a.nlist = nlist;
        a.ppT = c->d_ppT.p; a.sh_bf = c->d_sh_bf.p; a.Ds = b.Ds; a.n = c->nbf;
        a.dq_base = c->d_dq_base.p; a.dq = c->d_dq.p;
        const int p0 = c->cls_list[Q][0];
        if (fk_jeng_launch_dq(c->sh_l[c->pr_sa[p0]], c->sh_l[c->pr_sb[p0]], &a, st))
            return fail(c, FK_ERR_HIP, "J engine: D_q kernel launch failed");
    }
    FkJengArgs a;
    a.pair_ppoff = c->d_pr_ppoff.p; a.pair_npp = c->d_pr_npp.p; a.pair_G = c->d_pr_G.p; a.pp = c->d_pp.p;
    a.jp_off = c->d_jp_off.p; a.jp = c->d_jp.p; a.ppT = c->d_ppT.p; a.groups = c->d_groups.p;
    a.lst_G = c->d_lst_G.p; a.lst_sa = c->d_lst_sa.p; a.lst_sb = c->d_lst_sb.p;
    a.dq_base = c->d_dq_base.p; a.dq = c->d_dq.p; a.Dsh = b.Dsh; a.ns = c->nshell;
    a.dscreen = c->opts.density_screen && c->opts.tau > 0 ? 1 : 0;
    a.tau = c->opts.tau * c->dscreen_scale;
    for (int lp = 0; lp < kJengNB; ++lp)
        for (int lq = 0; lq < kJengNB; ++lq) {
            const int k = lp * kJengNB + lq;
            const int64_t nt = c->jeng_toff[k + 1] - c->jeng_toff[k];
            if (nt <= 0) continue;
            a.tiles = c->d_jeng_tiles.p + c->jeng_toff[k];
            a.ntiles = nt;
            a.rys_tab = c->d_rys.p + rys_staged_offset((lp + lq) / 2 + 1);
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nt + 3) / 4, 8LL * std::max(c->ncu, 1)));
            if (fk_jeng_launch_jp(lp, lq, &a, grid, st)) return fail(c, FK_ERR_HIP, "J engine: J_p kernel launch failed");
        }
    for (int P = 0; P < NPC; ++P) {
        if (c->cls_list[P].empty()) continue;
        FkJengJabArgs j;
        j.pairs = c->d_ket.p + c->ket_off[P]; j.npairs = (int)c->cls_list[P].size();
        j.pair_sa = c->d_pr_sa.p; j.pair_sb = c->d_pr_sb.p; j.pair_ppoff = c->d_pr_ppoff.p; j.pair_npp = c->d_pr_npp.p;
        j.pair_AB = c->d_pr_AB.p; j.pp = c->d_pp.p; j.jp_off = c->d_jp_off.p; j.jp = c->d_jp.p;
        j.sh_bf = c->d_sh_bf.p; j.XJ = b.X; j.n = c->nbf;
        const int p0 = c->cls_list[P][0];
        if (fk_jeng_launch_jab(c->sh_l[c->pr_sa[p0]], c->sh_l[c->pr_sb[p0]], &j, st))
            return fail(c, FK_ERR_HIP, "J engine: J_ab kernel launch failed");
    }
    return FK_OK;
}

// multi: the class launches may be spread over the caller's stream and the
// device's class-launch streams (never for the entry point without allocation,
// never while the caller's stream is being captured, never with per-class
// timing).
int build_jk_impl(fk_ctx *c, const double *D, double *J, double *K, unsigned flags, void *stream, const JKBufs &b,
                  bool multi)
{
    if ((flags & FK_J_ONLY) && (flags & FK_K_ONLY))
        return fail(c, FK_ERR_ARG, "fk_build_jk: FK_J_ONLY and FK_K_ONLY together");
    const int want = (flags & FK_J_ONLY) ? FK_WANT_J : ((flags & FK_K_ONLY) ? FK_WANT_K : FK_WANT_J | FK_WANT_K);
    if (!D || (!J && (want & FK_WANT_J)) || (!K && (want & FK_WANT_K)))
        return fail(c, FK_ERR_ARG, "fk_build_jk: null matrix pointer");
    if (!(want & FK_WANT_J)) J = nullptr;
    if (!(want & FK_WANT_K)) K = nullptr;
    const bool jeng = (flags & FK_J_ENGINE) && (want & FK_WANT_J);
    hipSetDevice(c->device);
    int rcj;
    if (jeng && (rcj = ensure_jeng(c))) return rcj;
    hipStream_t st = (hipStream_t)stream;
    // one nbf_m^2 block per molecule, concatenated
    const size_t nn = (size_t)c->mol_base[c->nmol];
    FkMolArgs ma;
    ma.sh_lbf = c->d_sh_bf.p; ma.sh_lend = c->d_sh_lend.p; ma.mol_sh0 = c->d_mol_sh0.p; ma.mol_nsh = c->d_mol_nsh.p;
    ma.mol_nbf = c->d_mol_nbf.p; ma.mol_bf0 = c->d_mol_bf0.p; ma.mol_base = c->d_mol_base.p;
    ma.mol_shbase = c->d_mol_shbase.p; ma.nmol = c->nmol; ma.nmat = (long long)nn; ma.nshmat = c->mol_shbase[c->nmol];
    const bool devp = flags & FK_DEVICE_PTRS;
    int rc;
    const double *Dd = D;
    double *Jd = J, *Kd = K;
    if (!devp) {
        if ((rc = dev_upload<double>(c, c->d_Din, nullptr, nn))) return rc;
        if ((rc = dev_upload<double>(c, c->d_Jout, nullptr, nn))) return rc;
        if ((rc = dev_upload<double>(c, c->d_Kout, nullptr, nn))) return rc;
        HIPCHK(c, hipMemcpyAsync(c->d_Din.p, D, nn * sizeof(double), hipMemcpyHostToDevice, st));
        Dd = c->d_Din.p;
        Jd = J ? c->d_Jout.p : nullptr;
        Kd = K ? c->d_Kout.p : nullptr;
    }
    if (fk_kernels_launch_prep(Dd, c->d_bf_scale.p, &ma, b.Ds, b.Dsh, st))
        return fail(c, FK_ERR_HIP, "prep kernel launch failed");
    if (fk_kernels_launch_fill(b.X, (long long)(2 * nn * b.ncopy), st) ||
        fk_kernels_launch_fill((double *)b.cnt, 2 * FK_MAX_QCLASS, st))
        return fail(c, FK_ERR_HIP, "fill kernel launch failed");
    c->timed = (flags & FK_TIME_CLASSES) != 0;
    if (c->timed)
        while (c->ev.size() < 2 * c->qclasses.size()) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    // with the J engine the Rys kernels form K only (or nothing)
    const int want_rys = jeng ? (want & FK_WANT_K) : want;
    // the density-bound fit the K classes read, before the other streams fork
    if (jeng && (want_rys & FK_WANT_K) && c->opts.tau_k > 0 &&
        fk_kernels_launch_dfit(Dd, c->nbf, c->d_bf_atom.p, c->d_atom_xyz.p, c->dfit_dr, c->d_dfit_bins.p, c->d_dfit.p, st))
        return fail(c, FK_ERR_HIP, "density-bound kernel launch failed");
    // Several streams: the classes, largest estimated work first, each go to
    // the stream with the least work so far, so that the long, latency-bound
    // launches of the small high-L classes run beside the large ones instead
    // of leaving most of the GPU idle.  The classes only add into X with
    // atomics; the other streams fork from and join the caller's.
    std::vector<hipStream_t> cls_st(c->qclasses.size(), st);
    int nfork = 0;
    const int nst = 1 + (int)c->aux.size();
    if (multi && nst > 1 && !c->timed && want_rys && c->qclasses.size() > 1) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(c, hipStreamIsCapturing(st, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            std::vector<size_t> ord(c->qclasses.size());
            std::iota(ord.begin(), ord.end(), 0);
            // estimated work per launch; an FP32 twin (its counts belong to the
            // FP64 entry) walks the same tiles and is given its twin's estimate
            std::vector<double> wk(c->qclasses.size(), 0.0);
            for (size_t i = 0; i < wk.size(); ++i) {
                const QuartetClass &q = c->qclasses[i];
                wk[i] = (double)q.prim_slots * q.flops_prim() + (double)q.nquartet * q.flops_quartet();
            }
            for (size_t i = 0; i < wk.size(); ++i)
                if (c->qclasses[i].prec != 0)
                    for (size_t j = 0; j < wk.size(); ++j)
                        if (c->qclasses[j].P == c->qclasses[i].P && c->qclasses[j].Q == c->qclasses[i].Q &&
                            c->qclasses[j].prec == 0)
                            wk[i] = wk[j];
            auto work = [&](size_t i) { return wk[i]; };
            std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
            std::vector<double> wsum(nst, 0.0);
            for (size_t i : ord) {
                const int k = (int)(std::min_element(wsum.begin(), wsum.end()) - wsum.begin());
                cls_st[i] = k == 0 ? st : c->aux[k - 1];
                wsum[k] += work(i);
            }
            HIPCHK(c, hipEventRecord(c->ev_fork, st));
            for (int k = 1; k < nst; ++k) HIPCHK(c, hipStreamWaitEvent(c->aux[k - 1], c->ev_fork, 0));
            nfork = nst - 1;
        }
    }
    for (size_t i = 0; i < c->qclasses.size(); ++i) {
        const QuartetClass &qc = c->qclasses[i];
        if (c->timed) HIPCHK(c, hipEventRecord(c->ev[2 * i], st));
        if (want_rys == 0) {
            if (c->timed) HIPCHK(c, hipEventRecord(c->ev[2 * i + 1], st));
            continue;
        }
        FkJKArgs a;
        a.sh_bf = c->d_sh_bf.p;
        a.mol_sh0 = c->d_mol_sh0.p;
        a.mol_nbf = c->d_mol_nbf.p;
        a.mol_nsh = c->d_mol_nsh.p;
        a.mol_base = c->d_mol_base.p;
        a.mol_shbase = c->d_mol_shbase.p;
        a.pair_sa = c->d_pr_sa.p;
        a.pair_sb = c->d_pr_sb.p;
        a.pair_ppoff = c->d_pr_ppoff.p;
        a.pair_npp = c->d_pr_npp.p;
        a.pair_AB = c->d_pr_AB.p;
        a.pair_G = c->d_pr_G.p;
        a.pp = c->d_pp.p;
        a.ket_list = c->d_ket.p;
        a.lst_sa = c->d_lst_sa.p;
        a.lst_sb = c->d_lst_sb.p;
        a.lst_CD = c->d_lst_CD.p;
        a.lst_G = c->d_lst_G.p;
        a.nlist = (int)c->ket_list_all.size();
        a.groups = c->d_groups.p;
        a.ppT = c->d_ppT.p;
        a.tiles = c->d_tiles.p + qc.tile_off;
        a.ntiles = (int)qc.ntile;
        a.tasks = qc.ntask > 0 ? c->d_tasks.p + qc.task_off : nullptr;
        a.ntask = (int)qc.ntask;
        a.krow_ncol = qc.krow_ncol;
        a.krow_col = c->d_krow_col.p;
        a.krow_cnt = c->d_krow_cnt.p;
        a.krow_off = c->d_krow_off.p;
        a.krow_fn = c->d_krow_fn.p;
        a.Dsh = b.Dsh;
        a.Ds = b.Ds;
        a.XJ = b.X;
        a.XK = b.X + nn;
        // workgroups add into copy blockIdx mod FK_XCD_COPIES; one copy: all alias it
        a.xcopy = b.ncopy > 1 ? b.xcopy : 0;
        a.dscreen = c->opts.density_screen && c->opts.tau > 0;
        a.want = want_rys;
        a.tau = c->opts.tau * c->dscreen_scale;
        // K beside the J engine: K blocks the fitted density bound proves
        // below tau_k are skipped (their quartets' other blocks still count)
        a.ks_shell = nullptr;
        a.ks_fit = nullptr;
        a.ks_tau = 0.0;
        if (jeng && c->opts.tau_k > 0) {
            a.ks_shell = c->d_ks_shell.p;
            a.ks_fit = c->d_dfit.p;
            a.ks_tau = c->opts.tau_k;
            a.dscreen = 1;
        }
        a.rys_tab = c->d_rys.p + rys_staged_offset(qc.info.nroot);
        a.counters = b.cnt + 2 * i;
        a.bra_slot = qc.bra_slot;
        a.prec = qc.prec;
        // a class with an FP32 twin splits its work by the per-quartet bound
        bool twin = false;
        for (const auto &o : c->qclasses) twin = twin || (o.P == qc.P && o.Q == qc.Q && o.prec != qc.prec);
        a.tau_fp32 = twin ? c->opts.tau_fp32 : 0.0;
        a.engine = qc.engine;
        a.kind = qc.info.wave_per_quartet;
        a.nw = qc.nw;
        a.krow_nbk = qc.krow_nbk;
        a.blocks = c->d_blocks.p;
        a.blk_bra = c->d_blk_bra.p;
        a.blk_pos = c->d_blk_pos.p;
        // Enough workgroups for the hardware to fill every CU to its register and
        // LDS limit; the persistent loop covers the rest.
        const int64_t wgs = qc.ntask > 0 ? qc.ntask : (qc.ntile + 3) / 4;
        const int64_t cap = std::max<int64_t>(1, (int64_t)(qc.grid_frac * std::max(8, qc.blocks_per_cu) * std::max(c->ncu, 1)));
        const int grid = (int)std::max<int64_t>(1, std::min(wgs, cap));
        if (fk_kernels_launch_jk(qc.P, qc.Q, &a, grid, cls_st[i]))
            return fail(c, FK_ERR_HIP, "J/K kernel launch failed for class (%d|%d)", qc.P, qc.Q);
        if (c->timed) HIPCHK(c, hipEventRecord(c->ev[2 * i + 1], st));
    }
    if (jeng && (rcj = jeng_build(c, b, st))) return rcj;
    for (int k = 0; k < nfork; ++k) {
        HIPCHK(c, hipEventRecord(c->ev_join[k], c->aux[k]));
        HIPCHK(c, hipStreamWaitEvent(st, c->ev_join[k], 0));
    }
    if (fk_kernels_launch_finalize(b.X, b.X + nn, b.xcopy, b.ncopy, c->d_bf_scale.p, &ma, Jd, Kd, st))
        return fail(c, FK_ERR_HIP, "finalize kernel launch failed");
    c->stats_pending = true;
    c->cnt_last = b.cnt;
    if (!devp) {
        if (J) HIPCHK(c, hipMemcpyAsync(J, Jd, nn * sizeof(double), hipMemcpyDeviceToHost, st));
        if (K) HIPCHK(c, hipMemcpyAsync(K, Kd, nn * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
    } else if (flags & FK_SYNC) {
        HIPCHK(c, hipStreamSynchronize(st));
    }
    return FK_OK;
}

}  // namespace

extern "C" {

int fk_density_bound(fk_ctx *c, const double *D, unsigned flags, double *H, double *Lambda)
{
    if (!c) return FK_ERR_ARG;
    if (!D || !H || !Lambda) return fail(c, FK_ERR_ARG, "fk_density_bound: null pointer");
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_density_bound: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_density_bound: call fk_build_quartets first");
    hipSetDevice(c->device);
    int rc;
    if ((rc = ensure_dfit(c))) return rc;
    const size_t nn = (size_t)c->nbf * c->nbf;
    const double *Dd = D;
    if (!(flags & FK_DEVICE_PTRS)) {
        if ((rc = dev_upload(c, c->d_Din, D, nn))) return rc;
        Dd = c->d_Din.p;
    }
    if (fk_kernels_launch_dfit(Dd, c->nbf, c->d_bf_atom.p, c->d_atom_xyz.p, c->dfit_dr, c->d_dfit_bins.p, c->d_dfit.p, nullptr))
        return fail(c, FK_ERR_HIP, "density-bound kernel launch failed");
    double f[2];
    HIPCHK(c, hipMemcpy(f, c->d_dfit.p, sizeof f, hipMemcpyDeviceToHost));
    *H = f[0];
    *Lambda = f[1];
    return FK_OK;
}

int fk_build_jk(fk_ctx *c, const double *D, double *J, double *K, unsigned flags, void *stream)
{
    if (!c) return FK_ERR_ARG;
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_build_jk: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_build_jk: call fk_build_quartets first");
    const size_t nn = (size_t)c->mol_base[c->nmol];
    const JKBufs b{c->d_Ds.p, c->d_Dsh.p, c->d_X.p, (long long)(2 * nn), FK_XCD_COPIES, c->d_cnt.p};
    return build_jk_impl(c, D, J, K, flags, stream, b, true);
}

int fk_build_jk_noalloc(fk_ctx *c, const double *D, double *J, double *K, unsigned flags, void *stream)
{
    if (!c) return FK_ERR_ARG;
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_build_jk_noalloc: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_build_jk_noalloc: call fk_build_quartets first");
    if (!(flags & FK_DEVICE_PTRS) || (flags & (FK_TIME_CLASSES | FK_J_ENGINE)))
        return fail(c, FK_ERR_ARG, "fk_build_jk_noalloc: needs FK_DEVICE_PTRS and takes no FK_TIME_CLASSES or FK_J_ENGINE");
    const long long nn = c->mol_base[c->nmol], nsh = c->mol_shbase[c->nmol];
    if (nn > FK_NOALLOC_MAX_NMAT || nsh > FK_NOALLOC_MAX_NSHMAT)
        return fail(c, FK_ERR_ARG,
                    "fk_build_jk_noalloc: %lld matrix elements and %lld shell-block elements exceed the "
                    "scratch limits (%d and %d); use fk_build_jk", nn, nsh, FK_NOALLOC_MAX_NMAT, FK_NOALLOC_MAX_NSHMAT);
    if (!c->scratch) return fail(c, FK_ERR_STATE, "fk_build_jk_noalloc: no scratch address for this device");
    double *base = c->scratch;
    const JKBufs b{base, base + 3 * (size_t)FK_NOALLOC_MAX_NMAT, base + FK_NOALLOC_MAX_NMAT, 0, 1,
                   (unsigned long long *)(base + 3 * (size_t)FK_NOALLOC_MAX_NMAT + FK_NOALLOC_MAX_NSHMAT)};
    return build_jk_impl(c, D, J, K, flags, stream, b, false);
}

int fk_stats(fk_ctx *c, fk_stats_t *s)
{
    if (!c || !s) return FK_ERR_ARG;
    std::memset(s, 0, sizeof *s);
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_stats: call fk_build_quartets first");
    std::vector<unsigned long long> cnt(2 * FK_MAX_QCLASS, 0);
    if (c->device >= 0 && c->stats_pending) {
        hipSetDevice(c->device);
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipMemcpy(cnt.data(), c->cnt_last, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    }
    s->nclass = (int)c->qclasses.size();
    for (size_t i = 0; i < c->qclasses.size(); ++i) {
        const auto &q = c->qclasses[i];
        s->la[i] = q.info.la; s->lb[i] = q.info.lb; s->lc[i] = q.info.lc; s->ld[i] = q.info.ld;
        s->quartets[i] = (int64_t)cnt[2 * i];
        s->prim_quartets[i] = (int64_t)cnt[2 * i + 1];
        s->flops_per_prim[i] = q.flops_prim();
        s->flops_per_quartet[i] = q.flops_quartet();
        s->engine[i] = q.engine;
        s->bra_block[i] = q.bra_block;
        s->kets_per_tile[i] = q.kets_per_tile;
        s->grid_fraction[i] = q.grid_frac;
        s->block_tasks[i] = q.ntask;
        s->waves_per_group[i] = q.nw;
        s->tiles[i] = q.ntile;
        s->team_size[i] = std::max(1, q.info.team_size);
        s->precision[i] = q.prec ? 32 : 64;
        s->prim_slots[i] = q.prim_slots;
        s->flops_total += s->prim_quartets[i] * q.flops_prim() + s->quartets[i] * q.flops_quartet();
        if (c->timed && 2 * i + 1 < c->ev.size()) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) s->class_ms[i] = ms;
        }
    }
    return FK_OK;
}

int fk_build_progress(fk_ctx *c, int *done, int *total)
{
    if (!c || !done || !total) return FK_ERR_ARG;
    *done = 0;
    *total = (int)c->qclasses.size();
    if (c->device < 0 || !c->timed) return fail(c, FK_ERR_STATE, "fk_build_progress: last build was not timed (FK_TIME_CLASSES)");
    hipSetDevice(c->device);
    for (size_t i = 0; i < c->qclasses.size() && 2 * i + 1 < c->ev.size(); ++i) {
        const hipError_t e = hipEventQuery(c->ev[2 * i + 1]);
        if (e == hipSuccess) ++*done;
        else if (e != hipErrorNotReady) return fail(c, FK_ERR_HIP, "fk_build_progress: %s", hipGetErrorString(e));
    }
    return FK_OK;
}

int fk_set_class_schedule(fk_ctx *c, int la, int lb, int lc, int ld, int bra_block, int kets_per_tile,
                          double grid_fraction)
{
    if (!c) return FK_ERR_ARG;
    if (la < lb || lc < ld || la > FK_MAX_L || lc > FK_MAX_L || lb < 0 || ld < 0)
        return fail(c, FK_ERR_ARG, "fk_set_class_schedule: need la >= lb, lc >= ld, l <= %d", FK_MAX_L);
    int P = pair_class(la, lb), Q = pair_class(lc, ld);
    if (P < Q) std::swap(P, Q);
    if (bra_block < 0 || bra_block > FK_MAX_BRA_BLOCK || kets_per_tile < 0 || kets_per_tile > 64 ||
        !(grid_fraction > 0 && grid_fraction <= 4))
        return fail(c, FK_ERR_ARG, "fk_set_class_schedule: bra_block 0..%d, kets_per_tile 0..64, grid_fraction (0, 4]",
                    FK_MAX_BRA_BLOCK);
    const fk_ctx::ClassSched old = c->sched.count(P * NPC + Q) ? c->sched[P * NPC + Q] : fk_ctx::ClassSched{};
    c->sched[P * NPC + Q] = fk_ctx::ClassSched{bra_block, kets_per_tile, grid_fraction, old.eng, old.bt, old.alt};
    return FK_OK;
}

int fk_set_class_lanes(fk_ctx *c, int la, int lb, int lc, int ld, int lanes)
{
    if (!c) return FK_ERR_ARG;
    if (la < lb || lc < ld || la > FK_MAX_L || lc > FK_MAX_L || lb < 0 || ld < 0)
        return fail(c, FK_ERR_ARG, "fk_set_class_lanes: need la >= lb, lc >= ld, l <= %d", FK_MAX_L);
    int P = pair_class(la, lb), Q = pair_class(lc, ld);
    if (P < Q) std::swap(P, Q);
    FkClassInfo info;
    if (fk_kernels_class_info(P, Q, &info))
        return fail(c, FK_ERR_UNSUPPORTED, "fk_set_class_lanes: class (%d%d|%d%d) is not built", la, lb, lc, ld);
    const int own = info.wave_per_quartet == 0 ? 1 : info.team_size;
    if (lanes != own && !(info.alt_team > 0 && lanes == info.alt_team))
        return fail(c, FK_ERR_UNSUPPORTED, "fk_set_class_lanes: class (%d%d|%d%d) has no kernel with %d lanes per quartet",
                    la, lb, lc, ld, lanes);
    c->sched[P * NPC + Q].alt = (info.alt_team > 0 && lanes == info.alt_team) ? 1 : 0;
    return FK_OK;
}

int fk_set_class_block_tasks(fk_ctx *c, int la, int lb, int lc, int ld, int enable)
{
    if (!c) return FK_ERR_ARG;
    if (la < lb || lc < ld || la > FK_MAX_L || lc > FK_MAX_L || lb < 0 || ld < 0)
        return fail(c, FK_ERR_ARG, "fk_set_class_block_tasks: need la >= lb, lc >= ld, l <= %d", FK_MAX_L);
    if (enable != 0 && enable != 1) return fail(c, FK_ERR_ARG, "fk_set_class_block_tasks: enable must be 0 or 1");
    int P = pair_class(la, lb), Q = pair_class(lc, ld);
    if (P < Q) std::swap(P, Q);
    FkClassInfo info;
    if (fk_kernels_class_info(P, Q, &info))
        return fail(c, FK_ERR_UNSUPPORTED, "fk_set_class_block_tasks: class (%d%d|%d%d) is not built", la, lb, lc, ld);
    c->sched[P * NPC + Q].bt = enable ? 1 : 0;
    return FK_OK;
}

int fk_set_class_engine(fk_ctx *c, int la, int lb, int lc, int ld, int engine)
{
    if (!c) return FK_ERR_ARG;
    if (la < lb || lc < ld || la > FK_MAX_L || lc > FK_MAX_L || lb < 0 || ld < 0)
        return fail(c, FK_ERR_ARG, "fk_set_class_engine: need la >= lb, lc >= ld, l <= %d", FK_MAX_L);
    if (engine != FK_ENGINE_RYS && engine != FK_ENGINE_HGP)
        return fail(c, FK_ERR_ARG, "fk_set_class_engine: engine must be FK_ENGINE_RYS or FK_ENGINE_HGP");
    int P = pair_class(la, lb), Q = pair_class(lc, ld);
    if (P < Q) std::swap(P, Q);
    FkClassInfo info;
    if (fk_kernels_class_info(P, Q, &info))
        return fail(c, FK_ERR_UNSUPPORTED, "fk_set_class_engine: class (%d%d|%d%d) is not built", la, lb, lc, ld);
    if (engine == FK_ENGINE_HGP && !info.hgp)
        return fail(c, FK_ERR_UNSUPPORTED, "fk_set_class_engine: the HGP engine is not built for class (%d%d|%d%d)",
                    la, lb, lc, ld);
    c->sched[P * NPC + Q].eng = engine;
    return FK_OK;
}

int fk_save_schedules(fk_ctx *c, const char *path)
{
    if (!c) return FK_ERR_ARG;
    if (!path) return fail(c, FK_ERR_ARG, "fk_save_schedules: null path");
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(c, FK_ERR_ARG, "fk_save_schedules: cannot write %s", path);
    std::fprintf(f, "# fockjk class schedules: la lb lc ld bra_block kets_per_tile grid_fraction engine block_tasks "
                    "alt_lanes\n");
    std::fprintf(f, "arch %s\n", c->arch.c_str());
    for (const auto &kv : c->sched) {
        int l[4] = {0, 0, 0, 0};
        for (int k = 0; k < 2; ++k) {
            const int pc = k == 0 ? kv.first / NPC : kv.first % NPC;
            int la = 0;
            while (pair_class(la + 1, 0) <= pc) ++la;
            l[2 * k] = la;
            l[2 * k + 1] = pc - pair_class(la, 0);
        }
        const auto &x = kv.second;
        int alt_lanes = 0, bt = x.bt;
        FkClassInfo info;
        if (!fk_kernels_class_info(kv.first / NPC, kv.first % NPC, &info)) {
            if (x.alt) alt_lanes = info.alt_team;
            if (bt < 0) bt = info.ket_outer > 0 ? 1 : 0;
        }
        std::fprintf(f, "class %d %d %d %d %d %d %.17g %d %d %d\n", l[0], l[1], l[2], l[3], x.bb, x.kt, x.gf, x.eng,
                     bt < 0 ? 0 : bt, alt_lanes);
    }
    const bool ok = std::ferror(f) == 0;
    if (std::fclose(f) != 0 || !ok) return fail(c, FK_ERR_ARG, "fk_save_schedules: write error on %s", path);
    return FK_OK;
}

int fk_load_schedules(fk_ctx *c, const char *path)
{
    if (!c) return FK_ERR_ARG;
    if (!path) return fail(c, FK_ERR_ARG, "fk_load_schedules: null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(c, FK_ERR_ARG, "fk_load_schedules: cannot read %s", path);
    std::map<int, fk_ctx::ClassSched> sched = c->sched;
    char line[512];
    int lineno = 0;
    bool arch_ok = false;
    int rc = FK_OK;
    while (rc == FK_OK && std::fgets(line, sizeof line, f)) {
        ++lineno;
        char word[32] = {0};
        if (std::sscanf(line, "%31s", word) != 1 || word[0] == '#') continue;
        if (std::strcmp(word, "arch") == 0) {
            char a[64] = {0};
            if (std::sscanf(line, "arch %63s", a) != 1) { rc = fail(c, FK_ERR_ARG, "fk_load_schedules: %s:%d: bad arch line", path, lineno); break; }
            if (c->arch != a) { rc = fail(c, FK_ERR_UNSUPPORTED, "fk_load_schedules: %s is for %s, the device is %s", path, a, c->arch.c_str()); break; }
            arch_ok = true;
        } else if (std::strcmp(word, "class") == 0) {
            int la, lb, lc, ld, bb, kt, eng, bt = -1, al = 0;
            double gf;
            const int nf = std::sscanf(line, "class %d %d %d %d %d %d %lf %d %d %d", &la, &lb, &lc, &ld, &bb, &kt, &gf, &eng,
                                       &bt, &al);
            if (nf < 8 || nf > 10) {
                rc = fail(c, FK_ERR_ARG, "fk_load_schedules: %s:%d: expected 8 to 10 fields", path, lineno);
                break;
            }
            if (!arch_ok) { rc = fail(c, FK_ERR_ARG, "fk_load_schedules: %s: class line before the arch line", path); break; }
            if (la < lb || lc < ld || la > FK_MAX_L || lc > FK_MAX_L || lb < 0 || ld < 0 || bb < 0 ||
                bb > FK_MAX_BRA_BLOCK || kt < 0 || kt > 64 || !(gf > 0 && gf <= 4) || (eng != 0 && eng != 1) ||
                (nf >= 9 && bt != 0 && bt != 1)) {
                rc = fail(c, FK_ERR_ARG, "fk_load_schedules: %s:%d: value out of range", path, lineno);
                break;
            }
            int P = pair_class(la, lb), Q = pair_class(lc, ld);
            if (P < Q) std::swap(P, Q);
            FkClassInfo info;
            if (fk_kernels_class_info(P, Q, &info) || (eng == 1 && !info.hgp) || (al != 0 && al != info.alt_team)) {
                rc = fail(c, FK_ERR_UNSUPPORTED, "fk_load_schedules: %s:%d: class, engine or kernel not built", path, lineno);
                break;
            }
            sched[P * NPC + Q] = fk_ctx::ClassSched{bb, kt, gf, eng, bt, al ? 1 : 0};
        } else {
            rc = fail(c, FK_ERR_ARG, "fk_load_schedules: %s:%d: unknown record '%s'", path, lineno, word);
        }
    }
    std::fclose(f);
    if (rc) return rc;
    if (!arch_ok) return fail(c, FK_ERR_ARG, "fk_load_schedules: %s has no arch line", path);
    c->sched = sched;
    return FK_OK;
}

int fk_autotune(fk_ctx *c, const double *D, unsigned flags, int reps, void *stream, fk_tune_report *rep)
{
    if (!c) return FK_ERR_ARG;
    if (!D) return fail(c, FK_ERR_ARG, "fk_autotune: null density");
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_autotune: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_autotune: call fk_build_quartets first");
    if (reps < 1 || reps > 100) return fail(c, FK_ERR_ARG, "fk_autotune: reps must be 1..100");
    if (rep) std::memset(rep, 0, sizeof *rep);
    hipSetDevice(c->device);
    hipStream_t st = (hipStream_t)stream;
    const fk_screen_opts opts = c->opts;
    int rc;
    // resident copies of D, J, K for the timed builds
    DevBuf<double> dD, dJ, dK;
    struct Free { DevBuf<double> *b[3]; ~Free() { for (auto *x : b) dev_free(*x); } } fr{{&dD, &dJ, &dK}};
    const size_t nm = c->mol_base.empty() ? (size_t)c->nbf * c->nbf : (size_t)c->mol_base[c->nmol];
    if ((rc = dev_upload<double>(c, dD, nullptr, nm)) || (rc = dev_upload<double>(c, dJ, nullptr, nm)) ||
        (rc = dev_upload<double>(c, dK, nullptr, nm)))
        return rc;
    HIPCHK(c, hipMemcpy(dD.p, D, nm * sizeof(double), (flags & FK_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    // times of the class launches (key P * NPC + Q, both precisions summed) for
    // the current schedules: min over reps of each launch
    int configs = 0;
    auto measure = [&](std::map<int, double> &t, std::vector<double> *per_launch) -> int {
        int r;
        if ((r = fk_build_quartets(c, &opts))) return r;
        ++configs;
        std::vector<double> best(c->qclasses.size(), 1e300);
        for (int k = 0; k <= reps; ++k) {  // the first build warms up
            if ((r = fk_build_jk(c, dD.p, dJ.p, dK.p, FK_DEVICE_PTRS | FK_SYNC | FK_TIME_CLASSES, st))) return r;
            if (k == 0) continue;
            for (size_t i = 0; i < c->qclasses.size(); ++i) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) best[i] = std::min(best[i], (double)ms);
            }
        }
        t.clear();
        for (size_t i = 0; i < c->qclasses.size(); ++i) t[c->qclasses[i].P * NPC + c->qclasses[i].Q] += best[i];
        if (per_launch) *per_launch = best;
        return FK_OK;
    };
    const std::map<int, fk_ctx::ClassSched> start = c->sched;
    std::map<int, double> t0;
    std::vector<double> launch0;
    if ((rc = measure(t0, &launch0))) return rc;
    struct Key { int P, Q, prec; };
    std::vector<Key> keys0;
    for (const auto &q : c->qclasses) keys0.push_back({q.P, q.Q, q.prec});
    std::map<int, fk_ctx::ClassSched> cur;
    for (const auto &kv : t0) {
        auto it = start.find(kv.first);
        cur[kv.first] = it == start.end() ? fk_ctx::ClassSched{} : it->second;
    }
    std::map<int, double> tbest = t0;
    // one axis at a time, every class measured under each candidate value
    for (int axis = 0; axis < 6; ++axis) {
        std::vector<double> vals;
        if (axis == 0) vals = {1, 2, 4, 8, 16, 32};
        else if (axis == 1) vals = {1, 2, 4, 8};   // rounds of kets (team and wave kernels)
        else if (axis == 2) vals = {1.0, 0.5, 0.25, 2.0, 4.0};
        else if (axis == 4) {
            // block tasks switched, for the classes that take them
            bool any = false;
            for (const auto &q : c->qclasses) any = any || q.info.ket_outer > 0 || q.info.wide > 0;
            if (!any || opts.block_tasks != 0) continue;
            vals = {-1};
        } else if (axis == 5) {
            // lanes per quartet: the other kernel, for the lane classes with a team alternative
            bool any = false;
            for (const auto &kv : cur) {
                FkClassInfo info;
                if (!fk_kernels_class_info(kv.first / NPC, kv.first % NPC, &info) && info.alt_team > 0) any = true;
            }
            if (!any) continue;
            vals = {-1};
        } else {
            // the other engine, for the classes that have both
            bool any = false;
            for (const auto &kv : cur) {
                FkClassInfo info;
                if (!fk_kernels_class_info(kv.first / NPC, kv.first % NPC, &info) && info.hgp) any = true;
            }
            if (!any) continue;
            vals = {-1};
        }
        for (double v : vals) {
            std::map<int, fk_ctx::ClassSched> trial = cur;
            for (auto &kv : trial) {
                const int P = kv.first / NPC, Q = kv.first % NPC;
                FkClassInfo info;
                if (fk_kernels_class_info(P, Q, &info)) continue;
                if (axis == 0) kv.second.bb = (int)v;
                else if (axis == 4) {
                    if (info.wave_per_quartet == 0 && (info.ket_outer > 0 || info.wide > 0)) {
                        const int on = kv.second.bt < 0 ? (info.ket_outer > 0 ? 1 : 0) : kv.second.bt;
                        kv.second.bt = 1 - on;
                    }
                } else if (axis == 5) {
                    if (info.alt_team > 0) kv.second.alt = 1 - kv.second.alt;
                } else if (axis == 3) {
                    if (info.hgp) kv.second.eng = 1 - kv.second.eng;
                } else if (axis == 1) {
                    if (info.wave_per_quartet == 0) continue;
                    const int qpw = info.wave_per_quartet == 3 ? 1 : 64 / std::max(1, info.team_size);
                    kv.second.kt = std::min(64, (int)v * qpw);
                } else kv.second.gf = v;
            }
            c->sched = trial;
            std::map<int, double> t;
            if ((rc = measure(t, nullptr))) { c->sched = start; fk_build_quartets(c, &opts); return rc; }
            for (auto &kv : t) {
                auto b = tbest.find(kv.first);
                if (b == tbest.end() || kv.second < b->second * 0.98) {  // 2 %: above timing noise
                    tbest[kv.first] = kv.second;
                    cur[kv.first] = trial[kv.first];
                }
            }
        }
    }
    c->sched = cur;
    std::map<int, double> t1;
    std::vector<double> launch1;
    if ((rc = measure(t1, &launch1))) return rc;
    if (rep) {
        rep->nclass = (int)c->qclasses.size();
        rep->configurations = configs;
        for (size_t i = 0; i < c->qclasses.size(); ++i) {
            const auto &q = c->qclasses[i];
            const auto &sc = c->sched[q.P * NPC + q.Q];
            rep->la[i] = q.info.la; rep->lb[i] = q.info.lb; rep->lc[i] = q.info.lc; rep->ld[i] = q.info.ld;
            rep->precision[i] = q.prec ? 32 : 64;
            rep->bra_block[i] = std::max(1, std::min(sc.bb > 0 ? sc.bb : (opts.bra_block > 0 ? opts.bra_block : 8), q.info.bra_block));
            rep->kets_per_tile[i] = q.info.wave_per_quartet == 0 ? 64 : (sc.kt > 0 ? sc.kt : 2 * (q.info.wave_per_quartet == 3 ? 1 : 64 / std::max(1, q.info.team_size)));
            rep->grid_fraction[i] = sc.gf;
            rep->engine[i] = q.engine;
            rep->block_tasks[i] = q.ntask > 0 ? 1 : 0;
            rep->lanes_per_quartet[i] = q.info.wave_per_quartet == 0 ? 1 : q.info.team_size;
            const auto s0 = start.find(q.P * NPC + q.Q);
            const fk_ctx::ClassSched sc0 = s0 == start.end() ? fk_ctx::ClassSched{} : s0->second;
            // compare the schedules in effect (a candidate equal to the default is no change)
            auto eff_bb = [&](const fk_ctx::ClassSched &x) {
                return std::max(1, std::min(x.bb > 0 ? x.bb : (opts.bra_block > 0 ? opts.bra_block : 8), q.info.bra_block));
            };
            auto eff_kt = [&](const fk_ctx::ClassSched &x) {
                if (q.info.wave_per_quartet == 0) return 64;
                return x.kt > 0 ? x.kt : 2 * (q.info.wave_per_quartet == 3 ? 1 : 64 / std::max(1, q.info.team_size));
            };
            rep->changed[i] =
                (eff_bb(sc0) != eff_bb(sc) || eff_kt(sc0) != eff_kt(sc) || sc0.gf != sc.gf || sc0.eng != sc.eng ||
                 ((sc0.bt < 0 ? (q.info.ket_outer > 0 ? 1 : 0) : sc0.bt) !=
                  (sc.bt < 0 ? (q.info.ket_outer > 0 ? 1 : 0) : sc.bt)) || sc0.alt != sc.alt) ? 1 : 0;
            rep->ms_tuned[i] = launch1[i];
            for (size_t j = 0; j < keys0.size(); ++j)
                if (keys0[j].P == q.P && keys0[j].Q == q.Q && keys0[j].prec == q.prec) rep->ms_default[i] = launch0[j];
            rep->build_ms_tuned += launch1[i];
        }
        for (double x : launch0) rep->build_ms_default += x;
    }
    return FK_OK;
}

int fk_debug_eri(fk_ctx *c, int nq, const int *quartets, double *out, int mode)
{
    if (!c) return FK_ERR_ARG;
    if (mode < 0 || mode > 5) return fail(c, FK_ERR_ARG, "fk_debug_eri: mode must be 0..5");
    const int on_device = mode & 1, engine = mode >> 1;
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "fk_debug_eri: not available for a batch of molecules");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_debug_eri: call fk_build_quartets first");
    if (nq < 0 || (nq > 0 && (!quartets || !out))) return fail(c, FK_ERR_ARG, "fk_debug_eri: bad arguments");
    if (on_device && c->device < 0) return fail(c, FK_ERR_STATE, "fk_debug_eri: context has no device");
    if (on_device) hipSetDevice(c->device);
    // pair index lookup for arbitrary shell pairs
    auto pair_index = [&](int a, int b) {
        const int hi = std::max(a, b), lo = std::min(a, b);
        return hi * (hi + 1) / 2 + lo;  // pairs were generated for a >= b in this order
    };
    size_t off = 0;
    std::vector<size_t> offs(nq);
    for (int q = 0; q < nq; ++q) {
        for (int k = 0; k < 4; ++k)
            if (quartets[4 * q + k] < 0 || quartets[4 * q + k] >= c->nshell)
                return fail(c, FK_ERR_ARG, "fk_debug_eri: shell index out of range in quartet %d", q);
        offs[q] = off;
        off += (size_t)ncart(c->sh_l[quartets[4 * q]]) * ncart(c->sh_l[quartets[4 * q + 1]]) *
               ncart(c->sh_l[quartets[4 * q + 2]]) * ncart(c->sh_l[quartets[4 * q + 3]]);
    }
    // group by canonical class
    struct Item { int q, bra, ket; bool swap; };
    std::vector<std::vector<Item>> groups(NPC * NPC);
    for (int q = 0; q < nq; ++q) {
        const int *s = quartets + 4 * q;
        int p1 = pair_index(s[0], s[1]), p2 = pair_index(s[2], s[3]);
        int c1 = c->pr_cls[p1], c2 = c->pr_cls[p2];
        bool swap = c1 < c2;
        if (swap) { std::swap(p1, p2); std::swap(c1, c2); }
        groups[c1 * NPC + c2].push_back({q, p1, p2, swap});
    }
    for (int P = 0; P < NPC; ++P)
        for (int Q = 0; Q <= P; ++Q) {
            auto &g = groups[P * NPC + Q];
            if (g.empty()) continue;
            std::vector<int> qs;
            for (auto &it : g) { qs.push_back(it.bra); qs.push_back(it.ket); }
            std::vector<double> raw;
            int rc = eval_quartets(c, P, Q, qs, raw, on_device != 0, engine);
            if (rc) return rc;
            for (size_t k = 0; k < g.size(); ++k) {
                const Item &it = g[k];
                const int *s = quartets + 4 * it.q;
                // canonical shells in raw order: (pa, pb | pc, pd)
                const int pa = c->pr_sa[it.bra], pb = c->pr_sb[it.bra], pc = c->pr_sa[it.ket], pd = c->pr_sb[it.ket];
                const int cs[4] = {pa, pb, pc, pd};
                const int cn[4] = {ncart(c->sh_l[pa]), ncart(c->sh_l[pb]), ncart(c->sh_l[pc]), ncart(c->sh_l[pd])};
                const int rn[4] = {ncart(c->sh_l[s[0]]), ncart(c->sh_l[s[1]]), ncart(c->sh_l[s[2]]), ncart(c->sh_l[s[3]])};
                // position of requested shell slot r in the canonical tuple
                int pos[4];
                const int req_pair_first = it.swap ? 2 : 0;
                // requested (s0,s1) maps to canonical pair (bra if !swap else ket)
                for (int r = 0; r < 2; ++r) {
                    const int base = it.swap ? 2 : 0;  // canonical slots of requested bra pair
                    const int x = s[r];
                    // if the pair has two equal shells, keep the slot order
                    if (cs[base] == x && (cs[base + 1] != x || r == 0)) pos[r] = base;
                    else pos[r] = base + 1;
                }
                for (int r = 2; r < 4; ++r) {
                    const int base = it.swap ? 0 : 2;
                    const int x = s[r];
                    if (cs[base] == x && (cs[base + 1] != x || r == 2)) pos[r] = base;
                    else pos[r] = base + 1;
                }
                (void)req_pair_first;
                const double *src = raw.data() + k * (size_t)(cn[0] * cn[1] * cn[2] * cn[3]);
                double *dst = out + offs[it.q];
                const double *sc[4];
                for (int r = 0; r < 4; ++r) sc[r] = &c->bf_scale[c->sh_bf[s[r]]];
                int i[4];
                for (i[0] = 0; i[0] < rn[0]; ++i[0])
                    for (i[1] = 0; i[1] < rn[1]; ++i[1])
                        for (i[2] = 0; i[2] < rn[2]; ++i[2])
                            for (i[3] = 0; i[3] < rn[3]; ++i[3]) {
                                int ci[4];
                                for (int r = 0; r < 4; ++r) ci[pos[r]] = i[r];
                                const double v = src[((ci[0] * cn[1] + ci[1]) * cn[2] + ci[2]) * cn[3] + ci[3]];
                                dst[((i[0] * rn[1] + i[1]) * rn[2] + i[2]) * rn[3] + i[3]] =
                                    v * sc[0][i[0]] * sc[1][i[1]] * sc[2][i[2]] * sc[3][i[3]];
                            }
            }
        }
    return FK_OK;
}

int fk_rys_host(int n, double T, double *u, double *w);

// Walks every tile the J/K kernels will visit and checks each address they
// form (list positions, transposed and bra primitive records, LDS slot,
// density, shell-block maxima and Fock accumulators) against its array.
// Returns FK_OK or FK_ERR_STATE with the first violation in fk_last_error.
int fk_check_indices(fk_ctx *c)
{
    if (!c) return FK_ERR_ARG;
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_check_indices: no quartet lists");
    const long long nl = (long long)c->ket_list_all.size();
    const long long npair = (long long)c->pr_sa.size(), nppr = (long long)(c->pp.size() / FK_NPP_REC);
    const long long nT = (long long)c->ppT.size();
    for (size_t qi = 0; qi < c->qclasses.size(); ++qi) {
        const QuartetClass &qc = c->qclasses[qi];
        const int NA = ncart(qc.info.la), NB = ncart(qc.info.lb), NC = ncart(qc.info.lc), ND = ncart(qc.info.ld);
        for (int64_t t = qc.tile_off; t < qc.tile_off + qc.ntile; ++t) {
            const FkTile &T = c->tiles[t];
            const long long gid = T.grp & ~FK_TILE_SAME;
            if (T.blk < 0 || T.blk >= (long long)c->blocks.size() || gid < 0 || gid >= (long long)c->groups.size())
                return fail(c, FK_ERR_STATE, "class %zu tile %lld: block/group out of range", qi, (long long)t);
            const FkGroup &g = c->groups[gid];
            const FkBraBlock &BB = c->blocks[T.blk];
            // the kernels address the tile's molecule: its nbf_m^2 and nshell_m^2 blocks
            if (g.mol < 0 || g.mol >= c->nmol) return fail(c, FK_ERR_STATE, "tile %lld: molecule out of range", (long long)t);
            const long long n = c->mol_nbf[g.mol], ns = c->mol_nsh[g.mol];
            if (BB.first < 0 || BB.count < 1 || BB.count > FK_MAX_BRA_BLOCK || (size_t)BB.first + BB.count > c->blk_bra.size())
                return fail(c, FK_ERR_STATE, "tile %lld: bra block range", (long long)t);
          for (int jb = 0; jb < BB.count; ++jb) {
            const long long bra = c->blk_bra[BB.first + jb], bpos = c->blk_pos[BB.first + jb];
            if (bra < 0 || bra >= npair || bpos < 0 || bpos >= nl) return fail(c, FK_ERR_STATE, "tile %lld: bra %d index", (long long)t, jb);
            const int gsa = c->pr_sa[bra], gsb = c->pr_sb[bra];
            if (c->sh_mol[gsa] != g.mol || c->sh_mol[gsb] != g.mol)
                return fail(c, FK_ERR_STATE, "tile %lld: bra outside the tile's molecule", (long long)t);
            const int sa = c->sh_loc[gsa], sb = c->sh_loc[gsb];
            const long long ppo = c->pr_ppoff[bra], bnp = c->pr_npp[bra];
            if (ppo < 0 || ppo + bnp > nppr) return fail(c, FK_ERR_STATE, "tile %lld: bra records", (long long)t);
            if (bnp * FK_NFLD > qc.bra_slot) return fail(c, FK_ERR_STATE, "tile %lld: LDS bra slot", (long long)t);
            const long long oa = c->sh_lbf[gsa], ob = c->sh_lbf[gsb];
            if (oa + NA > n || ob + NB > n || ncart(c->sh_l[gsa]) != NA || ncart(c->sh_l[gsb]) != NB)
                return fail(c, FK_ERR_STATE, "tile %lld: bra shells do not match the class", (long long)t);
            if (gsa != c->pr_sa[c->blk_bra[BB.first]])
                return fail(c, FK_ERR_STATE, "tile %lld: bra block members differ in their first shell", (long long)t);
            if (T.ket_count < 1 || T.ket_count > 64)
                return fail(c, FK_ERR_STATE, "tile %lld: ket count %d", (long long)t, T.ket_count);
            for (int k = 0; k < 64; ++k) {
                // every lane reads position ket_begin + (lane < count ? lane : 0)
                const long long pos = T.ket_begin + (k < T.ket_count ? k : 0);
                if (pos < 0 || pos >= nl) return fail(c, FK_ERR_STATE, "tile %lld lane %d: position %lld", (long long)t, k, pos);
                const long long r = pos - g.begin;
                if (r < 0 || r >= g.len) return fail(c, FK_ERR_STATE, "tile %lld lane %d: outside its group", (long long)t, k);
                const long long kp = c->ket_list_all[pos];
                if (kp < 0 || kp >= npair) return fail(c, FK_ERR_STATE, "tile %lld lane %d: ket pair", (long long)t, k);
                const int gsc = c->lst_sa[pos], gsd = c->lst_sb[pos];
                if (gsc != c->pr_sa[kp] || gsd != c->pr_sb[kp] || c->lst_sa_loc[pos] != c->sh_loc[gsc] ||
                    c->lst_sb_loc[pos] != c->sh_loc[gsd])
                    return fail(c, FK_ERR_STATE, "tile %lld lane %d: list data disagree with the pair", (long long)t, k);
                if (c->sh_mol[gsc] != g.mol || c->sh_mol[gsd] != g.mol)
                    return fail(c, FK_ERR_STATE, "tile %lld lane %d: ket outside the tile's molecule", (long long)t, k);
                const int sc = c->sh_loc[gsc], sd = c->sh_loc[gsd];
                if (ncart(c->sh_l[gsc]) != NC || ncart(c->sh_l[gsd]) != ND || c->pr_npp[kp] != g.npp)
                    return fail(c, FK_ERR_STATE, "tile %lld lane %d: ket does not match class/group", (long long)t, k);
                const long long last = g.base + ((long long)(g.npp - 1) * FK_NFLD + FK_NFLD - 1) * g.len + r;
                if (g.base < 0 || last >= nT) return fail(c, FK_ERR_STATE, "tile %lld lane %d: ket records", (long long)t, k);
                const long long oc = c->sh_lbf[gsc], od = c->sh_lbf[gsd];
                if (oc + NC > n || od + ND > n) return fail(c, FK_ERR_STATE, "tile %lld lane %d: ket functions", (long long)t, k);
                const long long dsh[6] = {sa * ns + sb, sc * ns + sd, sa * ns + sc, sa * ns + sd, sb * ns + sc, sb * ns + sd};
                for (long long x : dsh)
                    if (x < 0 || x >= ns * ns) return fail(c, FK_ERR_STATE, "tile %lld lane %d: shell block", (long long)t, k);
            }
          }
        }
    }
    return FK_OK;
}

// One-electron integrals on the host.  Overlap and kinetic energy by the
// Obara-Saika 1-D recurrences; nuclear attraction by Rys quadrature of the
// one-centre operator: V_ab = -Z_C (2 pi/p) K_AB sum_r w_r Ix Iy Iz with
// I(a+1,0) = (PA - u PC) I(a,0) + a (1-u)/(2p) I(a-1,0) and the horizontal
// transfer I(a,b+1) = I(a+1,b) + AB I(a,b).
int fk_one_electron(fk_ctx *c, double *S, double *T, double *V, double *e_nuc)
{
    if (!c) return FK_ERR_ARG;
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "fk_one_electron: not available for a batch of molecules");
    if (!c->have_basis) return fail(c, FK_ERR_STATE, "fk_one_electron: basis not set");
    const int n = c->nbf;
    if (e_nuc) {
        double e = 0;
        for (int a = 0; a < c->natom; ++a)
            for (int b = 0; b < a; ++b) {
                double r2 = 0;
                for (int k = 0; k < 3; ++k) r2 += (c->xyz[3 * a + k] - c->xyz[3 * b + k]) * (c->xyz[3 * a + k] - c->xyz[3 * b + k]);
                e += (double)c->Z[a] * c->Z[b] / std::sqrt(r2);
            }
        *e_nuc = e;
    }
    if (!S && !T && !V) return FK_OK;
    const size_t nn = (size_t)n * n;
    if (c->oe_S.size() != nn) {
        // computed once per geometry and basis: shell pairs sa >= sb, both
        // triangles written, shared out over host threads
        std::vector<double> Sv(nn), Tv(nn), Vv(nn);
        double *Sc = Sv.data(), *Tc = Tv.data(), *Vc = Vv.data();
        constexpr int LM = FK_MAX_L + 3;
        std::atomic<int> next{0};
        auto work = [&]() {
            for (int sa; (sa = next.fetch_add(1)) < c->nshell;)
                for (int sb = 0; sb <= sa; ++sb) {
                    const int la = c->sh_l[sa], lb = c->sh_l[sb];
                    const int na = ncart(la), nb = ncart(lb);
                    const double *A = &c->xyz[3 * c->sh_atom[sa]], *B = &c->xyz[3 * c->sh_atom[sb]];
                    double AB[3], ab2 = 0;
                    for (int k = 0; k < 3; ++k) { AB[k] = A[k] - B[k]; ab2 += AB[k] * AB[k]; }
                    std::vector<double> bs(na * nb, 0.0), bt(na * nb, 0.0), bv(na * nb, 0.0);
                    for (int i = c->sh_poff[sa]; i < c->sh_poff[sa + 1]; ++i)
                        for (int j = c->sh_poff[sb]; j < c->sh_poff[sb + 1]; ++j) {
                            const double al = c->exps[i], be = c->exps[j], p = al + be;
                            const double Kab = std::exp(-al * be / p * ab2) * c->coef[i] * c->coef[j];
                            double P[3], PA[3], PB[3];
                            for (int k = 0; k < 3; ++k) {
                                P[k] = (al * A[k] + be * B[k]) / p;
                                PA[k] = P[k] - A[k];
                                PB[k] = P[k] - B[k];
                            }
                            // 1-D overlaps O[k][i][j], i <= la, j <= lb + 2
                            double O[3][LM][LM] = {};
                            for (int k = 0; k < 3; ++k) {
                                O[k][0][0] = std::sqrt(M_PI / p);
                                for (int x = 0; x <= la; ++x)
                                    for (int y = 0; y <= lb + 2; ++y) {
                                        if (x == 0 && y == 0) continue;
                                        double v;
                                        if (x > 0) {
                                            v = PA[k] * O[k][x - 1][y];
                                            if (x > 1) v += (x - 1) / (2 * p) * O[k][x - 2][y];
                                            if (y > 0) v += y / (2 * p) * O[k][x - 1][y - 1];
                                        } else {
                                            v = PB[k] * O[k][x][y - 1];
                                            if (y > 1) v += (y - 1) / (2 * p) * O[k][x][y - 2];
                                        }
                                        O[k][x][y] = v;
                                    }
                            }
                            for (int ia = 0; ia < na; ++ia)
                                for (int ib = 0; ib < nb; ++ib) {
                                    int a[3], b[3];
                                    cart_exps(la, ia, a[0], a[1], a[2]);
                                    cart_exps(lb, ib, b[0], b[1], b[2]);
                                    double s1[3], t1[3];
                                    for (int k = 0; k < 3; ++k) {
                                        s1[k] = O[k][a[k]][b[k]];
                                        double tk = -2 * be * be * O[k][a[k]][b[k] + 2] + be * (2 * b[k] + 1) * s1[k];
                                        if (b[k] >= 2) tk -= 0.5 * b[k] * (b[k] - 1) * O[k][a[k]][b[k] - 2];
                                        t1[k] = tk;
                                    }
                                    bs[ia * nb + ib] += Kab * s1[0] * s1[1] * s1[2];
                                    bt[ia * nb + ib] += Kab * (t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2] + s1[0] * s1[1] * t1[2]);
                                }
                            const int nr = (la + lb) / 2 + 1;
                            for (int C = 0; C < c->natom; ++C) {
                                if (c->Z[C] == 0) continue;
                                double PC[3], pc2 = 0;
                                for (int k = 0; k < 3; ++k) { PC[k] = P[k] - c->xyz[3 * C + k]; pc2 += PC[k] * PC[k]; }
                                double u[RYS_NMAX], w[RYS_NMAX];
                                fk_rys_host(nr, p * pc2, u, w);
                                const double pre = -c->Z[C] * 2 * M_PI / p * Kab;
                                for (int r = 0; r < nr; ++r) {
                                    double I[3][LM][LM];
                                    for (int k = 0; k < 3; ++k) {
                                        double G[2 * LM];
                                        G[0] = 1.0;
                                        const double c00 = PA[k] - u[r] * PC[k], b10 = (1 - u[r]) / (2 * p);
                                        if (la + lb > 0) G[1] = c00;
                                        for (int e = 1; e < la + lb; ++e) G[e + 1] = c00 * G[e] + e * b10 * G[e - 1];
                                        // transfer to b: H[x][y] with x + y <= la + lb
                                        double H[2 * LM][LM];
                                        for (int e = 0; e <= la + lb; ++e) H[e][0] = G[e];
                                        for (int y = 0; y < lb; ++y)
                                            for (int x = 0; x < la + lb - y; ++x) H[x][y + 1] = H[x + 1][y] + AB[k] * H[x][y];
                                        for (int x = 0; x <= la; ++x)
                                            for (int y = 0; y <= lb; ++y) I[k][x][y] = H[x][y];
                                    }
                                    for (int ia = 0; ia < na; ++ia)
                                        for (int ib = 0; ib < nb; ++ib) {
                                            int a[3], b[3];
                                            cart_exps(la, ia, a[0], a[1], a[2]);
                                            cart_exps(lb, ib, b[0], b[1], b[2]);
                                            bv[ia * nb + ib] += pre * w[r] * I[0][a[0]][b[0]] * I[1][a[1]][b[1]] * I[2][a[2]][b[2]];
                                        }
                                }
                            }
                        }
                    for (int ia = 0; ia < na; ++ia)
                        for (int ib = 0; ib < nb; ++ib) {
                            const int r = c->sh_bf[sa] + ia, col = c->sh_bf[sb] + ib;
                            const double f = c->bf_scale[r] * c->bf_scale[col];
                            const size_t e1 = (size_t)r * n + col, e2 = (size_t)col * n + r;
                            Sc[e1] = Sc[e2] = f * bs[ia * nb + ib];
                            Tc[e1] = Tc[e2] = f * bt[ia * nb + ib];
                            Vc[e1] = Vc[e2] = f * bv[ia * nb + ib];
                        }
        
                }
        };
        int nth = (int)std::thread::hardware_concurrency();
        if (const char *e = std::getenv("OMP_NUM_THREADS")) nth = std::min(nth, std::max(1, std::atoi(e)));
        nth = std::max(1, std::min({nth, 32, c->nshell}));
        std::vector<std::thread> pool;
        for (int k = 1; k < nth; ++k) pool.emplace_back(work);
        work();
        for (auto &th : pool) th.join();
        c->oe_S.swap(Sv);
        c->oe_T.swap(Tv);
        c->oe_V.swap(Vv);
    }
    if (S) std::copy(c->oe_S.begin(), c->oe_S.end(), S);
    if (T) std::copy(c->oe_T.begin(), c->oe_T.end(), T);
    if (V) std::copy(c->oe_V.begin(), c->oe_V.end(), V);
    return FK_OK;
}

// ---------------------------------------------------------------- SCF ----
// Restricted closed-shell SCF around the device J/K build.  Every per-iteration
// matrix operation is a device kernel (fk_scf.hip): F = h + J - K/2, the
// energy, F' = X F X, the DIIS commutator F'D' - D'F' and its inner products,
// the DIIS combination, the purification that turns F' into the density and
// D = X D' X.  The host solves the (m+1) x (m+1) DIIS system and decides
// convergence from scalars read back each step.
namespace {

int guess_predict_device(fk_ctx *c, double *D, hipStream_t st);  // learned guess, defined below

// Largest entry of S^(-1/2) the SCF accepts (overlap eigenvalues down to
// about 1e-7); beyond it the orthonormal-basis steps lose all accuracy.
constexpr double kMaxOrthoEntry = 3.0e3;
// Fock eigenvalue (hartree) given to the overlap directions the canonical
// orthogonaliser drops: far above any occupied level, so that they stay empty.
constexpr double kNullShift = 1.0;

struct ScfWork {
    fk_ctx *c = nullptr;
    hipStream_t st = nullptr;
    int n = 0;
    DevBuf<double> h, X, Xi, D, Do, J, K, F, Fo, G, E, T1, T2, T3, part, scal;
    DevBuf<double> Dlast, dD, Jacc, Kacc;  // incremental builds
    DevBuf<double> Pn, ev, wk;             // canonical orthogonaliser: projector onto the dropped directions
    DevBuf<int> info;
    int ndrop = 0;
    std::vector<DevBuf<double>> ringF, ringE;
    ~ScfWork()
    {
        for (auto *b : {&h, &X, &Xi, &D, &Do, &J, &K, &F, &Fo, &G, &E, &T1, &T2, &T3, &part, &scal, &Dlast, &dD, &Jacc, &Kacc,
                        &Pn, &ev, &wk})
            dev_free(*b);
        dev_free(info);
        for (auto &b : ringF) dev_free(b);
        for (auto &b : ringE) dev_free(b);
    }
};

#define SCFCHK(w, call)                                                                          \
    do {                                                                                        \
        if ((call) != 0) return fail((w).c, FK_ERR_HIP, "fk_run_scf: kernel launch failed: %s", #call); \
    } while (0)

// reduction `op` of x (and y) into a host scalar (op 3 returns two values)
int scf_reduce(ScfWork &w, const double *x, const double *y, int op, double *out)
{
    SCFCHK(w, fk_scf_reduce(x, y, w.n, op, w.part.p, w.scal.p, 0, w.st));
    HIPCHK(w.c, hipMemcpyAsync(out, w.scal.p, (op == 3 ? 2 : 1) * sizeof(double), hipMemcpyDeviceToHost, w.st));
    HIPCHK(w.c, hipStreamSynchronize(w.st));
    return FK_OK;
}

// A <- swap helper for device buffers
inline void swapbuf(DevBuf<double> &a, DevBuf<double> &b) { std::swap(a, b); }

// Orthogonaliser X = S^(-1/2) and S^(1/2) by the coupled Newton-Schulz
// iteration on S / c, c an upper bound of the spectrum (Gershgorin).
int scf_orthogonaliser(ScfWork &w, double tol)
{
    const int n = w.n;
    double gb[2];
    int rc;
    // T3 holds S on entry
    if ((rc = scf_reduce(w, w.T3.p, nullptr, 3, gb))) return rc;
    const double cs = gb[1];
    if (!(cs > 0)) return fail(w.c, FK_ERR_ARG, "fk_run_scf: overlap matrix has no positive bound");
    SCFCHK(w, fk_scf_lincomb(w.Xi.p, w.T3.p, nullptr, nullptr, n, 1.0 / cs, 0, 0, 0, w.st));  // Y
    SCFCHK(w, fk_scf_lincomb(w.X.p, w.T3.p, nullptr, nullptr, n, 0.0, 0, 0, 1.0, w.st));       // Z = I
    double prev = 1e300, err = 1e300;
    for (int it = 0; it < 200; ++it) {
        SCFCHK(w, fk_scf_gemm(w.X.p, w.Xi.p, w.T1.p, n, 1.0, 0.0, w.st));                      // ZY
        SCFCHK(w, fk_scf_lincomb(w.T2.p, w.T1.p, nullptr, nullptr, n, 1.0, 0, 0, -1.0, w.st));  // ZY - I
        if ((rc = scf_reduce(w, w.T2.p, nullptr, 1, &err))) return rc;
        if (err < tol * 1e-3 || (err < 1e-9 && err > 0.5 * prev)) break;  // converged or at the rounding floor
        prev = err;
        SCFCHK(w, fk_scf_lincomb(w.T2.p, w.T1.p, nullptr, nullptr, n, -0.5, 0, 0, 1.5, w.st));  // T = (3I - ZY)/2
        SCFCHK(w, fk_scf_gemm(w.Xi.p, w.T2.p, w.T1.p, n, 1.0, 0.0, w.st));                     // Y T
        SCFCHK(w, fk_scf_gemm(w.T2.p, w.X.p, w.G.p, n, 1.0, 0.0, w.st));                       // T Z
        swapbuf(w.Xi, w.T1);
        swapbuf(w.X, w.G);
    }
    if (!(err < tol)) return fail(w.c, FK_ERR_ARG, "fk_run_scf: S^(-1/2) did not converge (max|ZY - I| = %.3g); overlap too ill-conditioned", err);
    SCFCHK(w, fk_scf_lincomb(w.X.p, w.X.p, nullptr, nullptr, n, 1.0 / std::sqrt(cs), 0, 0, 0, w.st));
    SCFCHK(w, fk_scf_lincomb(w.Xi.p, w.Xi.p, nullptr, nullptr, n, std::sqrt(cs), 0, 0, 0, w.st));
    // every direction of S is kept: a nearly linearly dependent basis (overlap
    // eigenvalues about 1e-7 or below) would amplify rounding past use
    double xmax = 0;
    if ((rc = scf_reduce(w, w.X.p, nullptr, 1, &xmax))) return rc;
    if (!(xmax < kMaxOrthoEntry))
        return fail(w.c, FK_ERR_ARG, "fk_run_scf: max |S^(-1/2)| = %.3g: the basis is nearly linearly dependent", xmax);
    return FK_OK;
}

// Canonical orthogonaliser: S = U s U^T (w.T3 holds S), X = U s^(-1/2) U^T and
// Xi = U s^(1/2) U^T over the eigenvalues above `cutoff`; the dropped
// directions' projector I - X Xi goes to w.Pn (when any is dropped).
int scf_orthogonaliser_canonical(ScfWork &w, double cutoff)
{
    const int n = w.n;
    const size_t nn = (size_t)n * n;
    int rc;
    if ((rc = dev_upload<double>(w.c, w.ev, nullptr, n)) || (rc = dev_upload<double>(w.c, w.wk, nullptr, n)) ||
        (rc = dev_upload<int>(w.c, w.info, nullptr, 1)))
        return rc;
    HIPCHK(w.c, hipMemcpyAsync(w.T1.p, w.T3.p, nn * sizeof(double), hipMemcpyDeviceToDevice, w.st));
    SCFCHK(w, fk_scf_eigh(w.T1.p, w.ev.p, w.wk.p, w.info.p, n, w.st));
    int info = 0;
    std::vector<double> s(n);
    HIPCHK(w.c, hipMemcpy(&info, w.info.p, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(w.c, hipMemcpy(s.data(), w.ev.p, n * sizeof(double), hipMemcpyDeviceToHost));
    if (info != 0) return fail(w.c, FK_ERR_HIP, "fk_run_scf: overlap eigen-decomposition failed (info %d)", info);
    w.ndrop = 0;
    for (double v : s) w.ndrop += v > cutoff ? 0 : 1;
    if (w.ndrop >= n) return fail(w.c, FK_ERR_ARG, "fk_run_scf: every overlap eigenvalue is below the cutoff %.3g", cutoff);
    SCFCHK(w, fk_scf_eig_scale(w.T1.p, w.ev.p, w.T2.p, n, cutoff, -0.5, w.st));
    SCFCHK(w, fk_scf_gemm(w.T2.p, w.T1.p, w.X.p, n, 1.0, 0.0, w.st));
    SCFCHK(w, fk_scf_eig_scale(w.T1.p, w.ev.p, w.T2.p, n, cutoff, 0.5, w.st));
    SCFCHK(w, fk_scf_gemm(w.T2.p, w.T1.p, w.Xi.p, n, 1.0, 0.0, w.st));
    if (w.ndrop > 0) {
        if ((rc = dev_upload<double>(w.c, w.Pn, nullptr, nn))) return rc;
        SCFCHK(w, fk_scf_gemm(w.X.p, w.Xi.p, w.T2.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_lincomb(w.Pn.p, w.T2.p, nullptr, nullptr, n, -1.0, 0, 0, 1.0, w.st));
    }
    return FK_OK;
}

// F' (w.Fo) plus the shift of the dropped directions, when there are any.
int scf_shift_null(ScfWork &w)
{
    if (w.ndrop > 0) SCFCHK(w, fk_scf_lincomb(w.Fo.p, w.Fo.p, w.Pn.p, nullptr, w.n, 1.0, kNullShift, 0, 0, w.st));
    return FK_OK;
}

// Orthonormal density D' = 2 P, P the projector onto the nocc lowest states of
// the symmetric matrix in w.Fo (trace-correcting purification); result in w.Do.
int scf_purify(ScfWork &w, int nocc, int *steps)
{
    const int n = w.n;
    double gb[2];
    int rc;
    if ((rc = scf_reduce(w, w.Fo.p, nullptr, 3, gb))) return rc;
    const double lo = gb[0], hi = gb[1];
    if (!(hi > lo)) return fail(w.c, FK_ERR_ARG, "fk_run_scf: degenerate Fock spectrum bounds");
    // P0 = (hi I - F') / (hi - lo): occupied (low) states near 1
    SCFCHK(w, fk_scf_lincomb(w.T1.p, w.Fo.p, nullptr, nullptr, n, -1.0 / (hi - lo), 0, 0, hi / (hi - lo), w.st));
    int extra = -1, it = 0;
    for (; it < 300; ++it) {
        SCFCHK(w, fk_scf_gemm(w.T1.p, w.T1.p, w.T2.p, n, 1.0, 0.0, w.st));
        double t1, t2;
        if ((rc = scf_reduce(w, w.T1.p, nullptr, 2, &t1))) return rc;
        if ((rc = scf_reduce(w, w.T2.p, nullptr, 2, &t2))) return rc;
        const double idem = t1 - t2;  // sum of x(1 - x) over the eigenvalues
        if (extra < 0 && std::fabs(idem) < 1e-11) extra = 2;  // quadratic convergence: two more steps
        if (extra == 0) break;
        if (extra > 0) --extra;
        if (std::fabs(t2 - nocc) < std::fabs(2 * t1 - t2 - nocc)) {
            swapbuf(w.T1, w.T2);                                                                  // P <- P^2
        } else {
            SCFCHK(w, fk_scf_lincomb(w.T1.p, w.T1.p, w.T2.p, nullptr, n, 2.0, -1.0, 0, 0, w.st)); // P <- 2P - P^2
        }
    }
    if (extra != 0) return fail(w.c, FK_ERR_NOT_CONVERGED, "fk_run_scf: purification did not converge (no gap?)");
    if (steps) *steps = it;
    SCFCHK(w, fk_scf_lincomb(w.Do.p, w.T1.p, nullptr, nullptr, n, 2.0, 0, 0, 0, w.st));
    return FK_OK;
}

// Orthonormal density D' = 2 C_o C_o^T from the eigenvectors of the nocc
// lowest states of the symmetric matrix in w.Fo (rocSOLVER); result in w.Do.
int scf_density_eig(ScfWork &w, int nocc)
{
    const int n = w.n;
    fk_ctx *c = w.c;
    HIPCHK(c, hipMemcpyAsync(w.T1.p, w.Fo.p, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, w.st));
    if (fk_scf_eigh(w.T1.p, w.ev.p, w.wk.p, w.info.p, n, w.st))
        return fail(c, FK_ERR_HIP, "fk_run_scf: eigen-decomposition launch failed");
    int info = 0;
    std::vector<double> occ(n);
    HIPCHK(c, hipMemcpy(&info, w.info.p, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(occ.data(), w.ev.p, n * sizeof(double), hipMemcpyDeviceToHost));
    if (info != 0) return fail(c, FK_ERR_HIP, "fk_run_scf: eigen-decomposition of X F X failed (info %d)", info);
    if (nocc < n && !(occ[nocc] > occ[nocc - 1]))
        return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf: no gap between the occupied and virtual states");
    for (int k = 0; k < n; ++k) occ[k] = k < nocc ? 2.0 : 0.0;
    HIPCHK(c, hipMemcpy(w.ev.p, occ.data(), n * sizeof(double), hipMemcpyHostToDevice));
    // C diag(occ) C^T: rows of the row-major eigenvector matrix are the states
    SCFCHK(w, fk_scf_eig_scale(w.T1.p, w.ev.p, w.T2.p, n, 1.0, 1.0, w.st));
    SCFCHK(w, fk_scf_gemm(w.T2.p, w.T1.p, w.Do.p, n, 1.0, 0.0, w.st));
    return FK_OK;
}

// Solves the Pulay system [B 1; 1 0] [c; l] = [0; 1] for m vectors (Gaussian
// elimination with partial pivoting).  Returns false if singular.
bool diis_solve(const std::vector<double> &B, int m, std::vector<double> &coef)
{
    const int k = m + 1;
    std::vector<double> A((size_t)k * (k + 1), 0.0);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i * (k + 1) + j] = B[(size_t)i * m + j];
        A[i * (k + 1) + m] = 1.0;
        A[m * (k + 1) + i] = 1.0;
    }
    A[m * (k + 1) + k] = 1.0;  // right-hand side of the constraint row
    // scale the error block so that pivoting compares like with like
    double bmax = 0;
    for (int i = 0; i < m; ++i) bmax = std::max(bmax, std::fabs(B[(size_t)i * m + i]));
    if (!(bmax > 0)) return false;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A[i * (k + 1) + j] /= bmax;
    for (int col = 0; col < k; ++col) {
        int piv = col;
        for (int r = col + 1; r < k; ++r)
            if (std::fabs(A[r * (k + 1) + col]) > std::fabs(A[piv * (k + 1) + col])) piv = r;
        if (std::fabs(A[piv * (k + 1) + col]) < 1e-300) return false;
        if (piv != col)
            for (int j = 0; j <= k; ++j) std::swap(A[col * (k + 1) + j], A[piv * (k + 1) + j]);
        for (int r = 0; r < k; ++r) {
            if (r == col) continue;
            const double f = A[r * (k + 1) + col] / A[col * (k + 1) + col];
            for (int j = col; j <= k; ++j) A[r * (k + 1) + j] -= f * A[col * (k + 1) + j];
        }
    }
    coef.assign(m, 0.0);
    for (int i = 0; i < m; ++i) coef[i] = A[i * (k + 1) + k] / A[i * (k + 1) + i];
    for (double v : coef)
        if (!std::isfinite(v)) return false;
    return true;
}

}  // namespace

int fk_run_scf(fk_ctx *c, const fk_scf_opts *opts, fk_scf_result *result, double *D_inout)
{
    if (!c) return FK_ERR_ARG;
    if (!result || !D_inout) return fail(c, FK_ERR_ARG, "fk_run_scf: null result or density pointer");
    std::memset(result, 0, sizeof *result);
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_run_scf: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_run_scf: call fk_build_quartets first");
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "fk_run_scf: one molecule per context (batches: one context each)");
    fk_scf_opts o = {100, 1e-10, 1e-8, 8, 0, 1e-8, 0, 0, 0.0, 0, 0};
    if (opts) o = *opts;
    if (o.max_iter < 0 || o.diis_n < 0 || o.diis_n > 32 || !(o.e_tol > 0) || !(o.g_tol > 0) || !(o.lindep > 0) ||
        !(o.canonical >= 0 && o.canonical < 1) || (o.j_engine != 0 && o.j_engine != 1) ||
        (o.density_eig != 0 && o.density_eig != 1) ||
        o.guess < 0 || o.guess > 3 || (o.graph != 0 && o.graph != 1) || o.incremental < 0 ||
        (o.graph && o.incremental))
        return fail(c, FK_ERR_ARG, "fk_run_scf: invalid options");
    if (c->nelec % 2 != 0 || c->nelec <= 0) return fail(c, FK_ERR_ARG, "fk_run_scf: closed shell needs an even, positive electron count");
    const int n = c->nbf, nocc = c->nelec / 2;
    if (nocc > n) return fail(c, FK_ERR_ARG, "fk_run_scf: more occupied orbitals than basis functions");
    const auto t_start = std::chrono::steady_clock::now();
    hipSetDevice(c->device);
    const size_t nn = (size_t)n * n;
    // one-electron part on the host, once per geometry
    std::vector<double> S(nn), T(nn), V(nn), h(nn);
    double enuc = 0;
    int rc;
    if ((rc = fk_one_electron(c, S.data(), T.data(), V.data(), &enuc))) return rc;
    for (size_t i = 0; i < nn; ++i) h[i] = T[i] + V[i];
    result->e_nuc = enuc;

    ScfWork w;
    w.c = c;
    w.n = n;
    w.st = nullptr;
    // graph mode runs on a stream of its own (capture needs one); a blocking
    // stream keeps the order with the synchronous copies of the set-up
    struct GraphRes {
        hipStream_t st = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        ~GraphRes()
        {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
            if (st) (void)hipStreamDestroy(st);
        }
    } gr;
    if (o.graph) {
        HIPCHK(c, hipStreamCreate(&gr.st));
        w.st = gr.st;
    }
    if (o.incremental)
        for (auto *b : {&w.Dlast, &w.dD, &w.Jacc, &w.Kacc})
            if ((rc = dev_upload<double>(c, *b, nullptr, nn))) return rc;
    for (auto *b : {&w.h, &w.X, &w.Xi, &w.D, &w.Do, &w.J, &w.K, &w.F, &w.Fo, &w.G, &w.E, &w.T1, &w.T2, &w.T3})
        if ((rc = dev_upload<double>(c, *b, nullptr, nn))) return rc;
    if ((rc = dev_upload<double>(c, w.part, nullptr, (size_t)fk_scf_reduce_scratch() + 2))) return rc;
    if ((rc = dev_upload<double>(c, w.scal, nullptr, 4))) return rc;
    w.ringF.resize(std::max(o.diis_n, 1));
    w.ringE.resize(std::max(o.diis_n, 1));
    if (o.diis_n > 0)
        for (int k = 0; k < o.diis_n; ++k)
            if ((rc = dev_upload<double>(c, w.ringF[k], nullptr, nn)) || (rc = dev_upload<double>(c, w.ringE[k], nullptr, nn)))
                return rc;
    if ((rc = dev_upload(c, w.h, h.data(), nn))) return rc;
    if ((rc = dev_upload(c, w.T3, S.data(), nn))) return rc;
    if ((rc = o.canonical > 0 ? scf_orthogonaliser_canonical(w, o.canonical) : scf_orthogonaliser(w, o.lindep))) return rc;
    result->ndropped = w.ndrop;
    if (o.density_eig &&
        ((rc = dev_upload<double>(c, w.ev, nullptr, n)) || (rc = dev_upload<double>(c, w.wk, nullptr, n)) ||
         (rc = dev_upload<int>(c, w.info, nullptr, 1))))
        return rc;
    auto density = [&]() { return o.density_eig ? scf_density_eig(w, nocc) : scf_purify(w, nocc, nullptr); };

    // initial orthonormal density D' (w.Do); a learned or SAD guess that
    // cannot be formed falls back to SAD, then to the core Hamiltonian
    const auto t_guess = std::chrono::steady_clock::now();
    int gused = o.guess;
    if (gused == 3) {
        rc = guess_predict_device(c, w.D.p, w.st);
        double ss = 0;
        if (!rc) rc = scf_reduce(w, w.D.p, w.D.p, 0, &ss);
        if (!rc && !std::isfinite(ss)) rc = fail(c, FK_ERR_ARG, "learned guess: non-finite prediction");
        if (!rc) {
            // projector onto the nocc largest eigenvalues of P' = S^1/2 D S^1/2 / 2:
            // purification of F' = -P' (its nocc lowest states)
            SCFCHK(w, fk_scf_gemm(w.Xi.p, w.D.p, w.T3.p, n, 1.0, 0.0, w.st));
            SCFCHK(w, fk_scf_gemm(w.T3.p, w.Xi.p, w.Fo.p, n, -0.5, 0.0, w.st));
            rc = scf_shift_null(w);
            if (!rc) rc = density();
        }
        if (rc) gused = 2;
    }
    if (gused == 2) {
        std::vector<double> Dsad(nn);
        rc = fk_sad_density(c, Dsad.data());
        if (!rc) rc = dev_upload(c, w.D, Dsad.data(), nn);
        if (rc) {
            gused = 0;
        } else {
            SCFCHK(w, fk_scf_gemm(w.Xi.p, w.D.p, w.T3.p, n, 1.0, 0.0, w.st));
            SCFCHK(w, fk_scf_gemm(w.T3.p, w.Xi.p, w.Do.p, n, 1.0, 0.0, w.st));
        }
    }
    if (gused != o.guess) c->err.clear();
    if (gused == 0) {
        SCFCHK(w, fk_scf_gemm(w.X.p, w.h.p, w.T3.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_gemm(w.T3.p, w.X.p, w.Fo.p, n, 1.0, 0.0, w.st));
        if ((rc = scf_shift_null(w)) || (rc = density())) return rc;
    } else if (gused == 1) {
        if ((rc = dev_upload(c, w.D, D_inout, nn))) return rc;
        SCFCHK(w, fk_scf_gemm(w.Xi.p, w.D.p, w.T3.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_gemm(w.T3.p, w.Xi.p, w.Do.p, n, 1.0, 0.0, w.st));
    }
    // D = X D' X
    SCFCHK(w, fk_scf_gemm(w.X.p, w.Do.p, w.T3.p, n, 1.0, 0.0, w.st));
    SCFCHK(w, fk_scf_gemm(w.T3.p, w.X.p, w.D.p, n, 1.0, 0.0, w.st));
    HIPCHK(c, hipStreamSynchronize(w.st));
    result->guess_used = gused;
    result->guess_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_guess).count();
    if (o.max_iter == 0) {
        HIPCHK(c, hipMemcpy(D_inout, w.D.p, nn * sizeof(double), hipMemcpyDeviceToHost));
        result->total_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        return FK_OK;
    }

    std::vector<double> B;  // DIIS inner products, row-major m x m over ring slots
    const int dn = std::max(o.diis_n, 1);
    B.assign((size_t)dn * dn, 0.0);
    std::vector<int> slot_age;  // ring slots in insertion order
    double e_prev = 0, e_cur = 0, err = 0, jk_s = 0;
    bool converged = false;
    int it = 0;
    // the Fock stage: J, K, F = h + J - K/2, D.h and D.F, F' = X F X, the
    // commutator F'D' - D'F' and its largest element, into scal[0..2]
    int since_full = 0;
    const unsigned jflag = o.j_engine ? FK_J_ENGINE : 0u;
    auto fock_stage = [&](bool eager) -> int {
        int r;
        if (eager && o.incremental) {
            // J, K from the density change since the last build (screened by
            // its own, smaller, density bounds) added to the running sums; a
            // full build every `incremental` iterations
            const bool full = since_full == 0;
            const double *Dsrc = w.D.p;
            if (!full) {
                SCFCHK(w, fk_scf_lincomb(w.dD.p, w.D.p, w.Dlast.p, nullptr, n, 1.0, -1.0, 0, 0, w.st));
                Dsrc = w.dD.p;
            }
            const auto tb = std::chrono::steady_clock::now();
            // a density change is screened 1000 times tighter, so that the
            // running sums stay as accurate as full builds
            c->dscreen_scale = full ? 1.0 : 1e-3;
            r = fk_build_jk(c, Dsrc, w.J.p, w.K.p, FK_DEVICE_PTRS | FK_SYNC | jflag, w.st);
            c->dscreen_scale = 1.0;
            if (r) return r;
            jk_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
            SCFCHK(w, fk_scf_lincomb(w.Jacc.p, w.J.p, w.Jacc.p, nullptr, n, 1.0, full ? 0.0 : 1.0, 0, 0, w.st));
            SCFCHK(w, fk_scf_lincomb(w.Kacc.p, w.K.p, w.Kacc.p, nullptr, n, 1.0, full ? 0.0 : 1.0, 0, 0, w.st));
            HIPCHK(c, hipMemcpyAsync(w.Dlast.p, w.D.p, nn * sizeof(double), hipMemcpyDeviceToDevice, w.st));
            since_full = (since_full + 1) % o.incremental;
            SCFCHK(w, fk_scf_lincomb(w.F.p, w.h.p, w.Jacc.p, w.Kacc.p, n, 1.0, 1.0, -0.5, 0, w.st));
        } else {
            if (eager) {  // the build timed on its own
                const auto tb = std::chrono::steady_clock::now();
                if ((r = fk_build_jk(c, w.D.p, w.J.p, w.K.p, FK_DEVICE_PTRS | FK_SYNC | jflag, w.st))) return r;
                jk_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
            } else if ((r = fk_build_jk(c, w.D.p, w.J.p, w.K.p, FK_DEVICE_PTRS | jflag, w.st))) {
                return r;
            }
            SCFCHK(w, fk_scf_lincomb(w.F.p, w.h.p, w.J.p, w.K.p, n, 1.0, 1.0, -0.5, 0, w.st));
        }
        SCFCHK(w, fk_scf_reduce(w.D.p, w.h.p, n, 0, w.part.p, w.scal.p, 0, w.st));
        SCFCHK(w, fk_scf_reduce(w.D.p, w.F.p, n, 0, w.part.p, w.scal.p, 1, w.st));
        SCFCHK(w, fk_scf_gemm(w.X.p, w.F.p, w.T3.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_gemm(w.T3.p, w.X.p, w.Fo.p, n, 1.0, 0.0, w.st));
        if ((r = scf_shift_null(w))) return r;
        SCFCHK(w, fk_scf_gemm(w.Fo.p, w.Do.p, w.G.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_antisym(w.E.p, w.G.p, n, w.st));
        SCFCHK(w, fk_scf_reduce(w.E.p, nullptr, n, 1, w.part.p, w.scal.p, 2, w.st));
        return FK_OK;
    };
    for (; it < o.max_iter; ++it) {
        const auto t0 = std::chrono::steady_clock::now();
        if (o.graph && it > 0) {
            if (!gr.x) {  // captured once, after an eager stage has set every buffer up
                HIPCHK(c, hipStreamBeginCapture(w.st, hipStreamCaptureModeThreadLocal));
                rc = fock_stage(false);
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(w.st, &g);
                gr.g = g;
                if (rc) return rc;
                if (e != hipSuccess) return fail(c, FK_ERR_HIP, "fk_run_scf: graph capture failed: %s", hipGetErrorString(e));
                HIPCHK(c, hipGraphInstantiate(&gr.x, gr.g, nullptr, nullptr, 0));
            }
            HIPCHK(c, hipGraphLaunch(gr.x, w.st));
        } else if ((rc = fock_stage(true))) {
            return rc;
        }
        double sc[3];
        HIPCHK(c, hipMemcpyAsync(sc, w.scal.p, 3 * sizeof(double), hipMemcpyDeviceToHost, w.st));
        HIPCHK(c, hipStreamSynchronize(w.st));
        if (o.graph && it > 0) jk_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const double dh = sc[0], df = sc[1];
        err = sc[2];
        e_prev = e_cur;
        e_cur = 0.5 * (dh + df) + enuc;
        if (!std::isfinite(e_cur) || !std::isfinite(err))
            return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf: non-finite energy or error at iteration %d", it + 1);
        if (it > 0 && std::fabs(e_cur - e_prev) < o.e_tol && err < o.g_tol) {
            converged = true;
            ++it;
            break;
        }
        // DIIS extrapolation of F'
        if (o.diis_n > 1) {
            int k;
            if ((int)slot_age.size() < o.diis_n) {
                k = (int)slot_age.size();
            } else {
                k = slot_age.front();
                slot_age.erase(slot_age.begin());
            }
            slot_age.push_back(k);
            HIPCHK(c, hipMemcpyAsync(w.ringF[k].p, w.Fo.p, nn * sizeof(double), hipMemcpyDeviceToDevice, w.st));
            HIPCHK(c, hipMemcpyAsync(w.ringE[k].p, w.E.p, nn * sizeof(double), hipMemcpyDeviceToDevice, w.st));
            for (int j : slot_age) {
                double v;
                if ((rc = scf_reduce(w, w.ringE[k].p, w.ringE[j].p, 0, &v))) return rc;
                B[(size_t)k * dn + j] = B[(size_t)j * dn + k] = v;
            }
            const int m = (int)slot_age.size();
            if (m >= 2) {
                std::vector<double> Bm((size_t)m * m), coef;
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j) Bm[(size_t)i * m + j] = B[(size_t)slot_age[i] * dn + slot_age[j]];
                if (diis_solve(Bm, m, coef)) {
                    SCFCHK(w, fk_scf_lincomb(w.Fo.p, w.ringF[slot_age[0]].p, nullptr, nullptr, n, coef[0], 0, 0, 0, w.st));
                    for (int i = 1; i < m; ++i)
                        SCFCHK(w, fk_scf_lincomb(w.Fo.p, w.Fo.p, w.ringF[slot_age[i]].p, nullptr, n, 1.0, coef[i], 0, 0, w.st));
                }
            }
        }
        // new density: D' from F', D = X D' X
        if ((rc = density())) return rc;
        SCFCHK(w, fk_scf_gemm(w.X.p, w.Do.p, w.T3.p, n, 1.0, 0.0, w.st));
        SCFCHK(w, fk_scf_gemm(w.T3.p, w.X.p, w.D.p, n, 1.0, 0.0, w.st));
    }
    HIPCHK(c, hipMemcpy(D_inout, w.D.p, nn * sizeof(double), hipMemcpyDeviceToHost));
    result->energy = e_cur;
    result->iterations = it;
    result->converged = converged ? 1 : 0;
    result->error = err;
    result->delta_e = e_cur - e_prev;
    result->jk_seconds = jk_s;
    result->total_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (!converged) return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf: not converged in %d iterations", o.max_iter);
    return FK_OK;
}

int fk_rys_host(int n, double T, double *u, double *w)
{
    if (n < 1 || n > RYS_NMAX || !u || !w || !(T >= 0)) return FK_ERR_ARG;
    const double *tab = rys_staged_host() + rys_staged_offset(n);
    switch (n) {
    case 1: rys_roots<1, true>(T, tab, u, w); break;
    case 2: rys_roots<2, true>(T, tab, u, w); break;
    case 3: rys_roots<3, true>(T, tab, u, w); break;
    case 4: rys_roots<4, true>(T, tab, u, w); break;
    case 5: rys_roots<5, true>(T, tab, u, w); break;
    case 6: rys_roots<6, true>(T, tab, u, w); break;
    case 7: rys_roots<7, true>(T, tab, u, w); break;
    }
    return FK_OK;
}

}  // extern "C"

// ============================================================ initial guesses
// Learned initial density and superposition of atomic densities (an
// extension: the paper's SCF starts from a conventional guess).
namespace {

// Position of the Cartesian component x^x y^y z^(l-x-y) in the library order.
inline int cart_index(int l, int x, int y) { return (l - x) * (l - x + 1) / 2 + (l - x - y); }

// T with phi_a(Q r) = sum_b T_ab phi_b(r) for the normalised Cartesian
// components of momentum l (Q row-major 3 x 3, T row-major ncart x ncart):
// the component's monomial is a product of l linear forms (Q r)_axis, whose
// expansion runs over the 3^l choices of one coordinate per factor.
void cart_rotation(int l, const double *Q, double *T)
{
    const int n = ncart(l);
    for (int i = 0; i < n * n; ++i) T[i] = 0.0;
    for (int a = 0; a < n; ++a) {
        int ex, ey, ez;
        cart_exps(l, a, ex, ey, ez);
        int axis[3] = {0, 0, 0};
        for (int f = 0; f < l; ++f) axis[f] = f < ex ? 0 : (f < ex + ey ? 1 : 2);
        const double na = 1.0 / std::sqrt(dfact(2 * ex - 1) * dfact(2 * ey - 1) * dfact(2 * ez - 1));
        int total = 1;
        for (int f = 0; f < l; ++f) total *= 3;
        for (int code = 0; code < total; ++code) {
            int cnt[3] = {0, 0, 0}, cc = code;
            double cf = 1.0;
            for (int f = 0; f < l; ++f) {
                const int j = cc % 3;
                cc /= 3;
                cf *= Q[axis[f] * 3 + j];
                ++cnt[j];
            }
            const double nb = 1.0 / std::sqrt(dfact(2 * cnt[0] - 1) * dfact(2 * cnt[1] - 1) * dfact(2 * cnt[2] - 1));
            T[a * n + cart_index(l, cnt[0], cnt[1])] += cf * na / nb;
        }
    }
}

// Block-diagonal rotation over the shells of atom `at` into T (FK_GUESS_NB^2,
// zero-padded); returns the atom's function count.
int atom_rotation(const fk_ctx *c, int at, const double *Q, double *T)
{
    for (int i = 0; i < FK_GUESS_NB * FK_GUESS_NB; ++i) T[i] = 0.0;
    int o = 0;
    double blk[100];
    for (int s = 0; s < c->nshell; ++s) {
        if (c->sh_atom[s] != at) continue;
        const int l = c->sh_l[s], n = ncart(l);
        cart_rotation(l, Q, blk);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) T[(o + i) * FK_GUESS_NB + o + j] = blk[i * n + j];
        o += n;
    }
    return o;
}

// Frame with e_z = ez (unit) and e_x along the part of ref orthogonal to e_z,
// or, for ref == NULL, along the lab axis least aligned with e_z (lowest
// index on ties); columns e_x, e_y, e_z of Q, row-major.
void frame_from(const double *ez, const double *ref, double *Q)
{
    double ex[3] = {0, 0, 0};
    if (ref) {
        for (int i = 0; i < 3; ++i) ex[i] = ref[i];
    } else {
        int k = 0;
        for (int i = 1; i < 3; ++i)
            if (std::fabs(ez[i]) < std::fabs(ez[k])) k = i;
        ex[k] = 1.0;
    }
    const double p = ex[0] * ez[0] + ex[1] * ez[1] + ex[2] * ez[2];
    for (int i = 0; i < 3; ++i) ex[i] -= p * ez[i];
    const double nx = std::sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
    for (int i = 0; i < 3; ++i) ex[i] /= nx;
    const double ey[3] = {ez[1] * ex[2] - ez[2] * ex[1], ez[2] * ex[0] - ez[0] * ex[2], ez[0] * ex[1] - ez[1] * ex[0]};
    for (int i = 0; i < 3; ++i) {
        Q[i * 3 + 0] = ex[i];
        Q[i * 3 + 1] = ey[i];
        Q[i * 3 + 2] = ez[i];
    }
}

// Atoms within FK_GUESS_RCUT of `centre`, other than e1 and e2, ordered by
// distance on a 1e-6 bohr grid, then index (atoms at distances equal by
// symmetry keep one order in any orientation).
void guess_neighbours(const fk_ctx *c, int centre, int e1, int e2, std::vector<std::pair<long long, int>> &out)
{
    out.clear();
    for (int k = 0; k < c->natom; ++k) {
        if (k == e1 || k == e2) continue;
        double r2 = 0;
        for (int i = 0; i < 3; ++i) {
            const double d = c->xyz[3 * k + i] - c->xyz[3 * centre + i];
            r2 += d * d;
        }
        const double r = std::sqrt(r2);
        if (r < FK_GUESS_RCUT) out.push_back({(long long)std::floor(r * 1e6), k});
    }
    std::sort(out.begin(), out.end());
}

// First neighbour (from position `start`) whose direction from `origin` has a
// component orthogonal to ez above 0.1 of its length; its vector in ref.
bool guess_off_axis(const fk_ctx *c, int origin, const double *ez, const std::vector<std::pair<long long, int>> &nb,
                    size_t start, double *ref)
{
    for (size_t i = start; i < nb.size(); ++i) {
        const int k = nb[i].second;
        double v[3], vv = 0, p = 0;
        for (int j = 0; j < 3; ++j) {
            v[j] = c->xyz[3 * k + j] - c->xyz[3 * origin + j];
            vv += v[j] * v[j];
            p += v[j] * ez[j];
        }
        double pp = 0;
        for (int j = 0; j < 3; ++j) {
            const double w = v[j] - p * ez[j];
            pp += w * w;
        }
        if (std::sqrt(pp) > 0.1 * std::sqrt(vv)) {
            for (int j = 0; j < 3; ++j) ref[j] = v[j];
            return true;
        }
    }
    return false;
}

// Frame of the pair (a, b): a != b: e_z from a to b, e_x towards the nearest
// off-axis neighbour of a (else of b); a == b: e_z towards a's nearest
// neighbour, e_x towards the next nearest off-axis one; missing neighbours:
// lab axes (a lone atom: the lab frame).
void local_frame(const fk_ctx *c, int a, int b, double *Q)
{
    std::vector<std::pair<long long, int>> nb;
    double ez[3], ref[3];
    if (a != b) {
        double R = 0;
        for (int i = 0; i < 3; ++i) {
            ez[i] = c->xyz[3 * b + i] - c->xyz[3 * a + i];
            R += ez[i] * ez[i];
        }
        R = std::sqrt(R);
        for (int i = 0; i < 3; ++i) ez[i] /= R;
        guess_neighbours(c, a, a, b, nb);
        bool have = guess_off_axis(c, a, ez, nb, 0, ref);
        if (!have) {
            guess_neighbours(c, b, a, b, nb);
            have = guess_off_axis(c, b, ez, nb, 0, ref);
        }
        frame_from(ez, have ? ref : nullptr, Q);
        return;
    }
    guess_neighbours(c, a, a, a, nb);
    if (nb.empty()) {
        for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const int k = nb[0].second;
    double R = 0;
    for (int i = 0; i < 3; ++i) {
        ez[i] = c->xyz[3 * k + i] - c->xyz[3 * a + i];
        R += ez[i] * ez[i];
    }
    R = std::sqrt(R);
    for (int i = 0; i < 3; ++i) ez[i] /= R;
    const bool have = guess_off_axis(c, a, ez, nb, 1, ref);
    frame_from(ez, have ? ref : nullptr, Q);
}

void transpose3(const double *Q, double *Qt)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Qt[j * 3 + i] = Q[i * 3 + j];
}

int element_slot(int Z)
{
    switch (Z) {
    case 1: return 0;
    case 6: return 1;
    case 7: return 2;
    case 8: return 3;
    default: return -1;
    }
}

struct GuessPairHost {
    int a1, a2;
};

// Atom function ranges; FK_ERR_UNSUPPORTED if an atom's shells are not
// consecutive or it has more than FK_GUESS_NB functions.
int atom_ranges(fk_ctx *c, std::vector<int> &f0, std::vector<int> &nf)
{
    f0.assign(c->natom, -1);
    nf.assign(c->natom, 0);
    for (int s = 0; s < c->nshell; ++s) {
        const int a = c->sh_atom[s];
        if (f0[a] < 0) f0[a] = c->sh_bf[s];
        else if (f0[a] + nf[a] != c->sh_bf[s])
            return fail(c, FK_ERR_UNSUPPORTED, "initial guess: the shells of atom %d are not consecutive", a);
        nf[a] += ncart(c->sh_l[s]);
        if (nf[a] > FK_GUESS_NB)
            return fail(c, FK_ERR_UNSUPPORTED, "initial guess: atom %d has more than %d functions", a, FK_GUESS_NB);
    }
    return FK_OK;
}

int guess_pair_list(fk_ctx *c, std::vector<GuessPairHost> &pairs)
{
    pairs.clear();
    if (!c->have_basis) return fail(c, FK_ERR_STATE, "initial guess: geometry and basis not set");
    if (c->nmol > 1) return fail(c, FK_ERR_UNSUPPORTED, "initial guess: one molecule per context");
    for (int a = 0; a < c->natom; ++a)
        if (element_slot(c->Z[a]) < 0)
            return fail(c, FK_ERR_UNSUPPORTED, "learned guess: element Z = %d is not one of H, C, N, O", c->Z[a]);
    const double rc2 = FK_GUESS_RCUT * FK_GUESS_RCUT;
    for (int i = 0; i < c->natom; ++i)
        for (int j = i; j < c->natom; ++j) {
            if (i != j) {
                double r2 = 0;
                for (int k = 0; k < 3; ++k) {
                    const double d = c->xyz[3 * i + k] - c->xyz[3 * j + k];
                    r2 += d * d;
                }
                if (!(r2 < rc2)) continue;
            }
            pairs.push_back(c->Z[j] > c->Z[i] ? GuessPairHost{j, i} : GuessPairHost{i, j});
        }
    return FK_OK;
}

// Features of a pair: element one-hots, radial Gaussians of the distance, and
// for each of the two atoms the moments (1, u, u u^T) of the directions u (in
// the pair frame Q) to its other neighbours within the cutoff, weighted by
// two radial shells exp(-((r - c0) / w)^2), per neighbour element.
constexpr double kEnvShell[2][2] = {{0.0, 3.0}, {5.0, 1.5}};
constexpr int kEnvMom = 10;
constexpr int kNEnv = 4 * 2 * kEnvMom;
static_assert(8 + FK_GUESS_NRBF + 2 * kNEnv == FK_GUESS_NFEAT, "feature layout");

void guess_features(const fk_ctx *c, const GuessPairHost &p, const double *Q, float *x)
{
    for (int k = 0; k < FK_GUESS_NFEAT; ++k) x[k] = 0.0f;
    x[element_slot(c->Z[p.a1])] = 1.0f;
    x[4 + element_slot(c->Z[p.a2])] = 1.0f;
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double d = c->xyz[3 * p.a2 + k] - c->xyz[3 * p.a1 + k];
        r2 += d * d;
    }
    const double R = std::sqrt(r2), step = FK_GUESS_RCUT / (FK_GUESS_NRBF - 1);
    for (int k = 0; k < FK_GUESS_NRBF; ++k) {
        const double u = (R - k * step) / step;
        x[8 + k] = (float)std::exp(-u * u);
    }
    const int base = 8 + FK_GUESS_NRBF;
    double acc[2][kNEnv];
    for (int side = 0; side < 2; ++side) {
        const int at = side ? p.a2 : p.a1;
        for (int i = 0; i < kNEnv; ++i) acc[side][i] = 0.0;
        for (int k = 0; k < c->natom; ++k) {
            if (k == p.a1 || k == p.a2) continue;
            double v[3], rr = 0;
            for (int j = 0; j < 3; ++j) {
                v[j] = c->xyz[3 * k + j] - c->xyz[3 * at + j];
                rr += v[j] * v[j];
            }
            const double r = std::sqrt(rr);
            if (!(r < FK_GUESS_RCUT)) continue;
            double u[3];
            for (int j = 0; j < 3; ++j) u[j] = (Q[0 * 3 + j] * v[0] + Q[1 * 3 + j] * v[1] + Q[2 * 3 + j] * v[2]) / r;
            const double mom[kEnvMom] = {1.0,         u[0],        u[1],        u[2],        u[0] * u[0],
                                         u[0] * u[1], u[0] * u[2], u[1] * u[1], u[1] * u[2], u[2] * u[2]};
            const int e = element_slot(c->Z[k]);
            for (int sh = 0; sh < 2; ++sh) {
                const double t = (r - kEnvShell[sh][0]) / kEnvShell[sh][1];
                const double w = std::exp(-t * t);
                for (int m = 0; m < kEnvMom; ++m) acc[side][(e * 2 + sh) * kEnvMom + m] += w * mom[m];
            }
        }
        for (int i = 0; i < kNEnv; ++i) x[base + side * kNEnv + i] = (float)acc[side][i];
    }
}

// C = A^T B C' helpers on FK_GUESS_NB x FK_GUESS_NB row-major blocks
void blk_mul(const double *A, bool ta, const double *B, bool tb, double *C)
{
    constexpr int W = FK_GUESS_NB;
    for (int i = 0; i < W; ++i)
        for (int j = 0; j < W; ++j) {
            double s = 0;
            for (int k = 0; k < W; ++k) s += (ta ? A[k * W + i] : A[i * W + k]) * (tb ? B[j * W + k] : B[k * W + j]);
            C[i * W + j] = s;
        }
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix: A = V diag(w) V^T.
void jacobi_eigen(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                const double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// Fractional-occupation SCF of atom `at` alone (its shells at the origin, Z
// electrons); result: its nf x nf density block.
int atomic_density(fk_ctx *c, int at, std::vector<double> &Dat)
{
    std::vector<int> shells;
    for (int s = 0; s < c->nshell; ++s)
        if (c->sh_atom[s] == at) shells.push_back(s);
    const int ns = (int)shells.size();
    std::vector<int> satom(ns, 0), sl(ns), snp(ns);
    std::vector<double> ex, cf;
    for (int k = 0; k < ns; ++k) {
        const int s = shells[k];
        sl[k] = c->sh_l[s];
        snp[k] = c->sh_nprim[s];
        for (int p = c->sh_poff[s]; p < c->sh_poff[s + 1]; ++p) {
            ex.push_back(c->exps[p]);
            cf.push_back(c->coef_in[p]);
        }
    }
    const int Z = c->Z[at];
    const double origin[3] = {0, 0, 0};
    fk_ctx *t = nullptr;
    if (fk_create(&t, -1) != FK_OK) return fail(c, FK_ERR_OOM, "SAD: cannot create an atomic context");
    struct Guard { fk_ctx *t; ~Guard() { fk_destroy(t); } } guard{t};
    fk_screen_opts so{};
    // the geometry's own electron count is not used (odd Z gets charge -1 to
    // pass the closed-shell check); the atom holds Z electrons below
    if (fk_set_geometry(t, 1, &Z, origin, (Z & 1) ? -1 : 0) || fk_set_basis(t, ns, satom.data(), sl.data(), snp.data(), ex.data(), cf.data()) ||
        fk_build_quartets(t, &so))
        return fail(c, FK_ERR_ARG, "SAD: atomic set-up failed: %s", t->err.c_str());
    const int n = t->nbf;
    const size_t n2 = (size_t)n * n;
    std::vector<double> S(n2), T(n2), V(n2), h(n2);
    if (fk_one_electron(t, S.data(), T.data(), V.data(), nullptr))
        return fail(c, FK_ERR_ARG, "SAD: atomic one-electron integrals failed: %s", t->err.c_str());
    for (size_t i = 0; i < n2; ++i) h[i] = T[i] + V[i];
    // every shell quartet's integrals, scattered into G[i][j][k][l] = (ij|kl)
    std::vector<int> q;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int cc = 0; cc < ns; ++cc)
                for (int d = 0; d < ns; ++d) q.insert(q.end(), {a, b, cc, d});
    size_t tot = 0;
    for (size_t k = 0; k < q.size(); k += 4)
        tot += (size_t)ncart(sl[q[k]]) * ncart(sl[q[k + 1]]) * ncart(sl[q[k + 2]]) * ncart(sl[q[k + 3]]);
    std::vector<double> out(tot), G(n2 * n2);
    if (fk_debug_eri(t, (int)(q.size() / 4), q.data(), out.data(), 0))
        return fail(c, FK_ERR_ARG, "SAD: atomic integrals failed: %s", t->err.c_str());
    size_t o = 0;
    for (size_t k = 0; k < q.size(); k += 4) {
        const int s0 = q[k], s1 = q[k + 1], s2 = q[k + 2], s3 = q[k + 3];
        const int n0 = ncart(sl[s0]), n1 = ncart(sl[s1]), n2_ = ncart(sl[s2]), n3 = ncart(sl[s3]);
        for (int i = 0; i < n0; ++i)
            for (int j = 0; j < n1; ++j)
                for (int kk = 0; kk < n2_; ++kk)
                    for (int l = 0; l < n3; ++l) {
                        const size_t I = t->sh_bf[s0] + i, J = t->sh_bf[s1] + j, K = t->sh_bf[s2] + kk, L = t->sh_bf[s3] + l;
                        G[((I * n + J) * n + K) * n + L] = out[o++];
                    }
    }
    // X = S^(-1/2)
    std::vector<double> w, U;
    jacobi_eigen(n, S, w, U);
    std::vector<double> X(n2, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0;
            for (int k = 0; k < n; ++k) s += U[(size_t)i * n + k] * U[(size_t)j * n + k] / std::sqrt(w[k]);
            X[(size_t)i * n + j] = s;
        }
    auto density_of = [&](const std::vector<double> &F, std::vector<double> &D) {
        std::vector<double> XF(n2, 0.0), Fp(n2, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0;
                for (int k = 0; k < n; ++k) s += X[(size_t)i * n + k] * F[(size_t)k * n + j];
                XF[(size_t)i * n + j] = s;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0;
                for (int k = 0; k < n; ++k) s += XF[(size_t)i * n + k] * X[(size_t)k * n + j];
                Fp[(size_t)i * n + j] = s;
            }
        std::vector<double> e, Cp;
        jacobi_eigen(n, Fp, e, Cp);
        std::vector<int> ord(n);
        for (int i = 0; i < n; ++i) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return e[a] < e[b]; });
        std::vector<double> occ(n, 0.0);
        double left = Z;
        for (int i = 0; i < n && left > 0;) {
            int j = i;
            while (j < n && e[ord[j]] - e[ord[i]] < 1e-4) ++j;
            const double each = std::min(2.0, left / (j - i));
            for (int k = i; k < j; ++k) occ[ord[k]] = each;
            left -= each * (j - i);
            i = j;
        }
        // C = X C'; D = sum_k occ_k c_k c_k^T
        std::vector<double> C(n2, 0.0);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double s = 0;
                for (int m = 0; m < n; ++m) s += X[(size_t)i * n + m] * Cp[(size_t)m * n + k];
                C[(size_t)i * n + k] = s;
            }
        D.assign(n2, 0.0);
        for (int k = 0; k < n; ++k) {
            if (occ[k] == 0.0) continue;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) D[(size_t)i * n + j] += occ[k] * C[(size_t)i * n + k] * C[(size_t)j * n + k];
        }
    };
    std::vector<double> D, Dn, F(n2);
    density_of(h, D);
    for (int it = 0; it < 500; ++it) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double jv = 0, kv = 0;
                for (int k = 0; k < n; ++k)
                    for (int l = 0; l < n; ++l) {
                        jv += G[(((size_t)i * n + j) * n + k) * n + l] * D[(size_t)k * n + l];
                        kv += G[(((size_t)i * n + k) * n + j) * n + l] * D[(size_t)k * n + l];
                    }
                F[(size_t)i * n + j] = h[(size_t)i * n + j] + jv - 0.5 * kv;
            }
        density_of(F, Dn);
        double delta = 0;
        for (size_t i = 0; i < n2; ++i) delta = std::max(delta, std::fabs(Dn[i] - D[i]));
        if (delta < 1e-10) {
            D = Dn;
            break;
        }
        for (size_t i = 0; i < n2; ++i) D[i] = 0.5 * Dn[i] + 0.5 * D[i];
    }
    Dat = D;
    return FK_OK;
}

}  // namespace

extern "C" {

int fk_sad_density(fk_ctx *c, double *D_out)
{
    if (!c) return FK_ERR_ARG;
    if (!D_out) return fail(c, FK_ERR_ARG, "fk_sad_density: null output");
    if (!c->have_basis) return fail(c, FK_ERR_STATE, "fk_sad_density: geometry and basis not set");
    // each atom's block sits in its molecule's block (one molecule: the whole matrix)
    std::vector<int> lf0(c->natom, -1), nf(c->natom, 0);
    for (int s = 0; s < c->nshell; ++s) {
        const int a = c->sh_atom[s];
        if (lf0[a] < 0) lf0[a] = c->sh_lbf[s];
        else if (lf0[a] + nf[a] != c->sh_lbf[s])
            return fail(c, FK_ERR_UNSUPPORTED, "fk_sad_density: the shells of atom %d are not consecutive", a);
        nf[a] += ncart(c->sh_l[s]);
    }
    std::fill(D_out, D_out + (size_t)c->mol_base[c->nmol], 0.0);
    int rc;
    for (int a = 0; a < c->natom; ++a) {
        if (nf[a] == 0) continue;
        // one atomic calculation per element and shell set (a batch may mix bases)
        std::vector<double> key{(double)c->Z[a]};
        for (int sh = 0; sh < c->nshell; ++sh) {
            if (c->sh_atom[sh] != a) continue;
            key.push_back(c->sh_l[sh]);
            key.push_back(c->sh_nprim[sh]);
            for (int p = c->sh_poff[sh]; p < c->sh_poff[sh + 1]; ++p) {
                key.push_back(c->exps[p]);
                key.push_back(c->coef_in[p]);
            }
        }
        auto it = c->sad_cache.find(key);
        if (it == c->sad_cache.end()) {
            std::vector<double> Dat;
            if ((rc = atomic_density(c, a, Dat))) return rc;
            it = c->sad_cache.emplace(std::move(key), std::move(Dat)).first;
        }
        const std::vector<double> &Dat = it->second;
        const int m = nf[a];
        if ((int)Dat.size() != m * m) return fail(c, FK_ERR_ARG, "fk_sad_density: internal: atomic block size");
        const int mol = c->atom_mol[a], n = c->mol_nbf[mol];
        double *Dm = D_out + c->mol_base[mol];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Dm[(size_t)(lf0[a] + i) * n + lf0[a] + j] = Dat[(size_t)i * m + j];
    }
    return FK_OK;
}

int fk_guess_pairs(fk_ctx *c, int *npair, float *features, int *shape)
{
    if (!c) return FK_ERR_ARG;
    if (!npair) return fail(c, FK_ERR_ARG, "fk_guess_pairs: null npair");
    std::vector<GuessPairHost> pairs;
    std::vector<int> f0, nf;
    int rc;
    if ((rc = guess_pair_list(c, pairs)) || (rc = atom_ranges(c, f0, nf))) return rc;
    *npair = (int)pairs.size();
    double Q[9];
    for (size_t p = 0; p < pairs.size(); ++p) {
        if (features) {
            local_frame(c, pairs[p].a1, pairs[p].a2, Q);
            guess_features(c, pairs[p], Q, features + p * FK_GUESS_NFEAT);
        }
        if (shape) shape[p] = (nf[pairs[p].a1] << 8) | nf[pairs[p].a2];
    }
    return FK_OK;
}

int fk_guess_targets(fk_ctx *c, const double *D, float *Y)
{
    if (!c) return FK_ERR_ARG;
    if (!D || !Y) return fail(c, FK_ERR_ARG, "fk_guess_targets: null argument");
    std::vector<GuessPairHost> pairs;
    std::vector<int> f0, nf;
    int rc;
    if ((rc = guess_pair_list(c, pairs)) || (rc = atom_ranges(c, f0, nf))) return rc;
    constexpr int W = FK_GUESS_NB;
    const int n = c->nbf;
    double B[W * W], Bb[W * W], T1[W * W], T2[W * W], H[W * W], Q[9];
    for (size_t p = 0; p < pairs.size(); ++p) {
        const int a1 = pairs[p].a1, a2 = pairs[p].a2, n1 = nf[a1], n2 = nf[a2];
        for (int i = 0; i < W * W; ++i) B[i] = 0.0;
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) B[i * W + j] = D[(size_t)(f0[a1] + i) * n + f0[a2] + j];
        // pair frame: D_frame = T(Q)^T D T(Q)
        local_frame(c, a1, a2, Q);
        atom_rotation(c, a1, Q, T1);
        atom_rotation(c, a2, Q, T2);
        blk_mul(B, false, T2, false, H);
        blk_mul(T1, true, H, false, Bb);
        float *y = Y + p * FK_GUESS_NOUT;
        for (int i = 0; i < W; ++i)
            for (int j = 0; j < W; ++j) y[i * W + j] = (i < n1 && j < n2) ? (float)Bb[i * W + j] : 0.0f;
    }
    return FK_OK;
}

int64_t fk_mlp_work_floats(const fk_mlp *m, int n)
{
    if (!m || m->nlayer < 1 || m->nlayer > FK_MLP_MAX_LAYERS || n < 0) return -1;
    int64_t w = 0, hmax = 0;
    for (int k = 0; k + 1 < m->nlayer; ++k) {
        w += 2 * (int64_t)n * m->dims[k + 1];
        hmax = std::max<int64_t>(hmax, m->dims[k + 1]);
    }
    return w + 2 * (int64_t)n * hmax;
}

static int mlp_check(const fk_mlp *m)
{
    if (!m || m->nlayer < 1 || m->nlayer > FK_MLP_MAX_LAYERS) return FK_ERR_ARG;
    for (int k = 0; k <= m->nlayer; ++k)
        if (m->dims[k] < 1 || m->dims[k] > 4096) return FK_ERR_ARG;
    for (int k = 0; k < m->nlayer; ++k)
        if (!m->W[k] || !m->b[k]) return FK_ERR_ARG;
    return FK_OK;
}

int fk_mlp_forward(const fk_mlp *m, const float *X, int n, float *Y, float *work, void *stream)
{
    if (mlp_check(m) || n < 0 || (n > 0 && (!X || !Y || (m->nlayer > 1 && !work)))) return FK_ERR_ARG;
    if (n == 0) return FK_OK;
    const float *in = X;
    float *wp = work;
    for (int k = 0; k < m->nlayer; ++k) {
        const int din = m->dims[k], dout = m->dims[k + 1];
        if (k + 1 < m->nlayer) {
            float *Z = wp, *A = wp + (size_t)n * dout;
            if (fk_guess_mm(0, 0, in, din, m->W[k], dout, Z, A, m->b[k], n, dout, din, stream)) return FK_ERR_HIP;
            in = A;
            wp += 2 * (size_t)n * dout;
        } else {
            if (fk_guess_mm(0, 0, in, din, m->W[k], dout, Y, nullptr, m->b[k], n, dout, din, stream)) return FK_ERR_HIP;
        }
    }
    return FK_OK;
}

int fk_mlp_backward(const fk_mlp *m, const float *X, int n, float *work, float *dY, const fk_mlp *grad, void *stream)
{
    if (mlp_check(m) || mlp_check(grad) || n < 0 || (n > 0 && (!X || !dY || (m->nlayer > 1 && !work)))) return FK_ERR_ARG;
    for (int k = 0; k <= m->nlayer; ++k)
        if (grad->dims[k] != m->dims[k] || grad->nlayer != m->nlayer) return FK_ERR_ARG;
    if (n == 0) return FK_OK;
    const int L = m->nlayer;
    // activations: layer k < L-1 keeps Z_k, A_k at zoff[k]
    std::vector<size_t> zoff(L, 0);
    size_t o = 0, hmax = 0;
    for (int k = 0; k + 1 < L; ++k) {
        zoff[k] = o;
        o += 2 * (size_t)n * m->dims[k + 1];
        hmax = std::max<size_t>(hmax, m->dims[k + 1]);
    }
    float *hbuf[2] = {work + o, work + o + (size_t)n * hmax};
    float *G = dY;
    for (int k = L - 1; k >= 0; --k) {
        const int din = m->dims[k], dout = m->dims[k + 1];
        const float *Ain = k == 0 ? X : work + zoff[k - 1] + (size_t)n * din;
        if (fk_guess_mm(1, 0, Ain, din, G, dout, grad->W[k], nullptr, nullptr, din, dout, n, stream)) return FK_ERR_HIP;
        if (fk_guess_colsum(G, n, dout, grad->b[k], stream)) return FK_ERR_HIP;
        if (k > 0) {
            float *H = hbuf[k & 1];
            if (fk_guess_mm(0, 1, G, dout, m->W[k], dout, H, nullptr, nullptr, n, din, dout, stream)) return FK_ERR_HIP;
            if (fk_guess_silu_back(H, work + zoff[k - 1], (long long)n * din, stream)) return FK_ERR_HIP;
            G = H;
        }
    }
    return FK_OK;
}

int fk_mlp_mse_scratch(void) { return fk_guess_mse_parts(); }

int fk_mlp_block_mse(const float *Y, const float *T, const int *shape, int n, double count, float *dY, double *part,
                     double *loss, void *stream)
{
    if (n < 0 || (n > 0 && (!Y || !T || !shape || !dY || !part || !loss)) || !(count > 0)) return FK_ERR_ARG;
    if (n == 0) return FK_OK;
    return fk_guess_block_mse(Y, T, shape, n, FK_GUESS_NB, count, dY, part, loss, stream) ? FK_ERR_HIP : FK_OK;
}

int fk_mlp_adam(const fk_mlp *m, const fk_mlp *grad, const fk_mlp *m1, const fk_mlp *m2, int step, float lr, float b1,
                float b2, float eps, void *stream)
{
    if (mlp_check(m) || mlp_check(grad) || mlp_check(m1) || mlp_check(m2) || step < 1) return FK_ERR_ARG;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
    for (int k = 0; k < m->nlayer; ++k) {
        const long long nw = (long long)m->dims[k] * m->dims[k + 1], nb = m->dims[k + 1];
        if (fk_guess_adam(m->W[k], grad->W[k], m1->W[k], m2->W[k], nw, lr, b1, b2, eps, c1, c2, stream) ||
            fk_guess_adam(m->b[k], grad->b[k], m1->b[k], m2->b[k], nb, lr, b1, b2, eps, c1, c2, stream))
            return FK_ERR_HIP;
    }
    return FK_OK;
}

int fk_set_guess_model(fk_ctx *c, const fk_mlp *hm)
{
    if (!c) return FK_ERR_ARG;
    if (!hm) {
        c->have_model = false;
        return FK_OK;
    }
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_set_guess_model: context has no device");
    if (mlp_check(hm) || hm->dims[0] != FK_GUESS_NFEAT || hm->dims[hm->nlayer] != FK_GUESS_NOUT)
        return fail(c, FK_ERR_ARG, "fk_set_guess_model: need 1..%d layers, %d inputs, %d outputs, dims <= 4096",
                    FK_MLP_MAX_LAYERS, FK_GUESS_NFEAT, FK_GUESS_NOUT);
    for (int k = 0; k < hm->nlayer; ++k)
        for (size_t i = 0; i < (size_t)hm->dims[k] * hm->dims[k + 1]; ++i)
            if (!std::isfinite(hm->W[k][i])) return fail(c, FK_ERR_ARG, "fk_set_guess_model: non-finite weight");
    hipSetDevice(c->device);
    c->g_model = *hm;
    int rc;
    for (int k = 0; k < hm->nlayer; ++k) {
        if ((rc = dev_upload<float>(c, c->g_W[k], hm->W[k], (size_t)hm->dims[k] * hm->dims[k + 1])) ||
            (rc = dev_upload<float>(c, c->g_b[k], hm->b[k], (size_t)hm->dims[k + 1])))
            return rc;
        c->g_model.W[k] = c->g_W[k].p;
        c->g_model.b[k] = c->g_b[k].p;
    }
    c->have_model = true;
    return FK_OK;
}

}  // extern "C"

namespace {

// Predicted (unpurified) density into the device array D (nbf x nbf) on `st`.
int guess_predict_device(fk_ctx *c, double *D, hipStream_t st)
{
    if (!c->have_model) return fail(c, FK_ERR_STATE, "learned guess: no model (fk_set_guess_model)");
    std::vector<GuessPairHost> pairs;
    std::vector<int> f0, nf;
    int rc;
    if ((rc = guess_pair_list(c, pairs)) || (rc = atom_ranges(c, f0, nf))) return rc;
    constexpr int W = FK_GUESS_NB;
    const int np = (int)pairs.size();
    std::vector<float> X((size_t)np * FK_GUESS_NFEAT);
    std::vector<FkGuessPair> gp(np);
    std::vector<double> rot((size_t)np * 2 * W * W);
    double Q[9], Qt[9];
    for (int p = 0; p < np; ++p) {
        const int a1 = pairs[p].a1, a2 = pairs[p].a2;
        local_frame(c, a1, a2, Q);
        guess_features(c, pairs[p], Q, &X[(size_t)p * FK_GUESS_NFEAT]);
        gp[p] = FkGuessPair{a1, a2, f0[a1], f0[a2], nf[a1], nf[a2]};
        // D_lab = T(Q^T)^T B T(Q^T)
        transpose3(Q, Qt);
        atom_rotation(c, a1, Qt, &rot[(size_t)p * 2 * W * W]);
        atom_rotation(c, a2, Qt, &rot[(size_t)p * 2 * W * W + W * W]);
    }
    const int64_t wf = fk_mlp_work_floats(&c->g_model, np);
    if ((rc = dev_upload(c, c->g_X, X.data(), X.size())) || (rc = dev_upload<float>(c, c->g_Y, nullptr, (size_t)np * FK_GUESS_NOUT)) ||
        (rc = dev_upload<float>(c, c->g_work, nullptr, (size_t)std::max<int64_t>(wf, 1))) ||
        (rc = dev_upload(c, c->g_pairs, gp.data(), gp.size())) || (rc = dev_upload(c, c->g_rot, rot.data(), rot.size())))
        return rc;
    if (fk_mlp_forward(&c->g_model, c->g_X.p, np, c->g_Y.p, c->g_work.p, st))
        return fail(c, FK_ERR_HIP, "learned guess: network launch failed");
    if (fk_guess_scatter(c->g_Y.p, c->g_pairs.p, c->g_rot.p, np, c->nbf, D, st))
        return fail(c, FK_ERR_HIP, "learned guess: scatter launch failed");
    return FK_OK;
}

}  // namespace

extern "C" int fk_guess_predict(fk_ctx *c, double *D_out)
{
    if (!c) return FK_ERR_ARG;
    if (!D_out) return fail(c, FK_ERR_ARG, "fk_guess_predict: null output");
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_guess_predict: context has no device");
    hipSetDevice(c->device);
    const size_t nn = (size_t)c->nbf * c->nbf;
    int rc;
    if ((rc = dev_upload<double>(c, c->g_D, nullptr, nn))) return rc;
    if ((rc = guess_predict_device(c, c->g_D.p, nullptr))) return rc;
    HIPCHK(c, hipMemcpy(D_out, c->g_D.p, nn * sizeof(double), hipMemcpyDeviceToHost));
    return FK_OK;
}

// ============================================================== batched SCF
// The SCF step for every molecule of a batch at once: one batched J/K build
// per iteration, and the dense steps as batched kernels over the
// concatenated per-molecule blocks, with per-molecule scalars (energies,
// DIIS systems, purification choices) on the host.
namespace {

// A host context holding molecule m of the batch alone (its atoms and shells).
int molecule_context(fk_ctx *c, int m, fk_ctx **out)
{
    *out = nullptr;
    int a0 = -1, na = 0;
    for (int a = 0; a < c->natom; ++a)
        if (c->atom_mol[a] == m) {
            if (a0 < 0) a0 = a;
            ++na;
        }
    const int s0 = c->mol_sh0[m], ns = c->mol_nsh[m];
    std::vector<int> Z(c->Z.begin() + a0, c->Z.begin() + a0 + na), satom(ns), sl(ns), snp(ns);
    std::vector<double> xyz(c->xyz.begin() + 3 * a0, c->xyz.begin() + 3 * (a0 + na)), ex, cf;
    for (int k = 0; k < ns; ++k) {
        const int s = s0 + k;
        satom[k] = c->sh_atom[s] - a0;
        sl[k] = c->sh_l[s];
        snp[k] = c->sh_nprim[s];
        for (int p = c->sh_poff[s]; p < c->sh_poff[s + 1]; ++p) {
            ex.push_back(c->exps[p]);
            cf.push_back(c->coef_in[p]);
        }
    }
    fk_ctx *t = nullptr;
    if (fk_create(&t, -1) != FK_OK) return fail(c, FK_ERR_OOM, "batched SCF: cannot create a molecule context");
    if (fk_set_geometry(t, na, Z.data(), xyz.data(), 0) || fk_set_basis(t, ns, satom.data(), sl.data(), snp.data(), ex.data(), cf.data())) {
        const int rc = fail(c, FK_ERR_ARG, "batched SCF: molecule %d: %s", m, t->err.c_str());
        fk_destroy(t);
        return rc;
    }
    *out = t;
    return FK_OK;
}

struct ScfBatch {
    fk_ctx *c = nullptr;
    hipStream_t st = nullptr;
    int nmol = 0, nmax = 0;
    size_t nm = 0;
    DevBuf<double> h, X, Xi, D, Do, J, K, F, Fo, G, E, T1, T2, T3, part, out, coef;
    DevBuf<double> Pn, ev, wk;  // canonical orthogonaliser
    DevBuf<int> info;
    std::vector<int> ndrop;     // per molecule
    std::vector<DevBuf<double>> ringF, ringE;
    ~ScfBatch()
    {
        for (auto *b : {&h, &X, &Xi, &D, &Do, &J, &K, &F, &Fo, &G, &E, &T1, &T2, &T3, &part, &out, &coef, &Pn, &ev, &wk})
            dev_free(*b);
        dev_free(info);
        for (auto &b : ringF) dev_free(b);
        for (auto &b : ringE) dev_free(b);
    }
    const int *nbf() const { return c->d_mol_nbf.p; }
    const long long *off() const { return c->d_mol_base.p; }
    int gemm(const double *A, const double *B, double *C, double alpha = 1.0, double beta = 0.0)
    {
        return fk_scfb_gemm(A, B, C, nmol, nmax, nbf(), off(), alpha, beta, st) ? fail(c, FK_ERR_HIP, "batched SCF: GEMM launch failed") : FK_OK;
    }
    // out = a_m x + b_m y + c_m z + d_m I, coefficients [4 nmol] from the host
    int lincomb(double *o, const double *x, const double *y, const double *z, const std::vector<double> &cf)
    {
        HIPCHK(c, hipMemcpy(coef.p, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice));
        return fk_scfb_lincomb(o, x, y, z, nmol, nmax, nbf(), off(), coef.p, st) ? fail(c, FK_ERR_HIP, "batched SCF: launch failed") : FK_OK;
    }
    int lincomb_u(double *o, const double *x, const double *y, const double *z, double a, double b, double cc, double d)
    {
        std::vector<double> cf(4 * (size_t)nmol);
        for (int m = 0; m < nmol; ++m) { cf[4 * m] = a; cf[4 * m + 1] = b; cf[4 * m + 2] = cc; cf[4 * m + 3] = d; }
        return lincomb(o, x, y, z, cf);
    }
    int reduce(const double *x, const double *y, int op, std::vector<double> &r)
    {
        if (fk_scfb_reduce(x, y, nmol, nbf(), off(), op, part.p, out.p, st)) return fail(c, FK_ERR_HIP, "batched SCF: reduction launch failed");
        r.resize((op == 3 ? 2 : 1) * (size_t)nmol);
        HIPCHK(c, hipMemcpyAsync(r.data(), out.p, r.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return FK_OK;
    }
};

int scfb_orthogonaliser(ScfBatch &w, double tol)
{
    const int nm = w.nmol;
    std::vector<double> gb, err, prev(nm, 1e300);
    int rc;
    if ((rc = w.reduce(w.T3.p, nullptr, 3, gb))) return rc;  // T3 holds S
    std::vector<double> cs(nm), cf(4 * (size_t)nm, 0.0);
    for (int m = 0; m < nm; ++m) {
        cs[m] = gb[nm + m];
        if (!(cs[m] > 0)) return fail(w.c, FK_ERR_ARG, "batched SCF: molecule %d: overlap matrix has no positive bound", m);
        cf[4 * m] = 1.0 / cs[m];
    }
    if ((rc = w.lincomb(w.Xi.p, w.T3.p, nullptr, nullptr, cf)) || (rc = w.lincomb_u(w.X.p, w.T3.p, nullptr, nullptr, 0, 0, 0, 1)))
        return rc;
    std::vector<char> done(nm, 0);
    for (int it = 0; it < 200; ++it) {
        if ((rc = w.gemm(w.X.p, w.Xi.p, w.T1.p)) || (rc = w.lincomb_u(w.T2.p, w.T1.p, nullptr, nullptr, 1, 0, 0, -1)) ||
            (rc = w.reduce(w.T2.p, nullptr, 1, err)))
            return rc;
        bool all = true;
        for (int m = 0; m < nm; ++m) {
            if (err[m] < tol * 1e-3 || (err[m] < 1e-9 && err[m] > 0.5 * prev[m])) done[m] = 1;
            prev[m] = err[m];
            all = all && done[m];
        }
        if (all) break;
        if ((rc = w.lincomb_u(w.T2.p, w.T1.p, nullptr, nullptr, -0.5, 0, 0, 1.5)) || (rc = w.gemm(w.Xi.p, w.T2.p, w.T1.p)) ||
            (rc = w.gemm(w.T2.p, w.X.p, w.G.p)))
            return rc;
        std::swap(w.Xi, w.T1);
        std::swap(w.X, w.G);
    }
    for (int m = 0; m < nm; ++m)
        if (!(err[m] < tol))
            return fail(w.c, FK_ERR_ARG, "batched SCF: molecule %d: S^(-1/2) did not converge (%.3g)", m, err[m]);
    std::vector<double> c1(4 * (size_t)nm, 0.0), c2(4 * (size_t)nm, 0.0);
    for (int m = 0; m < nm; ++m) {
        c1[4 * m] = 1.0 / std::sqrt(cs[m]);
        c2[4 * m] = std::sqrt(cs[m]);
    }
    if ((rc = w.lincomb(w.X.p, w.X.p, nullptr, nullptr, c1)) || (rc = w.lincomb(w.Xi.p, w.Xi.p, nullptr, nullptr, c2))) return rc;
    std::vector<double> xmax;
    if ((rc = w.reduce(w.X.p, nullptr, 1, xmax))) return rc;
    for (int m = 0; m < nm; ++m)
        if (!(xmax[m] < kMaxOrthoEntry))
            return fail(w.c, FK_ERR_ARG, "batched SCF: molecule %d: max |S^(-1/2)| = %.3g: the basis is nearly linearly dependent", m, xmax[m]);
    return FK_OK;
}

// Canonical orthogonalisers of every molecule (w.T3 holds the overlap blocks):
// per molecule S = U s U^T, X = U s^(-1/2) U^T, Xi = U s^(1/2) U^T over the
// eigenvalues above `cutoff`, and the dropped directions' projector in w.Pn.
int scfb_orthogonaliser_canonical(ScfBatch &w, double cutoff)
{
    fk_ctx *c = w.c;
    const int nm = w.nmol;
    int rc;
    if ((rc = dev_upload<double>(c, w.ev, nullptr, w.nm)) || (rc = dev_upload<double>(c, w.wk, nullptr, w.nmax)) ||
        (rc = dev_upload<int>(c, w.info, nullptr, nm)))
        return rc;
    HIPCHK(c, hipMemcpyAsync(w.T1.p, w.T3.p, w.nm * sizeof(double), hipMemcpyDeviceToDevice, w.st));
    for (int m = 0; m < nm; ++m)
        if (fk_scf_eigh(w.T1.p + c->mol_base[m], w.ev.p + c->mol_base[m], w.wk.p, w.info.p + m, c->mol_nbf[m], w.st))
            return fail(c, FK_ERR_HIP, "batched SCF: molecule %d: eigen-decomposition launch failed", m);
    std::vector<int> info(nm);
    std::vector<double> s(w.nm);
    HIPCHK(c, hipMemcpy(info.data(), w.info.p, nm * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(s.data(), w.ev.p, w.nm * sizeof(double), hipMemcpyDeviceToHost));
    w.ndrop.assign(nm, 0);
    bool any = false;
    for (int m = 0; m < nm; ++m) {
        if (info[m] != 0) return fail(c, FK_ERR_HIP, "batched SCF: molecule %d: overlap eigen-decomposition failed (info %d)", m, info[m]);
        const int n = c->mol_nbf[m];
        for (int i = 0; i < n; ++i) w.ndrop[m] += s[c->mol_base[m] + i] > cutoff ? 0 : 1;
        if (w.ndrop[m] >= n) return fail(c, FK_ERR_ARG, "batched SCF: molecule %d: every overlap eigenvalue is below the cutoff", m);
        any = any || w.ndrop[m] > 0;
    }
    for (int k = 0; k < 2; ++k) {
        for (int m = 0; m < nm; ++m)
            if (fk_scf_eig_scale(w.T1.p + c->mol_base[m], w.ev.p + c->mol_base[m], w.T2.p + c->mol_base[m],
                                 c->mol_nbf[m], cutoff, k == 0 ? -0.5 : 0.5, w.st))
                return fail(c, FK_ERR_HIP, "batched SCF: launch failed");
        if ((rc = w.gemm(w.T2.p, w.T1.p, k == 0 ? w.X.p : w.Xi.p))) return rc;
    }
    if (any) {
        if ((rc = dev_upload<double>(c, w.Pn, nullptr, w.nm)) || (rc = w.gemm(w.X.p, w.Xi.p, w.T2.p)) ||
            (rc = w.lincomb_u(w.Pn.p, w.T2.p, nullptr, nullptr, -1.0, 0, 0, 1.0)))
            return rc;
    }
    return FK_OK;
}

// F'_m (w.Fo) plus the shift of each molecule's dropped directions.
int scfb_shift_null(ScfBatch &w)
{
    if (w.ndrop.empty() || std::find_if(w.ndrop.begin(), w.ndrop.end(), [](int x) { return x > 0; }) == w.ndrop.end())
        return FK_OK;
    std::vector<double> cf(4 * (size_t)w.nmol, 0.0);
    for (int m = 0; m < w.nmol; ++m) {
        cf[4 * m] = 1.0;
        cf[4 * m + 1] = w.ndrop[m] > 0 ? kNullShift : 0.0;
    }
    return w.lincomb(w.Fo.p, w.Fo.p, w.Pn.p, nullptr, cf);
}

// Orthonormal densities D'_m = 2 P_m from F'_m in Fo (trace-correcting
// purification per molecule; molecules that have converged keep P).
int scfb_purify(ScfBatch &w, const std::vector<int> &nocc)
{
    const int nm = w.nmol;
    std::vector<double> gb, t1, t2, cf(4 * (size_t)nm, 0.0);
    int rc;
    if ((rc = w.reduce(w.Fo.p, nullptr, 3, gb))) return rc;
    for (int m = 0; m < nm; ++m) {
        const double lo = gb[m], hi = gb[nm + m];
        if (!(hi > lo)) return fail(w.c, FK_ERR_ARG, "batched SCF: molecule %d: degenerate Fock spectrum bounds", m);
        cf[4 * m] = -1.0 / (hi - lo);
        cf[4 * m + 3] = hi / (hi - lo);
    }
    if ((rc = w.lincomb(w.T1.p, w.Fo.p, nullptr, nullptr, cf))) return rc;
    std::vector<int> extra(nm, -1);
    bool all = false;
    for (int it = 0; it < 300 && !all; ++it) {
        if ((rc = w.gemm(w.T1.p, w.T1.p, w.T2.p)) || (rc = w.reduce(w.T1.p, nullptr, 2, t1)) || (rc = w.reduce(w.T2.p, nullptr, 2, t2)))
            return rc;
        all = true;
        for (int m = 0; m < nm; ++m) {
            double a = 1.0, b = 0.0;  // keep P
            if (extra[m] != 0) {
                const double idem = t1[m] - t2[m];
                if (extra[m] < 0 && std::fabs(idem) < 1e-11) extra[m] = 2;
                if (extra[m] != 0) {
                    if (extra[m] > 0) --extra[m];
                    if (std::fabs(t2[m] - nocc[m]) < std::fabs(2 * t1[m] - t2[m] - nocc[m])) { a = 0.0; b = 1.0; }
                    else { a = 2.0; b = -1.0; }
                }
            }
            cf[4 * m] = a; cf[4 * m + 1] = b; cf[4 * m + 2] = 0.0; cf[4 * m + 3] = 0.0;
            all = all && extra[m] == 0;
        }
        if (all) break;
        if ((rc = w.lincomb(w.T1.p, w.T1.p, w.T2.p, nullptr, cf))) return rc;
    }
    if (!all) return fail(w.c, FK_ERR_NOT_CONVERGED, "batched SCF: purification did not converge (no gap?)");
    return w.lincomb_u(w.Do.p, w.T1.p, nullptr, nullptr, 2.0, 0, 0, 0);
}

// Orthonormal densities D'_m = 2 C_o C_o^T from the eigenvectors of each
// molecule's nocc_m lowest states of F'_m in Fo (rocSOLVER per molecule).
int scfb_density_eig(ScfBatch &w, const std::vector<int> &nocc)
{
    fk_ctx *c = w.c;
    const int nm = w.nmol;
    int rc;
    if ((rc = dev_upload<double>(c, w.ev, nullptr, w.nm)) || (rc = dev_upload<double>(c, w.wk, nullptr, w.nmax)) ||
        (rc = dev_upload<int>(c, w.info, nullptr, nm)))
        return rc;
    HIPCHK(c, hipMemcpyAsync(w.T1.p, w.Fo.p, w.nm * sizeof(double), hipMemcpyDeviceToDevice, w.st));
    for (int m = 0; m < nm; ++m)
        if (fk_scf_eigh(w.T1.p + c->mol_base[m], w.ev.p + c->mol_base[m], w.wk.p, w.info.p + m, c->mol_nbf[m], w.st))
            return fail(c, FK_ERR_HIP, "batched SCF: molecule %d: eigen-decomposition launch failed", m);
    std::vector<int> info(nm);
    std::vector<double> occ(w.nm);
    HIPCHK(c, hipMemcpy(info.data(), w.info.p, nm * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(occ.data(), w.ev.p, w.nm * sizeof(double), hipMemcpyDeviceToHost));
    for (int m = 0; m < nm; ++m) {
        if (info[m] != 0) return fail(c, FK_ERR_HIP, "batched SCF: molecule %d: eigen-decomposition of X F X failed (info %d)", m, info[m]);
        const int n = c->mol_nbf[m];
        double *e = occ.data() + c->mol_base[m];
        if (nocc[m] < n && !(e[nocc[m]] > e[nocc[m] - 1]))
            return fail(c, FK_ERR_NOT_CONVERGED, "batched SCF: molecule %d: no gap between the occupied and virtual states", m);
        for (int k = 0; k < n; ++k) e[k] = k < nocc[m] ? 2.0 : 0.0;
    }
    HIPCHK(c, hipMemcpy(w.ev.p, occ.data(), w.nm * sizeof(double), hipMemcpyHostToDevice));
    for (int m = 0; m < nm; ++m)
        if (fk_scf_eig_scale(w.T1.p + c->mol_base[m], w.ev.p + c->mol_base[m], w.T2.p + c->mol_base[m], c->mol_nbf[m], 1.0,
                             1.0, w.st))
            return fail(c, FK_ERR_HIP, "batched SCF: launch failed");
    return w.gemm(w.T2.p, w.T1.p, w.Do.p);
}

// The batched SCF with every per-iteration decision on the device (the
// convergence flags, the DIIS ring slot and Pulay solve, the purification's
// choices with a fixed budget of steps, the density of converged molecules
// kept), so that one iteration -- J/K build included -- is captured once as
// a HIP graph and replayed; the host reads the energies, errors and flags
// after each replay to stop.  Results equal the eager loop's up to rounding.
constexpr int kScfbGraphPurSteps = 128;

int scfb_graph_loop(ScfBatch &w, const fk_scf_opts &o, const std::vector<int> &nocc, const std::vector<double> &enuc,
                    fk_scf_result *results, double *D_inout, std::chrono::steady_clock::time_point t_start)
{
    fk_ctx *c = w.c;
    const int nmol = w.nmol, nmax = w.nmax;
    const size_t nmat = w.nm;
    const int dn = std::max(o.diis_n, 1);
    if (dn > FK_SCFB_MAX_DIIS) return fail(c, FK_ERR_ARG, "batched SCF graph: at most %d DIIS vectors", FK_SCFB_MAX_DIIS);
    int rc;
    struct Res {
        hipStream_t st = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        ~Res()
        {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
            if (st) (void)hipStreamDestroy(st);
        }
    } gr;
    HIPCHK(c, hipStreamCreate(&gr.st));
    hipStream_t st = gr.st;
    DevBuf<int> ictl, conv, pstate, pdone, dnocc;
    DevBuf<double> eprev, dh, df, errv, gb, t1, t2, denuc, status, cF, cShift, cP, cDo, cKeep, Bm, dcoef, dpart, ringF, ringE;
    struct Free {
        std::vector<DevBuf<int> *> i;
        std::vector<DevBuf<double> *> d;
        ~Free() { for (auto *b : i) dev_free(*b); for (auto *b : d) dev_free(*b); }
    } fr{{&ictl, &conv, &pstate, &pdone, &dnocc},
         {&eprev, &dh, &df, &errv, &gb, &t1, &t2, &denuc, &status, &cF, &cShift, &cP, &cDo, &cKeep, &Bm, &dcoef, &dpart, &ringF, &ringE}};
    std::vector<double> k4(4 * (size_t)nmol, 0.0), kS(4 * (size_t)nmol, 0.0), kD(4 * (size_t)nmol, 0.0);
    for (int m = 0; m < nmol; ++m) {
        k4[4 * m] = 1.0; k4[4 * m + 1] = 1.0; k4[4 * m + 2] = -0.5;
        kS[4 * m] = 1.0; kS[4 * m + 1] = (!w.ndrop.empty() && w.ndrop[m] > 0) ? kNullShift : 0.0;
        kD[4 * m] = 2.0;
    }
    const bool shifted = !w.ndrop.empty() && std::find_if(w.ndrop.begin(), w.ndrop.end(), [](int x) { return x > 0; }) != w.ndrop.end();
    const std::vector<int> zi(std::max(nmol, 4), 0);
    const std::vector<double> zd(std::max<size_t>((size_t)nmol * dn * dn, 3 * (size_t)nmol), 0.0);
    if ((rc = dev_upload(c, ictl, zi.data(), 4)) || (rc = dev_upload(c, conv, zi.data(), nmol)) ||
        (rc = dev_upload<int>(c, pstate, nullptr, nmol)) || (rc = dev_upload<int>(c, pdone, nullptr, nmol)) ||
        (rc = dev_upload(c, dnocc, nocc.data(), nmol)) || (rc = dev_upload(c, eprev, zd.data(), nmol)) ||
        (rc = dev_upload<double>(c, dh, nullptr, nmol)) || (rc = dev_upload<double>(c, df, nullptr, nmol)) ||
        (rc = dev_upload<double>(c, errv, nullptr, nmol)) || (rc = dev_upload<double>(c, gb, nullptr, 2 * (size_t)nmol)) ||
        (rc = dev_upload<double>(c, t1, nullptr, nmol)) || (rc = dev_upload<double>(c, t2, nullptr, nmol)) ||
        (rc = dev_upload(c, denuc, enuc.data(), nmol)) || (rc = dev_upload(c, status, zd.data(), 3 * (size_t)nmol)) ||
        (rc = dev_upload(c, cF, k4.data(), k4.size())) || (rc = dev_upload(c, cShift, kS.data(), kS.size())) ||
        (rc = dev_upload<double>(c, cP, nullptr, 4 * (size_t)nmol)) || (rc = dev_upload(c, cDo, kD.data(), kD.size())) ||
        (rc = dev_upload<double>(c, cKeep, nullptr, 4 * (size_t)nmol)) || (rc = dev_upload(c, Bm, zd.data(), (size_t)nmol * dn * dn)) ||
        (rc = dev_upload<double>(c, dcoef, nullptr, (size_t)nmol * dn)) ||
        (rc = dev_upload<double>(c, dpart, nullptr, (size_t)nmol * dn * 32)) ||
        (rc = dev_upload<double>(c, ringF, nullptr, (size_t)dn * nmat)) || (rc = dev_upload<double>(c, ringE, nullptr, (size_t)dn * nmat)))
        return rc;
    // empty ring slots read as zeros (their inner products are never used)
    if (fk_kernels_launch_fill(ringF.p, (long long)(dn * nmat), st) || fk_kernels_launch_fill(ringE.p, (long long)(dn * nmat), st))
        return fail(c, FK_ERR_HIP, "batched SCF graph: fill launch failed");
    HIPCHK(c, hipStreamSynchronize(st));
    const int *nbf = w.nbf();
    const long long *off = w.off();
    auto L = [&](double *o_, const double *x, const double *y, const double *z, const double *cf) {
        return fk_scfb_lincomb(o_, x, y, z, nmol, nmax, nbf, off, cf, st);
    };
    auto G = [&](const double *A, const double *B, double *C_) { return fk_scfb_gemm(A, B, C_, nmol, nmax, nbf, off, 1.0, 0.0, st); };
    auto R = [&](const double *x, const double *y, int op, double *out) {
        return fk_scfb_reduce(x, y, nmol, nbf, off, op, w.part.p, out, st);
    };
    // one iteration, every step a kernel or a device copy
    auto enqueue = [&]() -> int {
        int r = 0;
        r |= fk_scfb_iter_begin(ictl.p, dn, st);
        if (r) return fail(c, FK_ERR_HIP, "batched SCF graph: launch failed");
        if ((r = fk_build_jk(c, w.D.p, w.J.p, w.K.p, FK_DEVICE_PTRS, st))) return r;
        r |= L(w.F.p, w.h.p, w.J.p, w.K.p, cF.p);
        r |= R(w.D.p, w.h.p, 0, dh.p);
        r |= R(w.D.p, w.F.p, 0, df.p);
        r |= G(w.X.p, w.F.p, w.T3.p);
        r |= G(w.T3.p, w.X.p, w.Fo.p);
        if (shifted) r |= L(w.Fo.p, w.Fo.p, w.Pn.p, nullptr, cShift.p);
        r |= G(w.Fo.p, w.Do.p, w.G.p);
        r |= fk_scfb_antisym(w.E.p, w.G.p, nmol, nmax, nbf, off, st);
        r |= R(w.E.p, nullptr, 1, errv.p);
        r |= fk_scfb_conv(dh.p, df.p, errv.p, denuc.p, nmol, o.e_tol, o.g_tol, ictl.p, conv.p, eprev.p, cKeep.p, status.p, st);
        if (o.diis_n > 1)
            r |= fk_scfb_diis(ringF.p, ringE.p, w.Fo.p, w.E.p, w.Fo.p, nmol, nmax, nbf, off, (long long)nmat, dn, ictl.p,
                              dpart.p, Bm.p, dcoef.p, st);
        if (r) return fail(c, FK_ERR_HIP, "batched SCF graph: launch failed");
        // the converged molecules' densities, kept below
        HIPCHK(c, hipMemcpyAsync(w.G.p, w.Do.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(w.E.p, w.D.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, st));
        r |= R(w.Fo.p, nullptr, 3, gb.p);
        r |= fk_scfb_pur_start(gb.p, nmol, cP.p, pstate.p, pdone.p, ictl.p, st);
        r |= L(w.T1.p, w.Fo.p, nullptr, nullptr, cP.p);
        for (int k = 0; k < kScfbGraphPurSteps; ++k) {
            r |= fk_scfb_gemm_skip(w.T1.p, w.T1.p, w.T2.p, nmol, nmax, nbf, off, pdone.p, st);
            r |= R(w.T1.p, nullptr, 2, t1.p);
            r |= R(w.T2.p, nullptr, 2, t2.p);
            r |= fk_scfb_pur_step(t1.p, t2.p, dnocc.p, nmol, cP.p, pstate.p, pdone.p, st);
            r |= L(w.T1.p, w.T1.p, w.T2.p, nullptr, cP.p);
        }
        r |= fk_scfb_pur_check(pstate.p, nmol, ictl.p, st);
        r |= L(w.Do.p, w.T1.p, nullptr, nullptr, cDo.p);
        r |= G(w.X.p, w.Do.p, w.T3.p);
        r |= G(w.T3.p, w.X.p, w.D.p);
        r |= L(w.Do.p, w.Do.p, w.G.p, nullptr, cKeep.p);
        r |= L(w.D.p, w.D.p, w.E.p, nullptr, cKeep.p);
        return r ? fail(c, FK_ERR_HIP, "batched SCF graph: launch failed") : FK_OK;
    };
    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = enqueue();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    gr.g = g;
    if (rc) return rc;
    if (e != hipSuccess) return fail(c, FK_ERR_HIP, "batched SCF graph: capture failed: %s", hipGetErrorString(e));
    HIPCHK(c, hipGraphInstantiate(&gr.x, gr.g, nullptr, nullptr, 0));
    std::vector<double> stat(3 * (size_t)nmol);
    std::vector<int> ic(4);
    std::vector<char> done(nmol, 0);
    std::vector<double> e_prev(nmol, 0.0), de_cur(nmol, 0.0), e_fin(nmol, 0.0), err_fin(nmol, 0.0), de_fin(nmol, 0.0);
    std::vector<int> it_fin(nmol, 0);
    const char *lg = std::getenv("FK_SCF_LOG");
    const bool log = lg && *lg && *lg != '0';
    double jk_s = 0;
    int it = 0;
    bool all_conv = false;
    for (; it < o.max_iter; ++it) {
        const auto t0 = std::chrono::steady_clock::now();
        HIPCHK(c, hipGraphLaunch(gr.x, st));
        HIPCHK(c, hipMemcpyAsync(stat.data(), status.p, stat.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(ic.data(), ictl.p, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        jk_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        all_conv = true;
        for (int m = 0; m < nmol; ++m) {
            const double em = stat[m], er = stat[nmol + m];
            const bool cm = stat[2 * nmol + m] != 0.0;
            if (!done[m] && (!std::isfinite(em) || !std::isfinite(er)))
                return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf_batch: molecule %d: non-finite energy or error at iteration %d", m, it + 1);
            if (cm && !done[m]) {
                done[m] = 1;
                e_fin[m] = em;
                err_fin[m] = er;
                de_fin[m] = em - e_prev[m];
                it_fin[m] = it + 1;
            }
            de_cur[m] = em - e_prev[m];
            e_prev[m] = em;
            all_conv = all_conv && done[m];
        }
        if (log)
            std::fprintf(stderr, "fk_run_scf_batch (graph): iteration %d: %d of %d converged, %.1f s\n", it + 1,
                         (int)std::count(done.begin(), done.end(), 1), nmol,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
        if (all_conv) {
            ++it;
            break;
        }
        if (ic[3] == 1) return fail(c, FK_ERR_ARG, "batched SCF: degenerate Fock spectrum bounds");
        if (ic[3] == 2) return fail(c, FK_ERR_NOT_CONVERGED, "batched SCF: purification did not converge in %d steps", kScfbGraphPurSteps);
    }
    HIPCHK(c, hipMemcpy(D_inout, w.D.p, nmat * sizeof(double), hipMemcpyDeviceToHost));
    const double tot = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int m = 0; m < nmol; ++m) {
        fk_scf_result &r = results[m];
        r.energy = done[m] ? e_fin[m] : stat[m];
        r.iterations = done[m] ? it_fin[m] : it;
        r.converged = done[m] ? 1 : 0;
        r.error = done[m] ? err_fin[m] : stat[nmol + m];
        r.delta_e = done[m] ? de_fin[m] : de_cur[m];
        r.jk_seconds = jk_s;
        r.total_seconds = tot;
        r.ndropped = w.ndrop.empty() ? 0 : w.ndrop[m];
    }
    if (!all_conv) return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf_batch: not every molecule converged in %d iterations", o.max_iter);
    return FK_OK;
}

}  // namespace

extern "C" int fk_run_scf_batch(fk_ctx *c, const fk_scf_opts *opts, fk_scf_result *results, double *D_inout)
{
    if (!c) return FK_ERR_ARG;
    if (!results || !D_inout) return fail(c, FK_ERR_ARG, "fk_run_scf_batch: null results or density pointer");
    if (c->device < 0) return fail(c, FK_ERR_STATE, "fk_run_scf_batch: context has no device");
    if (!c->have_quartets) return fail(c, FK_ERR_STATE, "fk_run_scf_batch: call fk_build_quartets first");
    const int nmol = c->nmol;
    std::memset(results, 0, sizeof(fk_scf_result) * (size_t)nmol);
    fk_scf_opts o = {100, 1e-10, 1e-8, 8, 0, 1e-8, 0, 0, 0.0, 0, 0};
    if (opts) o = *opts;
    if (o.max_iter < 0 || o.diis_n < 0 || o.diis_n > 32 || !(o.e_tol > 0) || !(o.g_tol > 0) || !(o.lindep > 0) ||
        !(o.canonical >= 0 && o.canonical < 1) || o.j_engine != 0 || o.guess < 0 || o.guess > 3 ||
        (o.graph != 0 && o.graph != 1) || o.incremental != 0 || (o.density_eig != 0 && o.density_eig != 1))
        return fail(c, FK_ERR_ARG, "fk_run_scf_batch: invalid options");
    if (o.graph && o.density_eig)
        return fail(c, FK_ERR_UNSUPPORTED, "fk_run_scf_batch: the graph loop forms densities by purification only");
    if (c->charge != 0) return fail(c, FK_ERR_UNSUPPORTED, "fk_run_scf_batch: the molecules of a batch must be neutral");
    const auto t_start = std::chrono::steady_clock::now();
    hipSetDevice(c->device);
    int rc;
    // one-electron part per molecule (host threads, molecules round-robin),
    // electron counts
    const size_t nmat = (size_t)c->mol_base[nmol];
    std::vector<double> Sh(nmat), hh(nmat), enuc(nmol);
    std::vector<int> nocc(nmol), mrc(nmol, FK_OK), nel(nmol, 0);
    int nmax = 0;
    for (int m = 0; m < nmol; ++m) nmax = std::max(nmax, c->mol_nbf[m]);
    {
        std::vector<fk_ctx *> tc(nmol, nullptr);
        for (int m = 0; m < nmol; ++m)  // contexts first: their errors go to c
            if ((rc = molecule_context(c, m, &tc[m]))) {
                for (fk_ctx *t : tc) fk_destroy(t);
                return rc;
            }
        const int nth = std::max(1, std::min<int>({16, nmol, (int)std::max(1u, std::thread::hardware_concurrency())}));
        auto work = [&](int tid) {
            for (int m = tid; m < nmol; m += nth) {
                const int n = c->mol_nbf[m];
                std::vector<double> S(n * (size_t)n), T(S.size()), V(S.size());
                mrc[m] = fk_one_electron(tc[m], S.data(), T.data(), V.data(), &enuc[m]);
                nel[m] = tc[m]->nelec;
                if (mrc[m]) continue;
                for (size_t i = 0; i < S.size(); ++i) {
                    Sh[c->mol_base[m] + i] = S[i];
                    hh[c->mol_base[m] + i] = T[i] + V[i];
                }
            }
        };
        std::vector<std::thread> pool;
        for (int k = 1; k < nth; ++k) pool.emplace_back(work, k);
        work(0);
        for (auto &th : pool) th.join();
        for (fk_ctx *t : tc) fk_destroy(t);
    }
    for (int m = 0; m < nmol; ++m) {
        if (mrc[m]) return fail(c, mrc[m], "fk_run_scf_batch: molecule %d: one-electron integrals failed", m);
        const int ne = nel[m];
        if (ne % 2 || ne <= 0 || ne / 2 > c->mol_nbf[m])
            return fail(c, FK_ERR_ARG, "fk_run_scf_batch: molecule %d: %d electrons", m, ne);
        nocc[m] = ne / 2;
    }
    ScfBatch w;
    w.c = c;
    w.nmol = nmol;
    w.nmax = nmax;
    w.nm = nmat;
    for (auto *b : {&w.h, &w.X, &w.Xi, &w.D, &w.Do, &w.J, &w.K, &w.F, &w.Fo, &w.G, &w.E, &w.T1, &w.T2, &w.T3})
        if ((rc = dev_upload<double>(c, *b, nullptr, nmat))) return rc;
    if ((rc = dev_upload<double>(c, w.part, nullptr, (size_t)fk_scfb_reduce_scratch(nmol))) ||
        (rc = dev_upload<double>(c, w.out, nullptr, 2 * (size_t)nmol)) || (rc = dev_upload<double>(c, w.coef, nullptr, 4 * (size_t)nmol)))
        return rc;
    const int dn = std::max(o.diis_n, 1);
    w.ringF.resize(dn);
    w.ringE.resize(dn);
    if (o.diis_n > 1)
        for (int k = 0; k < dn; ++k)
            if ((rc = dev_upload<double>(c, w.ringF[k], nullptr, nmat)) || (rc = dev_upload<double>(c, w.ringE[k], nullptr, nmat)))
                return rc;
    if ((rc = dev_upload(c, w.h, hh.data(), nmat)) || (rc = dev_upload(c, w.T3, Sh.data(), nmat))) return rc;
    if ((rc = o.canonical > 0 ? scfb_orthogonaliser_canonical(w, o.canonical) : scfb_orthogonaliser(w, o.lindep))) return rc;

    // initial orthonormal densities: the learned guess is per molecule only,
    // so a batch starts it from SAD
    const auto t_guess = std::chrono::steady_clock::now();
    int gused = o.guess == 3 ? 2 : o.guess;
    if (gused == 2) {
        std::vector<double> Dsad(nmat);
        if (fk_sad_density(c, Dsad.data()) || dev_upload(c, w.D, Dsad.data(), nmat)) {
            gused = 0;
            c->err.clear();
        }
    } else if (gused == 1) {
        if ((rc = dev_upload(c, w.D, D_inout, nmat))) return rc;
    }
    if (gused == 0) {
        if ((rc = w.gemm(w.X.p, w.h.p, w.T3.p)) || (rc = w.gemm(w.T3.p, w.X.p, w.Fo.p)) || (rc = scfb_shift_null(w)) ||
            (rc = o.density_eig ? scfb_density_eig(w, nocc) : scfb_purify(w, nocc)))
            return rc;
    } else {
        if ((rc = w.gemm(w.Xi.p, w.D.p, w.T3.p)) || (rc = w.gemm(w.T3.p, w.Xi.p, w.Do.p))) return rc;
    }
    if ((rc = w.gemm(w.X.p, w.Do.p, w.T3.p)) || (rc = w.gemm(w.T3.p, w.X.p, w.D.p))) return rc;
    HIPCHK(c, hipStreamSynchronize(w.st));
    const double guess_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_guess).count();
    for (int m = 0; m < nmol; ++m) {
        results[m].e_nuc = enuc[m];
        results[m].guess_used = gused;
        results[m].guess_seconds = guess_s;
    }
    if (o.max_iter == 0) {
        HIPCHK(c, hipMemcpy(D_inout, w.D.p, nmat * sizeof(double), hipMemcpyDeviceToHost));
        const double tot = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        for (int m = 0; m < nmol; ++m) results[m].total_seconds = tot;
        return FK_OK;
    }

    if (o.graph) return scfb_graph_loop(w, o, nocc, enuc, results, D_inout, t_start);

    std::vector<double> e_prev(nmol, 0.0), e_cur(nmol, 0.0), err(nmol, 0.0), dh, df, ev;
    std::vector<std::vector<double>> Bm(nmol, std::vector<double>((size_t)dn * dn, 0.0));
    std::vector<int> slot_age;
    // a molecule that meets the criteria keeps that density (and its results)
    // while the others iterate on
    std::vector<char> conv(nmol, 0);
    std::vector<double> e_fin(nmol, 0.0), err_fin(nmol, 0.0), de_fin(nmol, 0.0);
    std::vector<int> it_fin(nmol, 0);
    double jk_s = 0;
    bool all_conv = false;
    // progress lines on stderr when FK_SCF_LOG is set (long batches)
    const char *lg = std::getenv("FK_SCF_LOG");
    const bool log = lg && *lg && *lg != '0';
    int it = 0;
    for (; it < o.max_iter; ++it) {
        const auto t0 = std::chrono::steady_clock::now();
        if ((rc = fk_build_jk(c, w.D.p, w.J.p, w.K.p, FK_DEVICE_PTRS | FK_SYNC, w.st))) return rc;
        jk_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if ((rc = w.lincomb_u(w.F.p, w.h.p, w.J.p, w.K.p, 1.0, 1.0, -0.5, 0)) || (rc = w.reduce(w.D.p, w.h.p, 0, dh)) ||
            (rc = w.reduce(w.D.p, w.F.p, 0, df)))
            return rc;
        for (int m = 0; m < nmol; ++m) {
            e_prev[m] = e_cur[m];
            e_cur[m] = 0.5 * (dh[m] + df[m]) + enuc[m];
        }
        if ((rc = w.gemm(w.X.p, w.F.p, w.T3.p)) || (rc = w.gemm(w.T3.p, w.X.p, w.Fo.p)) || (rc = scfb_shift_null(w)) ||
            (rc = w.gemm(w.Fo.p, w.Do.p, w.G.p)))
            return rc;
        if (fk_scfb_antisym(w.E.p, w.G.p, nmol, nmax, w.nbf(), w.off(), w.st)) return fail(c, FK_ERR_HIP, "batched SCF: launch failed");
        if ((rc = w.reduce(w.E.p, nullptr, 1, err))) return rc;
        all_conv = true;
        int nconv = 0;
        double de_max = 0, err_max = 0;
        for (int m = 0; m < nmol; ++m) {
            if (conv[m]) {  // frozen at its converged density
                ++nconv;
                continue;
            }
            if (!std::isfinite(e_cur[m]) || !std::isfinite(err[m]))
                return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf_batch: molecule %d: non-finite energy or error at iteration %d", m, it + 1);
            conv[m] = it > 0 && std::fabs(e_cur[m] - e_prev[m]) < o.e_tol && err[m] < o.g_tol;
            if (conv[m]) {
                ++nconv;
                e_fin[m] = e_cur[m];
                err_fin[m] = err[m];
                de_fin[m] = e_cur[m] - e_prev[m];
                it_fin[m] = it + 1;
            }
            all_conv = all_conv && conv[m];
            de_max = std::max(de_max, std::fabs(e_cur[m] - e_prev[m]));
            err_max = std::max(err_max, err[m]);
        }
        if (log)
            std::fprintf(stderr, "fk_run_scf_batch: iteration %d: %d of %d converged, max |dE| %.3e, max error %.3e, %.1f s\n",
                         it + 1, nconv, nmol, de_max, err_max,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
        if (all_conv) {
            ++it;
            break;
        }
        if (o.diis_n > 1) {
            int k;
            if ((int)slot_age.size() < o.diis_n) {
                k = (int)slot_age.size();
            } else {
                k = slot_age.front();
                slot_age.erase(slot_age.begin());
            }
            slot_age.push_back(k);
            HIPCHK(c, hipMemcpyAsync(w.ringF[k].p, w.Fo.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, w.st));
            HIPCHK(c, hipMemcpyAsync(w.ringE[k].p, w.E.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, w.st));
            for (int j : slot_age) {
                if ((rc = w.reduce(w.ringE[k].p, w.ringE[j].p, 0, ev))) return rc;
                for (int m = 0; m < nmol; ++m) Bm[m][(size_t)k * dn + j] = Bm[m][(size_t)j * dn + k] = ev[m];
            }
            const int ms = (int)slot_age.size();
            if (ms >= 2) {
                // per molecule the Pulay coefficients (the newest F' alone if singular)
                std::vector<std::vector<double>> coefs(nmol);
                for (int m = 0; m < nmol; ++m) {
                    std::vector<double> B((size_t)ms * ms);
                    for (int i = 0; i < ms; ++i)
                        for (int j = 0; j < ms; ++j) B[(size_t)i * ms + j] = Bm[m][(size_t)slot_age[i] * dn + slot_age[j]];
                    if (!diis_solve(B, ms, coefs[m])) {
                        coefs[m].assign(ms, 0.0);
                        coefs[m][ms - 1] = 1.0;
                    }
                }
                std::vector<double> cf(4 * (size_t)nmol, 0.0);
                for (int m = 0; m < nmol; ++m) cf[4 * m] = coefs[m][0];
                if ((rc = w.lincomb(w.Fo.p, w.ringF[slot_age[0]].p, nullptr, nullptr, cf))) return rc;
                for (int i = 1; i < ms; ++i) {
                    for (int m = 0; m < nmol; ++m) { cf[4 * m] = 1.0; cf[4 * m + 1] = coefs[m][i]; }
                    if ((rc = w.lincomb(w.Fo.p, w.Fo.p, w.ringF[slot_age[i]].p, nullptr, cf))) return rc;
                }
            }
        }
        // new densities; frozen molecules keep theirs (D' and D: keep = 1)
        HIPCHK(c, hipMemcpyAsync(w.G.p, w.Do.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, w.st));
        HIPCHK(c, hipMemcpyAsync(w.E.p, w.D.p, nmat * sizeof(double), hipMemcpyDeviceToDevice, w.st));
        if ((rc = o.density_eig ? scfb_density_eig(w, nocc) : scfb_purify(w, nocc))) return rc;
        if ((rc = w.gemm(w.X.p, w.Do.p, w.T3.p)) || (rc = w.gemm(w.T3.p, w.X.p, w.D.p))) return rc;
        if (std::find(conv.begin(), conv.end(), 1) != conv.end()) {
            std::vector<double> cf(4 * (size_t)nmol, 0.0);
            for (int m = 0; m < nmol; ++m) {
                cf[4 * m] = conv[m] ? 0.0 : 1.0;
                cf[4 * m + 1] = conv[m] ? 1.0 : 0.0;
            }
            if ((rc = w.lincomb(w.Do.p, w.Do.p, w.G.p, nullptr, cf)) || (rc = w.lincomb(w.D.p, w.D.p, w.E.p, nullptr, cf)))
                return rc;
        }
    }
    HIPCHK(c, hipMemcpy(D_inout, w.D.p, nmat * sizeof(double), hipMemcpyDeviceToHost));
    const double tot = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int m = 0; m < nmol; ++m) {
        fk_scf_result &r = results[m];
        r.energy = conv[m] ? e_fin[m] : e_cur[m];
        r.iterations = conv[m] ? it_fin[m] : it;
        r.converged = conv[m] ? 1 : 0;
        r.error = conv[m] ? err_fin[m] : err[m];
        r.delta_e = conv[m] ? de_fin[m] : e_cur[m] - e_prev[m];
        r.jk_seconds = jk_s;
        r.total_seconds = tot;
        r.ndropped = w.ndrop.empty() ? 0 : w.ndrop[m];
    }
    if (!all_conv) return fail(c, FK_ERR_NOT_CONVERGED, "fk_run_scf_batch: not every molecule converged in %d iterations", o.max_iter);
    return FK_OK;
}
