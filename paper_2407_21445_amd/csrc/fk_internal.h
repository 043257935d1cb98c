// Structures shared by the host library and the kernels (not part of the ABI).
#pragma once

#include <stdint.h>

#define FK_NPP_REC 10  // doubles per primitive-pair record

// Primitive-pair record layout (FK_NPP_REC doubles):
//   0 zeta, 1 1/(2 zeta), 2-4 P, 5-7 P - A, 8 K (see fk::PrimPair), 9 G_[ab].

#define FK_NFLD 9  // fields of a transposed primitive-pair record (no G)

// Work tile: a block of bra shell pairs that share their first shell, and up to
// 64 consecutive ket shell pairs of one ket class, all from one
// primitive-count group.  Every (bra, ket) combination of the tile is a
// candidate quartet; the kernels apply the Schwarz, same-class and density
// tests per combination.
struct FkTile {
    int blk;        // bra block (index into FkJKArgs::blocks)
    int ket_begin;  // position in the concatenated sorted pair lists
    int ket_count;  // 1..64
    int grp;        // primitive-count group of the kets; bit 30: bra and ket from the same class
};
#define FK_TILE_SAME (1 << 30)

// Matrices a build forms (FkJKArgs::want).
#define FK_WANT_J 1
#define FK_WANT_K 2

// Bra block: blk_bra[first .. first + count) are shell-pair indices with the
// same first shell; blk_pos holds their positions in the sorted pair lists.
struct FkBraBlock {
    int first;
    int count;
};
#define FK_MAX_BRA_BLOCK 32

// A run of equal primitive-pair count inside one class's sorted pair list.
// Its primitive records are stored transposed, [j][field][position in run],
// so that lanes holding consecutive kets read consecutive addresses.
struct FkGroup {
    int begin;      // first list position
    int len;        // number of pairs
    int npp;        // primitive pairs per pair
    int mol;        // molecule of the run's pairs (0 unless the context holds a batch)
    long long base; // offset of the run's records in the transposed array
};

// Declaration of a kernel's dynamically sized LDS block (as doubles).
#ifndef FK_DYN_LDS
#define FK_DYN_LDS(name) extern __shared__ double name[]
#endif

struct FkJKArgs {
    // Shells are numbered within their molecule: a kernel offsets these arrays
    // by the tile's molecule (FkGroup::mol).
    const int *sh_bf;        // [nshell] first basis function of each shell, within its molecule
    const int *mol_sh0;      // [nmol] first shell of each molecule
    const int *mol_nbf;      // [nmol] functions per molecule
    const int *mol_nsh;      // [nmol] shells per molecule
    const long long *mol_base;    // [nmol + 1] offset of each molecule's nbf^2 block in Ds, XJ, XK
    const long long *mol_shbase;  // [nmol + 1] offset of each molecule's nshell^2 block in Dsh
    const int *pair_sa;      // [npair] first shell (higher l), index within the molecule
    const int *pair_sb;      // [npair] second shell, index within the molecule
    const int *pair_ppoff;   // [npair] first primitive pair
    const int *pair_npp;     // [npair] number of primitive pairs
    const double *pair_AB;   // [npair * 3] A - B
    const double *pair_G;    // [npair] Schwarz factor
    const double *pp;        // [nprimpair * FK_NPP_REC]
    const int *ket_list;     // sorted pair indices (all classes, concatenated)
    const int *lst_sa, *lst_sb;   // shells (within the molecule) of the pair at each list position
    const double *lst_CD;    // [3][nlist] A - B of the pair at each list position
    const double *lst_G;     // Schwarz factor at each list position
    int nlist;
    const FkGroup *groups;
    const double *ppT;       // transposed primitive records of every group
    const FkTile *tiles;
    int ntiles;
    const FkBraBlock *blocks;
    const int *blk_bra;      // shell-pair index of each bra of each block
    const int *blk_pos;      // its position in the sorted pair lists
    const double *Dsh;       // per molecule [nshell_m * nshell_m] max |D| per shell block
    const double *Ds;        // per molecule [nbf_m * nbf_m] component-scaled density
    double *XJ;              // per molecule [nbf_m * nbf_m] unsymmetrised Coulomb accumulator
    double *XK;              // per molecule [nbf_m * nbf_m] unsymmetrised exchange accumulator
    long long xcopy;         // distance between the FK_XCD_COPIES copies of (XJ, XK)
    int dscreen;             // apply the density screen
    int want;                // FK_WANT_J | FK_WANT_K: the matrices this build forms
    double tau;
    const double *rys_tab;   // staged Rys segment (table + Gauss-Hermite) of this class's root count
    unsigned long long *counters;  // [2]: contracted quartets, primitive quartets
    int bra_slot;            // doubles per wave for the staged bra primitive records
    int prec;                // 0: FP64 kernel, 1: FP32 kernel of the precision split
    int engine;              // 0: Rys quadrature, 1: HGP with early contraction
    int kind;                // kernel kind of the launch: the class's own, or 1 for a lane class's team alternative
    int nw;                  // waves per workgroup of the launch (4; 8 for the wide lane kernels)
    double tau_fp32;         // precision split (0: none): per bra and tile, the FP32
                             // launch takes the work when G_ab G_cd D_max < tau_fp32
    // K-block skip (K launches beside the J engine; null: off): per shell
    // x, y, z, R_x, G_x, and the fitted density bound |D| <= H exp(-Lambda r)
    // in ks_fit[0..1]; block K_xy is insignificant when
    // H exp(-Lambda max(0, |XY| - R_x - R_y)) G_x G_y <= ks_tau
    const double *ks_shell;
    const double *ks_fit;
    double ks_tau;
    // Block tasks of the ket-outer lane classes (ntask 0: each wave takes tiles
    // on its own).  A workgroup takes task i = tasks[i] = (first tile, tile
    // count), tiles of one bra block (a, b_j); its waves share those tiles and
    // sum X_K[b_j, x], X_K[a, x] and X_J[a, b_j] of the block in LDS, which
    // reaches memory once per task.  The columns x are the functions of the
    // ket shells' types, numbered per molecule: krow_col[shell] is a shell's
    // first column among the shells of its type, krow_cnt[4 mol + l] the
    // columns of type l, and krow_fn[krow_off[4 mol + l] + x] the function of
    // column x.  The ket's c columns come first, then (types differing) d's.
    const int2 *tasks;
    int ntask;
    int krow_ncol;           // LDS row length: the class's largest column count over the molecules
    int krow_nbk;            // bras per block the rows are laid out for (the class's bra block)
    const int *krow_col, *krow_cnt, *krow_off, *krow_fn;
};

// The accumulators X_J, X_K exist once per XCD (CDNA3/4 parts have 8 XCDs,
// each with its own L2; workgroups are dispatched to them round-robin).  A
// workgroup adds into copy blockIdx.x mod FK_XCD_COPIES, so the atomics of one
// XCD stay on lines its L2 owns; the finalize kernel sums the copies.  Any
// assignment is correct, the round-robin one keeps the traffic local.
#define FK_XCD_COPIES 8

// Molecule layout for the density preprocessing and finalize kernels.
struct FkMolArgs {
    const int *sh_lbf, *sh_lend;  // [nshell] first and end function of each shell within its molecule
    const int *mol_sh0, *mol_nsh, *mol_nbf, *mol_bf0;  // [nmol]; mol_bf0: first function in the flat numbering
    const long long *mol_base, *mol_shbase;           // [nmol + 1]
    int nmol;
    long long nmat, nshmat;       // total elements of the nbf^2 and nshell^2 blocks
};

// Quartet list for the debug/Schwarz kernels (canonical orientation).
struct FkDebugArgs {
    const int *pair_ppoff, *pair_npp;
    const double *pair_AB;
    const double *pp;
    const int2 *quartets;    // (bra pair, ket pair)
    int nq;
    double *out;             // [nq * NOUT]
    const double *rys_tab;
    int engine;              // 0: Rys quadrature, 1: HGP
};

// Per-class launch entry points (defined in fk_kernels.hip).
struct FkClassInfo {
    int la, lb, lc, ld, nroot, nout;
    int wave_per_quartet;    // kernel kind: 0 lane, 1 team over a, 2 team over (a,b), 3 wave per quartet
    int team_size;           // lanes per quartet
    int bra_block;           // largest bra block the class kernel takes per tile
    double flops_prim, flops_quartet;
    int ket_outer;           // bra block of the ket-outer loop order (0: bra-outer)
    int alt_team;            // lane classes with a team-per-quartet alternative: its lanes per quartet (else 0)
    int alt_bra_block;       // and the largest bra block of that kernel
    int wide;                // waves per workgroup of a wider build of the lane kernel (0: none)
    int hgp;                 // 1: the HGP engine is built for the class
    double flops_prim_hgp, flops_quartet_hgp;
};
// HGP kernels are built for lane-per-quartet classes up to this total momentum
#define FK_HGP_MAX_L 4

extern "C" {
int fk_kernels_class_info(int P, int Q, FkClassInfo *info);
int fk_kernels_launch_jk(int P, int Q, const FkJKArgs *args, int grid, void *stream);
int fk_kernels_launch_debug(int P, int Q, const FkDebugArgs *args, void *stream);
int fk_kernels_max_blocks(int P, int Q, int dyn_lds_bytes, int engine, int kind, int nw, int *blocks_per_cu);
// dynamic LDS of a class launch; krow_ncol > 0 adds the block-task K rows
int fk_kernels_jk_lds_bytes(int P, int Q, int bra_slot, int krow_ncol, int kind, int nbk, int nw);
int fk_kernels_launch_prep(const double *D, const double *bf_scale, const FkMolArgs *m, double *Ds, double *Dsh,
                           void *stream);
int fk_kernels_launch_finalize(const double *XJ, const double *XK, long long xcopy, int ncopy, const double *bf_scale,
                               const FkMolArgs *m, double *J, double *K, void *stream);
int fk_kernels_launch_fill(double *p, long long n, void *stream);
int fk_kernels_debug_host(int P, int Q, const int *pair_ppoff, const int *pair_npp, const double *pair_AB,
                          const double *pp, const int *quartets, int nq, double *out, int engine);
// ---- J engine (McMurchie-Davidson; paper, "J matrix implementation") ----
// Work tile of the J_p kernel: one bra pair against up to 64 kets of one
// primitive-count group (consecutive list positions).
struct FkJengTile {
    int bra, ket_begin, ket_count, grp;
};
// Hermite-contracted ket density D_q and the J_p accumulation.
struct FkJengArgs {
    const int *pair_ppoff, *pair_npp;
    const double *pair_G, *pp;
    const long long *jp_off;  // per pair: first element of its J_p block [npp][nherm(la+lb)]
    double *jp;
    const double *ppT;        // transposed ket primitive records (see FkGroup)
    const FkGroup *groups;
    const double *lst_G;
    const int *lst_sa, *lst_sb;
    const long long *dq_base; // per group: first element of its D_q block [npp][nherm(lc+ld)][len]
    const double *dq;
    const double *Dsh;
    int ns, dscreen;
    double tau;
    const FkJengTile *tiles;
    long long ntiles;
    const double *rys_tab;
};
struct FkJengDqArgs {
    const FkGroup *groups;
    const int *pos_grp;       // group of each list position
    int pos0, npos;           // the list positions of one ket class
    const int *lst_sa, *lst_sb;
    const double *lst_CD;
    int nlist;
    const double *ppT;
    const int *sh_bf;
    const double *Ds;
    int n;
    const long long *dq_base;
    double *dq;
};
struct FkJengJabArgs {
    const int *pairs;         // pair indices of one bra class
    int npairs;
    const int *pair_sa, *pair_sb, *pair_ppoff, *pair_npp;
    const double *pair_AB, *pp;
    const long long *jp_off;
    const double *jp;
    const int *sh_bf;
    double *XJ;
    int n;
};
// the J engine is built for total pair momenta up to this (s, p, d shells)
#define FK_JENG_MAX_LP 4
// density-decay fit (paper, "K matrix implementation", eq. density_bound):
// bins of the centre distance for the binned maxima of |D|
#define FK_DFIT_BINS 64
int fk_kernels_launch_dfit(const double *D, int n, const int *bf_atom, const double *atom_xyz, double dr,
                           unsigned long long *bins, double *fit, void *stream);

// dense SCF kernels (fk_scf.hip); n x n row-major FP64 device matrices
int fk_jeng_launch_dq(int lc, int ld, const FkJengDqArgs *a, void *stream);
int fk_jeng_launch_jp(int LP, int LQ, const FkJengArgs *a, int grid, void *stream);
int fk_jeng_launch_jab(int la, int lb, const FkJengJabArgs *a, void *stream);
int fk_scf_gemm(const double *A, const double *B, double *C, int n, double alpha, double beta, void *stream);
int fk_scf_lincomb(double *out, const double *x, const double *y, const double *z, int n, double a, double b,
                   double c, double d, void *stream);
int fk_scf_antisym(double *e, const double *G, int n, void *stream);
int fk_scf_reduce(const double *x, const double *y, int n, int op, double *part, double *out, int slot,
                  void *stream);
int fk_scf_reduce_scratch();
int fk_scf_eig_scale(const double *V, const double *s, double *out, int n, double cutoff, double power, void *stream);
int fk_scf_eigh(double *A, double *w, double *work, int *info, int n, void *stream);
}
