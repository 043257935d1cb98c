/*
 * fockjk -- Coulomb (J) and exchange (K) matrices of direct Hartree-Fock on
 * one AMD Instinct MI355X (gfx950).
 *
 * The library evaluates J_uv = sum_ls (uv|ls) D_ls and K_uv = sum_ls (ul|vs) D_ls
 * (paper, "Hartree-Fock Energy Formulation", eqs. for J and K) from the
 * electron repulsion integrals of contracted Cartesian Gaussian shells
 * (paper, "Notation", eqs. cgf and prim) up to f, screened by the Cauchy-
 * Schwarz bounds G_ab G_cd (eq. cauchy-schwarz) and by the density block
 * maximum D_max of the six density blocks of each quartet (paper, section
 * "Optimised GPU Implementation" of the Brc21 scheme), and exploiting the
 * 8-fold permutational symmetry of the integrals (paper, "Algorithmic
 * Challenges").  Integrals are evaluated by Rys quadrature.
 *
 * Conventions
 *   - Units: bohr and hartree.  D includes the factor 2 (D = 2 C_occ C_occ^T).
 *   - Matrices are nbf x nbf, row-major, full (both triangles), FP64.
 *   - Basis functions follow the shell order given to fk_set_basis; inside a
 *     shell the Cartesian components are ordered x^l, x^(l-1)y, x^(l-1)z,
 *     x^(l-2)y^2, ... z^l (descending x power, then descending y power).
 *     Every component is normalised to unit self-overlap.
 *   - Contraction coefficients multiply primitives normalised as the
 *     axis-aligned component: N(a,l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!).
 *
 * Ownership and threading
 *   - The caller owns every array it passes.  Host inputs are copied during
 *     the call.  Device pointers are borrowed for the duration of the call and
 *     used on the HIP stream passed in (NULL = the null stream); the call
 *     returns after enqueueing unless stated otherwise.
 *   - The library owns its device buffers (allocated with hipMalloc on the
 *     context's device when the basis or screening changes).
 *   - A context is used from one host thread at a time; separate contexts are
 *     independent.
 *
 * Errors
 *   Every function returns an fk_status (0 = success).  Arguments are fully
 *   validated on the host before any device work; nothing throws across the
 *   ABI.  fk_last_error returns a message describing the last failure of the
 *   context (valid until the next call on it); fk_last_error(NULL) describes
 *   the last failed fk_create on the calling thread.
 */
#ifndef FOCKJK_H
#define FOCKJK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fk_ctx fk_ctx;

typedef enum {
    FK_OK = 0,
    FK_ERR_ARG = -1,          /* invalid argument (checked on the host) */
    FK_ERR_UNSUPPORTED = -2,  /* l > FK_MAX_L, contraction depth > FK_MAX_K, ... */
    FK_ERR_HIP = -3,          /* a HIP runtime call failed */
    FK_ERR_OOM = -4,          /* device allocation failed */
    FK_ERR_NOT_CONVERGED = -5,/* SCF reached max_iter */
    FK_ERR_STATE = -6         /* call out of order (e.g. build_jk before build_quartets) */
} fk_status;

#define FK_MAX_L 3            /* s, p, d, f */
#define FK_MAX_K 9            /* primitives per contracted shell */

/* flags for fk_build_jk */
#define FK_DEVICE_PTRS 1u     /* D, J, K are device pointers (else host pointers) */
#define FK_SYNC 2u            /* synchronise the stream before returning */
#define FK_TIME_CLASSES 4u    /* record HIP events around each class kernel (read by fk_stats) */
#define FK_J_ONLY 8u          /* form J only (paper, "Hartree-Fock Energy Formulation": J_uv =
                                 sum_ls (uv|ls) D_ls); K is not written and may be NULL.  The
                                 density screen then uses D_ab and D_cd only */
#define FK_K_ONLY 16u         /* form K only (K_uv = sum_ls (ul|vs) D_ls); J is not written and
                                 may be NULL; the density screen uses D_ac, D_ad, D_bc, D_bd.
                                 FK_J_ONLY | FK_K_ONLY is FK_ERR_ARG */
#define FK_J_ENGINE 32u       /* J by the McMurchie-Davidson J engine (paper, "J matrix
                                 implementation": J_ab = sum_p E^ab_p J_p, J_p = sum_q [p|q] D_q,
                                 D_q = sum_cd E^cd_q D_cd, per primitive pair); K, unless
                                 FK_J_ONLY, by the Rys kernels with the K-only density screen.
                                 Every bra takes all its Schwarz- and density-screened kets (no
                                 bra-ket symmetry).  One molecule with s, p and d shells
                                 (FK_ERR_UNSUPPORTED otherwise); its lists are built at the first
                                 such build after fk_build_quartets */

/* Screening options (paper: Cauchy-Schwarz screening, eq. cauchy-schwarz, and
 * the density screen G_ab G_cd D_max < tau of the Brc21 scheme). */
typedef struct {
    double tau;        /* quartet threshold; 0 disables screening (every quartet) */
    double tau_prim;   /* primitive-pair pruning: drop primitive pairs whose
                          bound G_[ab] * max_all G_[cd] < tau_prim; 0 = keep all */
    int    density_screen; /* 1: apply the per-quartet D_max screen in fk_build_jk */
    int    bra_block;  /* bras sharing their first shell that one work tile
                          pairs with the same kets (1..32; 0 = default 8).
                          Contributions to K[a, c], K[a, d] and J[c, d] are
                          summed over the block before they reach memory */
    double tau_fp32;   /* precision split (an extension: the paper runs FP64 only):
                          each class gets a second, FP32 launch over the same work
                          tiles; per bra and tile, the quartets of a wave run their
                          recurrences in FP32 when every one has G_ab G_cd D_max <
                          tau_fp32 (D_max of the build's density, as in the density
                          screen), in FP64 otherwise.  Set-up, roots, weights,
                          digestion and all accumulation stay FP64; f-f bras stay
                          FP64.  0 = FP64 only */
    double tau_k;      /* K-block threshold of the K launches in a build with
                          FK_J_ENGINE (paper, "K matrix implementation": blocks
                          K_xy whose fitted density bound stays below tau_k are
                          skipped, see fk_density_bound; the paper uses 5e-6).
                          0 = no block skip */
    int    block_tasks; /* lane classes: 0 = a workgroup takes all ket tiles of
                          one bra block (a, b_1..b_m) at a time and sums
                          X_K[b_j, x], X_K[a, x] and X_J[a, b_j] in LDS, which
                          reaches memory once per block instead of once per tile
                          and bra.  Used where the rows fit without costing
                          waves per CU: the ket-outer classes ((ss|ss), (ps|ss))
                          with four-wave workgroups, and, where the schedule
                          asks for them (fk_set_class_block_tasks, the
                          autotuner), the bra-outer (ps|ps), (pp|ss), (pp|ps),
                          (ds|ss), (ds|ps), (dp|ss), (dp|ps) with eight-wave
                          workgroups, the bra block lowered until the rows fit
                          (fk_stats reports both);
                          -1 = every wave takes tiles on its own */
} fk_screen_opts;

typedef struct {
    int    nbf, nshell, natom, nelec;
    int    npair;            /* unique shell pairs (a >= b) */
    int    npair_kept;       /* pairs with G_ab * G_max >= tau */
    int    nclass_pair;      /* angular-momentum pair classes present */
    int    nquartet_class;   /* quartet classes with work */
    int64_t nprim_pair;      /* primitive pairs kept */
    int64_t nquartet_schwarz;/* unique shell quartets surviving the Schwarz screen */
    int64_t ntile;           /* work tiles (bra pair x up to 64 ket pairs) */
    double  flops_schwarz;   /* algorithmic FP64 flops of one build if no quartet
                                were removed by the density screen */
    int     nmol;            /* molecules in the context (1 unless fk_set_molecules) */
    int     reserved;
    int64_t nmat;            /* elements of D, J, K: sum over molecules of nbf_m^2 */
} fk_info_t;

/* Per-build statistics of the last fk_build_jk (filled by fk_stats).  On a
 * context without a device, or before the first build, only the host-side
 * fields (class, tiles, prim_slots, flops per unit) are filled. */
#define FK_MAX_QCLASS 110  /* 55 classes, each with an FP64 and an FP32 launch */
typedef struct {
    int     nclass;                       /* quartet classes launched */
    int     la[FK_MAX_QCLASS], lb[FK_MAX_QCLASS], lc[FK_MAX_QCLASS], ld[FK_MAX_QCLASS];
    int64_t quartets[FK_MAX_QCLASS];      /* contracted quartets computed */
    int64_t prim_quartets[FK_MAX_QCLASS]; /* primitive quartets computed */
    double  flops_per_prim[FK_MAX_QCLASS];/* algorithmic flops per primitive quartet */
    double  flops_per_quartet[FK_MAX_QCLASS]; /* per contracted quartet (digestion) */
    double  flops_total;                  /* algorithmic flops of the build */
    double  class_ms[FK_MAX_QCLASS];      /* kernel time per class (FK_TIME_CLASSES builds), else 0 */
    int64_t tiles[FK_MAX_QCLASS];         /* work tiles of the class */
    int     team_size[FK_MAX_QCLASS];     /* lanes computing one quartet (1, a team, or 64) */
    int     precision[FK_MAX_QCLASS];     /* 64: FP64 launch, 32: FP32 launch of the split */
    int64_t prim_slots[FK_MAX_QCLASS];    /* lane x primitive-quartet slots the waves step
                                             through if no quartet fails the density screen:
                                             per tile, rounds x 64 lanes x bra x ket primitive
                                             pairs.  prim_quartets * team_size / prim_slots is
                                             the lane utilisation of the primitive loops */
    int     engine[FK_MAX_QCLASS];        /* FK_ENGINE_RYS or FK_ENGINE_HGP */
    int     bra_block[FK_MAX_QCLASS];     /* the schedule in effect (fk_set_class_schedule) */
    int     kets_per_tile[FK_MAX_QCLASS];
    double  grid_fraction[FK_MAX_QCLASS];
    int64_t block_tasks[FK_MAX_QCLASS];   /* workgroup tasks of the class (fk_screen_opts
                                             .block_tasks), 0 if its waves take tiles */
    int     waves_per_group[FK_MAX_QCLASS]; /* waves per workgroup of the launch (4, or 8 for
                                             the bra-outer lane classes with block tasks) */
} fk_stats_t;

/* ---- context ---------------------------------------------------------- */
/* Create a context on HIP device `device`. */
int fk_create(fk_ctx **out, int device);
void fk_destroy(fk_ctx *ctx);
const char *fk_last_error(const fk_ctx *ctx);

/* ---- inputs (paper: "Notation") -------------------------------------- */
/* natom atoms with nuclear charges Z[natom] at xyz[natom*3] (bohr); the
 * molecule carries `charge` (electrons = sum Z - charge, must be even). */
int fk_set_geometry(fk_ctx *ctx, int natom, const int *Z, const double *xyz, int charge);

/* nshell contracted shells; shell s sits on atom shell_atom[s], has angular
 * momentum shell_l[s] (0..FK_MAX_L) and shell_nprim[s] (1..FK_MAX_K)
 * primitives whose exponents (> 0) and contraction coefficients are stored
 * consecutively in exps[] and coefs[] (sum of shell_nprim entries).
 * Requires fk_set_geometry first.  Invalidates quartet lists. */
int fk_set_basis(fk_ctx *ctx, int nshell, const int *shell_atom, const int *shell_l,
                 const int *shell_nprim, const double *exps, const double *coefs);

/* Batch of independent molecules in one context: atom a belongs to molecule
 * atom_mol[a] (0..nmol-1, non-decreasing over the atoms, so that each
 * molecule's atoms, shells and functions are contiguous).  Call after
 * fk_set_geometry (before or after fk_set_basis; it invalidates the quartet
 * lists).  Shell pairs and quartets never span two molecules; one
 * fk_build_jk then runs every molecule's quartets in the same class launches.
 * D, J and K become the concatenation of the molecules' nbf_m x nbf_m
 * row-major blocks (fk_molecule_layout gives the sizes and offsets).
 * fk_one_electron, fk_run_scf and fk_debug_eri return FK_ERR_UNSUPPORTED
 * for a batch (one context per molecule for those). */
int fk_set_molecules(fk_ctx *ctx, int nmol, const int *atom_mol);

/* nbf[m] and offset[m] (m = 0..nmol; offset[nmol] = total elements) of each
 * molecule's block of D, J, K.  Arrays of nmol and nmol + 1 entries. */
int fk_molecule_layout(const fk_ctx *ctx, int *nbf, int64_t *offset);

/* ---- screening and work lists (paper: Cauchy-Schwarz bounds; shell-pair
 * batching and upper-triangle class launches of the Brc21 scheme) -------- */
/* Builds shell pairs and primitive pairs, the Schwarz factors
 * G_ab = max sqrt((ab|ab)) (computed on the device), sorts pairs by class and
 * bound, and builds the work tiles.  opts == NULL means tau = 1e-10,
 * tau_prim = 0, density_screen = 1.  Synchronous. */
int fk_build_quartets(fk_ctx *ctx, const fk_screen_opts *opts);
int fk_info(const fk_ctx *ctx, fk_info_t *info);

/* ---- the hot path (paper: eq. fock_build; J and K) --------------------- */
/* J and K for the density D (all nbf x nbf, row-major, symmetric D).
 * flags: FK_DEVICE_PTRS (D, J, K in device memory, used on `stream`);
 * otherwise host arrays, copied in and out synchronously.  FK_SYNC waits for
 * completion.  FK_J_ONLY or FK_K_ONLY form one of the two matrices (the
 * other pointer may be NULL and is not written); a quartet is then skipped
 * when G_ab G_cd times the largest |D| over only the blocks that matrix
 * multiplies falls below tau.  Asymmetric D gives J, K of its symmetric part only when
 * density screening is off; callers pass symmetric D.  The call is ordered on
 * `stream`: the class kernels may run on two more streams (the library's,
 * one pair per device, shared by its contexts), which wait for `stream`
 * before the first of them and which `stream` waits for before the final
 * reduction (not while `stream` is being captured into a
 * graph, and not with FK_TIME_CLASSES: then every launch is on `stream`). */
int fk_build_jk(fk_ctx *ctx, const double *D, double *J, double *K, unsigned flags, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the build of
 * fk_build_jk that allocates nothing.  Its working buffers (scaled density,
 * shell-block maxima, one copy of the Coulomb and exchange accumulators,
 * counters) live in a fixed device array that each GPU the library runs on
 * holds for the life of the process: 3 FK_NOALLOC_MAX_NMAT + FK_NOALLOC_MAX_NSHMAT
 * + 2 FK_MAX_QCLASS doubles (about 52 MB).  Limits: the context's matrices
 * hold at most FK_NOALLOC_MAX_NMAT elements in all (one molecule: nbf <= 1448)
 * and its shell blocks at most FK_NOALLOC_MAX_NSHMAT (nshell <= 512); larger
 * contexts get FK_ERR_ARG (use fk_build_jk).  flags must contain
 * FK_DEVICE_PTRS (D, J, K device arrays of the caller) and may contain
 * FK_SYNC, FK_J_ONLY or FK_K_ONLY; FK_TIME_CLASSES and FK_J_ENGINE (whose
 * lists the context allocates) are FK_ERR_ARG.  The array
 * is shared by every context on a GPU and keeps the last call's contents (the
 * call clears what must start at zero): calls that overlap on one GPU, on any
 * streams, race and must be ordered by the caller.  Every launch is on
 * `stream` (the library's class-launch streams of fk_build_jk are not used).
 * Results equal fk_build_jk's up to the order of the accumulation; fk_stats
 * reports this call when it was the last build. */
#define FK_NOALLOC_MAX_NMAT (1 << 21)
#define FK_NOALLOC_MAX_NSHMAT (1 << 18)
int fk_build_jk_noalloc(fk_ctx *ctx, const double *D, double *J, double *K, unsigned flags, void *stream);

/* Density-decay bound (paper, "K matrix implementation", eq. density_bound):
 * H and Lambda with |D_uv| <= H exp(-Lambda r_uv) for every element whose
 * functions sit on different atoms r_uv apart: a least-squares line through
 * the logarithms of the largest |D| in 64 distance bins (same-atom elements
 * excluded), raised until it lies on or above every bin's maximum at the bin's
 * far edge (the printed fit alone is not a bound); Lambda >= 0.  D as in
 * fk_build_jk (FK_DEVICE_PTRS for a device pointer).  One molecule.  The K
 * launches of an FK_J_ENGINE build with fk_screen_opts.tau_k > 0 compute it
 * on the device for their density and skip every K block xy with
 * H exp(-Lambda max(0, |XY| - R_x - R_y)) G_x G_y <= tau_k (R_x: the largest
 * distance from shell x to the partner of a pair with G >= tau; G_x: its
 * largest pair factor); the quartets' other K blocks still count. */
int fk_density_bound(fk_ctx *ctx, const double *D, unsigned flags, double *H, double *Lambda);

/* Statistics of the last fk_build_jk (waits for it to finish). */
int fk_stats(fk_ctx *ctx, fk_stats_t *stats);

/* Progress of the last fk_build_jk issued with FK_TIME_CLASSES (and without
 * FK_SYNC): *done of *total class launches have finished on the device.
 * Does not block.  FK_ERR_STATE if the last build was not timed. */
int fk_build_progress(fk_ctx *ctx, int *done, int *total);

/* ---- kernel schedules ---------------------------------------------------
 * Per quartet class (named by its momenta as fk_stats lists them), the
 * schedule of its J/K kernel: bra_block = bras sharing their first shell per
 * work tile (0 = fk_screen_opts.bra_block; capped by the class kernel),
 * kets_per_tile = 1..64 kets per tile for the team and wave-per-quartet
 * kernels (0 = two rounds; lane-per-quartet kernels always take 64),
 * grid_fraction = size (0, 4] of the launched grid relative to the
 * resident-workgroup grid (the persistent loop covers every tile either way;
 * above 1 the later workgroups start as the first ones finish).  A schedule
 * changes the work order only, never the result beyond rounding order.
 * Takes effect at the next fk_build_quartets; fk_set_geometry, fk_set_basis
 * and fk_set_molecules clear all schedules. */
int fk_set_class_schedule(fk_ctx *ctx, int la, int lb, int lc, int ld, int bra_block, int kets_per_tile,
                          double grid_fraction);

/* Integral engine of a quartet class (a per-class schedule choice like the
 * ones above, with the same lifetime).  FK_ENGINE_RYS: Rys quadrature over
 * the 2D integrals, built for every class.  FK_ENGINE_HGP: the Obara-Saika
 * vertical recurrences per primitive quartet, contracted, then the
 * horizontal recurrences on the contracted integrals (paper: "HGP Recursive
 * Scheme", the vrr and hrr equations; the early contraction its "Optimised
 * GPU Implementation" builds on), with the Boys function values F_m(T) taken
 * as moments of the same Rys rule; built for the
 * lane-per-quartet classes up to L = la+lb+lc+ld = 4 (fk_stats reports the
 * choice per launch; FK_ERR_UNSUPPORTED for other classes).  Both engines
 * give the same integrals up to rounding. */
#define FK_ENGINE_RYS 0
#define FK_ENGINE_HGP 1
int fk_set_class_engine(fk_ctx *ctx, int la, int lb, int lc, int ld, int engine);

/* Block tasks per class (see fk_screen_opts.block_tasks, which turns them off
 * for every class): enable = 1 lets the class's workgroups take whole bra
 * blocks where the LDS rows fit, 0 keeps its waves on single tiles.  Without
 * a call (or a schedule file) the ket-outer lane classes take them and the
 * bra-outer ones do not.  Takes effect at the next fk_build_quartets;
 * FK_ERR_UNSUPPORTED for a class not built.  Classes other than the lane
 * classes listed at fk_screen_opts.block_tasks never take block tasks,
 * whatever is set. */
int fk_set_class_block_tasks(fk_ctx *ctx, int la, int lb, int lc, int ld, int enable);

/* Lanes per quartet of a class's kernel.  Every class has its own kernel
 * kind (a lane per quartet up to 54 integrals, a team of lanes per quartet,
 * or a wave per quartet for f-f bras; fk_stats.team_size); the lane classes
 * with 18 or more integrals and a bra shell of at least three components
 * ((pp|ps), (ds|ps), (ds|pp), (ds|ds), (dp|ss), (dp|ps), (dd|ss), (fs|ps),
 * (fp|ss)) also have a team kernel with one lane per component of the first
 * bra shell.  lanes = 1 selects the lane kernel, lanes = that component
 * count the team kernel; any other value, or a class without the kernel,
 * gives FK_ERR_UNSUPPORTED.  Takes effect at the next fk_build_quartets; the
 * team kernel takes the Rys engine and no block tasks. */
int fk_set_class_lanes(fk_ctx *ctx, int la, int lb, int lc, int ld, int lanes);

/* Schedule cache: fk_save_schedules writes every schedule and engine set on
 * the context (by fk_set_class_schedule, fk_set_class_engine,
 * fk_set_class_block_tasks, fk_set_class_lanes, fk_autotune or
 * an earlier load) to a text file, one line per class
 * ("class la lb lc ld bra_block kets_per_tile grid_fraction engine
 * block_tasks alt_lanes", alt_lanes 0 for the class's own kernel, else the
 * lanes per quartet of its team alternative; files without the last fields
 * read as the class's default block tasks and alt_lanes 0) after a
 * line naming the device architecture ("arch gfx950"; "host" for a context
 * without a device).  fk_load_schedules reads such a file into the context,
 * on top of the schedules already set; FK_ERR_UNSUPPORTED if the file was
 * written for another architecture or names a class or engine this library
 * does not build, FK_ERR_ARG for a malformed file (the context is then left
 * unchanged).  Like fk_set_class_schedule, a load takes effect at the next
 * fk_build_quartets.  A schedule set tuned on one workload suits workloads
 * of the same basis family and size; it never changes results beyond rounding
 * order. */
int fk_save_schedules(fk_ctx *ctx, const char *path);
int fk_load_schedules(fk_ctx *ctx, const char *path);

typedef struct {
    int    nclass;                      /* class launches after tuning (as fk_stats) */
    int    la[FK_MAX_QCLASS], lb[FK_MAX_QCLASS], lc[FK_MAX_QCLASS], ld[FK_MAX_QCLASS];
    int    precision[FK_MAX_QCLASS];    /* 64 or 32 */
    int    bra_block[FK_MAX_QCLASS], kets_per_tile[FK_MAX_QCLASS];
    double grid_fraction[FK_MAX_QCLASS];
    int    engine[FK_MAX_QCLASS];       /* FK_ENGINE_RYS or FK_ENGINE_HGP */
    int    changed[FK_MAX_QCLASS];      /* 1 if the schedule differs from the one before tuning */
    double ms_default[FK_MAX_QCLASS];   /* the launch's kernel time before tuning */
    double ms_tuned[FK_MAX_QCLASS];
    double build_ms_default, build_ms_tuned;  /* sums over the class launches */
    int    configurations;              /* list configurations built and timed */
    int    block_tasks[FK_MAX_QCLASS];  /* 1 if the class's schedule allows block tasks */
    int    lanes_per_quartet[FK_MAX_QCLASS]; /* 1 (lane kernel), a team's lanes, or 64 */
} fk_tune_report;

/* Autotuner for the schedules above: on the current geometry, basis and
 * screening options (those of the last fk_build_quartets) and density D
 * (as in fk_build_jk: FK_DEVICE_PTRS for a device pointer, else host), it
 * tries one axis at a time for all classes at once -- bra_block 1..32, then
 * 1, 2, 4, 8 rounds of kets per tile, then grid fractions 1, 1/2, 1/4, 2, 4,
 * then the other integral engine where a class has both, then block tasks
 * switched for the classes that take them (an LDS staging choice), then the
 * other kernel kind (lanes per quartet) where a class has two --
 * rebuilding the lists and timing each class launch with HIP events (one
 * warm-up and `reps` timed builds, the minimum kept), keeps for each class the
 * candidate more than 2 % faster than its best so far, and leaves the lists
 * built with the chosen schedules.  report may be NULL.  Runs about
 * 20 (reps + 1) builds and 20 list builds; allocates three nbf^2 buffers for
 * its duration. */
int fk_autotune(fk_ctx *ctx, const double *D, unsigned flags, int reps, void *stream, fk_tune_report *report);

/* ---- one-electron part and SCF (paper: "Hartree-Fock Energy Formulation") */
/* Overlap S, kinetic T and nuclear attraction V (host arrays nbf x nbf) and the
 * nuclear repulsion energy.  Any output pointer may be NULL. */
int fk_one_electron(fk_ctx *ctx, double *S, double *T, double *V, double *e_nuc);

typedef struct {
    int    max_iter;     /* default 100 */
    double e_tol;        /* |dE| threshold, default 1e-10 */
    double g_tol;        /* max |X (FDS - SDF) X| threshold, default 1e-8 */
    int    diis_n;       /* DIIS subspace size (0 or 1: no DIIS), default 8, at most 32 */
    int    guess;        /* 0 = core Hamiltonian, 1 = density given in D_inout,
                            2 = superposition of atomic densities (fk_sad_density),
                            3 = learned (the model of fk_set_guess_model; falls
                                back to 2, then 0, if the model is missing, an
                                element is not covered, the prediction is not
                                finite or its purification fails) */
    double lindep;       /* required accuracy of the orthogonaliser: max |Z S Z - I|
                            with Z = S^(-1/2) from the Newton-Schulz iteration;
                            fails with FK_ERR_ARG for an overlap matrix too
                            ill-conditioned to reach it, or when an entry of
                            S^(-1/2) exceeds 3e3 (overlap eigenvalues near
                            1e-7: the basis is nearly linearly dependent and
                            no direction is dropped).  Default 1e-8 */
    int    graph;        /* fk_run_scf: 1: from the second iteration on, the
                            Fock stage of an iteration (J/K build, F, the
                            energy terms, X F X, the commutator and its norm)
                            is one HIP graph, captured once and replayed, on a
                            stream of the run's own; DIIS and purification
                            stay eager.  fk_run_scf_batch: 1: the whole
                            iteration is one HIP graph -- the build, the Fock
                            stage, the convergence flags, the DIIS ring and
                            Pulay solve, the purification's choices (at most
                            128 steps) and the kept densities of converged
                            molecules are all decided by kernels; the host
                            reads the energies and flags after each replay.
                            jk_seconds then times the whole stage or
                            iteration.  Default 0 */
    int    incremental;  /* k > 0: J and K from the density change since the
                            previous build, added to running sums, with a full
                            build every k iterations; the change is screened
                            with tau / 1000 (its smaller density bounds still
                            drop most quartets late in the run); 0 = full
                            builds.  Not together with graph.  Default 0 */
    double canonical;    /* 0: the orthogonaliser is S^(-1/2) by Newton-Schulz,
                            every overlap direction kept (lindep applies);
                            c in (0, 1): canonical orthogonalisation: the
                            overlap matrix is diagonalised once per geometry
                            on the device (rocSOLVER), eigenvectors with
                            eigenvalue <= c are dropped and X = U s^(-1/2) U^T
                            over the rest; the dropped directions are given
                            Fock eigenvalue +1 hartree so that they stay
                            empty.  For nearly linearly dependent bases.
                            Default 0 */
    int    j_engine;     /* 1: every build of the run uses FK_J_ENGINE (J by the
                            J engine, K by the Rys kernels at fk_screen_opts
                            .tau_k).  Default 0 */
    int    density_eig;  /* 1: each density from the eigenvectors of X F X
                            (rocSOLVER, the nelec/2 lowest states) instead of
                            purification.  Purification reaches the commutator
                            criterion only where X F X is well conditioned: in
                            a basis with overlap eigenvalues near 1e-5 its
                            relative gap is small and the density's occupied-
                            virtual mixing stays near 1e-7; the eigensolver
                            density converges there.  Not with graph for
                            fk_run_scf_batch.  Default 0 */
} fk_scf_opts;

typedef struct {
    double energy;       /* total energy (hartree) of the last density */
    double e_nuc;
    int    iterations;   /* Fock builds performed */
    int    converged;
    double jk_seconds;   /* wall time spent in fk_build_jk */
    double total_seconds;
    double error;        /* max |X (FDS - SDF) X| at the last iteration */
    double delta_e;      /* energy change of the last iteration */
    int    guess_used;   /* the guess the run started from (see fk_scf_opts.guess) */
    double guess_seconds;/* wall time of the initial density */
    int    ndropped;     /* overlap directions the canonical orthogonaliser dropped */
} fk_scf_result;

/* Restricted closed-shell SCF (paper: "Hartree-Fock Energy Formulation"):
 * F = h + J - K/2 with J, K from fk_build_jk on the quartet lists of the last
 * fk_build_quartets; E = (D.h + D.F)/2 + E_nuc; Pulay DIIS on the commutator
 * X (FDS - SDF) X.  Every per-iteration matrix step runs on the device: the
 * orthogonaliser X = S^(-1/2) comes from a Newton-Schulz iteration, and the
 * density D = 2 X P X from trace-correcting purification of X F X (P the
 * projector onto the nelec/2 lowest states), so no eigensolver is used
 * (opts->density_eig = 1: P from rocSOLVER eigenvectors instead); the
 * host solves the small DIIS system.  Converged when |dE| < e_tol and the
 * error < g_tol.  D_inout (host, nbf x nbf, row-major) holds the guess when
 * opts->guess == 1 and the final density on return.  opts may be NULL
 * (defaults).  max_iter = 0 returns the initial density in D_inout and
 * performs no Fock build.  Returns FK_ERR_NOT_CONVERGED (with the result
 * filled) if max_iter is reached, or if the purification (or the
 * eigensolver density) finds no gap. */
int fk_run_scf(fk_ctx *ctx, const fk_scf_opts *opts, fk_scf_result *result, double *D_inout);

/* Batched SCF (several molecules in one context, fk_set_molecules): the SCF
 * step above for every molecule at once -- one batched fk_build_jk per
 * iteration, every dense step (orthogonaliser, Fock matrix, energies, DIIS
 * commutators, purification, D = X D' X) a batched kernel over the
 * concatenated per-molecule blocks, with each molecule's DIIS system and
 * purification choices solved on the host.  Molecules must be neutral and
 * closed shell.  A molecule that meets the criteria of fk_run_scf keeps
 * that density (and those results) while the others iterate on; the run ends
 * when every molecule has converged.  results: nmol entries (iterations: the
 * Fock builds until that molecule converged; jk_seconds and total_seconds are
 * the batch's); D_inout: host array of the
 * batch layout (fk_molecule_layout), the guess for guess = 1 and the final
 * densities on return.  guess = 3 starts from SAD (guess_used = 2): the
 * learned guess is per molecule.  max_iter = 0 returns the initial densities.
 * graph = 1 with density_eig = 1: FK_ERR_UNSUPPORTED.
 * With the environment variable FK_SCF_LOG set (not "0") each iteration
 * prints one progress line to stderr. */
int fk_run_scf_batch(fk_ctx *ctx, const fk_scf_opts *opts, fk_scf_result *results, double *D_inout);

/* ---- initial densities (an extension: the paper's SCF starts from a
 * conventional guess and has no learned part) ---------------------------- */

/* Superposition of atomic densities: for each element, the atom alone (its
 * shells, Z electrons) in a fractional-occupation SCF (F = h + J - K/2,
 * D = sum n_i c_i c_i^T, aufbau over levels of orbitals within 1e-4 hartree,
 * a partly filled level sharing its electrons equally, damped iteration
 * from the core guess until max |dD| < 1e-10); the molecule's density is
 * block diagonal over its atoms.  Host computation; D_out is a host array
 * of nbf x nbf (a batch: of the batch layout, fk_molecule_layout).  Works on
 * a context without a device. */
int fk_sad_density(fk_ctx *ctx, double *D_out);

/* Learned guess.  Atom pairs: every atom with itself and every pair closer
 * than FK_GUESS_RCUT, in row-major order over (i <= j); the pair's first atom
 * is the one of higher Z (lower index on ties).
 * Pair frame (columns e_x, e_y, e_z): for two atoms, e_z from the first to
 * the second and e_x towards the first atom's nearest neighbour off that axis
 * (else the second atom's); for an atom with itself, e_z towards its nearest
 * neighbour and e_x towards the next nearest off-axis one.  "Off-axis": the
 * direction's component orthogonal to e_z exceeds 0.1 of its length;
 * neighbours (within FK_GUESS_RCUT) are ordered by distance on a 1e-6 bohr
 * grid, then index; without a suitable neighbour e_x comes from the lab axis
 * least aligned with e_z (a lone atom keeps the lab frame).
 * Features of a pair (FK_GUESS_NFEAT floats): one-hot of the first atom's
 * element over (H, C, N, O), one-hot of the second's, FK_GUESS_NRBF
 * Gaussians exp(-g (R - mu_k)^2), mu_k = k RCUT / (NRBF - 1),
 * g = ((NRBF - 1) / RCUT)^2, then for the first and then the second atom the
 * moments (1, u_x, u_y, u_z, u_x^2, u_x u_y, u_x u_z, u_y^2, u_y u_z, u_z^2)
 * of the unit vectors u (pair-frame coordinates) to each other atom within
 * FK_GUESS_RCUT except the pair's two, weighted by exp(-(r / 3)^2) and
 * exp(-((r - 5) / 1.5)^2) (r in bohr), summed per element:
 * [atom][element][weight][moment].
 * Output of a pair: the block D[first's functions][second's functions] in the
 * pair frame, row-major, padded to FK_GUESS_NB x FK_GUESS_NB. */
#define FK_GUESS_NB 15
#define FK_GUESS_NOUT (FK_GUESS_NB * FK_GUESS_NB)
#define FK_GUESS_NRBF 24
#define FK_GUESS_NFEAT (8 + FK_GUESS_NRBF + 160)
#define FK_GUESS_RCUT 8.0      /* bohr */
#define FK_MLP_MAX_LAYERS 4

/* Multilayer perceptron: y = L_{n-1}(s(... s(L_0(x)))), L_k(x) = x W_k + b_k,
 * s(z) = z / (1 + exp(-z)) (SiLU).  W_k is dims[k] x dims[k+1] row-major,
 * b_k has dims[k+1] entries, FP32.  The pointers are host or device pointers
 * as each function states; the caller owns them. */
typedef struct {
    int    nlayer;                        /* 1..FK_MLP_MAX_LAYERS */
    int    dims[FK_MLP_MAX_LAYERS + 1];   /* each 1..4096 */
    float *W[FK_MLP_MAX_LAYERS];
    float *b[FK_MLP_MAX_LAYERS];
} fk_mlp;

/* Pairs of the current geometry: *npair always; features [npair][NFEAT] and
 * shape[npair] = (functions of the first atom << 8) | functions of the
 * second, if non-NULL (host arrays).  FK_ERR_UNSUPPORTED if an atom is not
 * H, C, N or O or has more than FK_GUESS_NB functions. */
int fk_guess_pairs(fk_ctx *ctx, int *npair, float *features, int *shape);

/* Training targets: the pair blocks of density D (host nbf x nbf) in the
 * pair frames, D_frame = T(Q)^T D_block T(Q) with T the Cartesian rotation
 * of each atom's shells, as Y[npair][FK_GUESS_NOUT] (host), zero-padded. */
int fk_guess_targets(fk_ctx *ctx, const double *D, float *Y);

/* Copies a network (host pointers; dims[0] = FK_GUESS_NFEAT, last dims =
 * FK_GUESS_NOUT) to the context's device; used by fk_guess_predict and by
 * fk_run_scf with guess = 3.  NULL removes it. */
int fk_set_guess_model(fk_ctx *ctx, const fk_mlp *host_model);

/* The network's prediction assembled into an nbf x nbf density before
 * purification (host D_out): each pair's block rotated back with the
 * Cartesian transforms of its atoms' shells and written to both triangles;
 * an atom's own block symmetrised; pairs beyond the cutoff zero. */
int fk_guess_predict(fk_ctx *ctx, double *D_out);

/* ---- network primitives on the device (training and inference) ----------
 * Device pointers, FP32, on `stream`; these return FK_ERR_ARG for invalid
 * sizes and FK_ERR_HIP for a failed launch and need no context. */

/* Floats of workspace fk_mlp_forward needs for n rows (activations kept for
 * the backward pass). */
int64_t fk_mlp_work_floats(const fk_mlp *m, int n);

/* Y[n][dims[nlayer]] from X[n][dims[0]]; work as sized above. */
int fk_mlp_forward(const fk_mlp *m, const float *X, int n, float *Y, float *work, void *stream);

/* Gradients of a loss whose gradient in Y is dY (overwritten as scratch),
 * after fk_mlp_forward on the same X and work: grad->W[k], grad->b[k]
 * (device buffers of the weights' sizes) receive dL/dW_k, dL/db_k. */
int fk_mlp_backward(const fk_mlp *m, const float *X, int n, float *work, float *dY, const fk_mlp *grad, void *stream);

/* Masked mean squared error over rows of FK_GUESS_NB x FK_GUESS_NB blocks:
 * entries (i, j) with i < shape[r] >> 8 and j < shape[r] & 255 count.
 * loss[0] (device double) = sum (Y - T)^2 / count; dY = 2 (Y - T) / count
 * on those entries, 0 elsewhere.  count = sum over rows of the two sizes'
 * product (given by the caller).  part: fk_mlp_mse_scratch() doubles. */
int fk_mlp_block_mse(const float *Y, const float *T, const int *shape, int n, double count, float *dY, double *part,
                     double *loss, void *stream);
int fk_mlp_mse_scratch(void);

/* One Adam step (Kingma and Ba 2015) on every weight and bias:
 * m1 = b1 m1 + (1 - b1) g, m2 = b2 m2 + (1 - b2) g^2,
 * w -= lr (m1 / (1 - b1^step)) / (sqrt(m2 / (1 - b2^step)) + eps).
 * grad, m1, m2 have the model's shapes (device); step >= 1. */
int fk_mlp_adam(const fk_mlp *m, const fk_mlp *grad, const fk_mlp *m1, const fk_mlp *m2, int step, float lr, float b1,
                float b2, float eps, void *stream);

/* ---- diagnostics -------------------------------------------------------- */
/* Raw contracted integrals (ab|cd) for nq shell quartets (shell indices
 * quartets[4q..4q+3], any order and any angular momenta), written
 * consecutively as [na][nb][nc][nd] blocks into out (host array of
 * sum na*nb*nc*nd doubles).  mode bit 0: 1 evaluates on the GPU with the
 * production per-quartet code, 0 evaluates the same code on the host;
 * mode >> 1: 0 = Rys engine, 1 = HGP engine (FK_ERR_UNSUPPORTED if a
 * quartet's class has no HGP kernel), 2 = the Hermite (McMurchie-Davidson)
 * expansion the J engine's E and R pieces define (host only, L <= 8). */
int fk_debug_eri(fk_ctx *ctx, int nq, const int *quartets, double *out, int mode);

/* Host-side check of every address the J/K kernels will form for the current
 * quartet lists (list positions, primitive records, LDS slots, density and
 * Fock indices).  FK_OK, or FK_ERR_STATE with the first violation in
 * fk_last_error.  Intended for tests and diagnostics. */
int fk_check_indices(fk_ctx *ctx);

/* Rys roots u[n] and weights w[n] for argument T from the library's tables,
 * evaluated on the host (n = 1..7). */
int fk_rys_host(int n, double T, double *u, double *w);

#ifdef __cplusplus
}
#endif
#endif
