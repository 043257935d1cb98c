// Structures shared by the host library and the kernels (not part of the ABI).
#pragma once

#include <stdint.h>

#define FK_NPP_REC 10  // doubles per primitive-pair record

// Primitive-pair record layout (FK_NPP_REC doubles):
//   0 zeta, 1 1/(2 zeta), 2-4 P, 5-7 P - A, 8 K (see fk::PrimPair), 9 G_[ab].

// Work tile: one bra shell pair and up to 64 consecutive ket shell pairs of one
// ket class (all with the same number of primitive pairs).
struct FkTile {
    int bra;        // shell-pair index
    int ket_begin;  // index into the ket class's sorted pair list
    int ket_count;  // 1..64
    int flags;      // bit 0: bra and ket from the same class
};

struct FkJKArgs {
    const int *sh_bf;        // [nshell + 1] first basis function of each shell
    const int *pair_sa;      // [npair] first shell (higher l)
    const int *pair_sb;      // [npair] second shell
    const int *pair_ppoff;   // [npair] first primitive pair
    const int *pair_npp;     // [npair] number of primitive pairs
    const double *pair_AB;   // [npair * 3] A - B
    const double *pair_G;    // [npair] Schwarz factor
    const double *pp;        // [nprimpair * FK_NPP_REC]
    const int *ket_list;     // sorted pair indices of the ket class
    const FkTile *tiles;
    int ntiles;
    int nshell;
    const double *Dsh;       // [nshell * nshell] max |D| per shell block
    const double *Ds;        // [nbf * nbf] component-scaled density
    double *XJ;              // [nbf * nbf] unsymmetrised Coulomb accumulator
    double *XK;              // [nbf * nbf] unsymmetrised exchange accumulator
    int nbf;
    int dscreen;             // apply the density screen
    double tau;
    const double *rys_tab;   // staged Rys segment (table + Gauss-Hermite) of this class's root count
    unsigned long long *counters;  // [2]: contracted quartets, primitive quartets
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
};

// Per-class launch entry points (defined in fk_kernels.hip).
struct FkClassInfo {
    int la, lb, lc, ld, nroot, nout;
    int wave_per_quartet;    // 1: wave-per-quartet kernel, 0: lane-per-quartet
    double flops_prim, flops_quartet;
};

extern "C" {
int fk_kernels_class_info(int P, int Q, FkClassInfo *info);
int fk_kernels_launch_jk(int P, int Q, const FkJKArgs *args, int grid, void *stream);
int fk_kernels_launch_debug(int P, int Q, const FkDebugArgs *args, void *stream);
int fk_kernels_max_blocks(int P, int Q, int *blocks_per_cu);
int fk_kernels_launch_prep(const double *D, const int *sh_bf, const double *bf_scale, int nshell, int nbf,
                           double *Ds, double *Dsh, void *stream);
int fk_kernels_launch_finalize(const double *XJ, const double *XK, const double *bf_scale, int nbf,
                               double *J, double *K, void *stream);
int fk_kernels_launch_fill(double *p, long long n, void *stream);
int fk_kernels_debug_host(int P, int Q, const int *pair_ppoff, const int *pair_npp, const double *pair_AB,
                          const double *pp, const int *quartets, int nq, double *out);
}
