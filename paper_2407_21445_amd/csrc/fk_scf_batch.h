// Launchers of the batched SCF-step kernels (fk_scf_batch.hip); not part of
// the ABI.  Matrices are concatenations of per-molecule n_m x n_m row-major
// FP64 blocks: nbf[m], off[m] (device arrays), nmax = max n_m.
#pragma once

extern "C" {
int fk_scfb_gemm(const double *A, const double *B, double *C, int nmol, int nmax, const int *nbf, const long long *off,
                 double alpha, double beta, void *stream);
// out = a_m x + b_m y + c_m z + d_m I, coef = device array [4 nmol]
int fk_scfb_lincomb(double *out, const double *x, const double *y, const double *z, int nmol, int nmax, const int *nbf,
                    const long long *off, const double *coef, void *stream);
int fk_scfb_antisym(double *E, const double *G, int nmol, int nmax, const int *nbf, const long long *off, void *stream);
// per-molecule reductions into out[nmol] (op 3: out[2 nmol]); ops as fk_scf_reduce
int fk_scfb_reduce(const double *x, const double *y, int nmol, const int *nbf, const long long *off, int op,
                   double *part, double *out, void *stream);
long long fk_scfb_reduce_scratch(int nmol);

// ---- device-decided iteration (graph replay) ----
#define FK_SCFB_MAX_DIIS 32
// C = A B per molecule, molecules with skip[m] != 0 left untouched
int fk_scfb_gemm_skip(const double *A, const double *B, double *C, int nmol, int nmax, const int *nbf,
                      const long long *off, const int *skip, void *stream);
int fk_scfb_iter_begin(int *ictl, int dn, void *stream);
int fk_scfb_conv(const double *dh, const double *df, const double *err, const double *enuc, int nmol, double e_tol,
                 double g_tol, const int *ictl, int *conv, double *eprev, double *keep, double *status, void *stream);
// ring slot copy of F' and the error, the B row, the Pulay solve and F' from
// the ring; part: nmol * dn * 32 doubles; Bm: nmol dn^2; dcoef: nmol dn
int fk_scfb_diis(double *ringF, double *ringE, const double *Fo, const double *E, double *Fo_out, int nmol, int nmax,
                 const int *nbf, const long long *off, long long nmat, int dn, const int *ictl, double *part,
                 double *Bm, double *dcoef, void *stream);
int fk_scfb_pur_start(const double *gb, int nmol, double *coef, int *pstate, int *pdone, int *ictl, void *stream);
int fk_scfb_pur_step(const double *t1, const double *t2, const int *nocc, int nmol, double *coef, int *pstate,
                     int *pdone, void *stream);
int fk_scfb_pur_check(const int *pstate, int nmol, int *ictl, void *stream);
}
