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
}
