// Structures and launchers of the learned-guess kernels (fk_guess.hip),
// shared with the host code; not part of the ABI.
#pragma once

// Atom pair of the learned density guess: its atoms (a1 is the pair's first
// atom, the origin of its frame), their first basis functions and function
// counts (at most FK_GUESS_NB each).
#ifndef FK_GUESS_NB
#define FK_GUESS_NB 15
#endif
struct FkGuessPair {
    int a1, a2, f1, f2, n1, n2;
};

extern "C" {
// FP32 row-major matrices
int fk_guess_mm(int ta, int tb, const float *A, int lda, const float *B, int ldb, float *C, float *A_out,
                const float *bias, int M, int N, int K, void *stream);
int fk_guess_silu_back(float *G, const float *Z, long long n, void *stream);
int fk_guess_colsum(const float *G, int rows, int cols, float *out, void *stream);
int fk_guess_mse_parts();
int fk_guess_block_mse(const float *Y, const float *T, const int *shape, int rows, int width, double count, float *dY,
                       double *part, double *loss, void *stream);
int fk_guess_adam(float *W, const float *g, float *m1, float *m2, long long n, float lr, float b1, float b2, float eps,
                  float c1, float c2, void *stream);
int fk_guess_scatter(const float *Y, const FkGuessPair *pairs, const double *rot, int npair, int n, double *D,
                     void *stream);
}
