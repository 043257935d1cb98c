// Kernels of the learned initial density (an extension: the paper's SCF starts
// from a conventional guess).  A small multilayer perceptron maps features of
// an atom pair to that pair's density block in the pair's bond frame; the
// blocks are rotated to the molecular frame and scattered into D, which the
// SCF step then purifies.  The same library trains the network: forward,
// backward, a masked squared-error loss and Adam are the kernels below.
//
// Everything here is FP32 except the scatter (FP64 rotation and output).  The
// products are small (pairs x 256 x 256 per layer, well under a millisecond
// per geometry), so a plain LDS-tiled FMA GEMM is used rather than MFMA.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "fk_guess.h"

namespace {

constexpr int MT = 64;  // output tile (MT x MT) per workgroup
constexpr int MK = 16;  // k-slab staged in LDS

// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias, activation), row-major.
//   TA = 0: A[m][k] at A[m * lda + k];  TA = 1: A stored [K][M], A[k * lda + m]
//   TB = 0: B[k][n] at B[k * ldb + n];  TB = 1: B stored [N][K], B[n * ldb + k]
// epilogue: bias (may be null) added; if A_out is non-null it receives
// SiLU(C) = C / (1 + exp(-C)) as well.  256 threads; thread (ty, tx) of a
// 16 x 16 grid owns outputs (ty + 16 i, tx + 16 j), i, j < 4.
template <int TA, int TB>
__global__ void __launch_bounds__(256) k_mm(const float *__restrict A, int lda, const float *__restrict B, int ldb,
                                            float *__restrict C, float *__restrict A_out, const float *__restrict bias,
                                            int M, int N, int K)
{
    __shared__ float As[MK][MT + 1];
    __shared__ float Bs[MK][MT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * MT, n0 = blockIdx.x * MT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += MK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = threadIdx.x + 256 * r;  // 0 .. 1023 = 64 x 16 elements
            // A slab: element (m, k) = (idx >> 4, idx & 15) or, transposed, (idx & 63, idx >> 6)
            int am, ak;
            if (TA) { am = idx & 63; ak = idx >> 6; } else { am = idx >> 4; ak = idx & 15; }
            const int gm = m0 + am, gk = k0 + ak;
            float va = 0.0f;
            if (gm < M && gk < K) va = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[ak][am] = va;
            int bk, bn;
            if (TB) { bn = idx >> 4; bk = idx & 15; } else { bk = idx >> 6; bn = idx & 63; }
            const int hk = k0 + bk, hn = n0 + bn;
            float vb = 0.0f;
            if (hk < K && hn < N) vb = TB ? B[(size_t)hn * ldb + hk] : B[(size_t)hk * ldb + hn];
            Bs[bk][bn] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty + 16 * i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx + 16 * j;
            if (n >= N) continue;
            float v = acc[i][j];
            if (bias) v += bias[n];
            C[(size_t)m * N + n] = v;
            if (A_out) A_out[(size_t)m * N + n] = v / (1.0f + expf(-v));
        }
    }
}

// G <- G * SiLU'(Z), SiLU'(z) = s (1 + z (1 - s)), s = 1 / (1 + exp(-z))
__global__ void __launch_bounds__(256) k_silu_back(float *__restrict G, const float *__restrict Z, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float z = Z[i];
    const float s = 1.0f / (1.0f + expf(-z));
    G[i] *= s * (1.0f + z * (1.0f - s));
}

// out[j] = sum_r G[r][j]: 64 columns per workgroup, 4 row phases reduced in
// LDS (fixed order, so the result is deterministic).
__global__ void __launch_bounds__(256) k_colsum(const float *__restrict G, int rows, int cols, float *__restrict out)
{
    __shared__ float part[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    float s = 0.0f;
    if (c < cols)
        for (int r = ph; r < rows; r += 4) s += G[(size_t)r * cols + c];
    part[ph][threadIdx.x & 63] = s;
    __syncthreads();
    if (ph == 0 && c < cols) out[c] = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

// Masked squared error over the (width x width) blocks of each row: entry
// (i, j) of row r counts if i < shape_r >> 8 and j < shape_r & 255.
// dY = 2 (Y - T) mask / count; per-workgroup partial sums of the squares.
constexpr int LB = 256;
__global__ void __launch_bounds__(LB) k_block_mse(const float *__restrict Y, const float *__restrict T,
                                                  const int *__restrict shape, int rows, int width, double inv_count,
                                                  float *__restrict dY, double *__restrict part)
{
    __shared__ double red[LB];
    const int m = width * width;
    const long long total = (long long)rows * m;
    double s = 0.0;
    for (long long e = (long long)blockIdx.x * LB + threadIdx.x; e < total; e += (long long)gridDim.x * LB) {
        const int r = (int)(e / m), k = (int)(e % m);
        const int i = k / width, j = k % width;
        const int sh = shape[r];
        float g = 0.0f;
        if (i < (sh >> 8) && j < (sh & 255)) {
            const double d = (double)Y[e] - (double)T[e];
            s += d * d;
            g = (float)(2.0 * d * inv_count);
        }
        dY[e] = g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = LB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(64) k_sum_parts(const double *__restrict part, int n, double scale, double *out)
{
    __shared__ double red[64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// Adam (Kingma and Ba) with bias corrections c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ void __launch_bounds__(256) k_adam(float *__restrict W, const float *__restrict g, float *__restrict m1,
                                              float *__restrict m2, long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    W[i] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
}

// One workgroup per atom pair: L = T_1^T B T_2 with B the predicted
// bond-frame block (rows: functions of the pair's first atom) and T_k the
// block-diagonal rotation of atom k's Cartesian components, written to D at
// (first, second) and its transpose; an on-site block is symmetrised.
__global__ void __launch_bounds__(256) k_guess_scatter(const float *__restrict Y, const FkGuessPair *__restrict pairs,
                                                       const double *__restrict rot, int n, double *__restrict D)
{
    constexpr int W = FK_GUESS_NB;
    __shared__ double B[W][W + 1];
    __shared__ double H[W][W + 1];
    const FkGuessPair p = pairs[blockIdx.x];
    const double *T1 = rot + (size_t)blockIdx.x * 2 * W * W;
    const double *T2 = T1 + W * W;
    const int t = threadIdx.x;
    const int i = t / W, j = t % W;
    const bool act = t < W * W;
    if (act) B[i][j] = (i < p.n1 && j < p.n2) ? (double)Y[(size_t)blockIdx.x * W * W + t] : 0.0;
    __syncthreads();
    // H = B T_2
    if (act) {
        double v = 0.0;
        if (i < p.n1 && j < p.n2)
            for (int k = 0; k < p.n2; ++k) v += B[i][k] * T2[k * W + j];
        H[i][j] = v;
    }
    __syncthreads();
    // L = T_1^T H (kept in B)
    double v = 0.0;
    if (act && i < p.n1 && j < p.n2)
        for (int k = 0; k < p.n1; ++k) v += T1[k * W + i] * H[k][j];
    __syncthreads();
    if (act) B[i][j] = v;
    __syncthreads();
    if (!act || i >= p.n1 || j >= p.n2) return;
    if (p.a1 == p.a2) {
        D[(size_t)(p.f1 + i) * n + p.f2 + j] = 0.5 * (B[i][j] + B[j][i]);
    } else {
        D[(size_t)(p.f1 + i) * n + p.f2 + j] = B[i][j];
        D[(size_t)(p.f2 + j) * n + p.f1 + i] = B[i][j];
    }
}

__global__ void __launch_bounds__(256) k_fill(double *__restrict p, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int fk_guess_mm(int ta, int tb, const float *A, int lda, const float *B, int ldb, float *C, float *A_out,
                const float *bias, int M, int N, int K, void *stream)
{
    if (M <= 0 || N <= 0) return 0;
    const dim3 grid((N + MT - 1) / MT, (M + MT - 1) / MT);
    const hipStream_t st = (hipStream_t)stream;
    if (!ta && !tb) hipLaunchKernelGGL((k_mm<0, 0>), grid, dim3(256), 0, st, A, lda, B, ldb, C, A_out, bias, M, N, K);
    else if (!ta && tb) hipLaunchKernelGGL((k_mm<0, 1>), grid, dim3(256), 0, st, A, lda, B, ldb, C, A_out, bias, M, N, K);
    else if (ta && !tb) hipLaunchKernelGGL((k_mm<1, 0>), grid, dim3(256), 0, st, A, lda, B, ldb, C, A_out, bias, M, N, K);
    else return -1;
    return ok();
}

int fk_guess_silu_back(float *G, const float *Z, long long n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_silu_back, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, G, Z, n);
    return ok();
}

int fk_guess_colsum(const float *G, int rows, int cols, float *out, void *stream)
{
    if (cols <= 0) return 0;
    hipLaunchKernelGGL(k_colsum, dim3((cols + 63) / 64), dim3(256), 0, (hipStream_t)stream, G, rows, cols, out);
    return ok();
}

int fk_guess_mse_parts() { return 480; }

int fk_guess_block_mse(const float *Y, const float *T, const int *shape, int rows, int width, double count, float *dY,
                       double *part, double *loss, void *stream)
{
    if (rows <= 0) return 0;
    const long long total = (long long)rows * width * width;
    const int g = (int)std::min<long long>(fk_guess_mse_parts(), (total + LB - 1) / LB);
    hipLaunchKernelGGL(k_block_mse, dim3(g), dim3(LB), 0, (hipStream_t)stream, Y, T, shape, rows, width,
                       1.0 / count, dY, part);
    if (ok()) return -3;
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, (hipStream_t)stream, part, g, 1.0 / count, loss);
    return ok();
}

int fk_guess_adam(float *W, const float *g, float *m1, float *m2, long long n, float lr, float b1, float b2, float eps,
                  float c1, float c2, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, W, g, m1, m2, n, lr, b1, b2, eps, c1,
                       c2);
    return ok();
}

int fk_guess_scatter(const float *Y, const FkGuessPair *pairs, const double *rot, int npair, int n, double *D,
                     void *stream)
{
    const long long nn = (long long)n * n;
    if (nn <= 0) return 0;
    hipLaunchKernelGGL(k_fill, dim3(nblk(nn)), dim3(256), 0, (hipStream_t)stream, D, nn);
    if (ok()) return -3;
    if (npair <= 0) return 0;
    hipLaunchKernelGGL(k_guess_scatter, dim3(npair), dim3(256), 0, (hipStream_t)stream, Y, pairs, rot, n, D);
    return ok();
}

}  // extern "C"
