// Dense kernels of the SCF step for a batch of molecules (the same operations
// as fk_scf.hip, per molecule): every matrix is the concatenation of the
// molecules' n_m x n_m row-major FP64 blocks, block m at offset off[m].
// Per-molecule scalars (coefficients, reduction results) are device arrays
// indexed by molecule, so one launch serves the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fk_scf_batch.h"

namespace {

constexpr int GT = 64;   // output tile (GT x GT) per workgroup
constexpr int GK = 16;   // k-slab staged in LDS
constexpr int GPAD = 1;

// C_m = alpha A_m B_m + beta C_m; molecule blockIdx.z; tiles outside the
// molecule's n_m x n_m block exit (the whole workgroup, before any barrier).
__global__ void __launch_bounds__(256) k_bgemm(const double *__restrict A, const double *__restrict B,
                                               double *__restrict C, const int *__restrict nbf,
                                               const long long *__restrict off, double alpha, double beta)
{
    __shared__ double As[GK][GT + GPAD];
    __shared__ double Bs[GK][GT + GPAD];
    const int m = blockIdx.z;
    const int n = nbf[m];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    if (m0 >= n || n0 >= n) return;
    const size_t base = (size_t)off[m];
    A += base;
    B += base;
    C += base;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += GK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = threadIdx.x + 256 * r;
            const int am = idx >> 4, ak = idx & 15;
            const int gm = m0 + am, gk = k0 + ak;
            As[ak][am] = (gm < n && gk < n) ? A[(size_t)gm * n + gk] : 0.0;
            const int bk = idx >> 6, bn = idx & 63;
            const int hk = k0 + bk, hn = n0 + bn;
            Bs[bk][bn] = (hk < n && hn < n) ? B[(size_t)hk * n + hn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < GK; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty + 16 * i;
        if (gm >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx + 16 * j;
            if (gn >= n) continue;
            double *c = C + (size_t)gm * n + gn;
            *c = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *c);
        }
    }
}

// out = a_m x + b_m y + c_m z + d_m I with coef[4 m .. 4 m + 3] = (a, b, c, d);
// y, z may be null; out may alias x, y or z.  Molecule blockIdx.y.
__global__ void __launch_bounds__(256) k_blincomb(double *out, const double *x, const double *y, const double *z,
                                                  const int *__restrict nbf, const long long *__restrict off,
                                                  const double *__restrict coef)
{
    const int m = blockIdx.y;
    const int n = nbf[m];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * n) return;
    const size_t e = (size_t)off[m] + (size_t)i;
    const double a = coef[4 * m], b = coef[4 * m + 1], c = coef[4 * m + 2], d = coef[4 * m + 3];
    double v = a * x[e];
    if (y) v += b * y[e];
    if (z) v += c * z[e];
    if (i / n == i % n) v += d;
    out[e] = v;
}

// E_m = G_m - G_m^T
__global__ void __launch_bounds__(256) k_bantisym(double *__restrict E, const double *__restrict G,
                                                  const int *__restrict nbf, const long long *__restrict off)
{
    const int m = blockIdx.y;
    const int n = nbf[m];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * n) return;
    const size_t base = (size_t)off[m];
    const int r = (int)(i / n), c = (int)(i % n);
    E[base + i] = G[base + i] - G[base + (size_t)c * n + r];
}

__device__ __forceinline__ double bwsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double bwmax(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double bwmin(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int RB = 256;   // threads per reduction workgroup
constexpr int RCH = 32;   // workgroups (chunks) per molecule in the first pass

// Partial reductions of molecule blockIdx.y, chunk blockIdx.x (ops as in
// fk_scf.hip: 0 sum x*y, 1 max|x|, 2 trace, 3 Gershgorin (min, max) of a
// symmetric block).  part[(m * RCH + chunk) * 2 + {0, 1}].
__global__ void __launch_bounds__(RB) k_breduce1(const double *__restrict x, const double *__restrict y,
                                                 const int *__restrict nbf, const long long *__restrict off, int op,
                                                 double *__restrict part)
{
    __shared__ double s0[RB / 64], s1[RB / 64];
    const int m = blockIdx.y;
    const int n = nbf[m];
    const size_t base = (size_t)off[m];
    double v0 = (op == 3) ? 1e300 : 0.0, v1 = -1e300;
    if (op == 2 || op == 3) {
        for (int r = blockIdx.x * RB + threadIdx.x; r < n; r += RCH * RB) {
            if (op == 2) {
                v0 += x[base + (size_t)r * n + r];
            } else {
                double rad = 0.0;
                for (int k = 0; k < n; ++k) rad += (k == r) ? 0.0 : fabs(x[base + (size_t)k * n + r]);
                const double d = x[base + (size_t)r * n + r];
                v0 = fmin(v0, d - rad);
                v1 = fmax(v1, d + rad);
            }
        }
    } else {
        const long long nn = (long long)n * n;
        for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < nn; i += (long long)RCH * RB) {
            if (op == 0) v0 += x[base + i] * y[base + i];
            else v0 = fmax(v0, fabs(x[base + i]));
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (op == 1) v0 = bwmax(v0);
    else if (op == 3) { v0 = bwmin(v0); v1 = bwmax(v1); }
    else v0 = bwsum(v0);
    if (lane == 0) { s0[w] = v0; s1[w] = v1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = s0[0], b = s1[0];
        for (int k = 1; k < RB / 64; ++k) {
            if (op == 1) a = fmax(a, s0[k]);
            else if (op == 3) { a = fmin(a, s0[k]); b = fmax(b, s1[k]); }
            else a += s0[k];
        }
        part[((size_t)m * RCH + blockIdx.x) * 2] = a;
        part[((size_t)m * RCH + blockIdx.x) * 2 + 1] = b;
    }
}

// out[m] (and out[nmol + m] for op 3) from the chunks, in a fixed order.
__global__ void __launch_bounds__(64) k_breduce2(const double *__restrict part, int nmol, int op,
                                                 double *__restrict out)
{
    const int m = blockIdx.x * 64 + threadIdx.x;
    if (m >= nmol) return;
    const double *p = part + (size_t)m * RCH * 2;
    double a = p[0], b = p[1];
    for (int k = 1; k < RCH; ++k) {
        if (op == 1) a = fmax(a, p[2 * k]);
        else if (op == 3) { a = fmin(a, p[2 * k]); b = fmax(b, p[2 * k + 1]); }
        else a += p[2 * k];
    }
    out[m] = a;
    if (op == 3) out[nmol + m] = b;
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

int fk_scfb_gemm(const double *A, const double *B, double *C, int nmol, int nmax, const int *nbf, const long long *off,
                 double alpha, double beta, void *stream)
{
    if (nmol <= 0 || nmax <= 0) return 0;
    const dim3 grid((nmax + GT - 1) / GT, (nmax + GT - 1) / GT, nmol);
    hipLaunchKernelGGL(k_bgemm, grid, dim3(256), 0, (hipStream_t)stream, A, B, C, nbf, off, alpha, beta);
    return ok();
}

int fk_scfb_lincomb(double *out, const double *x, const double *y, const double *z, int nmol, int nmax, const int *nbf,
                    const long long *off, const double *coef, void *stream)
{
    if (nmol <= 0 || nmax <= 0) return 0;
    const long long nn = (long long)nmax * nmax;
    const dim3 grid((unsigned)((nn + 255) / 256), nmol);
    hipLaunchKernelGGL(k_blincomb, grid, dim3(256), 0, (hipStream_t)stream, out, x, y, z, nbf, off, coef);
    return ok();
}

int fk_scfb_antisym(double *E, const double *G, int nmol, int nmax, const int *nbf, const long long *off, void *stream)
{
    if (nmol <= 0 || nmax <= 0) return 0;
    const long long nn = (long long)nmax * nmax;
    const dim3 grid((unsigned)((nn + 255) / 256), nmol);
    hipLaunchKernelGGL(k_bantisym, grid, dim3(256), 0, (hipStream_t)stream, E, G, nbf, off);
    return ok();
}

// part: fk_scfb_reduce_scratch(nmol) doubles; out: nmol doubles (2 nmol for op 3)
int fk_scfb_reduce(const double *x, const double *y, int nmol, const int *nbf, const long long *off, int op,
                   double *part, double *out, void *stream)
{
    if (nmol <= 0) return 0;
    hipLaunchKernelGGL(k_breduce1, dim3(RCH, nmol), dim3(RB), 0, (hipStream_t)stream, x, y, nbf, off, op, part);
    if (ok()) return -3;
    hipLaunchKernelGGL(k_breduce2, dim3((nmol + 63) / 64), dim3(64), 0, (hipStream_t)stream, part, nmol, op, out);
    return ok();
}

long long fk_scfb_reduce_scratch(int nmol) { return (long long)nmol * RCH * 2; }

}  // extern "C"
