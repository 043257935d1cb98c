// Dense kernels of the SCF step (paper §2.2: F = h + J - K/2, the generalised
// eigenproblem FC = SCe, D = 2 C_occ C_occ^T).
//
// The step is written as dense n x n FP64 products so that no eigensolver is
// needed on the device:
//   * the orthogonaliser X = S^(-1/2) comes from the coupled Newton-Schulz
//     iteration Y <- Y T, Z <- T Z, T = (3I - ZY)/2 (Higham, "Functions of
//     Matrices", 2008, eq. 6.35), started from Y = S/c, Z = I;
//   * the density is the spectral projector onto the N_occ lowest states of
//     F' = X F X, obtained by trace-correcting purification (Niklasson,
//     Phys. Rev. B 66, 155115 (2002)): X0 = (e_max I - F')/(e_max - e_min)
//     with Gershgorin bounds, then X <- X^2 or X <- 2X - X^2, whichever moves
//     the trace towards N_occ, until X is idempotent;
//   * the DIIS error is the commutator F'D' - D'F' in the orthonormal basis.
// The products are rocBLAS dgemm calls from n = 256 on (the LDS-tiled kernel
// below for smaller n and under graph capture).  The density can also come
// from the eigenvectors of F' (rocSOLVER), for bases where purification
// leaves too much occupied-virtual mixing.
// For nearly linearly dependent bases the orthogonaliser can instead be the
// canonical one: S = U s U^T once per geometry (rocSOLVER), X = U f(s) U^T
// with f(s) = s^(-1/2) above a cutoff and 0 below it (eigenvectors dropped).
// All matrices are n x n, row-major, FP64, device resident.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fk_internal.h"

namespace {

// rocBLAS handles of fk_scf_gemm, one per device
constexpr int kBlasDevices = 64;
rocblas_handle g_blas[kBlasDevices] = {};
std::mutex g_blas_mutex;

constexpr int GT = 64;   // output tile (GT x GT) per workgroup
constexpr int GK = 16;   // k-slab staged in LDS
constexpr int GPAD = 1;  // LDS row padding (doubles)

// C = alpha A B + beta C for n x n row-major matrices.  256 threads; thread
// (ty, tx) of a 16 x 16 grid owns the 4 x 4 outputs (ty + 16 i, tx + 16 j).
__global__ void __launch_bounds__(256) k_gemm(const double *__restrict A, const double *__restrict B,
                                              double *__restrict C, int n, double alpha, double beta)
{
    __shared__ double As[GK][GT + GPAD];
    __shared__ double Bs[GK][GT + GPAD];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += GK) {
        // A tile: 64 rows x 16 columns, stored transposed; B tile: 16 rows x 64 columns
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

// out = a x + b y + c z + d I (y, z may be null when b, c are 0); out may
// alias x, y or z (each element is read before it is written)
__global__ void k_lincomb(double *out, const double *x, const double *y, const double *z, int n, double a, double b,
                          double c, double d)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    double v = a * x[i];
    if (y) v += b * y[i];
    if (z) v += c * z[i];
    if (i / n == i % n) v += d;
    out[i] = v;
}

// e = G - G^T
__global__ void k_antisym(double *__restrict e, const double *__restrict G, int n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    const int r = (int)(i / n), c = (int)(i % n);
    e[i] = G[i] - G[(size_t)c * n + r];
}

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmax(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wmin(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int RB = 256;      // threads per reduction block
constexpr int RBLK = 240;    // blocks of the first reduction pass

// Per-block partial results of a reduction over n x n elements:
//   op 0: sum x*y;  op 1: max |x|;  op 2: sum of diagonal of x;
//   op 3: (min, max) Gershgorin bounds of x (two outputs); x must be
//         symmetric: the discs are formed from columns, so that consecutive
//         threads read consecutive addresses.
__global__ void __launch_bounds__(RB) k_reduce1(const double *__restrict x, const double *__restrict y, int n, int op,
                                                double *__restrict part)
{
    __shared__ double s0[RB / 64], s1[RB / 64];
    double v0 = (op == 3) ? 1e300 : 0.0, v1 = -1e300;
    if (op == 2 || op == 3) {
        for (int r = blockIdx.x * RB + threadIdx.x; r < n; r += gridDim.x * RB) {
            if (op == 2) {
                v0 += x[(size_t)r * n + r];
            } else {
                double rad = 0.0;
                for (int k = 0; k < n; ++k) rad += (k == r) ? 0.0 : fabs(x[(size_t)k * n + r]);
                const double d = x[(size_t)r * n + r];
                v0 = fmin(v0, d - rad);
                v1 = fmax(v1, d + rad);
            }
        }
    } else {
        const long long nn = (long long)n * n;
        for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < nn; i += (long long)gridDim.x * RB) {
            if (op == 0) v0 += x[i] * y[i];
            else v0 = fmax(v0, fabs(x[i]));
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (op == 1) v0 = wmax(v0);
    else if (op == 3) { v0 = wmin(v0); v1 = wmax(v1); }
    else v0 = wsum(v0);
    if (lane == 0) { s0[w] = v0; s1[w] = v1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = s0[0], b = s1[0];
        for (int k = 1; k < RB / 64; ++k) {
            if (op == 1) a = fmax(a, s0[k]);
            else if (op == 3) { a = fmin(a, s0[k]); b = fmax(b, s1[k]); }
            else a += s0[k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// Combines the per-block partials into out[slot] (and out[slot + 1] for op 3),
// in a fixed order so results do not depend on timing.
__global__ void k_reduce2(const double *__restrict part, int nblk, int op, double *__restrict out, int slot)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = part[0], b = part[1];
    for (int k = 1; k < nblk; ++k) {
        if (op == 1) a = fmax(a, part[2 * k]);
        else if (op == 3) { a = fmin(a, part[2 * k]); b = fmax(b, part[2 * k + 1]); }
        else a += part[2 * k];
    }
    out[slot] = a;
    if (op == 3) out[slot + 1] = b;
}

// Canonical orthogonaliser pieces.  V holds the eigenvectors of S as rows
// (rocSOLVER's column-major output read row-major), s the eigenvalues:
// out = V^T diag(f(s)), f(s) = s^power for s > cutoff and 0 otherwise, so
// that out V = U f(s) U^T over the kept eigenvectors.
__global__ void k_eig_scale(const double *__restrict V, const double *__restrict s, double *__restrict out, int n,
                            double cutoff, double power)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    const int r = (int)(i / n), c = (int)(i % n);  // out[r][c] = V[c][r] f(s_c)
    const double sv = s[c];
    out[i] = sv > cutoff ? V[(size_t)c * n + r] * pow(sv, power) : 0.0;
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

// C = alpha A B + beta C (row-major, n x n).  From n = 256 on, rocBLAS dgemm
// on the stream (in column-major terms C^T = B^T A^T), with one handle per
// device created on first use and kept for the life of the process; the
// kernel above for smaller n, and while the stream is being captured into a
// graph (the library call may allocate).
int fk_scf_gemm(const double *A, const double *B, double *C, int n, double alpha, double beta, void *stream)
{
    if (n <= 0) return 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusActive;
    int dev = -1;
    if (n >= 256 && cs == hipStreamCaptureStatusNone && hipGetDevice(&dev) == hipSuccess && dev >= 0 &&
        dev < kBlasDevices) {
        std::lock_guard<std::mutex> lock(g_blas_mutex);
        if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success) g_blas[dev] = nullptr;
        rocblas_handle h = g_blas[dev];
        if (h && rocblas_set_stream(h, (hipStream_t)stream) == rocblas_status_success &&
            rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &alpha, B, n, A, n, &beta, C,
                          n) == rocblas_status_success)
            return 0;
    }
    const dim3 grid((n + GT - 1) / GT, (n + GT - 1) / GT);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, (hipStream_t)stream, A, B, C, n, alpha, beta);
    return ok();
}

int fk_scf_lincomb(double *out, const double *x, const double *y, const double *z, int n, double a, double b,
                   double c, double d, void *stream)
{
    const long long nn = (long long)n * n;
    if (nn <= 0) return 0;
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, (hipStream_t)stream, out, x, y,
                       z, n, a, b, c, d);
    return ok();
}

int fk_scf_antisym(double *e, const double *G, int n, void *stream)
{
    const long long nn = (long long)n * n;
    if (nn <= 0) return 0;
    hipLaunchKernelGGL(k_antisym, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, (hipStream_t)stream, e, G, n);
    return ok();
}

// op as in k_reduce1; `part` holds 2 * 240 doubles of scratch; the result goes
// to out[slot] (and out[slot + 1] for op 3) on the device.
int fk_scf_reduce(const double *x, const double *y, int n, int op, double *part, double *out, int slot,
                  void *stream)
{
    if (n <= 0) return 0;
    const long long work = (op == 2 || op == 3) ? n : (long long)n * n;
    const int nblk = (int)std::min<long long>(RBLK, (work + RB - 1) / RB);
    hipLaunchKernelGGL(k_reduce1, dim3(nblk), dim3(RB), 0, (hipStream_t)stream, x, y, n, op, part);
    if (ok()) return -3;
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(64), 0, (hipStream_t)stream, part, nblk, op, out, slot);
    return ok();
}

int fk_scf_reduce_scratch() { return 2 * RBLK; }

int fk_scf_eig_scale(const double *V, const double *s, double *out, int n, double cutoff, double power, void *stream)
{
    const long long nn = (long long)n * n;
    if (nn <= 0) return 0;
    hipLaunchKernelGGL(k_eig_scale, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, (hipStream_t)stream, V, s, out,
                       n, cutoff, power);
    return ok();
}

// Eigen-decomposition of the symmetric n x n device matrix A (overwritten by
// the eigenvectors, rows of the row-major view) with rocSOLVER's divide and
// conquer solver; eigenvalues ascending into w; work holds n doubles, info one
// int (0 on success), all on the device.  Returns 0 or -3.
int fk_scf_eigh(double *A, double *w, double *work, int *info, int n, void *stream)
{
    if (n <= 0) return 0;
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return -3;
    int rc = 0;
    if (rocblas_set_stream(h, (hipStream_t)stream) != rocblas_status_success ||
        rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, A, n, w, work, info) !=
            rocblas_status_success)
        rc = -3;
    // the handle may own workspace the solver still uses: wait before freeing it
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = -3;
    rocblas_destroy_handle(h);
    return rc;
}

}  // extern "C"
