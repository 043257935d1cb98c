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
                                               const long long *__restrict off, double alpha, double beta,
                                               const int *__restrict skip)
{
    __shared__ double As[GK][GT + GPAD];
    __shared__ double Bs[GK][GT + GPAD];
    const int m = blockIdx.z;
    const int n = nbf[m];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    if (m0 >= n || n0 >= n) return;
    if (skip && skip[m]) return;  // molecule whose product is not needed (whole workgroup)
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

// ---- device-decided SCF iteration (every choice of the host loop made by
// kernels, so that one iteration is a fixed launch sequence a HIP graph can
// replay).  ictl: [0] iterations begun, [1] DIIS ring slot of this
// iteration, [2] filled slots, [3] failure (1 degenerate spectrum, 2
// purification not converged).

__global__ void k_biter_begin(int *ictl, int dn)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int it = ictl[0] + 1;
    ictl[0] = it;
    ictl[1] = (it - 1) % dn;
    ictl[2] = it < dn ? it : dn;
    ictl[3] = 0;
}

// Energies and the per-molecule convergence test (|dE| < e_tol and error <
// g_tol from the second iteration on; a converged molecule stays converged),
// the coefficients that keep a converged molecule's density (keep: a = 0,
// b = 1; else a = 1, b = 0) and the status the host reads: e[m], err[m],
// conv[m] at status[0 .. 3 nmol).
__global__ void k_bconv(const double *__restrict dh, const double *__restrict df, const double *__restrict err,
                        const double *__restrict enuc, int nmol, double e_tol, double g_tol,
                        const int *__restrict ictl, int *__restrict conv, double *__restrict eprev,
                        double *__restrict keep, double *__restrict status)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol) return;
    const double e = 0.5 * (dh[m] + df[m]) + enuc[m];
    if (!conv[m] && ictl[0] > 1 && fabs(e - eprev[m]) < e_tol && err[m] < g_tol) conv[m] = 1;
    eprev[m] = e;
    keep[4 * m] = conv[m] ? 0.0 : 1.0;
    keep[4 * m + 1] = conv[m] ? 1.0 : 0.0;
    keep[4 * m + 2] = 0.0;
    keep[4 * m + 3] = 0.0;
    status[m] = e;
    status[nmol + m] = err[m];
    status[2 * nmol + m] = conv[m];
}

// ring[slot] = src, per molecule block (ring slots nmat apart)
__global__ void __launch_bounds__(256) k_bslot_copy(double *__restrict ring, const double *__restrict src,
                                                    const int *__restrict ictl, const int *__restrict nbf,
                                                    const long long *__restrict off, long long nmat)
{
    const int m = blockIdx.y;
    const int n = nbf[m];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * n) return;
    const size_t e = (size_t)off[m] + (size_t)i;
    ring[(size_t)ictl[1] * nmat + e] = src[e];
}

// Partial inner products of this iteration's error (ring slot ictl[1]) with
// every slot j = blockIdx.z, chunk blockIdx.x of molecule blockIdx.y.
__global__ void __launch_bounds__(RB) k_bdots(const double *__restrict ring, const int *__restrict ictl,
                                              const int *__restrict nbf, const long long *__restrict off,
                                              long long nmat, double *__restrict part)
{
    __shared__ double s0[RB / 64];
    const int m = blockIdx.y, j = blockIdx.z;
    const int n = nbf[m];
    const int dn = gridDim.z;
    const double *x = ring + (size_t)ictl[1] * nmat + off[m];
    const double *y = ring + (size_t)j * nmat + off[m];
    double v = 0.0;
    for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < (long long)n * n; i += (long long)RCH * RB)
        v += x[i] * y[i];
    v = bwsum(v);
    if ((threadIdx.x & 63) == 0) s0[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = s0[0];
        for (int k = 1; k < RB / 64; ++k) a += s0[k];
        part[((size_t)m * dn + j) * RCH + blockIdx.x] = a;
    }
}

// Per molecule: the new row of the DIIS inner products B (in a fixed order
// of the chunks), then the Pulay coefficients of the filled slots from
// [B 1; 1 0] [c; l] = [0; 1] (Gaussian elimination with partial pivoting on
// B scaled by its largest diagonal); the newest slot alone when fewer than
// two are filled or the system is singular.
__global__ void k_bdiis(const double *__restrict part, int nmol, int dn, const int *__restrict ictl,
                        double *__restrict Bm, double *__restrict dcoef)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol) return;
    const int k = ictl[1], nf = ictl[2];
    double *B = Bm + (size_t)m * dn * dn;
    for (int j = 0; j < dn; ++j) {
        double d = 0.0;
        for (int c = 0; c < RCH; ++c) d += part[((size_t)m * dn + j) * RCH + c];
        B[k * dn + j] = d;
        B[j * dn + k] = d;
    }
    double *cf = dcoef + (size_t)m * dn;
    for (int j = 0; j < dn; ++j) cf[j] = 0.0;
    cf[k] = 1.0;
    if (nf < 2) return;
    constexpr int KM = FK_SCFB_MAX_DIIS + 1;
    double A[KM][KM + 1];
    const int kk = nf + 1;
    double bmax = 0.0;
    for (int i = 0; i < nf; ++i) bmax = fmax(bmax, fabs(B[i * dn + i]));
    if (!(bmax > 0)) return;
    for (int i = 0; i < kk; ++i)
        for (int j = 0; j <= kk; ++j) A[i][j] = 0.0;
    for (int i = 0; i < nf; ++i) {
        for (int j = 0; j < nf; ++j) A[i][j] = B[i * dn + j] / bmax;
        A[i][nf] = 1.0;
        A[nf][i] = 1.0;
    }
    A[nf][kk] = 1.0;
    for (int col = 0; col < kk; ++col) {
        int piv = col;
        for (int r = col + 1; r < kk; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (fabs(A[piv][col]) < 1e-300) return;
        if (piv != col)
            for (int j = 0; j <= kk; ++j) {
                const double t = A[col][j];
                A[col][j] = A[piv][j];
                A[piv][j] = t;
            }
        for (int r = 0; r < kk; ++r) {
            if (r == col) continue;
            const double f = A[r][col] / A[col][col];
            for (int j = col; j <= kk; ++j) A[r][j] -= f * A[col][j];
        }
    }
    double c[KM];
    for (int i = 0; i < nf; ++i) {
        c[i] = A[i][kk] / A[i][i];
        if (!isfinite(c[i])) return;
    }
    for (int i = 0; i < nf; ++i) cf[i] = c[i];
}

// Fo_m = sum over the filled slots j of dcoef[m][j] ringF[j]
__global__ void __launch_bounds__(256) k_bcombine(double *__restrict Fo, const double *__restrict ring,
                                                  const double *__restrict dcoef, int dn, const int *__restrict ictl,
                                                  const int *__restrict nbf, const long long *__restrict off,
                                                  long long nmat)
{
    const int m = blockIdx.y;
    const int n = nbf[m];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * n) return;
    const size_t e = (size_t)off[m] + (size_t)i;
    const int nf = ictl[2];
    double v = 0.0;
    for (int j = 0; j < nf; ++j) v += dcoef[(size_t)m * dn + j] * ring[(size_t)j * nmat + e];
    Fo[e] = v;
}

// Purification start: P0 = (hi I - F')/(hi - lo) from the Gershgorin bounds
// (gb[m], gb[nmol + m]); a degenerate spectrum sets the failure flag.
__global__ void k_bpur_start(const double *__restrict gb, int nmol, double *__restrict coef, int *__restrict pstate,
                             int *__restrict pdone, int *__restrict ictl)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol) return;
    const double lo = gb[m], hi = gb[nmol + m];
    const bool okb = hi > lo;
    if (!okb) atomicMax(&ictl[3], 1);
    coef[4 * m] = okb ? -1.0 / (hi - lo) : 0.0;
    coef[4 * m + 1] = 0.0;
    coef[4 * m + 2] = 0.0;
    coef[4 * m + 3] = okb ? hi / (hi - lo) : 0.0;
    pstate[m] = -1;
    pdone[m] = 0;
}

// One trace-correcting step per molecule from t1 = tr P, t2 = tr P^2: the
// host loop's choice (P^2 or 2P - P^2, whichever moves the trace towards
// nocc; two more steps after sum x(1 - x) < 1e-11; then P is kept).
__global__ void k_bpur_step(const double *__restrict t1, const double *__restrict t2, const int *__restrict nocc,
                            int nmol, double *__restrict coef, int *__restrict pstate, int *__restrict pdone)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol) return;
    double a = 1.0, b = 0.0;
    int ex = pstate[m];
    if (ex != 0) {
        if (ex < 0 && fabs(t1[m] - t2[m]) < 1e-11) ex = 2;
        if (ex != 0) {
            if (ex > 0) --ex;
            if (fabs(t2[m] - nocc[m]) < fabs(2 * t1[m] - t2[m] - nocc[m])) { a = 0.0; b = 1.0; }
            else { a = 2.0; b = -1.0; }
        }
    }
    pstate[m] = ex;
    pdone[m] = ex == 0 ? 1 : 0;
    coef[4 * m] = a;
    coef[4 * m + 1] = b;
    coef[4 * m + 2] = 0.0;
    coef[4 * m + 3] = 0.0;
}

__global__ void k_bpur_check(const int *__restrict pstate, int nmol, int *__restrict ictl)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nmol && pstate[m] != 0) atomicMax(&ictl[3], 2);
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

int fk_scfb_gemm(const double *A, const double *B, double *C, int nmol, int nmax, const int *nbf, const long long *off,
                 double alpha, double beta, void *stream)
{
    if (nmol <= 0 || nmax <= 0) return 0;
    const dim3 grid((nmax + GT - 1) / GT, (nmax + GT - 1) / GT, nmol);
    hipLaunchKernelGGL(k_bgemm, grid, dim3(256), 0, (hipStream_t)stream, A, B, C, nbf, off, alpha, beta,
                       (const int *)nullptr);
    return ok();
}

int fk_scfb_gemm_skip(const double *A, const double *B, double *C, int nmol, int nmax, const int *nbf,
                      const long long *off, const int *skip, void *stream)
{
    if (nmol <= 0 || nmax <= 0) return 0;
    const dim3 grid((nmax + GT - 1) / GT, (nmax + GT - 1) / GT, nmol);
    hipLaunchKernelGGL(k_bgemm, grid, dim3(256), 0, (hipStream_t)stream, A, B, C, nbf, off, 1.0, 0.0, skip);
    return ok();
}

int fk_scfb_iter_begin(int *ictl, int dn, void *stream)
{
    hipLaunchKernelGGL(k_biter_begin, dim3(1), dim3(1), 0, (hipStream_t)stream, ictl, dn);
    return ok();
}

int fk_scfb_conv(const double *dh, const double *df, const double *err, const double *enuc, int nmol, double e_tol,
                 double g_tol, const int *ictl, int *conv, double *eprev, double *keep, double *status, void *stream)
{
    hipLaunchKernelGGL(k_bconv, dim3((nmol + 63) / 64), dim3(64), 0, (hipStream_t)stream, dh, df, err, enuc, nmol,
                       e_tol, g_tol, ictl, conv, eprev, keep, status);
    return ok();
}

int fk_scfb_diis(double *ringF, double *ringE, const double *Fo, const double *E, double *Fo_out, int nmol, int nmax,
                 const int *nbf, const long long *off, long long nmat, int dn, const int *ictl, double *part,
                 double *Bm, double *dcoef, void *stream)
{
    if (dn > FK_SCFB_MAX_DIIS) return -1;
    hipStream_t st = (hipStream_t)stream;
    const long long nn = (long long)nmax * nmax;
    const dim3 g2((unsigned)((nn + 255) / 256), nmol);
    hipLaunchKernelGGL(k_bslot_copy, g2, dim3(256), 0, st, ringF, Fo, ictl, nbf, off, nmat);
    hipLaunchKernelGGL(k_bslot_copy, g2, dim3(256), 0, st, ringE, E, ictl, nbf, off, nmat);
    hipLaunchKernelGGL(k_bdots, dim3(RCH, nmol, dn), dim3(RB), 0, st, (const double *)ringE, ictl, nbf, off, nmat, part);
    hipLaunchKernelGGL(k_bdiis, dim3((nmol + 63) / 64), dim3(64), 0, st, (const double *)part, nmol, dn, ictl, Bm, dcoef);
    hipLaunchKernelGGL(k_bcombine, g2, dim3(256), 0, st, Fo_out, (const double *)ringF, (const double *)dcoef, dn, ictl,
                       nbf, off, nmat);
    return ok();
}

int fk_scfb_pur_start(const double *gb, int nmol, double *coef, int *pstate, int *pdone, int *ictl, void *stream)
{
    hipLaunchKernelGGL(k_bpur_start, dim3((nmol + 63) / 64), dim3(64), 0, (hipStream_t)stream, gb, nmol, coef, pstate,
                       pdone, ictl);
    return ok();
}

int fk_scfb_pur_step(const double *t1, const double *t2, const int *nocc, int nmol, double *coef, int *pstate,
                     int *pdone, void *stream)
{
    hipLaunchKernelGGL(k_bpur_step, dim3((nmol + 63) / 64), dim3(64), 0, (hipStream_t)stream, t1, t2, nocc, nmol, coef,
                       pstate, pdone);
    return ok();
}

int fk_scfb_pur_check(const int *pstate, int nmol, int *ictl, void *stream)
{
    hipLaunchKernelGGL(k_bpur_check, dim3((nmol + 63) / 64), dim3(64), 0, (hipStream_t)stream, pstate, nmol, ictl);
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
