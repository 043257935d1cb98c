// Rys quadrature roots and weights from the generated piecewise-polynomial
// tables (see gen_rys_table.py for how the tables are made).
//
// The n-point rule reproduces the Boys-function moments
// sum_r w_r u_r^k = F_k(T), k < 2n, of the paper's auxiliary integrals
// (eq. boys-fn-def), which is what lets a product of three 1-D factors per root
// stand in for the m-indexed auxiliary integrals of the vertical recurrences.
#pragma once

#include <math.h>

#include <vector>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FK_HD __host__ __device__ __forceinline__
#else
#define FK_HD inline
#endif

#include "rys_table.inc"

namespace fk {

// offset of the n-point rule in the half-range Gauss-Hermite arrays
constexpr int gh_offset(int n) { return n * (n - 1) / 2; }

struct GHConst {
    double y2[28], w[28];
};

// 1/sqrt(x) for x > 0: on the device the hardware estimate refined by two
// Newton steps y <- y (3 - x y^2)/2 (each doubles the correct bits).
FK_HD double rys_rsqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
#else
    return 1.0 / sqrt(x);
#endif
}

// Evaluate the n-point rule at T.  `tab` points at the n-point segment of the
// table ([interval][coefficient][function]); gy2/gw at the n-point
// Gauss-Hermite data (y_i^2 and h_i).  NEED_U = false evaluates the weights
// only (enough when L = 0).
template <int N, bool NEED_U>
FK_HD void rys_roots_from(double T, const double *__restrict tab, const double *__restrict gy2,
                          const double *__restrict gw, double *u, double *w)
{
    constexpr int NF = 2 * N;
    // table path, evaluated at T clamped into the table's range.  Region k =
    // floor(T/16) (k <= 3) has interval width 2^(k-1) and starts at interval
    // 64 - 2^(6-k).
    const double Tc = T < RYS_TMAX ? T : 0.0;
    static_assert(RYS_NREG == 4 && RYS_REG1_T0 == 16.0 && RYS_REG1_INVH == 1.0 && RYS_REG3_BASE == 56,
                  "closed-form region selection assumes the generated four-region layout");
    int k = (int)(Tc * (1.0 / 16.0));
    k = k < 3 ? k : 3;
    const double ih = (double)(2 >> k) + (k == 3 ? 0.25 : 0.0) + (k == 2 ? 0.5 : 0.0);
    const double y = (Tc - 16.0 * k) * ih;
    const int j = (int)y;
    const int iv = 64 - (64 >> k) + j;
    const double x = 2.0 * (y - j) - 1.0;
    const double *c = tab + iv * ((RYS_DEG + 1) * NF);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double vw = c[RYS_DEG * NF + 2 * i + 1];
#pragma unroll
        for (int k = RYS_DEG - 1; k >= 0; --k) vw = vw * x + c[k * NF + 2 * i + 1];
        w[i] = vw;
        if constexpr (NEED_U) {
            double vu = c[RYS_DEG * NF + 2 * i];
#pragma unroll
            for (int k = RYS_DEG - 1; k >= 0; --k) vu = vu * x + c[k * NF + 2 * i];
            u[i] = vu;
        }
    }
    // half-range Gauss-Hermite rule beyond the table
    if (T >= RYS_TMAX) {
        const double sT = rys_rsqrt(T);
        const double rT = sT * sT;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if constexpr (NEED_U) u[i] = gy2[i] * rT;
            w[i] = gw[i] * sT;
        }
    }
}

}  // namespace fk

// Size of one n-point table segment and of the segment plus its
// Gauss-Hermite data (y_i^2 then h_i), which is how kernels stage it in LDS.
constexpr int rys_seg_size(int n) { return RYS_NINT * (RYS_DEG + 1) * 2 * n; }
constexpr int rys_lds_size(int n) { return rys_seg_size(n) + 2 * n; }

// `tab` holds rys_lds_size(N) doubles: the segment followed by y_i^2 and h_i.
template <int N, bool NEED_U>
FK_HD void rys_roots(double T, const double *__restrict tab, double *u, double *w)
{
    fk::rys_roots_from<N, NEED_U>(T, tab, tab + rys_seg_size(N), tab + rys_seg_size(N) + N, u, w);
}

constexpr int rys_staged_offset(int n)
{
    int o = 0;
    for (int m = 1; m < n; ++m) o += rys_lds_size(m);
    return o;
}
constexpr int rys_staged_total() { return rys_staged_offset(RYS_NMAX + 1); }

// Host copy of every n-point segment followed by its Gauss-Hermite data, the
// layout uploaded to the device and staged into LDS by the kernels.
inline const double *rys_staged_host()
{
    static const std::vector<double> v = [] {
        std::vector<double> t;
        t.reserve(rys_staged_total());
        for (int n = 1; n <= RYS_NMAX; ++n) {
            t.insert(t.end(), rys_table_data + rys_table_offset[n - 1], rys_table_data + rys_table_offset[n]);
            for (int i = 0; i < n; ++i) t.push_back(rys_gh_y2[fk::gh_offset(n) + i]);
            for (int i = 0; i < n; ++i) t.push_back(rys_gh_w[fk::gh_offset(n) + i]);
        }
        return t;
    }();
    return v.data();
}
