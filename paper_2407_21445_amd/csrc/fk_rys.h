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

// Doubles between consecutive intervals of the n-point segment as staged for
// the kernels: the (RYS_DEG + 1) 2n coefficients padded to 2 mod 16, so that
// lanes reading the same coefficient of different intervals start 16 bytes
// apart modulo 128 bytes and spread over the LDS banks (a multiple of 8 or 16
// doubles would put every interval on the same few banks).
constexpr int rys_stride(int n)
{
    const int d = (RYS_DEG + 1) * 2 * n;
    return d + ((2 - d % 16) + 16) % 16;
}

// T from which the n-point rule is the half-range Gauss-Hermite rule: the
// asymptotic moments Gamma(k+1/2)/(2 T^(k+1/2)) it reproduces differ from
// F_k(T), k < 2n, by e^-T T^(k-1/2)/Gamma(k+1/2) relative, below 3e-15 from
// here on (checked by the generator against 80-digit Boys values).
constexpr double rys_tswitch(int n)
{
    return n == 1 ? RYS_TSWITCH_1 : n == 2 ? RYS_TSWITCH_2 : n == 3 ? RYS_TSWITCH_3 : n == 4 ? RYS_TSWITCH_4
         : n == 5 ? RYS_TSWITCH_5 : n == 6 ? RYS_TSWITCH_6 : RYS_TSWITCH_7;
}

// Intervals of the n-point table: a uniform grid up to the switch for small n,
// the four-region grid up to RYS_TMAX for the others.
constexpr int rys_nint(int n) { return rys_table_nint[n]; }
static_assert(rys_table_nint[1] == (int)(RYS_TSWITCH_1 * RYS_UNI_INVH) &&
              rys_table_nint[RYS_UNI_NMAX] == (int)(RYS_TSWITCH_4 * RYS_UNI_INVH) &&
              rys_table_nint[RYS_UNI_NMAX + 1] == RYS_NINT, "table layout");

// Evaluate the n-point rule at T.  `tab` points at the n-point segment of the
// table ([interval][coefficient][function], intervals rys_stride(n) apart);
// gy2/gw at the n-point Gauss-Hermite data (y_i^2 and h_i) for the region
// tables (the uniform-grid case takes them as constants).  NEED_U = false
// evaluates the weights only (enough when L = 0).
//
// Uniform grid (small n), BRANCHLESS: both rules are evaluated -- a lane
// beyond the switch reads interval 0, which every such lane shares (one LDS
// broadcast) -- and the lane's rule selected, so that the code of a primitive
// quartet is one basic block the compiler can interleave with the next one's
// (at the cost of both results being live at once).  Otherwise the two rules
// are separate branches, so a wave whose lanes all lie beyond the switch
// skips the table and only lanes below it read the LDS.
template <int N, bool NEED_U, bool BRANCHLESS = false>
FK_HD void rys_roots_from(double T, const double *__restrict tab, const double *__restrict gy2,
                          const double *__restrict gw, double *u, double *w)
{
    constexpr int NF = 2 * N;
    static_assert(rys_tswitch(N) <= RYS_TMAX, "the table must cover T below the switch");
    static_assert(RYS_NREG == 4 && RYS_REG1_T0 == 16.0 && RYS_REG1_INVH == 1.0 && RYS_REG3_BASE == 56,
                  "closed-form region selection assumes the generated four-region layout");
    if constexpr (N <= RYS_UNI_NMAX && BRANCHLESS) {
        const bool in_tab = T < rys_tswitch(N);
        const double y = (in_tab ? T : 0.0) * RYS_UNI_INVH;
        const int iv = (int)y;
        const double x = fma(2.0, y - (double)iv, -1.0);
        const double *c = tab + iv * rys_stride(N);
        const double sT = rys_rsqrt(in_tab ? 1.0 : T);
        const double rT = sT * sT;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double vw = c[RYS_DEG * NF + 2 * i + 1];
#pragma unroll
            for (int k = RYS_DEG - 1; k >= 0; --k) vw = vw * x + c[k * NF + 2 * i + 1];
            w[i] = in_tab ? vw : rys_gh_w[gh_offset(N) + i] * sT;
            if constexpr (NEED_U) {
                double vu = c[RYS_DEG * NF + 2 * i];
#pragma unroll
                for (int k = RYS_DEG - 1; k >= 0; --k) vu = vu * x + c[k * NF + 2 * i];
                u[i] = in_tab ? vu : rys_gh_y2[gh_offset(N) + i] * rT;
            }
        }
    } else if (T < rys_tswitch(N)) {
        int iv;
        double x;
        if constexpr (N <= RYS_UNI_NMAX) {
            const double y = T * RYS_UNI_INVH;
            iv = (int)y;
            x = fma(2.0, y - (double)iv, -1.0);
        } else {
            // region k = floor(T/16) (k <= 3) has interval width 2^(k-1) and
            // starts at interval 64 - 2^(6-k)
            int k = (int)(T * (1.0 / 16.0));
            k = k < 3 ? k : 3;
            const double ih = (double)(2 >> k) + (k == 3 ? 0.25 : 0.0) + (k == 2 ? 0.5 : 0.0);
            const double y = (T - 16.0 * k) * ih;
            const int j = (int)y;
            iv = 64 - (64 >> k) + j;
            x = 2.0 * (y - j) - 1.0;
        }
        const double *c = tab + iv * rys_stride(N);
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
    } else {
        const double sT = rys_rsqrt(T);
        const double rT = sT * sT;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if constexpr (NEED_U) u[i] = rys_gh_y2[gh_offset(N) + i] * rT;
            w[i] = rys_gh_w[gh_offset(N) + i] * sT;
        }
    }
}

}  // namespace fk

// Size of one staged n-point table segment and of the segment plus its
// Gauss-Hermite data (y_i^2 then h_i), which is how kernels stage it in LDS.
constexpr int rys_seg_size(int n) { return fk::rys_nint(n) * fk::rys_stride(n); }
constexpr int rys_lds_size(int n) { return rys_seg_size(n) + 2 * n; }

// `tab` holds rys_lds_size(N) doubles: the segment followed by y_i^2 and h_i.
template <int N, bool NEED_U, bool BRANCHLESS = false>
FK_HD void rys_roots(double T, const double *__restrict tab, double *u, double *w)
{
    fk::rys_roots_from<N, NEED_U, BRANCHLESS>(T, tab, tab + rys_seg_size(N), tab + rys_seg_size(N) + N, u, w);
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
            const int d = (RYS_DEG + 1) * 2 * n;
            for (int iv = 0; iv < fk::rys_nint(n); ++iv) {
                const double *src = rys_table_data + rys_table_offset[n - 1] + (size_t)iv * d;
                t.insert(t.end(), src, src + d);
                t.insert(t.end(), fk::rys_stride(n) - d, 0.0);
            }
            for (int i = 0; i < n; ++i) t.push_back(rys_gh_y2[fk::gh_offset(n) + i]);
            for (int i = 0; i < n; ++i) t.push_back(rys_gh_w[fk::gh_offset(n) + i]);
        }
        return t;
    }();
    return v.data();
}
