"""Generator of the Rys quadrature tables used by the ERI kernels.

The n-point Rys rule for a primitive quartet with argument T is the Gauss rule
of the weight exp(-T t^2) on t in [0, 1], written in the variable u = t^2:
    sum_i w_i u_i^k = F_k(T) = int_0^1 t^(2k) exp(-T t^2) dt,  k < 2n,
where F_k is the Boys function of the paper's auxiliary integrals.  The paper
gives no algorithm for the roots and weights; they are computed here from the
moments F_k(T) in 80-digit arithmetic (mpmath) by the modified Chebyshev
algorithm (Gautschi, Orthogonal Polynomials, 2004, sec. 2.1.7) and the
Golub-Welsch eigenvalue method, then fitted per T interval by Chebyshev
interpolation.  Above T_max the rule is the half-range Gauss-Hermite rule
u_i = y_i^2 / T, w_i = h_i / sqrt(T) (y_i > 0 the roots of H_{2n}).

Output: ``rys_table.inc`` with, for every n = 1..RYS_NMAX, coefficients laid
out [interval][coefficient][function], function 2i = u_i and 2i+1 = w_i, in
the monomial basis of x = 2 (T - T_lo)/h - 1 (Horner evaluation).

Intervals: for n <= UNI_NMAX a uniform grid of width UNI_H from 0 up to the
switch T_s(n) to the Gauss-Hermite rule (the interval of T is then a single
multiply and truncation); for larger n, whose tables would not fit the LDS
on a uniform grid, four regions of doubling width up to TMAX.  T_s(n) is the
smallest integer T from which the Gauss-Hermite moments agree with F_k(T),
k < 2n, to 3e-15 relative (64 at most).
"""
from __future__ import annotations

import argparse
import math
import os
import sys

import mpmath as mp

NMAX = 7
# (start of region, interval width); the last region ends at TMAX
REGIONS = [(0.0, 0.5), (16.0, 1.0), (32.0, 2.0), (48.0, 4.0)]
TMAX = 64.0          # end of the region tables
DEG = 9              # polynomial degree per interval
UNI_NMAX = 4         # n up to this: uniform grid
UNI_H = 0.5          # its interval width
TSWITCH = {1: 36.0, 2: 42.0, 3: 47.0, 4: 52.0, 5: 57.0, 6: 61.0, 7: 64.0}


def tswitch_check(n, T):
    """Largest relative difference between the Gauss-Hermite (asymptotic)
    moments and F_k(T), k < 2n."""
    mom = moments(T, 2 * n)
    T = mp.mpf(T)
    return max(abs(mp.gamma(k + mp.mpf(1) / 2) / (2 * T ** (k + mp.mpf(1) / 2)) - mom[k]) / mom[k]
               for k in range(2 * n))


def moments(T, kmax):
    T = mp.mpf(T)
    if T == 0:
        return [mp.mpf(1) / (2 * k + 1) for k in range(kmax + 1)]
    return [mp.gammainc(k + mp.mpf(1) / 2, 0, T) / (2 * T ** (k + mp.mpf(1) / 2)) for k in range(kmax + 1)]


def gauss_rule(mom, n):
    """Nodes/weights of the n-point Gauss rule from ordinary moments."""
    sig_prev = [mp.mpf(0)] * (2 * n)
    sig = list(mom[:2 * n])
    alpha = [mom[1] / mom[0]]
    beta = [mom[0]]
    for k in range(1, n):
        new = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_prev[l]
        alpha.append(new[k + 1] / new[k] - sig[k] / sig[k - 1])
        beta.append(new[k] / sig[k - 1])
        sig_prev, sig = sig, new
    Jm = mp.matrix(n, n)
    for i in range(n):
        Jm[i, i] = alpha[i]
        if i + 1 < n:
            Jm[i, i + 1] = Jm[i + 1, i] = mp.sqrt(beta[i + 1])
    E, Q = mp.eigsy(Jm)
    pairs = sorted((E[i], beta[0] * Q[0, i] ** 2) for i in range(n))
    return [p[0] for p in pairs], [p[1] for p in pairs]


def rule(T, n):
    return gauss_rule(moments(T, 2 * n), n)


def cheb_fit(fvals, deg):
    """Chebyshev coefficients from values at the Chebyshev-Gauss nodes."""
    N = deg + 1
    c = []
    for k in range(N):
        s = mp.fsum(fvals[j] * mp.cos(mp.pi * k * (j + mp.mpf(1) / 2) / N) for j in range(N))
        c.append(2 * s / N)
    c[0] /= 2
    return c


def cheb_to_mono(c):
    """Chebyshev series -> monomial coefficients (exact in mp arithmetic)."""
    N = len(c)
    Tk = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for k in range(2, N):
        a = [mp.mpf(0)] + [2 * x for x in Tk[k - 1]]
        b = Tk[k - 2] + [mp.mpf(0)] * (len(a) - len(Tk[k - 2]))
        Tk.append([x - y for x, y in zip(a, b)])
    mono = [mp.mpf(0)] * N
    for k in range(N):
        for i, v in enumerate(Tk[k]):
            mono[i] += c[k] * v
    return mono


def nodes(lo, h, deg):
    N = deg + 1
    xs = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / N) for j in range(N)]
    return xs, [lo + (x + 1) * h / 2 for x in xs]


def gauss_hermite_half(n):
    """Positive nodes y_i and weights h_i of the 2n-point Gauss-Hermite rule."""
    ys, ws = [], []
    # roots of H_{2n} via the Golub-Welsch matrix of the Hermite recurrence
    m = 2 * n
    Jm = mp.matrix(m, m)
    for i in range(m - 1):
        Jm[i, i + 1] = Jm[i + 1, i] = mp.sqrt(mp.mpf(i + 1) / 2)
    E, Q = mp.eigsy(Jm)
    for i in range(m):
        if E[i] > 0:
            ys.append(E[i])
            ws.append(mp.sqrt(mp.pi) * Q[0, i] ** 2)
    pairs = sorted(zip(ys, ws))
    return [p[0] for p in pairs], [p[1] for p in pairs]


def intervals():
    """(T_lo, width) of every interval of the region tables, region by region."""
    out = []
    ends = [r[0] for r in REGIONS[1:]] + [TMAX]
    for (t0, h), t1 in zip(REGIONS, ends):
        for i in range(int(round((t1 - t0) / h))):
            out.append((t0 + i * h, h))
    return out


def intervals_n(n):
    """(T_lo, width) of the intervals of the n-point table."""
    if n <= UNI_NMAX:
        return [(i * UNI_H, UNI_H) for i in range(int(round(TSWITCH[n] / UNI_H)))]
    return intervals()


def build_tables(nmax=NMAX, deg=DEG, progress=False):
    mp.mp.dps = 80
    for n in range(1, nmax + 1):
        assert tswitch_check(n, TSWITCH[n]) < 3e-15 or TSWITCH[n] == TMAX, n
    # every distinct interval once, with the rules of the n that use it
    users = {}
    for n in range(1, nmax + 1):
        for iv in intervals_n(n):
            users.setdefault(iv, []).append(n)
    rules = {}
    for it, ((lo, h), ns) in enumerate(sorted(users.items())):
        xs, Ts = nodes(mp.mpf(lo), mp.mpf(h), deg)
        vals = {n: [[] for _ in range(2 * n)] for n in ns}
        for T in Ts:
            mom = moments(T, 2 * max(ns))
            for n in ns:
                u, w = gauss_rule(mom, n)
                for i in range(n):
                    vals[n][2 * i].append(u[i])
                    vals[n][2 * i + 1].append(w[i])
        for n in ns:
            rules[(n, lo, h)] = [cheb_to_mono(cheb_fit(vals[n][f], deg)) for f in range(2 * n)]
        if progress:
            print(f"interval {it + 1}/{len(users)}", file=sys.stderr, flush=True)
    tabs = {n: [rules[(n, lo, h)] for lo, h in intervals_n(n)] for n in range(1, nmax + 1)}
    gh = {n: gauss_hermite_half(n) for n in range(1, nmax + 1)}
    return tabs, gh


def write_inc(path, tabs, gh, nmax=NMAX, deg=DEG):
    nint = len(intervals())
    L = []
    L.append("/* Generated by gen_rys_table.py -- do not edit.  Rys roots u_i and weights w_i")
    L.append(" * of the n-point rule for exp(-T t^2) on [0,1] in u = t^2, as degree-RYS_DEG")
    L.append(" * polynomials in x = 2 (T - T_lo)/h - 1 per interval of T below the switch")
    L.append(" * RYS_TSWITCH_n.  n <= RYS_UNI_NMAX: uniform intervals of width 1/RYS_UNI_INVH from")
    L.append(" * 0 (rys_table_nint[n] of them); larger n: region r starts at RYS_REGr_T0 with width")
    L.append(" * 1/RYS_REGr_INVH, its first interval has index RYS_REGr_BASE (RYS_NINT in all).")
    L.append(" * layout [interval][coefficient][function], function 2i = u_i, 2i+1 = w_i.")
    L.append(" * From the switch on: u_i = y_i^2/T, w_i = h_i/sqrt(T) (half-range Gauss-Hermite). */")
    L.append(f"#define RYS_NMAX {nmax}")
    L.append(f"#define RYS_NREG {len(REGIONS)}")
    L.append(f"#define RYS_TMAX {TMAX!r}")
    L.append(f"#define RYS_UNI_NMAX {UNI_NMAX}")
    L.append(f"#define RYS_UNI_INVH {1.0 / UNI_H!r}")
    for n in range(1, nmax + 1):
        L.append(f"#define RYS_TSWITCH_{n} {TSWITCH[n]!r}")
    L.append("static constexpr int rys_table_nint[RYS_NMAX + 1] = {0, " +
             ", ".join(str(len(tabs[n])) for n in range(1, nmax + 1)) + "};")
    bases, b = [], 0
    ends = [r[0] for r in REGIONS[1:]] + [TMAX]
    for (t0, h), t1 in zip(REGIONS, ends):
        bases.append(b)
        b += int(round((t1 - t0) / h))
    for r, ((t0, h), base) in enumerate(zip(REGIONS, bases)):
        L.append(f"#define RYS_REG{r}_T0 {t0!r}")
        L.append(f"#define RYS_REG{r}_INVH {1.0 / h!r}")
        L.append(f"#define RYS_REG{r}_BASE {base}")
    L.append(f"#define RYS_NINT {nint}")
    L.append(f"#define RYS_DEG {deg}")
    offs = []
    o = 0
    for n in range(1, nmax + 1):
        offs.append(o)
        o += len(tabs[n]) * (deg + 1) * 2 * n
    L.append(f"#define RYS_TABLE_SIZE {o}")
    L.append("static const int rys_table_offset[RYS_NMAX + 1] = {" + ", ".join(str(x) for x in offs) + f", {o}}};")
    L.append("static const double rys_table_data[RYS_TABLE_SIZE] = {")
    for n in range(1, nmax + 1):
        for it in range(len(tabs[n])):
            for k in range(deg + 1):
                row = ", ".join(mp.nstr(tabs[n][it][f][k], 17, min_fixed=1, max_fixed=0) for f in range(2 * n))
                L.append("  " + row + ",")
    L.append("};")
    ys, ws = [], []
    for n in range(1, nmax + 1):
        y, w = gh[n]
        ys += [mp.nstr(v * v, 17, min_fixed=1, max_fixed=0) for v in y]   # y_i^2
        ws += [mp.nstr(v, 17, min_fixed=1, max_fixed=0) for v in w]
    L.append("/* half-range Gauss-Hermite: y_i^2 and h_i, n = 1..RYS_NMAX concatenated */")
    L.append("static constexpr double rys_gh_y2[" + str(len(ys)) + "] = {" + ", ".join(ys) + "};")
    L.append("static constexpr double rys_gh_w[" + str(len(ws)) + "] = {" + ", ".join(ws) + "};")
    with open(path, "w") as f:
        f.write("\n".join(L) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "rys_table.inc"))
    args = ap.parse_args()
    tabs, gh = build_tables(progress=True)
    write_inc(args.out, tabs, gh)


if __name__ == "__main__":
    main()
