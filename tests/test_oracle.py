"""Pins of the CPU oracle against facts that do not come from the oracle:
closed forms, an arbitrary-precision Boys function, quadrature, calculus,
brute-force sums, a textbook energy, and invariants of the method.  Each test
names what a plausible mistake would break."""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.special import erf, hyp1f1

import oracle
from oracle.scf import run_scf
from synth import geometry as geom
from synth import workloads as wl
from synth.workloads import flatten

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sys(atoms, shells, Z=None):
    mol = {"Z": np.array(Z if Z is not None else [1] * len(atoms), dtype=np.int32),
           "xyz": np.array(atoms, dtype=np.float64), "charge": 0, "name": "t"}
    return flatten(mol, shells)


def _rand_sys(seed, lmax=3, natom=4, kmax=2):
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(-1.5, 1.5, size=(natom, 3))
    shells = []
    for a in range(natom):
        for l in range(lmax + 1):
            k = int(rng.integers(1, kmax + 1))
            shells.append({"atom": a, "l": l, "exps": list(rng.uniform(0.2, 3.0, size=k)),
                           "coefs": list(rng.uniform(0.3, 1.0, size=k))})
    return _sys(atoms, shells)


# ------------------------------------------------------------- Boys ---------
@pytest.mark.parametrize("m", range(0, 13))
def test_boys_zero(m):
    assert oracle.boys(m, 0.0)[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)


def test_boys_vs_mpmath():
    """F_m(T) = gamma(m+1/2, T) / (2 T^(m+1/2)), 30 significant digits."""
    mpmath.mp.dps = 30
    worst = 0.0
    for T in [1e-6, 1e-3, 0.1, 0.7, 2.5, 7.0, 15.0, 30.0, 34.99, 35.01, 40.0, 60.0, 120.0]:
        F = oracle.boys(12, T)
        for m in range(13):
            ref = mpmath.gammainc(m + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (m + 0.5))
            worst = max(worst, abs(F[m] - float(ref)) / float(ref))
    assert worst < 5e-14


def test_boys_erf_and_hyp1f1():
    for T in np.linspace(0.05, 34.0, 40):
        F = oracle.boys(6, T)
        assert F[0] == pytest.approx(0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T)), rel=1e-13)
        for m in range(7):
            assert F[m] == pytest.approx(hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1), rel=1e-11)


def test_boys_downward_identity():
    for T in [0.3, 5.0, 33.0, 36.0, 80.0]:
        F = oracle.boys(10, T)
        for m in range(10):
            assert 2 * T * F[m + 1] == pytest.approx((2 * m + 1) * F[m] - math.exp(-T), rel=1e-12, abs=1e-300)


# ------------------------------------------------------ ERI closed forms ----
@pytest.mark.parametrize("a,b,R", [(0.7, 1.3, 1.1), (2.0, 0.15, 3.7), (0.5, 0.5, 0.0), (5.0, 0.9, 0.4)])
def test_ssss_closed_form(a, b, R):
    """(aa|bb) of single normalised s primitives is the Coulomb energy of two
    normalised Gaussian charges: erf(sqrt(rho) R)/R, rho = 2a 2b/(2a+2b)."""
    s = _sys([[0, 0, 0], [0, 0, R]], [{"atom": 0, "l": 0, "exps": [a], "coefs": [1.0]},
                                      {"atom": 1, "l": 0, "exps": [b], "coefs": [1.0]}])
    v = oracle.eri_quartet(s, 0, 0, 1, 1)[0, 0, 0, 0]
    rho = (2 * a) * (2 * b) / (2 * a + 2 * b)
    ref = 2 * math.sqrt(rho / math.pi) if R == 0 else erf(math.sqrt(rho) * R) / R
    assert v == pytest.approx(ref, rel=1e-13)
    assert oracle.eri_quartet(s, 0, 0, 1, 1, method="os")[0, 0, 0, 0] == pytest.approx(ref, rel=1e-13)


def test_p_function_is_centre_derivative_of_s():
    """For normalised primitives p_x = a^(-1/2) d/dA_x s (Boys' derivative
    formula); check (p s|s s) against a 4-point finite difference of (s s|s s)."""
    rng = np.random.default_rng(7)
    atoms = rng.uniform(-1.0, 1.0, size=(4, 3))
    ex = [0.9, 0.6, 1.4, 0.35]

    def ssss(shift):
        at = atoms.copy()
        at[0, 0] += shift
        s = _sys(at, [{"atom": i, "l": 0, "exps": [ex[i]], "coefs": [1.0]} for i in range(4)])
        return oracle.eri_quartet(s, 0, 1, 2, 3)[0, 0, 0, 0]

    h = 1e-3
    fd = (-ssss(2 * h) + 8 * ssss(h) - 8 * ssss(-h) + ssss(-2 * h)) / (12 * h)
    sp = _sys(atoms, [{"atom": 0, "l": 1, "exps": [ex[0]], "coefs": [1.0]}] +
              [{"atom": i, "l": 0, "exps": [ex[i]], "coefs": [1.0]} for i in range(1, 4)])
    v = oracle.eri_quartet(sp, 0, 1, 2, 3)[0, 0, 0, 0]
    assert v == pytest.approx(fd / math.sqrt(ex[0]), rel=1e-8)


# ------------------------------------------------- recurrences agree --------
@pytest.mark.parametrize("seed", range(6))
def test_mmd_equals_os(seed):
    """Two different recurrence schemes (Hermite/MMD and OS VRR + HRR) agree up
    to (ff|ff); pins the garbled prefactors and the vrr2 sign reading."""
    s = _rand_sys(100 + seed)
    rng = np.random.default_rng(seed)
    for _ in range(8):
        q = rng.integers(0, s["nshell"], size=4)
        a = oracle.eri_quartet(s, *q, method="mmd")
        b = oracle.eri_quartet(s, *q, method="os")
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(a)))
    q = (3, 7, 11, 15)  # (ff|ff)
    a = oracle.eri_quartet(s, *q)
    b = oracle.eri_quartet(s, *q, method="os")
    assert a.shape == (10, 10, 10, 10)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(a)))


def test_eightfold_symmetry_and_schwarz():
    s = _rand_sys(5)
    rng = np.random.default_rng(3)
    for _ in range(10):
        a, b, c, d = (int(x) for x in rng.integers(0, s["nshell"], size=4))
        v = oracle.eri_quartet(s, a, b, c, d)
        assert np.allclose(oracle.eri_quartet(s, b, a, c, d), v.transpose(1, 0, 2, 3), rtol=1e-12, atol=1e-15)
        assert np.allclose(oracle.eri_quartet(s, a, b, d, c), v.transpose(0, 1, 3, 2), rtol=1e-12, atol=1e-15)
        assert np.allclose(oracle.eri_quartet(s, c, d, a, b), v.transpose(2, 3, 0, 1), rtol=1e-12, atol=1e-15)
        vab = oracle.eri_quartet(s, a, b, a, b)
        vcd = oracle.eri_quartet(s, c, d, c, d)
        gab = np.sqrt(np.einsum("ijij->ij", vab))
        gcd = np.sqrt(np.einsum("klkl->kl", vcd))
        assert np.all(np.abs(v) <= gab[:, :, None, None] * gcd[None, None, :, :] * (1 + 1e-12) + 1e-300)


def test_pppp_has_81_integrals_and_dd_hermite_sparsity():
    s = _rand_sys(9, lmax=1)
    assert oracle.eri_quartet(s, 1, 3, 5, 7).size == 81
    assert oracle.hermite_nnz(2, 2) == (1260, 336)


# ---------------------------------------------------- one-electron pins -----
def _gh_overlap_1d(i, j, a, b, A, B, n=30):
    x, w = np.polynomial.hermite.hermgauss(n)
    p = a + b
    P = (a * A + b * B) / p
    xs = P + x / math.sqrt(p)
    K = math.exp(-a * b / p * (A - B) ** 2)
    return K / math.sqrt(p) * np.sum(w * (xs - A) ** i * (xs - B) ** j)


def _gh_kinetic_1d(i, j, a, b, A, B):
    t = 0.0
    if j >= 2:
        t += -0.5 * j * (j - 1) * _gh_overlap_1d(i, j - 2, a, b, A, B)
    t += b * (2 * j + 1) * _gh_overlap_1d(i, j, a, b, A, B)
    t += -2 * b * b * _gh_overlap_1d(i, j + 2, a, b, A, B)
    return t


def _carts(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def test_overlap_kinetic_by_quadrature():
    """S and T of random contracted p/d/f shells against Gauss-Hermite
    quadrature with the unit-self-overlap convention applied in the test."""
    rng = np.random.default_rng(11)
    atoms = rng.uniform(-1, 1, size=(2, 3))
    shells = [{"atom": 0, "l": 2, "exps": [1.3, 0.4], "coefs": [0.6, 0.5]},
              {"atom": 1, "l": 3, "exps": [0.8], "coefs": [1.0]},
              {"atom": 1, "l": 1, "exps": [2.1, 0.3, 0.1], "coefs": [0.2, 0.5, 0.4]}]
    s = _sys(atoms, shells)
    S, T, _ = oracle.oneel(s)
    funcs = []
    for sh in shells:
        for c in _carts(sh["l"]):
            funcs.append((atoms[sh["atom"]], c, sh["exps"], sh["coefs"], sh["l"]))

    def raw(f, g, kin):
        A, ca, ea, da, la = f
        B, cb, eb, db, lb = g
        tot = 0.0
        for a, d1 in zip(ea, da):
            n1 = (2 * a / math.pi) ** 0.75 * (4 * a) ** (la / 2) / math.sqrt(float(np.prod(range(2 * la - 1, 0, -2)) or 1))
            for b, d2 in zip(eb, db):
                n2 = (2 * b / math.pi) ** 0.75 * (4 * b) ** (lb / 2) / math.sqrt(float(np.prod(range(2 * lb - 1, 0, -2)) or 1))
                s1 = [_gh_overlap_1d(ca[k], cb[k], a, b, A[k], B[k]) for k in range(3)]
                if kin:
                    t1 = [_gh_kinetic_1d(ca[k], cb[k], a, b, A[k], B[k]) for k in range(3)]
                    v = t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2] + s1[0] * s1[1] * t1[2]
                else:
                    v = s1[0] * s1[1] * s1[2]
                tot += d1 * d2 * n1 * n2 * v
        return tot

    n = len(funcs)
    norm = np.array([1 / math.sqrt(raw(f, f, False)) for f in funcs])
    for i in range(n):
        for j in range(n):
            assert S[i, j] == pytest.approx(raw(funcs[i], funcs[j], False) * norm[i] * norm[j], rel=1e-11, abs=1e-14)
            assert T[i, j] == pytest.approx(raw(funcs[i], funcs[j], True) * norm[i] * norm[j], rel=1e-11, abs=1e-13)


def test_nuclear_attraction_gaussian_charge():
    """<s|-Z/|r-C||s> for a normalised s primitive is minus Z times the
    potential of a normalised Gaussian charge of exponent 2a at distance R."""
    a, R = 0.8, 1.7
    s = _sys([[0, 0, 0], [0, R, 0]], [{"atom": 0, "l": 0, "exps": [a], "coefs": [1.0]}], Z=[1, 3])
    _, _, V = oracle.oneel(s)
    ref = -1 * 2 * math.sqrt(2 * a / math.pi) - 3 * erf(math.sqrt(2 * a) * R) / R
    assert V[0, 0] == pytest.approx(ref, rel=1e-13)


def _v_elem(atoms, Z, la, ea, lb, eb, comp_a, comp_b):
    """One element of the oracle's V between a single primitive of momentum la
    on atom 0 and one of momentum lb on atom 1 (Cartesian components by index)."""
    s = _sys(atoms, [{"atom": 0, "l": la, "exps": [ea], "coefs": [1.0]},
                     {"atom": 1, "l": lb, "exps": [eb], "coefs": [1.0]}], Z=Z)
    _, _, V = oracle.oneel(s)
    na = (la + 1) * (la + 2) // 2
    return V[comp_a, na + comp_b]


def _fd(f, h=1e-3):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


def test_nuclear_attraction_p_d_f_are_centre_derivatives():
    """Nuclear attraction of p, d and f functions (Hermite form with the Boys
    function) against centre derivatives of lower momenta.  The moving function
    sits on a ghost centre (Z = 0), so only the function moves, never a nucleus;
    two real nuclei elsewhere.  For primitives normalised per component:
        p_x   = a^(-1/2) d/dA_x s,
        d_xy  = a^(-1/2) d/dA_y p_x,
        d_xx  = (d/dA_x p_x + 2 a^(1/2) s) / (3a)^(1/2),
        f_xyz = a^(-1/2) d/dA_z d_xy,
    each checked by a 4-point central difference of the oracle's own lower
    element, starting from the s-s element that the Gaussian-charge test
    pins.  A sign error in the centre reflection, a wrong index of the R
    tensor or a transposed component fails one of them.  Both sides (bra and
    ket function) are moved."""
    rng = np.random.default_rng(17)
    base = np.vstack([rng.uniform(-1, 1, size=(2, 3)), [[0.3, -1.1, 0.8], [-0.9, 0.6, -0.4]]])
    Z = [0, 0, 3, 1]
    ea, eb = 0.85, 0.55

    def moved(atom, axis, h):
        at = base.copy()
        at[atom, axis] += h
        return at

    # bra side: function on atom 0 moves
    p_x = _v_elem(base, Z, 1, ea, 0, eb, 0, 0)
    fd = _fd(lambda h: _v_elem(moved(0, 0, h), Z, 0, ea, 0, eb, 0, 0))
    assert p_x == pytest.approx(fd / math.sqrt(ea), rel=1e-8)
    p_y = _v_elem(base, Z, 1, ea, 0, eb, 1, 0)
    fd = _fd(lambda h: _v_elem(moved(0, 1, h), Z, 0, ea, 0, eb, 0, 0))
    assert p_y == pytest.approx(fd / math.sqrt(ea), rel=1e-8)
    # d_xy (component 1 of xx, xy, xz, yy, yz, zz) from p_x moved along y
    d_xy = _v_elem(base, Z, 2, ea, 0, eb, 1, 0)
    fd = _fd(lambda h: _v_elem(moved(0, 1, h), Z, 1, ea, 0, eb, 0, 0))
    assert d_xy == pytest.approx(fd / math.sqrt(ea), rel=1e-7)
    # d_xx from p_x moved along x and the s element
    d_xx = _v_elem(base, Z, 2, ea, 0, eb, 0, 0)
    s_s = _v_elem(base, Z, 0, ea, 0, eb, 0, 0)
    fd = _fd(lambda h: _v_elem(moved(0, 0, h), Z, 1, ea, 0, eb, 0, 0))
    assert d_xx == pytest.approx((fd + 2 * math.sqrt(ea) * s_s) / math.sqrt(3 * ea), rel=1e-7)
    # f_xyz (component 4 of xxx, xxy, xxz, xyy, xyz, ...) from d_xy moved along z
    f_xyz = _v_elem(base, Z, 3, ea, 0, eb, 4, 0)
    fd = _fd(lambda h: _v_elem(moved(0, 2, h), Z, 2, ea, 0, eb, 1, 0))
    assert f_xyz == pytest.approx(fd / math.sqrt(ea), rel=1e-7)
    # ket side: function on atom 1 moves; p on both sides
    s_pz = _v_elem(base, Z, 0, ea, 1, eb, 0, 2)
    fd = _fd(lambda h: _v_elem(moved(1, 2, h), Z, 0, ea, 0, eb, 0, 0))
    assert s_pz == pytest.approx(fd / math.sqrt(eb), rel=1e-8)
    px_dyz = _v_elem(base, Z, 1, ea, 2, eb, 0, 4)
    fd = _fd(lambda h: _v_elem(moved(1, 1, h), Z, 1, ea, 1, eb, 0, 2))
    assert px_dyz == pytest.approx(fd / math.sqrt(eb), rel=1e-7)


# ------------------------------------------------------- J/K brute force ---
@pytest.mark.parametrize("seed", [0, 1])
def test_jk_matches_brute_force(seed):
    """The orbit-based literal J/K equals the plain N^4 sums (catches dropped
    permutations, double counting and transposed density indices)."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(-1.2, 1.2, size=(3, 3))
    shells = [{"atom": 0, "l": 0, "exps": [1.1, 0.3], "coefs": [0.5, 0.6]},
              {"atom": 0, "l": 1, "exps": [0.7], "coefs": [1.0]},
              {"atom": 0, "l": 1, "exps": [0.25], "coefs": [1.0]},
              {"atom": 1, "l": 2, "exps": [0.9], "coefs": [1.0]},
              {"atom": 2, "l": 0, "exps": [0.5], "coefs": [1.0]},
              {"atom": 2, "l": 3, "exps": [0.6], "coefs": [1.0]}]
    s = _sys(atoms, shells)
    assert s["nbf"] <= 30
    D = rng.normal(size=(s["nbf"], s["nbf"]))
    D = D + D.T
    eri = oracle.eri_full(s)
    J, K = oracle.jk(s, D)
    assert np.allclose(J, np.einsum("ijkl,kl->ij", eri, D), rtol=1e-12, atol=1e-12)
    assert np.allclose(K, np.einsum("ikjl,kl->ij", eri, D), rtol=1e-12, atol=1e-12)
    assert np.allclose(J, J.T, atol=1e-12) and np.allclose(K, K.T, atol=1e-12)
    off = oracle.bf_offsets(s)
    jp = [(3, 1), (5, 5), (0, 2)]
    kp = [(5, 0), (1, 3), (2, 2)]
    Jb, Kb = oracle.jk_blocks(s, D, jp, kp)
    for (a, b), blk in zip(jp, Jb):
        assert np.allclose(blk, J[off[a]:off[a + 1], off[b]:off[b + 1]], rtol=1e-12, atol=1e-12)
    for (a, c), blk in zip(kp, Kb):
        assert np.allclose(blk, K[off[a]:off[a + 1], off[c]:off[c + 1]], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------- SCF-level pins -------
def test_h2_textbook():
    g = json.load(open(os.path.join(GOLD, "h2_sto3g_szabo_ostlund.json")))
    s = wl.h2_sto3g(g["R_bohr"])
    S, T, V = oracle.oneel(s)
    eri = oracle.eri_full(s)
    I, tol = g["integrals_4dp"], g["integral_tol"]
    assert abs(S[0, 1] - I["S12"]) < tol
    assert abs(T[0, 0] - I["T11"]) < tol and abs(T[0, 1] - I["T12"]) < tol
    assert abs(V[0, 0] - I["V11_total"]) < tol and abs(V[0, 1] - I["V12_total"]) < tol
    assert abs(eri[0, 0, 0, 0] - I["eri_1111"]) < tol
    assert abs(eri[0, 0, 1, 1] - I["eri_1122"]) < tol
    assert abs(eri[0, 1, 0, 1] - I["eri_1212"]) < tol
    assert abs(eri[0, 0, 0, 1] - I["eri_1112"]) < tol
    r = run_scf(s)
    assert r["converged"]
    assert abs(r["E"] - g["E_total"]) < g["E_tol"]
    # two electrons in one orbital: c^T J c == c^T K c
    # D = 2 c c^T, so sum(D*J) = 4 (cc|cc) = sum(D*K)
    J, K = oracle.jk(s, r["D"])
    assert float(np.sum(r["D"] * J)) == pytest.approx(float(np.sum(r["D"] * K)), rel=1e-12)


def test_water_dimer_invariants():
    mol = geom.water_cluster(2, 42)
    s = wl.make_system(mol, "sto-3g")
    r = run_scf(s)
    assert r["converged"]
    D, S = r["D"], r["S"]
    assert np.trace(D @ S) == pytest.approx(s["nelec"], abs=1e-10)
    DS = D @ S
    assert np.allclose(DS @ DS, 2 * DS, atol=1e-7)
    # rigid rotation + translation
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    mol2 = dict(mol)
    mol2["xyz"] = mol["xyz"] @ Q.T + np.array([1.3, -0.7, 2.2])
    r2 = run_scf(wl.make_system(mol2, "sto-3g"))
    assert r2["E"] == pytest.approx(r["E"], abs=1e-8)
    # atom (molecule) reordering
    mol3 = dict(mol)
    mol3["xyz"] = np.concatenate([mol["xyz"][3:], mol["xyz"][:3]])
    mol3["Z"] = np.concatenate([mol["Z"][3:], mol["Z"][:3]])
    r3 = run_scf(wl.make_system(mol3, "sto-3g"))
    assert r3["E"] == pytest.approx(r["E"], abs=1e-8)


def test_far_fragments_additive():
    e1 = run_scf(wl.h2_sto3g())["E"]
    mol = {"Z": np.array([1, 1, 1, 1], dtype=np.int32),
           "xyz": np.array([[0, 0, 0], [0, 0, 1.4], [1000.0, 0, 0], [1000.0, 0, 1.4]]), "charge": 0, "name": "2H2"}
    e2 = run_scf(wl.make_system(mol, "sto-3g"))["E"]
    assert e2 == pytest.approx(2 * e1, abs=1e-9)
