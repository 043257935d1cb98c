"""Seeded synthetic Cartesian Gaussian basis sets.

No basis-set library is available, so the basis sets used by the workloads are
generated here from physical scale parameters:

* ``sto-3g``: every contracted shell is a least-squares fit of n Gaussians to a
  Slater function, the published construction of the STO-nG family
  (Hehre, Stewart & Pople 1969).  ``s`` and ``p`` shells of the same valence
  level share exponents, as in that family.  Slater exponents are the standard
  molecular values (H 1.24; C 5.67/1.72; N 6.67/1.95; O 7.66/2.25).
* ``6-31gs-type``: split-valence shell structure of 6-31G* built from the same
  fits (core s6; inner valence s3+p3; outer valence s1+p1; one Cartesian d).
* ``ccpvdz-type``: the shell structure of cc-pVDZ (O: s9 s9 s1 p4 p1 d1;
  H: s3 s1 p1) built from even-tempered exponents whose contraction
  coefficients are linear least-squares fits to Slater functions.
* ``tzvp-type``: a def2-TZVP-like structure up to f (C/N/O [5s3p2d1f],
  H [3s1p]) with contraction depth at most 6.

Conventions shared by every consumer (they are input format, not method):
contraction coefficients multiply primitives normalised as the axis-aligned
component, N(a,l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!).  How the
contracted functions are normalised is left to each consumer.

This module holds no arithmetic of the Hartree-Fock method; its overlap
integrals are those of single-centre radial functions used only for fitting.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy import integrate, optimize

# Slater exponents: (1s, 2sp) per element.
SLATER_ZETA = {1: (1.24, None), 6: (5.67, 1.72), 7: (6.67, 1.95), 8: (7.66, 2.25)}


# ---------------------------------------------------------------- fitting --
def _radial(fn, k, alpha):
    """int_0^inf r^k exp(-r - alpha r^2) dr for the Slater(zeta=1) fits."""
    val, _ = integrate.quad(lambda r: r ** k * math.exp(-r - alpha * r * r), 0, np.inf,
                            epsabs=1e-15, epsrel=1e-13, limit=400)
    return val


def _ovl_slater(kind, alpha):
    """Overlap of a normalised Slater function (zeta=1) with a normalised
    Gaussian of exponent alpha of the same angular type."""
    if kind == "1s":
        return 4 * math.pi * (1 / math.sqrt(math.pi)) * (2 * alpha / math.pi) ** 0.75 * _radial(None, 2, alpha)
    if kind == "2s":
        return 4 * math.pi * (1 / math.sqrt(3 * math.pi)) * (2 * alpha / math.pi) ** 0.75 * _radial(None, 3, alpha)
    if kind == "2p":
        return (4 * math.pi / 3) * (1 / math.sqrt(math.pi)) * (128 * alpha ** 5 / math.pi ** 3) ** 0.25 * _radial(None, 4, alpha)
    raise ValueError(kind)


def _ovl_gauss(l, a, b):
    return (2 * math.sqrt(a * b) / (a + b)) ** (1.5 + l)


def _ls(kind, alphas):
    """Linear least-squares coefficients for fixed exponents; returns (d, residual)."""
    l = 1 if kind == "2p" else 0
    S = np.array([[_ovl_gauss(l, a, b) for b in alphas] for a in alphas])
    bvec = np.array([_ovl_slater(kind, a) for a in alphas])
    d = np.linalg.solve(S, bvec)
    return d, 1.0 - float(bvec @ d)


@functools.lru_cache(maxsize=None)
def sto_fit(kinds: tuple, n: int):
    """Least-squares STO-nG fit (zeta = 1) of the Slater functions in ``kinds``
    with n shared exponents.  Returns (alphas, {kind: coefs})."""
    start = np.log(np.geomspace(0.07 * (5.0 ** (n - 1)) if kinds[0] != "1s" else 0.1 * (4.5 ** (n - 1)),
                                0.07 if kinds[0] != "1s" else 0.1, n))

    def obj(x):
        al = np.exp(x)
        if np.min(np.abs(np.diff(np.sort(al)))) < 1e-6:
            return 10.0
        try:
            return sum(_ls(k, al)[1] for k in kinds)
        except np.linalg.LinAlgError:
            return 10.0

    res = optimize.minimize(obj, start, method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-15, "maxiter": 40000, "maxfev": 40000})
    res = optimize.minimize(obj, res.x, method="BFGS", options={"gtol": 1e-12})
    al = np.sort(np.exp(res.x))[::-1]
    return tuple(al), {k: tuple(_ls(k, al)[0]) for k in kinds}


def _scaled(kinds, n, zeta):
    al, co = sto_fit(tuple(kinds), n)
    return [a * zeta * zeta for a in al], {k: list(v) for k, v in co.items()}


def _even_tempered(amax, amin, n):
    return list(np.geomspace(amax, amin, n))


def _fixed_fit(kind, alphas, zeta):
    """Coefficients of fixed exponents (already scaled to zeta) fitted to a
    Slater function of exponent zeta."""
    d, _ = _ls(kind, [a / (zeta * zeta) for a in alphas])
    return list(d)


# ----------------------------------------------------------- basis sets ----
def _shell(l, exps, coefs):
    return {"l": int(l), "exps": [float(x) for x in exps], "coefs": [float(c) for c in coefs]}


@functools.lru_cache(maxsize=None)
def _atom_shells(name: str, Z: int):
    z1, z2 = SLATER_ZETA[Z]
    out = []
    if name == "sto-3g":
        a, c = _scaled(("1s",), 3, z1)
        out.append(_shell(0, a, c["1s"]))
        if Z > 2:
            a, c = _scaled(("2s", "2p"), 3, z2)
            out.append(_shell(0, a, c["2s"]))
            out.append(_shell(1, a, c["2p"]))
    elif name == "6-31gs-type":
        if Z == 1:
            a, c = _scaled(("1s",), 3, 1.6 * z1)
            out.append(_shell(0, a, c["1s"]))
            out.append(_shell(0, [0.161], [1.0]))
        else:
            a, c = _scaled(("1s",), 6, z1)
            out.append(_shell(0, a, c["1s"]))
            a, c = _scaled(("2s", "2p"), 3, 1.25 * z2)
            out.append(_shell(0, a, c["2s"]))
            out.append(_shell(1, a, c["2p"]))
            aout = 0.057 * z2 * z2
            out.append(_shell(0, [aout], [1.0]))
            out.append(_shell(1, [aout], [1.0]))
            out.append(_shell(2, [0.8], [1.0]))
    elif name == "ccpvdz-type":
        if Z == 1:
            a, c = _scaled(("1s",), 3, 1.6 * z1)
            out.append(_shell(0, a, c["1s"]))
            out.append(_shell(0, [0.122], [1.0]))
            out.append(_shell(1, [0.727], [1.0]))
        else:
            ex = _even_tempered(200.0 * z1 * z1, 0.06 * z2 * z2 * 1.3, 9)
            out.append(_shell(0, ex, _fixed_fit("1s", ex, z1)))
            out.append(_shell(0, ex, _fixed_fit("2s", ex, z2)))
            out.append(_shell(0, [0.06 * z2 * z2], [1.0]))
            a, c = _scaled(("2p",), 4, 1.1 * z2)
            out.append(_shell(1, a, c["2p"]))
            out.append(_shell(1, [0.042 * z2 * z2], [1.0]))
            out.append(_shell(2, [1.185], [1.0]))
    elif name == "tzvp-type":
        if Z == 1:
            a, c = _scaled(("1s",), 3, 1.6 * z1)
            out.append(_shell(0, a, c["1s"]))
            out.append(_shell(0, [0.33], [1.0]))
            out.append(_shell(0, [0.12], [1.0]))
            out.append(_shell(1, [0.8], [1.0]))
        else:
            a, c = _scaled(("1s",), 6, z1)
            out.append(_shell(0, a, c["1s"]))
            a, c = _scaled(("2s",), 2, 2.2 * z2)
            out.append(_shell(0, a, c["2s"]))
            # a tight contracted 2s and three uncontracted s spread below it, so that
            # no one-centre combination is nearly redundant
            for e in (0.40, 0.17, 0.08):
                out.append(_shell(0, [e * z2 * z2 / 2.96], [1.0]))
            a, c = _scaled(("2p",), 4, 1.1 * z2)
            out.append(_shell(1, a, c["2p"]))
            for e in (0.30, 0.12):
                out.append(_shell(1, [e * z2 * z2 / 2.96], [1.0]))
            out.append(_shell(2, [1.1], [1.0]))
            out.append(_shell(2, [0.32], [1.0]))
            out.append(_shell(3, [0.76], [1.0]))
    else:
        raise ValueError(f"unknown basis {name}")
    return tuple(tuple(sorted(s.items())) for s in out)


def basis_for(name: str, Z) -> list:
    """Shell list for atoms with nuclear charges ``Z`` (atom-major order)."""
    shells = []
    for ia, z in enumerate(Z):
        for s in _atom_shells(name, int(z)):
            d = dict(s)
            shells.append({"atom": ia, "l": d["l"], "exps": list(d["exps"]), "coefs": list(d["coefs"])})
    return shells


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nbf(shells) -> int:
    return sum(ncart(s["l"]) for s in shells)
