"""Plain FP64 CPU oracle for the direct Hartree-Fock J/K build.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product library never
imports, links or calls anything here, and nothing here calls the product.

The arithmetic lives in ``oracle.c`` (compiled with gcc on first use or by the
build step); ``scf.py`` holds the textbook RHF/DIIS loop on top of it.
Every function cites the paper passage it follows in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        I, D, P = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        ob = [I, P, P, I, P, P, P, P, P]
        L.oracle_boys.argtypes = [I, D, P]
        L.oracle_nbf.argtypes = ob
        L.oracle_eri_quartet.argtypes = ob + [I, I, I, I, I, P]
        L.oracle_eri_full.argtypes = ob + [P]
        L.oracle_eri_list.argtypes = ob + [I, P, I, P]
        L.oracle_jk.argtypes = ob + [P, P, P, I]
        L.oracle_jk_blocks.argtypes = ob + [P, I, P, P, I, P, P, I]
        L.oracle_oneel.argtypes = ob + [P, P, P]
        L.oracle_enuc.argtypes = [I, P, P]
        L.oracle_enuc.restype = D
        L.oracle_hermite_nnz.argtypes = [I, I, D, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Args:
    """Keeps contiguous copies alive for the duration of a call."""

    def __init__(self, sys):
        self.Z = np.ascontiguousarray(sys["Z"], dtype=np.int32)
        self.xyz = np.ascontiguousarray(sys["xyz"], dtype=np.float64).reshape(-1)
        self.sa = np.ascontiguousarray(sys["sh_atom"], dtype=np.int32)
        self.sl = np.ascontiguousarray(sys["sh_l"], dtype=np.int32)
        self.sn = np.ascontiguousarray(sys["sh_nprim"], dtype=np.int32)
        self.ex = np.ascontiguousarray(sys["exps"], dtype=np.float64)
        self.co = np.ascontiguousarray(sys["coefs"], dtype=np.float64)

    def tup(self):
        return (len(self.Z), _ptr(self.Z), _ptr(self.xyz), len(self.sl), _ptr(self.sa), _ptr(self.sl),
                _ptr(self.sn), _ptr(self.ex), _ptr(self.co))


def ncart(l):
    return (l + 1) * (l + 2) // 2


def boys(mmax, T):
    F = np.zeros(mmax + 1)
    lib().oracle_boys(mmax, float(T), _ptr(F))
    return F


def eri_quartet(sys, a, b, c, d, method="mmd"):
    """Contracted normalised (ab|cd) as an array [na, nb, nc, nd]."""
    A = _Args(sys)
    l = sys["sh_l"]
    shape = tuple(ncart(int(l[s])) for s in (a, b, c, d))
    out = np.zeros(shape)
    rc = lib().oracle_eri_quartet(*A.tup(), a, b, c, d, 1 if method == "os" else 0, _ptr(out))
    if rc:
        raise ValueError("oracle: invalid basis")
    return out


def eri_list(sys, quartets, nthreads=0):
    """Evaluates the listed shell quartets (rows a, b, c, d) with the oracle's
    MMD code, OpenMP over the list; returns the sum of |(ab|cd)| (timing aid)."""
    A = _Args(sys)
    q = np.ascontiguousarray(np.asarray(quartets, dtype=np.int32).reshape(-1, 4))
    sink = ctypes.c_double()
    if lib().oracle_eri_list(*A.tup(), len(q), _ptr(q), int(nthreads), ctypes.byref(sink)):
        raise ValueError("oracle: invalid basis")
    return sink.value


def eri_full(sys):
    A = _Args(sys)
    n = sys["nbf"]
    out = np.zeros((n, n, n, n))
    if lib().oracle_eri_full(*A.tup(), _ptr(out)):
        raise ValueError("oracle: invalid basis")
    return out


def jk(sys, D, nthreads=0):
    """Unscreened J and K (literal sums over every distinct permutation)."""
    A = _Args(sys)
    n = sys["nbf"]
    D = np.ascontiguousarray(D, dtype=np.float64)
    J = np.zeros((n, n))
    K = np.zeros((n, n))
    if lib().oracle_jk(*A.tup(), _ptr(D), _ptr(J), _ptr(K), nthreads):
        raise ValueError("oracle: invalid basis")
    return J, K


def bf_offsets(sys):
    return np.concatenate([[0], np.cumsum([ncart(int(l)) for l in sys["sh_l"]])]).astype(int)


def jk_blocks(sys, D, jpairs, kpairs, nthreads=0):
    """Shell blocks J[A,B] and K[A,C] by literal unsymmetrised sums.
    Returns two lists of 2-D arrays."""
    A = _Args(sys)
    D = np.ascontiguousarray(D, dtype=np.float64)
    l = sys["sh_l"]
    jp = np.ascontiguousarray(np.asarray(jpairs, dtype=np.int32).reshape(-1, 2))
    kp = np.ascontiguousarray(np.asarray(kpairs, dtype=np.int32).reshape(-1, 2))
    js = [(ncart(int(l[a])), ncart(int(l[b]))) for a, b in jp]
    ks = [(ncart(int(l[a])), ncart(int(l[c]))) for a, c in kp]
    Jo = np.zeros(max(1, sum(x * y for x, y in js)))
    Ko = np.zeros(max(1, sum(x * y for x, y in ks)))
    if lib().oracle_jk_blocks(*A.tup(), _ptr(D), len(jp), _ptr(jp), _ptr(Jo), len(kp), _ptr(kp), _ptr(Ko),
                              nthreads):
        raise ValueError("oracle: invalid basis")
    outJ, outK, o = [], [], 0
    for s in js:
        outJ.append(Jo[o:o + s[0] * s[1]].reshape(s))
        o += s[0] * s[1]
    o = 0
    for s in ks:
        outK.append(Ko[o:o + s[0] * s[1]].reshape(s))
        o += s[0] * s[1]
    return outJ, outK


def oneel(sys):
    A = _Args(sys)
    n = sys["nbf"]
    S, T, V = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    if lib().oracle_oneel(*A.tup(), _ptr(S), _ptr(T), _ptr(V)):
        raise ValueError("oracle: invalid basis")
    return S, T, V


def enuc(sys):
    A = _Args(sys)
    return float(lib().oracle_enuc(len(A.Z), _ptr(A.Z), _ptr(A.xyz)))


def hermite_nnz(la, lb, zeta=1.3, PA=(0.31, -0.27, 0.19), PB=(-0.42, 0.23, -0.37)):
    """(dense, nonzero) counts of the pair's Hermite expansion tensor."""
    pa = np.array(PA, dtype=np.float64)
    pb = np.array(PB, dtype=np.float64)
    d = ctypes.c_int()
    n = ctypes.c_int()
    lib().oracle_hermite_nnz(la, lb, zeta, _ptr(pa), _ptr(pb), ctypes.byref(d), ctypes.byref(n))
    return d.value, n.value
