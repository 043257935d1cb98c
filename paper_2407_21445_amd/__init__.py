"""Python binding of libfockjk (see include/fockjk.h): argument marshalling only.

Every step of the J/K build runs in the library's HIP kernels; this module
only converts arrays, device pointers and streams.  Importing it loads
``libfockjk.so`` from this directory and fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfockjk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfockjk.so not built at {LIB_PATH}; run __graft_entry__.build() "
                      "(or python -m paper_2407_21445_amd.build)")

# One HIP runtime per process.  PyTorch ships its own copy of the runtime
# (linked by its unversioned name); loading the library first would pull in the
# system copy as well, and two runtimes in one process do not share the device.
# Importing torch first makes the library bind to the copy torch has loaded.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # host-only use (tables, validation) without PyTorch
    _torch = None

_lib = ctypes.CDLL(LIB_PATH)

FK_OK, FK_ERR_ARG, FK_ERR_UNSUPPORTED, FK_ERR_HIP, FK_ERR_OOM, FK_ERR_NOT_CONVERGED, FK_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
FK_DEVICE_PTRS, FK_SYNC, FK_TIME_CLASSES, FK_J_ONLY, FK_K_ONLY, FK_J_ENGINE = 1, 2, 4, 8, 16, 32
FK_MAX_QCLASS = 110
MAX_L, MAX_K = 3, 9


class ScreenOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("tau_prim", ctypes.c_double),
                ("density_screen", ctypes.c_int), ("bra_block", ctypes.c_int), ("tau_fp32", ctypes.c_double),
                ("tau_k", ctypes.c_double), ("block_tasks", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("nbf", ctypes.c_int), ("nshell", ctypes.c_int), ("natom", ctypes.c_int), ("nelec", ctypes.c_int),
                ("npair", ctypes.c_int), ("npair_kept", ctypes.c_int), ("nclass_pair", ctypes.c_int),
                ("nquartet_class", ctypes.c_int), ("nprim_pair", ctypes.c_int64),
                ("nquartet_schwarz", ctypes.c_int64), ("ntile", ctypes.c_int64), ("flops_schwarz", ctypes.c_double),
                ("nmol", ctypes.c_int), ("reserved", ctypes.c_int), ("nmat", ctypes.c_int64)]


_Q = FK_MAX_QCLASS


class Stats(ctypes.Structure):
    _fields_ = [("nclass", ctypes.c_int), ("la", ctypes.c_int * _Q), ("lb", ctypes.c_int * _Q),
                ("lc", ctypes.c_int * _Q), ("ld", ctypes.c_int * _Q), ("quartets", ctypes.c_int64 * _Q),
                ("prim_quartets", ctypes.c_int64 * _Q), ("flops_per_prim", ctypes.c_double * _Q),
                ("flops_per_quartet", ctypes.c_double * _Q), ("flops_total", ctypes.c_double),
                ("class_ms", ctypes.c_double * _Q), ("tiles", ctypes.c_int64 * _Q),
                ("team_size", ctypes.c_int * _Q), ("precision", ctypes.c_int * _Q), ("prim_slots", ctypes.c_int64 * _Q),
                ("engine", ctypes.c_int * _Q), ("bra_block", ctypes.c_int * _Q), ("kets_per_tile", ctypes.c_int * _Q),
                ("grid_fraction", ctypes.c_double * _Q), ("block_tasks", ctypes.c_int64 * _Q),
                ("waves_per_group", ctypes.c_int * _Q)]


class TuneReport(ctypes.Structure):
    _fields_ = [("nclass", ctypes.c_int), ("la", ctypes.c_int * _Q), ("lb", ctypes.c_int * _Q),
                ("lc", ctypes.c_int * _Q), ("ld", ctypes.c_int * _Q), ("precision", ctypes.c_int * _Q),
                ("bra_block", ctypes.c_int * _Q), ("kets_per_tile", ctypes.c_int * _Q),
                ("grid_fraction", ctypes.c_double * _Q), ("engine", ctypes.c_int * _Q), ("changed", ctypes.c_int * _Q),
                ("ms_default", ctypes.c_double * _Q),
                ("ms_tuned", ctypes.c_double * _Q), ("build_ms_default", ctypes.c_double),
                ("build_ms_tuned", ctypes.c_double), ("configurations", ctypes.c_int),
                ("block_tasks", ctypes.c_int * _Q), ("lanes_per_quartet", ctypes.c_int * _Q)]


class ScfOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("e_tol", ctypes.c_double), ("g_tol", ctypes.c_double),
                ("diis_n", ctypes.c_int), ("guess", ctypes.c_int), ("lindep", ctypes.c_double),
                ("graph", ctypes.c_int), ("incremental", ctypes.c_int), ("canonical", ctypes.c_double),
                ("j_engine", ctypes.c_int), ("density_eig", ctypes.c_int)]


class ScfResult(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("e_nuc", ctypes.c_double), ("iterations", ctypes.c_int),
                ("converged", ctypes.c_int), ("jk_seconds", ctypes.c_double), ("total_seconds", ctypes.c_double),
                ("error", ctypes.c_double), ("delta_e", ctypes.c_double), ("guess_used", ctypes.c_int),
                ("guess_seconds", ctypes.c_double), ("ndropped", ctypes.c_int)]


GUESS_CORE, GUESS_GIVEN, GUESS_SAD, GUESS_LEARNED = 0, 1, 2, 3
ENGINE_RYS, ENGINE_HGP = 0, 1
GUESS_NB, GUESS_NOUT, GUESS_NRBF, GUESS_NFEAT, GUESS_RCUT = 15, 225, 24, 192, 8.0
MLP_MAX_LAYERS = 4


class Mlp(ctypes.Structure):
    _fields_ = [("nlayer", ctypes.c_int), ("dims", ctypes.c_int * (MLP_MAX_LAYERS + 1)),
                ("W", ctypes.c_void_p * MLP_MAX_LAYERS), ("b", ctypes.c_void_p * MLP_MAX_LAYERS)]


_P, _I, _D, _U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
_sig = {
    "fk_create": ([ctypes.POINTER(_P), _I], _I),
    "fk_destroy": ([_P], None),
    "fk_last_error": ([_P], ctypes.c_char_p),
    "fk_set_geometry": ([_P, _I, _P, _P, _I], _I),
    "fk_set_basis": ([_P, _I, _P, _P, _P, _P, _P], _I),
    "fk_build_quartets": ([_P, ctypes.POINTER(ScreenOpts)], _I),
    "fk_info": ([_P, ctypes.POINTER(Info)], _I),
    "fk_build_jk": ([_P, _P, _P, _P, _U, _P], _I),
    "fk_build_jk_noalloc": ([_P, _P, _P, _P, _U, _P], _I),
    "fk_density_bound": ([_P, _P, _U, _P, _P], _I),
    "fk_stats": ([_P, ctypes.POINTER(Stats)], _I),
    "fk_one_electron": ([_P, _P, _P, _P, _P], _I),
    "fk_run_scf": ([_P, ctypes.POINTER(ScfOpts), ctypes.POINTER(ScfResult), _P], _I),
    "fk_debug_eri": ([_P, _I, _P, _P, _I], _I),
    "fk_rys_host": ([_I, _D, _P, _P], _I),
    "fk_check_indices": ([_P], _I),
    "fk_set_molecules": ([_P, _I, _P], _I),
    "fk_molecule_layout": ([_P, _P, _P], _I),
    "fk_sad_density": ([_P, _P], _I),
    "fk_build_progress": ([_P, _P, _P], _I),
    "fk_run_scf_batch": ([_P, ctypes.POINTER(ScfOpts), _P, _P], _I),
    "fk_set_class_schedule": ([_P, _I, _I, _I, _I, _I, _I, _D], _I),
    "fk_set_class_engine": ([_P, _I, _I, _I, _I, _I], _I),

    "fk_set_class_block_tasks": ([_P, _I, _I, _I, _I, _I], _I),


    "fk_set_class_lanes": ([_P, _I, _I, _I, _I, _I], _I),
    "fk_save_schedules": ([_P, ctypes.c_char_p], _I),
    "fk_load_schedules": ([_P, ctypes.c_char_p], _I),
    "fk_autotune": ([_P, _P, _U, _I, _P, ctypes.POINTER(TuneReport)], _I),
    "fk_guess_pairs": ([_P, _P, _P, _P], _I),
    "fk_guess_targets": ([_P, _P, _P], _I),
    "fk_set_guess_model": ([_P, ctypes.POINTER(Mlp)], _I),
    "fk_guess_predict": ([_P, _P], _I),
    "fk_mlp_work_floats": ([ctypes.POINTER(Mlp), _I], ctypes.c_int64),
    "fk_mlp_forward": ([ctypes.POINTER(Mlp), _P, _I, _P, _P, _P], _I),
    "fk_mlp_backward": ([ctypes.POINTER(Mlp), _P, _I, _P, _P, ctypes.POINTER(Mlp), _P], _I),
    "fk_mlp_block_mse": ([_P, _P, _P, _I, _D, _P, _P, _P, _P], _I),
    "fk_mlp_mse_scratch": ([], _I),
    "fk_mlp_adam": ([ctypes.POINTER(Mlp), ctypes.POINTER(Mlp), ctypes.POINTER(Mlp), ctypes.POINTER(Mlp), _I,
                     ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P], _I),
}
EXPORTS = tuple(_sig)
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class FockJKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fockjk error {code}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ncart(l):
    return (l + 1) * (l + 2) // 2


def rys_host(n, T):
    """Rys roots and weights of the library's tables, evaluated on the host."""
    u = np.zeros(n)
    w = np.zeros(n)
    rc = _lib.fk_rys_host(int(n), float(T), _ptr(u), _ptr(w))
    if rc:
        raise FockJKError(rc, "fk_rys_host: bad arguments")
    return u, w


class FockJK:
    """One library context on one device (device=-1: host-only context, which
    can build screening lists and evaluate integrals on the host for checks,
    but cannot run fk_build_jk)."""

    def __init__(self, device=0):
        self._ctx = ctypes.c_void_p()
        rc = _lib.fk_create(ctypes.byref(self._ctx), int(device))
        if rc:
            raise FockJKError(rc, f"fk_create(device={device}) failed: " + _lib.fk_last_error(None).decode())
        self.device = device
        self.nbf = 0
        self._keep = []

    def close(self):
        if self._ctx:
            _lib.fk_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc not in (FK_OK,):
            raise FockJKError(rc, _lib.fk_last_error(self._ctx).decode())
        return rc

    # ---- inputs ----
    def set_system(self, sys):
        Z = np.ascontiguousarray(sys["Z"], dtype=np.int32)
        xyz = np.ascontiguousarray(sys["xyz"], dtype=np.float64).reshape(-1)
        self._check(_lib.fk_set_geometry(self._ctx, len(Z), _ptr(Z), _ptr(xyz), int(sys.get("charge", 0))))
        sa = np.ascontiguousarray(sys["sh_atom"], dtype=np.int32)
        sl = np.ascontiguousarray(sys["sh_l"], dtype=np.int32)
        sn = np.ascontiguousarray(sys["sh_nprim"], dtype=np.int32)
        ex = np.ascontiguousarray(sys["exps"], dtype=np.float64)
        co = np.ascontiguousarray(sys["coefs"], dtype=np.float64)
        self._check(_lib.fk_set_basis(self._ctx, len(sl), _ptr(sa), _ptr(sl), _ptr(sn), _ptr(ex), _ptr(co)))
        self.sh_l = sl.copy()
        self.nbf = int(sum(_ncart(int(l)) for l in sl))
        return self

    def set_molecules(self, atom_mol):
        """Splits the atoms into independent molecules (batch); atom_mol is
        non-decreasing.  D, J, K are then flat concatenations of the
        molecules' nbf_m x nbf_m blocks (see molecule_layout)."""
        am = np.ascontiguousarray(atom_mol, dtype=np.int32)
        self._check(_lib.fk_set_molecules(self._ctx, int(am.max()) + 1, _ptr(am)))
        return self

    def molecule_layout(self):
        """(nbf per molecule, offsets of the blocks (nmol + 1 entries))."""
        nmol = self.info()["nmol"]
        nbf = np.zeros(nmol, dtype=np.int32)
        off = np.zeros(nmol + 1, dtype=np.int64)
        self._check(_lib.fk_molecule_layout(self._ctx, _ptr(nbf), _ptr(off)))
        return nbf, off

    def build_quartets(self, tau=1e-10, tau_prim=0.0, density_screen=True, bra_block=0, tau_fp32=0.0, tau_k=0.0,
                       block_tasks=True):
        o = ScreenOpts(float(tau), float(tau_prim), 1 if density_screen else 0, int(bra_block), float(tau_fp32),
                       float(tau_k), 0 if block_tasks else -1)
        self._check(_lib.fk_build_quartets(self._ctx, ctypes.byref(o)))
        return self

    def info(self):
        i = Info()
        self._check(_lib.fk_info(self._ctx, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    # ---- hot path ----
    def build_jk(self, D, J=None, K=None, stream=None, sync=False, time_classes=False, only=None, j_engine=False):
        """J, K for density D.  torch CUDA tensors (float64, contiguous) stay on
        the device and run on `stream` (default: torch's current stream);
        numpy arrays go through host copies.  only="J" or "K" forms one
        matrix (FK_J_ONLY / FK_K_ONLY); the other is returned as None.
        j_engine: J by the McMurchie-Davidson J engine (FK_J_ENGINE)."""
        if only not in (None, "J", "K"):
            raise ValueError("only must be None, 'J' or 'K'")
        oflag = {None: 0, "J": FK_J_ONLY, "K": FK_K_ONLY}[only] | (FK_J_ENGINE if j_engine else 0)
        nmat = self.info()["nmat"]
        if isinstance(D, np.ndarray):
            Dh = np.ascontiguousarray(D, dtype=np.float64)
            if Dh.size != nmat:
                raise ValueError(f"D must hold {nmat} elements (nbf x nbf, or the concatenated blocks of a batch)")
            Jh = np.zeros(Dh.shape) if only != "K" else None
            Kh = np.zeros(Dh.shape) if only != "J" else None
            self._check(_lib.fk_build_jk(self._ctx, _ptr(Dh), _ptr(Jh) if Jh is not None else None,
                                         _ptr(Kh) if Kh is not None else None, oflag, None))
            return Jh, Kh
        import torch
        if not (D.is_cuda and D.dtype == torch.float64 and D.is_contiguous() and D.numel() == nmat):
            raise ValueError(f"D must be a contiguous float64 CUDA tensor of {nmat} elements")
        if J is None and only != "K":
            J = torch.empty_like(D)
        if K is None and only != "J":
            K = torch.empty_like(D)
        if only == "J":
            K = None
        if only == "K":
            J = None
        for M in (J, K):
            if M is not None and not (M.is_cuda and M.dtype == torch.float64 and M.is_contiguous()
                                      and M.numel() == nmat):
                raise ValueError(f"J and K must be contiguous float64 CUDA tensors of {nmat} elements")
        st = stream if stream is not None else torch.cuda.current_stream(D.device)
        flags = FK_DEVICE_PTRS | (FK_SYNC if sync else 0) | (FK_TIME_CLASSES if time_classes else 0) | oflag
        self._check(_lib.fk_build_jk(self._ctx, ctypes.c_void_p(D.data_ptr()),
                                     ctypes.c_void_p(J.data_ptr() if J is not None else None),
                                     ctypes.c_void_p(K.data_ptr() if K is not None else None), flags,
                                     ctypes.c_void_p(st.cuda_stream)))
        return J, K

    def density_bound(self, D):
        """(H, Lambda) of the density-decay bound |D_uv| <= H exp(-Lambda r_uv)."""
        H, L = ctypes.c_double(), ctypes.c_double()
        if _torch is not None and isinstance(D, _torch.Tensor):
            self._check(_lib.fk_density_bound(self._ctx, ctypes.c_void_p(D.data_ptr()), FK_DEVICE_PTRS,
                                              ctypes.byref(H), ctypes.byref(L)))
        else:
            Dh = np.ascontiguousarray(D, dtype=np.float64)
            self._check(_lib.fk_density_bound(self._ctx, _ptr(Dh), 0, ctypes.byref(H), ctypes.byref(L)))
        return H.value, L.value

    def build_jk_noalloc(self, D, J, K, stream=None, sync=False, only=None):
        """fk_build_jk_noalloc: the build in the library's fixed device scratch
        array (no allocation).  D, J, K: contiguous float64 CUDA tensors of
        the caller (J or K may be None with only="K" or "J")."""
        import torch
        oflag = {None: 0, "J": FK_J_ONLY, "K": FK_K_ONLY}[only]
        st = stream if stream is not None else torch.cuda.current_stream(D.device)
        flags = FK_DEVICE_PTRS | (FK_SYNC if sync else 0) | oflag
        self._check(_lib.fk_build_jk_noalloc(self._ctx, ctypes.c_void_p(D.data_ptr()),
                                             ctypes.c_void_p(J.data_ptr() if J is not None else None),
                                             ctypes.c_void_p(K.data_ptr() if K is not None else None), flags,
                                             ctypes.c_void_p(st.cuda_stream)))
        return J, K

    def build_progress(self):
        """(finished, total) class launches of the last timed build."""
        d, t = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.fk_build_progress(self._ctx, ctypes.byref(d), ctypes.byref(t)))
        return d.value, t.value

    def stats(self):
        s = Stats()
        self._check(_lib.fk_stats(self._ctx, ctypes.byref(s)))
        out = []
        for i in range(s.nclass):
            out.append({"class": (s.la[i], s.lb[i], s.lc[i], s.ld[i]), "quartets": s.quartets[i],
                        "prim_quartets": s.prim_quartets[i], "flops_per_prim": s.flops_per_prim[i],
                        "flops_per_quartet": s.flops_per_quartet[i], "ms": s.class_ms[i],
                        "tiles": s.tiles[i], "team_size": s.team_size[i], "precision": s.precision[i],
                        "prim_slots": s.prim_slots[i], "engine": s.engine[i],
                        "schedule": [s.bra_block[i], s.kets_per_tile[i], s.grid_fraction[i]],
                        "block_tasks": s.block_tasks[i], "waves_per_group": s.waves_per_group[i]})
        return {"classes": out, "flops_total": s.flops_total,
                "quartets": sum(c["quartets"] for c in out), "prim_quartets": sum(c["prim_quartets"] for c in out)}

    # ---- one-electron / SCF ----
    def one_electron(self):
        n = self.nbf
        S, T, V = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
        e = ctypes.c_double()
        self._check(_lib.fk_one_electron(self._ctx, _ptr(S), _ptr(T), _ptr(V), ctypes.byref(e)))
        return S, T, V, e.value

    def run_scf(self, D0=None, max_iter=100, e_tol=1e-10, g_tol=1e-8, diis_n=8, lindep=1e-8, guess=None,
                graph=False, incremental=0, canonical=0.0, j_engine=False, density_eig=False):
        """guess: GUESS_CORE (default without D0), GUESS_GIVEN (default with
        D0), GUESS_SAD or GUESS_LEARNED; max_iter=0 returns the initial
        density only; canonical > 0: canonical orthogonalisation dropping
        overlap eigenvalues up to it."""
        n = self.nbf
        D = np.zeros((n, n)) if D0 is None else np.ascontiguousarray(D0, dtype=np.float64).copy()
        if guess is None:
            guess = GUESS_CORE if D0 is None else GUESS_GIVEN
        o = ScfOpts(int(max_iter), float(e_tol), float(g_tol), int(diis_n), int(guess), float(lindep), int(bool(graph)),
                    int(incremental), float(canonical), int(bool(j_engine)), int(bool(density_eig)))
        r = ScfResult()
        rc = _lib.fk_run_scf(self._ctx, ctypes.byref(o), ctypes.byref(r), _ptr(D))
        if rc not in (FK_OK, FK_ERR_NOT_CONVERGED):
            self._check(rc)
        res = {k: getattr(r, k) for k, _ in ScfResult._fields_}
        res["D"] = D
        return res

    # ---- kernel schedules ----
    def set_class_schedule(self, la, lb, lc, ld, bra_block=0, kets_per_tile=0, grid_fraction=1.0):
        self._check(_lib.fk_set_class_schedule(self._ctx, int(la), int(lb), int(lc), int(ld), int(bra_block),
                                               int(kets_per_tile), float(grid_fraction)))
        return self

    def set_class_lanes(self, la, lb, lc, ld, lanes):
        """Lanes per quartet of the class's kernel (1: lane kernel; the team
        alternative's lane count where the class has one)."""
        self._check(_lib.fk_set_class_lanes(self._ctx, int(la), int(lb), int(lc), int(ld), int(lanes)))
        return self

    def set_class_block_tasks(self, la, lb, lc, ld, enable=True):
        """Allow (default) or forbid block tasks for the class."""
        self._check(_lib.fk_set_class_block_tasks(self._ctx, int(la), int(lb), int(lc), int(ld), 1 if enable else 0))
        return self

    def set_class_engine(self, la, lb, lc, ld, engine):
        """engine: "rys" / "hgp" (or ENGINE_RYS / ENGINE_HGP) for the class."""
        e = {"rys": ENGINE_RYS, "hgp": ENGINE_HGP}.get(engine, engine)
        self._check(_lib.fk_set_class_engine(self._ctx, int(la), int(lb), int(lc), int(ld), int(e)))
        return self

    def save_schedules(self, path):
        self._check(_lib.fk_save_schedules(self._ctx, os.fsencode(path)))
        return self

    def load_schedules(self, path):
        self._check(_lib.fk_load_schedules(self._ctx, os.fsencode(path)))
        return self

    def autotune(self, D, reps=2, stream=None):
        """Tunes the class schedules on density D (numpy or device tensor);
        returns the report as a dict with a per-launch list."""
        r = TuneReport()
        if _torch is not None and isinstance(D, _torch.Tensor):
            rc = _lib.fk_autotune(self._ctx, ctypes.c_void_p(D.data_ptr()), FK_DEVICE_PTRS, int(reps),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(r))
        else:
            Dc = np.ascontiguousarray(D, dtype=np.float64)
            rc = _lib.fk_autotune(self._ctx, _ptr(Dc), 0, int(reps), None, ctypes.byref(r))
        self._check(rc)
        rows = [{k: getattr(r, k)[i] for k in ("la", "lb", "lc", "ld", "precision", "bra_block", "kets_per_tile",
                                                 "grid_fraction", "engine", "changed", "ms_default", "ms_tuned",
                                                 "block_tasks", "lanes_per_quartet")} for i in range(r.nclass)]
        return {"classes": rows, "build_ms_default": r.build_ms_default, "build_ms_tuned": r.build_ms_tuned,
                "configurations": r.configurations}

    def run_scf_batch(self, D0=None, max_iter=100, e_tol=1e-10, g_tol=1e-8, diis_n=8, lindep=1e-8, guess=None,
                      canonical=0.0, graph=False, density_eig=False):
        """SCF of every molecule of a batch at once; returns (list of per-molecule
        result dicts, flat density array in the batch layout)."""
        nmol = self.info()["nmol"]
        nmat = self.info()["nmat"]
        D = np.zeros(nmat) if D0 is None else np.ascontiguousarray(D0, dtype=np.float64).reshape(-1).copy()
        if guess is None:
            guess = GUESS_CORE if D0 is None else GUESS_GIVEN
        o = ScfOpts(int(max_iter), float(e_tol), float(g_tol), int(diis_n), int(guess), float(lindep), int(bool(graph)),
                    0, float(canonical), 0, int(bool(density_eig)))
        rs = (ScfResult * nmol)()
        rc = _lib.fk_run_scf_batch(self._ctx, ctypes.byref(o), rs, _ptr(D))
        if rc not in (FK_OK, FK_ERR_NOT_CONVERGED):
            self._check(rc)
        return [{k: getattr(r, k) for k, _ in ScfResult._fields_} for r in rs], D

    # ---- initial guesses ----
    def sad_density(self):
        """SAD density (nbf x nbf; a batch: the flat batch layout)."""
        info = self.info()
        if info["nmol"] > 1:
            D = np.zeros(info["nmat"])
        else:
            D = np.zeros((self.nbf, self.nbf))
        self._check(_lib.fk_sad_density(self._ctx, _ptr(D)))
        return D

    def guess_pairs(self):
        """(features [npair, GUESS_NFEAT] float32, shape codes [npair] int32)."""
        n = ctypes.c_int()
        self._check(_lib.fk_guess_pairs(self._ctx, ctypes.byref(n), None, None))
        X = np.zeros((n.value, GUESS_NFEAT), dtype=np.float32)
        sh = np.zeros(n.value, dtype=np.int32)
        self._check(_lib.fk_guess_pairs(self._ctx, ctypes.byref(n), _ptr(X), _ptr(sh)))
        return X, sh

    def guess_targets(self, D):
        n = ctypes.c_int()
        self._check(_lib.fk_guess_pairs(self._ctx, ctypes.byref(n), None, None))
        Y = np.zeros((n.value, GUESS_NOUT), dtype=np.float32)
        Dc = np.ascontiguousarray(D, dtype=np.float64)
        self._check(_lib.fk_guess_targets(self._ctx, _ptr(Dc), _ptr(Y)))
        return Y

    def set_guess_model(self, Ws, bs):
        """Ws[k]: (dims[k], dims[k+1]) arrays, bs[k]: (dims[k+1],); None removes."""
        if Ws is None:
            self._check(_lib.fk_set_guess_model(self._ctx, None))
            return self
        Wc = [np.ascontiguousarray(W, dtype=np.float32) for W in Ws]
        bc = [np.ascontiguousarray(b, dtype=np.float32) for b in bs]
        m = mlp_struct([W.shape[0] for W in Wc] + [Wc[-1].shape[1]], [_ptr(W) for W in Wc], [_ptr(b) for b in bc])
        self._check(_lib.fk_set_guess_model(self._ctx, ctypes.byref(m)))
        return self

    def guess_predict(self):
        D = np.zeros((self.nbf, self.nbf))
        self._check(_lib.fk_guess_predict(self._ctx, _ptr(D)))
        return D

    # ---- diagnostics ----
    def check_indices(self):
        self._check(_lib.fk_check_indices(self._ctx))
    def debug_eri(self, quartets, on_device=True, engine="rys"):
        q = np.ascontiguousarray(np.asarray(quartets, dtype=np.int32).reshape(-1, 4))
        shapes = [tuple(_ncart(int(self.sh_l[s])) for s in row) for row in q]
        tot = sum(int(np.prod(s)) for s in shapes)
        out = np.zeros(max(tot, 1))
        e = {"rys": ENGINE_RYS, "hgp": ENGINE_HGP, "mmd": 2}.get(engine, engine)
        self._check(_lib.fk_debug_eri(self._ctx, len(q), _ptr(q), _ptr(out), (1 if on_device else 0) | (2 * int(e))))
        res, o = [], 0
        for s in shapes:
            m = int(np.prod(s))
            res.append(out[o:o + m].reshape(s))
            o += m
        return res


# ---- network primitives on device tensors (training and inference) ----------
def mlp_struct(dims, Wptrs, bptrs):
    m = Mlp()
    m.nlayer = len(dims) - 1
    for k, d in enumerate(dims):
        m.dims[k] = int(d)
    for k in range(m.nlayer):
        m.W[k] = Wptrs[k]
        m.b[k] = bptrs[k]
    return m


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(_torch.cuda.current_stream().cuda_stream)


def _mlp_dev(Ws, bs):
    return mlp_struct([W.shape[0] for W in Ws] + [Ws[-1].shape[1]], [_dev(W) for W in Ws], [_dev(b) for b in bs])


def _rc(rc, what):
    if rc:
        raise FockJKError(rc, what + " failed")


def mlp_work(Ws, n):
    """Device workspace (float32 tensor) for mlp_forward on n rows."""
    m = mlp_struct([W.shape[0] for W in Ws] + [Ws[-1].shape[1]], [None] * len(Ws), [None] * len(Ws))
    k = _lib.fk_mlp_work_floats(ctypes.byref(m), int(n))
    return _torch.empty(max(int(k), 1), dtype=_torch.float32, device=Ws[0].device)


def mlp_forward(Ws, bs, X, work):
    """Y = network(X) on the device (float32 CUDA tensors, contiguous)."""
    m = _mlp_dev(Ws, bs)
    Y = _torch.empty((X.shape[0], Ws[-1].shape[1]), dtype=_torch.float32, device=X.device)
    _rc(_lib.fk_mlp_forward(ctypes.byref(m), _dev(X), int(X.shape[0]), _dev(Y), _dev(work), _stream()),
        "fk_mlp_forward")
    return Y


def mlp_backward(Ws, bs, X, work, dY, gWs, gbs):
    """Fills gWs, gbs with the gradients; dY is overwritten."""
    m, g = _mlp_dev(Ws, bs), _mlp_dev(gWs, gbs)
    _rc(_lib.fk_mlp_backward(ctypes.byref(m), _dev(X), int(X.shape[0]), _dev(work), _dev(dY), ctypes.byref(g),
                             _stream()), "fk_mlp_backward")


def block_mse(Y, T, shape, count, dY, part, loss):
    _rc(_lib.fk_mlp_block_mse(_dev(Y), _dev(T), _dev(shape), int(Y.shape[0]), float(count), _dev(dY), _dev(part),
                              _dev(loss), _stream()), "fk_mlp_block_mse")


def mse_scratch(device):
    return _torch.empty(_lib.fk_mlp_mse_scratch(), dtype=_torch.float64, device=device)


def mlp_adam(Ws, bs, gWs, gbs, m1W, m1b, m2W, m2b, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m, g = _mlp_dev(Ws, bs), _mlp_dev(gWs, gbs)
    a, v = _mlp_dev(m1W, m1b), _mlp_dev(m2W, m2b)
    _rc(_lib.fk_mlp_adam(ctypes.byref(m), ctypes.byref(g), ctypes.byref(a), ctypes.byref(v), int(step), float(lr),
                         float(b1), float(b2), float(eps), _stream()), "fk_mlp_adam")
