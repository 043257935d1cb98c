"""Host-side checks of libfockjk that need no GPU: exported symbols, the Rys
tables, the per-quartet integral code evaluated on the host, one-electron
integrals, screening lists and argument validation."""
import json
import math
import os
import re

import mpmath
import numpy as np
import pytest

import oracle
import paper_2407_21445_amd as fk
from synth import workloads as wl
from test_oracle import _rand_sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "fockjk.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|void|const char \*)\s*(fk_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 12
    import ctypes
    lib = ctypes.CDLL(fk.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(fk.EXPORTS)


@pytest.mark.parametrize("n", range(1, 8))
def test_rys_moments(n):
    """sum_i w_i u_i^k = F_k(T) for k < 2n (the defining property of the rule),
    against 30-digit Boys values, across the table, its interval edges and the
    asymptotic region."""
    mpmath.mp.dps = 30
    Ts = [0.0, 1e-9, 0.25, 0.5, 3.7, 15.999, 16.0, 16.001, 29.3, 47.0, 63.999, 64.0, 64.5, 90.0, 400.0]
    # either side of the switch from the table to the Gauss-Hermite rule
    sw = {1: 36.0, 2: 42.0, 3: 47.0, 4: 52.0, 5: 57.0, 6: 61.0, 7: 64.0}[n]
    Ts += [sw - 1e-9, sw, sw + 1e-9, sw + 0.5]
    for T in Ts:
        u, w = fk.rys_host(n, T)
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0)
        for k in range(2 * n):
            if T == 0:
                ref = 1.0 / (2 * k + 1)
            else:
                ref = float(mpmath.gammainc(k + 0.5, 0, T) / (2 * mpmath.mpf(T) ** (k + 0.5)))
            got = float(np.sum(w * u ** k))
            assert abs(got - ref) <= 1e-13 * ref + 1e-300, (n, T, k, got, ref)


def test_rys_n1_closed_form():
    for T in [0.0, 0.3, 2.0, 11.0, 40.0, 70.0]:
        F = oracle.boys(1, T)
        u, w = fk.rys_host(1, T)
        assert w[0] == pytest.approx(F[0], rel=1e-14)
        assert u[0] == pytest.approx(F[1] / F[0], rel=1e-13)


def test_host_eri_matches_oracle_all_classes():
    """The production per-quartet Rys code (run on the host) against the
    oracle's McMurchie-Davidson integrals, random shells up to (ff|ff)."""
    s = _rand_sys(21, lmax=3, natom=4, kmax=2)
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0)
    rng = np.random.default_rng(4)
    qs = [rng.integers(0, s["nshell"], size=4) for _ in range(60)]
    qs += [[3, 7, 11, 15], [2, 6, 10, 14], [1, 5, 9, 13], [0, 4, 8, 12], [3, 3, 3, 3], [7, 3, 3, 7]]
    res = c.debug_eri(qs, on_device=False)
    for q, a in zip(qs, res):
        b = oracle.eri_quartet(s, *q)
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b))), q


def _hgp_built(la, lb, lc, ld):
    """Classes with an HGP kernel: lane-per-quartet classes (at most 54
    Cartesian integrals) with la+lb+lc+ld <= 4."""
    n = [(l + 1) * (l + 2) // 2 for l in (la, lb, lc, ld)]
    return la + lb + lc + ld <= 4 and n[0] * n[1] * n[2] * n[3] <= 54


def test_host_hgp_matches_oracle():
    """The HGP engine's per-quartet code (vertical recurrences per primitive
    quartet, early contraction, horizontal recurrences), run on the host,
    against the oracle's McMurchie-Davidson integrals for every ordered
    (la, lb, lc, ld) with L <= 4 it is built for, three primitives per shell;
    the other classes are refused with FK_ERR_UNSUPPORTED."""
    s = _rand_sys(21, lmax=3, natom=4, kmax=3)
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0)
    rng = np.random.default_rng(5)
    nb = 0
    for la in range(4):
        for lb in range(4):
            for lc in range(4):
                for ld in range(4):
                    if la + lb + lc + ld > 4:
                        continue
                    at = rng.integers(0, 4, size=4)
                    q = [4 * at[0] + la, 4 * at[1] + lb, 4 * at[2] + lc, 4 * at[3] + ld]
                    cl = sorted([tuple(sorted((la, lb), reverse=True)), tuple(sorted((lc, ld), reverse=True))],
                                reverse=True)
                    if not _hgp_built(*cl[0], *cl[1]):
                        with pytest.raises(fk.FockJKError) as e:
                            c.debug_eri([q], on_device=False, engine="hgp")
                        assert e.value.code == fk.FK_ERR_UNSUPPORTED
                        continue
                    a = c.debug_eri([q], on_device=False, engine="hgp")[0]
                    r = c.debug_eri([q], on_device=False)[0]
                    b = oracle.eri_quartet(s, *q)
                    scale = max(1.0, float(np.max(np.abs(b))))
                    assert np.max(np.abs(a - b)) <= 1e-12 * scale, q
                    assert np.max(np.abs(a - r)) <= 1e-13 * scale, q
                    nb += 1
    assert nb == 65


def test_class_engine_arguments():
    s = _rand_sys(21, lmax=3, natom=4, kmax=2)
    c = fk.FockJK(device=-1).set_system(s)
    c.set_class_engine(1, 0, 1, 0, "hgp").set_class_engine(0, 0, 2, 2, "hgp").set_class_engine(1, 1, 1, 1, "rys")
    for bad in [(1, 1, 1, 1, "hgp"), (3, 3, 0, 0, "hgp")]:
        with pytest.raises(fk.FockJKError) as e:
            c.set_class_engine(*bad)
        assert e.value.code == fk.FK_ERR_UNSUPPORTED
    with pytest.raises(fk.FockJKError) as e:
        c.set_class_engine(1, 0, 0, 0, 2)
    assert e.value.code == fk.FK_ERR_ARG
    with pytest.raises(fk.FockJKError) as e:
        c.set_class_engine(0, 1, 0, 0, "rys")
    assert e.value.code == fk.FK_ERR_ARG


def test_one_electron_matches_oracle():
    s = _rand_sys(22, lmax=3, natom=3, kmax=3)
    s["charge"] = 1  # three H nuclei: keep the electron count even
    c = fk.FockJK(device=-1).set_system(s)
    S, T, V, en = c.one_electron()
    So, To, Vo = oracle.oneel(s)
    assert np.max(np.abs(S - So)) < 1e-13
    assert np.max(np.abs(T - To)) < 1e-12
    assert np.max(np.abs(V - Vo)) < 1e-11
    assert en == pytest.approx(oracle.enuc(s), rel=1e-14)


def _schwarz_oracle(s):
    n = s["nshell"]
    G = {}
    for a in range(n):
        for b in range(a + 1):
            v = oracle.eri_quartet(s, a, b, a, b)
            G[(a, b)] = math.sqrt(float(np.max(np.abs(np.einsum("ijij->ij", v)))))
    return G


@pytest.mark.parametrize("tau", [0.0, 1e-10, 1e-6, 1e-3])
def test_schwarz_quartet_count(tau):
    """Unique quartets kept by the ket-prefix lists equal the brute-force count
    of unordered pair pairs with G_ab G_cd >= tau."""
    s = wl.water4_sto3g()
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=tau)
    G = np.array(list(_schwarz_oracle(s).values()))
    npair = len(G)
    assert c.info()["npair"] == npair == s["nshell"] * (s["nshell"] + 1) // 2
    prod = np.outer(G, G)
    iu = np.tril_indices(npair)
    ref = int(np.sum(prod[iu] >= tau)) if tau > 0 else len(iu[0])
    got = c.info()["nquartet_schwarz"]
    # pairs whose product sits within rounding of tau may fall either side
    near = int(np.sum(np.abs(prod[iu] - tau) <= 1e-12 * tau)) if tau > 0 else 0
    assert abs(got - ref) <= near
    if tau == 0:
        assert got == 22155


def test_argument_validation():
    s = wl.h2_sto3g()
    c = fk.FockJK(device=-1)
    Z = np.array([1, 1], dtype=np.int32)
    xyz = np.zeros(6)
    P = fk._ptr
    with pytest.raises(fk.FockJKError) as e:
        c._check(fk._lib.fk_set_geometry(c._ctx, 0, P(Z), P(xyz), 0))
    assert e.value.code == fk.FK_ERR_ARG
    with pytest.raises(fk.FockJKError) as e:  # odd electron count
        c._check(fk._lib.fk_set_geometry(c._ctx, 2, P(Z), P(xyz), 1))
    assert e.value.code == fk.FK_ERR_ARG
    with pytest.raises(fk.FockJKError) as e:  # basis before geometry
        c._check(fk._lib.fk_set_basis(c._ctx, 1, P(np.zeros(1, np.int32)), P(np.zeros(1, np.int32)),
                                      P(np.ones(1, np.int32)), P(np.ones(1)), P(np.ones(1))))
    assert e.value.code == fk.FK_ERR_STATE
    c.set_system(s)
    bad = dict(s)
    bad["sh_l"] = np.array([4, 0], dtype=np.int32)
    with pytest.raises(fk.FockJKError) as e:
        c.set_system(bad)
    assert e.value.code == fk.FK_ERR_UNSUPPORTED
    bad = dict(s)
    bad["exps"] = s["exps"].copy()
    bad["exps"][1] = -1.0
    with pytest.raises(fk.FockJKError) as e:
        c.set_system(bad)
    assert e.value.code == fk.FK_ERR_ARG
    bad = dict(s)
    bad["sh_nprim"] = np.array([10, 3], dtype=np.int32)
    with pytest.raises(fk.FockJKError):
        c.set_system(bad)
    c.set_system(s)
    with pytest.raises(fk.FockJKError) as e:  # J/K before the quartet lists
        c.build_jk(np.eye(2))
    assert e.value.code == fk.FK_ERR_STATE
    c.build_quartets(tau=0.0)
    with pytest.raises(fk.FockJKError) as e:  # host-only context has no device
        c.build_jk(np.eye(2))
    assert e.value.code == fk.FK_ERR_STATE


@pytest.mark.parametrize("name,tau,tau_prim,tau_fp32", [
    ("spdf", 0.0, 0.0, 0.0), ("water4", 1e-10, 1e-12, 0.0),
    ("c20h42", 0.0, 0.0, 0.0), ("c20h42", 1e-10, 0.0, 0.0), ("c20h42", 1e-10, 1e-12, 0.0),
    ("water64", 1e-10, 1e-12, 1e-5), ("organic2", 1e-10, 1e-12, 0.0)])
def test_kernel_indices_in_bounds(name, tau, tau_prim, tau_fp32):
    """Every address the J/K kernels form from the tile, list, group and pair
    tables (positions, transposed ket records, bra records, density,
    shell-block maxima, Fock accumulators) lies inside its array, for the test
    systems and the full-size benchmark configurations: C20H42, (H2O)64 with
    the precision split (its FP64 and FP32 launches walk the same tiles), and
    the first two molecules of the organic batch (f shells, molecule
    offsets)."""
    if name == "spdf":
        s = _rand_sys(33, lmax=3, natom=3, kmax=2)
        s["charge"] = 1
    elif name == "water4":
        s = wl.water4_sto3g()
    elif name == "water64":
        s = wl.water64_ccpvdz()
    elif name == "organic2":
        s = wl.organic_batch(2)
    else:
        s = wl.c20h42_631gs()
    c = fk.FockJK(device=-1).set_system(s)
    if name == "organic2":
        c.set_molecules(s["atom_mol"])
    c.build_quartets(tau=tau, tau_prim=tau_prim, tau_fp32=tau_fp32)
    c.check_indices()
    assert c.info()["ntile"] > 0


def test_scf_needs_device():
    s = wl.water4_sto3g()
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0)
    with pytest.raises(fk.FockJKError) as e:
        c.run_scf()
    assert e.value.code == fk.FK_ERR_STATE


@pytest.mark.parametrize("tau_fp32", [1e-5, 1e-3])
def test_precision_split_lists(tau_fp32):
    """The split adds an FP32 launch per class (but f-f bras) over the same
    tiles: the Schwarz quartet count is unchanged and every kernel address
    stays in bounds (which launch computes a quartet is decided per build
    from the density)."""
    s = wl.water4_sto3g()
    ref = fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0)
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0, tau_fp32=tau_fp32)
    assert c.info()["nquartet_schwarz"] == ref.info()["nquartet_schwarz"] == 22155
    prec = [x["precision"] for x in c.stats()["classes"]]
    assert 32 in prec and 64 in prec and len(prec) > len(ref.stats()["classes"])
    c.check_indices()
    with pytest.raises(fk.FockJKError):
        fk.FockJK(device=-1).set_system(s).build_quartets(tau=0.0, tau_fp32=-1.0)


def _small_batch():
    spdf = _rand_sys(33, lmax=3, natom=3, kmax=2)
    spdf["charge"] = 1
    spdf["nelec"] -= 1
    return wl.batch([wl.water4_sto3g(), wl.h2_sto3g(), wl.alkane_sys(2, "6-31gs-type"), spdf])


@pytest.mark.parametrize("tau", [0.0, 1e-10])
def test_batch_lists(tau):
    """A batch holds each molecule's own quartets and nothing across
    molecules: unique quartet count = sum of the separate counts; the block
    layout follows the molecules' sizes; every kernel address stays inside
    its molecule's blocks."""
    b = _small_batch()
    c = fk.FockJK(device=-1).set_system(b).set_molecules(b["atom_mol"]).build_quartets(tau=tau)
    sep = sum(fk.FockJK(device=-1).set_system(m).build_quartets(tau=tau).info()["nquartet_schwarz"] for m in b["mols"])
    assert c.info()["nquartet_schwarz"] == sep
    nbf, off = c.molecule_layout()
    assert list(nbf) == [m["nbf"] for m in b["mols"]]
    assert off[-1] == c.info()["nmat"] == sum(m["nbf"] ** 2 for m in b["mols"])
    c.check_indices()


def test_batch_validation():
    b = _small_batch()
    c = fk.FockJK(device=-1).set_system(b)
    bad = b["atom_mol"].copy()
    bad[0], bad[-1] = bad[-1], bad[0]  # not non-decreasing
    with pytest.raises(fk.FockJKError):
        c.set_molecules(bad)
    c.set_molecules(b["atom_mol"]).build_quartets(tau=0.0)
    with pytest.raises(fk.FockJKError) as e:
        c.one_electron()
    assert e.value.code == fk.FK_ERR_UNSUPPORTED


# ------------------------------------------------------------ initial guesses
def _guess_sys(kind):
    from synth import geometry as geom
    if kind == "water2":
        return wl.make_system(geom.water_cluster(2, 8), "6-31gs-type")
    if kind == "propane":
        return wl.make_system(geom.alkane(3, 5, jitter=0.05), "6-31gs-type")
    return wl.make_system(geom.water_cluster(2, 9), "sto-3g")


@pytest.mark.parametrize("kind", ["water2", "propane", "water2_sto3g"])
def test_guess_features_and_targets_match_oracle(kind):
    """Pair list, features, shapes and pair-frame targets (host) against the
    oracle on a random density: the same pairs in the same order, features
    and targets to FP32 rounding."""
    from oracle import guess as og
    s = _guess_sys(kind)
    c = fk.FockJK(device=-1).set_system(s)
    X, sh = c.guess_pairs()
    pairs = og.pair_list(s)
    assert len(X) == len(pairs)
    assert np.max(np.abs(X - og.features(s, pairs))) < 1e-6
    assert [(int(v) >> 8, int(v) & 255) for v in sh] == og.pair_shape(s, pairs)
    D = wl.random_density(s, 3)
    Yo = og.targets(s, D, pairs)
    assert np.max(np.abs(c.guess_targets(D) - Yo)) <= 1e-6 * max(1.0, np.max(np.abs(Yo)))


@pytest.mark.parametrize("kind", ["water2", "propane"])
def test_sad_density_matches_oracle(kind):
    from oracle import guess as og
    s = _guess_sys(kind)
    c = fk.FockJK(device=-1).set_system(s)
    assert np.max(np.abs(c.sad_density() - og.sad_density(s))) < 1e-9


def test_guess_errors():
    s = _guess_sys("water2")
    c = fk.FockJK(device=-1).set_system(s)
    with pytest.raises(fk.FockJKError) as e:  # weights live on a device
        c.set_guess_model([np.zeros((fk.GUESS_NFEAT, 225))], [np.zeros(225)])
    assert e.value.code == fk.FK_ERR_STATE
    b = _small_batch()
    cb = fk.FockJK(device=-1).set_system(b).set_molecules(b["atom_mol"])
    with pytest.raises(fk.FockJKError) as e:
        cb.guess_pairs()
    assert e.value.code == fk.FK_ERR_UNSUPPORTED
    m = fk.mlp_struct([32, 225], [None], [None])
    assert fk._lib.fk_mlp_forward(fk.ctypes.byref(m), None, 1, None, None, None) == fk.FK_ERR_ARG


# ------------------------------------------------------------ kernel schedules
@pytest.mark.parametrize("sched", [(32, 64, 0.25), (1, 1, 1.0), (3, 17, 0.5)])
def test_class_schedules_keep_the_lists(sched):
    """Any schedule regroups the same Schwarz quartets into tiles: the quartet
    count is unchanged and every kernel address stays in bounds."""
    s = wl.alkane_sys(3, "6-31gs-type")
    ref = fk.FockJK(device=-1).set_system(s).build_quartets(tau=1e-10).info()
    c = fk.FockJK(device=-1).set_system(s)
    for la in range(3):
        for lb in range(la + 1):
            for lc in range(3):
                for ld in range(lc + 1):
                    c.set_class_schedule(la, lb, lc, ld, *sched)
    c.build_quartets(tau=1e-10)
    c.check_indices()
    assert c.info()["nquartet_schwarz"] == ref["nquartet_schwarz"]


def test_class_schedule_errors():
    c = fk.FockJK(device=-1).set_system(wl.water4_sto3g())
    for bad in [(0, 1, 0, 0, 0, 0, 1.0), (1, 0, 0, 0, 33, 0, 1.0), (1, 0, 0, 0, 0, 65, 1.0), (1, 0, 0, 0, 0, 0, 0.0), (1, 0, 0, 0, 0, 0, 4.5)]:
        with pytest.raises(fk.FockJKError) as e:
            c.set_class_schedule(*bad)
        assert e.value.code == fk.FK_ERR_ARG
    c.build_quartets(tau=0.0)
    with pytest.raises(fk.FockJKError) as e:
        c.autotune(np.zeros((28, 28)))
    assert e.value.code == fk.FK_ERR_STATE


def test_sad_density_batch_layout():
    """SAD of a batch: each molecule's block equals the oracle's SAD of that
    molecule alone, in the batch layout."""
    from oracle import guess as og
    from synth import geometry as geom
    mols = [wl.make_system(geom.water_cluster(2, 8), "6-31gs-type"), wl.alkane_sys(2, "6-31gs-type")]
    b = wl.batch(mols)
    c = fk.FockJK(device=-1).set_system(b).set_molecules(b["atom_mol"])
    D = c.sad_density()
    nbf, off = c.molecule_layout()
    for m, s in enumerate(mols):
        assert np.max(np.abs(D[off[m]:off[m + 1]].reshape(nbf[m], nbf[m]) - og.sad_density(s))) < 1e-9
    with pytest.raises(fk.FockJKError) as e:
        c.build_quartets(tau=1e-10).run_scf_batch()
    assert e.value.code == fk.FK_ERR_STATE


def test_sad_density_mixed_bases():
    """A batch mixing bases gives each atom the atomic density of its own
    shells (hydrogen in STO-3G and in 6-31G*-type)."""
    from oracle import guess as og
    mols = [wl.h2_sto3g(), wl.alkane_sys(2, "6-31gs-type")]
    b = wl.batch(mols)
    c = fk.FockJK(device=-1).set_system(b).set_molecules(b["atom_mol"])
    D = c.sad_density()
    nbf, off = c.molecule_layout()
    for m, s in enumerate(mols):
        assert np.max(np.abs(D[off[m]:off[m + 1]].reshape(nbf[m], nbf[m]) - og.sad_density(s))) < 1e-9


def test_bench_traffic_follows_the_schedule(tmp_path, monkeypatch):
    """bench.py reports the committed counter traffic only for the kernel
    sources, the class schedule and the integral engine it was measured
    under."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = {"workload": "c20h42", "source_sha256": bench._kernel_source_hash(), "copy_scale_fetch": 2.0,
         "copy_scale_write": 1.0,
         "kernels": [{"kernel": "J/K class (ps|ss)", "schedule": [8, 64, 1.0], "fetch_bytes_per_launch": 10.0,
                      "write_bytes_per_launch": 100.0},
                     {"kernel": "J/K class (ps|ss)", "schedule": [8, 64, 4.0], "fetch_bytes_per_launch": 20.0,
                      "write_bytes_per_launch": 300.0},
                     {"kernel": "J/K class (ps|ss)", "schedule": [8, 64, 1.0], "engine": "hgp",
                      "fetch_bytes_per_launch": 30.0, "write_bytes_per_launch": 300.0},
                     {"kernel": "J/K class (ss|ss)", "fetch_bytes_per_launch": 1.0, "write_bytes_per_launch": 1.0}]}
    os.makedirs(tmp_path / "profiles")
    with open(tmp_path / "profiles" / "roofline_traffic.json", "w") as f:
        json.dump(t, f)
    # the hash is taken from the real sources; only the profile directory moves
    real_hash = bench._kernel_source_hash()
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: real_hash)
    assert bench._traffic("J/K class (ps|ss)", "c20h42", [8, 64, 1.0]) == 120.0
    assert bench._traffic("J/K class (ps|ss)", "c20h42", (8, 64, 4.0)) == 340.0
    assert bench._traffic("J/K class (ps|ss)", "c20h42", [8, 64, 1.0], "hgp") == 360.0
    assert bench._traffic("J/K class (ps|ss)", "c20h42", [8, 64, 2.0]) is None
    assert bench._traffic("J/K class (ss|ss)", "c20h42", [8, 64, 1.0]) is None   # no schedule: never matched
    assert bench._traffic("J/K class (ps|ss)", "water64", [8, 64, 1.0]) is None
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "other sources")
    assert bench._traffic("J/K class (ps|ss)", "c20h42", [8, 64, 1.0]) is None


def test_schedule_cache_round_trip(tmp_path):
    """fk_save_schedules / fk_load_schedules: the schedules and engines set
    on one context reach another through the file; files for another
    architecture, malformed lines and engines a class lacks are refused and
    leave the context unchanged."""
    s = _rand_sys(21, lmax=2, natom=4, kmax=2)
    a = fk.FockJK(device=-1).set_system(s)
    a.set_class_schedule(1, 0, 0, 0, 4, 0, 2.0).set_class_schedule(2, 2, 1, 1, 1, 16, 0.5)
    a.set_class_engine(1, 0, 0, 0, "hgp").set_class_block_tasks(1, 0, 0, 0, False)
    p = str(tmp_path / "sched.txt")
    a.save_schedules(p)
    text = open(p).read()
    assert "arch host" in text
    assert "class 1 0 0 0 4 0 2 1 0 0" in text and "class 2 2 1 1 1 16 0.5 0 0 0" in text
    b = fk.FockJK(device=-1).set_system(s).load_schedules(p)
    p2 = str(tmp_path / "sched2.txt")
    b.save_schedules(p2)
    assert open(p2).read() == text
    for bad, code in [("arch gfx942\nclass 1 0 0 0 4 0 2 0\n", fk.FK_ERR_UNSUPPORTED),
                      ("arch host\nclass 1 0 0 0 4 0\n", fk.FK_ERR_ARG),
                      ("arch host\nclass 1 1 1 1 4 0 1 1\n", fk.FK_ERR_UNSUPPORTED),
                      ("class 1 0 0 0 4 0 2 0\n", fk.FK_ERR_ARG),
                      ("arch host\nclass 0 1 0 0 4 0 2 0\n", fk.FK_ERR_ARG),
                      ("arch host\nclass 1 0 0 0 4 0 2 0 2\n", fk.FK_ERR_ARG)]:
        q = tmp_path / "bad.txt"
        q.write_text(bad)
        c = fk.FockJK(device=-1).set_system(s).load_schedules(p)
        with pytest.raises(fk.FockJKError) as e:
            c.load_schedules(str(q))
        assert e.value.code == code, bad
        c.save_schedules(p2)
        assert open(p2).read() == text
    # a file without the block-task field (an older cache) allows block tasks
    q = tmp_path / "old.txt"
    q.write_text("arch host\nclass 1 0 0 0 4 0 2 0\n")
    d = fk.FockJK(device=-1).set_system(s).load_schedules(str(q))
    d.save_schedules(p2)
    assert "class 1 0 0 0 4 0 2 0 1 0" in open(p2).read()
    # the team alternative of a lane class travels as its lanes per quartet
    e = fk.FockJK(device=-1).set_system(s).set_class_lanes(2, 0, 1, 0, 6)
    e.save_schedules(p2)
    assert "class 2 0 1 0 0 0 1 0 0 6" in open(p2).read()
    f = fk.FockJK(device=-1).set_system(s).load_schedules(p2)
    f.save_schedules(str(tmp_path / "sched3.txt"))
    assert open(str(tmp_path / "sched3.txt")).read() == open(p2).read()
    q.write_text("arch host\nclass 2 0 1 0 0 0 1 0 1 3\n")
    with pytest.raises(fk.FockJKError) as ex:
        fk.FockJK(device=-1).set_system(s).load_schedules(str(q))
    assert ex.value.code == fk.FK_ERR_UNSUPPORTED


def test_class_kernel_choice():
    """Lanes per contracted quartet for every class up to f: one lane up to 54
    integrals; above it a team of NA lanes while a lane keeps at most 80
    integrals (NB NC ND), else NA NB lanes (NC ND <= 80), else the whole wave.
    (pp|pp), (fs|ds) and (fd|ss) are team classes (measured faster than as
    lane classes), (dp|ps) with 54 integrals a lane class; the wave classes
    (more than 64 bra component pairs: f-f bras) split each quartet over two
    waves (128 lanes)."""
    s = wl.organic_batch(1)
    c = fk.FockJK(device=-1).set_system(s).build_quartets(tau=1e-10)
    nc = [1, 3, 6, 10]
    got = {r["class"]: r["team_size"] for r in c.stats()["classes"]}
    assert len(got) == 55
    for (la, lb, lc, ld), ts in got.items():
        NA, NB, NC, ND = nc[la], nc[lb], nc[lc], nc[ld]
        if NA * NB * NC * ND <= 54:
            want = 1
        elif NB * NC * ND <= 80:
            want = NA
        elif NA * NB <= 64 and NC * ND <= 80:
            want = NA * NB
        else:
            want = 64 if NA * NB <= 64 else 128
        assert ts == want, ((la, lb, lc, ld), ts, want)
    assert got[(1, 1, 1, 1)] == 3 and got[(3, 0, 2, 0)] == 10 and got[(3, 2, 0, 0)] == 10
    assert got[(2, 1, 1, 0)] == 1
    c.close()


def test_block_tasks_partition_the_tiles():
    """Block tasks (fk_screen_opts.block_tasks = 0): the tiles of the ket-outer
    lane classes ((ss|ss), (ps|ss): four-wave workgroups, the same tiles; on by
    default) and of the bra-outer lane classes built for eight-wave workgroups
    (on where the schedule asks; their bra block lowered until the K rows fit)
    are regrouped so that each workgroup task holds tiles of one bra block; the
    other classes are untouched.  fk_build_quartets checks the partition, the
    bras per block against the rows and every ket's LDS row columns itself
    (validate_lists).  Without a device the LDS bound alone decides."""
    s = wl.c20h42_631gs()
    wide = {(1, 0, 1, 0), (1, 1, 0, 0), (1, 1, 1, 0), (2, 0, 0, 0), (2, 0, 1, 0), (2, 1, 0, 0), (2, 1, 1, 0)}
    dflt = {x["class"]: x for x in fk.FockJK(device=-1).set_system(s).build_quartets(
        tau=1e-10, tau_prim=1e-12).stats()["classes"]}
    assert all(x["block_tasks"] == 0 for k, x in dflt.items() if k in wide)
    c = fk.FockJK(device=-1).set_system(s)
    for w in wide:
        c.set_class_block_tasks(*w, True)
    on = c.build_quartets(tau=1e-10, tau_prim=1e-12).stats()["classes"]
    off = fk.FockJK(device=-1).set_system(s).build_quartets(tau=1e-10, tau_prim=1e-12,
                                                             block_tasks=False).stats()["classes"]
    assert len(on) == len(off)
    ko = {(0, 0, 0, 0), (1, 0, 0, 0)}
    seen = set()
    for a, b in zip(on, off):
        assert a["class"] == b["class"]
        assert b["block_tasks"] == 0 and b["waves_per_group"] == 4
        if a["class"] in ko:
            assert 0 < a["block_tasks"] <= a["tiles"] and a["waves_per_group"] == 4
            assert (a["tiles"], a["prim_slots"]) == (b["tiles"], b["prim_slots"])
            seen.add(a["class"])
        elif a["block_tasks"] > 0:
            assert a["class"] in wide and a["waves_per_group"] == 8
            assert a["schedule"][0] <= b["schedule"][0] and a["tiles"] >= b["tiles"]
            seen.add(a["class"])
        else:
            assert (a["tiles"], a["prim_slots"], a["waves_per_group"]) == (b["tiles"], b["prim_slots"], 4)
    assert ko <= seen and len(seen & wide) >= 5
    one = fk.FockJK(device=-1).set_system(s).set_class_block_tasks(1, 0, 0, 0, False)
    st = {x["class"]: x["block_tasks"] for x in one.build_quartets(tau=1e-10, tau_prim=1e-12).stats()["classes"]}
    assert st[(1, 0, 0, 0)] == 0 and st[(0, 0, 0, 0)] > 0


def test_class_lanes_select_the_team_alternative():
    """fk_set_class_lanes: a lane class with a team alternative runs it with
    one lane per component of its first bra shell (fk_stats team_size), over
    the same quartets; lane counts a class has no kernel for are refused."""
    s = wl.alkane_sys(2, "6-31gs-type")
    base = {x["class"]: x for x in fk.FockJK(device=-1).set_system(s).build_quartets(tau=1e-10).stats()["classes"]}
    c = fk.FockJK(device=-1).set_system(s)
    for cls, lanes in (((2, 0, 1, 0), 6), ((1, 1, 1, 0), 3), ((2, 1, 0, 0), 6)):
        c.set_class_lanes(*cls, lanes)
    st = {x["class"]: x for x in c.build_quartets(tau=1e-10).stats()["classes"]}
    assert st[(2, 0, 1, 0)]["team_size"] == 6 and st[(1, 1, 1, 0)]["team_size"] == 3
    assert st[(2, 1, 0, 0)]["team_size"] == 6 and st[(1, 0, 0, 0)]["team_size"] == 1
    for k, x in st.items():
        assert x["quartets"] == base[k]["quartets"]
    c.set_class_lanes(2, 0, 1, 0, 1)
    assert {x["class"]: x for x in c.build_quartets(tau=1e-10).stats()["classes"]}[(2, 0, 1, 0)]["team_size"] == 1
    for cls, lanes in (((1, 0, 0, 0), 3), ((2, 0, 1, 0), 3), ((1, 1, 1, 1), 1)):
        with pytest.raises(fk.FockJKError) as e:
            c.set_class_lanes(*cls, lanes)
        assert e.value.code == fk.FK_ERR_UNSUPPORTED
    c.set_class_lanes(1, 1, 1, 1, 3)  # a team class keeps its own kernel


def test_screen_option_validation():
    s = wl.water4_sto3g()
    c = fk.FockJK(device=-1).set_system(s)
    for kw in ({"tau": -1.0}, {"tau_fp32": -1e-5}, {"tau_k": -5e-6}):
        with pytest.raises(fk.FockJKError) as e:
            c.build_quartets(**kw)
        assert e.value.code == fk.FK_ERR_ARG
    o = fk.ScreenOpts(1e-10, 0.0, 1, 0, 0.0, 0.0, 1)
    assert fk._lib.fk_build_quartets(c._ctx, fk.ctypes.byref(o)) == fk.FK_ERR_ARG
    c.build_quartets(tau=1e-10, tau_k=5e-6)


def test_xcd_region_order_keeps_the_lists_valid():
    """A molecule whose density exceeds one XCD's L2 ((H2O)32, 800 functions)
    gets its lane classes' tiles, and block tasks with their tiles, placed by
    XCD region.  The lists stay a valid partition (fk_build_quartets checks
    tiles, tasks and LDS row columns itself), both builds hold the same
    Schwarz quartets per class, and every address the kernels would form lies
    inside its buffer (the host index walk), with block tasks off and on for
    every class that has them."""
    from synth import geometry as geom
    s = wl.make_system(geom.water_sphere(32, wl.SEED + 3), "ccpvdz-type")
    assert s["nbf"] > 724
    wide = {(1, 0, 1, 0), (1, 1, 0, 0), (1, 1, 1, 0), (2, 0, 0, 0), (2, 0, 1, 0), (2, 1, 0, 0), (2, 1, 1, 0)}
    off = fk.FockJK(device=-1).set_system(s)
    off.build_quartets(tau=1e-10, tau_prim=1e-12, block_tasks=False)
    off.check_indices()
    on = fk.FockJK(device=-1).set_system(s)
    for w in wide:
        on.set_class_block_tasks(*w, True)
    on.build_quartets(tau=1e-10, tau_prim=1e-12)
    on.check_indices()
    a, b = on.stats()["classes"], off.stats()["classes"]
    assert any(x["block_tasks"] > 0 for x in a)
    for x, y in zip(a, b):
        assert x["class"] == y["class"] and x["quartets"] == y["quartets"]
