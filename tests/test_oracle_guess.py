"""Pins of the guess oracle (oracle/guess.py) against facts that do not come
from it: the oracle's independently pinned integrals and SCF, group theory,
finite differences and closed forms.  Each test names what a plausible
mistake would break."""
import math

import numpy as np
import pytest

import oracle
from oracle import guess as og
from oracle.scf import run_scf
from synth import geometry as geom
from synth import workloads as wl


def _rot(seed):
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.normal(size=(3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def _rotated(mol, Q):
    m = dict(mol)
    m["xyz"] = np.asarray(mol["xyz"]) @ Q.T
    return m


def _full_rotation(sys, Q):
    n = sys["nbf"]
    T = np.zeros((n, n))
    for a in range(len(sys["Z"])):
        f = og.atom_functions(sys, a)
        T[np.ix_(f, f)] = og.atom_rotation(sys, a, Q)
    return T


def test_rotation_matches_overlap_of_rotated_molecule():
    """S of the rotated molecule is T(Q) S T(Q)^T; the overlap integrals are
    pinned on their own, so a wrong component order, normalisation ratio
    (x^2 vs xy) or transposed Q fails here.  6-31G*-type water has s, p, d."""
    mol = geom.water_cluster(1, 3)
    s = wl.make_system(mol, "6-31gs-type")
    Q = _rot(1)
    s2 = wl.make_system(_rotated(mol, Q), "6-31gs-type")
    S, S2 = oracle.oneel(s)[0], oracle.oneel(s2)[0]
    T = _full_rotation(s, Q)
    assert np.max(np.abs(T @ S @ T.T - S2)) < 1e-12


def test_rotation_is_a_representation():
    """T(Q1 Q2) = T(Q1) T(Q2), T(I) = I, T(Q^T) = T(Q)^-1, up to f."""
    Q1, Q2 = _rot(2), _rot(3)
    for l in range(4):
        n = og.ncart(l)
        assert np.allclose(og.cart_rotation(l, np.eye(3)), np.eye(n), atol=1e-14)
        assert np.allclose(og.cart_rotation(l, Q1 @ Q2), og.cart_rotation(l, Q1) @ og.cart_rotation(l, Q2),
                           atol=1e-12)
        assert np.allclose(og.cart_rotation(l, Q1.T) @ og.cart_rotation(l, Q1), np.eye(n), atol=1e-12)


def test_density_transforms_contravariantly():
    """The SCF density of the rotated molecule is T(Q^T)^T D T(Q^T) (the
    oracle's SCF is pinned by the textbook H2 energy and invariants)."""
    mol = geom.water_cluster(1, 5)
    s = wl.make_system(mol, "6-31gs-type")
    Q = _rot(4)
    s2 = wl.make_system(_rotated(mol, Q), "6-31gs-type")
    D, D2 = run_scf(s)["D"], run_scf(s2)["D"]
    Tt = _full_rotation(s, Q.T)
    assert np.max(np.abs(Tt.T @ D @ Tt - D2)) < 1e-6


def test_local_frame():
    """Right-handed orthonormal frames: a pair's e_z along the pair and its
    nearest off-axis neighbour in the x-z half-plane with x > 0; an atom's
    own frame points e_z at its nearest neighbour; a lone atom keeps the lab
    frame."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.8, 0.2, -0.1], [-0.6, 1.9, 0.3], [0.1, -0.2, 6.0]])
    for a, b in [(0, 1), (1, 0), (0, 0), (2, 2), (3, 3), (0, 3)]:
        Q = og.local_frame(xyz, a, b)
        assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-14) and np.linalg.det(Q) > 0
    Q = og.local_frame(xyz, 0, 1)
    assert np.allclose(Q[:, 2], xyz[1] / np.linalg.norm(xyz[1]))
    v = Q.T @ (xyz[2] - xyz[0])  # atom 2, nearest off-axis neighbour of atom 0
    assert v[0] > 0 and abs(v[1]) < 1e-14
    Q = og.local_frame(xyz, 0, 0)
    assert np.allclose(Q[:, 2], xyz[1] / np.linalg.norm(xyz[1]))
    v = Q.T @ xyz[2]
    assert v[0] > 0 and abs(v[1]) < 1e-14
    assert np.allclose(og.local_frame(xyz[:1], 0, 0), np.eye(3))


def _dimer():
    return wl.make_system(geom.water_cluster(2, 8), "6-31gs-type")


def test_targets_round_trip():
    """Blocks taken into their frames and assembled back reproduce every pair
    block of a random symmetric density."""
    s = _dimer()
    rng = np.random.default_rng(2)
    A = rng.normal(size=(s["nbf"], s["nbf"]))
    D = A + A.T
    pairs = og.pair_list(s)
    Da = og.assemble(s, pairs, og.targets(s, D, pairs))
    for a, b in pairs:
        fa, fb = og.atom_functions(s, a), og.atom_functions(s, b)
        assert np.max(np.abs(Da[np.ix_(fa, fb)] - D[np.ix_(fa, fb)])) < 1e-12


def test_features_and_targets_turn_with_the_molecule():
    """Rotating and translating the molecule changes neither the features nor
    the pair-frame blocks of its SCF density: the frames are built from the
    atoms, and the blocks transform with T (pinned above by the overlaps)."""
    mol = geom.water_cluster(2, 8)
    s = wl.make_system(mol, "6-31gs-type")
    m2 = _rotated(mol, _rot(21))
    m2["xyz"] = m2["xyz"] + np.array([0.7, -1.1, 0.4])
    s2 = wl.make_system(m2, "6-31gs-type")
    p1, p2 = og.pair_list(s), og.pair_list(s2)
    assert p1 == p2
    assert np.max(np.abs(og.features(s, p1) - og.features(s2, p2))) < 1e-12
    Y1 = og.targets(s, run_scf(s)["D"], p1)
    Y2 = og.targets(s2, run_scf(s2)["D"], p2)
    assert np.max(np.abs(Y1 - Y2)) < 1e-6


def _co():
    mol = {"Z": np.array([6, 8], dtype=np.int32), "charge": 0, "name": "CO",
           "xyz": np.array([[0.1, 0.2, -0.3], [0.1, 0.2, -0.3]]) + np.array([[0, 0, 0], [1.2, -0.9, 1.5]])}
    return mol


def test_features_closed_form():
    s = wl.make_system(_co(), "6-31gs-type")
    pairs = og.pair_list(s)
    X = og.features(s, pairs)
    assert X.shape == (3, og.N_FEAT)
    # one-hots: C = index 1, O = index 3
    assert list(X[1, :8]) == [0, 0, 0, 1, 0, 1, 0, 0]
    R = float(np.linalg.norm(s["xyz"][1] - s["xyz"][0]))
    step = og.R_CUT / (og.N_RBF - 1)
    k = 3
    assert X[1, 8 + k] == pytest.approx(math.exp(-((R - k * step) / step) ** 2), rel=1e-14)
    assert X[0, 8] == 1.0  # on-site pair: R = 0 at the first centre
    assert og.pair_shape(s, pairs) == [(15, 15), (15, 15), (15, 15)]
    base = 8 + og.N_RBF
    # the C-O pair: neither atom has a neighbour besides its partner
    assert np.all(X[1, base:] == 0)
    # carbon's own pair: oxygen (slot 3) on the frame's z axis, both shells
    env = X[0, base:base + og.N_ENV].reshape(len(og.ELEMENTS), len(og.ENV_SHELLS), og.ENV_MOMENTS)
    for sh, (c0, w) in enumerate(og.ENV_SHELLS):
        wt = math.exp(-((R - c0) / w) ** 2)
        assert np.allclose(env[3, sh], wt * np.array([1, 0, 0, 1, 0, 0, 0, 0, 0, 1]), atol=1e-15)
    assert np.all(env[:3] == 0)
    assert np.all(X[0, base:base + og.N_ENV] == X[0, base + og.N_ENV:])


def test_pair_list_cutoff():
    mol = {"Z": np.array([1, 1, 1, 1], dtype=np.int32), "charge": 0, "name": "H4",
           "xyz": np.array([[0, 0, 0], [0, 0, 1.9], [0, 0, 8.5], [0, 0, 20.0]])}  # bohr
    s = wl.make_system(mol, "sto-3g")
    r = np.asarray(s["xyz"]).reshape(-1, 3)[:, 2]
    pairs = og.pair_list(s)
    expect = [(i, j) for i in range(4) for j in range(i, 4) if i == j or abs(r[i] - r[j]) < og.R_CUT]
    assert pairs == expect


def test_purify_fixed_point_and_invariants():
    """A converged SCF density is its own projection; any symmetric input
    gives Tr(DS) = N and DSD = 2D; the projection ignores positive scaling."""
    s = wl.water4_sto3g()
    r = run_scf(s)
    S, D = r["S"], r["D"]
    nocc = s["nelec"] // 2
    assert np.max(np.abs(og.purify(S, D, nocc) - D)) < 1e-9
    assert np.max(np.abs(og.purify(S, 3.7 * D, nocc) - D)) < 1e-9
    rng = np.random.default_rng(3)
    A = rng.normal(size=D.shape)
    P = og.purify(S, D + 0.05 * (A + A.T), nocc)
    assert np.trace(P @ S) == pytest.approx(s["nelec"], abs=1e-9)
    assert np.max(np.abs(P @ S @ P - 2 * P)) < 1e-9


def _mlp(seed, dims):
    rng = np.random.default_rng(seed)
    Ws = [rng.normal(size=(dims[k], dims[k + 1])) / math.sqrt(dims[k]) for k in range(len(dims) - 1)]
    bs = [0.1 * rng.normal(size=dims[k + 1]) for k in range(len(dims) - 1)]
    return Ws, bs


def test_silu_closed_forms():
    assert og.silu(np.array(0.0)) == 0.0 and og.dsilu(np.array(0.0)) == 0.5
    assert og.silu(np.array(40.0)) == pytest.approx(40.0, rel=1e-15)
    z = np.linspace(-4, 4, 9)
    h = 1e-6
    assert np.allclose(og.dsilu(z), (og.silu(z + h) - og.silu(z - h)) / (2 * h), atol=1e-8)


def test_mlp_gradient_finite_differences():
    """Backward pass and masked loss against central differences: a dropped
    activation derivative, a transposed weight or a mask off by a row fails."""
    dims = [og.N_FEAT, 7, 5, og.NB_PAD * og.NB_PAD]
    Ws, bs = _mlp(5, dims)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(4, dims[0]))
    T = rng.normal(size=(4, dims[-1]))
    shapes = [(15, 15), (15, 2), (2, 2), (2, 15)]

    def loss():
        return og.block_mse(og.mlp_forward(Ws, bs, X)[0], T, shapes)[0]

    Y, pre = og.mlp_forward(Ws, bs, X)
    _, dY = og.block_mse(Y, T, shapes)
    dWs, dbs = og.mlp_backward(Ws, bs, X, pre, dY)
    h = 1e-6
    for k in range(3):
        for (i, j) in [(0, 0), (1, 3), (dims[k] - 1, dims[k + 1] - 1)]:
            w0 = Ws[k][i, j]
            Ws[k][i, j] = w0 + h
            lp = loss()
            Ws[k][i, j] = w0 - h
            lm = loss()
            Ws[k][i, j] = w0
            assert dWs[k][i, j] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)
        j = dims[k + 1] // 2
        b0 = bs[k][j]
        bs[k][j] = b0 + h
        lp = loss()
        bs[k][j] = b0 - h
        lm = loss()
        bs[k][j] = b0
        assert dbs[k][j] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)
    # entries outside a row's block do not reach the loss
    assert np.all(dY[2].reshape(15, 15)[2:, :] == 0) and np.all(dY[1].reshape(15, 15)[:, 2:] == 0)


def test_adam_first_step_closed_form():
    """From zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 0.0, 1e-3])
    W, m, v = og.adam(np.ones(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(W, 1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_occupations():
    e = np.array([-1.0, -0.5, -0.2, -0.2 + 1e-6, -0.2 - 1e-6, 0.3])
    assert list(og.occupations(e, 6)) == pytest.approx([2, 2, 2 / 3, 2 / 3, 2 / 3, 0])
    assert list(og.occupations(e, 5)) == pytest.approx([2, 2, 1 / 3, 1 / 3, 1 / 3, 0])


def test_sad_closed_shell_atom_is_rhf():
    """For the oxide ion (10 electrons, every level full) the fractional
    scheme is plain RHF: its density equals the pinned oracle SCF's."""
    mol = {"Z": np.array([8], dtype=np.int32), "xyz": np.zeros((1, 3)), "charge": -2, "name": "O2-"}
    s = wl.make_system(mol, "6-31gs-type")
    a = og.atom_system(s, 0)
    a["nelec"] = 10
    D = og.atomic_density(a)
    assert np.max(np.abs(D - run_scf(s)["D"])) < 1e-7


def test_sad_invariants():
    """Trace = electron count; each atom's block is spherically symmetric
    (invariant under any rotation) and the blocks between atoms vanish."""
    s = wl.make_system(geom.water_cluster(2, 8), "6-31gs-type")
    D = og.sad_density(s)
    S = oracle.oneel(s)[0]
    assert np.trace(D @ S) == pytest.approx(s["nelec"], abs=1e-9)
    fO = og.atom_functions(s, 0)
    T = og.atom_rotation(s, 0, _rot(13).T)
    blk = D[np.ix_(fO, fO)]
    assert np.max(np.abs(T.T @ blk @ T - blk)) < 1e-9
    fH = og.atom_functions(s, 1)
    assert np.all(D[np.ix_(fO, fH)] == 0)
