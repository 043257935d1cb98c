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


def test_icosahedral_group():
    """60 distinct proper rotations, closed under products; averaging over
    them leaves a d-d block (degree 4 in the rotation) invariant under any
    rotation, i.e. it is the full rotational average."""
    G = og.icosahedral_rotations()
    assert len(G) == 60
    keys = {tuple(np.round(g, 6).ravel()) for g in G}
    for g in G:
        assert np.allclose(g @ g.T, np.eye(3), atol=1e-12) and np.linalg.det(g) > 0
    for g, h in [(G[7], G[31]), (G[59], G[12])]:
        assert tuple(np.round(g @ h, 6).ravel()) in keys
    rng = np.random.default_rng(7)
    B = rng.normal(size=(6, 6))
    avg = sum(og.cart_rotation(2, g.T).T @ B @ og.cart_rotation(2, g.T) for g in G) / 60
    Q = _rot(9)
    assert np.allclose(og.cart_rotation(2, Q.T).T @ avg @ og.cart_rotation(2, Q.T), avg, atol=1e-12)


def test_bond_frame():
    """Right-handed orthonormal frame with e_z along the bond."""
    a, b = np.array([0.3, -1.0, 2.0]), np.array([1.1, 0.4, 1.7])
    Q = og.bond_frame(a, b)
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-14) and np.linalg.det(Q) > 0
    assert np.allclose(Q[:, 2], (b - a) / np.linalg.norm(b - a))
    assert np.allclose(og.bond_frame(a, a), np.eye(3))


def _co():
    mol = {"Z": np.array([6, 8], dtype=np.int32), "charge": 0, "name": "CO",
           "xyz": np.array([[0.1, 0.2, -0.3], [0.1, 0.2, -0.3]]) + np.array([[0, 0, 0], [1.2, -0.9, 1.5]])}
    return mol


def test_targets_round_trip_linear_molecule():
    """The density of a closed-shell linear molecule is symmetric about its
    axis, so the bond block survives the azimuthal average and assembly
    unchanged (a wrong frame, rotation direction or average breaks this);
    the block is also independent of how the molecule is oriented."""
    mol = _co()
    s = wl.make_system(mol, "6-31gs-type")
    D = run_scf(s)["D"]
    pairs = og.pair_list(s)
    assert pairs == [(0, 0), (1, 0), (1, 1)]  # O (Z=8) first in the C-O pair
    Y = og.targets(s, D, pairs)
    Da = og.assemble(s, pairs, Y)
    fC, fO = og.atom_functions(s, 0), og.atom_functions(s, 1)
    assert np.max(np.abs(Da[np.ix_(fO, fC)] - D[np.ix_(fO, fC)])) < 1e-9
    s2 = wl.make_system(_rotated(mol, _rot(11)), "6-31gs-type")
    Y2 = og.targets(s2, run_scf(s2)["D"], og.pair_list(s2))
    assert np.max(np.abs(Y2 - Y)) < 1e-6


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
