"""Learned initial density and the superposition-of-atomic-densities guess:
plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing else).  The
product library never imports, links or calls anything here, and nothing here
calls the product.

The paper has no initial-guess model (its SCF starts from a conventional
guess); this module states, in plain NumPy, what the library's learned guess
and its SAD fallback compute, so that they can be checked element by element.

Pieces (each written out from its definition, no blocking or fusion):

* ``cart_rotation(l, Q)``: the matrix T with phi_a(Q r) = sum_b T_ab phi_b(r)
  for the normalised Cartesian components phi of angular momentum l (the
  component order and normalisation of the paper's Cartesian Gaussians,
  "Notation").  A density block transforms as D' = T(Q^T)^T D T(Q^T) when the
  molecule is rotated by Q.
* ``pair_list`` / ``local_frame`` / ``features``: atom pairs within
  ``R_CUT`` (and every atom with itself), oriented heavier atom first; each
  pair's frame is fixed by its own atoms and their nearest neighbours (z
  along the pair, or towards an atom's nearest neighbour; x towards the
  nearest neighbour off that axis), so the frame turns with the molecule;
  features are element one-hots, Gaussian radial features of the distance,
  and each atom's environment as weighted moments (1, u, u u^T) of its
  neighbours' directions u in the pair frame, per element and radial shell.
* ``targets``: a density's pair blocks in each pair's frame, padded to
  15 x 15.
* ``assemble``: predicted blocks rotated back to the molecular frame and
  scattered into an nbf x nbf density (on-site blocks symmetrised).
* ``purify``: the projection onto an idempotent density with the right
  electron count: D0 = 2 S^-1/2 P S^-1/2, P the projector onto the nelec/2
  largest eigenvalues of S^1/2 D S^1/2 / 2.
* ``mlp_forward`` / ``mlp_backward`` / ``block_mse`` / ``adam``: the FP64
  statement of the network, its loss and its optimiser.
* ``sad_density``: block-diagonal density of spherically averaged atoms, each
  from an SCF with fractional occupations (F = h + J - K/2, D = sum n_i c_i
  c_i^T, equal occupation within a degenerate level).
"""
from __future__ import annotations

import math

import numpy as np

from . import eri_full, ncart, oneel

ELEMENTS = (1, 6, 7, 8)          # one-hot order: H, C, N, O
R_CUT = 8.0                      # bohr
N_RBF = 24
NB_PAD = 15                      # functions per atom in the padded block
ENV_SHELLS = ((0.0, 3.0), (5.0, 1.5))   # (centre, width) in bohr of the environment weights
ENV_MOMENTS = 10                 # 1, u_x, u_y, u_z, u_x^2, u_x u_y, u_x u_z, u_y^2, u_y u_z, u_z^2
N_ENV = len(ELEMENTS) * len(ENV_SHELLS) * ENV_MOMENTS
N_FEAT = 2 * len(ELEMENTS) + N_RBF + 2 * N_ENV
OFF_AXIS = 0.1                   # a reference direction needs |sin| above this


# ------------------------------------------------------------ rotations --
def cart_components(l):
    """(x, y, z) exponents in the library order: descending x, then y."""
    return [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


def _norm(e):
    """Relative normalisation of a Cartesian component (unit self-overlap)."""
    return 1.0 / math.sqrt(_dfact(2 * e[0] - 1) * _dfact(2 * e[1] - 1) * _dfact(2 * e[2] - 1))


def cart_rotation(l, Q):
    """T with phi_a(Q r) = sum_b T_ab phi_b(r), by expanding the monomial
    prod_i ((Q r)_i)^(e_i) into monomials of r."""
    comps = cart_components(l)
    index = {c: k for k, c in enumerate(comps)}
    T = np.zeros((len(comps), len(comps)))
    for a, e in enumerate(comps):
        # polynomial as {exponent triple: coefficient}
        poly = {(0, 0, 0): 1.0}
        for axis in range(3):
            for _ in range(e[axis]):
                new = {}
                for mono, cf in poly.items():
                    for j in range(3):
                        m = list(mono)
                        m[j] += 1
                        m = tuple(m)
                        new[m] = new.get(m, 0.0) + cf * Q[axis, j]
                poly = new
        for mono, cf in poly.items():
            b = index[mono]
            T[a, b] += cf * _norm(e) / _norm(mono)
    return T


def atom_shells(sys, atom):
    return [s for s in range(sys["nshell"]) if sys["sh_atom"][s] == atom]


def bf_offsets(sys):
    off = [0]
    for l in sys["sh_l"]:
        off.append(off[-1] + ncart(int(l)))
    return off


def atom_functions(sys, atom):
    off = bf_offsets(sys)
    return [f for s in atom_shells(sys, atom) for f in range(off[s], off[s + 1])]


def atom_rotation(sys, atom, Q):
    """Block-diagonal T(Q) over the atom's shells."""
    blocks = [cart_rotation(int(sys["sh_l"][s]), Q) for s in atom_shells(sys, atom)]
    n = sum(b.shape[0] for b in blocks)
    T = np.zeros((n, n))
    o = 0
    for b in blocks:
        T[o:o + len(b), o:o + len(b)] = b
        o += len(b)
    return T


def _frame_from(ez, ref):
    """Columns e_x, e_y, e_z: e_x along the part of ref orthogonal to e_z, or,
    without ref, along the lab axis least aligned with e_z (lowest index on
    ties)."""
    if ref is None:
        k = int(np.argmin(np.abs(ez)))
        ref = np.zeros(3)
        ref[k] = 1.0
    ex = ref - (ref @ ez) * ez
    ex /= np.linalg.norm(ex)
    return np.column_stack([ex, np.cross(ez, ex), ez])


def _neighbours(xyz, centre, exclude, r_cut=R_CUT):
    """Atoms within r_cut of atom `centre`, not in `exclude`, by distance on a
    1e-6 bohr grid, then index (so that distances equal by symmetry order the
    same way in any orientation)."""
    d = np.linalg.norm(xyz - xyz[centre], axis=1)
    ks = [k for k in range(len(xyz)) if k not in exclude and d[k] < r_cut]
    return sorted(ks, key=lambda k: (math.floor(d[k] * 1e6), k))


def _off_axis(xyz, origin, ez, cands):
    """First candidate whose direction from `origin` is off the e_z axis."""
    for k in cands:
        v = xyz[k] - xyz[origin]
        perp = v - (v @ ez) * ez
        if np.linalg.norm(perp) > OFF_AXIS * np.linalg.norm(v):
            return v
    return None


def local_frame(xyz, a, b):
    """Frame of the pair (a, b), columns e_x, e_y, e_z.  a != b: e_z from a to
    b; e_x towards the nearest off-axis neighbour of a (else of b).  a == b:
    e_z towards a's nearest neighbour, e_x towards the next nearest off-axis
    one.  Missing neighbours: lab axes (a lone atom: the lab frame)."""
    xyz = np.asarray(xyz, float).reshape(-1, 3)
    if a != b:
        ez = xyz[b] - xyz[a]
        ez = ez / np.linalg.norm(ez)
        ref = _off_axis(xyz, a, ez, _neighbours(xyz, a, {a, b}))
        if ref is None:
            ref = _off_axis(xyz, b, ez, _neighbours(xyz, b, {a, b}))
        return _frame_from(ez, ref)
    nb = _neighbours(xyz, a, {a})
    if not nb:
        return np.eye(3)
    ez = xyz[nb[0]] - xyz[a]
    ez = ez / np.linalg.norm(ez)
    return _frame_from(ez, _off_axis(xyz, a, ez, nb[1:]))


# ---------------------------------------------------------------- pairs --
def pair_list(sys, r_cut=R_CUT):
    """[(first, second)]: for i <= j (row-major over the atoms) every i == j,
    and every i < j with |R_i - R_j| < r_cut; first is the atom of higher Z
    (the lower index for equal Z)."""
    Z, xyz = sys["Z"], np.asarray(sys["xyz"], float).reshape(-1, 3)
    out = []
    for i in range(len(Z)):
        for j in range(i, len(Z)):
            if i != j and np.linalg.norm(xyz[i] - xyz[j]) >= r_cut:
                continue
            out.append((j, i) if Z[j] > Z[i] else (i, j))
    return out


def features(sys, pairs, r_cut=R_CUT):
    Z, xyz = sys["Z"], np.asarray(sys["xyz"], float).reshape(-1, 3)
    X = np.zeros((len(pairs), N_FEAT))
    mu = np.arange(N_RBF) * (r_cut / (N_RBF - 1))
    gamma = ((N_RBF - 1) / r_cut) ** 2
    base = 2 * len(ELEMENTS) + N_RBF
    for p, (a, b) in enumerate(pairs):
        X[p, ELEMENTS.index(int(Z[a]))] = 1.0
        X[p, len(ELEMENTS) + ELEMENTS.index(int(Z[b]))] = 1.0
        R = np.linalg.norm(xyz[b] - xyz[a])
        X[p, 2 * len(ELEMENTS):base] = np.exp(-gamma * (R - mu) ** 2)
        Q = local_frame(xyz, a, b)
        for side, atom in enumerate((a, b)):
            for k in range(len(Z)):
                if k in (a, b):
                    continue
                v = xyz[k] - xyz[atom]
                r = np.linalg.norm(v)
                if r >= r_cut:
                    continue
                u = Q.T @ (v / r)
                mom = [1.0, u[0], u[1], u[2], u[0] * u[0], u[0] * u[1], u[0] * u[2], u[1] * u[1], u[1] * u[2],
                       u[2] * u[2]]
                e = ELEMENTS.index(int(Z[k]))
                for sh, (c0, w) in enumerate(ENV_SHELLS):
                    wt = math.exp(-((r - c0) / w) ** 2)
                    o = base + side * N_ENV + (e * len(ENV_SHELLS) + sh) * ENV_MOMENTS
                    X[p, o:o + ENV_MOMENTS] += wt * np.array(mom)
    return X


def pair_shape(sys, pairs):
    return [(len(atom_functions(sys, a)), len(atom_functions(sys, b))) for a, b in pairs]


def targets(sys, D, pairs):
    """Pair blocks of D in each pair's frame (padded, flattened row-major
    15 x 15): D_frame = T(Q)^T D T(Q), the molecule rotated by Q^T."""
    xyz = np.asarray(sys["xyz"], float).reshape(-1, 3)
    Y = np.zeros((len(pairs), NB_PAD * NB_PAD))
    for p, (a, b) in enumerate(pairs):
        fa, fb = atom_functions(sys, a), atom_functions(sys, b)
        Q = local_frame(xyz, a, b)
        blk = atom_rotation(sys, a, Q).T @ D[np.ix_(fa, fb)] @ atom_rotation(sys, b, Q)
        pad = np.zeros((NB_PAD, NB_PAD))
        pad[:len(fa), :len(fb)] = blk
        Y[p] = pad.ravel()
    return Y


def assemble(sys, pairs, Y):
    """nbf x nbf density from pair-frame blocks: D_lab = T(Q^T)^T B T(Q^T)."""
    xyz = np.asarray(sys["xyz"], float).reshape(-1, 3)
    n = sys["nbf"]
    D = np.zeros((n, n))
    for p, (a, b) in enumerate(pairs):
        fa, fb = atom_functions(sys, a), atom_functions(sys, b)
        B = np.asarray(Y[p], float).reshape(NB_PAD, NB_PAD)[:len(fa), :len(fb)]
        Q = local_frame(xyz, a, b)
        L = atom_rotation(sys, a, Q.T).T @ B @ atom_rotation(sys, b, Q.T)
        if a == b:
            D[np.ix_(fa, fa)] = 0.5 * (L + L.T)
        else:
            D[np.ix_(fa, fb)] = L
            D[np.ix_(fb, fa)] = L.T
    return D


def purify(S, D, nocc):
    """2 S^-1/2 P S^-1/2 with P the projector onto the nocc largest
    eigenvalues of S^1/2 D S^1/2 / 2."""
    w, U = np.linalg.eigh(S)
    Sh = (U * np.sqrt(w)) @ U.T
    Si = (U / np.sqrt(w)) @ U.T
    e, V = np.linalg.eigh(Sh @ D @ Sh / 2)
    Vo = V[:, np.argsort(e)[::-1][:nocc]]
    return 2.0 * Si @ (Vo @ Vo.T) @ Si


# ------------------------------------------------------------------ MLP --
def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mlp_forward(Ws, bs, X):
    """Returns (output, pre-activations of every layer); SiLU after every
    layer but the last."""
    A, pre = np.asarray(X, float), []
    for k, (W, b) in enumerate(zip(Ws, bs)):
        Z = A @ W + b
        pre.append(Z)
        A = silu(Z) if k < len(Ws) - 1 else Z
    return A, pre


def mlp_backward(Ws, bs, X, pre, dY):
    """Gradients (dW list, db list) of a scalar whose gradient in the output
    is dY."""
    L = len(Ws)
    dWs, dbs = [None] * L, [None] * L
    G = np.asarray(dY, float)
    for k in range(L - 1, -1, -1):
        A_in = np.asarray(X, float) if k == 0 else silu(pre[k - 1])
        dWs[k] = A_in.T @ G
        dbs[k] = G.sum(axis=0)
        if k > 0:
            G = (G @ Ws[k].T) * dsilu(pre[k - 1])
    return dWs, dbs


def block_mse(Y, T, shapes, width=NB_PAD):
    """Mean of (Y - T)^2 over the entries (i, j), i < nA, j < nB, of each
    row's block; returns (loss, dloss/dY)."""
    M = np.zeros_like(np.asarray(Y, float))
    for r, (na, nb) in enumerate(shapes):
        m = np.zeros((width, width))
        m[:na, :nb] = 1.0
        M[r] = m.ravel()
    cnt = M.sum()
    R = (np.asarray(Y, float) - T) * M
    return float((R * R).sum() / cnt), 2.0 * R / cnt


def adam(W, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) with bias correction; returns the new
    (W, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return W - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ SAD --
def atom_system(sys, atom):
    """The atom's shells alone, at the origin, with its own electron count."""
    shells = atom_shells(sys, atom)
    poff = np.concatenate([[0], np.cumsum(sys["sh_nprim"])])
    exps = np.concatenate([sys["exps"][poff[s]:poff[s + 1]] for s in shells])
    coefs = np.concatenate([sys["coefs"][poff[s]:poff[s + 1]] for s in shells])
    Z = int(sys["Z"][atom])
    return {"Z": np.array([Z], dtype=np.int32), "xyz": np.zeros((1, 3)), "charge": 0, "nelec": Z,
            "sh_atom": np.zeros(len(shells), dtype=np.int32),
            "sh_l": np.asarray(sys["sh_l"])[shells].astype(np.int32),
            "sh_nprim": np.asarray(sys["sh_nprim"])[shells].astype(np.int32),
            "exps": exps, "coefs": coefs, "nshell": len(shells),
            "nbf": sum(ncart(int(sys["sh_l"][s])) for s in shells)}


def occupations(eps, nelec, tol=1e-4):
    """Aufbau over levels of orbitals within tol (hartree) of the level's
    lowest; a partly filled level shares its electrons equally."""
    order = np.argsort(eps)
    n = np.zeros(len(eps))
    left = float(nelec)
    i = 0
    while i < len(order) and left > 0:
        j = i
        while j < len(order) and eps[order[j]] - eps[order[i]] < tol:
            j += 1
        g = j - i
        each = min(2.0, left / g)
        n[order[i:j]] = each
        left -= each * g
        i = j
    return n


def atomic_density(asys, max_iter=500, tol=1e-10, mix=0.5):
    """Fractional-occupation SCF of one atom (damped fixed-point iteration
    on D from the core-Hamiltonian start)."""
    S, T, V = oneel(asys)
    h = T + V
    G = eri_full(asys)
    w, U = np.linalg.eigh(S)
    X = (U / np.sqrt(w)) @ U.T

    def density_of(F):
        e, C = np.linalg.eigh(X @ F @ X)
        C = X @ C
        n = occupations(e, asys["nelec"])
        return (C * n) @ C.T

    D = density_of(h)
    for _ in range(max_iter):
        J = np.einsum("ijkl,kl->ij", G, D)
        K = np.einsum("ikjl,kl->ij", G, D)
        Dn = density_of(h + J - 0.5 * K)
        delta = np.max(np.abs(Dn - D))
        D = Dn if delta < tol else mix * Dn + (1 - mix) * D
        if delta < tol:
            break
    return D


def sad_density(sys):
    """Block-diagonal superposition of the atoms' densities (one atomic
    calculation per element, on the first atom of that element)."""
    n = sys["nbf"]
    D = np.zeros((n, n))
    cache = {}
    for atom, Z in enumerate(sys["Z"]):
        key = int(Z)
        if key not in cache:
            cache[key] = atomic_density(atom_system(sys, atom))
        f = atom_functions(sys, atom)
        D[np.ix_(f, f)] = cache[key]
    return D
