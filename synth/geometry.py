"""Seeded synthetic molecular geometries (all returned in bohr).

Workloads (the paper's own molecules and basis data are not available, so
these stand in for its linear and globular benchmark systems):

* ``water_cluster(n, seed)``: rigid waters (O-H 0.9572 A, H-O-H 104.52 deg),
  uniformly random orientations; water i >= 1 is placed with its O at a
  distance U(2.7, 3.5) A from the O of a uniformly chosen earlier water;
  rejected if any O-O < 2.7 A or any intermolecular atom pair < 1.5 A.
* ``alkane(n, seed, jitter)``: all-trans n-CnH(2n+2), C-C 1.54 A, C-H 1.09 A,
  tetrahedral angles, staggered methyl caps, per-coordinate uniform jitter.
* ``water_sphere(n, seed)``: n rigid waters packed at 1.0 g/cm^3 inside a
  sphere, O by random sequential addition (min O-O 2.5 A), random orientation,
  min intermolecular atom-atom 1.2 A.
* ``h2(R)``: the hydrogen molecule at bond length R bohr.
* ``organic(seed)``: a random closed-shell organic molecule: 3-30 heavy atoms
  (C/N/O with probabilities 0.7/0.15/0.15 under their valences 4/3/2) on a
  random branched tree, with probability 0.4 a planar 5- or 6-membered carbon
  ring first; heavy-heavy bonds U(1.30, 1.55) A, X-H U(1.00, 1.10) A; every
  free valence capped with H; placements rejected if a non-bonded pair comes
  closer than 1.7 A (heavy) or 1.2 A (involving H).

Holds none of the method's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

ANGSTROM = 1.0 / 0.529177210903  # bohr per angstrom
MASTER_SEED = 20240731

ROH, HOH = 0.9572, math.radians(104.52)


def _rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _water_body():
    h = HOH / 2
    return np.array([[0.0, 0.0, 0.0],
                     [ROH * math.sin(h), 0.0, ROH * math.cos(h)],
                     [-ROH * math.sin(h), 0.0, ROH * math.cos(h)]])


def _mol(Z, xyz_ang, charge=0, name=""):
    return {"name": name, "Z": np.asarray(Z, dtype=np.int32),
            "xyz": np.asarray(xyz_ang, dtype=np.float64) * ANGSTROM, "charge": int(charge)}


def water_cluster(n: int, seed: int, dmin=2.7, dmax=3.5, jitter=0.0):
    rng = np.random.default_rng(seed)
    body = _water_body()
    mols = [body @ _rand_rot(rng).T]
    tries = 0
    while len(mols) < n:
        tries += 1
        if tries > 100000:
            raise RuntimeError("water_cluster: placement failed")
        j = int(rng.integers(len(mols)))
        o = mols[j][0] + rng.uniform(dmin, dmax) * _unit(rng)
        w = body @ _rand_rot(rng).T + o
        ok = True
        for m in mols:
            if np.linalg.norm(m[0] - w[0]) < dmin:
                ok = False
                break
            if np.min(np.linalg.norm(m[:, None, :] - w[None, :, :], axis=-1)) < 1.5:
                ok = False
                break
        if ok:
            mols.append(w)
    xyz = np.concatenate(mols)
    if jitter:
        xyz = xyz + rng.uniform(-jitter, jitter, size=xyz.shape)
    return _mol([8, 1, 1] * n, xyz, name=f"(H2O){n}")


def water_sphere(n: int, seed: int, density=1.0, dmin=2.5, amin=1.2):
    rng = np.random.default_rng(seed)
    vol_per = 18.01528 / (density * 0.602214076)  # A^3 per molecule
    R = (3 * n * vol_per / (4 * math.pi)) ** (1 / 3)
    body = _water_body()
    mols = []
    tries = 0
    while len(mols) < n:
        tries += 1
        if tries > 2000000:
            raise RuntimeError("water_sphere: placement failed")
        o = R * rng.uniform() ** (1 / 3) * _unit(rng)
        if any(np.linalg.norm(m[0] - o) < dmin for m in mols):
            continue
        for _ in range(20):
            w = body @ _rand_rot(rng).T + o
            if all(np.min(np.linalg.norm(m[:, None, :] - w[None, :, :], axis=-1)) >= amin for m in mols):
                mols.append(w)
                break
    return _mol([8, 1, 1] * n, np.concatenate(mols), name=f"(H2O){n}-sphere")


def alkane(n: int, seed: int, jitter=0.02, rcc=1.54, rch=1.09):
    rng = np.random.default_rng(seed)
    th = math.acos(-1 / 3)  # tetrahedral angle
    half = th / 2
    C = np.array([[i * rcc * math.sin(half), (0.5 if i % 2 else -0.5) * rcc * math.cos(half), 0.0]
                  for i in range(n)])
    H = []
    for i in range(n):
        nb = [C[j] - C[i] for j in (i - 1, i + 1) if 0 <= j < n]
        if len(nb) == 2:
            u1, u2 = (v / np.linalg.norm(v) for v in nb)
            b = -(u1 + u2)
            b /= np.linalg.norm(b)
            nrm = np.cross(u1, u2)
            nrm /= np.linalg.norm(nrm)
            for s in (1, -1):
                H.append(C[i] + rch * (math.cos(half) * b + s * math.sin(half) * nrm))
        else:
            if n == 1:
                a = np.array([1.0, 0, 0])
                e1 = np.array([0, 1.0, 0])
            else:
                a = nb[0] / np.linalg.norm(nb[0])
                # in-plane direction trans to the next carbon: away from the zig-zag
                e1 = np.array([0.0, -1.0 if C[i][1] > 0 else 1.0, 0.0]) if n > 1 else np.array([0, 1.0, 0])
                e1 = e1 - (e1 @ a) * a
                e1 /= np.linalg.norm(e1)
            e2 = np.cross(a, e1)
            for k in range(3 if n > 1 else 4):
                if n == 1:
                    break
                phi = 2 * math.pi * k / 3
                d = math.cos(th) * a + math.sin(th) * (math.cos(phi) * e1 + math.sin(phi) * e2)
                H.append(C[i] + rch * d)
    xyz = np.concatenate([C, np.array(H)])
    xyz = xyz + rng.uniform(-jitter, jitter, size=xyz.shape)
    return _mol([6] * n + [1] * len(H), xyz, name=f"C{n}H{2*n+2}")


def _free_direction(rng, pos, center, bonded, tries=200):
    """Unit vector from `center` that keeps the new atom away from the bonded
    neighbours' directions (best of random candidates)."""
    best, score = None, -1e9
    dirs = [(pos[j] - center) / np.linalg.norm(pos[j] - center) for j in bonded]
    for _ in range(tries):
        d = _unit(rng)
        s_ = min((-(d @ u) for u in dirs), default=1.0)
        if s_ > score:
            best, score = d, s_
    return best


def organic(seed: int, hmin=3, hmax=30):
    rng = np.random.default_rng(seed)
    valence = {6: 4, 7: 3, 8: 2}
    for _attempt in range(200):
        nh = int(rng.integers(hmin, hmax + 1))
        Z, pos, nbrs = [], [], []
        if rng.random() < 0.4 and nh >= 6:
            ring = 6 if rng.random() < 0.5 else 5
            r = 1.40 / (2 * math.sin(math.pi / ring))
            for k in range(ring):
                a = 2 * math.pi * k / ring
                Z.append(6)
                pos.append(np.array([r * math.cos(a), r * math.sin(a), 0.0]))
                nbrs.append([(k - 1) % ring, (k + 1) % ring])
        else:
            Z.append(6)
            pos.append(np.zeros(3))
            nbrs.append([])
        ok = True
        while len(Z) < nh and ok:
            el = int(rng.choice([6, 7, 8], p=[0.7, 0.15, 0.15]))
            free = [i for i in range(len(Z)) if len(nbrs[i]) < valence[Z[i]] - (1 if len(Z) < nh - 1 else 0)]
            if not free:
                free = [i for i in range(len(Z)) if len(nbrs[i]) < valence[Z[i]]]
            if not free:
                ok = False
                break
            placed = False
            for _t in range(30):
                i = int(rng.choice(free))
                d = _free_direction(rng, pos, pos[i], nbrs[i])
                p_new = pos[i] + rng.uniform(1.30, 1.55) * d
                if all(np.linalg.norm(p_new - pos[j]) >= 1.7 for j in range(len(Z)) if j != i):
                    Z.append(el)
                    pos.append(p_new)
                    nbrs.append([i])
                    nbrs[i].append(len(Z) - 1)
                    placed = True
                    break
            if not placed:
                ok = False
        if not ok:
            continue
        heavy = len(Z)
        H = []
        for i in range(heavy):
            for _ in range(valence[Z[i]] - len(nbrs[i])):
                placed = False
                for _t in range(60):
                    d = _free_direction(rng, pos + H, pos[i], nbrs[i], tries=60)
                    p_new = pos[i] + rng.uniform(1.00, 1.10) * d
                    # H keeps 1.2 A from every atom other than its own
                    if all(np.linalg.norm(p_new - q) >= 1.2 for j, q in enumerate(pos + H) if j != i):
                        H.append(p_new)
                        nbrs[i].append(len(pos) + len(H) - 1)
                        placed = True
                        break
                if not placed:
                    break
            else:
                continue
            break
        else:
            xyz = np.array(pos + H)
            return _mol(Z + [1] * len(H), xyz, name=f"org{seed}-h{heavy}")
    raise RuntimeError("organic: no valid molecule after 200 attempts")


def h2(R=1.4):
    return {"name": "H2", "Z": np.array([1, 1], dtype=np.int32),
            "xyz": np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]]), "charge": 0}


def nelec(mol):
    return int(np.sum(mol["Z"])) - int(mol["charge"])
