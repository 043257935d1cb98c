"""Named seeded workloads: a molecule plus a synthetic basis, flattened into the
plain arrays that both the oracle and the library consume.

* ``water4_sto3g``  -- 4 waters, STO-3G-type (28 functions, s and p).
* ``c20h42_631gs``  -- all-trans C20H42 with 0.02 A jitter, 6-31G*-type
  (384 Cartesian functions, s, p and d).
* ``water64_ccpvdz`` -- 64 waters at 1.0 g/cm^3, cc-pVDZ-type (1600 functions).
* ``batch(systems)`` -- several systems as one batch (atoms, shells and
  primitives concatenated; ``atom_mol`` maps atoms to molecules).
* ``organic_batch(n)`` -- n random organic molecules in the def2-TZVP-like
  ``tzvp-type`` basis (s to f), the 256-molecule batched workload.
* small test systems (H2, short alkanes, water dimers) in any basis.
"""
from __future__ import annotations

import numpy as np

from . import basis as _basis
from . import geometry as _geom

SEED = _geom.MASTER_SEED


def make_system(mol, basis_name):
    shells = _basis.basis_for(basis_name, mol["Z"])
    return flatten(mol, shells, basis_name)


def flatten(mol, shells, basis_name="custom"):
    sh_atom = np.array([s["atom"] for s in shells], dtype=np.int32)
    sh_l = np.array([s["l"] for s in shells], dtype=np.int32)
    sh_nprim = np.array([len(s["exps"]) for s in shells], dtype=np.int32)
    exps = np.array([e for s in shells for e in s["exps"]], dtype=np.float64)
    coefs = np.array([c for s in shells for c in s["coefs"]], dtype=np.float64)
    nb = _basis.nbf(shells)
    return {
        "name": f"{mol.get('name', 'mol')}/{basis_name}",
        "Z": np.asarray(mol["Z"], dtype=np.int32),
        "xyz": np.ascontiguousarray(mol["xyz"], dtype=np.float64),
        "charge": int(mol["charge"]),
        "nelec": _geom.nelec(mol),
        "sh_atom": sh_atom, "sh_l": sh_l, "sh_nprim": sh_nprim,
        "exps": exps, "coefs": coefs, "nbf": nb, "nshell": len(shells),
    }


def water4_sto3g(seed=SEED + 1):
    return make_system(_geom.water_cluster(4, seed), "sto-3g")


def c20h42_631gs(seed=SEED + 2):
    return make_system(_geom.alkane(20, seed, jitter=0.02), "6-31gs-type")


def water64_ccpvdz(seed=SEED + 3):
    return make_system(_geom.water_sphere(64, seed), "ccpvdz-type")


def h2_sto3g(R=1.4):
    return make_system(_geom.h2(R), "sto-3g")


def alkane_sys(n, basis_name, seed=SEED + 10, jitter=0.02):
    return make_system(_geom.alkane(n, seed + n, jitter=jitter), basis_name)


def water_sys(n, basis_name, seed=SEED + 20):
    return make_system(_geom.water_cluster(n, seed + n), basis_name)


def subset_shells(sys, keep):
    """A system restricted to the shells whose indices are in ``keep``
    (used for tiny brute-force cases)."""
    keep = np.asarray(sorted(keep))
    off = np.concatenate([[0], np.cumsum(sys["sh_nprim"])])
    exps = np.concatenate([sys["exps"][off[i]:off[i + 1]] for i in keep])
    coefs = np.concatenate([sys["coefs"][off[i]:off[i + 1]] for i in keep])
    out = dict(sys)
    out.update(sh_atom=sys["sh_atom"][keep].copy(), sh_l=sys["sh_l"][keep].copy(),
               sh_nprim=sys["sh_nprim"][keep].copy(), exps=exps, coefs=coefs,
               nshell=len(keep), nbf=int(sum(_basis.ncart(int(l)) for l in sys["sh_l"][keep])))
    out["name"] = sys["name"] + f"[{len(keep)} shells]"
    return out


def random_density(sys, seed):
    """A symmetric, positive semi-definite density-like matrix (no physics):
    D = 2 C C^T with C of shape nbf x nocc drawn from a normal distribution."""
    rng = np.random.default_rng(seed)
    n = sys["nbf"]
    nocc = max(1, sys["nelec"] // 2)
    C = rng.normal(scale=0.3, size=(n, nocc))
    return 2.0 * C @ C.T


def batch(systems):
    """Concatenates systems into one batch: the flattened arrays of all
    molecules plus ``atom_mol`` (molecule of each atom) and ``mols`` (the
    input systems, for per-molecule checks)."""
    natoms = np.cumsum([0] + [len(x["Z"]) for x in systems])
    out = {
        "name": f"batch of {len(systems)}",
        "Z": np.concatenate([x["Z"] for x in systems]).astype(np.int32),
        "xyz": np.concatenate([x["xyz"] for x in systems]),
        "charge": int(sum(x["charge"] for x in systems)),
        "nelec": int(sum(x["nelec"] for x in systems)),
        "sh_atom": np.concatenate([x["sh_atom"] + natoms[i] for i, x in enumerate(systems)]).astype(np.int32),
        "sh_l": np.concatenate([x["sh_l"] for x in systems]).astype(np.int32),
        "sh_nprim": np.concatenate([x["sh_nprim"] for x in systems]).astype(np.int32),
        "exps": np.concatenate([x["exps"] for x in systems]),
        "coefs": np.concatenate([x["coefs"] for x in systems]),
        "nbf": int(sum(x["nbf"] for x in systems)),
        "nshell": int(sum(x["nshell"] for x in systems)),
        "atom_mol": np.concatenate([np.full(len(x["Z"]), i, dtype=np.int32) for i, x in enumerate(systems)]),
        "mols": list(systems),
    }
    return out


def organic_batch(n=256, basis_name="tzvp-type", seed=SEED + 40):
    return batch([make_system(_geom.organic(seed + i), basis_name) for i in range(n)])


# ------------------------------------------------- learned-guess geometry set --
GUESS_SET_SIZE = 2000
GUESS_HELD_OUT = 200   # the last 200 indices are never trained on


def guess_geometry(i, seed=SEED + 60):
    """Geometry i of the learned-guess set: even i a linear alkane C4-C16 in
    a random orientation, odd i a water cluster of 4-32 molecules; every
    coordinate jittered by up to 0.05 angstrom."""
    rng = np.random.default_rng(seed + 7919 * i)
    if i % 2 == 0:
        n = int(rng.integers(4, 17))
        mol = _geom.alkane(n, seed + i, jitter=0.05)
        mol["xyz"] = mol["xyz"] @ _geom._rand_rot(rng).T
    else:
        n = int(rng.integers(4, 33))
        mol = _geom.water_cluster(n, seed + i, jitter=0.05)
    return mol


def guess_system(i, basis_name="6-31gs-type", seed=SEED + 60):
    return make_system(guess_geometry(i, seed), basis_name)
