"""Textbook restricted closed-shell SCF on top of the oracle's integrals.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the Hartree-Fock section of the paper: solve FC = SC eps with
F = h + J - K/2 and D = 2 C_occ C_occ^T.  The paper prints no energy
expression; the standard one is used: E = 1/2 sum D (h + F) + E_nuc.
Orthogonalisation is canonical (S^-1/2 over eigenvalues above a cutoff);
convergence is accelerated by Pulay's DIIS on the commutator FDS - SDF.
"""
from __future__ import annotations

import numpy as np

from . import enuc, jk, oneel


def orthogonalizer(S, cutoff=1e-8):
    w, U = np.linalg.eigh(S)
    keep = w > cutoff
    return U[:, keep] / np.sqrt(w[keep])


def density(C, nocc):
    Co = C[:, :nocc]
    return 2.0 * Co @ Co.T


def energy(D, h, F, e_nuc):
    return 0.5 * float(np.sum(D * (h + F))) + e_nuc


def core_guess(h, X, nocc):
    e, Cp = np.linalg.eigh(X.T @ h @ X)
    return density(X @ Cp, nocc)


def run_scf(sys, D0=None, max_iter=100, e_tol=1e-10, g_tol=1e-8, diis_n=8, nthreads=0, jk_fn=None,
            ortho_cutoff=1e-8):
    """Returns dict(E, D, iters, converged, energies); overlap eigenvectors with
    eigenvalue at or below ortho_cutoff are left out of the orthogonal basis."""
    S, T, V = oneel(sys)
    h = T + V
    e_nuc = enuc(sys)
    nocc = sys["nelec"] // 2
    X = orthogonalizer(S, ortho_cutoff)
    D = core_guess(h, X, nocc) if D0 is None else np.array(D0)
    jk_fn = jk_fn or (lambda Dm: jk(sys, Dm, nthreads))
    focks, errs, energies = [], [], []
    E_old = None
    for it in range(1, max_iter + 1):
        J, K = jk_fn(D)
        F = h + J - 0.5 * K
        E = energy(D, h, F, e_nuc)
        energies.append(E)
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        gnorm = float(np.max(np.abs(err)))
        if E_old is not None and abs(E - E_old) < e_tol and gnorm < g_tol:
            return {"E": E, "D": D, "iters": it, "converged": True, "energies": energies, "F": F, "h": h, "S": S}
        E_old = E
        focks.append(F)
        errs.append(err)
        if len(focks) > diis_n:
            focks.pop(0)
            errs.pop(0)
        if len(focks) >= 2:
            n = len(focks)
            B = -np.ones((n + 1, n + 1))
            B[n, n] = 0.0
            for i in range(n):
                for j in range(n):
                    B[i, j] = float(np.sum(errs[i] * errs[j]))
            rhs = np.zeros(n + 1)
            rhs[n] = -1.0
            try:
                c = np.linalg.solve(B, rhs)[:n]
                F = sum(ci * Fi for ci, Fi in zip(c, focks))
            except np.linalg.LinAlgError:
                pass
        e, Cp = np.linalg.eigh(X.T @ F @ X)
        D = density(X @ Cp, nocc)
    return {"E": E, "D": D, "iters": max_iter, "converged": False, "energies": energies, "F": F, "h": h, "S": S}
