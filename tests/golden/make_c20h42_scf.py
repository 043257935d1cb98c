"""Writes c20h42_631gs_scf.json: the oracle's converged RHF energy of the
C20H42 / 6-31G*-type workload (the seeded all-trans chain with 0.02 A jitter,
384 Cartesian functions), unscreened, from the core-Hamiltonian guess, to the
convergence criteria |dE| < 1e-10 Eh and max |X^T (FDS - SDF) X| < 1e-8.

Calls only the oracle (literal J/K sums over every unique shell quartet,
canonical orthogonalisation, DIIS).  One oracle J/K build takes minutes on a
few host cores, so the result is stored rather than recomputed by the tests.

    python tests/golden/make_c20h42_scf.py [nthreads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.scf import run_scf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    s = wl.c20h42_631gs()
    t0 = time.time()

    def jk_fn(D):
        t = time.time()
        J, K = oracle.jk(s, D, nthreads)
        print(f"oracle J/K build {time.time() - t:.0f} s", file=sys.stderr, flush=True)
        return J, K

    r = run_scf(s, jk_fn=jk_fn)
    out = {
        "source": "oracle/ (this script): unscreened literal J/K, canonical orthogonalisation (cutoff 1e-8), "
                  "DIIS on FDS - SDF, core-Hamiltonian guess",
        "workload": s["name"], "nbf": int(s["nbf"]), "nelec": int(s["nelec"]),
        "criteria": {"e_tol": 1e-10, "g_tol": 1e-8},
        "E_total": r["E"], "iterations": r["iters"], "converged": bool(r["converged"]),
        "energies": r["energies"], "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "c20h42_631gs_scf.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("E_total", "iterations", "converged", "seconds")}))


if __name__ == "__main__":
    main()
