#!/usr/bin/env python
"""J+K Fock-build throughput on one MI355X.

A step is one full pass of the J/K hot path for one density: density
preprocessing (scaled D, shell-block maxima), every quartet-class Rys ERI +
digestion kernel, and the symmetrisation into J and K, on resident device
buffers.  Workload (default): all-trans C20H42 with 0.02 A seeded jitter in the
6-31G*-type basis (384 Cartesian functions, s/p/d), Schwarz threshold 1e-10
with the per-quartet density screen, at the core-Hamiltonian guess density.

Prints one JSON line (see the fields below).  --gpus above 1 is refused: the
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "J+K Fock builds/s & ERI quartets/s, FP64 vs mixed @1e-6 Eh; SCF iters"
PEAK_FP64_VALU = 78.6  # TFLOP/s, MI355X dense FP64 vector
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X dense FP32 vector


def _kernel_source_hash():
    """Hash of the kernel sources: a committed counter measurement applies
    only to the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("fk_kernels.hip", "fk_eri.h", "fk_rys.h", "fk_internal.h"):
        with open(os.path.join(HERE, "paper_2407_21445_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic(kernel_name, workload, schedule="default"):
    """HBM bytes per launch of the named kernel from profiles/roofline_traffic.json
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a
    plain copy of known size), or None when absent, taken on other kernels or
    under another schedule of the class ("default", or [bra block, kets per
    tile, grid fraction])."""
    path = os.path.join(HERE, "profiles", "roofline_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != _kernel_source_hash() or t.get("workload") != workload:
        return None
    for k in t.get("kernels", []):
        if k["kernel"] == kernel_name and k.get("schedule", "default") == schedule:
            return k["fetch_bytes_per_launch"] * t["copy_scale_fetch"] + k["write_bytes_per_launch"] * t["copy_scale_write"]
    return None


def _workload(name):
    from synth import workloads as wl
    if name == "c20h42":
        return wl.c20h42_631gs(), "C20H42 all-trans (0.02 A jitter), 6-31G*-type, 384 Cartesian bf"
    if name == "water4":
        return wl.water4_sto3g(), "(H2O)4 STO-3G-type, 28 bf, tau=1e-10"
    if name == "c4":
        raise SystemExit("c4 is a batch workload (bench_batch)")
    if name == "water64":
        return wl.water64_ccpvdz(), "(H2O)64 1.0 g/cm3, cc-pVDZ-type, 1600 Cartesian bf, tau=1e-10"
    raise SystemExit(f"unknown workload {name}")


def _core_density(S, h, nocc):
    w, U = np.linalg.eigh(S)
    keep = w > 1e-8
    X = U[:, keep] / np.sqrt(w[keep])
    e, Cp = np.linalg.eigh(X.T @ h @ X)
    C = X @ Cp[:, :nocc]
    return 2.0 * C @ C.T


def cpu_baseline(sys_, D, target_s=15.0):
    """The oracle (test infrastructure) timed on host cores over a bounded
    sample of the same workload: whole shell blocks J[A,B] by literal sums
    (every (AB|CD) over all C, D), scaled to one full unscreened oracle build
    (one evaluation per unique shell quartet)."""
    import oracle
    nthreads = min(16, os.cpu_count() or 1)
    ns = sys_["nshell"]
    rng = np.random.default_rng(99)
    done_q, t_used, nblk = 0, 0.0, 0
    while t_used < target_s and nblk < 4096:
        a, b = (int(x) for x in rng.integers(0, ns, size=2))
        t0 = time.perf_counter()
        oracle.jk_blocks(sys_, D, [(a, b)], [], nthreads=nthreads)
        t_used += time.perf_counter() - t0
        done_q += ns * ns
        nblk += 1
    npair = ns * (ns + 1) // 2
    unique_q = npair * (npair + 1) // 2
    per_q = t_used / done_q
    est_build_s = per_q * unique_q
    return {"value": 1.0 / est_build_s, "unit": "builds/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{nblk} random J shell blocks ({done_q} shell quartets, {t_used:.1f} s) scaled to one "
                      f"unscreened build of {unique_q} unique shell quartets",
            "quartets_per_s": 1.0 / per_q, "est_build_s": est_build_s}


def _progress(msg):
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def bench_batch(args, torch, fk):
    """Batched builds: the first --nmol molecules of the seeded 256-molecule
    organic set (tzvp-type basis, s to f) in one context, every class launch
    covering all molecules; eager builds and replays of the build captured in
    a HIP graph are timed with HIP events."""
    from synth import workloads as wl
    b = wl.organic_batch(args.nmol)
    ctx = fk.FockJK(0).set_system(b).set_molecules(b["atom_mol"])
    Ds = []
    if args.batch_density == "core":
        for m in b["mols"]:
            h = fk.FockJK(-1).set_system(m)
            S, T, V, _ = h.one_electron()
            Ds.append(_core_density(S, T + V, m["nelec"] // 2).ravel())
    _progress(f"batch of {args.nmol} molecules set up")
    tune = None
    if args.autotune:
        # schedules tuned on a two-molecule batch of the same set, applied to all
        t_tune = time.perf_counter()
        nsub = min(2, args.nmol)
        sb = wl.batch(b["mols"][:nsub])
        sub = fk.FockJK(0).set_system(sb).set_molecules(sb["atom_mol"])
        sub.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=args.tau_fp32)
        Dsub = np.concatenate(Ds[:nsub]) if Ds else sub.sad_density()
        rep = sub.autotune(Dsub, reps=1)
        for r in rep["classes"]:
            ctx.set_class_schedule(r["la"], r["lb"], r["lc"], r["ld"], r["bra_block"], r["kets_per_tile"],
                                   r["grid_fraction"])
        tune = {"seconds": time.perf_counter() - t_tune, "tuned_on": f"first {nsub} molecules",
                "configurations": rep["configurations"], "class_ms_sum_default": rep["build_ms_default"],
                "class_ms_sum_tuned": rep["build_ms_tuned"],
                "changed_classes": sum(r["changed"] for r in rep["classes"])}
        del sub
        _progress(f"schedules tuned in {tune['seconds']:.0f} s")
    ctx.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=args.tau_fp32)
    info = ctx.info()
    _progress(f"lists built: {info['ntile']} tiles, {info['nquartet_schwarz']} Schwarz quartets")
    dev = torch.device("cuda:0")
    Dh = np.concatenate(Ds) if Ds else ctx.sad_density()
    Dd = torch.tensor(Dh, dtype=torch.float64, device=dev)
    J = torch.empty_like(Dd)
    K = torch.empty_like(Dd)
    stream = torch.cuda.current_stream(dev)
    def build(timed):
        ctx.build_jk(Dd, J, K, stream=stream, time_classes=args.progress)
        if args.progress:
            # long builds report each finished class launch (work-derived progress)
            last = -1
            while True:
                done, total = ctx.build_progress()
                if done != last:
                    _progress(f"{'timed' if timed else 'warm-up'} build: {done} of {total} class launches finished")
                    last = done
                if done == total:
                    break
                # short polls: the next build is queued only after this one
                # ends, so the poll interval is idle time inside the timed region
                time.sleep(0.02)

    for _ in range(args.warmup):
        build(False)
    torch.cuda.synchronize()
    st = ctx.stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        build(True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    if args.warmup == 0:
        st = ctx.stats()
    ms_graph = None
    if not args.progress:
        # the same build captured once in a HIP graph, replayed
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.build_jk(Dd, J, K)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
    _progress(f"builds timed: {ms:.0f} ms eager" + (f", {ms_graph:.0f} ms graph" if ms_graph else ""))
    nbf = [m["nbf"] for m in b["mols"]]
    out = {
        "metric": METRIC, "value": 1000.0 / ms, "unit": "batch builds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.tau_fp32 <= 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"organic batch, first {args.nmol} of 256 seeded molecules (3-30 C/N/O + H), "
                               f"tzvp-type basis (s-f), one launch per class for all molecules",
                   "nmol": args.nmol, "nbf_total": int(sum(nbf)), "nbf_min": int(min(nbf)), "nbf_max": int(max(nbf)),
                   "tau": args.tau, "tau_prim": args.tau_prim,
                   "density": "core-Hamiltonian guess per molecule" if args.batch_density == "core" else "SAD"},
        "molecule_builds_per_s": args.nmol * 1000.0 / ms,
        "graph_ms_per_step": ms_graph,
        "quartets_per_s": st["quartets"] / (ms * 1e-3),
        "quartets_per_build": st["quartets"], "schwarz_quartets": info["nquartet_schwarz"],
        "tflops_build": st["flops_total"] / (ms * 1e-3) / 1e12,
    }
    if tune:
        out["autotune"] = tune
    if args.batch_scf:
        # batched SCF of every molecule from SAD (outside the timed region)
        # criteria of the organic set: its overlap eigenvalues reach ~1e-6, so
        # the orthonormal-basis commutator has a noise floor near 1e-6
        tol = dict(e_tol=1e-7, g_tol=1e-5)
        rs, _ = ctx.run_scf_batch(guess=fk.GUESS_SAD, **tol)
        _progress(f"batched SCF: {max(r['iterations'] for r in rs)} iterations")
        out["scf_batch"] = {"criteria": tol, "iterations": [r["iterations"] for r in rs],
                            "converged": int(sum(r["converged"] for r in rs)),
                            "seconds": rs[0]["total_seconds"], "jk_seconds": rs[0]["jk_seconds"],
                            "energies": [r["energy"] for r in rs]}
        if args.tau_fp32 > 0:
            ref = fk.FockJK(0).set_system(b).set_molecules(b["atom_mol"])
            ref.build_quartets(tau=args.tau, tau_prim=args.tau_prim)
            r64, _ = ref.run_scf_batch(guess=fk.GUESS_SAD, **tol)
            out["scf_batch"]["fp64_seconds"] = r64[0]["total_seconds"]
            out["scf_batch"]["max_abs_energy_diff_vs_fp64"] = max(abs(a["energy"] - c["energy"]) for a, c in zip(rs, r64))
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c20h42")
    ap.add_argument("--tau", type=float, default=1e-10)
    ap.add_argument("--tau-prim", type=float, default=1e-12, help="primitive-pair pruning threshold")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--classes", action="store_true", help="print the per-class kernel table to stderr")
    ap.add_argument("--schedule", action="append", default=[], metavar="LA,LB,LC,LD,BB,KT,GF",
                    help="fix a class schedule (bra block, kets per tile, grid fraction) before the lists "
                         "are built; with --no-autotune it is the one timed")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF run reported beside the build rate")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the default kernel schedules (the autotuner runs by default, before timing)")
    ap.add_argument("--nmol", type=int, default=8, help="molecules of the organic batch (--workload c4)")
    ap.add_argument("--batch-scf", action="store_true", help="--workload c4: also run the batched SCF")
    ap.add_argument("--batch-density", choices=("core", "sad"), default="core",
                    help="--workload c4: density of the timed builds")
    ap.add_argument("--progress", action="store_true",
                    help="--workload c4: report finished class launches during each build (long batches)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 5 times (calibrates HBM byte counters)")
    ap.add_argument("--tau-fp32", type=float, default=0.0,
                    help="precision split: FP32 recurrences for quartets with G_ab G_cd * 2 below this (0: FP64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2
    import torch
    import paper_2407_21445_amd as fk

    if args.copy_probe > 0:
        x = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8}), flush=True)
        return 0
    if args.workload == "c4":
        return bench_batch(args, torch, fk)
    sys_, desc = _workload(args.workload)
    ctx = fk.FockJK(0).set_system(sys_)
    pinned = {}
    for spec in args.schedule:
        v = spec.split(",")
        if len(v) != 7:
            raise SystemExit(f"--schedule {spec}: expected LA,LB,LC,LD,BRA_BLOCK,KETS,GRID_FRACTION")
        cls, sch = tuple(int(x) for x in v[:4]), (int(v[4]), int(v[5]), float(v[6]))
        ctx.set_class_schedule(*cls, *sch)
        pinned[cls] = list(sch)
    ctx.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=args.tau_fp32)
    info = ctx.info()
    S, T, V, _ = ctx.one_electron()
    D = _core_density(S, T + V, sys_["nelec"] // 2)
    dev = torch.device("cuda:0")
    Dd = torch.tensor(D, dtype=torch.float64, device=dev)
    J = torch.empty_like(Dd)
    K = torch.empty_like(Dd)
    stream = torch.cuda.current_stream(dev)
    tune, tuned_rows = None, []
    if args.autotune:
        # schedule tuning before the timed region (lists rebuilt with the choice)
        t_tune = time.perf_counter()
        rep = ctx.autotune(Dd, reps=2, stream=stream.cuda_stream)
        tuned_rows = rep["classes"]
        tune = {"seconds": time.perf_counter() - t_tune, "configurations": rep["configurations"],
                "class_ms_sum_default": rep["build_ms_default"], "class_ms_sum_tuned": rep["build_ms_tuned"],
                "classes": {f"({r['la']}{r['lb']}|{r['lc']}{r['ld']})/fp{r['precision']}":
                            [r["bra_block"], r["kets_per_tile"], r["grid_fraction"], round(r["ms_default"], 4),
                             round(r["ms_tuned"], 4)]
                            for r in rep["classes"] if r["ms_default"] > 0.1},
                "fields": "bra_block, kets_per_tile, grid_fraction, ms_default, ms_tuned (classes above 0.1 ms)"}

    for _ in range(args.warmup):
        ctx.build_jk(Dd, J, K, stream=stream)
    torch.cuda.synchronize()
    st = ctx.stats()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.build_jk(Dd, J, K, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps

    # per-class kernel times (HIP events around each class launch on the same stream)
    reps = 3
    acc = None
    for _ in range(reps):
        ctx.build_jk(Dd, J, K, stream=stream, time_classes=True)
        s2 = ctx.stats()
        t = np.array([c["ms"] for c in s2["classes"]])
        acc = t if acc is None else acc + t
    cls_ms = acc / reps
    i = int(np.argmax(cls_ms))
    c = s2["classes"][i]
    if args.classes:
        print(f"{'class':>10} {'ms':>8} {'share':>6} {'quartets':>11} {'prims':>13} {'GFLOP':>9} {'TFLOP/s':>8} {'frac':>6}",
              file=sys.stderr)
        for k in np.argsort(-cls_ms):
            cc = s2["classes"][k]
            f = cc["prim_quartets"] * cc["flops_per_prim"] + cc["quartets"] * cc["flops_per_quartet"]
            tf = f / (cls_ms[k] * 1e-3) / 1e12 if cls_ms[k] > 0 else 0.0
            nm = "({}{}|{}{})".format(*("spdf"[x] for x in cc["class"]))
            print(f"{nm:>10} {cls_ms[k]:8.3f} {cls_ms[k] / cls_ms.sum():6.3f} {cc['quartets']:11d} "
                  f"{cc['prim_quartets']:13d} {f / 1e9:9.2f} {tf:8.3f} {tf / PEAK_FP64_VALU:6.3f}", file=sys.stderr)
    cflops = c["prim_quartets"] * c["flops_per_prim"] + c["quartets"] * c["flops_per_quartet"]
    achieved = cflops / (cls_ms[i] * 1e-3) / 1e12
    peak = PEAK_FP32_VALU if c["precision"] == 32 else PEAK_FP64_VALU
    lname = "spdf"
    cname = "({}{}|{}{})".format(*(lname[x] for x in c["class"]))
    # the committed counter figures name the schedule they were taken under
    sched = pinned.get(tuple(c["class"]), "default")
    for r in tuned_rows:
        if (r["la"], r["lb"], r["lc"], r["ld"]) == tuple(c["class"]) and r["precision"] == c["precision"] \
                and r["changed"]:
            sched = [r["bra_block"], r["kets_per_tile"], r["grid_fraction"]]
    out = {
        "metric": METRIC, "value": 1000.0 / ms, "unit": "builds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.tau_fp32 <= 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": desc, "nbf": info["nbf"], "nshell": info["nshell"], "tau": args.tau,
                   "tau_prim": args.tau_prim,
                   "density": "core-Hamiltonian guess",
                   "precision": "fp64" if args.tau_fp32 <= 0 else f"mixed (FP32 below tau_fp32={args.tau_fp32:g})"},
        "quartets_per_s": st["quartets"] / (ms * 1e-3),
        "prim_quartets_per_s": st["prim_quartets"] / (ms * 1e-3),
        "quartets_per_build": st["quartets"], "schwarz_quartets": info["nquartet_schwarz"],
        "flops_per_build": st["flops_total"], "tflops_build": st["flops_total"] / (ms * 1e-3) / 1e12,
        "wall_s_timed": wall,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": _traffic(f"J/K class {cname}", args.workload, sched),
                     "kernel": f"J/K class {cname}" + (" (FP32 part)" if c["precision"] == 32 else ""),
                     "kernel_ms": float(cls_ms[i]), "schedule": sched,
                     "class_share": float(cls_ms[i] / cls_ms.sum())},
    }
    if args.tau_fp32 > 0:
        # the same build in FP64 only: J/K and one-build energy differences
        ref = fk.FockJK(0).set_system(sys_).build_quartets(tau=args.tau, tau_prim=args.tau_prim)
        if args.autotune:  # the FP64 reference with its own tuned schedules
            ref.autotune(Dd, reps=2, stream=stream.cuda_stream)
        J64, K64 = ref.build_jk(Dd, sync=True)
        torch.cuda.synchronize()
        for _ in range(2):
            ref.build_jk(Dd, J64, K64, stream=stream)
        r0 = torch.cuda.Event(enable_timing=True)
        r1 = torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _ in range(args.steps):
            ref.build_jk(Dd, J64, K64, stream=stream)
        r1.record(stream)
        torch.cuda.synchronize()
        ms64 = r0.elapsed_time(r1) / args.steps
        dJ = (J - J64).cpu().numpy()
        dK = (K - K64).cpu().numpy()
        n32 = sum(x["quartets"] for x in st["classes"] if x["precision"] == 32)
        out["mixed"] = {"tau_fp32": args.tau_fp32, "fp32_quartet_fraction": n32 / max(1, st["quartets"]),
                        "fp64_builds_per_s": 1000.0 / ms64, "speedup": ms64 / ms,
                        "max_abs_dJ": float(np.max(np.abs(dJ))), "max_abs_dK": float(np.max(np.abs(dK))),
                        "dE_one_build": float(0.5 * np.sum(D * dJ) - 0.25 * np.sum(D * dK))}
    if tune:
        out["autotune"] = tune
    if not args.no_scf:
        # SCF from the core-Hamiltonian guess on the same quartet lists (outside
        # the timed region): iterations to |dE| < 1e-10, max|error| < 1e-8
        r = ctx.run_scf()
        if args.tau_fp32 > 0:
            r64 = ref.run_scf()
            out["mixed"]["scf_energy_fp64"] = r64["energy"]
            out["mixed"]["scf_energy_diff"] = r["energy"] - r64["energy"]
        out["scf"] = {"iterations": r["iterations"], "converged": bool(r["converged"]), "energy": r["energy"],
                      "seconds": r["total_seconds"], "jk_seconds": r["jk_seconds"],
                      "jk_ms_per_iteration": 1000.0 * r["jk_seconds"] / max(1, r["iterations"]),
                      "guess": "core Hamiltonian"}
        # the same SCF from the SAD guess and from the learned guess (when the
        # trained network for this basis is present)
        guesses = {"sad": fk.GUESS_SAD}
        model = os.path.join(HERE, "paper_2407_21445_amd", "guess_631gs.npz")
        if sys_["name"].endswith("/6-31gs-type") and os.path.exists(model):
            from paper_2407_21445_amd.guess_train import load_model
            try:
                ctx.set_guess_model(*load_model(model))
                guesses["learned"] = fk.GUESS_LEARNED
            except fk.FockJKError as e:  # weights of another feature layout
                print(f"bench.py: learned guess skipped: {e}", file=sys.stderr)
        # the core-guess SCF with incremental builds (full build every 8 iterations)
        rin = ctx.run_scf(incremental=8)
        out["scf"]["incremental"] = {"iterations": rin["iterations"], "converged": bool(rin["converged"]),
                                     "seconds": rin["total_seconds"], "jk_seconds": rin["jk_seconds"],
                                     "energy_minus_full": rin["energy"] - r["energy"]}
        # the core-guess SCF again with its Fock stage replayed from a HIP graph
        rgr = ctx.run_scf(graph=True)
        out["scf"]["graph"] = {"iterations": rgr["iterations"], "converged": bool(rgr["converged"]),
                               "seconds": rgr["total_seconds"], "stage_seconds": rgr["jk_seconds"],
                               "energy_minus_eager": rgr["energy"] - r["energy"]}
        for name, g in guesses.items():
            rg = ctx.run_scf(guess=g)
            out["scf"][name] = {"iterations": rg["iterations"], "converged": bool(rg["converged"]),
                                "seconds": rg["total_seconds"], "guess_seconds": rg["guess_seconds"],
                                "energy_minus_core_start": rg["energy"] - r["energy"],
                                "guess_used": {0: "core", 2: "sad", 3: "learned"}.get(rg["guess_used"], "?")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sys_, D, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
