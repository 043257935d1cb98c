#!/usr/bin/env python
"""J+K Fock-build throughput on one MI355X.

A step is one full pass of the J/K hot path for one density: density
preprocessing (scaled D, shell-block maxima), every quartet-class Rys ERI +
digestion kernel, and the symmetrisation into J and K, on resident device
buffers.  Workload (default): 64 seeded waters at 1.0 g/cm^3 in the
cc-pVDZ-type basis (1600 Cartesian functions, s/p/d), Schwarz threshold 1e-10
with the per-quartet density screen, primitive pairs pruned at 1e-12, at the
core-Hamiltonian guess density.  `value` is the FP64 build rate; the line
also carries the same build with the precision split at tau_fp32 = 1e-5
(`mixed`: rate, speed-up, J/K and energy differences, SCF energies of both),
SCF iteration counts, the dominant kernel against the FP64 roofline, a
C20H42 / 6-31G*-type reference rate and the oracle's CPU baseline.

Prints one JSON line.  --gpus above 1 is refused: the build runs on one GPU.
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


def _traffic(kernel_name, workload, schedule, engine="rys"):
    """HBM bytes per launch of the named kernel from profiles/roofline_traffic.json
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a
    plain copy of known size), or None when absent, taken on other kernels,
    under another schedule of the class ([bra block, kets per tile, grid
    fraction]) or with the other integral engine."""
    path = os.path.join(HERE, "profiles", "roofline_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != _kernel_source_hash() or t.get("workload") != workload:
        return None
    for k in t.get("kernels", []):
        if k["kernel"] == kernel_name and k.get("schedule") == list(schedule) and k.get("engine", "rys") == engine:
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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sys_, gpu_classes, target_s=20.0):
    """The oracle (test infrastructure: plain MMD, unscreened) timed on the
    host's cores over a bounded sample of the same workload.  Per quartet
    class, random shell quartets of that class (uniform over the unscreened
    unique quartets) are evaluated by the oracle's MMD code, on all cores and
    on one; their time per primitive quartet, times the primitive quartets the
    GPU build computes in that class, estimates the oracle doing the GPU's
    (screened) work; time per shell quartet times the class's unique quartets
    estimates one unscreened oracle build.  value = 1 / the screened estimate
    (all cores)."""
    import oracle
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    ls = np.asarray(sys_["sh_l"])
    npr = np.asarray(sys_["sh_nprim"])
    ns = len(ls)

    def pcls(la, lb):
        return la * (la + 1) // 2 + lb
    pairs = {}
    for a in range(ns):
        for b in range(a + 1):
            x, y = (a, b) if (ls[a], a) >= (ls[b], b) else (b, a)
            pairs.setdefault(pcls(ls[x], ls[y]), []).append((x, y))
    pairs = {k: np.array(v, dtype=np.int32) for k, v in pairs.items()}
    gpu = {}
    for c in gpu_classes:
        key = tuple(c["class"])
        q, p = gpu.get(key, (0, 0))
        gpu[key] = (q + c["quartets"], p + c["prim_quartets"])
    rng = np.random.default_rng(2024)
    per = max(0.05, target_s / max(1, len(gpu)))
    rows, est_scr, est_scr1, est_uns, t_used = [], 0.0, 0.0, 0.0, 0.0
    for (la, lb, lc, ld), (gq, gp) in sorted(gpu.items()):
        P, Q = pcls(la, lb), pcls(lc, ld)
        B, K = pairs[P], pairs[Q]
        n_unique = len(B) * len(K) if P != Q else len(B) * (len(B) + 1) // 2

        def sample(n):
            qs = np.concatenate([B[rng.integers(len(B), size=n)], K[rng.integers(len(K), size=n)]], axis=1)
            prims = float(np.sum(npr[qs[:, 0]] * npr[qs[:, 1]] * npr[qs[:, 2]] * npr[qs[:, 3]]))
            return qs, prims

        def timed(n, threads):
            qs, prims = sample(n)
            t0 = time.perf_counter()
            oracle.eri_list(sys_, qs, nthreads=threads)
            return time.perf_counter() - t0, n, prims
        # grow the sample until it takes a fair share of the budget
        n = 64
        while True:
            t_all, n_all, p_all = timed(n, ncpu)
            if t_all >= 0.3 * per or n >= 2_000_000:
                break
            n = int(min(2_000_000, n * min(16.0, max(2.0, 0.7 * per / max(t_all, 1e-4)))))
        n1 = int(min(n_all, max(16, n_all * 0.3 * per / max(t_all * ncpu, 1e-4))))
        t_one, n_one, p_one = timed(n1, 1)
        t_used += t_all + t_one
        est_scr += t_all / p_all * gp
        est_scr1 += t_one / p_one * gp
        est_uns += t_all / n_all * n_unique
        rows.append({"class": "({}{}|{}{})".format(*("spdf"[x] for x in (la, lb, lc, ld))),
                     "sampled_quartets": n_all, "sampled_quartets_1core": n_one,
                     "s_per_prim_quartet": t_all / p_all, "s_per_prim_quartet_1core": t_one / p_one})
    return {"value": 1.0 / est_scr, "unit": "builds/s", "cores": ncpu, "kind": "oracle",
            "sample": f"per quartet class, random unscreened shell quartets of this workload evaluated by the "
                      f"oracle's MMD code ({sum(r['sampled_quartets'] for r in rows)} quartets on {ncpu} threads, "
                      f"{sum(r['sampled_quartets_1core'] for r in rows)} on 1, {t_used:.1f} s); time per primitive "
                      f"quartet x the GPU build's primitive quartets per class = one build of the same screened "
                      f"work",
            "nproc": ncpu, "cpu_model": _cpu_model(), "value_1core": 1.0 / est_scr1,
            "est_screened_build_s": est_scr, "est_screened_build_s_1core": est_scr1,
            "est_unscreened_build_s": est_uns, "classes": rows}


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
    _progress(f"batch of {args.nmol} molecules set up")

    def start_density(c):
        # core-Hamiltonian densities of every molecule, by the library's own
        # batched SCF start (device orthogonaliser and purification), or SAD
        if args.batch_density == "core":
            return c.run_scf_batch(max_iter=0, guess=fk.GUESS_CORE)[1]
        return c.sad_density()
    tune = None
    if args.autotune:
        # schedules tuned on a two-molecule batch of the same set, applied to all
        t_tune = time.perf_counter()
        nsub = min(2, args.nmol)
        sb = wl.batch(b["mols"][:nsub])
        sub = fk.FockJK(0).set_system(sb).set_molecules(sb["atom_mol"])
        sub.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=args.tau_fp32,
                            block_tasks=args.block_tasks)
        Dsub = start_density(sub)
        rep = sub.autotune(Dsub, reps=1)
        for r in rep["classes"]:
            ctx.set_class_schedule(r["la"], r["lb"], r["lc"], r["ld"], r["bra_block"], r["kets_per_tile"],
                                   r["grid_fraction"])
            ctx.set_class_engine(r["la"], r["lb"], r["lc"], r["ld"], r["engine"])
        tune = {"seconds": time.perf_counter() - t_tune, "tuned_on": f"first {nsub} molecules",
                "configurations": rep["configurations"], "class_ms_sum_default": rep["build_ms_default"],
                "class_ms_sum_tuned": rep["build_ms_tuned"],
                "changed_classes": sum(r["changed"] for r in rep["classes"])}
        del sub
        _progress(f"schedules tuned in {tune['seconds']:.0f} s")
    ctx.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=args.tau_fp32, block_tasks=args.block_tasks)
    info = ctx.info()
    _progress(f"lists built: {info['ntile']} tiles, {info['nquartet_schwarz']} Schwarz quartets")
    dev = torch.device("cuda:0")
    Dh = start_density(ctx)
    _progress("start densities formed")
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
        # batched SCF of every molecule from SAD (outside the timed region),
        # to the default criteria.  The organic set's bases are ill
        # conditioned (smallest overlap eigenvalues 1.7e-6..1.2e-5): densities
        # by purification of X F X stall near a commutator of 1e-5, so the
        # densities come from the eigensolver
        tol = dict(e_tol=1e-10, g_tol=1e-8, canonical=args.canonical, density_eig=True)
        rs, _ = ctx.run_scf_batch(guess=fk.GUESS_SAD, **tol)
        _progress(f"batched SCF: {max(r['iterations'] for r in rs)} iterations")
        out["scf_batch"] = {"criteria": tol, "iterations": [r["iterations"] for r in rs],
                            "converged": int(sum(r["converged"] for r in rs)),
                            "seconds": rs[0]["total_seconds"], "jk_seconds": rs[0]["jk_seconds"],
                            "energies": [r["energy"] for r in rs],
                            "dropped_directions": [r["ndropped"] for r in rs]}
        if args.tau_fp32 > 0:
            ref = fk.FockJK(0).set_system(b).set_molecules(b["atom_mol"])
            ref.build_quartets(tau=args.tau, tau_prim=args.tau_prim)
            r64, _ = ref.run_scf_batch(guess=fk.GUESS_SAD, **tol)
            out["scf_batch"]["fp64_seconds"] = r64[0]["total_seconds"]
            out["scf_batch"]["max_abs_energy_diff_vs_fp64"] = max(abs(a["energy"] - c["energy"]) for a, c in zip(rs, r64))
    print(json.dumps(out), flush=True)
    return 0


def _time_builds(torch, ctx, Dd, J, K, stream, warmup, steps, j_engine=False):
    """Milliseconds per build: `warmup` untimed builds, then `steps` builds
    between HIP events on the build stream, bracketed by device syncs."""
    for _ in range(warmup):
        ctx.build_jk(Dd, J, K, stream=stream, j_engine=j_engine)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.build_jk(Dd, J, K, stream=stream, j_engine=j_engine)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _class_times(ctx, Dd, J, K, stream, reps=3):
    """Per-launch kernel times (HIP events around each class launch, on the
    build stream), averaged over `reps` builds; returns (times, stats)."""
    acc = None
    for _ in range(reps):
        ctx.build_jk(Dd, J, K, stream=stream, time_classes=True)
        st = ctx.stats()
        t = np.array([c["ms"] for c in st["classes"]])
        acc = t if acc is None else acc + t
    return acc / reps, st


def _cname(c):
    return "({}{}|{}{})".format(*("spdf"[x] for x in c["class"]))


def _print_classes(cls_ms, st):
    print(f"{'class':>10} {'prec':>4} {'eng':>4} {'ms':>8} {'share':>6} {'quartets':>11} {'prims':>13} {'GFLOP':>9} "
          f"{'TFLOP/s':>8} {'frac':>6}", file=sys.stderr)
    for k in np.argsort(-cls_ms):
        cc = st["classes"][k]
        f = cc["prim_quartets"] * cc["flops_per_prim"] + cc["quartets"] * cc["flops_per_quartet"]
        tf = f / (cls_ms[k] * 1e-3) / 1e12 if cls_ms[k] > 0 else 0.0
        peak = PEAK_FP32_VALU if cc["precision"] == 32 else PEAK_FP64_VALU
        print(f"{_cname(cc):>10} {cc['precision']:>4} {('rys', 'hgp')[cc['engine']]:>4} {cls_ms[k]:8.3f} {cls_ms[k] / cls_ms.sum():6.3f} "
              f"{cc['quartets']:11d} {cc['prim_quartets']:13d} {f / 1e9:9.2f} {tf:8.3f} {tf / peak:6.3f}",
              file=sys.stderr)


def _hgp_everywhere(fk, c):
    """The HGP engine for every class it is built for (the others keep Rys)."""
    for la in range(4):
        for lb in range(la + 1):
            for lc in range(4):
                for ld in range(lc + 1):
                    if (la, lb) >= (lc, ld):
                        try:
                            c.set_class_engine(la, lb, lc, ld, "hgp")
                        except fk.FockJKError as e:
                            if e.code != fk.FK_ERR_UNSUPPORTED:
                                raise


SCHED_DIR = os.path.join(HERE, "paper_2407_21445_amd", "schedules")


def _load_cached(ctx, key, arch, args):
    """Schedule source of a context: 'default' (--no-autotune), 'cache' (the
    committed schedules of this workload and architecture, loaded here) or
    'autotune' (no cache, or --retune)."""
    if not args.autotune:
        return "default"
    path = os.path.join(SCHED_DIR, f"{key}.{arch}.txt")
    if args.retune or not os.path.exists(path):
        return "autotune"
    ctx.load_schedules(path)
    return "cache"


def _save_tuned(ctx, key, arch, args):
    if args.save_schedules:
        os.makedirs(args.save_schedules, exist_ok=True)
        ctx.save_schedules(os.path.join(args.save_schedules, f"{key}.{arch}.txt"))


def _tune(ctx, Dd, stream):
    t0 = time.perf_counter()
    rep = ctx.autotune(Dd, reps=2, stream=stream.cuda_stream)
    return rep, {"source": "autotune", "seconds": time.perf_counter() - t0, "configurations": rep["configurations"],
                 "class_ms_sum_default": rep["build_ms_default"], "class_ms_sum_tuned": rep["build_ms_tuned"],
                 "changed_classes": int(sum(r["changed"] for r in rep["classes"]))}


def _sched_of(c):
    """The schedule a class launch ran with: [bra block, kets per tile, grid fraction]."""
    return [int(c["schedule"][0]), int(c["schedule"][1]), float(c["schedule"][2])]


def bench_single(args, torch, fk):
    """One molecule: the FP64 build timed (the line's value), the dominant
    class kernel against the FP64 roofline, the same build with the precision
    split (mixed) timed and compared, SCF runs of both, a C20H42 line and the
    oracle's CPU baseline."""
    sys_, desc = _workload(args.workload)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    pinned = {}

    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]

    def make(tau_fp32, key, tau_k=0.0):
        c = fk.FockJK(0).set_system(sys_)
        for spec in args.schedule:
            v = spec.split(",")
            if len(v) != 7:
                raise SystemExit(f"--schedule {spec}: expected LA,LB,LC,LD,BRA_BLOCK,KETS,GRID_FRACTION")
            cls, sch = tuple(int(x) for x in v[:4]), (int(v[4]), int(v[5]), float(v[6]))
            c.set_class_schedule(*cls, *sch)
            pinned[cls] = list(sch)
        if args.engine == "hgp":
            _hgp_everywhere(fk, c)
        src = _load_cached(c, key, arch, args)
        return c.build_quartets(tau=args.tau, tau_prim=args.tau_prim, tau_fp32=tau_fp32, tau_k=tau_k,
                                block_tasks=args.block_tasks), src

    ctx, src64 = make(0.0, f"{args.workload}_fp64")
    info = ctx.info()
    S, T, V, _ = ctx.one_electron()
    D = _core_density(S, T + V, sys_["nelec"] // 2)
    Dd = torch.tensor(D, dtype=torch.float64, device=dev)
    J = torch.empty_like(Dd)
    K = torch.empty_like(Dd)
    _progress(f"{desc}: lists built ({info['nquartet_schwarz']} Schwarz quartets)")
    tune, tuned_rows = {"source": src64}, []
    if src64 == "autotune":
        rep, tune = _tune(ctx, Dd, stream)
        tuned_rows = rep["classes"]
        _save_tuned(ctx, f"{args.workload}_fp64", arch, args)
        _progress(f"FP64 schedules tuned in {tune['seconds']:.0f} s")
    ms = _time_builds(torch, ctx, Dd, J, K, stream, args.warmup, args.steps)
    st = ctx.stats()
    _progress(f"FP64 build {ms:.2f} ms")
    cls_ms, s2 = _class_times(ctx, Dd, J, K, stream)
    if args.classes:
        _print_classes(cls_ms, s2)
    i = int(np.argmax(cls_ms))
    c = s2["classes"][i]
    cflops = c["prim_quartets"] * c["flops_per_prim"] + c["quartets"] * c["flops_per_quartet"]
    achieved = cflops / (cls_ms[i] * 1e-3) / 1e12
    sched = _sched_of(c)
    out = {
        "metric": METRIC, "value": 1000.0 / ms, "unit": "builds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nbf": info["nbf"], "nshell": info["nshell"], "tau": args.tau,
                   "tau_prim": args.tau_prim, "density": "core-Hamiltonian guess", "precision": "fp64",
                   "mixed_leg_tau_fp32": args.tau_fp32},
        "quartets_per_s": st["quartets"] / (ms * 1e-3),
        "prim_quartets_per_s": st["prim_quartets"] / (ms * 1e-3),
        "quartets_per_build": st["quartets"], "schwarz_quartets": info["nquartet_schwarz"],
        "hgp_launches": int(sum(1 for x in st["classes"] if x["engine"] == fk.ENGINE_HGP)),
        "flops_per_build": st["flops_total"], "tflops_build": st["flops_total"] / (ms * 1e-3) / 1e12,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU,
                     "traffic": _traffic(f"J/K class {_cname(c)}", args.workload, sched, ("rys", "hgp")[c["engine"]]),
                     "kernel": f"J/K class {_cname(c)}", "kernel_ms": float(cls_ms[i]), "schedule": sched,
                     "engine": ("rys", "hgp")[c["engine"]],
                     "class_share": float(cls_ms[i] / cls_ms.sum()),
                     "flops_per_launch": cflops, "quartets_per_launch": c["quartets"],
                     "prim_quartets_per_launch": c["prim_quartets"]},
    }
    out["schedules"] = tune
    ref = None
    if args.tau_fp32 > 0:
        # the same build with the precision split: FP32 recurrences for the
        # waves whose quartets all have G_ab G_cd D_max below tau_fp32
        mx, src_mx = make(args.tau_fp32, f"{args.workload}_mixed")
        tune_mx = {"source": src_mx}
        if src_mx == "autotune":
            _, tune_mx = _tune(mx, Dd, stream)
            _save_tuned(mx, f"{args.workload}_mixed", arch, args)
        Jm = torch.empty_like(Dd)
        Km = torch.empty_like(Dd)
        ms_mx = _time_builds(torch, mx, Dd, Jm, Km, stream, args.warmup, args.steps)
        stm = mx.stats()
        ctx.build_jk(Dd, J, K, stream=stream)
        torch.cuda.synchronize()
        dJ = (Jm - J).cpu().numpy()
        dK = (Km - K).cpu().numpy()
        n32 = sum(x["quartets"] for x in stm["classes"] if x["precision"] == 32)
        cms, s3 = _class_times(mx, Dd, Jm, Km, stream)
        f64 = sum(x["prim_quartets"] * x["flops_per_prim"] + x["quartets"] * x["flops_per_quartet"]
                  for x in s3["classes"] if x["precision"] == 64)
        f32 = sum(x["prim_quartets"] * x["flops_per_prim"] + x["quartets"] * x["flops_per_quartet"]
                  for x in s3["classes"] if x["precision"] == 32)
        t_ideal = f64 / (PEAK_FP64_VALU * 1e12) + f32 / (PEAK_FP32_VALU * 1e12)
        out["mixed"] = {"tau_fp32": args.tau_fp32, "builds_per_s": 1000.0 / ms_mx, "ms_per_step": ms_mx,
                        "speedup_vs_fp64": ms / ms_mx, "fp32_quartet_fraction": n32 / max(1, stm["quartets"]),
                        "quartets_per_s": stm["quartets"] / (ms_mx * 1e-3),
                        "max_abs_dJ": float(np.max(np.abs(dJ))), "max_abs_dK": float(np.max(np.abs(dK))),
                        "dE_one_build": float(0.5 * np.sum(D * dJ) - 0.25 * np.sum(D * dK)),
                        "roofline_frac_t_ideal": t_ideal / (float(cms.sum()) * 1e-3)}
        out["mixed"]["schedules"] = tune_mx
        _progress(f"mixed build {ms_mx:.2f} ms ({n32 / max(1, stm['quartets']):.2f} FP32 quartets)")
        ref = mx
    split = None
    if args.split and all(l <= 2 for l in sys_["sh_l"]):
        # the split build of the paper's opt-UM scheme: J by the McMurchie-
        # Davidson J engine, K by the Rys kernels at the looser K threshold
        split, _ = make(0.0, f"{args.workload}_fp64", tau_k=args.tau_k)
        Js, Ks = torch.empty_like(Dd), torch.empty_like(Dd)
        split.build_jk(Dd, Js, Ks, stream=stream, j_engine=True, sync=True)  # its lists
        ms_sp = _time_builds(torch, split, Dd, Js, Ks, stream, args.warmup, args.steps, j_engine=True)
        ctx.build_jk(Dd, J, K, stream=stream)
        torch.cuda.synchronize()
        dJ = (Js - J).cpu().numpy()
        dK = (Ks - K).cpu().numpy()
        out["split_jk"] = {"tau_k": args.tau_k, "ms_per_step": ms_sp, "builds_per_s": 1000.0 / ms_sp,
                           "speedup_vs_fused": ms / ms_sp,
                           "max_abs_dJ": float(np.max(np.abs(dJ))), "max_abs_dK": float(np.max(np.abs(dK))),
                           "dE_one_build": float(0.5 * np.sum(D * dJ) - 0.25 * np.sum(D * dK))}
        _progress(f"split J-engine/K build {ms_sp:.2f} ms")
    if not args.no_scf:
        # SCF from the core-Hamiltonian guess on the same lists (outside the
        # timed region): |dE| < 1e-10, max |error| < 1e-8
        r = ctx.run_scf()
        out["scf"] = {"iterations": r["iterations"], "converged": bool(r["converged"]), "energy": r["energy"],
                      "seconds": r["total_seconds"], "jk_seconds": r["jk_seconds"],
                      "jk_ms_per_iteration": 1000.0 * r["jk_seconds"] / max(1, r["iterations"]),
                      "guess": "core Hamiltonian"}
        if ref is not None:
            rm = ref.run_scf()
            out["mixed"]["scf"] = {"iterations": rm["iterations"], "converged": bool(rm["converged"]),
                                   "energy": rm["energy"], "seconds": rm["total_seconds"],
                                   "jk_seconds": rm["jk_seconds"],
                                   "energy_minus_fp64": rm["energy"] - r["energy"]}
        if split is not None:
            # the loose K screen follows D from one iteration to the next, so
            # this SCF stops at |dE| < 1e-7, max |error| < 1e-5
            rs = split.run_scf(j_engine=True, e_tol=1e-7, g_tol=1e-5)
            out["split_jk"]["scf"] = {"iterations": rs["iterations"], "converged": bool(rs["converged"]),
                                      "energy": rs["energy"], "seconds": rs["total_seconds"],
                                      "jk_seconds": rs["jk_seconds"], "energy_minus_fused": rs["energy"] - r["energy"]}
        guesses = {"sad": fk.GUESS_SAD}
        model = os.path.join(HERE, "paper_2407_21445_amd", "guess_631gs.npz")
        if sys_["name"].endswith("/6-31gs-type") and os.path.exists(model):
            from paper_2407_21445_amd.guess_train import load_model
            try:
                ctx.set_guess_model(*load_model(model))
                guesses["learned"] = fk.GUESS_LEARNED
            except fk.FockJKError as e:  # weights of another feature layout
                print(f"bench.py: learned guess skipped: {e}", file=sys.stderr)
        for name, g in guesses.items():
            rg = ctx.run_scf(guess=g)
            out["scf"][name] = {"iterations": rg["iterations"], "converged": bool(rg["converged"]),
                                "seconds": rg["total_seconds"], "guess_seconds": rg["guess_seconds"],
                                "energy_minus_core_start": rg["energy"] - r["energy"],
                                "guess_used": {0: "core", 2: "sad", 3: "learned"}.get(rg["guess_used"], "?")}
        _progress(f"SCF: {r['iterations']} iterations")
    if args.workload != "c20h42" and not args.no_extra:
        # the C20H42 / 6-31G*-type workload, FP64, as a second line of reference
        from synth import workloads as wl
        s2y = wl.c20h42_631gs()
        c2 = fk.FockJK(0).set_system(s2y)
        src2 = _load_cached(c2, "c20h42_fp64", arch, args)
        c2.build_quartets(tau=args.tau, tau_prim=args.tau_prim, block_tasks=args.block_tasks)
        S2, T2, V2, _ = c2.one_electron()
        D2 = torch.tensor(_core_density(S2, T2 + V2, s2y["nelec"] // 2), dtype=torch.float64, device=dev)
        J2, K2 = torch.empty_like(D2), torch.empty_like(D2)
        if src2 == "autotune":
            _tune(c2, D2, stream)
            _save_tuned(c2, "c20h42_fp64", arch, args)
        ms2 = _time_builds(torch, c2, D2, J2, K2, stream, 3, 20)
        st2 = c2.stats()
        out["c20h42"] = {"workload": "C20H42 all-trans (0.02 A jitter), 6-31G*-type, 384 Cartesian bf, fp64",
                         "builds_per_s": 1000.0 / ms2, "ms_per_step": ms2, "schedules": src2,
                         "quartets_per_s": st2["quartets"] / (ms2 * 1e-3)}
        _progress(f"C20H42 build {ms2:.2f} ms")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sys_, st["classes"], args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="water64", choices=("water64", "c20h42", "water4", "c4"))
    ap.add_argument("--tau", type=float, default=1e-10)
    ap.add_argument("--tau-prim", type=float, default=1e-12, help="primitive-pair pruning threshold")
    ap.add_argument("--tau-fp32", type=float, default=1e-5,
                    help="mixed leg: FP32 recurrences for waves whose quartets all have G_ab G_cd D_max below "
                         "this (0: no mixed leg; for --workload c4 the precision of the timed batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--classes", action="store_true", help="print the per-class kernel table to stderr")
    ap.add_argument("--schedule", action="append", default=[], metavar="LA,LB,LC,LD,BB,KT,GF",
                    help="fix a class schedule (bra block, kets per tile, grid fraction) before the lists "
                         "are built; with --no-autotune it is the one timed")
    ap.add_argument("--engine", choices=("rys", "hgp"), default="rys",
                    help="integral engine before tuning: hgp selects it for every class it is built for "
                         "(the autotuner may still switch a class)")
    ap.add_argument("--no-split", dest="split", action="store_false",
                    help="skip the split build (J engine + K at --tau-k) timed beside the fused one")
    ap.add_argument("--tau-k", type=float, default=5e-6, help="K threshold of the split build")
    ap.add_argument("--no-block-tasks", dest="block_tasks", action="store_false",
                    help="ket-outer classes take tiles per wave instead of whole bra blocks per workgroup")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF runs reported beside the build rate")
    ap.add_argument("--no-extra", action="store_true", help="skip the C20H42 reference line")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the default kernel schedules (by default the committed schedule cache of the "
                         "workload is loaded, or the autotuner runs before timing if there is none)")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even where a schedule cache exists")
    ap.add_argument("--save-schedules", metavar="DIR", default="",
                    help="write the schedules the autotuner chose to DIR/<workload>_<leg>.<arch>.txt")
    ap.add_argument("--nmol", type=int, default=8, help="molecules of the organic batch (--workload c4)")
    ap.add_argument("--batch-scf", action="store_true", help="--workload c4: also run the batched SCF")
    ap.add_argument("--canonical", type=float, default=0.0,
                    help="--batch-scf: canonical orthogonalisation cutoff (overlap eigenvalues dropped; 0: "
                         "symmetric S^(-1/2))")
    ap.add_argument("--batch-density", choices=("core", "sad"), default="core",
                    help="--workload c4: density of the timed builds")
    ap.add_argument("--progress", action="store_true",
                    help="--workload c4: report finished class launches during each build (long batches)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 5 times (calibrates HBM byte counters)")
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
        if "--tau-fp32" not in " ".join(sys.argv):
            args.tau_fp32 = 0.0
        return bench_batch(args, torch, fk)
    return bench_single(args, torch, fk)


if __name__ == "__main__":
    sys.exit(main())
