"""Trains the learned initial-density network on the library's own converged
densities and evaluates it against the SAD guess.

    python -m paper_2407_21445_amd.guess_train train --out guess_631gs.npz
    python -m paper_2407_21445_amd.guess_train eval --model guess_631gs.npz

Training data: the geometries of ``synth.workloads.guess_geometry`` (alkanes
C4-C16 and water clusters of 4-32 molecules, 6-31G*-type basis) except the
held-out tail; each is converged by the library's SCF (from the SAD guess),
and its density is cut into bond-frame pair blocks by ``fk_guess_targets``.
The network (192 -> 256 -> 256 -> 225, SiLU) is trained with the library's
forward, backward, masked-MSE and Adam kernels; PyTorch only holds the device
arrays and gathers the shuffled minibatch rows.

Evaluation: SCF from SAD and from the learned guess on the held-out
geometries; iterations, wall times and the energy difference per geometry.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402  (before the library: one HIP runtime)

import paper_2407_21445_amd as fk  # noqa: E402
from synth import workloads as wl  # noqa: E402

DIMS = (fk.GUESS_NFEAT, 256, 256, fk.GUESS_NOUT)
DEFAULT_MODEL = os.path.join(HERE, "guess_631gs.npz")


def log(*a):
    print(*a, flush=True)


def load_model(path=DEFAULT_MODEL):
    z = np.load(path, allow_pickle=False)
    L = int(z["nlayer"])
    return [z[f"W{k}"] for k in range(L)], [z[f"b{k}"] for k in range(L)]


def _converge(i, tau=1e-10):
    s = wl.guess_system(i)
    c = fk.FockJK(0).set_system(s).build_quartets(tau=tau)
    r = c.run_scf(guess=fk.GUESS_SAD, e_tol=1e-8, g_tol=1e-6)
    if not r["converged"]:
        return i, None
    X, sh = c.guess_pairs()
    Y = c.guess_targets(r["D"])
    c.close()
    return i, (X, sh, Y, r["iterations"])


def generate(indices, budget_s, workers=4):
    """Converged pair data for as many geometries as fit in the budget."""
    t0 = time.time()
    out, stop = {}, threading.Event()
    def job(i):
        if stop.is_set():
            return i, None
        return _converge(i)
    with cf.ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(job, i) for i in indices]
        done = 0
        for f in cf.as_completed(futs):
            i, d = f.result()
            if d is not None:
                out[i] = d
            done += 1
            if done % 50 == 0:
                log(f"data: {done}/{len(indices)} geometries, {sum(len(v[0]) for v in out.values())} pairs, "
                    f"{time.time() - t0:.0f} s")
            if time.time() - t0 > budget_s:
                stop.set()
    return out


def train(data, epochs, budget_s, batch=2048, lr=1e-3, seed=2407, val_frac=0.05):
    dev = torch.device("cuda:0")
    keys = sorted(data)
    rng = np.random.default_rng(seed)
    rng.shuffle(keys)
    nval = max(1, int(len(keys) * val_frac))
    # inputs are standardised on the host with the training set's mean and
    # spread; the affine map is folded into the first layer afterwards
    Xall = np.concatenate([data[k][0] for k in keys[nval:]]).astype(np.float64)
    mu = Xall.mean(axis=0)
    sd = Xall.std(axis=0)
    sd[sd < 1e-6] = 1.0
    del Xall

    def stack(ks):
        X = ((np.concatenate([data[k][0] for k in ks]) - mu) / sd).astype(np.float32)
        S = np.concatenate([data[k][1] for k in ks])
        Y = np.concatenate([data[k][2] for k in ks])
        return (torch.from_numpy(X).to(dev), torch.from_numpy(S).to(dev), torch.from_numpy(Y).to(dev),
                float(sum((int(v) >> 8) * (int(v) & 255) for v in S)))
    Xv, Sv, Yv, cv = stack(keys[:nval])
    Xt, St, Yt, _ = stack(keys[nval:])
    n = Xt.shape[0]
    batch = min(batch, n)
    log(f"train: {len(keys) - nval} geometries / {n} pairs, validation {nval} / {Xv.shape[0]}")
    # He-type initialisation; the last bias starts at the mean target
    Ws = [torch.from_numpy((rng.normal(size=(DIMS[k], DIMS[k + 1])) * math.sqrt(1.0 / DIMS[k])).astype(np.float32))
          .to(dev) for k in range(3)]
    bs = [torch.zeros(DIMS[k + 1], dtype=torch.float32, device=dev) for k in range(3)]
    bs[2].copy_(Yt.mean(dim=0))
    gW = [torch.zeros_like(W) for W in Ws]
    gb = [torch.zeros_like(b) for b in bs]
    m1W, m1b = [torch.zeros_like(W) for W in Ws], [torch.zeros_like(b) for b in bs]
    m2W, m2b = [torch.zeros_like(W) for W in Ws], [torch.zeros_like(b) for b in bs]
    work = fk.mlp_work(Ws, batch)
    dY = torch.empty((batch, DIMS[-1]), dtype=torch.float32, device=dev)
    part, loss = fk.mse_scratch(dev), torch.zeros(1, dtype=torch.float64, device=dev)

    def evaluate(X, S, Y, cnt):
        tot = 0.0
        wk = fk.mlp_work(Ws, X.shape[0])
        P = fk.mlp_forward(Ws, bs, X, wk)
        g = torch.empty_like(P)
        fk.block_mse(P, Y, S, cnt, g, part, loss)
        tot = float(loss.item())
        return tot

    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    t0, step, hist = time.time(), 0, []
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=gen)
        run = 0.0
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            X, S, Y = Xt[idx].contiguous(), St[idx].contiguous(), Yt[idx].contiguous()
            cnt = float(((S >> 8) * (S & 255)).sum().item())
            P = fk.mlp_forward(Ws, bs, X, work)
            fk.block_mse(P, Y, S, cnt, dY, part, loss)
            fk.mlp_backward(Ws, bs, X, work, dY, gW, gb)
            step += 1
            rate = lr * 0.5 * (1 + math.cos(math.pi * min(step, total) / total)) + 1e-5
            fk.mlp_adam(Ws, bs, gW, gb, m1W, m1b, m2W, m2b, step, rate)
            if b % 50 == 0:
                run = float(loss.item())
        vl = evaluate(Xv, Sv, Yv, cv)
        hist.append((ep, run, vl))
        log(f"epoch {ep}: train batch loss {run:.3e}  validation {vl:.3e}  ({time.time() - t0:.0f} s)")
        if time.time() - t0 > budget_s:
            break
    torch.cuda.synchronize()
    W = [w.cpu().numpy().astype(np.float64) for w in Ws]
    b = [v.cpu().numpy().astype(np.float64) for v in bs]
    # fold the standardisation: ((x - mu) / sd) W0 + b0 = x (W0 / sd) + (b0 - (mu / sd) W0)
    b[0] = b[0] - (mu / sd) @ W[0]
    W[0] = W[0] / sd[:, None]
    return [w.astype(np.float32) for w in W], [v.astype(np.float32) for v in b], hist


def cmd_train(a):
    t0 = time.time()
    ntrain = wl.GUESS_SET_SIZE - wl.GUESS_HELD_OUT
    data = generate(range(min(a.n_train, ntrain)), a.data_budget, a.workers)
    log(f"data: {len(data)} geometries in {time.time() - t0:.0f} s")
    Ws, bs, hist = train(data, a.epochs, a.train_budget)
    meta = {"basis": "6-31gs-type", "geometries": len(data), "pairs": int(sum(len(v[0]) for v in data.values())),
            "epochs": len(hist), "final_validation_mse": hist[-1][2], "dims": list(DIMS),
            "rcut_bohr": fk.GUESS_RCUT, "nrbf": fk.GUESS_NRBF, "seconds": time.time() - t0}
    arrs = {f"W{k}": Ws[k] for k in range(3)}
    arrs.update({f"b{k}": bs[k] for k in range(3)})
    np.savez(a.out, nlayer=np.int32(3), meta=np.array(json.dumps(meta)), **arrs)
    log("saved", a.out, json.dumps(meta))


def cmd_eval(a):
    Ws, bs = load_model(a.model)
    first = wl.GUESS_SET_SIZE - wl.GUESS_HELD_OUT
    idx = list(range(first, first + a.n_eval))
    rows = []
    t0 = time.time()
    for k, i in enumerate(idx):
        s = wl.guess_system(i)
        c = fk.FockJK(0).set_system(s).build_quartets(tau=1e-10)
        c.set_guess_model(Ws, bs)
        # the one-electron matrices are computed once per geometry and kept:
        # form them before either timed run so that both start alike
        c.run_scf(max_iter=0, guess=fk.GUESS_CORE)
        r0 = c.run_scf(guess=fk.GUESS_SAD)
        r1 = c.run_scf(guess=fk.GUESS_LEARNED)
        rows.append({"i": i, "name": s["name"], "nbf": s["nbf"], "sad_iter": r0["iterations"],
                     "learned_iter": r1["iterations"], "sad_s": r0["total_seconds"], "learned_s": r1["total_seconds"],
                     "guess_s": r1["guess_seconds"], "used": r1["guess_used"], "conv": bool(r0["converged"] and r1["converged"]),
                     "dE": r1["energy"] - r0["energy"]})
        c.close()
        if (k + 1) % 20 == 0:
            log(f"eval: {k + 1}/{len(idx)} ({time.time() - t0:.0f} s)")
    it0 = np.array([r["sad_iter"] for r in rows])
    it1 = np.array([r["learned_iter"] for r in rows])
    s0 = np.array([r["sad_s"] for r in rows])
    s1 = np.array([r["learned_s"] for r in rows])
    summ = {"geometries": len(rows), "sad_iterations_mean": float(it0.mean()), "learned_iterations_mean": float(it1.mean()),
            "sad_seconds_total": float(s0.sum()), "learned_seconds_total": float(s1.sum()),
            "guess_seconds_mean": float(np.mean([r["guess_s"] for r in rows])),
            "max_abs_dE": float(max(abs(r["dE"]) for r in rows)), "all_converged": all(r["conv"] for r in rows),
            "learned_used": sum(r["used"] == fk.GUESS_LEARNED for r in rows),
            "fewer": int((it1 < it0).sum()), "equal": int((it1 == it0).sum()), "more": int((it1 > it0).sum())}
    log(json.dumps(summ))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": summ, "rows": rows}, f, indent=1)


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=1800)
    t.add_argument("--data-budget", type=float, default=600.0, help="seconds for the SCF data")
    t.add_argument("--train-budget", type=float, default=240.0)
    t.add_argument("--epochs", type=int, default=60)
    t.add_argument("--workers", type=int, default=4)
    t.add_argument("--out", default=DEFAULT_MODEL)
    e = sub.add_parser("eval")
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--n-eval", type=int, default=wl.GUESS_HELD_OUT)
    e.add_argument("--out", default="")
    a = p.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("guess_train needs a GPU")
    {"train": cmd_train, "eval": cmd_eval}[a.cmd](a)


if __name__ == "__main__":
    main()
