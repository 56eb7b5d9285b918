"""Training and evaluation of the learned basis surrogate on the GPU.

The data are the shape vectors the method computes itself: for seeded 64^3
pore domains with a lognormal modulus (8^3-voxel box grains), hplmm_setup
builds every grain's exact basis and hplmm_sg_samples turns a random subset
of the (grain, interface, mortar) samples into network inputs and targets.
Training runs the library's own convolution, loss and Adam kernels; PyTorch
only holds the device tensors and draws the mini-batches.

    python -m paper_2509_19777_amd.surrogate train --domains 40 --per-grain 4 --epochs 32 --out w.npz
    python -m paper_2509_19777_amd.surrogate eval --weights w.npz
    python -m paper_2509_19777_amd.surrogate compare   (exact vs surrogate set-up on a fresh 64^3 domain)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import hplmm as hp
from . import synth

CHANNELS = (4, 32, 32, 32, 9)
TRAIN_SEED0, EVAL_SEED = 1000, 7
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "basis_surrogate_poresE64_n4.npz")


def conv_macs(channels=CHANNELS):
    """Multiply-adds of one sample's forward pass (27 offsets x 729 positions)."""
    return 27 * 729 * sum(a * b for a, b in zip(channels[:-1], channels[1:]))


def train_flops(channels=CHANNELS):
    """Flops of one training sample: forward, weight gradients of every layer,
    data gradients of every layer but the first."""
    f = conv_macs(channels)
    d = f - 27 * 729 * channels[0] * channels[1]
    return 2 * (2 * f + d)


def domain_samples(p, per_grain, rng):
    """Inputs and targets of per_grain random samples of every grain of one domain."""
    import torch
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=p.n_mortar)
    S.setup()
    x, y, meta = hp.surrogate_samples(S)
    idx = []
    for m in np.unique(meta[:, 0]):
        cand = np.flatnonzero(meta[:, 0] == m)
        idx.extend(rng.choice(cand, size=min(per_grain, cand.size), replace=False).tolist())
    it = torch.from_numpy(np.sort(np.asarray(idx, dtype=np.int64))).cuda()
    xs, ys = x.index_select(0, it), y.index_select(0, it)
    n_grains = int(np.unique(meta[:, 0]).size)
    del S, x, y
    return xs, ys, n_grains


def _make_problem(args):
    seed, n, box, n_mortar = args
    return synth.config_pores_lognormal(n, box, seed=seed, n_mortar=n_mortar)


def problems(seeds, n=64, box=8, n_mortar=4, workers=8):
    """The voxel problems of the given seeds, generated in worker processes
    that import NumPy only (started with 'spawn', so none of them touches the
    GPU)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    args = [(s, n, box, n_mortar) for s in seeds]
    if workers <= 1 or len(args) == 1:
        return [_make_problem(a) for a in args]
    with ProcessPoolExecutor(max_workers=min(workers, len(args)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_make_problem, args))


def dataset(probs, per_grain, rng_seed=0, log=None):
    """Samples of the given problems (generate them with problems() before the
    process first touches the GPU)."""
    import torch
    rng = np.random.default_rng(rng_seed)
    n_domains = len(probs)
    xs, ys, grains = [], [], 0
    for d in range(n_domains):
        x, y, g = domain_samples(probs[d], per_grain, rng)
        xs.append(x)
        ys.append(y)
        grains += g
        if log:
            log(f"domain {d + 1}/{n_domains}: {grains} grains, {sum(t.shape[0] for t in xs)} samples")
    return torch.cat(xs), torch.cat(ys), grains


def init_params(seed, channels=CHANNELS, last_scale=0.1):
    """He-normal weights (the output layer scaled down so that the first
    predictions are small), zero biases, in the library's flat order."""
    rng = np.random.default_rng(seed)
    out = []
    nl = len(channels) - 1
    for l, (ci, co) in enumerate(zip(channels[:-1], channels[1:])):
        sc = last_scale if l == nl - 1 else 1.0
        out.append((rng.standard_normal((3, 3, 3, ci, co)) * sc * np.sqrt(2.0 / (27 * ci)), np.zeros(co)))
    return hp.flatten_params(out)


def train(net, X, Y, epochs, batch, lr, seed=0, Xv=None, Yv=None, log=None, decay_every=24):
    """Mini-batch Adam on (X, Y); returns the per-epoch history."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        lr_ep = lr * (0.5 ** (ep // decay_every))
        tot, cnt, kernel_ms = 0.0, 0, 0.0
        t0 = time.perf_counter()
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, yb = X.index_select(0, idx), Y.index_select(0, idx)
            ev0.record()
            loss = net.gradient(xb, yb)
            net.adam(lr_ep)
            ev1.record()
            ev1.synchronize()
            kernel_ms += ev0.elapsed_time(ev1)
            tot += loss * batch
            cnt += batch
        rec = {"epoch": ep + 1, "lr": lr_ep, "train_loss": tot / max(cnt, 1), "samples": cnt,
               "wall_s": time.perf_counter() - t0, "kernel_s": kernel_ms / 1e3,
               "tflops": train_flops(net.channels) * cnt / (kernel_ms * 1e-3) / 1e12 if kernel_ms else None}
        if Xv is not None:
            rec["val_loss"] = evaluate_loss(net, Xv, Yv, batch)
        hist.append(rec)
        if log:
            log(json.dumps(rec))
    return hist


def evaluate_loss(net, X, Y, batch):
    """Mean per-sample relative squared error (the training loss) without updates."""
    tot = 0.0
    n = X.shape[0]
    for b0 in range(0, n, batch):
        xb, yb = X[b0:b0 + batch].contiguous(), Y[b0:b0 + batch].contiguous()
        tot += net.gradient(xb, yb) * xb.shape[0]
    return tot / n


def per_sample_error(net, X, Y, batch):
    """Relative L2 error of every sample's prediction on the interior nodes."""
    import torch
    errs = []
    for b0 in range(0, X.shape[0], batch):
        xb, yb = X[b0:b0 + batch].contiguous(), Y[b0:b0 + batch].contiguous()
        pb = net.forward(xb)
        m = (xb[..., 0:1] > 0.5).float()
        num = (((pb - yb) * m) ** 2).sum(dim=(1, 2, 3, 4))
        den = ((yb * m) ** 2).sum(dim=(1, 2, 3, 4)) + 1e-30
        errs.append(torch.sqrt(num / den).cpu().numpy())
    return np.concatenate(errs)


def compare(net, prob, thresholds, reps=3, log=None):
    """Exact set-up versus the surrogate set-up at each threshold on one
    problem: FGMRES(50) iterations to 1e-8 and the set-up / solve times (best
    of reps, host clock around synchronised calls)."""
    import torch
    sysm, part = hp.build_problem(prob)
    S = hp.Solver(sysm, part, n_mortar=prob.n_mortar)
    rows = []

    def timed(fn):
        best, out = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3
            best = t if best is None else min(best, t)
        return best, out

    for thr in [None] + list(thresholds):
        if thr is None:
            t_set, st = timed(lambda: S.setup())
        else:
            t_set, st = timed(lambda: S.setup_surrogate(net, thr))
        t_sol, (x, info) = timed(lambda: S.solve(rtol=1e-8, restart=50, maxit=300))
        rec = {"basis": "exact" if thr is None else f"surrogate, threshold {thr:g}",
               "setup_ms": round(t_set, 2), "solve_ms": round(t_sol, 2), "iters": info["iters"],
               "status": info["status"], "rel_res": info["rel_res"]}
        if thr is not None:
            rec.update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()})
        rows.append(rec)
        if log:
            log(json.dumps(rec))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "compare"])
    ap.add_argument("--domains", type=int, default=40)
    ap.add_argument("--per-grain", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=96)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    # voxel problems first, in worker processes, before this process uses the GPU
    if a.cmd == "train":
        probs = problems([TRAIN_SEED0 + d for d in range(a.domains)] + [EVAL_SEED + 500])
        train_probs, val_probs = probs[:-1], probs[-1:]
    else:
        eval_probs = problems([EVAL_SEED], workers=1)
        if a.cmd == "compare":
            import torch
            torch.cuda.set_device(0)
            net = hp.SurrogateNet(CHANNELS, max_batch=a.batch)
            net.set_params(np.load(a.weights or DEFAULT_WEIGHTS)["params"])
            compare(net, eval_probs[0], [1e-3, 1e-2, 1e-1, 1.0, 1e300], log=log)
            return 0
    log("problems generated")
    import torch
    torch.cuda.set_device(0)
    net = hp.SurrogateNet(CHANNELS, max_batch=a.batch)
    if a.weights:
        net.set_params(np.load(a.weights)["params"])
    else:
        net.set_params(init_params(0))
    if a.cmd == "train":
        X, Y, grains = dataset(train_probs, a.per_grain, log=log)
        Xv, Yv, _ = dataset(val_probs, 2, rng_seed=1)
        log(f"training on {X.shape[0]} samples from {grains} grains; validation {Xv.shape[0]} samples")
        hist = train(net, X, Y, a.epochs, a.batch, a.lr, Xv=Xv, Yv=Yv, log=log)
        if a.out:
            np.savez(a.out, params=net.get_params(), channels=np.array(CHANNELS), history=json.dumps(hist),
                     grains=grains, samples=X.shape[0])
            log(f"saved {a.out}")
    else:
        Xe, Ye, g = dataset(eval_probs, 1 << 30)
        e = per_sample_error(net, Xe, Ye, a.batch)
        log(json.dumps({"grains": g, "samples": int(e.size), "median_rel_err": float(np.median(e)),
                        "p90_rel_err": float(np.quantile(e, 0.9)), "max_rel_err": float(e.max())}))


if __name__ == "__main__":
    sys.exit(main())
