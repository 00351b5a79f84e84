"""Learned-warm-start experiment on the 137M-parameter network.

    python -m paper_2509_22462_amd.warmstart_run [--train 4096] [--test 256]
        [--hess-prec bf16] [--epochs 300] [--out dataset.npz]

Reduced-space problems  min ||x - x0||^2  s.t.  NN(x)_t - NN(x)_c >= 0.5,
0 <= x <= 1  with the tanh MLP 784-4096-8192-8192-4096-10 (weights
N(0, 1/fan_in), seed 0) and synthetic 28x28 blob images x0.  Cold-solves the
training set (lock-step batches, GPU oracles), trains the 794-512-512-804
warm-start MLP with the library's kernels, then solves the held-out set cold
and warm.  Progress lines go to stderr; one JSON summary line to stdout.
The solved dataset is saved to --out and reused when it already holds the
same configuration (resume).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import datagen, evaluator, ipm, nnc, warmstart

DIMS = datagen.C2_DIMS
ACTS = ["tanh"] * 4 + ["identity"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def solve_chunked(probs, ev, opts, chunk, label):
    out = []
    t0 = time.perf_counter()
    for k in range(0, len(probs), chunk):
        out.extend(ipm.solve_batch(probs[k:k + chunk], ev, None, opts, max_batch=chunk))
        it = np.mean([r.iters for r in out])
        log(f"{label}: {len(out)}/{len(probs)} solved, mean iters {it:.1f}, "
            f"{time.perf_counter() - t0:.1f}s")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--prec", default="fp32")
    ap.add_argument("--hess-prec", default="bf16")
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="warmstart_dataset.npz")
    a = ap.parse_args(argv)

    ctx = nnc.Context(0)
    Ws, bs = datagen.mlp_weights(DIMS, seed=0)
    ev = evaluator.GpuEvaluator(ctx, DIMS, ACTS, Ws, bs, prec=a.prec, hess_prec=a.hess_prec,
                                max_points=a.chunk)
    opts = ipm.Options()
    m = DIMS[-1]
    train = warmstart.make_problems(ev.nn, a.train, seed=500, m=m)
    test = warmstart.make_problems(ev.nn, a.test, seed=900, m=m)
    cfg = np.array([a.train, a.hess_prec == "bf16"], dtype=np.float64)
    if os.path.exists(a.out) and np.array_equal(np.load(a.out)["cfg"], cfg):
        d = np.load(a.out)
        F, Y, cold_train_iters = d["F"], d["Y"], d["iters"]
        log(f"loaded {F.shape[0]} solved instances from {a.out}")
    else:
        res = solve_chunked(train, ev, opts, a.chunk, "train cold")
        ok = [i for i, r in enumerate(res) if r.status == "converged"]
        F = warmstart.features([train[i] for i in ok], m)
        Y = warmstart.targets([res[i] for i in ok])
        cold_train_iters = np.array([res[i].iters for i in ok])
        np.savez(a.out, F=F, Y=Y, iters=cold_train_iters, cfg=cfg)
    model = warmstart.WarmStartModel(ctx, DIMS[0], m, hidden=(512, 512), batch=256, prec="bf16")
    rep = model.fit(F, Y, epochs=a.epochs, lr=a.lr)
    log(f"trained: val loss {rep.val_loss[0]:.4f} -> {rep.val_loss[-1]:.4f} in {rep.seconds:.1f}s")
    starts = model.starts(test)
    cmp_ = warmstart.compare(test, starts, ev, opts, max_batch=a.chunk)
    summary = dict(
        workload="learned warm start, tanh MLP 784-4096-8192-8192-4096-10, blob images",
        train_instances=int(F.shape[0]), test_instances=a.test,
        cold_iters_mean=float(cmp_.cold_iters.mean()), warm_iters_mean=float(cmp_.warm_iters.mean()),
        cold_seconds=cmp_.cold_seconds, warm_seconds=cmp_.warm_seconds,
        cold_obj_mean=float(cmp_.cold_obj.mean()), warm_obj_mean=float(cmp_.warm_obj.mean()),
        obj_max_abs_diff=float(np.max(np.abs(cmp_.cold_obj - cmp_.warm_obj))),
        fallbacks=cmp_.fallbacks, rejected=cmp_.rejected,
        train_seconds=rep.seconds, val_loss_first=rep.val_loss[0], val_loss_last=rep.val_loss[-1],
        oracle_seconds=ev.seconds, oracle_calls=ev.calls)
    print(json.dumps(summary), flush=True)
    model.close()
    ev.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
