"""Learned-warm-start experiment on the 137M-parameter network.

    python -m paper_2509_22462_amd.warmstart_run [--train 4096] [--test 256]
        [--hess-prec bf16] [--epochs 300] [--out dataset.npz]

Reduced-space problems  min ||x - x0||^2  s.t.  NN(x)_t - NN(x)_c >= 0.5,
0 <= x <= 1  with the tanh MLP 784-4096-8192-8192-4096-10 (weights
N(0, 1/fan_in), seed 0) and synthetic 28x28 blob images x0.  Cold-solves the
training set (lock-step batches, GPU oracles, Newton systems by the device
KKT solve unless --host-kkt; the line search allows for the FP32 rounding
of the network values), trains the 794-512-512-804 warm-start MLP with the
library's kernels, then solves the held-out set cold and warm.  Solves that
do not converge are classified by a projected-gradient ascent of the margin
from the returned point (reachable / locally infeasible).  Progress lines go to stderr; one JSON summary line to stdout.
The solved training set is checkpointed to --out after every chunk and
resumed from there when the file holds the same configuration; with
--max-seconds the cold solves stop after that budget (exit status 75, the
checkpoint kept) so that a long dataset can be built over several runs.
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


def load_checkpoint(path, cfg):
    if not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        d = dict(np.load(f))
    if not np.array_equal(d["cfg"], cfg):
        return None
    return d


def save_checkpoint(path, **arrays):
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:  # a file object: numpy adds no suffix
        np.savez_compressed(f, **arrays)
    os.replace(tmp, path)


def build_dataset(train, ev, opts, a, m, cfg):
    """Cold-solve the training problems chunk by chunk, checkpointing as it goes."""
    n = train[0].n
    d = load_checkpoint(a.out, cfg)
    if d is None:
        d = dict(cfg=cfg, done=np.array(0), F=np.zeros((len(train), n + m)),
                 Y=np.zeros((len(train), n + 2 * m)), iters=np.zeros(len(train), dtype=np.int64),
                 ok=np.zeros(len(train), dtype=bool), status=np.array([""] * len(train), dtype="<U20"))
    if "status" not in d:  # checkpoints written before statuses were kept
        d["status"] = np.array([""] * len(train), dtype="<U20")
    done = int(d["done"])
    if done:
        log(f"resuming: {done}/{len(train)} training problems already solved in {a.out}")
    t0 = time.perf_counter()
    while done < len(train):
        chunk = train[done:done + a.chunk]
        res = ipm.solve_batch(chunk, ev, None, opts, max_batch=a.chunk)
        sl = slice(done, done + len(chunk))
        d["F"][sl] = warmstart.features(chunk, m)
        d["Y"][sl] = warmstart.targets(res)
        d["iters"][sl] = [r.iters for r in res]
        d["ok"][sl] = [r.status == "converged" for r in res]
        d["status"][sl] = [r.status for r in res]
        done += len(chunk)
        d["done"] = np.array(done)
        save_checkpoint(a.out, **d)
        log(f"train cold: {done}/{len(train)} solved ({int(d['ok'][:done].sum())} converged), "
            f"mean iters {d['iters'][:done].mean():.1f}, {time.perf_counter() - t0:.1f}s")
        # every run solves at least one chunk; the budget is checked between chunks
        if a.max_seconds and done < len(train) and time.perf_counter() - t0 > a.max_seconds:
            return d, False
    return d, True


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
    ap.add_argument("--max-seconds", type=float, default=0.0)
    ap.add_argument("--host-kkt", action="store_true",
                    help="Newton systems solved on the host (numpy) instead of the device KKT solve")
    a = ap.parse_args(argv)

    ctx = nnc.Context(0)
    Ws, bs = datagen.mlp_weights(DIMS, seed=0)
    ev = evaluator.GpuEvaluator(ctx, DIMS, ACTS, Ws, bs, prec=a.prec, hess_prec=a.hess_prec,
                                max_points=a.chunk)
    opts = ipm.Options(device_kkt=not a.host_kkt, merit_noise=ev.merit_noise)
    m = DIMS[-1]
    train = warmstart.make_problems(ev.nn, a.train, seed=500, m=m)
    test = warmstart.make_problems(ev.nn, a.test, seed=900, m=m)
    cfg = np.array([a.train, a.hess_prec == "bf16", a.chunk, not a.host_kkt, ev.merit_noise], dtype=np.float64)
    d, complete = build_dataset(train, ev, opts, a, m, cfg)
    if not complete:
        log(f"time budget reached after {int(d['done'])}/{a.train} problems; rerun to resume")
        ev.close()
        ctx.close()
        return 75  # EX_TEMPFAIL: rerun to resume
    ok = d["ok"]
    n = DIMS[0]
    # failed training solves: can the margin be met from the returned point?
    bad = np.nonzero(~ok)[0]
    train_classes = {}
    if bad.size:
        t0 = time.perf_counter()
        _, reached, stationary = ipm.margin_ascent([train[i] for i in bad], d["Y"][bad, :n], ev)
        train_classes = dict(reachable=int(reached.sum()), locally_infeasible=int((~reached & stationary).sum()),
                             undecided=int((~reached & ~stationary).sum()))
        log(f"failed training solves classified in {time.perf_counter() - t0:.1f}s: {train_classes}")
    F, Y, cold_train_iters = d["F"][ok], d["Y"][ok], d["iters"][ok]
    model = warmstart.WarmStartModel(ctx, DIMS[0], m, hidden=(512, 512), batch=256, prec="bf16")
    rep = model.fit(F, Y, epochs=a.epochs, lr=a.lr)
    log(f"trained: val loss {rep.val_loss[0]:.4f} -> {rep.val_loss[-1]:.4f} in {rep.seconds:.1f}s")
    starts = model.starts(test)
    cmp_ = warmstart.compare(test, starts, ev, opts, max_batch=a.chunk)
    both = np.array([cs == "converged" and ws == "converged"
                     for cs, ws in zip(cmp_.cold_status, cmp_.warm_status)])
    cold_bad = [i for i, st in enumerate(cmp_.cold_status) if st != "converged"]
    test_classes = {}
    if cold_bad:
        _, reached, stationary = ipm.margin_ascent([test[i] for i in cold_bad], cmp_.cold_x[cold_bad], ev)
        test_classes = dict(reachable=int(reached.sum()), locally_infeasible=int((~reached & stationary).sum()),
                            undecided=int((~reached & ~stationary).sum()))
    counts = lambda st: {k: int(sum(1 for x in st if x == k)) for k in sorted(set(st))}  # noqa: E731
    summary = dict(
        workload="learned warm start, tanh MLP 784-4096-8192-8192-4096-10, blob images",
        train_problems=a.train, train_instances=int(F.shape[0]), test_instances=a.test,
        cold_train_iters_mean=float(cold_train_iters.mean()),
        cold_test_converged=int(sum(s == "converged" for s in cmp_.cold_status)),
        cold_iters_mean=float(cmp_.cold_iters.mean()), warm_iters_mean=float(cmp_.warm_iters.mean()),
        cold_seconds=cmp_.cold_seconds, warm_seconds=cmp_.warm_seconds,
        cold_obj_mean=float(cmp_.cold_obj.mean()), warm_obj_mean=float(cmp_.warm_obj.mean()),
        obj_max_abs_diff=float(np.max(np.abs(cmp_.cold_obj - cmp_.warm_obj))),
        fallbacks=cmp_.fallbacks, rejected=cmp_.rejected,
        cold_status=counts(cmp_.cold_status), warm_status=counts(cmp_.warm_status),
        train_failures=dict(count=int(bad.size), statuses=counts([str(x) for x in d["status"][bad]]),
                            classes=train_classes),
        cold_test_failure_classes=test_classes,
        both_converged=int(both.sum()),
        both_cold_iters_mean=float(cmp_.cold_iters[both].mean()),
        both_warm_iters_mean=float(cmp_.warm_iters[both].mean()),
        both_cold_iters_median=float(np.median(cmp_.cold_iters[both])),
        both_warm_iters_median=float(np.median(cmp_.warm_iters[both])),
        both_obj_max_abs_diff=float(np.max(np.abs(cmp_.cold_obj[both] - cmp_.warm_obj[both]))),
        warm_fewer_iters_frac=float(np.mean(cmp_.warm_iters[both] < cmp_.cold_iters[both])),
        train_seconds=rep.seconds, val_loss_first=rep.val_loss[0], val_loss_last=rep.val_loss[-1],
        oracle_seconds=ev.seconds, oracle_calls=ev.calls)
    print(json.dumps(summary), flush=True)
    model.close()
    ev.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
