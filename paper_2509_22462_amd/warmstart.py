"""Learned warm start for the reduced-space interior-point solves.

Pipeline (all on one GPU, host IPM in FP64):
  1. instances: synthetic 28x28 blob images x0, c = argmax NN(x0), target t
     drawn uniformly among the other labels; problem
         min ||x - x0||^2  s.t.  NN(x)_t - NN(x)_c >= margin,  0 <= x <= 1;
  2. cold solves with the host IPM (many problems in lock step, oracles from
     the GPU library) -> primal-dual solutions (x*, y*, lambda*);
  3. a small MLP  [x0 || e_t - e_c]  ->  [x* || y* || lambda*]  (standardised
     targets) trained on the GPU by the library's own forward/backward GEMM
     kernels and Adam (nnc_train_*);
  4. warm starts for held-out problems: x = clip(x_hat), lambda = lambda_hat,
     nu from lambda_hat (the y-stationarity lambda + nu (e_t - e_c) = 0), and
     a small initial barrier parameter; the cold start is the fallback (a
     non-finite prediction is rejected; a warm solve that does not converge
     is re-solved cold) and the reference for iteration counts and final
     objectives.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import datagen, ipm, nnc


def make_problems(nn_fn, count: int, seed: int, m: int, margin: float = 0.5,
                  side: int = 28) -> List[ipm.Problem]:
    X0 = datagen.blob_images(count, seed, side)
    logits = np.asarray(nn_fn(X0))
    c = np.argmax(logits, axis=1)
    rng = np.random.default_rng(seed + 7919)
    t = (c + rng.integers(1, m, size=count)) % m
    return [ipm.Problem(x0=X0[i], t=int(t[i]), c=int(c[i]), margin=margin) for i in range(count)]


def features(probs: List[ipm.Problem], m: int) -> np.ndarray:
    n = probs[0].n
    F = np.zeros((len(probs), n + m))
    for i, p in enumerate(probs):
        F[i, :n] = p.x0
        F[i, n + p.t] += 1.0
        F[i, n + p.c] -= 1.0
    return F


def targets(results: List[ipm.Result]) -> np.ndarray:
    return np.stack([np.concatenate([r.x, r.y, r.lam]) for r in results])


@dataclasses.dataclass
class FitReport:
    epochs: int
    train_loss: List[float]
    val_loss: List[float]
    seconds: float


class WarmStartModel:
    """The warm-start MLP, trained with the library's GPU kernels."""

    def __init__(self, ctx: "nnc.Context", n: int, m: int, hidden=(512, 512), batch: int = 256,
                 prec: str = "bf16", seed: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.n, self.m = n, m
        self.dims = [n + m, *hidden, n + 2 * m]
        self.batch = batch
        self.h = nnc.nnc_train_create(ctx.h, self.dims, batch, nnc.PREC_CODES[prec], seed)
        dev = ctx.device
        self.Xb = torch.zeros(batch, self.dims[0], dtype=torch.float64, device=dev)
        self.Yb = torch.zeros(batch, self.dims[-1], dtype=torch.float64, device=dev)
        self.Pb = torch.zeros(batch, self.dims[-1], dtype=torch.float64, device=dev)
        self.mu = np.zeros(self.dims[-1])
        self.sd = np.ones(self.dims[-1])

    def fit(self, F, Y, epochs: int = 200, lr: float = 1e-3, val_frac: float = 0.1,
            seed: int = 0, verbose: bool = False) -> FitReport:
        torch = self.torch
        t0 = time.perf_counter()
        rng = np.random.default_rng(seed)
        idx = rng.permutation(F.shape[0])
        nval = max(1, int(round(val_frac * F.shape[0])))
        val, tr = idx[:nval], idx[nval:]
        self.mu = Y[tr].mean(axis=0)
        self.sd = np.maximum(Y[tr].std(axis=0), 1e-3)
        Z = (Y - self.mu) / self.sd
        tl, vl = [], []
        steps = max(1, -(-len(tr) // self.batch))  # ceil: every row seen once per epoch
        for ep in range(epochs):
            # wrap the permutation so every step has a full batch, even when
            # the training set is smaller than one batch
            order = np.resize(rng.permutation(tr), steps * self.batch)
            losses = []
            for k in range(steps):
                rows = order[k * self.batch:(k + 1) * self.batch]
                self.Xb.copy_(torch.from_numpy(F[rows]))
                self.Yb.copy_(torch.from_numpy(Z[rows]))
                want = (k == 0)
                loss = nnc.nnc_train_step(self.ctx.h, self.h, self.Xb.data_ptr(), self.Yb.data_ptr(),
                                          lr, want_loss=want)
                if want:
                    losses.append(loss)
            tl.append(float(np.mean(losses)) if losses else float("nan"))
            if ep % 10 == 0 or ep == epochs - 1:
                P = self.predict_std(F[val])
                vl.append(float(np.mean((P - Z[val]) ** 2)))
                if verbose:
                    print(f"epoch {ep} train {tl[-1]:.4f} val {vl[-1]:.4f}", flush=True)
        return FitReport(epochs, tl, vl, time.perf_counter() - t0)

    def predict_std(self, F) -> np.ndarray:
        torch = self.torch
        out = np.empty((F.shape[0], self.dims[-1]))
        for k in range(0, F.shape[0], self.batch):
            b = min(self.batch, F.shape[0] - k)
            self.Xb[:b].copy_(torch.from_numpy(F[k:k + b]))
            nnc.nnc_train_predict(self.ctx.h, self.h, b, self.Xb.data_ptr(), self.Pb.data_ptr())
            out[k:k + b] = self.Pb[:b].cpu().numpy()
        return out

    def predict(self, F) -> np.ndarray:
        return self.predict_std(F) * self.sd + self.mu

    def starts(self, probs: List[ipm.Problem], mu0: float = 1e-2) -> List[Optional[ipm.Start]]:
        P = self.predict(features(probs, self.m))
        return [start_from_prediction(p, row, self.n, self.m, mu0) for p, row in zip(probs, P)]

    def close(self):
        if self.h is not None:
            nnc.nnc_train_destroy(self.ctx.h, self.h)
            self.h = None


def start_from_prediction(prob: ipm.Problem, row: np.ndarray, n: int, m: int,
                          mu0: float) -> Optional[ipm.Start]:
    """Turn one predicted [x || y || lambda] into an IPM start (None = reject)."""
    if not np.all(np.isfinite(row)):
        return None
    x = np.clip(row[:n], 0.0, 1.0)
    lam = row[n + m:n + 2 * m].copy()
    # y-stationarity lambda + nu (e_t - e_c) = 0 fixes nu from lambda_t, lambda_c
    nu = 0.5 * (lam[prob.c] - lam[prob.t])
    return ipm.Start(x=x, y=None, lam=lam, nu=min(nu, 0.0), mu0=mu0)


@dataclasses.dataclass
class Comparison:
    cold_iters: np.ndarray
    warm_iters: np.ndarray
    cold_obj: np.ndarray
    warm_obj: np.ndarray
    cold_seconds: float
    warm_seconds: float
    fallbacks: int
    rejected: int
    warm_status: list
    cold_status: list
    cold_x: np.ndarray = None  # returned points of the cold solves (failure classification)


def compare(probs, starts, ev, opts=None, max_batch=None) -> Comparison:
    """Cold vs warm solves of the same problems; warm failures fall back to cold."""
    t0 = time.perf_counter()
    cold = ipm.solve_batch(probs, ev, None, opts, max_batch)
    t1 = time.perf_counter()
    rejected = sum(s is None for s in starts)
    warm = ipm.solve_batch(probs, ev, starts, opts, max_batch)
    fb = [i for i, r in enumerate(warm) if r.status != "converged"]
    if fb:
        redo = ipm.solve_batch([probs[i] for i in fb], ev, None, opts, max_batch)
        for i, r in zip(fb, redo):
            r.iters += warm[i].iters  # the wasted warm iterations count against it
            warm[i] = r
    t2 = time.perf_counter()
    return Comparison(
        cold_iters=np.array([r.iters for r in cold]), warm_iters=np.array([r.iters for r in warm]),
        cold_obj=np.array([r.obj for r in cold]), warm_obj=np.array([r.obj for r in warm]),
        cold_seconds=t1 - t0, warm_seconds=t2 - t1, fallbacks=len(fb), rejected=rejected,
        warm_status=[r.status for r in warm], cold_status=[r.status for r in cold],
        cold_x=np.stack([r.x for r in cold]))
