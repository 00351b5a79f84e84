"""GPU oracle evaluator for the host interior-point driver.

Wraps one (or two) library networks: ``nn``/``jac`` run on the network of
precision ``prec`` and ``hess`` on ``hess_prec`` (the Hessian only shapes the
Newton step, so it may run in BF16 while g and J -- which decide the KKT
residuals -- stay FP32).  Rows are evaluated in chunks of ``max_points`` with
device buffers (and pinned host staging buffers for the copies back)
allocated once.  ``newton`` keeps the Hessian on the device and solves the
reduced Newton system there (nnc_kkt_solve; only dx returns).  Wall-clock
per oracle is accumulated in the categories of the paper's Table 4
(function, Jacobian, Hessian, and the device solver when it is used).
"""
from __future__ import annotations

import time

import numpy as np

from . import ipm, nnc


class GpuEvaluator(ipm.Evaluator):
    def __init__(self, ctx: "nnc.Context", dims, acts, Ws, bs, prec="fp32", hess_prec=None,
                 max_points=64):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.dims = list(dims)
        self.n, self.m = dims[0], dims[-1]
        self.B = max_points
        self.net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=max_points)
        hp = hess_prec or prec
        self.hnet = self.net if hp == prec else ctx.net(dims, acts, Ws, bs, prec=hp,
                                                         max_points=max_points)
        dev = ctx.device
        f64 = torch.float64
        self.x = torch.zeros(max_points, self.n, dtype=f64, device=dev)
        self.lam = torch.zeros(max_points, self.m, dtype=f64, device=dev)
        self.g = torch.zeros(max_points, self.m, dtype=f64, device=dev)
        self.J = torch.zeros(max_points, self.m, self.n, dtype=f64, device=dev)
        self.H = torch.zeros(max_points, self.n, self.n, dtype=f64, device=dev)
        # pinned host staging for the results (fast device-to-host copies)
        self.gh = torch.empty(max_points, self.m, dtype=f64, pin_memory=True)
        self.Jh = torch.empty(max_points, self.m, self.n, dtype=f64, pin_memory=True)
        self.Hh = None  # allocated on the first host-side Hessian request
        # device KKT solve (Newton steps with H kept on the GPU)
        self.kkt = None
        self.seconds = {"function": 0.0, "jacobian": 0.0, "hessian": 0.0, "solver": 0.0}
        self.calls = {"function": 0, "jacobian": 0, "hessian": 0, "newton": 0}

    def _chunks(self, X):
        for k in range(0, X.shape[0], self.B):
            yield k, X[k:k + self.B]

    def _load(self, buf, A):
        buf[:A.shape[0]].copy_(self.torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)))

    def nn(self, X):
        t0 = time.perf_counter()
        X = np.atleast_2d(X)
        out = np.empty((X.shape[0], self.m))
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            self._load(self.x, Xc)
            nnc._chk(nnc.nnc_eval_g(self.ctx.h, self.net.h, b, self.x.data_ptr(), None,
                                    self.g.data_ptr()), self.ctx.h, "nnc_eval_g")
            self.gh[:b].copy_(self.g[:b])
            out[k:k + b] = self.gh[:b].numpy()
        self.seconds["function"] += time.perf_counter() - t0
        self.calls["function"] += 1
        return out

    def jac(self, X):
        t0 = time.perf_counter()
        X = np.atleast_2d(X)
        out = np.empty((X.shape[0], self.m, self.n))
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            self._load(self.x, Xc)
            nnc._chk(nnc.nnc_eval_jac_g(self.ctx.h, self.net.h, b, self.x.data_ptr(),
                                        self.J.data_ptr()), self.ctx.h, "nnc_eval_jac_g")
            self.Jh[:b].copy_(self.J[:b])
            out[k:k + b] = self.Jh[:b].numpy()
        self.seconds["jacobian"] += time.perf_counter() - t0
        self.calls["jacobian"] += 1
        return out

    def hess(self, X, Lam):
        t0 = time.perf_counter()
        X = np.atleast_2d(X)
        Lam = np.atleast_2d(Lam)
        out = np.empty((X.shape[0], self.n, self.n))
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            self._load(self.x, Xc)
            self._load(self.lam, Lam[k:k + b])
            nnc._chk(nnc.nnc_eval_hess_lag(self.ctx.h, self.hnet.h, b, self.x.data_ptr(), 0.0,
                                           self.lam.data_ptr(), self.H.data_ptr()), self.ctx.h,
                     "nnc_eval_hess_lag")
            if self.Hh is None:
                self.Hh = self.torch.empty(self.B, self.n, self.n, dtype=self.torch.float64, pin_memory=True)
            self.Hh[:b].copy_(self.H[:b])
            out[k:k + b] = self.Hh[:b].numpy()
        self.seconds["hessian"] += time.perf_counter() - t0
        self.calls["hessian"] += 1
        return out

    def newton(self, X, Lam, D, A, S, R, delta_w0, delta_w_max):
        """Newton steps with the Hessian kept on the device: H from
        nnc_eval_hess_lag into HBM, then (H + diag(D) + S a a^T + delta I) dx = R
        by nnc_kkt_solve, delta raised from 0 to delta_w0 and then by 8x for
        the systems whose factorisation fails (the host driver's inertia
        correction); only dx (and the failure flags) come back."""
        torch = self.torch
        X = np.atleast_2d(X)
        Bt = X.shape[0]
        if self.kkt is None:
            f64 = torch.float64
            dev = self.ctx.device
            self.kkt = nnc.nnc_kkt_create(self.ctx.h, self.n, self.B)
            self.kd = torch.zeros(self.B, self.n, dtype=f64, device=dev)
            self.ka = torch.zeros(self.B, self.n, dtype=f64, device=dev)
            self.ks = torch.zeros(self.B, dtype=f64, device=dev)
            self.kr = torch.zeros(self.B, self.n, dtype=f64, device=dev)
            self.kdelta = torch.zeros(self.B, dtype=f64, device=dev)
            self.kdx = torch.zeros(self.B, self.n, dtype=f64, device=dev)
            self.kinfo = torch.zeros(self.B, dtype=torch.int32, device=dev)
            self.kdxh = torch.empty(self.B, self.n, dtype=f64, pin_memory=True)
            self.kinfoh = torch.empty(self.B, dtype=torch.int32, pin_memory=True)
        out = [None] * Bt
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            t0 = time.perf_counter()
            self._load(self.x, Xc)
            self._load(self.lam, np.atleast_2d(Lam)[k:k + b])
            nnc._chk(nnc.nnc_eval_hess_lag(self.ctx.h, self.hnet.h, b, self.x.data_ptr(), 0.0,
                                           self.lam.data_ptr(), self.H.data_ptr()), self.ctx.h,
                     "nnc_eval_hess_lag")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            self.seconds["hessian"] += t1 - t0
            self._load(self.kd, D[k:k + b])
            self._load(self.ka, A[k:k + b])
            self.ks[:b].copy_(torch.from_numpy(np.ascontiguousarray(S[k:k + b], dtype=np.float64)))
            self._load(self.kr, R[k:k + b])
            delta = np.zeros(b)
            pending = np.ones(b, dtype=bool)
            for _ in range(60):
                self.kdelta[:b].copy_(torch.from_numpy(delta))
                nnc._chk(nnc.nnc_kkt_solve(self.ctx.h, self.kkt, b, self.H.data_ptr(), self.kd.data_ptr(),
                                           self.ka.data_ptr(), self.ks.data_ptr(), self.kdelta.data_ptr(),
                                           self.kr.data_ptr(), self.kdx.data_ptr(), self.kinfo.data_ptr()),
                         self.ctx.h, "nnc_kkt_solve")
                self.kinfoh[:b].copy_(self.kinfo[:b])
                self.kdxh[:b].copy_(self.kdx[:b])
                info = self.kinfoh[:b].numpy()
                dx = self.kdxh[:b].numpy()
                for i in np.nonzero(pending)[0]:
                    if info[i] == 0 and np.all(np.isfinite(dx[i])):
                        out[k + i] = dx[i].copy()
                        pending[i] = False
                    else:
                        delta[i] = delta_w0 if delta[i] == 0.0 else delta[i] * 8.0
                        if delta[i] > delta_w_max:
                            pending[i] = False  # stays None: the step failed
                if not pending.any():
                    break
            self.seconds["solver"] += time.perf_counter() - t1
        self.calls["newton"] += 1
        self.calls["hessian"] += 1
        return out

    def close(self):
        if self.kkt is not None:
            nnc.nnc_kkt_destroy(self.ctx.h, self.kkt)
            self.kkt = None
        if self.hnet is not self.net:
            self.hnet.destroy()
        self.net.destroy()
