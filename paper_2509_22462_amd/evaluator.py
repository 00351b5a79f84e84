"""GPU oracle evaluator for the host interior-point driver.

Wraps one (or two) library networks: ``nn``/``jac`` run on the network of
precision ``prec`` and ``hess`` on ``hess_prec`` (the Hessian only shapes the
Newton step, so it may run in BF16 while g and J -- which decide the KKT
residuals -- stay FP32).  Rows are evaluated in chunks of ``max_points`` with
device buffers allocated once.  Wall-clock per oracle is accumulated in the
four categories of the paper's Table 4 (function, Jacobian, Hessian; the
driver adds the solver time).
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
        self.seconds = {"function": 0.0, "jacobian": 0.0, "hessian": 0.0}
        self.calls = {"function": 0, "jacobian": 0, "hessian": 0}

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
            out[k:k + b] = self.g[:b].cpu().numpy()
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
            out[k:k + b] = self.J[:b].cpu().numpy()
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
            out[k:k + b] = self.H[:b].cpu().numpy()
        self.seconds["hessian"] += time.perf_counter() - t0
        self.calls["hessian"] += 1
        return out

    def close(self):
        if self.hnet is not self.net:
            self.hnet.destroy()
        self.net.destroy()
