"""GPU oracle evaluator for the host interior-point driver.

Wraps one (or two) library networks: ``nn``/``jac`` run on the network of
precision ``prec`` and ``hess`` on ``hess_prec`` (the Hessian only shapes the
Newton step, so it may run in BF16 while g and J -- which decide the KKT
residuals -- stay FP32).  Rows are evaluated in chunks of ``max_points`` with
device buffers (and pinned host staging buffers for the copies back)
allocated once.  ``jac_hess`` serves J and H from one nnc_eval (one shared
forward pass), optionally keeping H in HBM; ``newton`` solves the reduced
Newton system there (nnc_kkt_solve; only dx returns), against the kept H
when the points match, else after computing H.  Wall-clock
per oracle is accumulated in the categories of the paper's Table 4
(function, Jacobian, Hessian, and the device solver when it is used).
"""
from __future__ import annotations

import time

import numpy as np

from . import ipm, nnc


class GpuEvaluator(ipm.Evaluator):
    # batches are split into max_points chunks here, so the driver hands over
    # whole rounds (the Hessians kept by one jac_hess call then cover them all)
    chunks_internally = True

    def __init__(self, ctx: "nnc.Context", dims, acts, Ws, bs, prec="fp32", hess_prec=None,
                 max_points=64):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.dims = list(dims)
        self.n, self.m = dims[0], dims[-1]
        self.B = max_points
        self.net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=max_points)
        # relative rounding noise of the network values this evaluator returns
        # (FP64 output layer, hidden layers in `prec`): the driver's
        # Options.merit_noise for solves on it
        self.merit_noise = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}[prec]
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
        # Hessians kept on the device by jac_hess(keep=True): row slot k of
        # self.hstore holds H at the (x, lambda) whose bytes key self.hslot
        self.hstore = None
        self.hslot = {}
        self.seconds = {"function": 0.0, "jacobian": 0.0, "hessian": 0.0, "jacobian+hessian": 0.0, "solver": 0.0}
        self.calls = {"function": 0, "jacobian": 0, "hessian": 0, "jacobian+hessian": 0, "newton": 0}

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

    @staticmethod
    def _key(x, lam):
        return np.ascontiguousarray(x, dtype=np.float64).tobytes() + np.ascontiguousarray(lam, dtype=np.float64).tobytes()

    def jac_hess(self, X, Lam, keep=False):
        """J and H at the same points from one nnc_eval per chunk (one shared
        forward pass).  keep: H stays in a device store, one slot per row,
        for newton() at the same (x, lambda); None is returned in its place."""
        torch = self.torch
        if self.hnet is not self.net:  # H on a network of another precision: two calls
            J = self.jac(X)
            if not keep:
                return list(zip(J, self.hess(X, Lam)))
            self._hess_to_store(X, Lam)
            return [(j, None) for j in J]
        t0 = time.perf_counter()
        X = np.atleast_2d(X)
        Lam = np.atleast_2d(Lam)
        Bt = X.shape[0]
        if keep:
            self._store_capacity(Bt)
        Jout = np.empty((Bt, self.m, self.n))
        Hout = None if keep else np.empty((Bt, self.n, self.n))
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            self._load(self.x, Xc)
            self._load(self.lam, Lam[k:k + b])
            Hd = self.hstore[k:k + b] if keep else self.H
            nnc._chk(nnc.nnc_eval(self.ctx.h, self.net.h, b, self.x.data_ptr(), None, 0.0, self.lam.data_ptr(),
                                  None, self.J.data_ptr(), Hd.data_ptr()), self.ctx.h, "nnc_eval")
            self.Jh[:b].copy_(self.J[:b])
            Jout[k:k + b] = self.Jh[:b].numpy()
            if not keep:
                if self.Hh is None:
                    self.Hh = torch.empty(self.B, self.n, self.n, dtype=torch.float64, pin_memory=True)
                self.Hh[:b].copy_(self.H[:b])
                Hout[k:k + b] = self.Hh[:b].numpy()
        if keep:
            self.hslot = {self._key(X[i], Lam[i]): i for i in range(Bt)}
        self.seconds["jacobian+hessian"] += time.perf_counter() - t0
        self.calls["jacobian+hessian"] += 1
        return [(Jout[i], None if keep else Hout[i]) for i in range(Bt)]

    def _store_capacity(self, Bt):
        if self.hstore is None or self.hstore.shape[0] < Bt:
            self.hstore = None
            self.hstore = self.torch.empty(Bt, self.n, self.n, dtype=self.torch.float64, device=self.ctx.device)
        self.hslot = {}

    def _hess_to_store(self, X, Lam):
        t0 = time.perf_counter()
        X = np.atleast_2d(X)
        Lam = np.atleast_2d(Lam)
        self._store_capacity(X.shape[0])
        for k, Xc in self._chunks(X):
            b = Xc.shape[0]
            self._load(self.x, Xc)
            self._load(self.lam, Lam[k:k + b])
            nnc._chk(nnc.nnc_eval_hess_lag(self.ctx.h, self.hnet.h, b, self.x.data_ptr(), 0.0,
                                           self.lam.data_ptr(), self.hstore[k:k + b].data_ptr()), self.ctx.h,
                     "nnc_eval_hess_lag")
        self.hslot = {self._key(X[i], Lam[i]): i for i in range(X.shape[0])}
        self.seconds["hessian"] += time.perf_counter() - t0
        self.calls["hessian"] += 1

    def newton(self, X, Lam, D, A, S, R, delta_w0, delta_w_max):
        """Newton steps with the Hessian kept on the device: H in HBM (kept
        by jac_hess at the same (x, lambda), else from nnc_eval_hess_lag now),
        then (H + diag(D) + S a a^T + delta I) dx = R by nnc_kkt_solve, delta
        raised from 0 to delta_w0 and then by 8x for the systems whose
        factorisation fails (the host driver's inertia correction); only dx
        (and the failure flags) come back."""
        X = np.atleast_2d(X)
        Lam = np.atleast_2d(Lam)
        Bt = X.shape[0]
        self._kkt_buffers()
        out = [None] * Bt
        slots = [self.hslot.get(self._key(X[i], Lam[i])) for i in range(Bt)] if self.hslot else [None] * Bt
        kept = [i for i in range(Bt) if slots[i] is not None]
        if kept:
            # solve against the kept Hessians in place: rows in slot order,
            # runs of consecutive slots (at most max_points rows) per call
            order = sorted(kept, key=lambda i: slots[i])
            rowbytes = self.n * self.n * 8
            r = 0
            while r < len(order):
                e = r + 1
                while e < len(order) and e - r < self.B and slots[order[e]] == slots[order[e - 1]] + 1:
                    e += 1
                rows = order[r:e]
                t1 = time.perf_counter()
                self._solve_rows(self.hstore.data_ptr() + slots[rows[0]] * rowbytes, rows, D, A, S, R,
                                 delta_w0, delta_w_max, out)
                self.seconds["solver"] += time.perf_counter() - t1
                r = e
        rest = [i for i in range(Bt) if slots[i] is None]
        for k in range(0, len(rest), self.B):
            rows = rest[k:k + self.B]
            b = len(rows)
            t0 = time.perf_counter()
            self._load(self.x, X[rows])
            self._load(self.lam, Lam[rows])
            nnc._chk(nnc.nnc_eval_hess_lag(self.ctx.h, self.hnet.h, b, self.x.data_ptr(), 0.0,
                                           self.lam.data_ptr(), self.H.data_ptr()), self.ctx.h,
                     "nnc_eval_hess_lag")
            self.torch.cuda.synchronize()
            t1 = time.perf_counter()
            self.seconds["hessian"] += t1 - t0
            self._solve_rows(self.H.data_ptr(), rows, D, A, S, R, delta_w0, delta_w_max, out)
            self.seconds["solver"] += time.perf_counter() - t1
        self.calls["newton"] += 1
        if rest:
            self.calls["hessian"] += 1
        return out

    def _kkt_buffers(self):
        if self.kkt is not None:
            return
        torch = self.torch
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

    def _solve_rows(self, Hptr, rows, D, A, S, R, delta_w0, delta_w_max, out):
        """The Newton systems of rows `rows` (at most max_points) with their
        Hessians contiguous at device address Hptr; dx into out[row]."""
        torch = self.torch
        b = len(rows)
        self._load(self.kd, D[rows])
        self._load(self.ka, A[rows])
        self.ks[:b].copy_(torch.from_numpy(np.ascontiguousarray(np.asarray(S)[rows], dtype=np.float64)))
        self._load(self.kr, R[rows])
        delta = np.zeros(b)
        pending = np.ones(b, dtype=bool)
        for _ in range(60):
            self.kdelta[:b].copy_(torch.from_numpy(delta))
            nnc._chk(nnc.nnc_kkt_solve(self.ctx.h, self.kkt, b, Hptr, self.kd.data_ptr(), self.ka.data_ptr(),
                                       self.ks.data_ptr(), self.kdelta.data_ptr(), self.kr.data_ptr(),
                                       self.kdx.data_ptr(), self.kinfo.data_ptr()), self.ctx.h, "nnc_kkt_solve")
            self.kinfoh[:b].copy_(self.kinfo[:b])
            self.kdxh[:b].copy_(self.kdx[:b])
            info = self.kinfoh[:b].numpy()
            dx = self.kdxh[:b].numpy()
            for i in np.nonzero(pending)[0]:
                if info[i] == 0 and np.all(np.isfinite(dx[i])):
                    out[rows[i]] = dx[i].copy()
                    pending[i] = False
                else:
                    delta[i] = delta_w0 if delta[i] == 0.0 else delta[i] * 8.0
                    if delta[i] > delta_w_max:
                        pending[i] = False  # stays None: the step failed
            if not pending.any():
                break

    def close(self):
        if self.kkt is not None:
            nnc.nnc_kkt_destroy(self.ctx.h, self.kkt)
            self.kkt = None
        if self.hnet is not self.net:
            self.hnet.destroy()
        self.net.destroy()
