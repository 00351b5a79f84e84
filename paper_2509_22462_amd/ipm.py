"""Host primal-dual interior-point driver for the reduced-space formulation.

The paper solves its problems with IPOPT (Section 2, Eq. 1-2): each
iteration needs the oracles g, grad g and the Hessian of the Lagrangian and
solves the Newton/KKT system of Eq. 2.  This module is a plain FP64 host
implementation of that loop in the reduced-space form of Section 3.2:

    variables  w = (x, y, s),   0 <= x <= 1,  s >= 0,  y free
    minimise   f(x) = ||x - x0||^2
    subject to c1 = y - NN(x) = 0                    (the gray-box constraint, Eq. 5)
               c2 = y_t - y_c - s - margin = 0        (NN_t - NN_c >= margin, slack s)

The NN oracles come from an *evaluator* (the GPU library, or any object with
the same three methods); the KKT algebra runs on the host in FP64.

Algorithm (after the IPOPT paper the paper cites, simplified):
  * barrier subproblems min f - mu sum log(bound slacks) s.t. c = 0, with the
    monotone Fiacco-McCormick mu update mu <- max(tol/10, min(k_mu mu, mu^th_mu))
    once the barrier error is below k_eps mu;
  * Newton step on the primal-dual equations (Eq. 2 with the barrier terms:
    alpha = Sigma = Z/X, beta = the barrier gradient).  Because y enters the
    constraints linearly with an identity and the slack row is scalar, (dy,
    dlambda, ds, dnu) are eliminated in closed form, leaving the n x n system
        (W_xx + Sigma_x + sigma_s a a^T + delta_w I) dx = rhs,   a = J^T (e_t - e_c),
    where W_xx = 2 I + sum_i (-lambda_i) Hess NN_i(x) is the Hessian of the
    Lagrangian from eval_hess_lag (lambda_nn = -lambda: the constraint is y - NN).
    The full KKT matrix has the correct inertia exactly when this reduced
    matrix is positive definite, so inertia correction raises delta_w until a
    Cholesky factorisation succeeds;
  * fraction-to-the-boundary rule tau = max(0.99, 1 - mu);
  * backtracking Armijo line search on the l1 merit phi_mu + rho ||c||_1
    (in place of IPOPT's filter), rho above the infinity norm of the
    multipliers after the step (so the Newton step descends), never decreased,
    with an allowance for the merit's evaluation noise (Options.merit_noise);
  * convergence: scaled max(dual infeasibility, ||c||_inf, complementarity)
    <= tol (1e-6, the paper's tolerance).

Every solve is written as a generator that *yields* oracle requests, so that
``solve_batch`` can run many problems in lock step and serve each round of
requests with one batched GPU call.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Any, Callable, Generator, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Options:
    tol: float = 1e-6
    max_iter: int = 200
    mu0: float = 0.1
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    kappa_eps: float = 10.0
    tau_min: float = 0.99
    bound_push: float = 1e-2
    armijo_eta: float = 1e-4
    max_backtracks: int = 30
    delta_w0: float = 1e-4
    delta_w_max: float = 1e40
    time_limit: float = 3600.0
    s_max: float = 100.0  # dual-infeasibility scaling cap (IPOPT s_max)
    device_kkt: bool = False  # Newton steps by the evaluator's device KKT solve (H stays on the GPU)
    # ask for J and H in one request (one shared forward pass) while the last
    # scaled KKT error exceeds merge_jac_hess * tol; closer to convergence J
    # comes alone first, so a converged iterate costs no Hessian (0: never)
    merge_jac_hess: float = 100.0
    # relative noise of the merit function as evaluated (network values from
    # FP32 or BF16 kernels): a trial point within merit_noise * max(1, |phi|)
    # of the Armijo bound is accepted, so that the line search does not fail
    # on rounding once the remaining decrease is below the evaluation noise
    merit_noise: float = 0.0
    verbose: bool = False


@dataclasses.dataclass
class Problem:
    """min ||x - x0||^2 s.t. NN(x)_t - NN(x)_c >= margin, 0 <= x <= 1."""
    x0: np.ndarray
    t: int
    c: int
    margin: float = 0.5

    @property
    def n(self):
        return int(self.x0.shape[0])


@dataclasses.dataclass
class L1Problem:
    """The paper's adversarial-image problem (Section 4.1, Eq. 7):
    min ||x - x_ref||_1 s.t. y = NN(x), y_t >= threshold (NN ends in SoftMax,
    so y_t is the probability of the target label).  As printed, x has no box.
    Solved with the slack split x = x_ref + p - q, p, q >= 0, objective
    sum(p) + sum(q)."""
    x_ref: np.ndarray
    t: int
    threshold: float = 0.6

    @property
    def n(self):
        return int(self.x_ref.shape[0])


@dataclasses.dataclass
class Start:
    """Optional starting point (a warm start): any field may be None."""
    x: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None
    lam: Optional[np.ndarray] = None
    nu: Optional[float] = None
    mu0: Optional[float] = None


@dataclasses.dataclass
class Result:
    status: str
    x: np.ndarray
    y: np.ndarray
    s: float
    zs: float
    lam: np.ndarray
    nu: float
    zL: np.ndarray
    zU: np.ndarray
    iters: int
    obj: float
    kkt_error: float
    primal_inf: float
    dual_inf: float
    evals: dict
    seconds: float = 0.0
    history: list = dataclasses.field(default_factory=list)


STATUSES = ("converged", "max_iter", "time_limit", "eval_error", "line_search_fail",
            "warmstart_rejected")

Request = tuple  # ("nn", x) | ("jac", x) | ("jach", x, lam_nn, keep) | ("hess", x, lam_nn)
#                  | ("newton", x, lam_nn, d, a, s, r, dw0, dwmax)


def _push_into_box(x, lo, hi, push):
    """Move x strictly inside [lo, hi] (IPOPT's bound_push, relative form)."""
    pl = push * np.maximum(1.0, np.abs(lo))
    pu = push * np.maximum(1.0, np.abs(hi))
    width = hi - lo
    pl = np.minimum(pl, 0.5 * width)
    pu = np.minimum(pu, 0.5 * width)
    return np.minimum(np.maximum(x, lo + pl), hi - pu)


def ipm_generator(prob: Problem, start: Optional[Start] = None,
                  opts: Optional[Options] = None) -> Generator[Request, Any, Result]:
    """The interior-point solve as a generator of oracle requests."""
    opts = opts or Options()
    start = start or Start()
    n = prob.n
    x0 = np.asarray(prob.x0, dtype=np.float64)
    lo = np.zeros(n)
    hi = np.ones(n)
    evals = {"nn": 0, "jac": 0, "hess": 0}
    t_start = time.perf_counter()

    # ------------------------------------------------------------ initial point
    x = x0.copy() if start.x is None else np.asarray(start.x, dtype=np.float64).copy()
    if not np.all(np.isfinite(x)):
        x = x0.copy()
    x = _push_into_box(x, lo, hi, opts.bound_push)
    nnx = yield ("nn", x)
    evals["nn"] += 1
    nnx = np.asarray(nnx, dtype=np.float64)
    m = nnx.shape[0]
    d = np.zeros(m)
    d[prob.t] += 1.0
    d[prob.c] -= 1.0
    y = nnx.copy() if start.y is None else np.asarray(start.y, dtype=np.float64).copy()
    h = float(d @ y) - prob.margin
    s = max(h, opts.bound_push)
    mu = opts.mu0 if start.mu0 is None else float(start.mu0)
    lam = np.zeros(m) if start.lam is None else np.asarray(start.lam, dtype=np.float64).copy()
    nu = 0.0 if start.nu is None else float(start.nu)
    zL = mu / (x - lo)
    zU = mu / (hi - x)
    zs = mu / s

    def objective(xx):
        r = xx - x0
        return float(r @ r)

    def constraints(xx_nn, yy, ss):
        return yy - xx_nn, float(d @ yy) - ss - prob.margin

    history = []
    it = 0
    status = "max_iter"
    J = None
    rho_pen = 0.0
    kkt = np.inf
    pinf = np.inf
    dinf = np.inf
    while True:
        # ------------------------------------------------------------ oracles
        Hpre = None
        merged = opts.merge_jac_hess > 0 and kkt > opts.merge_jac_hess * opts.tol
        if merged:
            J, Hpre = yield ("jach", x, -lam, opts.device_kkt)  # H kept by the evaluator when None
            evals["hess"] += 1
        else:
            J = yield ("jac", x)
        evals["jac"] += 1
        J = np.asarray(J, dtype=np.float64)
        c1, c2 = constraints(nnx, y, s)
        grad_f = 2.0 * (x - x0)
        # dual residuals of the Lagrangian f + lam^T c1 + nu c2 - zL (x-lo) - zU (hi-x) - zs s
        rx = grad_f - J.T @ lam - zL + zU
        ry = lam + nu * d
        rs = -nu - zs
        pinf = max(float(np.max(np.abs(c1))), abs(c2))
        dinf = max(float(np.max(np.abs(rx))), float(np.max(np.abs(ry))), abs(rs))
        comp = max(float(np.max(np.abs((x - lo) * zL))), float(np.max(np.abs((hi - x) * zU))),
                   abs(s * zs))
        zsum = float(np.sum(zL) + np.sum(zU) + zs)
        sd = max(opts.s_max, (float(np.sum(np.abs(lam))) + abs(nu) + zsum) / (m + 2 * n + 2)) / opts.s_max
        sc = max(opts.s_max, zsum / (2 * n + 1)) / opts.s_max
        kkt = max(dinf / sd, pinf, comp / sc)
        obj = objective(x)
        history.append((it, obj, pinf, dinf, mu))
        if opts.verbose:
            print(f"it {it:3d} obj {obj:.6e} inf_pr {pinf:.2e} inf_du {dinf:.2e} mu {mu:.1e}")
        if not (np.all(np.isfinite(J)) and np.isfinite(kkt)):
            status = "eval_error"
            break
        if kkt <= opts.tol:
            status = "converged"
            break
        if it >= opts.max_iter:
            status = "max_iter"
            break
        if time.perf_counter() - t_start > opts.time_limit:
            status = "time_limit"
            break
        # barrier subproblem error and mu update (monotone strategy)
        while True:
            comp_mu = max(float(np.max(np.abs((x - lo) * zL - mu))),
                          float(np.max(np.abs((hi - x) * zU - mu))), abs(s * zs - mu))
            err_mu = max(dinf / sd, pinf, comp_mu / sc)
            if err_mu > opts.kappa_eps * mu or mu <= opts.tol / 10.0:
                break
            mu = max(opts.tol / 10.0, min(opts.kappa_mu * mu, mu ** opts.theta_mu))
        tau = max(opts.tau_min, 1.0 - mu)

        # ------------------------------------------------------------ Newton step
        sig_x = zL / (x - lo) + zU / (hi - x)
        sig_s = zs / s
        # barrier gradients (beta of Eq. 2)
        gphi_x = grad_f - mu / (x - lo) + mu / (hi - x)
        gphi_s = -mu / s
        # right-hand sides: -[grad phi + A^T mult ; c]
        rx_mu = gphi_x - J.T @ lam
        ry_mu = lam + nu * d
        rs_mu = gphi_s - nu
        a = J.T @ d
        rhs = -rx_mu - J.T @ ry_mu - a * (sig_s * (c2 - d @ c1) + rs_mu)
        # Sign conventions of the eliminated rows (see module docstring):
        #   dy = J dx - c1, ds = d^T dy + c2, dnu = sig_s ds + rs_mu, dlam = -ry_mu - d dnu
        # Reduced system (W_xx + Sigma_x + sig_s a a^T + delta I) dx = rhs with
        # W_xx = Hess NN-term + 2 I; delta escalates until the factorisation
        # succeeds (inertia correction).
        if opts.device_kkt:
            dx = yield ("newton", x, -lam, sig_x + 2.0, a, sig_s, rhs, opts.delta_w0, opts.delta_w_max)
            if not merged:
                evals["hess"] += 1  # else H was made (and kept) by the "jach" request
            if dx is None or not np.all(np.isfinite(dx)):
                status = "eval_error"
                break
            dx = np.asarray(dx, dtype=np.float64)
        else:
            if Hpre is not None:
                Hnn = Hpre
            else:
                Hnn = yield ("hess", x, -lam)
                evals["hess"] += 1
            Hnn = np.asarray(Hnn, dtype=np.float64)
            if not np.all(np.isfinite(Hnn)):
                status = "eval_error"
                break
            W = Hnn + 2.0 * np.eye(n)
            M = W + np.diag(sig_x) + sig_s * np.outer(a, a)
            delta = 0.0
            Lc = None
            for _ in range(60):
                try:
                    Lc = np.linalg.cholesky(M + delta * np.eye(n))
                    break
                except np.linalg.LinAlgError:
                    delta = opts.delta_w0 if delta == 0.0 else delta * 8.0
                    if delta > opts.delta_w_max:
                        break
            if Lc is None:
                status = "eval_error"
                break
            dx = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rhs))
        dy = J @ dx - c1
        ds = float(d @ dy) + c2
        dnu = sig_s * ds + rs_mu
        dlam = -ry_mu - d * dnu
        dzL = mu / (x - lo) - zL - (zL / (x - lo)) * dx
        dzU = mu / (hi - x) - zU + (zU / (hi - x)) * dx
        dzs = mu / s - zs - (zs / s) * ds

        # ------------------------------------------------------------ step sizes
        def max_step(v, dv):
            neg = dv < 0
            if not np.any(neg):
                return 1.0
            return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))

        a_pr = min(max_step(x - lo, dx), max_step(hi - x, -dx), max_step(np.array([s]), np.array([ds])))
        a_du = min(max_step(zL, dzL), max_step(zU, dzU), max_step(np.array([zs]), np.array([dzs])))

        # ------------------------------------------------------------ line search
        # l1 penalty above the multipliers the step leads to (so the Newton step
        # is a descent direction of the merit function), never decreased
        rho_pen = max(rho_pen, max(float(np.max(np.abs(lam + dlam))) if m else 0.0, abs(nu + dnu)) + 1.0)
        rho = rho_pen

        def merit(xx, yy, ss, nn_xx):
            cc1, cc2 = constraints(nn_xx, yy, ss)
            with np.errstate(divide="ignore", invalid="ignore"):
                bar = -mu * (np.sum(np.log(xx - lo)) + np.sum(np.log(hi - xx)) + math.log(ss))
            return objective(xx) + bar + rho * (float(np.sum(np.abs(cc1))) + abs(cc2))

        phi0 = merit(x, y, s, nnx)
        dphi = float(gphi_x @ dx) + gphi_s * ds - rho * (float(np.sum(np.abs(c1))) + abs(c2))
        alpha = a_pr
        accepted = False
        for _ in range(opts.max_backtracks):
            xt = x + alpha * dx
            yt = y + alpha * dy
            st = s + alpha * ds
            nnt = yield ("nn", xt)
            evals["nn"] += 1
            nnt = np.asarray(nnt, dtype=np.float64)
            if np.all(np.isfinite(nnt)):
                phit = merit(xt, yt, st, nnt)
                bound = phi0 + opts.armijo_eta * alpha * min(dphi, 0.0) + opts.merit_noise * max(1.0, abs(phi0))
                if np.isfinite(phit) and phit <= bound:
                    accepted = True
                    break
            alpha *= 0.5
        if not accepted:
            status = "line_search_fail"
            break
        x, y, s, nnx = xt, yt, st, nnt
        lam = lam + alpha * dlam
        nu = nu + alpha * dnu
        zL = zL + a_du * dzL
        zU = zU + a_du * dzU
        zs = zs + a_du * dzs
        # keep bound multipliers within IPOPT's kappa_Sigma band of mu / slack
        ks = 1e10
        zL = np.clip(zL, mu / (ks * (x - lo)), ks * mu / (x - lo))
        zU = np.clip(zU, mu / (ks * (hi - x)), ks * mu / (hi - x))
        zs = min(max(zs, mu / (ks * s)), ks * mu / s)
        it += 1

    return Result(status=status, x=x, y=y, s=s, zs=zs, lam=lam, nu=nu, zL=zL, zU=zU, iters=it,
                  obj=objective(x), kkt_error=float(kkt), primal_inf=float(pinf),
                  dual_inf=float(dinf), evals=evals, seconds=time.perf_counter() - t_start,
                  history=history)


def ipm_l1_generator(prob: L1Problem, start: Optional[Start] = None,
                     opts: Optional[Options] = None) -> Generator[Request, Any, Result]:
    """Eq. 7 by the same primal-dual barrier method.

    Variables p, q >= 0 (x = x_ref + p - q), y free, slack s >= 0; constraints
    c1 = y - NN(x) = 0 and c2 = y_t - s - threshold = 0; objective 1^T (p + q).
    The Lagrangian's Hessian in (p, q) is [[W, -W], [-W, W]] with
    W = sum_i (-lambda_i) Hess NN_i(x) (the objective is linear).  After the
    closed-form elimination of y, s and the multipliers (as in
    ``ipm_generator``, with the margin row d = e_t), the p and q rows read
        K dx + Sigma_p dp = R_p,   -K dx + Sigma_q dq = R_q,   dx = dp - dq,
    K = W + sigma_s a a^T; eliminating dp and dq leaves the same reduced system
        (W + diag(1 / (1/Sigma_p + 1/Sigma_q)) + sigma_s a a^T) dx = rhs,
    and then dp = (R_p + R_q + Sigma_q dx) / (Sigma_p + Sigma_q), dq = dp - dx
    (the K dx terms cancel in the sum of the two rows)."""
    opts = opts or Options()
    start = start or Start()
    n = prob.n
    xr = np.asarray(prob.x_ref, dtype=np.float64)
    evals = {"nn": 0, "jac": 0, "hess": 0}
    t_start = time.perf_counter()
    push = opts.bound_push
    if start.x is not None and np.all(np.isfinite(start.x)):
        dxs = np.asarray(start.x, dtype=np.float64) - xr
        p = np.maximum(dxs, 0.0) + push
        q = np.maximum(-dxs, 0.0) + push
    else:
        p = np.full(n, push)
        q = np.full(n, push)
    x = xr + p - q
    nnx = yield ("nn", x)
    evals["nn"] += 1
    nnx = np.asarray(nnx, dtype=np.float64)
    m = nnx.shape[0]
    d = np.zeros(m)
    d[prob.t] = 1.0
    y = nnx.copy() if start.y is None else np.asarray(start.y, dtype=np.float64).copy()
    s = max(float(d @ y) - prob.threshold, push)
    mu = opts.mu0 if start.mu0 is None else float(start.mu0)
    lam = np.zeros(m) if start.lam is None else np.asarray(start.lam, dtype=np.float64).copy()
    nu = 0.0 if start.nu is None else float(start.nu)
    zp = mu / p
    zq = mu / q
    zs = mu / s

    def constraints(xx_nn, yy, ss):
        return yy - xx_nn, float(d @ yy) - ss - prob.threshold

    history = []
    it = 0
    status = "max_iter"
    rho_pen = 0.0
    kkt = pinf = dinf = np.inf
    while True:
        Hpre = None
        merged = opts.merge_jac_hess > 0 and kkt > opts.merge_jac_hess * opts.tol
        if merged:
            J, Hpre = yield ("jach", x, -lam, opts.device_kkt)  # H kept by the evaluator when None
            evals["hess"] += 1
        else:
            J = yield ("jac", x)
        evals["jac"] += 1
        J = np.asarray(J, dtype=np.float64)
        c1, c2 = constraints(nnx, y, s)
        jl = J.T @ lam
        rp = 1.0 - jl - zp
        rq = 1.0 + jl - zq
        ry = lam + nu * d
        rs = -nu - zs
        pinf = max(float(np.max(np.abs(c1))), abs(c2))
        dinf = max(float(np.max(np.abs(rp))), float(np.max(np.abs(rq))), float(np.max(np.abs(ry))), abs(rs))
        comp = max(float(np.max(np.abs(p * zp))), float(np.max(np.abs(q * zq))), abs(s * zs))
        zsum = float(np.sum(zp) + np.sum(zq) + zs)
        sd = max(opts.s_max, (float(np.sum(np.abs(lam))) + abs(nu) + zsum) / (m + 2 * n + 2)) / opts.s_max
        sc = max(opts.s_max, zsum / (2 * n + 1)) / opts.s_max
        kkt = max(dinf / sd, pinf, comp / sc)
        obj = float(np.sum(np.abs(x - xr)))
        history.append((it, obj, pinf, dinf, mu))
        if opts.verbose:
            print(f"it {it:3d} obj {obj:.6e} inf_pr {pinf:.2e} inf_du {dinf:.2e} mu {mu:.1e}")
        if not (np.all(np.isfinite(J)) and np.isfinite(kkt)):
            status = "eval_error"
            break
        if kkt <= opts.tol:
            status = "converged"
            break
        if it >= opts.max_iter:
            break
        if time.perf_counter() - t_start > opts.time_limit:
            status = "time_limit"
            break
        while True:
            comp_mu = max(float(np.max(np.abs(p * zp - mu))), float(np.max(np.abs(q * zq - mu))),
                          abs(s * zs - mu))
            if max(dinf / sd, pinf, comp_mu / sc) > opts.kappa_eps * mu or mu <= opts.tol / 10.0:
                break
            mu = max(opts.tol / 10.0, min(opts.kappa_mu * mu, mu ** opts.theta_mu))
        tau = max(opts.tau_min, 1.0 - mu)

        # ------------------------------------------------------------ Newton step
        sig_p = zp / p
        sig_q = zq / q
        sig_s = zs / s
        gp = 1.0 - mu / p  # barrier gradients in p, q, s
        gq = 1.0 - mu / q
        gs = -mu / s
        ry_mu = lam + nu * d
        rs_mu = gs - nu
        a = J.T @ d
        k0 = sig_s * (c2 - d @ c1) + rs_mu
        rho = J.T @ ry_mu + a * k0
        Rp = -(gp - jl) - rho
        Rq = -(gq + jl) + rho
        dinv = 1.0 / sig_p + 1.0 / sig_q
        dvec = 1.0 / dinv
        rhs = dvec * (Rp / sig_p - Rq / sig_q)
        if opts.device_kkt:
            dx = yield ("newton", x, -lam, dvec, a, sig_s, rhs, opts.delta_w0, opts.delta_w_max)
            if not merged:
                evals["hess"] += 1  # else H was made (and kept) by the "jach" request
            if dx is None or not np.all(np.isfinite(dx)):
                status = "eval_error"
                break
            dx = np.asarray(dx, dtype=np.float64)
        else:
            if Hpre is not None:
                Hnn = Hpre
            else:
                Hnn = yield ("hess", x, -lam)
                evals["hess"] += 1
            Hnn = np.asarray(Hnn, dtype=np.float64)
            if not np.all(np.isfinite(Hnn)):
                status = "eval_error"
                break
            M = Hnn + np.diag(dvec) + sig_s * np.outer(a, a)
            delta = 0.0
            Lc = None
            for _ in range(60):
                try:
                    Lc = np.linalg.cholesky(M + delta * np.eye(n))
                    break
                except np.linalg.LinAlgError:
                    delta = opts.delta_w0 if delta == 0.0 else delta * 8.0
                    if delta > opts.delta_w_max:
                        break
            if Lc is None:
                status = "eval_error"
                break
            dx = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rhs))
        dp = (Rp + Rq + sig_q * dx) / (sig_p + sig_q)
        dq = dp - dx
        dy = J @ dx - c1
        ds = float(d @ dy) + c2
        dnu = sig_s * ds + rs_mu
        dlam = -ry_mu - d * dnu
        dzp = mu / p - zp - sig_p * dp
        dzq = mu / q - zq - sig_q * dq
        dzs = mu / s - zs - sig_s * ds

        def max_step(v, dv):
            neg = dv < 0
            if not np.any(neg):
                return 1.0
            return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))

        a_pr = min(max_step(p, dp), max_step(q, dq), max_step(np.array([s]), np.array([ds])))
        a_du = min(max_step(zp, dzp), max_step(zq, dzq), max_step(np.array([zs]), np.array([dzs])))
        rho_pen = max(rho_pen, max(float(np.max(np.abs(lam + dlam))) if m else 0.0, abs(nu + dnu)) + 1.0)
        rho_m = rho_pen

        def merit(pp, qq, yy, ss, nn_xx):
            cc1, cc2 = constraints(nn_xx, yy, ss)
            with np.errstate(divide="ignore", invalid="ignore"):
                bar = -mu * (np.sum(np.log(pp)) + np.sum(np.log(qq)) + math.log(ss))
            return float(np.sum(pp) + np.sum(qq)) + bar + rho_m * (float(np.sum(np.abs(cc1))) + abs(cc2))

        phi0 = merit(p, q, y, s, nnx)
        dphi = float(gp @ dp) + float(gq @ dq) + gs * ds - rho_m * (float(np.sum(np.abs(c1))) + abs(c2))
        alpha = a_pr
        accepted = False
        for _ in range(opts.max_backtracks):
            pt, qt = p + alpha * dp, q + alpha * dq
            yt = y + alpha * dy
            st = s + alpha * ds
            xt = xr + pt - qt
            nnt = yield ("nn", xt)
            evals["nn"] += 1
            nnt = np.asarray(nnt, dtype=np.float64)
            if np.all(np.isfinite(nnt)):
                phit = merit(pt, qt, yt, st, nnt)
                bound = phi0 + opts.armijo_eta * alpha * min(dphi, 0.0) + opts.merit_noise * max(1.0, abs(phi0))
                if np.isfinite(phit) and phit <= bound:
                    accepted = True
                    break
            alpha *= 0.5
        if not accepted:
            status = "line_search_fail"
            break
        p, q, y, s, nnx, x = pt, qt, yt, st, nnt, xt
        lam = lam + alpha * dlam
        nu = nu + alpha * dnu
        zp = zp + a_du * dzp
        zq = zq + a_du * dzq
        zs = zs + a_du * dzs
        ks = 1e10
        zp = np.clip(zp, mu / (ks * p), ks * mu / p)
        zq = np.clip(zq, mu / (ks * q), ks * mu / q)
        zs = min(max(zs, mu / (ks * s)), ks * mu / s)
        it += 1

    # report x-space multipliers of the (absent) box as zeros: zL/zU hold the
    # split variables' bound multipliers p and q for inspection
    return Result(status=status, x=x, y=y, s=s, zs=zs, lam=lam, nu=nu, zL=zp, zU=zq, iters=it,
                  obj=float(np.sum(np.abs(x - xr))), kkt_error=float(kkt), primal_inf=float(pinf),
                  dual_inf=float(dinf), evals=evals, seconds=time.perf_counter() - t_start,
                  history=history)


def l1_kkt_residual(prob: L1Problem, res: Result, nn_fn: Callable, jac_fn: Callable):
    """Unscaled first-order optimality residuals of an Eq. 7 solve in the
    split variables (res.zL, res.zU hold the multipliers of p >= 0, q >= 0)."""
    x, y, s = res.x, res.y, res.s
    xr = np.asarray(prob.x_ref, dtype=np.float64)
    p = np.maximum(x - xr, 0.0)
    q = np.maximum(xr - x, 0.0)
    m = y.shape[0]
    d = np.zeros(m)
    d[prob.t] = 1.0
    J = jac_fn(x)
    c1 = y - nn_fn(x)
    c2 = float(d @ y) - s - prob.threshold
    jl = J.T @ res.lam
    return dict(primal=max(float(np.max(np.abs(c1))), abs(c2)),
                dual=max(float(np.max(np.abs(1.0 - jl - res.zL))), float(np.max(np.abs(1.0 + jl - res.zU))),
                         float(np.max(np.abs(res.lam + res.nu * d))), abs(res.nu + res.zs)),
                sign=min(float(np.min(res.zL)), float(np.min(res.zU)), res.zs),
                kink=float(np.max(np.minimum(p, q))))


class Evaluator:
    """Interface of the NN oracles used by the driver (batched over rows)."""

    def nn(self, X: np.ndarray) -> np.ndarray:  # (B, n) -> (B, m)
        raise NotImplementedError

    def jac(self, X: np.ndarray) -> np.ndarray:  # (B, n) -> (B, m, n)
        raise NotImplementedError

    def hess(self, X: np.ndarray, Lam: np.ndarray) -> np.ndarray:  # -> (B, n, n)
        """sum_i Lam[b, i] Hess NN_i(X[b])."""
        raise NotImplementedError

    def jac_hess(self, X: np.ndarray, Lam: np.ndarray, keep: bool = False):
        """Per row (J, H): both oracles at the same points, from one evaluation
        where the evaluator can share the forward pass.  keep: the evaluator
        may hold H for a following newton() at the same (X[b], Lam[b]) and
        return None in its place."""
        return list(zip(self.jac(X), self.hess(X, Lam)))

    def newton(self, X, Lam, D, A, S, R, delta_w0, delta_w_max):
        """Optional (Options.device_kkt): for each row b the solution dx of
        (Hess_b + diag(D[b]) + S[b] A[b] A[b]^T + delta I) dx = R[b], with
        Hess_b = sum_i Lam[b, i] Hess NN_i(X[b]) and delta raised from 0 to
        delta_w0, then by 8x, until the matrix factorises (None past
        delta_w_max)."""
        raise NotImplementedError


def _serve(ev: Evaluator, kind: str, reqs: List[Request]):
    X = np.stack([r[1] for r in reqs])
    if kind == "nn":
        return list(ev.nn(X))
    if kind == "jac":
        return list(ev.jac(X))
    Lam = np.stack([r[2] for r in reqs])
    if kind == "jach":
        return list(ev.jac_hess(X, Lam, bool(reqs[0][3])))
    if kind == "newton":
        D, A, R = (np.stack([r[i] for r in reqs]) for i in (3, 4, 6))
        S = np.array([r[5] for r in reqs])
        return list(ev.newton(X, Lam, D, A, S, R, reqs[0][7], reqs[0][8]))
    return list(ev.hess(X, Lam))


def solve(prob: Problem, ev: Evaluator, start: Optional[Start] = None,
          opts: Optional[Options] = None) -> Result:
    return solve_batch([prob], ev, [start], opts)[0]


def solve_batch(probs: Sequence[Problem], ev: Evaluator, starts=None,
                opts: Optional[Options] = None, max_batch: Optional[int] = None) -> List[Result]:
    """Run the solves in lock step; each round's requests of one kind are
    served by one batched evaluator call (at most ``max_batch`` rows)."""
    starts = list(starts) if starts is not None else [None] * len(probs)
    t0 = time.perf_counter()
    gens = [(ipm_l1_generator if isinstance(p, L1Problem) else ipm_generator)(p, s, opts)
            for p, s in zip(probs, starts)]
    results: List[Optional[Result]] = [None] * len(gens)
    pending = {}
    for i, g in enumerate(gens):
        pending[i] = next(g)
    while pending:
        by_kind = {}
        for i, r in pending.items():
            by_kind.setdefault(r[0], []).append(i)
        answers = {}
        for kind, idx in by_kind.items():
            # evaluators that chunk by themselves get the whole round (so the
            # Hessians a "jach" round keeps cover every problem of it)
            step = len(idx) if getattr(ev, "chunks_internally", False) else (max_batch or len(idx))
            for k in range(0, len(idx), step):
                chunk = idx[k:k + step]
                out = _serve(ev, kind, [pending[i] for i in chunk])
                for i, o in zip(chunk, out):
                    answers[i] = o
        nxt = {}
        for i, ans in answers.items():
            try:
                nxt[i] = gens[i].send(ans)
            except StopIteration as e:
                results[i] = e.value
        pending = nxt
    for r in results:
        r.seconds = max(r.seconds, 0.0)
    return results


def margin_ascent(probs: Sequence[Problem], X0: np.ndarray, ev: Evaluator, max_steps: int = 200,
                  rtol: float = 1e-4, atol: float = 1e-7):
    """Projected-gradient ascent of the margin NN_t(x) - NN_c(x) over the
    box [0, 1]^n from each row of X0, all rows in lock step (batched oracle
    calls); backtracking (Armijo, step doubled after each accepted step)
    along the projected path.  A row stops when its margin reaches the
    problem's, or when its projected gradient falls below
    max(atol, rtol * |gradient at the start|) (a stationary point of the
    margin over the box).  Returns (best margin, reached, stationary) arrays."""
    B = len(probs)
    X = np.clip(np.asarray(X0, dtype=np.float64), 0.0, 1.0)
    NN = np.asarray(ev.nn(X), dtype=np.float64)
    m = NN.shape[1]
    D = np.zeros((B, m))
    for b, pr in enumerate(probs):
        D[b, pr.t] += 1.0
        D[b, pr.c] -= 1.0
    target = np.array([pr.margin for pr in probs])
    marg = np.sum(D * NN, axis=1)
    reached = marg >= target
    stationary = np.zeros(B, dtype=bool)
    step = np.ones(B)
    g0 = np.full(B, np.nan)
    for _ in range(max_steps):
        idx = np.nonzero(~reached & ~stationary)[0]
        if idx.size == 0:
            break
        J = np.asarray(ev.jac(X[idx]), dtype=np.float64)
        G = np.einsum("kmn,km->kn", J, D[idx])
        Xi = X[idx]
        blocked = ((Xi <= 0.0) & (G < 0.0)) | ((Xi >= 1.0) & (G > 0.0))
        pgn = np.max(np.abs(np.where(blocked, 0.0, G)), axis=1)
        first = np.isnan(g0[idx])
        g0[idx[first]] = np.max(np.abs(G[first]), axis=1)
        st = pgn <= np.maximum(atol, rtol * g0[idx])
        stationary[idx[st]] = True
        live, G = idx[~st], G[~st]
        if live.size == 0:
            continue
        t = step[live] * 2.0
        done = np.zeros(live.size, dtype=bool)
        for _ in range(40):
            todo = np.nonzero(~done)[0]
            Xt = np.clip(X[live[todo]] + t[todo, None] * G[todo], 0.0, 1.0)
            Mt = np.sum(D[live[todo]] * np.asarray(ev.nn(Xt), dtype=np.float64), axis=1)
            gain = np.sum(G[todo] * (Xt - X[live[todo]]), axis=1)
            ok = (Mt >= marg[live[todo]] + 1e-4 * gain) & (gain > 0.0)
            acc = todo[ok]
            X[live[acc]] = Xt[ok]
            marg[live[acc]] = Mt[ok]
            done[acc] = True
            t[todo[~ok]] *= 0.5
            if done.all():
                break
        step[live] = t
        # a row whose step underflowed without progress is at a stationary point
        stationary[live[~done]] = True
        reached = marg >= target
    return marg, reached, stationary


def classify_failures(probs: Sequence[Problem], results: Sequence[Result], ev: Evaluator, **kw):
    """Label each solve: "converged"; "reachable" (the margin constraint can
    be met from the returned point: the driver failed on a problem that is
    feasible there); "locally_infeasible" (projected-gradient ascent of the
    margin from the returned point stops at a stationary point of the margin
    over the box below the required margin: IPOPT's point of local
    infeasibility); "undecided" (neither within the ascent's steps)."""
    labels = ["converged" if r.status == "converged" else None for r in results]
    bad = [i for i, lab in enumerate(labels) if lab is None]
    if bad:
        marg, reached, stationary = margin_ascent([probs[i] for i in bad], np.stack([results[i].x for i in bad]),
                                                  ev, **kw)
        for k, i in enumerate(bad):
            labels[i] = "reachable" if reached[k] else ("locally_infeasible" if stationary[k] else "undecided")
    return labels


def kkt_residual(prob: Problem, res: Result, nn_fn: Callable, jac_fn: Callable):
    """Unscaled first-order optimality residuals of a returned point."""
    x, y, s = res.x, res.y, res.s
    m = y.shape[0]
    d = np.zeros(m)
    d[prob.t] += 1.0
    d[prob.c] -= 1.0
    J = jac_fn(x)
    c1 = y - nn_fn(x)
    c2 = float(d @ y) - s - prob.margin
    rx = 2.0 * (x - prob.x0) - J.T @ res.lam - res.zL + res.zU
    ry = res.lam + res.nu * d
    rs = -res.nu - res.zs
    return dict(primal=max(float(np.max(np.abs(c1))), abs(c2)),
                dual_x=float(np.max(np.abs(rx))), dual_y=float(np.max(np.abs(ry))),
                dual_s=abs(rs),
                comp=float(max(np.max(x * res.zL), np.max((1 - x) * res.zU), s * res.zs)))
