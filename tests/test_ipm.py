"""Host interior-point driver on the oracle evaluator (CPU only).

Pins: the convex special case against its closed form (bisection on the
single multiplier), first-order optimality of the returned point on a
nonconvex tanh network, lock-step batching equal to single solves, and the
failure statuses forced from the host.
"""
import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, ipm


class OracleEval(ipm.Evaluator):
    def __init__(self, Ws, bs, acts):
        self.Ws, self.bs, self.acts = Ws, bs, acts
        self.calls = {"nn": 0, "jac": 0, "hess": 0}

    def nn(self, X):
        self.calls["nn"] += 1
        return O.residual(self.Ws, self.bs, self.acts, X)

    def jac(self, X):
        self.calls["jac"] += 1
        return O.jacobians(self.Ws, self.bs, self.acts, X)

    def hess(self, X, Lam):
        self.calls["hess"] += 1
        return O.hess_lag(self.Ws, self.bs, self.acts, X, Lam)


def bisect_projection(x0, a, beta):
    """argmin ||x - x0||^2 s.t. a^T x >= beta, 0 <= x <= 1 (closed form in nu)."""
    def xs(nu):
        return np.clip(x0 + 0.5 * nu * a, 0.0, 1.0)

    if a @ xs(0.0) >= beta:
        return xs(0.0)
    lo, hi = 0.0, 1.0
    while a @ xs(hi) < beta:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if a @ xs(mid) < beta:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    return xs(hi)


def test_convex_special_case_matches_closed_form():
    n, m = 30, 4
    rng = np.random.default_rng(40)
    W = rng.standard_normal((m, n)) / np.sqrt(n)
    b = 0.1 * rng.standard_normal(m)
    ev = OracleEval([W], [b], ["identity"])
    x0 = rng.random(n)
    logits = W @ x0 + b
    c = int(np.argmax(logits))
    t = (c + 1) % m
    prob = ipm.Problem(x0=x0, t=t, c=c, margin=0.5)
    res = ipm.solve(prob, ev, opts=ipm.Options(tol=1e-10))
    assert res.status == "converged", res.status
    xstar = bisect_projection(x0, W[t] - W[c], 0.5 - (b[t] - b[c]))
    assert np.max(np.abs(res.x - xstar)) < 1e-6
    assert abs(res.obj - np.sum((xstar - x0) ** 2)) < 1e-8
    # at the paper's tolerance the point is already close
    res6 = ipm.solve(prob, ev)
    assert res6.status == "converged" and np.max(np.abs(res6.x - xstar)) < 1e-4


@pytest.mark.parametrize("seed", [41, 42])
def test_nonconvex_tanh_network_reaches_kkt_point(seed):
    dims = (24, 32, 16, 5)
    acts = ["tanh", "tanh", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=seed)
    ev = OracleEval(Ws, bs, acts)
    x0 = np.random.default_rng(seed).random(24)
    c = int(np.argmax(O.nn(Ws, bs, acts, x0)))
    t = (c + 2) % 5
    prob = ipm.Problem(x0=x0, t=t, c=c, margin=0.5)
    res = ipm.solve(prob, ev)
    assert res.status == "converged", (res.status, res.iters)
    r = ipm.kkt_residual(prob, res, lambda x: O.nn(Ws, bs, acts, x),
                         lambda x: O.jacobian(Ws, bs, acts, x))
    assert r["primal"] < 1e-6
    assert r["dual_y"] < 1e-6
    assert r["dual_x"] < 1e-4
    assert r["comp"] < 1e-5
    # feasibility of y = NN(x) and of the margin through the oracle
    y = O.nn(Ws, bs, acts, res.x)
    assert y[t] - y[c] >= 0.5 - 1e-6
    assert np.all(res.x >= 0) and np.all(res.x <= 1)


def test_lockstep_batch_equals_single_solves():
    dims = (16, 20, 4)
    acts = ["sigmoid", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=43)
    ev = OracleEval(Ws, bs, acts)
    rng = np.random.default_rng(44)
    probs = []
    for _ in range(3):
        x0 = rng.random(16)
        c = int(np.argmax(O.nn(Ws, bs, acts, x0)))
        probs.append(ipm.Problem(x0=x0, t=(c + 1) % 4, c=c, margin=0.2))
    batch = ipm.solve_batch(probs, ev)
    for p, rb in zip(probs, batch):
        rs = ipm.solve(p, ev)
        assert rs.status == rb.status
        assert rs.iters == rb.iters
        np.testing.assert_allclose(rs.x, rb.x, rtol=0, atol=1e-12)


def test_failure_statuses_forced_from_host():
    dims = (8, 6, 3)
    acts = ["tanh", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=45)
    x0 = np.full(8, 0.5)
    c = int(np.argmax(O.nn(Ws, bs, acts, x0)))
    prob = ipm.Problem(x0=x0, t=(c + 1) % 3, c=c)

    class NaNHess(OracleEval):
        def hess(self, X, Lam):
            return np.full((X.shape[0], 8, 8), np.nan)

    assert ipm.solve(prob, NaNHess(Ws, bs, acts)).status == "eval_error"
    res = ipm.solve(prob, OracleEval(Ws, bs, acts), opts=ipm.Options(max_iter=1))
    assert res.status == "max_iter" and res.iters == 1
    res = ipm.solve(prob, OracleEval(Ws, bs, acts), opts=ipm.Options(time_limit=0.0))
    assert res.status == "time_limit"
    # a NaN starting guess is replaced by x0 instead of poisoning the solve
    res = ipm.solve(prob, OracleEval(Ws, bs, acts), start=ipm.Start(x=np.full(8, np.nan)))
    assert res.status == "converged"


# ---------------------------------------------------------------- Eq. 7: l1 objective, SoftMax threshold
def test_l1_linear_special_case_matches_closed_form():
    """With a linear network (identity activation) Eq. 7 is the linear program
    min ||x - x_ref||_1 s.t. w^T x >= beta: the l1-cheapest change puts all of
    the shortfall on the coordinate with the largest |w_i| (the l-infinity norm
    is the dual of l1), objective (beta - w^T x_ref) / max |w_i|."""
    n, m = 20, 3
    rng = np.random.default_rng(46)
    W = rng.standard_normal((m, n)) / np.sqrt(n)
    b = 0.1 * rng.standard_normal(m)
    ev = OracleEval([W], [b], ["identity"])
    x_ref = rng.random(n)
    t = 1
    thr = float(W[t] @ x_ref + b[t]) + 0.8  # infeasible at x_ref by 0.8
    prob = ipm.L1Problem(x_ref=x_ref, t=t, threshold=thr)
    res = ipm.solve(prob, ev, opts=ipm.Options(tol=1e-9))
    assert res.status == "converged", res.status
    i = int(np.argmax(np.abs(W[t])))
    x_star = x_ref.copy()
    x_star[i] += 0.8 / W[t][i]
    assert abs(res.obj - 0.8 / abs(W[t][i])) < 1e-6
    assert np.max(np.abs(res.x - x_star)) < 1e-5
    # already feasible: the reference image itself
    prob2 = ipm.L1Problem(x_ref=x_ref, t=t, threshold=thr - 1.0)
    res2 = ipm.solve(prob2, ev, opts=ipm.Options(tol=1e-9))
    assert res2.status == "converged" and res2.obj < 1e-6


def test_l1_softmax_problem_reaches_kkt_point():
    """Eq. 7 on a small tanh + SoftMax network: the target label reaches the
    0.6 probability threshold, the point is first-order optimal through the
    oracle, and the lock-step batch equals the single solves."""
    dims = (16, 12, 5)
    acts = ["tanh", "softmax"]
    Ws, bs = datagen.mlp_weights(dims, seed=47, bias_scale=0.2)
    ev = OracleEval(Ws, bs, acts)
    rng = np.random.default_rng(48)
    probs = []
    for _ in range(3):
        x_ref = rng.random(16)
        c = int(np.argmax(O.nn(Ws, bs, acts, x_ref)))
        probs.append(ipm.L1Problem(x_ref=x_ref, t=(c + 1) % 5, threshold=0.6))
    batch = ipm.solve_batch(probs, ev)
    for prob, rb in zip(probs, batch):
        assert rb.status == "converged", rb.status
        y = O.nn(Ws, bs, acts, rb.x)
        assert y[prob.t] >= 0.6 - 1e-6
        r = ipm.l1_kkt_residual(prob, rb, lambda x: O.nn(Ws, bs, acts, x),
                                lambda x: O.jacobian(Ws, bs, acts, x))
        assert r["primal"] < 1e-6 and r["dual"] < 1e-5 and r["sign"] > 0, r
        rs = ipm.solve(prob, ev)
        assert rs.iters == rb.iters
        np.testing.assert_allclose(rs.x, rb.x, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- failure classification
def test_margin_ascent_reaches_the_box_maximum_of_a_linear_margin():
    """Linear network NN(x) = W x + b: the margin d^T (W x + b) is largest over
    [0, 1]^n at x_i = [(W^T d)_i > 0], value d^T b + sum_i max((W^T d)_i, 0)
    (closed form); with a target above it the ascent stops there, stationary."""
    dims = (12, 4)
    Ws, bs = datagen.mlp_weights(dims, seed=71, bias_scale=0.3)
    ev = OracleEval(Ws, bs, ["identity"])
    probs = [ipm.Problem(x0=np.full(12, 0.5), t=t, c=c, margin=50.0) for t, c in ((0, 1), (2, 3), (3, 0))]
    X0 = np.random.default_rng(3).uniform(0.0, 1.0, (3, 12))
    marg, reached, stationary = ipm.margin_ascent(probs, X0, ev)
    for k, p in enumerate(probs):
        d = np.zeros(4)
        d[p.t], d[p.c] = 1.0, -1.0
        g = Ws[0].T @ d
        best = float(d @ bs[0] + np.sum(np.maximum(g, 0.0)))
        assert abs(marg[k] - best) <= 1e-9 * max(1.0, abs(best)), (marg[k], best)
    assert stationary.all() and not reached.any()


def test_unreachable_margin_is_labelled_locally_infeasible():
    """tanh outputs bound the margin NN_t - NN_c by 2: a required margin of
    2.5 cannot be met anywhere; the solve fails and the classification finds
    a stationary point of the margin below 2.5.  A reachable margin from a
    non-converged result is labelled reachable."""
    dims = (8, 6, 3)
    acts = ["tanh", "tanh"]
    Ws, bs = datagen.mlp_weights(dims, seed=46)
    ev = OracleEval(Ws, bs, acts)
    x0 = np.full(8, 0.5)
    c = int(np.argmax(O.nn(Ws, bs, acts, x0)))
    bad = ipm.Problem(x0=x0, t=(c + 1) % 3, c=c, margin=2.5)
    res = ipm.solve(bad, ev, opts=ipm.Options(max_iter=60))
    assert res.status != "converged"
    assert ipm.classify_failures([bad], [res], ev) == ["locally_infeasible"]
    ok = ipm.Problem(x0=x0, t=(c + 1) % 3, c=c, margin=0.0)
    fake = ipm.solve(ok, ev, opts=ipm.Options(max_iter=0))
    assert fake.status == "max_iter"
    assert ipm.classify_failures([ok], [fake], ev) == ["reachable"]
    good = ipm.solve(ok, ev)
    assert ipm.classify_failures([ok, bad], [good, res], ev) == ["converged", "locally_infeasible"]


def test_merit_noise_allowance_lets_noisy_evaluations_converge():
    """Network values with 1e-6 relative noise (the rounding of FP32 kernels)
    make the Armijo test compare merit values that differ by less than their
    noise near convergence: some solves end in line_search_fail.  With the
    noise allowance every solve converges, to a KKT point of the noise-free
    problem (residuals recomputed through the oracle)."""
    dims = (64, 48, 48, 5)
    acts = ["tanh", "tanh", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=8)
    clean = OracleEval(Ws, bs, acts)

    class Noisy(OracleEval):
        def __init__(self):
            super().__init__(Ws, bs, acts)
            self.rng = np.random.default_rng(0)

        def nn(self, X):
            v = super().nn(X)
            return v * (1.0 + 1e-6 * self.rng.uniform(-1.0, 1.0, v.shape))

    from paper_2509_22462_amd import warmstart
    probs = warmstart.make_problems(clean.nn, 40, seed=3, m=5, side=8)
    plain = ipm.solve_batch(probs, Noisy(), None, ipm.Options())
    assert sum(r.status == "line_search_fail" for r in plain) >= 1
    allowed = ipm.solve_batch(probs, Noisy(), None, ipm.Options(merit_noise=1e-5))
    assert all(r.status == "converged" for r in allowed)
    for p, r in zip(probs, allowed):
        k = ipm.kkt_residual(p, r, lambda x: O.nn(Ws, bs, acts, x), lambda x: O.jacobian(Ws, bs, acts, x))
        assert k["primal"] < 1e-5 and k["dual_x"] < 1e-4, k
