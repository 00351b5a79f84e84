"""Host interior-point solves on the GPU evaluator against the same solves on
the FP64 oracle evaluator (small 784 -> 64 -> 64 -> 10 tanh network, blob-image
problems min ||x - x0||^2 s.t. NN_t - NN_c >= 0.5, 0 <= x <= 1).

Both solves must end with the same status at the same point, and the GPU
solve's point must be a KKT point to the paper's tolerance (1e-6) when its
residuals are recomputed through the oracle."""
import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, evaluator, ipm, warmstart

pytestmark = pytest.mark.gpu

DIMS = datagen.C1_DIMS
ACTS = ["tanh", "tanh", "identity"]


class OracleEval(ipm.Evaluator):
    def __init__(self, Ws, bs, acts):
        self.Ws, self.bs, self.acts = Ws, bs, acts

    def nn(self, X):
        return O.residual(self.Ws, self.bs, self.acts, X)

    def jac(self, X):
        return O.jacobians(self.Ws, self.bs, self.acts, X)

    def hess(self, X, Lam):
        return O.hess_lag(self.Ws, self.bs, self.acts, X, Lam)


def scaled_kkt_through_oracle(prob, res, Ws, bs, opts):
    """The solver's scaled optimality error (dual infeasibility / s_d,
    primal infeasibility, complementarity / s_c) with NN and J from the oracle."""
    r = ipm.kkt_residual(prob, res, lambda x: O.nn(Ws, bs, ACTS, x),
                         lambda x: O.jacobian(Ws, bs, ACTS, x))
    n, m = prob.n, res.y.shape[0]
    zsum = float(np.sum(res.zL) + np.sum(res.zU) + res.zs)
    sd = max(opts.s_max, (float(np.sum(np.abs(res.lam))) + abs(res.nu) + zsum) / (m + 2 * n + 2)) / opts.s_max
    sc = max(opts.s_max, zsum / (2 * n + 1)) / opts.s_max
    dual = max(r["dual_x"], r["dual_y"], r["dual_s"])
    return max(dual / sd, r["primal"], r["comp"] / sc), r


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2509_22462_amd import nnc
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("prec,xtol,ktol", [("fp64", 1e-8, 1e-6), ("fp32", 1e-4, 1e-5)])
def test_gpu_solves_match_oracle_solves(ctx, prec, xtol, ktol):
    Ws, bs = datagen.mlp_weights(DIMS, seed=0)
    oracle_ev = OracleEval(Ws, bs, ACTS)
    probs = warmstart.make_problems(oracle_ev.nn, 4, seed=300, m=10)
    opts = ipm.Options()
    ref = ipm.solve_batch(probs, oracle_ev, opts=opts)
    ev = evaluator.GpuEvaluator(ctx, DIMS, ACTS, Ws, bs, prec=prec, max_points=4)
    try:
        res = ipm.solve_batch(probs, ev, opts=opts, max_batch=4)
    finally:
        ev.close()
    converged = 0
    for p, r0, r1 in zip(probs, ref, res):
        assert r1.status == r0.status, (r0.status, r1.status)
        if r0.status != "converged":
            continue
        converged += 1
        assert np.max(np.abs(r1.x - r0.x)) < xtol, np.max(np.abs(r1.x - r0.x))
        assert abs(r1.obj - r0.obj) < 10 * xtol * max(1.0, r0.obj)
        err, parts = scaled_kkt_through_oracle(p, r1, Ws, bs, opts)
        assert err <= ktol, (err, parts)
        # the margin holds through the oracle
        y = O.nn(Ws, bs, ACTS, r1.x)
        assert y[p.t] - y[p.c] >= p.margin - ktol
        assert np.all(r1.x >= 0.0) and np.all(r1.x <= 1.0)
    assert converged >= 3


@pytest.mark.parametrize("prec,xtol,device_kkt", [("fp64", 1e-8, False), ("fp32", 1e-4, False),
                                                  ("fp32", 1e-4, True)])
def test_adversarial_image_problem_matches_oracle(ctx, prec, xtol, device_kkt):
    """The paper's Eq. 7 on a 784 -> 64 -> 64 -> 10 tanh + SoftMax network:
    min ||x - x_ref||_1 s.t. y = NN(x), y_t >= 0.6 (slack split x = x_ref + p - q),
    blob images as x_ref, a target label other than the predicted one.  The GPU
    evaluator's solves (host or device Newton steps) end with the oracle
    evaluator's status at its point, with the target probability at 0.6."""
    acts = ["tanh", "tanh", "softmax"]
    Ws, bs = datagen.mlp_weights(DIMS, seed=7)

    class SoftmaxOracle(ipm.Evaluator):
        def nn(self, X):
            return O.residual(Ws, bs, acts, X)

        def jac(self, X):
            return O.jacobians(Ws, bs, acts, X)

        def hess(self, X, Lam):
            return O.hess_lag(Ws, bs, acts, X, Lam, method="layersum")

    oracle_ev = SoftmaxOracle()
    X0 = datagen.blob_images(3, seed=310)
    probs = []
    for i in range(3):
        c = int(np.argmax(O.nn(Ws, bs, acts, X0[i])))
        probs.append(ipm.L1Problem(x_ref=X0[i], t=(c + 3 + i) % 10, threshold=0.6))
    opts = ipm.Options()
    ref = ipm.solve_batch(probs, oracle_ev, opts=opts)
    ev = evaluator.GpuEvaluator(ctx, DIMS, acts, Ws, bs, prec=prec, max_points=3)
    try:
        # the evaluator's allowance for the rounding noise of its merit values
        opts_gpu = ipm.Options(device_kkt=device_kkt, merit_noise=ev.merit_noise)
        res = ipm.solve_batch(probs, ev, opts=opts_gpu, max_batch=3)
    finally:
        ev.close()
    converged = 0
    for p, r0, r1 in zip(probs, ref, res):
        assert r1.status == r0.status, (r0.status, r1.status)
        if r0.status != "converged":
            continue
        converged += 1
        assert np.max(np.abs(r1.x - r0.x)) < xtol, np.max(np.abs(r1.x - r0.x))
        y = O.nn(Ws, bs, acts, r1.x)
        assert y[p.t] >= 0.6 - 1e-5
        r = ipm.l1_kkt_residual(p, r1, lambda x: O.nn(Ws, bs, acts, x),
                                lambda x: O.jacobian(Ws, bs, acts, x))
        assert r["primal"] < 1e-5 and r["sign"] > 0, r
    assert converged >= 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_merged_jac_hess_and_kept_hessians(ctx, prec):
    """jac_hess (one nnc_eval per chunk) gives the bits of the separate jac
    and hess calls, across chunks of max_points rows; Newton steps solved
    against the Hessians it kept on the device (rows reordered and partly
    dropped, so the kept slots form several runs) give the bits of the steps
    that recompute H."""
    Ws, bs = datagen.mlp_weights(DIMS, seed=5, bias_scale=0.2)
    X, Lam = datagen.points(DIMS[0], DIMS[-1], 7, seed=6)
    ev = evaluator.GpuEvaluator(ctx, DIMS, ACTS, Ws, bs, prec=prec, max_points=3)
    try:
        J, H = ev.jac(X), ev.hess(X, Lam)
        pairs = ev.jac_hess(X, Lam)
        assert np.array_equal(np.stack([p[0] for p in pairs]), J)
        assert np.array_equal(np.stack([p[1] for p in pairs]), H)
        kept = ev.jac_hess(X, Lam, keep=True)
        assert all(p[1] is None for p in kept)
        assert np.array_equal(np.stack([p[0] for p in kept]), J)
        rng = np.random.default_rng(7)
        rows = [5, 0, 1, 3, 6]  # row 2 and 4 converged: slots {0, 1}, {3}, {5, 6}
        n = DIMS[0]
        D = rng.uniform(1.0, 3.0, (len(rows), n)) + 2.0
        A = rng.standard_normal((len(rows), n))
        S = rng.uniform(0.1, 1.0, len(rows))
        R = rng.standard_normal((len(rows), n))
        dx_kept = ev.newton(X[rows], Lam[rows], D, A, S, R, 1e-4, 1e40)
        ev.hslot = {}
        dx_new = ev.newton(X[rows], Lam[rows], D, A, S, R, 1e-4, 1e40)
        for a, b in zip(dx_kept, dx_new):
            assert a is not None and np.array_equal(a, b)
    finally:
        ev.close()
