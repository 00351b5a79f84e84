"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (normwise relative error per point, ||A - A_ref|| / ||A_ref||):
1e-10 for the FP64 path, 1e-5 for FP32 GEMMs, 2e-2 for BF16 GEMMs.
Sizes span several GEMM tiles with ragged tails (n and widths not multiples
of the tile or padding sizes), every activation, both output-layer readings,
biases, several points per call, the degenerate depths (L = 1, 2) and the
full 137M-parameter network (whole 784 x 784 Hessians).  Every comparison
bounds both the normwise error and max|A - A_ref| / max|A_ref|.
"""
import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, nnc

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 2e-2}
PRECS = ["fp64", "fp32", "bf16"]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def relmax(a, b):
    """Largest elementwise error against the largest reference entry."""
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


def close(a, b, tol, what=""):
    """Normwise (Frobenius / 2-norm) relative error and the elementwise bound
    max|a - b| / max|b|, both within tol: a tile that is wrong over a small
    part of a large matrix fails the second even when the first passes."""
    e, em = rel(a, b), relmax(a, b)
    assert e < tol and em < tol, (what, e, em, tol)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


HESS = ["for", "layersum"]


def check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, obj=0.0, q=None, tol=None, hess="auto"):
    tol = tol or TOL[prec]
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=X.shape[0], hess=hess)
    if q is not None:
        net.set_objective_diag(q)
    Y = np.cos(np.arange(X.shape[0] * dims[-1])).reshape(X.shape[0], dims[-1])
    g = net.eval_g(X, Y).cpu().numpy()
    nn_out = net.eval_g(X).cpu().numpy()
    J = net.eval_jac_g(X).cpu().numpy()
    H = net.eval_hess_lag(X, Lam, obj_factor=obj).cpu().numpy()
    for b in range(X.shape[0]):
        ref_nn = O.nn(Ws, bs, acts, X[b])
        close(nn_out[b], ref_nn, tol, ("NN", b))
        close(g[b], Y[b] - ref_nn, max(tol, 1e-14), ("g", b))
        Jr = O.jacobian(Ws, bs, acts, X[b])
        close(J[b], Jr, tol, ("J", b))
        Hr = O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1], obj_factor=obj, q=q)[0]
        if np.linalg.norm(Hr) == 0:
            assert np.all(H[b] == 0)
        else:
            close(H[b], Hr, tol, ("H", b))
        assert np.array_equal(H[b], H[b].T)
    net.destroy()


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
def test_c1_parity(ctx, prec, hess):
    """784 -> 64 -> 64 -> 10 tanh, the small workload with one point."""
    Ws, bs = datagen.mlp_weights(datagen.C1_DIMS, seed=0)
    X, Lam = datagen.points(784, 10, 1, seed=1001)
    check_all(ctx, datagen.C1_DIMS, ["tanh", "tanh", "identity"], Ws, bs, X, Lam, prec, hess=hess)


ACT_CASES = [
    ["tanh", "tanh", "identity"],
    ["sigmoid", "sigmoid", "identity"],
    ["softplus", "softplus", "identity"],
    ["tanh", "softplus", "sigmoid"],  # sigma applied at the output as well
]


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("acts", ACT_CASES, ids=lambda a: "-".join(a))
def test_ragged_nets(ctx, prec, acts, hess):
    dims = (37, 150, 70, 5)  # nothing a multiple of 16 or 64
    Ws, bs = datagen.mlp_weights(dims, seed=3, bias_scale=0.2)
    X, Lam = datagen.points(37, 5, 3, seed=7)
    check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, hess=hess)


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims,acts", [
    ((9, 4), ["identity"]),           # affine: H = 0 (only the objective term)
    ((9, 4), ["tanh"]),               # one layer with sigma at the output
    ((12, 20, 3), ["sigmoid", "identity"]),  # one hidden layer, identity output
    ((12, 20, 3), ["tanh", "tanh"]),
    ((200, 300, 260, 90, 7), ["tanh", "sigmoid", "softplus", "identity"]),
])
def test_depths_and_objective(ctx, prec, dims, acts, hess):
    Ws, bs = datagen.mlp_weights(dims, seed=11, bias_scale=0.1)
    X, Lam = datagen.points(dims[0], dims[-1], 2, seed=12)
    q = np.linspace(0.5, 2.0, dims[0])
    check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, obj=0.75, q=q, hess=hess)


@pytest.mark.parametrize("hess", HESS)
def test_softplus_surrogate_batch(ctx, hess):
    """Net A of the surrogate workload (120 -> 512x4 -> 4, softplus) at 64 points."""
    dims = datagen.C3_DIMS["A"]
    acts = ["softplus"] * 4 + ["identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=0)
    X, Lam = datagen.surrogate_points(120, 4, 64, seed=1003)
    net = ctx.net(dims, acts, Ws, bs, prec="fp32", max_points=64, hess=hess)
    H = net.eval_hess_lag(X, Lam).cpu().numpy()
    J = net.eval_jac_g(X).cpu().numpy()
    for b in (0, 17, 63):
        close(H[b], O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1])[0], 1e-5, ("H", b))
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), 1e-5, ("J", b))
    net.destroy()


@pytest.mark.parametrize("hess", HESS)
def test_determinism_and_batch_consistency(ctx, hess):
    dims = (64, 192, 128, 6)
    acts = ["tanh", "tanh", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=21, bias_scale=0.1)
    X, Lam = datagen.points(64, 6, 4, seed=22)
    net = ctx.net(dims, acts, Ws, bs, prec="fp32", max_points=4, hess=hess)
    H1 = net.eval_hess_lag(X, Lam).cpu().numpy()
    for _ in range(20):
        assert np.array_equal(net.eval_hess_lag(X, Lam).cpu().numpy(), H1)
    # a point evaluated alone gives the same bits as inside the batch
    H2 = net.eval_hess_lag(X[2:3], Lam[2:3]).cpu().numpy()
    assert np.array_equal(H2[0], H1[2])
    g1 = net.eval_g(X).cpu().numpy()
    assert np.array_equal(net.eval_g(X).cpu().numpy(), g1)
    net.destroy()


def test_error_paths(ctx):
    import torch
    dims = (8, 16, 2)
    Ws, bs = datagen.mlp_weights(dims, seed=1)
    net = ctx.net(dims, ["tanh", "identity"], Ws, bs, prec="fp32", max_points=2)
    h = ctx.h
    x = torch.zeros(3, 8, dtype=torch.float64, device="cuda")
    g = torch.zeros(3, 2, dtype=torch.float64, device="cuda")
    assert nnc.nnc_eval_g(h, net.h, 3, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_E_SHAPE
    assert nnc.nnc_eval_g(h, net.h, -1, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_E_SHAPE
    assert nnc.nnc_eval_g(h, net.h, 1, None, None, g.data_ptr()) == nnc.NNC_E_ARG
    assert nnc.nnc_eval_g(h, 99, 1, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_E_ARG
    assert nnc.nnc_eval_hess_lag(h, net.h, 1, x.data_ptr(), 0.0, None, g.data_ptr()) == nnc.NNC_E_ARG
    assert nnc.nnc_eval_g(h, net.h, 0, None, None, None) == nnc.NNC_OK  # B = 0 is a no-op
    with pytest.raises(nnc.NNCError):
        ctx.net((8, 0, 2), ["tanh", "identity"], Ws, bs)
    with pytest.raises(nnc.NNCError):
        ctx.net(dims, [7, 0], Ws, bs)  # activation code out of range
    net.destroy()
    assert nnc.nnc_eval_g(h, net.h, 1, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_E_ARG


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("B", [1, 3])
def test_combined_eval_matches_separate_calls(ctx, prec, B, hess):
    """nnc_eval (one forward pass for g, J and H; at one point the Jacobian
    rows and the FP64 adjoint share each hidden layer's weight stream) gives
    the bits of the three separate oracle calls, for any subset of outputs,
    and matches the oracle."""
    dims = (37, 150, 300, 70, 6)  # m = 6: Jacobian rows on the MFMA stream
    acts = ["tanh", "softplus", "sigmoid", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=17, bias_scale=0.1)
    X, Lam = datagen.points(37, 6, B, seed=18)
    Y = np.sin(np.arange(6.0 * B)).reshape(B, 6)
    q = np.linspace(1.0, 3.0, 37)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=3, hess=hess)
    net.set_objective_diag(q)
    g1 = net.eval_g(X, Y).cpu().numpy()
    J1 = net.eval_jac_g(X).cpu().numpy()
    H1 = net.eval_hess_lag(X, Lam, obj_factor=0.5).cpu().numpy()
    g, J, H = (t.cpu().numpy() for t in net.eval(X, Lam, y=Y, obj_factor=0.5))
    assert np.array_equal(g, g1) and np.array_equal(J, J1) and np.array_equal(H, H1)
    g2, J2, H2 = net.eval(X, want=("J",))
    assert g2 is None and H2 is None and np.array_equal(J2.cpu().numpy(), J1)
    _, _, H3 = net.eval(X, Lam, obj_factor=0.5, want=("H",))
    assert np.array_equal(H3.cpu().numpy(), H1)
    g4, _, _ = net.eval(X, y=Y, want=("g",))
    assert np.array_equal(g4.cpu().numpy(), g1)
    tol = TOL[prec]
    for b in range(B):
        close(g[b], Y[b] - O.nn(Ws, bs, acts, X[b]), max(tol, 1e-14), ("g", b))
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), tol, ("J", b))
        Hr = O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1], obj_factor=0.5, q=q)[0]
        close(H[b], Hr, tol, ("H", b))
    import torch
    x = torch.as_tensor(X, device="cuda")
    out = torch.zeros(B, 37, 37, dtype=torch.float64, device="cuda")
    h = ctx.h
    assert nnc.nnc_eval(h, net.h, B, x.data_ptr(), None, 0.0, None, None, None, None) == nnc.NNC_E_ARG
    assert nnc.nnc_eval(h, net.h, B, x.data_ptr(), None, 0.0, None, None, None,
                        out.data_ptr()) == nnc.NNC_E_ARG  # H needs lambda
    assert nnc.nnc_eval(h, net.h, 4, x.data_ptr(), None, 0.0, None, None, None,
                        out.data_ptr()) == nnc.NNC_E_SHAPE  # beyond max_points, nothing read
    net.destroy()


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims,acts", [
    ((37, 150, 300, 70, 5), ["tanh", "softplus", "sigmoid", "identity"]),
    ((37, 150, 300, 70, 5), ["sigmoid", "tanh", "softplus", "tanh"]),  # sigma at the output
    ((12, 20, 3), ["softplus", "identity"]),  # one hidden layer: output-layer adjoint only
    ((9, 4), ["tanh"]),                       # one layer: no hidden adjoint
])
def test_many_points(ctx, prec, dims, acts, hess):
    """From 64 points on, the primal pass and the FP64 adjoint run as MFMA
    GEMMs over all points (fewer points: weight-streaming kernels).  70 points
    (a ragged last row tile): sampled points against the oracle, the combined
    call bit for bit against the separate calls, and the same points evaluated
    three at a time through the streaming path agree to the tolerance."""
    B = 70
    n, m = dims[0], dims[-1]
    Ws, bs = datagen.mlp_weights(dims, seed=23, bias_scale=0.2)
    X, Lam = datagen.points(n, m, B, seed=24)
    Y = np.cos(np.arange(m * B)).reshape(B, m)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=B, hess=hess)
    g1 = net.eval_g(X, Y).cpu().numpy()
    J1 = net.eval_jac_g(X).cpu().numpy()
    H1 = net.eval_hess_lag(X, Lam).cpu().numpy()
    g, J, H = (t.cpu().numpy() for t in net.eval(X, Lam, y=Y))
    assert np.array_equal(g, g1) and np.array_equal(J, J1) and np.array_equal(H, H1)
    tol = TOL[prec]
    sample = (0, 1, 35, 63, 64, 69)
    for b in sample:
        close(g[b], Y[b] - O.nn(Ws, bs, acts, X[b]), max(tol, 1e-14), ("g", b))
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), tol, ("J", b))
        Hr = O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1])[0]
        close(H[b], Hr, tol, ("H", b))
        assert np.array_equal(H[b], H[b].T)
    idx = np.array(sample[:3])
    gs, Js, Hs = (t.cpu().numpy() for t in net.eval(X[idx], Lam[idx], y=Y[idx]))
    for k, b in enumerate(idx):
        assert rel(gs[k], g[b]) < 2 * max(tol, 1e-14)
        assert rel(Js[k], J[b]) < 2 * tol and rel(Hs[k], H[b]) < 2 * tol
    net.destroy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("B", [1, 2, 3])
@pytest.mark.parametrize("out", ["identity", "softmax"])
def test_jacobian_row_blocks(ctx, prec, B, out):
    """B * m = 20, 40 and 60 Jacobian rows (two to four 16-row blocks) through
    the reverse weight streams, whose rows are staged in LDS per workgroup of
    8 weight blocks with K split over workgroups: the 1000-wide layer (K =
    1024) gives several K slices, the 300-wide one (K = 320) a ragged last
    chunk, 300 and 37 weight rows a last workgroup with fewer blocks than
    waves.  Every point's J against the oracle; the combined call (Jacobian
    rows and FP64 adjoint in one stream) gives the separate call's bits."""
    dims = (37, 300, 1000, 20)
    acts = ["tanh", "sigmoid", out]
    Ws, bs = datagen.mlp_weights(dims, seed=47, bias_scale=0.2)
    X, Lam = datagen.points(dims[0], dims[-1], B, seed=48)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=B)
    J = net.eval_jac_g(X).cpu().numpy()
    _, J2, _ = (t.cpu().numpy() for t in net.eval(X, Lam))
    assert np.array_equal(J, J2)
    for b in range(B):
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), TOL[prec], ("J", b))
    net.destroy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("B", [1, 2])
def test_jacobian_one_row_block_wide_layer(ctx, prec, B):
    """6 or 12 Jacobian rows (one 16-row block) on a 2000-wide layer: the
    row-staged stream at one row block (16 workgroups of weight blocks), with
    K = 1088 leaving a ragged last chunk for both chunk sizes (128 and 256 K
    elements); against the oracle, and the combined call's bits."""
    dims = (37, 2000, 1060, 6)
    acts = ["tanh", "softplus", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=49, bias_scale=0.2)
    X, Lam = datagen.points(dims[0], dims[-1], B, seed=50)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=B)
    J = net.eval_jac_g(X).cpu().numpy()
    g2, J2, H2 = (t.cpu().numpy() for t in net.eval(X, Lam))
    assert np.array_equal(J, J2)
    for b in range(B):
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), TOL[prec], ("J", b))
        close(H2[b], O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1])[0], TOL[prec], ("H", b))
    net.destroy()


@pytest.mark.parametrize("dims,acts", [
    ((37, 600, 500, 400, 12), ["tanh", "softplus", "sigmoid", "identity"]),
    ((37, 150, 70, 5), ["tanh", "sigmoid", "softmax"]),
])
def test_sweep_beside_reverse_passes(ctx, monkeypatch, dims, acts):
    """BF16 layer sum at one point: the forward sweep runs on the library's
    second stream beside the Jacobian + adjoint streams, and S = diag(s) T is
    formed after both.  Against a context created with NNC_SWEEP_OVERLAP=0
    (everything on one stream, S in the sweep epilogue): g and J bit for bit,
    H within the BF16 tolerance of the oracle on both (S is rounded from the
    stored T instead of the accumulator)."""
    Ws, bs = datagen.mlp_weights(dims, seed=51, bias_scale=0.2)
    X, Lam = datagen.points(dims[0], dims[-1], 1, seed=52)
    monkeypatch.setenv("NNC_SWEEP_OVERLAP", "0")
    c1 = nnc.Context(0)
    monkeypatch.delenv("NNC_SWEEP_OVERLAP")
    try:
        n1 = c1.net(dims, acts, Ws, bs, prec="bf16", max_points=1, hess="layersum")
        n2 = ctx.net(dims, acts, Ws, bs, prec="bf16", max_points=1, hess="layersum")
        r1 = [t.cpu().numpy() for t in n1.eval(X, Lam)]
        r2 = [t.cpu().numpy() for t in n2.eval(X, Lam)]
        H2b = n2.eval_hess_lag(X, Lam).cpu().numpy()
        assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
        assert np.array_equal(r2[2], H2b)  # the H-only call takes the same path
        Hr = O.hess_lag(Ws, bs, acts, X, Lam)[0]
        close(r1[2][0], Hr, TOL["bf16"], "H one stream")
        close(r2[2][0], Hr, TOL["bf16"], "H two streams")
        assert np.array_equal(r2[2][0], r2[2][0].T)
        n1.destroy()
        n2.destroy()
    finally:
        c1.close()


# ---------------------------------------------------------------- full-size network
@pytest.fixture(scope="module")
def c2_weights():
    return datagen.mlp_weights(datagen.C2_DIMS, seed=0)


_C2_REFS = {}


def c2_reference(Ws, bs, acts, seed, B, b):
    """NN, J and the whole 784 x 784 H of point b of a seeded draw (FP64
    oracle, forward-over-reverse), computed once per module run."""
    key = (seed, B, b)
    if key not in _C2_REFS:
        X, Lam = datagen.points(784, 10, B, seed=seed)
        _C2_REFS[key] = (O.nn(Ws, bs, acts, X[b]), O.jacobian_reverse(Ws, bs, acts, X[b]),
                         O.hess_for(Ws, bs, acts, X[b], Lam[b]))
    return _C2_REFS[key]


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
def test_c2_full_size_whole(ctx, c2_weights, prec, hess):
    """784 -> 4096 -> 8192 -> 8192 -> 4096 -> 10 tanh (137M weights), 2 points:
    g, J and the whole 784 x 784 H of each point against the oracle, normwise
    and elementwise; also the one-point combined call."""
    Ws, bs = c2_weights
    acts = ["tanh"] * 4 + ["identity"]
    X, Lam = datagen.points(784, 10, 2, seed=1004)
    net = ctx.net(datagen.C2_DIMS, acts, Ws, bs, prec=prec, max_points=2, hess=hess)
    g = net.eval_g(X).cpu().numpy()
    J = net.eval_jac_g(X).cpu().numpy()
    H = net.eval_hess_lag(X, Lam).cpu().numpy()
    tol = TOL[prec]
    for b in range(2):
        nn_ref, J_ref, H_ref = c2_reference(Ws, bs, acts, 1004, 2, b)
        close(g[b], nn_ref, tol, (prec, "g", b))
        close(J[b], J_ref, tol, (prec, "J", b))
        close(H[b], H_ref, tol, (prec, "H", b))
        assert np.array_equal(H[b], H[b].T)
        if b == 0:
            # the one-point combined call (shared weight streams) on the full network
            g1, J1, H1 = (t.cpu().numpy()[0] for t in net.eval(X[:1], Lam[:1]))
            close(g1, nn_ref, tol, (prec, "g1"))
            close(J1, J_ref, tol, (prec, "J1"))
            close(H1, H_ref, tol, (prec, "H1"))
    net.destroy()


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
def test_every_gemm_tiling(ctx, prec, hess):
    """Each compiled tile configuration, forced on every sweep GEMM, against the oracle."""
    dims = (37, 150, 300, 70, 5)
    acts = ["tanh", "softplus", "sigmoid", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=13, bias_scale=0.1)
    X, Lam = datagen.points(37, 5, 3, seed=14)
    code = nnc.PREC_CODES[prec]
    try:
        for cfg in range(nnc.nnc_gemm_config_count()):
            nnc.nnc_set_gemm_config(ctx.h, code, cfg)
            check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, hess=hess)
    finally:
        nnc.nnc_set_gemm_config(ctx.h, code, -1)
    with pytest.raises(nnc.NNCError):
        nnc.nnc_set_gemm_config(ctx.h, code, nnc.nnc_gemm_config_count())


@pytest.mark.parametrize("n", [1, 5, 784])
def test_pack_lower_triangle(ctx, n):
    """nnc_hess_pack_lower: row-major lower triangle, bit for bit; at n = 784
    it holds the 307,720 entries of the reduced-space Hessian structure."""
    import torch
    B = 3
    H = torch.randn(B, n, n, dtype=torch.float64, device="cuda")
    tri = n * (n + 1) // 2
    Hp = torch.full((B, tri), float("nan"), dtype=torch.float64, device="cuda")
    assert nnc.nnc_hess_pack_lower(ctx.h, B, n, H.data_ptr(), Hp.data_ptr()) == nnc.NNC_OK
    ii, jj = np.tril_indices(n)
    np.testing.assert_array_equal(Hp.cpu().numpy(), H.cpu().numpy()[:, ii, jj])
    if n == 784:
        assert tri == 307720
    assert nnc.nnc_hess_pack_lower(ctx.h, B, n, H.data_ptr(), H.data_ptr()) == nnc.NNC_E_ARG
    assert nnc.nnc_hess_pack_lower(ctx.h, B, 0, H.data_ptr(), Hp.data_ptr()) == nnc.NNC_E_SHAPE
    assert nnc.nnc_hess_pack_lower(ctx.h, 0, n, None, None) == nnc.NNC_OK


@pytest.mark.parametrize("hess", HESS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("ks", [2, 3])
def test_ksplit_sweeps_every_tiling(ctx, prec, ks, hess):
    """Sweep GEMMs as K slices (FP32 partials, FP64 for FP64 GEMMs; slice-order
    sum; fused epilogue) under every tiling, against the oracle; the same bits
    on a repeat."""
    dims = (37, 150, 300, 70, 5)  # K = 192, 320, 128 after padding: ragged slices
    acts = ["tanh", "softplus", "sigmoid", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=23, bias_scale=0.1)
    X, Lam = datagen.points(37, 5, 3, seed=24)
    code = nnc.PREC_CODES[prec]
    try:
        assert nnc.nnc_set_gemm_ksplit(ctx.h, code, ks) == nnc.NNC_OK
        for cfg in range(nnc.nnc_gemm_config_count()):
            nnc.nnc_set_gemm_config(ctx.h, code, cfg)
            check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, hess=hess)
        nnc.nnc_set_gemm_config(ctx.h, code, -1)
        net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=3, hess=hess)
        H1 = net.eval_hess_lag(X, Lam).cpu().numpy()
        assert np.array_equal(net.eval_hess_lag(X, Lam).cpu().numpy(), H1)
        net.destroy()
    finally:
        nnc.nnc_set_gemm_config(ctx.h, code, -1)
        nnc.nnc_set_gemm_ksplit(ctx.h, code, -1)
    assert nnc.nnc_set_gemm_ksplit(ctx.h, code, 9) == nnc.NNC_E_ARG


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("points", [1, 32])
def test_c2_benchmark_configuration(c2_weights, prec, points, monkeypatch):
    """The 137M network in the launch configuration bench.py times: the
    committed gfx950 tiling table (K-split sweep GEMMs where it says so) and
    one combined nnc_eval call, at 1 point (the headline) and 32 points (the
    precision sweep); g, J and the whole H of the first and last point
    against the oracle, normwise and elementwise."""
    import torch
    monkeypatch.setenv("NNC_AUTOTUNE_CACHE", nnc.TUNED_TABLE)
    c = nnc.Context(0)
    try:
        Ws, bs = c2_weights
        acts = ["tanh"] * 4 + ["identity"]
        seed = 1002 if points == 1 else 1004
        X, Lam = datagen.points(784, 10, points, seed=seed)
        net = c.net(datagen.C2_DIMS, acts, Ws, bs, prec=prec, max_points=points)
        # n = 784 below the hidden widths: the layer sum is the cheaper method
        assert net.hess_method == "layersum"
        g, J, H = (t.cpu().numpy() for t in net.eval(X, Lam))
        torch.cuda.synchronize()
        tol = TOL[prec]
        for b in sorted({0, points - 1}):
            nn_ref, J_ref, H_ref = c2_reference(Ws, bs, acts, seed, points, b)
            close(g[b], nn_ref, tol, (prec, points, "g", b))
            close(J[b], J_ref, tol, (prec, points, "J", b))
            close(H[b], H_ref, tol, (prec, points, "H", b))
            assert np.array_equal(H[b], H[b].T)
        net.destroy()
    finally:
        torch.cuda.synchronize()
        c.close()


def test_hess_method_selection_and_errors(ctx):
    """The automatic choice follows the algorithmic flops of the two methods
    (784 -> 64 -> 64 -> 10: forward-over-reverse; widths above n: the layer
    sum); switching keeps results; bad codes are rejected."""
    Ws, bs = datagen.mlp_weights(datagen.C1_DIMS, seed=0)
    acts = ["tanh", "tanh", "identity"]
    net = ctx.net(datagen.C1_DIMS, acts, Ws, bs, prec="fp64", max_points=2)
    assert net.hess_method == "for"
    dims = (40, 300, 200, 3)
    Ws2, bs2 = datagen.mlp_weights(dims, seed=5, bias_scale=0.1)
    net2 = ctx.net(dims, acts, Ws2, bs2, prec="fp64", max_points=2)
    assert net2.hess_method == "layersum"
    X, Lam = datagen.points(40, 3, 2, seed=6)
    H_ls = net2.eval_hess_lag(X, Lam).cpu().numpy()
    net2.set_hess_method("for")
    assert net2.hess_method == "for"
    H_for = net2.eval_hess_lag(X, Lam).cpu().numpy()
    net2.set_hess_method("auto")
    assert net2.hess_method == "layersum"
    assert np.array_equal(net2.eval_hess_lag(X, Lam).cpu().numpy(), H_ls)
    for b in range(2):
        Hr = O.hess_layersum(Ws2, bs2, acts, X[b], Lam[b])
        close(H_ls[b], Hr, 1e-10, ("layersum", b))
        close(H_for[b], Hr, 1e-10, ("for", b))
    assert nnc.load_library().nnc_net_set_hess_method(ctx.h, net2.h, 3) == nnc.NNC_E_ARG
    assert nnc.load_library().nnc_net_set_hess_method(ctx.h, 99, 1) == nnc.NNC_E_ARG
    net.destroy()
    net2.destroy()


# ---------------------------------------------------------------- SoftMax output layer
SOFTMAX_CASES = [
    ((37, 150, 70, 5), ["tanh", "sigmoid", "softmax"]),
    ((12, 20, 3), ["tanh", "softmax"]),         # one hidden layer
    ((9, 4), ["softmax"]),                       # the SoftMax layer alone (multinomial logistic)
    ((200, 300, 260, 90, 7), ["sigmoid", "tanh", "softplus", "softmax"]),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims,acts", SOFTMAX_CASES)
def test_softmax_output(ctx, prec, dims, acts):
    """SoftMax output layer (Table 1's classifiers): g, J and H (layer sum with
    the rank-two SoftMax term) against the oracle at 3 points, with an
    objective diagonal; the combined call gives the separate calls' bits."""
    Ws, bs = datagen.mlp_weights(dims, seed=41, bias_scale=0.3)
    X, Lam = datagen.points(dims[0], dims[-1], 3, seed=42)
    q = np.linspace(0.5, 1.5, dims[0])
    check_all(ctx, dims, acts, Ws, bs, X, Lam, prec, obj=0.5, q=q)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=3)
    assert net.hess_method == "layersum"
    g1 = net.eval_g(X).cpu().numpy()
    J1 = net.eval_jac_g(X).cpu().numpy()
    H1 = net.eval_hess_lag(X, Lam).cpu().numpy()
    g, J, H = (t.cpu().numpy() for t in net.eval(X, Lam))
    assert np.array_equal(g, g1) and np.array_equal(J, J1) and np.array_equal(H, H1)
    assert np.allclose(g.sum(axis=1), 1.0, rtol=0, atol=1e-12)  # probabilities
    with pytest.raises(nnc.NNCError):
        net.set_hess_method("for")
    net.destroy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_softmax_mnist_shape_and_many_points(ctx, prec):
    """784 -> 128 x 5 -> 10 tanh + SoftMax (Table 1's smallest MNIST network)
    at 70 points (the many-point GEMM primal and adjoint paths), sampled
    points whole against the oracle, normwise and elementwise."""
    dims = (784,) + (128,) * 5 + (10,)
    acts = ["tanh"] * 5 + ["softmax"]
    Ws, bs = datagen.mlp_weights(dims, seed=43, bias_scale=0.1)
    X = datagen.blob_images(70, seed=44)
    _, Lam = datagen.points(784, 10, 70, seed=45)
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=70)
    g, J, H = (t.cpu().numpy() for t in net.eval(X, Lam))
    tol = TOL[prec]
    for b in (0, 33, 69):
        close(g[b], O.nn(Ws, bs, acts, X[b]), tol, ("g", b))
        close(J[b], O.jacobian(Ws, bs, acts, X[b]), tol, ("J", b))
        close(H[b], O.hess_layersum(Ws, bs, acts, X[b], Lam[b]), tol, ("H", b))
    net.destroy()
    with pytest.raises(nnc.NNCError):  # SoftMax on a hidden layer
        ctx.net((5, 4, 3), ["softmax", "identity"], *datagen.mlp_weights((5, 4, 3), seed=1))
