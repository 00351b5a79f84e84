"""nnc_eval_g_static (no allocation; forward-pass vectors in the library's
static device workspace) against nnc_eval_g through the C ABI: the same
bits, on two calls in a row (the second with fewer points), and the FP64
oracle; oversized calls are refused."""
import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, nnc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2), ("fp64", 1e-10)])
def test_static_eval_g_matches_eval_g(prec, tol):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    ctx = nnc.Context(0)
    try:
        dims = (37, 150, 300, 70, 5)
        acts = ["tanh", "softplus", "sigmoid", "identity"]
        Ws, bs = datagen.mlp_weights(dims, seed=61, bias_scale=0.2)
        net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=70)
        h = ctx.h
        # 70 points (many-point GEMM primal pass for FP32/FP64), then 3 (weight streams)
        for B, seed in ((70, 62), (3, 63)):
            X, _ = datagen.points(37, 5, B, seed=seed)
            Y = np.cos(np.arange(5.0 * B)).reshape(B, 5)
            x = torch.as_tensor(X, device="cuda")
            y = torch.as_tensor(Y, device="cuda")
            g_ref = torch.full((B, 5), np.nan, dtype=torch.float64, device="cuda")
            g_st = torch.full((B, 5), np.nan, dtype=torch.float64, device="cuda")
            assert nnc.nnc_eval_g(h, net.h, B, x.data_ptr(), y.data_ptr(), g_ref.data_ptr()) == nnc.NNC_OK
            rc = nnc.nnc_eval_g_static(h, net.h, B, x.data_ptr(), y.data_ptr(), g_st.data_ptr())
            assert rc == nnc.NNC_OK, nnc.nnc_last_error(h)
            torch.cuda.synchronize()
            a, b = g_st.cpu().numpy(), g_ref.cpu().numpy()
            assert np.array_equal(a, b), (B, np.max(np.abs(a - b)))
            for p in (0, B - 1):
                ref = Y[p] - O.nn(Ws, bs, acts, X[p])
                assert np.linalg.norm(a[p] - ref) / np.linalg.norm(ref) < max(tol, 1e-14)
        # NN(x) form (y NULL), B = 0 no-op, null pointers
        X, _ = datagen.points(37, 5, 2, seed=64)
        x = torch.as_tensor(X, device="cuda")
        g_st = torch.empty(2, 5, dtype=torch.float64, device="cuda")
        assert nnc.nnc_eval_g_static(h, net.h, 2, x.data_ptr(), None, g_st.data_ptr()) == nnc.NNC_OK
        torch.cuda.synchronize()
        for p in range(2):
            ref = O.nn(Ws, bs, acts, X[p])
            assert np.linalg.norm(g_st.cpu().numpy()[p] - ref) / np.linalg.norm(ref) < tol
        assert nnc.nnc_eval_g_static(h, net.h, 0, None, None, None) == nnc.NNC_OK
        assert nnc.nnc_eval_g_static(h, net.h, 2, None, None, g_st.data_ptr()) == nnc.NNC_E_ARG
        assert nnc.nnc_eval_g_static(h, net.h, 71, x.data_ptr(), None, g_st.data_ptr()) == nnc.NNC_E_SHAPE
        net.destroy()
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_static_eval_g_refuses_beyond_workspace():
    """A network whose points need more than the 64 MiB workspace: the call
    returns NNC_E_SHAPE before launching anything; a call that fits works."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    ctx = nnc.Context(0)
    try:
        dims = (16, 4096, 4096, 4096, 4096, 3)  # about 264 KB of vectors per point
        acts = ["tanh"] * 4 + ["identity"]
        Ws, bs = datagen.mlp_weights(dims, seed=65)
        net = ctx.net(dims, acts, Ws, bs, prec="fp32", max_points=300)
        X, _ = datagen.points(16, 3, 300, seed=66)
        x = torch.as_tensor(X, device="cuda")
        g = torch.full((300, 3), np.nan, dtype=torch.float64, device="cuda")
        assert nnc.nnc_eval_g_static(ctx.h, net.h, 300, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_E_SHAPE
        assert "static workspace" in nnc.nnc_last_error(ctx.h)
        torch.cuda.synchronize()
        assert np.all(np.isnan(g.cpu().numpy()))  # nothing written
        assert nnc.nnc_eval_g_static(ctx.h, net.h, 200, x.data_ptr(), None, g.data_ptr()) == nnc.NNC_OK
        g_ref = net.eval_g(X[:200]).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy()[:200], g_ref)
        net.destroy()
    finally:
        torch.cuda.synchronize()
        ctx.close()
