"""Warm-start MLP training kernels against the FP64 backprop/Adam oracle (GPU)."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2509_22462_amd import datagen, nnc

pytestmark = pytest.mark.gpu

ACTS3 = ["tanh", "tanh", "identity"]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def flatten(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])


def unflatten(v, dims):
    Ws, bs, o = [], [], 0
    for l in range(1, len(dims)):
        n = dims[l] * dims[l - 1]
        Ws.append(v[o:o + n].reshape(dims[l], dims[l - 1]).copy())
        o += n
        bs.append(v[o:o + dims[l]].copy())
        o += dims[l]
    return Ws, bs


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
def test_one_step_matches_oracle(ctx, prec, tol):
    import torch
    dims = (20, 64, 48, 12)
    batch = 50  # not a multiple of the 64-row padding
    Ws, bs = datagen.mlp_weights(dims, seed=30, bias_scale=0.1)
    rng = np.random.default_rng(31)
    X = rng.random((batch, 20))
    Y = rng.standard_normal((batch, 12))
    h = ctx.h
    mlp = nnc.nnc_train_create(h, list(dims), batch, nnc.PREC_CODES[prec], 7)
    nnc.nnc_train_set_params(h, mlp, flatten(Ws, bs))
    Xd = torch.as_tensor(X, device="cuda")
    Yd = torch.as_tensor(Y, device="cuda")
    lr = 1e-3
    loss = nnc.nnc_train_step(h, mlp, Xd.data_ptr(), Yd.data_ptr(), lr)
    ref_loss, gW, gb = M.grads(Ws, bs, ACTS3, X, Y)
    assert abs(loss - ref_loss) / ref_loss < tol
    g_gpu = nnc.nnc_train_get_grads(h, mlp)
    g_ref = flatten(gW, gb)
    assert rel(g_gpu, g_ref) < tol, rel(g_gpu, g_ref)
    # parameters after one Adam step
    params = Ws + bs
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    M.adam_step(params, gW + gb, m, v, 1, lr=lr)
    p_gpu = nnc.nnc_train_get_params(h, mlp)
    p_ref = flatten(params[:3], params[3:])
    p0 = flatten(*datagen.mlp_weights(dims, seed=30, bias_scale=0.1))
    # the first Adam step moves every parameter by about lr * sign(g): compare the
    # update, allowing sign flips only where the gradient is tiny
    d_gpu = p_gpu - p0
    d_ref = p_ref - p0
    big = np.abs(g_ref) > 1e-3 * np.max(np.abs(g_ref))
    assert np.max(np.abs(d_gpu[big] - d_ref[big])) < (1e-6 if prec == "fp32" else 2e-4)
    nnc.nnc_train_destroy(h, mlp)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_training_reduces_loss_and_predict_matches(ctx, prec):
    import torch
    dims = (16, 128, 128, 8)
    batch = 128
    rng = np.random.default_rng(33)
    X = rng.random((batch, 16))
    Wt = rng.standard_normal((8, 16))
    Y = np.tanh(X @ Wt.T)
    h = ctx.h
    mlp = nnc.nnc_train_create(h, list(dims), batch, nnc.PREC_CODES[prec], 11)
    Xd = torch.as_tensor(X, device="cuda")
    Yd = torch.as_tensor(Y, device="cuda")
    l0 = nnc.nnc_train_step(h, mlp, Xd.data_ptr(), Yd.data_ptr(), 3e-3)
    for _ in range(300):
        nnc.nnc_train_step(h, mlp, Xd.data_ptr(), Yd.data_ptr(), 3e-3, want_loss=False)
    l1 = nnc.nnc_train_step(h, mlp, Xd.data_ptr(), Yd.data_ptr(), 3e-3)
    assert l1 < 0.1 * l0, (l0, l1)
    out = torch.empty(40, 8, dtype=torch.float64, device="cuda")
    nnc.nnc_train_predict(h, mlp, 40, Xd.data_ptr(), out.data_ptr())
    Ws, bs = unflatten(nnc.nnc_train_get_params(h, mlp), dims)
    _, ref = M.forward(Ws, bs, ACTS3, X[:40])
    assert rel(out.cpu().numpy(), ref) < (1e-5 if prec == "fp32" else 3e-2)
    with pytest.raises(nnc.NNCError):
        nnc.nnc_train_predict(h, mlp, batch + 1, Xd.data_ptr(), out.data_ptr())
    nnc.nnc_train_destroy(h, mlp)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
def test_six_adam_steps_match_oracle(ctx, prec, tol):
    """Six training steps: at every step the gradients against backprop at the
    GPU's current parameters, and the parameters after the step against the
    oracle's Adam (bias corrections of steps 1..6, both moments carried over)
    applied to the same gradients."""
    import torch
    dims = (20, 64, 48, 12)
    batch = 50
    Ws, bs = datagen.mlp_weights(dims, seed=34, bias_scale=0.1)
    rng = np.random.default_rng(35)
    X = rng.random((batch, 20))
    Y = rng.standard_normal((batch, 12))
    h = ctx.h
    mlp = nnc.nnc_train_create(h, list(dims), batch, nnc.PREC_CODES[prec], 9)
    nnc.nnc_train_set_params(h, mlp, flatten(Ws, bs))
    Xd = torch.as_tensor(X, device="cuda")
    Yd = torch.as_tensor(Y, device="cuda")
    lr = 2e-3
    ref = nnc.nnc_train_get_params(h, mlp)  # FP32 master values, as FP64
    m = [np.zeros_like(ref)]
    v = [np.zeros_like(ref)]
    for t in range(1, 7):
        before = nnc.nnc_train_get_params(h, mlp)
        nnc.nnc_train_step(h, mlp, Xd.data_ptr(), Yd.data_ptr(), lr, want_loss=False)
        g_gpu = nnc.nnc_train_get_grads(h, mlp)
        _, gW, gb = M.grads(*unflatten(before, dims), ACTS3, X, Y)
        assert rel(g_gpu, flatten(gW, gb)) < tol, (t, rel(g_gpu, flatten(gW, gb)))
        p = [ref]
        M.adam_step(p, [g_gpu], m, v, t, lr=lr)
        after = nnc.nnc_train_get_params(h, mlp)
        # FP32 master parameters and FP32 Adam arithmetic: a few ulps per step
        assert np.max(np.abs(after - ref)) < 1e-6 * t, (t, np.max(np.abs(after - ref)))
        # steps after the first are not sign(g) * lr: momentum and bias correction matter
        if t >= 2:
            assert np.max(np.abs(np.abs(after - before) - lr)) > 1e-2 * lr
    nnc.nnc_train_destroy(h, mlp)
