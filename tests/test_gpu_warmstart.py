"""Learned warm start end to end on the GPU (small network).

Cold-solve blob-image problems with the host IPM on the GPU evaluator, train
the warm-start MLP with the library's training kernels, and show that warm
starts on held-out problems need fewer IPM iterations than cold starts,
while every solve still ends at a KKT point (warm failures fall back)."""
import numpy as np
import pytest

from paper_2509_22462_amd import datagen, evaluator, ipm, nnc, warmstart

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def test_warm_start_beats_cold_start(ctx):
    dims = (64, 256, 256, 5)
    acts = ["tanh", "tanh", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=8)
    ev = evaluator.GpuEvaluator(ctx, dims, acts, Ws, bs, prec="fp32", max_points=64)
    train = warmstart.make_problems(ev.nn, 640, seed=100, m=5, side=8)
    test = warmstart.make_problems(ev.nn, 64, seed=200, m=5, side=8)
    res = ipm.solve_batch(train, ev, max_batch=64)
    ok = [i for i, r in enumerate(res) if r.status == "converged"]
    assert len(ok) > 0.9 * len(train)
    F = warmstart.features([train[i] for i in ok], 5)
    Y = warmstart.targets([res[i] for i in ok])
    model = warmstart.WarmStartModel(ctx, 64, 5, hidden=(256, 256), batch=64, prec="bf16", seed=1)
    rep = model.fit(F, Y, epochs=150, lr=2e-3)
    assert rep.val_loss[-1] < 0.5 * rep.val_loss[0]
    starts = model.starts(test)
    cmp_ = warmstart.compare(test, starts, ev, max_batch=64)
    print(f"cold iters {cmp_.cold_iters.mean():.2f} warm iters {cmp_.warm_iters.mean():.2f} "
          f"fallbacks {cmp_.fallbacks} rejected {cmp_.rejected}")
    assert all(s == "converged" for s in cmp_.warm_status)
    assert cmp_.warm_iters.mean() < cmp_.cold_iters.mean()
    model.close()
    ev.close()
