"""The autotuner validates its candidates: every tiling it times is compared,
on the same inputs, with the plain 64 x 64 register-staged tiling (max |diff|
relative to max |reference| of the GEMM's primary output), and only
candidates within the tolerance of their precision can be chosen.  Each line
it appends to the tuning cache records the check; after tuning, g, J and H
still match the oracle."""
import json

import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, nnc

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 2e-2, "fp64": 1e-10}
ORACLE_TOL = {"fp32": 1e-5, "bf16": 2e-2, "fp64": 1e-10}


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("hess", ["for", "layersum"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_autotune_validates_candidates(ctx, tmp_path, monkeypatch, prec, hess):
    dims, acts = (37, 150, 70, 5), ["tanh", "softplus", "identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=61, bias_scale=0.2)
    X, Lam = datagen.points(dims[0], dims[-1], 3, seed=62)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("NNC_AUTOTUNE_CACHE", str(cache))
    net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=3, hess=hess)
    try:
        assert nnc.nnc_autotune(ctx.h, net.h, 3) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
        rows = [json.loads(line) for line in cache.read_text().splitlines()]
        assert rows, "no tuned GEMM recorded"
        for r in rows:
            assert r["validated"] is True, r
            assert r["rejected"] == 0, r  # every tiling computes the same product
            assert r["candidates"] >= 2, r
            assert 0.0 <= r["max_rel_err"] <= TOL[prec], r
        H = net.eval_hess_lag(X, Lam).cpu().numpy()
        J = net.eval_jac_g(X).cpu().numpy()
        for b in range(3):
            Hr = O.hess_lag(Ws, bs, acts, X[b:b + 1], Lam[b:b + 1])[0]
            assert np.linalg.norm(H[b] - Hr) <= ORACLE_TOL[prec] * np.linalg.norm(Hr)
            Jr = O.jacobian(Ws, bs, acts, X[b])
            assert np.linalg.norm(J[b] - Jr) <= ORACLE_TOL[prec] * np.linalg.norm(Jr)
    finally:
        net.destroy()
