"""Batched multi-network evaluation (grouped persistent launches + HIP graph)."""
import numpy as np
import pytest

from oracle import nn as O
from paper_2509_22462_amd import datagen, nnc

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def close(a, b, tol, what=""):
    """Normwise relative error and max|a - b| / max|b| both within tol."""
    e = rel(a, b)
    em = float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))
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


def make_jobs(ctx, specs, prec, seed, hess="auto"):
    import torch
    nets, bufs, data = [], [], []
    for k, (dims, npts) in enumerate(specs):
        acts = ["softplus"] * (len(dims) - 2) + ["identity"]
        Ws, bs = datagen.mlp_weights(dims, seed=seed + k, bias_scale=0.05)
        X, Lam = datagen.surrogate_points(dims[0], dims[-1], npts, seed=seed + 100 + k)
        net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=npts, hess=hess)
        x = torch.as_tensor(X, device="cuda")
        lam = torch.as_tensor(Lam, device="cuda")
        g = torch.empty(npts, dims[-1], dtype=torch.float64, device="cuda")
        J = torch.empty(npts, dims[-1], dims[0], dtype=torch.float64, device="cuda")
        H = torch.empty(npts, dims[0], dims[0], dtype=torch.float64, device="cuda")
        nets.append(net)
        bufs.append(dict(x=x, lam=lam, g=g, J=J, H=H))
        data.append((dims, acts, Ws, bs, X, Lam))
    jobs = [dict(net=n.h, B=b["x"].shape[0], x=b["x"].data_ptr(), lam=b["lam"].data_ptr(),
                 obj_factor=0.0, g=b["g"].data_ptr(), J=b["J"].data_ptr(), H=b["H"].data_ptr())
            for n, b in zip(nets, bufs)]
    return nets, bufs, data, jobs


SPECS = [((120, 64, 64, 4), 8), ((120, 128, 128, 128, 4), 16), ((120, 256, 256, 256, 256, 4), 20)]


@pytest.mark.parametrize("hess", ["auto", "for", "layersum"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-10), ("bf16", 2e-2)])
def test_batch_matches_oracle(ctx, prec, tol, hess):
    """Three networks of different depths and widths in one batched call
    (with "auto" the first picks forward-over-reverse and the other two the
    layer sum, so one H launch holds both kinds of product)."""
    import torch
    nets, bufs, data, jobs = make_jobs(ctx, SPECS, prec, seed=50, hess=hess)
    assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
    torch.cuda.synchronize()
    for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
        H = b["H"].cpu().numpy()
        J = b["J"].cpu().numpy()
        g = b["g"].cpu().numpy()
        for p in (0, X.shape[0] - 1):
            close(g[p], O.nn(Ws, bs, acts, X[p]), tol, (dims, "g", p))
            close(J[p], O.jacobian(Ws, bs, acts, X[p]), tol, (dims, "J", p))
            Hr = O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1])[0]
            close(H[p], Hr, tol, (dims, "H", p))
    for n in nets:
        n.destroy()


def test_graph_replay_bitwise_and_input_updates(ctx):
    import torch
    nets, bufs, data, jobs = make_jobs(ctx, SPECS, "fp32", seed=60)
    assert nnc.nnc_eval_batch(ctx.h, jobs) == 0
    torch.cuda.synchronize()
    first = [b["H"].clone() for b in bufs]
    # eager single-network results on the same inputs (same kernels, other grid)
    for n, b in zip(nets, bufs):
        He = n.eval_hess_lag(b["x"], b["lam"])
        torch.cuda.synchronize()
        assert rel(first[nets.index(n)].cpu().numpy(), He.cpu().numpy()) < 1e-6
    for rep in range(4):
        for b in bufs:
            b["H"].zero_()
        torch.cuda.synchronize()
        assert nnc.nnc_eval_batch(ctx.h, jobs) == 0  # replay of the captured graph
        torch.cuda.synchronize()
        for b, f in zip(bufs, first):
            assert torch.equal(b["H"], f), f"replay {rep} differs"
        _ = bufs[0]["x"].sum().item()  # eager work between replays
    # new values in the same buffers: the replay must see them
    for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
        X2 = np.clip(X + 0.05, 0.0, 1.5)
        b["x"].copy_(torch.as_tensor(X2, device="cuda"))
        b["X2"] = X2
    assert nnc.nnc_eval_batch(ctx.h, jobs) == 0
    torch.cuda.synchronize()
    for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
        H = b["H"].cpu().numpy()
        Hr = O.hess_lag(Ws, bs, acts, b["X2"][:1], Lam[:1])[0]
        assert rel(H[0], Hr) < 1e-5
    # a different job list re-captures
    jobs2 = [dict(j) for j in jobs[:2]]
    jobs2[1]["B"] = 5
    assert nnc.nnc_eval_batch(ctx.h, jobs2) == 0
    torch.cuda.synchronize()
    dims, acts, Ws, bs, X, Lam = data[1]
    H = bufs[1]["H"].cpu().numpy()
    Hr = O.hess_lag(Ws, bs, acts, bufs[1]["X2"][4:5], Lam[4:5])[0]
    assert rel(H[4], Hr) < 1e-5
    for n in nets:
        n.destroy()


def test_batch_argument_errors(ctx):
    nets, bufs, data, jobs = make_jobs(ctx, SPECS[:2], "fp32", seed=70)
    bad = [dict(j) for j in jobs]
    bad[0]["B"] = 999
    assert nnc.nnc_eval_batch(ctx.h, bad) == nnc.NNC_E_SHAPE
    dup = [dict(jobs[0]), dict(jobs[0])]
    assert nnc.nnc_eval_batch(ctx.h, dup) == nnc.NNC_E_ARG
    nolam = [dict(jobs[0])]
    nolam[0]["lam"] = 0
    assert nnc.nnc_eval_batch(ctx.h, nolam) == nnc.NNC_E_ARG
    assert nnc.nnc_eval_batch(ctx.h, []) == nnc.NNC_OK
    for n in nets:
        n.destroy()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_surrogate_workload_full_size(ctx, prec, tol):
    """The three softplus surrogates (120 -> 512x4 / 1024x6 / 2048x8 -> 4) at
    64, 512 and 1024 points in one batched call (g, J and H requested): the
    first, middle and last point of every net against the oracle, whole
    g, J and H, normwise and elementwise."""
    import torch
    specs = [(datagen.C3_DIMS[k], datagen.C3_POINTS[k]) for k in ("A", "B", "C")]
    nets, bufs, data, jobs = make_jobs(ctx, specs, prec, seed=0)
    assert nnc.nnc_eval_batch(ctx.h, jobs) == 0, nnc.nnc_last_error(ctx.h)
    torch.cuda.synchronize()
    for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
        g = b["g"].cpu().numpy()
        J = b["J"].cpu().numpy()
        H = b["H"].cpu().numpy()
        for p in (0, X.shape[0] // 2, X.shape[0] - 1):
            close(g[p], O.nn(Ws, bs, acts, X[p]), tol, (dims, "g", p))
            close(J[p], O.jacobian(Ws, bs, acts, X[p]), tol, (dims, "J", p))
            Hr = O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1])[0]
            close(H[p], Hr, tol, (dims, "H", p))
    for n in nets:
        n.destroy()


def test_batch_replans_after_autotune(ctx):
    """A batch graph captured before nnc_autotune (which can grow the K-split
    workspace and changes tilings) is not replayed afterwards: the same job
    list re-plans, and the results still match the oracle."""
    import torch
    nets, bufs, data, jobs = make_jobs(ctx, SPECS, "fp32", seed=95)
    code = nnc.PREC_CODES["fp32"]
    try:
        assert nnc.nnc_set_gemm_ksplit(ctx.h, code, 2) == nnc.NNC_OK  # small workspace, K-split GEMMs
        assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
        torch.cuda.synchronize()
        assert nnc.nnc_set_gemm_ksplit(ctx.h, code, -1) == nnc.NNC_OK
        for n, b in zip(nets, bufs):
            assert nnc.nnc_autotune(ctx.h, n.h, b["x"].shape[0]) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
        for b in bufs:
            b["H"].zero_()
        assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
        torch.cuda.synchronize()
        for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
            H = b["H"].cpu().numpy()
            for p in (0, X.shape[0] - 1):
                close(H[p], O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1])[0], 1e-5, (dims, p))
    finally:
        nnc.nnc_set_gemm_ksplit(ctx.h, code, -1)
    for n in nets:
        n.destroy()


def test_batch_objective_diag_change_replans(ctx):
    """Changing a network's registered objective diagonal between two batched
    calls with identical job lists: the second call uses the new diagonal."""
    import torch
    nets, bufs, data, jobs = make_jobs(ctx, SPECS[:2], "fp32", seed=96)
    for j in jobs:
        j["obj_factor"] = 0.5
    q1 = torch.linspace(1.0, 2.0, 120, dtype=torch.float64, device="cuda")
    q2 = torch.linspace(-3.0, 0.5, 120, dtype=torch.float64, device="cuda")
    for q in (q1, q2):
        for n in nets:
            n.set_objective_diag(q)
        assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
        torch.cuda.synchronize()
        qh = q.cpu().numpy()
        for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
            H = b["H"].cpu().numpy()
            p = X.shape[0] - 1
            Hr = O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1], obj_factor=0.5, q=qh)[0]
            close(H[p], Hr, 1e-5, (dims, p))
    for n in nets:
        n.destroy()


@pytest.mark.parametrize("hess", ["for", "layersum"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_batch_every_grouped_tiling(ctx, prec, tol, hess):
    """Every tiling forced on the batched sweep launches (register-staged and
    LDS-DMA-staged grouped kernels; a tiling the grouped kernel lacks falls
    back to the default one), against the oracle."""
    import torch
    code = nnc.PREC_CODES[prec]
    nets, bufs, data, jobs = make_jobs(ctx, SPECS, prec, seed=80, hess=hess)
    try:
        for cfg in range(nnc.nnc_gemm_config_count()):
            nnc.nnc_set_gemm_config(ctx.h, code, cfg)
            for b in bufs:
                b["H"].zero_()
            assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
            torch.cuda.synchronize()
            for (dims, acts, Ws, bs, X, Lam), b in zip(data, bufs):
                H = b["H"].cpu().numpy()
                p = X.shape[0] - 1
                Hr = O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1])[0]
                assert rel(H[p], Hr) < tol, (cfg, dims, rel(H[p], Hr))
    finally:
        nnc.nnc_set_gemm_config(ctx.h, code, -1)
    for n in nets:
        n.destroy()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_batch_persistent_items_every_tiling(ctx, prec, tol):
    """Two 120 -> 1024 -> 1024 -> 4 nets at 64 points (7680 tangent rows):
    each batched sweep launch holds more tiles than the persistent grid has
    workgroups, so workgroups walk several work items and refill their LDS
    stages between items.  Every tiling forced, sampled points vs the oracle."""
    import torch
    code = nnc.PREC_CODES[prec]
    specs = [((120, 1024, 1024, 4), 64), ((120, 1024, 1024, 4), 64)]
    nets, bufs, data, jobs = make_jobs(ctx, specs, prec, seed=90)
    for j in jobs:
        j["J"] = 0
    refs = [{p: O.hess_lag(Ws, bs, acts, X[p:p + 1], Lam[p:p + 1])[0] for p in (0, 37, 63)}
            for (dims, acts, Ws, bs, X, Lam) in data]
    try:
        for cfg in range(nnc.nnc_gemm_config_count()):
            nnc.nnc_set_gemm_config(ctx.h, code, cfg)
            for b in bufs:
                b["H"].zero_()
            assert nnc.nnc_eval_batch(ctx.h, jobs) == nnc.NNC_OK, nnc.nnc_last_error(ctx.h)
            torch.cuda.synchronize()
            for ref, b in zip(refs, bufs):
                H = b["H"].cpu().numpy()
                for p, Hr in ref.items():
                    assert rel(H[p], Hr) < tol, (cfg, p, rel(H[p], Hr))
    finally:
        nnc.nnc_set_gemm_config(ctx.h, code, -1)
    for n in nets:
        n.destroy()
