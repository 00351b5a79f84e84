"""Benchmark: Hessian-of-Lagrangian evaluations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|bf16|fp64]

Workload: the 137M-parameter tanh MLP 784 -> 4096 -> 8192 -> 8192 -> 4096 -> 10
(weights N(0, 1/fan_in), biases 0, seed 0), one point x ~ U[0,1)^784 and
lambda ~ N(0,1)^10.  One step is one interior-point iteration's oracle set at
that point: g, J and the Hessian of the Lagrangian from one nnc_eval call
(forward pass, FP64 output layer, Jacobian, FP64 adjoint, forward- and
reverse-tangent MFMA sweeps, FP64 H accumulation, finalize; the primal
forward pass is shared by the three).  Inputs are device-resident before
timing.

Prints one JSON line.  ``roofline`` describes the dominant kernel (the MFMA
tangent GEMM): algorithmic flops per launch / average launch time measured
with HIP events on the library's stream over the timed region.
``cpu_baseline`` times the FP64 numpy oracle on the host on a bounded sample
of the same workload (and reports the GPU result's error against it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp64": 78.6}  # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
DIMS = (784, 4096, 8192, 8192, 4096, 10)
ACTS = ["tanh", "tanh", "tanh", "tanh", "identity"]


def sweep_flops(dims, identity_out=True, method="for"):
    """Algorithmic flops of the tangent-sweep GEMMs (n seeds): forward and
    reverse sweeps for forward-over-reverse, the forward sweep alone for the
    layer sum."""
    n = dims[0]
    Lt = len(dims) - 2 if identity_out else len(dims) - 1
    per_sweep = 2.0 * n * sum(dims[l] * dims[l - 1] for l in range(2, Lt + 1))
    return per_sweep if method == "layersum" else 2.0 * per_sweep


def hprod_flops(dims, identity_out=True, method="for"):
    """Algorithmic flops of the final H product: H = G_1 W_1 (n x n x d_1)
    for forward-over-reverse; for the layer sum the n(n+1)/2 entries on and
    below the diagonal of sum_l T_l^T diag(s_l) T_l (2 sum_l d_l flops each)."""
    n = dims[0]
    Lt = len(dims) - 2 if identity_out else len(dims) - 1
    if method == "layersum":
        return float(n) * (n + 1) * sum(dims[l] for l in range(1, Lt + 1))
    return 2.0 * n * n * dims[1]


def hess_flops(dims, identity_out=True, method="for"):
    """Algorithmic flops of one n x n Hessian by the given method (sweeps
    plus the final product)."""
    return sweep_flops(dims, identity_out, method) + hprod_flops(dims, identity_out, method)


def weight_bytes(dims, esize):
    return sum(dims[l] * dims[l - 1] for l in range(1, len(dims))) * esize


def gemm_source_sha():
    """Digest of what decides the sweep GEMMs' memory traffic: the GEMM kernel
    sources and the committed tiling table."""
    pkg = os.path.join(ROOT, "paper_2509_22462_amd")
    h = hashlib.sha256()
    for rel in ("csrc/gemm.hip", "csrc/gemm_kernels.h", "csrc/gemm_dma.hip", "csrc/gemm_common.h",
                "tuning/gfx950.jsonl"):
        h.update(open(os.path.join(pkg, rel), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(prec, flops_per_launch_bytes=None):
    """HBM traffic per GEMM launch from committed PMC counter runs, if current."""
    p = os.path.join(ROOT, "profiles", f"gemm_c2_{prec}_traffic.json")  # PMC FETCH/WRITE_SIZE
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("gemm_source_sha") != gemm_source_sha():
        return None
    return d.get("bytes_per_launch")


def load_mfma_busy(prec, key="mfma_busy_pct"):
    """MFMA-busy percentage from a committed rocprofv3 counter run
    (SQ_VALU_MFMA_BUSY_CYCLES), if the GEMM sources are unchanged since: of the
    sweep GEMM (mfma_busy_pct) or of all kernels of one evaluation
    (whole_eval_mfma_busy_pct)."""
    p = os.path.join(ROOT, "profiles", "gemm_c2_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("gemm_source_sha") != gemm_source_sha():
        return None
    return d.get(key, {}).get(prec)


def time_gpu(prec, steps, warmup, Ws, bs, X, Lam, autotune=True, hess="auto"):
    import torch

    from paper_2509_22462_amd import nnc

    P = X.shape[0]
    ctx = nnc.Context(0)
    net = ctx.net(DIMS, ACTS, Ws, bs, prec=prec, max_points=P, hess=hess)
    method = net.hess_method
    if autotune:  # set-up: pick the GEMM tilings for these shapes
        rc = nnc.nnc_autotune(ctx.h, net.h, P)
        if rc:
            raise RuntimeError(nnc.nnc_last_error(ctx.h))
    dev = ctx.device
    x = torch.as_tensor(X, device=dev)
    lam = torch.as_tensor(Lam, device=dev)
    g = torch.empty(P, DIMS[-1], dtype=torch.float64, device=dev)
    J = torch.empty(P, DIMS[-1], DIMS[0], dtype=torch.float64, device=dev)
    H = torch.empty(P, DIMS[0], DIMS[0], dtype=torch.float64, device=dev)

    def step():
        # g, J and H at the same points, one call (one primal forward pass)
        rc = nnc.nnc_eval(ctx.h, net.h, P, x.data_ptr(), None, 0.0, lam.data_ptr(), g.data_ptr(),
                          J.data_ptr(), H.data_ptr())
        if rc:
            raise RuntimeError(nnc.nnc_last_error(ctx.h))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events only around the dominant kernel's launches
    # (the sweep GEMMs; every recorded launch adds two queue markers)
    nnc.nnc_profile_classes(ctx.h, 1 << nnc.NNC_KC_GEMM)
    nnc.nnc_profile(ctx.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nnc.nnc_profile(ctx.h, False)
    gemm_ms, gemm_n = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM)
    # per-class breakdown from a separate profiled pass (all classes)
    nb = max(3, min(steps, 10))
    nnc.nnc_profile_classes(ctx.h, 0xF)
    nnc.nnc_profile(ctx.h, True)
    for _ in range(nb):
        step()
    nnc.nnc_profile(ctx.h, False)
    scale = steps / nb  # breakdown totals expressed per timed run
    h_ms, h_n = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM_H)
    sk_ms, sk_n = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_SKINNY)
    ot_ms, ot_n = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_OTHER)
    h_ms, sk_ms, ot_ms = h_ms * scale, sk_ms * scale, ot_ms * scale
    h_n, sk_n, ot_n = int(h_n * scale), int(sk_n * scale), int(ot_n * scale)

    # After the timed region: per-step latency spread (each step synchronised),
    # the single-oracle rates, and the device-to-host copy of H that a host
    # solver adds per iteration (not part of `value`).
    lat = []
    for _ in range(min(steps, 20)):
        s0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - s0) * 1e3)

    def rate(**outs):
        n = max(5, min(steps, 20))
        ptr = {k: (v.data_ptr() if v is not None else None) for k, v in outs.items()}
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(n):
            rc = nnc.nnc_eval(ctx.h, net.h, P, x.data_ptr(), None, 0.0, ptr.get("lam"), ptr.get("g"),
                              ptr.get("J"), ptr.get("H"))
            if rc:
                raise RuntimeError(nnc.nnc_last_error(ctx.h))
        torch.cuda.synchronize()
        return round(P * n / (time.perf_counter() - s0), 1)

    Hh = torch.empty(H.shape, dtype=H.dtype, pin_memory=True)
    Hh.copy_(H)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(10):
        Hh.copy_(H)
    torch.cuda.synchronize()
    d2h_ms = (time.perf_counter() - s0) / 10 * 1e3
    extra = dict(step_ms_p10=round(float(np.percentile(lat, 10)), 4),
                 step_ms_p50=round(float(np.percentile(lat, 50)), 4),
                 step_ms_p90=round(float(np.percentile(lat, 90)), 4),
                 g_evals_per_s=rate(g=g), jac_evals_per_s=rate(J=J),
                 hess_evals_per_s=rate(lam=lam, H=H),
                 h_d2h_ms=round(d2h_ms, 4), h_d2h_gb_per_s=round(H.numel() * 8 / (d2h_ms * 1e-3) / 1e9, 2))
    out = dict(
        extra=extra, method=method,
        seconds=t1 - t0, steps=steps, gemm_ms=gemm_ms, gemm_launches=gemm_n, h_ms=h_ms, h_launches=h_n,
        skinny_ms=sk_ms,
        skinny_launches=sk_n, other_ms=ot_ms, other_launches=ot_n,
        g=g.cpu().numpy()[0], J=J.cpu().numpy()[0], H=H.cpu().numpy()[0])
    net.destroy()
    ctx.close()
    return out


def bench_surrogates(steps, warmup, prec="fp32", autotune=False):
    """Three softplus surrogates (120 -> 512x4 / 1024x6 / 2048x8 -> 4) at
    64 / 512 / 1024 points in one batched call (graph replay per step).
    The grouped launches take the tiling the table holds for their largest
    product; --autotune re-tunes each network's shapes first (set-up)."""
    import torch

    from paper_2509_22462_amd import datagen, nnc

    ctx = nnc.Context(0)
    jobs, keep, flops, pts = [], [], 0.0, 0
    methods = {}
    for k in ("A", "B", "C"):
        dims = datagen.C3_DIMS[k]
        B = datagen.C3_POINTS[k]
        acts = ["softplus"] * (len(dims) - 2) + ["identity"]
        Ws, bs = datagen.mlp_weights(dims, seed=0)
        X, Lam = datagen.surrogate_points(dims[0], dims[-1], B, seed=1003)
        net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=B)
        if autotune:
            assert nnc.nnc_autotune(ctx.h, net.h, B) == 0, nnc.nnc_last_error(ctx.h)
        x = torch.as_tensor(X, device="cuda")
        lam = torch.as_tensor(Lam, device="cuda")
        H = torch.empty(B, dims[0], dims[0], dtype=torch.float64, device="cuda")
        g = torch.empty(B, dims[-1], dtype=torch.float64, device="cuda")
        J = torch.empty(B, dims[-1], dims[0], dtype=torch.float64, device="cuda")
        keep += [net, x, lam, H, g, J]
        jobs.append(dict(net=net.h, B=B, x=x.data_ptr(), lam=lam.data_ptr(), obj_factor=0.0,
                         g=g.data_ptr(), J=J.data_ptr(), H=H.data_ptr()))
        flops += B * hess_flops(dims, method=net.hess_method)
        methods[k] = net.hess_method
        pts += B
    for _ in range(warmup):
        assert nnc.nnc_eval_batch(ctx.h, jobs) == 0, nnc.nnc_last_error(ctx.h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        nnc.nnc_eval_batch(ctx.h, jobs)
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = e0.elapsed_time(e1) / steps
    # after the timed region: each network once through the eager path, per
    # kernel class (where the time of a batched call goes outside the GEMMs)
    eager = {}
    nets = [keep[i] for i in range(0, len(keep), 6)]
    for k, net, j in zip(("A", "B", "C"), nets, jobs):
        nnc.nnc_profile_classes(ctx.h, 0xF)
        nnc.nnc_profile(ctx.h, True)
        rc = nnc.nnc_eval(ctx.h, net.h, j["B"], j["x"], None, 0.0, j["lam"], j["g"], j["J"], j["H"])
        assert rc == 0, nnc.nnc_last_error(ctx.h)
        nnc.nnc_profile(ctx.h, False)
        eager[k] = {name: round(nnc.nnc_profile_read(ctx.h, cls)[0], 3)
                    for name, cls in (("sweep_gemm_ms", nnc.NNC_KC_GEMM), ("h_gemm_ms", nnc.NNC_KC_GEMM_H),
                                      ("stream_ms", nnc.NNC_KC_SKINNY), ("other_ms", nnc.NNC_KC_OTHER))}
    out = dict(workload="softplus surrogates 120-512x4-4 (64 pts), 120-1024x6-4 (512 pts), "
                        "120-2048x8-4 (1024 pts): g, J, H per point, one batched call",
               precision=prec, points_per_call=pts, ms_per_call=round(ms, 3),
               h_evals_per_s=round(pts / (ms * 1e-3), 1), wall_s=round(t1 - t0, 3),
               tflops=round(flops / (ms * 1e-3) / 1e12, 2),
               frac=round(flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec], 4),
               hess_tflop_per_call=round(flops / 1e12, 3), hess_method=methods, eager_per_net=eager)
    ctx.close()
    return out


def bench_sweep(steps, warmup, points=32, h_sample=4, autotune=True):
    """Precision sweep on the 137M-parameter MLP: `points` points per call,
    BF16 / FP32 / FP64 GEMMs (FP64 residual, adjoint and H accumulation in
    all), throughput and normwise error of g, J (all points) and H (a sample
    of points) against the FP64 oracle."""
    import torch

    from oracle import nn as O
    from paper_2509_22462_amd import datagen, nnc

    Ws, bs = datagen.mlp_weights(DIMS, seed=0)
    X, Lam = datagen.points(784, 10, points, seed=1004)
    ref_g = np.stack([O.nn(Ws, bs, ACTS, x) for x in X])
    ref_J = np.stack([O.jacobian_reverse(Ws, bs, ACTS, x) for x in X])
    ref_H = [O.hess_for(Ws, bs, ACTS, X[p], Lam[p]) for p in range(h_sample)]

    def rel(u, v):
        return float(np.linalg.norm(u - v) / np.linalg.norm(v))

    out = {}
    for prec in ("bf16", "fp32", "fp64"):
        ctx = nnc.Context(0)
        net = ctx.net(DIMS, ACTS, Ws, bs, prec=prec, max_points=points)
        FHp = hess_flops(DIMS, method=net.hess_method)
        if autotune:
            assert nnc.nnc_autotune(ctx.h, net.h, points) == 0, nnc.nnc_last_error(ctx.h)
        x = torch.as_tensor(X, device="cuda")
        lam = torch.as_tensor(Lam, device="cuda")
        g = torch.empty(points, 10, dtype=torch.float64, device="cuda")
        J = torch.empty(points, 10, 784, dtype=torch.float64, device="cuda")
        H = torch.empty(points, 784, 784, dtype=torch.float64, device="cuda")

        def step():
            rc = nnc.nnc_eval(ctx.h, net.h, points, x.data_ptr(), None, 0.0, lam.data_ptr(),
                              g.data_ptr(), J.data_ptr(), H.data_ptr())
            assert rc == 0, nnc.nnc_last_error(ctx.h)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        nnc.nnc_profile_classes(ctx.h, (1 << nnc.NNC_KC_GEMM) | (1 << nnc.NNC_KC_GEMM_H))
        nnc.nnc_profile(ctx.h, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nnc.nnc_profile(ctx.h, False)
        nnc.nnc_profile_classes(ctx.h, 0xF)
        gm, gn = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM)
        hm, hn = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM_H)
        gh, Jh, Hh = g.cpu().numpy(), J.cpu().numpy(), H.cpu().numpy()
        out[prec] = dict(
            h_evals_per_s=round(points * steps / dt, 2), ms_per_call=round(dt / steps * 1e3, 3),
            hess_method=net.hess_method,
            mfma_tflops=round(points * FHp * steps / ((gm + hm) * 1e-3) / 1e12, 2),
            mfma_frac=round(points * FHp * steps / ((gm + hm) * 1e-3) / 1e12
                            / PEAK_TFLOPS[prec], 4),
            rel_err_g_max=max(rel(gh[p], ref_g[p]) for p in range(points)),
            rel_err_J_max=max(rel(Jh[p], ref_J[p]) for p in range(points)),
            rel_err_H_max=max(rel(Hh[p], ref_H[p]) for p in range(h_sample)),
            rel_err_H_median=float(np.median([rel(Hh[p], ref_H[p]) for p in range(h_sample)])))
        net.destroy()
        ctx.close()
    return dict(workload=f"precision sweep: tanh MLP 784-4096-8192-8192-4096-10, {points} points, "
                         "step = g + J + H", points=points, h_error_sample=h_sample, results=out)


def bench_scopf(steps, warmup, precs=("fp32", "bf16")):
    """The deep, narrow surrogate shape (117 -> 4000 x 38 -> 37 tanh, 592.6M
    weights) at one point: step = g + J + H (nnc_eval), committed tiling
    table; the sweep GEMMs (37 sequential products at 117 tangent columns)
    timed with HIP events on the library's stream."""
    import torch

    from paper_2509_22462_amd import datagen, nnc

    dims = datagen.SCOPF_DIMS
    acts = ["tanh"] * 38 + ["identity"]
    Ws, bs = datagen.mlp_weights(dims, seed=0)
    X, Lam = datagen.scopf_points(1, seed=1006)
    out = {}
    for prec in precs:
        ctx = nnc.Context(0)
        net = ctx.net(dims, acts, Ws, bs, prec=prec, max_points=1)
        method = net.hess_method
        x = torch.as_tensor(X, device="cuda")
        lam = torch.as_tensor(Lam, device="cuda")
        g = torch.empty(1, 37, dtype=torch.float64, device="cuda")
        J = torch.empty(1, 37, 117, dtype=torch.float64, device="cuda")
        H = torch.empty(1, 117, 117, dtype=torch.float64, device="cuda")

        def step():
            rc = nnc.nnc_eval(ctx.h, net.h, 1, x.data_ptr(), None, 0.0, lam.data_ptr(), g.data_ptr(),
                              J.data_ptr(), H.data_ptr())
            assert rc == 0, nnc.nnc_last_error(ctx.h)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        nnc.nnc_profile_classes(ctx.h, (1 << nnc.NNC_KC_GEMM) | (1 << nnc.NNC_KC_GEMM_H) | (1 << nnc.NNC_KC_SKINNY))
        nnc.nnc_profile(ctx.h, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nnc.nnc_profile(ctx.h, False)
        nnc.nnc_profile_classes(ctx.h, 0xF)
        gm, gn = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM)
        hm, _ = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_GEMM_H)
        sm, _ = nnc.nnc_profile_read(ctx.h, nnc.NNC_KC_SKINNY)
        fs = sweep_flops(dims, method=method)
        ach = fs * steps / (gm * 1e-3) / 1e12
        esz = {"fp32": 4, "bf16": 2, "fp64": 8}[prec]
        out[prec] = dict(h_evals_per_s=round(steps / dt, 2), ms_per_step=round(dt / steps * 1e3, 3),
                         hess_method=method, sweep_gemm_ms_per_step=round(gm / steps, 4),
                         sweep_gemm_tflops=round(ach, 2), sweep_gemm_frac=round(ach / PEAK_TFLOPS[prec], 4),
                         h_product_ms_per_step=round(hm / steps, 4),
                         stream_ms_per_step=round(sm / steps, 4),
                         stream_tb_per_s=round(2 * weight_bytes(dims, esz) / (sm / steps * 1e-3) / 1e12, 2))
        net.destroy()
        ctx.close()
    return dict(workload="tanh MLP 117-4000x38-37 (592.6M weights), 1 point, step = g + J + H",
                hess_gflop_per_eval=round(hess_flops(dims, method=out[precs[0]]["hess_method"]) / 1e9, 2),
                results=out)


MFMA_KIND = {"fp32": "fp32_16x16x4", "bf16": "bf16_16x16x32", "fp64": "fp64_16x16x4"}


def measured_ceilings(nbytes=1 << 30, reps=3):
    """The MFMA rates and HBM stream rates that plain loops reach on this GPU
    (nnc_peak_mfma / nnc_peak_hbm): the measured ceilings beside the datasheet
    peaks.  Each MFMA shape is timed twice and the faster run kept."""
    import torch
    from paper_2509_22462_amd import nnc
    ctx = nnc.Context(0)
    try:
        mfma = {}
        for kind in nnc.PEAK_KINDS:
            iters = 2000 if kind.startswith("bf16") else 500
            mfma[kind] = round(max(nnc.nnc_peak_mfma(ctx.h, kind, iters) for _ in range(2)), 1)
        src = torch.full((nbytes // 4,), 7, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        rd, cp = nnc.nnc_peak_hbm(ctx.h, src.data_ptr(), dst.data_ptr(), nbytes, reps)
        del src, dst
    finally:
        ctx.close()
    return dict(mfma_tflops=mfma, hbm_read_gb_per_s=round(rd, 1), hbm_copy_gb_per_s=round(cp, 1),
                note=f"plain-loop probes: 16 waves/CU of independent MFMA chains; grid-stride 16-byte loads over "
                     f"{nbytes >> 20} MiB (read; copy counts read + write bytes)")


def bench_kkt(reps=20, n=784, batches=(1, 64)):
    """Device Newton step (nnc_kkt_solve: assemble M = H + diag(d) + s a a^T,
    FP64 Cholesky, two triangular solves) against the host route it replaces
    (copy H to pinned host memory, numpy Cholesky and solve), at the 137M
    net's n = 784, per system."""
    import torch

    from paper_2509_22462_amd import nnc

    rng = np.random.default_rng(5)
    ctx = nnc.Context(0)
    out = {}
    for B in batches:
        G = rng.standard_normal((B, n, n)) / np.sqrt(n)
        H = 0.5 * (G + G.transpose(0, 2, 1))
        d = 2.0 + rng.random((B, n))
        a = rng.standard_normal((B, n)) / np.sqrt(n)
        sv = rng.random(B)
        r = rng.standard_normal((B, n))
        dev = lambda v: torch.as_tensor(np.ascontiguousarray(v), device="cuda")
        Ht, dt, at, st, rt = dev(H), dev(d), dev(a), dev(sv), dev(r)
        dx = torch.empty(B, n, dtype=torch.float64, device="cuda")
        info = torch.empty(B, dtype=torch.int32, device="cuda")
        kkt = nnc.nnc_kkt_create(ctx.h, n, B)

        def solve():
            rc = nnc.nnc_kkt_solve(ctx.h, kkt, B, Ht.data_ptr(), dt.data_ptr(), at.data_ptr(), st.data_ptr(), None,
                                   rt.data_ptr(), dx.data_ptr(), info.data_ptr())
            assert rc == 0, nnc.nnc_last_error(ctx.h)

        solve()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            solve()
        e1.record()
        torch.cuda.synchronize()
        dev_ms = e0.elapsed_time(e1) / reps
        assert int(info.abs().sum().item()) == 0
        # host route: H to pinned memory, Cholesky and two solves per system
        Hh = torch.empty(B, n, n, dtype=torch.float64, pin_memory=True)
        hreps = max(2, min(reps, 200 // B))
        t0 = time.perf_counter()
        for _ in range(hreps):
            Hh.copy_(Ht)
            Hn = Hh.numpy()
            for b in range(B):
                M = Hn[b] + np.diag(d[b]) + sv[b] * np.outer(a[b], a[b])
                Lc = np.linalg.cholesky(M)
                np.linalg.solve(Lc.T, np.linalg.solve(Lc, r[b]))
        host_ms = (time.perf_counter() - t0) / hreps * 1e3
        ref = np.linalg.solve(H[0] + np.diag(d[0]) + sv[0] * np.outer(a[0], a[0]), r[0])
        err = float(np.linalg.norm(dx.cpu().numpy()[0] - ref) / np.linalg.norm(ref))
        out[f"B{B}"] = dict(device_ms=round(dev_ms, 4), device_ms_per_system=round(dev_ms / B, 4),
                            host_ms=round(host_ms, 3), host_ms_per_system=round(host_ms / B, 4),
                            rel_err_vs_numpy=err)
        nnc.nnc_kkt_destroy(ctx.h, kkt)
    ctx.close()
    return dict(workload=f"reduced Newton system n = {n} (dense FP64 SPD), device Cholesky vs host numpy "
                         "(H copied to pinned host memory)", results=out)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def cpu_baseline(Ws, bs, X, Lam, budget_s=12.0, max_steps=5, other_configs=True):
    """Time the FP64 oracle (g, J, H at the same point) on the host cores:
    the headline workload as a bounded sample, then one oracle step per point
    of the other workloads (small net, each surrogate net), and the headline
    step again with BLAS on one thread."""
    from oracle import nn as O
    from paper_2509_22462_amd import datagen
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = cores
    t0 = time.perf_counter()
    done = 0
    res = None
    while done < max_steps and (time.perf_counter() - t0) < budget_s:
        g = O.nn(Ws, bs, ACTS, X[0])
        J = O.jacobian_reverse(Ws, bs, ACTS, X[0])
        H = O.hess_for(Ws, bs, ACTS, X[0], Lam[0])
        done += 1
        res = (g, J, H)
    dt = time.perf_counter() - t0
    out = dict(value=done / dt, unit="H evals/s", cores=int(min(cores, blas_threads)), kind="oracle",
               sample=f"{done} oracle steps (g, J, H by forward-over-reverse) at one point of the "
                      "137M-param MLP, FP64 numpy",
               seconds=dt, affinity_cores=cores, blas_threads=int(blas_threads), cpu_model=cpu_model())

    def step_seconds(dims, acts, x, lam, reps):
        Wc, bc = datagen.mlp_weights(dims, seed=0)
        t = time.perf_counter()
        for _ in range(reps):
            O.nn(Wc, bc, acts, x)
            O.jacobian_reverse(Wc, bc, acts, x)
            O.hess_for(Wc, bc, acts, x, lam)
        return (time.perf_counter() - t) / reps

    if other_configs:
        per = {}
        x1, l1 = datagen.points(784, 10, 1, seed=1001)
        per["tanh 784-64-64-10 (1 point)"] = step_seconds(datagen.C1_DIMS, ["tanh", "tanh", "identity"],
                                                          x1[0], l1[0], 5)
        for k in ("A", "B", "C"):
            dims = datagen.C3_DIMS[k]
            xs, ls = datagen.surrogate_points(dims[0], dims[-1], 1, seed=1003)
            acts = ["softplus"] * (len(dims) - 2) + ["identity"]
            name = f"softplus {dims[0]}-{dims[1]}x{len(dims) - 2}-{dims[-1]} (per point)"
            per[name] = step_seconds(dims, acts, xs[0], ls[0], 3)
        per["137M MLP, 32-point sweep (per point)"] = dt / max(done, 1)
        out["seconds_per_step"] = {k: round(v, 5) for k, v in per.items()}
    # the same step on one core (BLAS limited to one thread)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            O.nn(Ws, bs, ACTS, X[0])
            O.jacobian_reverse(Ws, bs, ACTS, X[0])
            O.hess_for(Ws, bs, ACTS, X[0], Lam[0])
            d1 = time.perf_counter() - t1
        out["single_core"] = dict(value=round(1.0 / d1, 4), cores=1, seconds=round(d1, 3),
                                  sample="1 oracle step (g, J, H), BLAS on one thread")
    except ImportError:  # pragma: no cover
        pass
    return out, res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--variants", default="bf16,fp64",
                    help="other precisions to time briefly (comma list, '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the surrogate-batch and 32-point precision-sweep keys of the default line")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune the GEMM tilings live (default: the committed gfx950 table)")
    ap.add_argument("--hess", default="auto", choices=["auto", "for", "layersum"],
                    help="Hessian method (auto: the cheaper by algorithmic flops; layer sum here)")
    ap.add_argument("--points", type=int, default=1,
                    help="points per call (the headline workload is 1)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the MFMA / HBM ceiling probes (nnc_peak_mfma, nnc_peak_hbm)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", default="mlp137m", choices=["mlp137m", "surrogates", "sweep", "scopf"],
                    help="surrogates: the batched three-network workload (extra report, "
                         "not the headline line)")
    a = ap.parse_args(argv)
    from paper_2509_22462_amd import nnc as _nnc
    if a.autotune:
        os.environ.setdefault("NNC_AUTOTUNE_CACHE", os.path.join("/tmp", "nnc_tune.jsonl"))
    else:
        os.environ.setdefault("NNC_AUTOTUNE_CACHE", _nnc.TUNED_TABLE)
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    if a.workload == "surrogates":
        print(json.dumps(bench_surrogates(a.steps, a.warmup, a.prec, autotune=a.autotune)), flush=True)
        return 0
    if a.workload == "sweep":
        print(json.dumps(bench_sweep(a.steps, a.warmup, autotune=a.autotune)), flush=True)
        return 0
    if a.workload == "scopf":
        if a.autotune:  # set-up: tune the 117-column sweep shapes, then time
            from paper_2509_22462_amd import datagen, nnc as _n
            Wt, bt = datagen.mlp_weights(datagen.SCOPF_DIMS, seed=0)
            for prec in ("fp32", "bf16"):
                c = _n.Context(0)
                nt = c.net(datagen.SCOPF_DIMS, ["tanh"] * 38 + ["identity"], Wt, bt, prec=prec, max_points=1)
                assert _n.nnc_autotune(c.h, nt.h, 1) == 0, _n.nnc_last_error(c.h)
                nt.destroy()
                c.close()
        print(json.dumps(bench_scopf(a.steps, a.warmup)), flush=True)
        return 0

    from paper_2509_22462_amd import datagen
    Ws, bs = datagen.mlp_weights(DIMS, seed=0)
    X, Lam = datagen.points(784, 10, a.points, seed=1002)

    if a.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    r = time_gpu(a.prec, a.steps, a.warmup, Ws, bs, X, Lam, autotune=a.autotune, hess=a.hess)
    method = r["method"]
    FH = hess_flops(DIMS, method=method) * a.points
    ms_step = r["seconds"] / a.steps * 1e3
    value = a.points * a.steps / r["seconds"]
    # dominant kernel: the tangent-sweep GEMM (forward + reverse sweeps)
    FS = sweep_flops(DIMS, method=method) * a.points
    gemm_per_launch_ms = r["gemm_ms"] / max(r["gemm_launches"], 1)
    launches_per_step = r["gemm_launches"] / a.steps
    flops_per_launch = FS / launches_per_step
    achieved = flops_per_launch / (gemm_per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[a.prec]
    traffic = load_traffic(a.prec)
    roofline = dict(bound="mfma", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=traffic,
                    kernel=("tangent-sweep GEMM launches (" + ("forward sweep only: the layer-sum method" if method == "layersum"
                            else "forward and reverse sweeps") + "; gemm_nt_kernel or gemm_dma_kernel as the tiling table "
                            "assigns, with the split-K reduction where K is split)"),
                    flops_per_launch=flops_per_launch, avg_launch_ms=round(gemm_per_launch_ms, 4),
                    launches_per_step=launches_per_step)
    h_launch_ms = r["h_ms"] / max(r["h_launches"], 1)
    all_gemm_tflops = FH / ((r["gemm_ms"] + r["h_ms"]) / a.steps * 1e-3) / 1e12
    esz = {"fp32": 4, "bf16": 2, "fp64": 8}[a.prec]
    # weight-streaming kernels: at one point nnc_eval reads every weight twice
    # per step (forward pass; Jacobian rows + FP64 adjoint in one reverse pass)
    sk_step_ms = r["skinny_ms"] / a.steps
    breakdown = dict(source="sweep GEMM from the timed region; other classes from a separate "
                            "profiled pass of the same step",
                     sweep_gemm_ms_per_step=round(r["gemm_ms"] / a.steps, 4),
                     skinny_stream_tb_per_s=(round(2 * weight_bytes(DIMS, esz) / (sk_step_ms * 1e-3) / 1e12, 2)
                                             if a.points == 1 and sk_step_ms > 0 else None),
                     h_gemm_ms_per_step=round(r["h_ms"] / a.steps, 4),
                     h_gemm_tflops=round(a.points * hprod_flops(DIMS, method=method) / (h_launch_ms * 1e-3) / 1e12, 2),
                     all_mfma_tflops=round(all_gemm_tflops, 2),
                     skinny_ms_per_step=round(r["skinny_ms"] / a.steps, 4),
                     other_ms_per_step=round(r["other_ms"] / a.steps, 4),
                     **r["extra"])

    variants = {}
    for p in [v for v in a.variants.split(",") if v and v != a.prec]:
        rv = time_gpu(p, max(5, a.steps // 3), 2, Ws, bs, X, Lam, autotune=a.autotune, hess=a.hess)
        lp = rv["gemm_launches"] / rv["steps"]
        FSv = sweep_flops(DIMS, method=rv["method"]) * a.points
        ach = (FSv / lp) / ((rv["gemm_ms"] / max(rv["gemm_launches"], 1)) * 1e-3) / 1e12
        variants[p] = dict(value=round(a.points * rv["steps"] / rv["seconds"], 3),
                           ms_per_step=round(rv["seconds"] / rv["steps"] * 1e3, 4),
                           gemm_tflops=round(ach, 2), gemm_frac=round(ach / PEAK_TFLOPS[p], 4),
                           hess_method=rv["method"],
                           _res=rv)

    extras = {}
    if not a.no_extras:
        # the other two throughput workloads, briefly: the batched surrogates
        # (one persistent graph replay per step) and the 32-point precision sweep
        extras["surrogate_batch"] = bench_surrogates(max(3, a.steps // 6), 2, "fp32")
        extras["precision_sweep_32pts"] = bench_sweep(max(3, a.steps // 10), 1, points=32, h_sample=2,
                                                      autotune=a.autotune)
        extras["deep_narrow_592m_1pt"] = bench_scopf(max(5, a.steps // 3), 2)
        extras["device_kkt_newton_step"] = bench_kkt()
    ceilings = None
    if not a.no_peaks:
        ceilings = measured_ceilings()
        mk = ceilings["mfma_tflops"][MFMA_KIND[a.prec]]
        ceilings["sweep_gemm_frac_of_measured_mfma"] = round(achieved / mk, 4)
        if breakdown.get("skinny_stream_tb_per_s"):
            ceilings["weight_stream_frac_of_measured_read"] = round(
                breakdown["skinny_stream_tb_per_s"] * 1e3 / ceilings["hbm_read_gb_per_s"], 4)
    cpu = None
    errors = None
    if not a.no_cpu_baseline:
        cpu, ref = cpu_baseline(Ws, bs, X, Lam)

        def rel(u, v):
            return float(np.linalg.norm(u - v) / np.linalg.norm(v))

        errors = {a.prec: dict(g=rel(r["g"], ref[0]), J=rel(r["J"], ref[1]), H=rel(r["H"], ref[2]))}
        for p, v in variants.items():
            rv = v["_res"]
            errors[p] = dict(g=rel(rv["g"], ref[0]), J=rel(rv["J"], ref[1]), H=rel(rv["H"], ref[2]))
        cpu = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in cpu.items()}
    for v in variants.values():
        v.pop("_res", None)

    line = {
        "metric": "Hessian-of-Lagrangian evals/s (137M-param MLP)",
        "value": round(value, 3),
        "unit": "H evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[a.prec],
        "data": "synthetic",
        "config": {"workload": f"tanh MLP 784-4096-8192-8192-4096-10 (137.5M weights), {a.points} "
                               "point(s), step = g + J + H at the point(s) (nnc_eval)",
                   "points": a.points, "precision": a.prec, "hess_method": method,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "measured_ceilings": ceilings,
        "mfma_util_pct": round(100 * achieved / peak, 2),
        "mfma_util_basis": "algorithmic flops of the dominant kernel / its HIP-event time / peak",
        "mfma_busy_pct_rocprof": load_mfma_busy(a.prec),
        "mfma_busy_whole_eval_pct_rocprof": load_mfma_busy(a.prec, "whole_eval_mfma_busy_pct"),
        "rel_err_vs_fp64_oracle": errors,
        "cpu_baseline": cpu,
        "breakdown": breakdown,
        "variants": variants,
        "other_workloads": extras,
        "hess_gflop_per_eval": round(FH / 1e9, 2),
        "weight_bytes": weight_bytes(DIMS, esz),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
