"""CPU checks of the work accounting behind bench.py's roofline figures.

The flop counts are recomputed here by enumerating the GEMMs of the two
tangent sweeps and the H product one by one (shapes M x N x K, 2MNK flops),
an independent route to the closed forms bench.py uses."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def enumerate_gemms(dims):
    """Forward sweep T_{l+1} = W_{l+1} D_l T_l (l = 1..Lt-1), reverse sweep
    E_{l-1} = W_l^T G_l (l = Lt..2), then H = W_1^T G_1, with n tangent
    columns and an identity output layer (Lt = L - 1)."""
    n, L = dims[0], len(dims) - 1
    Lt = L - 1
    gemms = [(n, dims[l + 1], dims[l]) for l in range(1, Lt)]       # forward
    gemms += [(n, dims[l - 1], dims[l]) for l in range(Lt, 1, -1)]  # reverse
    gemms.append((n, n, dims[1]))                                   # H
    return gemms


def test_flop_counts_match_gemm_enumeration():
    b = load_bench()
    for dims in [(784, 4096, 8192, 8192, 4096, 10), (784, 64, 64, 10), (120, 512, 512, 512, 512, 4)]:
        g = enumerate_gemms(dims)
        total = sum(2.0 * m * nn * k for m, nn, k in g)
        sweeps = sum(2.0 * m * nn * k for m, nn, k in g[:-1])
        assert b.hess_flops(dims) == total
        assert b.sweep_flops(dims) == sweeps
    # the 137M network: six sweep GEMMs, 420.9 GF, plus 5.04 GF for H
    g = enumerate_gemms((784, 4096, 8192, 8192, 4096, 10))
    assert len(g) == 7
    assert abs(b.sweep_flops((784, 4096, 8192, 8192, 4096, 10)) / 1e9 - 420.907) < 1e-3
    assert abs(b.hess_flops((784, 4096, 8192, 8192, 4096, 10)) / 1e9 - 425.942) < 1e-3


def test_weight_bytes_and_traffic_gate():
    b = load_bench()
    dims = (784, 4096, 8192, 8192, 4096, 10)
    nw = 784 * 4096 + 4096 * 8192 + 8192 * 8192 + 8192 * 4096 + 4096 * 10
    assert nw == 137_469_952  # weights of the 137M network (biases excluded)
    assert b.weight_bytes(dims, 4) == 4 * nw
    # the committed traffic figure is reported only while the GEMM source matches
    import json
    for prec in ("fp32", "bf16"):
        t = b.load_traffic(prec)
        d = json.load(open(os.path.join(ROOT, "profiles", f"gemm_c2_{prec}_traffic.json")))
        if d["gemm_source_sha"] == b.gemm_source_sha():
            assert t == d["bytes_per_launch"]
        else:
            assert t is None
    assert b.load_traffic("fp64") is None  # never measured for FP64


def test_layersum_flop_accounting():
    """The layer sum is counted at its own flops: the forward sweep plus the
    n(n+1)/2 entries of the lower triangle, 2 sum_l d_l flops each (never at
    the forward-over-reverse count)."""
    b = load_bench()
    c2 = (784, 4096, 8192, 8192, 4096, 10)
    fwd = 2.0 * 784 * (8192 * 4096 + 8192 * 8192 + 4096 * 8192)
    assert b.sweep_flops(c2, method="layersum") == fwd
    assert abs(b.hprod_flops(c2, method="layersum") - 784 * 785 * (4096 + 8192 + 8192 + 4096)) < 1
    assert abs(b.hess_flops(c2, method="layersum") / 1e9 - 225.575) < 1e-2
    assert b.hess_flops(c2, method="layersum") < 0.53 * b.hess_flops(c2, method="for")
    # with sigma applied at the output too, the output layer joins both sums
    dims = (5, 7, 3)
    assert b.sweep_flops(dims, identity_out=False, method="layersum") == 2.0 * 5 * 7 * 3
    assert b.hprod_flops(dims, identity_out=False, method="layersum") == 5 * 6 * (7 + 3)


def test_peaks_are_the_published_ones():
    b = load_bench()
    assert b.PEAK_TFLOPS["fp32"] == 157.3
    assert b.PEAK_TFLOPS["fp64"] == 78.6
    assert np.isclose(b.PEAK_TFLOPS["bf16"], 2516.6, rtol=1e-3)
