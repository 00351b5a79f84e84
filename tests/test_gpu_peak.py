"""Peak microbenchmarks (nnc_peak_mfma, nnc_peak_hbm): every MFMA shape
reports a rate that is positive and no higher than the datasheet peak of its
type (plus a margin for clock boost); the stream probe's copy leaves dst
equal to src, its rates stay below the HBM datasheet figure on a buffer
larger than the Infinity Cache, and invalid arguments are rejected before
anything is launched."""
import numpy as np
import pytest

from paper_2509_22462_amd import nnc

pytestmark = pytest.mark.gpu

# MI355X datasheet peaks (dense), TFLOP/s, and HBM bandwidth, GB/s
DATASHEET = {"bf16_16x16x32": 2516.6, "bf16_32x32x16": 2516.6, "fp32_16x16x4": 157.3, "fp64_16x16x4": 78.6}
HBM_GBS = 8000.0


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    c = nnc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("kind", list(nnc.PEAK_KINDS))
def test_mfma_rate_is_plausible(ctx, kind):
    tf = nnc.nnc_peak_mfma(ctx.h, kind, 200)
    print(f"{kind}: {tf:.1f} TFLOP/s")
    assert 0.2 * DATASHEET[kind] < tf < 1.1 * DATASHEET[kind]


def test_stream_probe_copies_and_rates_are_plausible(ctx):
    import torch
    nbytes = 512 << 20  # above the 256 MB Infinity Cache
    src = torch.arange(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    rd, cp = nnc.nnc_peak_hbm(ctx.h, src.data_ptr(), dst.data_ptr(), nbytes, 2)
    print(f"read {rd:.0f} GB/s, copy {cp:.0f} GB/s")
    assert torch.equal(src, dst)
    assert 500.0 < rd < 1.1 * HBM_GBS
    assert 500.0 < cp < 1.1 * HBM_GBS


def test_stream_probe_ragged_tail(ctx):
    """A size that leaves a tail after the four-way unrolled loop."""
    import torch
    n16 = 1000003  # 16-byte words
    src = torch.randint(-2**31, 2**31 - 1, (n16 * 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    nnc.nnc_peak_hbm(ctx.h, src.data_ptr(), dst.data_ptr(), n16 * 16, 1)
    assert torch.equal(src, dst)


def test_invalid_arguments_are_rejected(ctx):
    import torch
    src = torch.zeros(1024, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    lib = nnc.load_library()
    out = nnc.C.c_double(0.0)
    assert lib.nnc_peak_mfma(ctx.h, 7, 10, nnc.C.byref(out)) == nnc.NNC_E_ARG
    assert lib.nnc_peak_mfma(ctx.h, 0, 0, nnc.C.byref(out)) == nnc.NNC_E_SHAPE
    assert lib.nnc_peak_mfma(ctx.h, 0, 10, None) == nnc.NNC_E_ARG
    rd, cp = nnc.C.c_double(0.0), nnc.C.c_double(0.0)
    p, q = src.data_ptr(), dst.data_ptr()
    # size not a multiple of 16, misaligned pointer, overlap, no output
    assert lib.nnc_peak_hbm(ctx.h, p, q, 4004, 1, nnc.C.byref(rd), nnc.C.byref(cp)) == nnc.NNC_E_SHAPE
    assert lib.nnc_peak_hbm(ctx.h, p + 4, q, 1024, 1, nnc.C.byref(rd), nnc.C.byref(cp)) == nnc.NNC_E_ARG
    assert lib.nnc_peak_hbm(ctx.h, p, p + 1024, 2048, 1, nnc.C.byref(rd), nnc.C.byref(cp)) == nnc.NNC_E_ARG
    assert lib.nnc_peak_hbm(ctx.h, p, q, 1024, 1, None, None) == nnc.NNC_E_ARG
    assert lib.nnc_peak_hbm(ctx.h, p, q, 1024, 0, nnc.C.byref(rd), None) == nnc.NNC_E_SHAPE
    assert np.all(dst.cpu().numpy() == 0)  # nothing was launched
