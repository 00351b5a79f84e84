"""The C-ABI library loads and exports every symbol include/nnc.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_2509_22462_amd import nnc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nnc.LIB_PATH):
        pytest.fail("libnnc.so is not built: run python -m paper_2509_22462_amd.build")
    return ctypes.CDLL(nnc.LIB_PATH)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("nnc_create", "nnc_eval_g", "nnc_eval_jac_g", "nnc_eval_hess_lag", "nnc_eval_batch",
              "nnc_autotune", "nnc_train_step"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    assert set(declared_symbols()) == set(nnc.SIGNATURES)


def test_strerror_and_null_handles_without_gpu():
    nnc.load_library()
    assert nnc.nnc_strerror(0) == "ok"
    assert nnc.nnc_strerror(nnc.NNC_E_SHAPE) == "invalid shape"
    assert nnc.nnc_strerror(12345) == "unknown status"
    lib = nnc.load_library()
    assert lib.nnc_destroy(None) == nnc.NNC_OK
    assert lib.nnc_eval_g(None, 0, 1, None, None, None) == nnc.NNC_E_ARG
    assert lib.nnc_last_error(None) == b"null context"


def test_enum_values_match_header():
    text = open(HEADER).read()
    for name in ("NNC_IDENTITY", "NNC_TANH", "NNC_SIGMOID", "NNC_SOFTPLUS", "NNC_FP64", "NNC_FP32",
                 "NNC_BF16", "NNC_E_ARG", "NNC_E_SHAPE", "NNC_E_UNSUPPORTED"):
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(nnc, name), name


def test_tiling_table_names_compiled_tilings(lib):
    """Every entry of the committed tiling table names a tiling the library
    compiles, a K split the launcher accepts, and a shape listed once."""
    import json
    count = lib.nnc_gemm_config_count()
    seen = set()
    with open(nnc.TUNED_TABLE) as f:
        rows = [json.loads(line) for line in f if line.strip()]
    assert rows
    for r in rows:
        assert 0 <= r["cfg"] < count, r
        assert 1 <= r["ksplit"] <= 8, r
        assert r["dt"] in (0, 1, 2) and r["acc64"] in (0, 1), r
        assert r["acc64"] == 0 or r["ksplit"] == 1, r  # FP64-accumulated products are never K-split
        key = (r["dt"], r["M"], r["N"], r["K"], r["acc64"], r["splits"])
        assert key not in seen, key
        seen.add(key)
