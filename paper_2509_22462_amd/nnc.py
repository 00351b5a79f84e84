"""ctypes binding of libnnc (``include/nnc.h``).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  The functions carry the C names (``nnc_create``, ``nnc_eval_g``,
...) and take plain integers for device pointers, so any allocator works;
:class:`Context` / :class:`Net` add a thin convenience layer over torch
device tensors (torch is used only for device memory and streams).

Importing this module loads nothing; the library is loaded on first use and
a missing or unloadable ``libnnc.so`` raises :class:`NNCError` — there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnnc.so")
# GEMM tilings chosen by nnc_autotune on gfx950 for the shipped workloads
TUNED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.jsonl")

# enum nnc_act / nnc_prec / nnc_status (mirrors include/nnc.h)
NNC_IDENTITY, NNC_TANH, NNC_SIGMOID, NNC_SOFTPLUS, NNC_SOFTMAX = 0, 1, 2, 3, 4
NNC_FP64, NNC_FP32, NNC_BF16 = 0, 1, 2
NNC_KC_GEMM, NNC_KC_SKINNY, NNC_KC_OTHER, NNC_KC_GEMM_H = 0, 1, 2, 3
NNC_HESS_AUTO, NNC_HESS_FOR, NNC_HESS_LAYERSUM = 0, 1, 2
HESS_CODES = {"auto": NNC_HESS_AUTO, "for": NNC_HESS_FOR, "layersum": NNC_HESS_LAYERSUM}
NNC_OK, NNC_E_ARG, NNC_E_SHAPE, NNC_E_NOMEM, NNC_E_HIP, NNC_E_NONFINITE, NNC_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)

ACT_CODES = {"identity": NNC_IDENTITY, "tanh": NNC_TANH, "sigmoid": NNC_SIGMOID,
             "softplus": NNC_SOFTPLUS, "softmax": NNC_SOFTMAX}
PREC_CODES = {"fp64": NNC_FP64, "fp32": NNC_FP32, "bf16": NNC_BF16}

# Every symbol include/nnc.h declares, with (restype, argtypes).
_p = C.c_void_p
_i = C.c_int
_d = C.c_double
SIGNATURES = {
    "nnc_create": (_i, [_i, _p, C.POINTER(_p)]),
    "nnc_destroy": (_i, [_p]),
    "nnc_set_stream": (_i, [_p, _p]),
    "nnc_strerror": (C.c_char_p, [_i]),
    "nnc_last_error": (C.c_char_p, [_p]),
    "nnc_net_create": (_i, [_p, _i, C.POINTER(_i), C.POINTER(_i), C.POINTER(_p), C.POINTER(_p),
                            _i, _i, C.POINTER(_i)]),
    "nnc_net_destroy": (_i, [_p, _i]),
    "nnc_net_set_objective_diag": (_i, [_p, _i, _p]),
    "nnc_net_info": (_i, [_p, _i, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i), C.POINTER(_i),
                          C.POINTER(_i)]),
    "nnc_net_set_hess_method": (_i, [_p, _i, _i]),
    "nnc_net_hess_method": (_i, [_p, _i, C.POINTER(_i)]),
    "nnc_eval_g": (_i, [_p, _i, _i, _p, _p, _p]),
    "nnc_eval_g_static": (_i, [_p, _i, _i, _p, _p, _p]),
    "nnc_eval_jac_g": (_i, [_p, _i, _i, _p, _p]),
    "nnc_eval_hess_lag": (_i, [_p, _i, _i, _p, _d, _p, _p]),
    "nnc_eval": (_i, [_p, _i, _i, _p, _p, _d, _p, _p, _p, _p]),
    "nnc_hess_pack_lower": (_i, [_p, _i, _i, _p, _p]),
    "nnc_kkt_create": (_i, [_p, _i, _i, C.POINTER(_i)]),
    "nnc_kkt_destroy": (_i, [_p, _i]),
    "nnc_kkt_solve": (_i, [_p, _i, _i, _p, _p, _p, _p, _p, _p, _p, _p]),
    "nnc_profile_classes": (_i, [_p, _i]),
    "nnc_set_gemm_ksplit": (_i, [_p, _i, _i]),
    "nnc_eval_batch": (_i, [_p, _i, _p]),
    "nnc_autotune": (_i, [_p, _i, _i]),
    "nnc_autotune_query": (_i, [_p, _i, _i, _i, _i, _i, _i]),
    "nnc_set_gemm_config": (_i, [_p, _i, _i]),
    "nnc_gemm_config_count": (_i, []),
    "nnc_profile": (_i, [_p, _i]),
    "nnc_profile_read": (_i, [_p, _i, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "nnc_train_create": (_i, [_p, _i, C.POINTER(_i), _i, _i, C.c_ulonglong, C.POINTER(_i)]),
    "nnc_train_destroy": (_i, [_p, _i]),
    "nnc_train_step": (_i, [_p, _i, _p, _p, C.c_float, C.POINTER(C.c_float)]),
    "nnc_train_predict": (_i, [_p, _i, _i, _p, _p]),
    "nnc_train_num_params": (_i, [_p, _i, C.POINTER(C.c_longlong)]),
    "nnc_train_get_params": (_i, [_p, _i, _p]),
    "nnc_train_set_params": (_i, [_p, _i, _p]),
    "nnc_train_get_grads": (_i, [_p, _i, _p]),
    "nnc_peak_mfma": (_i, [_p, _i, _i, C.POINTER(_d)]),
    "nnc_peak_hbm": (_i, [_p, _p, _p, C.c_size_t, _i, C.POINTER(_d), C.POINTER(_d)]),
}

# MFMA shapes of nnc_peak_mfma (include/nnc.h NNC_PEAK_*)
PEAK_KINDS = {"bf16_16x16x32": 0, "bf16_32x32x16": 1, "fp32_16x16x4": 2, "fp64_16x16x4": 3}


class NNCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class nnc_job(C.Structure):
    _fields_ = [("net", C.c_int), ("B", C.c_int), ("x", C.c_void_p), ("lam", C.c_void_p),
                ("obj_factor", C.c_double), ("g", C.c_void_p), ("J", C.c_void_p),
                ("H", C.c_void_p)]


_LIB = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libnnc.so once; raise NNCError if it is missing (no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise NNCError(NNC_E_UNSUPPORTED,
                       f"{path} not built; run `python -m paper_2509_22462_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _chk(rc: int, ctx=None, what: str = ""):
    if rc != NNC_OK:
        lib = load_library()
        msg = lib.nnc_strerror(rc).decode()
        if ctx is not None:
            detail = lib.nnc_last_error(ctx)
            if detail:
                msg += ": " + detail.decode()
        raise NNCError(rc, f"{what}: {msg}" if what else msg)
    return rc


# ---------------------------------------------------------------- C-named calls
def nnc_create(device: int = 0, stream: int | None = None):
    lib = load_library()
    h = C.c_void_p()
    _chk(lib.nnc_create(device, stream or None, C.byref(h)), None, "nnc_create")
    return h


def nnc_destroy(ctx):
    return load_library().nnc_destroy(ctx)


def nnc_set_stream(ctx, stream: int | None):
    return _chk(load_library().nnc_set_stream(ctx, stream or None), ctx, "nnc_set_stream")


def nnc_strerror(status: int) -> str:
    return load_library().nnc_strerror(status).decode()


def nnc_last_error(ctx) -> str:
    return load_library().nnc_last_error(ctx).decode()


def nnc_net_create(ctx, dims: Sequence[int], acts: Sequence[int], Ws, bs, prec: int,
                   max_points: int) -> int:
    """Ws/bs: float64 numpy arrays (host); returns the network handle."""
    lib = load_library()
    L = len(dims) - 1
    Wc = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
    bc = [None if b is None else np.ascontiguousarray(b, dtype=np.float64) for b in (bs or [None] * L)]
    d = (C.c_int * (L + 1))(*dims)
    a = (C.c_int * L)(*acts)
    wp = (C.c_void_p * L)(*[w.ctypes.data for w in Wc])
    bp = (C.c_void_p * L)(*[0 if b is None else b.ctypes.data for b in bc])
    out = C.c_int(-1)
    _chk(lib.nnc_net_create(ctx, L, d, a, wp, bp, prec, max_points, C.byref(out)), ctx,
         "nnc_net_create")
    return out.value


def nnc_net_destroy(ctx, net: int):
    return _chk(load_library().nnc_net_destroy(ctx, net), ctx, "nnc_net_destroy")


def nnc_net_set_objective_diag(ctx, net: int, q_ptr: int | None):
    return _chk(load_library().nnc_net_set_objective_diag(ctx, net, q_ptr or None), ctx,
                "nnc_net_set_objective_diag")


def nnc_net_info(ctx, net: int):
    v = [C.c_int() for _ in range(5)]
    _chk(load_library().nnc_net_info(ctx, net, *[C.byref(x) for x in v]), ctx, "nnc_net_info")
    return dict(zip(("L", "n", "m", "prec", "max_points"), (x.value for x in v)))


def nnc_net_set_hess_method(ctx, net: int, method: int):
    return _chk(load_library().nnc_net_set_hess_method(ctx, net, method), ctx, "nnc_net_set_hess_method")


def nnc_net_hess_method(ctx, net: int) -> int:
    v = C.c_int(-1)
    _chk(load_library().nnc_net_hess_method(ctx, net, C.byref(v)), ctx, "nnc_net_hess_method")
    return v.value


def nnc_eval_g(ctx, net: int, B: int, x: int, y: int | None, g: int) -> int:
    return load_library().nnc_eval_g(ctx, net, B, x or None, y or None, g or None)


def nnc_eval_g_static(ctx, net: int, B: int, x: int, y: int | None, g: int) -> int:
    return load_library().nnc_eval_g_static(ctx, net, B, x or None, y or None, g or None)


def nnc_eval_jac_g(ctx, net: int, B: int, x: int, J: int) -> int:
    return load_library().nnc_eval_jac_g(ctx, net, B, x or None, J or None)


def nnc_eval_hess_lag(ctx, net: int, B: int, x: int, obj_factor: float, lam: int, H: int) -> int:
    return load_library().nnc_eval_hess_lag(ctx, net, B, x or None, float(obj_factor), lam or None,
                                            H or None)


def nnc_eval(ctx, net: int, B: int, x: int, y: int, obj_factor: float, lam: int, g: int, J: int,
             H: int) -> int:
    return load_library().nnc_eval(ctx, net, B, x or None, y or None, float(obj_factor), lam or None,
                                   g or None, J or None, H or None)


def nnc_peak_mfma(ctx, kind: str, iters: int) -> float:
    """Measured MFMA throughput (TFLOP/s) of one instruction shape."""
    out = C.c_double(0.0)
    _chk(load_library().nnc_peak_mfma(ctx, PEAK_KINDS[kind], int(iters), C.byref(out)), ctx, "nnc_peak_mfma")
    return out.value


def nnc_peak_hbm(ctx, src: int, dst: int, nbytes: int, reps: int):
    """Measured (read, copy) stream rates in GB/s over device buffers src, dst."""
    rd, cp = C.c_double(0.0), C.c_double(0.0)
    _chk(load_library().nnc_peak_hbm(ctx, src, dst, int(nbytes), int(reps), C.byref(rd), C.byref(cp)),
         ctx, "nnc_peak_hbm")
    return rd.value, cp.value


def nnc_kkt_create(ctx, n: int, max_B: int) -> int:
    out = C.c_int(-1)
    _chk(load_library().nnc_kkt_create(ctx, n, max_B, C.byref(out)), ctx, "nnc_kkt_create")
    return out.value


def nnc_kkt_destroy(ctx, kkt: int):
    return _chk(load_library().nnc_kkt_destroy(ctx, kkt), ctx, "nnc_kkt_destroy")


def nnc_kkt_solve(ctx, kkt: int, B: int, H: int, d: int | None, a: int | None, s: int | None,
                  delta: int | None, r: int, dx: int, info: int) -> int:
    return load_library().nnc_kkt_solve(ctx, kkt, B, H or None, d or None, a or None, s or None,
                                        delta or None, r or None, dx or None, info or None)


def nnc_hess_pack_lower(ctx, B: int, n: int, H: int, Hp: int) -> int:
    return load_library().nnc_hess_pack_lower(ctx, B, n, H or None, Hp or None)


def nnc_profile_classes(ctx, class_mask: int) -> int:
    return load_library().nnc_profile_classes(ctx, int(class_mask))


def nnc_set_gemm_ksplit(ctx, prec: int, ksplit: int) -> int:
    return load_library().nnc_set_gemm_ksplit(ctx, int(prec), int(ksplit))


def nnc_eval_batch(ctx, jobs: Sequence[dict]) -> int:
    arr = (nnc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = nnc_job(j["net"], j["B"], j.get("x") or None, j.get("lam") or None,
                         float(j.get("obj_factor", 0.0)), j.get("g") or None, j.get("J") or None,
                         j.get("H") or None)
    return load_library().nnc_eval_batch(ctx, len(jobs), arr)


def nnc_autotune(ctx, net: int, B: int) -> int:
    return load_library().nnc_autotune(ctx, net, B)


def nnc_autotune_query(ctx, prec: int, M: int, N: int, K: int, acc64: int, splits: int) -> int:
    return load_library().nnc_autotune_query(ctx, prec, M, N, K, acc64, splits)


def nnc_set_gemm_config(ctx, prec: int, config: int):
    return _chk(load_library().nnc_set_gemm_config(ctx, prec, config), ctx, "nnc_set_gemm_config")


def nnc_gemm_config_count() -> int:
    return load_library().nnc_gemm_config_count()


def nnc_profile(ctx, enable: bool):
    return _chk(load_library().nnc_profile(ctx, int(bool(enable))), ctx, "nnc_profile")


def nnc_profile_read(ctx, kernel_class: int):
    """(total milliseconds, launches) recorded for one kernel class."""
    ms = C.c_double()
    cnt = C.c_longlong()
    _chk(load_library().nnc_profile_read(ctx, kernel_class, C.byref(ms), C.byref(cnt)), ctx,
         "nnc_profile_read")
    return ms.value, cnt.value


def nnc_train_create(ctx, dims: Sequence[int], batch: int, prec: int, seed: int) -> int:
    L = len(dims) - 1
    d = (C.c_int * (L + 1))(*dims)
    out = C.c_int(-1)
    _chk(load_library().nnc_train_create(ctx, L, d, batch, prec, seed, C.byref(out)), ctx,
         "nnc_train_create")
    return out.value


def nnc_train_destroy(ctx, mlp: int):
    return _chk(load_library().nnc_train_destroy(ctx, mlp), ctx, "nnc_train_destroy")


def nnc_train_step(ctx, mlp: int, X: int, Y: int, lr: float, want_loss: bool = True):
    loss = C.c_float(float("nan"))
    _chk(load_library().nnc_train_step(ctx, mlp, X, Y, lr, C.byref(loss) if want_loss else None),
         ctx, "nnc_train_step")
    return loss.value if want_loss else None


def nnc_train_predict(ctx, mlp: int, B: int, X: int, Yhat: int):
    return _chk(load_library().nnc_train_predict(ctx, mlp, B, X, Yhat), ctx, "nnc_train_predict")


def nnc_train_num_params(ctx, mlp: int) -> int:
    v = C.c_longlong()
    _chk(load_library().nnc_train_num_params(ctx, mlp, C.byref(v)), ctx, "nnc_train_num_params")
    return v.value


def nnc_train_get_params(ctx, mlp: int) -> np.ndarray:
    out = np.empty(nnc_train_num_params(ctx, mlp), dtype=np.float64)
    _chk(load_library().nnc_train_get_params(ctx, mlp, out.ctypes.data), ctx, "nnc_train_get_params")
    return out


def nnc_train_get_grads(ctx, mlp: int) -> np.ndarray:
    out = np.empty(nnc_train_num_params(ctx, mlp), dtype=np.float64)
    _chk(load_library().nnc_train_get_grads(ctx, mlp, out.ctypes.data), ctx, "nnc_train_get_grads")
    return out


def nnc_train_set_params(ctx, mlp: int, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float64)
    _chk(load_library().nnc_train_set_params(ctx, mlp, p.ctypes.data), ctx, "nnc_train_set_params")


# ---------------------------------------------------------------- torch convenience
def _torch():
    import torch  # noqa: WPS433 (device memory and streams only)
    return torch


def _dev_f64(a, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    return t.contiguous()


class Context:
    """A library context bound to a torch CUDA (HIP) device and stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.h = nnc_create(device, stream.cuda_stream)

    def net(self, dims, acts, Ws, bs=None, prec="fp32", max_points=1, hess="auto") -> "Net":
        acts_c = [ACT_CODES[a] if isinstance(a, str) else int(a) for a in acts]
        p = PREC_CODES[prec] if isinstance(prec, str) else int(prec)
        net = Net(self, nnc_net_create(self.h, list(dims), acts_c, Ws, bs, p, max_points), list(dims))
        if hess != "auto":
            net.set_hess_method(hess)
        return net

    def close(self):
        if self.h:
            nnc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    def __init__(self, ctx: Context, handle: int, dims):
        self.ctx = ctx
        self.h = handle
        self.n = dims[0]
        self.m = dims[-1]
        self._q = None

    def set_objective_diag(self, q):
        self._q = None if q is None else _dev_f64(q, self.ctx.device)
        nnc_net_set_objective_diag(self.ctx.h, self.h, None if q is None else self._q.data_ptr())

    def set_hess_method(self, method: str):
        """"auto", "for" (forward-over-reverse) or "layersum"."""
        nnc_net_set_hess_method(self.ctx.h, self.h, HESS_CODES[method])

    @property
    def hess_method(self) -> str:
        code = nnc_net_hess_method(self.ctx.h, self.h)
        return {v: k for k, v in HESS_CODES.items()}[code]

    def eval_g(self, x, y=None, out=None):
        torch = _torch()
        x = _dev_f64(x, self.ctx.device).reshape(-1, self.n)
        B = x.shape[0]
        yy = None if y is None else _dev_f64(y, self.ctx.device).reshape(B, self.m)
        g = out if out is not None else torch.empty(B, self.m, dtype=torch.float64, device=self.ctx.device)
        _chk(nnc_eval_g(self.ctx.h, self.h, B, x.data_ptr(), None if yy is None else yy.data_ptr(),
                        g.data_ptr()), self.ctx.h, "nnc_eval_g")
        return g

    def eval_jac_g(self, x, out=None):
        torch = _torch()
        x = _dev_f64(x, self.ctx.device).reshape(-1, self.n)
        B = x.shape[0]
        J = out if out is not None else torch.empty(B, self.m, self.n, dtype=torch.float64,
                                                    device=self.ctx.device)
        _chk(nnc_eval_jac_g(self.ctx.h, self.h, B, x.data_ptr(), J.data_ptr()), self.ctx.h,
             "nnc_eval_jac_g")
        return J

    def eval_hess_lag(self, x, lam, obj_factor=0.0, out=None):
        torch = _torch()
        x = _dev_f64(x, self.ctx.device).reshape(-1, self.n)
        B = x.shape[0]
        lam = _dev_f64(lam, self.ctx.device).reshape(B, self.m)
        H = out if out is not None else torch.empty(B, self.n, self.n, dtype=torch.float64,
                                                    device=self.ctx.device)
        _chk(nnc_eval_hess_lag(self.ctx.h, self.h, B, x.data_ptr(), obj_factor, lam.data_ptr(),
                               H.data_ptr()), self.ctx.h, "nnc_eval_hess_lag")
        return H

    def eval(self, x, lam=None, y=None, obj_factor=0.0, want=("g", "J", "H")):
        """g, J and/or H at the same points in one call (one forward pass)."""
        torch = _torch()
        dev = self.ctx.device
        x = _dev_f64(x, dev).reshape(-1, self.n)
        B = x.shape[0]
        f64 = torch.float64
        g = torch.empty(B, self.m, dtype=f64, device=dev) if "g" in want else None
        J = torch.empty(B, self.m, self.n, dtype=f64, device=dev) if "J" in want else None
        H = torch.empty(B, self.n, self.n, dtype=f64, device=dev) if "H" in want else None
        yy = None if y is None else _dev_f64(y, dev).reshape(B, self.m)
        ll = None if lam is None else _dev_f64(lam, dev).reshape(B, self.m)
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        _chk(nnc_eval(self.ctx.h, self.h, B, x.data_ptr(), ptr(yy), obj_factor, ptr(ll), ptr(g),
                      ptr(J), ptr(H)), self.ctx.h, "nnc_eval")
        return g, J, H

    def destroy(self):
        nnc_net_destroy(self.ctx.h, self.h)
