"""Python binding of libzf (ctypes).  Argument marshalling only: every step of the
refinement runs in the library's HIP kernels.  Tensors are torch CUDA (HIP)
tensors; PyTorch supplies device memory and the current stream.

The binding never falls back to another implementation: if libzf.so is missing
or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzf.so")

# enums of include/zf.h
FP64, BF16X3, FP16X3 = 0, 1, 2
STOP_RATIO, STOP_MONOTONE = 0, 1
REFINE_OFF, REFINE_F64_DELTA, REFINE_F64_FULL = 0, 1, 2
WARN_MAXSWEEPS, WARN_HIST_TRUNC = 1, 4
ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_NONFINITE, ERR_NOT_CONVERGED = -1, -2, -3, -4, -5

_PREC = {"fp64": FP64, "bf16x3": BF16X3, "fp16x3": FP16X3}
_STOP = {"ratio": STOP_RATIO, "monotone": STOP_MONOTONE}
_REFINE = {"off": REFINE_OFF, "f64_delta": REFINE_F64_DELTA, "f64_full": REFINE_F64_FULL}
KERNEL_CLASSES = ("gemm_x3", "gemm_x3_sym", "gemm_f64", "gemm_f64_sym")


class ZFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libzf error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("precision", ctypes.c_int), ("stop", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("refine", ctypes.c_int),
                ("max_refine", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("low_evals", ctypes.c_int),
                ("high_evals", ctypes.c_int), ("hist_len", ctypes.c_int),
                ("flags", ctypes.c_int), ("final_err", ctypes.c_double),
                ("final_rms", ctypes.c_double)]


EXPORTS = ("zf_default_opts", "zf_refine", "zf_refine_ex", "zf_residual", "zf_release",
           "zf_last_error", "zf_version", "zf_t_split", "zf_t_gemm", "zf_t_gershgorin",
           "zf_profile_enable", "zf_profile_reset", "zf_profile_read")

_lib = None


def lib() -> ctypes.CDLL:
    """Load libzf.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    P = ctypes.POINTER
    L.zf_default_opts.argtypes = [P(Opts)]
    L.zf_default_opts.restype = None
    L.zf_refine.argtypes = [vp, vp, i, i, i, vp, P(i), P(d), i, P(i), vp]
    L.zf_refine.restype = i
    L.zf_refine_ex.argtypes = [vp, vp, i, P(Opts), vp, P(Result), P(d), i, vp]
    L.zf_refine_ex.restype = i
    L.zf_residual.argtypes = [vp, vp, i, P(d), vp]
    L.zf_residual.restype = i
    L.zf_release.argtypes = []
    L.zf_release.restype = None
    L.zf_last_error.argtypes = []
    L.zf_last_error.restype = ctypes.c_char_p
    L.zf_version.argtypes = []
    L.zf_version.restype = i
    L.zf_t_split.argtypes = [vp, i64, vp, vp, i, vp]
    L.zf_t_split.restype = i
    L.zf_t_gemm.argtypes = [i, i, i, i, i, vp, vp, d, vp, d, d, vp, P(d), vp]
    L.zf_t_gemm.restype = i
    L.zf_t_gershgorin.argtypes = [vp, i, P(d), vp]
    L.zf_t_gershgorin.restype = i
    L.zf_profile_enable.argtypes = [i]
    L.zf_profile_enable.restype = None
    L.zf_profile_reset.argtypes = []
    L.zf_profile_reset.restype = None
    L.zf_profile_read.argtypes = [i, P(ctypes.c_char_p), P(ctypes.c_longlong), P(d), P(d)]
    L.zf_profile_read.restype = i
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        raise ZFError(rc, lib().zf_last_error().decode())
    return rc


def _dev(t: torch.Tensor, name: str, n: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    if n is not None and tuple(t.shape) != (n, n):
        raise ValueError(f"{name} must be {n}x{n}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


@dataclass
class Refined:
    Z: torch.Tensor
    iters: int
    hist: list = field(default_factory=list)
    low_evals: int = 0
    high_evals: int = 0
    flags: int = 0
    final_err: float = math.nan
    final_rms: float = math.nan


def refine(S: torch.Tensor, Z0: torch.Tensor | None = None, *, order: int = 2,
           precision: str = "bf16x3", stop: str = "ratio", max_sweeps: int = 100,
           refine: str = "f64_delta", max_refine: int = 10, out: torch.Tensor | None = None,
           hist_cap: int = 256, stream=None) -> Refined:
    """Refine Z0 (None: scaled identity) to Z with Z^T S Z = I (zf_refine_ex)."""
    n = S.shape[0]
    s_ptr = _dev(S, "S", n)
    z0_ptr = _dev(Z0, "Z0", n) if Z0 is not None else None
    if out is None:
        out = torch.empty_like(S)
    z_ptr = _dev(out, "out", n)
    o = Opts(order, _PREC[precision], _STOP[stop], max_sweeps, _REFINE[refine], max_refine)
    r = Result()
    hist = (ctypes.c_double * max(hist_cap, 1))()
    rc = lib().zf_refine_ex(s_ptr, z0_ptr, n, ctypes.byref(o), z_ptr, ctypes.byref(r), hist,
                            hist_cap, _stream(stream))
    _check(rc)
    return Refined(out, r.iters, list(hist[: r.hist_len]), r.low_evals, r.high_evals, r.flags,
                   r.final_err, r.final_rms)


def refine_basic(S, Z0, order, precision, out, hist_cap=256, stream=None):
    """The short form zf_refine(S, Z0, n, order, precision) -> (rc, iters, hist)."""
    n = S.shape[0]
    iters = ctypes.c_int(0)
    hl = ctypes.c_int(0)
    hist = (ctypes.c_double * max(hist_cap, 1))()
    rc = lib().zf_refine(_dev(S, "S", n), _dev(Z0, "Z0", n) if Z0 is not None else None, n, order,
                         _PREC[precision] if isinstance(precision, str) else precision,
                         _dev(out, "out", n), ctypes.byref(iters), hist, hist_cap,
                         ctypes.byref(hl), _stream(stream))
    _check(rc)
    return rc, iters.value, list(hist[: hl.value])


def residual(S: torch.Tensor, Z: torch.Tensor, stream=None) -> float:
    """||Z^T S Z - I||_F with FP64 products (zf_residual)."""
    n = S.shape[0]
    v = ctypes.c_double(0.0)
    _check(lib().zf_residual(_dev(S, "S", n), _dev(Z, "Z", n), n, ctypes.byref(v), _stream(stream)))
    return v.value


def release() -> None:
    lib().zf_release()


def last_error() -> str:
    return lib().zf_last_error().decode()


# ---- kernel-level hooks (unit tests) ---------------------------------------
def t_split(a: torch.Tensor, fmt: str = "bf16", stream=None):
    """Two-term split of FP64 values -> (hi, lo) raw 16-bit patterns (int16 tensors)."""
    if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous():
        raise TypeError("a must be a contiguous CUDA float64 tensor")
    hi = torch.empty(a.shape, dtype=torch.int16, device=a.device)
    lo = torch.empty_like(hi)
    _check(lib().zf_t_split(a.data_ptr(), a.numel(), hi.data_ptr(), lo.data_ptr(),
                            1 if fmt == "bf16" else 2, _stream(stream)))
    return hi, lo


def t_gemm(precision: str, A: torch.Tensor, B: torch.Tensor, *, sym: bool = False,
           alpha: float = 0.0, D: torch.Tensor | None = None, beta: float = 1.0,
           gamma: float = 0.0, stream=None):
    """C = alpha D + beta A B^T + gamma I through one library GEMM; returns (C, sum C^2)."""
    m, k = A.shape
    nn = B.shape[0]
    for t, nm in ((A, "A"), (B, "B")):
        _dev(t, nm)
    if B.shape[1] != k:
        raise ValueError("A and B must share the inner dimension")
    if D is not None:
        _dev(D, "D")
        if tuple(D.shape) != (m, nn):
            raise ValueError("D must be m x nn")
    C = torch.empty((m, nn), dtype=torch.float64, device=A.device)
    nrm = ctypes.c_double(0.0)
    _check(lib().zf_t_gemm(_PREC[precision], 1 if sym else 0, m, nn, k, A.data_ptr(), B.data_ptr(),
                           alpha, D.data_ptr() if D is not None else None, beta, gamma,
                           C.data_ptr(), ctypes.byref(nrm), _stream(stream)))
    return C, nrm.value


def t_gershgorin(S: torch.Tensor, stream=None) -> float:
    n = S.shape[0]
    v = ctypes.c_double(0.0)
    _check(lib().zf_t_gershgorin(_dev(S, "S", n), n, ctypes.byref(v), _stream(stream)))
    return v.value


# ---- per-kernel timing ------------------------------------------------------
def profile_enable(on: bool = True) -> None:
    lib().zf_profile_enable(1 if on else 0)


def profile_reset() -> None:
    lib().zf_profile_reset()


def profile_read() -> dict:
    """{class: (launches, total_ms, executed_flops)} from HIP events around each GEMM."""
    out = {}
    for c in range(len(KERNEL_CLASSES)):
        name = ctypes.c_char_p()
        n = ctypes.c_longlong(0)
        ms = ctypes.c_double(0.0)
        fl = ctypes.c_double(0.0)
        _check(lib().zf_profile_read(c, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms),
                                     ctypes.byref(fl)))
        out[name.value.decode()] = (n.value, ms.value, fl.value)
    return out
