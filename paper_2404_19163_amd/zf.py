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
FP64, BF16X3, FP16X3, BF16, FP32, FP16 = 0, 1, 2, 3, 4, 5
STOP_RATIO, STOP_MONOTONE = 0, 1
REFINE_OFF, REFINE_F64_DELTA, REFINE_F64_FULL, REFINE_F32, REFINE_EMU = 0, 1, 2, 3, 4
REFINE_CRT, REFINE_CRT_FIRST = 5, 6
WARN_MAXSWEEPS, WARN_Z0_FALLBACK, WARN_HIST_TRUNC = 1, 2, 4
Z0_GIVEN, Z0_SCALED_IDENTITY, Z0_LEARNED = 0, 1, 2
ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_NONFINITE, ERR_NOT_CONVERGED = -1, -2, -3, -4, -5

_PREC = {"fp64": FP64, "bf16x3": BF16X3, "fp16x3": FP16X3, "bf16": BF16, "fp32": FP32,
         "fp16": FP16}
_STOP = {"ratio": STOP_RATIO, "monotone": STOP_MONOTONE}
_GUESS = {"identity": Z0_SCALED_IDENTITY, "learned": Z0_LEARNED, "given": Z0_GIVEN}
_REFINE = {"off": REFINE_OFF, "f64_delta": REFINE_F64_DELTA, "f64_full": REFINE_F64_FULL,
           "f32": REFINE_F32, "emu": REFINE_EMU, "crt": REFINE_CRT, "crt_first": REFINE_CRT_FIRST}
KERNEL_CLASSES = ("gemm_x3", "gemm_x3_sym", "gemm_f64", "gemm_f64_sym", "gemm_hh", "gemm_hh_sym",
                  "gemm_f32", "gemm_f32_sym", "gemm_x3f16", "gemm_x3f16_sym", "gemm_hhf16",
                  "gemm_hhf16_sym", "gemm_oz", "gemm_oz_sym", "gemm_crt", "gemm_crt_sym")


class ZFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libzf error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("precision", ctypes.c_int), ("stop", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("refine", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("z0", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("low_evals", ctypes.c_int),
                ("high_evals", ctypes.c_int), ("hist_len", ctypes.c_int),
                ("flags", ctypes.c_int), ("final_err", ctypes.c_double),
                ("final_rms", ctypes.c_double), ("status", ctypes.c_int),
                ("z0_used", ctypes.c_int)]


EXPORTS = ("zf_default_opts", "zf_refine", "zf_refine_ex", "zf_residual", "zf_release", "zf_residual_noalloc",
           "zf_last_error", "zf_version", "zf_t_split", "zf_t_gemm", "zf_t_gershgorin",
           "zf_profile_enable", "zf_profile_reset", "zf_profile_read", "zf_refine_batched",
           "zf_batched_set_tiles", "zf_batched_get_tiles", "zf_batched_autotune",
           "zf_batched_use_graph", "zf_batched_set_graph_sweeps", "zf_batched_last_stats",
           "zf_batched_release", "zf_features", "zf_guess_label",
           "zf_mlp_set_params", "zf_mlp_get_params", "zf_mlp_set_norm", "zf_mlp_train_step",
           "zf_mlp_grad", "zf_mlp_predict", "zf_mlp_save", "zf_mlp_load", "zf_congruence", "zf_t_ozaki",
           "zf_t_crt", "zf_t_gemm_kb")
N_PARAMS = 4931

_lib = None


def lib() -> ctypes.CDLL:
    """Load libzf.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python paper_2404_19163_amd/csrc/build.py")
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
    L.zf_residual_noalloc.argtypes = [vp, vp, i, vp, vp]
    L.zf_residual_noalloc.restype = i
    L.zf_congruence.argtypes = [vp, vp, i, i, vp, vp]
    L.zf_congruence.restype = i
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
    L.zf_t_gemm_kb.argtypes = [i, i, i, i, i, vp, vp, d, vp, d, d, vp, P(d), vp]
    L.zf_t_gemm_kb.restype = i
    L.zf_t_ozaki.argtypes = [i, i, i, i, i, vp, vp, d, vp, d, d, vp, P(d), vp]
    L.zf_t_ozaki.restype = i
    L.zf_t_crt.argtypes = [i, i, i, i, i, vp, vp, d, vp, d, d, vp, P(d), vp]
    L.zf_t_crt.restype = i
    L.zf_t_gershgorin.argtypes = [vp, i, P(d), vp]
    L.zf_t_gershgorin.restype = i
    L.zf_profile_enable.argtypes = [i]
    L.zf_profile_enable.restype = None
    L.zf_profile_reset.argtypes = []
    L.zf_profile_reset.restype = None
    L.zf_profile_read.argtypes = [i, P(ctypes.c_char_p), P(ctypes.c_longlong), P(d), P(d)]
    L.zf_profile_read.restype = i
    L.zf_refine_batched.argtypes = [i, P(vp), P(vp), P(i), P(Opts), P(vp), P(Result), P(d), i, vp]
    L.zf_refine_batched.restype = i
    L.zf_batched_set_tiles.argtypes = [P(i), P(i), i]
    L.zf_batched_set_tiles.restype = i
    L.zf_batched_get_tiles.argtypes = [P(i), P(i), i]
    L.zf_batched_get_tiles.restype = i
    L.zf_batched_autotune.argtypes = [P(i), i, i, i, P(i), P(d), vp]
    L.zf_batched_autotune.restype = i
    L.zf_batched_use_graph.argtypes = [i]
    L.zf_batched_use_graph.restype = None
    L.zf_batched_set_graph_sweeps.argtypes = [i]
    L.zf_batched_set_graph_sweeps.restype = i
    L.zf_batched_last_stats.argtypes = [P(i), P(i)]
    L.zf_batched_last_stats.restype = i
    L.zf_batched_release.argtypes = []
    L.zf_batched_release.restype = None
    F = P(ctypes.c_float)
    L.zf_features.argtypes = [vp, i, vp, vp]
    L.zf_features.restype = i
    L.zf_guess_label.argtypes = [vp, vp, i, P(d), vp]
    L.zf_guess_label.restype = i
    L.zf_mlp_set_params.argtypes = [F, i]
    L.zf_mlp_set_params.restype = i
    L.zf_mlp_get_params.argtypes = [F, i]
    L.zf_mlp_get_params.restype = i
    L.zf_mlp_set_norm.argtypes = [F, F, F, F]
    L.zf_mlp_set_norm.restype = i
    L.zf_mlp_train_step.argtypes = [vp, vp, i, ctypes.c_float, F, vp]
    L.zf_mlp_train_step.restype = i
    L.zf_mlp_grad.argtypes = [vp, vp, i, F, F, vp]
    L.zf_mlp_grad.restype = i
    L.zf_mlp_predict.argtypes = [vp, P(d), vp]
    L.zf_mlp_predict.restype = i
    L.zf_mlp_save.argtypes = [ctypes.c_char_p]
    L.zf_mlp_save.restype = i
    L.zf_mlp_load.argtypes = [ctypes.c_char_p]
    L.zf_mlp_load.restype = i
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
    status: int = 0
    z0_used: int = -1


def refine(S: torch.Tensor, Z0: torch.Tensor | None = None, *, order: int = 2,
           precision: str = "bf16x3", stop: str = "ratio", max_sweeps: int = 100,
           refine: str = "f64_delta", max_refine: int = 10, out: torch.Tensor | None = None,
           hist_cap: int = 256, stream=None, guess: str = "identity") -> Refined:
    """Refine Z0 to Z with Z^T S Z = I (zf_refine_ex).  With Z0 None the guess is the
    scaled identity, or the learned polynomial (guess="learned", needs a loaded net)."""
    n = S.shape[0]
    s_ptr = _dev(S, "S", n)
    z0_ptr = _dev(Z0, "Z0", n) if Z0 is not None else None
    if out is None:
        out = torch.empty_like(S)
    z_ptr = _dev(out, "out", n)
    o = Opts(order, _PREC[precision], _STOP[stop], max_sweeps, _REFINE[refine], max_refine,
             _GUESS[guess])
    r = Result()
    hist = (ctypes.c_double * max(hist_cap, 1))()
    rc = lib().zf_refine_ex(s_ptr, z0_ptr, n, ctypes.byref(o), z_ptr, ctypes.byref(r), hist,
                            hist_cap, _stream(stream))
    _check(rc)
    res = Refined(out, r.iters, list(hist[: r.hist_len]), r.low_evals, r.high_evals, r.flags,
                  r.final_err, r.final_rms)
    res.z0_used = r.z0_used
    return res


@dataclass
class BatchResult:
    results: list
    rc: int


def refine_batched(S_list, Z0_list=None, *, order: int = 2, precision: str = "bf16x3",
                   stop: str = "ratio", max_sweeps: int = 100, refine: str = "f64_delta",
                   max_refine: int = 10, out=None, hist_cap: int = 64, stream=None,
                   raise_on_error: bool = True, guess: str = "identity") -> BatchResult:
    """Refine many matrices together (zf_refine_batched).  Matrices without a Z0 start
    from the scaled identity, or the learned polynomial (guess="learned").  Returns one
    Refined per matrix (with .status and .z0_used) and the call's return code."""
    count = len(S_list)
    ns = [int(S.shape[0]) for S in S_list]
    sp = (ctypes.c_void_p * count)(*[_dev(S, "S", n) for S, n in zip(S_list, ns)])
    if Z0_list is None:
        z0p = None
    else:
        z0p = (ctypes.c_void_p * count)(*[(_dev(Z, "Z0", n) if Z is not None else None)
                                          for Z, n in zip(Z0_list, ns)])
    if out is None:
        out = [torch.empty_like(S) for S in S_list]
    zp = (ctypes.c_void_p * count)(*[_dev(Z, "out", n) for Z, n in zip(out, ns)])
    narr = (ctypes.c_int * count)(*ns)
    o = Opts(order, _PREC[precision], _STOP[stop], max_sweeps, _REFINE[refine], max_refine,
             _GUESS[guess])
    res = (Result * count)()
    hist = (ctypes.c_double * max(count * hist_cap, 1))()
    rc = lib().zf_refine_batched(count, sp, z0p, narr, ctypes.byref(o), zp, res, hist, hist_cap,
                                 _stream(stream))
    if rc < 0 and raise_on_error:
        raise ZFError(rc, lib().zf_last_error().decode())
    outl = []
    for m in range(count):
        r = res[m]
        h = list(hist[m * hist_cap: m * hist_cap + r.hist_len])
        outl.append(Refined(out[m], r.iters, h, r.low_evals, r.high_evals, r.flags, r.final_err,
                            r.final_rms))
        outl[-1].status = r.status
        outl[-1].z0_used = r.z0_used
    return BatchResult(outl, rc)


def batched_set_tiles(max_n, tiles) -> None:
    k = len(max_n)
    _check(lib().zf_batched_set_tiles((ctypes.c_int * k)(*max_n), (ctypes.c_int * k)(*tiles), k))


def batched_get_tiles():
    mx = (ctypes.c_int * 16)()
    tl = (ctypes.c_int * 16)()
    k = _check(lib().zf_batched_get_tiles(mx, tl, 16))
    return list(mx[:k]), list(tl[:k])


def batched_autotune(bucket_n, batch: int = 32, reps: int = 5, stream=None):
    """Time 64- and 128-wide tiles per order bucket, install the faster; returns
    (tiles, [(ms64, ms128), ...])."""
    k = len(bucket_n)
    best = (ctypes.c_int * k)()
    ms = (ctypes.c_double * (2 * k))()
    _check(lib().zf_batched_autotune((ctypes.c_int * k)(*bucket_n), k, batch, reps, best, ms,
                                     _stream(stream)))
    return list(best), [(ms[2 * b], ms[2 * b + 1]) for b in range(k)]


def batched_use_graph(on: bool = True) -> None:
    lib().zf_batched_use_graph(1 if on else 0)


def batched_set_graph_sweeps(sweeps: int = 8) -> None:
    """Macro-sweeps captured per graph launch (default 8; 0: every one the caps allow,
    so one launch and one synchronization per call)."""
    _check(lib().zf_batched_set_graph_sweeps(sweeps))


def batched_last_stats():
    """(macro-sweeps that had a live matrix, graph launches) of the last batched call."""
    a, b = ctypes.c_int(0), ctypes.c_int(0)
    lib().zf_batched_last_stats(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def batched_release() -> None:
    """Free the batched path's cached arena and graph (zf_batched_release)."""
    lib().zf_batched_release()


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
    """||Z^T S Z - I||_F / sqrt(n) with FP64 products (zf_residual)."""
    n = S.shape[0]
    v = ctypes.c_double(0.0)
    _check(lib().zf_residual(_dev(S, "S", n), _dev(Z, "Z", n), n, ctypes.byref(v), _stream(stream)))
    return v.value


def residual_noalloc(S: torch.Tensor, Z: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """zf_residual_noalloc: the RMS residual into the device scalar `out` (float64, one
    element), stream-ordered, without allocating device memory (n <= 1024)."""
    n = S.shape[0]
    if out.dtype != torch.float64 or out.numel() < 1 or not out.is_cuda:
        raise ValueError("out must be a CUDA float64 tensor with at least one element")
    _check(lib().zf_residual_noalloc(_dev(S, "S", n), _dev(Z, "Z", n), n, out.data_ptr(),
                                     _stream(stream)))


def congruence(H: torch.Tensor, Z: torch.Tensor, *, precision: str = "fp64",
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """H_perp = Z^T H Z (zf_congruence): the standard-form Hamiltonian once Z^T S Z = I.
    `out` may be H or Z itself."""
    n = H.shape[0]
    h_ptr, z_ptr = _dev(H, "H", n), _dev(Z, "Z", n)
    if out is None:
        out = torch.empty_like(H)
    _check(lib().zf_congruence(h_ptr, z_ptr, n, _PREC[precision], _dev(out, "out", n),
                               _stream(stream)))
    return out


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
           gamma: float = 0.0, stream=None, slices: int = 0, kblocked: bool = False):
    """C = alpha D + beta A B^T + gamma I through one library GEMM; returns (C, sum C^2).
    precision "emu" runs the emulated FP64 product with `slices` integer slices, "crt"
    the residue-emulated product with `slices` moduli; kblocked (pair precisions) splits
    A and B into the solver's K-blocked pair layout (zf_t_gemm_kb)."""
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
    dptr = D.data_ptr() if D is not None else None
    if precision in ("emu", "crt"):
        fn = lib().zf_t_ozaki if precision == "emu" else lib().zf_t_crt
        rc = fn(slices, 1 if sym else 0, m, nn, k, A.data_ptr(), B.data_ptr(), alpha,
                dptr, beta, gamma, C.data_ptr(), ctypes.byref(nrm), _stream(stream))
    else:
        fn = lib().zf_t_gemm_kb if kblocked else lib().zf_t_gemm
        rc = fn(_PREC[precision], 1 if sym else 0, m, nn, k, A.data_ptr(),
                             B.data_ptr(), alpha, dptr, beta, gamma, C.data_ptr(),
                             ctypes.byref(nrm), _stream(stream))
    _check(rc)
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


# ---- learned guess -----------------------------------------------------------
def _f32p(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def features(S: torch.Tensor, stream=None) -> torch.Tensor:
    """The 8 spectral features of S (device FP32 tensor)."""
    n = S.shape[0]
    f = torch.empty(8, dtype=torch.float32, device=S.device)
    _check(lib().zf_features(_dev(S, "S", n), n, f.data_ptr(), _stream(stream)))
    return f


def guess_label(S: torch.Tensor, Z: torch.Tensor, stream=None):
    """Least-squares coefficients of p in the S^(1/2)-weighted norm (3 floats)."""
    n = S.shape[0]
    c = (ctypes.c_double * 3)()
    _check(lib().zf_guess_label(_dev(S, "S", n), _dev(Z, "Z", n), n, c, _stream(stream)))
    return [c[0], c[1], c[2]]


def mlp_set_params(theta) -> None:
    a, p = _f32p(theta)
    if a.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} parameters")
    _check(lib().zf_mlp_set_params(p, N_PARAMS))


def mlp_get_params():
    import numpy as np
    a = np.empty(N_PARAMS, dtype=np.float32)
    _check(lib().zf_mlp_get_params(a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), N_PARAMS))
    return a


def mlp_set_norm(mu_x, sd_x, mu_y, sd_y) -> None:
    arrs = [_f32p(x) for x in (mu_x, sd_x, mu_y, sd_y)]
    _check(lib().zf_mlp_set_norm(*[p for _, p in arrs]))


def _f32dev(t: torch.Tensor, cols: int, name: str) -> int:
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 \
            or t.shape[1] != cols:
        raise TypeError(f"{name} must be a contiguous CUDA float32 (batch, {cols}) tensor")
    return t.data_ptr()


def mlp_train_step(feats: torch.Tensor, labels: torch.Tensor, lr: float, stream=None) -> float:
    loss = ctypes.c_float(0.0)
    _check(lib().zf_mlp_train_step(_f32dev(feats, 8, "feats"), _f32dev(labels, 3, "labels"),
                                   feats.shape[0], lr, ctypes.byref(loss), _stream(stream)))
    return loss.value


def mlp_grad(feats: torch.Tensor, labels: torch.Tensor, stream=None):
    import numpy as np
    g = np.empty(N_PARAMS, dtype=np.float32)
    loss = ctypes.c_float(0.0)
    _check(lib().zf_mlp_grad(_f32dev(feats, 8, "feats"), _f32dev(labels, 3, "labels"),
                             feats.shape[0], g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                             ctypes.byref(loss), _stream(stream)))
    return g, loss.value


def mlp_predict(feat: torch.Tensor, stream=None):
    if feat.dtype != torch.float32 or not feat.is_cuda or feat.numel() != 8:
        raise TypeError("feat must be 8 CUDA float32 values")
    c = (ctypes.c_double * 3)()
    _check(lib().zf_mlp_predict(feat.data_ptr(), c, _stream(stream)))
    return [c[0], c[1], c[2]]


def mlp_save(path) -> None:
    """Write the loaded network (normalization + parameters) to path (zf_mlp_save)."""
    _check(lib().zf_mlp_save(os.fsencode(path)))


def mlp_load(path) -> None:
    """Load a network written by mlp_save (zf_mlp_load)."""
    _check(lib().zf_mlp_load(os.fsencode(path)))
