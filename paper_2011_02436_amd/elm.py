"""Python binding of libelm (ctypes over the C ABI in include/elm.h).

Argument marshalling only: tensors are torch device tensors, passed to the
library as raw device pointers with their leading dimension, on the current
torch stream.  Every step of the training path runs in the library's HIP
kernels; there is no CPU fallback, and importing this module fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libelm.so")

ELM_OK = 0
ELM_ERR_NO_CONVERGENCE = 6
ELM_F64, ELM_F32, ELM_BF16, ELM_F16 = 0, 1, 2, 3
ELM_SAMPLE_MAJOR, ELM_NODE_MAJOR = 0, 1

_DT = {torch.float64: ELM_F64, torch.float32: ELM_F32, torch.bfloat16: ELM_BF16,
       torch.float16: ELM_F16}
_LP = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}
_DT_NAME = {ELM_F64: "fp64", ELM_F32: "fp32", ELM_BF16: "bf16", ELM_F16: "fp16"}


class ElmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status} ({_status_string(status)}): {message}")
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("transposed", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("ne_residual", ctypes.c_double),
                ("ne_history", ctypes.c_double * 32)]

    def as_dict(self):
        n = self.iterations + 1 if self.ne_residual >= 0 else 0
        return {"rank": int(self.rank), "transposed": bool(self.transposed),
                "iterations": int(self.iterations), "ne_residual": float(self.ne_residual),
                "ne_history": [float(self.ne_history[i]) for i in range(min(n, 32))]}


class FactorInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("n", ctypes.c_int64), ("transposed", ctypes.c_int32),
                ("gram_dtype", ctypes.c_int32), ("max_diag", ctypes.c_double),
                ("last_pivot", ctypes.c_double), ("first_rejected", ctypes.c_double),
                ("tau", ctypes.c_double), ("noise_floor", ctypes.c_double), ("reliable", ctypes.c_int32),
                ("certified_full_rank", ctypes.c_int32)]

    def as_dict(self):
        return {"rank": int(self.rank), "n": int(self.n), "transposed": bool(self.transposed),
                "gram_dtype": _DT_NAME.get(int(self.gram_dtype), "?"), "max_diag": float(self.max_diag),
                "last_pivot": float(self.last_pivot), "first_rejected": float(self.first_rejected),
                "tau": float(self.tau), "noise_floor": float(self.noise_floor),
                "reliable": bool(self.reliable), "certified_full_rank": int(self.certified_full_rank)}


class TrainInfo(ctypes.Structure):
    _fields_ = [("solve", SolveInfo), ("factor", FactorInfo), ("gram_dtype", ctypes.c_int32),
                ("escalations", ctypes.c_int32), ("guard", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("d", ctypes.c_int64), ("L", ctypes.c_int64), ("m", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("W", ctypes.c_void_p), ("ldw", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("T", ctypes.c_void_p), ("ldt", ctypes.c_int64),
                ("H64", ctypes.c_void_p), ("ldh64", ctypes.c_int64),
                ("beta", ctypes.c_void_p), ("ldbeta", ctypes.c_int64)]


STAGES = ["hidden", "gram", "gram_reduce", "rank", "factor", "solve", "rhs", "residual", "predict"]


class BatchReport(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("grouped_problems", ctypes.c_int32),
                ("worker_problems", ctypes.c_int32), ("escalations", ctypes.c_int32),
                ("batch_stream_syncs", ctypes.c_int32), ("graph_captures", ctypes.c_int32),
                ("graph_launches", ctypes.c_int32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n_log2", ctypes.c_int32),
                ("k_log2", ctypes.c_int32), ("value", ctypes.c_int32)]


TUNE_KINDS = {1: "gram_splits", 2: "gram_chunks", 3: "panel"}


class StageTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("count", ctypes.c_int64 * 9)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2011_02436_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "elm_create": ([ctypes.POINTER(vp), vp], i32),
        "elm_destroy": ([vp], i32),
        "elm_set_stream": ([vp, vp], i32),
        "elm_status_string": ([i32], ctypes.c_char_p),
        "elm_last_error": ([vp], ctypes.c_char_p),
        "elm_hidden": ([vp, i64, i64, i64, vp, i64, vp, i64, vp, i32, vp, i64, vp, i64, i32], i32),
        "elm_rank_factor": ([vp, i64, i64, vp, i64, i32, i32, dbl, ctypes.POINTER(vp),
                             ctypes.POINTER(i64)], i32),
        "elm_gram": ([vp, i64, i64, vp, i64, i32, i32, vp, i64], i32),
        "elm_gram_noalloc": ([vp, i64, i64, vp, i64, i32, i32, vp, i64], i32),
        "elm_factor_rank": ([vp, ctypes.POINTER(i64)], i32),
        "elm_factor_grow": ([vp, vp, i64, i64, vp, i64, dbl, ctypes.POINTER(vp), ctypes.POINTER(i64),
                             ctypes.POINTER(i32)], i32),
        "elm_factor_pivots": ([vp, vp, ctypes.POINTER(i32)], i32),
        "elm_factor_destroy": ([vp], i32),
        "elm_factor_get_info": ([vp, ctypes.POINTER(FactorInfo)], i32),
        "elm_train_batched": ([vp, i32, ctypes.POINTER(Problem), i32, dbl, dbl, i32,
                               ctypes.POINTER(TrainInfo), ctypes.POINTER(i32)], i32),
        "elm_train": ([vp, i64, i64, i64, i64, vp, i64, vp, i64, vp, vp, i64, i32, vp, i64, vp, i64,
                       dbl, dbl, i32, vp, i64, vp, i64, vp, ctypes.POINTER(TrainInfo),
                       ctypes.POINTER(vp)], i32),
        "elm_pinv_solve": ([vp, vp, i64, vp, i64, vp, i64, dbl, i32, vp, i64,
                            ctypes.POINTER(SolveInfo)], i32),
        "elm_train_streamed": ([vp, i64, i64, i64, i64, vp, i64, vp, i64, vp, vp, i64, i32, i64, dbl, dbl,
                                i32, vp, i64, ctypes.POINTER(TrainInfo)], i32),
        "elm_block_solve": ([vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, i64, vp, vp, i64], i32),
        "elm_predict": ([vp, i64, i64, i64, i64, vp, i64, vp, i64, vp, i32, vp, i64, vp, i64, vp],
                        i32),
        "elm_predict_hidden": ([vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp], i32),
        "elm_autotune_gram": ([vp, i64, i64, vp, i64, i32, ctypes.POINTER(i32),
                               ctypes.POINTER(dbl)], i32),
        "elm_set_option": ([vp, i32, i64], i32),
        "elm_get_option": ([vp, i32, ctypes.POINTER(i64)], i32),
        "elm_profile_enable": ([vp, i32], i32),
        "elm_profile_read": ([vp, ctypes.POINTER(StageTimes)], i32),
        "elm_batch_get_report": ([vp, ctypes.POINTER(BatchReport)], i32),
        "elm_tune_table_get": ([vp, ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)], i32),
        "elm_probe_mfma": ([vp, i32, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], i32),
        "elm_probe_stream": ([vp, vp, i64, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], i32),
        "elm_probe_dma": ([vp, vp, i64, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], i32),
        "elm_tune_table_set": ([vp, ctypes.POINTER(TuneEntry), i32], i32),
        "elm_tune_table_save": ([vp, ctypes.c_char_p], i32),
        "elm_tune_table_load": ([vp, ctypes.c_char_p], i32),
        "elm_autotune_batch": ([vp, i32, ctypes.POINTER(Problem), i32, dbl, dbl, i32, ctypes.POINTER(dbl),
                                ctypes.POINTER(dbl)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ["elm_create", "elm_destroy", "elm_set_stream", "elm_status_string", "elm_last_error",
            "elm_hidden", "elm_gram", "elm_gram_noalloc", "elm_rank_factor", "elm_factor_rank", "elm_factor_grow", "elm_factor_pivots",
            "elm_factor_destroy", "elm_factor_get_info", "elm_train", "elm_train_streamed", "elm_train_batched",
            "elm_pinv_solve", "elm_block_solve", "elm_predict", "elm_predict_hidden",
            "elm_autotune_gram", "elm_set_option", "elm_get_option", "elm_profile_enable",
            "elm_profile_read", "elm_batch_get_report", "elm_tune_table_get", "elm_tune_table_set",
            "elm_tune_table_save", "elm_tune_table_load", "elm_autotune_batch", "elm_probe_mfma",
            "elm_probe_stream", "elm_probe_dma"]


def _status_string(st: int) -> str:
    return _lib.elm_status_string(st).decode()


# ----------------------------------------------------------------------------
# handle: one per (device, stream)
# ----------------------------------------------------------------------------
class Handle:
    def __init__(self, device: Optional[int] = None):
        dev = torch.cuda.current_device() if device is None else device
        self.device = dev
        with torch.cuda.device(dev):
            h = ctypes.c_void_p()
            st = _lib.elm_create(ctypes.byref(h), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            if st != ELM_OK:
                raise ElmError(st, "elm_create", "")
        self.ptr = h

    def bind_current_stream(self):
        _lib.elm_set_stream(self.ptr, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, st: int, where: str):
        if st != ELM_OK:
            raise ElmError(st, where, _lib.elm_last_error(self.ptr).decode())

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                _lib.elm_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass


_handles = {}


def handle() -> Handle:
    dev = torch.cuda.current_device()
    h = _handles.get(dev)
    if h is None:
        h = Handle(dev)
        _handles[dev] = h
    h.bind_current_stream()
    return h


def _mat(t: torch.Tensor, name: str):
    """(pointer, leading dimension) of a row-major 2-D device tensor."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    rows, cols = t.shape
    if cols > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit stride along rows")
    ld = t.stride(0) if rows > 1 else cols
    if ld < cols:
        raise ValueError(f"{name}: row stride smaller than the row length")
    return ctypes.c_void_p(t.data_ptr()), max(ld, 1)


def _vec(t: torch.Tensor, name: str):
    if not t.is_cuda or t.dim() != 1 or t.stride(0) != 1:
        raise ValueError(f"{name} must be a contiguous 1-D device tensor")
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------
def elm_hidden(X: torch.Tensor, W: torch.Tensor, b: torch.Tensor,
               H: Optional[torch.Tensor] = None, Hlp: Optional[torch.Tensor] = None) -> None:
    """H = sigmoid(X W + b) into H (N x L, dtype of X) and/or Hlp (L x N)."""
    h = handle()
    N, d = X.shape
    L = W.shape[1]
    if X.dtype not in (torch.float64, torch.float32) or W.dtype != X.dtype or b.dtype != X.dtype:
        raise ValueError("X, W, b must share dtype float64 or float32")
    xp, ldx = _mat(X, "X")
    wp, ldw = _mat(W, "W")
    bp = _vec(b, "b")
    hp, ldh = (ctypes.c_void_p(), 0) if H is None else _mat(H, "H")
    if H is not None and (H.dtype != X.dtype or tuple(H.shape) != (N, L)):
        raise ValueError("H must be N x L with the dtype of X")
    if Hlp is not None:
        if tuple(Hlp.shape) != (L, N) or Hlp.dtype not in (torch.bfloat16, torch.float16, torch.float32):
            raise ValueError("Hlp must be L x N in bfloat16, float16 or float32")
        lp, ldlp = _mat(Hlp, "Hlp")
        lpdt = _DT[Hlp.dtype]
    else:
        lp, ldlp, lpdt = ctypes.c_void_p(), 0, ELM_BF16
    h.check(_lib.elm_hidden(h.ptr, N, d, L, xp, ldx, wp, ldw, bp, _DT[X.dtype], hp, ldh, lp, ldlp,
                            lpdt), "elm_hidden")


def elm_gram(H: torch.Tensor, layout: str = "sample", M: Optional[torch.Tensor] = None,
             noalloc: bool = False) -> torch.Tensor:
    """The FP64 Gram (H^T H, or H H^T when N < L) of a sample-major FP64 H or a
    node-major low-precision copy.  M: optional preallocated n x n float64
    output.  noalloc=True calls elm_gram_noalloc (partials in the library's
    static device array, no device allocation by the library)."""
    h = handle()
    if layout == "sample":
        N, L = H.shape
        lay = ELM_SAMPLE_MAJOR
    else:
        L, N = H.shape
        lay = ELM_NODE_MAJOR
    n = min(N, L)
    if M is None:
        M = torch.empty((n, n), dtype=torch.float64, device=H.device)
    elif M.dtype != torch.float64 or M.shape[0] != n or M.shape[1] < n:
        raise ValueError("M must be float64 with n rows and at least n columns")
    hp, ldh = _mat(H, "H")
    mp, ldm = _mat(M, "M")
    fn, name = (_lib.elm_gram_noalloc, "elm_gram_noalloc") if noalloc else (_lib.elm_gram, "elm_gram")
    h.check(fn(h.ptr, N, L, hp, ldh, _DT[H.dtype], lay, mp, ldm), name)
    return M


class Factor:
    """Library-owned rank factor (permutation, rank, full-rank factorisation)."""

    def __init__(self, ptr: ctypes.c_void_p, N: int, L: int, rank: int):
        self.ptr = ptr
        self.N, self.L, self.rank = N, L, rank

    @property
    def n(self) -> int:
        return min(self.N, self.L)

    def info(self) -> dict:
        """Rank-decision diagnostics: pivots, noise floor, reliability."""
        out = FactorInfo()
        st = _lib.elm_factor_get_info(self.ptr, ctypes.byref(out))
        if st != 0:
            raise ElmError(st, "elm_factor_get_info", "")
        return out.as_dict()

    def pivots(self):
        import numpy as np
        out = np.empty(self.n, dtype=np.int32)
        h = handle()
        h.check(_lib.elm_factor_pivots(h.ptr, self.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                "elm_factor_pivots")
        return out

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                _lib.elm_factor_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass


def elm_rank_factor(H: torch.Tensor, layout: str = "sample", tau_rel: float = 0.0) -> Factor:
    """Rank step on H: FP64 sample-major (N x L), or a node-major (L x N)
    low-precision copy from elm_hidden."""
    h = handle()
    if layout == "sample":
        N, L = H.shape
        lay = ELM_SAMPLE_MAJOR
    elif layout == "node":
        L, N = H.shape
        lay = ELM_NODE_MAJOR
    else:
        raise ValueError("layout must be 'sample' or 'node'")
    hp, ldh = _mat(H, "H")
    f = ctypes.c_void_p()
    r = ctypes.c_int64()
    h.check(_lib.elm_rank_factor(h.ptr, N, L, hp, ldh, _DT[H.dtype], lay, float(tau_rel), ctypes.byref(f),
                                 ctypes.byref(r)), "elm_rank_factor")
    return Factor(f, N, L, int(r.value))


def elm_factor_grow(factor: Factor, H64: torch.Tensor, tau_rel: float = 0.0) -> Tuple[Factor, bool]:
    """The factor of H' = [H Hn] grown from `factor` (of the FP64 column Gram of
    H, the first columns of H64).  Returns (new factor, grown), grown False
    when the library factored H' from scratch."""
    h = handle()
    N, L = H64.shape
    if H64.dtype != torch.float64:
        raise TypeError("H64 must be float64")
    hp, ldh = _mat(H64, "H64")
    out = ctypes.c_void_p()
    r = ctypes.c_int64()
    grown = ctypes.c_int32()
    h.check(_lib.elm_factor_grow(h.ptr, factor.ptr, N, L, hp, ldh, tau_rel, ctypes.byref(out),
                                 ctypes.byref(r), ctypes.byref(grown)), "elm_factor_grow")
    return Factor(out, N, L, int(r.value)), bool(grown.value)


def elm_pinv_solve(factor: Factor, T: torch.Tensor, H64: torch.Tensor, ir_tol: float = 1e-10,
                   ir_max_iter: int = 0, beta: Optional[torch.Tensor] = None,
                   check_convergence: bool = True):
    """beta = H^+ T through the factor, with optional FP64 refinement.
    Returns (beta, info dict)."""
    h = handle()
    N, m = T.shape
    L = factor.L
    if T.dtype != torch.float64 or H64.dtype != torch.float64:
        raise ValueError("T and H64 must be float64")
    if tuple(H64.shape) != (factor.N, factor.L) or N != factor.N:
        raise ValueError("T / H64 shapes do not match the factor")
    if beta is None:
        beta = torch.empty((L, m), dtype=torch.float64, device=T.device)
    tp, ldt = _mat(T, "T")
    hp, ldh = _mat(H64, "H64")
    bp, ldb = _mat(beta, "beta")
    info = SolveInfo()
    st = _lib.elm_pinv_solve(h.ptr, factor.ptr, m, tp, ldt, hp, ldh, float(ir_tol), int(ir_max_iter),
                             bp, ldb, ctypes.byref(info))
    if st == ELM_ERR_NO_CONVERGENCE and not check_convergence:
        st = ELM_OK
    h.check(st, "elm_pinv_solve")
    return beta, info.as_dict()


def elm_block_solve(H64: torch.Tensor, T: torch.Tensor, split: int, M: Optional[torch.Tensor] = None,
                    piv: Optional[torch.Tensor] = None) -> torch.Tensor:
    """beta by the paper's block form (eqs. 19-23) for a full-column-rank
    sample-major FP64 H split after `split` columns of the order piv (int32
    device tensor of L indices; None = identity).  M: optional FP64 Gram
    H^T H (formed by the library when None)."""
    h = handle()
    N, L = H64.shape
    m = T.shape[1]
    if H64.dtype != torch.float64 or T.dtype != torch.float64:
        raise TypeError("H64 and T must be float64")
    hp, ldh = _mat(H64, "H64")
    tp, ldt = _mat(T, "T")
    mp, ldm = (None, 0) if M is None else _mat(M, "M")
    if piv is not None and (piv.dtype != torch.int32 or piv.numel() != L or not piv.is_contiguous()):
        raise ValueError("piv must be a contiguous int32 tensor of L entries")
    pp = None if piv is None else ctypes.c_void_p(piv.data_ptr())
    beta = torch.empty((L, m), dtype=torch.float64, device=H64.device)
    bp, ldb = _mat(beta, "beta")
    h.check(_lib.elm_block_solve(h.ptr, N, L, m, hp, ldh, tp, ldt, mp, ldm, split, pp, bp, ldb),
            "elm_block_solve")
    return beta


def elm_predict(X: torch.Tensor, W: torch.Tensor, b: torch.Tensor, beta: torch.Tensor,
                want_Y: bool = True, want_labels: bool = True):
    """Y = sigmoid(X W + b) beta (dtype of X) and arg-max labels (int32)."""
    h = handle()
    N, d = X.shape
    L = W.shape[1]
    m = beta.shape[1]
    xp, ldx = _mat(X, "X")
    wp, ldw = _mat(W, "W")
    bp = _vec(b, "b")
    betap, ldbeta = _mat(beta, "beta")
    if beta.dtype != torch.float64:
        raise ValueError("beta must be float64")
    Y = torch.empty((N, m), dtype=X.dtype, device=X.device) if want_Y else None
    labels = torch.empty(N, dtype=torch.int32, device=X.device) if want_labels else None
    yp, ldy = (ctypes.c_void_p(), 0) if Y is None else _mat(Y, "Y")
    lp = ctypes.c_void_p() if labels is None else ctypes.c_void_p(labels.data_ptr())
    h.check(_lib.elm_predict(h.ptr, N, d, L, m, xp, ldx, wp, ldw, bp, _DT[X.dtype], betap, ldbeta, yp, ldy,
                             lp), "elm_predict")
    return Y, labels


def autotune_gram(H: torch.Tensor, layout: str = "node") -> Tuple[int, float]:
    """elm_autotune_gram: times the Gram of H with several K-split (16-bit,
    node-major L x N copy) or K-chunk (FP32 node-major, FP64 sample-major
    N x L) counts and keeps the fastest as the handle's table row for this
    shape's buckets.  Returns (count, milliseconds)."""
    if H.dim() != 2 or H.stride(1) != 1:
        raise ValueError("H must be a row-major 2-D tensor")
    if layout == "sample":
        if H.dtype != torch.float64:
            raise ValueError("a sample-major H must be float64")
        N, L = H.shape
    else:
        if H.dtype not in (torch.bfloat16, torch.float16, torch.float32):
            raise ValueError("a node-major H must be bfloat16, float16 or float32")
        L, N = H.shape
    h = handle()
    sp = ctypes.c_int32()
    ms = ctypes.c_double()
    h.check(_lib.elm_autotune_gram(h.ptr, N, L, ctypes.c_void_p(H.data_ptr()), H.stride(0),
                                   _DT[H.dtype], ctypes.byref(sp), ctypes.byref(ms)),
            "elm_autotune_gram")
    return int(sp.value), float(ms.value)


OPTIONS = {"full_rank_min_order": 1, "batch_workers": 2}


def set_option(name: str, value: int) -> int:
    """Set a tuning option of the current device's handle (elm_set_option);
    returns the previous value."""
    if name not in OPTIONS:
        raise ValueError(f"unknown option {name!r}; known: {sorted(OPTIONS)}")
    h = handle()
    old = ctypes.c_int64()
    h.check(_lib.elm_get_option(h.ptr, OPTIONS[name], ctypes.byref(old)), "elm_get_option")
    h.check(_lib.elm_set_option(h.ptr, OPTIONS[name], int(value)), "elm_set_option")
    return int(old.value)


def get_option(name: str) -> int:
    if name not in OPTIONS:
        raise ValueError(f"unknown option {name!r}; known: {sorted(OPTIONS)}")
    h = handle()
    v = ctypes.c_int64()
    h.check(_lib.elm_get_option(h.ptr, OPTIONS[name], ctypes.byref(v)), "elm_get_option")
    return int(v.value)


def profile_enable(on: bool = True) -> None:
    """Start (and reset) or stop the library's HIP-event stage timers."""
    h = handle()
    h.check(_lib.elm_profile_enable(h.ptr, 1 if on else 0), "elm_profile_enable")


def profile_read() -> dict:
    """{stage: (total_ms, count)} since the last profile_enable(True)."""
    h = handle()
    st = StageTimes()
    h.check(_lib.elm_profile_read(h.ptr, ctypes.byref(st)), "elm_profile_read")
    return {name: (float(st.ms[i]), int(st.count[i])) for i, name in enumerate(STAGES)}


def tune_table() -> list:
    """The handle's tuning table as a list of dicts."""
    h = handle()
    n = ctypes.c_int32()
    h.check(_lib.elm_tune_table_get(h.ptr, None, 0, ctypes.byref(n)), "elm_tune_table_get")
    rows = (TuneEntry * max(n.value, 1))()
    h.check(_lib.elm_tune_table_get(h.ptr, rows, n.value, ctypes.byref(n)), "elm_tune_table_get")
    return [{"kind": TUNE_KINDS.get(r.kind, r.kind), "dtype": _DT_NAME.get(r.dtype, "any"),
             "n_log2": r.n_log2, "k_log2": r.k_log2, "value": r.value} for r in rows[:n.value]]


def tune_table_set(rows: list) -> None:
    """Replace the table (rows as returned by tune_table)."""
    h = handle()
    kinds = {v: k for k, v in TUNE_KINDS.items()}
    dts = {v: k for k, v in _DT_NAME.items()}
    arr = (TuneEntry * max(len(rows), 1))()
    for i, r in enumerate(rows):
        arr[i] = TuneEntry(kinds[r["kind"]], dts.get(r["dtype"], -1), r["n_log2"], r["k_log2"], r["value"])
    h.check(_lib.elm_tune_table_set(h.ptr, arr, len(rows)), "elm_tune_table_set")


def tune_table_save(path: str) -> None:
    h = handle()
    h.check(_lib.elm_tune_table_save(h.ptr, path.encode()), "elm_tune_table_save")


def tune_table_load(path: str) -> None:
    h = handle()
    h.check(_lib.elm_tune_table_load(h.ptr, path.encode()), "elm_tune_table_load")


def _problem_array(problems, H64s=None, betas=None):
    count = len(problems)
    arr = (Problem * max(count, 1))()
    keep = []
    for e, (X, W, b, T) in enumerate(problems):
        N, d = X.shape
        L = W.shape[1]
        m = T.shape[1]
        H64 = H64s[e] if H64s is not None else torch.empty((N, L), dtype=torch.float64, device=X.device)
        beta = betas[e] if betas is not None else torch.empty((L, m), dtype=torch.float64, device=X.device)
        keep += [H64, beta]
        xp, ldx = _mat(X, "X")
        wp, ldw = _mat(W, "W")
        tp, ldt = _mat(T, "T")
        hp, ldh = _mat(H64, "H64")
        bp, ldb = _mat(beta, "beta")
        arr[e] = Problem(N, d, L, m, xp.value, ldx, wp.value, ldw, _vec(b, "b").value, tp.value, ldt,
                         hp.value, ldh, bp.value, ldb)
    return arr, keep


def autotune_batch(problems, precision: str = "bf16", ir_tol: float = 1e-10,
                   ir_max_iter: Optional[int] = None, tau_rel: float = 0.0, H64s=None, betas=None):
    """elm_autotune_batch over a list of (X, W, b, T): returns (ms before,
    ms after); the choice goes to the handle's tuning table."""
    h = handle()
    arr, keep = _problem_array(problems, H64s, betas)
    gdt = {"fp64": ELM_F64, "fp32": ELM_F32, "bf16": ELM_BF16, "fp16": ELM_F16}[precision]
    its = (2 if precision == "fp64" else 30) if ir_max_iter is None else ir_max_iter
    before, after = ctypes.c_double(), ctypes.c_double()
    h.check(_lib.elm_autotune_batch(h.ptr, len(problems), arr, gdt, tau_rel, ir_tol, its, ctypes.byref(before),
                                    ctypes.byref(after)), "elm_autotune_batch")
    del keep
    return before.value, after.value


def probe_mfma(dtype: str = "bf16", random_operands: bool = True, shape: int = 0) -> Tuple[float, float]:
    """Sustained MFMA rate from registers: (TFLOP/s, ms).  shape 0: 32x32x16
    BF16 or 16x16x4 FP64; shape 1 (FP64): the four-block 4x4x4 instruction."""
    h = handle()
    tf, ms = ctypes.c_double(), ctypes.c_double()
    h.check(_lib.elm_probe_mfma(h.ptr, {"bf16": ELM_BF16, "fp64": ELM_F64}[dtype], int(shape),
                                1 if random_operands else 0, ctypes.byref(tf), ctypes.byref(ms)),
            "elm_probe_mfma")
    return tf.value, ms.value


def probe_stream(buf: torch.Tensor) -> Tuple[float, float]:
    """Streaming read of a device tensor: (GB/s, ms)."""
    h = handle()
    gbs, ms = ctypes.c_double(), ctypes.c_double()
    h.check(_lib.elm_probe_stream(h.ptr, ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                  ctypes.byref(gbs), ctypes.byref(ms)), "elm_probe_stream")
    return gbs.value, ms.value


def probe_dma(buf: torch.Tensor, resident: bool = False) -> Tuple[float, float]:
    """Direct global->LDS staging as the 16-bit Gram does it: (GB/s, ms)."""
    h = handle()
    gbs, ms = ctypes.c_double(), ctypes.c_double()
    h.check(_lib.elm_probe_dma(h.ptr, ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                               1 if resident else 0, ctypes.byref(gbs), ctypes.byref(ms)), "elm_probe_dma")
    return gbs.value, ms.value


def batch_report() -> dict:
    """How the last train_batched call ran (groups, grouped and worker
    problems, escalations, batch-stream synchronisations, HIP graphs)."""
    h = handle()
    out = BatchReport()
    h.check(_lib.elm_batch_get_report(h.ptr, ctypes.byref(out)), "elm_batch_get_report")
    return out.as_dict()


def elm_predict_hidden(H: torch.Tensor, beta: torch.Tensor, want_Y: bool = True,
                       want_labels: bool = True):
    """Y = H beta and arg-max labels from a stored FP64 sample-major H."""
    h = handle()
    N, L = H.shape
    m = beta.shape[1]
    if H.dtype != torch.float64 or beta.dtype != torch.float64:
        raise ValueError("H and beta must be float64")
    if beta.shape[0] != L:
        raise ValueError("beta must have L rows")
    hp, ldh = _mat(H, "H")
    bp, ldb = _mat(beta, "beta")
    Y = torch.empty((N, m), dtype=torch.float64, device=H.device) if want_Y else None
    labels = torch.empty(N, dtype=torch.int32, device=H.device) if want_labels else None
    yp, ldy = (ctypes.c_void_p(), 0) if Y is None else _mat(Y, "Y")
    lp = ctypes.c_void_p() if labels is None else ctypes.c_void_p(labels.data_ptr())
    h.check(_lib.elm_predict_hidden(h.ptr, N, L, m, hp, ldh, bp, ldb, yp, ldy, lp), "elm_predict_hidden")
    return Y, labels


# ----------------------------------------------------------------------------
# the whole training path as one call (composition of the entry points)
# ----------------------------------------------------------------------------
@dataclass
class TrainResult:
    beta: torch.Tensor
    rank: int
    info: dict
    factor: Factor = field(repr=False, default=None)
    Y: Optional[torch.Tensor] = field(repr=False, default=None)       # H beta (training set)
    labels: Optional[torch.Tensor] = field(repr=False, default=None)  # row arg-max of H beta


def train(X: torch.Tensor, W: torch.Tensor, b: torch.Tensor, T: torch.Tensor, precision: str = "fp64",
          ir_tol: float = 1e-10, ir_max_iter: Optional[int] = None, tau_rel: float = 0.0,
          H64: Optional[torch.Tensor] = None, Hlp: Optional[torch.Tensor] = None,
          check_convergence: bool = True, outputs: bool = False) -> TrainResult:
    """H = g(XW + b) -> rank factor -> beta = H^+ T (+ FP64 refinement), one
    elm_train call.  outputs=True also returns the training-set outputs
    Y = H beta and their arg-max labels, taken from the last refinement pass.

    precision: 'fp64' (FP64 Gram), or 'fp32' / 'bf16' / 'fp16' (Gram of a
    node-major low-precision copy; the rank decision and the refinement
    residual stay in FP64, and a failed guard moves the Gram one precision
    up).  X, W, b, T must be float64; H64 (N x L float64) and Hlp (L x N of
    the precision's dtype; for the fastest Gram a view of rows padded to a
    multiple of 64 elements, e.g. torch.empty((L, -(-N // 64) * 64))[:, :N])
    may be passed preallocated to keep allocation out of timed regions.  info
    holds the solve report plus 'factor' (rank
    diagnostics), 'gram_dtype', 'escalations' and 'guard'."""
    if precision not in ("fp64", "fp32", "bf16", "fp16"):
        raise ValueError("precision must be one of fp64, fp32, bf16, fp16")
    h = handle()
    N, d = X.shape
    L = W.shape[1]
    m = T.shape[1]
    for name, t in (("X", X), ("W", W), ("b", b), ("T", T)):
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
    if H64 is None:
        H64 = torch.empty((N, L), dtype=torch.float64, device=X.device)
    gdt = {"fp64": ELM_F64, "fp32": ELM_F32, "bf16": ELM_BF16, "fp16": ELM_F16}[precision]
    lp_ptr, ldlp = None, 0
    if precision != "fp64" and Hlp is not None:
        if Hlp.dtype != _LP[precision] or tuple(Hlp.shape) != (L, N):
            raise ValueError("Hlp must be L x N of the precision's dtype")
        lp_ptr, ldlp = _mat(Hlp, "Hlp")
    its = (2 if precision == "fp64" else 30) if ir_max_iter is None else ir_max_iter
    xp, ldx = _mat(X, "X")
    wp, ldw = _mat(W, "W")
    tp, ldt = _mat(T, "T")
    hp, ldh = _mat(H64, "H64")
    beta = torch.empty((L, m), dtype=torch.float64, device=X.device)
    bp, ldb = _mat(beta, "beta")
    Y = labels = None
    yp, ldy, lp_lab = None, 0, None
    if outputs:
        Y = torch.empty((N, m), dtype=torch.float64, device=X.device)
        labels = torch.empty((N,), dtype=torch.int32, device=X.device)
        yp, ldy = _mat(Y, "Y")
        lp_lab = _vec(labels, "labels")
    ti = TrainInfo()
    fptr = ctypes.c_void_p()
    st = _lib.elm_train(h.ptr, N, d, L, m, xp, ldx, wp, ldw, _vec(b, "b"), tp, ldt, gdt, hp, ldh,
                        lp_ptr, ldlp, tau_rel, ir_tol, its, bp, ldb, yp, ldy, lp_lab, ctypes.byref(ti),
                        ctypes.byref(fptr))
    if st == ELM_ERR_NO_CONVERGENCE and not check_convergence:
        pass
    else:
        h.check(st, "elm_train")
    info = ti.solve.as_dict()
    info["factor"] = ti.factor.as_dict()
    info["gram_dtype"] = _DT_NAME.get(int(ti.gram_dtype), "?")
    info["escalations"] = int(ti.escalations)
    info["guard"] = int(ti.guard)
    factor = Factor(fptr, N, L, int(ti.factor.rank)) if fptr.value else None
    return TrainResult(beta, int(ti.factor.rank), info, factor, Y, labels)


def train_streamed(X: torch.Tensor, W: torch.Tensor, b: torch.Tensor, T: torch.Tensor,
                   precision: str = "fp64", chunk_rows: int = 65536, ir_tol: float = 1e-10,
                   ir_max_iter: Optional[int] = None, tau_rel: float = 0.0,
                   check_convergence: bool = True) -> TrainResult:
    """elm_train_streamed: the training without storing H (formed chunk_rows
    samples at a time for the Gram and again for each refinement residual)."""
    if precision not in ("fp64", "fp32", "bf16", "fp16"):
        raise ValueError("precision must be one of fp64, fp32, bf16, fp16")
    h = handle()
    N, d = X.shape
    L = W.shape[1]
    m = T.shape[1]
    for name, t in (("X", X), ("W", W), ("b", b), ("T", T)):
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
    gdt = {"fp64": ELM_F64, "fp32": ELM_F32, "bf16": ELM_BF16, "fp16": ELM_F16}[precision]
    its = (2 if precision == "fp64" else 30) if ir_max_iter is None else ir_max_iter
    xp, ldx = _mat(X, "X")
    wp, ldw = _mat(W, "W")
    tp, ldt = _mat(T, "T")
    beta = torch.empty((L, m), dtype=torch.float64, device=X.device)
    bp, ldb = _mat(beta, "beta")
    ti = TrainInfo()
    st = _lib.elm_train_streamed(h.ptr, N, d, L, m, xp, ldx, wp, ldw, _vec(b, "b"), tp, ldt, gdt,
                                 int(chunk_rows), tau_rel, ir_tol, its, bp, ldb, ctypes.byref(ti))
    if not (st == ELM_ERR_NO_CONVERGENCE and not check_convergence):
        h.check(st, "elm_train_streamed")
    info = _train_info_dict(ti)
    return TrainResult(beta, int(ti.factor.rank), info)


def _train_info_dict(ti: TrainInfo) -> dict:
    info = ti.solve.as_dict()
    info["factor"] = ti.factor.as_dict()
    info["gram_dtype"] = _DT_NAME.get(int(ti.gram_dtype), "?")
    info["escalations"] = int(ti.escalations)
    info["guard"] = int(ti.guard)
    return info


def train_batched(problems, precision: str = "fp64", ir_tol: float = 1e-10,
                  ir_max_iter: Optional[int] = None, tau_rel: float = 0.0, H64s=None,
                  betas=None, check: bool = True):
    """elm_train_batched over a list of (X, W, b, T) float64 device tensors.

    H64s / betas: optional lists of preallocated N x L / L x m float64
    buffers.  Returns (betas, infos, statuses); with check=True a failed
    problem raises ElmError."""
    if precision not in ("fp64", "fp32", "bf16", "fp16"):
        raise ValueError("precision must be one of fp64, fp32, bf16, fp16")
    h = handle()
    count = len(problems)
    arr = (Problem * max(count, 1))()
    keep = []
    out_betas = []
    for e, (X, W, b, T) in enumerate(problems):
        for name, t in (("X", X), ("W", W), ("b", b), ("T", T)):
            if t.dtype != torch.float64:
                raise TypeError(f"problem {e}: {name} must be float64")
        N, d = X.shape
        L = W.shape[1]
        m = T.shape[1]
        H64 = H64s[e] if H64s is not None else torch.empty((N, L), dtype=torch.float64, device=X.device)
        beta = betas[e] if betas is not None else torch.empty((L, m), dtype=torch.float64, device=X.device)
        keep.append(H64)
        out_betas.append(beta)
        xp, ldx = _mat(X, "X")
        wp, ldw = _mat(W, "W")
        tp, ldt = _mat(T, "T")
        hp, ldh = _mat(H64, "H64")
        bp, ldb = _mat(beta, "beta")
        arr[e] = Problem(N, d, L, m, xp.value, ldx, wp.value, ldw, _vec(b, "b").value, tp.value, ldt,
                         hp.value, ldh, bp.value, ldb)
    gdt = {"fp64": ELM_F64, "fp32": ELM_F32, "bf16": ELM_BF16, "fp16": ELM_F16}[precision]
    its = (2 if precision == "fp64" else 30) if ir_max_iter is None else ir_max_iter
    infos = (TrainInfo * max(count, 1))()
    stats = (ctypes.c_int32 * max(count, 1))()
    st = _lib.elm_train_batched(h.ptr, count, arr, gdt, tau_rel, ir_tol, its, infos, stats)
    if check:
        h.check(st, "elm_train_batched")
    return out_betas, [_train_info_dict(infos[e]) for e in range(count)], [int(stats[e]) for e in range(count)]
