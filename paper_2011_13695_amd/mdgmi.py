"""Thin ctypes binding of libmdgmi (include/mdgmi.h), same names as the C ABI.

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every step of the computation runs in the library's HIP
kernels. Importing this module never falls back to anything else: if the
shared library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import re
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().with_name("libmdgmi.so")
HEADER = Path(__file__).resolve().parents[1] / "include" / "mdgmi.h"

MDGMI_OK = 0
MDGMI_E_NULL = -1
MDGMI_E_SHAPE = -2
MDGMI_E_LABELS = -3
MDGMI_E_SIGMA2 = -4
MDGMI_E_UNSUPPORTED = -5
MDGMI_E_WORKSPACE = -6
MDGMI_E_HIP = -7
MDGMI_E_DEVICE = -8
MDGMI_E_ARG = -9

MDGMI_PATH_F64 = 0
MDGMI_PATH_F32_DIRECT = 1
MDGMI_PATH_F32_MFMA_F16SPLIT = 2
MDGMI_PATH_F32_MFMA_BF16SPLIT = 3
MDGMI_PATH_LEARNED_BF16 = 4
MDGMI_PATH_AUTO = 5
PATHS = {"f64": MDGMI_PATH_F64, "direct": MDGMI_PATH_F32_DIRECT,
         "mfma": MDGMI_PATH_F32_MFMA_F16SPLIT, "mfma_bf16": MDGMI_PATH_F32_MFMA_BF16SPLIT,
         "learned": MDGMI_PATH_LEARNED_BF16, "auto": MDGMI_PATH_AUTO}

MDGMI_NFIELDS = 6
FIELDS = ("gmi", "mi", "se_gmi", "se_mi", "n", "n_nonfinite")
MDGMI_NFIELDS_HD = 8
FIELDS_HD = FIELDS + ("ber", "ser")
MDGMI_NFIELDS_S = 9
FIELDS_S = ("gmi_s1", "se_s1", "s_opt", "gmi_sopt", "se_sopt", "ngmi", "n", "n_nonfinite", "iterations")


class MdgmiError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        super().__init__(f"{fn}: {mdgmi_status_string(code)} ({code})")


_lib = None
_P = ctypes.c_void_p


def lib():
    """Load libmdgmi.so (built in-tree by paper_2011_13695_amd.build)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2011_13695_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        L.mdgmi_status_string.restype = ctypes.c_char_p
        L.mdgmi_status_string.argtypes = [ctypes.c_int]
        L.mdgmi_validate_labels.argtypes = [_P, ctypes.c_int32]
        L.mdgmi_format_create.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]
        L.mdgmi_format_destroy.argtypes = [_P]
        L.mdgmi_generate.argtypes = [_P, ctypes.c_uint64, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                     _P, _P, ctypes.c_int32, _P]
        L.mdgmi_llr_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.mdgmi_llr.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_double, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P]
        L.mdgmi_gmi_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.mdgmi_gmi.argtypes = [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                ctypes.c_size_t, _P]
        L.mdgmi_gmi_hd_workspace_size.argtypes = L.mdgmi_gmi_workspace_size.argtypes
        L.mdgmi_gmi_static.argtypes = [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]
        L.mdgmi_gmi_hd.argtypes = L.mdgmi_gmi.argtypes
        L.mdgmi_llr_maxlog.argtypes = L.mdgmi_llr.argtypes
        L.mdgmi_gmi_maxlog.argtypes = L.mdgmi_gmi.argtypes
        L.mdgmi_gmi_sopt_workspace_size.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.mdgmi_gmi_sopt.argtypes = [_P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P]
        L.mdgmi_gmi_bits_workspace_size.argtypes = L.mdgmi_gmi_sopt_workspace_size.argtypes
        L.mdgmi_gmi_bits.argtypes = L.mdgmi_gmi_sopt.argtypes
        L.mdgmi_q_factor_db.restype = ctypes.c_double
        L.mdgmi_q_factor_db.argtypes = [ctypes.c_double]
        L.mdgmi_set_tuning.argtypes = [ctypes.c_int]
        L.mdgmi_probe_rates.argtypes = [_P]
        _lib = L
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions include/mdgmi.h declares."""
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(mdgmi_\w+)\s*\(", text, re.M)))


def _check(fn: str, code: int):
    if code != MDGMI_OK:
        raise MdgmiError(fn, code)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _path(path) -> int:
    return PATHS[path] if isinstance(path, str) else int(path)


def _check_y(y, path: int, tx_idx=None):
    """The element type of y follows the path (double on the FP64 path, float
    otherwise; AUTO never resolves to FP64); sent rows are 32-bit."""
    import torch
    want = torch.float64 if path == MDGMI_PATH_F64 else torch.float32
    if y.dtype != want:
        raise TypeError(f"y must be {want} on this path, got {y.dtype}")
    if tx_idx is not None and tx_idx.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"tx_idx must be a 32-bit integer tensor, got {tx_idx.dtype}")


def mdgmi_status_string(code: int) -> str:
    return lib().mdgmi_status_string(int(code)).decode()


def mdgmi_validate_labels(labels) -> int:
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    return int(lib().mdgmi_validate_labels(lab.ctypes.data_as(_P), lab.size))


def mdgmi_set_tuning(mfma_variant: int) -> None:
    lib().mdgmi_set_tuning(int(mfma_variant))


class Format:
    """An mdgmi_format handle: a constellation staged on the current device."""

    def __init__(self, X, labels):
        X = np.ascontiguousarray(X, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.uint32)
        self.M, self.dim = X.shape
        self.m = int(self.M).bit_length() - 1
        h = _P()
        _check("mdgmi_format_create",
               lib().mdgmi_format_create(X.ctypes.data_as(_P), lab.ctypes.data_as(_P), self.M, self.dim,
                                         ctypes.byref(h)))
        self.handle = h

    @classmethod
    def of(cls, fmt):
        """From a workloads.Format (or anything with X and labels)."""
        return cls(fmt.X, fmt.labels)

    def close(self):
        if getattr(self, "handle", None):
            lib().mdgmi_format_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdgmi_generate(fmt: Format, seed: int, sigma2, n: int, snr_slot0: int = 0, y=None, tx_idx=None,
                   dtype=None, stream=None):
    """Seeded channel samples on the device: returns (y [n_snr, n, dim], tx [n_snr, n])."""
    import torch
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    dtype = dtype or (y.dtype if y is not None else torch.float32)
    if y is None:
        y = torch.empty((n_snr, n, fmt.dim), dtype=dtype, device="cuda")
    if tx_idx is None:
        tx_idx = torch.empty((n_snr, n), dtype=torch.int32, device="cuda")
    assert y.is_contiguous() and tx_idx.is_contiguous() and y.dtype in (torch.float32, torch.float64)
    assert tuple(y.shape) == (n_snr, n, fmt.dim) and tuple(tx_idx.shape) == (n_snr, n)
    _check("mdgmi_generate",
           lib().mdgmi_generate(fmt.handle, int(seed) & 0xFFFFFFFFFFFFFFFF, s2.ctypes.data_as(_P), n_snr, n,
                                snr_slot0, _dptr(y), _dptr(tx_idx), int(y.dtype == torch.float64),
                                _stream(stream)))
    return y, tx_idx


def mdgmi_llr_workspace_size(fmt: Format, n: int, path="auto") -> int:
    b = ctypes.c_size_t()
    _check("mdgmi_llr_workspace_size", lib().mdgmi_llr_workspace_size(fmt.handle, n, _path(path), ctypes.byref(b)))
    return int(b.value)


def mdgmi_gmi_workspace_size(fmt: Format, n: int, n_snr: int, path="auto") -> int:
    b = ctypes.c_size_t()
    _check("mdgmi_gmi_workspace_size",
           lib().mdgmi_gmi_workspace_size(fmt.handle, n, n_snr, _path(path), ctypes.byref(b)))
    return int(b.value)


def workspace(nbytes: int):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def mdgmi_llr(fmt: Format, y, sigma2: float, path="auto", llr=None, ws=None, stream=None):
    """Per-bit LLRs (nats) of y [n, dim] -> [n, m] (FP64 path: double, else float)."""
    import torch
    assert y.is_cuda and y.is_contiguous() and y.shape[-1] == fmt.dim
    n = y.numel() // fmt.dim
    p = _path(path)
    _check_y(y, p)
    if llr is None:
        llr = torch.empty((n, fmt.m), dtype=y.dtype, device=y.device)
    if ws is None:
        ws = workspace(mdgmi_llr_workspace_size(fmt, n, p))
    _check("mdgmi_llr", lib().mdgmi_llr(fmt.handle, _dptr(y), n, float(sigma2), _dptr(llr), p, _dptr(ws),
                                        ws.numel(), _stream(stream)))
    return llr


def mdgmi_gmi(fmt: Format, y, tx_idx, sigma2, path="auto", out=None, ws=None, stream=None):
    """GMI/MI per SNR: y [n_snr, n, dim], tx [n_snr, n] -> out [n_snr, 6] (double)."""
    import torch
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    assert y.is_cuda and y.is_contiguous() and tx_idx.is_contiguous()
    n = y.numel() // (fmt.dim * n_snr)
    assert y.numel() == n_snr * n * fmt.dim and tx_idx.numel() == n_snr * n
    p = _path(path)
    _check_y(y, p, tx_idx)
    if out is None:
        out = torch.empty((n_snr, MDGMI_NFIELDS), dtype=torch.float64, device=y.device)
    if ws is None:
        ws = workspace(mdgmi_gmi_workspace_size(fmt, n, n_snr, p))
    _check("mdgmi_gmi", lib().mdgmi_gmi(fmt.handle, _dptr(y), _dptr(tx_idx), n, s2.ctypes.data_as(_P), n_snr, p,
                                        _dptr(out), _dptr(ws), ws.numel(), _stream(stream)))
    return out


MDGMI_STATIC_SCRATCH_BYTES = 16 << 20


def mdgmi_gmi_static(fmt: Format, y, tx_idx, sigma2, path="auto", out=None, stream=None):
    """mdgmi_gmi with the library's static scratch array instead of a
    workspace (no allocation inside the call; `out` may be preallocated)."""
    import torch
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    assert y.is_cuda and y.is_contiguous() and tx_idx.is_contiguous()
    n = y.numel() // (fmt.dim * n_snr)
    assert y.numel() == n_snr * n * fmt.dim and tx_idx.numel() == n_snr * n
    p = _path(path)
    _check_y(y, p, tx_idx)
    if out is None:
        out = torch.empty((n_snr, MDGMI_NFIELDS), dtype=torch.float64, device=y.device)
    _check("mdgmi_gmi_static", lib().mdgmi_gmi_static(fmt.handle, _dptr(y), _dptr(tx_idx), n,
                                                      s2.ctypes.data_as(_P), n_snr, p, _dptr(out), _stream(stream)))
    return out


def mdgmi_gmi_hd_workspace_size(fmt: Format, n: int, n_snr: int, path="auto") -> int:
    b = ctypes.c_size_t()
    _check("mdgmi_gmi_hd_workspace_size",
           lib().mdgmi_gmi_hd_workspace_size(fmt.handle, n, n_snr, _path(path), ctypes.byref(b)))
    return int(b.value)


def mdgmi_gmi_hd(fmt: Format, y, tx_idx, sigma2, path="auto", out=None, ws=None, stream=None):
    """GMI/MI plus hard-decision BER and SER per SNR -> out [n_snr, 8] (double)."""
    import torch
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    assert y.is_cuda and y.is_contiguous() and tx_idx.is_contiguous()
    n = y.numel() // (fmt.dim * n_snr)
    assert y.numel() == n_snr * n * fmt.dim and tx_idx.numel() == n_snr * n
    p = _path(path)
    _check_y(y, p, tx_idx)
    if out is None:
        out = torch.empty((n_snr, MDGMI_NFIELDS_HD), dtype=torch.float64, device=y.device)
    if ws is None:
        ws = workspace(mdgmi_gmi_hd_workspace_size(fmt, n, n_snr, p))
    _check("mdgmi_gmi_hd", lib().mdgmi_gmi_hd(fmt.handle, _dptr(y), _dptr(tx_idx), n, s2.ctypes.data_as(_P), n_snr,
                                              p, _dptr(out), _dptr(ws), ws.numel(), _stream(stream)))
    return out


def mdgmi_llr_maxlog(fmt: Format, y, sigma2: float, path="auto", llr=None, ws=None, stream=None):
    """Max-log LLRs (nats) of y [n, dim] -> [n, m] (FP64 path: double, else float)."""
    import torch
    assert y.is_cuda and y.is_contiguous() and y.shape[-1] == fmt.dim
    n = y.numel() // fmt.dim
    p = _path(path)
    _check_y(y, p)
    if llr is None:
        llr = torch.empty((n, fmt.m), dtype=y.dtype, device=y.device)
    if ws is None:
        ws = workspace(mdgmi_llr_workspace_size(fmt, n, p))
    _check("mdgmi_llr_maxlog", lib().mdgmi_llr_maxlog(fmt.handle, _dptr(y), n, float(sigma2), _dptr(llr), p,
                                                      _dptr(ws), ws.numel(), _stream(stream)))
    return llr


def mdgmi_gmi_maxlog(fmt: Format, y, tx_idx, sigma2, path="auto", out=None, ws=None, stream=None):
    """GMI of the max-log LLRs per SNR -> out [n_snr, 6] (MI fields NaN)."""
    import torch
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    assert y.is_cuda and y.is_contiguous() and tx_idx.is_contiguous()
    n = y.numel() // (fmt.dim * n_snr)
    assert y.numel() == n_snr * n * fmt.dim and tx_idx.numel() == n_snr * n
    p = _path(path)
    _check_y(y, p, tx_idx)
    if out is None:
        out = torch.empty((n_snr, MDGMI_NFIELDS), dtype=torch.float64, device=y.device)
    if ws is None:
        ws = workspace(mdgmi_gmi_workspace_size(fmt, n, n_snr, p))
    _check("mdgmi_gmi_maxlog", lib().mdgmi_gmi_maxlog(fmt.handle, _dptr(y), _dptr(tx_idx), n, s2.ctypes.data_as(_P),
                                                      n_snr, p, _dptr(out), _dptr(ws), ws.numel(), _stream(stream)))
    return out


def mdgmi_gmi_sopt_workspace_size(n: int) -> int:
    b = ctypes.c_size_t()
    _check("mdgmi_gmi_sopt_workspace_size", lib().mdgmi_gmi_sopt_workspace_size(n, ctypes.byref(b)))
    return int(b.value)


def mdgmi_gmi_sopt(fmt: Format, llr, tx_idx, out=None, ws=None, stream=None):
    """s-optimised GMI of LLRs [n, m] (float32 or float64, nats) for the sent
    rows tx [n] -> out [9] (double, fields FIELDS_S)."""
    import torch
    assert llr.is_cuda and llr.is_contiguous() and tx_idx.is_contiguous()
    assert llr.dtype in (torch.float32, torch.float64)
    n = llr.numel() // fmt.m
    assert llr.numel() == n * fmt.m and tx_idx.numel() == n
    if out is None:
        out = torch.empty(MDGMI_NFIELDS_S, dtype=torch.float64, device=llr.device)
    if ws is None:
        ws = workspace(mdgmi_gmi_sopt_workspace_size(n))
    _check("mdgmi_gmi_sopt", lib().mdgmi_gmi_sopt(fmt.handle, _dptr(llr), int(llr.dtype == torch.float64),
                                                  _dptr(tx_idx), n, _dptr(out), _dptr(ws), ws.numel(),
                                                  _stream(stream)))
    return out


def mdgmi_gmi_bits(fmt: Format, llr, tx_idx, out=None, ws=None, stream=None):
    """Per-bit GMI of LLRs [n, m] (float32 or float64, nats) for the sent rows
    tx [n] -> out [2 m + 2] (double): GMI_k and its standard error per bit,
    then n and the non-finite count."""
    import torch
    assert llr.is_cuda and llr.is_contiguous() and tx_idx.is_contiguous()
    assert llr.dtype in (torch.float32, torch.float64)
    n = llr.numel() // fmt.m
    assert llr.numel() == n * fmt.m and tx_idx.numel() == n
    if out is None:
        out = torch.empty(2 * fmt.m + 2, dtype=torch.float64, device=llr.device)
    if ws is None:
        b = ctypes.c_size_t()
        _check("mdgmi_gmi_bits_workspace_size", lib().mdgmi_gmi_bits_workspace_size(n, ctypes.byref(b)))
        ws = workspace(b.value)
    _check("mdgmi_gmi_bits", lib().mdgmi_gmi_bits(fmt.handle, _dptr(llr), int(llr.dtype == torch.float64),
                                                  _dptr(tx_idx), n, _dptr(out), _dptr(ws), ws.numel(),
                                                  _stream(stream)))
    return out


def _stream_sigs():
    L = lib()
    if getattr(L, "_stream_sigs", False):
        return L
    L.mdgmi_stream_create.argtypes = [_P, ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.POINTER(_P)]
    L.mdgmi_stream_push.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    L.mdgmi_stream_wait.argtypes = [_P, ctypes.c_int64]
    L.mdgmi_stream_result.argtypes = [_P, ctypes.c_int64, _P]
    L.mdgmi_stream_total.argtypes = [_P, _P]
    L.mdgmi_stream_reset.argtypes = [_P]
    L.mdgmi_stream_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    L.mdgmi_stream_destroy.argtypes = [_P]
    L._stream_sigs = True
    return L


class Stream:
    """Streaming GMI/MI monitor over fixed-size buffers (mdgmi_stream_*)."""

    def __init__(self, fmt: Format, sigma2: float, buffer_n: int, n_lanes: int = 4, path="auto", ring: int = 1024):
        L = _stream_sigs()
        self.fmt = fmt
        h = _P()
        _check("mdgmi_stream_create", L.mdgmi_stream_create(fmt.handle, float(sigma2), int(buffer_n), int(n_lanes),
                                                            _path(path), int(ring), ctypes.byref(h)))
        self.handle = h
        self._inflight = {}
        self.path = self.info()[1]

    def push(self, y, tx_idx) -> int:
        """y [n, dim], tx [n]: torch tensors (device: read in place; CPU,
        preferably pinned: copied asynchronously) or numpy arrays (copied;
        kept alive here until the buffer has been waited for)."""
        import torch
        if isinstance(y, torch.Tensor):
            assert y.is_contiguous() and tx_idx.is_contiguous()
            _check_y(y, self.path, tx_idx)
            host = int(not y.is_cuda)
            yp, tp = _P(y.data_ptr()), _P(tx_idx.data_ptr())
            n = y.numel() // self.fmt.dim
        else:
            y = np.ascontiguousarray(y, dtype=np.float64 if self.path == MDGMI_PATH_F64 else np.float32)
            tx_idx = np.ascontiguousarray(tx_idx, dtype=np.uint32)
            host, yp, tp, n = 1, y.ctypes.data_as(_P), tx_idx.ctypes.data_as(_P), y.size // self.fmt.dim
        idx = ctypes.c_int64()
        _check("mdgmi_stream_push", _stream_sigs().mdgmi_stream_push(self.handle, yp, tp, n, host, ctypes.byref(idx)))
        self._inflight[int(idx.value)] = (y, tx_idx)
        return int(idx.value)

    def _release(self, upto=None):
        for k in [k for k in self._inflight if upto is None or k <= upto]:
            del self._inflight[k]

    def wait(self, index: int = -1) -> None:
        _check("mdgmi_stream_wait", _stream_sigs().mdgmi_stream_wait(self.handle, int(index)))
        self._release(None if index < 0 else index)

    def result(self, index: int):
        out = np.empty(MDGMI_NFIELDS)
        _check("mdgmi_stream_result", _stream_sigs().mdgmi_stream_result(self.handle, int(index),
                                                                          out.ctypes.data_as(_P)))
        self._release(index)
        return out

    def total(self):
        out = np.empty(MDGMI_NFIELDS)
        _check("mdgmi_stream_total", _stream_sigs().mdgmi_stream_total(self.handle, out.ctypes.data_as(_P)))
        self._release()
        return out

    def reset(self) -> None:
        _check("mdgmi_stream_reset", _stream_sigs().mdgmi_stream_reset(self.handle))
        self._release()

    def info(self):
        n, p = ctypes.c_int64(), ctypes.c_int32()
        _check("mdgmi_stream_info", _stream_sigs().mdgmi_stream_info(self.handle, ctypes.byref(n), ctypes.byref(p)))
        return int(n.value), int(p.value)

    def close(self):
        if getattr(self, "handle", None):
            _stream_sigs().mdgmi_stream_destroy(self.handle)
            self.handle = None
            self._inflight = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdgmi_q_factor_db(ber: float) -> float:
    """Q-factor (dB) of a bit error rate under the Gaussian-noise conversion."""
    return float(lib().mdgmi_q_factor_db(float(ber)))


# ------------------------------------------------------------------ batches
class mdgmi_instance(ctypes.Structure):
    _fields_ = [("fmt", _P), ("y", _P), ("tx_idx", _P), ("n", ctypes.c_int64), ("sigma2", ctypes.c_double)]


MDGMI_TUNE_BULK, MDGMI_TUNE_SHORT = 0, 1
MDGMI_TUNE_SHORT_SAMPLES = 1 << 18


class mdgmi_tune_entry(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("M", ctypes.c_int32), ("regime", ctypes.c_int32), ("path", ctypes.c_int32),
                ("mfma_variant", ctypes.c_int32), ("pad", ctypes.c_int32), ("samples", ctypes.c_int64),
                ("direct_rate", ctypes.c_double), ("mfma_rate", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def _batch_sigs():
    L = lib()
    if getattr(L, "_batch_sigs", False):
        return L
    IP = ctypes.POINTER(mdgmi_instance)
    L.mdgmi_gmi_batched_workspace_size.argtypes = [IP, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.mdgmi_gmi_batched.argtypes = [IP, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]
    L.mdgmi_batch_create.argtypes = [IP, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]
    L.mdgmi_batch_run.argtypes = [_P, _P, ctypes.c_int32, _P]
    L.mdgmi_batch_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.mdgmi_batch_destroy.argtypes = [_P]
    L.mdgmi_autotune.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(mdgmi_tune_entry)]
    L.mdgmi_tune_lookup.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(mdgmi_tune_entry)]
    L.mdgmi_tune_save.argtypes = [ctypes.c_char_p]
    L.mdgmi_tune_load.argtypes = [ctypes.c_char_p]
    L._batch_sigs = True
    return L


def instances(items):
    """items: sequence of (Format, y [n, dim] float32 tensor, tx [n] tensor, sigma2)."""
    arr = (mdgmi_instance * len(items))()
    for q, (f, y, tx, s2) in enumerate(items):
        assert y.is_contiguous() and tx.is_contiguous() and y.dtype == __import__("torch").float32
        n = y.numel() // f.dim
        assert tx.numel() == n
        arr[q] = mdgmi_instance(f.handle, y.data_ptr(), tx.data_ptr(), n, float(s2))
    return arr


def mdgmi_gmi_batched_workspace_size(inst, path="auto") -> int:
    L = _batch_sigs()
    b = ctypes.c_size_t()
    _check("mdgmi_gmi_batched_workspace_size",
           L.mdgmi_gmi_batched_workspace_size(inst, len(inst), _path(path), ctypes.byref(b)))
    return int(b.value)


def mdgmi_gmi_batched(inst, path="auto", out=None, ws=None, stream=None):
    """One-shot ragged batch -> out [n_inst, 6] (double, device)."""
    import torch
    L = _batch_sigs()
    if out is None:
        out = torch.empty((len(inst), MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    if ws is None:
        ws = workspace(mdgmi_gmi_batched_workspace_size(inst, path))
    _check("mdgmi_gmi_batched", L.mdgmi_gmi_batched(inst, len(inst), _path(path), _dptr(out), _dptr(ws),
                                                    ws.numel(), _stream(stream)))
    return out


class Batch:
    """mdgmi_batch plan handle (keeps the instance tensors alive)."""

    def __init__(self, items, path="auto"):
        L = _batch_sigs()
        self._keep = list(items)
        self.inst = instances(items)
        h = _P()
        _check("mdgmi_batch_create", L.mdgmi_batch_create(self.inst, len(self.inst), _path(path), ctypes.byref(h)))
        self.handle = h
        self.n_inst = len(self.inst)

    def info(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check("mdgmi_batch_info", lib().mdgmi_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return {"items": a.value, "pairs": b.value}

    def run(self, out=None, use_graph=True, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.n_inst, MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
        _check("mdgmi_batch_run", lib().mdgmi_batch_run(self.handle, _dptr(out), int(bool(use_graph)),
                                                        _stream(stream)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().mdgmi_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdgmi_autotune(dim: int, M: int, force: bool = False) -> dict:
    """Bulk-regime entry as a dict, the short-regime entry under "short"."""
    L = _batch_sigs()
    e = (mdgmi_tune_entry * 2)()
    _check("mdgmi_autotune", L.mdgmi_autotune(dim, M, int(force), e))
    d = e[0].as_dict()
    d["short"] = e[1].as_dict()
    return d


def mdgmi_tune_lookup(dim: int, M: int, regime: int = MDGMI_TUNE_BULK):
    L = _batch_sigs()
    e = mdgmi_tune_entry()
    rc = L.mdgmi_tune_lookup(dim, M, int(regime), ctypes.byref(e))
    return e.as_dict() if rc == MDGMI_OK else None


def mdgmi_tune_save(path) -> None:
    _check("mdgmi_tune_save", _batch_sigs().mdgmi_tune_save(str(path).encode()))


def mdgmi_tune_load(path) -> None:
    _check("mdgmi_tune_load", _batch_sigs().mdgmi_tune_load(str(path).encode()))


def mdgmi_tune_clear() -> None:
    lib().mdgmi_tune_clear()


def mdgmi_get_tuning() -> int:
    return int(lib().mdgmi_get_tuning())


# ------------------------------------------------------------------ learned demapper
def _mlp_sigs():
    L = lib()
    if getattr(L, "_mlp_sigs", False):
        return L
    L.mdgmi_mlp_create.argtypes = [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(_P)]
    L.mdgmi_mlp_destroy.argtypes = [_P]
    L.mdgmi_mlp_param_count.argtypes = [_P, ctypes.POINTER(ctypes.c_int64)]
    L.mdgmi_mlp_get_params.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int32]
    L.mdgmi_mlp_set_params.argtypes = [_P, _P, ctypes.c_int64]
    L.mdgmi_mlp_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    L.mdgmi_mlp_features.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _P, _P]
    L.mdgmi_mlp_forward.argtypes = [_P, _P, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P]
    L.mdgmi_mlp_loss_grad.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P]
    L.mdgmi_mlp_adam_step.argtypes = [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]
    L.mdgmi_mlp_save.argtypes = [_P, ctypes.c_char_p]
    L.mdgmi_mlp_load.argtypes = [_P, ctypes.c_char_p]
    L.mdgmi_mlp_train_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    L.mdgmi_mlp_train_step.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float, _P, _P, ctypes.c_size_t, _P]
    L.mdgmi_mlp_llr_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    L.mdgmi_mlp_llr.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P]
    L.mdgmi_learned_calibrate_workspace_size.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                                         ctypes.POINTER(ctypes.c_size_t)]
    L.mdgmi_learned_calibrate.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P, ctypes.c_int64, _P,
                                          ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]
    L._mlp_sigs = True
    return L


class MLP:
    """mdgmi_mlp handle: FP32 masters + bf16 copies on the device."""

    def __init__(self, sizes, seed: int = 0):
        L = _mlp_sigs()
        self.sizes = [int(v) for v in sizes]
        arr = (ctypes.c_int32 * len(self.sizes))(*self.sizes)
        h = _P()
        _check("mdgmi_mlp_create", L.mdgmi_mlp_create(ctypes.cast(arr, _P), len(self.sizes) - 1, int(seed),
                                                      ctypes.byref(h)))
        self.handle = h
        c = ctypes.c_int64()
        _check("mdgmi_mlp_param_count", L.mdgmi_mlp_param_count(h, ctypes.byref(c)))
        self.P = c.value
        self._ws = None

    def close(self):
        if getattr(self, "handle", None):
            lib().mdgmi_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _get(self, which):
        out = np.empty(self.P, dtype=np.float32)
        _check("mdgmi_mlp_get_params", lib().mdgmi_mlp_get_params(self.handle, out.ctypes.data_as(_P), self.P, which))
        return out

    def params(self):
        return self._get(0)

    def grad(self):
        return self._get(1)

    def moments(self):
        return self._get(2), self._get(3)

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.P
        _check("mdgmi_mlp_set_params", lib().mdgmi_mlp_set_params(self.handle, p.ctypes.data_as(_P), self.P))

    def workspace(self, n):
        b = ctypes.c_size_t()
        _check("mdgmi_mlp_workspace_size", lib().mdgmi_mlp_workspace_size(self.handle, n, ctypes.byref(b)))
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = workspace(b.value)
        return self._ws

    def forward(self, x, out=None, stream=None):
        import torch
        n = x.shape[0]
        assert x.is_contiguous() and x.dtype == torch.float32 and x.shape[1] == self.sizes[0]
        if out is None:
            out = torch.empty((n, self.sizes[-1]), dtype=torch.float32, device="cuda")
        ws = self.workspace(n)
        _check("mdgmi_mlp_forward", lib().mdgmi_mlp_forward(self.handle, _dptr(x), n, _dptr(out), _dptr(ws),
                                                            ws.numel(), _stream(stream)))
        return out

    def loss_grad(self, x, target_llr, loss=None, stream=None):
        import torch
        n = x.shape[0]
        assert x.is_contiguous() and target_llr.is_contiguous() and target_llr.shape == (n, self.sizes[-1])
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device="cuda")
        ws = self.workspace(n)
        _check("mdgmi_mlp_loss_grad", lib().mdgmi_mlp_loss_grad(self.handle, _dptr(x), _dptr(target_llr), n,
                                                                _dptr(loss), _dptr(ws), ws.numel(), _stream(stream)))
        return loss

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check("mdgmi_mlp_adam_step", lib().mdgmi_mlp_adam_step(self.handle, lr, beta1, beta2, eps, _stream(stream)))

    def train_workspace_size(self, n):
        b = ctypes.c_size_t()
        _check("mdgmi_mlp_train_workspace_size",
               _mlp_sigs().mdgmi_mlp_train_workspace_size(self.handle, n, ctypes.byref(b)))
        return b.value

    def train_step(self, y, snr_db, target_llr, lr, loss=None, ws=None, stream=None):
        """mdgmi_mlp_train_step: features from y [n, dim] and per-sample SNRs
        snr_db [n] (dB), BCE forward/backward and one Adam step."""
        import torch
        L = _mlp_sigs()
        n = y.shape[0]
        assert y.is_contiguous() and snr_db.is_contiguous() and target_llr.is_contiguous()
        assert y.dtype == snr_db.dtype == target_llr.dtype == torch.float32 and snr_db.numel() == n
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device="cuda")
        if ws is None:
            b = ctypes.c_size_t()
            _check("mdgmi_mlp_train_workspace_size", L.mdgmi_mlp_train_workspace_size(self.handle, n, ctypes.byref(b)))
            ws = workspace(b.value)
        _check("mdgmi_mlp_train_step", L.mdgmi_mlp_train_step(self.handle, _dptr(y), _dptr(snr_db), _dptr(target_llr),
                                                              n, float(lr), _dptr(loss), _dptr(ws), ws.numel(),
                                                              _stream(stream)))
        return loss

    def llr(self, y, snr_db, out=None, stream=None):
        """mdgmi_mlp_llr: logits [n, out] of y [n, dim] at per-sample SNRs snr_db [n] (dB)."""
        import torch
        L = _mlp_sigs()
        n = y.shape[0]
        assert y.is_contiguous() and snr_db.is_contiguous() and snr_db.numel() == n
        if out is None:
            out = torch.empty((n, self.sizes[-1]), dtype=torch.float32, device="cuda")
        b = ctypes.c_size_t()
        _check("mdgmi_mlp_llr_workspace_size", L.mdgmi_mlp_llr_workspace_size(self.handle, n, ctypes.byref(b)))
        ws = workspace(b.value) if b.value else None
        _check("mdgmi_mlp_llr", L.mdgmi_mlp_llr(self.handle, _dptr(y), _dptr(snr_db), n, _dptr(out),
                                                _dptr(ws) if ws is not None else None, b.value, _stream(stream)))
        return out

    def save(self, path):
        _check("mdgmi_mlp_save", lib().mdgmi_mlp_save(self.handle, str(path).encode()))

    def load(self, path):
        _check("mdgmi_mlp_load", lib().mdgmi_mlp_load(self.handle, str(path).encode()))


def mdgmi_mlp_features(y, snr_db: float, x=None, stream=None):
    """x [n, dim + 1] = [y, (snr_db - 9.5) / 4.5] on the device."""
    import torch
    n, dim = y.shape
    if x is None:
        x = torch.empty((n, dim + 1), dtype=torch.float32, device="cuda")
    _check("mdgmi_mlp_features", _mlp_sigs().mdgmi_mlp_features(_dptr(y), n, dim, float(snr_db), _dptr(x),
                                                                 _stream(stream)))
    return x


def _mlp_gmi_sigs():
    L = _mlp_sigs()
    if not getattr(L, "_mlp_gmi_sigs", False):
        L.mdgmi_mlp_gmi_workspace_size.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.mdgmi_mlp_gmi.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int64, _P, _P,
                                    ctypes.c_size_t, _P]
        L._mlp_gmi_sigs = True
    return L


def mdgmi_mlp_gmi_workspace_size(net: "MLP", chunk: int) -> int:
    b = ctypes.c_size_t()
    _check("mdgmi_mlp_gmi_workspace_size",
           _mlp_gmi_sigs().mdgmi_mlp_gmi_workspace_size(net.handle, int(chunk), ctypes.byref(b)))
    return b.value


def mdgmi_mlp_gmi(net: "MLP", fmt: Format, y, tx_idx, snr_db, chunk: int = 1 << 20, out=None, ws=None, stream=None):
    """Learned GMI per SNR point: y [n_snr, n, dim], tx [n_snr, n] -> out [n_snr, 6] (MI fields NaN)."""
    import torch
    L = _mlp_gmi_sigs()
    snr = np.ascontiguousarray(np.atleast_1d(snr_db), dtype=np.float64)
    n_snr = snr.size
    n = y.numel() // (fmt.dim * n_snr)
    chunk = int(min(chunk, n))
    if out is None:
        out = torch.empty((n_snr, MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    if ws is None:
        ws = workspace(mdgmi_mlp_gmi_workspace_size(net, chunk))
    _check("mdgmi_mlp_gmi", L.mdgmi_mlp_gmi(net.handle, fmt.handle, _dptr(y), _dptr(tx_idx), n, snr.ctypes.data_as(_P),
                                            n_snr, chunk, _dptr(out), _dptr(ws), ws.numel(), _stream(stream)))
    return out


def mdgmi_learned_calibrate(fmt: Format, net: "MLP", y, tx_idx, sigma2, exact_path="auto", max_loss=0.01,
                            stream=None):
    """Attach net to fmt and route each sigma2 (paired GMI loss on these
    held-out samples <= max_loss -> the network). Returns [n_snr, 4]:
    GMI_exact, GMI_learned, loss, route (1 learned)."""
    L = _mlp_sigs()
    s2 = np.ascontiguousarray(np.atleast_1d(sigma2), dtype=np.float64)
    n_snr = s2.size
    n = y.numel() // (fmt.dim * n_snr)
    p = _path(exact_path)
    b = ctypes.c_size_t()
    _check("mdgmi_learned_calibrate_workspace_size",
           L.mdgmi_learned_calibrate_workspace_size(fmt.handle, net.handle, p, n, n_snr, ctypes.byref(b)))
    ws = workspace(b.value)
    res = np.empty((n_snr, 4), dtype=np.float64)
    _check("mdgmi_learned_calibrate", L.mdgmi_learned_calibrate(fmt.handle, net.handle, p, float(max_loss), _dptr(y),
                                                                _dptr(tx_idx), n, s2.ctypes.data_as(_P), n_snr,
                                                                res.ctypes.data_as(_P), _dptr(ws), ws.numel(),
                                                                _stream(stream)))
    fmt._learned_net = net   # keep the network alive while the format uses it
    return res


def mdgmi_mlp_set_fused(waves: int) -> None:
    """Inference kernel of mdgmi_mlp_gmi: 8 (default) or 4 waves fused, 0 layer by layer."""
    _check("mdgmi_mlp_set_fused", lib().mdgmi_mlp_set_fused(int(waves)))


def mdgmi_probe_rates() -> dict:
    """Measured peaks of the current device (mdgmi_probe_rates)."""
    out = np.zeros(9, dtype=np.float64)
    _check("mdgmi_probe_rates", lib().mdgmi_probe_rates(out.ctypes.data_as(_P)))
    return {"exp_per_s": float(out[0]), "clock_hz_exp": float(out[1]), "fma_lane_ops_per_s": float(out[2]),
            "clock_hz_fma": float(out[3]), "mfma_bf16_flops_per_s": float(out[4]),
            "mfma_2waves_flops_per_s": float(out[5]), "mfma_with_4_fma_flops_per_s": float(out[6]),
            "mfma_with_8_fma_flops_per_s": float(out[7]), "split_waves_iters_per_s": float(out[8])}
