"""FP64 CPU oracle (plain C, see oracle.c) and its ctypes loader.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py. The product path (the HIP library and its
binding) never imports, links or calls anything here.

Definitions followed (standard BICM/BMD information theory; the paper names
GMI, MI and LLR only in its glossary): see the header of oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "oracle.c"
LIB = HERE / "liboracle.so"

_lib = None


def build(force: bool = True) -> Path:
    """Compile oracle.c with gcc (IEEE semantics: no fast-math)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               str(SRC), "-o", str(tmp), "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
            build(force=True)
        L = ctypes.CDLL(str(LIB))
        P = ctypes.c_void_p
        L.oracle_llr.argtypes = [P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, P]
        L.oracle_costs.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int,
                                   ctypes.c_double, P, P]
        L.oracle_gmi.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int,
                                 ctypes.c_double, P]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def llr(y, X, labels, sigma2):
    """Per-bit LLRs in nats, shape (n, m); column k is label bit k (LSB first),
    positive values favour bit 1."""
    X = _c(X, np.float64)
    M, dim = X.shape
    m = int(M).bit_length() - 1
    y = _c(np.reshape(y, (-1, dim)), np.float64)
    lab = _c(labels, np.uint32)
    out = np.empty((y.shape[0], m), dtype=np.float64)
    rc = lib().oracle_llr(_ptr(y), y.shape[0], dim, _ptr(X), _ptr(lab), M, float(sigma2), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_llr failed ({rc})")
    return out


def costs(y, tx_idx, X, labels, sigma2):
    """Per-sample (GMI cost, MI cost) in bits."""
    X = _c(X, np.float64)
    M, dim = X.shape
    y = _c(np.reshape(y, (-1, dim)), np.float64)
    tx = _c(tx_idx, np.uint32)
    lab = _c(labels, np.uint32)
    n = y.shape[0]
    cg = np.empty(n)
    cm = np.empty(n)
    rc = lib().oracle_costs(_ptr(y), _ptr(tx), n, dim, _ptr(X), _ptr(lab), M, float(sigma2),
                            _ptr(cg), _ptr(cm))
    if rc != 0:
        raise RuntimeError(f"oracle_costs failed ({rc})")
    return cg, cm


FIELDS = ("gmi", "mi", "se_gmi", "se_mi", "n", "n_nonfinite")


def gmi(y, tx_idx, X, labels, sigma2):
    """{GMI, MI, SE_GMI, SE_MI, N, n_nonfinite} for one SNR point (bits/symbol)."""
    X = _c(X, np.float64)
    M, dim = X.shape
    y = _c(np.reshape(y, (-1, dim)), np.float64)
    tx = _c(tx_idx, np.uint32)
    lab = _c(labels, np.uint32)
    out = np.empty(6)
    rc = lib().oracle_gmi(_ptr(y), _ptr(tx), y.shape[0], dim, _ptr(X), _ptr(lab), M, float(sigma2),
                          _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_gmi failed ({rc})")
    return out


def gmi_per_snr(y, tx_idx, X, labels, sigma2s):
    """Rows of gmi() for y (n_snr, n, N), tx (n_snr, n) and one sigma2 per SNR."""
    return np.stack([gmi(y[s], tx_idx[s], X, labels, s2) for s, s2 in enumerate(sigma2s)])
