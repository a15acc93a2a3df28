"""FP64 CPU oracle (plain C, see oracle.c) and its ctypes loader.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py. The product path (the HIP library and its
binding) never imports, links or calls anything here.

Definitions followed (standard BICM/BMD information theory; the paper names
GMI, MI and LLR only in its glossary): see the header of oracle.c.
"""
from __future__ import annotations

import ctypes
import math
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
        L.oracle_hd.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, P]
        L.oracle_llr_maxlog.argtypes = [P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, P]
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


def hd(y, tx_idx, X, labels, sigma2):
    """Hard decisions: (BER of the bitwise MAP decisions, SER of the
    nearest-point decisions, n, non-finite count)."""
    X = _c(X, np.float64)
    M, dim = X.shape
    y = _c(np.reshape(y, (-1, dim)), np.float64)
    tx = _c(tx_idx, np.uint32)
    lab = _c(labels, np.uint32)
    out = np.empty(4)
    rc = lib().oracle_hd(_ptr(y), _ptr(tx), y.shape[0], dim, _ptr(X), _ptr(lab), M, float(sigma2), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_hd failed ({rc})")
    return out


# ---------------------------------------------------------------- MLP demapper
def _mlp_sigs():
    L = lib()
    if getattr(L, "_mlp_sigs", False):
        return L
    P = ctypes.c_void_p
    L.oracle_gelu.restype = ctypes.c_double
    L.oracle_gelu.argtypes = [ctypes.c_double]
    L.oracle_mlp_param_count.restype = ctypes.c_int64
    L.oracle_mlp_param_count.argtypes = [P, ctypes.c_int]
    L.oracle_mlp_forward.argtypes = [P, P, ctypes.c_int, P, ctypes.c_int64, P]
    L.oracle_mlp_loss_grad.restype = ctypes.c_double
    L.oracle_mlp_loss_grad.argtypes = [P, P, ctypes.c_int, P, P, ctypes.c_int64, P]
    L.oracle_adam.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double]
    L.oracle_gmi_cost_from_llr.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P]
    L._mlp_sigs = True
    return L


def gelu(x: float) -> float:
    return float(_mlp_sigs().oracle_gelu(float(x)))


def mlp_param_count(sizes) -> int:
    s = _c(sizes, np.int32)
    return int(_mlp_sigs().oracle_mlp_param_count(_ptr(s), len(sizes) - 1))


def mlp_forward(params, sizes, x):
    """Logits [n, sizes[-1]] (nats) of inputs x [n, sizes[0]]."""
    s = _c(sizes, np.int32)
    p = _c(params, np.float64)
    assert p.size == mlp_param_count(sizes)
    x = _c(np.reshape(x, (-1, sizes[0])), np.float64)
    out = np.empty((x.shape[0], sizes[-1]))
    rc = _mlp_sigs().oracle_mlp_forward(_ptr(p), _ptr(s), len(sizes) - 1, _ptr(x), x.shape[0], _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle_mlp_forward failed")
    return out


def mlp_loss_grad(params, sizes, x, target):
    """(mean BCE-with-logits loss in nats summed over outputs, gradient [P])."""
    s = _c(sizes, np.int32)
    p = _c(params, np.float64)
    x = _c(np.reshape(x, (-1, sizes[0])), np.float64)
    t = _c(np.reshape(target, (-1, sizes[-1])), np.float64)
    g = np.empty_like(p)
    loss = _mlp_sigs().oracle_mlp_loss_grad(_ptr(p), _ptr(s), len(sizes) - 1, _ptr(x), _ptr(t), x.shape[0], _ptr(g))
    return float(loss), g


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays (step number t >= 1)."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _mlp_sigs().oracle_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.size, int(t), float(lr), float(b1),
                            float(b2), float(eps))


def gmi_cost_from_llr(llr, sent_label):
    """Per-sample GMI cost (bits) of arbitrary LLRs [n, m] for the sent labels."""
    llr = _c(llr, np.float64)
    lab = _c(sent_label, np.uint32)
    out = np.empty(llr.shape[0])
    _mlp_sigs().oracle_gmi_cost_from_llr(_ptr(llr), _ptr(lab), llr.shape[0], llr.shape[1], _ptr(out))
    return out


# ------------------------------------------------- max-log LLRs, GMI(s), s-opt
def llr_maxlog(y, X, labels, sigma2):
    """Max-log LLRs in nats, shape (n, m): per bit, the squared distance to
    the nearest point labelled 0 minus that to the nearest point labelled 1,
    over 2 sigma2."""
    X = _c(X, np.float64)
    M, dim = X.shape
    m = int(M).bit_length() - 1
    y = _c(np.reshape(y, (-1, dim)), np.float64)
    lab = _c(labels, np.uint32)
    out = np.empty((y.shape[0], m), dtype=np.float64)
    rc = lib().oracle_llr_maxlog(_ptr(y), y.shape[0], dim, _ptr(X), _ptr(lab), M, float(sigma2), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_llr_maxlog failed ({rc})")
    return out


def gmi_s(llr, sent_label, s):
    """(GMI(s), its standard error) in bits of a bit-metric decoder that uses
    the given LLRs scaled by s >= 0:
        GMI(s) = m - mean_i sum_k log2(1 + exp(-s (2 b_k(i) - 1) lambda_k(i))).
    s = 1 is the GMI of the LLRs as they are; for the exact LLRs of the
    channel it is also the maximum over s."""
    llr = _c(llr, np.float64)
    n, m = llr.shape
    c = gmi_cost_from_llr(float(s) * llr, sent_label)
    se = float(np.std(c, ddof=1) / np.sqrt(n)) if n > 1 else 0.0
    return float(m - np.mean(c)), se


GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0


def gmi_sopt(llr, sent_label, iters=120):
    """(s*, GMI(s*), SE at s*): the s-optimised GMI, max over s >= 0 of
    gmi_s. Every cost term log(1 + e^{-s v}) is convex in s, so GMI(s) is
    concave and a golden-section search finds the maximum: first an upper
    end s_hi, doubled from 1 until GMI(s_hi) no longer exceeds GMI(s_hi / 2),
    then the search on [0, s_hi]."""
    f = lambda s: gmi_s(llr, sent_label, s)[0]   # noqa: E731
    hi = 1.0
    while f(2.0 * hi) > f(hi) and hi < 2.0 ** 40:
        hi *= 2.0
    hi *= 2.0
    lo = 0.0
    a = hi - GOLDEN * (hi - lo)
    b = lo + GOLDEN * (hi - lo)
    fa, fb = f(a), f(b)
    for _ in range(iters):
        if fa < fb:
            lo, a, fa = a, b, fb
            b = lo + GOLDEN * (hi - lo)
            fb = f(b)
        else:
            hi, b, fb = b, a, fa
            a = hi - GOLDEN * (hi - lo)
            fa = f(a)
    s = 0.5 * (lo + hi)
    g, se = gmi_s(llr, sent_label, s)
    if f(0.0) >= g:       # non-informative LLRs: the maximum is at s = 0
        s = 0.0
        g, se = gmi_s(llr, sent_label, 0.0)
    return s, g, se


def gmi_bits(llr, sent_label):
    """Per-bit GMI of given LLRs: for each label bit k,
        GMI_k = 1 - mean_i log2(1 + exp(-(2 b_k(i) - 1) lambda_ik))
    and its standard error; sum_k GMI_k is the GMI at s = 1. Returns
    (gmi [m], se [m]) in bits."""
    llr = _c(llr, np.float64)
    n, m = llr.shape
    lab = _c(sent_label, np.uint32)
    gmi = np.empty(m)
    se = np.empty(m)
    for k in range(m):
        col = np.ascontiguousarray(llr[:, k:k + 1])
        bit = ((lab >> k) & 1).astype(np.uint32)        # the cost of one bit as a one-bit label
        c = gmi_cost_from_llr(col, bit)
        gmi[k] = 1.0 - float(np.mean(c))
        se[k] = float(np.std(c, ddof=1) / np.sqrt(n)) if n > 1 else 0.0
    return gmi, se
