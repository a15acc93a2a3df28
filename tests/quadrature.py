"""Reference values that do not come from the oracle, used to pin it.

* Gauss-Hermite closed forms for Gray BPSK / QPSK: the BPSK LLR is 2y/sigma^2
  (derived by hand), so E[log2(1 + exp(-lambda))] is a one-dimensional
  Gaussian integral.
* Density-based integration on a grid: MI = E[log2 p(y|x)/p(y)] and the BICM
  GMI (s = 1) as the sum of the bit-wise mutual informations
  sum_k I(B_k; Y) = sum_k E[log2 p(y|b_k)/p(y)]. This route never forms an LLR
  or a softplus, so it checks the estimator's formula rather than retyping it.
* oracle_expectation(): the expectation of the oracle's own per-sample costs
  under a tensor Gauss-Hermite rule, i.e. the noise-free version of the
  Monte-Carlo average, for comparison with the references above.
"""
from __future__ import annotations

import math

import numpy as np

LOG2E = 1.0 / math.log(2.0)


def gh(n: int):
    """Gauss-Hermite nodes/weights for E[f(Z)], Z ~ N(0,1): f(sqrt(2) t) w / sqrt(pi)."""
    t, w = np.polynomial.hermite.hermgauss(n)
    return math.sqrt(2.0) * t, w / math.sqrt(math.pi)


def bpsk_mi(gamma: float, n: int = 150) -> float:
    """Gray BPSK, x = +-1, real noise variance 1/gamma: the LLR is 2 y gamma,
    so MI = GMI = 1 - E_z[log2(1 + exp(-2 gamma - 2 sqrt(gamma) z))]."""
    z, w = gh(n)
    u = -2.0 * gamma - 2.0 * math.sqrt(gamma) * z
    sp = np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))
    return 1.0 - float(np.sum(w * sp)) * LOG2E


def qpsk_mi(snr_lin: float, n: int = 150) -> float:
    """Gray QPSK with E_s = 1 over complex AWGN, SNR = E_s/N0: two independent
    BPSK channels of SNR gamma = SNR each."""
    return 2.0 * bpsk_mi(snr_lin, n)


def _logsumexp(a, axis):
    mx = np.max(a, axis=axis, keepdims=True)
    return np.squeeze(mx, axis=axis) + np.log(np.sum(np.exp(a - mx), axis=axis))


def density_gmi_mi_1d(X, labels, sigma2, n_grid: int = 20001, span: float = 9.0):
    """Bit-wise MI sum and MI of a 1-D constellation by grid integration of
    the channel densities (trapezoid-like Riemann sum on a fine uniform grid)."""
    x = np.asarray(X, dtype=np.float64).reshape(-1)
    M = x.size
    m = int(M).bit_length() - 1
    s = math.sqrt(sigma2)
    y = np.linspace(x.min() - span * s, x.max() + span * s, n_grid)
    dy = y[1] - y[0]
    # log p(y | x_j) up to the common normalisation
    lp = -((y[:, None] - x[None, :]) ** 2) / (2 * sigma2) - 0.5 * math.log(2 * math.pi * sigma2)
    return _density_terms(lp, labels, M, m, dy)


def density_gmi_mi_2d(X, labels, sigma2, n_grid: int = 801, span: float = 9.0):
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    m = int(M).bit_length() - 1
    s = math.sqrt(sigma2)
    g0 = np.linspace(X[:, 0].min() - span * s, X[:, 0].max() + span * s, n_grid)
    g1 = np.linspace(X[:, 1].min() - span * s, X[:, 1].max() + span * s, n_grid)
    Y0, Y1 = np.meshgrid(g0, g1, indexing="ij")
    Y = np.stack([Y0.ravel(), Y1.ravel()], axis=1)
    dA = (g0[1] - g0[0]) * (g1[1] - g1[0])
    d2 = ((Y[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    lp = -d2 / (2 * sigma2) - math.log(2 * math.pi * sigma2)
    return _density_terms(lp, labels, M, m, dA)


def _density_terms(lp, labels, M, m, dvol, per_bit=False):
    """lp[g, j] = log p(y_g | x_j). Returns (sum_k I(B_k;Y), I(X;Y)) in bits,
    or with per_bit the list of I(B_k;Y) instead of their sum."""
    labels = np.asarray(labels, dtype=np.int64)
    lpy = _logsumexp(lp, 1) - math.log(M)                    # log p(y)
    py_j = np.exp(lp)                                        # p(y | x_j)
    # I(X;Y) = (1/M) sum_j int p(y|x_j) log2(p(y|x_j)/p(y)) dy
    mi = float(np.sum(py_j * (lp - lpy[:, None])) * dvol / M) * LOG2E
    bits = []
    for k in range(m):
        ik = 0.0
        for b in (0, 1):
            sel = ((labels >> k) & 1) == b
            lpb = _logsumexp(lp[:, sel], 1) - math.log(sel.sum())   # log p(y | b_k = b)
            pb = np.exp(lpb)
            ik += 0.5 * float(np.sum(pb * (lpb - lpy)) * dvol) * LOG2E
        bits.append(ik)
    return (bits if per_bit else sum(bits)), mi


def density_bitwise_1d(X, labels, sigma2, n_grid: int = 20001, span: float = 9.0):
    """[I(B_k; Y) for each label bit k] of a 1-D constellation (bits)."""
    x = np.asarray(X, dtype=np.float64).reshape(-1)
    M = x.size
    m = int(M).bit_length() - 1
    s = math.sqrt(sigma2)
    y = np.linspace(x.min() - span * s, x.max() + span * s, n_grid)
    lp = -((y[:, None] - x[None, :]) ** 2) / (2 * sigma2) - 0.5 * math.log(2 * math.pi * sigma2)
    return _density_terms(lp, labels, M, m, y[1] - y[0], per_bit=True)[0]


def oracle_expectation(oracle_costs, X, labels, sigma2, n: int = 40):
    """E[c_G], E[c_M] of the oracle's per-sample costs by tensor Gauss-Hermite
    over the noise for every transmitted point, returned as (GMI, MI)."""
    X = np.asarray(X, dtype=np.float64)
    M, dim = X.shape
    m = int(M).bit_length() - 1
    z, w = gh(n)
    grids = np.meshgrid(*([z] * dim), indexing="ij")
    Z = np.stack([g.ravel() for g in grids], axis=1)
    W = np.ones(Z.shape[0])
    for wg in np.meshgrid(*([w] * dim), indexing="ij"):
        W = W * wg.ravel()
    s = math.sqrt(sigma2)
    eg = em = 0.0
    for i in range(M):
        y = X[i][None, :] + s * Z
        cg, cm = oracle_costs(y, np.full(Z.shape[0], i, dtype=np.uint32), X, labels, sigma2)
        eg += float(np.sum(W * cg))
        em += float(np.sum(W * cm))
    return m - eg / M, m - em / M
