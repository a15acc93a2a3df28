"""Pins of the oracle's max-log LLRs, GMI(s) and s-optimised GMI.

Max-log LLRs replace each class log-sum-exp by its largest term:
lambda_k = (min over class 0 of ||y - x||^2 - min over class 1) / (2 sigma2).
* two-point formats: each class has one point, so max-log equals the exact LLR;
* Gray QPSK: each bit's classes differ in one coordinate only and the other
  coordinate contributes the same factor to both class sums, so max-log
  again equals the exact LLR;
* Gray 4-PAM at hand-computed points;
* 0 <= ln sum_C e^{-t} + min_C t <= ln |C| for each class, hence
  |lambda_exact - lambda_maxlog| <= ln(M / 2); and the relative gap
  vanishes at high SNR.
GMI(s) = m - mean sum_k log2(1 + exp(-s (2 b_k - 1) lambda_k)):
* GMI(0) = 0 for any LLRs; GMI(1) of the exact LLRs is the exact GMI;
* binary symmetric LLRs (+-L, a fraction p of them on the sent bit's side):
  GMI(s) is maximal at s* = ln(p / (1 - p)) / L with GMI(s*) = 1 - h2(p);
* scaling the LLRs by c divides s* by c and leaves the maximum unchanged;
* exact LLRs: s* close to 1; max-log LLRs: s-optimisation gains, and stays
  below the exact GMI.
"""
import math

import numpy as np
import pytest

import workloads as w


def h2(p):
    return -p * math.log2(p) - (1 - p) * math.log2(1 - p)


@pytest.mark.parametrize("dim", [1, 2, 4, 8])
def test_two_point_formats_equal_exact(orc, dim):
    rng = np.random.default_rng(dim)
    X = rng.standard_normal((2, dim))
    lab = np.array([1, 0], np.uint32)
    y = rng.standard_normal((500, dim)) * 1.5
    np.testing.assert_allclose(orc.llr_maxlog(y, X, lab, 0.3), orc.llr(y, X, lab, 0.3), rtol=1e-12, atol=1e-12)


def test_gray_qpsk_equals_exact(orc):
    f = w.square_qam(2)
    y, _ = w.channel_samples(f, 0.2, seed=3, snr_slot=0, n=2000)
    np.testing.assert_allclose(orc.llr_maxlog(y, f.X, f.labels, 0.2), orc.llr(y, f.X, f.labels, 0.2),
                               rtol=1e-10, atol=1e-10)


def test_4pam_hand_values(orc):
    # levels -3, -1, 1, 3 with Gray labels 0, 1, 3, 2: bit 1 is 1 on {1, 3},
    # bit 0 is 1 on {-1, 1}; sigma2 = 0.5 so lambda = difference of d^2.
    X = np.array([[-3.0], [-1.0], [1.0], [3.0]])
    lab = np.array([0, 1, 3, 2], np.uint32)
    y = np.array([[0.5], [-2.5], [2.0]])
    # y = 0.5:  d^2 = 12.25, 2.25, 0.25, 6.25 -> bit0: 6.25 - 0.25 = 6, bit1: 2.25 - 0.25 = 2
    # y = -2.5: d^2 = 0.25, 2.25, 12.25, 30.25 -> bit0: 0.25 - 2.25 = -2, bit1: 0.25 - 12.25 = -12
    # y = 2:    d^2 = 25, 9, 1, 1 -> bit0: 1 - 1 = 0, bit1: 9 - 1 = 8
    want = np.array([[6.0, 2.0], [-2.0, -12.0], [0.0, 8.0]])
    np.testing.assert_array_equal(orc.llr_maxlog(y, X, lab, 0.5), want)


@pytest.mark.parametrize("dim,M", [(2, 16), (4, 64), (8, 256)])
def test_within_log_class_size_of_exact(orc, dim, M):
    f = w.random_shells(dim, M, 5 + M)
    for snr in (0.0, 10.0):
        s2 = float(w.sigma2_from_snr_db(snr, dim))
        y, _ = w.channel_samples(f, s2, seed=1, snr_slot=0, n=1500)
        gap = orc.llr(y, f.X, f.labels, s2) - orc.llr_maxlog(y, f.X, f.labels, s2)
        assert np.max(np.abs(gap)) <= math.log(M / 2) + 1e-9
        assert np.max(np.abs(gap)) > 1e-3       # and not identical for these formats


def test_high_snr_limit(orc):
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(40.0, 2))
    y, _ = w.channel_samples(f, s2, seed=2, snr_slot=0, n=2000)
    ex = orc.llr(y, f.X, f.labels, s2)
    ml = orc.llr_maxlog(y, f.X, f.labels, s2)
    assert np.max(np.abs(ex - ml) / np.abs(ex)) < 1e-3


def test_gmi_s_zero_and_one(orc):
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(9.0, 2))
    y, tx = w.channel_samples(f, s2, seed=4, snr_slot=0, n=5000)
    lam = orc.llr(y, f.X, f.labels, s2)
    sent = f.labels[tx]
    assert orc.gmi_s(lam, sent, 0.0)[0] == 0.0
    g1, se1 = orc.gmi_s(lam, sent, 1.0)
    ref = orc.gmi(y, tx, f.X, f.labels, s2)
    assert g1 == pytest.approx(ref[0], abs=1e-12) and se1 == pytest.approx(ref[2], rel=1e-9)


@pytest.mark.parametrize("p,L,m", [(0.9, 3.7, 1), (0.75, 0.4, 1), (0.97, 12.0, 3)])
def test_binary_symmetric_closed_form(orc, p, L, m):
    n = 4000
    k = int(round(p * n))
    rng = np.random.default_rng(7)
    sent = rng.integers(0, 1 << m, n).astype(np.uint32)
    bits = ((sent[:, None] >> np.arange(m)) & 1).astype(np.float64)
    right = np.zeros((n, m), bool)
    for j in range(m):
        right[rng.permutation(n)[:k], j] = True
    lam = np.where(right, 1.0, -1.0) * (2.0 * bits - 1.0) * L
    pe = k / n
    s, g, _ = orc.gmi_sopt(lam, sent)
    assert s == pytest.approx(math.log(pe / (1 - pe)) / L, rel=1e-7)
    assert g == pytest.approx(m * (1 - h2(pe)), abs=1e-12)


def test_scaling_invariance(orc):
    f = w.format_4d64()
    s2 = float(w.sigma2_from_snr_db(8.0, 4))
    y, tx = w.channel_samples(f, s2, seed=9, snr_slot=0, n=3000)
    lam = orc.llr_maxlog(y, f.X, f.labels, s2)
    sent = f.labels[tx]
    s0, g0, _ = orc.gmi_sopt(lam, sent)
    for c in (0.25, 3.0):
        s, g, _ = orc.gmi_sopt(c * lam, sent)
        assert s == pytest.approx(s0 / c, rel=1e-6)
        assert g == pytest.approx(g0, abs=1e-12)


def test_exact_llrs_optimum_near_one_and_maxlog_gains(orc):
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(6.0, 2))
    y, tx = w.channel_samples(f, s2, seed=11, snr_slot=0, n=100_000)
    sent = f.labels[tx]
    ex = orc.llr(y, f.X, f.labels, s2)
    s, g, se = orc.gmi_sopt(ex, sent)
    g1 = orc.gmi_s(ex, sent, 1.0)[0]
    assert abs(s - 1.0) < 0.03 and 0.0 <= g - g1 < 2e-4
    ml = orc.llr_maxlog(y, f.X, f.labels, s2)
    sm, gm, _ = orc.gmi_sopt(ml, sent)
    gm1 = orc.gmi_s(ml, sent, 1.0)[0]
    assert gm > gm1 and abs(sm - 1.0) > 0.02
    assert gm <= g + 3 * se


def test_uninformative_llrs_give_zero(orc):
    rng = np.random.default_rng(12)
    sent = rng.integers(0, 4, 1000).astype(np.uint32)
    bits = ((sent[:, None] >> np.arange(2)) & 1).astype(np.float64)
    lam = -(2.0 * bits - 1.0) * 2.0          # every LLR points at the wrong bit
    s, g, _ = orc.gmi_sopt(lam, sent)
    assert s == 0.0 and g == 0.0
