"""Pins of the oracle's hard decisions (bitwise MAP from the LLR signs and
nearest-point symbol decisions) against textbook error probabilities of
Gray-labelled formats over AWGN, their limits and hand-built samples.

Closed forms (Es/N0 = SNR for unit-energy 2-D formats, noise variance
1/(2 SNR) per real dimension, Q(x) = erfc(x / sqrt 2) / 2):
* BPSK on one axis: BER = SER = Q(sqrt(2 SNR));
* Gray QPSK: BER = Q(sqrt(SNR)), SER = 1 - (1 - BER)^2;
* square 16-QAM, nearest point: P = 1.5 Q(sqrt(SNR / 5)) per axis,
  SER = 1 - (1 - P)^2.
Monte-Carlo estimates are compared within 4 standard errors."""
import math

import numpy as np
import pytest

import workloads as w


def Q(x):
    return 0.5 * math.erfc(x / math.sqrt(2.0))


def mc(orc, f, snr_db, n, seed=21):
    s2 = float(w.sigma2_from_snr_db(snr_db, f.dim))
    y, tx = w.channel_samples(f, s2, seed=seed, snr_slot=int(snr_db * 10) & 0xFFFF, n=n)
    return orc.hd(y, tx, f.X, f.labels, s2)


def within(est, p, n, k=4.0):
    se = math.sqrt(max(p * (1 - p), 1e-12) / n)
    return abs(est - p) <= k * se


@pytest.mark.parametrize("snr_db", [0.0, 4.0, 8.0])
def test_bpsk(orc, snr_db):
    f = w.Format("bpsk2d", np.array([[-1.0, 0.0], [1.0, 0.0]]), np.array([0, 1], np.uint32))
    r = mc(orc, f, snr_db, 200_000)
    p = Q(math.sqrt(2 * 10 ** (snr_db / 10)))
    assert within(r[0], p, 200_000) and within(r[1], p, 200_000)


@pytest.mark.parametrize("snr_db", [2.0, 6.0, 10.0])
def test_gray_qpsk(orc, snr_db):
    f = w.square_qam(2)
    n = 200_000
    r = mc(orc, f, snr_db, n)
    ber = Q(math.sqrt(10 ** (snr_db / 10)))
    assert within(r[0], ber, 2 * n)
    assert within(r[1], 1 - (1 - ber) ** 2, n)


@pytest.mark.parametrize("snr_db", [8.0, 12.0, 16.0])
def test_16qam_nearest_point_ser(orc, snr_db):
    f = w.format_16qam()
    n = 100_000
    r = mc(orc, f, snr_db, n)
    p = 1.5 * Q(math.sqrt(10 ** (snr_db / 10) / 5))
    assert within(r[1], 1 - (1 - p) ** 2, n)


def test_limits(orc):
    f = w.format_16qam()
    lo = mc(orc, f, -40.0, 40_000)
    assert within(lo[0], 0.5, 4 * 40_000) and within(lo[1], 1 - 1 / 16, 40_000)
    hi = mc(orc, f, 40.0, 20_000)
    assert hi[0] == 0.0 and hi[1] == 0.0


def test_hand_built_samples(orc):
    f = w.square_qam(2)                       # Gray QPSK
    i = 1
    x = f.X[i]
    far = -3.0 * x                            # mirrored through the origin: both bits wrong
    side = np.array([-x[0], x[1]]) * 2.0      # mirrored on one axis: one bit wrong
    y = np.stack([x, far, side])
    tx = np.array([i, i, i], np.uint32)
    r = orc.hd(y, tx, f.X, f.labels, 0.1)
    assert r[0] == pytest.approx(3 / 6) and r[1] == pytest.approx(2 / 3)


def test_nonfinite_samples_are_errors(orc):
    f = w.square_qam(2)
    y = np.array([[np.nan, 0.0], [0.5, 0.5]])
    tx = np.array([0, 0], np.uint32)
    r = orc.hd(y, tx, f.X, f.labels, 0.1)
    assert r[3] == 1 and r[1] >= 0.5 and r[0] >= 0.5


def test_exact_ties_go_to_the_lowest_label(orc):
    """A sample exactly half-way between two points is decided for the one
    with the lower label: a symbol error only when the other was sent; moved
    off the bisector, the nearer point wins whatever its label. Where two
    labels share one point, the lower label is always decided, so sending
    the higher one is always a symbol error (its bit decisions are unaffected:
    they come from the LLR signs)."""
    f = w.square_qam(2)
    a, b = 0, 1
    if np.count_nonzero(f.X[a] != f.X[b]) != 1:   # want neighbours on one axis
        b = 2
    mid = 0.5 * (f.X[a] + f.X[b])
    d = ((mid[None] - f.X[[a, b]]) ** 2).sum(1)
    assert d[0] == d[1]                           # an exact tie in FP64
    lo, hi = (a, b) if f.labels[a] < f.labels[b] else (b, a)
    assert orc.hd(mid[None], np.array([lo], np.uint32), f.X, f.labels, 0.1)[1] == 0.0
    assert orc.hd(mid[None], np.array([hi], np.uint32), f.X, f.labels, 0.1)[1] == 1.0
    off = mid + 1e-3 * (f.X[b] - f.X[a])
    assert orc.hd(off[None], np.array([a], np.uint32), f.X, f.labels, 0.1)[1] == 1.0
    assert orc.hd(off[None], np.array([b], np.uint32), f.X, f.labels, 0.1)[1] == 0.0
    X = f.X.copy()
    X[3] = X[2]                                  # two labels on one point
    g = w.Format("dup-qpsk", X, f.labels.copy())
    lo, hi = (2, 3) if g.labels[2] < g.labels[3] else (3, 2)
    assert orc.hd(X[2][None] + 0.01, np.array([lo], np.uint32), g.X, g.labels, 0.1)[1] == 0.0
    assert orc.hd(X[2][None] + 0.01, np.array([hi], np.uint32), g.X, g.labels, 0.1)[1] == 1.0
    # the rule follows labels, not rows: swap the two rows' labels
    lab = g.labels.copy()
    lab[2], lab[3] = lab[3], lab[2]
    assert orc.hd(X[2][None] + 0.01, np.array([hi], np.uint32), g.X, lab, 0.1)[1] == 0.0
    assert orc.hd(X[2][None] + 0.01, np.array([lo], np.uint32), g.X, lab, 0.1)[1] == 1.0