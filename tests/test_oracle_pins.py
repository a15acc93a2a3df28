"""Pins of the FP64 oracle against things other than itself (CPU only).

Each pin is chosen so that a plausible slip in the oracle (a sign, a factor of
two in the noise variance, a dropped class term, a transposed operand, a wrong
label bit) fails at least one of them:

* hand-derived closed-form LLRs of BPSK / Gray QPSK;
* the Gauss-Hermite closed form of Gray QPSK GMI = MI;
* density-based grid integration (MI as E log p(y|x)/p(y), GMI as the sum of
  bit-wise mutual informations) for 1-D PAM and 2-D PSK/ring/QAM formats;
* 16-QAM = 4-PAM x 4-PAM separability;
* low- and high-SNR limits, GMI <= MI, label and geometry invariances.
"""
import math

import numpy as np
import pytest

import quadrature as q
import workloads as w

LOG2E = 1.0 / math.log(2.0)


def bpsk_format():
    return w.Format("BPSK", np.array([[-1.0], [1.0]]), np.array([0, 1], dtype=np.uint32))


def pam4_1d():
    return np.array([[-3.0], [-1.0], [1.0], [3.0]]) / math.sqrt(10.0), np.array([0, 1, 3, 2], np.uint32)


# --------------------------------------------------------------------------- generator
def test_philox_known_answers():
    """Published Philox-4x32-10 known-answer vectors (Random123 distribution)."""
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for c, k, exp in cases:
        out = w.philox4x32_10(np.array([c], np.uint32), np.array([k], np.uint32))[0]
        assert [int(v) for v in out] == exp


def test_generator_random_access_and_moments():
    f = w.format_4d64()
    y, tx = w.channel_samples(f, 0.01, seed=5, snr_slot=3, n=20000)
    idx = np.array([0, 17, 19999, 12345], dtype=np.uint64)
    y2, tx2 = w.channel_samples(f, 0.01, seed=5, snr_slot=3, idx=idx)
    np.testing.assert_array_equal(tx[idx.astype(int)], tx2)
    np.testing.assert_array_equal(y[idx.astype(int)], y2)
    z = (y - f.X[tx]) / 0.1
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    counts = np.bincount(tx, minlength=64)
    chi2 = float(((counts - 20000 / 64) ** 2 / (20000 / 64)).sum())
    assert chi2 < 120  # 63 dof, p ~ 1e-5


def test_formats_are_valid():
    fmts = [w.format_16qam(), w.format_4d64(), w.format_8d2048(), w.psk(3), w.pam(3)]
    fmts += w.ragged_formats()
    assert len(fmts) == 5 + 48
    for f in fmts:
        assert w.check_labels(f.labels, f.M), f.name
        assert abs(np.mean(np.sum(f.X ** 2, axis=1)) - 1.0) < 1e-12, f.name
    rf = w.ragged_formats()
    assert sorted({f.dim for f in rf}) == [2, 4, 8]
    assert {f.M for f in rf} == {1 << m for m in range(2, 13)}


def test_named_format_geometry():
    f = w.format_16qam()
    lev = np.array([-3, -1, 1, 3]) / math.sqrt(10)
    assert set(np.round(f.X[:, 0], 12)) == set(np.round(lev, 12))
    # Gray: nearest neighbours differ in exactly one label bit
    for a in range(16):
        for b in range(16):
            if abs(np.linalg.norm(f.X[a] - f.X[b]) - 2 / math.sqrt(10)) < 1e-9:
                assert bin(int(f.labels[a]) ^ int(f.labels[b])).count("1") == 1
    g = w.format_8d2048()
    r = np.linalg.norm(g.X, axis=1)
    assert np.allclose(r[:1024], r[0]) and np.allclose(r[1024:], 1.6 * r[0])


# --------------------------------------------------------------------------- closed forms
def test_bpsk_llr_closed_form(orc):
    f = bpsk_format()
    rng = np.random.default_rng(0)
    for s2 in (0.05, 0.5, 3.0):
        y = rng.normal(size=(500, 1)) * 2
        lam = orc.llr(y, f.X, f.labels, s2)
        np.testing.assert_allclose(lam[:, 0], 2.0 * y[:, 0] / s2, rtol=1e-12, atol=1e-12)


def test_qpsk_llr_closed_form(orc):
    f = w.square_qam(2)          # label = aI<<1 | aQ, bit 0 on the Q axis
    a = 1.0 / math.sqrt(2.0)
    rng = np.random.default_rng(1)
    for s2 in (0.02, 0.3):
        y = rng.normal(size=(400, 2))
        lam = orc.llr(y, f.X, f.labels, s2)
        np.testing.assert_allclose(lam[:, 0], 2 * a * y[:, 1] / s2, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(lam[:, 1], 2 * a * y[:, 0] / s2, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("snr_db", [-6, 0, 2, 4, 6, 8, 10, 12, 14])
def test_qpsk_gauss_hermite(orc, snr_db):
    f = w.square_qam(2)
    s2 = float(w.sigma2_from_snr_db(snr_db, 2))
    ref = q.qpsk_mi(10 ** (snr_db / 10))
    g, mi = q.oracle_expectation(orc.costs, f.X, f.labels, s2, n=150)
    assert abs(g - ref) < 1e-8 and abs(mi - ref) < 1e-8


def test_per_sample_identity_bpsk_qpsk(orc):
    """With m = 1 per real axis (BPSK, Gray QPSK) the GMI and MI costs coincide
    sample by sample."""
    for f, s2 in ((bpsk_format(), 0.4), (w.square_qam(2), 0.1), (w.square_qam(2), 0.01)):
        y, tx = w.channel_samples(f, s2, seed=11, snr_slot=0, n=3000)
        cg, cm = orc.costs(y, tx, f.X, f.labels, s2)
        np.testing.assert_allclose(cg, cm, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------- density integration
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("snr_db", [0, 8, 16])
def test_pam_density_integration(orc, m, snr_db):
    f = w.pam(m)
    s2 = float(w.sigma2_from_snr_db(snr_db, 1))
    dg, dm = q.density_gmi_mi_1d(f.X, f.labels, s2, n_grid=100001)
    og, om = q.oracle_expectation(orc.costs, f.X, f.labels, s2, n=200)
    assert abs(og - dg) < 1e-6 and abs(om - dm) < 1e-6


@pytest.mark.parametrize("fmt", ["qpsk", "8psk", "2ring8", "8qam"])
@pytest.mark.parametrize("snr_db", [2, 9])
def test_2d_density_integration(orc, fmt, snr_db):
    f = {"qpsk": w.psk(2, offset=math.pi / 4), "8psk": w.psk(3), "2ring8": w.two_ring_8(1.8),
         "8qam": w.qam(2, 1)}[fmt]
    s2 = float(w.sigma2_from_snr_db(snr_db, 2))
    dg, dm = q.density_gmi_mi_2d(f.X, f.labels, s2, n_grid=801)
    og, om = q.oracle_expectation(orc.costs, f.X, f.labels, s2, n=100)
    assert abs(og - dg) < 2e-6 and abs(om - dm) < 2e-6


@pytest.mark.parametrize("snr_db", [0, 6, 12, 18])
def test_16qam_equals_two_4pam(orc, snr_db):
    """Gray square 16-QAM is the product of two Gray 4-PAMs with independent
    I/Q noise, so both rates are twice the 4-PAM rates (grid integration)."""
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(snr_db, 2))
    X1, l1 = pam4_1d()
    dg, dm = q.density_gmi_mi_1d(X1, l1, s2, n_grid=200001)
    og, om = q.oracle_expectation(orc.costs, f.X, f.labels, s2, n=120)
    assert abs(og - 2 * dg) < 2e-6 and abs(om - 2 * dm) < 2e-6


def test_product_separability_per_sample(orc):
    """For a product format with concatenated labels, LLRs of the bits of one
    component depend only on that component, and both costs add per sample."""
    fa, fb = w.two_ring_8(1.8), w.psk(2, offset=0.3)
    f = w.product(fa, fb)
    # the product is normalised as a whole: read the components back at that scale
    Xa = f.X[::fb.M, :2]
    Xb = f.X[:fb.M, 2:]
    s2 = 0.03
    y, tx = w.channel_samples(f, s2, seed=4, snr_slot=0, n=2000)
    lam = orc.llr(y, f.X, f.labels, s2)
    lam_a = orc.llr(y[:, :2], Xa, fa.labels, s2)
    lam_b = orc.llr(y[:, 2:], Xb, fb.labels, s2)
    np.testing.assert_allclose(lam[:, :fb.m], lam_b, rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(lam[:, fb.m:], lam_a, rtol=1e-10, atol=1e-9)
    cg, cm = orc.costs(y, tx, f.X, f.labels, s2)
    cga, cma = orc.costs(y[:, :2], tx // fb.M, Xa, fa.labels, s2)
    cgb, cmb = orc.costs(y[:, 2:], tx % fb.M, Xb, fb.labels, s2)
    np.testing.assert_allclose(cg, cga + cgb, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(cm, cma + cmb, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------- limits and invariants
def test_low_snr_limit(orc):
    f = w.square_qam(2)
    for snr_db in (-30.0, -40.0):
        snr = 10 ** (snr_db / 10)
        g, mi = q.oracle_expectation(orc.costs, f.X, f.labels, float(w.sigma2_from_snr_db(snr_db, 2)), n=60)
        assert 0.998 < mi / (snr * LOG2E) < 1.0001
        assert 0.998 < g / (snr * LOG2E) < 1.0001
    f = w.format_8d2048()
    y, tx = w.channel_samples(f, float(w.sigma2_from_snr_db(-40, 8)), seed=1, snr_slot=0, n=300)
    r = orc.gmi(y, tx, f.X, f.labels, float(w.sigma2_from_snr_db(-40, 8)))
    assert abs(r[0]) < 5 * r[2] + 1e-3 and abs(r[1]) < 5 * r[3] + 1e-3


def test_high_snr_limit(orc):
    for f in (w.format_16qam(), w.format_4d64(), w.format_8d2048()):
        s2 = float(w.sigma2_from_snr_db(45, f.dim))
        y, tx = w.channel_samples(f, s2, seed=2, snr_slot=0, n=500)
        r = orc.gmi(y, tx, f.X, f.labels, s2)
        assert abs(r[0] - f.m) < 1e-9 and abs(r[1] - f.m) < 1e-9


@pytest.mark.parametrize("name,snr_db", [("8d", 2.0), ("8d", 12.0), ("4d", 0.0), ("16qam", 4.0)])
def test_gmi_le_mi(orc, name, snr_db):
    f = {"8d": w.format_8d2048(), "4d": w.format_4d64(), "16qam": w.format_16qam()}[name]
    s2 = float(w.sigma2_from_snr_db(snr_db, f.dim))
    y, tx = w.channel_samples(f, s2, seed=3, snr_slot=0, n=3000 if f.M > 64 else 20000)
    cg, cm = orc.costs(y, tx, f.X, f.labels, s2)
    d = cg - cm                          # MI - GMI estimated as mean(cg - cm)
    se = d.std(ddof=1) / math.sqrt(d.size)
    assert d.mean() >= -3 * se
    assert np.all(cm >= -1e-12)          # log2 sum_j e^{-(t_j - t_i)} >= 0 (term j = i)


def test_invariances(orc):
    f = w.format_4d64()
    s2 = 0.02
    y, tx = w.channel_samples(f, s2, seed=6, snr_slot=0, n=800)
    lam = orc.llr(y, f.X, f.labels, s2)
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    t = rng.normal(size=4)
    np.testing.assert_allclose(orc.llr(y @ Q.T + t, f.X @ Q.T + t, f.labels, s2), lam, rtol=1e-8, atol=1e-8)
    perm = rng.permutation(f.M)
    np.testing.assert_allclose(orc.llr(y, f.X[perm], f.labels[perm], s2), lam, rtol=1e-12, atol=1e-12)
    # complementing label bit 2 negates LLR column 2 only
    lab = f.labels ^ np.uint32(1 << 2)
    lam2 = orc.llr(y, f.X, lab, s2)
    np.testing.assert_allclose(lam2[:, 2], -lam[:, 2], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.delete(lam2, 2, 1), np.delete(lam, 2, 1), rtol=1e-12, atol=1e-12)
    # swapping label bits 0 and 5 swaps the LLR columns
    b0, b5 = (f.labels >> 0) & 1, (f.labels >> 5) & 1
    lab = (f.labels & ~np.uint32(0b100001)) | (b0 << 5) | b5
    lam3 = orc.llr(y, f.X, lab.astype(np.uint32), s2)
    np.testing.assert_allclose(lam3[:, [5, 1, 2, 3, 4, 0]], lam, rtol=1e-12, atol=1e-12)


def test_sign_convention_high_snr(orc):
    """Near point j at high SNR, sign(lambda_k) equals bit k of labels[j]."""
    f = w.format_4d64()
    s2 = float(w.sigma2_from_snr_db(25, 4))
    lam = orc.llr(f.X, f.X, f.labels, s2)
    bits = (f.labels[:, None] >> np.arange(6)) & 1
    assert np.all((lam > 0) == (bits == 1))


def test_far_classes_do_not_underflow(orc):
    """A 16-QAM corner sample at 30 dB: the far classes sit hundreds of nats
    away; the LLR equals the max-log value up to ln(M/2) and stays finite."""
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(30, 2))
    y = f.X[[0, 5, 15]] + 0.01
    lam = orc.llr(y, f.X, f.labels, s2)
    assert np.all(np.isfinite(lam)) and np.abs(lam).max() > 700
    d2 = ((y[:, None, :] - f.X[None]) ** 2).sum(-1) / (2 * s2)
    for k in range(4):
        b = ((f.labels >> k) & 1).astype(bool)
        maxlog = d2[:, ~b].min(1) - d2[:, b].min(1)
        assert np.all(np.abs(lam[:, k] - maxlog) <= math.log(8) + 1e-9)


def test_mc_against_quadrature_16qam(orc):
    """The Monte-Carlo estimate on the seeded 16-QAM workload agrees with the
    2 x 4-PAM grid integral within 4 standard errors."""
    wl = w.workload_qam16(n=100_000)
    X1, l1 = pam4_1d()
    for s in (0, 2, 5):
        s2 = float(wl.sigma2[s])
        y, tx = w.channel_samples(wl.fmt, s2, wl.seed, s, n=wl.n)
        r = orc.gmi(y, tx, wl.fmt.X, wl.fmt.labels, s2)
        dg, dm = q.density_gmi_mi_1d(X1, l1, s2, n_grid=100001)
        assert abs(r[0] - 2 * dg) < 4 * r[2] and abs(r[1] - 2 * dm) < 4 * r[3]
        assert r[4] == wl.n and r[5] == 0


def test_nonfinite_is_flagged(orc):
    f = w.format_16qam()
    y, tx = w.channel_samples(f, 0.05, seed=0, snr_slot=0, n=100)
    y[7, 1] = np.nan
    r = orc.gmi(y, tx, f.X, f.labels, 0.05)
    assert np.isnan(r[0]) and r[5] == 1
