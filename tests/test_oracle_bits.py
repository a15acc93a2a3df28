"""Pins of the oracle's per-bit GMI (each label bit's share of the GMI at
s = 1): it sums to the GMI; for Gray 4-PAM and 8-PAM each bit's estimate
agrees within Monte-Carlo error with the bit-wise mutual information
I(B_k; Y) from grid integration of the channel densities (which never forms
an LLR); for Gray 16-QAM the in-phase and quadrature bits mirror each other."""
import numpy as np
import pytest

import quadrature as qd
import workloads as w


@pytest.mark.parametrize("m,snr_db", [(2, 6.0), (2, 12.0), (3, 10.0), (3, 16.0)])
def test_pam_bits_against_quadrature(orc, m, snr_db):
    f = w.pam(m)
    s2 = float(w.sigma2_from_snr_db(snr_db, 1))
    n = 200_000
    y, tx = w.channel_samples(f, s2, seed=m, snr_slot=int(snr_db), n=n)
    g, se = orc.gmi_bits(orc.llr(y, f.X, f.labels, s2), f.labels[tx])
    ref = qd.density_bitwise_1d(f.X, f.labels, s2)
    assert len(ref) == m
    for k in range(m):
        assert abs(g[k] - ref[k]) <= 4 * se[k] + 1e-6, (k, g[k], ref[k], se[k])
    # Gray PAM: the bits are not alike (the sign bit is the most reliable)
    assert max(ref) - min(ref) > 0.01


def test_sum_is_the_gmi_and_qam_symmetry(orc):
    f = w.format_16qam()
    s2 = float(w.sigma2_from_snr_db(9.0, 2))
    y, tx = w.channel_samples(f, s2, seed=7, snr_slot=0, n=100_000)
    lam = orc.llr(y, f.X, f.labels, s2)
    g, se = orc.gmi_bits(lam, f.labels[tx])
    assert np.sum(g) == pytest.approx(orc.gmi(y, tx, f.X, f.labels, s2)[0], abs=1e-12)
    # label = g(I) << 2 | g(Q): bits 0/1 on the quadrature axis mirror bits 2/3 on the in-phase axis
    assert abs(g[0] - g[2]) <= 4 * np.hypot(se[0], se[2])
    assert abs(g[1] - g[3]) <= 4 * np.hypot(se[1], se[3])
