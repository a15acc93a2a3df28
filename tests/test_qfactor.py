"""The host-only Q-factor conversion of the C ABI (no GPU call): the
Gaussian-noise relation BER = erfc(Q / sqrt 2) / 2, checked against
scipy's inverse complementary error function, round trips at the two
HD-FEC thresholds the paper quotes (8.4 dB for 6.7 % overhead and 5.7 dB
for 20 % overhead, experimental-results subsections), the textbook point
Q = 6 <-> BER = 9.87e-10, and the end points."""
import math

import numpy as np
import pytest
from scipy.special import erfcinv

from paper_2011_13695_amd import mdgmi


def ber_of_q_db(q_db):
    return 0.5 * math.erfc(10 ** (q_db / 20) / math.sqrt(2.0))


@pytest.mark.parametrize("ber", [1e-300, 1e-15, 1e-9, 1e-6, 1e-3, 3.8e-3, 4.5e-3, 2e-2, 0.1, 0.3, 0.49])
def test_matches_erfcinv(ber):
    ref = 20 * math.log10(math.sqrt(2.0) * erfcinv(2 * ber))
    assert mdgmi.mdgmi_q_factor_db(ber) == pytest.approx(ref, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("q_db", [8.4, 5.7, 12.0, 3.0])
def test_round_trip_thresholds(q_db):
    assert mdgmi.mdgmi_q_factor_db(ber_of_q_db(q_db)) == pytest.approx(q_db, abs=1e-10)


def test_textbook_q6():
    ber = ber_of_q_db(20 * math.log10(6.0))
    assert ber == pytest.approx(9.8659e-10, rel=1e-4)
    assert mdgmi.mdgmi_q_factor_db(ber) == pytest.approx(20 * math.log10(6.0), abs=1e-10)


def test_end_points_and_monotone():
    assert mdgmi.mdgmi_q_factor_db(0.0) == math.inf
    assert mdgmi.mdgmi_q_factor_db(0.5) == -math.inf
    for bad in (-1e-3, 0.5000001, math.nan, math.inf):
        assert math.isnan(mdgmi.mdgmi_q_factor_db(bad))
    b = np.logspace(-12, math.log10(0.49), 200)
    q = [mdgmi.mdgmi_q_factor_db(float(v)) for v in b]
    assert all(x > y for x, y in zip(q, q[1:]))
