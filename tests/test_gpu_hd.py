"""Hard decisions through the C ABI (mdgmi_gmi_hd) against the FP64 oracle
on the same inputs, every exact path:
* bit errors of the bitwise MAP decision (sign of the exact LLR) and symbol
  errors of the nearest-point decision, as counts over n samples;
* the GMI/MI fields of the same call against the oracle and against
  mdgmi_gmi.

The FP32 paths decide from sums and distances carrying rounding: a decision
the oracle takes within that rounding of its threshold may go either way.
Such decisions are counted from the oracle's own values (LLRs with
|lambda| <= 2e-3 max(|lambda|, 1), distance margins within 5e-3 + 1e-5 of
the log2 metric), and the counts must agree to within them; every other
decision must agree exactly. The FP64 path uses 1e-9 for both.
Exact ties between points that share their coordinates are no rounding
question: both sides decide them for the lowest label, so they are not
counted as ambiguous and must agree exactly.
Edge cases: coincident points (ties go to the lowest label), non-finite
samples (m bit errors, one symbol error), noiseless 30 dB, and samples
received far from their sent point (the per-class path of the FP32 kernels).
"""
import math
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import mdgmi  # noqa: E402

PATHS = ["f64", "direct", "mfma", "mfma_bf16"]
GMI_TOL = {"f64": 1e-10, "direct": 1e-4, "mfma": 1e-4, "mfma_bf16": 1e-4}
LOG2E = 1.0 / math.log(2.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dt(path):
    return torch.float64 if path == "f64" else torch.float32


def ambiguous(orc, y, tx, X, labels, s2, path):
    """(bits, symbols) whose oracle decision lies within the path's rounding
    of its threshold."""
    lam = orc.llr(y, X, labels, s2)
    rel = 1e-9 if path == "f64" else 2e-3
    amb_bits = int(np.count_nonzero(np.abs(lam) <= rel * np.maximum(np.abs(lam), 1.0)))
    d = np.concatenate([((y[a:a + 256, None, :] - X[None, :, :]) ** 2).sum(axis=2)
                        for a in range(0, len(y), 256)])
    s = LOG2E / (2.0 * s2)
    rows = np.arange(len(tx))
    di = d[rows, tx]
    d[rows, tx] = np.inf
    # points with the sent point's coordinates tie exactly: decided by label
    d[np.all(X[None, :, :] == X[tx][:, None, :], axis=2)] = np.inf
    margin = s * (d.min(axis=1) - di)
    if path == "f64":
        tol = 1e-9 * np.maximum(s * di, 1.0)
    else:
        tol = 5e-3 + 1e-5 * s * (np.sum(y * y, axis=1) + np.max(np.sum(X * X, axis=1)))
    amb_sym = int(np.count_nonzero(np.abs(margin) <= tol))
    return amb_bits, amb_sym


def check_hd(orc, f, y, tx, s2s, path, label):
    gf = mdgmi.Format.of(f)
    n = y.shape[1]
    out = mdgmi.mdgmi_gmi_hd(gf, dev(y, dt(path)), dev_u32(tx), s2s, path=path).cpu().numpy()
    gmi = mdgmi.mdgmi_gmi(gf, dev(y, dt(path)), dev_u32(tx), s2s, path=path).cpu().numpy()
    ref = orc.gmi_per_snr(y, tx, f.X, f.labels, s2s)
    for q, s2 in enumerate(s2s):
        r = orc.hd(y[q], tx[q], f.X, f.labels, float(s2))
        ab, asym = ambiguous(orc, y[q], tx[q], f.X, f.labels, float(s2), path)
        be_gpu, be_ref = out[q, 6] * n * f.m, r[0] * n * f.m
        se_gpu, se_ref = out[q, 7] * n, r[1] * n
        say(f"[hd] {label} {path} q={q}: bit errors {be_gpu:.0f} vs {be_ref:.0f} (amb {ab}), "
            f"symbol errors {se_gpu:.0f} vs {se_ref:.0f} (amb {asym})")
        assert abs(be_gpu - round(be_gpu)) < 1e-6 and abs(se_gpu - round(se_gpu)) < 1e-6
        assert abs(be_gpu - be_ref) <= ab, (q, be_gpu, be_ref, ab)
        assert abs(se_gpu - se_ref) <= asym, (q, se_gpu, se_ref, asym)
        assert out[q, 4] == n and out[q, 5] == r[3]
    fin = np.all(np.isfinite(ref[:, :2]), axis=1)
    assert np.max(np.abs(out[fin, :2] - ref[fin, :2]), initial=0.0) <= GMI_TOL[path]
    np.testing.assert_allclose(out[fin, :4], gmi[fin, :4], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(out[:, 4:6], gmi[:, 4:6])
    return out


FORMATS = {
    "qam16": (w.format_16qam, [6.0, 12.0, 18.0]),
    "4d64": (w.format_4d64, [4.0, 10.0, 16.0]),
    "8d256": (lambda: w.random_shells(8, 256, 11), [2.0, 8.0, 14.0]),
    "8d2048": (w.format_8d2048, [6.0, 12.0, 18.0]),
}


@pytest.mark.parametrize("name", list(FORMATS))
@pytest.mark.parametrize("path", PATHS)
def test_hd_parity(orc, name, path):
    make, snrs = FORMATS[name]
    f = make()
    s2s = w.sigma2_from_snr_db(np.array(snrs), f.dim)
    n = 3001
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=31, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y = np.stack(ys)
    tx = np.stack(txs)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    out = check_hd(orc, f, y, tx, s2s, path, name)
    assert out[0, 6] > out[-1, 6] and out[0, 7] > out[-1, 7]   # errors fall with SNR


@pytest.mark.parametrize("path", PATHS)
def test_hd_coincident_points(orc, path):
    """Rows 5 and 9 share one point (labels 5 and 9): the nearest-point
    decision goes to the lower label, so every sample sent on row 9 and
    received next to it is a symbol error and every such sample sent on
    row 5 is none; the kernels must count exactly those."""
    f = w.random_shells(4, 16, 77)
    X = f.X.copy()
    X[5] = X[9]
    g = w.Format("dup4d-16", X, f.labels.copy())
    assert g.labels[5] < g.labels[9]
    s2 = float(w.sigma2_from_snr_db(14.0, 4))
    y, tx = w.channel_samples(g, s2, seed=5, snr_slot=0, n=3001)
    rng = np.random.default_rng(55)
    for k0, j in ((0, 5), (3, 9)):                      # sent on the shared point, received near it
        tx[k0::7] = j
        y[k0::7] = X[j] + 0.02 * rng.standard_normal((len(y[k0::7]), 4))
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    check_hd(orc, g, y[None], tx[None], np.array([s2]), path, "coincident")
    gf = mdgmi.Format.of(g)
    for k0, j, want in ((0, 5, 0.0), (3, 9, 1.0)):
        ys, ts = y[k0::7], tx[k0::7]
        assert orc.hd(ys, ts, g.X, g.labels, s2)[1] == want
        out = mdgmi.mdgmi_gmi_hd(gf, dev(ys[None], dt(path)), dev_u32(ts[None]), [s2], path=path).cpu().numpy()
        assert out[0, 7] == want, (j, out[0, 7])


@pytest.mark.parametrize("path", PATHS)
def test_hd_nonfinite_samples(orc, path):
    f = w.format_4d64()
    s2 = float(w.sigma2_from_snr_db(10.0, 4))
    y, tx = w.channel_samples(f, s2, seed=6, snr_slot=0, n=1000)
    y[17, 2] = np.nan
    y[400, 0] = np.inf
    y[999, 3] = np.nan
    gf = mdgmi.Format.of(f)
    yy = y if path == "f64" else y.astype(np.float32).astype(np.float64)
    out = mdgmi.mdgmi_gmi_hd(gf, dev(yy[None], dt(path)), dev_u32(tx[None]), [s2], path=path).cpu().numpy()
    r = orc.hd(yy, tx, f.X, f.labels, s2)
    assert out[0, 5] == 3 and r[3] == 3
    ok = np.isfinite(yy).all(axis=1)
    ab, asym = ambiguous(orc, yy[ok], tx[ok], f.X, f.labels, s2, path)
    assert abs(out[0, 6] - r[0]) * 1000 * f.m <= ab + 1e-6
    assert abs(out[0, 7] - r[1]) * 1000 <= asym + 1e-6
    assert out[0, 6] * 1000 * f.m >= 3 * f.m and out[0, 7] * 1000 >= 3


@pytest.mark.parametrize("path", PATHS)
def test_hd_noiseless(orc, path):
    f = w.format_4d64()
    s2 = float(w.sigma2_from_snr_db(30.0, 4))
    y, tx = w.channel_samples(f, s2, seed=7, snr_slot=0, n=4099)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    out = mdgmi.mdgmi_gmi_hd(mdgmi.Format.of(f), dev(y[None], dt(path)), dev_u32(tx[None]), [s2],
                             path=path).cpu().numpy()
    r = orc.hd(y, tx, f.X, f.labels, s2)
    assert r[0] == 0.0 and r[1] == 0.0
    assert out[0, 6] == 0.0 and out[0, 7] == 0.0


@pytest.mark.parametrize("path", PATHS)
def test_hd_far_from_sent_point(orc, path):
    """Received near a random point other than the sent one at low noise:
    the sent point's metric exceeds the common exponent window, so the FP32
    kernels take their per-class path for the costs and the decisions."""
    f = w.format_4d64()
    rng = np.random.default_rng(99)
    n = 2003
    s2 = 0.002
    tx = rng.integers(0, f.M, n).astype(np.uint32)
    near = rng.integers(0, f.M, n)
    y = f.X[near] + math.sqrt(s2) * rng.standard_normal((n, f.dim))
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    d_sent = ((y - f.X[tx]) ** 2).sum(axis=1)
    far = LOG2E / (2 * s2) * d_sent > 200.0
    assert far.sum() > n // 2
    check_hd(orc, f, y[None], tx[None], np.array([s2]), path, "far")


def test_hd_workspace_and_errors():
    f = w.format_16qam()
    gf = mdgmi.Format.of(f)
    for p in ("f64", "direct", "mfma", "auto"):
        assert mdgmi.mdgmi_gmi_hd_workspace_size(gf, 1000, 3, p) >= mdgmi.mdgmi_gmi_workspace_size(gf, 1000, 3, p)
    y = torch.zeros((1, 8, 2), dtype=torch.float32, device="cuda")
    tx = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_hd(gf, y, tx, [-1.0], path="direct")
    assert e.value.code == mdgmi.MDGMI_E_SIGMA2
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_hd(gf, y, tx, [0.1], path="direct", ws=mdgmi.workspace(8))
    assert e.value.code == mdgmi.MDGMI_E_WORKSPACE


@pytest.mark.parametrize("path", PATHS)
def test_hd_and_maxlog_many_snrs_in_one_call(path):
    """41 SNR points in one call (two launches of at most 32 points, and
    per-SNR partials of 7 values with hard decisions): every row equals the
    call for that SNR point alone; error counts are integers, so BER/SER
    agree exactly, GMI/MI to rounding."""
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    snrs = np.linspace(-5.0, 25.0, 41)
    s2s = w.sigma2_from_snr_db(snrs, 4)
    n = 1501
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=61, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y = np.stack(ys)
    tx = np.stack(txs)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    yd, td = dev(y, dt(path)), dev_u32(tx)
    out = mdgmi.mdgmi_gmi_hd(gf, yd, td, s2s, path=path).cpu().numpy()
    ml = mdgmi.mdgmi_gmi_maxlog(gf, yd, td, s2s, path=path).cpu().numpy()
    for q in (0, 20, 31, 32, 40):
        one = mdgmi.mdgmi_gmi_hd(gf, yd[q:q + 1].contiguous(), td[q:q + 1].contiguous(), [s2s[q]],
                                 path=path).cpu().numpy()[0]
        np.testing.assert_array_equal(out[q, 4:], one[4:])
        np.testing.assert_allclose(out[q, :4], one[:4], rtol=1e-12, atol=1e-12)
        mo = mdgmi.mdgmi_gmi_maxlog(gf, yd[q:q + 1].contiguous(), td[q:q + 1].contiguous(), [s2s[q]],
                                    path=path).cpu().numpy()[0]
        np.testing.assert_allclose(ml[q, [0, 2]], mo[[0, 2]], rtol=1e-12, atol=1e-12)
        assert np.isnan(ml[q, 1]) and ml[q, 4] == n
