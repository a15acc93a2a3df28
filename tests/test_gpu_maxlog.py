"""Max-log metrics and the s-optimised GMI through the C ABI, against the
FP64 oracle on the same inputs:
* mdgmi_llr_maxlog on every path: |d lambda| <= 1e-3 max(|lambda|, 1) nats
  (FP64 path 1e-9), formats from M = 16 (padding rows in the MFMA image) to
  M = 2048, samples far from every point (the FP32 per-class path) and
  non-finite samples;
* mdgmi_gmi_maxlog: the GMI of the oracle's max-log LLRs at s = 1 within
  1e-4 bit (FP64 path 1e-10), MI fields NaN;
* mdgmi_gmi_sopt on the very LLRs the GPU produced (copied to the host for
  the oracle): GMI at s = 1 and at s* within 1e-6 bit, s* within 1e-3
  relative; the binary-symmetric closed form; s* = 0 for LLRs that favour
  the wrong bit; non-finite LLRs and sent rows out of range.
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
LLR_RTOL = {"f64": 1e-9, "direct": 1e-3, "mfma": 1e-3, "mfma_bf16": 1e-3}
GMI_TOL = {"f64": 1e-10, "direct": 1e-4, "mfma": 1e-4, "mfma_bf16": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dt(path):
    return torch.float64 if path == "f64" else torch.float32


def ratio(got, ref, path):
    return float(np.max(np.abs(got - ref) / (LLR_RTOL[path] * np.maximum(np.abs(ref), 1.0))))


FORMATS = {
    "qam16": (w.format_16qam, [4.0, 12.0, 24.0]),
    "4d64": (w.format_4d64, [2.0, 10.0, 20.0]),
    "8d256": (lambda: w.random_shells(8, 256, 11), [0.0, 8.0, 16.0]),
    "8d2048": (w.format_8d2048, [2.0, 10.0, 17.0]),
}


def inputs(f, snrs, n, path, seed=41):
    s2s = w.sigma2_from_snr_db(np.array(snrs), f.dim)
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=seed, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y = np.stack(ys)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    return y, np.stack(txs), s2s


@pytest.mark.parametrize("name", list(FORMATS))
@pytest.mark.parametrize("path", PATHS)
def test_maxlog_llr_and_gmi(orc, name, path):
    make, snrs = FORMATS[name]
    f = make()
    gf = mdgmi.Format.of(f)
    n = 3001
    y, tx, s2s = inputs(f, snrs, n, path)
    out = mdgmi.mdgmi_gmi_maxlog(gf, dev(y, dt(path)), dev_u32(tx), s2s, path=path).cpu().numpy()
    for q, s2 in enumerate(s2s):
        lam = mdgmi.mdgmi_llr_maxlog(gf, dev(y[q], dt(path)), float(s2), path=path).cpu().numpy()
        ref = orc.llr_maxlog(y[q], f.X, f.labels, float(s2))
        r = ratio(lam.astype(np.float64), ref, path)
        g, se = orc.gmi_s(ref, f.labels[tx[q]], 1.0)
        say(f"[maxlog] {name} {path} q={q}: LLR err/bar {r:.3f}, GMI {out[q, 0]:.6f} vs {g:.6f}")
        assert r <= 1.0, (q, r)
        assert abs(out[q, 0] - g) <= GMI_TOL[path], (q, out[q, 0], g)
        assert out[q, 2] == pytest.approx(se, rel=1e-3, abs=1e-9)
        assert np.isnan(out[q, 1]) and np.isnan(out[q, 3])
        assert out[q, 4] == n and out[q, 5] == 0


@pytest.mark.parametrize("path", PATHS)
def test_maxlog_far_and_nonfinite(orc, path):
    """Samples far outside the constellation (nearest point beyond the
    exponent window) and non-finite samples."""
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(15.0, 4))
    y, tx = w.channel_samples(f, s2, seed=13, snr_slot=0, n=1003)
    y[::5] *= 6.0                       # far from every point
    y[7, 1] = np.nan
    y[500, 3] = np.inf
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    lam = mdgmi.mdgmi_llr_maxlog(gf, dev(y, dt(path)), s2, path=path).cpu().numpy().astype(np.float64)
    ref = orc.llr_maxlog(y, f.X, f.labels, s2)
    ok = np.isfinite(y).all(axis=1)
    assert np.all(np.isnan(lam[~ok]))
    assert ratio(lam[ok], ref[ok], path) <= 1.0
    far = LOG2E_OVER_2 / s2 * np.min(((y[ok, None, :] - f.X[None]) ** 2).sum(-1), axis=1) > 200.0
    assert far.sum() > 50
    out = mdgmi.mdgmi_gmi_maxlog(gf, dev(y[None], dt(path)), dev_u32(tx[None]), [s2], path=path).cpu().numpy()
    assert out[0, 5] == 2 and np.isnan(out[0, 0])
    good = mdgmi.mdgmi_gmi_maxlog(gf, dev(y[ok][None], dt(path)), dev_u32(tx[ok][None]), [s2],
                                  path=path).cpu().numpy()
    g, _ = orc.gmi_s(ref[ok], f.labels[tx[ok]], 1.0)
    assert abs(good[0, 0] - g) <= GMI_TOL[path]


LOG2E_OVER_2 = 0.5 / math.log(2.0)


@pytest.mark.parametrize("source", ["exact", "maxlog"])
@pytest.mark.parametrize("path", PATHS)
def test_sopt_on_gpu_llrs(orc, source, path):
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    n = 20011
    s2 = float(w.sigma2_from_snr_db(7.0, 4))
    y, tx = w.channel_samples(f, s2, seed=17, snr_slot=0, n=n)
    fn = mdgmi.mdgmi_llr if source == "exact" else mdgmi.mdgmi_llr_maxlog
    lam = fn(gf, dev(y, dt(path)), s2, path=path)
    out = mdgmi.mdgmi_gmi_sopt(gf, lam, dev_u32(tx)).cpu().numpy()
    lh = lam.cpu().numpy().astype(np.float64)
    sent = f.labels[tx]
    g1, se1 = orc.gmi_s(lh, sent, 1.0)
    s, g, se = orc.gmi_sopt(lh, sent)
    tol = 1e-9 if path == "f64" else 1e-6
    say(f"[sopt] {source} {path}: s* {out[2]:.6f} vs {s:.6f}, GMI* {out[3]:.7f} vs {g:.7f}, "
        f"GMI(1) {out[0]:.7f}, {int(out[8])} passes")
    assert abs(out[0] - g1) <= tol and out[1] == pytest.approx(se1, rel=1e-4)
    assert abs(out[3] - g) <= tol and out[2] == pytest.approx(s, rel=1e-3)
    assert out[4] == pytest.approx(se, rel=1e-3)
    assert out[5] == pytest.approx(out[3] / f.m, rel=1e-12)
    assert out[6] == n and out[7] == 0 and out[8] <= 8      # Newton converges in a few passes
    assert out[3] >= out[0] - 1e-12


@pytest.mark.parametrize("p,L,m", [(0.9, 3.7, 1), (0.75, 0.4, 2), (0.97, 12.0, 3)])
def test_sopt_binary_symmetric_closed_form(p, L, m):
    n = 4000
    k = int(round(p * n))
    rng = np.random.default_rng(7)
    M = 1 << m
    X = rng.standard_normal((M, 2))
    f = w.Format(f"bsc{m}", X, np.arange(M, dtype=np.uint32))
    gf = mdgmi.Format.of(f)
    tx = rng.integers(0, M, n).astype(np.uint32)
    bits = ((tx[:, None] >> np.arange(m)) & 1).astype(np.float64)
    right = np.zeros((n, m), bool)
    for j in range(m):
        right[rng.permutation(n)[:k], j] = True
    lam = np.where(right, 1.0, -1.0) * (2.0 * bits - 1.0) * L
    pe = k / n
    for dtype in (torch.float32, torch.float64):
        out = mdgmi.mdgmi_gmi_sopt(gf, dev(lam, dtype), dev_u32(tx)).cpu().numpy()
        assert out[2] == pytest.approx(math.log(pe / (1 - pe)) / L, rel=1e-6)
        h = -pe * math.log2(pe) - (1 - pe) * math.log2(1 - pe)
        assert out[3] == pytest.approx(m * (1 - h), abs=1e-6)


def test_sopt_edge_cases():
    f = w.square_qam(2)
    gf = mdgmi.Format.of(f)
    rng = np.random.default_rng(3)
    n = 1000
    tx = rng.integers(0, 4, n).astype(np.uint32)
    bits = ((tx[:, None] >> np.arange(2)) & 1).astype(np.float64)
    wrong = -(2.0 * bits - 1.0) * 2.0
    out = mdgmi.mdgmi_gmi_sopt(gf, dev(wrong, torch.float32), dev_u32(tx)).cpu().numpy()
    assert out[2] == 0.0 and out[3] == 0.0 and out[0] < 0.0
    right = -wrong
    out = mdgmi.mdgmi_gmi_sopt(gf, dev(right, torch.float32), dev_u32(tx)).cpu().numpy()
    assert out[3] > 2.0 - 1e-6 and out[2] > 10.0          # all correct: GMI -> m as s grows
    bad = right.copy()
    bad[10, 1] = np.nan
    out = mdgmi.mdgmi_gmi_sopt(gf, dev(bad, torch.float32), dev_u32(tx)).cpu().numpy()
    assert out[7] == 1 and np.isnan(out[3]) and np.isnan(out[0])
    tx2 = tx.copy()
    tx2[5] = 99
    out = mdgmi.mdgmi_gmi_sopt(gf, dev(right, torch.float32), dev_u32(tx2)).cpu().numpy()
    assert out[7] == 1 and np.isnan(out[3])
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_sopt(gf, dev(right, torch.float32), dev_u32(tx), ws=mdgmi.workspace(8))
    assert e.value.code == mdgmi.MDGMI_E_WORKSPACE


@pytest.mark.parametrize("source", ["exact", "maxlog"])
@pytest.mark.parametrize("path", PATHS)
def test_per_bit_gmi_on_gpu_llrs(orc, source, path):
    """mdgmi_gmi_bits on the LLRs the GPU produced, against the oracle's
    per-bit GMI of the same values; the bits sum to the GMI at s = 1."""
    f = w.format_16qam() if path == "direct" else w.format_4d64()
    gf = mdgmi.Format.of(f)
    n = 30011
    s2 = float(w.sigma2_from_snr_db(8.0, f.dim))
    y, tx = w.channel_samples(f, s2, seed=29, snr_slot=0, n=n)
    fn = mdgmi.mdgmi_llr if source == "exact" else mdgmi.mdgmi_llr_maxlog
    lam = fn(gf, dev(y, dt(path)), s2, path=path)
    out = mdgmi.mdgmi_gmi_bits(gf, lam, dev_u32(tx)).cpu().numpy()
    so = mdgmi.mdgmi_gmi_sopt(gf, lam, dev_u32(tx)).cpu().numpy()
    g, se = orc.gmi_bits(lam.cpu().numpy().astype(np.float64), f.labels[tx])
    tol = 1e-9 if path == "f64" else 1e-6
    m = f.m
    assert np.max(np.abs(out[0:2 * m:2] - g)) <= tol
    np.testing.assert_allclose(out[1:2 * m:2], se, rtol=1e-3)
    assert out[2 * m] == n and out[2 * m + 1] == 0
    # same costs, summed per bit vs per sample: FP32 terms round differently
    assert abs(np.sum(out[0:2 * m:2]) - so[0]) <= (1e-12 if path == "f64" else 1e-6)
    say(f"[bits] {source} {path}: " + " ".join(f"{v:.4f}" for v in out[0:2 * m:2]))


def test_per_bit_gmi_edges():
    f = w.square_qam(2)
    gf = mdgmi.Format.of(f)
    rng = np.random.default_rng(5)
    n = 777
    tx = rng.integers(0, 4, n).astype(np.uint32)
    bits = ((tx[:, None] >> np.arange(2)) & 1).astype(np.float64)
    lam = (2.0 * bits - 1.0) * 3.0
    out = mdgmi.mdgmi_gmi_bits(gf, dev(lam, torch.float32), dev_u32(tx)).cpu().numpy()
    want = 1.0 - np.log2(1.0 + np.exp(-3.0))
    np.testing.assert_allclose(out[[0, 2]], [want, want], rtol=1e-6)
    assert out[1] == pytest.approx(0.0, abs=1e-12) and out[4] == n and out[5] == 0
    bad = lam.copy()
    bad[3, 1] = np.nan
    out = mdgmi.mdgmi_gmi_bits(gf, dev(bad, torch.float32), dev_u32(tx)).cpu().numpy()
    assert out[5] == 1 and np.isnan(out[2])
    tx2 = tx.copy()
    tx2[0] = 4
    out = mdgmi.mdgmi_gmi_bits(gf, dev(lam, torch.float64), dev_u32(tx2)).cpu().numpy()
    assert out[5] == 1 and np.isnan(out[0]) and np.isnan(out[2])
