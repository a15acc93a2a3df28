"""The per-sample 4x4-block shape of the fp16-split MFMA path (4 <= M <= 512,
8-D up to M = 256; one sample per lane, v_mfma_f32_4x4x4_16b_f16 with the
point operands broadcast from one block to all sixteen) through the
C ABI, against the FP64 oracle on the same samples, in every mode:
* GMI/MI within 1e-4 bit with exact sample counts; exact LLRs within
  1e-3 max(|lambda|, 1) nats; hard-decision error counts within the
  decisions that sit at their thresholds; max-log LLRs (1e-3) and their GMI
  (1e-4);
* every format size the shape serves in 1, 2, 4 and 8 dimensions, n not a
  multiple of 64 (a ragged last batch of lanes), several SNR points in one
  launch, up to SNRs where classes lie beyond the common exponent offset
  (the lane's FP32 per-class path);
* samples far from every point, non-finite samples, samples beyond the fp16
  range of the operand split, and sent rows out of range;
* the shape against the 32 x 32 shape of the same path on the same samples;
* small instances of a ragged batch (their own 4x4-shape kind) against
  per-instance calls: the same per-sample arithmetic, so GMI/MI agree to
  FP64 summation order.
"""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import mdgmi  # noqa: E402

SMALL = 8        # mdgmi_set_tuning variant of the per-sample 4x4 shape
BIG = 4          # a 32 x 32 shape (one column, 16 waves, LDS image)
LLR_RTOL = 1e-3
GMI_TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def ratio(got, ref):
    return float(np.max(np.abs(got - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))))


@pytest.fixture
def shape():
    """Selects a launch shape for the test and restores the default after."""
    def use(v):
        mdgmi.mdgmi_set_tuning(v)
    yield use
    mdgmi.mdgmi_set_tuning(-1)


def fmt(dim, M):
    if dim == 1:
        return w.pam(int(np.log2(M)))
    if dim == 2 and M in (4, 16, 64):
        return w.square_qam(int(np.log2(M)))
    return w.random_shells(dim, M, 100 + 7 * dim + M)


CASES = [(1, 4), (1, 16), (1, 64), (1, 256), (1, 512), (2, 4), (2, 8), (2, 16), (2, 32), (2, 64), (2, 128),
         (2, 256), (2, 512), (4, 4), (4, 16), (4, 32), (4, 64), (4, 128), (4, 256), (4, 512), (8, 4),
         (8, 8), (8, 16), (8, 32), (8, 64), (8, 128), (8, 256)]


def sigma2s_for(f):
    """From a noisy regime to one where classes of a sample lie beyond the
    common exponent offset. The top is capped at s max||x||^2 = 1500: the
    expanded form K - s||x||^2 + <2 s x, y> cancels terms of that size, so
    an LLR near zero carries an absolute error that grows with s (about
    2.3e-7 s max||x||^2 nats for the fp16 split), and the 1e-3 bar holds
    up to s max||x||^2 of about 4000."""
    base = 6.0 * f.m / max(f.dim, 1) ** 0.5
    s2 = w.sigma2_from_snr_db(np.array([0.0, base + 6.0, base + 26.0]), f.dim)
    max_n2 = float((f.X ** 2).sum(1).max())
    return np.maximum(s2, np.log2(np.e) / (2.0 * 1500.0 / max_n2))


@pytest.mark.parametrize("dim,M", CASES)
def test_small_shape_parity(orc, shape, dim, M):
    shape(SMALL)
    f = fmt(dim, M)
    gf = mdgmi.Format.of(f)
    s2s = sigma2s_for(f)
    n = 2053
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=31, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y = np.stack(ys).astype(np.float32).astype(np.float64)
    tx = np.stack(txs)
    out = mdgmi.mdgmi_gmi_hd(gf, dev(y), dev_u32(tx), s2s, path="mfma").cpu().numpy()
    ml = mdgmi.mdgmi_gmi_maxlog(gf, dev(y), dev_u32(tx), s2s, path="mfma").cpu().numpy()
    ref = orc.gmi_per_snr(y, tx, f.X, f.labels, s2s)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert np.all(out[:, 5] == 0)
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL, (out[:, :2], ref[:, :2])
    far_seen = 0
    for q, s2 in enumerate(s2s):
        s2 = float(s2)
        lam = mdgmi.mdgmi_llr(gf, dev(y[q]), s2, path="mfma").cpu().numpy().astype(np.float64)
        lex = orc.llr(y[q], f.X, f.labels, s2)
        assert ratio(lam, lex) <= 1.0, q
        far_seen += int(np.count_nonzero(np.abs(lex) > 150.0))
        lml = mdgmi.mdgmi_llr_maxlog(gf, dev(y[q]), s2, path="mfma").cpu().numpy().astype(np.float64)
        rml = orc.llr_maxlog(y[q], f.X, f.labels, s2)
        assert ratio(lml, rml) <= 1.0, q
        assert abs(ml[q, 0] - orc.gmi_s(rml, f.labels[tx[q]], 1.0)[0]) <= GMI_TOL, q
        assert np.isnan(ml[q, 1])
        # hard decisions: bit errors may differ only where the oracle's LLR
        # is within FP32 rounding of zero, symbol errors only where two
        # distances tie within it
        hd = orc.hd(y[q], tx[q], f.X, f.labels, s2)
        amb = int(np.count_nonzero(np.abs(lex) <= 2e-3 * np.maximum(np.abs(lex), 1.0)))
        assert abs(out[q, 6] - hd[0]) * n * f.m <= amb + 1e-6, q
        d = ((y[q][:, None, :] - f.X[None]) ** 2).sum(-1)
        di = d[np.arange(n), tx[q]]
        d2 = d.copy()
        d2[np.arange(n), tx[q]] = np.inf
        tol = 1e-5 * (1.0 + np.max(np.abs(y[q])) ** 2) / s2
        amb_s = int(np.count_nonzero(np.abs(d2.min(axis=1) - di) / (2 * s2) <= tol))
        assert abs(out[q, 7] - hd[1]) * n <= amb_s + 1e-6, q
    # the highest SNR point reaches LLRs beyond the common offset's window
    assert far_seen > 0
    say(f"[small] dim={dim} M={M}: GMI {out[:, 0]} max-log {ml[:, 0]} BER {out[:, 6]}")


@pytest.mark.parametrize("dim,M", [(2, 16), (4, 64), (8, 32), (1, 8), (2, 256), (8, 64)])
def test_small_against_32x32_shape(shape, dim, M):
    """Both shapes split the same factors into fp16 parts; they differ in
    the order of FP32 roundings only."""
    f = fmt(dim, M)
    gf = mdgmi.Format.of(f)
    s2s = w.sigma2_from_snr_db(np.array([3.0, 12.0]), f.dim)
    n = 5000
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=5, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y, tx = dev(np.stack(ys)), dev_u32(np.stack(txs))
    res = {}
    for v in (SMALL, BIG):
        shape(v)
        res[v] = (mdgmi.mdgmi_gmi_hd(gf, y, tx, s2s, path="mfma").cpu().numpy(),
                  mdgmi.mdgmi_llr(gf, y[1].contiguous(), float(s2s[1]), path="mfma").cpu().numpy())
    a, b = res[SMALL], res[BIG]
    np.testing.assert_array_equal(a[0][:, 4:6], b[0][:, 4:6])
    assert np.max(np.abs(a[0][:, :2] - b[0][:, :2])) <= 1e-6
    assert ratio(a[1].astype(np.float64), b[1].astype(np.float64)) <= 1.0
    say(f"[small vs 32x32] dim={dim} M={M}: dGMI {np.max(np.abs(a[0][:, 0] - b[0][:, 0])):.2e}")


@pytest.mark.parametrize("dim,M", [(2, 16), (4, 64), (8, 16), (4, 256)])
def test_small_shape_edge_samples(orc, shape, dim, M):
    """Far samples, y beyond the fp16 range of the split, non-finite samples
    and a sent row out of range, mixed into ordinary ones."""
    shape(SMALL)
    f = fmt(dim, M)
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(15.0, f.dim))
    n = 300
    y, tx = w.channel_samples(f, s2, seed=9, snr_slot=0, n=n)
    y = y.astype(np.float32).astype(np.float64)
    y[10] = 40.0                       # far from every point: exponents underflow
    y[11] = -7.5
    lam = mdgmi.mdgmi_llr(gf, dev(y), s2, path="mfma").cpu().numpy().astype(np.float64)
    ref = orc.llr(y, f.X, f.labels, s2)
    assert ratio(lam, ref) <= 1.0 and np.abs(ref[10:12]).max() > 1000
    lml = mdgmi.mdgmi_llr_maxlog(gf, dev(y), s2, path="mfma").cpu().numpy().astype(np.float64)
    assert ratio(lml, orc.llr_maxlog(y, f.X, f.labels, s2)) <= 1.0
    out = mdgmi.mdgmi_gmi(gf, dev(y[None]), dev_u32(tx[None]), [s2], path="mfma").cpu().numpy()
    r = orc.gmi(y, tx, f.X, f.labels, s2)
    # per-sample costs of the far samples are large: compare relative to size
    assert abs(out[0, 0] - r[0]) <= 1e-4 * max(1.0, abs(r[0]))
    assert abs(out[0, 1] - r[1]) <= 1e-4 * max(1.0, abs(r[1]))
    # |y| beyond the fp16 range of the split (and ||y||^2 far beyond FP32's
    # resolution of a difference of squared distances): the per-class path
    # forms distance differences in factored form, so the LLRs of every
    # FP32 path meet the bar against the oracle, and so do GMI and MI
    yh = y.copy()
    yh[12] = 5.0e4
    yh[13, 0] = -3.0e5
    yh[14] = [(-1.0) ** q * 7.0e3 * (q + 1) for q in range(dim)]
    ro = orc.llr(yh, f.X, f.labels, s2)
    rg = orc.gmi(yh, tx, f.X, f.labels, s2)
    for path in ("mfma", "direct", "mfma_bf16"):
        a = mdgmi.mdgmi_llr(gf, dev(yh), s2, path=path).cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(a)), path
        assert ratio(a, ro) <= 1.0, (path, ratio(a, ro))
        ga = mdgmi.mdgmi_gmi(gf, dev(yh[None]), dev_u32(tx[None]), [s2], path=path).cpu().numpy()
        assert ga[0, 5] == 0
        assert abs(ga[0, 0] - rg[0]) <= 1e-4 * max(1.0, abs(rg[0])), (path, ga[0, 0], rg[0])
        assert abs(ga[0, 1] - rg[1]) <= 1e-4 * max(1.0, abs(rg[1])), (path, ga[0, 1], rg[1])
        lml = mdgmi.mdgmi_llr_maxlog(gf, dev(yh), s2, path=path).cpu().numpy().astype(np.float64)
        assert ratio(lml, orc.llr_maxlog(yh, f.X, f.labels, s2)) <= 1.0, path
    # a NaN sample and a sent row out of range are counted as non-finite
    good = np.ones(n, bool)
    yb = y.copy()
    yb[20, 0] = np.nan
    txb = tx.copy()
    txb[21] = M + 3
    good[20] = False
    out = mdgmi.mdgmi_gmi_hd(gf, dev(yb[None]), dev_u32(txb[None]), [s2], path="mfma").cpu().numpy()
    assert out[0, 4] == n and out[0, 5] == 2 and np.isnan(out[0, 0]) and np.isnan(out[0, 1])
    lam = mdgmi.mdgmi_llr(gf, dev(yb), s2, path="mfma").cpu().numpy()
    assert np.all(np.isnan(lam[20])) and np.all(np.isfinite(lam[good]))
    ml = mdgmi.mdgmi_gmi_maxlog(gf, dev(yb[None]), dev_u32(txb[None]), [s2], path="mfma").cpu().numpy()
    assert ml[0, 5] == 2 and np.isnan(ml[0, 0])
    say(f"[small edges] dim={dim} M={M}: far GMI {r[0]:.1f}")


def test_small_shape_is_the_default_and_can_be_declined(shape):
    """Untuned small formats run the 4x4 shape on the fp16-split path (and
    AUTO takes that path); asking for a 32 x 32 variant runs that shape; the
    two agree to FP32 rounding and each is bit-reproducible."""
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    mdgmi.mdgmi_tune_clear()
    s2s = w.sigma2_from_snr_db(np.array([2.0, 10.0]), 4)
    y, tx = mdgmi.mdgmi_generate(gf, 3, s2s, 20000, dtype=torch.float32)
    shape(-1)
    dflt = mdgmi.mdgmi_gmi(gf, y, tx, s2s, path="mfma").cpu().numpy()
    auto = mdgmi.mdgmi_gmi(gf, y, tx, s2s, path="auto").cpu().numpy()
    shape(SMALL)
    small = mdgmi.mdgmi_gmi(gf, y, tx, s2s, path="mfma").cpu().numpy()
    small2 = mdgmi.mdgmi_gmi(gf, y, tx, s2s, path="mfma").cpu().numpy()
    shape(BIG)
    big = mdgmi.mdgmi_gmi(gf, y, tx, s2s, path="mfma").cpu().numpy()
    np.testing.assert_array_equal(dflt, small)
    np.testing.assert_array_equal(auto, small)
    np.testing.assert_array_equal(small, small2)
    assert np.max(np.abs(small[:, :2] - big[:, :2])) <= 1e-6


@pytest.mark.parametrize("path", ["mfma", "auto"])
def test_small_instances_in_a_batch(shape, path):
    """Ragged sample counts (1, below and above one item alignment of 256,
    large), every dimension, M = 4 .. 256, in one batch; each row against
    mdgmi_gmi on the same samples."""
    shape(-1)
    mdgmi.mdgmi_tune_clear()
    specs = [(1, 4, 1), (1, 64, 255), (2, 16, 257), (2, 256, 70001), (4, 64, 4099), (4, 128, 600),
             (8, 8, 63), (8, 64, 9000), (2, 4, 1000), (4, 256, 20000), (4, 512, 3000), (8, 256, 2000),
             (1, 512, 30011)]
    items, refs = [], []
    for k, (dim, M, n) in enumerate(specs):
        f = fmt(dim, M)
        gf = mdgmi.Format.of(f)
        s2 = float(w.sigma2_from_snr_db(4.0 + 2.0 * k, dim))
        y, tx = w.channel_samples(f, s2, seed=50 + k, snr_slot=k, n=n)
        yd, td = dev(y), dev_u32(tx)
        items.append((gf, yd, td, s2))
        refs.append(mdgmi.mdgmi_gmi(gf, yd[None], td[None], [s2], path="mfma").cpu().numpy()[0])
    out = mdgmi.mdgmi_gmi_batched(mdgmi.instances(items), path=path).cpu().numpy()
    ref = np.array(refs)
    np.testing.assert_array_equal(out[:, 4:6], ref[:, 4:6])
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= 1e-12
    plan = mdgmi.Batch(items, path=path)
    a = plan.run(use_graph=True).cpu().numpy()
    b = plan.run(use_graph=True).cpu().numpy()
    plan.close()
    np.testing.assert_array_equal(a, b)
    assert np.max(np.abs(a[:, :2] - ref[:, :2])) <= 1e-12
    say(f"[small batch] {path}: max dGMI vs per-instance {np.max(np.abs(out[:, 0] - ref[:, 0])):.1e}")


@pytest.mark.parametrize("name", ["64-PAM", "16-QAM"])
@pytest.mark.parametrize("path", ["mfma", "mfma32", "direct"])
def test_llr_near_zero_at_large_s(orc, shape, name, path):
    """At s max||x||^2 = 1.3e4 (inside the fp16 range of the split) the
    expanded distance form cancels terms of that size; LLRs near zero are
    recomputed on the per-class path, so exact and max-log LLRs meet the
    1e-3 max(|lambda|, 1) bar there too: 4x4 shape, 32 x 32 shape, direct."""
    shape(BIG if path == "mfma32" else -1)
    path = "mfma" if path == "mfma32" else path
    f = w.pam(6) if name == "64-PAM" else w.square_qam(4)
    gf = mdgmi.Format.of(f)
    max_n2 = float((f.X ** 2).sum(1).max())
    s = 1.3e4 / max_n2
    s2 = float(np.log2(np.e) / (2.0 * s))
    n = 20000
    # y spread over the constellation's extent: at this noise level channel
    # samples would hardly ever sit near a decision boundary
    lim = float(np.abs(f.X).max()) + 0.1
    y = np.random.default_rng(71).uniform(-lim, lim, size=(n, f.dim)).astype(np.float32).astype(np.float64)
    lam = mdgmi.mdgmi_llr(gf, dev(y), s2, path=path).cpu().numpy().astype(np.float64)
    ref = orc.llr(y, f.X, f.labels, s2)
    near = int(np.count_nonzero(np.abs(ref) < 2.0))    # 34 (16-QAM) to 4192 (64-PAM) of 1.2e5
    assert near > 20 and ratio(lam, ref) <= 1.0, (near, ratio(lam, ref))
    lml = mdgmi.mdgmi_llr_maxlog(gf, dev(y), s2, path=path).cpu().numpy().astype(np.float64)
    rml = orc.llr_maxlog(y, f.X, f.labels, s2)
    assert ratio(lml, rml) <= 1.0, ratio(lml, rml)
    say(f"[large s] {name} {path}: {near} LLRs below 2 nats, worst {ratio(lam, ref):.2f} / {ratio(lml, rml):.2f} of the bar")
