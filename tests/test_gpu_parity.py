"""GPU parity: the HIP paths through the C ABI against the FP64 oracle on the
very same seeded inputs (generated on the host by workloads, copied over).

Bars (stated in the tests):
* LLRs, FP32 paths: |d lambda| <= 1e-3 * max(|lambda_oracle|, 1) nats;
  FP64 path: <= 1e-9 * max(|lambda|, 1).
* GMI / MI: |d| <= 1e-4 bit/symbol on FP32 paths, <= 1e-10 on the FP64 path.
* Counts (N, non-finite) exact; repeated calls bit-identical.
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

F32_PATHS = ["direct", "mfma", "mfma_bf16"]
LLR_RTOL = 1e-3
GMI_TOL32 = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def llr_bar(lam_gpu, lam_ref, rtol):
    err = np.abs(lam_gpu - lam_ref)
    bar = rtol * np.maximum(np.abs(lam_ref), 1.0)
    return float(np.max(err / bar)), float(np.max(err))


FORMATS = {
    "16qam": lambda: w.format_16qam(),
    "4d64": lambda: w.format_4d64(),
    "8d2048": lambda: w.format_8d2048(),
    "qpsk": lambda: w.square_qam(2),
    "bpsk2d": lambda: w.Format("bpsk2d", np.array([[-1.0, 0.0], [1.0, 0.0]]), np.array([1, 0], np.uint32)),
    "8psk": lambda: w.psk(3),
    "sh2d-32": lambda: w.random_shells(2, 32, 11),
    "sh4d-128": lambda: w.random_shells(4, 128, 12),
    "sh8d-16": lambda: w.random_shells(8, 16, 13),
    "sh8d-512": lambda: w.random_shells(8, 512, 14),
    "sh2d-4096": lambda: w.random_shells(2, 4096, 15),
    "sh8d-4096": lambda: w.random_shells(8, 4096, 16),
    "sh4d-4096": lambda: w.random_shells(4, 4096, 17),
    "qp8d-256": lambda: w.qam_product(8, 8),
    "qp4d-32": lambda: w.qam_product(4, 5),
}

_fmt_cache = {}


def gfmt(name):
    if name not in _fmt_cache:
        f = FORMATS[name]()
        _fmt_cache[name] = (f, mdgmi.Format.of(f))
    return _fmt_cache[name]


def n_for(f, base=1037):
    # keep the oracle to about a second: n * M * m pairs
    return int(max(97, min(base, 3e6 // (f.M * max(f.m, 1)))))


LLR_CASES = [
    ("16qam", 0.0), ("16qam", 12.0), ("16qam", 24.0),
    ("4d64", -2.0), ("4d64", 8.0), ("4d64", 18.0),
    ("8d2048", 2.0), ("8d2048", 17.0),
    ("qpsk", 5.0), ("bpsk2d", 3.0), ("8psk", 14.0),
    ("sh2d-32", 10.0), ("sh4d-128", 20.0), ("sh8d-16", 6.0), ("sh8d-512", 12.0),
    ("sh2d-4096", 25.0), ("sh8d-4096", 9.0), ("sh4d-4096", 14.0), ("qp8d-256", 15.0), ("qp4d-32", 22.0),
]


@pytest.mark.parametrize("name,snr_db", LLR_CASES)
@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_llr_parity(orc, name, snr_db, path):
    f, gf = gfmt(name)
    s2 = float(w.sigma2_from_snr_db(snr_db, f.dim))
    n = n_for(f)
    y, _ = w.channel_samples(f, s2, seed=101, snr_slot=0, n=n)
    say(f"[llr] {name} {snr_db} dB path={path} n={n}")
    if path == "f64":
        lam = mdgmi.mdgmi_llr(gf, dev(y, torch.float64), s2, path=path).cpu().numpy()
        ref = orc.llr(y, f.X, f.labels, s2)
        ratio, _ = llr_bar(lam, ref, 1e-9)
    else:
        y32 = y.astype(np.float32)
        lam = mdgmi.mdgmi_llr(gf, dev(y32, torch.float32), s2, path=path).cpu().numpy().astype(np.float64)
        ref = orc.llr(y32.astype(np.float64), f.X, f.labels, s2)
        ratio, _ = llr_bar(lam, ref, LLR_RTOL)
    assert lam.shape == ref.shape
    assert np.all(np.isfinite(lam))
    assert ratio <= 1.0, f"max |dlambda| / bar = {ratio}"


GMI_CASES = [
    ("16qam", [0.0, 6.0, 14.0, 20.0]),
    ("4d64", [-2.0, 4.0, 10.0, 18.0]),
    ("8d2048", [2.0, 9.0, 17.0]),
    ("bpsk2d", [0.0, 10.0]),
    ("sh2d-32", [3.0, 25.0]),
    ("sh4d-128", [-5.0, 15.0]),
    ("sh8d-16", [0.0, 20.0]),
    ("sh2d-4096", [10.0, 25.0]),
    ("sh8d-4096", [5.0]),
    ("qp8d-256", [8.0, 16.0]),
]


def gmi_inputs(f, snrs, n, seed=202):
    ys, txs = [], []
    s2 = w.sigma2_from_snr_db(np.array(snrs), f.dim)
    for q, v in enumerate(s2):
        y, tx = w.channel_samples(f, float(v), seed=seed, snr_slot=q, n=n)
        ys.append(y)
        txs.append(tx)
    return np.stack(ys), np.stack(txs), s2


@pytest.mark.parametrize("name,snrs", GMI_CASES)
@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_gmi_parity(orc, name, snrs, path):
    f, gf = gfmt(name)
    n = n_for(f, base=4099)
    y, tx, s2 = gmi_inputs(f, snrs, n)
    say(f"[gmi] {name} {snrs} path={path} n={n}")
    if path == "f64":
        out = mdgmi.mdgmi_gmi(gf, dev(y, torch.float64), dev_u32(tx), s2, path=path).cpu().numpy()
        yref, tol = y, 1e-10
    else:
        y32 = y.astype(np.float32)
        out = mdgmi.mdgmi_gmi(gf, dev(y32, torch.float32), dev_u32(tx), s2, path=path).cpu().numpy()
        yref, tol = y32.astype(np.float64), GMI_TOL32
    ref = orc.gmi_per_snr(yref, tx, f.X, f.labels, s2)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    np.testing.assert_array_equal(out[:, 5], ref[:, 5])
    assert np.max(np.abs(out[:, 0] - ref[:, 0])) <= tol, (out[:, 0], ref[:, 0])
    assert np.max(np.abs(out[:, 1] - ref[:, 1])) <= tol, (out[:, 1], ref[:, 1])
    np.testing.assert_allclose(out[:, 2:4], ref[:, 2:4], rtol=1e-3, atol=1e-6)


def test_many_snrs_in_one_call(orc):
    """More SNR points than one launch carries (launches are chunked)."""
    f, gf = gfmt("qpsk")
    snrs = np.linspace(-5, 25, 41)
    y, tx, s2 = gmi_inputs(f, snrs, 300, seed=7)
    say("[gmi] qpsk 41 SNRs")
    for path in F32_PATHS:
        out = mdgmi.mdgmi_gmi(gf, dev(y.astype(np.float32), torch.float32), dev_u32(tx), s2, path=path).cpu().numpy()
        ref = orc.gmi_per_snr(y.astype(np.float32).astype(np.float64), tx, f.X, f.labels, s2)
        assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL32
        # with the sent point's u taken from the matrix cores themselves the MI
        # of the split path is as close as the direct path's
        assert np.max(np.abs(out[:, 1] - ref[:, 1])) <= 1e-5


@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_single_sample_and_ragged_tails(orc, path):
    f, gf = gfmt("sh8d-512")
    for n in (1, 31, 33, 257):
        y, tx, s2 = gmi_inputs(f, [7.0], n, seed=n)
        say(f"[gmi] ragged n={n} path={path}")
        dt = torch.float64 if path == "f64" else torch.float32
        yy = y if path == "f64" else y.astype(np.float32)
        out = mdgmi.mdgmi_gmi(gf, dev(yy, dt), dev_u32(tx), s2, path=path).cpu().numpy()
        ref = orc.gmi_per_snr(yy.astype(np.float64), tx, f.X, f.labels, s2)
        assert out[0, 4] == n
        assert abs(out[0, 0] - ref[0, 0]) <= GMI_TOL32 and abs(out[0, 1] - ref[0, 1]) <= GMI_TOL32
        if n == 1:
            assert out[0, 2] == 0.0 and out[0, 3] == 0.0


@pytest.mark.parametrize("path", F32_PATHS)
def test_far_samples_take_the_exact_per_class_path(orc, path):
    """Samples far from every point (outside the common exponent window) are
    still exact: LLRs and costs match the oracle."""
    f, gf = gfmt("16qam")
    s2 = float(w.sigma2_from_snr_db(20, 2))
    rng = np.random.default_rng(3)
    y = (rng.normal(size=(200, 2)) * 3.0).astype(np.float32)     # many far from the grid
    tx = rng.integers(0, 16, size=200).astype(np.uint32)
    say(f"[far] path={path}")
    lam = mdgmi.mdgmi_llr(gf, dev(y, torch.float32), s2, path=path).cpu().numpy().astype(np.float64)
    ref = orc.llr(y.astype(np.float64), f.X, f.labels, s2)
    ratio, _ = llr_bar(lam, ref, LLR_RTOL)
    assert ratio <= 1.0 and np.abs(ref).max() > 200
    out = mdgmi.mdgmi_gmi(gf, dev(y[None], torch.float32), dev_u32(tx[None]), [s2], path=path).cpu().numpy()
    r = orc.gmi(y.astype(np.float64), tx, f.X, f.labels, s2)
    # per-sample costs reach thousands of bits here: compare relative to their size
    assert abs(out[0, 0] - r[0]) <= 1e-4 * max(1.0, abs(r[0]))
    assert abs(out[0, 1] - r[1]) <= 1e-4 * max(1.0, abs(r[1]))


@pytest.mark.parametrize("path", F32_PATHS)
def test_far_class_windows(orc, path):
    """LLRs of samples whose farthest class lies inside the common exponent
    window, in the window of the raised offset (the second pass of the MFMA
    path) and beyond both (exact per-class path), all against the oracle.
    The regimes are counted on the host from the class distances."""
    f, gf = gfmt("16qam")
    s2 = float(w.sigma2_from_snr_db(20, 2))
    s = 1.0 / (math.log(2.0) * 2.0 * s2)
    rng = np.random.default_rng(11)
    r = rng.uniform(0.3, 2.0, size=3000)
    th = rng.uniform(0.0, 2.0 * np.pi, size=3000)
    y = np.stack([r * np.cos(th), r * np.sin(th)], axis=1).astype(np.float32)
    d = s * ((y.astype(np.float64)[:, None, :] - f.X[None]) ** 2).sum(-1)   # s |y - x|^2, log2 units
    far = np.zeros(len(y))           # distance of the farthest class (its nearest point)
    for k in range(f.m):
        b = (f.labels >> k) & 1
        far = np.maximum(far, np.maximum(d[:, b == 0].min(1), d[:, b == 1].min(1)))
    assert (far < 180).sum() > 100 and ((far > 220) & (far < 280)).sum() > 100 and (far > 320).sum() > 100
    say(f"[far windows] path={path}")
    lam = mdgmi.mdgmi_llr(gf, dev(y, torch.float32), s2, path=path).cpu().numpy().astype(np.float64)
    ref = orc.llr(y.astype(np.float64), f.X, f.labels, s2)
    ratio, _ = llr_bar(lam, ref, LLR_RTOL)
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_nonfinite_input_is_flagged(orc, path):
    f, gf = gfmt("4d64")
    y, tx, s2 = gmi_inputs(f, [5.0, 6.0], 500)
    y[1, 123, 2] = np.nan
    dt = torch.float64 if path == "f64" else torch.float32
    yy = y if path == "f64" else y.astype(np.float32)
    say(f"[nan] path={path}")
    out = mdgmi.mdgmi_gmi(gf, dev(yy, dt), dev_u32(tx), s2, path=path).cpu().numpy()
    assert out[0, 5] == 0 and np.isfinite(out[0, 0])
    assert out[1, 5] == 1 and np.isnan(out[1, 0]) and np.isnan(out[1, 1])


@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_bit_reproducible(path):
    f, gf = gfmt("8d2048")
    y, tx, s2 = gmi_inputs(f, [4.0, 12.0], 3000)
    dt = torch.float64 if path == "f64" else torch.float32
    yd, txd = dev(y, dt), dev_u32(tx)
    say(f"[repro] path={path}")
    a = mdgmi.mdgmi_gmi(gf, yd, txd, s2, path=path).cpu().numpy()
    b = mdgmi.mdgmi_gmi(gf, yd, txd, s2, path=path).cpu().numpy()
    assert a.tobytes() == b.tobytes()


def test_generator_matches_host_generator():
    for name in ("16qam", "4d64", "8d2048"):
        f, gf = gfmt(name)
        snrs = [0.0, 10.0]
        s2 = w.sigma2_from_snr_db(np.array(snrs), f.dim)
        n = 5003
        say(f"[gen] {name}")
        y32, tx = mdgmi.mdgmi_generate(gf, 99, s2, n, snr_slot0=3, dtype=torch.float32)
        y64, tx64 = mdgmi.mdgmi_generate(gf, 99, s2, n, snr_slot0=3, dtype=torch.float64)
        y32, tx, y64, tx64 = (t.cpu().numpy() for t in (y32, tx, y64, tx64))
        for q in range(2):
            yh, txh = w.channel_samples(f, float(s2[q]), seed=99, snr_slot=3 + q, n=n)
            np.testing.assert_array_equal(tx[q].view(np.uint32), txh)
            np.testing.assert_array_equal(tx64[q].view(np.uint32), txh)
            # device and host libm may differ in the last bit of log/cos/sin
            np.testing.assert_allclose(y64[q], yh, rtol=1e-14, atol=1e-15)
            d = np.abs(y32[q].astype(np.float64) - yh.astype(np.float32).astype(np.float64))
            ulp = np.spacing(np.abs(yh.astype(np.float32))).astype(np.float64)
            assert np.all(d <= ulp)
            assert np.mean(d == 0) > 0.999


def test_error_codes_before_launch():
    f, gf = gfmt("16qam")
    y = torch.zeros((1, 10, 2), dtype=torch.float32, device="cuda")
    tx = torch.zeros((1, 10), dtype=torch.int32, device="cuda")
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi(gf, y, tx, [0.0], path="direct")
    assert e.value.code == mdgmi.MDGMI_E_SIGMA2
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi(gf, y, tx, [float("nan")], path="direct")
    assert e.value.code == mdgmi.MDGMI_E_SIGMA2
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi(gf, y, tx, [0.1], path="direct", ws=mdgmi.workspace(8))
    assert e.value.code == mdgmi.MDGMI_E_WORKSPACE
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi(gf, y, tx, [1e-9], path="mfma")     # s far outside the fp16 split range
    assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi(gf, y, tx, [0.1], path=7)
    assert e.value.code == mdgmi.MDGMI_E_ARG
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.Format(np.zeros((4, 2)), [0, 1, 2, 2])
    assert e.value.code == mdgmi.MDGMI_E_LABELS


@pytest.mark.parametrize("path", ["f64"] + F32_PATHS)
def test_sent_row_out_of_range_gives_nan(path):
    f, gf = gfmt("16qam")
    y, tx, s2 = gmi_inputs(f, [5.0], 100)
    tx[0, 17] = 16
    dt = torch.float64 if path == "f64" else torch.float32
    say(f"[badrow] path={path}")
    out = mdgmi.mdgmi_gmi(gf, dev(y, dt), dev_u32(tx), s2, path=path).cpu().numpy()
    assert out[0, 5] == 1 and np.isnan(out[0, 0])
