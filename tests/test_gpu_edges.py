"""Edge and degenerate cases of the exact paths through the C ABI, against
the FP64 oracle where there is something to compare:
* empty inputs (n = 0, no SNR points) are rejected before any launch;
* one-bit formats (M = 2) in 2, 4 and 8 dimensions;
* coincident points carrying different labels (class sums tie);
* SNRs far below and far above the working range (GMI -> 0 and -> m);
* the 16-QAM workload at its full size (11 SNR points x 1e5 samples) on
  every path, all samples against the oracle.
"""
import ctypes
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
LLR_RTOL = 1e-3
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


def llr_ratio(lam, ref):
    return float(np.max(np.abs(lam - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))))


def test_empty_inputs_are_rejected():
    f = w.format_16qam()
    gf = mdgmi.Format.of(f)
    L = mdgmi.lib()
    y = torch.zeros((1, 4, 2), dtype=torch.float32, device="cuda")
    tx = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    out = torch.zeros((1, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    ws = mdgmi.workspace(1 << 20)
    s2 = np.array([0.1])
    P = ctypes.c_void_p
    sp = s2.ctypes.data_as(P)
    stream = P(torch.cuda.current_stream().cuda_stream)
    say("[edge] empty inputs")
    for n, n_snr in ((0, 1), (4, 0)):
        rc = L.mdgmi_gmi(gf.handle, P(y.data_ptr()), P(tx.data_ptr()), n, sp, n_snr, mdgmi.MDGMI_PATH_AUTO,
                         P(out.data_ptr()), P(ws.data_ptr()), ws.numel(), stream)
        assert rc == mdgmi.MDGMI_E_SHAPE
        rc = L.mdgmi_generate(gf.handle, 1, sp, n_snr, n, 0, P(y.data_ptr()), P(tx.data_ptr()), 0, stream)
        assert rc == mdgmi.MDGMI_E_SHAPE
    rc = L.mdgmi_llr(gf.handle, P(y.data_ptr()), 0, 0.1, P(out.data_ptr()), mdgmi.MDGMI_PATH_AUTO,
                     P(ws.data_ptr()), ws.numel(), stream)
    assert rc == mdgmi.MDGMI_E_SHAPE
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_batched(mdgmi.instances([]), path="auto")
    assert e.value.code == mdgmi.MDGMI_E_SHAPE
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0)        # nothing was launched


@pytest.mark.parametrize("dim", [2, 4, 8])
@pytest.mark.parametrize("path", PATHS)
def test_one_bit_formats(orc, dim, path):
    f = w.random_shells(dim, 2, 40 + dim)
    gf = mdgmi.Format.of(f)
    snrs = [-6.0, 3.0, 15.0]
    s2 = w.sigma2_from_snr_db(np.array(snrs), dim)
    n = 2053
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=dim, snr_slot=q, n=n) for q, v in enumerate(s2)))
    y = np.stack(ys)
    tx = np.stack(txs)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    say(f"[edge] M=2 dim={dim} path={path}")
    out = mdgmi.mdgmi_gmi(gf, dev(y, dt(path)), dev_u32(tx), s2, path=path).cpu().numpy()
    ref = orc.gmi_per_snr(y, tx, f.X, f.labels, s2)
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL[path]
    lam = mdgmi.mdgmi_llr(gf, dev(y[1], dt(path)), float(s2[1]), path=path).cpu().numpy().astype(np.float64)
    assert llr_ratio(lam, orc.llr(y[1], f.X, f.labels, float(s2[1]))) <= (1e-6 if path == "f64" else 1.0)
    # one bit: the GMI and the MI of a binary input are the same quantity
    np.testing.assert_allclose(out[:, 0], out[:, 1], rtol=0, atol=1e-6)


@pytest.mark.parametrize("path", PATHS)
def test_coincident_points(orc, path):
    """Two labels on the same point: their class sums tie exactly."""
    f = w.random_shells(4, 16, 77)
    X = f.X.copy()
    X[5] = X[9]
    g = w.Format("dup4d-16", X, f.labels.copy())
    gf = mdgmi.Format.of(g)
    s2 = float(w.sigma2_from_snr_db(12.0, 4))
    y, tx = w.channel_samples(g, s2, seed=5, snr_slot=0, n=3001)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    say(f"[edge] coincident points path={path}")
    lam = mdgmi.mdgmi_llr(gf, dev(y, dt(path)), s2, path=path).cpu().numpy().astype(np.float64)
    assert llr_ratio(lam, orc.llr(y, g.X, g.labels, s2)) <= (1e-6 if path == "f64" else 1.0)
    out = mdgmi.mdgmi_gmi(gf, dev(y[None], dt(path)), dev_u32(tx[None]), [s2], path=path).cpu().numpy()
    ref = orc.gmi(y, tx, g.X, g.labels, s2)
    assert np.max(np.abs(out[0, :2] - ref[:2])) <= GMI_TOL[path]


@pytest.mark.parametrize("path", PATHS)
def test_extreme_snrs(orc, path):
    """-30 dB: GMI and MI near 0; +30 dB: m within rounding (the top of the
    fp16 split's range for this format). Both against the oracle on the
    same samples."""
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    snrs = np.array([-30.0, 30.0])
    s2 = w.sigma2_from_snr_db(snrs, f.dim)
    n = 4099
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=8, snr_slot=q, n=n) for q, v in enumerate(s2)))
    y = np.stack(ys)
    tx = np.stack(txs)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    say(f"[edge] extreme SNRs path={path}")
    out = mdgmi.mdgmi_gmi(gf, dev(y, dt(path)), dev_u32(tx), s2, path=path).cpu().numpy()
    ref = orc.gmi_per_snr(y, tx, f.X, f.labels, s2)
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL[path]
    assert abs(out[0, 1]) < 0.05 and abs(out[1, 0] - f.m) < 1e-6 and abs(out[1, 1] - f.m) < 1e-6


@pytest.mark.parametrize("path", PATHS)
def test_qam16_workload_full_size(orc, path):
    """The 16-QAM workload (11 SNR points x 1e5 seeded samples, generated on
    the device) with every sample checked by the oracle."""
    wl = w.workload_qam16()
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    say(f"[edge] 16-QAM full size path={path}")
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, wl.sigma2, wl.n, dtype=dt(path))
    out = mdgmi.mdgmi_gmi(gf, y, tx, wl.sigma2, path=path).cpu().numpy()
    yh = y.cpu().numpy().astype(np.float64)
    th = tx.cpu().numpy().view(np.uint32)
    ref = orc.gmi_per_snr(yh, th, f.X, f.labels, wl.sigma2)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL[path]
    q = 5
    lam = mdgmi.mdgmi_llr(gf, y[q], float(wl.sigma2[q]), path=path).cpu().numpy().astype(np.float64)
    assert llr_ratio(lam, orc.llr(yh[q], f.X, f.labels, float(wl.sigma2[q]))) <= (1e-6 if path == "f64" else 1.0)


def test_bf16_split_beyond_the_fp16_range(orc):
    """At SNRs where the fp16 split's factors overflow (the path reports
    MDGMI_E_UNSUPPORTED), the bf16 three-part split still runs the distance
    term on the matrix cores and matches the oracle."""
    for f, snr in ((w.format_4d64(), 48.0), (w.format_16qam(), 50.0), (w.pam(4), 55.0)):
        gf = mdgmi.Format.of(f)
        s2 = float(w.sigma2_from_snr_db(snr, f.dim))
        y, tx = w.channel_samples(f, s2, seed=12, snr_slot=0, n=3001)
        y = y.astype(np.float32).astype(np.float64)
        say(f"[edge] bf16 split {f.name} at {snr} dB")
        with pytest.raises(mdgmi.MdgmiError) as e:
            mdgmi.mdgmi_gmi(gf, dev(y[None], torch.float32), dev_u32(tx[None]), [s2], path="mfma")
        assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED
        out = mdgmi.mdgmi_gmi(gf, dev(y[None], torch.float32), dev_u32(tx[None]), [s2],
                              path="mfma_bf16").cpu().numpy()
        ref = orc.gmi(y, tx, f.X, f.labels, s2)
        assert np.max(np.abs(out[0, :2] - ref[:2])) <= 1e-4
        lam = mdgmi.mdgmi_llr(gf, dev(y, torch.float32), s2, path="mfma_bf16").cpu().numpy().astype(np.float64)
        assert llr_ratio(lam, orc.llr(y, f.X, f.labels, s2)) <= 1.0


def test_auto_takes_the_bf16_split_beyond_the_fp16_range(orc):
    """AUTO on a large format at an SNR outside the fp16 split's range runs
    the bf16 split (bit-identical to asking for it) rather than the slower
    direct path; within range it keeps the fp16 split."""
    f = w.random_shells(8, 256, 19)
    gf = mdgmi.Format.of(f)
    mdgmi.mdgmi_tune_clear()
    for snr, expect in ((45.0, "mfma_bf16"), (10.0, "mfma")):
        s2 = float(w.sigma2_from_snr_db(snr, 8))
        y, tx = w.channel_samples(f, s2, seed=4, snr_slot=0, n=2500)
        yd, td = dev(y[None], torch.float32), dev_u32(tx[None])
        auto = mdgmi.mdgmi_gmi(gf, yd, td, [s2], path="auto").cpu().numpy()
        same = mdgmi.mdgmi_gmi(gf, yd, td, [s2], path=expect).cpu().numpy()
        np.testing.assert_array_equal(auto, same)
        ref = orc.gmi(y.astype(np.float32).astype(np.float64), tx, f.X, f.labels, s2)
        assert np.max(np.abs(auto[0, :2] - ref[:2])) <= 1e-4
        say(f"[edge] AUTO at {snr} dB -> {expect}: GMI {auto[0, 0]:.6f}")


def test_peak_probe_rates_are_plausible():
    """mdgmi_probe_rates: the exponential, FMA and bf16 MFMA rates it measures
    on this device are positive and ordered as the hardware is built (a plain
    FMA issues at least as fast as v_exp_f32) and no larger than the chip's
    nominal figures allow (256 CUs at 2.4 GHz with some clock margin)."""
    r = mdgmi.mdgmi_probe_rates()
    say(f"[probe] {r}")
    assert 1e12 < r["exp_per_s"] <= 1.1 * 256 * 32 * 2.4e9
    assert r["exp_per_s"] <= r["fma_lane_ops_per_s"] <= 1.1 * 256 * 64 * 2.4e9
    assert 1e14 < r["mfma_bf16_flops_per_s"] <= 1.1 * 2.5e15
    # vector instructions beside the MFMAs can only slow the matrix core down
    assert 1e14 < r["mfma_with_8_fma_flops_per_s"] <= 1.05 * r["mfma_with_4_fma_flops_per_s"]
    assert r["mfma_with_4_fma_flops_per_s"] <= 1.05 * r["mfma_2waves_flops_per_s"] <= 1.1 * 2.5e15
    # MFMA and FMA waves side by side: an iteration (2 MFMAs of one wave, 16 FMAs of
    # the other) takes at least as long as the longer of its two parts alone
    simd = torch.cuda.get_device_properties(0).multi_processor_count * 4
    t_mfma = 2 * 32768 / (r["mfma_2waves_flops_per_s"] / simd)
    t_fma = 16 * 64 / (r["fma_lane_ops_per_s"] / simd)
    t_split = 1.0 / r["split_waves_iters_per_s"]
    say(f"[probe] split waves: {t_split * 1e9:.1f} ns per iteration; MFMA part {t_mfma * 1e9:.1f}, FMA part {t_fma * 1e9:.1f}")
    assert 0.95 * max(t_mfma, t_fma) <= t_split <= 1.5 * (t_mfma + t_fma)
