"""The paper's own modulation formats as GMI workloads, through the C ABI on
every path, against the FP64 oracle on the same samples: Gray PAM-2/4/8/16
on one real axis (a one-dimensional format: its own kernel instantiations,
MFMA image layout and generator case) and Gray square QAM-4/16/64.
* GMI/MI within 1e-4 bit (FP64 path 1e-10) and sample counts;
* exact and max-log LLRs within 1e-3 max(|lambda|, 1) nats (FP64 1e-9);
* hard-decision error counts within the decisions near their thresholds;
* the device generator against the host generator for a 1-D format;
* one-dimensional instances in a ragged batch (the per-sample 4x4 MFMA
  kind from M = 4, the direct kernel for M = 2) against per-instance calls
  that take the same kernels, and the autotuner on a 1-D format.
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

PATHS = ["f64", "direct", "mfma", "mfma_bf16"]
GMI_TOL = {"f64": 1e-10, "direct": 1e-4, "mfma": 1e-4, "mfma_bf16": 1e-4}
LLR_RTOL = {"f64": 1e-9, "direct": 1e-3, "mfma": 1e-3, "mfma_bf16": 1e-3}
FORMATS = {f.name: f for f in w.paper_formats()}
SNRS = {"2-PAM": [0.0, 6.0, 12.0], "4-PAM": [4.0, 12.0, 20.0], "8-PAM": [8.0, 18.0, 28.0],
        "16-PAM": [14.0, 24.0, 34.0], "4-QAM": [0.0, 6.0, 12.0], "16-QAM": [4.0, 12.0, 20.0],
        "64-QAM": [10.0, 18.0, 26.0]}


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


@pytest.mark.parametrize("name", list(FORMATS))
@pytest.mark.parametrize("path", PATHS)
def test_paper_format_parity(orc, name, path):
    f = FORMATS[name]
    gf = mdgmi.Format.of(f)
    s2s = w.sigma2_from_snr_db(np.array(SNRS[name]), f.dim)
    n = 4099
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=23, snr_slot=q, n=n) for q, v in enumerate(s2s)))
    y = np.stack(ys)
    tx = np.stack(txs)
    if path != "f64":
        y = y.astype(np.float32).astype(np.float64)
    out = mdgmi.mdgmi_gmi_hd(gf, dev(y, dt(path)), dev_u32(tx), s2s, path=path).cpu().numpy()
    ml = mdgmi.mdgmi_gmi_maxlog(gf, dev(y, dt(path)), dev_u32(tx), s2s, path=path).cpu().numpy()
    ref = orc.gmi_per_snr(y, tx, f.X, f.labels, s2s)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= GMI_TOL[path]
    for q, s2 in enumerate(s2s):
        s2 = float(s2)
        lam = mdgmi.mdgmi_llr(gf, dev(y[q], dt(path)), s2, path=path).cpu().numpy().astype(np.float64)
        lex = orc.llr(y[q], f.X, f.labels, s2)
        assert ratio(lam, lex, path) <= 1.0, q
        lml = mdgmi.mdgmi_llr_maxlog(gf, dev(y[q], dt(path)), s2, path=path).cpu().numpy().astype(np.float64)
        rml = orc.llr_maxlog(y[q], f.X, f.labels, s2)
        assert ratio(lml, rml, path) <= 1.0, q
        g_ml = orc.gmi_s(rml, f.labels[tx[q]], 1.0)[0]
        assert abs(ml[q, 0] - g_ml) <= GMI_TOL[path], q
        hd = orc.hd(y[q], tx[q], f.X, f.labels, s2)
        rel = 1e-9 if path == "f64" else 2e-3
        amb = int(np.count_nonzero(np.abs(lex) <= rel * np.maximum(np.abs(lex), 1.0)))
        assert abs(out[q, 6] - hd[0]) * n * f.m <= amb + 1e-6, q
        # nearest-point margins of the oracle for the symbol decisions
        d = ((y[q][:, None, :] - f.X[None]) ** 2).sum(-1)
        di = d[np.arange(n), tx[q]].copy()
        d[np.arange(n), tx[q]] = np.inf
        tol = 1e-9 if path == "f64" else 1e-5 * (1.0 + np.max(np.abs(y[q])) ** 2) / s2
        amb_s = int(np.count_nonzero(np.abs(d.min(axis=1) - di) / (2 * s2) <= tol))
        assert abs(out[q, 7] - hd[1]) * n <= amb_s + 1e-6, q
        say(f"[paper] {name} {path} SNR {SNRS[name][q]} dB: GMI {out[q, 0]:.5f} MI {out[q, 1]:.5f} "
            f"max-log GMI {ml[q, 0]:.5f} BER {out[q, 6]:.3e} SER {out[q, 7]:.3e}")


def test_generator_one_dimensional():
    f = FORMATS["8-PAM"]
    gf = mdgmi.Format.of(f)
    s2 = w.sigma2_from_snr_db(np.array([5.0, 15.0]), 1)
    n = 5003
    y32, tx = mdgmi.mdgmi_generate(gf, 7, s2, n, snr_slot0=2, dtype=torch.float32)
    y64, _ = mdgmi.mdgmi_generate(gf, 7, s2, n, snr_slot0=2, dtype=torch.float64)
    y32, tx, y64 = (t.cpu().numpy() for t in (y32, tx, y64))
    assert y32.shape == (2, n, 1)
    for q in range(2):
        yh, txh = w.channel_samples(f, float(s2[q]), seed=7, snr_slot=2 + q, n=n)
        np.testing.assert_array_equal(tx[q].view(np.uint32), txh)
        np.testing.assert_allclose(y64[q], yh, rtol=1e-14, atol=1e-15)
        d = np.abs(y32[q].astype(np.float64) - yh.astype(np.float32).astype(np.float64))
        assert np.all(d <= np.spacing(np.abs(yh.astype(np.float32))).astype(np.float64))


def test_one_dimensional_instances_in_a_batch():
    mdgmi.mdgmi_tune_clear()
    items, refs = [], []
    for k, name in enumerate(["2-PAM", "4-PAM", "16-PAM", "64-QAM"]):
        f = FORMATS[name]
        gf = mdgmi.Format.of(f)
        s2 = float(w.sigma2_from_snr_db(10.0 + 3 * k, f.dim))
        y, tx = w.channel_samples(f, s2, seed=k, snr_slot=k, n=3000 + 517 * k)
        yd = dev(y.astype(np.float32), torch.float32)
        td = dev_u32(tx)
        items.append((gf, yd, td, s2))
        refs.append(mdgmi.mdgmi_gmi(gf, yd[None], td[None], [s2], path="auto").cpu().numpy()[0])
    out = mdgmi.mdgmi_gmi_batched(mdgmi.instances(items), path="auto").cpu().numpy()
    ref = np.array(refs)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert np.max(np.abs(out[:, :2] - ref[:, :2])) <= 1e-9
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_batched(mdgmi.instances(items[:1]), path="mfma")
    assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED


def test_autotune_one_dimensional():
    e = mdgmi.mdgmi_autotune(1, 16, force=True)
    assert e["dim"] == 1 and e["M"] == 16
    assert e["path"] in (mdgmi.MDGMI_PATH_F32_DIRECT, mdgmi.MDGMI_PATH_F32_MFMA_F16SPLIT)
    f = FORMATS["16-PAM"]
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(20.0, 1))
    y, tx = w.channel_samples(f, s2, seed=1, snr_slot=0, n=2000)
    out = mdgmi.mdgmi_gmi(gf, dev(y[None].astype(np.float32), torch.float32), dev_u32(tx[None]), [s2],
                          path="auto").cpu().numpy()
    yy = y.astype(np.float32).astype(np.float64)
    ref = mdgmi.mdgmi_gmi(gf, dev(yy[None], torch.float64), dev_u32(tx[None]), [s2], path="f64").cpu().numpy()
    assert abs(out[0, 0] - ref[0, 0]) <= 1e-4
    mdgmi.mdgmi_tune_clear()
