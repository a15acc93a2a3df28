"""Parity at the full size of the 8-D workload (M = 2048 two-shell format,
16 SNR points x 1e7 samples, generated on the device), in the launch
configuration the benchmark times, and of the 4-D workload (M = 64
two-ring product, 21 SNR points x 1e7 samples) on its default path.

The oracle cannot evaluate 3.3e11 pairs, so the full-size results are tied
to it through outputs it can compute one by one and through properties that
hold at any size:
* LLR mode over all 1e7 samples of every SNR point; 384 seeded random rows
  per point against the FP64 oracle on the very same (device) inputs, bar
  |d lambda| <= 1e-3 * max(|lambda|, 1) nats;
* the GMI-mode result of the timed launch equals m - mean of the bit costs
  formed from those full LLR arrays (same samples), within 1e-4 bit;
* additivity of the reduction: the full-size sums equal the sample-weighted
  sums of two halves run separately (1e-9 relative);
* the full-size MI agrees with the oracle's MI of the sampled rows within
  Monte-Carlo error, and MI >= GMI within 3 standard errors;
* max-log metrics and the s-optimised GMI in the same way (sampled rows,
  the launch's GMI against the full LLR arrays, s* against the oracle's
  GMI(s) on the sample).
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

LLR_RTOL = 1e-3
GMI_TOL32 = 1e-4
ROWS = 384


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    wl = w.workload_8d2048()
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    say(f"[full] generating {len(wl.snr_db)} x {wl.n} samples of {f.name}")
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, wl.sigma2, wl.n, dtype=torch.float32)
    out = mdgmi.mdgmi_gmi(gf, y, tx, wl.sigma2, path="mfma").cpu().numpy()
    torch.cuda.synchronize()
    return wl, f, gf, y, tx, out


def test_counts_and_finiteness(full):
    wl, f, gf, y, tx, out = full
    assert np.all(out[:, 4] == wl.n) and np.all(out[:, 5] == 0)
    assert np.all(np.isfinite(out[:, :4]))


def test_sampled_llrs_and_gmi_formula_at_full_size(full, orc):
    wl, f, gf, y, tx, out = full
    rng = np.random.default_rng(2048)
    ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, "mfma"))
    lab = torch.from_numpy(f.labels.astype(np.int64)).cuda()
    bits = torch.arange(f.m, device="cuda", dtype=torch.int64)
    worst = 0.0
    for q, s2 in enumerate(wl.sigma2):
        say(f"[full] SNR {wl.snr_db[q]} dB: LLRs of {wl.n} samples")
        lam = mdgmi.mdgmi_llr(gf, y[q], float(s2), path="mfma", ws=ws)
        rows = np.sort(rng.choice(wl.n, size=ROWS, replace=False))
        ri = torch.from_numpy(rows).cuda()
        yr = y[q].index_select(0, ri).cpu().numpy().astype(np.float64)
        ref = orc.llr(yr, f.X, f.labels, float(s2))
        got = lam.index_select(0, ri).cpu().numpy().astype(np.float64)
        ratio = float(np.max(np.abs(got - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))))
        worst = max(worst, ratio)
        assert ratio <= 1.0, (q, ratio)
        # GMI of the timed launch vs the bit costs of the full LLR arrays
        b = ((lab[tx[q].long()].unsqueeze(1) >> bits) & 1).double()
        u = -(2.0 * b - 1.0) * lam.double()
        cg = (torch.clamp(u, min=0.0) + torch.log1p(torch.exp(-u.abs()))).sum(dim=1) / math.log(2.0)
        gmi = f.m - float(cg.mean())
        assert abs(gmi - out[q, 0]) <= GMI_TOL32, (q, gmi, out[q, 0])
        del lam, b, u, cg
    say(f"[full] worst sampled LLR error / bar = {worst:.3f}")


def test_reduction_is_additive_over_halves(full):
    wl, f, gf, y, tx, out = full
    h = wl.n // 2
    parts = []
    for sl in (slice(0, h), slice(h, wl.n)):
        ys = y[:, sl].contiguous()
        ts = tx[:, sl].contiguous()
        parts.append(mdgmi.mdgmi_gmi(gf, ys, ts, wl.sigma2, path="mfma").cpu().numpy())
        del ys, ts
    n1, n2 = h, wl.n - h
    for col in (0, 1):
        comb = (n1 * parts[0][:, col] + n2 * parts[1][:, col]) / wl.n
        np.testing.assert_allclose(comb, out[:, col], rtol=1e-9, atol=1e-9)


def test_mi_against_sampled_oracle(full, orc):
    wl, f, gf, y, tx, out = full
    rng = np.random.default_rng(4096)
    for q in (0, 7, 15):
        s2 = float(wl.sigma2[q])
        rows = np.sort(rng.choice(wl.n, size=2000, replace=False))
        ri = torch.from_numpy(rows).cuda()
        yr = y[q].index_select(0, ri).cpu().numpy().astype(np.float64)
        tr = tx[q].index_select(0, ri).cpu().numpy().view(np.uint32)
        r = orc.gmi(yr, tr, f.X, f.labels, s2)
        say(f"[full] q={q}: MI full {out[q, 1]:.5f} vs sample {r[1]:.5f} +- {r[3]:.5f}")
        assert abs(out[q, 1] - r[1]) <= 5.0 * r[3] + 1e-6
        assert abs(out[q, 0] - r[0]) <= 5.0 * r[2] + 1e-6
        assert out[q, 1] >= out[q, 0] - 3.0 * math.hypot(out[q, 2], out[q, 3])


def test_maxlog_and_sopt_at_full_size(full, orc):
    """Max-log metrics on the full 8-D workload in the launch the benchmark
    times: sampled max-log LLR rows against the oracle, the GMI of the one
    mdgmi_gmi_maxlog launch against the bit costs of the full max-log LLR
    arrays, and per SNR point the s-optimised GMI of those arrays: its GMI at
    s = 1 equals the launch's GMI, GMI(s*) >= GMI(1), and s* maximises the
    oracle's GMI(s) on a sample within Monte-Carlo error."""
    wl, f, gf, y, tx, out = full
    ml = mdgmi.mdgmi_gmi_maxlog(gf, y, tx, wl.sigma2, path="mfma").cpu().numpy()
    assert np.all(ml[:, 4] == wl.n) and np.all(ml[:, 5] == 0)
    rng = np.random.default_rng(77)
    ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, "mfma"))
    lab = torch.from_numpy(f.labels.astype(np.int64)).cuda()
    bits = torch.arange(f.m, device="cuda", dtype=torch.int64)
    for q in range(0, len(wl.sigma2), 3):
        s2 = float(wl.sigma2[q])
        lam = mdgmi.mdgmi_llr_maxlog(gf, y[q], s2, path="mfma", ws=ws)
        rows = np.sort(rng.choice(wl.n, size=ROWS, replace=False))
        ri = torch.from_numpy(rows).cuda()
        yr = y[q].index_select(0, ri).cpu().numpy().astype(np.float64)
        ref = orc.llr_maxlog(yr, f.X, f.labels, s2)
        got = lam.index_select(0, ri).cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))) <= 1.0, q
        b = ((lab[tx[q].long()].unsqueeze(1) >> bits) & 1).double()
        u = -(2.0 * b - 1.0) * lam.double()
        cg = (torch.clamp(u, min=0.0) + torch.log1p(torch.exp(-u.abs()))).sum(dim=1) / math.log(2.0)
        assert abs(f.m - float(cg.mean()) - ml[q, 0]) <= GMI_TOL32, q
        so = mdgmi.mdgmi_gmi_sopt(gf, lam, tx[q]).cpu().numpy()
        assert abs(so[0] - ml[q, 0]) <= 1e-5 and so[3] >= so[0] - 1e-9 and so[8] <= 8
        tr = tx[q].index_select(0, ri).cpu().numpy().view(np.uint32)
        g_at = orc.gmi_s(got, f.labels[tr], so[2])
        s_o, g_o, se_o = orc.gmi_sopt(got, f.labels[tr])
        assert g_o - g_at[0] <= 3.0 * se_o + 1e-9
        say(f"[full] max-log q={q}: GMI {ml[q, 0]:.5f} (exact {out[q, 0]:.5f}), s* {so[2]:.4f}, "
            f"GMI(s*) {so[3]:.5f}")
        del lam, b, u, cg


def test_bf16_split_at_full_size(full, orc):
    """The bf16 three-part split on the full 8-D workload: sampled LLR rows
    against the oracle, and its one-launch GMI/MI against the fp16 split's
    (both within 1e-4 of the same exact values, so within 2e-4 of each other)
    and against the bit costs of its own full LLR arrays."""
    wl, f, gf, y, tx, out = full
    ob = mdgmi.mdgmi_gmi(gf, y, tx, wl.sigma2, path="mfma_bf16").cpu().numpy()
    assert np.all(ob[:, 4] == wl.n) and np.all(ob[:, 5] == 0)
    assert np.max(np.abs(ob[:, :2] - out[:, :2])) <= 2e-4
    rng = np.random.default_rng(1616)
    ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, "mfma_bf16"))
    lab = torch.from_numpy(f.labels.astype(np.int64)).cuda()
    bits = torch.arange(f.m, device="cuda", dtype=torch.int64)
    for q in (0, 8, 15):
        s2 = float(wl.sigma2[q])
        lam = mdgmi.mdgmi_llr(gf, y[q], s2, path="mfma_bf16", ws=ws)
        rows = np.sort(rng.choice(wl.n, size=ROWS, replace=False))
        ri = torch.from_numpy(rows).cuda()
        yr = y[q].index_select(0, ri).cpu().numpy().astype(np.float64)
        ref = orc.llr(yr, f.X, f.labels, s2)
        got = lam.index_select(0, ri).cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))) <= 1.0, q
        b = ((lab[tx[q].long()].unsqueeze(1) >> bits) & 1).double()
        u = -(2.0 * b - 1.0) * lam.double()
        cg = (torch.clamp(u, min=0.0) + torch.log1p(torch.exp(-u.abs()))).sum(dim=1) / math.log(2.0)
        assert abs(f.m - float(cg.mean()) - ob[q, 0]) <= GMI_TOL32, q
        say(f"[full] bf16 q={q}: GMI {ob[q, 0]:.6f} (fp16 {out[q, 0]:.6f})")
        del lam, b, u, cg


def test_4d64_workload_full_size(orc):
    """21 SNR points x 1e7 samples of the 4-D M = 64 format on the default
    (autotuned or untuned) path: sampled LLR rows against the oracle, the
    GMI of the one launch against the bit costs of the full LLR arrays, and
    the sampled GMI/MI within Monte-Carlo error."""
    wl = w.workload_4d64()
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    say(f"[full] generating {len(wl.snr_db)} x {wl.n} samples of {f.name}")
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, wl.sigma2, wl.n, dtype=torch.float32)
    out = mdgmi.mdgmi_gmi(gf, y, tx, wl.sigma2, path="auto").cpu().numpy()
    assert np.all(out[:, 4] == wl.n) and np.all(out[:, 5] == 0)
    rng = np.random.default_rng(64)
    ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, "auto"))
    lab = torch.from_numpy(f.labels.astype(np.int64)).cuda()
    bits = torch.arange(f.m, device="cuda", dtype=torch.int64)
    for q in range(0, len(wl.snr_db), 4):
        s2 = float(wl.sigma2[q])
        lam = mdgmi.mdgmi_llr(gf, y[q], s2, path="auto", ws=ws)
        rows = np.sort(rng.choice(wl.n, size=2000, replace=False))
        ri = torch.from_numpy(rows).cuda()
        yr = y[q].index_select(0, ri).cpu().numpy().astype(np.float64)
        ref = orc.llr(yr, f.X, f.labels, s2)
        got = lam.index_select(0, ri).cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref) / (LLR_RTOL * np.maximum(np.abs(ref), 1.0))) <= 1.0, q
        b = ((lab[tx[q].long()].unsqueeze(1) >> bits) & 1).double()
        u = -(2.0 * b - 1.0) * lam.double()
        cg = (torch.clamp(u, min=0.0) + torch.log1p(torch.exp(-u.abs()))).sum(dim=1) / math.log(2.0)
        assert abs(f.m - float(cg.mean()) - out[q, 0]) <= GMI_TOL32, q
        tr = tx[q].index_select(0, ri).cpu().numpy().view(np.uint32)
        r = orc.gmi(yr, tr, f.X, f.labels, s2)
        assert abs(out[q, 1] - r[1]) <= 5.0 * r[3] + 1e-6
        say(f"[full] 4D q={q}: GMI {out[q, 0]:.5f} MI {out[q, 1]:.5f}")
        del lam, b, u, cg
