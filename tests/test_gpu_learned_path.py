"""The learned demapper through the C ABI: mdgmi_mlp_llr (the fused kernel's
LLR mode) element-wise against the FP64 oracle's forward pass,
mdgmi_mlp_train_step against its parts, a 50-step Adam trajectory against
the oracle's forward/backward/Adam, and MDGMI_PATH_LEARNED_BF16 in
mdgmi_gmi / mdgmi_llr with the per-SNR fallback decided by
mdgmi_learned_calibrate inside the library.

Bars: logits within K = 8 standard deviations of the bf16 rounding error
model (mlp_bounds) plus FP32 slack; routed results bit-identical to the
call they route to; the trajectory's losses within 1e-4 (relative) of the
oracle's and its parameter displacement within 3% (relative L2) of the
oracle's: the gradients carry bf16 errors of about 1e-3 of their size,
Adam normalises each step, and an element whose gradient is near zero can
take a step of another sign (measured: 7e-6 and 0.3%)."""
import sys

import numpy as np
import pytest

import mlp_bounds as mb
import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import mdgmi  # noqa: E402

SIZES = [9, 256, 256, 256, 11]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def feats(y, snr):
    """Features as the kernels form them: [y, (SNR_dB - 9.5) / 4.5] (SNR values
    that float32 represents exactly, so host and device agree)."""
    snr = np.asarray(snr, dtype=np.float32).astype(np.float64)
    return np.concatenate([y.astype(np.float64), ((snr - 9.5) / 4.5)[:, None]], axis=1)


@pytest.fixture(scope="module")
def fmt8():
    f = w.format_8d2048()
    return f, mdgmi.Format.of(f)


@pytest.mark.parametrize("n", [97, 4099])
def test_mlp_llr_elementwise_against_oracle(orc, fmt8, n):
    f, gf = fmt8
    net = mdgmi.MLP(SIZES, seed=21)
    rng = np.random.default_rng(n)
    snr = rng.choice(np.arange(2.0, 17.25, 0.25), size=n)
    s2 = w.sigma2_from_snr_db(snr, 8)
    y = (f.X[rng.integers(0, f.M, n)] + np.sqrt(s2)[:, None] * rng.standard_normal((n, 8))).astype(np.float32)
    say(f"[learned] mdgmi_mlp_llr n={n}")
    lam = net.llr(torch.from_numpy(y).cuda(), torch.from_numpy(snr.astype(np.float32)).cuda()).cpu().numpy()
    p = net.params().astype(np.float64)
    x = feats(y, snr)
    ref = orc.mlp_forward(p, SIZES, x)
    r = mb.check(lam, ref, mb.logits_sd(p, SIZES, x))
    say(f"[learned] fused LLR mode: max |d| / bar = {r:.3f}")
    assert lam.shape == (n, 11) and r <= 1.0
    # the layer-by-layer GEMM path computes the same logits within the same model
    mdgmi.mdgmi_mlp_set_fused(0)
    try:
        lam2 = net.llr(torch.from_numpy(y).cuda(), torch.from_numpy(snr.astype(np.float32)).cuda()).cpu().numpy()
    finally:
        mdgmi.mdgmi_mlp_set_fused(8)
    assert mb.check(lam2, ref, mb.logits_sd(p, SIZES, x)) <= 1.0


@pytest.mark.parametrize("out", [1, 5, 16, 21, 32])
def test_mlp_llr_output_widths(orc, out):
    """The fused kernel's LLR stores for output widths that fill whole
    groups of four rows (16, 32) and that end inside one (1, 5, 21), each
    row against the oracle's logits."""
    sizes = [9, 256, 256, 256, out]
    net = mdgmi.MLP(sizes, seed=40 + out)
    rng = np.random.default_rng(out)
    n = 301
    snr = rng.choice(np.arange(2.0, 17.25, 0.25), size=n)
    y = rng.normal(0.0, 0.7, (n, 8)).astype(np.float32)
    say(f"[learned] mdgmi_mlp_llr out={out}")
    lam = net.llr(torch.from_numpy(y).cuda(), torch.from_numpy(snr.astype(np.float32)).cuda()).cpu().numpy()
    assert lam.shape == (n, out)
    p = net.params().astype(np.float64)
    x = feats(y, snr)
    ref = orc.mlp_forward(p, sizes, x)
    assert mb.check(lam, ref, mb.logits_sd(p, sizes, x)) <= 1.0


def test_mlp_llr_saturated_gelus_and_nan_rows(orc, fmt8):
    """Inputs far outside the trained range drive most pre-activations past
    |x| = 4, where the fused kernel's GELU gate is exactly 0 or 1: the LLRs
    still follow the oracle within the error model; a NaN input row gives NaN
    logits on that row only."""
    f, gf = fmt8
    net = mdgmi.MLP(SIZES, seed=33)
    rng = np.random.default_rng(5)
    n = 515
    snr = rng.choice(np.arange(2.0, 17.25, 0.25), size=n)
    y = (300.0 * rng.standard_normal((n, 8))).astype(np.float32)
    y[7, 3] = np.nan
    say("[learned] mdgmi_mlp_llr saturated inputs")
    lam = net.llr(torch.from_numpy(y).cuda(), torch.from_numpy(snr.astype(np.float32)).cuda()).cpu().numpy()
    assert np.all(np.isnan(lam[7])) and np.all(np.isfinite(np.delete(lam, 7, axis=0)))
    p = net.params().astype(np.float64)
    keep = np.arange(n) != 7
    x = feats(y[keep], snr[keep])
    ref = orc.mlp_forward(p, SIZES, x)
    zs, _, _ = mb.forward_sd(p, SIZES, x)
    assert np.mean(np.abs(zs[0]) >= 4.0) > 0.5           # most first-layer GELUs saturated
    r = mb.check(lam[keep], ref, mb.logits_sd(p, SIZES, x))
    say(f"[learned] saturated: max |d| / bar = {r:.3f}")
    assert r <= 1.0


def test_fused_gmi_is_the_gmi_of_its_llrs(orc, fmt8):
    """The fused GMI mode costs the same logits its LLR mode stores."""
    f, gf = fmt8
    net = mdgmi.MLP(SIZES, seed=5)
    snrs = np.array([3.0, 11.5])
    s2 = w.sigma2_from_snr_db(snrs, 8)
    n = 3001
    ys, txs = zip(*(w.channel_samples(f, float(v), seed=8, snr_slot=q, n=n) for q, v in enumerate(s2)))
    y = np.stack(ys).astype(np.float32)
    tx = np.stack(txs)
    out = mdgmi.mdgmi_mlp_gmi(net, gf, torch.from_numpy(y).cuda(), dev_u32(tx), snrs).cpu().numpy()
    for q in range(2):
        lam = net.llr(torch.from_numpy(y[q]).cuda(), torch.full((n,), float(snrs[q]), device="cuda")).cpu().numpy()
        c = orc.gmi_cost_from_llr(lam.astype(np.float64), f.labels[tx[q]])
        assert abs(out[q, 0] - (f.m - c.mean())) <= 1e-5, (out[q, 0], f.m - c.mean())
        assert np.isnan(out[q, 1]) and out[q, 4] == n


def test_train_step_is_loss_grad_then_adam(orc, fmt8):
    f, gf = fmt8
    a = mdgmi.MLP([9, 64, 11], seed=4)
    b = mdgmi.MLP([9, 64, 11], seed=4)
    n = 512
    snr = np.repeat([4.0, 12.5], n // 2)
    s2 = w.sigma2_from_snr_db(snr, 8)
    rng = np.random.default_rng(1)
    tx = rng.integers(0, f.M, n)
    y = (f.X[tx] + np.sqrt(s2)[:, None] * rng.standard_normal((n, 8))).astype(np.float32)
    lam = np.concatenate([orc.llr(y[:n // 2].astype(np.float64), f.X, f.labels, float(s2[0])),
                          orc.llr(y[n // 2:].astype(np.float64), f.X, f.labels, float(s2[-1]))]).astype(np.float32)
    yd, ld = torch.from_numpy(y).cuda(), torch.from_numpy(lam).cuda()
    say("[learned] train_step")
    for _ in range(3):
        a.train_step(yd, torch.from_numpy(snr.astype(np.float32)).cuda(), ld, 2e-3)
        x = torch.cat([mdgmi.mdgmi_mlp_features(yd[:n // 2], 4.0), mdgmi.mdgmi_mlp_features(yd[n // 2:], 12.5)])
        b.loss_grad(x.contiguous(), ld)
        b.adam_step(2e-3)
    np.testing.assert_array_equal(a.params(), b.params())


def test_adam_trajectory_against_oracle(orc, fmt8):
    """50 Adam steps of a [9, 64, 11] network on the same batches: the GPU
    (bf16 GEMMs, FP32 masters) against the oracle's FP64 forward, backward
    and Adam."""
    f, gf = fmt8
    sizes = [9, 64, 11]
    net = mdgmi.MLP(sizes, seed=12)
    p = net.params().astype(np.float64)
    p0 = p.copy()
    mm, vv = np.zeros_like(p), np.zeros_like(p)
    rng = np.random.default_rng(77)
    n, lr = 512, 2e-3
    loss_gpu, loss_ref = [], []
    say("[learned] 50-step trajectory")
    for t in range(1, 51):
        snr = rng.choice(np.arange(2.0, 17.25, 0.25), size=n).astype(np.float32)
        s2 = w.sigma2_from_snr_db(snr.astype(np.float64), 8)
        tx = rng.integers(0, f.M, n)
        y = (f.X[tx] + np.sqrt(s2)[:, None] * rng.standard_normal((n, 8))).astype(np.float32)
        lam = np.empty((n, f.m), dtype=np.float32)
        for v in np.unique(snr):                     # oracle targets per SNR value
            k = snr == v
            lam[k] = orc.llr(y[k].astype(np.float64), f.X, f.labels, float(w.sigma2_from_snr_db(float(v), 8)))
        loss = net.train_step(torch.from_numpy(y).cuda(), torch.from_numpy(snr).cuda(), torch.from_numpy(lam).cuda(),
                              lr)
        loss_gpu.append(float(loss.item()))
        target = 1.0 / (1.0 + np.exp(-lam.astype(np.float64)))
        lr_, g = orc.mlp_loss_grad(p, sizes, feats(y, snr), target)
        loss_ref.append(lr_)
        orc.adam(p, g, mm, vv, t, lr)
    loss_gpu, loss_ref = np.array(loss_gpu), np.array(loss_ref)
    dl = np.max(np.abs(loss_gpu - loss_ref) / loss_ref)
    pg = net.params().astype(np.float64)
    dd = np.linalg.norm((pg - p0) - (p - p0)) / np.linalg.norm(p - p0)
    say(f"[learned] trajectory: loss {loss_ref[0]:.4f} -> {loss_ref[-1]:.4f} nats, max rel loss diff {dl:.2e}, "
        f"displacement rel diff {dd:.3f}")
    assert loss_ref[-10:].mean() < loss_ref[:10].mean()   # it learns (fresh batches each step)
    assert dl <= 1e-4 and dd <= 0.03, (dl, dd)


def test_learned_path_routes_per_snr(orc, fmt8):
    """Calibration decides per SNR point inside the library; the learned path
    then gives exactly the network's result where routed to it and exactly
    the exact path's result elsewhere (also for an uncalibrated SNR)."""
    f, gf = fmt8
    g2 = mdgmi.Format.of(f)          # a format object of its own for the attachment
    net = mdgmi.MLP(SIZES, seed=31)
    snrs = np.array([2.0, 6.0, 10.0, 14.0])
    s2 = w.sigma2_from_snr_db(snrs, 8)
    n = 8192
    y, tx = mdgmi.mdgmi_generate(g2, 17, s2, n, snr_slot0=900)
    ex = mdgmi.mdgmi_gmi(g2, y, tx, s2, path="auto").cpu().numpy()
    le = mdgmi.mdgmi_mlp_gmi(net, g2, y, tx, snrs).cpu().numpy()
    with pytest.raises(mdgmi.MdgmiError) as e:              # nothing attached yet
        mdgmi.mdgmi_gmi(g2, y, tx, s2, path="learned")
    assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED
    say("[learned] calibrate: every point to the network")
    res = mdgmi.mdgmi_learned_calibrate(g2, net, y, tx, s2, max_loss=1e6)
    np.testing.assert_array_equal(res[:, 0], ex[:, 0])
    np.testing.assert_array_equal(res[:, 1], le[:, 0])
    np.testing.assert_allclose(res[:, 2], ex[:, 0] - le[:, 0], rtol=0, atol=0)
    assert np.all(res[:, 3] == 1)
    out = mdgmi.mdgmi_gmi(g2, y, tx, s2, path="learned").cpu().numpy()
    assert out.tobytes() == le.tobytes()
    say("[learned] calibrate: a bound between the losses")
    bound = float(np.sort(res[:, 2])[1]) + 1e-9
    res = mdgmi.mdgmi_learned_calibrate(g2, net, y, tx, s2, max_loss=bound)
    routed = res[:, 3] == 1
    assert 0 < routed.sum() < len(snrs)
    out = mdgmi.mdgmi_gmi(g2, y, tx, s2, path="learned").cpu().numpy()
    for q in range(len(snrs)):
        want = le[q] if routed[q] else ex[q]
        assert out[q].tobytes() == want.tobytes(), (q, out[q], want)
    # LLRs follow the same route
    for q in range(len(snrs)):
        lam = mdgmi.mdgmi_llr(g2, y[q], float(s2[q]), path="learned").cpu().numpy()
        if routed[q]:
            ref = net.llr(y[q], torch.full((n,), float(snrs[q]), device="cuda")).cpu().numpy()
        else:
            ref = mdgmi.mdgmi_llr(g2, y[q], float(s2[q]), path="auto").cpu().numpy()
        assert lam.tobytes() == ref.tobytes(), q
    # an SNR never calibrated takes the exact path
    s2x = w.sigma2_from_snr_db(np.array([7.0]), 8)
    ox = mdgmi.mdgmi_gmi(g2, y[1:2], tx[1:2], s2x, path="learned").cpu().numpy()
    assert ox.tobytes() == mdgmi.mdgmi_gmi(g2, y[1:2], tx[1:2], s2x, path="auto").cpu().numpy().tobytes()
    say("[learned] calibrate: bound 0 routes everything to the exact path")
    res = mdgmi.mdgmi_learned_calibrate(g2, net, y, tx, s2, max_loss=0.0)
    assert np.all(res[:, 3] == 0)
    out = mdgmi.mdgmi_gmi(g2, y, tx, s2, path="learned").cpu().numpy()
    assert out.tobytes() == ex.tobytes()
