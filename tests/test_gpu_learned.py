"""The learned demapper end to end on the GPU: training on exact-demapper
targets lowers the loss, the device learned-GMI kernel agrees with the
oracle's GMI cost of the very same logits, the hard-bit BCE identity holds,
and the per-SNR fallback routes to the exact path where the network is
worse than the 0.01 bit/symbol bound (forced here with a zeroed network)."""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import learned, mdgmi  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qam16():
    f = w.format_16qam()
    return f, mdgmi.Format.of(f)


def test_learned_gmi_kernel_matches_oracle_cost(qam16, orc):
    f, gf = qam16
    net = mdgmi.MLP([3, 32, 4], seed=5)
    snr = np.array([4.0, 12.0])
    s2 = learned.sigma2_of(snr, 2)
    n = 3001
    y, tx = mdgmi.mdgmi_generate(gf, 17, s2, n, dtype=torch.float32)
    say("[learned] gmi kernel vs oracle")
    out = mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr, chunk=1000).cpu().numpy()
    for q in range(2):
        x = mdgmi.mdgmi_mlp_features(y[q].contiguous(), float(snr[q]))
        logits = net.forward(x).cpu().numpy().astype(np.float64)
        lab = f.labels[tx[q].cpu().numpy().view(np.uint32)]
        cost = orc.gmi_cost_from_llr(logits, lab)
        assert abs(out[q, 0] - (4 - cost.mean())) <= 1e-5
        assert out[q, 4] == n and out[q, 5] == 0 and np.isnan(out[q, 1])


def test_training_lowers_loss_and_approaches_exact_gmi(qam16):
    f, gf = qam16
    cfg = learned.TrainConfig(hidden=(64, 64), batch=4096, slices=8, snr_lo=2.0, snr_hi=14.0, steps=400,
                              lr=3e-3, log_every=50, seed=3)
    tr = learned.Trainer(gf, cfg)
    say("[learned] training 16-QAM")
    res = tr.train(log=say)
    first, last = res.losses[0][1], res.losses[-1][1]
    assert last < 0.5 * first
    ev, _, _ = learned.evaluate(tr.net, gf, [4.0, 8.0, 12.0], 20000, sopt=True)
    say(f"[learned] exact {ev.gmi_exact} learned {ev.gmi_learned} s* {ev.s_opt} GMI(s*) {ev.gmi_learned_sopt}")
    assert max(ev.loss) < 0.1          # 16-QAM is easy for a small network
    assert min(ev.loss) > -0.01        # a mismatched metric cannot beat the exact GMI by more than MC noise
    # the s-optimised GMI of the learned LLRs: at least GMI(1), at most the exact GMI (within MC noise)
    for g1, gs, ge in zip(ev.gmi_learned, ev.gmi_learned_sopt, ev.gmi_exact):
        assert gs >= g1 - 1e-6 and gs <= ge + 0.01


def test_fallback_routes_to_exact(qam16):
    f, gf = qam16
    net = mdgmi.MLP([3, 16, 4], seed=1)
    net.set_params(np.zeros(net.P, dtype=np.float32))   # logits 0: learned GMI = 0
    ev, _, _ = learned.evaluate(net, gf, [5.0, 15.0], 5000)
    assert ev.route == ["exact", "exact"]
    assert ev.gmi == ev.gmi_exact
    assert all(abs(g) < 1e-12 for g in ev.gmi_learned)
    p = np.zeros(net.P, dtype=np.float32)
    p[:] = np.nan
    net.set_params(p)
    ev, _, _ = learned.evaluate(net, gf, [5.0], 2000)
    assert ev.route == ["exact"] and np.isnan(ev.gmi_learned[0])


@pytest.mark.parametrize("waves", [4, 8])
def test_fused_inference_matches_layered_path(waves, orc):
    """The fused kernel (activations in registers) gives the GMI of the same
    network as the layer-by-layer GEMM path and as the oracle's cost of the
    layered path's logits."""
    f = w.format_8d2048()
    gf = mdgmi.Format.of(f)
    net = mdgmi.MLP([9, 256, 256, 256, 11], seed=11)
    snr = np.array([5.0, 12.0])
    y, tx = mdgmi.mdgmi_generate(gf, 21, learned.sigma2_of(snr, 8), 5003, dtype=torch.float32)
    say(f"[learned] fused waves={waves}")
    try:
        mdgmi.mdgmi_mlp_set_fused(0)
        ref = mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr).cpu().numpy()
        mdgmi.mdgmi_mlp_set_fused(waves)
        out = mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr).cpu().numpy()
    finally:
        mdgmi.mdgmi_mlp_set_fused(8)
    np.testing.assert_array_equal(out[:, 4], ref[:, 4])
    assert np.max(np.abs(out[:, 0] - ref[:, 0])) <= 1e-3, (out[:, 0], ref[:, 0])
    x = mdgmi.mdgmi_mlp_features(y[0].contiguous(), float(snr[0]))
    logits = net.forward(x).cpu().numpy().astype(np.float64)
    cost = orc.gmi_cost_from_llr(logits, f.labels[tx[0].cpu().numpy().view(np.uint32)])
    assert abs(ref[0, 0] - (11 - cost.mean())) <= 1e-5


def _ms(fn, reps=5):
    """Median device time of fn over reps calls (after one warm-up call)."""
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def test_what_the_network_gains_on_a_structured_format():
    """What the trained network gains: on the 8-D M = 4096 Gray 8-QAM
    product, 2.5e7 training samples bring the paired GMI loss within the
    0.01-bit bound at every SNR point of 2..17 dB, so the library routes all
    of them to the network, and the learned GMI (and the routed path) takes
    less device time than the exact demapper on the same samples: 272k MFMA
    flops and 768 GELUs per sample against 4096 exponentials and their class
    sums."""
    f = w.qam_product(8, 12)
    gf = mdgmi.Format.of(f)
    cfg = learned.TrainConfig(steps=int(2.5e7) // 4096)
    tr = learned.Trainer(gf, cfg)
    say("[gain] training 2.5e7 samples on the 8-D M=4096 Gray 8-QAM product")
    tr.train()
    snr = np.arange(2.0, 18.0)
    s2 = learned.sigma2_of(snr, gf.dim)
    ev, y, tx = learned.evaluate(tr.net, gf, snr, n=1 << 20)
    say(f"[gain] paired loss max {max(ev.loss):.4f}, routes {ev.route.count('learned')}/16 learned")
    assert max(ev.loss) <= 0.01 and all(r == "learned" for r in ev.route), ev.loss
    out = torch.empty((snr.size, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    lws = mdgmi.workspace(mdgmi.mdgmi_mlp_gmi_workspace_size(tr.net, 1 << 20))
    ews = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, 1 << 20, snr.size, "mfma"))
    rws = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, 1 << 20, snr.size, "learned"))
    t_learned = _ms(lambda: mdgmi.mdgmi_mlp_gmi(tr.net, gf, y, tx, snr, out=out, ws=lws))
    t_exact = _ms(lambda: mdgmi.mdgmi_gmi(gf, y, tx, s2, path="mfma", out=out, ws=ews))
    t_routed = _ms(lambda: mdgmi.mdgmi_gmi(gf, y, tx, s2, path="learned", out=out, ws=rws))
    routed = out.cpu().numpy()
    say(f"[gain] learned {t_learned:.2f} ms, routed {t_routed:.2f} ms, exact {t_exact:.2f} ms")
    np.testing.assert_allclose(routed[:, 0], ev.gmi_learned, rtol=0, atol=1e-9)
    assert t_learned < t_exact and t_routed < t_exact
