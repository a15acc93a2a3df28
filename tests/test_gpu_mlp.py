"""GPU parity of the MLP demapper kernels against the FP64 oracle.

bf16 operands (weights, inputs, activations, back-propagated gradients) with
FP32 accumulation bound the agreement. Every logit, the loss and every
gradient element is held to K = 8 standard deviations of the rounding error
the bf16 arithmetic makes on that element (mlp_bounds: propagated from the
exact |W|, |h| and |D| magnitudes at bf16 resolution) plus FP32 slack;
logits against the oracle at the FP32 masters, the loss and gradients (sums
over samples, in which a weight's fixed rounding error does not average
out) against the oracle at the bf16-rounded weights and features the
kernels multiply. Adam and checkpoints are checked exactly."""
import math
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def layer_slices(sizes):
    off = 0
    out = []
    for l in range(len(sizes) - 1):
        nw = sizes[l + 1] * sizes[l]
        out.append((slice(off, off + nw), slice(off + nw, off + nw + sizes[l + 1])))
        off += nw + sizes[l + 1]
    return out


def demapper_inputs(n, seed=0):
    f = w.format_8d2048()
    snr = 9.0
    s2 = float(w.sigma2_from_snr_db(snr, 8))
    y, tx = w.channel_samples(f, s2, seed=seed, snr_slot=0, n=n)
    x = np.concatenate([y, np.full((n, 1), (snr - 9.5) / 4.5)], axis=1)
    return f, y, tx, x, s2


@pytest.fixture(scope="module")
def net():
    return mdgmi.MLP(SIZES, seed=7)


def test_init_is_seeded_and_bounded(net):
    p = net.params()
    assert p.size == net.P == 9 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 11 + 11
    for l, (ws, bs) in enumerate(layer_slices(SIZES)):
        bound = 1 / math.sqrt(SIZES[l])
        assert np.abs(p[ws]).max() <= bound and np.abs(p[bs]).max() <= bound
        assert np.abs(p[ws]).max() > 0.9 * bound
    again = mdgmi.MLP(SIZES, seed=7).params()
    np.testing.assert_array_equal(p, again)
    assert not np.array_equal(p, mdgmi.MLP(SIZES, seed=8).params())


def test_forward_matches_oracle(net, orc):
    n = 1037
    _, _, _, x, _ = demapper_inputs(n)
    say("[mlp] forward")
    logits = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    p = net.params().astype(np.float64)
    x64 = x.astype(np.float32).astype(np.float64)
    ref = orc.mlp_forward(p, SIZES, x64)
    assert logits.shape == ref.shape
    r = mb.check(logits, ref, mb.logits_sd(p, SIZES, x64))
    say(f"[mlp] forward: max |d| / bar = {r:.3f}")
    assert r <= 1.0, r


def test_features_kernel():
    y = torch.randn(333, 8, device="cuda")
    x = mdgmi.mdgmi_mlp_features(y, 12.5).cpu().numpy()
    np.testing.assert_array_equal(x[:, :8], y.cpu().numpy())
    assert np.all(x[:, 8] == np.float32((12.5 - 9.5) / 4.5))


@pytest.mark.parametrize("n", [129, 5000])
def test_loss_and_gradient_match_oracle(net, orc, n):
    f, y, tx, x, s2 = demapper_inputs(n, seed=n)
    lam = orc.llr(y, f.X, f.labels, s2)           # exact targets from the oracle
    x32 = x.astype(np.float32)
    say(f"[mlp] loss/grad n={n}")
    loss = net.loss_grad(torch.from_numpy(x32).cuda(), torch.from_numpy(lam.astype(np.float32)).cuda())
    g = net.grad().astype(np.float64)
    p = net.params().astype(np.float64)
    target = 1.0 / (1.0 + np.exp(-lam.astype(np.float32).astype(np.float64)))
    # the gradient at the bf16 weights and features the kernels multiply
    pq, xq = mb.round_operands(p, SIZES, x32.astype(np.float64))
    ref_loss, ref_g = orc.mlp_loss_grad(pq, SIZES, xq, target)
    sd_loss, sd_w, sd_b = mb.grad_sd(pq, SIZES, xq, target)
    assert abs(float(loss.item()) - ref_loss) <= mb.K_SIGMA * sd_loss + 1e-6 * abs(ref_loss)
    worst = 0.0
    for l, (ws, bs) in enumerate(layer_slices(SIZES)):
        for sl, sd, name in ((ws, sd_w[l].ravel(), "W"), (bs, sd_b[l], "b")):
            r = mb.check(g[sl], ref_g[sl], sd)
            worst = max(worst, r)
            assert r <= 1.0, (l, name, r)
            # the gradient is resolved: its error is small against its own size
            assert rel(g[sl], ref_g[sl]) <= 0.1, (l, name, rel(g[sl], ref_g[sl]))
    say(f"[mlp] gradient n={n}: max |d| / bar = {worst:.3f}")


@pytest.mark.parametrize("n", [776, 777])
def test_gradient_of_ragged_widths_matches_oracle(orc, n):
    """Widths that fill neither a 64-wide GEMM tile nor a 32-wide K-step
    (40, 24: multiples of 8, so the 16-byte operand path runs with its row
    and k masks) and sample counts on both sides of a multiple of 8 (776:
    the weight gradients take the 16-byte path over ragged K slices; 777:
    the element path)."""
    sizes = [9, 40, 24, 11]
    m_ = mdgmi.MLP(sizes, seed=11)
    f, y, tx, x, s2 = demapper_inputs(n, seed=n)
    lam = orc.llr(y, f.X, f.labels, s2)
    x32 = x.astype(np.float32)
    say(f"[mlp] ragged widths {sizes} n={n}")
    loss = m_.loss_grad(torch.from_numpy(x32).cuda(), torch.from_numpy(lam.astype(np.float32)).cuda())
    g = m_.grad().astype(np.float64)
    p = m_.params().astype(np.float64)
    target = 1.0 / (1.0 + np.exp(-lam.astype(np.float32).astype(np.float64)))
    pq, xq = mb.round_operands(p, sizes, x32.astype(np.float64))
    ref_loss, ref_g = orc.mlp_loss_grad(pq, sizes, xq, target)
    sd_loss, sd_w, sd_b = mb.grad_sd(pq, sizes, xq, target)
    assert abs(float(loss.item()) - ref_loss) <= mb.K_SIGMA * sd_loss + 1e-6 * abs(ref_loss)
    for l, (ws, bs) in enumerate(layer_slices(sizes)):
        for sl, sd, name in ((ws, sd_w[l].ravel(), "W"), (bs, sd_b[l], "b")):
            r = mb.check(g[sl], ref_g[sl], sd)
            assert r <= 1.0, (l, name, r)
            assert rel(g[sl], ref_g[sl]) <= 0.1, (l, name, rel(g[sl], ref_g[sl]))
    logits = m_.forward(torch.from_numpy(x32).cuda()).cpu().numpy()
    ref = orc.mlp_forward(p, sizes, x32.astype(np.float64))
    r = mb.check(logits, ref, mb.logits_sd(p, sizes, x32.astype(np.float64)))
    say(f"[mlp] ragged widths n={n}: logits max |d| / bar = {r:.3f}")
    assert r <= 1.0, r


def test_adam_matches_oracle_on_the_gpu_gradient(orc):
    sizes = [9, 64, 11]
    m_ = mdgmi.MLP(sizes, seed=3)
    f, y, tx, x, s2 = demapper_inputs(300, seed=9)
    lam = orc.llr(y, f.X, f.labels, s2).astype(np.float32)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    ld = torch.from_numpy(lam).cuda()
    p = m_.params().astype(np.float64)
    mm = np.zeros_like(p)
    vv = np.zeros_like(p)
    for t in range(1, 4):
        m_.loss_grad(xd, ld)
        g = m_.grad().astype(np.float64)
        m_.adam_step(1e-3)
        orc.adam(p, g, mm, vv, t, 1e-3)
        np.testing.assert_allclose(m_.params(), p, rtol=2e-6, atol=2e-8)
        p = m_.params().astype(np.float64)   # follow the FP32 trajectory
        a, b = m_.moments()
        mm, vv = a.astype(np.float64), b.astype(np.float64)


def test_checkpoint_roundtrip(tmp_path, orc):
    sizes = [9, 32, 11]
    a = mdgmi.MLP(sizes, seed=1)
    f, y, tx, x, s2 = demapper_inputs(100, seed=2)
    lam = orc.llr(y, f.X, f.labels, s2).astype(np.float32)
    a.loss_grad(torch.from_numpy(x.astype(np.float32)).cuda(), torch.from_numpy(lam).cuda())
    a.adam_step(1e-2)
    path = tmp_path / "mlp.bin"
    a.save(path)
    b = mdgmi.MLP(sizes, seed=99)
    b.load(path)
    np.testing.assert_array_equal(a.params(), b.params())
    for u, v in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(u, v)
    # identical next step from both
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    for net in (a, b):
        net.loss_grad(xd, torch.from_numpy(lam).cuda())
        net.adam_step(1e-2)
    np.testing.assert_array_equal(a.params(), b.params())
    with pytest.raises(mdgmi.MdgmiError):
        mdgmi.MLP([9, 33, 11]).load(path)   # widths must match
