"""Pins of the FP64 MLP-demapper oracle (CPU only): finite differences for
the backward pass, closed forms for GELU, the loss and Adam, a one-path
network computed by hand (catches transposed weight layouts), and the
identity between the hard-target cross-entropy and the GMI cost."""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
import workloads as w


def rand_params(sizes, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(size=oracle.mlp_param_count(sizes)) * scale


def test_gelu_matches_erf_form_and_symmetry():
    xs = np.linspace(-6, 6, 241)
    g = np.array([oracle.gelu(x) for x in xs])
    exact = 0.5 * xs * (1 + erf(xs / math.sqrt(2)))
    assert np.max(np.abs(g - exact)) < 1e-3          # the tanh form is a published 1e-3-class approximation
    assert oracle.gelu(0.0) == 0.0
    np.testing.assert_allclose([oracle.gelu(-x) for x in xs], g - xs, atol=1e-14)   # gelu(-x) = gelu(x) - x
    assert abs(oracle.gelu(1.0) - 0.8411919906082768) < 1e-15   # 0.5 (1 + tanh(sqrt(2/pi) * 1.044715))


def test_param_count():
    assert oracle.mlp_param_count([9, 256, 256, 256, 11]) == 9 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 11 + 11


def test_one_path_network_by_hand():
    """Only one weight per layer is non-zero: the logit is a scalar chain."""
    sizes = [3, 4, 5, 2]
    p = np.zeros(oracle.mlp_param_count(sizes))
    # W1[o=2][i=1] = 1.5, b1[2] = 0.25 ; W2[o=4][i=2] = -0.7, b2[4] = 0.1 ; W3[o=1][i=4] = 2.0, b3 = (0.3, -0.2)
    off = 0
    W1 = p[off:off + 12].reshape(4, 3); off += 12
    b1 = p[off:off + 4]; off += 4
    W2 = p[off:off + 20].reshape(5, 4); off += 20
    b2 = p[off:off + 5]; off += 5
    W3 = p[off:off + 10].reshape(2, 5); off += 10
    b3 = p[off:off + 2]
    W1[2, 1] = 1.5; b1[2] = 0.25
    W2[4, 2] = -0.7; b2[4] = 0.1
    W3[1, 4] = 2.0; b3[:] = [0.3, -0.2]
    x = np.array([[0.9, -0.4, 2.0]])
    h1 = oracle.gelu(1.5 * -0.4 + 0.25)
    h2 = oracle.gelu(-0.7 * h1 + 0.1)
    want = np.array([0.3, 2.0 * h2 - 0.2])
    # hidden units that see only a bias still pass gelu(bias) on; here all other biases are 0
    np.testing.assert_allclose(oracle.mlp_forward(p, sizes, x)[0], want, rtol=1e-14, atol=1e-15)


def test_gradient_matches_central_differences():
    sizes = [5, 7, 6, 3]
    p = rand_params(sizes, 1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(13, 5))
    t = rng.uniform(size=(13, 3))
    loss, g = oracle.mlp_loss_grad(p, sizes, x, t)
    eps = 1e-6
    idx = rng.choice(p.size, size=60, replace=False)
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (oracle.mlp_loss_grad(pp, sizes, x, t)[0] - oracle.mlp_loss_grad(pm, sizes, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_closed_forms():
    sizes = [2, 3, 4]
    p = np.zeros(oracle.mlp_param_count(sizes))
    x = np.ones((5, 2))
    # zero network: logits 0, BCE = ln 2 per output whatever the target
    loss, _ = oracle.mlp_loss_grad(p, sizes, x, np.full((5, 4), 0.3))
    assert abs(loss - 4 * math.log(2)) < 1e-14
    # bias-only output: softplus(b) - p b
    p[-4:] = [1.0, -2.0, 0.5, 3.0]
    t = np.full((5, 4), 0.25)
    want = sum(math.log1p(math.exp(b)) - 0.25 * b for b in [1.0, -2.0, 0.5, 3.0])
    assert abs(oracle.mlp_loss_grad(p, sizes, x, t)[0] - want) < 1e-13


def test_adam_closed_form_constant_gradient():
    """With a constant gradient g the bias-corrected moments are g and g^2,
    so every step moves by lr * g / (|g| + eps)."""
    P = 7
    p = np.linspace(-1, 1, P)
    g = np.linspace(-0.3, 0.5, P)
    m = np.zeros(P)
    v = np.zeros(P)
    p0 = p.copy()
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        oracle.adam(p, g, m, v, t, lr, eps=eps)
    np.testing.assert_allclose(p, p0 - 5 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_hard_target_bce_equals_gmi_cost():
    """BCE with hard targets (the sent bits) in bits is m - GMI of the logits
    read as LLRs: ties the loss code to the GMI cost code."""
    sizes = [9, 16, 11]
    p = rand_params(sizes, 3)
    f = w.format_8d2048()
    y, tx = w.channel_samples(f, 0.02, seed=4, snr_slot=0, n=200)
    x = np.concatenate([y, np.full((200, 1), 0.3)], axis=1)
    lab = f.labels[tx]
    bits = ((lab[:, None] >> np.arange(11)) & 1).astype(np.float64)
    loss, _ = oracle.mlp_loss_grad(p, sizes, x, bits)
    logits = oracle.mlp_forward(p, sizes, x)
    cost = oracle.gmi_cost_from_llr(logits, lab)
    assert abs(loss / math.log(2) - cost.mean()) < 1e-12


def test_exact_llrs_as_logits_reproduce_the_exact_gmi(orc):
    """gmi_cost_from_llr on the exact LLRs equals the oracle's own GMI cost."""
    f = w.format_4d64()
    y, tx = w.channel_samples(f, 0.03, seed=5, snr_slot=0, n=300)
    lam = orc.llr(y, f.X, f.labels, 0.03)
    cg, _ = orc.costs(y, tx, f.X, f.labels, 0.03)
    np.testing.assert_allclose(oracle.gmi_cost_from_llr(lam, f.labels[tx]), cg, rtol=1e-12, atol=1e-12)
