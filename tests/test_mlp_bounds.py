"""The bf16 error model behind the MLP parity bars (mlp_bounds), checked on
the CPU against an emulation of the kernels' arithmetic: operands rounded
to bf16, products accumulated in FP32, activations and back-propagated
gradients stored in bf16 (the order of operations of the GPU's forward,
BCE and backward passes). The normalised deviations (emulated - exact) / sd
must have a spread near 1 (the model is neither loose nor tight) and stay
inside the K = 8 bar."""
import numpy as np
import pytest

import mlp_bounds as mb

torch = pytest.importorskip("torch")


def bf(a):
    return torch.as_tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float32)


def f32(a):
    return torch.as_tensor(a, dtype=torch.float32)


def gelu_t(z):
    return 0.5 * z * (1.0 + torch.tanh(mb.C * (z + 0.044715 * z ** 3)))


def gelu1_t(z):
    t = torch.tanh(mb.C * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * mb.C * (1.0 + 3.0 * 0.044715 * z * z)


def emulate(params, sizes, x, p):
    """Logits, loss and gradient as the GPU forms them (bf16 operands)."""
    Ws, bs = mb.unpack(params, sizes)
    L = len(Ws)
    h = bf(x)
    Hs, Zs = [h], []
    for l in range(L):
        z = h @ bf(Ws[l]).T + f32(bs[l])
        Zs.append(z)
        if l < L - 1:
            h = bf(gelu_t(z))
            Hs.append(h)
    n = x.shape[0]
    zL = Zs[-1]
    pt = f32(p)
    loss = (torch.nn.functional.softplus(zL.double()) - pt.double() * zL.double()).sum(1).mean().item()
    D = bf((torch.sigmoid(zL) - pt) / n)
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = (D.T @ Hs[l]).double().numpy()
        gb[l] = D.sum(0).double().numpy()
        if l > 0:
            D = bf((D @ bf(Ws[l])) * gelu1_t(Zs[l - 1]))
    return zL.double().numpy(), loss, gW, gb


def exact(params, sizes, x, p):
    Ws, bs = mb.unpack(params, sizes)
    zs, h, _ = mb.forward_sd(params, sizes, x)
    n = x.shape[0]
    zL = zs[-1]
    loss = float(np.mean(np.sum(np.logaddexp(0.0, zL) - p * zL, axis=1)))
    D = (1.0 / (1.0 + np.exp(-zL)) - p) / n
    L = len(Ws)
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = D.T @ h[l]
        gb[l] = D.sum(0)
        if l > 0:
            D = (D @ Ws[l]) * mb.gelu1(zs[l - 1])
    return zL, loss, gW, gb


@pytest.mark.parametrize("seed", [0, 1])
def test_error_model_matches_emulated_bf16_arithmetic(seed):
    sizes = [9, 256, 256, 256, 11]
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(sizes) - 1):
        bound = 1.0 / np.sqrt(sizes[l])
        params.append(rng.uniform(-bound, bound, sizes[l + 1] * sizes[l] + sizes[l + 1]))
    params = np.concatenate(params).astype(np.float32).astype(np.float64)
    n = 600
    x = np.concatenate([rng.normal(0, 0.4, (n, 8)), rng.uniform(-1.6, 1.6, (n, 1))], axis=1)
    x = x.astype(np.float32).astype(np.float64)
    p = 1.0 / (1.0 + np.exp(-rng.normal(0, 3, (n, 11))))
    ze, loss_e, gWe, gbe = emulate(params, sizes, x, p)
    zx, _, _, _ = exact(params, sizes, x, p)
    sd_z = mb.logits_sd(params, sizes, x)
    # sums over samples: against the exact values at the rounded operands
    pq, xq = mb.round_operands(params, sizes, x)
    _, loss_x, gWx, gbx = exact(pq, sizes, xq, p)
    sd_loss, sd_w, sd_b = mb.grad_sd(pq, sizes, xq, p)
    groups = [("logits", ze, zx, sd_z)]
    groups += [(f"dW{l}", gWe[l], gWx[l], sd_w[l]) for l in range(len(gWe))]
    groups += [(f"db{l}", gbe[l], gbx[l], sd_b[l]) for l in range(len(gbe))]
    for name, e, r, sd in groups:
        t = (e - r) / np.maximum(sd, 1e-300)
        spread = float(np.std(t))
        # the model describes the spread (not a loose bound) ...
        assert 0.5 <= spread <= 1.3, (name, spread)
        # ... and the bar holds
        assert mb.check(e, r, sd) <= 1.0, (name, mb.check(e, r, sd))
    assert abs(loss_e - loss_x) <= mb.K_SIGMA * sd_loss + 1e-6 * abs(loss_x)
