"""Element-wise error model of the MLP kernels' bf16 arithmetic, for parity
tests against the FP64 oracle.

The GPU rounds weights, activations and back-propagated gradients to bf16
(8 significant bits, round to nearest even: the error of a value v is
uniform within +-ulp(v) / 2, ulp(v) = 2^(floor(log2 |v|) - 7), so its
variance is ulp(v)^2 / 12 = v^2 rv(v)) and accumulates in FP32. Each rounding
is an independent zero-mean error; a sum of many such terms is close to
Gaussian, so the deviation of a GPU output from the exact value is modelled
by its standard deviation, propagated layer by layer from the magnitudes
of the exact quantities:

  forward   z_o = sum_i W_oi h_i + b_o:
            Var dz_o = sum_i (W_oi h_i)^2 (rv(W_oi) + rv(h_i)) + sum_i W_oi^2 Var dh_i
            (the rounding of W_oi and of h_i), dh = gelu'(z) dz.
  backward  D_L = bf16((sigmoid(z_L) - p) / n), D_(l-1) = bf16((D_l W_l) gelu'(z_(l-1))),
            dW_l = D_l^T H_(l-1) (bf16 operands), db_l = sum_s D_l:
            the same rule for every product and sum, with the rounding of
            each stored operand and the error of its inputs.

Tests accept |gpu - oracle| <= K sd + FP32 slack with K = 8. Against an
emulation of the kernels' bf16 arithmetic (tests/test_mlp_bounds.py) the
normalised deviations spread by 0.98-1.14 sd (correlations between the
forward error of an activation and the gradient it meets are not modelled)
and reach 6 sd among 65536 weight-gradient elements, hence K = 8.

The rounding of a weight (and of a feature every sample shares, such as
the SNR input) is one fixed error for all samples: it averages out of no
sum over samples. The weight gradient sums over samples, so its parity is
taken against the oracle at the bf16-rounded weights and features the
kernels actually use (exact=True below drops their rounding from the
model); per-sample outputs (logits) against the oracle at the FP32 masters. The exact intermediate values needed
for the magnitudes are formed here in FP64 with numpy; the reference
values the tests compare with come from the oracle.
"""
import math

import numpy as np

K_SIGMA = 8.0


def rv(v):
    """Relative variance of rounding v to bf16: (ulp(v) / v)^2 / 12."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.exp2(np.floor(np.log2(a)) - 7.0) / a
    return np.where(a > 0, u * u / 12.0, 0.0)
C = math.sqrt(2.0 / math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C * (z + 0.044715 * z ** 3)))


def gelu1(z):
    t = np.tanh(C * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C * (1.0 + 3.0 * 0.044715 * z * z)


def gelu2(z, h=1e-4):
    return (gelu1(z + h) - gelu1(z - h)) / (2.0 * h)


def unpack(params, sizes):
    Ws, bs, off = [], [], 0
    for l in range(len(sizes) - 1):
        nw = sizes[l + 1] * sizes[l]
        Ws.append(params[off:off + nw].reshape(sizes[l + 1], sizes[l]).astype(np.float64))
        bs.append(params[off + nw:off + nw + sizes[l + 1]].astype(np.float64))
        off += nw + sizes[l + 1]
    return Ws, bs


def forward_sd(params, sizes, x, exact=False):
    """(z per layer, h per layer (h[0] = x), var of dz per layer). exact:
    weights and features are taken as already rounded (no error of theirs)."""
    Ws, bs = unpack(params, sizes)
    h = [np.asarray(x, dtype=np.float64)]
    zs, vz = [], []
    vh = np.zeros_like(h[0])
    L = len(Ws)
    for l in range(L):
        W = Ws[l]
        z = h[-1] @ W.T + bs[l]
        hh = h[-1] ** 2
        v = vh @ (W.T ** 2)
        if l > 0 or not exact:
            v = v + (hh * rv(h[-1])) @ (W.T ** 2)
        if not exact:
            v = v + hh @ (W.T ** 2 * rv(W.T))
        zs.append(z)
        vz.append(v)
        if l < L - 1:
            hn = gelu(z)
            vh = gelu1(z) ** 2 * v
            h.append(hn)
    return zs, h, vz


def logits_sd(params, sizes, x):
    zs, _, vz = forward_sd(params, sizes, x)
    return np.sqrt(vz[-1])


def grad_sd(params, sizes, x, p, exact=True):
    """Standard deviations of the GPU's loss and of each layer's dW, db
    (lists, layer order), for targets p = sigmoid(lambda), against the
    gradient at the rounded weights and features (exact=True)."""
    Ws, bs = unpack(params, sizes)
    zs, h, vz = forward_sd(params, sizes, x, exact)
    n = x.shape[0]
    L = len(Ws)
    zL = zs[-1]
    sg = 1.0 / (1.0 + np.exp(-zL))
    G = (sg - p) / n
    sd_loss = math.sqrt(np.sum(np.sum(np.abs(sg - p) * np.sqrt(vz[-1]), axis=1) ** 2)) / n
    D = G
    # logit error through sigmoid, bf16 storage, FP32 evaluation of sigmoid(z) - p
    vD = (sg * (1.0 - sg) / n) ** 2 * vz[-1] + rv(G) * G ** 2 + (1.2e-7 / n) ** 2
    vW, vb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        hp = h[l]
        if l > 0:
            vhp = gelu1(zs[l - 1]) ** 2 * vz[l - 1] + rv(hp) * hp ** 2   # forward error + bf16 storage
        else:
            vhp = np.zeros_like(hp) if exact else rv(hp) * hp ** 2          # the features rounded to bf16
        vW[l] = vD.T @ (hp ** 2) + (D ** 2).T @ vhp
        vb[l] = vD.sum(axis=0)
        if l > 0:
            W = Ws[l]
            P = D @ W
            vP = vD @ (W ** 2) + (0.0 if exact else (D ** 2) @ (W ** 2 * rv(W)))
            g1 = gelu1(zs[l - 1])
            Dn = P * g1
            vDn = g1 ** 2 * vP + (P * gelu2(zs[l - 1])) ** 2 * vz[l - 1] + rv(Dn) * Dn ** 2
            D, vD = Dn, vDn
    return sd_loss, [np.sqrt(v) for v in vW], [np.sqrt(v) for v in vb]


def round_operands(params, sizes, x):
    """(params with every weight rounded to bf16 and biases kept, features
    rounded to bf16): the operands the kernels multiply."""
    import torch
    bf = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double().numpy()  # noqa: E731
    q = np.array(params, dtype=np.float64)
    off = 0
    for l in range(len(sizes) - 1):
        nw = sizes[l + 1] * sizes[l]
        q[off:off + nw] = bf(q[off:off + nw])
        off += nw + sizes[l + 1]
    return q, bf(x)


def check(gpu, ref, sd, fp32_rel=1e-6, floor=1e-12):
    """Largest |gpu - ref| / (K sd + FP32 slack) over the elements (<= 1 passes)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    bar = K_SIGMA * np.asarray(sd) + fp32_rel * np.abs(ref) + floor
    return float(np.max(np.abs(gpu - ref) / bar))
