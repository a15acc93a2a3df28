"""The fused MLP kernel's GELU (packed fp16, no transcendentals) against the
oracle's tanh-form GELU, on the CPU.

The kernel's arithmetic is emulated exactly: the FP32 accumulator s = x / 4
rounded toward zero to fp16, v = clamp(1 - s^2), the polynomial P(v) and the
gate clamp(1/2 + s P(v)) in fused fp16 operations (each an exact FP64 value
rounded once to fp16: every operand here is an fp16 number, and the products
and sums involved fit FP64's 53 bits), the product with the FP32 s rounded
once to FP32 and then to bf16. The coefficients are read from the kernel
source. Bars: |gate - Phi_tanh(x)| <= 8e-4 and |GELU(x) - GELU_tanh(x)|
<= 2.1e-3 over a dense sweep of FP32 inputs; exactly 1 / 0 beyond +-4;
NaN and infinities as the tanh form gives them."""
import re
from pathlib import Path

import numpy as np
import pytest

import mlp_bounds as mb

SRC = Path(__file__).resolve().parents[1] / "paper_2011_13695_amd" / "csrc" / "mlp_fused.hip"


def gate_coefficients():
    m = re.search(r"kGateP\[7\]\s*=\s*\{([^}]*)\}", SRC.read_text())
    assert m, "kGateP not found in the fused kernel source"
    c = [float(t.strip().rstrip("f")) for t in m.group(1).split(",")]
    assert len(c) == 7
    return np.array(c)


def f16(v):
    return np.asarray(v, dtype=np.float64).astype(np.float16).astype(np.float64)


def f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def rtz16(v):
    """FP32 -> fp16 rounded toward zero (v_cvt_pkrtz_f16_f32)."""
    v = np.asarray(v, dtype=np.float64)
    with np.errstate(over="ignore"):
        r = v.astype(np.float16)
    away = np.abs(r.astype(np.float64)) > np.abs(v)
    return np.where(away, np.nextafter(r, np.float16(0)), r).astype(np.float64)


def kernel_gate(s, c):
    """The gate Phi(4 s) as the kernel forms it (NaN where the input is NaN)."""
    c16 = f16(c)
    sh = rtz16(s)
    with np.errstate(invalid="ignore", over="ignore"):
        v = np.clip(f16(1.0 - sh * sh), 0.0, 1.0)
        v = np.where(np.isnan(v), 0.0, v)
        p = np.full_like(v, c16[-1])
        for k in range(len(c16) - 2, -1, -1):
            p = f16(p * v + c16[k])
        return np.clip(f16(sh * p + 0.5), 0.0, 1.0)


def kernel_gelu_quarter(s, c):
    """GELU(4 s) / 4 as stored (before the bf16 rounding)."""
    with np.errstate(invalid="ignore", over="ignore"):
        return f32(np.asarray(s, dtype=np.float64) * kernel_gate(s, c))


def phi_tanh(x):
    return 0.5 * (1.0 + np.tanh(mb.C * (x + 0.044715 * x ** 3)))


def test_gate_polynomial_shape():
    c = gate_coefficients()
    assert c[0] == 0.5                                   # P(0) = 1/2: gate exactly 1 at x = 4
    np.testing.assert_array_equal(f16(c), c)             # the coefficients are fp16 numbers
    # at s -> 0 the gate is 1/2 + s P(1): its slope in s, P(1), is 4 Phi'(0) = 4 sqrt(2/pi) / 2
    assert abs(c.sum() - 2.0 * mb.C) < 4e-3


def test_gate_and_gelu_error_over_fp32_inputs(orc):
    c = gate_coefficients()
    s = f32(np.concatenate([np.linspace(-1.3, 1.3, 2_600_001), np.linspace(-0.02, 0.02, 400_001)]))
    x = 4.0 * s
    gate = kernel_gate(s, c)
    e_gate = np.abs(gate - phi_tanh(x))
    e_gelu = np.abs(4.0 * kernel_gelu_quarter(s, c) - x * phi_tanh(x))
    assert e_gate.max() <= 8e-4, (e_gate.max(), x[np.argmax(e_gate)])
    assert e_gelu.max() <= 2.1e-3, (e_gelu.max(), x[np.argmax(e_gelu)])
    # the numpy tanh form above is the oracle's GELU: check it on a subset, incl. the worst points
    idx = np.unique(np.concatenate([np.arange(0, s.size, 9973), [np.argmax(e_gate), np.argmax(e_gelu)]]))
    ref = np.array([orc.gelu(float(v)) for v in x[idx]])
    np.testing.assert_allclose(x[idx] * phi_tanh(x[idx]), ref, rtol=1e-13, atol=1e-15)
    assert np.max(np.abs(4.0 * kernel_gelu_quarter(s[idx], c) - ref)) <= 2.1e-3


def test_gate_saturates_and_special_values():
    c = gate_coefficients()
    big = f32(np.array([1.0, 1.0000001, 1.5, 7.0, 1e4, 3e38]))
    np.testing.assert_array_equal(kernel_gate(big, c), 1.0)
    np.testing.assert_array_equal(kernel_gate(-big, c), 0.0)
    np.testing.assert_array_equal(kernel_gelu_quarter(big, c), big)      # GELU(x) = x for x >= 4
    assert np.all(kernel_gelu_quarter(-big, c) == 0.0)                    # and 0 for x <= -4
    assert kernel_gelu_quarter(np.array([0.0]), c)[0] == 0.0
    inf = kernel_gelu_quarter(np.array([np.inf, np.nan]), c)
    assert inf[0] == np.inf and np.isnan(inf[1])
    # -inf: -inf * 0, NaN, as x * Phi(x) of the tanh form
    assert np.isnan(kernel_gelu_quarter(np.array([-np.inf]), c)[0])


def test_gate_is_monotone_enough():
    """The gate never leaves [0, 1] and is non-decreasing within its
    rounding (2 fp16 ulps at 1/2..1) over the dense sweep."""
    c = gate_coefficients()
    s = f32(np.linspace(-1.2, 1.2, 400_001))
    g = kernel_gate(s, c)
    assert g.min() >= 0.0 and g.max() <= 1.0
    assert np.min(np.diff(g)) >= -2 * 2.0 ** -11


@pytest.mark.parametrize("seed", [0, 1])
def test_error_model_holds_for_the_fused_gate(seed):
    """The fused kernel's forward pass (bf16 operands, FP32 accumulation,
    this GELU, x / 4 scaling) stays inside the bf16 error model's bar with a
    spread near 1, as the exact-GELU arithmetic does."""
    torch = pytest.importorskip("torch")
    c = gate_coefficients()
    sizes = [9, 256, 256, 256, 11]
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(sizes) - 1):
        bound = 1.0 / np.sqrt(sizes[l])
        params.append(rng.uniform(-bound, bound, sizes[l + 1] * sizes[l] + sizes[l + 1]))
    params = np.concatenate(params).astype(np.float32).astype(np.float64)
    n = 1500
    x = np.concatenate([rng.normal(0, 0.6, (n, 8)), rng.uniform(-1.6, 1.6, (n, 1))], axis=1)
    x = x.astype(np.float32).astype(np.float64)

    def bf(a):
        return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double().numpy()

    Ws, bs = mb.unpack(params, sizes)
    h = bf(x)
    L = len(Ws)
    for l in range(L):
        scale = 0.25 if l == 0 else 4.0 if l == L - 1 else 1.0
        bias = 0.25 * bs[l] if l < L - 1 else bs[l]
        z = f32(h @ bf(Ws[l] * scale).T + bias)
        if l < L - 1:
            h = bf(kernel_gelu_quarter(z, c))
    zs, _, vz = mb.forward_sd(params, sizes, x)
    t = (z - zs[-1]) / np.sqrt(vz[-1])
    assert 0.7 <= float(np.std(t)) <= 1.3, float(np.std(t))
    assert mb.check(z, zs[-1], np.sqrt(vz[-1])) <= 1.0
