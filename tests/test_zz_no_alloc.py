"""mdgmi_gmi_static (no allocation: scratch in a static device array)
through the C ABI against mdgmi_gmi on the same samples: bit-identical
results for two calls in a row, the second smaller than the first, on every
path; a call needing more scratch than the array holds is refused before
any launch."""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import mdgmi  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def inputs(f, snrs, n, seed, dtype=np.float32):
    s2 = w.sigma2_from_snr_db(np.asarray(snrs, dtype=np.float64), f.dim)
    ys, txs = [], []
    for q, v in enumerate(s2):
        y, tx = w.channel_samples(f, float(v), seed=seed, snr_slot=q, n=n)
        ys.append(y.astype(dtype))
        txs.append(tx)
    return torch.from_numpy(np.stack(ys)).cuda(), dev_u32(np.stack(txs)), s2


@pytest.mark.parametrize("name,path", [("8d2048", "mfma"), ("8d2048", "mfma_bf16"), ("8d2048", "direct"),
                                       ("4d64", "auto"), ("16qam", "f64")])
def test_static_scratch_matches_workspace_call(name, path):
    f = {"8d2048": w.format_8d2048, "4d64": w.format_4d64, "16qam": w.format_16qam}[name]()
    gf = mdgmi.Format.of(f)
    dt = np.float64 if path == "f64" else np.float32
    # two calls in a row, the second with fewer SNR points and samples
    for k, (snrs, n) in enumerate([(np.arange(2.0, 18.0), 20011), ([5.0, 11.0], 3001)]):
        y, tx, s2 = inputs(f, snrs, n, seed=40 + k, dtype=dt)
        say(f"[static] {name} {path} call {k}: {len(s2)} SNR points x {n}")
        a = mdgmi.mdgmi_gmi_static(gf, y, tx, s2, path=path).cpu().numpy()
        b = mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path).cpu().numpy()
        assert a.tobytes() == b.tobytes()
        assert np.all(a[:, 4] == n) and np.all(np.isfinite(a[:, :2]))


def test_static_scratch_refuses_oversized_calls():
    """8-D M = 4096 on the bf16 split holds a 512 KiB operand image per SNR
    point: 32 points in one launch fill the whole array before any partial
    sums, so the call is refused (valid, correctly sized inputs)."""
    f = w.random_shells(8, 4096, 3)
    gf = mdgmi.Format.of(f)
    n_snr, n = 32, 4096
    need = mdgmi.mdgmi_gmi_workspace_size(gf, n, n_snr, mdgmi._path("mfma_bf16"))
    assert need > mdgmi.MDGMI_STATIC_SCRATCH_BYTES
    y = torch.zeros((n_snr, n, 8), dtype=torch.float32, device="cuda")
    tx = torch.zeros((n_snr, n), dtype=torch.int32, device="cuda")
    s2 = np.full(n_snr, 0.01)
    out = torch.zeros((n_snr, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    say("[static] oversized call")
    rc = mdgmi.lib().mdgmi_gmi_static(gf.handle, mdgmi._dptr(y), mdgmi._dptr(tx), n, s2.ctypes.data_as(mdgmi._P),
                                      n_snr, mdgmi._path("mfma_bf16"), mdgmi._dptr(out), None)
    assert rc == mdgmi.MDGMI_E_WORKSPACE
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    # a smaller call on the same format fits and matches mdgmi_gmi
    a = mdgmi.mdgmi_gmi_static(gf, y[:4].contiguous(), tx[:4].contiguous(), s2[:4], path="mfma_bf16").cpu().numpy()
    b = mdgmi.mdgmi_gmi(gf, y[:4].contiguous(), tx[:4].contiguous(), s2[:4], path="mfma_bf16").cpu().numpy()
    assert a.tobytes() == b.tobytes()
