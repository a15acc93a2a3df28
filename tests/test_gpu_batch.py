"""GPU parity of the ragged persistent batch and of the autotuner's choices:
every instance of a mixed batch (dims 2/4/8, M from 2 to 4096, ragged
sample counts, both paths) against the FP64 oracle on the same samples, the
hipGraph replay against direct launches, and bit-reproducibility."""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2011_13695_amd import mdgmi  # noqa: E402

GMI_TOL32 = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_batch(seed=0, max_pairs=4e6):
    """(format, gpu format, y, tx, sigma2) for a mix that covers every code path."""
    specs = [(2, 2), (2, 4), (4, 8), (8, 16), (2, 32), (4, 64), (8, 128), (2, 256), (4, 1024), (8, 2048),
             (2, 4096), (8, 4096), (4, 512), (8, 64)]
    rng = np.random.default_rng(seed)
    out = []
    for k, (dim, M) in enumerate(specs):
        m = M.bit_length() - 1
        f = w.random_shells(dim, M, 100 + k) if (k % 2 == 0 or dim == 2 and m == 1) else w.qam_product(dim, m)
        snr = float(rng.uniform(-3, 25))
        s2 = float(w.sigma2_from_snr_db(snr, dim))
        n = int(max(33, min(max_pairs / (M * m), 10 ** rng.uniform(2.0, 3.6))))
        y, tx = w.channel_samples(f, s2, seed=seed + k, snr_slot=k, n=n)
        out.append((f, mdgmi.Format.of(f), y.astype(np.float32), tx, s2))
    return out


def to_items(batch):
    items = []
    for f, gf, y, tx, s2 in batch:
        yd = torch.from_numpy(y).cuda()
        td = torch.from_numpy(tx.view(np.int32)).cuda()
        items.append((gf, yd, td, s2))
    return items


@pytest.fixture(scope="module")
def mixed():
    b = mixed_batch()
    return b, to_items(b)


@pytest.fixture(scope="module")
def oracle_rows(mixed, orc):
    b, _ = mixed
    return np.stack([orc.gmi(y.astype(np.float64), tx, f.X, f.labels, s2) for f, _, y, tx, s2 in b])


@pytest.mark.parametrize("path", ["auto", "direct"])
def test_batched_one_shot_matches_oracle(mixed, oracle_rows, path):
    b, items = mixed
    say(f"[batch] one-shot path={path} instances={len(items)}")
    inst = mdgmi.instances(items)
    out = mdgmi.mdgmi_gmi_batched(inst, path=path).cpu().numpy()
    np.testing.assert_array_equal(out[:, 4], oracle_rows[:, 4])
    np.testing.assert_array_equal(out[:, 5], oracle_rows[:, 5])
    assert np.max(np.abs(out[:, 0] - oracle_rows[:, 0])) <= GMI_TOL32
    assert np.max(np.abs(out[:, 1] - oracle_rows[:, 1])) <= GMI_TOL32


def test_batch_plan_graph_and_direct_launches_agree(mixed, oracle_rows):
    b, items = mixed
    say("[batch] plan + graph")
    plan = mdgmi.Batch(items, path="auto")
    info = plan.info()
    assert info["items"] >= len(items)
    g1 = plan.run(use_graph=True).cpu().numpy()
    g2 = plan.run(use_graph=True).cpu().numpy()   # replay
    torch.cuda.synchronize()
    d1 = plan.run(use_graph=False).cpu().numpy()
    assert g1.tobytes() == g2.tobytes() == d1.tobytes()
    assert np.max(np.abs(g1[:, :2] - oracle_rows[:, :2])) <= GMI_TOL32
    # a replay into another output buffer recaptures
    out2 = torch.empty_like(torch.from_numpy(g1)).cuda()
    g3 = plan.run(out=out2, use_graph=True).cpu().numpy()
    assert g3.tobytes() == g1.tobytes()
    plan.close()


def test_batch_matches_per_instance_calls(mixed):
    b, items = mixed
    say("[batch] vs one call per instance")
    inst = mdgmi.instances(items)
    out = mdgmi.mdgmi_gmi_batched(inst, path="direct").cpu().numpy()
    for q, (gf, yd, td, s2) in enumerate(items):
        one = mdgmi.mdgmi_gmi(gf, yd.view(1, -1, gf.dim), td.view(1, -1), [s2], path="direct").cpu().numpy()
        assert abs(one[0, 0] - out[q, 0]) <= 1e-9 and abs(one[0, 1] - out[q, 1]) <= 1e-9


def test_autotuner_table_roundtrip(tmp_path):
    say("[tune] autotune 8D M=256 and 2D M=16")
    e = mdgmi.mdgmi_autotune(8, 256, force=True)
    assert e["dim"] == 8 and e["M"] == 256 and e["direct_rate"] > 0 and e["mfma_rate"] > 0
    assert e["path"] in (mdgmi.MDGMI_PATH_F32_DIRECT, mdgmi.MDGMI_PATH_F32_MFMA_F16SPLIT)
    # bulk timing on at least 2^20 samples, the short regime on 2^15
    assert e["regime"] == mdgmi.MDGMI_TUNE_BULK and e["samples"] >= 1 << 20
    s = e["short"]
    assert s["regime"] == mdgmi.MDGMI_TUNE_SHORT and s["samples"] == 1 << 15 and s["direct_rate"] > 0
    assert mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_SHORT) == s
    e2 = mdgmi.mdgmi_autotune(2, 16, force=True)
    # small formats time the MFMA shapes too (the per-sample 4x4 shape among them)
    assert e2["path"] in (mdgmi.MDGMI_PATH_F32_DIRECT, mdgmi.MDGMI_PATH_F32_MFMA_F16SPLIT)
    assert e2["mfma_rate"] > 0 and 0 <= e2["mfma_variant"] <= 8
    p = tmp_path / "tune.json"
    mdgmi.mdgmi_tune_save(p)
    mdgmi.mdgmi_tune_clear()
    assert mdgmi.mdgmi_tune_lookup(8, 256) is None
    mdgmi.mdgmi_tune_load(p)
    assert mdgmi.mdgmi_tune_lookup(8, 256)["path"] == e["path"]


def test_batch_rejects_bad_instances(mixed):
    b, items = mixed
    gf, yd, td, s2 = items[0]
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_batched(mdgmi.instances([(gf, yd, td, -1.0)]), path="auto")
    assert e.value.code == mdgmi.MDGMI_E_SIGMA2
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.mdgmi_gmi_batched(mdgmi.instances([(gf, yd, td, s2)]), path="f64")
    assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED
    with pytest.raises(mdgmi.MdgmiError) as e:     # M = 2 cannot take the MFMA batch path
        mdgmi.mdgmi_gmi_batched(mdgmi.instances([(gf, yd, td, s2)]), path="mfma")
    assert e.value.code == mdgmi.MDGMI_E_UNSUPPORTED


def test_auto_path_follows_the_regime_of_the_call(tmp_path):
    """A table whose bulk entry says "direct" and whose short entry says "the
    fp16 split, variant 4": AUTO calls of fewer than 2^18 samples give
    exactly the fp16-split result, larger ones exactly the direct result."""
    f = w.random_shells(8, 256, seed=3)
    gf = mdgmi.Format.of(f)
    p = tmp_path / "regimes.json"
    rows = [f'  {{"dim": 8, "M": {f.M}, "regime": 0, "samples": 1048576, "path": 1, "variant": -1, '
            f'"direct_rate": 2.000000e+12, "mfma_rate": 1.000000e+12}}',
            f'  {{"dim": 8, "M": {f.M}, "regime": 1, "samples": 32768, "path": 2, "variant": 4, '
            f'"direct_rate": 1.000000e+12, "mfma_rate": 3.000000e+12}}']
    p.write_text('{"arch": "gfx950", "entries": [\n' + ",\n".join(rows) + "\n]}\n")
    mdgmi.mdgmi_tune_clear()
    try:
        mdgmi.mdgmi_tune_load(p)
        s2 = float(w.sigma2_from_snr_db(10.0, 8))
        for n, ref_path in ((5000, "mfma"), (300_000, "direct")):
            say(f"[tune] AUTO at n={n}: expect the {ref_path} path")
            y, tx = mdgmi.mdgmi_generate(gf, 21, [s2], n, dtype=torch.float32)
            a = mdgmi.mdgmi_gmi(gf, y, tx, [s2], path="auto").cpu().numpy()
            b = mdgmi.mdgmi_gmi(gf, y, tx, [s2], path=ref_path).cpu().numpy()
            np.testing.assert_array_equal(a, b)
    finally:
        mdgmi.mdgmi_tune_clear()
