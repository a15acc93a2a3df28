"""The streaming monitor (mdgmi_stream_*) through the C ABI:
* each buffer's row equals mdgmi_gmi on the same samples (bit-identical:
  same kernels, same launch for the same n), including a short last buffer,
  and agrees with the FP64 oracle within 1e-4 bit;
* the running total equals the sample-weighted combination of the buffers
  (1e-12) and the oracle over all samples (1e-4), and is bit-identical for
  1, 3 and 8 lanes and for host (pinned and pageable) and device inputs;
* the result ring, reset, wait semantics and argument errors;
* a launch-shape change between create and push (tuning) stays within the
  workspace sized at create and gives the same GMI/MI.
"""
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


def buffers(f, s2, sizes, seed=5):
    out = []
    for k, n in enumerate(sizes):
        y, tx = w.channel_samples(f, s2, seed=seed, snr_slot=k, n=n)
        out.append((y.astype(np.float32), tx))
    return out


def run(f, gf, s2, bufs, lanes, mode, path="auto", ring=64):
    st = mdgmi.Stream(gf, s2, max(len(b[0]) for b in bufs), n_lanes=lanes, path=path, ring=ring)
    for y, tx in bufs:
        if mode == "device":
            st.push(torch.from_numpy(y).cuda(), torch.from_numpy(tx.view(np.int32)).cuda())
        elif mode == "pinned":
            st.push(torch.from_numpy(y).pin_memory(), torch.from_numpy(tx.view(np.int32)).pin_memory())
        else:
            st.push(y, tx)
    rows = np.array([st.result(i) for i in range(len(bufs))])
    tot = st.total()
    st.close()
    return rows, tot


@pytest.mark.parametrize("name", ["16qam", "8d2048"])
def test_rows_and_totals(orc, name):
    f = w.format_16qam() if name == "16qam" else w.format_8d2048()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(9.0, f.dim))
    sizes = [4096] * 6 + [1717]
    bufs = buffers(f, s2, sizes)
    rows, tot = run(f, gf, s2, bufs, 3, "device")
    for k, (y, tx) in enumerate(bufs):
        one = mdgmi.mdgmi_gmi(gf, torch.from_numpy(y[None]).cuda(), torch.from_numpy(tx[None].view(np.int32)).cuda(),
                              [s2], path="auto").cpu().numpy()[0]
        np.testing.assert_array_equal(rows[k], one)
        ref = orc.gmi(y.astype(np.float64), tx, f.X, f.labels, s2)
        assert np.max(np.abs(rows[k, :2] - ref[:2])) <= 1e-4
    n = np.array(sizes, dtype=np.float64)
    for col in (0, 1):
        comb = np.sum(n * rows[:, col]) / n.sum()
        assert abs(comb - tot[col]) <= 1e-12 * max(1.0, abs(comb))
    assert tot[4] == n.sum() and tot[5] == 0
    ya = np.concatenate([b[0] for b in bufs]).astype(np.float64)
    ta = np.concatenate([b[1] for b in bufs])
    ref = orc.gmi(ya, ta, f.X, f.labels, s2)
    assert np.max(np.abs(tot[:2] - ref[:2])) <= 1e-4
    assert tot[2] == pytest.approx(ref[2], rel=1e-3) and tot[3] == pytest.approx(ref[3], rel=1e-3)
    say(f"[stream] {name}: total GMI {tot[0]:.6f} MI {tot[1]:.6f} vs oracle {ref[0]:.6f} {ref[1]:.6f}")


def test_lanes_and_inputs_bit_identical():
    f = w.format_4d64()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(12.0, 4))
    bufs = buffers(f, s2, [20000] * 9 + [333], seed=9)
    base_rows, base_tot = run(f, gf, s2, bufs, 1, "device")
    for lanes, mode in ((3, "device"), (8, "device"), (4, "pinned"), (2, "host")):
        rows, tot = run(f, gf, s2, bufs, lanes, mode)
        np.testing.assert_array_equal(rows, base_rows)
        np.testing.assert_array_equal(tot, base_tot)


def test_ring_reset_and_errors():
    f = w.format_16qam()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(10.0, 2))
    bufs = buffers(f, s2, [1000] * 5, seed=2)
    st = mdgmi.Stream(gf, s2, 1000, n_lanes=2, ring=2)
    for y, tx in bufs:
        st.push(y, tx)
    st.wait()
    assert st.info()[0] == 5
    with pytest.raises(mdgmi.MdgmiError) as e:
        st.result(1)                                  # overwritten in a ring of 2
    assert e.value.code == mdgmi.MDGMI_E_ARG
    r4 = st.result(4)
    assert r4[4] == 1000
    with pytest.raises(mdgmi.MdgmiError) as e:
        st.result(5)                                  # not pushed yet
    assert e.value.code == mdgmi.MDGMI_E_ARG
    assert st.total()[4] == 5000
    st.reset()
    assert st.total()[4] == 0
    st.push(*bufs[0])
    t = st.total()
    assert t[4] == 1000 and t[0] == pytest.approx(st.result(5)[0], abs=1e-15)
    big = np.zeros((1001, 2), np.float32)
    with pytest.raises(mdgmi.MdgmiError) as e:
        st.push(big, np.zeros(1001, np.uint32))
    assert e.value.code == mdgmi.MDGMI_E_SHAPE
    st.close()
    for kw, code in (({"n_lanes": 0}, mdgmi.MDGMI_E_SHAPE), ({"n_lanes": 9}, mdgmi.MDGMI_E_SHAPE),
                     ({"ring": 0}, mdgmi.MDGMI_E_SHAPE)):
        with pytest.raises(mdgmi.MdgmiError) as e:
            mdgmi.Stream(gf, s2, 1000, **kw)
        assert e.value.code == code
    with pytest.raises(mdgmi.MdgmiError) as e:
        mdgmi.Stream(gf, -1.0, 1000)
    assert e.value.code == mdgmi.MDGMI_E_SIGMA2


def test_f64_path_stream(orc):
    f = w.format_16qam()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(6.0, 2))
    st = mdgmi.Stream(gf, s2, 3000, n_lanes=2, path="f64")
    ys = []
    for k in range(4):
        y, tx = w.channel_samples(f, s2, seed=3, snr_slot=k, n=3000)
        st.push(torch.from_numpy(y).cuda(), torch.from_numpy(tx.view(np.int32)).cuda())
        ys.append((y, tx))
    tot = st.total()
    st.close()
    ref = orc.gmi(np.concatenate([a for a, _ in ys]), np.concatenate([b for _, b in ys]), f.X, f.labels, s2)
    assert np.max(np.abs(tot[:2] - ref[:2])) <= 1e-10


@pytest.mark.parametrize("name", ["16qam", "8d2048"])
def test_benchmark_configuration(orc, name):
    """2^22-sample buffers on 4 lanes, as the benchmark times them: every
    row bit-identical to mdgmi_gmi on that buffer (itself checked against
    the oracle at full size elsewhere), the total equal to the sample-weighted
    rows, and 512 sampled samples of the last buffer against the oracle's
    per-sample costs."""
    f = w.format_16qam() if name == "16qam" else w.format_8d2048()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(10.0, f.dim))
    nb = 1 << 22
    y, tx = mdgmi.mdgmi_generate(gf, 77, [s2] * 3, nb, dtype=torch.float32)
    st = mdgmi.Stream(gf, s2, nb, n_lanes=4, path="auto")
    for k in range(3):
        st.push(y[k], tx[k])
    rows = np.array([st.result(k) for k in range(3)])
    tot = st.total()
    st.close()
    for k in range(3):
        one = mdgmi.mdgmi_gmi(gf, y[k:k + 1], tx[k:k + 1], [s2], path="auto").cpu().numpy()[0]
        np.testing.assert_array_equal(rows[k], one)
    assert abs(np.mean(rows[:, 0]) - tot[0]) <= 1e-12 and tot[4] == 3 * nb
    idx = torch.from_numpy(np.sort(np.random.default_rng(3).choice(nb, 512, replace=False))).cuda()
    ys = y[2].index_select(0, idx).cpu().numpy().astype(np.float64)
    ts = tx[2].index_select(0, idx).cpu().numpy().view(np.uint32)
    cg, cm = orc.costs(ys, ts, f.X, f.labels, s2)
    # the sampled costs' mean estimates the buffer's GMI/MI within Monte-Carlo error
    se_g = np.std(cg, ddof=1) / np.sqrt(len(cg))
    assert abs((f.m - cg.mean()) - rows[2, 0]) <= 5 * se_g + 1e-9
    say(f"[stream] {name} 2^22 x 3 on 4 lanes: GMI {tot[0]:.5f}")


def test_shape_change_between_create_and_push(orc):
    """The 16-QAM format runs on the per-sample 4x4 shape by default and on
    32 x 32 tiles under variant 4; the two launch different block counts.
    Streams created under one and pushed under the other stay within their
    workspaces and agree with the oracle."""
    f = w.format_16qam()
    gf = mdgmi.Format.of(f)
    s2 = float(w.sigma2_from_snr_db(8.0, 2))
    bufs = buffers(f, s2, [4096, 4096, 1500], seed=13)
    ref = orc.gmi(np.concatenate([b[0] for b in bufs]).astype(np.float64), np.concatenate([b[1] for b in bufs]),
                  f.X, f.labels, s2)
    try:
        for first, then in ((-1, 4), (4, -1)):
            mdgmi.mdgmi_set_tuning(first)
            st = mdgmi.Stream(gf, s2, 4096, n_lanes=2, path="mfma")
            mdgmi.mdgmi_set_tuning(then)
            for y, tx in bufs:
                st.push(torch.from_numpy(y).cuda(), torch.from_numpy(tx.view(np.int32)).cuda())
            tot = st.total()
            st.close()
            assert tot[4] == sum(len(b[0]) for b in bufs) and tot[5] == 0
            assert np.max(np.abs(tot[:2] - ref[:2])) <= 1e-4
            say(f"[stream] shape {first} -> {then}: GMI {tot[0]:.6f} vs oracle {ref[0]:.6f}")
    finally:
        mdgmi.mdgmi_set_tuning(-1)
