"""The C-ABI library loads, exports every symbol include/mdgmi.h declares, and
its host-only entry points behave (no GPU needed)."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_2011_13695_amd import mdgmi


def test_library_exports_every_declared_symbol():
    names = mdgmi.declared_functions()
    assert {"mdgmi_llr", "mdgmi_gmi", "mdgmi_generate", "mdgmi_format_create"} <= set(names)
    L = mdgmi.lib()
    for fn in names:
        assert hasattr(L, fn), fn
    out = subprocess.run(["nm", "-D", "--defined-only", str(mdgmi.LIB_PATH)], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported


def test_library_carries_gfx950_code_object():
    """The fat binary built here holds a gfx950 device code object."""
    data = mdgmi.LIB_PATH.read_bytes()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_status_strings():
    for code in range(0, -10, -1):
        s = mdgmi.mdgmi_status_string(code)
        assert s and s != "unknown status"
    assert mdgmi.mdgmi_status_string(123) == "unknown status"


def test_validate_labels_host_only():
    assert mdgmi.mdgmi_validate_labels(np.arange(16)[::-1]) == mdgmi.MDGMI_OK
    assert mdgmi.mdgmi_validate_labels([0, 1, 1, 3]) == mdgmi.MDGMI_E_LABELS
    assert mdgmi.mdgmi_validate_labels([0, 1, 2, 4]) == mdgmi.MDGMI_E_LABELS
    L = mdgmi.lib()
    assert L.mdgmi_validate_labels(None, 4) == mdgmi.MDGMI_E_NULL
    lab = np.arange(4, dtype=np.uint32)
    assert L.mdgmi_validate_labels(lab.ctypes.data_as(ctypes.c_void_p), 0) == mdgmi.MDGMI_E_SHAPE


def test_format_create_rejects_bad_arguments_before_touching_the_device():
    L = mdgmi.lib()
    P = ctypes.c_void_p
    X = np.zeros((8, 2))
    lab = np.arange(8, dtype=np.uint32)
    h = P()
    assert L.mdgmi_format_create(None, lab.ctypes.data_as(P), 8, 2, ctypes.byref(h)) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_format_create(X.ctypes.data_as(P), lab.ctypes.data_as(P), 8, 3, ctypes.byref(h)) == mdgmi.MDGMI_E_SHAPE
    assert L.mdgmi_format_create(X.ctypes.data_as(P), lab.ctypes.data_as(P), 6, 2, ctypes.byref(h)) == mdgmi.MDGMI_E_SHAPE
    bad = lab.copy()
    bad[3] = 1
    assert L.mdgmi_format_create(X.ctypes.data_as(P), bad.ctypes.data_as(P), 8, 2, ctypes.byref(h)) == mdgmi.MDGMI_E_LABELS
    Xn = X.copy()
    Xn[2, 1] = np.nan
    assert L.mdgmi_format_create(Xn.ctypes.data_as(P), lab.ctypes.data_as(P), 8, 2, ctypes.byref(h)) == mdgmi.MDGMI_E_ARG


def test_null_handles_rejected():
    L = mdgmi.lib()
    b = ctypes.c_size_t()
    assert L.mdgmi_gmi_workspace_size(None, 10, 1, 1, ctypes.byref(b)) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_llr(None, None, 10, 1.0, None, 1, None, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_format_destroy(None) == mdgmi.MDGMI_E_NULL


def test_new_entry_points_reject_bad_arguments_host_side():
    """Checks that return before any device call (no GPU needed)."""
    L = mdgmi.lib()
    mdgmi._stream_sigs()
    P = ctypes.c_void_p
    b = ctypes.c_size_t()
    assert L.mdgmi_gmi_sopt_workspace_size(0, ctypes.byref(b)) == mdgmi.MDGMI_E_SHAPE
    assert L.mdgmi_gmi_sopt_workspace_size(10, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_bits_workspace_size(0, ctypes.byref(b)) == mdgmi.MDGMI_E_SHAPE
    assert L.mdgmi_gmi_bits_workspace_size(10, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_sopt(None, None, 0, None, 10, None, None, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_bits(None, None, 0, None, 10, None, None, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_hd_workspace_size(None, 10, 1, 1, ctypes.byref(b)) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_hd(None, None, None, 10, None, 1, 1, None, None, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_gmi_maxlog(None, None, None, 10, None, 1, 1, None, None, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_llr_maxlog(None, None, 10, 1.0, None, 1, None, 0, None) == mdgmi.MDGMI_E_NULL
    h = P()
    assert L.mdgmi_stream_create(None, 1.0, 10, 1, 1, 4, ctypes.byref(h)) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_stream_push(None, None, None, 10, 0, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_stream_wait(None, 0) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_stream_total(None, None) == mdgmi.MDGMI_E_NULL
    assert L.mdgmi_stream_destroy(None) == mdgmi.MDGMI_E_NULL


def test_bench_refuses_several_gpus_and_interpolates_q_thresholds():
    import json
    import sys

    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                         cwd=str(mdgmi.LIB_PATH.parents[1]), timeout=120)
    assert out.returncode == 2
    assert "single-GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]
    sys.path.insert(0, str(mdgmi.LIB_PATH.parents[1]))
    import bench
    snr = [0.0, 1.0, 2.0, 3.0]
    assert bench.q_crossing(snr, [1.0, 2.0, 3.0, 4.0], 2.5) == pytest.approx(1.5)
    assert bench.q_crossing(snr, [1.0, 2.0, None, None], 8.4) == pytest.approx(2.0)   # BER 0: Q unbounded
    assert bench.q_crossing(snr, [1.0, 2.0, 3.0, 4.0], 9.0) is None


def test_binding_checks_element_types():
    """The C ABI reads y as double on the FP64 path and float otherwise; the
    binding refuses a tensor of the other type instead of passing its bytes."""
    torch = pytest.importorskip("torch")
    y64 = torch.zeros((4, 2), dtype=torch.float64)
    y32 = torch.zeros((4, 2), dtype=torch.float32)
    tx = torch.zeros(4, dtype=torch.int32)
    mdgmi._check_y(y64, mdgmi.MDGMI_PATH_F64, tx)
    for p in (mdgmi.MDGMI_PATH_AUTO, mdgmi.MDGMI_PATH_F32_DIRECT, mdgmi.MDGMI_PATH_F32_MFMA_F16SPLIT,
              mdgmi.MDGMI_PATH_F32_MFMA_BF16SPLIT):
        mdgmi._check_y(y32, p, tx)
        with pytest.raises(TypeError):
            mdgmi._check_y(y64, p)
    with pytest.raises(TypeError):
        mdgmi._check_y(y32, mdgmi.MDGMI_PATH_F64)
    with pytest.raises(TypeError):
        mdgmi._check_y(y32, mdgmi.MDGMI_PATH_AUTO, tx.to(torch.int64))


def _tune_json(entries):
    rows = ",\n".join(
        f'  {{"dim": {d}, "M": {M}, "regime": {r}, "samples": {n}, "path": {p}, "variant": {v}, '
        f'"direct_rate": {dr:.6e}, "mfma_rate": {mr:.6e}}}' for d, M, r, n, p, v, dr, mr in entries)
    return '{"arch": "gfx950", "entries": [\n' + rows + "\n]}\n"


def test_tune_table_regimes_json_host_only(tmp_path):
    """The tuning table holds one entry per (dim, M, sample-count regime);
    it survives a save/load round trip, and the loader skips malformed
    entries (no device involved)."""
    p = tmp_path / "t.json"
    p.write_text(_tune_json([(8, 256, 0, 1 << 20, 1, -1, 2.0e12, 1.0e12),
                             (8, 256, 1, 1 << 15, 2, 4, 1.0e12, 3.0e12),
                             (4, 64, 1, 1 << 15, 2, 8, 1.0e12, 2.5e12),
                             (4, 48, 0, 1 << 20, 1, -1, 1.0e12, 0.0),      # M not a power of two
                             (2, 16, 2, 1 << 20, 1, -1, 1.0e12, 0.0)]))    # no such regime
    mdgmi.mdgmi_tune_clear()
    try:
        mdgmi.mdgmi_tune_load(p)
        bulk = mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_BULK)
        short = mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_SHORT)
        assert bulk["path"] == mdgmi.MDGMI_PATH_F32_DIRECT and bulk["samples"] == 1 << 20
        assert short["path"] == mdgmi.MDGMI_PATH_F32_MFMA_F16SPLIT and short["mfma_variant"] == 4
        assert short["regime"] == mdgmi.MDGMI_TUNE_SHORT and short["samples"] == 1 << 15
        assert mdgmi.mdgmi_tune_lookup(4, 64, mdgmi.MDGMI_TUNE_BULK) is None
        assert mdgmi.mdgmi_tune_lookup(4, 64, mdgmi.MDGMI_TUNE_SHORT)["mfma_variant"] == 8
        assert mdgmi.mdgmi_tune_lookup(4, 48, mdgmi.MDGMI_TUNE_BULK) is None
        assert mdgmi.mdgmi_tune_lookup(2, 16, mdgmi.MDGMI_TUNE_BULK) is None
        assert mdgmi.mdgmi_tune_lookup(8, 256, 2) is None
        q = tmp_path / "u.json"
        mdgmi.mdgmi_tune_save(q)
        mdgmi.mdgmi_tune_clear()
        assert mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_SHORT) is None
        mdgmi.mdgmi_tune_load(q)
        assert mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_SHORT) == short
        assert mdgmi.mdgmi_tune_lookup(8, 256, mdgmi.MDGMI_TUNE_BULK) == bulk
        bad = tmp_path / "bad.json"
        bad.write_text(_tune_json([(3, 256, 0, 1 << 20, 1, -1, 1.0, 0.0)]))
        with pytest.raises(mdgmi.MdgmiError):
            mdgmi.mdgmi_tune_load(bad)
    finally:
        mdgmi.mdgmi_tune_clear()


def test_probe_rejects_null_output():
    assert mdgmi.lib().mdgmi_probe_rates(None) == mdgmi.MDGMI_E_NULL
