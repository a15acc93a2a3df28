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
