"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the FP64 oracle (serial and with OpenMP threads) and the C-ABI's format
checks and preparation (csrc/format_host.cpp, the code behind
mdgmi_validate_labels and mdgmi_format_create's argument checks), each
driven over every dimension, edge inputs and every rejected argument by a
small driver under tests/sanitize/, and the fused inference layout's index
map. A sanitizer report aborts the driver."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout}\n{r.stderr}"
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_sanitizers(tmp_path, openmp):
    exe = tmp_path / "oracle_san"
    run(["gcc", "-std=c11", *SAN, *(["-fopenmp"] if openmp else []), str(ROOT / "oracle" / "oracle.c"),
         str(ROOT / "tests" / "sanitize" / "oracle_driver.c"), "-lm", "-o", str(exe)])
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    assert "oracle driver ok" in run([str(exe)], env=env)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_format_checks_under_sanitizers(tmp_path):
    exe = tmp_path / "format_san"
    csrc = ROOT / "paper_2011_13695_amd" / "csrc"
    run(["g++", "-std=c++17", "-Wall", *SAN, f"-I{ROOT / 'include'}", f"-I{csrc}", str(csrc / "format_host.cpp"),
         str(ROOT / "tests" / "sanitize" / "format_driver.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    assert "format driver ok" in run([str(exe)], env=env)


@pytest.mark.skipif(shutil.which("g++") is None or not Path("/opt/rocm/include/hip").is_dir(),
                    reason="g++ or the HIP headers not available")
def test_fused_layout_index_map(tmp_path):
    """csrc/mlp_layout.h on the host: the inverse index map the Adam step
    writes through agrees with the whole-layout builder's forward map."""
    exe = tmp_path / "layout_san"
    csrc = ROOT / "paper_2011_13695_amd" / "csrc"
    run(["g++", "-std=c++17", "-Wall", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{csrc}",
         str(ROOT / "tests" / "sanitize" / "layout_driver.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    assert "layout driver ok" in run([str(exe)], env=env)
