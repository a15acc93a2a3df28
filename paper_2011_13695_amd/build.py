"""Build libmdgmi.so (HIP, gfx950) in-tree with hipcc.

Every .hip and .cpp file under csrc/ is compiled separately (in parallel) and linked
into paper_2011_13695_amd/libmdgmi.so. Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
ROOT = PKG.parent
BUILD = ROOT / "_build" / "mdgmi"
LIB = PKG / "libmdgmi.so"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
    f"-I{ROOT / 'include'}",
]

# Per-file flags. The 4x4-block MFMA shape keeps its accumulators in
# ordinary VGPRs: the exponentials read every MFMA result, and AGPR results
# would cost one extra v_accvgpr_read per (sample, point).
EXTRA_FLAGS = {name: ["-mllvm", "-amdgpu-mfma-vgpr-form"] for name in ("exact_mfma4.hip", "batch_small.hip")}


def sources():
    """HIP sources, plus the host-only C++ ones (no device code)."""
    return sorted([*CSRC.glob("*.hip"), *CSRC.glob("*.cpp")])


def _compile(src: Path, incremental: bool = False) -> Path:
    obj = BUILD / (src.stem + ".o")
    if incremental and obj.exists():
        newest = max(p.stat().st_mtime for p in [src, *CSRC.glob("*.h"), ROOT / "include" / "mdgmi.h"])
        if obj.stat().st_mtime > newest:
            return obj
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(src.name, []), "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature: drop that warning
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err.strip():
        print(err, file=sys.stderr)
    return obj


def build(jobs: int | None = None, incremental: bool = False) -> Path:
    """Compile every source (incremental: only those older than their object
    file's inputs, for development) and link the library."""
    BUILD.mkdir(parents=True, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = LIB.with_name(LIB.name + ".tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="-i" in sys.argv[1:]))
