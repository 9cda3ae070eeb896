"""Build libswe.so (HIP, gfx950) in-tree with hipcc.

Every ``csrc/*.hip`` source is compiled to an object under ``_build/`` and
linked into ``paper_2301_12010_amd/libswe.so``.  ``csrc/calib/valu_calib.hip``
(the benchmark's vector-ALU calibration) becomes ``libswe_calib.so``.  Packed
FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "libswe.so"
CALIB_SRC = CSRC / "calib" / "valu_calib.hip"
CALIB_OUT = PKG / "libswe_calib.so"
BUILD = ROOT / "_build"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", str(ROOT / "include"), "-Wall", "-Wno-unused-function"]


def sources():
    return sorted(CSRC.glob("*.hip"))


def _compile(src: Path) -> Path:
    obj = BUILD / (src.stem + ".o")
    cmd = [HIPCC, *FLAGS, "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{r.stderr[-8000:]}")
    return obj


def _link(objs, out: Path):
    tmp = out.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp),
           *[str(o) for o in objs], "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, out)


def build(verbose: bool = True) -> Path:
    """Compile every HIP source and link libswe.so and libswe_calib.so
    (always rebuilds)."""
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs) + 1)) as ex:
        calib = ex.submit(_compile, CALIB_SRC)
        objs = list(ex.map(_compile, srcs))
        calib_obj = calib.result()
    _link([calib_obj], CALIB_OUT)
    _link(objs, OUT)
    if verbose:
        print(f"built {OUT} and {CALIB_OUT.name}")
    return OUT


if __name__ == "__main__":
    build()
