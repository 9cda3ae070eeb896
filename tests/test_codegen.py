"""CPU: code generation of the hot kernels (hipcc -S for gfx950, the library's
own flags).  Guards two properties measured on the GPU to matter:

* no flat memory instructions: flat accesses count on the same wait counter as
  LDS reads, so every LDS wait of the sweeps would also wait for HBM loads
  (the batched kernels read their scenario from a table and lost 8% that way);
* no scratch (spilled registers) and at most 256 VGPRs, so two 256-thread
  blocks still fit on a CU.
"""
import re
import shutil
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

from paper_2301_12010_amd import build  # noqa: E402

PROBE = """
#include "swe_batch_kernels.hpp"
namespace swe {
template __global__ void k_stage<TileCfg<128, 16, 8>, 2, 2>(Geo, int, int);
template __global__ void k_round<TileCfg<128, 16, 8>, 2, 2, false, false, false>(BatchTables, int, int);
template __global__ void k_persistent<TileCfg<128, 16, 8>, 2, false, false, false>(BatchTables);
}
"""


def kernels(asm: str):
    """(name, body, metadata) of every kernel in an assembly listing."""
    out = []
    for m in re.finditer(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", asm, re.S):
        name, meta = m.group(1), m.group(2)
        start = asm.index(f"{name}:")
        body = asm[start:asm.index("s_endpgm", start)]
        out.append((name, body, meta))
    return out


@pytest.mark.skipif(not Path(build.HIPCC).exists() and not shutil.which("hipcc"), reason="hipcc not installed")
def test_hot_kernels_use_global_accesses_without_spills(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    out = tmp_path / "probe.s"
    flags = [f for f in build.FLAGS if f != "-fPIC"]
    cmd = [build.HIPCC, *flags, "-I", str(build.CSRC), "--cuda-device-only", "-S", str(src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    found = kernels(out.read_text())
    names = [n for n, _, _ in found]
    assert len(found) == 3 and any("k_stage" in n for n in names) and any("k_round" in n for n in names) \
        and any("k_persistent" in n for n in names), names
    for name, body, meta in found:
        flat = re.findall(r"^\s*(flat_\w+)", body, re.M)
        assert not flat, (name, sorted(set(flat)))
        scratch = int(re.search(r"\.amdhsa_private_segment_fixed_size (\d+)", meta).group(1))
        assert scratch == 0, (name, scratch)
        vgprs = int(re.search(r"\.amdhsa_next_free_vgpr (\d+)", meta).group(1))
        assert vgprs <= 256, (name, vgprs)
