"""Every device kernel of the library keeps its per-lane data in registers:
each HIP source is compiled for gfx950 to assembly with the library's own
flags, and no kernel may reserve private (scratch) memory.  Scratch turns
register arrays into memory round trips inside the innermost loops (an
element kernel indexed by a run-time node count once ran 6.6x slower that
way), so a non-zero private segment is treated as a regression."""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_1204_2586_amd import build as B

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


def _kernel_resources(src, out):
    cmd = ["hipcc"] + [f for f in B.HIPFLAGS if f != "-fPIC"] + ["--cuda-device-only", "-S",
                                                                  os.path.join(B.CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    kernels, name = {}, None
    for line in open(out):
        m = re.match(r"\s*\.amdhsa_kernel\s+(\S+)", line)
        if m:
            name = m.group(1)
        m = re.match(r"\s*\.amdhsa_private_segment_fixed_size\s+(\d+)", line)
        if m and name:
            kernels[name] = int(m.group(1))
    return kernels


def test_no_kernel_uses_scratch(tmp_path):
    srcs = [s for s in B.HIP_SOURCES if s != "hip/solver.hip"]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        found = list(ex.map(lambda s: _kernel_resources(s, str(tmp_path / (os.path.basename(s) + ".s"))), srcs))
    total = 0
    for src, kernels in zip(srcs, found):
        assert kernels, f"no kernels found in {src}"
        total += len(kernels)
        spilled = {k: v for k, v in kernels.items() if v}
        assert not spilled, (src, spilled)
    assert total > 300
