"""Device code of the 23x23 and generic paths keeps its operands in registers.

Compiles the numeric kernels of those paths to gfx950 assembly with the
library's own flags and checks that no kernel has a private (scratch) segment:
a kernel whose operand arrays the compiler could not keep in registers runs
several times slower with the same results (the generic kernel once took
0.52 -> 1.23 ms that way), which no parity test would notice.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1708_03604_amd import build as B

SOURCES = ("kernels_numeric.hip", "kernels_split.hip", "kernels_slice.hip")


def private_segments(src, tmp_path):
    out = str(tmp_path / (src + ".s"))
    cmd = [B._hipcc(), "-x", "hip", "-S", "--offload-device-only", os.path.join(B.CSRC, src), "-o", out] + B.FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    sizes, kernel = {}, None
    for line in open(out):
        m = re.match(r"\s*\.amdhsa_kernel\s+(\S+)", line)
        if m:
            kernel = m.group(1)
        m = re.match(r"\s*\.amdhsa_private_segment_fixed_size\s+(\d+)", line)
        if m and kernel:
            sizes[kernel] = int(m.group(1))
    return sizes


@pytest.mark.parametrize("src", SOURCES)
def test_no_scratch_in_numeric_kernels(src, tmp_path):
    if shutil.which(B._hipcc()) is None and not os.path.exists(B._hipcc()):
        pytest.skip("hipcc not found")
    sizes = private_segments(src, tmp_path)
    assert sizes, "no kernels found"
    assert {k: v for k, v in sizes.items() if v} == {}
