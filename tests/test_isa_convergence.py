"""The device code keeps wave-uniform control flow around cross-lane
operations.

Kernels that broadcast a value with readfirstlane or move data between lanes
with ds_bpermute rely on every lane of the wave reaching those instructions
together. If the compiler gives a loop a per-lane (divergent) exit while such
an instruction sits inside the loop, lanes that stay behind compute with a
different set of active lanes; in the walk this once made part of a wave
re-walk the same group forever. This test compiles the library sources for
gfx950, keeps the assembly, and checks every loop whose latch narrows EXEC
for such instructions. It needs hipcc but no GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
from isa_convergence import check  # noqa: E402

SOURCES = ["walk.hip", "sort.hip", "scan.hip", "build.hip"]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
@pytest.mark.parametrize("src", SOURCES)
def test_no_convergent_op_in_divergent_loop(src, tmp_path):
    import re
    sys.path.insert(0, ROOT)
    from paper_1502_07442_amd.build import FLAGS
    flags = [f for f in FLAGS if f not in ("-shared",)]
    cmd = ["hipcc", *flags, "-c", os.path.join(ROOT, "paper_1502_07442_amd", "csrc", src), "-save-temps",
           "-o", str(tmp_path / "k.o")]
    subprocess.run(cmd, check=True, cwd=tmp_path, capture_output=True)
    asm = [f for f in os.listdir(tmp_path) if f.endswith("gfx950.s")]
    assert asm, "no device assembly produced"
    text = open(tmp_path / asm[0]).read()
    kernels = list(re.finditer(r"^(_Z\S+):\s*;", text, re.M))
    assert kernels
    for km in kernels:
        # a function's code ends at its .Lfunc_end label (a kernel at its
        # s_endpgm, an outlined device function at its return)
        end = text.find(".Lfunc_end", km.end())
        body = text[km.end(): end if end >= 0 else len(text)].splitlines()
        assert check(body) == [], f"{km.group(1)}: cross-lane op inside a divergent loop"
