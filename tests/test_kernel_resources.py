"""Kernel resources of the gfx950 build, read from the compiler (no GPU).

No kernel of the library may spill to private (scratch) memory: a kernel that
needs scratch makes the HIP runtime allocate its backing store when the kernel
is dispatched on a queue (every worker stream of the server is a new one), and
that allocation can fail with the device full of cached blocks, aborting the
process.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2511_00735_amd import build

HIP_SOURCES = sorted(s for s in build.sources() if s.endswith(".hip"))
# bytes per lane a kernel may use (by a substring of its mangled name): none
ALLOWED = {}

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


def kernel_scratch(src, tmp_path):
    """(mangled kernel name, scratch bytes per lane) of every kernel in src."""
    out = tmp_path / (os.path.basename(src) + ".o")
    flags = [f for f in build.FLAGS if f != "-fPIC"]
    r = subprocess.run(["hipcc", *flags, "-c", src, "-o", str(out), "-Rpass-analysis=kernel-resource-usage"],
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"remark:\s+Function Name: (\S+)", r.stderr)
    scratch = [int(v) for v in re.findall(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert len(names) == len(scratch), "resource remarks not paired"
    if "__global__" in open(src).read():
        assert names, "resource remarks not found"
    return list(zip(names, scratch))


@pytest.mark.parametrize("src", HIP_SOURCES, ids=os.path.basename)
def test_no_kernel_spills_to_scratch(src, tmp_path):
    over = []
    for name, nbytes in kernel_scratch(src, tmp_path):
        allowed = max([v for k, v in ALLOWED.items() if k in name], default=0)
        if nbytes > allowed:
            over.append((name, nbytes, allowed))
    assert not over, f"kernels using scratch beyond their allowance: {over}"
