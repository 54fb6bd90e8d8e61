"""The binding and torch share one HIP runtime (no GPU needed).

torch's wheel ships its own libamdhip64 with the system runtime's soname.  The
binding imports torch before it loads libpp.so, so the library's dependency on
libamdhip64.so.7 resolves to torch's copy, even in a process that loads the
library before anything else touches torch (as build() then smoke() does).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1907_00072_amd", "_lib", "libpp.so")

PROBE = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_1907_00072_amd import binding   # no torch import before this point
binding.lib()
import torch
maps = open("/proc/self/maps").read().splitlines()
hip = sorted({l.split()[-1] for l in maps if "libamdhip64" in l})
print("\n".join(hip))
"""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpp.so not built")
def test_library_binds_to_torchs_hip_runtime():
    out = subprocess.run([sys.executable, "-c", PROBE, ROOT], capture_output=True, text=True,
                         timeout=300, check=True).stdout.split()
    assert len(out) == 1, out                      # one HIP runtime mapped, not two
    import torch
    assert os.path.dirname(out[0]) == os.path.join(os.path.dirname(torch.__file__), "lib")
