"""Importing the package maps exactly one HIP runtime into the process: torch
is imported before the library is loaded, so the library's dependency on the
runtime resolves to the copy torch brought (loaded the other way round, the
system's runtime and torch's would both be mapped, and the library's calls
would not see torch's devices, streams or memory).  Checked from the
process's own memory map in a fresh interpreter; needs no GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import paper_1411_2141_amd
paths = set()
for line in open("/proc/self/maps"):
    if "libamdhip64" in line:
        paths.add(line.split()[-1])
print(len(paths), sorted(paths))
"""


@pytest.mark.skipif(not os.path.exists("/proc/self/maps"), reason="needs /proc")
def test_package_maps_one_hip_runtime():
    r = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    count = int(r.stdout.split()[0])
    assert count == 1, r.stdout
