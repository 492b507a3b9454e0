"""The package imported before torch: the library must still run on the same
HIP runtime as torch's tensors and streams (one runtime per process).  Run in
a fresh interpreter, since this process has imported torch already."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import paper_1411_2141_amd as pkg      # before any explicit torch import
import numpy as np
import torch
from synth import uniform_mesh
V, T, _ = uniform_mesh(32, 32, 8)
yy, xx = np.mgrid[0:32, 0:32]
te = np.exp(-((xx - 15.0) ** 2 + (yy - 17.0) ** 2) / 40.0).astype(np.float32)
re = np.exp(-((xx - 16.0) ** 2 + (yy - 16.0) ** 2) / 40.0).astype(np.float32)
ctx = pkg.MeshReg([dict(te=te, re=re, V=V, T=T, alpha=0.1)], tau=0.5)
u = ctx.zeros_u()
ctx.step(u, 3)
msd = ctx.warp_msd(u)
torch.cuda.synchronize()
assert np.isfinite(msd.item()) and torch.isfinite(u).all().item()
ctx.close()
print("OK", flush=True)
"""


def test_package_imported_before_torch_runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] package imported before torch, in a child interpreter", flush=True)
    r = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0 and "OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
