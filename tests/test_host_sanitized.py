"""The library's host pre-computation (tables, operators, nested dissection,
Cholesky factor, block schedule, apex inverse), built with g++ and the address
and undefined-behaviour sanitizers, on quadtree, unstructured and uniform
meshes: the triangular solves carried out on the CPU the way the device
schedule prescribes reproduce (I + tau alpha K)^-1 b to 1e-12, with and
without an apex and after a numeric refactorisation.  Any sanitizer report
fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import uniform_mesh
from tests._problems import small_pair, unstructured_pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1411_2141_amd", "csrc")


@pytest.fixture(scope="module")
def plan_check(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("host") / "plan_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           os.path.join(SRC, "host_mesh.cpp"), os.path.join(SRC, "host_factor.cpp"),
           "-o", out, "-lpthread"]
    subprocess.run(cmd, check=True, timeout=600)
    return out


def _write_mesh(path, V, T, H, W):
    V = np.ascontiguousarray(V, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.int32)
    with open(path, "wb") as f:
        np.array([H, W, V.shape[0], T.shape[0]], dtype=np.int32).tofile(f)
        V.tofile(f)
        T.tofile(f)


MESHES = {
    "quadtree_128": lambda: (small_pair(seed=1, side=128, s_min=1, s_max=16)[2:4], 128, 128),
    "unstructured_64": lambda: (unstructured_pair(seed=7, side=64)[2:4], 64, 64),
    "uniform_96x64": lambda: (uniform_mesh(64, 96, 2)[:2], 64, 96),
}


@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("apex", [0, 1 << 30])
def test_schedule_solves_the_system_under_sanitizers(plan_check, tmp_path, mesh, apex):
    (V, T), H, W = MESHES[mesh]()
    path = str(tmp_path / "mesh.bin")
    _write_mesh(path, V, T, H, W)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([plan_check, path, "0.5", "0.2", "1.3", str(apex)], capture_output=True,
                       text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    fields = r.stdout.split()
    res, res2 = float(fields[fields.index("residual") + 1]), float(fields[-1])
    assert res < 1e-12 and res2 < 1e-12, r.stdout
    apex_rows = int(fields[fields.index("apex_rows") + 1])
    assert (apex_rows > 0) == (apex > 0), r.stdout
