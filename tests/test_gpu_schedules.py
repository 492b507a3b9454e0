"""GPU parity of every solve schedule the library can run.

The autotuner picks, per level, one of nine level kernels (wavefront per
block with its factor data copied straight into LDS, or with 8 or 16 loads in
flight per lane, half a wavefront per block of at most 32 rows, or a
workgroup of 64 / 128 / 256 / 512 / 1024 threads per block);
``solve_kernel`` forces one of them wherever admissible.
Each schedule is checked against the FP64 oracle with and without the apex
(the explicit inverse of the top levels), with split backward panels, on a
single 512x512 pair and on a batch of ragged pairs: the solve alone (relative
1e-12) and whole iterations, whose first solve level also assembles the
right-hand side (displacements relative 1e-5).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import registration as reg
from synth import make_pair, uniform_mesh
from tests._problems import small_pair

pytestmark = pytest.mark.gpu

KERNELS = (1, 8, 16, 32, 33, 34, 64, 128, 256, 512, 1024)
SOLVE_TOL = 1e-12
U_TOL = 1e-5


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1411_2141_amd  # noqa: F401


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def as_dict(p):
    return dict(te=p.te, re=p.re, V=p.V, T=p.T, alpha=p.alpha)


@pytest.fixture(scope="module")
def batch():
    te, re_, V, T = small_pair(seed=5, side=48, s_min=1, s_max=16)[:4]
    Vr, Tr = uniform_mesh(24, 40, 4)[:2]
    t2, r2 = small_pair(seed=6, side=48)[:2]
    ds = [as_dict(make_pair(1)), dict(te=te, re=re_, V=V, T=T, alpha=0.2),
          dict(te=t2[:24, :40].copy(), re=r2[:24, :40].copy(), V=Vr, T=Tr, alpha=0.1),
          as_dict(make_pair(4, 3, side=256))]
    tau = 0.5
    pbs = [reg.setup(d["te"], d["re"], d["V"], d["T"], d["alpha"], tau) for d in ds]
    rng = np.random.default_rng(11)
    bs = [rng.normal(size=(d["V"].shape[0], 2)) for d in ds]
    x_or = [reg.solve(pb, b) for pb, b in zip(pbs, bs)]
    u_or = [reg.run(pb, None, 5)[0] for pb in pbs]
    return ds, tau, bs, x_or, u_or


@pytest.fixture(scope="module")
def single():
    d = as_dict(make_pair(2))
    tau = 0.5
    pb = reg.setup(d["te"], d["re"], d["V"], d["T"], d["alpha"], tau)
    b = np.random.default_rng(12).normal(size=(d["V"].shape[0], 2))
    return d, tau, b, reg.solve(pb, b), reg.run(pb, None, 3)[0]


@pytest.mark.parametrize("apex", [0, -1])
@pytest.mark.parametrize("kernel", KERNELS)
def test_batch_schedule(batch, kernel, apex):
    import paper_1411_2141_amd as pkg
    ds, tau, bs, x_or, u_or = batch
    say(f"batch of {len(ds)} ragged pairs, solve_kernel={kernel}, apex_rows={apex}")
    ctx = pkg.MeshReg(ds, tau=tau, solve_kernel=kernel, apex_rows=apex)
    x = ctx.solve(dev(np.concatenate(bs))).cpu().numpy()
    u = ctx.zeros_u()
    ctx.step(u, 5, record_msd=True)
    ug = u.cpu().numpy()
    for k in range(len(ds)):
        sl = slice(ctx.node_offsets[k], ctx.node_offsets[k + 1])
        assert rel(x[sl], x_or[k]) < SOLVE_TOL, (k, rel(x[sl], x_or[k]))
        assert rel(ug[sl], u_or[k]) < U_TOL, (k, rel(ug[sl], u_or[k]))
    ctx.close()


@pytest.mark.parametrize("split", [0, 16])
@pytest.mark.parametrize("kernel", KERNELS)
def test_single_pair_schedule(single, kernel, split):
    import paper_1411_2141_amd as pkg
    d, tau, b, x_or, u_or = single
    say(f"512x512 pair, solve_kernel={kernel}, bwd_split_rows={split}, no apex")
    # no apex, so every level of the tree runs through the level kernels
    ctx = pkg.MeshReg([d], tau=tau, solve_kernel=kernel, apex_rows=-1, bwd_split_rows=split)
    x = ctx.solve(dev(b)).cpu().numpy()
    assert rel(x, x_or) < SOLVE_TOL, rel(x, x_or)
    u = ctx.zeros_u()
    ctx.step(u, 3)
    assert rel(u.cpu().numpy(), u_or) < U_TOL
    ctx.close()


def test_invalid_solve_kernel_rejected():
    import paper_1411_2141_amd as pkg
    d = as_dict(make_pair(1))
    with pytest.raises(pkg.binding.MeshRegError):
        pkg.MeshReg([d], tau=0.5, solve_kernel=48)


@pytest.mark.parametrize("kernel", [0, 32, 256])
def test_separate_assembly(batch, kernel):
    """The force assembly in a launch of its own (MR_FLAG_SEPARATE_ASSEMBLY),
    autotuned or with a forced level kernel: iterations and the MSD trace
    match the oracle as in the fused form."""
    import paper_1411_2141_amd as pkg
    ds, tau, bs, x_or, u_or = batch
    say(f"batch of {len(ds)} ragged pairs, separate assembly, solve_kernel={kernel}")
    ctx = pkg.MeshReg(ds, tau=tau, solve_kernel=kernel, separate_assembly=True)
    assert ctx.info(0, "fused_assembly") == 0
    u = ctx.zeros_u()
    trace = ctx.step(u, 5, record_msd=True).cpu().numpy()
    ug = u.cpu().numpy()
    for k, d in enumerate(ds):
        sl = slice(ctx.node_offsets[k], ctx.node_offsets[k + 1])
        assert rel(ug[sl], u_or[k]) < U_TOL, (k, rel(ug[sl], u_or[k]))
        # the trace holds the MSD of each iterate: against the oracle's MSD of
        # the same displacements
        pb = reg.setup(d["te"], d["re"], d["V"], d["T"], d["alpha"], tau)
        msd_or = reg.msd(pb, ug[sl])
        assert abs(trace[4, k] - msd_or) <= 1e-6 * msd_or, (k, trace[4, k], msd_or)
    ctx.close()
    fused = pkg.MeshReg(ds, tau=tau, solve_kernel=kernel)
    assert fused.info(0, "fused_assembly") == 1
    fused.close()
