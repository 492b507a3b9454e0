"""The allocation-free warp + MSD entry point (mesh_reg_warp_msd_noalloc)
against mesh_reg_warp_msd on the same displacements: two calls in a row on
different contexts, the second with a smaller input (fewer pixel tiles), so
the second reads a static scratch that still holds the first call's partial
sums beyond its own tiles."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import make_pair

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def smooth_u(ctx, pairs, amp, seed):
    rng = np.random.default_rng(seed)
    out = []
    for p in pairs:
        a = rng.uniform(-amp, amp, (2, 2, 2))
        x, y = p.V[:, 0] / p.width, p.V[:, 1] / p.height
        u = np.zeros((p.n_nodes, 2))
        for c in range(2):
            for i in range(2):
                for j in range(2):
                    u[:, c] += a[c, i, j] * np.sin((i + 1) * np.pi * x) * np.sin((j + 1) * np.pi * y)
        out.append(u)
    return torch.as_tensor(np.concatenate(out), device="cuda")


def test_noalloc_warp_msd_matches_the_allocating_entry_point_twice():
    import paper_1411_2141_amd as pkg
    B = pkg.binding
    big = [make_pair(2), make_pair(1)]
    small = [make_pair(1, 1)]
    for k, pairs in enumerate((big, small)):
        say(f"noalloc call {k}: {len(pairs)} pairs, {sum(p.height * p.width for p in pairs)} pixels")
        ctx = pkg.MeshReg(pairs, tau=0.5)
        u = smooth_u(ctx, pairs, 3.0, seed=40 + k)
        msd_ref, w_ref = ctx.warp_msd(u, return_warped=True)
        msd = torch.empty(len(pairs), dtype=torch.float64, device="cuda")
        warped = torch.empty_like(w_ref)
        stream = torch.cuda.current_stream().cuda_stream
        B.mesh_reg_warp_msd_noalloc(ctx.ctx, u, msd, warped, stream)
        torch.cuda.synchronize()
        assert torch.equal(msd, msd_ref), (msd, msd_ref)
        assert torch.equal(warped, w_ref)
        msd2 = torch.empty_like(msd)
        B.mesh_reg_warp_msd_noalloc(ctx.ctx, u, msd2, None, stream)   # without the image
        torch.cuda.synchronize()
        assert torch.equal(msd2, msd_ref)
        ctx.close()
