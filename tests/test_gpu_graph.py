"""HIP-graph replay of mesh_reg_step against eager execution: several
replays with eager work and synchronisations between them, every replay
checked (bit-identical, since every kernel of the step is deterministic)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import make_pair
from tests._problems import small_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_graph_replays_match_eager():
    print("[gpu-case] graph replay vs eager (2 pairs, 6 iterations, MSD trace)", flush=True)
    import paper_1411_2141_amd as pkg
    te, re_, V, T, _ = small_pair(seed=1, side=48, s_min=1, s_max=16)
    p = make_pair(1)
    pairs = [dict(te=p.te, re=p.re, V=p.V, T=p.T, alpha=0.1), dict(te=te, re=re_, V=V, T=T, alpha=0.3)]
    # fixed schedules: two tuned contexts may pick different workgroup sizes,
    # which changes the rounding of the partial sums
    eager = pkg.MeshReg(pairs, tau=0.5, tune=False)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        graphed = pkg.MeshReg(pairs, tau=0.5, graph=True, tune=False)
        u = graphed.zeros_u()
        trace = torch.empty((6, 2), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(0)
    for rep in range(4):
        u0 = torch.as_tensor(rng.normal(scale=0.3, size=(eager.total_nodes, 2)), device="cuda")
        ue = u0.clone()
        te_trace = eager.step(ue, 6, record_msd=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            u.copy_(u0)
            pkg.binding.mesh_reg_step(graphed.ctx, u, 6, trace, side.cuda_stream)
        side.synchronize()
        assert torch.equal(u, ue), rep
        assert torch.equal(trace, te_trace), rep
        # unrelated eager work between replays
        eager.warp_msd(ue)
        torch.cuda.synchronize()
    eager.close()
    graphed.close()
