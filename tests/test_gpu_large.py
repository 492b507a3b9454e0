"""GPU parity at full workload sizes and the workloads' own iteration counts.

Expected values come from ``tests/golden/full_size_*.json``, written by
``tests/golden/make_full_size.py`` from the FP64 oracle on the same seeded
inputs (each record carries a digest of its inputs, checked here first).
Comparisons on sampled entries are normwise over the sample.

2048x2048 single pair (559k nodes): displacements after 50 iterations; the
gradient of the final MSD after 50 unrolled iterations (checkpoint 10) w.r.t.
u0, alpha and the template against the oracle's, also as projections on 64
seeded node directions; central finite differences of the GPU forward (h =
1e-3 px) along the same directions against the oracle's projections; warp at a
seeded smooth displacement on sampled pixels.

64-pair differentiable batch (512x512, per-pair alpha): gradients after 100
unrolled iterations (checkpoint 10) of four pairs against the oracle, and the
alpha gradient against GPU finite differences.

256-pair ragged batch in the launch configuration the benchmark times (graph
replay on a side stream, autotuned schedule, automatic apex): 100 iterations,
displacements of four sampled pairs of different sizes against the oracle.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj, bspline, mesh as omesh, registration as reg
from synth import make_pair, make_pairs, random_directions

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def pkg():
    import paper_1411_2141_amd
    return paper_1411_2141_amd


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def check_inputs(rec, p):
    from tests.golden.make_full_size import input_digest
    assert rec["digest"] == input_digest(p), "inputs differ from those the expected values were made on"


def at(rec, key, shape=(-1, 2)):
    return np.asarray(rec[key], dtype=np.float64).reshape(shape)


@pytest.fixture(scope="module")
def c3():
    say("building the 2048^2 pair")
    p = make_pair(3)
    ctx = pkg().MeshReg([p], tau=0.5)
    yield p, ctx
    ctx.close()


def smooth_u(V, H, W, amp, seed):
    """A seeded smooth displacement field sampled at the nodes (input only)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, (2, 3, 3))
    x, y = V[:, 0] / W, V[:, 1] / H
    u = np.zeros((V.shape[0], 2))
    for c in range(2):
        for p in range(3):
            for q in range(3):
                u[:, c] += a[c, p, q] * np.sin((p + 1) * np.pi * x) * np.sin((q + 1) * np.pi * y)
    return u


def test_c3_run_parity_50_iterations(c3):
    p, ctx = c3
    rec = golden("full_size_2048.json")
    check_inputs(rec, p)
    N = rec["n_iter"]
    say(f"c3 run parity: {p.n_nodes} nodes, {N} iterations")
    u = ctx.zeros_u()
    ctx.step(u, N)
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    idx = np.asarray(rec["node_index"])
    err = rel(ug[idx], at(rec, "u_at_nodes"))
    say(f"c3 u after {N}: sampled relative error {err:.2e}, norm {np.linalg.norm(ug):.6e} "
        f"(oracle {rec['u_norm']:.6e})")
    assert err < 1e-5
    assert abs(np.linalg.norm(ug) - rec["u_norm"]) <= 1e-5 * rec["u_norm"]


def test_c3_warp_on_sampled_pixels(c3):
    p, ctx = c3
    say("c3 warp parity on sampled pixels")
    H, W = p.height, p.width
    u = smooth_u(p.V, H, W, 6.0, seed=31)
    msd, warped = ctx.warp_msd(dev(u), return_warped=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    ii = rng.integers(0, H, 4000)
    jj = rng.integers(0, W, 4000)
    # oracle: locate each sampled pixel centre by the exact containment test
    t6 = omesh.table_t6(p.V, p.T, H, W)
    tri = t6[ii, jj]
    w = omesh.barycentric(p.V, p.T, tri, 2 * jj + 1, 2 * ii + 1)
    up = (w[:, :, None] * u[p.T[tri]]).sum(axis=1)
    c = bspline.prefilter(p.te.astype(np.float64))
    want = bspline.evaluate(c, jj + up[:, 0], ii + up[:, 1])[0]
    got = warped.cpu().numpy().reshape(H, W)[ii, jj]
    assert np.abs(got - want).max() < 2e-6 * max(1.0, np.abs(want).max())
    assert np.isfinite(msd.item())


def test_c3_gradient_against_oracle_50_iterations(c3):
    p, ctx = c3
    rec = golden("full_size_2048.json")
    check_inputs(rec, p)
    N, ck = rec["n_iter"], rec["ckpt_every"]
    say(f"c3 gradient vs oracle (N={N}, checkpoint {ck})")
    msd, g_u0, g_alpha, g_te = ctx.backward(ctx.zeros_u(), N, ck)
    torch.cuda.synchronize()
    g = g_u0.cpu().numpy()
    gt = g_te.cpu().numpy()
    idx, pix = np.asarray(rec["node_index"]), np.asarray(rec["pixel_index"])
    e_u = rel(g[idx], at(rec, "g_u0_at_nodes"))
    e_te = rel(gt[pix], at(rec, "g_te_at_pixels", (-1,)))
    e_a = abs(g_alpha.item() - rec["g_alpha"]) / abs(rec["g_alpha"])
    proj = np.array([float(np.sum(g * d)) for d in random_directions(p.n_nodes, 64, rec["direction_seed"])])
    e_p = rel(proj, rec["projections"])
    say(f"c3 gradient errors: u0 {e_u:.2e}, te {e_te:.2e}, alpha {e_a:.2e}, 64 projections {e_p:.2e}, "
        f"msd {abs(msd.item() - rec['msd']) / rec['msd']:.2e}")
    assert abs(msd.item() - rec["msd"]) <= 1e-5 * rec["msd"]
    assert e_u < 1e-4 and e_te < 1e-4 and e_a < 1e-4 and e_p < 1e-4
    assert abs(np.linalg.norm(g) - rec["g_u0_norm"]) <= 1e-4 * rec["g_u0_norm"]
    assert abs(np.linalg.norm(gt) - rec["g_te_norm"]) <= 1e-4 * rec["g_te_norm"]


def test_c3_central_differences_against_oracle_64_directions(c3):
    """Central differences of the GPU forward along the 64 seeded directions
    against the oracle's directional derivatives.  The forward samples and
    warps in FP32, so a difference quotient at h = 1e-3 px carries an absolute
    noise floor: each warped pixel W_p is rounded to ~delta = 2^-22 (FP32 tap
    sums of coefficients of magnitude ~1), and the loss difference
    (2/P) sum_p e_p (W_p(+h) - W_p(-h)) then carries ~2 e_rms delta / sqrt(P),
    i.e. eta = 2 sqrt(MSD) delta / (sqrt(P) 2h) in the quotient.  Each
    direction must agree to 5e-3 relative plus 5 eta, and the 64 together to
    5e-3 normwise."""
    p, ctx = c3
    rec = golden("full_size_2048.json")
    check_inputs(rec, p)
    N, h = rec["n_iter"], rec["fd_step_px"]
    say(f"c3 central differences on 64 directions vs oracle (N={N}, h={h} px)")
    u = ctx.zeros_u()

    def loss(v):
        u.copy_(dev(v))
        ctx.step(u, N)
        return ctx.warp_msd(u).item()

    fd = np.array([(loss(h * d) - loss(-h * d)) / (2 * h)
                   for d in random_directions(p.n_nodes, 64, rec["direction_seed"])])
    want = np.asarray(rec["projections"])
    eta = 2.0 * np.sqrt(rec["msd"]) * 2.0 ** -22 / (np.sqrt(p.height * p.width) * 2 * h)
    err = np.abs(fd - want)
    say(f"c3 FD vs oracle: normwise {rel(fd, want):.2e}, per direction median "
        f"{np.median(err / np.abs(want)):.2e}, worst (err - 5e-3 |p|) / eta "
        f"{np.max((err - 5e-3 * np.abs(want)) / eta):.2f} (eta {eta:.2e})")
    assert rel(fd, want) < 5e-3
    assert np.all(err <= 5e-3 * np.abs(want) + 5 * eta)


def test_c5_batched_gradients_on_four_pairs():
    rec = golden("full_size_diff_batch.json")
    N, ck = rec["pairs"][0]["n_iter"], rec["ckpt_every"]
    say(f"c5: 4 pairs of the 64-pair differentiable batch, N={N}, checkpoint {ck}")
    pairs = [make_pair(5, r["pair_index"]) for r in rec["pairs"]]
    for r, q in zip(rec["pairs"], pairs):
        check_inputs(r, q)
    assert len({round(q.alpha, 12) for q in pairs}) == 4
    ctx = pkg().MeshReg(pairs, tau=0.5)
    msd, g_u0, g_alpha, g_te = ctx.backward(ctx.zeros_u(), N, ck)
    torch.cuda.synchronize()
    gu_all, gt_all = g_u0.cpu().numpy(), g_te.cpu().numpy()
    for k, (r, q) in enumerate(zip(rec["pairs"], pairs)):
        gu = gu_all[ctx.node_offsets[k]:ctx.node_offsets[k + 1]]
        gt = gt_all[ctx.pixel_offsets[k]:ctx.pixel_offsets[k + 1]]
        idx, pix = np.asarray(r["node_index"]), np.asarray(r["pixel_index"])
        e_u = rel(gu[idx], at(r, "g_u0_at_nodes"))
        e_te = rel(gt[pix], at(r, "g_te_at_pixels", (-1,)))
        e_a = abs(g_alpha[k].item() - r["g_alpha"]) / abs(r["g_alpha"])
        say(f"c5 pair {k}: u0 {e_u:.2e}, te {e_te:.2e}, alpha {e_a:.2e}, "
            f"msd {abs(msd[k].item() - r['msd']) / r['msd']:.2e}")
        assert abs(msd[k].item() - r["msd"]) <= 1e-5 * r["msd"]
        assert e_u < 1e-4 and e_te < 1e-4 and e_a < 1e-4
        assert abs(np.linalg.norm(gu) - r["g_u0_norm"]) <= 1e-4 * r["g_u0_norm"]
        assert abs(np.linalg.norm(gt) - r["g_te_norm"]) <= 1e-4 * r["g_te_norm"]
    # alpha: GPU central differences per pair (relative step 1e-3)
    for k, q in enumerate(pairs):
        ha = 1e-3 * q.alpha
        vals = []
        for a in (q.alpha + ha, q.alpha - ha):
            ctx.set_alpha(k, a)
            u = ctx.zeros_u()
            ctx.step(u, N)
            vals.append(ctx.warp_msd(u)[k].item())
        ctx.set_alpha(k, q.alpha)
        fd = (vals[0] - vals[1]) / (2 * ha)
        assert abs(fd - g_alpha[k].item()) <= 2e-2 * abs(g_alpha[k].item()), (k, fd, g_alpha[k].item())
    ctx.close()


def test_c4_full_batch_sampled_pairs():
    rec = golden("full_size_batch.json")
    N = rec["pairs"][0]["n_iter"]
    say(f"c4: 256 ragged pairs, graph replay, {N} iterations, 4 sampled pairs vs oracle")
    pairs = make_pairs(4, rec["n_pairs_in_batch"], processes=8)
    for r in rec["pairs"]:
        check_inputs(r, pairs[r["pair_index"]])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ctx = pkg().MeshReg(pairs, tau=0.5, graph=True)
        u = ctx.zeros_u()
        pkg().binding.mesh_reg_step(ctx.ctx, u, N, None, side.cuda_stream)   # capture + replay
        u.zero_()
        pkg().binding.mesh_reg_step(ctx.ctx, u, N, None, side.cuda_stream)   # replay
        msd = ctx.warp_msd(u)
        side.synchronize()
        ug = u.cpu().numpy()
    for r in rec["pairs"]:
        k = r["pair_index"]
        uk = ug[ctx.node_offsets[k]:ctx.node_offsets[k + 1]]
        err = rel(uk[np.asarray(r["node_index"])], at(r, "u_at_nodes"))
        say(f"c4 pair {k} (side {r['height']}): sampled u error {err:.2e}, "
            f"msd {abs(msd[k].item() - r['msd']) / r['msd']:.2e}")
        assert err < 1e-5, (k, err)
        assert abs(np.linalg.norm(uk) - r["u_norm"]) <= 1e-5 * r["u_norm"]
    ctx.close()
