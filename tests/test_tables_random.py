"""Randomised host checks (hypothesis): on random quadtree and unstructured
meshes of random sizes the library's tables T1-T6 equal the oracle's bit for
bit, and the oracle's operators keep their closed-form invariants (symmetric
stiffness with zero row sums, mass summing to the image area, every pixel
covered)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import paper_1411_2141_amd as pkg
from oracle import mesh as omesh
from synth import quadtree_mesh, unstructured_mesh
from synth.images import draw_params, make_images

SETTINGS = dict(max_examples=12, deadline=None,
                suppress_health_check=[HealthCheck.too_slow], derandomize=True)


def _images(seed, H, W):
    rng = np.random.default_rng(seed)
    return make_images(draw_params(rng, H, W, 3.0, n_blobs=3))


@st.composite
def meshes(draw):
    s_max = draw(st.sampled_from([4, 8, 16]))
    H = s_max * draw(st.integers(1, 4))
    W = s_max * draw(st.integers(1, 4))
    s_min = draw(st.sampled_from([s for s in (1, 2, 4) if s <= s_max]))
    g = draw(st.sampled_from([0.02, 0.05, 0.2]))
    seed = draw(st.integers(0, 10_000))
    te, re = _images(seed, H, W)
    if draw(st.booleans()):
        V, T, _ = quadtree_mesh(te, s_min, s_max, g)
    else:
        V, T = unstructured_mesh(te, s_min, s_max, g, seed=seed)
    return te, re, V, T


@settings(**SETTINGS)
@given(meshes())
def test_library_tables_match_the_oracle_on_random_meshes(m):
    te, re, V, T = m
    H, W = te.shape
    ctx = pkg.MeshReg([dict(te=te, re=re, V=V, T=T, alpha=0.1)], tau=0.5, host_only=True)
    try:
        want = omesh.tables(V, T, H, W)
        for name in ("t1_ptr", "t1_slot", "t2_ptr", "t2_idx", "t3_ptr", "t3_idx", "t4", "t5"):
            assert np.array_equal(ctx.table(0, name), want[name]), name
        assert np.array_equal(ctx.table(0, "t6").reshape(H, W), want["t6"])
        assert np.array_equal(np.sort(ctx.table(0, "perm")), np.arange(V.shape[0]))
    finally:
        ctx.close()


@settings(**SETTINGS)
@given(meshes())
def test_operator_invariants_on_random_meshes(m):
    te, _, V, T = m
    H, W = te.shape
    K = omesh.stiffness(V, T).toarray()
    M = omesh.mass(V, T).toarray()
    assert np.abs(K - K.T).max() < 1e-12
    assert np.abs(K.sum(1)).max() < 1e-12
    assert np.linalg.eigvalsh(K).min() > -1e-9
    assert abs(M.sum() - H * W) < 1e-9 * H * W
    assert abs(omesh.lumped_mass(V, T).sum() - H * W) < 1e-9 * H * W
    assert np.all(omesh.table_t6(V, T, H, W) >= 0)
