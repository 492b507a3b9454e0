"""Pins for the oracle's mesh tables and P1 operators (Section 2.1 mesh,
Algorithm 1 pre-computation, eq. 9-10, Section 2.3)."""
import json
import os

import numpy as np
import pytest

from oracle import mesh
from synth import quadtree_mesh, uniform_mesh, unstructured_mesh
from synth.images import draw_params, make_images

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_adaptive(seed=0, side=64, s_min=1, s_max=16, g=0.05):
    rng = np.random.default_rng(seed)
    te, _ = make_images(draw_params(rng, side, side, 3.0, n_blobs=6))
    V, T, leaves = quadtree_mesh(te, s_min, s_max, g)
    return V, T, leaves, te


def test_one_leaf_golden():
    g = json.load(open(os.path.join(GOLDEN, "one_leaf_s4.json")))
    V, T = np.array(g["V"]), np.array(g["T"])
    tb = mesh.tables(V, T, g["height"], g["width"])
    for k in ("t1_ptr", "t1_slot", "t2_ptr", "t2_idx", "t3_ptr", "t3_idx", "t4", "t5", "t6"):
        assert np.array_equal(tb[k], np.array(g[k])), k
    assert np.array_equal(mesh.stiffness(V, T).toarray(), np.array(g["K_dense"]))
    assert np.allclose(6 * mesh.mass(V, T).toarray(), np.array(g["M_times_6_dense"]), atol=1e-13)
    assert np.allclose(3 * mesh.lumped_mass(V, T), np.array(g["m_times_3"]), atol=1e-13)


def test_eq9_equals_p1_gradient_and_exact_linear_gradient():
    """Eq. 9 as printed and the rotation formula both give the exact gradient
    of a linear function on arbitrary triangles."""
    rng = np.random.default_rng(10)
    P = rng.uniform(-10, 10, (400, 3, 2))
    cr = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - \
         (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
    P[cr < 0] = P[cr < 0][:, [0, 2, 1]]          # positive orientation
    a = rng.normal(size=(400, 2))
    c0 = rng.normal(size=400)
    f = c0[:, None] + np.einsum("tk,tvk->tv", a, P)
    g9 = mesh.eq9_gradient(P[:, 0], P[:, 1], P[:, 2], f[:, 0], f[:, 1], f[:, 2])
    assert np.abs(g9 - a).max() < 1e-9 * (1 + np.abs(a).max())
    # the rotation formula (integer areas) on integer triangles
    Pi = rng.integers(-20, 21, (400, 3, 2))
    cri = (Pi[:, 1, 0] - Pi[:, 0, 0]) * (Pi[:, 2, 1] - Pi[:, 0, 1]) - \
          (Pi[:, 1, 1] - Pi[:, 0, 1]) * (Pi[:, 2, 0] - Pi[:, 0, 0])
    keep = cri != 0
    Pi = Pi[keep]
    Pi[cri[keep] < 0] = Pi[cri[keep] < 0][:, [0, 2, 1]]
    Vi = Pi.reshape(-1, 2)
    Ti = np.arange(Vi.shape[0]).reshape(-1, 3)
    G = mesh.p1_gradients(Vi, Ti)
    fi = c0[: Pi.shape[0], None] + np.einsum("tk,tvk->tv", a[: Pi.shape[0]], Pi)
    grad_rot = np.einsum("tv,tvk->tk", fi, G)
    grad_9 = mesh.eq9_gradient(Pi[:, 0], Pi[:, 1], Pi[:, 2], fi[:, 0], fi[:, 1], fi[:, 2])
    assert np.abs(grad_rot - a[: Pi.shape[0]]).max() < 1e-10
    assert np.abs(grad_9 - grad_rot).max() < 1e-10


def test_quadtree_element_stiffness_closed_form():
    V, T, _ = uniform_mesh(8, 8, 8)        # one leaf -> two triangles
    G = mesh.p1_gradients(V, T)
    A = 0.5 * mesh.twice_areas(V, T)
    K0 = A[0] * np.einsum("ak,bk->ab", G[0], G[0])
    K1 = A[1] * np.einsum("ak,bk->ab", G[1], G[1])
    assert np.array_equal(K0, 0.5 * np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 1]]))
    assert np.array_equal(K1, 0.5 * np.array([[1, 0, -1], [0, 1, -1], [-1, -1, 2]]))


def test_stiffness_symmetric_zero_rowsum_and_energy_of_linear_fields():
    V, T, leaves, _ = small_adaptive()
    assert leaves[:, 2].min() < leaves[:, 2].max()     # really adaptive (hanging nodes)
    K = mesh.stiffness(V, T)
    Kd = K.toarray()
    assert np.array_equal(Kd, Kd.T)
    assert np.abs(Kd.sum(1)).max() == 0.0
    assert np.all(np.mod(2 * Kd, 1.0) == 0)            # multiples of 1/2, exact
    H = W = 64
    for a in ([1.0, 0.0], [0.3, -0.7]):
        u = V[:, 0] * a[0] + V[:, 1] * a[1]
        assert u @ (K @ u) == pytest.approx((a[0] ** 2 + a[1] ** 2) * W * H, rel=1e-13)
    ev = np.linalg.eigvalsh(Kd)
    assert ev[0] > -1e-10 and ev[1] > 1e-8             # PSD, null space = constants


def test_uniform_mesh_stiffness_is_five_point_laplacian():
    V, T, _ = uniform_mesh(16, 16, 2)
    K = mesh.stiffness(V, T).toarray()
    X = V[:, 0]
    Y = V[:, 1]
    key = {(int(x), int(y)): i for i, (x, y) in enumerate(V)}
    for i in range(V.shape[0]):
        x, y = int(X[i]), int(Y[i])
        if 0 < x < 16 and 0 < y < 16:
            row = K[i]
            assert row[i] == 4.0
            for dx, dy in ((2, 0), (-2, 0), (0, 2), (0, -2)):
                assert row[key[(x + dx, y + dy)]] == -1.0
            assert np.count_nonzero(row) == 5


def test_mass_and_lumped_mass():
    V, T, _, _ = small_adaptive()
    M = mesh.mass(V, T)
    one = np.ones(V.shape[0])
    assert one @ (M @ one) == pytest.approx(64 * 64, rel=1e-14)
    m = mesh.lumped_mass(V, T)
    assert np.allclose(M @ one, m, rtol=1e-14)
    assert np.array_equal(mesh.tables(V, T, 64, 64)["t5"], np.rint(6 * m).astype(np.int64))


def test_t6_brute_force_and_coverage():
    V, T, _, _ = small_adaptive(seed=3, side=32, s_max=16)
    t6 = mesh.table_t6(V, T, 32, 32)
    assert t6.min() >= 0
    V2 = 2 * V.astype(np.int64)
    for i in range(0, 32, 3):
        for j in range(32):
            p = np.array([2 * j + 1, 2 * i + 1])
            found = -1
            for t in range(T.shape[0]):
                P = V2[T[t]]
                ok = True
                for k in range(3):
                    a, b = P[k], P[(k + 1) % 3]
                    if (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0]) < 0:
                        ok = False
                if ok:
                    found = t
                    break
            assert t6[i, j] == found


def test_t6_ties_on_unit_leaves_go_to_lower_triangle():
    V, T, _ = uniform_mesh(6, 6, 1)
    t6 = mesh.table_t6(V, T, 6, 6)
    leaf = np.arange(36).reshape(6, 6)
    assert np.array_equal(t6, 2 * leaf)          # every centre is on its leaf's diagonal


def test_tables_structure():
    V, T, _, _ = small_adaptive(seed=4)
    n = V.shape[0]
    tb = mesh.tables(V, T, 64, 64)
    # T1: each triangle corner appears exactly once, under its node, in triangle order
    slots = tb["t1_slot"]
    assert np.array_equal(np.sort(slots), np.arange(3 * T.shape[0]))
    for i in range(0, n, 7):
        s = slots[tb["t1_ptr"][i]:tb["t1_ptr"][i + 1]]
        assert np.all(np.diff(s // 3) > 0)
        assert np.all(T[s // 3, s % 3] == i)
    # T3 = pattern of K (structural) and contains T2 plus the diagonal
    K = mesh.stiffness(V, T)
    K.sort_indices()
    assert np.array_equal(tb["t3_ptr"], K.indptr) and np.array_equal(tb["t3_idx"], K.indices)
    assert tb["t3_idx"].size == tb["t2_idx"].size + n
    # barycentric weights reproduce pixel centres
    H = W = 64
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    w = mesh.barycentric(V, T, tb["t6"].ravel(), 2 * jj.ravel() + 1, 2 * ii.ravel() + 1)
    assert w.min() >= 0 and np.abs(w.sum(1) - 1).max() < 1e-15
    P = V[T[tb["t6"].ravel()]].astype(float)
    assert np.abs((w[:, :, None] * P).sum(1) - np.stack([jj.ravel() + .5, ii.ravel() + .5], 1)).max() < 1e-12


def test_validate_rejects_bad_meshes():
    V, T, _ = uniform_mesh(4, 4, 2)
    mesh.validate(V, T, 4, 4)
    with pytest.raises(ValueError):
        mesh.validate(V, T[:, [0, 2, 1]], 4, 4)      # negative area
    bad = T.copy()
    bad[0, 0] = V.shape[0]
    with pytest.raises(ValueError):
        mesh.validate(V, bad, 4, 4)
    with pytest.raises(ValueError):
        mesh.validate(np.vstack([V, [[1, 1]]]), T, 4, 4)   # unreferenced node


def test_unstructured_mesh_operators_and_coverage():
    """General triangulations (irregular valence, edges in all directions):
    K symmetric with zero row sums and exact energy on linear fields, the
    mass sums to the image area, T6 covers every pixel and matches the
    brute-force lowest-id rule, including centres on shared edges."""
    rng = np.random.default_rng(4)
    te, _ = make_images(draw_params(rng, 40, 40, 3.0, n_blobs=5))
    V, T = unstructured_mesh(te, 1, 8, 0.05, seed=4)
    tb = mesh.tables(V, T, 40, 40)
    val = np.diff(tb["t2_ptr"])
    assert val.min() < 4 < val.max()                   # not a quadtree valence pattern
    P = V[T].astype(np.int64)
    d = P[:, 1] - P[:, 0]
    assert np.any((d[:, 0] != 0) & (d[:, 1] != 0) & (np.abs(d[:, 0]) != np.abs(d[:, 1])))
    K = mesh.stiffness(V, T)
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() <= 1e-14 * np.abs(Kd).max()
    assert np.abs(Kd.sum(1)).max() <= 1e-12 * np.abs(Kd).max()
    for a in ([1.0, 0.0], [0.3, -0.7]):
        u = V[:, 0] * a[0] + V[:, 1] * a[1]
        assert u @ (K @ u) == pytest.approx((a[0] ** 2 + a[1] ** 2) * 40 * 40, rel=1e-12)
    M = mesh.mass(V, T)
    one = np.ones(V.shape[0])
    assert one @ (M @ one) == pytest.approx(40 * 40, rel=1e-14)
    t6 = tb["t6"]
    assert t6.min() >= 0
    V2 = 2 * V.astype(np.int64)
    ties = 0
    for i in range(0, 40, 3):
        for j in range(40):
            p = np.array([2 * j + 1, 2 * i + 1])
            hits = []
            for t in range(T.shape[0]):
                Q = V2[T[t]]
                if all((Q[(k + 1) % 3][0] - Q[k][0]) * (p[1] - Q[k][1])
                       - (Q[(k + 1) % 3][1] - Q[k][1]) * (p[0] - Q[k][0]) >= 0 for k in range(3)):
                    hits.append(t)
            assert t6[i, j] == hits[0]
            ties += len(hits) > 1
    assert ties > 0                                     # shared-edge centres were exercised
