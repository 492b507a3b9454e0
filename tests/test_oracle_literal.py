"""Pins for the oracle of Algorithm 1 as printed (explicit update with the eq.
9-10 mesh gradient on the deformed mesh, eq. 11-14 umbrella smoothing)."""
import numpy as np
import scipy.sparse as sp

from oracle import literal as lit, registration as reg
from synth import uniform_mesh
from tests._problems import small_pair, unstructured_pair


def _adjacency(T, n):
    """Node adjacency from the triangles' edges (independent of table T2)."""
    T = np.asarray(T)
    r = np.concatenate([T[:, 0], T[:, 1], T[:, 1], T[:, 2], T[:, 2], T[:, 0]])
    c = np.concatenate([T[:, 1], T[:, 0], T[:, 2], T[:, 1], T[:, 0], T[:, 2]])
    A = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    A.data[:] = 1.0
    return A


def _brute_node_gradient(P, T, f):
    """Per triangle the gradient of the linear interpolant by a 3x3 solve, then
    the unsigned-area-weighted mean per node, zero-area triangles skipped."""
    n = P.shape[0]
    num = np.zeros((n, 2))
    den = np.zeros(n)
    for tri in np.asarray(T):
        Q = P[tri]
        area = 0.5 * abs((Q[1, 0] - Q[0, 0]) * (Q[2, 1] - Q[0, 1])
                         - (Q[1, 1] - Q[0, 1]) * (Q[2, 0] - Q[0, 0]))
        if area == 0.0:
            continue
        coef = np.linalg.solve(np.column_stack([Q, np.ones(3)]), f[tri])
        for v in tri:
            num[v] += area * coef[:2]
            den[v] += area
    g = np.zeros((n, 2))
    g[den > 0] = num[den > 0] / den[den > 0, None]
    return g


def test_umbrella_matrix_is_the_row_normalised_edge_adjacency():
    for V, T in [uniform_mesh(16, 16, 4)[:2], small_pair(seed=2, side=32)[2:4],
                 unstructured_pair(seed=7, side=32)[2:4]]:
        n = V.shape[0]
        A = lit.umbrella(T, n).toarray()
        E = _adjacency(T, n).toarray()
        want = E / E.sum(1, keepdims=True)
        assert np.array_equal(A != 0, E != 0)
        assert np.abs(A - want).max() < 1e-15
        assert np.abs(A.sum(1) - 1.0).max() < 1e-14


def test_node_gradient_against_triangle_solves_on_a_deformed_mesh():
    te, re, V, T, _ = small_pair(seed=4, side=32)
    rng = np.random.default_rng(3)
    P = V + rng.uniform(-0.2, 0.2, size=V.shape)          # deformed, no fold
    f = np.sin(0.3 * P[:, 0]) * np.cos(0.2 * P[:, 1]) + 0.01 * P[:, 0] ** 2
    g = lit.node_gradient(P, T, f)
    assert np.abs(g - _brute_node_gradient(P, T, f)).max() < 1e-11
    # a linear field has that gradient at every node, deformed mesh or not
    a = np.array([0.37, -1.25])
    gl = lit.node_gradient(P, T, P @ a + 2.0)
    assert np.abs(gl - a).max() < 1e-11
    # a collapsed triangle (its corners made collinear) is left out
    P2 = P.copy()
    t0 = T[0]
    P2[t0[2]] = 0.5 * (P2[t0[0]] + P2[t0[1]])
    g2 = lit.node_gradient(P2, T, f)
    assert np.abs(g2 - _brute_node_gradient(P2, T, f)).max() < 1e-11


def test_one_step_on_a_linear_template_is_closed_form():
    """Te = a x + b (pixel-centre samples), Re flat at c, u = 0, lambda = 0: at
    nodes away from the border (the mirrored boundary's influence on the
    spline decays like 0.268^distance) t = a (x - 1/2) + b and the mesh
    gradient is (a, 0), so u_0 = -tau (t - c) (a, 0)."""
    H = W = 64
    a, b, c, tau = 0.02, 0.1, 0.3, 7.0
    te = np.tile(a * np.arange(W) + b, (H, 1))
    re = np.full((H, W), c)
    V, T, _ = uniform_mesh(H, W, 4)
    pb = reg.setup(te, re, V, T, alpha=0.0, tau=1.0)
    u1 = lit.step(pb, np.zeros((V.shape[0], 2)), tau, 0.0)
    inner = (V[:, 0] >= 24) & (V[:, 0] <= W - 24) & (V[:, 1] >= 8) & (V[:, 1] <= H - 8)
    want_x = -tau * (a * (V[inner, 0] - 0.5) + b - c) * a
    assert inner.sum() > 20
    assert np.abs(u1[inner, 0] - want_x).max() < 1e-12
    assert np.abs(u1[inner, 1]).max() < 1e-12


def test_identical_images_only_smooth():
    te, re, V, T, _ = small_pair(seed=5, side=32)
    pb = reg.setup(te, te, V, T, alpha=0.0, tau=1.0)
    n = V.shape[0]
    u = np.random.default_rng(0).normal(scale=0.05, size=(n, 2))
    E = _adjacency(T, n)
    S = 0.2 * sp.identity(n) + 0.8 * sp.diags(1.0 / np.asarray(E.sum(1)).ravel()) @ E
    # one step from u = 0 stays at 0 (the samples equal the reference)
    u0, _ = lit.run(pb, None, 3, 20.0, 0.8)
    assert np.abs(u0).max() < 1e-12
    # a flat template: no force, u only smoothed
    pf = reg.setup(np.full_like(te, 0.4), re, V, T, alpha=0.0, tau=1.0)
    got = lit.step(pf, u, 20.0, 0.8)
    assert np.abs(got - S @ u).max() < 1e-14
    # constants are kept
    c = np.tile([0.3, -0.7], (n, 1))
    assert np.abs(lit.step(pf, c, 20.0, 0.8) - c).max() < 1e-14


def test_explicit_run_lowers_the_msd_at_a_stable_step():
    te, re, V, T, _ = small_pair(seed=1, side=48, s_min=1, s_max=16)
    pb = reg.setup(te, re, V, T, alpha=0.0, tau=1.0)
    m0 = reg.msd(pb, np.zeros((V.shape[0], 2)))
    _, ms = lit.run(pb, None, 20, 20.0, 0.8, record_msd=True)
    assert ms[-1] < 0.8 * m0


def test_division_free_form_of_the_node_gradient_equals_eq9_eq10():
    """The kernel's form of eq. 9-10: with cr the doubled signed area and
    S = sum_v t_v R(P_{v+2} - P_{v+1}), R(x, y) = (-y, x), the node mean is
    sum sign(cr) S / sum |cr|.  Checked against the oracle (eq. 9 as printed,
    unsigned areas) on a deformed mesh with folded triangles."""
    te, re, V, T, _ = small_pair(seed=6, side=32)
    rng = np.random.default_rng(11)
    P = V + rng.uniform(-1.5, 1.5, size=V.shape)          # large enough to fold some
    f = np.cos(0.2 * P[:, 0]) + 0.1 * P[:, 1]
    T = np.asarray(T)
    Q = P[T]                                              # [nT][3][2]
    cr = ((Q[:, 1, 0] - Q[:, 0, 0]) * (Q[:, 2, 1] - Q[:, 0, 1])
          - (Q[:, 1, 1] - Q[:, 0, 1]) * (Q[:, 2, 0] - Q[:, 0, 0]))
    assert (cr < 0).any() and (cr > 0).any()
    S = np.zeros((T.shape[0], 2))
    for v in range(3):
        a, b = (v + 1) % 3, (v + 2) % 3
        d = Q[:, b] - Q[:, a]
        S[:, 0] -= f[T[:, v]] * d[:, 1]
        S[:, 1] += f[T[:, v]] * d[:, 0]
    num = np.zeros((V.shape[0], 2))
    den = np.zeros(V.shape[0])
    for v in range(3):
        np.add.at(num, T[:, v], np.sign(cr)[:, None] * S)
        np.add.at(den, T[:, v], np.abs(cr))
    g = num / den[:, None]
    assert np.abs(g - lit.node_gradient(P, T, f)).max() < 1e-9 * max(1.0, np.abs(g).max())
