"""Pins for the oracle's iteration, solve, warp and MSD (eq. 3-8, eq. 10,
Algorithm 1, Section 1's MSD metric)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bspline, mesh, registration as reg
from synth import uniform_mesh
from tests._problems import small_pair, translation_pair


def test_force_of_constant_and_linear_density():
    te, re, V, T, _ = small_pair(seed=1, side=64, s_min=2, s_max=16)
    pb = reg.setup(te, re, V, T, alpha=0.1, tau=0.5)
    n = V.shape[0]
    h = np.tile([0.3, -1.2], (n, 1))
    f = (pb.M @ h) / pb.m[:, None]
    assert np.abs(f - h).max() < 1e-14
    # a linear density is reproduced at interior nodes of a uniform mesh
    Vu, Tu, _ = uniform_mesh(16, 16, 2)
    Mu, mu = mesh.mass(Vu, Tu), mesh.lumped_mass(Vu, Tu)
    hl = np.stack([0.5 * Vu[:, 0] - Vu[:, 1], 2.0 + 0.25 * Vu[:, 1]], 1).astype(float)
    fl = (Mu @ hl) / mu[:, None]
    inner = (Vu[:, 0] > 0) & (Vu[:, 0] < 16) & (Vu[:, 1] > 0) & (Vu[:, 1] < 16)
    assert np.abs(fl[inner] - hl[inner]).max() < 1e-13


def test_cg_matches_dense_solve_and_preserves_mean():
    te, re, V, T, _ = small_pair(seed=2, side=32, s_min=2, s_max=16)
    assert V.shape[0] <= 300
    pb = reg.setup(te, re, V, T, alpha=0.1, tau=0.5)
    b = np.random.default_rng(0).normal(size=(V.shape[0], 2))
    xd = np.linalg.solve(pb.S.toarray(), b)
    xc = reg.solve(pb, b)
    assert np.abs(xc - xd).max() < 1e-12 * np.abs(xd).max()
    assert np.abs(xc.sum(0) - b.sum(0)).max() < 1e-11          # S 1 = 1 and S symmetric


def test_constant_template_is_pure_diffusion():
    """With a flat template the force vanishes, so u^N = S^-N u^0."""
    _, _, V, T, _ = small_pair(seed=3, side=32, s_min=2, s_max=16)
    te = np.full((32, 32), 0.4, dtype=np.float32)
    pb = reg.setup(te, te, V, T, alpha=0.3, tau=0.7)
    u0 = np.random.default_rng(1).normal(size=(V.shape[0], 2))
    uN, _, _ = reg.run(pb, u0, 5)
    Sinv = np.linalg.inv(pb.S.toarray())
    ref = np.linalg.matrix_power(Sinv, 5) @ u0
    assert np.abs(uN - ref).max() < 1e-12


def test_identical_images_are_a_fixed_point():
    te, _, V, T, _ = small_pair(seed=4, side=64)
    pb = reg.setup(te, te, V, T, alpha=0.1, tau=0.5)
    u = reg.step(pb, np.zeros((V.shape[0], 2)))
    assert np.abs(u).max() < 1e-13


def test_zero_displacement_msd_is_pixel_msd():
    te, re, V, T, _ = small_pair(seed=5, side=64)
    pb = reg.setup(te, re, V, T, alpha=0.1, tau=0.5)
    want = np.mean((te.astype(float) - re.astype(float)) ** 2)
    assert reg.msd(pb, np.zeros((V.shape[0], 2))) == pytest.approx(want, rel=1e-12)


def test_integer_shift_warp_closed_form():
    """u = d (integer) warps every pixel to its shifted neighbour."""
    te, re, V, T, _ = translation_pair(side=128, shift=(0.0, 0.0))
    assert max(np.abs(te[:8]).max(), np.abs(te[:, -8:]).max()) < 1e-4 * np.abs(te).max()
    pb = reg.setup(te, re, V, T, alpha=0.1, tau=0.5)
    d = np.array([3, -2])
    W = reg.warp(pb, np.tile(d.astype(float), (V.shape[0], 1)))
    want = np.zeros((128, 128))
    # W[i][j] = Te[i + dy][j + dx]; the template is ~0 near its border
    want[2:, :125] = te[:-2, 3:]
    assert np.abs(W - want).max() < 1e-4 * np.abs(te).max()


def test_integer_translation_state_is_stationary():
    d = (2.0, -1.0)
    te, _, V, T, _ = translation_pair(side=128, shift=(0.0, 0.0))
    re = np.zeros_like(te)
    re[1:, :126] = te[:-1, 2:]                  # Re(x) = Te(x + d) exactly on the grid
    pb = reg.setup(te, re, V, T, alpha=0.5, tau=5.0)
    u = np.tile(np.array(d), (V.shape[0], 1))
    for _ in range(3):
        u = reg.step(pb, u)
    assert np.abs(u - np.array(d)).max() < 1e-9


@pytest.mark.slow
def test_translation_is_recovered():
    d = np.array([1.0, -2.0])
    te, re, V, T, _ = translation_pair(side=128, shift=tuple(d))
    pb = reg.setup(te, re, V, T, alpha=1.0, tau=20.0)
    m0 = reg.msd(pb, np.zeros((V.shape[0], 2)))
    u, _, _ = reg.run(pb, None, 200)
    assert np.abs(u - d).max() < 0.01
    assert reg.msd(pb, u) < m0 * 1e-4


def test_force_mode_nodal_uses_h_directly():
    te, re, V, T, _ = small_pair(seed=6, side=32)
    pb = reg.setup(te, re, V, T, alpha=0.1, tau=0.5, force_mode=reg.FORCE_NODAL)
    u = np.random.default_rng(2).normal(scale=0.3, size=(V.shape[0], 2))
    h, f = reg.force(pb, u)
    assert np.array_equal(h, f)
    t, gx, gy = bspline.evaluate(pb.c_te, V[:, 0] - 0.5 + u[:, 0], V[:, 1] - 0.5 + u[:, 1])
    assert np.abs(h[:, 0] - (t - pb.rho) * gx).max() < 1e-15


def test_descent_lowers_the_objective_for_small_steps():
    """The update is a proximal-gradient step on D + alpha S with the nodal
    force: for a small tau the objective decreases."""
    te, re, V, T, _ = small_pair(seed=7, side=64)
    pb = reg.setup(te, re, V, T, alpha=0.2, tau=0.05, force_mode=reg.FORCE_NODAL)

    def energy(u):
        t = reg.node_samples(pb, u)[0]
        return 0.5 * np.sum((t - pb.rho) ** 2) + 0.5 * pb.alpha * sum(
            u[:, c] @ (pb.K @ u[:, c]) for c in range(2))

    u = np.zeros((V.shape[0], 2))
    e0 = energy(u)
    for _ in range(5):
        u = reg.step(pb, u)
        e1 = energy(u)
        assert e1 <= e0 + 1e-15
        e0 = e1


def _scan_stop(msds, max_iter, check_every, rel_tol):
    """Brute force over a recorded MSD trajectory (msds[k] = MSD(u^k)): the
    first check point whose relative decrease over the last check_every
    iterations is below rel_tol (or that follows a non-positive MSD)."""
    prev = 0
    k = 0
    while k < max_iter:
        k = min(k + check_every, max_iter)
        a, b = msds[prev], msds[k]
        if not a > 0.0 or a - b < rel_tol * a:
            return k
        prev = k
    return k


@pytest.mark.parametrize("rel_tol", [0.0, 0.01, 0.02, 0.03, 1.0])
def test_run_until_stops_where_a_scan_of_the_trajectory_does(rel_tol):
    """Stopping rule of the loop to convergence against a scan of the full
    trajectory: same stop, same u, same final MSD; the last chunk is short
    (max_iter not a multiple of check_every)."""
    te, re, V, T, _ = small_pair(seed=3, side=32)
    pb = reg.setup(te, re, V, T, alpha=0.05, tau=0.5)
    max_iter, every = 38, 5
    _, ms, us = reg.run(pb, None, max_iter, record_msd=True, keep_all=True)
    msds = [reg.msd(pb, us[0])] + ms
    want = _scan_stop(msds, max_iter, every, rel_tol)
    u, iters, m_final, checks = reg.run_until(pb, None, max_iter, every, rel_tol)
    assert iters == want
    assert np.array_equal(u, us[want])
    assert m_final == msds[want]
    points = list(range(0, want, every)) + [want]      # the MSDs compared
    assert checks == [msds[k] for k in points]
    if rel_tol == 0.0:
        assert iters == max_iter          # this problem's MSD decreases throughout
    if rel_tol == 1.0:
        assert iters == every             # no chunk removes the whole misfit


def test_run_until_special_cases():
    te, re, V, T, _ = small_pair(seed=3, side=32)
    pb = reg.setup(te, re, V, T, alpha=0.05, tau=0.5)
    u0 = np.random.default_rng(1).normal(scale=0.3, size=(V.shape[0], 2))
    # no iterations: u0 and its MSD come back
    u, iters, m, checks = reg.run_until(pb, u0, 0, 4, 0.01)
    assert iters == 0 and np.array_equal(u, u0) and m == reg.msd(pb, u0) and checks == [m]
    # identical images: zero misfit from the start, so the first check stops
    pz = reg.setup(te, te, V, T, alpha=0.05, tau=0.5)
    u, iters, m, _ = reg.run_until(pz, None, 50, 4, 0.01)
    assert iters == 4 and np.abs(u).max() < 1e-12 and m < 1e-20
