"""Pins for the oracle's reverse-mode gradient of the final MSD: adjoint
identities of each linear piece and central finite differences of the whole
unrolled objective (eq. 1 unrolled by Algorithm 1)."""
import numpy as np
import pytest

from oracle import adjoint, bspline, mesh, registration as reg
from tests._problems import small_pair


def _problem(seed=0, side=32, alpha=0.1, tau=0.5):
    te, re, V, T, _ = small_pair(seed=seed, side=side, s_min=2, s_max=16)
    return reg.setup(te, re, V, T, alpha=alpha, tau=tau), te, re, V, T


def test_force_operator_adjoint_identity():
    pb, *_ = _problem(1)
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=(2, pb.V.shape[0]))
    fwd = (pb.M @ x) / pb.m          # f = D^-1 M h
    adj = pb.M @ (y / pb.m)          # hbar = M D^-1 fbar
    assert abs(fwd @ y - x @ adj) < 1e-12 * np.abs(fwd @ y)


def test_interpolation_and_tap_scatter_adjoint_identity():
    pb, *_ = _problem(2)
    H, W = pb.height, pb.width
    rng = np.random.default_rng(1)
    u = rng.normal(scale=0.5, size=(pb.V.shape[0], 2))
    # pixel interpolation u -> u(p) and its transpose
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    tri = pb.t6.ravel()
    w = mesh.barycentric(pb.V, pb.T, tri, 2 * jj.ravel() + 1, 2 * ii.ravel() + 1)
    z = rng.normal(size=H * W)
    up = reg.pixel_displacement(pb, u)[:, :, 0].ravel()
    back = np.zeros(pb.V.shape[0])
    for a in range(3):
        np.add.at(back, pb.T[tri, a], w[:, a] * z)
    assert abs(up @ z - u[:, 0] @ back) < 1e-11
    # spline evaluation c -> s(q) and the tap scatter
    c = rng.normal(size=(H, W))
    qx, qy = rng.uniform(-3, W + 2, 50), rng.uniform(-3, H + 2, 50)
    zz = rng.normal(size=50)
    sval = bspline.evaluate(c, qx, qy)[0]
    cbar = np.zeros((H, W))
    adjoint._scatter_taps(cbar, (H, W), qx, qy, zz)
    assert abs(sval @ zz - np.sum(c * cbar)) < 1e-11


def _loss(te, re, V, T, alpha, tau, u0, n_iter):
    pb = reg.setup(te, re, V, T, alpha=alpha, tau=tau)
    uN, _, _ = reg.run(pb, u0, n_iter)
    return reg.msd(pb, uN)


@pytest.mark.parametrize("force_mode", [reg.FORCE_P1, reg.FORCE_NODAL])
def test_gradient_matches_central_differences(force_mode):
    te, re, V, T, _ = small_pair(seed=3, side=32, s_min=2, s_max=16)
    alpha, tau, N = 0.2, 2.0, 4
    pb = reg.setup(te, re, V, T, alpha=alpha, tau=tau, force_mode=force_mode)
    rng = np.random.default_rng(4)
    u0 = rng.normal(scale=0.4, size=(V.shape[0], 2))
    L, g_u0, g_alpha, g_te = adjoint.gradient(pb, u0, N)

    def loss(te_=te, alpha_=alpha, u0_=u0):
        p = reg.setup(te_, re, V, T, alpha=alpha_, tau=tau, force_mode=force_mode)
        return reg.msd(p, reg.run(p, u0_, N)[0])

    assert loss() == pytest.approx(L, rel=1e-14)
    for k in range(3):
        d = rng.normal(size=u0.shape)
        h = 1e-4
        fd = (loss(u0_=u0 + h * d) - loss(u0_=u0 - h * d)) / (2 * h)
        assert fd == pytest.approx(np.sum(g_u0 * d), rel=1e-6, abs=1e-12)
    ha = 1e-4 * alpha
    fda = (loss(alpha_=alpha + ha) - loss(alpha_=alpha - ha)) / (2 * ha)
    assert fda == pytest.approx(g_alpha, rel=1e-6, abs=1e-12)
    dt = rng.normal(size=te.shape)
    ht = 1e-4
    fdt = (loss(te_=te.astype(float) + ht * dt) - loss(te_=te.astype(float) - ht * dt)) / (2 * ht)
    assert fdt == pytest.approx(np.sum(g_te * dt), rel=1e-6, abs=1e-12)
