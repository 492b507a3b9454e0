"""Reverse-mode gradient of ``L = MSD(u^N)`` through ``N`` iterations, in FP64.

Differentiates the objective of eq. 1 as unrolled by Algorithm 1 (in its
semi-implicit form) with respect to the initial displacements ``u^0``, the
regularisation weight ``alpha`` and the template intensities ``Te``.

For ``u^{k+1} = S^-1 b^k``, ``b^k = u^k - tau D^-1 M h(u^k)`` (``D = diag(m)``),
``h_i = r_i g_i`` and ``S = I + tau alpha K``:

* warp: ``lambda^N_v = (2/P) sum_p e_p w_v(p) grad s(q_p)`` and
  ``cbar += (2/P) sum_p e_p beta(x) beta(y)`` at ``q_p = x_p - 1/2 + u^N(p)``;
* step ``k`` (from ``N-1`` down to 0):
  ``mu = S^-1 lambda^{k+1}``;
  ``gbar_alpha -= tau sum_c mu_c^T K u_c^{k+1}``;
  ``eta = -tau M (mu / m)``;
  ``lambda^k_i = mu_i + (g_i . eta_i) g_i + r_i H_i eta_i``;
  ``cbar += (eta_i . g_i) beta beta + r_i (eta_ix beta' beta + eta_iy beta beta')``
  at node ``i``'s taps;
* ``gbar_Te = B^-1 cbar`` (the prefilter is symmetric, hence self-adjoint).
"""
from __future__ import annotations

import numpy as np

from . import bspline, mesh
from .registration import FORCE_NODAL, Problem, cg, node_samples, run


def _scatter_taps(cbar, shape, x, y, coef_v, coef_x=None, coef_y=None):
    rows, cols, wv, wx, wy = bspline.tap_weights(shape, x, y)
    val = coef_v[:, None] * wv
    if coef_x is not None:
        val = val + coef_x[:, None] * wx + coef_y[:, None] * wy
    np.add.at(cbar, (rows.ravel(), cols.ravel()), val.ravel())


def warp_adjoint(pb: Problem, u: np.ndarray):
    """``(lambda^N, cbar_warp, msd)`` for ``L = MSD(u)``."""
    H, W = pb.height, pb.width
    P = H * W
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    tri = pb.t6.ravel()
    w = mesh.barycentric(pb.V, pb.T, tri, 2 * jj.ravel() + 1, 2 * ii.ravel() + 1)
    nodes = pb.T[tri]
    up = (w[:, :, None] * u[nodes]).sum(axis=1)
    qx = jj.ravel() + up[:, 0]
    qy = ii.ravel() + up[:, 1]
    val, gx, gy = bspline.evaluate(pb.c_te, qx, qy)
    e = val - pb.re.ravel()
    msd = float(np.sum(e * e) / P)
    lam = np.zeros_like(u)
    for a in range(3):
        np.add.at(lam[:, 0], nodes[:, a], (2.0 / P) * e * w[:, a] * gx)
        np.add.at(lam[:, 1], nodes[:, a], (2.0 / P) * e * w[:, a] * gy)
    cbar = np.zeros((H, W))
    _scatter_taps(cbar, (H, W), qx, qy, (2.0 / P) * e)
    return lam, cbar, msd


def step_adjoint(pb: Problem, u_k: np.ndarray, u_k1: np.ndarray, lam_k1: np.ndarray,
                 cbar: np.ndarray):
    """One reverse step: returns ``(lambda^k, d gbar_alpha)`` and adds into ``cbar``."""
    S = pb.S
    mu = np.stack([cg(S, lam_k1[:, 0]), cg(S, lam_k1[:, 1])], axis=1)
    dalpha = -pb.tau * sum(float(mu[:, c] @ (pb.K @ u_k1[:, c])) for c in range(2))
    if pb.force_mode == FORCE_NODAL:
        eta = -pb.tau * mu
    else:
        eta = -pb.tau * (pb.M @ (mu / pb.m[:, None]))
    t, gx, gy, hxx, hxy, hyy = node_samples(pb, u_k, order=2)
    r = t - pb.rho
    eg = eta[:, 0] * gx + eta[:, 1] * gy
    lam = mu.copy()
    lam[:, 0] += eg * gx + r * (hxx * eta[:, 0] + hxy * eta[:, 1])
    lam[:, 1] += eg * gy + r * (hxy * eta[:, 0] + hyy * eta[:, 1])
    _scatter_taps(cbar, cbar.shape, pb.V[:, 0] - 0.5 + u_k[:, 0], pb.V[:, 1] - 0.5 + u_k[:, 1],
                  eg, r * eta[:, 0], r * eta[:, 1])
    return lam, dalpha


def gradient(pb: Problem, u0: np.ndarray | None, n_iter: int):
    """``(msd, g_u0, g_alpha, g_te)`` of ``L = MSD(u^N)``."""
    uN, _, us = run(pb, u0, n_iter, keep_all=True)
    lam, cbar, L = warp_adjoint(pb, uN)
    g_alpha = 0.0
    for k in range(n_iter - 1, -1, -1):
        lam, da = step_adjoint(pb, us[k], us[k + 1], lam, cbar)
        g_alpha += da
    g_te = bspline.prefilter(cbar)
    return L, lam, g_alpha, g_te
