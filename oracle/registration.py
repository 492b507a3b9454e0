"""The registration iteration, warp and MSD in plain FP64.

Objective (eq. 1): ``E[u] = D[Re, Te o u] + alpha S[u]`` with the nodal SSD
data term of eq. 4 and, as regulariser, the P1 diffusion energy
``S[u] = 1/2 sum_c u_c^T K u_c`` (the mesh Laplacian of Section 2.3 written
as a symmetric stiffness so that a direct sparse solve applies, as the
abstract describes).  One iteration (Algorithm 1: update, then smoothing;
eq. 5-8), made semi-implicit:

1. ``t_i, g_i = s_Te(V_i - 1/2 + u_i), grad s_Te(...)``  (eq. 3; spline, abstract)
2. ``r_i = t_i - rho_i``, ``rho_i = s_Re(V_i - 1/2)``    (eq. 4)
3. ``h_i = r_i g_i``                                       (eq. 6)
4. ``f = (M h) / m`` per component (the area-weighted triangle-to-node average
   of eq. 10 applied to the P1 load), or ``f = h`` in the nodal mode
5. ``b = u - tau f``                                       (eq. 5)
6. ``u+ = (I + tau alpha K)^-1 b`` per component           (eq. 7-8, implicit)

Warp and MSD (Section 1: final displacement reconstruction and the MSD
metric; Fig. 3): every pixel centre ``x_p = (j+1/2, i+1/2)`` takes the
piecewise-linear displacement of its triangle (table T6),
``W_p = s_Te(x_p - 1/2 + u(p))`` and ``MSD = mean_p (W_p - Re_p)^2``.

Steps 1-6 are a proximal-gradient step on ``D + alpha S``; the solve here is
conjugate gradients (not a Cholesky factorisation) to a relative residual of
1e-14.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import bspline, mesh

FORCE_P1 = 0
FORCE_NODAL = 1


def cg(A: sp.spmatrix, b: np.ndarray, rtol: float = 1e-14, maxiter: int = 1000) -> np.ndarray:
    """Plain conjugate gradients for SPD ``A``; stops at ``|r| <= rtol |b|``."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x
    r = b.copy()
    p = r.copy()
    rr = r @ r
    for _ in range(maxiter):
        if np.sqrt(rr) <= rtol * bn:
            break
        Ap = A @ p
        a = rr / (p @ Ap)
        x += a * p
        r -= a * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


@dataclass
class Problem:
    """Pre-computed state of one pair (Algorithm 1, pre-computation)."""
    V: np.ndarray
    T: np.ndarray
    height: int
    width: int
    te: np.ndarray
    re: np.ndarray
    c_te: np.ndarray
    c_re: np.ndarray
    rho: np.ndarray
    K: sp.csr_matrix
    M: sp.csr_matrix
    m: np.ndarray
    t6: np.ndarray
    alpha: float
    tau: float
    force_mode: int = FORCE_P1

    @property
    def S(self) -> sp.csr_matrix:
        n = self.V.shape[0]
        return (sp.identity(n, format="csr") + (self.tau * self.alpha) * self.K).tocsr()


def setup(te, re, V, T, alpha: float, tau: float, force_mode: int = FORCE_P1,
          t6: np.ndarray | None = None) -> Problem:
    te = np.asarray(te, dtype=np.float64)
    re = np.asarray(re, dtype=np.float64)
    H, W = te.shape
    V = np.asarray(V, dtype=np.int64)
    T = np.asarray(T, dtype=np.int64)
    mesh.validate(V, T, H, W)
    c_te = bspline.prefilter(te)
    c_re = bspline.prefilter(re)
    rho = bspline.evaluate(c_re, V[:, 0] - 0.5, V[:, 1] - 0.5)[0]
    if t6 is None:
        t6 = mesh.table_t6(V, T, H, W)
    return Problem(V=V, T=T, height=H, width=W, te=te, re=re, c_te=c_te, c_re=c_re, rho=rho,
                   K=mesh.stiffness(V, T), M=mesh.mass(V, T), m=mesh.lumped_mass(V, T),
                   t6=t6, alpha=float(alpha), tau=float(tau), force_mode=force_mode)


def node_samples(pb: Problem, u: np.ndarray, order: int = 1):
    """Template spline at the displaced nodes ``V - 1/2 + u``."""
    return bspline.evaluate(pb.c_te, pb.V[:, 0] - 0.5 + u[:, 0], pb.V[:, 1] - 0.5 + u[:, 1],
                            order=order)


def force(pb: Problem, u: np.ndarray):
    """``(h, f)``: nodal SSD force density and the force the step uses."""
    t, gx, gy = node_samples(pb, u)
    r = t - pb.rho
    h = np.stack([r * gx, r * gy], axis=1)
    if pb.force_mode == FORCE_NODAL:
        return h, h.copy()
    f = (pb.M @ h) / pb.m[:, None]
    return h, f


def rhs(pb: Problem, u: np.ndarray) -> np.ndarray:
    """``b = u - tau f``."""
    return u - pb.tau * force(pb, u)[1]


def solve(pb: Problem, b: np.ndarray, dense: bool = False) -> np.ndarray:
    S = pb.S
    if dense:
        return np.linalg.solve(S.toarray(), b)
    return np.stack([cg(S, b[:, 0]), cg(S, b[:, 1])], axis=1)


def step(pb: Problem, u: np.ndarray, dense: bool = False) -> np.ndarray:
    return solve(pb, rhs(pb, u), dense=dense)


def pixel_displacement(pb: Problem, u: np.ndarray) -> np.ndarray:
    """``u(p)`` at every pixel centre: ``[H][W][2]``."""
    H, W = pb.height, pb.width
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    tri = pb.t6.ravel()
    if np.any(tri < 0):
        raise ValueError("pixel not covered by the mesh")
    w = mesh.barycentric(pb.V, pb.T, tri, 2 * jj.ravel() + 1, 2 * ii.ravel() + 1)
    nodes = pb.T[tri]
    up = (w[:, :, None] * u[nodes]).sum(axis=1)
    return up.reshape(H, W, 2)


def warp(pb: Problem, u: np.ndarray) -> np.ndarray:
    """Registered image ``W_p = s_Te(j + u_x(p), i + u_y(p))``."""
    H, W = pb.height, pb.width
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    up = pixel_displacement(pb, u)
    return bspline.evaluate(pb.c_te, jj + up[:, :, 0], ii + up[:, :, 1])[0]


def msd(pb: Problem, u: np.ndarray) -> float:
    """Mean squared difference between the warped template and ``Re``."""
    e = warp(pb, u) - pb.re
    return float(np.sum(e * e) / e.size)


def run(pb: Problem, u0: np.ndarray | None, n_iter: int, record_msd: bool = False,
        keep_all: bool = False):
    """``n_iter`` iterations from ``u0`` (zeros if None).

    Returns ``(u_N, msds, us)``: ``msds[k] = MSD(u^{k+1})`` when recorded and
    ``us`` every iterate ``u^0 .. u^N`` when ``keep_all``.
    """
    u = np.zeros((pb.V.shape[0], 2)) if u0 is None else np.array(u0, dtype=np.float64)
    msds, us = [], [u.copy()] if keep_all else None
    for _ in range(n_iter):
        u = step(pb, u)
        if record_msd:
            msds.append(msd(pb, u))
        if keep_all:
            us.append(u.copy())
    return u, msds, us


def run_until(pb: Problem, u0: np.ndarray | None, max_iter: int, check_every: int,
              rel_tol: float):
    """Algorithm 1's loop "to convergence" with a relative-MSD stopping rule.

    The paper leaves the criterion open; this reading checks every
    ``check_every`` iterations: with ``m_prev`` the MSD ``check_every``
    iterations earlier (``MSD(u0)`` at first) and ``m_now`` the current one,
    the loop stops when ``m_prev <= 0`` or ``m_prev - m_now < rel_tol m_prev``
    (an increase stops it too), and after ``max_iter`` iterations at most (the
    last chunk may be shorter).  Returns ``(u, iters, m_final, checks)`` with
    ``checks`` the MSDs compared, ``MSD(u0)`` first.
    """
    u = np.zeros((pb.V.shape[0], 2)) if u0 is None else np.array(u0, dtype=np.float64)
    m_prev = msd(pb, u)
    checks = [m_prev]
    done = 0
    while done < max_iter:
        n = min(check_every, max_iter - done)
        for _ in range(n):
            u = step(pb, u)
        done += n
        m_now = msd(pb, u)
        checks.append(m_now)
        stop = not (m_prev > 0.0) or (m_prev - m_now) < rel_tol * m_prev
        m_prev = m_now
        if stop:
            break
    return u, done, m_prev, checks
