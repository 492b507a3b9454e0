"""Algorithm 1 as printed: explicit descent with the mesh gradient, then umbrella
smoothing -- TEST INFRASTRUCTURE (see the package docstring).

One iteration from ``u = u_1^k`` (Section 2 and Algorithm 1):

1. ``t_i = s_Te(V_i - 1/2 + u_i)``, ``r_i = t_i - rho_i`` with ``rho_i`` the
   reference at the undisplaced node (eq. 3-4, the reading of the main path).
2. The gradient of the nodal samples on the deformed mesh ``P = V + u``:
   on every triangle eq. 9 as printed, with its area computed from the
   deformed corners at the start of the iteration; at every node the
   area-weighted mean of eq. 10 over its triangles.  Areas are taken
   unsigned; a triangle whose deformed area is zero is left out, and a node
   left with no triangle gets a zero gradient (the paper does not say).
3. ``u_0^{k+1} = u - tau r g`` (eq. 5 with eq. 6).
4. ``u_1^{k+1} = ((1 - lambda) I + lambda A^Lap) u_0^{k+1}`` (eq. 14), with
   ``A^Lap`` the umbrella matrix of eq. 11-13: ``1 / m_i`` at the ``m_i``
   nodes of node i's 1-ring (the other corners of its triangles).

The paper uses ``tau = 0.005`` and ``lambda = 0.8`` on 0-255 intensities; the
force is quadratic in intensity, so on [0, 1] images the same step is
``tau = 0.005 * 255^2``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bspline, mesh
from .registration import Problem, msd

PAPER_TAU_0_255 = 0.005
PAPER_LAMBDA = 0.8
TAU_UNIT_RANGE = PAPER_TAU_0_255 * 255.0 ** 2


def umbrella(T: np.ndarray, n: int) -> sp.csr_matrix:
    """``A^Lap`` (eq. 13) from the 1-ring table T2."""
    ptr, idx = mesh.table_t2(T, n)
    rows, cols, vals = [], [], []
    for i in range(n):
        nb = idx[ptr[i]:ptr[i + 1]]
        for j in nb:
            rows.append(i)
            cols.append(int(j))
            vals.append(1.0 / len(nb))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def node_gradient(P: np.ndarray, T: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Eq. 10 at every node: ``sum_j A_j grad f_Tj / sum_j A_j`` over the
    node's triangles, ``grad f_Tj`` by eq. 9 on the corner positions ``P``
    (FP64), ``A_j`` the unsigned area; zero-area triangles are skipped."""
    P = np.asarray(P, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    f = np.asarray(f, dtype=np.float64)
    n = P.shape[0]
    Pi, Pj, Pk = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    e1, e2 = Pj - Pi, Pk - Pi
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    ok = area > 0.0
    g_tri = np.zeros((T.shape[0], 2))
    g_tri[ok] = mesh.eq9_gradient(Pi[ok], Pj[ok], Pk[ok], f[T[ok, 0]], f[T[ok, 1]], f[T[ok, 2]])
    num = np.zeros((n, 2))
    den = np.zeros(n)
    for a in range(3):
        np.add.at(num, T[ok, a], area[ok, None] * g_tri[ok])
        np.add.at(den, T[ok, a], area[ok])
    g = np.zeros((n, 2))
    has = den > 0.0
    g[has] = num[has] / den[has, None]
    return g


def samples(pb: Problem, u: np.ndarray) -> np.ndarray:
    """Template values at the displaced nodes (step 1)."""
    V = pb.V
    return bspline.evaluate(pb.c_te, V[:, 0] - 0.5 + u[:, 0], V[:, 1] - 0.5 + u[:, 1])[0]


def update(pb: Problem, u: np.ndarray, tau: float) -> np.ndarray:
    """Steps 1-3: ``u_0^{k+1}``."""
    t = samples(pb, u)
    r = t - pb.rho
    g = node_gradient(pb.V + u, pb.T, t)
    return u - tau * r[:, None] * g


def smooth(A: sp.csr_matrix, u0: np.ndarray, lam: float) -> np.ndarray:
    """Step 4 (eq. 14), one application."""
    return (1.0 - lam) * u0 + lam * (A @ u0)


def step(pb: Problem, u: np.ndarray, tau: float, lam: float,
         A: sp.csr_matrix | None = None) -> np.ndarray:
    if A is None:
        A = umbrella(pb.T, pb.V.shape[0])
    return smooth(A, update(pb, u, tau), lam)


def run(pb: Problem, u0: np.ndarray | None, n_iter: int, tau: float, lam: float,
        record_msd: bool = False):
    """``n_iter`` iterations; returns ``(u_N, msds)`` with ``msds[k] = MSD(u^{k+1})``."""
    A = umbrella(pb.T, pb.V.shape[0])
    u = np.zeros((pb.V.shape[0], 2)) if u0 is None else np.array(u0, dtype=np.float64)
    out = []
    for _ in range(n_iter):
        u = step(pb, u, tau, lam, A)
        if record_msd:
            out.append(msd(pb, u))
    return u, out
