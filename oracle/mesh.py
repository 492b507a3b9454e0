"""Mesh tables and P1 operators in plain FP64 / exact integers.

The mesh ``(V, T)`` follows Section 2.1: ``V`` holds node coordinates (here
integer pixel corners ``(x, y)``), ``T`` holds three node indices per triangle
and the triangles cover the image domain ``[0, W] x [0, H]``.  Algorithm 1's
pre-computation builds the 1-ring ``N_1`` and each node's neighbour triangles;
the tables below are those, in a fixed order:

* T1: node -> (triangle, corner) CSR, slots sorted by triangle id
  (each node's neighbour triangles).
* T2: 1-ring CSR, neighbours sorted ascending (``N_1``).
* T3: pattern of the stiffness / mass matrices: T2 plus the diagonal.
* T4: twice each triangle's signed area (integer cross product).
* T5: per node, the sum of T4 over its triangles (six times the lumped mass).
* T6: per pixel, the triangle containing its centre ``(j+1/2, i+1/2)``,
  ties to the lowest triangle id; -1 if none.

Operators (Section 2.2, eq. 9 and 10; Section 2.3):

* element gradients of the linear (P1) basis, ``grad phi_a = R e_a / (2 A)``
  with ``e_a`` the edge opposite vertex ``a`` and ``R`` the +90 degree rotation;
  this equals eq. 9 as printed (checked in the tests);
* stiffness ``K_T[a][b] = e_a . e_b / (4 A)`` and consistent mass
  ``M_T = (A/12) [[2,1,1],[1,2,1],[1,1,2]]``, summed over triangles;
* lumped mass ``m = M 1``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def twice_areas(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """T4: ``(b - a) x (c - a)`` per triangle, int64."""
    P = np.asarray(V, dtype=np.int64)[np.asarray(T, dtype=np.int64)]
    e1 = P[:, 1] - P[:, 0]
    e2 = P[:, 2] - P[:, 0]
    return e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]


def validate(V, T, height: int, width: int) -> None:
    """Raise ``ValueError`` for a mesh the method cannot use."""
    V = np.asarray(V)
    T = np.asarray(T)
    n = V.shape[0]
    if V.ndim != 2 or V.shape[1] != 2 or T.ndim != 2 or T.shape[1] != 3:
        raise ValueError("V must be [n][2] and T [n_T][3]")
    if n == 0 or T.shape[0] == 0:
        raise ValueError("empty mesh")
    if T.min() < 0 or T.max() >= n:
        raise ValueError("triangle index out of range")
    if (V[:, 0].min() < 0 or V[:, 0].max() > width or V[:, 1].min() < 0
            or V[:, 1].max() > height):
        raise ValueError("node outside [0, W] x [0, H]")
    if np.any(twice_areas(V, T) <= 0):
        raise ValueError("triangle with non-positive area")
    if np.unique(T).size != n:
        raise ValueError("unreferenced node")


def table_t1(T: np.ndarray, n: int):
    """Node -> slots ``3 * triangle + corner``, each node's slots in triangle order."""
    ptr = np.zeros(n + 1, dtype=np.int64)
    lists = [[] for _ in range(n)]
    for t in range(T.shape[0]):
        for a in range(3):
            lists[int(T[t, a])].append(3 * t + a)
    for i in range(n):
        ptr[i + 1] = ptr[i] + len(lists[i])
    slots = np.array([s for lst in lists for s in lst], dtype=np.int64)
    return ptr, slots


def table_t2(T: np.ndarray, n: int):
    """1-ring CSR: for each node the other nodes of its triangles, ascending."""
    nbrs = [set() for _ in range(n)]
    for t in range(T.shape[0]):
        a, b, c = (int(v) for v in T[t])
        nbrs[a].update((b, c))
        nbrs[b].update((a, c))
        nbrs[c].update((a, b))
    ptr = np.zeros(n + 1, dtype=np.int64)
    for i in range(n):
        ptr[i + 1] = ptr[i] + len(nbrs[i])
    idx = np.array([j for i in range(n) for j in sorted(nbrs[i])], dtype=np.int64)
    return ptr, idx


def table_t3(T: np.ndarray, n: int):
    """CSR pattern of K and M: the 1-ring plus the node itself, ascending."""
    ptr2, idx2 = table_t2(T, n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    out = []
    for i in range(n):
        row = sorted(list(idx2[ptr2[i]:ptr2[i + 1]]) + [i])
        out.extend(row)
        ptr[i + 1] = ptr[i] + len(row)
    return ptr, np.array(out, dtype=np.int64)


def table_t5(T: np.ndarray, t4: np.ndarray, n: int) -> np.ndarray:
    t5 = np.zeros(n, dtype=np.int64)
    for t in range(T.shape[0]):
        for a in range(3):
            t5[T[t, a]] += t4[t]
    return t5


def table_t6(V: np.ndarray, T: np.ndarray, height: int, width: int) -> np.ndarray:
    """Lowest-id triangle whose closed interior holds each pixel centre.

    Exact integer test in doubled coordinates: the centre of pixel ``(i, j)`` is
    ``(2j+1, 2i+1) / 2`` and ``p`` lies in triangle ``(a, b, c)`` iff the three
    edge cross products ``(b-a) x (p-a)``, ``(c-b) x (p-b)``, ``(a-c) x (p-c)``
    are all >= 0 (triangles have positive orientation).  Triangles are tested
    in groups of equal bounding-box size (all candidate pixels of a group at
    once); each pixel keeps the minimum id that contains it.
    """
    V2 = 2 * np.asarray(V, dtype=np.int64)
    T = np.asarray(T, dtype=np.int64)
    big = np.iinfo(np.int64).max
    t6 = np.full(height * width, big, dtype=np.int64)
    P = V2[T]                                   # [nT][3][2]
    xlo = np.clip((P[:, :, 0].min(1) - 1) // 2, 0, width)
    xhi = np.clip((P[:, :, 0].max(1) - 1) // 2 + 1, 0, width)
    ylo = np.clip((P[:, :, 1].min(1) - 1) // 2, 0, height)
    yhi = np.clip((P[:, :, 1].max(1) - 1) // 2 + 1, 0, height)
    bw, bh = xhi - xlo, yhi - ylo
    keys = bw * (height + 1) + bh
    for key in np.unique(keys):
        ts = np.nonzero(keys == key)[0]
        w, h = int(bw[ts[0]]), int(bh[ts[0]])
        if w <= 0 or h <= 0:
            continue
        for chunk in np.array_split(ts, max(1, ts.size * w * h // 4_000_000 + 1)):
            jj = xlo[chunk, None, None] + np.arange(w)[None, None, :]
            ii = ylo[chunk, None, None] + np.arange(h)[None, :, None]
            px, py = 2 * jj + 1, 2 * ii + 1
            inside = np.ones((chunk.size, h, w), dtype=bool)
            for k in range(3):
                a = P[chunk, k][:, :, None, None]
                b = P[chunk, (k + 1) % 3][:, :, None, None]
                cr = (b[:, 0] - a[:, 0]) * (py - a[:, 1]) - (b[:, 1] - a[:, 1]) * (px - a[:, 0])
                inside &= cr >= 0
            tid = np.broadcast_to(chunk[:, None, None], inside.shape)
            flat = (ii * width + jj)
            flat = np.broadcast_to(flat, inside.shape)
            np.minimum.at(t6, flat[inside], tid[inside])
    t6[t6 == big] = -1
    return t6.reshape(height, width)


def tables(V, T, height: int, width: int) -> dict:
    """All six tables as a dict of int64 arrays."""
    V = np.asarray(V)
    T = np.asarray(T)
    n = V.shape[0]
    t1p, t1s = table_t1(T, n)
    t2p, t2i = table_t2(T, n)
    t3p, t3i = table_t3(T, n)
    t4 = twice_areas(V, T)
    t5 = table_t5(T, t4, n)
    t6 = table_t6(V, T, height, width)
    return dict(t1_ptr=t1p, t1_slot=t1s, t2_ptr=t2p, t2_idx=t2i, t3_ptr=t3p, t3_idx=t3i,
                t4=t4, t5=t5, t6=t6)


def p1_gradients(V, T):
    """``grad phi_a`` for the three corners of every triangle: ``[nT][3][2]``."""
    P = np.asarray(V, dtype=np.float64)[np.asarray(T)]
    twoA = twice_areas(V, T).astype(np.float64)
    out = np.empty(P.shape)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        e = P[:, c] - P[:, b]                   # edge opposite a
        out[:, a, 0] = -e[:, 1] / twoA          # R(x, y) = (-y, x)
        out[:, a, 1] = e[:, 0] / twoA
    return out


def eq9_gradient(Vi, Vj, Vk, fi, fj, fk):
    """Eq. 9 as printed: the gradient on triangle (Vi, Vj, Vk) of the linear
    interpolant of nodal values (fi, fj, fk), with V_ab = V_b - V_a."""
    Vi, Vj, Vk = (np.asarray(v, dtype=np.float64) for v in (Vi, Vj, Vk))
    d = lambda p, q: p[..., 0] * q[..., 0] + p[..., 1] * q[..., 1]
    Vij, Vjk, Vik, Vkj = Vj - Vi, Vk - Vj, Vk - Vi, Vj - Vk
    Vji, Vki = Vi - Vj, Vi - Vk
    cr = (Vj - Vi)[..., 0] * (Vk - Vi)[..., 1] - (Vj - Vi)[..., 1] * (Vk - Vi)[..., 0]
    A = 0.5 * np.abs(cr)
    s = lambda v: v[..., None]
    g = (s(fi) * (s(d(Vij, Vjk)) * (Vk - Vi) + s(d(Vik, Vkj)) * (Vj - Vi))
         + s(fj) * (s(d(Vji, Vik)) * (Vk - Vj) + s(d(Vjk, Vki)) * (Vi - Vj))
         + s(fk) * (s(d(Vkj, Vji)) * (Vi - Vk) + s(d(Vki, Vij)) * (Vj - Vk)))
    return g / s(4.0 * A * A)


def stiffness(V, T) -> sp.csr_matrix:
    """P1 stiffness ``K = sum_T K_T``, ``K_T[a][b] = A grad phi_a . grad phi_b``."""
    n = np.asarray(V).shape[0]
    G = p1_gradients(V, T)
    A = 0.5 * twice_areas(V, T).astype(np.float64)
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(T[:, a])
            cols.append(T[:, b])
            vals.append(A * (G[:, a, 0] * G[:, b, 0] + G[:, a, 1] * G[:, b, 1]))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def mass(V, T) -> sp.csr_matrix:
    """Consistent P1 mass ``M = sum_T (A/12) [[2,1,1],[1,2,1],[1,1,2]]``."""
    n = np.asarray(V).shape[0]
    A = 0.5 * twice_areas(V, T).astype(np.float64)
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(T[:, a])
            cols.append(T[:, b])
            vals.append(A * (2.0 if a == b else 1.0) / 12.0)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def lumped_mass(V, T) -> np.ndarray:
    """``m = M 1``: a third of the area of every triangle at each of its corners."""
    n = np.asarray(V).shape[0]
    A = 0.5 * twice_areas(V, T).astype(np.float64)
    m = np.zeros(n)
    for a in range(3):
        np.add.at(m, T[:, a], A / 3.0)
    return m


def barycentric(V, T, tri: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Barycentric weights ``[npts][3]`` of points in their triangles.

    ``w_a = area(p, b, c) / area(a, b, c)`` and cyclically; exact for integer
    ``2 p`` since both areas are integers in doubled coordinates.
    """
    V2 = 2 * np.asarray(V, dtype=np.int64)
    P = V2[np.asarray(T, dtype=np.int64)[tri]]          # [npts][3][2]
    p = np.stack([np.asarray(px), np.asarray(py)], axis=-1)
    tot = ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
           - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])).astype(np.float64)
    w = np.empty((p.shape[0], 3))
    for a in range(3):
        b, c = P[:, (a + 1) % 3], P[:, (a + 2) % 3]
        cr = (b[:, 0] - p[:, 0]) * (c[:, 1] - p[:, 1]) - (b[:, 1] - p[:, 1]) * (c[:, 0] - p[:, 0])
        w[:, a] = cr / tot
    return w
