"""Content-adaptive quadtree triangulation used as the registration mesh.

The paper meshes the template with the content-adaptive mesher of its
reference [12] (Section 3.1); that mesher is outside this project, and the
paper notes quadtree/octree adaptive grids as the simpler adaptive option
(Section 1).  This module builds such a mesh; it produces the method's input
``(V, T)`` (Section 2.1: ``V`` is ``n_V x 2`` coordinates, ``T`` is
``n_T x 3`` node indices) and performs no step of the method itself.

Rules:

* The image ``W x H`` is tiled by roots of side ``s_max`` (both sides must be
  multiples of ``s_max``, a power of two).
* A cell of side ``s`` is split into four iff ``s > s_min`` and the intensity
  range (max - min) of the template over the cell's pixel block exceeds ``g``.
* No 2:1 balance: nodes that hang on a larger neighbour's edge are ordinary
  free nodes.
* Leaves are sorted by ``(y0, x0)``; nodes are the distinct leaf corners sorted
  by ``(y, x)``; leaf ``k`` with corners ``p00=(x0,y0)``, ``p10=(x0+s,y0)``,
  ``p01=(x0,y0+s)``, ``p11=(x0+s,y0+s)`` gives triangles
  ``T[2k] = (p00, p10, p11)`` and ``T[2k+1] = (p00, p11, p01)``, both with
  positive signed area ``s^2/2`` in (x, y).
"""
from __future__ import annotations

import numpy as np


def quadtree_leaves(img: np.ndarray, s_min: int, s_max: int, g: float) -> np.ndarray:
    """Leaves ``[n_leaves][3]`` as ``(x0, y0, s)`` int32, sorted by ``(y0, x0)``."""
    H, W = img.shape
    if s_max & (s_max - 1) or s_min & (s_min - 1) or s_min > s_max:
        raise ValueError("s_min and s_max must be powers of two with s_min <= s_max")
    if H % s_max or W % s_max:
        raise ValueError("image sides must be multiples of s_max")
    img = np.asarray(img, dtype=np.float64)
    leaves = []
    # cells at the current size, in block units of that size
    iy, ix = np.meshgrid(np.arange(H // s_max), np.arange(W // s_max), indexing="ij")
    iy, ix = iy.ravel(), ix.ravel()
    s = s_max
    while iy.size:
        blocks = img.reshape(H // s, s, W // s, s)
        rng_s = blocks.max(axis=(1, 3)) - blocks.min(axis=(1, 3))
        split = (s > s_min) & (rng_s[iy, ix] > g)
        keep = ~split
        leaves.append(np.stack([ix[keep] * s, iy[keep] * s,
                                np.full(int(keep.sum()), s)], axis=1))
        cy, cx = iy[split], ix[split]
        iy = np.concatenate([2 * cy, 2 * cy, 2 * cy + 1, 2 * cy + 1])
        ix = np.concatenate([2 * cx, 2 * cx + 1, 2 * cx, 2 * cx + 1])
        s //= 2
    lv = np.concatenate(leaves, axis=0).astype(np.int64)
    order = np.lexsort((lv[:, 0], lv[:, 1]))
    return lv[order].astype(np.int32)


def mesh_from_leaves(leaves: np.ndarray, height: int, width: int):
    """Nodes ``V [n][2] (x, y)`` int32 and triangles ``T [2 n_leaves][3]`` int32."""
    lv = np.asarray(leaves, dtype=np.int64)
    x0, y0, s = lv[:, 0], lv[:, 1], lv[:, 2]
    stride = width + 1
    k00 = y0 * stride + x0
    k10 = y0 * stride + x0 + s
    k01 = (y0 + s) * stride + x0
    k11 = (y0 + s) * stride + x0 + s
    keys = np.unique(np.concatenate([k00, k10, k01, k11]))
    V = np.stack([keys % stride, keys // stride], axis=1).astype(np.int32)
    n00, n10, n01, n11 = (np.searchsorted(keys, k) for k in (k00, k10, k01, k11))
    T = np.empty((2 * lv.shape[0], 3), dtype=np.int32)
    T[0::2, 0], T[0::2, 1], T[0::2, 2] = n00, n10, n11
    T[1::2, 0], T[1::2, 1], T[1::2, 2] = n00, n11, n01
    return V, T


def quadtree_mesh(img: np.ndarray, s_min: int, s_max: int, g: float):
    """``(V, T, leaves)`` for a template image."""
    leaves = quadtree_leaves(img, s_min, s_max, g)
    V, T = mesh_from_leaves(leaves, img.shape[0], img.shape[1])
    return V, T, leaves


def uniform_mesh(height: int, width: int, s: int):
    """A uniform quadtree mesh of side-``s`` leaves (every cell a leaf)."""
    ys, xs = np.meshgrid(np.arange(0, height, s), np.arange(0, width, s), indexing="ij")
    leaves = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, s)], axis=1).astype(np.int32)
    V, T = mesh_from_leaves(leaves, height, width)
    return V, T, leaves
