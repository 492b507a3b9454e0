"""Content-adaptive unstructured triangulation (irregular valence, arbitrary
edge directions) as a second mesh type for the registration path.

The paper's meshes come from the content-adaptive mesher of its reference
[12] (Section 3.1), which is outside this project.  This module stands in
for that kind of mesh: the node set is the corner set of a content-adaptive
quadtree (dense where the template has detail), every node that is not on
the image border or a fixed corner is moved by a seeded integer jitter
within its finest adjacent cell, and the nodes are connected by their
Delaunay triangulation (scipy).  The result covers ``[0, W] x [0, H]``
exactly (the four image corners and every border node stay on the border),
uses integer node coordinates, and has no quadtree structure left: node
valences vary and edges run in all directions.  Like ``quadtree``, this only
produces the method's input ``(V, T)``.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay

from .quadtree import quadtree_leaves


def unstructured_mesh(img: np.ndarray, s_min: int, s_max: int, g: float, seed: int,
                      jitter: float = 0.35):
    """``(V, T)``: V ``[n][2]`` int32 ``(x, y)``, T ``[n_T][3]`` int32 with
    positive signed area ``(b - a) x (c - a) > 0`` in ``(x, y)``."""
    H, W = img.shape
    leaves = quadtree_leaves(img, s_min, s_max, g).astype(np.int64)
    x0, y0, s = leaves[:, 0], leaves[:, 1], leaves[:, 2]
    stride = W + 1
    corners = np.concatenate([y0 * stride + x0, y0 * stride + x0 + s,
                              (y0 + s) * stride + x0, (y0 + s) * stride + x0 + s])
    sizes = np.concatenate([s, s, s, s])
    keys = np.unique(corners)
    # finest cell size adjacent to each node
    fine = np.full(keys.size, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(fine, np.searchsorted(keys, corners), sizes)
    x = (keys % stride).astype(np.int64)
    y = (keys // stride).astype(np.int64)
    rng = np.random.default_rng(seed)
    reach = np.floor(jitter * fine).astype(np.int64)
    dx = np.where(reach > 0, rng.integers(-reach, reach + 1), 0)
    dy = np.where(reach > 0, rng.integers(-reach, reach + 1), 0)
    interior_x = (x > 0) & (x < W)
    interior_y = (y > 0) & (y < H)
    # border nodes slide along their border only; corners stay
    x = np.where(interior_x, np.clip(x + dx, 1, W - 1), x)
    y = np.where(interior_y, np.clip(y + dy, 1, H - 1), y)
    pts = np.unique(np.stack([x, y], axis=1), axis=0)          # jitter may merge nodes
    tri = Delaunay(pts.astype(np.float64)).simplices.astype(np.int64)
    a, b, c = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    keep = area2 != 0                                         # collinear border triples
    tri, area2 = tri[keep], area2[keep]
    neg = area2 < 0
    tri[neg] = tri[neg][:, [0, 2, 1]]
    used = np.unique(tri)
    remap = np.full(pts.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    V = pts[used].astype(np.int32)
    T = remap[tri].astype(np.int32)
    # node order (y, x), triangle order by first node then the others: a
    # deterministic numbering independent of Qhull's output order
    order = np.lexsort((V[:, 0], V[:, 1]))
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    V = V[order]
    T = rank[T].astype(np.int32)
    rot = np.argmin(T, axis=1)                                # smallest id first, orientation kept
    T = np.stack([T[np.arange(T.shape[0]), (rot + k) % 3] for k in range(3)], axis=1)
    T = T[np.lexsort((T[:, 2], T[:, 1], T[:, 0]))].astype(np.int32)
    return V, T
