"""Seeded random node directions for directional-derivative checks (inputs only)."""
from __future__ import annotations

import numpy as np


def random_directions(n_nodes: int, count: int, seed: int):
    """``count`` directions of shape ``[n_nodes][2]``, each component uniform in
    [-1, 1], drawn one after the other from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    for _ in range(count):
        yield rng.uniform(-1.0, 1.0, size=(n_nodes, 2))
