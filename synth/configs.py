"""The five workloads, as seeded recipes.

Seeds are ``1000 * config_id + pair_index``.  Draw order per pair: the side
(batched ragged workload only), then the image parameters of
``synth.images.draw_params``, then (batched differentiable workload only) the
pair's alpha, log-uniform in [0.02, 0.2].

| id | workload | images | mesh (s_min, s_max, g) | alpha, tau, iterations |
|----|----------|--------|------------------------|------------------------|
| 1 | single pair, small | 128^2 FP32, 8 blobs, sine amplitude 3 | 2, 16, 0.05 | 0.1, 0.5, 50 |
| 2 | single pair, clinical slice size | 512^2, 12-bit, 128 blobs, amplitude 8 | 1, 32, 0.08 | 0.05, 0.5, 200 (MSD every iteration) |
| 3 | single large pair, differentiable | 2048^2 FP32, 2048 blobs, amplitude 8 | 1, 32, 0.08 | 0.05, 0.5, 50 |
| 4 | 256 ragged pairs | side in {128..1024}, FP32, amplitude 6 | 1, 32, 0.10 | 0.05, 0.5, 100 |
| 5 | 64 pairs, differentiable | 512^2 12-bit as id 2 | 1, 32, 0.08 | log-uniform alpha, 0.5, 100, checkpoint 10 |
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .images import draw_params, make_images
from .quadtree import quadtree_mesh

C4_SIDES = (128, 192, 256, 384, 512, 768, 1024)


@dataclass
class Pair:
    te: np.ndarray          # float32 [H][W]
    re: np.ndarray          # float32 [H][W]
    V: np.ndarray           # int32 [n][2] (x, y)
    T: np.ndarray           # int32 [n_T][3]
    leaves: np.ndarray      # int32 [n_leaves][3] (x0, y0, s)
    alpha: float
    seed: int
    params: dict = field(repr=False, default_factory=dict)

    @property
    def height(self) -> int:
        return int(self.te.shape[0])

    @property
    def width(self) -> int:
        return int(self.te.shape[1])

    @property
    def n_nodes(self) -> int:
        return int(self.V.shape[0])


@dataclass
class Workload:
    config_id: int
    name: str
    pairs: list
    tau: float
    n_iter: int
    msd_every_iter: bool = False
    ckpt_every: int = 0


SPECS = {
    1: dict(name="single-pair 128x128, quadtree s=2..16 g=0.05", side=128, amp=3.0,
            quant=False, s_min=2, s_max=16, g=0.05, alpha=0.1, tau=0.5, n_iter=50,
            n_pairs=1),
    2: dict(name="single-pair 512x512 12-bit, quadtree s=1..32 g=0.08", side=512, amp=8.0,
            quant=True, s_min=1, s_max=32, g=0.08, alpha=0.05, tau=0.5, n_iter=200,
            n_pairs=1, msd_every_iter=True),
    3: dict(name="single-pair 2048x2048, quadtree s=1..32 g=0.08, fwd+bwd", side=2048,
            amp=8.0, quant=False, s_min=1, s_max=32, g=0.08, alpha=0.05, tau=0.5,
            n_iter=50, n_pairs=1, ckpt_every=10),
    4: dict(name="256 ragged pairs 128..1024, quadtree s=1..32 g=0.10", side=None, amp=6.0,
            quant=False, s_min=1, s_max=32, g=0.10, alpha=0.05, tau=0.5, n_iter=100,
            n_pairs=256),
    5: dict(name="64 pairs 512x512 12-bit, fwd+bwd checkpoint 10", side=512, amp=8.0,
            quant=True, s_min=1, s_max=32, g=0.08, alpha=None, tau=0.5, n_iter=100,
            n_pairs=64, ckpt_every=10),
}


def make_pair(config_id: int, pair_index: int = 0, side: int | None = None) -> Pair:
    """One seeded pair of workload ``config_id``; ``side`` overrides the image side."""
    spec = SPECS[config_id]
    seed = 1000 * config_id + pair_index
    rng = np.random.default_rng(seed)
    if spec["side"] is None:
        drawn = int(rng.choice(C4_SIDES))
        side = drawn if side is None else side
    elif side is None:
        side = spec["side"]
    params = draw_params(rng, side, side, spec["amp"])
    alpha = spec["alpha"]
    if alpha is None:
        alpha = float(np.exp(rng.uniform(np.log(0.02), np.log(0.2))))
    te, re = make_images(params, quantise=spec["quant"])
    V, T, leaves = quadtree_mesh(te, spec["s_min"], spec["s_max"], spec["g"])
    return Pair(te=te, re=re, V=V, T=T, leaves=leaves, alpha=float(alpha), seed=seed,
                params=params)


def _make_pair_args(args):
    return make_pair(*args)


def make_pairs(config_id: int, n_pairs: int, processes: int = 1) -> list:
    """Pairs ``0 .. n_pairs-1`` of a workload, optionally in a process pool
    (``spawn`` start method, so no GPU state is inherited)."""
    if processes <= 1 or n_pairs <= 1:
        return [make_pair(config_id, p) for p in range(n_pairs)]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(processes) as pool:
        return pool.map(_make_pair_args, [(config_id, p) for p in range(n_pairs)], chunksize=1)


def make_workload(config_id: int, n_pairs: int | None = None, processes: int = 1) -> Workload:
    spec = SPECS[config_id]
    k = spec["n_pairs"] if n_pairs is None else n_pairs
    pairs = make_pairs(config_id, k, processes)
    return Workload(config_id=config_id, name=spec["name"], pairs=pairs, tau=spec["tau"],
                    n_iter=spec["n_iter"], msd_every_iter=spec.get("msd_every_iter", False),
                    ckpt_every=spec.get("ckpt_every", 0))
