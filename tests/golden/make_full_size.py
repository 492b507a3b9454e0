"""Writes the full-size expected values of the GPU parity tests.

Every value written here comes from the FP64 oracle (``oracle/``) run on the
seeded synthetic inputs of ``synth/``; nothing is read from the HIP library.
The workloads are run at their own iteration counts:

* ``full_size_2048.json`` -- the 2048x2048 pair (alpha 0.05, tau 0.5): the
  displacements after 50 iterations from zero, and the gradient of the final
  MSD after 50 unrolled iterations (the objective of eq. 1 unrolled by
  Algorithm 1) with respect to the initial displacements (at zero), alpha and
  the template; the gradient is stored as its projections on 64 seeded random
  node directions (uniform in [-1, 1] per component, generator seed 34), as
  sampled entries and as norms.
* ``full_size_diff_batch.json`` -- pairs 0-3 of the 64-pair 512x512
  differentiable batch (per-pair alpha): the gradients of the final MSD after
  100 unrolled iterations from zero (sampled entries, norms, alpha).
* ``full_size_batch.json`` -- four pairs of the 256-pair ragged batch (the
  smallest side, the largest, a 384 side and pair 137): the displacements after
  100 iterations from zero (sampled entries and norms).

Each record carries a digest of its inputs (images, nodes, triangles, alpha),
so a test run on other inputs fails instead of comparing unrelated numbers.

Usage: ``python tests/golden/make_full_size.py [2048|diff_batch|batch ...]``
(all three by default; about ten minutes on one core for the 2048x2048 pair).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from oracle import registration as reg  # noqa: E402
from synth import SPECS, make_pair, random_directions  # noqa: E402
from synth.configs import C4_SIDES  # noqa: E402

TAU = 0.5
N_NODE_SAMPLES = 512
N_PIXEL_SAMPLES = 2048
DIRECTION_SEED = 34
N_DIRECTIONS = 64


def input_digest(p) -> str:
    """sha256 over the pair's images, nodes, triangles and alpha."""
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(p.te, dtype=np.float32), np.ascontiguousarray(p.re, dtype=np.float32),
              np.ascontiguousarray(p.V, dtype=np.int32), np.ascontiguousarray(p.T, dtype=np.int32)):
        h.update(a.tobytes())
    h.update(repr(float(p.alpha)).encode())
    return h.hexdigest()


def node_sample(n: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(n, size=min(n, N_NODE_SAMPLES), replace=False))


def pixel_sample(H: int, W: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(H * W, size=min(H * W, N_PIXEL_SAMPLES),
                                                      replace=False))


def fl(a) -> list:
    return [float(x) for x in np.asarray(a, dtype=np.float64).ravel()]


def gradient_record(p, n_iter: int, seed: int) -> dict:
    pb = reg.setup(p.te, p.re, p.V, p.T, p.alpha, TAU)
    L, gu, ga, gt = oadj.gradient(pb, None, n_iter)
    nodes = node_sample(p.n_nodes, seed)
    pix = pixel_sample(p.height, p.width, seed + 1)
    return {"digest": input_digest(p), "n_nodes": p.n_nodes, "height": p.height, "width": p.width,
            "alpha": float(p.alpha), "n_iter": n_iter, "msd": float(L), "g_alpha": float(ga),
            "g_u0_norm": float(np.linalg.norm(gu)), "g_te_norm": float(np.linalg.norm(gt)),
            "node_index": [int(i) for i in nodes], "g_u0_at_nodes": fl(gu[nodes]),
            "pixel_index": [int(i) for i in pix], "g_te_at_pixels": fl(gt.ravel()[pix])}, gu


def make_2048() -> dict:
    t0 = time.time()
    p = make_pair(3)
    n_iter = SPECS[3]["n_iter"]
    pb = reg.setup(p.te, p.re, p.V, p.T, p.alpha, TAU)
    u, _, _ = reg.run(pb, None, n_iter)
    rec, gu = gradient_record(p, n_iter, seed=3100)
    nodes = np.asarray(rec["node_index"])
    rec.update({"u_norm": float(np.linalg.norm(u)), "u_at_nodes": fl(u[nodes]),
                "direction_seed": DIRECTION_SEED,
                "projections": [float(np.sum(gu * d)) for d in
                                random_directions(p.n_nodes, N_DIRECTIONS, DIRECTION_SEED)],
                "fd_step_px": 1e-3, "ckpt_every": SPECS[3]["ckpt_every"]})
    print(f"2048: {p.n_nodes} nodes, {time.time() - t0:.0f} s", flush=True)
    return rec


def make_diff_batch() -> dict:
    t0 = time.time()
    n_iter = SPECS[5]["n_iter"]
    recs = []
    for k in range(4):
        rec, _ = gradient_record(make_pair(5, k), n_iter, seed=5100 + 10 * k)
        rec["pair_index"] = k
        recs.append(rec)
    print(f"diff_batch: {time.time() - t0:.0f} s", flush=True)
    return {"n_pairs_in_batch": SPECS[5]["n_pairs"], "ckpt_every": SPECS[5]["ckpt_every"],
            "pairs": recs}


def batch_picks() -> list:
    """Pair indices: the first pair of the smallest side, the first of the
    largest, the first 384 side, and pair 137 (the side is the first draw of
    each pair's generator)."""
    sides = [int(np.random.default_rng(4000 + k).choice(C4_SIDES)) for k in range(SPECS[4]["n_pairs"])]
    picks = [sides.index(min(sides)), sides.index(max(sides)), sides.index(384), 137]
    return picks


def make_batch() -> dict:
    t0 = time.time()
    n_iter = SPECS[4]["n_iter"]
    recs = []
    for k in batch_picks():
        p = make_pair(4, k)
        pb = reg.setup(p.te, p.re, p.V, p.T, p.alpha, TAU)
        u, _, _ = reg.run(pb, None, n_iter)
        nodes = node_sample(p.n_nodes, 4100 + k)
        recs.append({"pair_index": k, "digest": input_digest(p), "n_nodes": p.n_nodes,
                     "height": p.height, "n_iter": n_iter, "u_norm": float(np.linalg.norm(u)),
                     "node_index": [int(i) for i in nodes], "u_at_nodes": fl(u[nodes]),
                     "msd": float(reg.msd(pb, u))})
    print(f"batch: {time.time() - t0:.0f} s", flush=True)
    return {"n_pairs_in_batch": SPECS[4]["n_pairs"], "pairs": recs}


MAKERS = {"2048": (make_2048, "full_size_2048.json"),
          "diff_batch": (make_diff_batch, "full_size_diff_batch.json"),
          "batch": (make_batch, "full_size_batch.json")}


def main(which) -> None:
    for name in which:
        fn, fname = MAKERS[name]
        rec = fn()
        rec["written_by"] = "tests/golden/make_full_size.py (FP64 oracle)"
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump(rec, f, separators=(",", ":"))
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(MAKERS))
