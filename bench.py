"""Throughput of the registration hot path on one MI355X.

One step = one iteration of the method on the 512x512 12-bit single-pair
workload (quadtree mesh s=1..32, g=0.08; alpha=0.05, tau=0.5): template
sampling at the displaced nodes, P1 force assembly, the two FP64 triangular
solves of (I + tau alpha K), and the full-pixel warp + MSD (every iteration).
The timed region runs exactly ``--steps`` iterations from u = 0 with every
input already resident in device memory.

Prints one JSON line: node-updates/s, plus the dominant kernel's roofline
(algorithmic bytes / HIP-event kernel time) and the FP64 oracle timed on a
bounded sample on the host cores.
"""
from __future__ import annotations

import os

# the oracle baseline runs single-threaded; pin BLAS/OpenMP before numpy loads
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse
import json
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-updates/s per registration iteration, fwd+bwd vs plain; achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(ctx, pair, V, H, W) -> dict:
    """Bytes each kernel family must move per launch (each datum once)."""
    n = int(V.shape[0])
    nt = ctx.info(0, "n_tris")
    nnz_m = ctx.info(0, "mass_nnz")
    off = ctx.info(0, "solve_offblock")
    dense = ctx.info(0, "solve_dense")
    # coefficients touched by the node samples at u = 0 (4x4 taps per node)
    fx = V[:, 0] - 1
    fy = V[:, 1] - 1
    taps = set()
    for dm in range(-1, 3):
        for dn in range(-1, 3):
            r = np.clip(fy + dm, 0, H - 1)
            c = np.clip(fx + dn, 0, W - 1)
            taps.update((r * W + c).tolist())
    sample = 36 * n + 4 * len(taps)                    # u 16, xy 8, rho 4, h 8 + coefficients
    assemble = 48 * n + 8 * nnz_m                       # ptr 4, u 16, iperm 4, h 8, b 16 + col/wt
    solve_call = 2 * (32 * n + 12 * off + 8 * dense + 8 * n) + 4 * n + 16 * n
    warp = 12 * H * W + 24 * n + 16 * nt                # t6, Re, coef per pixel; u, xy; triangles
    return dict(sample=sample, assemble=assemble, solve_call=solve_call, warp=warp)


def cpu_baseline(pair, tau, n_iter_sample: int) -> dict:
    from oracle import registration as reg
    pb = reg.setup(pair.te, pair.re, pair.V, pair.T, pair.alpha, tau)
    u = np.zeros((pair.V.shape[0], 2))
    t0 = time.perf_counter()
    for _ in range(n_iter_sample):
        u = reg.step(pb, u)
        reg.msd(pb, u)
    dt = time.perf_counter() - t0
    return {"value": pair.n_nodes * n_iter_sample / dt, "unit": "node-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {n_iter_sample} iterations (each with warp+MSD) of the same "
                      f"512x512 pair, FP64 NumPy/SciPy oracle with CG solves, 1 thread, "
                      f"{dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=60, help="oracle iterations timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the multi-GPU "
              f"sharding of this path is described in DESIGN.md and not built.", file=sys.stderr)
        return 2

    import torch
    import paper_1411_2141_amd as pkg
    from synth import make_pair

    pair = make_pair(2)
    tau = 0.5
    H, W = pair.height, pair.width
    n = pair.n_nodes
    ctx = pkg.MeshReg([pair], tau=tau)
    u = ctx.zeros_u()
    trace = torch.empty((max(args.steps, args.warmup), 1), dtype=torch.float64, device="cuda")

    def run(k):
        pkg.binding.mesh_reg_step(ctx.ctx, u, k, trace, torch.cuda.current_stream().cuda_stream)

    run(args.warmup)
    torch.cuda.synchronize()
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    final_msd = float(trace[args.steps - 1, 0].item())
    value = n * args.steps / dt

    roof = None
    kernels = {}
    if not args.no_profile:
        u.zero_()
        ctx.enable_timing(True)
        run(args.steps)
        torch.cuda.synchronize()
        times = ctx.kernel_times()
        ctx.enable_timing(False)
        nbytes = algorithmic_bytes(ctx, 0, pair.V, H, W)
        per_launch = {
            "sample": nbytes["sample"], "assemble": nbytes["assemble"], "warp": nbytes["warp"],
            "solve": nbytes["solve_call"] / max(1, times["solve"][1] / max(1, args.steps)),
        }
        for fam, (ms, cnt) in times.items():
            if cnt:
                avg_ms = ms / cnt
                kernels[fam] = {"avg_us": round(avg_ms * 1e3, 3), "launches": cnt,
                                "gbs": round(per_launch[fam] / (avg_ms * 1e-3) / 1e9, 2),
                                "share": round(ms / sum(t[0] for t in times.values()), 4)}
        dom = max(times, key=lambda f: times[f][0])
        ach = kernels[dom]["gbs"]
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": dom,
                "bytes_per_launch": int(per_launch[dom]),
                "avg_launch_us": kernels[dom]["avg_us"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pair, tau, args.cpu_iters)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "single pair 512x512 12-bit blobs+disk, sine warp A=8, quadtree "
                               "s=1..32 g=0.08, alpha=0.05 tau=0.5, warp+MSD every iteration",
                   "nodes": n, "triangles": int(pair.T.shape[0]), "pixels": H * W,
                   "iterations": args.steps, "parallelism": "single GPU",
                   "final_msd": final_msd},
        "kernels": kernels, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
