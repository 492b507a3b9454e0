"""Torch-facing wrapper around the C ABI: device buffers and streams only.

``MeshReg`` owns one library context (one or many pairs).  Tensors are
allocated with torch on the current device and passed by pointer; every
computation happens in the library's HIP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _stream():
    return torch.cuda.current_stream().cuda_stream


class MeshReg:
    """Registration context for a batch of pairs.

    ``pairs``: sequence of objects or dicts with ``te`` and ``re`` (FP32
    ``[H][W]`` numpy arrays or tensors), ``V`` (int ``[n][2]`` node corners
    ``(x, y)``), ``T`` (int ``[n_T][3]``) and ``alpha``.
    """

    def __init__(self, pairs, tau: float, force_mode: int = B.MR_FORCE_P1,
                 host_only: bool = False, device: str | torch.device = "cuda",
                 apex_rows: int = 0, bwd_split_rows: int = 0, graph: bool = False,
                 tune: bool = True, solve_kernel: int = 0, separate_assembly: bool = False):
        self.host_only = host_only
        self.device = torch.device(device) if not host_only else torch.device("cpu")
        get = (lambda p, k: p[k]) if isinstance(pairs[0], dict) else (lambda p, k: getattr(p, k))
        specs, self._images = [], []
        for p in pairs:
            te, re = get(p, "te"), get(p, "re")
            H, W = int(te.shape[0]), int(te.shape[1])
            spec = dict(V=np.asarray(get(p, "V")), T=np.asarray(get(p, "T")), height=H, width=W,
                        alpha=float(get(p, "alpha")))
            if not host_only:
                tt = torch.as_tensor(np.asarray(te, dtype=np.float32) if not torch.is_tensor(te) else te,
                                     dtype=torch.float32, device=self.device).contiguous()
                rr = torch.as_tensor(np.asarray(re, dtype=np.float32) if not torch.is_tensor(re) else re,
                                     dtype=torch.float32, device=self.device).contiguous()
                spec["te"], spec["re"] = tt, rr
                self._images.append((tt, rr))
            specs.append(spec)
        flags = B.MR_FLAG_HOST_ONLY if host_only else (B.MR_FLAG_GRAPH if graph else 0)
        if not tune:
            flags |= B.MR_FLAG_NO_TUNE
        if separate_assembly:
            flags |= B.MR_FLAG_SEPARATE_ASSEMBLY
        stream = None if host_only else _stream()
        self.ctx = B.mesh_reg_init(specs, tau, force_mode, flags, stream, apex_rows, bwd_split_rows,
                                   solve_kernel)
        self._images = []          # the library keeps its own copies
        self.tau = float(tau)
        self.n_pairs = len(pairs)
        self.shapes = [(s["height"], s["width"]) for s in specs]
        self._alpha = [s["alpha"] for s in specs]       # each pair's alpha in the library
        self.template_version = 0                         # counts set_template calls
        self.n_nodes = [int(s["V"].shape[0]) for s in specs]
        self.node_offsets = np.concatenate([[0], np.cumsum(self.n_nodes)]).astype(np.int64)
        self.pixel_offsets = np.concatenate(
            [[0], np.cumsum([h * w for h, w in self.shapes])]).astype(np.int64)

    # -- buffers -------------------------------------------------------------
    @property
    def total_nodes(self) -> int:
        return int(self.node_offsets[-1])

    @property
    def total_pixels(self) -> int:
        return int(self.pixel_offsets[-1])

    def zeros_u(self) -> torch.Tensor:
        return torch.zeros((self.total_nodes, 2), dtype=torch.float64, device=self.device)

    def pair_slice(self, x: torch.Tensor, pair: int) -> torch.Tensor:
        return x[self.node_offsets[pair]:self.node_offsets[pair + 1]]

    def pixel_slice(self, x: torch.Tensor, pair: int) -> torch.Tensor:
        H, W = self.shapes[pair]
        return x[self.pixel_offsets[pair]:self.pixel_offsets[pair + 1]].view(H, W)

    # -- the method ------------------------------------------------------------
    def step(self, u: torch.Tensor, n_iter: int, record_msd: bool = False):
        """``n_iter`` iterations in place on ``u``; returns the MSD trace if asked."""
        trace = (torch.empty((n_iter, self.n_pairs), dtype=torch.float64, device=self.device)
                 if record_msd else None)
        B.mesh_reg_step(self.ctx, u, n_iter, trace, _stream())
        return trace

    def step_explicit(self, u: torch.Tensor, n_iter: int, tau: float, lam: float = 0.8,
                      record_msd: bool = False):
        """Algorithm 1 as printed (explicit update with the mesh gradient on the
        deformed mesh, one umbrella smoothing), ``n_iter`` iterations in place."""
        trace = (torch.empty((n_iter, self.n_pairs), dtype=torch.float64, device=self.device)
                 if record_msd else None)
        B.mesh_reg_step_explicit(self.ctx, u, n_iter, tau, lam, trace, _stream())
        return trace

    def run(self, u: torch.Tensor, max_iter: int, check_every: int = 10, rel_tol: float = 1e-3):
        """Iterates in place until each pair's MSD falls by less than ``rel_tol``
        (relative) over ``check_every`` iterations, at most ``max_iter``; a pair
        that stops keeps its u while the others go on.  Returns ``(iters, msd)``:
        the per-pair iteration counts (list) and the final MSDs (device FP64)."""
        msd = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        iters = B.mesh_reg_run(self.ctx, u, max_iter, check_every, rel_tol, self.n_pairs, msd,
                               _stream())
        return iters, msd

    def warp_msd(self, u: torch.Tensor, return_warped: bool = False):
        msd = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        warped = (torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
                  if return_warped else None)
        B.mesh_reg_warp_msd(self.ctx, u, msd, warped, _stream())
        return (msd, warped) if return_warped else msd

    def force(self, u: torch.Tensor):
        h = torch.empty((self.total_nodes, 2), dtype=torch.float32, device=self.device)
        b = torch.empty((self.total_nodes, 2), dtype=torch.float64, device=self.device)
        B.mesh_reg_force(self.ctx, u, h, b, _stream())
        return h, b

    def solve(self, b: torch.Tensor) -> torch.Tensor:
        x = torch.empty_like(b)
        B.mesh_reg_solve(self.ctx, b.contiguous(), x, _stream())
        return x

    def backward(self, u0: torch.Tensor, n_iter: int, ckpt_every: int = 10, g_msd=None,
                 want_u0: bool = True, want_alpha: bool = True, want_te: bool = True):
        """Gradients of ``sum_p g_msd[p] MSD_p(u^N)``: ``(msd, g_u0, g_alpha, g_te)``."""
        if g_msd is None:
            g_msd = torch.ones(self.n_pairs, dtype=torch.float64, device=self.device)
        g_u0 = torch.empty_like(u0) if want_u0 else None
        g_alpha = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device) if want_alpha else None
        g_te = (torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
                if want_te else None)
        msd = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        B.mesh_reg_backward(self.ctx, u0.contiguous(), n_iter, ckpt_every, g_msd.contiguous(),
                            g_u0, g_alpha, g_te, msd, _stream())
        return msd, g_u0, g_alpha, g_te

    def checkpoints(self, n_iter: int, ckpt_every: int) -> torch.Tensor:
        """A checkpoint buffer for ``forward_ckpt``: ``[ceil(n_iter / ckpt_every) + 1][sum n][2]``."""
        n_seg = -(-int(n_iter) // int(ckpt_every))
        return torch.empty((n_seg + 1, self.total_nodes, 2), dtype=torch.float64, device=self.device)

    def forward_ckpt(self, u: torch.Tensor, n_iter: int, ckpt_every: int = 10, ckpt=None):
        """``n_iter`` iterations in place on ``u`` that also write the
        checkpoints the reverse pass needs; returns ``(msd, ckpt)`` with the
        per-pair MSD of the final ``u``."""
        if ckpt is None:
            ckpt = self.checkpoints(n_iter, ckpt_every)
        msd = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        B.mesh_reg_forward_ckpt(self.ctx, u, n_iter, ckpt_every, ckpt, msd, _stream())
        return msd, ckpt

    def backward_ckpt(self, ckpt: torch.Tensor, n_iter: int, ckpt_every: int = 10, g_msd=None,
                      want_u0: bool = True, want_alpha: bool = True, want_te: bool = True):
        """Gradients as ``backward`` from the checkpoints ``forward_ckpt`` wrote
        (no forward pass of its own): ``(msd, g_u0, g_alpha, g_te)``."""
        if g_msd is None:
            g_msd = torch.ones(self.n_pairs, dtype=torch.float64, device=self.device)
        g_u0 = (torch.empty((self.total_nodes, 2), dtype=torch.float64, device=self.device)
                if want_u0 else None)
        g_alpha = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device) if want_alpha else None
        g_te = (torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
                if want_te else None)
        msd = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        B.mesh_reg_backward_ckpt(self.ctx, ckpt, n_iter, ckpt_every, g_msd.contiguous(), g_u0,
                                 g_alpha, g_te, msd, _stream())
        return msd, g_u0, g_alpha, g_te

    def set_alpha(self, pair: int, alpha: float) -> None:
        """Re-factorises pair ``pair`` for ``alpha`` (skipped when it already has it)."""
        alpha = float(alpha)
        if self._alpha[pair] == alpha:
            return
        B.mesh_reg_set_alpha(self.ctx, pair, alpha, None if self.host_only else _stream())
        self._alpha[pair] = alpha

    def set_template(self, pair: int, te: torch.Tensor) -> None:
        B.mesh_reg_set_template(self.ctx, pair, te.contiguous(), _stream())
        self.template_version += 1

    def alphas(self) -> list:
        """Each pair's alpha as the library holds it."""
        return list(self._alpha)

    # -- introspection -------------------------------------------------------------
    def table(self, pair: int, name: str) -> np.ndarray:
        return B.mesh_reg_get_tables(self.ctx, pair, name)

    def info(self, pair: int, key: str) -> int:
        return B.mesh_reg_get_info(self.ctx, pair, key)

    def enable_timing(self, on: bool = True) -> None:
        B.mesh_reg_enable_timing(self.ctx, on)

    def set_graph(self, on: bool) -> None:
        """Graph replay of ``step`` on or off (off drops the cached graph)."""
        B.mesh_reg_set_graph(self.ctx, on)

    def kernel_times(self) -> dict:
        return B.mesh_reg_kernel_times(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            B.mesh_reg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
