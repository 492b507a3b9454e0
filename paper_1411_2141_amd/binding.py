"""ctypes binding of ``include/meshreg.h``: same names, argument marshalling only.

Every step of the registration runs in the HIP library; this module only
turns Python/torch objects into pointers and status codes into exceptions.
If ``libmeshreg.so`` is missing, loading fails loudly -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmeshreg.so")

MR_OK, MR_EINVAL, MR_ENOMEM, MR_EHIP, MR_ENOTSPD, MR_ESTATE, MR_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MR_FORCE_P1, MR_FORCE_NODAL = 0, 1
MR_FLAG_HOST_ONLY = 1
MR_FLAG_GRAPH = 2
MR_FLAG_NO_TUNE = 4
MR_FLAG_SEPARATE_ASSEMBLY = 8
TABLES = {"t1_ptr": 10, "t1_slot": 11, "t2_ptr": 20, "t2_idx": 21, "t3_ptr": 30, "t3_idx": 31,
          "t4": 40, "t5": 50, "t6": 60, "perm": 70}
INFO = {"n_nodes": 1, "n_tris": 2, "nnz_l": 3, "n_blocks": 4, "fwd_levels": 5, "bwd_levels": 6,
        "node_offset": 7, "pixel_offset": 8, "n_pairs": 9, "device_bytes": 10,
        "solve_offblock": 11, "solve_dense": 12, "mass_nnz": 13, "apex_rows": 14,
        "solve_bytes": 15, "fused_assembly": 16, "tile_entries": 17}
KERNEL_FAMILIES = ("sample", "assemble", "solve", "warp")

EXPORTED = ("mesh_reg_init", "mesh_reg_step", "mesh_reg_run", "mesh_reg_step_explicit",
            "mesh_reg_warp_msd", "mesh_reg_warp_msd_noalloc", "mesh_reg_force",
            "mesh_reg_solve", "mesh_reg_backward", "mesh_reg_forward_ckpt",
            "mesh_reg_backward_ckpt", "mesh_reg_set_alpha", "mesh_reg_set_template",
            "mesh_reg_get_tables", "mesh_reg_get_info", "mesh_reg_enable_timing",
            "mesh_reg_kernel_times", "mesh_reg_set_graph", "mesh_reg_destroy",
            "mesh_reg_last_error")


class MeshRegError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"meshreg error {code}: {message}")
        self.code = code


class MrPair(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("n_nodes", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("node_xy", ctypes.c_void_p), ("tris", ctypes.c_void_p),
                ("te", ctypes.c_void_p), ("re", ctypes.c_void_p), ("alpha", ctypes.c_double)]


class MrParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("force_mode", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("apex_rows", ctypes.c_int32),
                ("bwd_split_rows", ctypes.c_int32), ("solve_kernel", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libmeshreg.so`` (built in-tree by ``paper_1411_2141_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1411_2141_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mesh_reg_init": (ctypes.c_int, [ctypes.POINTER(MrPair), i32, ctypes.POINTER(MrParams), vp,
                                         ctypes.POINTER(vp)]),
        "mesh_reg_step": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "mesh_reg_run": (ctypes.c_int, [vp, vp, i32, i32, dbl, ctypes.POINTER(i32), vp, vp]),
        "mesh_reg_step_explicit": (ctypes.c_int, [vp, vp, i32, dbl, dbl, vp, vp]),
        "mesh_reg_warp_msd": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mesh_reg_warp_msd_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mesh_reg_force": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mesh_reg_solve": (ctypes.c_int, [vp, vp, vp, vp]),
        "mesh_reg_backward": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "mesh_reg_forward_ckpt": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        "mesh_reg_backward_ckpt": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "mesh_reg_set_alpha": (ctypes.c_int, [vp, i32, dbl, vp]),
        "mesh_reg_set_template": (ctypes.c_int, [vp, i32, vp, vp]),
        "mesh_reg_get_tables": (ctypes.c_int, [vp, i32, i32, vp, ctypes.POINTER(i64)]),
        "mesh_reg_get_info": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(i64)]),
        "mesh_reg_enable_timing": (ctypes.c_int, [vp, i32]),
        "mesh_reg_kernel_times": (ctypes.c_int, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "mesh_reg_set_graph": (ctypes.c_int, [vp, i32]),
        "mesh_reg_destroy": (None, [vp]),
        "mesh_reg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != MR_OK:
        msg = load_library().mesh_reg_last_error()
        raise MeshRegError(rc, msg.decode() if msg else "")


def _ptr(t) -> int | None:
    """Device pointer of a torch tensor (None stays NULL)."""
    return None if t is None else t.data_ptr()


def mesh_reg_init(pairs: list, tau: float, force_mode: int = MR_FORCE_P1, flags: int = 0,
                  stream: int | None = None, apex_rows: int = 0, bwd_split_rows: int = 0,
                  solve_kernel: int = 0):
    """``pairs``: sequence of dicts with ``V`` (int32 [n][2]), ``T`` (int32 [nT][3]),
    ``te``/``re`` (device FP32 [H][W] tensors, or None with the host-only flag),
    ``height``, ``width`` and ``alpha``.  Returns the opaque context handle."""
    lib = load_library()
    keep = []
    arr = (MrPair * len(pairs))()
    for k, p in enumerate(pairs):
        V = np.ascontiguousarray(p["V"], dtype=np.int32)
        T = np.ascontiguousarray(p["T"], dtype=np.int32)
        keep += [V, T]
        arr[k] = MrPair(int(p["height"]), int(p["width"]), V.shape[0], T.shape[0],
                        V.ctypes.data, T.ctypes.data, _ptr(p.get("te")), _ptr(p.get("re")),
                        float(p["alpha"]))
    params = MrParams(float(tau), int(force_mode), int(flags), int(apex_rows), int(bwd_split_rows),
                      int(solve_kernel))
    out = ctypes.c_void_p()
    _check(lib.mesh_reg_init(arr, len(pairs), ctypes.byref(params), stream, ctypes.byref(out)))
    return out


def mesh_reg_step(ctx, u, n_iter: int, msd_trace=None, stream=None) -> None:
    _check(load_library().mesh_reg_step(ctx, _ptr(u), int(n_iter), _ptr(msd_trace), stream))


def mesh_reg_run(ctx, u, max_iter: int, check_every: int, rel_tol: float, n_pairs: int, msd,
                 stream=None) -> list:
    """Runs to the relative-MSD stopping rule; returns the per-pair iteration counts."""
    iters = (ctypes.c_int32 * n_pairs)()
    _check(load_library().mesh_reg_run(ctx, _ptr(u), int(max_iter), int(check_every),
                                       float(rel_tol), iters, _ptr(msd), stream))
    return list(iters)


def mesh_reg_step_explicit(ctx, u, n_iter: int, tau: float, lam: float, msd_trace=None,
                           stream=None) -> None:
    _check(load_library().mesh_reg_step_explicit(ctx, _ptr(u), int(n_iter), float(tau),
                                                 float(lam), _ptr(msd_trace), stream))


def mesh_reg_warp_msd(ctx, u, msd, warped=None, stream=None) -> None:
    _check(load_library().mesh_reg_warp_msd(ctx, _ptr(u), _ptr(msd), _ptr(warped), stream))

def mesh_reg_warp_msd_noalloc(ctx, u, msd, warped=None, stream=None) -> None:
    """mesh_reg_warp_msd with its partial sums in the library's static device
    scratch (no allocation; calls on one GPU must not overlap)."""
    _check(load_library().mesh_reg_warp_msd_noalloc(ctx, _ptr(u), _ptr(msd), _ptr(warped), stream))


def mesh_reg_force(ctx, u, h=None, b=None, stream=None) -> None:
    _check(load_library().mesh_reg_force(ctx, _ptr(u), _ptr(h), _ptr(b), stream))


def mesh_reg_solve(ctx, b, x, stream=None) -> None:
    _check(load_library().mesh_reg_solve(ctx, _ptr(b), _ptr(x), stream))


def mesh_reg_backward(ctx, u0, n_iter: int, ckpt_every: int, g_msd, g_u0=None, g_alpha=None,
                      g_te=None, msd=None, stream=None) -> None:
    _check(load_library().mesh_reg_backward(ctx, _ptr(u0), int(n_iter), int(ckpt_every),
                                            _ptr(g_msd), _ptr(g_u0), _ptr(g_alpha), _ptr(g_te),
                                            _ptr(msd), stream))


def mesh_reg_forward_ckpt(ctx, u, n_iter: int, ckpt_every: int, ckpt, msd=None,
                          stream=None) -> None:
    _check(load_library().mesh_reg_forward_ckpt(ctx, _ptr(u), int(n_iter), int(ckpt_every),
                                                _ptr(ckpt), _ptr(msd), stream))


def mesh_reg_backward_ckpt(ctx, ckpt, n_iter: int, ckpt_every: int, g_msd, g_u0=None,
                           g_alpha=None, g_te=None, msd=None, stream=None) -> None:
    _check(load_library().mesh_reg_backward_ckpt(ctx, _ptr(ckpt), int(n_iter), int(ckpt_every),
                                                 _ptr(g_msd), _ptr(g_u0), _ptr(g_alpha),
                                                 _ptr(g_te), _ptr(msd), stream))


def mesh_reg_set_alpha(ctx, pair: int, alpha: float, stream=None) -> None:
    _check(load_library().mesh_reg_set_alpha(ctx, int(pair), float(alpha), stream))


def mesh_reg_set_template(ctx, pair: int, te, stream=None) -> None:
    _check(load_library().mesh_reg_set_template(ctx, int(pair), _ptr(te), stream))


def mesh_reg_get_tables(ctx, pair: int, table: str) -> np.ndarray:
    lib = load_library()
    tid = TABLES[table]
    n = ctypes.c_int64()
    _check(lib.mesh_reg_get_tables(ctx, int(pair), tid, None, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.int32 if table in ("t6", "perm") else np.int64)
    _check(lib.mesh_reg_get_tables(ctx, int(pair), tid, out.ctypes.data, ctypes.byref(n)))
    return out


def mesh_reg_get_info(ctx, pair: int, key: str) -> int:
    v = ctypes.c_int64()
    _check(load_library().mesh_reg_get_info(ctx, int(pair), INFO[key], ctypes.byref(v)))
    return int(v.value)


def mesh_reg_enable_timing(ctx, enable: bool) -> None:
    _check(load_library().mesh_reg_enable_timing(ctx, 1 if enable else 0))


def mesh_reg_set_graph(ctx, enable: bool) -> None:
    _check(load_library().mesh_reg_set_graph(ctx, 1 if enable else 0))


def mesh_reg_kernel_times(ctx) -> dict:
    """``{family: (total_ms, launches)}``; resets the accumulated events."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(load_library().mesh_reg_kernel_times(ctx, ms, n))
    return {f: (ms[k], int(n[k])) for k, f in enumerate(KERNEL_FAMILIES)}


def mesh_reg_destroy(ctx) -> None:
    if ctx:
        load_library().mesh_reg_destroy(ctx)


def mesh_reg_last_error() -> str:
    msg = load_library().mesh_reg_last_error()
    return msg.decode() if msg else ""
