"""CPU tests of the library's host side: the C ABI loads and exports every
declared symbol, tables T1-T6 equal the oracle's bit for bit, the ordering is
a permutation, and invalid inputs are rejected with the documented codes.
No GPU work is launched (contexts are built host-only)."""
import os
import re

import numpy as np
import pytest

from oracle import mesh as omesh
from synth import make_pair, uniform_mesh
from tests._problems import small_pair, unstructured_pair

import paper_1411_2141_amd as pkg
from paper_1411_2141_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "meshreg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mesh_reg_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == names


def host_ctx(pairs, tau=0.5, force_mode=0):
    return pkg.MeshReg(pairs, tau=tau, force_mode=force_mode, host_only=True)


def _pairs_for_tables():
    out = []
    te, re_, V, T, _ = small_pair(seed=1, side=48, s_min=1, s_max=16)
    out.append(dict(te=te, re=re_, V=V, T=T, alpha=0.1))
    p = make_pair(1)
    out.append(dict(te=p.te, re=p.re, V=p.V, T=p.T, alpha=p.alpha))
    V, T, _ = uniform_mesh(24, 40, 4)     # ragged, non-square
    out.append(dict(te=np.zeros((24, 40), np.float32), re=np.zeros((24, 40), np.float32),
                    V=V, T=T, alpha=0.3))
    te, re_, V, T = unstructured_pair(seed=9, side=48)     # general triangulation
    out.append(dict(te=te, re=re_, V=V, T=T, alpha=0.15))
    return out


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_tables_bit_exact_with_oracle(k):
    pair = _pairs_for_tables()[k]
    H, W = pair["te"].shape
    ctx = host_ctx([pair])
    want = omesh.tables(pair["V"], pair["T"], H, W)
    for name in ("t1_ptr", "t1_slot", "t2_ptr", "t2_idx", "t3_ptr", "t3_idx", "t4", "t5"):
        got = ctx.table(0, name)
        assert got.dtype == np.int64
        assert np.array_equal(got, want[name]), name
    assert np.array_equal(ctx.table(0, "t6").reshape(H, W), want["t6"])
    perm = ctx.table(0, "perm")
    assert np.array_equal(np.sort(perm), np.arange(pair["V"].shape[0]))
    assert ctx.info(0, "nnz_l") >= pair["V"].shape[0]
    assert ctx.info(0, "fwd_levels") >= 1 and ctx.info(0, "bwd_levels") >= 1
    ctx.close()


def test_tile_entries_count_distinct_triangles_per_pixel_tile():
    """MR_INFO_TILE_ENTRIES: the warp's per-tile triangle lists hold the
    distinct T6 triangles of each 16 x 16 pixel tile (T6 from the oracle)."""
    for pair in _pairs_for_tables():
        H, W = pair["te"].shape
        t6 = omesh.tables(pair["V"], pair["T"], H, W)["t6"]
        want = sum(len(np.unique(t6[y:y + 16, x:x + 16]))
                   for y in range(0, H, 16) for x in range(0, W, 16))
        ctx = host_ctx([pair])
        assert ctx.info(0, "tile_entries") == want
        ctx.close()


def test_batched_tables_per_pair():
    pairs = _pairs_for_tables()
    ctx = host_ctx(pairs)
    assert ctx.info(0, "n_pairs") == 4
    for k, pair in enumerate(pairs):
        H, W = pair["te"].shape
        want = omesh.tables(pair["V"], pair["T"], H, W)
        assert np.array_equal(ctx.table(k, "t1_slot"), want["t1_slot"])
        assert np.array_equal(ctx.table(k, "t6").reshape(H, W), want["t6"])
        assert ctx.info(k, "node_offset") == sum(p["V"].shape[0] for p in pairs[:k])
    ctx.close()


def _one_leaf():
    V, T, _ = uniform_mesh(4, 4, 4)
    z = np.zeros((4, 4), np.float32)
    return dict(te=z, re=z, V=V, T=T, alpha=0.1)


def _expect(code, pair=None, **kw):
    pair = pair or _one_leaf()
    with pytest.raises(B.MeshRegError) as ei:
        host_ctx([pair], **kw)
    assert ei.value.code == code
    return str(ei.value)


def test_invalid_inputs_are_rejected():
    p = _one_leaf()
    host_ctx([p]).close()
    bad = dict(p, T=p["T"].copy())
    bad["T"][0, 0] = 99
    assert "out of range" in _expect(B.MR_EINVAL, bad)
    bad = dict(p, T=p["T"][:, [0, 2, 1]].copy())
    assert "area" in _expect(B.MR_EINVAL, bad)
    bad = dict(p, V=np.vstack([p["V"], [[1, 1]]]))
    assert "not used" in _expect(B.MR_EINVAL, bad)
    bad = dict(p, T=p["T"][:1].copy())                   # half the square uncovered
    bad["V"] = p["V"]
    msg = _expect(B.MR_EINVAL, bad)
    assert "not used" in msg or "not covered" in msg
    bad = dict(p, V=p["V"] * 2)                         # outside the image
    assert "outside" in _expect(B.MR_EINVAL, bad)
    _expect(B.MR_EINVAL, tau=0.0)
    _expect(B.MR_EINVAL, tau=float("nan"))
    _expect(B.MR_EINVAL, dict(p, alpha=-1.0))
    _expect(B.MR_EINVAL, dict(p, alpha=float("inf")))
    # image sides up to 65535 (triangle corners are packed as 16-bit pairs)
    wide = np.zeros((1, 65536), np.float32)
    Vw = np.array([[0, 0], [65536, 0], [0, 1], [65536, 1]], np.int32)
    Tw = np.array([[0, 1, 3], [0, 3, 2]], np.int32)
    assert "65536" in _expect(B.MR_EINVAL, dict(te=wide, re=wide, V=Vw, T=Tw, alpha=0.1))
    # at most 2^31 - 1 pixels per image (32-bit offsets within a pair's image);
    # a zero-stride view stands in for the image, whose pixels are never read
    big = np.broadcast_to(np.float32(0.0), (65535, 32769))
    Vb = np.array([[0, 0], [32769, 0], [0, 65535], [32769, 65535]], np.int32)
    assert "2^31" in _expect(B.MR_EINVAL, dict(te=big, re=big, V=Vb, T=Tw, alpha=0.1))


def test_uncovered_pixel_is_rejected():
    # two triangles of a 4x4 leaf inside an 8x4 image: the right half is uncovered
    V, T, _ = uniform_mesh(4, 4, 4)
    z = np.zeros((4, 8), np.float32)
    assert "not covered" in _expect(B.MR_EINVAL, dict(te=z, re=z, V=V, T=T, alpha=0.1))


def test_host_only_context_refuses_device_calls():
    ctx = host_ctx([_one_leaf()])
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_step(ctx.ctx, None, 1)
    assert ei.value.code in (B.MR_ESTATE, B.MR_EINVAL)
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_run(ctx.ctx, None, 10, 5, 0.01, 1, None)
    assert ei.value.code == B.MR_ESTATE
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_step_explicit(ctx.ctx, None, 1, 20.0, 0.8)
    assert ei.value.code == B.MR_ESTATE
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_forward_ckpt(ctx.ctx, None, 4, 2, None)
    assert ei.value.code == B.MR_ESTATE
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_backward_ckpt(ctx.ctx, None, 4, 2, None)
    assert ei.value.code == B.MR_ESTATE
    ctx.close()


def test_set_alpha_host_only_and_rejects_negative():
    te, re_, V, T, _ = small_pair(seed=2, side=32)
    ctx = host_ctx([dict(te=te, re=re_, V=V, T=T, alpha=0.1)])
    ctx.set_alpha(0, 0.7)
    with pytest.raises(B.MeshRegError) as ei:
        ctx.set_alpha(0, -0.5)
    assert ei.value.code == B.MR_EINVAL
    ctx.close()


def test_overflowing_alpha_is_not_positive_definite_and_leaves_the_factor():
    """tau alpha K overflows the pivots for alpha near the largest double: the
    factorisation reports MR_ENOTSPD, at init and from set_alpha, and a failed
    set_alpha leaves the pair usable (a later set_alpha succeeds)."""
    te, re_, V, T, _ = small_pair(seed=2, side=32)
    with pytest.raises(B.MeshRegError) as ei:
        host_ctx([dict(te=te, re=re_, V=V, T=T, alpha=1e308)])
    assert ei.value.code == B.MR_ENOTSPD
    ctx = host_ctx([dict(te=te, re=re_, V=V, T=T, alpha=0.1)])
    nnz = ctx.info(0, "nnz_l")
    with pytest.raises(B.MeshRegError) as ei:
        B.mesh_reg_set_alpha(ctx.ctx, 0, 1e308, None)
    assert ei.value.code == B.MR_ENOTSPD
    assert ctx.alphas() == [0.1]
    B.mesh_reg_set_alpha(ctx.ctx, 0, 0.7, None)
    assert ctx.info(0, "nnz_l") == nnz
    ctx.close()
