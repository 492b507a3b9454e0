"""Small seeded problems shared by the oracle and parity tests (inputs only)."""
import numpy as np

from synth import quadtree_mesh, unstructured_mesh
from synth.images import draw_params, make_images, textured_translation_pair


def small_pair(seed=0, side=32, s_min=2, s_max=16, g=0.05, amp=3.0, n_blobs=4, quant=False):
    rng = np.random.default_rng(seed)
    te, re = make_images(draw_params(rng, side, side, amp, n_blobs=n_blobs), quantise=quant)
    V, T, leaves = quadtree_mesh(te, s_min, s_max, g)
    return te, re, V, T, leaves


def translation_pair(side=128, shift=(1.0, -2.0), seed=11, s_min=2, s_max=16, g=0.05):
    te, re = textured_translation_pair(side, side, shift, seed)
    V, T, leaves = quadtree_mesh(te, s_min, s_max, g)
    return te, re, V, T, leaves


def unstructured_pair(seed=7, side=64, s_min=1, s_max=16, g=0.05, amp=3.0, n_blobs=4):
    """Images as small_pair, mesh from synth.unstructured (irregular valence,
    edges in all directions)."""
    rng = np.random.default_rng(seed)
    te, re = make_images(draw_params(rng, side, side, amp, n_blobs=n_blobs))
    V, T = unstructured_mesh(te, s_min, s_max, g, seed=seed)
    return te, re, V, T
