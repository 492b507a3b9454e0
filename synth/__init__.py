"""Seeded synthetic inputs (images, quadtree and unstructured meshes) for the registration path.

This package holds none of the registration arithmetic; it only produces the
inputs that both the HIP library and the FP64 oracle consume.
"""
from .configs import SPECS, Pair, Workload, make_pair, make_pairs, make_workload
from .images import draw_params, make_images, textured_translation_pair
from .quadtree import mesh_from_leaves, quadtree_leaves, quadtree_mesh, uniform_mesh
from .directions import random_directions
from .unstructured import unstructured_mesh

__all__ = ["SPECS", "Pair", "Workload", "make_pair", "make_pairs", "make_workload", "draw_params",
           "make_images", "textured_translation_pair", "mesh_from_leaves",
           "quadtree_leaves", "quadtree_mesh", "uniform_mesh", "unstructured_mesh",
           "random_directions"]
