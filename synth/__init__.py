"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random inputs: images, point clouds, neighbour lists
and initial embeddings.  It contains none of the embedding method's arithmetic
(no edge weights, degrees, system matrices, solves or orthonormalisation); those
live separately in ``oracle/`` (CPU, FP64) and in the HIP library.

All generators use ``numpy.random.default_rng(seed)`` (PCG64) and return
float32 feature arrays, which both sides read as the same exact values.
"""
from .voronoi import voronoi_image, image_features, batch_image_shapes
from .points import gaussian_mixture, knn_edge_list, knn_edge_list_torch
from .embed import smooth_y0, gaussian_y0
from .workloads import (WORKLOADS, BATCHES, EDGE_WORKLOADS, Workload, make_workload, make_batch,
                        make_edges_workload, grid_workload, edges_workload)

__all__ = [
    "voronoi_image", "image_features", "batch_image_shapes",
    "gaussian_mixture", "knn_edge_list", "knn_edge_list_torch", "smooth_y0", "gaussian_y0",
    "WORKLOADS", "BATCHES", "EDGE_WORKLOADS", "Workload", "make_workload", "make_batch",
    "make_edges_workload", "grid_workload", "edges_workload",
]
