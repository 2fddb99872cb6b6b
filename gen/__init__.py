"""Seeded synthetic inputs shared by the oracle and the GPU path (data only)."""
from .graphs import Graph, grid2d, grid3d_box, gnp, grid3d_seg, grid3d_seg_slab, rmat_flowimprove, rmat_batch, workload, smooth_field  # noqa: F401
