"""Seeded synthetic graphs and random vector blocks.

This module is the only code shared by the oracle side and the GPU side of the
tests and the benchmark.  It draws numbers and builds canonical edge lists; it
holds none of the sparsification method's arithmetic (no Laplacian, smoothing,
scoring, selection, spanning tree or coarsening).

Canonical edge list: int32 arrays ``u``, ``v`` with ``u < v``, sorted by
``(u, v)``, unique, node ids in ``[0, n)``, plus positive finite weights
``w``.  The edge id is the list index.

Workload families (stand-ins for the paper's circuit, mesh and real-world
matrices, which are not available):

* ``grid2d``      -- 2-D 4-neighbour grid (the 64x64 case; also small meshes)
* ``powergrid``   -- 2-D grid plus a fraction of random cell-diagonal shortcuts
* ``knn3d``       -- symmetrised k-nearest-neighbour graph of uniform 3-D points
                     with Gaussian-kernel weights
* ``chung_lu``    -- power-law random graph (expected-degree model)
* ``mesh3d``      -- 3-D 7-point mesh

Seeds: graph seed = configuration number, vector seed = 1000 + 10*config + level.
"""
from .graphs import (  # noqa: F401
    Graph,
    grid2d,
    powergrid,
    knn3d,
    chung_lu,
    mesh3d,
    random_connected,
    random_block,
    workload_graph,
    workload_params,
    WORKLOADS,
    workload_block,
)
