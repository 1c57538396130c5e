"""MI355X (gfx950) implementation of the data-parallel hot path of SF-GRASS
(Zhang, Zhao, Feng, ICCAD 2020): smoothing of random vector blocks by
Laplacian sweeps, embedding-distance edge scores, top-k selection,
affinity-driven coarsening, and the sparsifier driver, behind the C ABI in
``include/sfg.h`` (``libsfg.so``).  ``sfg`` is the ctypes binding.
"""
from . import sfg  # noqa: F401

__all__ = ["sfg"]
