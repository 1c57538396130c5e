"""Condition numbers of many sparsifiers of seeded meshes, in CPU worker
processes (the oracle's Lanczos estimator; spawned workers never touch the GPU)."""
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _mesh(side, seed):
    import workloads as W

    return W.mesh3d(side, side, side, seed=seed, wdist=("lognormal", 0.0, 1.5))


def _kappa_job(job):
    import oracle

    side, seed, mask = job
    g = _mesh(side, seed)
    return float(oracle.kappa_sparse(g.n, g.u, g.v, g.w, np.asarray(mask, dtype=bool))[0])


def kappa_many(jobs, workers=4):
    """jobs: (side, seed, keep mask) tuples; returns their kappa estimates in order."""
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_kappa_job, jobs))
