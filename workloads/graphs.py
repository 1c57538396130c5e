"""Seeded generators for the synthetic workloads (canonical edge lists).

Every generator returns a :class:`Graph` whose edge list is canonical: ``u < v``,
sorted by ``(u, v)``, unique, connected.  Weights are drawn after the edge list
is in canonical order, so the i-th weight belongs to edge id i.  All random
numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class Graph:
    n: int
    u: np.ndarray            # int32[m]
    v: np.ndarray            # int32[m]
    w: np.ndarray            # float64[m]; exact widening when the workload states FP32 weights
    name: str = ""
    w32: Optional[np.ndarray] = None   # float32[m] when the workload's weights are FP32
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.u.shape[0])


# ----------------------------------------------------------------------------
# helpers (index bookkeeping only)
# ----------------------------------------------------------------------------

def _canonical(n: int, a: np.ndarray, b: np.ndarray):
    """Order endpoints, drop self loops and duplicates, sort by (u, v)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    keep = lo != hi
    key = np.unique(lo[keep] * n + hi[keep])
    return (key // n).astype(np.int32), (key % n).astype(np.int32)


def _largest_component(n: int, u: np.ndarray, v: np.ndarray, extra: dict):
    """Keep the largest connected component, relabelling nodes in ascending order.

    ``extra`` maps names to per-edge arrays that are filtered alongside.
    """
    adj = sp.coo_matrix((np.ones(u.shape[0], dtype=np.int8), (u, v)), shape=(n, n))
    ncomp, lab = connected_components(adj, directed=False)
    if ncomp == 1:
        return n, u, v, extra
    sizes = np.bincount(lab)
    big = int(np.argmax(sizes))
    keep_node = lab == big
    newid = np.full(n, -1, dtype=np.int64)
    newid[keep_node] = np.arange(int(keep_node.sum()))
    ek = keep_node[u]          # both endpoints share a component
    u2 = newid[u[ek]].astype(np.int32)
    v2 = newid[v[ek]].astype(np.int32)
    extra2 = {k: arr[ek] for k, arr in extra.items()}
    # relabelling is monotone, so (u, v) order is preserved
    return int(keep_node.sum()), u2, v2, extra2


def _weights(rng, m: int, dist: tuple):
    kind = dist[0]
    if kind == "uniform":
        return rng.uniform(dist[1], dist[2], m)
    if kind == "lognormal":
        return rng.lognormal(dist[1], dist[2], m)
    if kind == "unit":
        return np.ones(m)
    raise ValueError(f"unknown weight distribution {dist!r}")


# ----------------------------------------------------------------------------
# families
# ----------------------------------------------------------------------------

def grid2d(nx: int, ny: int, seed: int, wdist=("uniform", 0.5, 2.0)) -> Graph:
    """nx-by-ny 4-neighbour grid; node id = i*ny + j; edges right and down."""
    n = nx * ny
    p = np.arange(n, dtype=np.int64)
    i, j = p // ny, p % ny
    right = np.where(j < ny - 1, p + 1, -1)
    down = np.where(i < nx - 1, p + ny, -1)
    vv = np.stack([right, down], axis=1).reshape(-1)       # per node: +1 then +ny
    uu = np.repeat(p, 2)
    ok = vv >= 0
    u, v = uu[ok].astype(np.int32), vv[ok].astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _weights(rng, u.shape[0], wdist)
    return Graph(n, u, v, w, name=f"grid{nx}x{ny}")


def powergrid(nx: int, ny: int, frac: float, seed: int, wdist=("lognormal", 0.0, 1.0)) -> Graph:
    """Grid plus ``round(frac * grid edges)`` cell-diagonal shortcuts.

    Diagonal slots: every cell (i, j), i < nx-1, j < ny-1 has two, slot 2c is
    (i,j)-(i+1,j+1) and slot 2c+1 is (i,j+1)-(i+1,j).  They are sampled without
    replacement, then all weights are drawn in canonical edge order.
    """
    n = nx * ny
    g = grid2d(nx, ny, seed, wdist=("unit",))
    mg = g.m
    nd = int(round(frac * mg))
    rng = np.random.Generator(np.random.PCG64(seed))
    slots = rng.choice((nx - 1) * (ny - 1) * 2, size=nd, replace=False)
    c, t = slots // 2, slots % 2
    ci, cj = c // (ny - 1), c % (ny - 1)
    du = np.where(t == 0, ci * ny + cj, ci * ny + cj + 1)
    dv = np.where(t == 0, (ci + 1) * ny + cj + 1, (ci + 1) * ny + cj)
    u, v = _canonical(n, np.concatenate([g.u, du]), np.concatenate([g.v, dv]))
    w = _weights(rng, u.shape[0], wdist)
    return Graph(n, u, v, w, name=f"powergrid{nx}x{ny}+{frac:g}diag", meta={"diagonals": nd})


def knn3d(npts: int, k: int, seed: int) -> Graph:
    """Symmetrised k-NN graph of ``npts`` points uniform in [0,1]^3.

    Weight exp(-d^2/h^2), h = median of the npts*k directed k-NN distances;
    union symmetrisation; largest connected component.  FP64 weights, with an
    FP32 copy for reduced-precision runs.
    """
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((npts, 3))
    tree = cKDTree(pts)
    dist, idx = tree.query(pts, k=k + 1, workers=-1)
    dist, idx = dist[:, 1:], idx[:, 1:]        # drop self
    h = float(np.median(dist))
    a = np.repeat(np.arange(npts, dtype=np.int64), k)
    u, v = _canonical(npts, a, idx.reshape(-1))
    d2 = np.sum((pts[u] - pts[v]) ** 2, axis=1)
    w = np.exp(-d2 / (h * h))
    n, u, v, ex = _largest_component(npts, u, v, {"w": w})
    w = ex["w"]
    return Graph(n, u, v, w, name=f"knn3d_{npts}_k{k}", w32=w.astype(np.float32),
                 meta={"h": h, "points": npts})


def _chung_lu_i0(n: int, total: float, alpha: float) -> float:
    """Smallest offset i0 with w_max^2 <= sum(w) for w_i = c (i+i0)^-alpha, sum = total."""
    idx = np.arange(n, dtype=np.float64)

    def ok(i0):
        s = np.sum((idx + i0) ** (-alpha))
        c = total / s
        wmax = c * i0 ** (-alpha)
        return wmax * wmax <= total

    lo, hi = 1.0, 1.0
    while not ok(hi):
        hi *= 2.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


def chung_lu(n: int, m_pairs: int, gamma: float, seed: int, wdist=("uniform", 1.0, 10.0)) -> Graph:
    """Chung-Lu expected-degree graph with power-law exponent ``gamma``.

    Expected degrees w_i = c (i+i0)^(-1/(gamma-1)) with sum 2*m_pairs; endpoints
    of m_pairs pairs drawn iid proportional to w; self loops and duplicates are
    dropped; largest component kept.  FP32 weights.
    """
    alpha = 1.0 / (gamma - 1.0)
    total = 2.0 * m_pairs
    i0 = _chung_lu_i0(n, total, alpha)
    wexp = (np.arange(n, dtype=np.float64) + i0) ** (-alpha)
    wexp *= total / wexp.sum()
    cdf = np.cumsum(wexp)
    cdf /= cdf[-1]
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.searchsorted(cdf, rng.random(m_pairs), side="right")
    b = np.searchsorted(cdf, rng.random(m_pairs), side="right")
    np.minimum(a, n - 1, out=a)
    np.minimum(b, n - 1, out=b)
    u, v = _canonical(n, a, b)
    del a, b
    n2, u, v, _ = _largest_component(n, u, v, {})
    w32 = _weights(rng, u.shape[0], wdist).astype(np.float32)
    return Graph(n2, u, v, w32.astype(np.float64), name=f"chunglu_{n}_g{gamma:g}", w32=w32,
                 meta={"i0": i0, "wmax": float(wexp[0]), "pairs": m_pairs})


def mesh3d(nx: int, ny: int, nz: int, seed: int, wdist=("lognormal", 0.0, 1.5)) -> Graph:
    """3-D 7-point mesh; node id = (i*ny + j)*nz + k; edges +k, +j, +i."""
    n = nx * ny * nz
    p = np.arange(n, dtype=np.int64)
    k = p % nz
    j = (p // nz) % ny
    i = p // (ny * nz)
    e1 = np.where(k < nz - 1, p + 1, -1)
    e2 = np.where(j < ny - 1, p + nz, -1)
    e3 = np.where(i < nx - 1, p + ny * nz, -1)
    vv = np.stack([e1, e2, e3], axis=1).reshape(-1)
    del e1, e2, e3, i, j, k
    ok = vv >= 0
    u = np.repeat(p, 3)[ok].astype(np.int32)
    v = vv[ok].astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _weights(rng, u.shape[0], wdist)
    return Graph(n, u, v, w, name=f"mesh{nx}x{ny}x{nz}")


def random_connected(n: int, extra: int, seed: int, wdist=("uniform", 0.5, 2.0)) -> Graph:
    """Random recursive tree plus ``extra`` random chords (connected by construction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64) if n > 1 \
        else np.zeros(0, dtype=np.int64)
    a = np.concatenate([np.arange(1, n), rng.integers(0, n, extra)])
    b = np.concatenate([parent, rng.integers(0, n, extra)])
    u, v = _canonical(n, a, b)
    w = _weights(rng, u.shape[0], wdist)
    return Graph(n, u, v, w, name=f"rand{n}+{extra}")


def random_block(n: int, k: int, seed: int) -> np.ndarray:
    """n-by-k block of iid N(0,1) FP64 values, row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, k))


# ----------------------------------------------------------------------------
# named workloads (graph seed; random blocks use seed 1000 + 10 * seed + index)
# ----------------------------------------------------------------------------

WORKLOADS = {
    "grid64": dict(name="grid64x64", seed=1, k=8, sweeps=10, frac=0.05, dtype="f64"),
    "powergrid": dict(name="powergrid1000x1000+2%diag", seed=2, k=16, sweeps=20, frac=0.10, dtype="f64"),
    "knn": dict(name="knn3d_2M_k10", seed=3, k=32, sweeps=20, frac=0.10, dtype="f16", band=0.01),
    "chunglu": dict(name="chunglu_4M_g2.2", seed=4, k=16, sweeps=20, frac=0.10, dtype="f32", levels=5),
    "mesh": dict(name="mesh200x200x200", seed=5, k=16, sweeps=20, frac=0.10, dtype="f32", cand_frac=0.20),
}


def workload_params(name: str) -> dict:
    return dict(WORKLOADS[name])


def workload_graph(name: str, scale: float = 1.0) -> Graph:
    """Graph of a named workload; ``scale`` < 1 gives a same-shaped smaller case."""
    seed = WORKLOADS[name]["seed"]
    if name == "grid64":
        return grid2d(64, 64, seed=seed)
    if name == "powergrid":
        s = max(8, int(round(1000 * scale)))
        return powergrid(s, s, 0.02, seed=seed)
    if name == "knn":
        return knn3d(max(2000, int(round(2_000_000 * scale))), 10, seed=seed)
    if name == "chunglu":
        nn = max(4000, int(round(4_000_000 * scale)))
        return chung_lu(nn, int(round(40_000_000 * scale)), 2.2, seed=seed)
    if name == "mesh":
        s = max(4, int(round(200 * scale ** (1.0 / 3.0))))
        return mesh3d(s, s, s, seed=seed)
    raise ValueError(name)


def workload_block(name: str, n: int, level: int = 0, k: Optional[int] = None) -> np.ndarray:
    """The workload's random block number ``level`` (a level or a round)."""
    kk = WORKLOADS[name]["k"] if k is None else k
    return random_block(n, kk, 1000 + 10 * WORKLOADS[name]["seed"] + level)
