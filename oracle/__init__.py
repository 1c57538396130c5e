"""Plain CPU FP64 oracle of the SF-GRASS hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library: its arithmetic lives in ``sfg_oracle.c`` (plain C, FP64,
``-ffp-contract=off``) and in the NumPy/SciPy routines below, and it neither
imports nor loads anything from the product package.

Paper: Zhang, Zhao, Feng, "SF-GRASS: Solver-Free Graph Spectral
Sparsification", ICCAD 2020.  Section / equation / algorithm citations refer
to it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99", "-fopenmp",
           "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        D = ctypes.c_double
        lib.orc_laplacian_csr.argtypes = [I64, I64, P, P, P, P, P, P, P, P]
        lib.orc_laplacian_csr.restype = ctypes.c_int
        lib.orc_smooth.argtypes = [I64, P, P, P, P, I32, I32, D, P, P]
        lib.orc_smooth.restype = None
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox4x32_10.restype = None
        lib.orc_random_block.argtypes = [I64, I32, ctypes.c_uint64, ctypes.c_uint32, P]
        lib.orc_random_block.restype = None
        lib.orc_color.argtypes = [I64, P, P, P]
        lib.orc_color.restype = I32
        lib.orc_smooth_gs.argtypes = [I64, P, P, P, P, I32, I32, D, P, I32, P]
        lib.orc_smooth_gs.restype = None
        lib.orc_smooth_masked.argtypes = [I64, P, P, P, P, I32, I32, D, P, P, P]
        lib.orc_smooth_masked.restype = None
        lib.orc_edge_scores.argtypes = [I32, P, I64, P, P, P, P]
        lib.orc_edge_scores.restype = None
        lib.orc_affinity.argtypes = [I32, P, I64, P, P, P]
        lib.orc_affinity.restype = None
        lib.orc_select_topk.argtypes = [I64, P, P, I64, P, P]
        lib.orc_select_topk.restype = ctypes.c_int
        lib.orc_max_spanning_forest.argtypes = [I64, I64, P, P, P, P, P]
        lib.orc_max_spanning_forest.restype = I64
        lib.orc_components.argtypes = [I64, I64, P, P, P, P]
        lib.orc_components.restype = I64
        lib.orc_aggregate.argtypes = [I64, P, P, P, P, P, P]
        lib.orc_aggregate.restype = I64
        lib.orc_galerkin.argtypes = [I64, P, P, P, P, I64, P, P, P, P]
        lib.orc_galerkin.restype = I64
        lib.orc_exact_sum.argtypes = [I64, P, I64]
        lib.orc_exact_sum.restype = D
        lib.orc_center.argtypes = [I64, I32, P, P]
        lib.orc_center.restype = None
        lib.orc_set_threads.argtypes = [I32]
        lib.orc_set_threads.restype = None
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = I32
        _lib = lib
    return _lib


def set_threads(t: int) -> None:
    """Threads of the row- and edge-parallel loops (smoothing sweeps, scores).
    Each row or edge is computed by one thread in a fixed order, so results
    are the same bits for any count."""
    _L().orc_set_threads(int(t))


def max_threads() -> int:
    return int(_L().orc_max_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

@dataclass
class CSR:
    n: int
    rowptr: np.ndarray   # int64[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    eid: np.ndarray      # int32[nnz]
    deg: np.ndarray      # float64[n]


def laplacian_csr(n: int, u, v, w) -> CSR:
    """L = D - A of the weighted graph (Sec. 2.1, Eq. 1), stored as the CSR of A plus D."""
    u, v, w = _i32(u), _i32(v), _f64(w)
    m = u.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(2 * m, dtype=np.int32)
    val = np.zeros(2 * m, dtype=np.float64)
    eid = np.zeros(2 * m, dtype=np.int32)
    deg = np.zeros(n, dtype=np.float64)
    rc = _L().orc_laplacian_csr(n, m, _p(u), _p(v), _p(w), _p(rowptr), _p(col), _p(val), _p(eid), _p(deg))
    if rc != 0:
        raise MemoryError("orc_laplacian_csr")
    return CSR(n, rowptr, col, val, eid, deg)


def exact_sum(x) -> float:
    x = _f64(x).reshape(-1)
    return float(_L().orc_exact_sum(x.shape[0], _p(x), 1))


def center(X0) -> tuple[np.ndarray, np.ndarray]:
    """Random block made orthogonal to the all-one vector (Sec. 3.2): subtract
    each column's mean, mean = exactly rounded column sum / n."""
    X = np.array(X0, dtype=np.float64, order="C", copy=True)
    n, k = X.shape
    mean = np.zeros(k, dtype=np.float64)
    _L().orc_center(n, k, _p(X), _p(mean))
    return X, mean


def smooth(csr: CSR, X, sweeps: int, omega: float = 0.5) -> np.ndarray:
    """Low-pass smoothing of the block by damped-Jacobi sweeps on L x = 0 (Sec. 3.2)."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    Y = np.empty_like(X)
    k = X.shape[1]
    _L().orc_smooth(csr.n, _p(csr.rowptr), _p(csr.col), _p(csr.val), _p(csr.deg), k, sweeps, omega,
                    _p(X), _p(Y))
    return X


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words and 2 key words to 4 words."""
    c = np.asarray(ctr, dtype=np.uint32)
    kk = np.asarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _L().orc_philox4x32_10(_p(c), _p(kk), _p(out))
    return out


def random_block(n: int, k: int, seed: int, block: int = 0) -> np.ndarray:
    """n-by-k standard normals from (seed, block): Philox4x32-10 counters and Box-Muller."""
    X = np.empty((n, k), dtype=np.float64)
    _L().orc_random_block(n, k, ctypes.c_uint64(seed), ctypes.c_uint32(block), _p(X))
    return X


def color(csr: CSR):
    """Multicolouring for the Gauss-Seidel smoother: Jones-Plassmann rounds with
    a fixed hash priority, smallest free colour.  Returns (color[n], ncolors)."""
    c = np.empty(csr.n, dtype=np.int32)
    nc = _L().orc_color(csr.n, _p(csr.rowptr), _p(csr.col), _p(c))
    return c, int(nc)


def smooth_gs(csr: CSR, X, sweeps: int, omega: float, colors, ncolors: int) -> np.ndarray:
    """Multicolour Gauss-Seidel reading of the smoother (Sec. 3.2): colour by
    colour, in place, each row as in the Jacobi sweep."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    _L().orc_smooth_gs(csr.n, _p(csr.rowptr), _p(csr.col), _p(csr.val), _p(csr.deg), X.shape[1], sweeps, omega,
                       _p(_i32(colors)), ncolors, _p(X))
    return X


def smooth_masked(csr: CSR, X, sweeps: int, omega: float, dist) -> np.ndarray:
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    Y = np.empty_like(X)
    d = _i32(dist)
    _L().orc_smooth_masked(csr.n, _p(csr.rowptr), _p(csr.col), _p(csr.val), _p(csr.deg), X.shape[1],
                           sweeps, omega, _p(d), _p(X), _p(Y))
    return X


def edge_scores(X, u, v, w) -> np.ndarray:
    """Embedding-distance edge scores w_e * |X_p - X_q|^2 (Eq. 18, Alg. 1 distortion)."""
    X = _f64(X)
    u, v, w = _i32(u), _i32(v), _f64(w)
    s = np.zeros(u.shape[0], dtype=np.float64)
    _L().orc_edge_scores(X.shape[1], _p(X), u.shape[0], _p(u), _p(v), _p(w), _p(s))
    return s


def affinity(Xbar, u, v) -> np.ndarray:
    """Algebraic-distance node affinity of the centred block (Sec. 3.2)."""
    Xbar = _f64(Xbar)
    u, v = _i32(u), _i32(v)
    a = np.zeros(u.shape[0], dtype=np.float64)
    _L().orc_affinity(Xbar.shape[1], _p(Xbar), u.shape[0], _p(u), _p(v), _p(a))
    return a


def ksel(frac: float, n_cand: int) -> int:
    """Number of edges recovered: ceil(fl(frac * n_cand))."""
    return int(math.ceil(float(frac) * float(n_cand)))


def select_topk(score, eid, k: int) -> tuple[np.ndarray, float]:
    """Top k by (score desc, edge id asc); returns candidate positions and the k-th score."""
    score, eid = _f64(score), _i32(eid)
    chosen = np.zeros(max(k, 1), dtype=np.int64)
    tau = ctypes.c_double(0.0)
    rc = _L().orc_select_topk(score.shape[0], _p(score), _p(eid), k, _p(chosen), ctypes.byref(tau))
    if rc != 0:
        raise ValueError("bad k")
    return chosen[:k], float(tau.value)


def max_spanning_forest(n: int, u, v, w, allowed=None) -> tuple[np.ndarray, int]:
    """Kruskal maximum-weight spanning forest, order (w desc, eid asc) (Sec. 3.4 MST)."""
    u, v, w = _i32(u), _i32(v), _f64(w)
    intree = np.zeros(u.shape[0], dtype=np.uint8)
    al = None if allowed is None else np.ascontiguousarray(allowed, dtype=np.uint8)
    comps = _L().orc_max_spanning_forest(n, u.shape[0], _p(u), _p(v), _p(w), _p(al), _p(intree))
    return intree, int(comps)


def components(n: int, u, v, mask=None) -> tuple[int, np.ndarray]:
    u, v = _i32(u), _i32(v)
    lab = np.zeros(n, dtype=np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    c = _L().orc_components(n, u.shape[0], _p(u), _p(v), _p(mk), _p(lab))
    return int(c), lab


def aggregate(csr: CSR, aff_entry) -> tuple[np.ndarray, np.ndarray, int]:
    """Aggregation sets from the affinity pointer graph (reading of Sec. 3.2)."""
    a = _f64(aff_entry)
    ptr = np.zeros(csr.n, dtype=np.int32)
    agg = np.zeros(csr.n, dtype=np.int32)
    nc = _L().orc_aggregate(csr.n, _p(csr.rowptr), _p(csr.col), _p(csr.val), _p(a), _p(ptr), _p(agg))
    return agg, ptr, int(nc)


def galerkin(u, v, w, agg, nc: int):
    """Coarse graph L_c = H+^T L H+ as an edge list (Eq. 3-5) plus the heaviest fine edge per coarse edge."""
    u, v, w, agg = _i32(u), _i32(v), _f64(w), _i32(agg)
    m = u.shape[0]
    cu = np.zeros(max(m, 1), dtype=np.int32)
    cv = np.zeros(max(m, 1), dtype=np.int32)
    cw = np.zeros(max(m, 1), dtype=np.float64)
    rep = np.zeros(max(m, 1), dtype=np.int32)
    mc = _L().orc_galerkin(m, _p(u), _p(v), _p(w), _p(agg), nc, _p(cu), _p(cv), _p(cw), _p(rep))
    mc = int(mc)
    return cu[:mc].copy(), cv[:mc].copy(), cw[:mc].copy(), rep[:mc].copy()


# ----------------------------------------------------------------------------
# single-level and multilevel sparsifier (Sec. 3.4-3.6, Alg. 1)
# ----------------------------------------------------------------------------

@dataclass
class LevelResult:
    n: int
    m: int
    n_cand: int
    k_sel: int
    tau: float
    cand: np.ndarray = field(repr=False, default=None)     # candidate edge ids (ascending)
    score: np.ndarray = field(repr=False, default=None)    # FP64 scores of candidates
    chosen: np.ndarray = field(repr=False, default=None)   # chosen edge ids, in rank order


@dataclass
class Result:
    keep: np.ndarray                # uint8[m]: 0 off, 1 sparsifier before additions, 2 recovered
    levels: list                    # LevelResult per scored level (finest last)
    X: Optional[np.ndarray] = None  # smoothed block of the finest scoring pass


def score_level(n, u, v, w, base_mask, X0, k_sweeps, omega, frac, embed="sparsifier", k_take=None,
                smoother="jacobi"):
    """One round of Alg. 1's embed / score / include-top-few on a graph whose
    current sparsifier is ``base_mask``.  ``embed`` selects the smoothed graph:
    'sparsifier' (eigenvectors of L_P, Sec. 3.5) or 'graph' (Alg. 1, embed G).
    ``k_take`` (default ceil(frac * candidates)) is how many edges are added.
    ``smoother``: 'jacobi' (damped Jacobi) or 'gs' (multicolour Gauss-Seidel)."""
    u, v, w = _i32(u), _i32(v), _f64(w)
    base_mask = np.asarray(base_mask, dtype=bool)
    if embed == "sparsifier":
        hu, hv, hw = u[base_mask], v[base_mask], w[base_mask]
    elif embed == "graph":
        hu, hv, hw = u, v, w
    else:
        raise ValueError(embed)
    H = laplacian_csr(n, hu, hv, hw)
    Xc, _ = center(X0)
    if smoother == "gs":
        colors, ncolors = color(H)
        X = smooth_gs(H, Xc, k_sweeps, omega, colors, ncolors)
    elif smoother == "jacobi":
        X = smooth(H, Xc, k_sweeps, omega)
    else:
        raise ValueError(smoother)
    cand = np.nonzero(~base_mask)[0].astype(np.int32)
    s = edge_scores(X, u[cand], v[cand], w[cand])
    k = ksel(frac, cand.shape[0]) if k_take is None else int(k_take)
    pos, tau = select_topk(s, cand, k)
    lr = LevelResult(n, u.shape[0], int(cand.shape[0]), k, tau, cand, s, cand[pos])
    return lr, X


def sparsify_single(n, u, v, w, X0, sweeps, frac, omega=0.5, embed="sparsifier", smoother="jacobi") -> Result:
    """Spanning tree plus the top f of off-tree edges by embedding-distance score."""
    intree, comps = max_spanning_forest(n, u, v, w)
    if comps != 1:
        raise ValueError("graph is not connected")
    lr, X = score_level(n, u, v, w, intree.astype(bool), X0, sweeps, omega, frac, embed, smoother=smoother)
    keep = intree.astype(np.uint8)
    keep[lr.chosen] = 2
    return Result(keep, [lr], X)


def round_quotas(k_total, rounds):
    """Near-equal shares of k_total over ``rounds`` rounds (they sum to k_total)."""
    return [k_total * (r + 1) // rounds - k_total * r // rounds for r in range(rounds)]


def sparsify_rounds(n, u, v, w, X0s, rounds, sweeps, frac, omega=0.5, embed="sparsifier") -> Result:
    """Multi-round densification of the single-level method: the budget
    k_sel = ceil(f * off-tree edges) is split into ``rounds`` near-equal quotas;
    round r re-embeds the block X0s[r] on the current sparsifier (the tree plus
    the edges added so far, whose Laplacian the perturbation analysis of
    Sec. 3.5 is about), scores the edges outside it and adds its quota's top
    edges.  rounds = 1 is sparsify_single."""
    intree, comps = max_spanning_forest(n, u, v, w)
    if comps != 1:
        raise ValueError("graph is not connected")
    base = intree.astype(bool)
    keep = intree.astype(np.uint8)
    k_total = ksel(frac, int((~base).sum()))
    results, X = [], None
    for r, q in enumerate(round_quotas(k_total, rounds)):
        lr, X = score_level(n, u, v, w, base, X0s[r], sweeps, omega, frac, embed, k_take=q)
        keep[lr.chosen] = 2
        base[lr.chosen] = True
        results.append(lr)
    return Result(keep, results, X)


@dataclass
class Level:
    n: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    agg: Optional[np.ndarray] = None      # aggregate of each node (to the next coarser level)
    nc: int = 0
    rep: Optional[np.ndarray] = None      # per coarse edge: heaviest fine edge of this level


def coarsen_level(n, u, v, w, X0, sweeps, omega=0.5):
    """One spectral-coarsening step (Sec. 3.2-3.3): smooth on G, affinities,
    aggregation, Galerkin coarse graph."""
    G = laplacian_csr(n, u, v, w)
    Xc, _ = center(X0)
    X = smooth(G, Xc, sweeps, omega)
    Xbar, _ = center(X)
    a_edge = affinity(Xbar, u, v)
    a_entry = a_edge[G.eid]
    agg, ptr, nc = aggregate(G, a_entry)
    cu, cv, cw, rep = galerkin(u, v, w, agg, nc)
    return agg, nc, cu, cv, cw, rep, a_edge


def sparsify_multilevel(n, u, v, w, X0s, levels, sweeps, frac, omega=0.5, embed="sparsifier"):
    """Alg. 1: coarsen G_0..G_lf, P_lf = G_lf, then map back level by level,
    each time adding the top f of the off-subgraph edges.

    ``X0s[l]`` is an (>= N_l)-by-K FP64 block; level l uses its first N_l rows.
    """
    lv = [Level(n, _i32(u), _i32(v), _f64(w))]
    for l in range(levels - 1):
        L = lv[-1]
        agg, nc, cu, cv, cw, rep, _ = coarsen_level(L.n, L.u, L.v, L.w, X0s[l][:L.n], sweeps, omega)
        L.agg, L.nc, L.rep = agg, nc, rep
        lv.append(Level(nc, cu, cv, cw))
    lf = levels - 1
    P = np.ones(lv[lf].u.shape[0], dtype=np.uint8)     # Alg. 1: P_lf = G_lf
    results = []
    keep = P
    X = None
    for l in range(lf, 0, -1):
        F, C = lv[l - 1], lv[l]
        intra = F.agg[F.u] == F.agg[F.v]
        inner, _ = max_spanning_forest(F.n, F.u, F.v, F.w, allowed=intra)
        base = inner.astype(bool)
        sel_coarse = np.nonzero(P)[0]
        base[F.rep[sel_coarse]] = True
        lr, X = score_level(F.n, F.u, F.v, F.w, base, X0s[l - 1][:F.n], sweeps, omega, frac, embed)
        keep = base.astype(np.uint8)
        keep[lr.chosen] = 2
        results.append(lr)
        P = keep
    return Result(keep, results, X), lv


# ----------------------------------------------------------------------------
# quality checks: relative condition number (Eq. 2) and eigenvalues
# ----------------------------------------------------------------------------

def laplacian_dense(n, u, v, w) -> np.ndarray:
    L = np.zeros((n, n))
    for a, b, c in zip(np.asarray(u), np.asarray(v), np.asarray(w)):
        L[a, b] -= c
        L[b, a] -= c
        L[a, a] += c
        L[b, b] += c
    return L


def laplacian_sparse(n, u, v, w):
    import scipy.sparse as sp
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    A = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(n, n)).tocsr()
    d = np.asarray(A.sum(axis=1)).reshape(-1)
    return (sp.diags(d) - A).tocsc()


def kappa_dense(n, u, v, w, mask) -> tuple[float, float, float]:
    """kappa(L_G, L_P) = lambda_max / lambda_min of the grounded pencil (Eq. 2)."""
    from scipy.linalg import eigh

    mask = np.asarray(mask, dtype=bool)
    LG = laplacian_dense(n, u, v, w)[1:, 1:]
    LP = laplacian_dense(n, np.asarray(u)[mask], np.asarray(v)[mask], np.asarray(w)[mask])[1:, 1:]
    ev = eigh(LG, LP, eigvals_only=True)
    return float(ev[-1] / ev[0]), float(ev[-1]), float(ev[0])


def kappa_sparse(n, u, v, w, mask, tol=1e-8) -> tuple[float, float, float]:
    """Same quantity by Lanczos on the grounded pencil with sparse LU solves of L_P and L_G."""
    import scipy.sparse.linalg as sla

    mask = np.asarray(mask, dtype=bool)
    LG = laplacian_sparse(n, u, v, w)[1:, 1:].tocsc()
    LP = laplacian_sparse(n, np.asarray(u)[mask], np.asarray(v)[mask], np.asarray(w)[mask])[1:, 1:].tocsc()
    luP = sla.splu(LP)
    N = n - 1
    opA = sla.LinearOperator((N, N), matvec=lambda x: luP.solve(LG @ x), dtype=np.float64)
    lmax = float(np.real(sla.eigs(opA, k=1, which="LR", tol=tol, return_eigenvectors=False)[0]))
    luG = sla.splu(LG)
    opB = sla.LinearOperator((N, N), matvec=lambda x: luG.solve(LP @ x), dtype=np.float64)
    inv_lmin = float(np.real(sla.eigs(opB, k=1, which="LR", tol=tol, return_eigenvectors=False)[0]))
    lmin = 1.0 / inv_lmin
    return lmax / lmin, lmax, lmin


def pcg_iterations(n, u, v, w, mask=None, tol=1e-3, maxiter=20000, seed=0) -> int:
    """Iterations of preconditioned CG on the grounded system L_G x = b (node 0
    grounded, b standard normal from ``seed``) until ||r|| <= tol ||b||, with the
    grounded sparsifier Laplacian L_P (the edges of ``mask``) solved exactly by a
    sparse LU as the preconditioner (mask None: plain CG).  The sparsifier's
    downstream use in the paper's evaluation (Sec. 4, Table 3)."""
    import scipy.sparse.linalg as sla

    LG = laplacian_sparse(n, u, v, w)[1:, 1:].tocsr()
    if mask is None:
        def solve(r):
            return r.copy()
    else:
        mask = np.asarray(mask, dtype=bool)
        LP = laplacian_sparse(n, np.asarray(u)[mask], np.asarray(v)[mask], np.asarray(w)[mask])[1:, 1:].tocsc()
        solve = sla.splu(LP).solve
    b = np.random.default_rng(seed).standard_normal(n - 1)
    nb = float(np.linalg.norm(b))
    x = np.zeros(n - 1)
    r = b.copy()
    z = solve(r)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, maxiter + 1):
        Ap = LG @ p
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        if float(np.linalg.norm(r)) <= tol * nb:
            return it
        z = solve(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return maxiter


# ----------------------------------------------------------------------------
# sigma-driven stopping: spanning-tree solves and the condition-number estimate
# ----------------------------------------------------------------------------

@dataclass
class Tree:
    """A spanning tree rooted at node 0, laid out in depth-first preorder."""
    n: int
    order: np.ndarray    # int32[n]: node at each preorder position (order[0] = 0)
    parent: np.ndarray   # int32[n]: preorder position of the parent (-1 at the root)
    size: np.ndarray     # int32[n]: nodes in the subtree
    pw: np.ndarray       # float64[n]: weight of the edge to the parent (0 at the root)
    tdown: np.ndarray    # int32[n]: walk step that enters the node (-1 at the root)
    tup: np.ndarray      # int32[n]: walk step that leaves it (-1 at the root)


def tree_dfs(n: int, u, v, w, tree_mask) -> Tree:
    """Depth-first walk of the spanning tree given by ``tree_mask`` from node 0.
    A node's children are taken in ascending id order starting after its
    parent and wrapping round (the root starts at its smallest neighbour).
    Every traversal of a tree edge, down or up, is one walk step."""
    u, v, w = _i32(u), _i32(v), _f64(w)
    mk = np.asarray(tree_mask, dtype=bool)
    tu, tv, tw = u[mk], v[mk], w[mk]
    if tu.shape[0] != n - 1:
        raise ValueError("tree must have n - 1 edges")
    adj = [[] for _ in range(n)]
    for a, b, c in zip(tu.tolist(), tv.tolist(), tw.tolist()):
        adj[a].append((b, c))
        adj[b].append((a, c))
    for lst in adj:
        lst.sort()
    order, parent, size, pw, tdown, tup = [], [], [], [], [], []
    pre = np.full(n, -1, dtype=np.int64)
    step = 0

    def visit(q, par_pre, weight, enter_step):
        pre[q] = len(order)
        order.append(q)
        parent.append(par_pre)
        size.append(1)
        pw.append(weight)
        tdown.append(enter_step)
        tup.append(-1)

    visit(0, -1, 0.0, -1)
    # stack entries: [node, neighbours in visiting order, next index]
    stack = [[0, [b for b, _ in adj[0]], 0]]
    wt = [dict(lst) for lst in adj]
    while stack:
        top = stack[-1]
        q, nbrs, i = top
        if i < len(nbrs):
            top[2] += 1
            c = nbrs[i]
            if pre[c] >= 0:
                raise ValueError("tree edges contain a cycle")
            visit(c, int(pre[q]), wt[q][c], step)
            step += 1
            ids = [b for b, _ in adj[c]]
            j = ids.index(q)
            stack.append([c, ids[j + 1:] + ids[:j], 0])
        else:
            stack.pop()
            if stack:
                tup[pre[q]] = step
                step += 1
                size[int(pre[stack[-1][0]])] += size[pre[q]]
    if len(order) != n:
        raise ValueError("tree edges do not span the graph")
    return Tree(n, np.array(order, np.int32), np.array(parent, np.int32), np.array(size, np.int32),
                np.array(pw, np.float64), np.array(tdown, np.int32), np.array(tup, np.int32))


def tree_solve(tree: Tree, B) -> np.ndarray:
    """x = L_T^+ b for every column: the tree Laplacian system with b projected
    onto the complement of the all-one vector, solved by eliminating leaves
    upward (each edge carries the net demand of the subtree below it) and
    back-substituting potentials downward; the result has zero mean."""
    B = _f64(B)
    one = B.ndim == 1
    B2 = B.reshape(B.shape[0], -1)
    F = B2[tree.order] - B2.mean(axis=0)
    for i in range(tree.n - 1, 0, -1):
        F[tree.parent[i]] += F[i]
    Xp = np.zeros_like(F)
    for i in range(1, tree.n):
        Xp[i] = Xp[tree.parent[i]] + F[i] / tree.pw[i]
    X = np.empty_like(Xp)
    X[tree.order] = Xp
    X -= X.mean(axis=0)
    return X.reshape(-1) if one else X


def kappa_estimate(n, u, v, w, mask, Y0, steps: int) -> list:
    """Lower estimate of lambda_max of the pencil (L_G, L_P), P the edges of
    ``mask`` (a connected spanning subgraph of G with G's weights), by subspace
    iteration Y <- L_P^+ L_G Y with Rayleigh-Ritz after every step.  Because
    L_P <= L_G, lambda_min >= 1 and the relative condition number of Eq. 2 is
    at most lambda_max; any Ritz value is at most lambda_max (Courant-Fischer).
    L_P systems are solved exactly (sparse LU, node 0 grounded).  Returns the
    largest Ritz value after each step."""
    import scipy.linalg as dla
    import scipy.sparse.linalg as sla

    mask = np.asarray(mask, dtype=bool)
    u, v, w = _i32(u), _i32(v), _f64(w)
    LG = laplacian_sparse(n, u, v, w).tocsr()
    LP = laplacian_sparse(n, u[mask], v[mask], w[mask]).tocsr()
    lu = sla.splu(LP[1:, 1:].tocsc())

    def solve(Z):
        X = np.zeros_like(Z)
        X[1:] = lu.solve(Z[1:])
        return X - X.mean(axis=0)

    Y = _f64(Y0).copy()
    Y -= Y.mean(axis=0)
    out = []
    for _ in range(steps):
        Yn = solve(LG @ Y)
        A = Yn.T @ (LG @ Yn)
        Bm = Yn.T @ (LP @ Yn)
        A = 0.5 * (A + A.T)
        Bm = 0.5 * (Bm + Bm.T)
        theta, V = dla.eigh(A, Bm)
        out.append(float(theta[-1]))
        Y = Yn @ V
    return out


def sparsify_sigma(n, u, v, w, X0s, Y0s, sigma, frac, max_rounds, sweeps, est_steps, omega=0.5,
                   embed="sparsifier", smoother="jacobi"):
    """Sigma-driven stopping (Alg. 1 takes sigma but never uses it): start
    from the maximum-weight spanning tree and, while the condition-number
    estimate exceeds sigma^2 (Eq. 2) and rounds remain, add the next
    ceil(frac * off-tree edges) top-scored edges, each batch scored on the
    sparsifier grown so far.  X0s[r] is round r's smoothing block, Y0s[j]
    the starting block of the j-th estimate.  Returns (Result, estimates)."""
    intree, comps = max_spanning_forest(n, u, v, w)
    if comps != 1:
        raise ValueError("graph is not connected")
    base = intree.astype(bool)
    keep = intree.astype(np.uint8)
    q = ksel(frac, int((~base).sum()))
    kappas = [kappa_estimate(n, u, v, w, base, Y0s[0], est_steps)[-1]]
    results, X = [], None
    r = 0
    while kappas[-1] > sigma * sigma and r < max_rounds:
        take = min(q, int((~base).sum()))
        if take == 0:
            break
        lr, X = score_level(n, u, v, w, base, X0s[r], sweeps, omega, frac, embed, k_take=take, smoother=smoother)
        keep[lr.chosen] = 2
        base[lr.chosen] = True
        results.append(lr)
        r += 1
        kappas.append(kappa_estimate(n, u, v, w, base, Y0s[r], est_steps)[-1])
    return Result(keep, results, X), kappas


# ----------------------------------------------------------------------------
# precision form: reference for the reduced-precision selection
# ----------------------------------------------------------------------------

def score_errors(s, s_ref, tau) -> dict:
    """Error measures of reduced-precision scores against FP64 ones."""
    s = np.asarray(s, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    d = np.abs(s - s_ref)
    pos = s_ref > 0
    rel_all = float(np.max(d[pos] / s_ref[pos])) if np.any(pos) else 0.0
    top = s_ref >= tau
    rel_top = float(np.max(d[top] / s_ref[top])) if np.any(top) else 0.0
    return {"max_rel_all": rel_all, "max_rel_selected_region": rel_top,
            "max_abs_over_tau": float(np.max(d) / tau) if tau > 0 else float("inf")}
