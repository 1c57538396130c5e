"""Pin of the oracle's Alg. 1 composition (``oracle.sparsify_multilevel``)
against a dense brute force written independently of it.

The brute force restates the hierarchy from the paper with dense matrices and
plain loops, sharing no routine with the oracle:
  * coarsening (Sec. 3.2-3.3): dense damped-Jacobi smoothing of the centred
    random block on G_l, affinities (x_p . x_q)^2 / (|x_p|^2 |x_q|^2) of the
    re-centred block, every node pointing to its neighbour with the largest
    (affinity, weight, -id), aggregates = connected parts of the pointer graph
    (label propagation), numbered by their smallest member; the Galerkin
    graph as the dense product H^T W H of the aggregate indicator H (Eq. 3 with
    the H+ of Eq. 5), and per coarse edge the heaviest fine edge between the
    two aggregates;
  * Alg. 1 downwards: P_lf = G_lf; at level l-1 the union of a maximum
    spanning forest of every aggregate (SciPy's minimum spanning tree of the
    negated weights, restricted to intra-aggregate edges) and, for each edge of
    the coarse sparsifier P_l, its representative fine edge; then the
    sparsifier embedding (dense smoothing on the Laplacian of that union), the
    scores w |x_p - x_q|^2 of the edges outside it and the top ceil(f * n_cand)
    by (score desc, id asc).

Weights are drawn from a continuous distribution so every spanning tree and
every ranking is unique; scores are compared to a summation-order tolerance,
everything integer (aggregates, coarse edges, representatives, sparsifier
masks, selected sets) exactly.  The edge count of each mapped sparsifier is
also checked against (N_{l-1} - N_l) + |E(P_l)|: inner forests contribute one
edge fewer than their aggregate's size, and each coarse sparsifier edge maps to
one fine edge.
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

import workloads as W


# --------------------------------------------------------------------------- dense brute force

def _dense_w(n, u, v, w):
    A = np.zeros((n, n))
    A[u, v] = w
    A[v, u] = w
    return A


def _centre(X):
    X = np.array(X, dtype=np.float64)
    for c in range(X.shape[1]):
        X[:, c] -= math.fsum(X[:, c]) / X.shape[0]
    return X


def _jacobi(A, X, sweeps, omega):
    d = A.sum(axis=1)
    for _ in range(sweeps):
        X = (1.0 - omega) * X + omega * (A @ X) / d[:, None]
    return X


def _pointer_aggregates(n, u, v, w, a):
    best = [None] * n
    for e in range(len(u)):
        for p, q in ((int(u[e]), int(v[e])), (int(v[e]), int(u[e]))):
            key = (a[e], w[e], -q)
            if best[p] is None or key > best[p][0]:
                best[p] = (key, q)
    ptr = np.array([b[1] for b in best])
    lab = np.arange(n)
    changed = True
    while changed:                       # label propagation over the undirected pointer edges
        changed = False
        for p in range(n):
            lo = min(lab[p], lab[ptr[p]])
            if lab[p] != lo or lab[ptr[p]] != lo:
                lab[p] = lab[ptr[p]] = lo
                changed = True
    roots = sorted(set(lab.tolist()))     # each root is its part's smallest member
    return np.array([roots.index(x) for x in lab]), len(roots)


def _coarsen(n, u, v, w, X0, sweeps, omega):
    A = _dense_w(n, u, v, w)
    X = _jacobi(A, _centre(X0), sweeps, omega)
    Xb = _centre(X)
    a = np.zeros(len(u))
    for e in range(len(u)):
        xp, xq = Xb[u[e]], Xb[v[e]]
        den = (xp @ xp) * (xq @ xq)
        a[e] = (xp @ xq) ** 2 / den if den > 0 else 0.0
    agg, nc = _pointer_aggregates(n, u, v, w, a)
    H = np.zeros((n, nc))
    H[np.arange(n), agg] = 1.0
    Ac = H.T @ A @ H
    cu, cv = [], []
    for I in range(nc):
        for J in range(I + 1, nc):
            if Ac[I, J] > 0:
                cu.append(I)
                cv.append(J)
    cu, cv = np.array(cu, dtype=np.int32), np.array(cv, dtype=np.int32)
    cw = Ac[cu, cv]
    rep = np.zeros(len(cu), dtype=np.int64)
    for c in range(len(cu)):
        pair = {int(cu[c]), int(cv[c])}
        between = [e for e in range(len(u)) if {int(agg[u[e]]), int(agg[v[e]])} == pair]
        rep[c] = max(between, key=lambda e: (w[e], -e))
    return agg, nc, cu, cv, cw, rep


def _inner_forest(n, u, v, w, agg):
    intra = np.nonzero(agg[u] == agg[v])[0]
    M = coo_matrix((-w[intra], (u[intra], v[intra])), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(M).tocoo()
    pairs = {(min(a, b), max(a, b)) for a, b in zip(T.row.tolist(), T.col.tolist())}
    return np.array([(int(u[e]), int(v[e])) in pairs for e in range(len(u))])


def brute_multilevel(n, u, v, w, X0s, levels, sweeps, frac, omega=0.5):
    """Per level (finest first): dict of agg, coarse graph, representatives,
    mapped sparsifier, candidates, scores, chosen; and the final keep mask."""
    lv = [{"n": n, "u": np.asarray(u), "v": np.asarray(v), "w": np.asarray(w, dtype=np.float64)}]
    for l in range(levels - 1):
        L = lv[-1]
        agg, nc, cu, cv, cw, rep = _coarsen(L["n"], L["u"], L["v"], L["w"], X0s[l][:L["n"]], sweeps, omega)
        L.update(agg=agg, nc=nc, rep=rep)
        lv.append({"n": nc, "u": cu, "v": cv, "w": cw})
    P = np.ones(len(lv[-1]["u"]), dtype=bool)           # P_lf = G_lf
    for l in range(levels - 1, 0, -1):
        F = lv[l - 1]
        base = _inner_forest(F["n"], F["u"], F["v"], F["w"], F["agg"])
        assert base.sum() == F["n"] - lv[l]["n"]
        base[F["rep"][P]] = True
        assert base.sum() == (F["n"] - lv[l]["n"]) + P.sum()
        Ap = _dense_w(F["n"], F["u"][base], F["v"][base], F["w"][base])
        X = _jacobi(Ap, _centre(X0s[l - 1][:F["n"]]), sweeps, omega)
        cand = np.nonzero(~base)[0]
        s = F["w"][cand] * ((X[F["u"][cand]] - X[F["v"][cand]]) ** 2).sum(axis=1)
        k = math.ceil(frac * len(cand))
        order = sorted(range(len(cand)), key=lambda i: (-s[i], cand[i]))
        chosen = cand[order[:k]]
        F.update(base=base.copy(), cand=cand, score=s, chosen=np.sort(chosen))
        P = base.copy()
        P[chosen] = True
    keep = lv[0]["base"].astype(np.uint8)
    keep[lv[0]["chosen"]] = 2
    return lv, keep


# --------------------------------------------------------------------------- the pin

CASES = {
    "grid8x8_3lv": (lambda: W.grid2d(8, 8, seed=301, wdist=("lognormal", 0.0, 1.0)), 3, 0.1),
    "rand70_3lv": (lambda: W.random_connected(70, 170, seed=302, wdist=("lognormal", 0.0, 1.0)), 3, 0.2),
    "pgrid9_3lv": (lambda: W.powergrid(9, 9, 0.05, seed=303), 3, 0.15),
    "rand48_2lv": (lambda: W.random_connected(48, 110, seed=304, wdist=("lognormal", 0.0, 1.0)), 2, 0.1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_multilevel_matches_dense_brute_force(orc, case):
    make, levels, frac = CASES[case]
    g = make()
    k, T = 6, 8
    X0s = [W.random_block(g.n, k, 700 + l) for l in range(levels)]
    ref, keep_ref = brute_multilevel(g.n, g.u, g.v, g.w, X0s, levels, T, frac)
    r, lv = orc.sparsify_multilevel(g.n, g.u, g.v, g.w, X0s, levels, T, frac)
    # the hierarchy reaches at least one mapped level with candidates left unselected, so the mapping
    # of the coarse sparsifier (not the whole coarse graph) is exercised
    assert len(lv) == levels and lv[-1].n >= 2
    for l in range(levels - 1):
        assert np.array_equal(lv[l].agg, ref[l]["agg"]), (case, l)
        assert lv[l].nc == ref[l]["nc"]
        C = lv[l + 1]
        assert np.array_equal(C.u, ref[l + 1]["u"]) and np.array_equal(C.v, ref[l + 1]["v"]), (case, l)
        assert np.allclose(C.w, ref[l + 1]["w"], rtol=1e-13, atol=0)
        assert np.array_equal(lv[l].rep, ref[l]["rep"]), (case, l)
    # r.levels holds the scored levels from coarse to fine: level lf-1 first, level 0 last
    assert len(r.levels) == levels - 1
    for i, lr in enumerate(r.levels):
        R = ref[levels - 2 - i]
        assert np.array_equal(lr.cand, R["cand"]), (case, i)
        assert lr.k_sel == len(R["chosen"])
        np.testing.assert_allclose(lr.score, R["score"], rtol=1e-10, atol=1e-300)
        assert np.array_equal(np.sort(lr.chosen), R["chosen"]), (case, i)
    assert np.array_equal(r.keep, keep_ref), case
    # at least one coarse sparsifier is a strict subgraph of its level's graph (the mapping of P_l, not
    # G_l, matters) and holds recovered edges (the mapping keeps them, not only the tree)
    strict = [R for R in ref[1:levels - 1] if len(R["cand"]) > len(R["chosen"]) > 0]
    assert strict or levels == 2


def test_brute_force_mapping_counts_on_a_grid(orc):
    """The brute force's own invariant at every level: |P_{l-1} before additions| =
    (N_{l-1} - N_l) + |E(P_l)|, and each P_{l-1} is connected and spans G_{l-1}."""
    g = W.grid2d(9, 9, seed=305, wdist=("lognormal", 0.0, 1.0))
    X0s = [W.random_block(g.n, 6, 710 + l) for l in range(3)]
    ref, keep = brute_multilevel(g.n, g.u, g.v, g.w, X0s, 3, 8, 0.1)
    for l in range(2):
        L = ref[l]
        m = coo_matrix((np.ones(int(L["base"].sum())), (L["u"][L["base"]], L["v"][L["base"]])),
                       shape=(L["n"], L["n"]))
        assert connected_components(m, directed=False)[0] == 1
    c, _ = orc.components(g.n, g.u, g.v, keep > 0)
    assert c == 1
