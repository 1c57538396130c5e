"""Pins of the CPU FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a library
routine (SciPy/NumPy), a closed form, an invariant, or brute force on tiny
inputs.  None of these tests touches the GPU library.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, laplacian as csgraph_laplacian
from scipy.sparse.csgraph import minimum_spanning_tree

import workloads as W


def dense_from_csr(csr):
    n = csr.n
    A = np.zeros((n, n))
    for p in range(n):
        for j in range(csr.rowptr[p], csr.rowptr[p + 1]):
            A[p, csr.col[j]] += csr.val[j]
    return np.diag(csr.deg) - A


def adjacency(n, u, v, w):
    return sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                         shape=(n, n)).toarray()


TINY = [
    W.grid2d(4, 4, seed=11),
    W.grid2d(5, 7, seed=12, wdist=("lognormal", 0.0, 1.0)),
    W.random_connected(30, 40, seed=13),
    W.random_connected(64, 150, seed=14, wdist=("lognormal", 0.0, 1.5)),
]


# --------------------------------------------------------------------------- Laplacian (Sec. 2.1)

@pytest.mark.parametrize("g", TINY, ids=lambda g: g.name)
def test_laplacian_matches_scipy(orc, g):
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    L = dense_from_csr(csr)
    Lref = csgraph_laplacian(adjacency(g.n, g.u, g.v, g.w))
    assert np.allclose(L, Lref, rtol=0, atol=1e-14)
    # ascending columns, entry -> edge id consistent with the edge list
    for p in range(g.n):
        cols = csr.col[csr.rowptr[p]:csr.rowptr[p + 1]]
        assert np.all(np.diff(cols) > 0)
    e = csr.eid
    rows = np.repeat(np.arange(g.n), np.diff(csr.rowptr))
    assert np.all(csr.val == g.w[e])
    assert np.all(np.minimum(rows, csr.col) == g.u[e])
    assert np.all(np.maximum(rows, csr.col) == g.v[e])


def test_laplacian_integer_row_sums_exact(orc):
    g = W.random_connected(200, 500, seed=3)
    w = np.floor(g.w * 8.0) + 1.0             # small integers: sums are exact
    csr = orc.laplacian_csr(g.n, g.u, g.v, w)
    rowsum = np.zeros(g.n)
    for p in range(g.n):
        rowsum[p] = csr.deg[p] - sum(csr.val[csr.rowptr[p]:csr.rowptr[p + 1]])
    assert np.all(rowsum == 0.0)


def test_quadratic_form_identity(orc):
    # x^T L x = sum_E w (x_p - x_q)^2 (Sec. 2.1)
    g = TINY[3]
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    L = dense_from_csr(csr)
    x = np.random.default_rng(0).standard_normal(g.n)
    lhs = x @ L @ x
    rhs = math.fsum(g.w * (x[g.u] - x[g.v]) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


# --------------------------------------------------------------------------- exact sum / centring

def test_exact_sum_matches_fsum(orc):
    rng = np.random.default_rng(1)
    cases = [rng.standard_normal(10000),
             np.array([1e16, 1.0, -1e16, 1e-16, 3.0]),
             np.array([1e-16, 1.0, 1e16]),
             rng.standard_normal(1000) * 10.0 ** rng.integers(-20, 20, 1000)]
    for x in cases:
        assert orc.exact_sum(x) == math.fsum(x)


def test_center_orthogonal_to_ones(orc):
    X0 = W.random_block(1000, 8, 5)
    X, mean = orc.center(X0)
    for c in range(8):
        assert mean[c] == math.fsum(X0[:, c]) / 1000.0
        assert abs(math.fsum(X[:, c])) < 1e-12


# --------------------------------------------------------------------------- smoothing (Sec. 3.2)

def _closed_form_smooth(L, deg, X0, T, omega):
    """X_T = D^-1/2 V (I - omega Lambda)^T V^T D^1/2 X0 with V Lambda V^T = D^-1/2 L D^-1/2."""
    dh = np.sqrt(deg)
    Nrm = L / dh[:, None] / dh[None, :]
    lam, V = np.linalg.eigh(Nrm)
    f = (1.0 - omega * lam) ** T
    return (V * f) @ (V.T @ (dh[:, None] * X0)) / dh[:, None]


@pytest.mark.parametrize("g", TINY, ids=lambda g: g.name)
@pytest.mark.parametrize("omega", [0.5, 0.3])
def test_smoothing_closed_form(orc, g, omega):
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    L = dense_from_csr(csr)
    X0, _ = orc.center(W.random_block(g.n, 4, 7))
    T = 12
    X = orc.smooth(csr, X0, T, omega)
    Xref = _closed_form_smooth(L, csr.deg, X0, T, omega)
    assert np.max(np.abs(X - Xref)) <= 1e-12 * np.max(np.abs(X0))


def test_fp64_summation_order_noise_floor(orc):
    # not a pin: the oracle adds each row in ascending column order; the same sweeps with every row added in
    # the reverse order differ only by rounding, about 1e-16 of the values, far below the 1e-12 tolerance
    g = W.grid2d(20, 20, seed=12, wdist=("lognormal", 0.0, 1.0))
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    X0, _ = orc.center(W.random_block(g.n, 3, 13))
    T, omega = 10, 0.5
    ref = orc.smooth(csr, X0, T, omega)
    X = X0.copy()
    for _ in range(T):
        Y = np.empty_like(X)
        for p in range(g.n):
            acc = np.zeros(X.shape[1])
            for j in range(csr.rowptr[p + 1] - 1, csr.rowptr[p] - 1, -1):
                acc = acc + csr.val[j] * X[csr.col[j]]
            Y[p] = (1 - omega) * X[p] + omega * (acc / csr.deg[p])
        X = Y
    rel = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    assert 0 <= rel < 1e-14, rel


def test_smoothing_invariants(orc):
    g = W.grid2d(12, 9, seed=4, wdist=("lognormal", 0.0, 1.0))
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    L = dense_from_csr(csr)
    X, _ = orc.center(W.random_block(g.n, 3, 8))
    m0 = csr.deg @ X
    energy = np.trace(X.T @ L @ X)
    for _ in range(15):
        X = orc.smooth(csr, X, 1, 0.5)
        # 1^T D X is conserved by I - omega D^-1 L
        assert np.allclose(csr.deg @ X, m0, rtol=0, atol=1e-12)
        e2 = np.trace(X.T @ L @ X)
        assert e2 <= energy * (1 + 1e-13)        # Dirichlet energy never increases for omega <= 1
        energy = e2


def test_smoothing_complete_graph(orc):
    # unit-weight K_n: a centred x maps to x * (1 - omega n / (n - 1))
    n = 9
    a, b = np.triu_indices(n, 1)
    csr = orc.laplacian_csr(n, a, b, np.ones(a.shape[0]))
    X, _ = orc.center(W.random_block(n, 2, 9))
    for omega in (0.5, 0.25):
        Y = orc.smooth(csr, X, 1, omega)
        assert np.allclose(Y, X * (1 - omega * n / (n - 1)), rtol=0, atol=1e-14)


def test_smoothing_masked_cone(orc):
    from scipy.sparse.csgraph import shortest_path

    g = W.grid2d(15, 15, seed=6)
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    X0, _ = orc.center(W.random_block(g.n, 4, 10))
    T = 6
    full = orc.smooth(csr, X0, T, 0.5)
    seeds = [0, 37, 112]
    D = shortest_path(sp.csr_matrix(adjacency(g.n, g.u, g.v, np.ones(g.m))), unweighted=True,
                      indices=seeds)
    dist = np.minimum(D.min(axis=0), 1 << 20).astype(np.int32)
    part = orc.smooth_masked(csr, X0, T, 0.5, dist)
    assert np.array_equal(part[seeds], full[seeds])


# --------------------------------------------------------------------------- scores (Eq. 16-19)

@pytest.mark.parametrize("g", TINY[1:], ids=lambda g: g.name)
def test_scores_full_embedding_equal_leverage(orc, g):
    # with U_eff = [u_i / sqrt(lambda_i)] over all nontrivial pairs the score is w * R_eff (Eq. 19)
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    L = dense_from_csr(csr)
    lam, V = np.linalg.eigh(L)
    U = V[:, 1:] / np.sqrt(lam[1:])
    s = orc.edge_scores(U, g.u, g.v, g.w)
    Lp = np.linalg.pinv(L)
    reff = Lp[g.u, g.u] + Lp[g.v, g.v] - 2 * Lp[g.u, g.v]
    assert np.allclose(s, g.w * reff, rtol=1e-10, atol=0)
    # leverage scores of a connected graph sum to n - 1
    assert abs(s.sum() - (g.n - 1)) < 1e-9 * g.n


def test_scores_on_tree_are_path_stretch(orc):
    g = W.random_connected(40, 60, seed=21)
    intree, comps = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    assert comps == 1
    t = intree.astype(bool)
    L = dense_from_csr(orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t]))
    lam, V = np.linalg.eigh(L)
    U = V[:, 1:] / np.sqrt(lam[1:])
    s = orc.edge_scores(U, g.u, g.v, g.w)
    # brute force: walk the unique tree path and add 1/w of its edges
    adj = {p: [] for p in range(g.n)}
    for e in np.nonzero(t)[0]:
        adj[int(g.u[e])].append((int(g.v[e]), g.w[e]))
        adj[int(g.v[e])].append((int(g.u[e]), g.w[e]))

    def path_resistance(a, b):
        stack = [(a, -1, 0.0)]
        while stack:
            x, par, r = stack.pop()
            if x == b:
                return r
            for y, wy in adj[x]:
                if y != par:
                    stack.append((y, x, r + 1.0 / wy))
        raise AssertionError

    stretch = np.array([g.w[e] * path_resistance(int(g.u[e]), int(g.v[e])) for e in range(g.m)])
    assert np.allclose(s, stretch, rtol=1e-9, atol=0)


def test_first_order_perturbation(orc):
    # Eq. 16: adding an edge of tiny weight eps moves lambda_i by eps (u_i^T e_pq)^2 + O(eps^2)
    g = W.random_connected(12, 8, seed=2)
    L = dense_from_csr(orc.laplacian_csr(g.n, g.u, g.v, g.w))
    lam, V = np.linalg.eigh(L)
    p, q = 0, 7
    e = np.zeros(g.n); e[p], e[q] = 1, -1
    for eps in (1e-3, 1e-4):
        lam2 = np.linalg.eigvalsh(L + eps * np.outer(e, e))
        pred = eps * (V.T @ e) ** 2
        err = np.max(np.abs((lam2 - lam) - pred)[1:])
        assert err < 50 * eps * eps


# --------------------------------------------------------------------------- selection (Alg. 1)

def test_select_matches_sort(orc):
    rng = np.random.default_rng(3)
    s = np.round(rng.random(5000) * 50) / 7.0    # many ties
    eid = np.sort(rng.choice(100000, 5000, replace=False)).astype(np.int32)
    for k in (0, 1, 17, 999, 5000):
        pos, tau = orc.select_topk(s, eid, k)
        order = np.lexsort((eid, -s))
        assert np.array_equal(pos, order[:k])
        if k:
            assert tau == s[order[k - 1]]


def test_ksel_examples(orc):
    assert orc.ksel(0.05, 3969) == 199
    assert orc.ksel(0.10, 1037961) == 103797


# --------------------------------------------------------------------------- spanning tree (Sec. 3.4)

@pytest.mark.parametrize("g", TINY + [W.grid2d(30, 30, seed=5)], ids=lambda g: g.name)
def test_max_spanning_tree_matches_scipy(orc, g):
    intree, comps = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    assert comps == 1 and intree.sum() == g.n - 1
    ref = minimum_spanning_tree(sp.csr_matrix((-g.w, (g.u, g.v)), shape=(g.n, g.n))).tocoo()
    ref_set = set(zip(np.minimum(ref.row, ref.col), np.maximum(ref.row, ref.col)))
    got = set(zip(g.u[intree == 1], g.v[intree == 1]))
    assert got == ref_set


def test_max_spanning_tree_ties_take_smaller_id(orc):
    # unit-weight 4-cycle: Kruskal over ascending id keeps edges 0, 1, 2
    u = np.array([0, 0, 1, 2]); v = np.array([1, 3, 2, 3])
    intree, _ = orc.max_spanning_forest(4, u, v, np.ones(4))
    assert list(intree) == [1, 1, 1, 0]


def test_components_match_scipy(orc):
    g = W.random_connected(300, 100, seed=8)
    mask = (np.arange(g.m) % 3) != 0
    c, lab = orc.components(g.n, g.u, g.v, mask)
    A = sp.coo_matrix((np.ones(int(mask.sum())), (g.u[mask], g.v[mask])), shape=(g.n, g.n))
    c2, lab2 = connected_components(A, directed=False)
    assert c == c2
    # same partition
    assert len(set(zip(lab, lab2))) == c


# --------------------------------------------------------------------------- affinity (Sec. 3.2)

def test_affinity_is_squared_cosine(orc):
    from scipy.spatial.distance import cosine

    g = TINY[2]
    Xb = W.random_block(g.n, 6, 12)
    a = orc.affinity(Xb, g.u, g.v)
    ref = np.array([(1.0 - cosine(Xb[p], Xb[q])) ** 2 for p, q in zip(g.u, g.v)])
    assert np.allclose(a, ref, rtol=1e-12, atol=1e-15)
    # special values: parallel rows -> 1, orthogonal rows -> 0, a zero row -> 0
    Y = np.array([[1.0, 2.0], [-2.0, -4.0], [2.0, -1.0], [0.0, 0.0]])
    a2 = orc.affinity(Y, [0, 0, 0], [1, 2, 3])
    assert a2[0] == 1.0 and a2[1] == 0.0 and a2[2] == 0.0


# --------------------------------------------------------------------------- coarsening (Eq. 3-7)

def _coarsen_dense(orc, g, seed=3, T=8):
    agg, nc, cu, cv, cw, rep, a_edge = orc.coarsen_level(g.n, g.u, g.v, g.w,
                                                         W.random_block(g.n, 4, seed), T)
    Hp = np.zeros((g.n, nc))
    Hp[np.arange(g.n), agg] = 1.0                      # H+ of Eq. 5
    H = (Hp / Hp.sum(axis=0)).T                        # H of Eq. 4
    return agg, nc, cu, cv, cw, rep, Hp, H


@pytest.mark.parametrize("g", [W.grid2d(8, 8, seed=31), W.random_connected(60, 120, seed=32)],
                         ids=lambda g: g.name)
def test_galerkin_is_eq3(orc, g):
    agg, nc, cu, cv, cw, rep, Hp, H = _coarsen_dense(orc, g)
    assert 1 < nc <= g.n // 2                          # every aggregate has >= 2 nodes
    assert np.allclose(H @ Hp, np.eye(nc))             # H H+ = I
    L = dense_from_csr(orc.laplacian_csr(g.n, g.u, g.v, g.w))
    Lc_ref = Hp.T @ L @ Hp                             # Eq. 3 with H^{-T} = H+^T
    Lc = dense_from_csr(orc.laplacian_csr(nc, cu, cv, cw))
    assert np.allclose(Lc, Lc_ref, rtol=0, atol=1e-12)
    # every aggregate is connected inside G
    for I in range(nc):
        S = np.nonzero(agg == I)[0]
        inside = np.isin(g.u, S) & np.isin(g.v, S)
        c, _ = connected_components(sp.coo_matrix((np.ones(int(inside.sum())), (g.u[inside], g.v[inside])),
                                                  shape=(g.n, g.n)).tocsr()[S][:, S], directed=False)
        assert c == 1
    # representative fine edge: heaviest between the two aggregates, ties smallest id
    for e_c in range(cu.shape[0]):
        between = ((agg[g.u] == cu[e_c]) & (agg[g.v] == cv[e_c])) | ((agg[g.u] == cv[e_c]) & (agg[g.v] == cu[e_c]))
        ids = np.nonzero(between)[0]
        best = ids[np.lexsort((ids, -g.w[ids]))[0]]
        assert rep[e_c] == best
    # aggregates numbered by ascending smallest member
    firsts = [np.min(np.nonzero(agg == I)[0]) for I in range(nc)]
    assert firsts == sorted(firsts)


def test_coarse_eigenvalue_bounds(orc):
    # min|S| lambda_i(L) <= lambda_i(L_c) <= max|S| lambda_{i+N-Nc}(L)  (Eq. 7 lower bound, interlacing)
    g = W.grid2d(9, 8, seed=33, wdist=("lognormal", 0.0, 1.0))
    agg, nc, cu, cv, cw, rep, Hp, H = _coarsen_dense(orc, g)
    L = dense_from_csr(orc.laplacian_csr(g.n, g.u, g.v, g.w))
    Lc = dense_from_csr(orc.laplacian_csr(nc, cu, cv, cw))
    lam = np.linalg.eigvalsh(L)
    lamc = np.linalg.eigvalsh(Lc)
    sizes = np.bincount(agg)
    for i in range(nc):
        assert sizes.min() * lam[i] <= lamc[i] + 1e-10
        assert lamc[i] <= sizes.max() * lam[i + g.n - nc] + 1e-10


def test_aggregate_pointer_rule_brute_force(orc):
    g = W.random_connected(40, 50, seed=34)
    csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    a = np.round(np.random.default_rng(1).random(g.m) * 4) / 4     # ties in affinity
    agg, ptr, nc = orc.aggregate(csr, a[csr.eid])
    for p in range(g.n):
        best = None
        for e in range(g.m):
            if p not in (g.u[e], g.v[e]):
                continue
            q = int(g.v[e] if g.u[e] == p else g.u[e])
            key = (a[e], g.w[e], -q)
            if best is None or key > best[0]:
                best = (key, q)
        assert ptr[p] == best[1]
    c, lab = connected_components(sp.coo_matrix((np.ones(g.n), (np.arange(g.n), ptr)), shape=(g.n, g.n)),
                                  directed=False)
    assert c == nc and len(set(zip(lab, agg))) == nc


def test_backward_mapping_of_a_tree_is_a_tree(orc):
    g = W.grid2d(20, 20, seed=35)
    agg, nc, cu, cv, cw, rep, _ = orc.coarsen_level(g.n, g.u, g.v, g.w, W.random_block(g.n, 4, 2), 8)
    ctree, comps = orc.max_spanning_forest(nc, cu, cv, cw)
    assert comps == 1
    intra = agg[g.u] == agg[g.v]
    inner, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w, allowed=intra)
    base = inner.astype(bool)
    base[rep[ctree == 1]] = True
    assert base.sum() == g.n - 1
    c, _ = orc.components(g.n, g.u, g.v, base)
    assert c == 1


# --------------------------------------------------------------------------- sparsifier and kappa (Eq. 2)

def test_kappa_dense_and_sparse_agree(orc):
    g = W.grid2d(12, 12, seed=40)
    r = orc.sparsify_single(g.n, g.u, g.v, g.w, W.random_block(g.n, 8, 41), 10, 0.1)
    mask = r.keep > 0
    kd, lmax, lmin = orc.kappa_dense(g.n, g.u, g.v, g.w, mask)
    ks, _, _ = orc.kappa_sparse(g.n, g.u, g.v, g.w, mask)
    assert abs(kd - ks) <= 1e-6 * kd
    assert lmin >= 1 - 1e-9                    # P is a subgraph of G, so L_G >= L_P


def test_kappa_monotone_and_tree_bounds(orc):
    g = W.grid2d(10, 10, seed=42, wdist=("lognormal", 0.0, 1.0))
    intree, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    t = intree.astype(bool)
    k_tree, lmax, _ = orc.kappa_dense(g.n, g.u, g.v, g.w, t)
    # exact stretch bounds: max_e w_e R_T(e) <= lambda_max(L_T^+ L_G) <= sum_e w_e R_T(e)
    LT = dense_from_csr(orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t]))
    Lp = np.linalg.pinv(LT)
    st = g.w * (Lp[g.u, g.u] + Lp[g.v, g.v] - 2 * Lp[g.u, g.v])
    assert st.max() <= lmax * (1 + 1e-9) and lmax <= st.sum() * (1 + 1e-9)
    # adding edges never increases kappa
    order = np.argsort(-st)
    mask = t.copy()
    prev = k_tree
    for e in order[:10]:
        if mask[e]:
            continue
        mask[e] = True
        k2, _, _ = orc.kappa_dense(g.n, g.u, g.v, g.w, mask)
        assert k2 <= prev * (1 + 1e-9)
        prev = k2


def test_sparsifier_structure(orc):
    g = W.workload_graph("grid64")
    r = orc.sparsify_single(g.n, g.u, g.v, g.w, W.workload_block("grid64", g.n), 10, 0.05)
    lr = r.levels[0]
    assert lr.n_cand == 3969 and lr.k_sel == 199
    assert (r.keep == 1).sum() == g.n - 1 and (r.keep == 2).sum() == 199
    c, _ = orc.components(g.n, g.u, g.v, r.keep > 0)
    assert c == 1
    # the recovered edges are exactly the top 199 scores among off-tree edges
    s = lr.score
    thr = np.sort(s)[::-1][198]
    assert np.all(s[np.isin(lr.cand, lr.chosen)] >= thr)


def test_multilevel_structure(orc):
    g = W.grid2d(40, 40, seed=43, wdist=("lognormal", 0.0, 1.0))
    X0s = [W.random_block(g.n, 8, 50 + l) for l in range(3)]
    r, lv = orc.sparsify_multilevel(g.n, g.u, g.v, g.w, X0s, 3, 10, 0.1)
    assert lv[0].n > lv[1].n > lv[2].n
    keep = r.keep
    c, _ = orc.components(g.n, g.u, g.v, keep > 0)
    assert c == 1
    lr = r.levels[-1]
    assert (keep == 2).sum() == lr.k_sel
    assert (keep > 0).sum() < g.m


# --------------------------------------------------------------------------- multi-round densification

def test_round_quotas(orc):
    for k_total in (0, 1, 7, 199, 103797):
        for rounds in (1, 2, 3, 5, 16):
            q = orc.round_quotas(k_total, rounds)
            assert len(q) == rounds and sum(q) == k_total
            assert max(q) - min(q) <= 1


def test_rounds_one_is_single_pass(orc):
    g = W.powergrid(30, 25, 0.02, seed=91)
    X0 = W.random_block(g.n, 8, 92)
    a = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, 6, 0.1)
    b = orc.sparsify_rounds(g.n, g.u, g.v, g.w, [X0], 1, 6, 0.1)
    assert np.array_equal(a.keep, b.keep)
    assert a.levels[0].tau == b.levels[0].tau


def _dense_rounds(n, u, v, w, X0s, rounds, sweeps, frac, omega):
    """Brute force with dense matrices: Kruskal by sorting, the sweep as a
    matrix product, scores from the dense block, top-k by a full sort."""
    order = sorted(range(len(w)), key=lambda e: (-w[e], e))
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    inP = np.zeros(len(w), bool)
    for e in order:
        a, b = find(u[e]), find(v[e])
        if a != b:
            parent[a] = b
            inP[e] = True
    k_total = math.ceil(frac * float((~inP).sum()))
    added = []
    for r in range(rounds):
        q = k_total * (r + 1) // rounds - k_total * r // rounds
        A = np.zeros((n, n))
        for e in np.nonzero(inP)[0]:
            A[u[e], v[e]] = A[v[e], u[e]] = w[e]
        d = A.sum(1)
        X = X0s[r] - X0s[r].mean(0)
        for _ in range(sweeps):
            X = (1 - omega) * X + omega * (A @ X) / d[:, None]
        cand = np.nonzero(~inP)[0]
        s = w[cand] * ((X[u[cand]] - X[v[cand]]) ** 2).sum(1)
        take = sorted(range(len(cand)), key=lambda i: (-s[i], cand[i]))[:q]
        inP[cand[take]] = True
        added.append(set(cand[take].tolist()))
    return inP, added


def test_rounds_match_dense_brute_force(orc):
    # a tiny graph where the rounds' choices depend on re-embedding the growing sparsifier
    g = W.random_connected(40, 110, seed=93, wdist=("lognormal", 0.0, 1.0))
    rounds, sweeps, frac = 4, 5, 0.3
    X0s = [W.random_block(g.n, 6, 94 + r) for r in range(rounds)]
    res = orc.sparsify_rounds(g.n, g.u, g.v, g.w, X0s, rounds, sweeps, frac)
    inP, added = _dense_rounds(g.n, g.u, g.v, g.w, X0s, rounds, sweeps, frac, 0.5)
    assert np.array_equal(res.keep > 0, inP)
    for lr, ref in zip(res.levels, added):
        assert set(lr.chosen.tolist()) == ref
    # the rounds add disjoint sets that together are the whole budget
    chosen = np.concatenate([lr.chosen for lr in res.levels])
    assert len(set(chosen.tolist())) == len(chosen) == orc.ksel(frac, g.m - (g.n - 1))


def test_rounds_lower_the_condition_number(orc):
    # the 64x64 grid workload (K=8, T=10, f=5%): re-embedding on the grown
    # sparsifier in 5 rounds beats one pass with the same budget on every seed
    g = W.workload_graph("grid64")
    k1, k5 = [], []
    for seed in range(5):
        X0s = [W.random_block(g.n, 8, 500 + 10 * seed + r) for r in range(5)]
        r1 = orc.sparsify_rounds(g.n, g.u, g.v, g.w, X0s[:1], 1, 10, 0.05)
        r5 = orc.sparsify_rounds(g.n, g.u, g.v, g.w, X0s, 5, 10, 0.05)
        assert (r1.keep == 2).sum() == (r5.keep == 2).sum()
        k1.append(orc.kappa_sparse(g.n, g.u, g.v, g.w, r1.keep > 0)[0])
        k5.append(orc.kappa_sparse(g.n, g.u, g.v, g.w, r5.keep > 0)[0])
    assert all(b < a for a, b in zip(k1, k5)), (k1, k5)


# --------------------------------------------------------------------------- Gauss-Seidel reading

def _mix32(x):
    x &= 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def _jp_brute(n, adj):
    """Jones-Plassmann by sets: local maxima of (hash, id) among the uncoloured,
    smallest colour free among earlier-coloured neighbours."""
    prio = {p: (_mix32(p), p) for p in range(n)}
    color, left = {}, set(range(n))
    while left:
        chosen = [p for p in left if all(prio[p] > prio[q] for q in adj[p] if q in left)]
        for p in chosen:
            used = {color[q] for q in adj[p] if q in color}
            c = 0
            while c in used:
                c += 1
            color[p] = c
        left -= set(chosen)
    return np.array([color[p] for p in range(n)], np.int32)


@pytest.mark.parametrize("g", [W.grid2d(1, 30, seed=1), W.grid2d(9, 11, seed=2),
                               W.random_connected(60, 200, seed=3),
                               W.Graph(40, np.zeros(39, np.int32), np.arange(1, 40, dtype=np.int32), np.ones(39))],
                         ids=["path", "grid", "random", "star"])
def test_coloring_matches_brute_force(orc, g):
    H = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    c, nc = orc.color(H)
    adj = [set() for _ in range(g.n)]
    for a, b in zip(g.u, g.v):
        adj[a].add(int(b))
        adj[b].add(int(a))
    assert np.array_equal(c, _jp_brute(g.n, adj))
    assert nc == c.max() + 1
    assert np.all(c[g.u] != c[g.v])                       # proper
    deg = np.bincount(np.concatenate([g.u, g.v]), minlength=g.n)
    assert nc <= deg.max() + 1


def test_gauss_seidel_matches_dense(orc):
    g = W.random_connected(50, 140, seed=4, wdist=("lognormal", 0.0, 1.0))
    H = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    c, nc = orc.color(H)
    X0 = W.random_block(g.n, 5, 6)
    A = np.zeros((g.n, g.n))
    A[g.u, g.v] = g.w
    A[g.v, g.u] = g.w
    d = A.sum(1)
    for omega in (1.0, 0.5):
        X = X0.copy()
        for _ in range(4):
            for cc in range(nc):
                rows = np.nonzero(c == cc)[0]
                X[rows] = (1 - omega) * X[rows] + omega * (A[rows] @ X) / d[rows, None]
        got = orc.smooth_gs(H, X0, 4, omega, c, nc)
        assert np.max(np.abs(got - X)) < 1e-12 * np.max(np.abs(X0))


def test_gauss_seidel_against_jacobi_on_grid(orc):
    # the 64x64 grid workload (K=8, T=10, f=5%), 5 seeds: plain Gauss-Seidel
    # (omega 1, the paper's wording) against the damped Jacobi reading at equal
    # sweeps; measured medians 543 (GS, omega 1), 457 (Jacobi), 429 (GS, omega 1/2)
    g = W.workload_graph("grid64")
    kj, kg1, kg5 = [], [], []
    for seed in range(5):
        X0 = W.random_block(g.n, 8, 700 + seed)
        for out, kw in ((kj, {}), (kg1, {"omega": 1.0, "smoother": "gs"}), (kg5, {"omega": 0.5, "smoother": "gs"})):
            r = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, 10, 0.05, **kw)
            out.append(orc.kappa_sparse(g.n, g.u, g.v, g.w, r.keep > 0)[0])
    mj, m1, m5 = np.median(kj), np.median(kg1), np.median(kg5)
    assert m5 < mj < m1, (mj, m1, m5)


# --------------------------------------------------------------------------- downstream PCG

def test_pcg_special_cases(orc):
    g = W.mesh3d(8, 7, 6, seed=5, wdist=("lognormal", 0.0, 1.0))
    # the graph preconditioning itself: one iteration
    assert orc.pcg_iterations(g.n, g.u, g.v, g.w, np.ones(g.m, bool)) == 1
    # plain CG counts the same iterations as SciPy's CG with the same stopping rule
    import scipy.sparse.linalg as sla

    LG = orc.laplacian_sparse(g.n, g.u, g.v, g.w)[1:, 1:].tocsr()
    b = np.random.default_rng(0).standard_normal(g.n - 1)
    count = [0]

    def cb(_):
        count[0] += 1

    sla.cg(LG, b, rtol=1e-3, atol=0.0, maxiter=10000, callback=cb)
    assert abs(orc.pcg_iterations(g.n, g.u, g.v, g.w, None) - count[0]) <= 1
    # a spanning-tree preconditioner beats none
    tree = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    assert orc.pcg_iterations(g.n, g.u, g.v, g.w, tree) < count[0]


# --------------------------------------------------------------------------- random test vectors

def test_philox_known_answers(orc):
    # the known-answer values published with Philox4x32-10 (Salmon et al., SC'11)
    cases = [([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
             ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
             ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
              [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1])]
    for ctr, key, want in cases:
        assert orc.philox4x32_10(ctr, key).tolist() == want


def test_random_block_box_muller(orc):
    n, k, seed, block = 1001, 3, 0x123456789ABCDEF, 7      # odd total: the last pair keeps z0 only
    X = orc.random_block(n, k, seed, block).reshape(-1)
    for j in (0, 1, 17, (n * k - 1) // 2):
        r = orc.philox4x32_10([j & 0xFFFFFFFF, j >> 32, block, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u1 = float(((int(r[0]) << 32 | int(r[1])) >> 11)) * 2.0 ** -53
        u2 = float(((int(r[2]) << 32 | int(r[3])) >> 11)) * 2.0 ** -53
        rho = math.sqrt(-2.0 * math.log(1.0 - u1))
        assert abs(X[2 * j] - rho * math.cos(2 * math.pi * u2)) <= 4e-16 * max(1.0, rho)
        if 2 * j + 1 < n * k:
            assert abs(X[2 * j + 1] - rho * math.sin(2 * math.pi * u2)) <= 4e-16 * max(1.0, rho)


def test_random_block_is_standard_normal(orc):
    from scipy import stats

    X = orc.random_block(250000, 4, 2024, 0).reshape(-1)
    N = X.size
    assert abs(X.mean()) < 5 / math.sqrt(N)
    assert abs(X.var() - 1) < 5 * math.sqrt(2 / N)
    assert stats.kstest(X, "norm").pvalue > 1e-3
    # blocks and seeds give different streams
    assert not np.allclose(orc.random_block(100, 4, 2024, 1), orc.random_block(100, 4, 2024, 0))
    assert not np.allclose(orc.random_block(100, 4, 2025, 0), orc.random_block(100, 4, 2024, 0))


# --------------------------------------------------------------------------- sigma-driven stopping

def _canon(n, pairs, w):
    pairs = np.array(pairs, dtype=np.int64)
    a, b = np.minimum(pairs[:, 0], pairs[:, 1]), np.maximum(pairs[:, 0], pairs[:, 1])
    o = np.lexsort((b, a))
    return a[o].astype(np.int32), b[o].astype(np.int32), np.asarray(w, dtype=np.float64)[o]


def test_tree_dfs_hand_example(orc):
    # node 4 is entered from 2; its neighbours 1, 2, 3, 5 are taken after 2 and wrap round: 3, 5, 1
    u, v, w = _canon(6, [(0, 2), (1, 4), (2, 4), (3, 4), (4, 5)], [1.0, 2.0, 3.0, 4.0, 5.0])
    t = orc.tree_dfs(6, u, v, w, np.ones(5, bool))
    assert t.order.tolist() == [0, 2, 4, 3, 5, 1]
    assert t.parent.tolist() == [-1, 0, 1, 2, 2, 2]
    assert t.size.tolist() == [6, 5, 4, 1, 1, 1]
    assert t.pw.tolist() == [0.0, 1.0, 3.0, 4.0, 5.0, 2.0]
    assert t.tdown.tolist() == [-1, 0, 1, 2, 4, 6]
    assert t.tup.tolist() == [-1, 9, 8, 3, 5, 7]


@pytest.mark.parametrize("g", TINY + [W.grid2d(30, 30, seed=21)])
def test_tree_dfs_invariants(orc, g):
    tree = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    t = orc.tree_dfs(g.n, g.u, g.v, g.w, tree)
    n = g.n
    assert sorted(t.order.tolist()) == list(range(n)) and t.order[0] == 0
    assert np.all(t.parent[1:] < np.arange(1, n)) and t.parent[0] == -1
    # every subtree is the contiguous preorder range [i, i + size)
    sizes = np.ones(n, dtype=np.int64)
    for i in range(n - 1, 0, -1):
        sizes[t.parent[i]] += sizes[i]
    assert np.array_equal(sizes, t.size)
    for i in range(1, n):
        assert t.parent[i] <= i - 1 and i < t.parent[i] + t.size[t.parent[i]]
    # the walk crosses each edge once each way: 2(n-1) distinct steps, a subtree's
    # walk spans 2 size - 1 steps
    steps = np.concatenate([t.tdown[1:], t.tup[1:]])
    assert sorted(steps.tolist()) == list(range(2 * (n - 1)))
    assert np.array_equal(t.tup[1:] - t.tdown[1:], 2 * t.size[1:] - 1)
    # the parent edges are the tree edges, with their weights
    pe = {(min(a, b), max(a, b)): c for a, b, c in zip(g.u[tree], g.v[tree], g.w[tree])}
    for i in range(1, n):
        a, b = int(t.order[i]), int(t.order[t.parent[i]])
        assert pe[(min(a, b), max(a, b))] == t.pw[i]


def test_tree_solve_against_pseudo_inverse(orc):
    g = W.random_connected(40, 60, seed=31, wdist=("lognormal", 0.0, 1.0))
    tree = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    t = orc.tree_dfs(g.n, g.u, g.v, g.w, tree)
    B = np.random.default_rng(5).standard_normal((g.n, 3))
    L = csgraph_laplacian(adjacency(g.n, g.u[tree], g.v[tree], g.w[tree]))
    X = orc.tree_solve(t, B)
    assert np.allclose(X, np.linalg.pinv(L) @ B, rtol=0, atol=1e-10 * np.abs(X).max())


def test_tree_solve_path_closed_form(orc):
    # unit path 0-1-...-(n-1), demand +1 at 0 and -1 at n-1: potentials fall by 1 per edge
    n = 25
    u, v, w = _canon(n, [(i, i + 1) for i in range(n - 1)], np.ones(n - 1))
    t = orc.tree_dfs(n, u, v, w, np.ones(n - 1, bool))
    b = np.zeros(n)
    b[0], b[-1] = 1.0, -1.0
    x = orc.tree_solve(t, b)
    want = (n - 1) / 2.0 - np.arange(n)
    assert np.allclose(x, want, rtol=0, atol=1e-13)


def test_tree_solve_residual_on_grid(orc):
    g = W.grid2d(40, 40, seed=22, wdist=("lognormal", 0.0, 1.0))
    tree = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    t = orc.tree_dfs(g.n, g.u, g.v, g.w, tree)
    B = np.random.default_rng(6).standard_normal((g.n, 4))
    X = orc.tree_solve(t, B)
    L = orc.laplacian_sparse(g.n, g.u[tree], g.v[tree], g.w[tree])
    R = L @ X - (B - B.mean(axis=0))
    assert np.abs(R).max() <= 1e-11 * np.abs(B).max() * math.sqrt(g.n)
    assert np.abs(X.mean(axis=0)).max() <= 1e-12 * np.abs(X).max()


def test_kappa_estimate_one_edge_closed_form(orc):
    # G = cycle, P = G minus one edge e: L_G = L_P + w_e b b^T, so the pencil has one
    # eigenvalue 1 + w_e * R_P(e) (R_P: the path's resistance) and all others 1
    n = 60
    rng = np.random.default_rng(7)
    u, v, w = _canon(n, [(i, i + 1) for i in range(n - 1)] + [(0, n - 1)], rng.uniform(0.5, 2.0, n))
    off = int(np.nonzero((u == 0) & (v == n - 1))[0][0])
    mask = np.ones(n, bool)
    mask[off] = False
    want = 1.0 + w[off] * float(np.sum(1.0 / w[mask]))
    th = orc.kappa_estimate(n, u, v, w, mask, rng.standard_normal((n, 3)), 12)
    assert abs(th[-1] - want) <= 1e-10 * want
    assert all(t <= want * (1 + 1e-12) for t in th)


@pytest.mark.parametrize("frac", [0.0, 0.1])
def test_kappa_estimate_bounds_dense(orc, frac):
    g = W.grid2d(14, 14, seed=23, wdist=("lognormal", 0.0, 1.0))
    base = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    mask = base.copy()
    if frac:
        lr, _ = orc.score_level(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 8, 3), 10, 0.5, frac)
        mask[lr.chosen] = True
    _, lmax, lmin = orc.kappa_dense(g.n, g.u, g.v, g.w, mask)
    assert abs(lmin - 1.0) < 1e-9       # P inside G with G's weights: lambda_min = 1 here
    th = orc.kappa_estimate(g.n, g.u, g.v, g.w, mask, orc.random_block(g.n, 8, 4), 40)
    assert all(t <= lmax * (1 + 1e-9) for t in th)          # Ritz values never exceed lambda_max
    assert th[-1] >= lmax * (1 - 1e-6)                      # and converge to it
    assert th[4] >= 0.5 * lmax


def test_sigma_stopping(orc):
    g = W.grid2d(16, 16, seed=24, wdist=("lognormal", 0.0, 1.0))
    n, k, frac, sweeps, est = g.n, 8, 0.05, 10, 8
    X0s = [orc.random_block(n, k, 9, r) for r in range(16)]
    Y0s = [orc.random_block(n, 4, 9, 64 + j) for j in range(17)]
    base = orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0
    q = orc.ksel(frac, int((~base).sum()))
    # sigma large enough: the tree alone is accepted
    res, kap = orc.sparsify_sigma(n, g.u, g.v, g.w, X0s, Y0s, 1e4, frac, 16, sweeps, est)
    assert len(kap) == 1 and res.levels == [] and np.array_equal(res.keep, base.astype(np.uint8))
    # a tight sigma: batches of q edges until the estimate drops below sigma^2 or the cap
    sigma = math.sqrt(0.3 * kap[0])
    res, kap = orc.sparsify_sigma(n, g.u, g.v, g.w, X0s, Y0s, sigma, frac, 16, sweeps, est)
    r = len(res.levels)
    assert r >= 1 and len(kap) == r + 1
    assert kap[-1] <= sigma ** 2 and all(x > sigma ** 2 for x in kap[:-1])
    assert int((res.keep == 2).sum()) == r * q
    # the true condition number never rises as edges are added (L_P grows in the Loewner order)
    mask = base.copy()
    prev = orc.kappa_dense(n, g.u, g.v, g.w, mask)[1]
    for lr in res.levels:
        mask[lr.chosen] = True
        cur = orc.kappa_dense(n, g.u, g.v, g.w, mask)[1]
        assert cur <= prev * (1 + 1e-9)
        prev = cur
    # the round cap bounds the additions
    res2, kap2 = orc.sparsify_sigma(n, g.u, g.v, g.w, X0s, Y0s, 1.0, frac, 2, sweeps, est)
    assert len(res2.levels) == 2 and len(kap2) == 3


# --------------------------------------------------------------------------- threads

def test_threads_give_the_same_bits(orc):
    """Smoothing rows and edge scores are split over threads; each row or edge
    is one thread's work in the fixed order, so any thread count gives the same
    bits (the CPU baseline is timed on one thread and on all host cores)."""
    g = W.powergrid(60, 70, 0.02, seed=91)
    intree, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    t = intree.astype(bool)
    H = orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t])
    Xc, _ = orc.center(W.random_block(g.n, 16, 92))
    cand = np.nonzero(~t)[0]
    out = []
    for threads in (1, 3, max(orc.max_threads(), 2)):
        orc.set_threads(threads)
        X = orc.smooth(H, Xc, 12)
        out.append((X, orc.edge_scores(X, g.u[cand], g.v[cand], g.w[cand])))
    orc.set_threads(orc.max_threads())
    for X, s in out[1:]:
        assert np.array_equal(X, out[0][0]) and np.array_equal(s, out[0][1])
