"""GPU parity: libsfg (through its C ABI) against the CPU FP64 oracle.

FP64 paths are compared bit for bit: the GPU kernels add every row and every
score in the oracle's order with one rounding per operation.  Reduced
precision paths are compared with tolerances derived from their unit
roundoff.
"""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_07633_amd import sfg

    sfg.lib()
    return sfg


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


GRAPHS = {
    "grid64": lambda: W.workload_graph("grid64"),
    "rand1500": lambda: W.random_connected(1500, 4000, seed=71, wdist=("lognormal", 0.0, 1.0)),
    # over 4 edges per node: the CSR is built edge-parallel instead of by row walks
    "dense800": lambda: W.random_connected(800, 6400, seed=75, wdist=("lognormal", 0.0, 1.0)),
    "pgrid_97": lambda: W.powergrid(97, 103, 0.02, seed=72),
    "mesh_13": lambda: W.mesh3d(13, 11, 9, seed=73),
    "path2": lambda: W.grid2d(1, 2, seed=74),
    "star": lambda: W.Graph(300, np.zeros(299, np.int32), np.arange(1, 300, dtype=np.int32),
                            np.linspace(0.5, 2.0, 299), name="star"),
}


@pytest.fixture(scope="module", params=list(GRAPHS))
def graph(request):
    return GRAPHS[request.param]()


# --------------------------------------------------------------------------- a1: Laplacian CSR

@pytest.mark.parametrize("masked", [False, True])
def test_laplacian_csr_bitwise(S, orc, graph, masked):
    g = graph
    mask = None
    if masked:
        mask, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    for wdt in (np.float64, np.float32):
        w = g.w.astype(wdt)
        sel = np.ones(g.m, bool) if mask is None else mask.astype(bool)
        ref = orc.laplacian_csr(g.n, g.u[sel], g.v[sel], w[sel].astype(np.float64))
        H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(w), mask=None if mask is None else dev(mask))
        assert H.nnz == ref.col.shape[0]
        assert np.array_equal(host(H.rowptr), ref.rowptr.astype(np.int32))
        assert np.array_equal(host(H.col)[:H.nnz], ref.col)
        ids = np.nonzero(sel)[0]
        assert np.array_equal(host(H.eid)[:H.nnz], ids[ref.eid])
        assert np.array_equal(host(H.val)[:H.nnz], ref.val.astype(wdt))
        assert np.array_equal(host(H.deg), ref.deg.astype(wdt))


@pytest.mark.parametrize("which", ["tree", "half", "none", "all"])
def test_csr_select_bitwise(S, orc, graph, which):
    # the CSR of a subgraph taken from G's CSR equals the one built from the masked edge list
    g = graph
    rng = np.random.default_rng(41)
    mask = {"tree": orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0].astype(np.uint8),
            "half": (rng.random(g.m) < 0.5).astype(np.uint8),
            "none": np.zeros(g.m, np.uint8), "all": np.full(g.m, 3, np.uint8)}[which]
    for wdt in (np.float64, np.float32):
        u, v, w = dev(g.u), dev(g.v), dev(g.w.astype(wdt))
        G = S.sfg_laplacian_csr(g.n, u, v, w)
        ref = S.sfg_laplacian_csr(g.n, u, v, w, mask=dev(mask))
        got = S.sfg_csr_select(G, dev(mask))
        assert got.nnz == ref.nnz == 2 * int((mask != 0).sum())
        for f in ("rowptr", "deg"):
            assert np.array_equal(host(getattr(got, f)), host(getattr(ref, f))), f
        for f in ("col", "val", "eid"):
            assert np.array_equal(host(getattr(got, f))[:got.nnz], host(getattr(ref, f))[:ref.nnz]), f


def test_csr_select_errors(S):
    g = W.grid2d(5, 5, seed=42)
    G = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    mask = dev(np.ones(g.m, np.uint8))
    with pytest.raises(S.SfgError):
        S.sfg_csr_select(G, mask, ws=torch.empty(8, dtype=torch.uint8, device="cuda"))
    G.eid = None
    with pytest.raises((S.SfgError, AttributeError, TypeError)):
        S.sfg_csr_select(G, mask)


# --------------------------------------------------------------------------- a2+a3: smoothing

@pytest.mark.parametrize("k,sweeps", [(1, 3), (3, 5), (8, 10), (16, 20), (32, 4), (64, 2), (16, 0)])
def test_smooth_f64_bitwise(S, orc, graph, k, sweeps):
    g = graph
    X0 = W.random_block(g.n, k, 100 + k)
    ref_csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    Xc, _ = orc.center(X0)
    ref = orc.smooth(ref_csr, Xc, sweeps, 0.5)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    X = S.sfg_smooth(H, dev(X0), sweeps, 0.5, storage=torch.float64)
    np.testing.assert_array_equal(host(X), ref)


def test_column_mean_under_heavy_cancellation(S, orc):
    """Centring subtracts each column's mean; the oracle takes the exactly rounded column sum (fsum).  These
    columns defeat a plain FP64 sum (big values that cancel around small ones, near-opposite pairs that cancel
    to 2^-50 of their size) and are spread over many blocks of the GPU's partial sums; the GPU's double-double
    sum must still round to the same mean, so the centred block is bit-identical."""
    import math

    rng = np.random.default_rng(77)
    n = 300_000
    c0 = np.tile([2.0 ** 53, 1.0, -2.0 ** 53, 1.0], n // 4)
    x = rng.standard_normal(n // 2) * 2.0 ** 20
    a = x + rng.standard_normal(n // 2) * 2.0 ** -30         # rounded: the pair sums are what is left of delta
    c1 = np.empty(n)
    c1[0::2], c1[1::2] = a, -x
    c2 = rng.permutation(c1)
    c3 = rng.standard_normal(n)
    X0 = np.ascontiguousarray(np.stack([c0, c1, c2, c3], axis=1))
    for c in (0, 1, 2):
        assert sum(X0[:, c].tolist()) != math.fsum(X0[:, c])       # a plain sequential sum is wrong here
    g = W.grid2d(1, n, seed=78)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    got = host(S.sfg_smooth(H, dev(X0), 0, storage=torch.float64))
    ref, mean = orc.center(X0)
    assert all(mean[c] == math.fsum(X0[:, c]) / n for c in range(4))
    np.testing.assert_array_equal(got, ref)


def test_smooth_omega_and_tree(S, orc):
    g = W.powergrid(60, 70, 0.02, seed=75)
    tree, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    t = tree.astype(bool)
    X0 = W.random_block(g.n, 16, 9)
    ref_csr = orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t])
    for omega in (0.5, 0.3, 1.0):
        ref = orc.smooth(ref_csr, orc.center(X0)[0], 7, omega)
        H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w), mask=dev(tree))
        X = S.sfg_smooth(H, dev(X0), 7, omega)
        np.testing.assert_array_equal(host(X), ref)


@pytest.mark.parametrize("k,sweeps", [(16, 1), (16, 2), (24, 5), (40, 3), (8, 4)])
def test_smooth_f64_tree_column_parts(S, orc, k, sweeps, monkeypatch):
    # FP64 blocks are swept in 8-column parts when a part's working set fits the
    # memory-side cache (the 1M-node power grid); SFG_SWEEP_SPLIT=2 forces the
    # part sweeps (first sweep from x0, middle sweeps in part buffers, last into
    # the output columns) on a small tree
    monkeypatch.setenv("SFG_SWEEP_SPLIT", "2")
    g = W.powergrid(41, 53, 0.02, seed=76)
    tree, _ = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    t = tree.astype(bool)
    X0 = W.random_block(g.n, k, 300 + k)
    ref = orc.smooth(orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t]), orc.center(X0)[0], sweeps, 0.5)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w), mask=dev(tree))
    X = S.sfg_smooth(H, dev(X0), sweeps, 0.5, storage=torch.float64)
    np.testing.assert_array_equal(host(X), ref)
    # the graph itself (4 entries per row) under the forced split
    ref_g = orc.smooth(orc.laplacian_csr(g.n, g.u, g.v, g.w), orc.center(X0)[0], sweeps, 0.5)
    Hg = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    np.testing.assert_array_equal(host(S.sfg_smooth(Hg, dev(X0), sweeps, 0.5, storage=torch.float64)), ref_g)


@pytest.mark.parametrize("storage,final_f32,tol", [
    (torch.float32, False, 2e-5),
    (torch.float16, True, 6e-3),
    (torch.float16, False, 2e-2),
    (torch.bfloat16, True, 5e-2),
])
def test_smooth_reduced_precision(S, orc, storage, final_f32, tol):
    # Bound: every sweep is a convex combination, so the stored iterate carries
    # at most ~(sweeps + 1) storage roundings of |X| scale; tol is that bound
    # (u = 6e-8, 4.9e-4, 3.9e-3 for FP32, FP16, BF16) relative to max |X0|.
    g = W.powergrid(80, 80, 0.02, seed=76)
    k, T = 16, 20
    X0 = W.random_block(g.n, k, 11)
    ref = orc.smooth(orc.laplacian_csr(g.n, g.u, g.v, g.w), orc.center(X0)[0], T, 0.5)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w.astype(np.float32)))
    X = S.sfg_smooth(H, dev(X0), T, 0.5, storage=storage, final_f32=final_f32)
    err = np.max(np.abs(host(X.float()).astype(np.float64) - ref)) / np.max(np.abs(X0))
    assert err < tol, err


# --------------------------------------------------------------------------- a4: scores and affinities

def test_scores_f64_bitwise(S, orc, graph):
    g = graph
    k = 16
    X = W.random_block(g.n, k, 5)
    ref = orc.edge_scores(X, g.u, g.v, g.w)
    s = S.sfg_edge_scores(dev(X), dev(g.u), dev(g.v), dev(g.w))
    np.testing.assert_array_equal(host(s), ref)
    # candidate subset (every third edge)
    cand = np.arange(0, g.m, 3, dtype=np.int32)
    s2 = S.sfg_edge_scores(dev(X), dev(g.u), dev(g.v), dev(g.w), cand=dev(cand))
    np.testing.assert_array_equal(host(s2), ref[cand])


@pytest.mark.parametrize("k", [1, 5, 8, 32, 64])
def test_scores_and_affinity_shapes(S, orc, k):
    g = W.random_connected(700, 1500, seed=77)
    X = W.random_block(g.n, k, 6)
    np.testing.assert_array_equal(host(S.sfg_edge_scores(dev(X), dev(g.u), dev(g.v), dev(g.w))),
                                  orc.edge_scores(X, g.u, g.v, g.w))
    a = S.sfg_affinity(dev(X), dev(g.u), dev(g.v))
    np.testing.assert_array_equal(host(a), orc.affinity(orc.center(X)[0], g.u, g.v))


def test_scores_reduced_precision(S, orc):
    g = W.random_connected(2000, 6000, seed=78)
    X = W.random_block(g.n, 32, 7)
    ref = orc.edge_scores(X, g.u, g.v, g.w)
    w32 = dev(g.w.astype(np.float32))
    for xdt, tol in ((torch.float32, 1e-5), (torch.float16, 3e-2), (torch.bfloat16, 2e-1)):
        s = S.sfg_edge_scores(dev(X).to(xdt), dev(g.u), dev(g.v), w32)
        rel = np.abs(host(s).astype(np.float64) - ref) / np.max(ref)
        assert rel.max() < tol, (xdt, rel.max())


# --------------------------------------------------------------------------- a5: selection

@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_select_topk_matches_sort(S, orc, dt):
    rng = np.random.default_rng(8)
    for ne, ties in ((1, False), (5000, True), (123457, False), (300000, True)):
        s = rng.random(ne) * 10 - 2.0
        if ties:
            s = np.round(s * 16) / 16
        s = s.astype(dt == torch.float64 and np.float64 or np.float32).astype(np.float64)
        eid = np.arange(ne, dtype=np.int32)
        for k in sorted({0, 1, ne // 7, ne // 2, ne}):
            sel, tau = S.sfg_select_topk(dev(s, dt), k)
            pos, tau_ref = orc.select_topk(s, eid, k)
            want = np.zeros(ne, np.uint8)
            want[pos] = 1
            assert np.array_equal(host(sel), want), (ne, k)
            if k:
                assert tau == tau_ref
            else:
                assert tau == float("inf")


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_select_many_equal_keys_at_the_threshold(S, orc, dt):
    """A large run of equal keys straddles the k-th position, so the digit pick
    of every radix pass lands in the same crowded bucket; the marked set must
    still be the first k by (score desc, position asc)."""
    rng = np.random.default_rng(81)
    for ne, share in ((200003, 0.6), (70001, 0.99)):
        s = rng.random(ne) + 2.0
        tied = rng.random(ne) < share
        s[tied] = 1.5
        s[rng.random(ne) < 0.2] = 0.25
        s = s.astype(dt == torch.float64 and np.float64 or np.float32).astype(np.float64)
        eid = np.arange(ne, dtype=np.int32)
        n_above = int((s > 1.5).sum())
        n_tied = int((s == 1.5).sum())
        for k in (n_above + 1, n_above + n_tied // 2, n_above + n_tied - 1, n_above + n_tied):
            sel, tau = S.sfg_select_topk(dev(s, dt), k)
            pos, tau_ref = orc.select_topk(s, eid, k)
            want = np.zeros(ne, np.uint8)
            want[pos] = 1
            assert np.array_equal(host(sel), want), (ne, k)
            assert tau == tau_ref == 1.5


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_select_keys_sharing_their_high_digits(S, orc, dt):
    """Scores that agree in their top 22 bits (and many in more): the first
    radix passes leave almost every key in one bucket, so the pass that copies
    the matching keys to its buffer copies nearly all of them, and the later
    passes work on that buffer."""
    rng = np.random.default_rng(83)
    ne = 250001
    if dt == torch.float64:
        s = 1.0 + rng.integers(0, 1 << 22, ne) * 2.0 ** -50
    else:
        s = 1.0 + rng.integers(0, 1 << 12, ne) * 2.0 ** -23
    s = s.astype(dt == torch.float64 and np.float64 or np.float32).astype(np.float64)
    eid = np.arange(ne, dtype=np.int32)
    for k in (1, 17, ne // 3, ne - 1):
        sel, tau = S.sfg_select_topk(dev(s, dt), k)
        pos, tau_ref = orc.select_topk(s, eid, k)
        want = np.zeros(ne, np.uint8)
        want[pos] = 1
        assert np.array_equal(host(sel), want), k
        assert tau == tau_ref


def test_select_rejects_bad_scores(S):
    s = torch.tensor([1.0, float("nan"), 3.0], dtype=torch.float64, device="cuda")
    with pytest.raises(S.SfgError, match="SFG_ENUMERIC"):
        S.sfg_select_topk(s, 1)
    s = torch.tensor([1.0, -2.0, 3.0, -0.5, 0.0], dtype=torch.float64, device="cuda")
    sel, tau = S.sfg_select_topk(s, 3)          # signed values are ordered too
    assert sel.cpu().tolist() == [1, 0, 1, 0, 1] and tau == 0.0
    sel, tau = S.sfg_select_topk(s.float(), 4)
    assert sel.cpu().tolist() == [1, 0, 1, 1, 1] and tau == -0.5
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_select_topk(s, 6)


# --------------------------------------------------------------------------- spanning tree

def test_spanning_tree(S, orc, graph):
    g = graph
    ref, comps = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    t, c = S.sfg_spanning_tree(g.n, dev(g.u), dev(g.v), dev(g.w))
    assert c == comps == 1
    assert np.array_equal(host(t), ref)


# --------------------------------------------------------------------------- whole single-level pass

@pytest.mark.parametrize("embed", ["sparsifier", "graph"])
def test_sparsify_single_level_matches_oracle(S, orc, graph, embed):
    g = graph
    k, T, f = 8, 10, 0.05
    X0 = W.random_block(g.n, k, 31)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, T, f, embed=embed)
    p = S.make_params(k=k, sweeps=T, frac=f, embed=S.EMBED_GRAPH if embed == "graph" else S.EMBED_SPARSIFIER)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), p)
    assert np.array_equal(host(keep), ref.keep)
    lr = ref.levels[0]
    assert rep[0]["n_cand"] == lr.n_cand and rep[0]["k_sel"] == lr.k_sel
    if lr.k_sel:
        assert rep[0]["tau"] == lr.tau


@pytest.mark.parametrize("rounds", [2, 5])
def test_sparsify_rounds_match_oracle(S, orc, graph, rounds):
    # multi-round densification: each round re-embeds on the grown sparsifier
    g = graph
    k, T, f = 8, 6, 0.1
    X0s = np.stack([W.random_block(g.n, k, 40 + r) for r in range(rounds)])
    ref = orc.sparsify_rounds(g.n, g.u, g.v, g.w, list(X0s), rounds, T, f)
    p = S.make_params(k=k, sweeps=T, frac=f, rounds=rounds)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0s), p)
    assert np.array_equal(host(keep), ref.keep)
    assert len(rep) == rounds
    for r, lr in zip(rep, ref.levels):
        assert r["n_cand"] == lr.n_cand and r["k_sel"] == lr.k_sel
        if lr.k_sel:
            assert r["tau"] == lr.tau


def test_sparsify_rounds_precision_form(S, orc, monkeypatch):
    # FP16 embedding with FP64 re-scoring of the band, round by round (the predicted-cone shortcut is off)
    monkeypatch.setenv("SFG_PRECISION_PREDICT", "0")
    g = W.powergrid(90, 80, 0.02, seed=95)
    k, T, f, R = 16, 8, 0.1, 3
    X0s = np.stack([W.random_block(g.n, k, 96 + r) for r in range(R)])
    ref = orc.sparsify_rounds(g.n, g.u, g.v, g.w, list(X0s), R, T, f)
    p = S.make_params(k=k, sweeps=T, frac=f, rounds=R, storage=torch.float16, final_f32=True, band=0.01)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0s), p)
    assert np.array_equal(host(keep), ref.keep)
    assert all(r["band"] > 0 for r in rep)


def test_sparsify_rounds_errors(S):
    g = W.grid2d(10, 10, seed=97)
    # room for every block the parameters name, so the library itself rejects them
    X0 = dev(np.stack([W.random_block(g.n, 4, 98 + r) for r in range(17)]))
    for kw in ({"rounds": 17}, {"rounds": -1}, {"rounds": 2, "levels": 2}):
        with pytest.raises(S.SfgError):
            S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, S.make_params(k=4, sweeps=3, frac=0.1, **kw))


def test_sparsify_deterministic(S):
    g = W.powergrid(120, 110, 0.02, seed=79)
    X0 = dev(W.random_block(g.n, 16, 3))
    p = S.make_params(k=16, sweeps=20, frac=0.1)
    a, _ = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, p)
    b, _ = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, p)
    assert torch.equal(a, b)


# --------------------------------------------------------------------------- error paths

def test_sparsify_errors(S):
    g = W.grid2d(10, 10, seed=80)
    X0 = dev(W.random_block(g.n, 8, 1))
    p = S.make_params()
    # disconnected: drop every edge at node 0
    keepe = (g.u != 0)
    with pytest.raises(S.SfgError, match="SFG_ENOTCONN"):
        S.sfg_sparsify(g.n, dev(g.u[keepe]), dev(g.v[keepe]), dev(g.w[keepe]), X0, p)
    # malformed: swapped endpoints, unsorted, bad weight
    u2, v2 = g.u.copy(), g.v.copy()
    u2[3], v2[3] = v2[3], u2[3]
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_sparsify(g.n, dev(u2), dev(v2), dev(g.w), X0, p)
    w2 = g.w.copy()
    w2[5] = 0.0
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(w2), X0, p)
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_sparsify(g.n, dev(g.u[::-1].copy()), dev(g.v[::-1].copy()), dev(g.w), X0, p)
    # injected allocation failure
    os.environ["SFG_FAIL_ALLOC_AFTER"] = "3"
    try:
        with pytest.raises(S.SfgError, match="SFG_ENOMEM"):
            S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, p)
    finally:
        del os.environ["SFG_FAIL_ALLOC_AFTER"]
    keep, _ = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, p)   # still works afterwards
    assert int((keep == 1).sum()) == g.n - 1


def test_workspace_too_small(S):
    g = W.grid2d(8, 8, seed=81)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SfgError, match="SFG_EWORKSPACE"):
        S.sfg_smooth(H, dev(W.random_block(g.n, 4, 2)), 3, ws=ws)


# the *_large cases have >= 65536 edges, so later Boruvka rounds run on compacted edge lists
@pytest.mark.parametrize("case", ["unit_grid", "ties_f32", "forest", "chunglu", "ties_large", "forest_large",
                                  "mesh_large", "unit_large"])
def test_spanning_tree_ties_and_forests(S, orc, case):
    if case == "unit_grid":
        g = W.grid2d(37, 41, seed=90, wdist=("unit",))
        w, allowed = g.w, None
    elif case == "unit_large":
        g = W.grid2d(300, 310, seed=95, wdist=("unit",))    # every weight tied: ids decide
        w, allowed = g.w, None
    elif case == "ties_f32":
        g = W.random_connected(5000, 20000, seed=91)
        w, allowed = np.round(g.w * 4) / 4, None            # heavy ties
    elif case == "ties_large":
        g = W.random_connected(60000, 200000, seed=96)
        w, allowed = np.round(g.w * 4) / 4, None
    elif case == "forest":
        g = W.powergrid(60, 50, 0.02, seed=92)
        w = g.w
        allowed = (np.random.default_rng(1).random(g.m) < 0.6).astype(np.uint8)
    elif case == "forest_large":
        g = W.powergrid(250, 240, 0.02, seed=97)
        w = g.w
        allowed = (np.random.default_rng(2).random(g.m) < 0.7).astype(np.uint8)
    elif case == "mesh_large":
        g = W.mesh3d(40, 38, 36, seed=98)
        w, allowed = g.w, None
    else:
        g = W.chung_lu(30000, 300000, 2.2, seed=93)
        w, allowed = g.w32.astype(np.float64), None
    ref, comps = orc.max_spanning_forest(g.n, g.u, g.v, w, allowed=allowed)
    t, c = S.sfg_spanning_tree(g.n, dev(g.u), dev(g.v), dev(w), allowed=None if allowed is None else dev(allowed))
    assert c == comps
    assert np.array_equal(host(t), ref)
    if case == "chunglu":   # FP32 weights give the same forest
        t32, c32 = S.sfg_spanning_tree(g.n, dev(g.u), dev(g.v), dev(g.w32))
        assert c32 == comps and np.array_equal(host(t32), ref)


@pytest.mark.parametrize("storage,tol", [(torch.float32, 2e-5), (torch.float16, 6e-3)])
def test_smooth_hub_rows(S, orc, storage, tol):
    # power-law graph plus a star centre of degree 3000: rows longer than 256
    # entries are swept by a whole workgroup in reduced precision
    g = W.chung_lu(20000, 120000, 2.2, seed=94)
    hub_v = np.arange(1, 3001, dtype=np.int32)
    a = np.concatenate([g.u, np.zeros(3000, np.int32)])
    b = np.concatenate([g.v, hub_v])
    key = np.unique(a.astype(np.int64) * g.n + b)
    u, v = (key // g.n).astype(np.int32), (key % g.n).astype(np.int32)
    w = np.random.default_rng(3).uniform(1, 10, u.shape[0])
    deg = np.bincount(u, minlength=g.n) + np.bincount(v, minlength=g.n)
    assert deg.max() > 3000 and (deg > 256).sum() > 5
    X0 = W.random_block(g.n, 16, 12)
    ref = orc.smooth(orc.laplacian_csr(g.n, u, v, w), orc.center(X0)[0], 20, 0.5)
    H = S.sfg_laplacian_csr(g.n, dev(u), dev(v), dev(w.astype(np.float32)))
    X = S.sfg_smooth(H, dev(X0), 20, 0.5, storage=storage, final_f32=True)
    err = np.max(np.abs(host(X.float()).astype(np.float64) - ref)) / np.max(np.abs(X0))
    assert err < tol, err
    # deterministic
    X2 = S.sfg_smooth(H, dev(X0), 20, 0.5, storage=storage, final_f32=True)
    assert torch.equal(X, X2)


@pytest.mark.parametrize("n,center", [(6000, 5000), (10000, 9999), (3000, 0)])
def test_csr_long_lower_parts(S, orc, n, center):
    # a star whose centre has a lower part of up to n-1 entries (LDS and global rank paths)
    others = np.array([p for p in range(n) if p != center], dtype=np.int64)
    a = np.minimum(others, center)
    b = np.maximum(others, center)
    extra = np.arange(0, n - 1, 7)
    key = np.unique(np.concatenate([a * n + b, extra * n + extra + 1]))
    u, v = (key // n).astype(np.int32), (key % n).astype(np.int32)
    w = np.random.default_rng(n).uniform(0.5, 2.0, u.shape[0])
    ref = orc.laplacian_csr(n, u, v, w)
    H = S.sfg_laplacian_csr(n, dev(u), dev(v), dev(w))
    assert np.array_equal(host(H.col)[:H.nnz], ref.col)
    assert np.array_equal(host(H.eid)[:H.nnz], ref.eid)
    assert np.array_equal(host(H.val)[:H.nnz], ref.val)
    assert np.array_equal(host(H.deg), ref.deg)


@pytest.mark.parametrize("masked", [False, True])
def test_csr_medium_lower_parts(S, orc, masked):
    # a path (under 4 edges per node: the row walks) with rows whose lower parts hold 2..40 entries: in registers
    # up to 8, ranked by one thread from a copy up to 32, by a workgroup beyond
    n = 3000
    rng = np.random.default_rng(91)
    key = [np.arange(n - 1) * n + np.arange(1, n)]
    for q, cnt in ((2999, 20), (2998, 9), (2990, 32), (2980, 33), (2970, 40), (2960, 8), (2950, 2)):
        lo = rng.choice(q - 1, cnt, replace=False)
        key.append(lo * n + q)
    key = np.unique(np.concatenate(key))
    u, v = (key // n).astype(np.int32), (key % n).astype(np.int32)
    w = rng.uniform(0.5, 2.0, u.shape[0])
    sel = rng.random(u.shape[0]) < 0.8 if masked else np.ones(u.shape[0], bool)
    assert u.shape[0] <= 4 * n
    ref = orc.laplacian_csr(n, u[sel], v[sel], w[sel])
    H = S.sfg_laplacian_csr(n, dev(u), dev(v), dev(w), mask=dev(sel.astype(np.uint8)) if masked else None)
    assert H.nnz == ref.col.shape[0]
    assert np.array_equal(host(H.rowptr), ref.rowptr.astype(np.int32))
    assert np.array_equal(host(H.col)[:H.nnz], ref.col)
    assert np.array_equal(host(H.eid)[:H.nnz], np.nonzero(sel)[0][ref.eid])
    assert np.array_equal(host(H.val)[:H.nnz], ref.val)
    assert np.array_equal(host(H.deg), ref.deg)


@pytest.mark.parametrize("keep", [0.5, 0.03, 1.0])
def test_csr_masked_long_slices(S, orc, keep):
    # hubs whose upper slices (edges (p, q), q > p) run past one wavefront's 64 edges, with a random share of the
    # edges masked out, beside short rows: the walks count and place the kept edges in order
    n = 5000
    rng = np.random.default_rng(int(keep * 1000) + 17)
    hubs = np.array([0, 1, 7, 4000])
    key = [h * n + np.arange(h + 1, n) for h in hubs]
    key.append(np.arange(0, n - 1) * n + np.arange(1, n))
    key.append(rng.integers(0, n, 20000) * n + rng.integers(0, n, 20000))
    key = np.concatenate(key)
    a, b = key // n, key % n
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    key = key[key // n != key % n]
    u, v = (key // n).astype(np.int32), (key % n).astype(np.int32)
    w = rng.uniform(0.5, 2.0, u.shape[0])
    sel = rng.random(u.shape[0]) < keep
    for wdt in (np.float64, np.float32):
        wt = w.astype(wdt)
        ref = orc.laplacian_csr(n, u[sel], v[sel], wt[sel].astype(np.float64))
        H = S.sfg_laplacian_csr(n, dev(u), dev(v), dev(wt), mask=dev(sel.astype(np.uint8)))
        assert H.nnz == ref.col.shape[0]
        assert np.array_equal(host(H.rowptr), ref.rowptr.astype(np.int32))
        assert np.array_equal(host(H.col)[:H.nnz], ref.col)
        assert np.array_equal(host(H.eid)[:H.nnz], np.nonzero(sel)[0][ref.eid])
        assert np.array_equal(host(H.val)[:H.nnz], ref.val.astype(wdt))
        assert np.array_equal(host(H.deg), ref.deg.astype(wdt))


# --------------------------------------------------------------------------- Gauss-Seidel reading

def test_color_matches_oracle(S, orc, graph):
    g = graph
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    color, rows, ptr, nc = S.sfg_color(H)
    ref, nref = orc.color(orc.laplacian_csr(g.n, g.u, g.v, g.w))
    assert nc == nref
    assert np.array_equal(host(color), ref)
    want = np.concatenate([np.nonzero(ref == c)[0] for c in range(nref)]).astype(np.int32)
    assert np.array_equal(host(rows), want)
    assert np.array_equal(host(ptr)[:nc + 1], np.concatenate([[0], np.cumsum(np.bincount(ref, minlength=nref))]))


@pytest.mark.parametrize("k,sweeps,omega", [(8, 5, 1.0), (16, 3, 0.5), (3, 4, 1.0), (16, 0, 1.0)])
def test_smooth_gs_f64_bitwise(S, orc, graph, k, sweeps, omega):
    g = graph
    X0 = W.random_block(g.n, k, 60 + k)
    ref_csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    c, nc = orc.color(ref_csr)
    ref = orc.smooth_gs(ref_csr, orc.center(X0)[0], sweeps, omega, c, nc)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w))
    X = S.sfg_smooth_gs(H, S.sfg_color(H), dev(X0), sweeps, omega)
    np.testing.assert_array_equal(host(X), ref)


def test_smooth_gs_f32(S, orc):
    g = W.powergrid(70, 60, 0.02, seed=61)
    X0 = W.random_block(g.n, 16, 62)
    ref_csr = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    c, nc = orc.color(ref_csr)
    ref = orc.smooth_gs(ref_csr, orc.center(X0)[0], 10, 1.0, c, nc)
    H = S.sfg_laplacian_csr(g.n, dev(g.u), dev(g.v), dev(g.w.astype(np.float32)))
    X = S.sfg_smooth_gs(H, S.sfg_color(H), dev(X0), 10, 1.0, storage=torch.float32)
    err = np.max(np.abs(host(X).astype(np.float64) - ref)) / np.max(np.abs(X0))
    assert err < 2e-5, err


@pytest.mark.parametrize("omega", [1.0, 0.5])
def test_sparsify_gauss_seidel_matches_oracle(S, orc, graph, omega):
    g = graph
    k, T, f = 8, 6, 0.1
    X0 = W.random_block(g.n, k, 63)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, T, f, omega=omega, smoother="gs")
    p = S.make_params(k=k, sweeps=T, frac=f, omega=omega, smoother=S.SMOOTH_GAUSS_SEIDEL)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), p)
    assert np.array_equal(host(keep), ref.keep)
    if ref.levels[0].k_sel:
        assert rep[0]["tau"] == ref.levels[0].tau


def test_gauss_seidel_unsupported_combinations(S):
    g = W.grid2d(10, 10, seed=64)
    X0 = dev(W.random_block(g.n, 4, 65))
    for kw in ({"storage": torch.float16}, {"storage": torch.float32, "band": 0.01}, {"smoother": 2}):
        kw.setdefault("smoother", S.SMOOTH_GAUSS_SEIDEL)
        with pytest.raises(S.SfgError):
            S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), X0, S.make_params(k=4, sweeps=3, frac=0.1, **kw))


# --------------------------------------------------------------------------- random blocks on the device

@pytest.mark.parametrize("n,k,seed,block", [(1000, 16, 7, 0), (333, 3, 2 ** 40 + 5, 3), (1, 1, 0, 0)])
def test_random_block_matches_oracle(S, orc, n, k, seed, block):
    # the integer generator is exact; log/cos/sin are the device math library's
    got = host(S.sfg_random_block(n, k, seed, block))
    ref = orc.random_block(n, k, seed, block)
    assert np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))) < 1e-14


def test_sparsify_draws_blocks_from_the_seed(S, orc):
    g = W.powergrid(80, 70, 0.02, seed=66)
    k, T, f, seed = 16, 10, 0.1, 99
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), None, S.make_params(k=k, sweeps=T, frac=f, seed=seed))
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, orc.random_block(g.n, k, seed, 0), T, f)
    assert np.array_equal(host(keep), ref.keep)
    # rounds draw block r for round r
    keep2, _ = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), None,
                              S.make_params(k=k, sweeps=T, frac=f, seed=seed, rounds=3))
    ref2 = orc.sparsify_rounds(g.n, g.u, g.v, g.w, [orc.random_block(g.n, k, seed, r) for r in range(3)], 3, T, f)
    assert np.array_equal(host(keep2), ref2.keep)


def _hub_graph(seed):
    # a random connected graph plus three hubs joined to 1,500 random nodes each (rows far over 256 entries)
    base = W.random_connected(3000, 6000, seed=seed, wdist=("lognormal", 0.0, 1.0))
    rng = np.random.default_rng(seed)
    a = [base.u.astype(np.int64)]
    b = [base.v.astype(np.int64)]
    for h in (5, 1700, 2999):
        nb = rng.choice(np.setdiff1d(np.arange(3000), [h]), 1500, replace=False)
        a.append(np.minimum(nb, h))
        b.append(np.maximum(nb, h))
    key = np.unique(np.concatenate(a) * 3000 + np.concatenate(b))
    u, v = (key // 3000).astype(np.int32), (key % 3000).astype(np.int32)
    w = rng.lognormal(0.0, 1.0, u.shape[0])
    return W.Graph(3000, u, v, w, name="hubs")


@pytest.mark.parametrize("embed", ["sparsifier", "graph"])
def test_fp64_hub_rows_match_oracle(S, orc, embed):
    # sfg_sparsify knows its scoring graph's longest row, so FP64 hub rows are summed through LDS
    # (k_sweep_hub64), in the oracle's order: bit for bit
    g = _hub_graph(81)
    X0 = W.random_block(g.n, 16, 82)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, 12, 0.1, embed=embed)
    p = S.make_params(k=16, sweeps=12, frac=0.1, embed=S.EMBED_GRAPH if embed == "graph" else S.EMBED_SPARSIFIER)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), p)
    assert np.array_equal(host(keep), ref.keep)
    assert rep[0]["tau"] == ref.levels[0].tau
    # the graph embedding's rows: the hubs are over 256 entries
    Gc = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    assert embed == "sparsifier" or np.diff(Gc.rowptr).max() > 1000
