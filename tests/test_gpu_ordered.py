"""sfg_smooth_ordered: several sweeps per pass through LDS, in a given row
order, bit-identical to sfg_smooth (and so to the oracle's smoothing) on every
path it takes -- passes of 4, 3 or 2 sweeps, a shorter last pass, a layout
for fewer hops when a block's neighbourhood does not fit, and the plain
fallback."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def tree_and_order(S, g):
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    tree, comps = S.sfg_spanning_tree(g.n, u, v, w)
    assert comps == 1
    T = S.sfg_tree_order(g.n, u, v, w, tree)
    return u, v, w, tree, T.order


GRAPHS = {
    "mesh_17x13x11": lambda: W.mesh3d(17, 13, 11, seed=501, wdist=("lognormal", 0.0, 1.5)),
    "pgrid_150x140": lambda: W.powergrid(150, 140, 0.02, seed=502),
    "knn_20k": lambda: W.knn3d(20000, 10, seed=503),
    "path_50": lambda: W.grid2d(1, 50, seed=504),
}


@pytest.mark.parametrize("hops", ["4", "3", "2"])
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
@pytest.mark.parametrize("split", [False, True])
def test_ordered_tree_sweeps_are_bit_identical(S, name, storage, hops, split, monkeypatch):
    # sweep counts that leave every remainder of a pass (20 = 5 x 4, 7 = 4 + 3 = 2 x 3 + 1, ...); split: two
    # workgroups per block, one per 64-byte column group, where k allows
    monkeypatch.setenv("SFG_SWEEP_HOPS", hops)
    if split:
        monkeypatch.setenv("SFG_PASS_COLS", "8" if storage == torch.float64 else "16")
    g = GRAPHS[name]()
    u, v, w, tree, order = tree_and_order(S, g)
    H = S.sfg_laplacian_csr(g.n, u, v, w.to(storage), mask=tree)
    for k, sweeps in ((16, 20), (16, 7), (8, 2), (4, 3), (12, 5), (16, 6)):
        X0 = dev(W.random_block(g.n, k, 510 + k + sweeps))
        ref = S.sfg_smooth(H, X0, sweeps, 0.5, storage=storage)
        info = {}
        got = S.sfg_smooth_ordered(H, order, X0, sweeps, 0.5, storage=storage, info=info)
        assert torch.equal(got, ref), (name, k, sweeps)
        # the tree's preorder keeps every block's neighbourhood within the LDS capacity of the hops asked for
        # (the k-NN tree has nodes of higher degree: at least two hops fit there)
        if name == "knn_20k":
            assert 2 <= info["sweeps_per_pass"] <= int(hops), (name, k, sweeps)
        else:
            assert info["sweeps_per_pass"] == int(hops), (name, k, sweeps)


def two_hop_slots(n, tu, tv, order, rows=64):
    """Slots of each block's 2-hop layout (L0 = the block's rows of the order, L1 and L2 the new neighbours of
    the layer before), from the tree's edges, on the host."""
    import scipy.sparse as sp

    a = sp.coo_matrix((np.ones(2 * tu.size), (np.r_[tu, tv], np.r_[tv, tu])), shape=(n, n)).tocsr()
    ptr, ind = a.indptr, a.indices
    out = []
    for b in range(0, n, rows):
        l0 = set(order[b:b + rows].tolist())
        l1 = set()
        for p in l0:
            l1.update(ind[ptr[p]:ptr[p + 1]].tolist())
        l1 -= l0
        l2 = set()
        for p in l1:
            l2.update(ind[ptr[p]:ptr[p + 1]].tolist())
        l2 -= l0 | l1
        out.append(len(l0) + len(l1) + len(l2))
    return np.array(out)


def test_ordered_blocks_over_the_common_capacity(S):
    # FP64, 16 vectors, two hops: the common-case launch holds 123 slots a block. The blocks of this tree whose
    # 2-hop neighbourhood holds more (up to the layout's 168) stage nothing and gather their first sweep's X_t
    # from global memory in the same launch. The host checks that such blocks exist; the bits are sfg_smooth's.
    g = W.mesh3d(60, 60, 60, seed=540, wdist=("lognormal", 0.0, 1.5))
    u, v, w, tree, order = tree_and_order(S, g)
    t = tree.cpu().numpy().astype(bool)
    slots = two_hop_slots(g.n, g.u[t], g.v[t], order.cpu().numpy())
    assert (slots > 123).sum() >= 1 and (slots <= 168).all(), (int((slots > 123).sum()), int(slots.max()))
    H = S.sfg_laplacian_csr(g.n, u, v, w, mask=tree)
    for sweeps in (4, 5):
        X0 = dev(W.random_block(g.n, 16, 541 + sweeps))
        ref = S.sfg_smooth(H, X0, sweeps, 0.5)
        info = {}
        got = S.sfg_smooth_ordered(H, order, X0, sweeps, 0.5, info=info)
        assert info["sweeps_per_pass"] == 2, sweeps
        assert torch.equal(got, ref), sweeps


@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
def test_ordered_sweeps_on_a_whole_graph(S, storage):
    # the 3-D mesh itself in its tree's preorder: six neighbours per row, larger neighbourhoods; whatever
    # layout fits (or none), the bits are sfg_smooth's
    g = W.mesh3d(12, 11, 10, seed=520, wdist=("lognormal", 0.0, 1.0))
    u, v, w, tree, order = tree_and_order(S, g)
    H = S.sfg_laplacian_csr(g.n, u, v, w.to(storage))
    X0 = dev(W.random_block(g.n, 16, 521))
    ref = S.sfg_smooth(H, X0, 9, 0.5, storage=storage)
    info = {}
    got = S.sfg_smooth_ordered(H, order, X0, 9, 0.5, storage=storage, info=info)
    assert torch.equal(got, ref) and info["sweeps_per_pass"] in (1, 2, 3, 4)


def test_ordered_takes_fewer_hops_when_more_do_not_fit(S, monkeypatch):
    # the whole 2-D grid in its tree's preorder: four neighbours a row, so neighbourhoods grow fast with the
    # hops, and at some cap a block's layout exceeds its capacities.  The library then lays out for fewer hops
    # (or runs the plain sweeps): never more than the cap asked for, and the bits never change.
    g = W.grid2d(200, 200, seed=525)
    u, v, w, tree, order = tree_and_order(S, g)
    H = S.sfg_laplacian_csr(g.n, u, v, w)
    X0 = dev(W.random_block(g.n, 16, 526))
    ref = S.sfg_smooth(H, X0, 12, 0.5)
    for hops in ("4", "3", "2", "0"):
        monkeypatch.setenv("SFG_SWEEP_HOPS", hops)
        info = {}
        got = S.sfg_smooth_ordered(H, order, X0, 12, 0.5, info=info)
        assert torch.equal(got, ref), hops
        assert 1 <= info["sweeps_per_pass"] <= max(int(hops), 1), hops
    # the tree alone fits 4 hops; unset, FP64 takes 2 and FP32 3
    monkeypatch.setenv("SFG_SWEEP_HOPS", "4")
    Ht = S.sfg_laplacian_csr(g.n, u, v, w, mask=tree)
    info = {}
    assert torch.equal(S.sfg_smooth_ordered(Ht, order, X0, 12, 0.5, info=info), S.sfg_smooth(Ht, X0, 12, 0.5))
    assert info["sweeps_per_pass"] == 4
    monkeypatch.delenv("SFG_SWEEP_HOPS")
    for storage, hops in ((torch.float64, 2), (torch.float32, 3)):
        Hs = S.sfg_laplacian_csr(g.n, u, v, w.to(storage), mask=tree)
        info = {}
        got = S.sfg_smooth_ordered(Hs, order, X0, 12, 0.5, storage=storage, info=info)
        assert torch.equal(got, S.sfg_smooth(Hs, X0, 12, 0.5, storage=storage)) and info["sweeps_per_pass"] == hops


def test_ordered_falls_back_and_checks(S, orc):
    g = W.grid2d(64, 64, seed=530)
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    H = S.sfg_laplacian_csr(g.n, u, v, w)
    X0 = dev(W.random_block(g.n, 8, 531))
    ref = S.sfg_smooth(H, X0, 6, 0.5)
    # node order on the whole grid: a block of 64 nodes is one grid row, whose neighbours above and below
    # exceed even the 2-hop capacity, so the plain path runs
    info = {}
    ident = torch.arange(g.n, dtype=torch.int32, device="cuda")
    got = S.sfg_smooth_ordered(H, ident, X0, 6, 0.5, info=info)
    assert torch.equal(got, ref) and info["sweeps_per_pass"] == 1
    # and it is the oracle's smoothing
    Hc = orc.laplacian_csr(g.n, g.u, g.v, g.w)
    assert np.array_equal(got.cpu().numpy(), orc.smooth(Hc, orc.center(X0.cpu().numpy())[0], 6, 0.5))
    # shapes the passes do not take: zero and one sweep, k not a multiple of 4, and (unless SFG_SWEEP_HOPS
    # asks for them) narrow blocks with few sweeps: 4 FP32 vectors, 10 sweeps
    tree, _ = S.sfg_spanning_tree(g.n, u, v, w)
    Ht32 = S.sfg_laplacian_csr(g.n, u, v, w.float(), mask=tree)
    order = S.sfg_tree_order(g.n, u, v, w, tree).order
    X4 = dev(W.random_block(g.n, 4, 538))
    info = {}
    got = S.sfg_smooth_ordered(Ht32, order, X4, 10, 0.5, storage=torch.float32, info=info)
    assert torch.equal(got, S.sfg_smooth(Ht32, X4, 10, 0.5, storage=torch.float32)) and info["sweeps_per_pass"] == 1
    Ht = S.sfg_laplacian_csr(g.n, u, v, w, mask=tree)
    for sweeps, k in ((0, 8), (1, 8), (5, 6)):
        X0k = dev(W.random_block(g.n, k, 532 + k))
        info = {}
        got = S.sfg_smooth_ordered(Ht, order, X0k, sweeps, 0.5, info=info)
        assert torch.equal(got, S.sfg_smooth(Ht, X0k, sweeps, 0.5)) and info["sweeps_per_pass"] == 1
    # 16-bit rows over 16 columns
    X24 = dev(W.random_block(g.n, 24, 539))
    info = {}
    got = S.sfg_smooth_ordered(Ht32, order, X24, 6, 0.5, storage=torch.float16, final_f32=True, info=info)
    assert torch.equal(got, S.sfg_smooth(Ht32, X24, 6, 0.5, storage=torch.float16, final_f32=True))
    assert info["sweeps_per_pass"] == 1
    # an order that is not a permutation is refused where the passes would use it (16 FP64 vectors, 6 sweeps)
    X16 = dev(W.random_block(g.n, 16, 537))
    bad = order.clone()
    bad[5] = bad[6]
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_smooth_ordered(Ht, bad, X16, 6, 0.5)
    bad = order.clone()
    bad[0] = g.n
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_smooth_ordered(Ht, bad, X16, 6, 0.5)
    # a negative entry, and a duplicate at the two ends of the order, right after a valid call on the same graph
    bad = order.clone()
    bad[g.n // 2] = -1
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_smooth_ordered(Ht, bad, X16, 6, 0.5)
    S.sfg_smooth_ordered(Ht, order, X16, 6, 0.5)
    bad = order.clone()
    bad[g.n - 1] = bad[0]
    with pytest.raises(S.SfgError, match="SFG_EINVAL"):
        S.sfg_smooth_ordered(Ht, bad, X16, 6, 0.5)
    info = {}
    assert torch.equal(S.sfg_smooth_ordered(Ht, order, X16, 6, 0.5, info=info), S.sfg_smooth(Ht, X16, 6, 0.5))
    assert info["sweeps_per_pass"] == 2


@pytest.mark.parametrize("hops", ["4", "3", "2"])
@pytest.mark.parametrize("storage", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("final_f32", [False, True])
def test_ordered_sixteen_bit_storage_is_bit_identical(S, storage, final_f32, hops, monkeypatch):
    # FP16 / BF16 storage, FP32 weights and arithmetic; with final_f32 only the very last sweep stores FP32
    monkeypatch.setenv("SFG_SWEEP_HOPS", hops)
    g = W.mesh3d(17, 13, 11, seed=545, wdist=("lognormal", 0.0, 1.5))
    u, v, w, tree, order = tree_and_order(S, g)
    H = S.sfg_laplacian_csr(g.n, u, v, w.float(), mask=tree)
    for k, sweeps in ((4, 10), (16, 7), (8, 2), (12, 5)):
        X0 = dev(W.random_block(g.n, k, 550 + k + sweeps))
        ref = S.sfg_smooth(H, X0, sweeps, 0.5, storage=storage, final_f32=final_f32)
        info = {}
        got = S.sfg_smooth_ordered(H, order, X0, sweeps, 0.5, storage=storage, final_f32=final_f32, info=info)
        assert got.dtype == ref.dtype and torch.equal(got, ref), (k, sweeps)
        assert info["sweeps_per_pass"] == int(hops), (k, sweeps)


@pytest.mark.parametrize("storage", [torch.float32, torch.float64])
def test_ordered_hub_rows_keep_the_single_sweep_sums(S, storage, monkeypatch):
    # a star of 270 leaves on a path: in reduced precision sfg_smooth sums rows over 256 entries by lane groups,
    # so the passes must leave such a row to it (the FP64 row exceeds the local capacities instead)
    monkeypatch.setenv("SFG_SWEEP_HOPS", "2")
    n_leaf, n_path = 270, 500
    n = 1 + n_leaf + n_path
    u = list(range(1, n_leaf + 1)) + list(range(n_leaf, n - 1))
    v = [0] * n_leaf + list(range(n_leaf + 1, n))
    uu, vv = np.minimum(u, v).astype(np.int32), np.maximum(u, v).astype(np.int32)
    o = np.lexsort((vv, uu))
    rng = np.random.default_rng(560)
    w = rng.uniform(0.5, 2.0, n - 1)
    ut, vt, wt = dev(uu[o]), dev(vv[o]), dev(w)
    tree, _ = S.sfg_spanning_tree(n, ut, vt, wt)
    order = S.sfg_tree_order(n, ut, vt, wt, tree).order
    H = S.sfg_laplacian_csr(n, ut, vt, wt.to(storage))
    X0 = dev(W.random_block(n, 8, 561))
    info = {}
    got = S.sfg_smooth_ordered(H, order, X0, 6, 0.5, storage=storage, info=info)
    assert torch.equal(got, S.sfg_smooth(H, X0, 6, 0.5, storage=storage)) and info["sweeps_per_pass"] == 1


def test_ordered_matches_the_oracle_on_a_power_grid_tree(S, orc):
    g = W.powergrid(120, 110, 0.02, seed=540)
    u, v, w, tree, order = tree_and_order(S, g)
    t = tree.cpu().numpy().astype(bool)
    H = S.sfg_laplacian_csr(g.n, u, v, w, mask=tree)
    X0 = W.random_block(g.n, 16, 541)
    info = {}
    got = S.sfg_smooth_ordered(H, order, dev(X0), 20, 0.5, info=info)
    Hc = orc.laplacian_csr(g.n, g.u[t], g.v[t], g.w[t])
    assert info["sweeps_per_pass"] == 2
    assert np.array_equal(got.cpu().numpy(), orc.smooth(Hc, orc.center(X0)[0], 20, 0.5))
