"""Coarsening and the multilevel sparsifier (Alg. 1) against the oracle, FP64
(the aggregation argmax is taken in the oracle's precision)."""
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


GRAPHS = {
    "grid40": lambda: W.grid2d(40, 40, seed=61, wdist=("lognormal", 0.0, 1.0)),
    "rand3000": lambda: W.random_connected(3000, 9000, seed=62),
    "chunglu20k": lambda: W.chung_lu(20000, 200000, 2.2, seed=4),
    "mesh20": lambda: W.mesh3d(20, 20, 20, seed=63, wdist=("lognormal", 0.0, 1.5)),
    "unitgrid": lambda: W.grid2d(30, 31, seed=64, wdist=("unit",)),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_coarsen_matches_oracle(S, orc, name):
    g = GRAPHS[name]()
    k, T = 8, 10
    X0 = W.random_block(g.n, k, 70)
    agg_r, nc_r, cu_r, cv_r, cw_r, rep_r, aff_r = orc.coarsen_level(g.n, g.u, g.v, g.w, X0, T)
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    G = S.sfg_laplacian_csr(g.n, u, v, w)
    X = S.sfg_smooth(G, dev(X0), T, 0.5)
    aff = S.sfg_affinity(X, u, v)
    np.testing.assert_array_equal(aff.cpu().numpy(), aff_r)
    agg, nc, cu, cv, cw, crep = S.sfg_coarsen(G, u, v, w, aff)
    assert nc == nc_r
    np.testing.assert_array_equal(agg.cpu().numpy(), agg_r)
    np.testing.assert_array_equal(cu.cpu().numpy(), cu_r)
    np.testing.assert_array_equal(cv.cpu().numpy(), cv_r)
    np.testing.assert_array_equal(cw.cpu().numpy(), cw_r)
    np.testing.assert_array_equal(crep.cpu().numpy(), rep_r)


@pytest.mark.parametrize("name,levels", [("grid40", 3), ("rand3000", 4), ("chunglu20k", 5), ("mesh20", 3)])
def test_multilevel_matches_oracle(S, orc, name, levels):
    g = GRAPHS[name]()
    k, T, f = 8, 10, 0.1
    X0s = np.stack([W.random_block(g.n, k, 80 + l) for l in range(levels)])
    ref, lv = orc.sparsify_multilevel(g.n, g.u, g.v, g.w, list(X0s), levels, T, f)
    p = S.make_params(levels=levels, k=k, sweeps=T, frac=f)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0s), p)
    assert len(rep) == len(lv)
    for l, L in enumerate(lv[:-1]):
        assert rep[l]["n"] == L.n and rep[l]["m"] == L.u.shape[0]
    np.testing.assert_array_equal(keep.cpu().numpy(), ref.keep)
    # per-level additions equal the oracle's (finest level reported first)
    for lr_ref, lr in zip(ref.levels[::-1], rep):
        assert lr["n_cand"] == lr_ref.n_cand and lr["k_sel"] == lr_ref.k_sel and lr["tau"] == lr_ref.tau


@pytest.mark.parametrize("name,levels", [("chunglu20k", 5), ("mesh20", 3)])
def test_multilevel_in_tree_preorder_matches_oracle(S, orc, name, levels, monkeypatch):
    # every level's sweeps (on G_l for the affinities, on the level's sparsifier for the scores) in the preorder
    # of a spanning tree of G_l: rows keep their entry order, so the hierarchy is the oracle's bit for bit
    monkeypatch.setenv("SFG_NODE_ORDER", "1")
    g = GRAPHS[name]()
    k, T, f = 8, 10, 0.1
    X0s = np.stack([W.random_block(g.n, k, 80 + l) for l in range(levels)])
    ref, lv = orc.sparsify_multilevel(g.n, g.u, g.v, g.w, list(X0s), levels, T, f)
    p = S.make_params(levels=levels, k=k, sweeps=T, frac=f)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0s), p)
    # every swept level (the coarsest, P = G, is not swept)
    assert [r["node_order"] for r in rep[:-1]] == [1] * (len(rep) - 1)
    np.testing.assert_array_equal(keep.cpu().numpy(), ref.keep)
    for lr_ref, lr in zip(ref.levels[::-1], rep):
        assert lr["n_cand"] == lr_ref.n_cand and lr["k_sel"] == lr_ref.k_sel and lr["tau"] == lr_ref.tau


def test_multilevel_fp32_is_a_valid_sparsifier(S, orc):
    g = W.chung_lu(20000, 200000, 2.2, seed=4)
    levels, k, T, f = 5, 16, 20, 0.1
    X0s = np.stack([W.random_block(g.n, k, 90 + l) for l in range(levels)])
    p = S.make_params(levels=levels, k=k, sweeps=T, frac=f, storage=torch.float32)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w.astype(np.float32)), dev(X0s), p)
    kp = keep.cpu().numpy()
    c, _ = orc.components(g.n, g.u, g.v, kp > 0)
    assert c == 1
    assert (kp == 2).sum() == rep[0]["k_sel"]
    ns = [r["n"] for r in rep]
    assert all(a > b for a, b in zip(ns, ns[1:]))


@pytest.mark.parametrize("storage", [torch.float32, torch.float64])
def test_power_law_hierarchy_is_deterministic(S, storage):
    # the hub-row sweeps of a power-law graph's dense levels run on a side stream beside the main sweep; the
    # ordering between them (two events per iterate) must make every run give the same bits
    g = W.chung_lu(20000, 200000, 2.2, seed=4)
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    p = S.make_params(levels=5, k=16, sweeps=12, frac=0.1, storage=storage, seed=9)
    keeps, taus = [], []
    for _ in range(3):
        keep, rep = S.sfg_sparsify(g.n, u, v, w, None, p)
        keeps.append(keep.cpu().numpy())
        taus.append([r["tau"] for r in rep])
    assert all(np.array_equal(keeps[0], k) for k in keeps[1:])
    assert all(t == taus[0] for t in taus[1:])
