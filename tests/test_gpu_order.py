"""GPU: sweeping in the spanning tree's preorder changes no result.

sfg_sparsify may number the nodes in the preorder of the spanning tree
before smoothing (locality of the neighbour reads).  Every row keeps its
entries in their original order, so each row's sum is formed exactly as in
the input numbering: keep masks, thresholds and band statistics must be
bit-identical to the input-numbered run and, in FP64, to the oracle.
SFG_NODE_ORDER=0 / 1 forces either numbering; unset, the library decides.
"""
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
    "knn3000": lambda: W.knn3d(3000, 8, seed=301),
    "pgrid_61": lambda: W.powergrid(61, 67, 0.02, seed=302),
    "rand2000": lambda: W.random_connected(2000, 5000, seed=303, wdist=("lognormal", 0.0, 1.0)),
    "mesh_11": lambda: W.mesh3d(11, 9, 13, seed=304),
    "star": lambda: W.Graph(300, np.zeros(299, np.int32), np.arange(1, 300, dtype=np.int32),
                            np.linspace(0.5, 2.0, 299), name="star"),
    "path2": lambda: W.grid2d(1, 2, seed=305),
}


@pytest.fixture(scope="module", params=list(GRAPHS))
def graph(request):
    return GRAPHS[request.param]()


def run(S, g, X0, p, mode, monkeypatch, info=None):
    if mode is None:
        monkeypatch.delenv("SFG_NODE_ORDER", raising=False)
    else:
        monkeypatch.setenv("SFG_NODE_ORDER", mode)
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), None if X0 is None else dev(X0), p, info=info)
    return host(keep), rep


@pytest.mark.parametrize("embed", ["sparsifier", "graph"])
def test_preorder_matches_oracle(S, orc, graph, embed, monkeypatch):
    g = graph
    k, T, f = 8, 10, 0.05
    X0 = W.random_block(g.n, k, 311)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, T, f, embed=embed)
    p = S.make_params(k=k, sweeps=T, frac=f, embed=S.EMBED_GRAPH if embed == "graph" else S.EMBED_SPARSIFIER)
    keep, rep = run(S, g, X0, p, "1", monkeypatch)
    assert rep[0]["node_order"] == 1
    # in the preorder the tree embedding's FP64 sweeps run two per pass (sfg_smooth_ordered's passes) on the
    # grid-like trees; a row beyond the layout (the star's hub) or a larger neighbourhood (the random trees) may
    # send a level to one sweep per launch; the bits are the same either way
    if embed == "sparsifier":
        want = (2,) if g.name.startswith(("powergrid", "mesh", "grid")) else (1, 2)
        assert rep[0]["sweeps_per_pass"] in want, g.name
    assert np.array_equal(keep, ref.keep)
    lr = ref.levels[0]
    assert rep[0]["n_cand"] == lr.n_cand and rep[0]["k_sel"] == lr.k_sel
    if lr.k_sel:
        assert rep[0]["tau"] == lr.tau


@pytest.mark.parametrize("name", ["knn3000", "pgrid_61"])
@pytest.mark.parametrize("storage,final_f32,band", [
    (torch.float64, False, 0.0),
    (torch.float32, False, 0.0),
    (torch.float32, False, 0.01),
    (torch.float16, True, 0.01),
    (torch.bfloat16, True, 0.04),
    (torch.float16, False, 0.0),
])
def test_preorder_changes_nothing(S, name, storage, final_f32, band, monkeypatch):
    # reduced precision too: the same sums in the same order, so the same roundings
    monkeypatch.setenv("SFG_PRECISION_PREDICT", "0")
    g = GRAPHS[name]()
    X0 = W.random_block(g.n, 16, 312)
    p = S.make_params(k=16, sweeps=12, frac=0.1, storage=storage, final_f32=final_f32, band=band)
    k0, r0 = run(S, g, X0, p, "0", monkeypatch)
    k1, r1 = run(S, g, X0, p, "1", monkeypatch)
    assert r0[0]["node_order"] == 0 and r1[0]["node_order"] == 1
    assert np.array_equal(k0, k1)
    for f in ("n_cand", "k_sel", "tau", "band", "band_above", "band_rounds", "cone_rows"):
        assert r0[0][f] == r1[0][f], f


def test_preorder_with_predicted_fallback(S, monkeypatch):
    # the predicted-cone shortcut re-enters the level on the FP64 path in the same numbering
    g = W.knn3d(4000, 10, seed=313)
    X0 = W.random_block(g.n, 16, 314)
    p = S.make_params(k=16, sweeps=20, frac=0.1, storage=torch.float16, final_f32=True, band=0.01)
    k0, r0 = run(S, g, X0, p, "0", monkeypatch)
    k1, r1 = run(S, g, X0, p, "1", monkeypatch)
    assert r0[0]["precision_fallback"] == 1 and r1[0]["precision_fallback"] == 1
    assert r1[0]["node_order"] == 1
    assert np.array_equal(k0, k1) and r0[0]["tau"] == r1[0]["tau"]


@pytest.mark.parametrize("rounds", [2, 4])
def test_preorder_rounds_match_oracle(S, orc, rounds, monkeypatch):
    # the numbering is decided once and kept for every round
    g = W.knn3d(2500, 8, seed=315)
    k, T, f = 8, 6, 0.1
    X0s = np.stack([W.random_block(g.n, k, 316 + r) for r in range(rounds)])
    ref = orc.sparsify_rounds(g.n, g.u, g.v, g.w, list(X0s), rounds, T, f)
    keep, rep = run(S, g, X0s, S.make_params(k=k, sweeps=T, frac=f, rounds=rounds), "1", monkeypatch)
    assert np.array_equal(keep, ref.keep)
    assert all(r["node_order"] == 1 for r in rep)
    for r, lr in zip(rep, ref.levels):
        assert r["k_sel"] == lr.k_sel and r["tau"] == lr.tau


def test_preorder_sigma(S, monkeypatch):
    g = W.knn3d(3000, 8, seed=317)
    p = S.make_params(k=8, sweeps=10, frac=0.05, sigma=6.0, seed=318)
    i0, i1 = {}, {}
    k0, r0 = run(S, g, None, p, "0", monkeypatch, info=i0)
    k1, r1 = run(S, g, None, p, "1", monkeypatch, info=i1)
    assert len(r0) == len(r1) >= 1
    assert all(r["node_order"] == 1 for r in r1)
    assert np.array_equal(k0, k1)
    assert i0["kappa"] == i1["kappa"]


def test_auto_choice(S, monkeypatch):
    # points in random order: most tree neighbours lie far apart, so a call with
    # enough sweep launches (8 rounds x 20 sweeps x 4 column parts) relabels; a
    # power grid in grid order is already local; a single short pass never pays
    knn = W.knn3d(70000, 10, seed=319)
    pg = W.powergrid(300, 300, 0.02, seed=320)
    X0s = W.random_block(knn.n * 8, 32, 321).reshape(8, knn.n, 32)
    cases = ((knn, X0s, dict(k=32, sweeps=20, frac=0.1, rounds=8), 1),
             (knn, X0s[0], dict(k=8, sweeps=10, frac=0.1), 0),
             (pg, W.random_block(pg.n * 8, 32, 322).reshape(8, pg.n, 32), dict(k=32, sweeps=20, frac=0.1, rounds=8),
              0))
    for g, X0, kw, want in cases:
        p = S.make_params(**kw)
        ka, ra = run(S, g, X0, p, None, monkeypatch)
        k0, r0 = run(S, g, X0, p, "0", monkeypatch)
        assert all(r["node_order"] == want for r in ra), (g.name, kw)
        assert np.array_equal(ka, k0)
        assert [r["tau"] for r in ra] == [r["tau"] for r in r0]


def test_small_graphs_and_gauss_seidel_keep_input_order(S, orc, monkeypatch):
    # auto leaves graphs under 65,536 nodes alone; the Gauss-Seidel colouring is
    # defined on the input numbering, so that smoother never relabels
    g = W.knn3d(3000, 8, seed=322)
    X0 = W.random_block(g.n, 8, 323)
    _, r = run(S, g, X0, S.make_params(k=8, sweeps=6, frac=0.1), None, monkeypatch)
    assert r[0]["node_order"] == 0
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, 6, 0.1, smoother="gs", omega=1.0)
    p = S.make_params(k=8, sweeps=6, frac=0.1, omega=1.0, smoother=S.SMOOTH_GAUSS_SEIDEL)
    keep, r = run(S, g, X0, p, "1", monkeypatch)
    assert r[0]["node_order"] == 0
    assert np.array_equal(keep, ref.keep)
