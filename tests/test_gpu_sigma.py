"""GPU parity of sigma-driven stopping: spanning-tree layout and solves, the
condition-number estimate and the stopping loop of sfg_sparsify, against the
CPU oracle.

Integer layouts are compared exactly.  Tree solves add in a different order
than the oracle's elimination (prefix sums against a leaf-to-root pass): they
agree to a few ulps of the solution's scale.  The estimate is compared step
by step with tight inner solves (the oracle solves exactly); at the default
loose tolerance only the bounds that hold for any subspace are checked.
"""
import math

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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def star(n):
    return W.Graph(n, np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32), np.linspace(0.5, 2.0, n - 1),
                   name=f"star{n}")


TREES = {
    "grid64": lambda: W.workload_graph("grid64"),
    "rand1500": lambda: W.random_connected(1500, 4000, seed=81, wdist=("lognormal", 0.0, 1.0)),
    "pgrid_301": lambda: W.powergrid(301, 299, 0.02, seed=82),
    "mesh_17": lambda: W.mesh3d(17, 13, 11, seed=83),
    "star3000": lambda: star(3000),
    "path2": lambda: W.grid2d(1, 2, seed=84),
}


@pytest.fixture(scope="module", params=list(TREES))
def tgraph(request):
    return TREES[request.param]()


def tree_mask(orc, g):
    return orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0


def keep_of(mask):
    return dev(mask.astype(np.uint8))


def test_tree_order_exact(S, orc, tgraph):
    g = tgraph
    print(f"tree_order {g.name} n={g.n}", flush=True)
    tm = tree_mask(orc, g)
    t = S.sfg_tree_order(g.n, dev(g.u), dev(g.v), dev(g.w), keep_of(tm))
    want = orc.tree_dfs(g.n, g.u, g.v, g.w, tm)
    for name in ("order", "parent", "size", "tdown", "tup"):
        assert np.array_equal(host(getattr(t, name)), getattr(want, name)), name
    assert np.array_equal(host(t.pw), want.pw)


def test_tree_order_of_sparsifier_marks(S, orc):
    # edges marked 2 (recovered) are ignored: only the 1s form the tree
    g = W.powergrid(60, 50, 0.05, seed=85)
    tm = tree_mask(orc, g)
    keep = tm.astype(np.uint8)
    keep[np.nonzero(~tm)[0][::3]] = 2
    t = S.sfg_tree_order(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep))
    want = orc.tree_dfs(g.n, g.u, g.v, g.w, tm)
    assert np.array_equal(host(t.order), want.order)
    assert np.array_equal(host(t.tup), want.tup)


def test_tree_order_errors(S, orc):
    g = W.grid2d(10, 10, seed=86)
    tm = tree_mask(orc, g)
    U, V, Wt = dev(g.u), dev(g.v), dev(g.w)
    short = tm.copy()
    short[np.nonzero(tm)[0][0]] = False
    with pytest.raises(S.SfgError) as e:
        S.sfg_tree_order(g.n, U, V, Wt, keep_of(short))
    assert e.value.name == "SFG_EINVAL"
    # n - 1 edges with a cycle: swap one tree edge for an off-tree edge inside one of the two halves
    _, lab = orc.components(g.n, g.u, g.v, short.astype(np.uint8))
    inside = np.nonzero(~tm & (lab[g.u] == lab[g.v]))[0]
    cyc = short.copy()
    cyc[inside[0]] = True
    assert orc.components(g.n, g.u, g.v, cyc.astype(np.uint8))[0] == 2
    with pytest.raises(S.SfgError) as e:
        S.sfg_tree_order(g.n, U, V, Wt, keep_of(cyc))
    assert e.value.name == "SFG_ENOTCONN"
    with pytest.raises(S.SfgError) as e:
        S.sfg_tree_order(g.n, U, V, dev(g.w.astype(np.float32)), keep_of(tm))
    assert e.value.name == "SFG_EINVAL"


@pytest.mark.parametrize("k", [1, 3, 8, 17, 64])   # 17 does not divide the 256-thread workgroup; 64 is the largest
def test_tree_solve_matches_oracle(S, orc, tgraph, k):
    g = tgraph
    print(f"tree_solve {g.name} k={k}", flush=True)
    tm = tree_mask(orc, g)
    t = S.sfg_tree_order(g.n, dev(g.u), dev(g.v), dev(g.w), keep_of(tm))
    B = np.random.default_rng(11).standard_normal((g.n, k))
    X = host(S.sfg_tree_solve(t, dev(B)))
    want = orc.tree_solve(orc.tree_dfs(g.n, g.u, g.v, g.w, tm), B)
    scale = np.abs(want).max()
    assert np.abs(X - want).max() <= 1e-12 * scale * max(1.0, math.log2(g.n))
    assert np.abs(X.mean(axis=0)).max() <= 1e-13 * scale * max(1.0, math.log2(g.n))


def test_tree_solve_large_residual(S, orc):
    # 1M-node power grid tree: many scan tiles; the residual L_T x - (b - mean b) is checked on the host
    g = W.workload_graph("powergrid")
    tm = tree_mask(orc, g)
    t = S.sfg_tree_order(g.n, dev(g.u), dev(g.v), dev(g.w), keep_of(tm))
    B = np.random.default_rng(12).standard_normal((g.n, 4))
    X = host(S.sfg_tree_solve(t, dev(B)))
    want = orc.tree_solve(orc.tree_dfs(g.n, g.u, g.v, g.w, tm), B)
    scale = np.abs(want).max()
    assert np.abs(X - want).max() <= 1e-12 * scale * math.log2(g.n)
    # backward error: the residual is a few ulps of |L| |x| (the oracle's own is about 6e-17 of it)
    L = orc.laplacian_sparse(g.n, g.u[tm], g.v[tm], g.w[tm])
    R = L @ X - (B - B.mean(axis=0))
    dmax = float(np.asarray(abs(L).sum(axis=1)).max())
    assert np.abs(R).max() <= 1e-15 * dmax * np.abs(X).max()
    # sampled nodes of the layout against the walk's definition: a parent edge is a tree edge
    order, parent = host(t.order), host(t.parent)
    pe = set(zip(g.u[tm].tolist(), g.v[tm].tolist()))
    for i in np.random.default_rng(13).integers(1, g.n, 2000):
        a, b = int(order[i]), int(order[parent[i]])
        assert (min(a, b), max(a, b)) in pe


def test_tree_solve_inplace(S, orc):
    g = W.random_connected(700, 900, seed=87)
    tm = tree_mask(orc, g)
    t = S.sfg_tree_order(g.n, dev(g.u), dev(g.v), dev(g.w), keep_of(tm))
    B = np.random.default_rng(14).standard_normal((g.n, 2))
    b = dev(B)
    want = host(S.sfg_tree_solve(t, b.clone()))
    S.sfg_tree_solve(t, b, out=b)
    assert np.array_equal(host(b), want)


# --------------------------------------------------------------------------- estimate

def test_kappa_one_edge_closed_form(S, orc):
    n = 400
    rng = np.random.default_rng(15)
    pairs = [(i, i + 1) for i in range(n - 1)] + [(0, n - 1)]
    u = np.array([p[0] for p in pairs], np.int32)
    v = np.array([p[1] for p in pairs], np.int32)
    o = np.lexsort((v, u))
    u, v, w = u[o], v[o], rng.uniform(0.5, 2.0, n)
    off = int(np.nonzero((u == 0) & (v == n - 1))[0][0])
    keep = np.ones(n, np.uint8)
    keep[off] = 0
    want = 1.0 + w[off] * float(np.sum(1.0 / w[keep > 0]))
    kp = S.make_kappa_params(k=4, steps=10, tol=1e-12)
    kap, rep = S.sfg_kappa_estimate(n, dev(u), dev(v), dev(w), dev(keep), kp)
    assert abs(kap - want) <= 1e-8 * want
    assert all(x <= want * (1 + 1e-10) for x in rep["ritz"])


@pytest.mark.parametrize("name,frac", [("grid64", 0.0), ("grid64", 0.05), ("rand1500", 0.1), ("pgrid_301", 0.1)])
def test_kappa_steps_match_oracle(S, orc, name, frac):
    g = TREES[name]()
    print(f"kappa {name} frac={frac}", flush=True)
    base = tree_mask(orc, g)
    keep = base.astype(np.uint8)
    if frac:
        lr, _ = orc.score_level(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 8, 5), 10, 0.5, frac)
        keep[lr.chosen] = 2
    Y0 = orc.random_block(g.n, 6, 21, 3)
    want = orc.kappa_estimate(g.n, g.u, g.v, g.w, keep > 0, Y0, 5)
    kp = S.make_kappa_params(k=6, steps=5, tol=1e-11)
    kap, rep = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep), kp, y0=dev(Y0))
    assert rep["unconverged"] == 0
    assert np.allclose(rep["ritz"], want, rtol=1e-6, atol=0)
    assert kap == rep["ritz"][-1]


@pytest.mark.parametrize("k", [5, 32])   # odd: one column per thread in the Laplacian product; 32: the largest
def test_kappa_block_widths(S, orc, k):
    g = TREES["rand1500"]()
    base = tree_mask(orc, g)
    keep = base.astype(np.uint8)
    lr, _ = orc.score_level(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 8, 5), 10, 0.5, 0.1)
    keep[lr.chosen] = 2
    Y0 = orc.random_block(g.n, k, 22, 1)
    want = orc.kappa_estimate(g.n, g.u, g.v, g.w, keep > 0, Y0, 4)
    kap, rep = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep),
                                    S.make_kappa_params(k=k, steps=4, tol=1e-11), y0=dev(Y0))
    assert rep["unconverged"] == 0
    assert np.allclose(rep["ritz"], want, rtol=1e-6, atol=0)


def test_kappa_seeded_start(S, orc):
    # y0 = NULL draws the start block on the device: the same block as random_block(seed, block), up to
    # the last bits of the device's log / sin / cos in Box-Muller
    g = TREES["rand1500"]()
    keep = tree_mask(orc, g).astype(np.uint8)
    kp = S.make_kappa_params(k=4, steps=3, tol=1e-11, seed=99, block=5)
    k1, _ = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep), kp)
    k2, _ = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep), kp,
                                 y0=dev(orc.random_block(g.n, 4, 99, 5)))
    assert abs(k1 - k2) <= 1e-9 * k2


def test_kappa_default_tolerance_bounds(S, orc):
    g = W.grid2d(30, 30, seed=88, wdist=("lognormal", 0.0, 1.0))
    base = tree_mask(orc, g)
    keep = base.astype(np.uint8)
    lr, _ = orc.score_level(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 8, 6), 10, 0.5, 0.1)
    keep[lr.chosen] = 2
    _, lmax, _ = orc.kappa_dense(g.n, g.u, g.v, g.w, keep > 0)
    kap, rep = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(g.w), dev(keep))
    assert kap <= lmax * (1 + 1e-9)
    assert kap >= 0.9 * lmax
    assert rep["inner_iters"] > 0 and rep["unconverged"] == 0


def test_kappa_f32_weights(S, orc):
    g = W.powergrid(80, 70, 0.02, seed=89)
    w32 = g.w.astype(np.float32)
    keep = tree_mask(orc, g).astype(np.uint8)
    Y0 = orc.random_block(g.n, 4, 1, 0)
    kp = S.make_kappa_params(k=4, steps=4, tol=1e-11)
    kap, _ = S.sfg_kappa_estimate(g.n, dev(g.u), dev(g.v), dev(w32), dev(keep), kp, y0=dev(Y0))
    want = orc.kappa_estimate(g.n, g.u, g.v, w32.astype(np.float64), keep > 0, Y0, 4)[-1]
    assert abs(kap - want) <= 1e-6 * want


def test_kappa_errors(S, orc):
    g = W.grid2d(8, 8, seed=90)
    U, V, Wt = dev(g.u), dev(g.v), dev(g.w)
    keep = tree_mask(orc, g).astype(np.uint8)
    for kp in (S.make_kappa_params(k=33), S.make_kappa_params(k=64), S.make_kappa_params(steps=65),
               S.make_kappa_params(tol=1.5), S.make_kappa_params(k=4, max_iter=-1)):
        with pytest.raises(S.SfgError) as e:
            S.sfg_kappa_estimate(g.n, U, V, Wt, dev(keep), kp)
        assert e.value.name == "SFG_EINVAL"
    bad = keep.copy()
    bad[np.nonzero(keep)[0][0]] = 2      # no longer n - 1 edges marked 1
    with pytest.raises(S.SfgError) as e:
        S.sfg_kappa_estimate(g.n, U, V, Wt, dev(bad))
    assert e.value.name == "SFG_EINVAL"


# --------------------------------------------------------------------------- sigma-driven sparsify

def sigma_case(S, orc, g, sigma, frac, k=8, sweeps=10, rounds=16, est_k=4, est_steps=6, omega=0.5,
               embed="sparsifier", smoother="jacobi"):
    seed = 31
    X0s = [orc.random_block(g.n, k, seed, r) for r in range(16)]
    Y0s = [orc.random_block(g.n, est_k, seed, 64 + j) for j in range(17)]
    res, kaps = orc.sparsify_sigma(g.n, g.u, g.v, g.w, X0s, Y0s, sigma, frac, rounds, sweeps, est_steps, omega,
                                   embed, smoother)
    est = S.make_kappa_params(k=est_k, steps=est_steps, tol=1e-11)
    p = S.make_params(k=k, sweeps=sweeps, frac=frac, rounds=rounds, seed=seed, sigma=sigma, est=est, omega=omega,
                      embed=S.EMBED_GRAPH if embed == "graph" else S.EMBED_SPARSIFIER,
                      smoother=S.SMOOTH_GAUSS_SEIDEL if smoother == "gs" else S.SMOOTH_JACOBI)
    info = {}
    keep, levels = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), None, p, info=info)
    return res, kaps, host(keep), levels, info


@pytest.mark.parametrize("name", ["grid64", "pgrid_301"])
def test_sigma_sparsify_matches_oracle(S, orc, name):
    g = TREES[name]()
    print(f"sigma sparsify {name}", flush=True)
    # sigma^2 between the oracle's estimates so that the stopping round is not borderline
    seed = 31
    base = tree_mask(orc, g)
    k0 = orc.kappa_estimate(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 4, seed, 64), 6)[-1]
    sigma = math.sqrt(0.2 * k0)
    res, kaps, keep, levels, info = sigma_case(S, orc, g, sigma, 0.03)
    assert len(levels) == len(res.levels) >= 1
    for a, b in zip(kaps, info["kappa"]):
        assert abs(a - b) <= 1e-6 * a
    assert all(abs(x - sigma ** 2) > 1e-4 * sigma ** 2 for x in kaps)
    assert np.array_equal(keep, res.keep)
    for lv, lr in zip(levels, res.levels):
        assert lv["k_sel"] == lr.k_sel and lv["tau"] == lr.tau


def test_sigma_tree_accepted_and_cap(S, orc):
    g = TREES["grid64"]()
    res, kaps, keep, levels, info = sigma_case(S, orc, g, 1e4, 0.05)
    assert levels == [] and len(info["kappa"]) == 1
    assert np.array_equal(keep, res.keep) and int((keep == 2).sum()) == 0
    res, kaps, keep, levels, info = sigma_case(S, orc, g, 1.0, 0.05, rounds=3)
    assert len(levels) == 3 and len(info["kappa"]) == 4
    assert np.array_equal(keep, res.keep)


def test_sigma_exhausts_candidates(S, orc):
    # batches of 40% of the off-tree edges: the third batch takes what is left, then the loop ends
    g = W.grid2d(12, 12, seed=91, wdist=("lognormal", 0.0, 1.0))
    res, kaps, keep, levels, info = sigma_case(S, orc, g, 1.0, 0.4)
    n_off = g.u.shape[0] - (g.n - 1)
    assert [lv["k_sel"] for lv in levels] == [math.ceil(0.4 * n_off)] * 2 + [n_off - 2 * math.ceil(0.4 * n_off)]
    assert int((keep == 0).sum()) == 0
    assert np.array_equal(keep, res.keep)
    # P = G: the estimate is 1
    assert abs(info["kappa"][-1] - 1.0) < 1e-9


def test_sigma_param_errors(S, orc):
    g = TREES["grid64"]()
    U, V, Wt = dev(g.u), dev(g.v), dev(g.w)
    for kw in ({"sigma": -1.0}, {"sigma": 3.0, "levels": 2}, {"sigma": 3.0, "frac": 0.0}):
        p = S.make_params(**kw)
        with pytest.raises(S.SfgError) as e:
            S.sfg_sparsify(g.n, U, V, Wt, None, p)
        assert e.value.name in ("SFG_EINVAL", "SFG_EUNSUPPORTED")
    p = S.make_params(sigma=3.0, est=S.make_kappa_params(k=40))
    with pytest.raises(S.SfgError) as e:
        S.sfg_sparsify(g.n, U, V, Wt, None, p)
    assert e.value.name == "SFG_EINVAL"


@pytest.mark.parametrize("embed,smoother,omega", [("graph", "jacobi", 0.5), ("sparsifier", "gs", 1.0)])
def test_sigma_with_other_embeddings_and_smoothers(S, orc, embed, smoother, omega):
    g = TREES["grid64"]()
    base = tree_mask(orc, g)
    k0 = orc.kappa_estimate(g.n, g.u, g.v, g.w, base, orc.random_block(g.n, 4, 31, 64), 6)[-1]
    sigma = math.sqrt(0.25 * k0)
    res, kaps, keep, levels, info = sigma_case(S, orc, g, sigma, 0.03, omega=omega, embed=embed, smoother=smoother)
    assert len(levels) == len(res.levels) >= 1
    assert all(abs(x - sigma ** 2) > 1e-4 * sigma ** 2 for x in kaps)
    assert np.array_equal(keep, res.keep)
    for a, b in zip(kaps, info["kappa"]):
        assert abs(a - b) <= 1e-6 * a


def test_sigma_degenerate_graphs(S, orc):
    # a graph that is its own spanning tree: no candidates, the estimate is exactly the identity pencil's 1
    g = W.grid2d(1, 40, seed=92)                 # a path
    keep, levels = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), None,
                                  S.make_params(k=4, sweeps=5, frac=0.1, sigma=1.5,
                                                est=S.make_kappa_params(k=3, steps=3, tol=1e-11)),
                                  info=(info := {}))
    assert levels == [] and len(info["kappa"]) == 1 and abs(info["kappa"][0] - 1.0) < 1e-12
    assert int((host(keep) == 1).sum()) == g.n - 1
    # two nodes, one edge: the estimate needs k <= n - 1 = 1
    g2 = W.grid2d(1, 2, seed=93)
    kap, _ = S.sfg_kappa_estimate(2, dev(g2.u), dev(g2.v), dev(g2.w), dev(np.ones(1, np.uint8)),
                                  S.make_kappa_params(k=1, steps=2, tol=1e-11))
    assert abs(kap - 1.0) < 1e-12
    with pytest.raises(S.SfgError) as e:
        S.sfg_kappa_estimate(2, dev(g2.u), dev(g2.v), dev(g2.w), dev(np.ones(1, np.uint8)),
                             S.make_kappa_params(k=2, steps=2))
    assert e.value.name == "SFG_EINVAL"


# --------------------------------------------------------------------------- downstream PCG (Sec. 4)

def test_pcg_matches_oracle(S, orc):
    # CG on the grounded L_G preconditioned by the sparsifier: the GPU solves L_P by tree-preconditioned CG to
    # 1e-6, the oracle by sparse LU: both are exact for an outer tolerance of 1e-3, and over some 80 iterations
    # finite-precision CG drifts by an iteration or two, so the counts agree within max(2, 5%)
    import scipy.sparse as sp

    g = W.mesh3d(14, 14, 14, seed=401, wdist=("lognormal", 0.0, 1.5))
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    seed = 5
    bfull = np.zeros(g.n)
    bfull[1:] = np.random.default_rng(seed).standard_normal(g.n - 1)
    its = []
    for f in (0.0, 0.05, 0.2):
        keep, _ = S.sfg_sparsify(g.n, u, v, w, dev(W.random_block(g.n, 16, 402)),
                                 S.make_params(k=16, sweeps=20, frac=f))
        ref = orc.pcg_iterations(g.n, g.u, g.v, g.w, host(keep) > 0, tol=1e-3, seed=seed)
        x, rep = S.sfg_pcg(g.n, u, v, w, keep, dev(bfull), tol=1e-3)
        assert rep["converged"] == 1 and rep["inner_capped"] == 0, rep
        print("f", f, "gpu", rep["iters"], "oracle", ref, "inner", rep["inner_iters"], "ms", round(rep["ms"], 1),
              flush=True)
        assert abs(rep["iters"] - ref) <= max(2, 0.05 * ref), (f, rep["iters"], ref)
        assert rep["relres"] <= 1e-3
        # the returned solution: grounded residual below the tolerance
        L = sp.coo_matrix((np.r_[-g.w, -g.w], (np.r_[g.u, g.v], np.r_[g.v, g.u])), shape=(g.n, g.n)).tocsr()
        L = L + sp.diags(-np.asarray(L.sum(axis=1)).ravel())
        xh = host(x)
        assert xh[0] == 0.0
        res = L[1:, 1:] @ xh[1:] - bfull[1:]
        assert np.linalg.norm(res) <= 1.001e-3 * np.linalg.norm(bfull[1:])
        its.append(rep["iters"])
    assert its[0] > its[1] > its[2]


def test_pcg_errors(S):
    g = W.grid2d(8, 8, seed=403)
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    keep, _ = S.sfg_sparsify(g.n, u, v, w, dev(W.random_block(g.n, 4, 404)), S.make_params(k=4, sweeps=4, frac=0.1))
    b = dev(np.ones(g.n))
    for kw in ({"tol": 0.0}, {"tol": 1.0}, {"max_iter": 0}):
        with pytest.raises(S.SfgError, match="SFG_EINVAL"):
            S.sfg_pcg(g.n, u, v, w, keep, b, **kw)
    no_tree = keep.clone()
    no_tree[no_tree == 1] = 2
    with pytest.raises(S.SfgError):
        S.sfg_pcg(g.n, u, v, w, no_tree, b)
    # the iteration cap is reported, not an error
    x, rep = S.sfg_pcg(g.n, u, v, w, keep, b, tol=1e-12, max_iter=2)
    assert rep["iters"] == 2 and rep["converged"] == 0


def test_pcg_two_nodes(S):
    # the grounded system is 1 x 1: w x_1 = b_1, solved in one iteration
    g = W.grid2d(1, 2, seed=405)
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    keep = dev(np.ones(1, np.uint8))
    x, rep = S.sfg_pcg(g.n, u, v, w, keep, dev(np.array([7.0, 3.0])), tol=1e-6)
    assert rep["iters"] == 1 and rep["converged"] == 1
    xh = host(x)
    assert xh[0] == 0.0 and abs(xh[1] - 3.0 / g.w[0]) <= 1e-14 * abs(3.0 / g.w[0])
