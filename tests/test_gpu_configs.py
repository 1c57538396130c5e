"""Parity at the full sizes of the 3-D mesh workload (200^3: 8,000,000 nodes,
23,880,000 edges, 16 vectors, 20 sweeps, 10%) in the launch configuration the
benchmark times (two FP64 sweeps per pass in the spanning tree's preorder,
three in FP32), and of a 1M-node Chung-Lu graph through the 5-level hierarchy
of Alg. 1.  The oracle runs each whole computation on the CPU (about a minute
each); its results are shared by the tests of a module."""
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


# --------------------------------------------------------------------------- 200^3 mesh, one scoring pass

@pytest.fixture(scope="module")
def mesh(orc):
    g = W.workload_graph("mesh")
    prm = W.workload_params("mesh")
    X0 = W.workload_block("mesh", g.n)
    print(f"oracle: single-level pass on the {g.n}-node mesh", flush=True)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, prm["sweeps"], prm["frac"])
    return g, prm, X0, ref


@pytest.mark.parametrize("passes", [True, False])
def test_mesh200_full_size_f64_identical(S, orc, mesh, passes):
    """The benchmark's step (tree CSR, FP64 smoothing of the 16-vector block, scores, selection): every one of
    the 15,880,001 scores bit for bit, the selected set and the threshold.  passes: the smoothing as the
    benchmark times it, two sweeps per pass in the tree's preorder (sfg_smooth_ordered); else one sweep per
    launch in node order (--single-sweep)."""
    g, prm, X0, ref = mesh
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    tree, comps = S.sfg_spanning_tree(g.n, u, v, w)
    assert comps == 1
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    lr = ref.levels[0]
    assert np.array_equal(cand.cpu().numpy(), lr.cand)
    H = S.sfg_laplacian_csr(g.n, u, v, w, mask=tree)
    if passes:
        order = S.sfg_tree_order(g.n, u, v, w, tree).order
        info = {}
        X = S.sfg_smooth_ordered(H, order, dev(X0), prm["sweeps"], 0.5, storage=torch.float64, info=info)
        assert info["sweeps_per_pass"] == 2
    else:
        X = S.sfg_smooth(H, dev(X0), prm["sweeps"], 0.5, storage=torch.float64)
    s = S.sfg_edge_scores(X, u, v, w, cand=cand)
    assert np.array_equal(s.cpu().numpy(), lr.score)
    k = orc.ksel(prm["frac"], int(cand.numel()))
    sel, tau = S.sfg_select_topk(s, k)
    assert tau == lr.tau
    assert np.array_equal(np.sort(cand[sel.bool()].cpu().numpy()), np.sort(lr.chosen))


def test_mesh200_full_size_f32_close(S, orc, mesh):
    """The same pass in FP32 storage and arithmetic against the FP64 oracle: 20 sweeps of a few FP32 roundings
    each stay far below 1e-4 of the threshold, and the selections agree but for edges that close to it."""
    g, prm, X0, ref = mesh
    lr = ref.levels[0]
    u, v, w64 = dev(g.u), dev(g.v), dev(g.w)
    w32 = w64.float()
    tree, _ = S.sfg_spanning_tree(g.n, u, v, w64)
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    H = S.sfg_laplacian_csr(g.n, u, v, w32, mask=tree)
    # as the benchmark's FP32 pass: three sweeps per pass in the tree's preorder (the same bits as sfg_smooth)
    order = S.sfg_tree_order(g.n, u, v, w64, tree).order
    info = {}
    X = S.sfg_smooth_ordered(H, order, dev(X0), prm["sweeps"], 0.5, storage=torch.float32, info=info)
    assert info["sweeps_per_pass"] == 3
    s = S.sfg_edge_scores(X, u, v, w32, cand=cand)
    err = orc.score_errors(s.cpu().numpy().astype(np.float64), lr.score, lr.tau)
    assert err["max_abs_over_tau"] < 1e-4, err
    assert err["max_rel_selected_region"] < 1e-4, err
    k = orc.ksel(prm["frac"], int(cand.numel()))
    sel, _ = S.sfg_select_topk(s, k)
    got = set(cand[sel.bool()].cpu().numpy().tolist())
    want = set(lr.chosen.tolist())
    diff = np.array(sorted(got ^ want), dtype=np.int64)
    if diff.size:
        pos = np.searchsorted(lr.cand, diff)
        assert np.max(np.abs(lr.score[pos] - lr.tau)) <= err["max_abs_over_tau"] * lr.tau * 2


# --------------------------------------------------------------------------- 1M-node Chung-Lu, 5 levels

LEVELS, K, T, F = 5, 16, 20, 0.1


@pytest.fixture(scope="module")
def chunglu(orc):
    g = W.chung_lu(1_000_000, 10_000_000, 2.2, seed=4)
    X0s = np.stack([W.random_block(g.n, K, 500 + l) for l in range(LEVELS)])
    print(f"oracle: {LEVELS}-level hierarchy of the {g.n}-node Chung-Lu graph", flush=True)
    ref, lv = orc.sparsify_multilevel(g.n, g.u, g.v, g.w, list(X0s), LEVELS, T, F)
    return g, X0s, ref, lv


def test_chunglu_1m_hierarchy_f64_identical(S, chunglu):
    """The whole FP64 hierarchy (smoothing on every G_l, affinities, aggregation, Galerkin graphs, per-aggregate
    trees, backward mapping, scoring and selection at every level) gives the oracle's sparsifier bit for bit."""
    g, X0s, ref, lv = chunglu
    keep, rep = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0s),
                               S.make_params(levels=LEVELS, k=K, sweeps=T, frac=F))
    assert len(rep) == len(lv) == LEVELS
    for l, L in enumerate(lv[:-1]):
        assert rep[l]["n"] == L.n and rep[l]["m"] == L.u.shape[0], l
    for lr_ref, lr in zip(ref.levels[::-1], rep):
        assert (lr["n_cand"], lr["k_sel"], lr["tau"]) == (lr_ref.n_cand, lr_ref.k_sel, lr_ref.tau)
    assert np.array_equal(keep.cpu().numpy(), ref.keep)


def test_chunglu_1m_fp32_score_error_per_level(S, orc, chunglu):
    """FP32 scoring (the Chung-Lu workload's storage) on each level's graph and mapped sparsifier of the FP64
    hierarchy, against the oracle's FP64 scores of that level.  The error is bounded edge by edge by the
    arithmetic: the iteration matrix (1 - omega) I + omega D^-1 A has non-negative rows summing to 1, so it
    never amplifies earlier errors, and a sweep adds at most (L + 8) eps max|x| to an entry (L entries summed,
    the division, the damping and the FP32 rounding of the weights and degrees; L the longest row), so after T
    sweeps every entry is within delta = (T (L + 8) + 1) eps max|x0| of its FP64 value; a score
    w sum_c d_c^2 then errs by at most w sum_c e_c (2 |d_c| + e_c) + (k + 3) eps s with
    e_c = 2 delta + eps (|d_c| + 2 delta).  On the dense
    coarse levels the smoothed vectors are nearly constant, so the scores are differences of close numbers:
    the error relative to the threshold is reported per level (printed) and is largest there."""
    g, X0s, ref, lv = chunglu
    eps = 2.0 ** -24
    for i, lr in enumerate(ref.levels):            # coarse to fine: level LEVELS-2 .. 0
        l = LEVELS - 2 - i
        L = lv[l]
        base = np.ones(L.u.shape[0], dtype=np.uint8)
        base[lr.cand] = 0
        u, v = dev(L.u), dev(L.v)
        w32 = dev(L.w.astype(np.float32))
        H = S.sfg_laplacian_csr(L.n, u, v, w32, mask=dev(base))
        X = S.sfg_smooth(H, dev(X0s[l][:L.n]), T, 0.5, storage=torch.float32)
        s = S.sfg_edge_scores(X, u, v, w32, cand=dev(lr.cand.astype(np.int32))).cpu().numpy().astype(np.float64)
        # the oracle's FP64 embedding of the level, for the bound
        m = base.astype(bool)
        Hc = orc.laplacian_csr(L.n, L.u[m], L.v[m], L.w[m])
        Xc, _ = orc.center(X0s[l][:L.n])
        X64 = orc.smooth(Hc, Xc, T, 0.5)
        longest = int(np.max(np.diff(Hc.rowptr)))
        delta = (T * (longest + 8) + 1) * eps * float(np.max(np.abs(Xc)))
        d = np.abs(X64[L.u[lr.cand]] - X64[L.v[lr.cand]])
        e = 2 * delta + eps * (d + 2 * delta)
        bound = L.w[lr.cand] * np.sum(e * (2 * d + e), axis=1) + (K + 3) * eps * lr.score
        err = np.abs(s - lr.score)
        print(f"level {l}: {L.n} nodes, longest row {longest}, max |FP32 - FP64| / tau = "
              f"{np.max(err) / lr.tau:.3e}, largest error / bound = {np.max(err / bound):.3e}", flush=True)
        assert np.all(err <= bound), l
