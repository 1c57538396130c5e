"""Full-size checks of the extra workloads against the oracle.

* 2M-point kNN graph (32 vectors, 20 sweeps, 10%): reduced-precision scores
  against the FP64 oracle (three error measures), and the selected set after
  FP64 re-scoring of the 1% band identical to the oracle's.
* Surrogate on 3-D meshes: the condition numbers reached by the pruned and
  the ranked sparsifiers against the plain one (the oracle's kappa estimator).
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


def test_knn_full_size_precision(S, orc, monkeypatch):
    g = W.workload_graph("knn")
    prm = W.workload_params("knn")
    k, T, f, band = prm["k"], prm["sweeps"], prm["frac"], prm["band"]
    X0 = W.workload_block("knn", g.n)
    ref = orc.sparsify_single(g.n, g.u, g.v, g.w, X0, T, f)
    lr = ref.levels[0]
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    x0 = dev(X0)
    tree = dev((ref.keep == 1).astype(np.uint8))
    H = S.sfg_laplacian_csr(g.n, u, v, w.float(), mask=tree)
    cand = dev(lr.cand)
    errs = {}
    for name, storage, ff in (("f16+f32last", torch.float16, True), ("f16", torch.float16, False),
                              ("bf16+f32last", torch.bfloat16, True), ("f32", torch.float32, False)):
        X = S.sfg_smooth(H, x0, T, 0.5, storage=storage, final_f32=ff)
        s = S.sfg_edge_scores(X, u, v, w.float(), cand=cand).cpu().numpy().astype(np.float64)
        errs[name] = orc.score_errors(s, lr.score, lr.tau)
    print("score errors vs FP64 oracle:", errs, flush=True)
    assert errs["f16+f32last"]["max_rel_selected_region"] <= 1e-2
    assert errs["f32"]["max_abs_over_tau"] <= 1e-4
    # default calls: 20 hops of the tree reach most of the graph, so the predicted cone sends the level to the
    # FP64 path (precision_fallback): the selection is the FP64 oracle's whatever the storage
    for name, storage, ff in (("f16+f32last", torch.float16, True), ("bf16+f32last", torch.bfloat16, True)):
        p = S.make_params(k=k, sweeps=T, frac=f, storage=storage, final_f32=ff, band=band)
        keep, rep = S.sfg_sparsify(g.n, u, v, w, x0, p)
        assert rep[0]["precision_fallback"] == 1 and rep[0]["cone_rows"] == T * g.n
        assert np.array_equal(keep.cpu().numpy(), ref.keep), name
    # the band path itself (prediction off): reduced-precision scores, FP64 re-scoring of the band
    monkeypatch.setenv("SFG_PRECISION_PREDICT", "0")
    for name, storage, ff, m in (("f16+f32last", torch.float16, True, band),
                                 ("bf16+f32last", torch.bfloat16, True, band),
                                 ("bf16+f32last", torch.bfloat16, True, 0.04)):
        p = S.make_params(k=k, sweeps=T, frac=f, storage=storage, final_f32=ff, band=m)
        keep, rep = S.sfg_sparsify(g.n, u, v, w, x0, p)
        got = keep.cpu().numpy()
        diff = np.nonzero(got != ref.keep)[0]
        print(name, "band", m, "edges re-scored", rep[0]["band"], "doublings", rep[0]["band_rounds"],
              "differing edges", diff.size, flush=True)
        assert rep[0]["precision_fallback"] == 0 and rep[0]["band"] > 0
        # a score and the reduced-precision threshold each err by at most e = max|s~ - s| / tau (times tau), so
        # a margin m >= 2e (relative to the threshold, itself within e of tau) holds every edge that belongs to
        # the FP64 set: then the set is exactly the FP64 one
        e = errs[name]["max_abs_over_tau"]
        if m * (1 - e) >= 2 * e:
            assert diff.size == 0, (name, m)
        else:
            # BF16 at the workload's 1% band: its error (about 3% of tau) exceeds the margin, so edges whose
            # FP64 score lies within that error of the threshold can land on the wrong side, and only those
            pos = np.searchsorted(lr.cand, diff)
            assert np.all(lr.cand[pos] == diff)
            assert np.all(np.abs(lr.score[pos] - lr.tau) <= 2 * e * lr.tau), (name, m)
            assert diff.size <= 1e-4 * lr.k_sel


def test_surrogate_condition_number(S, orc):
    """The surrogate trained as the mesh benchmark trains it (50 seeded 40^3
    meshes, 60 epochs), on 5 held-out 24^3 meshes: the pruned path (exact
    scores of the top 20%) keeps the plain path's condition number, and the
    ranked path (surrogate order alone, 15% of the off-tree edges) reaches at
    least the plain default's median condition number; so does the 16-vector
    model ranked at 20%."""
    from paper_2008_07633_amd import surrogate as SG
    from kappa_pool import kappa_many

    graphs, targets = [], []
    for i in range(50):
        g = W.mesh3d(40, 40, 40, seed=100 + i, wdist=("lognormal", 0.0, 1.5))
        X0 = W.random_block(g.n, 16, 2000 + i)
        pp = SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0[:, :SG.KC]))
        pp.raw_nf, pp.raw_ef = SG.features(pp, None)
        graphs.append(pp)
        targets.append(torch.log(SG.plain_scores(pp, dev(X0), 20) + 1e-30))
    model, hist = SG.train(SG.TrainSet(graphs, targets), epochs=60)
    del graphs, targets
    # the recall configuration: all 16 vectors in the cheap embedding
    graphs, targets = [], []
    for i in range(50):
        g = W.mesh3d(40, 40, 40, seed=100 + i, wdist=("lognormal", 0.0, 1.5))
        X0 = W.random_block(g.n, 16, 2000 + i)
        pp = SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0[:, :SG.KC_RECALL]))
        pp.raw_nf, pp.raw_ef = SG.features(pp, None)
        graphs.append(pp)
        targets.append(torch.log(SG.plain_scores(pp, dev(X0), 20) + 1e-30))
    model16, _ = SG.train(SG.TrainSet(graphs, targets), epochs=60)
    del graphs, targets
    side, jobs = 24, []
    for i in range(5):
        g = W.mesh3d(side, side, side, seed=200 + i, wdist=("lognormal", 0.0, 1.5))
        X0 = dev(W.random_block(g.n, 16, 7000 + i))
        u, v, w = dev(g.u), dev(g.v), dev(g.w)
        plain, _ = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=16, sweeps=20, frac=0.1, storage=torch.float32))
        pruned = SG.sparsify_pruned(g.n, u, v, w, X0, model, 20, 0.1, 0.2)
        ranked = SG.sparsify_ranked(g.n, u, v, w, X0, model, 20, 0.15)
        ranked16 = SG.sparsify_ranked(g.n, u, v, w, X0, model16, 20, 0.2)
        assert not pruned.fallback and not ranked.fallback and not ranked16.fallback
        for keep in (plain, pruned.keep, ranked.keep, ranked16.keep):
            jobs.append((side, 200 + i, keep.cpu().numpy() > 0))
        jobs.append((side, 200 + i, plain.cpu().numpy() == 1))
    k = np.array(kappa_many(jobs)).reshape(5, 5)
    print("kappa plain / pruned / ranked(15%) / ranked 16-vector model (20%) / tree:", k.round(2).tolist(),
          flush=True)
    med = np.median(k, axis=0)
    assert np.all(k[:, 2] < k[:, 4] / 5)       # far better than the tree alone
    assert med[1] <= 1.25 * med[0]            # pruning keeps the plain condition number
    assert med[2] <= med[0]                   # ranking reaches the plain default's median
    assert med[3] <= med[0]                   # so does the recall configuration at 20%


def test_pcg_iterations_fall_with_recovered_edges(S, orc):
    """Downstream use (the paper's PCG evaluation): CG on the grounded Laplacian
    of a 30^3 log-normal mesh, preconditioned by the FP32 GPU sparsifier."""
    g = W.mesh3d(30, 30, 30, seed=300, wdist=("lognormal", 0.0, 1.5))
    X0 = dev(W.random_block(g.n, 16, 301))
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    plain = orc.pcg_iterations(g.n, g.u, g.v, g.w, None)
    its = []
    for f in (0.0, 0.02, 0.05, 0.1, 0.2):
        keep, _ = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=16, sweeps=20, frac=f, storage=torch.float32))
        its.append(orc.pcg_iterations(g.n, g.u, g.v, g.w, keep.cpu().numpy() > 0))
    print("PCG iterations: plain", plain, "tree / 2% / 5% / 10% / 20%:", its, flush=True)
    assert its[0] < plain / 3
    assert all(b < a for a, b in zip(its, its[1:]))
    assert its[3] < its[0] / 8
