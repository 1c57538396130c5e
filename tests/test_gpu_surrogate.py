"""Learned surrogate: GPU features, forward, gradient and Adam against the CPU
FP64 reference; training; recall against the plain scorer; fallback."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import mpnn as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_07633_amd import sfg

    sfg.lib()
    return sfg


@pytest.fixture(scope="module")
def SG(S):
    from paper_2008_07633_amd import surrogate

    return surrogate


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _prep(SG, g, seed=1, sweeps=20, kc=None):
    x0c = dev(W.random_block(g.n, SG.KC if kc is None else kc, seed))
    return SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), x0c, sweeps)


@pytest.mark.parametrize("kc", [4, 16, 6])   # the two vector-load paths and the generic one
def test_features_match_oracle(S, SG, orc, kc):
    g = W.mesh3d(9, 8, 7, seed=11, wdist=("lognormal", 0.0, 1.5))
    pp = _prep(SG, g, kc=kc)
    nf, ef = SG.features(pp, None)
    tree = pp.tree.cpu().numpy().astype(bool)
    xc = pp.xc.cpu().numpy().astype(np.float64)
    cand = pp.cand.cpu().numpy()
    w32 = g.w.astype(np.float32).astype(np.float64)
    rn, re = M.raw_features(g.n, g.u, g.v, w32, tree, xc, cand)
    np.testing.assert_allclose(nf.cpu().numpy(), rn, rtol=0, atol=2e-4)
    np.testing.assert_allclose(ef.cpu().numpy(), re, rtol=0, atol=2e-4)


def _random_case(SG, seed=3):
    g = W.mesh3d(8, 9, 10, seed=12, wdist=("lognormal", 0.0, 1.0))
    pp = _prep(SG, g, seed)
    nf_raw, ef_raw = SG.features(pp, None)
    rn, re = nf_raw.cpu().numpy().astype(np.float64), ef_raw.cpu().numpy().astype(np.float64)
    norm = np.concatenate([rn.mean(0), 1 / (rn.std(0) + 1e-3), re.mean(0), 1 / (re.std(0) + 1e-3)])
    norm[0], norm[8] = 0.0, 1.0
    norm = norm.astype(np.float32)
    nf, ef = SG.features(pp, dev(norm))
    theta = (M.init_params(seed) + 0.02).astype(np.float32)
    y = np.random.default_rng(seed).standard_normal(pp.cand.numel()).astype(np.float32)
    return g, pp, nf, ef, theta, y


def test_forward_and_gradient_match_oracle(S, SG):
    g, pp, nf, ef, theta, y = _random_case(SG)
    A, d = M.norm_adjacency(g.n, g.u, g.v, g.w.astype(np.float32).astype(np.float64))
    X = nf.cpu().numpy().astype(np.float64)
    E = ef.cpu().numpy().astype(np.float64)
    cand = pp.cand.cpu().numpy()
    th64 = theta.astype(np.float64)
    yhat_ref, cache = M.forward(th64, A, d, X, g.u, g.v, cand, E)
    grad_ref = M.backward(th64, A, d, X, y.astype(np.float64), yhat_ref, cache)
    pred, loss, grad = S.sfg_mpnn_loss_grad(pp.G, dev(theta), nf, pp.u, pp.v, ef, dev(y), cand=pp.cand)
    pred, grad = pred.cpu().numpy(), grad.cpu().numpy()
    scale = np.max(np.abs(yhat_ref))
    assert np.max(np.abs(pred - yhat_ref)) < 2e-5 * scale
    assert abs(loss.item() - M.loss(yhat_ref, y)) < 1e-4 * M.loss(yhat_ref, y)
    # per block of parameters, relative to that block's largest gradient
    o = 0
    for name, shape in M.LAYOUT:
        c = int(np.prod(shape))
        gr, gg = grad_ref[o:o + c], grad[o:o + c]
        assert np.max(np.abs(gg - gr)) <= 1e-4 * max(np.max(np.abs(gr)), 1e-12), name
        o += c
    # BF16 activations (inference): close to the FP64 reference
    pb = S.sfg_mpnn_forward(pp.G, dev(theta), nf, pp.u, pp.v, ef, cand=pp.cand, act=torch.bfloat16).cpu().numpy()
    assert np.max(np.abs(pb - yhat_ref)) < 3e-2 * scale
    pf = S.sfg_mpnn_forward(pp.G, dev(theta), nf, pp.u, pp.v, ef, cand=pp.cand, act=torch.float32).cpu().numpy()
    assert np.max(np.abs(pf - yhat_ref)) < 2e-5 * scale


def test_training_is_deterministic(S, SG):
    g, pp, nf, ef, theta, y = _random_case(SG, 4)
    a = S.sfg_mpnn_loss_grad(pp.G, dev(theta), nf, pp.u, pp.v, ef, dev(y), cand=pp.cand)[2]
    b = S.sfg_mpnn_loss_grad(pp.G, dev(theta), nf, pp.u, pp.v, ef, dev(y), cand=pp.cand)[2]
    assert torch.equal(a, b)


def test_adam_matches_oracle(S):
    rng = np.random.default_rng(0)
    th = rng.standard_normal(4865)
    m = np.zeros(4865)
    v = np.zeros(4865)
    tg, mg, vg = dev(th.astype(np.float32)), torch.zeros(4865, device="cuda"), torch.zeros(4865, device="cuda")
    for step in range(1, 6):
        gr = rng.standard_normal(4865)
        th, m, v = M.adam_step(th, gr, m, v, step, lr=1e-2)
        S.sfg_mpnn_adam(tg, dev(gr.astype(np.float32)), mg, vg, step, lr=1e-2)
    np.testing.assert_allclose(tg.cpu().numpy(), th, rtol=0, atol=1e-5)


def _mesh_case(S, SG, seed, side, kc=None):
    g = W.mesh3d(side, side, side, seed=seed, wdist=("lognormal", 0.0, 1.5))
    X0 = W.random_block(g.n, 16, 500 + seed)
    pp = SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0[:, :(SG.KC if kc is None else kc)]))
    pp.raw_nf, pp.raw_ef = SG.features(pp, None)
    return g, X0, pp, SG.plain_scores(pp, dev(X0), 20)


def _train_small(S, SG, n_train=10, side=20, epochs=30, kc=None):
    cases = [_mesh_case(S, SG, 300 + i, side, kc) for i in range(n_train)]
    ts = SG.TrainSet([c[2] for c in cases], [torch.log(c[3] + 1e-30) for c in cases])
    return SG.train(ts, epochs=epochs)


def test_training_learns_and_beats_the_cheap_score(S, SG):
    model, hist = _train_small(S, SG)
    assert hist[-1] < 0.1 * hist[0]
    # held-out mesh: recall of the plain method's top 10% inside the top candidates
    g, X0, pp, s = _mesh_case(S, SG, 350, 20)
    nc = int(pp.cand.numel())
    chosen = torch.nonzero(S.sfg_select_topk(s, int(np.ceil(0.1 * nc)))[0]).reshape(-1)
    pred = SG.predict(model, pp)
    # the method without the network: rank by the cheap embedding's own score
    cheap = S.sfg_edge_scores(pp.xc, pp.u, pp.v, pp.w32, cand=pp.cand, score_dtype=torch.float32)
    rec = {}
    for cf in (0.2, 0.5):
        kk = int(np.ceil(cf * nc))
        rec[("net", cf)] = SG.recall(chosen, torch.nonzero(S.sfg_select_topk(pred, kk)[0]).reshape(-1), nc)
        rec[("cheap", cf)] = SG.recall(chosen, torch.nonzero(S.sfg_select_topk(cheap, kk)[0]).reshape(-1), nc)
    assert rec[("net", 0.2)] > rec[("cheap", 0.2)] + 0.03, rec
    assert rec[("net", 0.5)] >= 0.98, rec
    # the pruned pipeline scores only the candidates and keeps the tree
    res = SG.sparsify_pruned(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), model, 20, 0.1, 0.5)
    assert not res.fallback and res.n_scored == int(np.ceil(0.5 * nc))
    kp = res.keep.cpu().numpy()
    assert (kp == 1).sum() == g.n - 1 and (kp == 2).sum() == res.k_sel


def test_recall_configuration(S, SG):
    # all 16 of the method's vectors in the cheap embedding: the candidates hold the plain selection
    model, hist = _train_small(S, SG, kc=SG.KC_RECALL)
    assert model.kc == SG.KC_RECALL and model.tc == SG.TC
    g, X0, pp, s = _mesh_case(S, SG, 351, 20, kc=SG.KC_RECALL)
    nc = int(pp.cand.numel())
    chosen = torch.nonzero(S.sfg_select_topk(s, int(np.ceil(0.1 * nc)))[0]).reshape(-1)
    pred = SG.predict(model, pp)
    rec = {cf: SG.recall(chosen, torch.nonzero(S.sfg_select_topk(pred, int(np.ceil(cf * nc)))[0]).reshape(-1), nc)
           for cf in (0.2, 0.3)}
    assert rec[0.2] >= 0.97 and rec[0.3] >= 0.99, rec
    # the pruned path takes the model's cheap embedding from the block
    res = SG.sparsify_pruned(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), model, 20, 0.1, 0.3)
    assert not res.fallback and res.n_scored == int(np.ceil(0.3 * nc))


def _fnv1a64(b: bytes) -> int:
    h = 0xcbf29ce484222325
    for x in b:
        h = ((h ^ x) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def _reseal(raw: bytes) -> bytes:
    """A model file with its hash recomputed (to reach the checks after the hash)."""
    import struct

    return raw[:-8] + struct.pack("<Q", _fnv1a64(raw[:-8]))


def test_model_file_roundtrip_and_fallback(S, SG, tmp_path):
    import struct

    model = SG.Model(SG.init_params(1), torch.linspace(0.5, 2.0, 24, device="cuda"), 0.25, 1.5, kc=16, tc=6)
    p = str(tmp_path / "m.sfgm")
    model.save(p)
    m2 = SG.load(p)
    assert torch.equal(m2.params, model.params) and torch.equal(m2.norm, model.norm)
    assert (m2.kc, m2.tc, m2.y_mean, m2.y_std) == (16, 6, 0.25, 1.5)
    raw = open(p, "rb").read()
    npar = S.sfg_mpnn_param_count()
    assert raw[:8] == b"SFGMPNN1" and len(raw) == 48 + 4 * (npar + 24) + 8
    assert struct.unpack_from("<IIIii", raw, 8) == (1, npar, 24, 16, 6)
    assert struct.unpack_from("<Q", raw, len(raw) - 8)[0] == _fnv1a64(raw[:-8])

    def write(name, b):
        q = str(tmp_path / name)
        open(q, "wb").write(b)
        return q

    def patched(off, fmt, *vals):
        b = bytearray(raw)
        struct.pack_into(fmt, b, off, *vals)
        return bytes(b)

    # the cheap embedding is covered by the hash, and must be sane
    with pytest.raises(SG.SurrogateInvalid, match="checksum"):
        SG.load(write("kc.sfgm", patched(20, "<i", 4)))
    with pytest.raises(SG.SurrogateInvalid, match="cheap embedding"):
        SG.load(write("kc0.sfgm", _reseal(patched(20, "<i", 0))))
    with pytest.raises(SG.SurrogateInvalid, match="version"):
        SG.load(write("v2.sfgm", _reseal(patched(8, "<I", 2))))
    with pytest.raises(SG.SurrogateInvalid, match="shapes"):
        SG.load(write("shape.sfgm", _reseal(patched(12, "<I", npar - 1))))
    with pytest.raises(SG.SurrogateInvalid, match="length"):
        SG.load(write("short.sfgm", _reseal(raw[:-12] + raw[-8:])))
    with pytest.raises(SG.SurrogateInvalid, match="not a surrogate model"):
        SG.load(write("magic.sfgm", b"NOTMODEL" + raw[8:]))
    # corrupted parameters: hash mismatch; a NaN with a valid hash: refused as non-finite
    with pytest.raises(SG.SurrogateInvalid, match="checksum"):
        SG.load(write("bad.sfgm", patched(48 + 4 * 5, "<f", 123.0)))
    nan_path = write("nan.sfgm", _reseal(patched(48 + 4 * 5, "<f", float("nan"))))
    with pytest.raises(SG.SurrogateInvalid, match="non-finite"):
        SG.load(nan_path)
    with pytest.raises(SG.SurrogateInvalid, match="cannot open"):
        SG.load(str(tmp_path / "missing.sfgm"))
    # a failed load leaves the caller's buffers alone
    params = torch.full((npar,), 7.0, device="cuda")
    norm = torch.full((24,), 7.0, device="cuda")
    meta = S.MpnnMeta()
    import ctypes

    st = S.lib().sfg_mpnn_load(nan_path.encode(), ctypes.c_void_p(params.data_ptr()),
                               ctypes.c_void_p(norm.data_ptr()), ctypes.byref(meta), S._stream())
    assert st == 1 and bool((params == 7.0).all()) and bool((norm == 7.0).all())
    # the pruned path falls back to the plain scorer on a bad model
    g = W.mesh3d(10, 10, 10, seed=360)
    X0 = W.random_block(g.n, 16, 1)
    res = SG.sparsify_pruned(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), nan_path, 20, 0.1, 0.2)
    assert res.fallback and "non-finite" in res.reason
    keep, _ = S.sfg_sparsify(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0), S.make_params(k=16, sweeps=20, frac=0.1,
                                                                                       storage=torch.float32))
    assert torch.equal(res.keep, keep)


def test_sparsify_with_surrogate_in_the_library(S, SG):
    # sfg_sparsify with sfg_params.surrogate runs the pruned path in the library: the same keep mask as the
    # Python composition of the primitives (surrogate.sparsify_pruned), for both models
    for kc in (SG.KC, SG.KC_RECALL):
        model, _ = _train_small(S, SG, n_train=6, side=16, epochs=10, kc=kc)
        for side, seed in ((18, 371), (23, 372)):
            g = W.mesh3d(side, side, side, seed=seed, wdist=("lognormal", 0.0, 1.5))
            X0 = dev(W.random_block(g.n, 16, seed))
            u, v, w = dev(g.u), dev(g.v), dev(g.w)
            ref = SG.sparsify_pruned(g.n, u, v, w, X0, model, 20, 0.1, 0.2)
            p = S.make_params(k=16, sweeps=20, frac=0.1, storage=torch.float32, surrogate=model, cand_frac=0.2)
            keep, rep = S.sfg_sparsify(g.n, u, v, w, X0, p)
            assert not ref.fallback and rep[0]["surrogate_fallback"] == 0
            assert torch.equal(keep, ref.keep), (kc, side)
            assert rep[0]["n_scored"] == ref.n_scored and rep[0]["k_sel"] == ref.k_sel
            assert rep[0]["n_cand"] == ref.n_cand


@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
def test_surrogate_scoring_everything_is_the_plain_path(S, SG, storage):
    # cand_frac = 1: every off-tree edge is scored exactly, so the result is the plain sparsifier's
    model = SG.Model(SG.init_params(3), torch.ones(24, device="cuda"), 0.0, 1.0, kc=4, tc=5)
    g = W.mesh3d(14, 15, 16, seed=373, wdist=("lognormal", 0.0, 1.5))
    X0 = dev(W.random_block(g.n, 8, 374))
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    plain, r0 = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=8, sweeps=12, frac=0.1, storage=storage))
    keep, r1 = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=8, sweeps=12, frac=0.1, storage=storage,
                                                              surrogate=model, cand_frac=1.0))
    assert torch.equal(keep, plain)
    assert r1[0]["tau"] == r0[0]["tau"] and r1[0]["n_scored"] == r0[0]["n_cand"] == r0[0]["n_scored"]


def test_surrogate_in_the_library_falls_back_and_checks(S, SG):
    g = W.mesh3d(10, 11, 12, seed=375)
    X0 = dev(W.random_block(g.n, 8, 376))
    u, v, w = dev(g.u), dev(g.v), dev(g.w)
    params = SG.init_params(4)
    params[7] = float("nan")
    bad = SG.Model(params, torch.ones(24, device="cuda"), 0.0, 1.0, kc=4, tc=5)
    plain, _ = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=8, sweeps=6, frac=0.1, storage=torch.float32))
    keep, rep = S.sfg_sparsify(g.n, u, v, w, X0, S.make_params(k=8, sweeps=6, frac=0.1, storage=torch.float32,
                                                               surrogate=bad))
    assert rep[0]["surrogate_fallback"] == 1 and torch.equal(keep, plain)
    good = SG.Model(SG.init_params(4), torch.ones(24, device="cuda"), 0.0, 1.0, kc=4, tc=5)
    for kw, status in (({"levels": 2}, "SFG_EUNSUPPORTED"), ({"band": 0.01, "storage": torch.float16},
                                                              "SFG_EUNSUPPORTED"),
                       ({"rounds": 2}, "SFG_EUNSUPPORTED"), ({"cand_frac": 0.0}, "SFG_EINVAL"),
                       ({"cand_frac": 1.5}, "SFG_EINVAL"), ({"k": 2}, "SFG_EINVAL")):
        args = dict(k=8, sweeps=6, frac=0.1, storage=torch.float32, surrogate=good)
        args.update(kw)
        x = X0 if args["k"] == 8 else X0[:, :args["k"]].contiguous()
        # room for every block the parameters name, so the library itself rejects them
        x = torch.cat([x.reshape(-1)] * 2)
        with pytest.raises(S.SfgError, match=status):
            S.sfg_sparsify(g.n, u, v, w, x, S.make_params(**args))


def test_standardisation_in_the_library_matches_fp64(S, SG):
    """sfg_mpnn_fit_norm and sfg_mpnn_standardize against the same statistics taken in FP64 by NumPy over
    the concatenated training arrays (population deviation, floor 1e-6, node feature 0 kept as 1)."""
    graphs, targets = [], []
    for i in range(3):
        g = W.mesh3d(9 + i, 10, 11, seed=390 + i)
        pp = SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), dev(W.random_block(g.n, 4, 391 + i)), 5)
        pp.raw_nf, pp.raw_ef = SG.features(pp, None)
        graphs.append(pp)
        targets.append(torch.log(SG.plain_scores(pp, dev(W.random_block(g.n, 8, 392 + i)), 6) + 1e-30))
    norm, ystat = SG.fit_norm(SG.TrainSet(graphs, targets))
    nf = np.concatenate([p.raw_nf.cpu().numpy() for p in graphs]).astype(np.float64)
    ef = np.concatenate([p.raw_ef.cpu().numpy() for p in graphs]).astype(np.float64)
    y = np.concatenate([t.cpu().numpy() for t in targets]).astype(np.float64)
    nm, ns, em, es = nf.mean(0), nf.std(0), ef.mean(0), ef.std(0)
    nm[0], ns[0] = 0.0, 1.0
    want = np.concatenate([nm, 1 / np.maximum(ns, 1e-6), em, 1 / np.maximum(es, 1e-6)])
    got = norm.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-6)
    ys = ystat.cpu().numpy()
    assert abs(ys[0] - y.mean()) <= 1e-12 * max(1.0, abs(y.mean())) and abs(ys[1] - y.std()) <= 1e-10 * y.std()
    z = S.sfg_mpnn_standardize(targets[1].contiguous(), ystat).cpu().numpy()
    zr = ((targets[1].cpu().numpy().astype(np.float64) - ys[0]) / ys[1]).astype(np.float32)
    assert np.array_equal(z, zr)
    # deterministic: the same statistics twice
    norm2, ystat2 = SG.fit_norm(SG.TrainSet(graphs, targets))
    assert torch.equal(norm, norm2) and torch.equal(ystat, ystat2)


def test_pruned_candidates_match_an_oracle_composition(S, SG, orc):
    """The pruned path's candidate set (the top 20% of the off-tree edges by prediction) against the same
    composition in FP64 on the CPU: the oracle's spanning tree, its FP64 cheap embedding (the first 4 vectors
    centred and smoothed 10 times on the tree), the reference features and forward pass, and its top 20%.  The
    library smooths the cheap embedding in BF16 and infers with BF16 activations, so the sets may differ, but
    only by edges whose FP64 prediction lies within the measured prediction error of the cut."""
    import math

    g = W.mesh3d(24, 22, 20, seed=395, wdist=("lognormal", 0.0, 1.5))
    kc, tc, cf = 4, 10, 0.2
    X0 = W.random_block(g.n, 16, 396)
    # oracle composition, FP64 (the surrogate works on the FP32 weights)
    intree, comps = orc.max_spanning_forest(g.n, g.u, g.v, g.w)
    assert comps == 1
    t = intree.astype(bool)
    w32 = g.w.astype(np.float32).astype(np.float64)
    Hc = orc.laplacian_csr(g.n, g.u[t], g.v[t], w32[t])
    xc = orc.smooth(Hc, orc.center(X0[:, :kc])[0], tc)
    cand = np.nonzero(~t)[0].astype(np.int32)
    rn, re = M.raw_features(g.n, g.u, g.v, w32, t, xc, cand)
    norm = np.concatenate([rn.mean(0), 1 / np.maximum(rn.std(0), 1e-6), re.mean(0), 1 / np.maximum(re.std(0), 1e-6)])
    norm[0], norm[8] = 0.0, 1.0
    norm32 = norm.astype(np.float32)
    nf, ef = M.standardise(rn, re, norm32.astype(np.float64))
    theta32 = (M.init_params(5) * 0.5 + 0.01).astype(np.float32)
    A, d = M.norm_adjacency(g.n, g.u, g.v, w32)
    pred_ref, _ = M.forward(theta32.astype(np.float64), A, d, nf, g.u, g.v, cand, ef)
    kcand = int(math.ceil(cf * cand.size))
    pos_ref, cut = orc.select_topk(pred_ref, cand, kcand)
    # the library's composition
    model = SG.Model(dev(theta32), dev(norm32), 0.0, 1.0, kc=kc, tc=tc)
    pp = SG.prepare(g.n, dev(g.u), dev(g.v), dev(g.w), dev(X0[:, :kc]), tc)
    assert np.array_equal(pp.cand.cpu().numpy(), cand)
    cpos, pred = SG.prune(model, pp, cf)
    pred = pred.cpu().numpy().astype(np.float64)
    delta = float(np.max(np.abs(pred - pred_ref)))
    scale = float(np.max(np.abs(pred_ref)))
    assert delta < 0.05 * scale, (delta, scale)
    got, want = set(cpos.cpu().numpy().tolist()), set(pos_ref.tolist())
    diff = np.array(sorted(got ^ want), dtype=np.int64)
    assert diff.size <= 0.02 * kcand, (diff.size, kcand)
    if diff.size:
        assert np.max(np.abs(pred_ref[diff] - cut)) <= 2 * delta
