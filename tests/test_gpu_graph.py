"""A HIP graph of one scoring step (tree CSR, centring and smoothing, scores,
top-k selection) replays to the eager result: several replays, each after
other eager work and a synchronisation, every one checked bit for bit."""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,split", [(torch.float64, "2"), (torch.float64, "0"), (torch.float32, "1")])
def test_graph_replay_matches_eager(orc, dtype, split, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_07633_amd import sfg as S

    monkeypatch.setenv("SFG_SWEEP_SPLIT", split)
    dev = "cuda"
    g = W.powergrid(150, 160, 0.02, seed=81)
    k, T, f = 16, 7, 0.1
    u, v = torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev)
    w64 = torch.from_numpy(g.w).to(dev)
    w = w64.to(dtype)
    x0 = torch.from_numpy(W.random_block(g.n, k, 82)).to(dev)
    tree = torch.from_numpy(orc.max_spanning_forest(g.n, g.u, g.v, g.w)[0]).to(dev)
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    nc = int(cand.numel())
    ksel = int(math.ceil(f * nc))
    nnz = 2 * (g.n - 1)
    ws_csr = torch.empty(S.sfg_workspace_bytes(S.OP_LAPLACIAN_CSR, g.n, g.m, 0, dtype), dtype=torch.uint8, device=dev)
    ws_sm = torch.empty(S.sfg_workspace_bytes(S.OP_SMOOTH, g.n, 0, k, dtype), dtype=torch.uint8, device=dev)
    ws_sel = torch.empty(S.sfg_workspace_bytes(S.OP_SELECT_TOPK, 0, nc, 0, dtype), dtype=torch.uint8, device=dev)
    H = S.Csr(g.n, nnz, torch.empty(g.n + 1, dtype=torch.int32, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(nnz, dtype=dtype, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(g.n, dtype=dtype, device=dev))
    X = torch.empty((g.n, k), dtype=dtype, device=dev)
    score = torch.empty(nc, dtype=dtype, device=dev)
    sel = torch.empty(nc, dtype=torch.uint8, device=dev)
    tau = torch.empty(1, dtype=torch.float64, device=dev)

    def step():
        S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz)
        S.sfg_smooth(H, x0, T, 0.5, storage=dtype, out=X, ws=ws_sm)
        S.sfg_edge_scores(X, u, v, w, cand=cand, out=score)
        S.sfg_select_topk(score, ksel, sel=sel, tau=tau, ws=ws_sel, sync=False)

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (H.rowptr, H.col, H.val, H.deg, X, score, sel, tau)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    # other eager work on other buffers between the replays
    X2 = torch.empty_like(X)
    ws2 = torch.empty_like(ws_sm)
    x1 = torch.from_numpy(W.random_block(g.n, k, 83)).to(dev)
    for r in range(4):
        S.sfg_smooth(H, x1, 3 + r, 0.5, storage=dtype, out=X2, ws=ws2)
        for t in (X, score, sel, tau, H.col, H.deg):
            t.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (H.rowptr, H.col, H.val, H.deg, X, score, sel, tau)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), r
