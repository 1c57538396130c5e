"""The Python binding checks every tensor against what the C ABI assumes of it
(element type, contiguity, element count, device) before it calls the library,
so a wrong tensor raises ValueError instead of letting a kernel read or write
past the end of a buffer.  CPU only: the library is replaced by a stub that
fails the test if it is reached."""
import pytest
import torch

from paper_2008_07633_amd import sfg as S


@pytest.fixture(autouse=True)
def no_library(monkeypatch):
    def reached():
        raise AssertionError("the library was called before the arguments were checked")

    monkeypatch.setattr(S, "lib", reached)


def _csr(n, nnz, vt=torch.float64):
    return S.Csr(n, nnz, torch.zeros(n + 1, dtype=torch.int32), torch.zeros(nnz, dtype=torch.int32),
                 torch.zeros(nnz, dtype=vt), torch.zeros(nnz, dtype=torch.int32), torch.zeros(n, dtype=vt))


def _edges(m):
    u = torch.arange(m, dtype=torch.int32)
    return u, u + 1, torch.ones(m, dtype=torch.float64)


def test_smooth_checks_the_block():
    H = _csr(10, 18)
    ws = torch.zeros(256, dtype=torch.uint8)
    with pytest.raises(ValueError, match="x0: dtype torch.float32"):
        S.sfg_smooth(H, torch.zeros(10, 4, dtype=torch.float32), 3, ws=ws)
    with pytest.raises(ValueError, match="x0: has 9 rows"):
        S.sfg_smooth(H, torch.zeros(9, 4, dtype=torch.float64), 3, ws=ws)
    with pytest.raises(ValueError, match="x0: must be contiguous"):
        S.sfg_smooth(H, torch.zeros(10, 8, dtype=torch.float64)[:, ::2], 3, ws=ws)
    with pytest.raises(ValueError, match="out: holds 20 elements, the call needs 40"):
        S.sfg_smooth(H, torch.zeros(10, 4, dtype=torch.float64), 3, out=torch.zeros(20, dtype=torch.float64),
                     ws=ws)
    with pytest.raises(ValueError, match="out: dtype torch.float64"):
        S.sfg_smooth(H, torch.zeros(10, 4, dtype=torch.float64), 3, storage=torch.float32,
                     out=torch.zeros(10, 4, dtype=torch.float64), ws=ws)
    # everything else right: host memory is refused
    with pytest.raises(ValueError, match="device tensors"):
        S.sfg_smooth(H, torch.zeros(10, 4, dtype=torch.float64), 3, ws=ws)


def test_csr_view_is_checked_against_n_and_nnz():
    H = _csr(10, 18)
    H.col = H.col[:10]
    with pytest.raises(ValueError, match="csr.col: holds 10 elements, the call needs 18"):
        H.struct()
    H = _csr(10, 18)
    H.deg = H.deg.float()
    with pytest.raises(ValueError, match="csr.deg: dtype torch.float32"):
        H.struct()


def test_edge_scores_checks_ids_and_weights():
    u, v, w = _edges(6)
    x = torch.zeros(7, 4, dtype=torch.float64)
    with pytest.raises(ValueError, match="u: dtype torch.int64"):
        S.sfg_edge_scores(x, u.long(), v, w)
    with pytest.raises(ValueError, match="w: holds 5 elements"):
        S.sfg_edge_scores(x, u, v, w[:5])
    with pytest.raises(ValueError, match="cand: dtype torch.int64"):
        S.sfg_edge_scores(x, u, v, w, cand=torch.tensor([0, 2]))
    with pytest.raises(ValueError, match="x: must be contiguous"):
        S.sfg_edge_scores(torch.zeros(7, 8, dtype=torch.float64)[:, 1:5], u, v, w)
    with pytest.raises(ValueError, match="out: holds 1 elements, the call needs 2"):
        S.sfg_edge_scores(x, u, v, w, cand=torch.tensor([0, 2], dtype=torch.int32),
                          out=torch.zeros(1, dtype=torch.float64))


def test_select_checks_scores_and_outputs():
    ws = torch.zeros(256, dtype=torch.uint8)
    with pytest.raises(ValueError, match="score: dtype torch.int32"):
        S.sfg_select_topk(torch.zeros(5, dtype=torch.int32), 2, ws=ws)
    with pytest.raises(ValueError, match="sel: holds 3 elements"):
        S.sfg_select_topk(torch.zeros(5, dtype=torch.float64), 2, sel=torch.zeros(3, dtype=torch.uint8), ws=ws)
    with pytest.raises(ValueError, match="tau: dtype torch.float32"):
        S.sfg_select_topk(torch.zeros(5), 2, tau=torch.zeros(1, dtype=torch.float32), ws=ws)


def test_sparsify_checks_the_extent_of_x0():
    u, v, w = _edges(6)
    keep = torch.zeros(6, dtype=torch.uint8)
    n, k = 7, 4
    p = S.make_params(levels=3, k=k)
    with pytest.raises(ValueError, match=f"x0: holds {n * k} elements, the call needs {3 * n * k}"):
        S.sfg_sparsify(n, u, v, w, torch.zeros(n, k, dtype=torch.float64), p, keep=keep)
    p = S.make_params(k=k, rounds=2)
    with pytest.raises(ValueError, match=f"the call needs {2 * n * k}"):
        S.sfg_sparsify(n, u, v, w, torch.zeros(n, k, dtype=torch.float64), p, keep=keep)
    p = S.make_params(k=k, sigma=5.0)      # sigma mode: up to 16 batches by default
    with pytest.raises(ValueError, match=f"the call needs {16 * n * k}"):
        S.sfg_sparsify(n, u, v, w, torch.zeros(2, n, k, dtype=torch.float64), p, keep=keep)
    with pytest.raises(ValueError, match="keep: holds 5 elements"):
        S.sfg_sparsify(n, u, v, w, None, S.make_params(k=k), keep=torch.zeros(5, dtype=torch.uint8))
    with pytest.raises(ValueError, match="v: 5 entries, u has 6"):
        S.sfg_sparsify(n, u, torch.cat([v[:5], torch.zeros(1, dtype=torch.int32)])[:5], w, None,
                       S.make_params(k=k), keep=keep)


def test_laplacian_csr_checks_outputs_against_nnz():
    u, v, w = _edges(6)
    out = _csr(7, 12)
    out.eid = out.eid[:8]
    with pytest.raises(ValueError, match="out.eid: holds 8 elements, the call needs 12"):
        S.sfg_laplacian_csr(7, u, v, w, ws=torch.zeros(256, dtype=torch.uint8), out=out, nnz=12)
    with pytest.raises(ValueError, match="out.val: dtype torch.float32, the weights are torch.float64"):
        S.sfg_laplacian_csr(7, u, v, w, ws=torch.zeros(256, dtype=torch.uint8), out=_csr(7, 12, torch.float32),
                            nnz=12)
    with pytest.raises(ValueError, match="mask: dtype torch.bool"):
        S.sfg_laplacian_csr(7, u, v, w, mask=torch.ones(6, dtype=torch.bool))
