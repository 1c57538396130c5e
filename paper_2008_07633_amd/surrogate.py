"""Learned edge-criticality surrogate: training, model files, pruning.

The network and its kernels are in ``csrc/mpnn.hip`` (C ABI ``sfg_mpnn_*``).
This module drives them.  It only marshals and orchestrates; every numeric step runs
in libsfg:
  * a cheap embedding -- the first ``kc`` of the method's own random
    vectors, smoothed ``tc`` times on the spanning tree with BF16 storage and
    an FP32 last iterate -- feeds the features (sharing the vectors makes the
    cheap scores close relatives of the exact ones).  ``kc`` and ``tc`` are
    properties of a model: the fast default takes 4 vectors (its cheap
    embedding costs a fifth of the plain smoothing; the network lifts the
    recall of its candidates from 0.79 to 0.90 at 20%), the recall
    configuration all 16 (recall 0.99 at 20%, though then the cheap score
    alone does as well, since the plain scores share all their randomness);
  * training targets are the plain method's own scores (``K`` vectors, ``T``
    sweeps, FP32), as standardised logs;
  * inference predicts every off-tree edge, keeps the top ``cand_frac`` as
    candidates, and the plain scorer ranks the candidates exactly.

Model files are written and read by the library (``sfg_mpnn_save`` /
``sfg_mpnn_load``: a versioned binary format with the shapes, the cheap
embedding, the standardisation constants and a 64-bit FNV-1a hash), so a C
caller can use a model trained here; a file that fails any check raises
:class:`SurrogateInvalid`, and callers fall back to the plain scorer.  The
feature and target standardisation of the training set is computed by the
library too (``sfg_mpnn_fit_norm``, ``sfg_mpnn_standardize``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import sfg as S

KC = 4                 # vectors of the cheap embedding (fast default)
KC_RECALL = 16         # the recall configuration: every vector of the plain method
TC = 10                # sweeps of the cheap embedding (half of the plain method's 20)
N_NODE_FEAT, N_EDGE_FEAT = 8, 4


class SurrogateInvalid(RuntimeError):
    """The model cannot be used (missing, corrupted, incompatible or not finite)."""


@dataclass
class Model:
    params: torch.Tensor                 # F32 [param_count] on the device
    norm: torch.Tensor                   # F32 [24]: node means, node inv stds, edge means, edge inv stds
    y_mean: float = 0.0                  # target standardisation (log score)
    y_std: float = 1.0
    meta: dict = field(default_factory=dict)
    kc: int = KC                         # cheap embedding: vectors (the first kc of the method's block)
    tc: int = TC                         # cheap embedding: sweeps

    def save(self, path: str) -> None:
        S.sfg_mpnn_save(path, self.params.contiguous(), self.norm.contiguous(), self.kc, self.tc, self.y_mean,
                        self.y_std)


def load(path: str, device="cuda") -> Model:
    """A model file written by Model.save (or by a C caller through sfg_mpnn_save)."""
    try:
        params, norm, meta = S.sfg_mpnn_load(path, device)
    except S.SfgError as e:     # unreadable, or a failed check (the message says which)
        raise SurrogateInvalid(str(e)) from e
    return Model(params, norm, meta["y_mean"], meta["y_std"], kc=meta["kc"], tc=meta["tc"])


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """Seeded He-style initial weights and zero biases, in the flat layout of sfg.h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = []
    for rows, fan_in in ((17, 8), (65, 32), (69, 68)):
        w = rng.standard_normal((rows, 32)) * math.sqrt(2.0 / fan_in)
        w[-1, :] = 0.0           # bias row
        blocks.append(w.reshape(-1))
    w4 = rng.standard_normal(33) * math.sqrt(1.0 / 32)
    w4[-1] = 0.0
    blocks.append(w4)
    return torch.from_numpy(np.concatenate(blocks).astype(np.float32)).to(device)


# ----------------------------------------------------------------------------- per-graph preparation

@dataclass
class Prepared:
    n: int
    u: torch.Tensor
    v: torch.Tensor
    w32: torch.Tensor
    tree: torch.Tensor
    cand: torch.Tensor            # off-tree edge ids, ascending
    G: S.Csr                      # F32 CSR of the graph
    T: S.Csr                      # F32 CSR of the tree
    xc: torch.Tensor              # cheap embedding (n x kc, F32)
    tc: int = TC                  # its sweeps
    raw_nf: Optional[torch.Tensor] = None
    raw_ef: Optional[torch.Tensor] = None


def prepare(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, x0c: torch.Tensor, sweeps: int = TC,
            tree: Optional[torch.Tensor] = None) -> Prepared:
    """Tree, CSRs of G and of the tree, and the cheap embedding from x0c (n x kc,
    FP64) smoothed ``sweeps`` times on the tree (a model is used with the kc and
    sweeps it was trained with)."""
    w32 = w.float()
    if tree is None:
        tree, comps = S.sfg_spanning_tree(n, u, v, w)
        if comps != 1:
            raise S.SfgError(2, "graph is not connected")
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    G = S.sfg_laplacian_csr(n, u, v, w32)
    T = S.sfg_csr_select(G, tree)
    xc = S.sfg_smooth(T, x0c, sweeps, 0.5, storage=torch.bfloat16, final_f32=True)
    return Prepared(n, u, v, w32, tree, cand, G, T, xc, sweeps)


def features(pp: Prepared, norm: Optional[torch.Tensor]):
    return S.sfg_mpnn_features(pp.G, pp.T, pp.xc, pp.u, pp.v, pp.w32, cand=pp.cand, norm=norm)


def plain_scores(pp: Prepared, x0: torch.Tensor, sweeps: int, storage=torch.float32) -> torch.Tensor:
    """The plain method's scores of the off-tree edges (the training target and the reference for recall)."""
    X = S.sfg_smooth(pp.T, x0, sweeps, 0.5, storage=storage)
    return S.sfg_edge_scores(X, pp.u, pp.v, pp.w32, cand=pp.cand, score_dtype=torch.float32)


# ----------------------------------------------------------------------------- training

@dataclass
class TrainSet:
    graphs: list                  # Prepared (with raw features)
    targets: list                 # raw log scores (device F32)


def fit_norm(ts: TrainSet):
    """Feature and target standardisation of the training set, computed by the library
    (sfg_mpnn_fit_norm).  Returns the 24-value feature normalisation and the target mean and
    standard deviation, on the device."""
    return S.sfg_mpnn_fit_norm([g.raw_nf for g in ts.graphs], [g.raw_ef for g in ts.graphs],
                               [t.contiguous() for t in ts.targets])


def train(ts: TrainSet, epochs: int = 20, lr: float = 3e-3, seed: int = 7, lr_min: float = 3e-4,
          log=None) -> tuple[Model, list]:
    """Full-batch Adam over the training graphs, one step per graph per epoch,
    cosine-decayed learning rate.  Returns the model and the per-epoch mean loss.
    The model records the cheap embedding of the training graphs (all alike)."""
    dev = ts.targets[0].device
    kc, tc = int(ts.graphs[0].xc.shape[1]), ts.graphs[0].tc
    if any(int(g.xc.shape[1]) != kc or g.tc != tc for g in ts.graphs):
        raise ValueError("training graphs must share one cheap embedding (vectors and sweeps)")
    norm, ystat = fit_norm(ts)
    ym, ysd = (float(x) for x in ystat.cpu())
    feats = []
    for g, t in zip(ts.graphs, ts.targets):
        nf, ef = features(g, norm)
        feats.append((nf, ef, S.sfg_mpnn_standardize(t.contiguous(), ystat)))
    params = init_params(seed, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    ws_cache = {}
    history = []
    step = 0
    total = epochs * len(ts.graphs)
    for ep in range(epochs):
        losses = []
        for gi, (g, (nf, ef, y)) in enumerate(zip(ts.graphs, feats)):
            key = (g.n, int(ef.shape[0]))
            if key not in ws_cache:
                ws_cache[key] = torch.empty(S.sfg_workspace_bytes(S.OP_MPNN_TRAIN, g.n, key[1], 0, S.F32),
                                            dtype=torch.uint8, device=dev)
            _, loss, _ = S.sfg_mpnn_loss_grad(g.G, params, nf, g.u, g.v, ef, y, cand=g.cand, ws=ws_cache[key],
                                              grad=grad)
            step += 1
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * (step - 1) / max(total - 1, 1)))
            S.sfg_mpnn_adam(params, grad, m, v, step, lr=lr_t)
            losses.append(loss)
        ep_loss = float(torch.stack(losses).mean().item())
        history.append(ep_loss)
        if log:
            log(f"epoch {ep}: loss {ep_loss:.4f}")
    return Model(params, norm, ym, ysd, {"epochs": epochs, "lr": lr, "seed": seed}, kc=kc, tc=tc), history


# ----------------------------------------------------------------------------- inference

def predict(model: Model, pp: Prepared, act=torch.bfloat16) -> torch.Tensor:
    nf, ef = features(pp, model.norm)
    return S.sfg_mpnn_forward(pp.G, model.params, nf, pp.u, pp.v, ef, cand=pp.cand, act=act)


def prune(model: Model, pp: Prepared, cand_frac: float, act=torch.bfloat16):
    """Positions (into pp.cand) of the top cand_frac of the off-tree edges by prediction."""
    pred = predict(model, pp, act)
    k = int(math.ceil(cand_frac * int(pp.cand.numel())))
    sel, _ = S.sfg_select_topk(pred, k)
    return torch.nonzero(sel).reshape(-1).to(torch.int32), pred


def recall(chosen_plain_pos: torch.Tensor, cand_pos: torch.Tensor, n_cand: int) -> float:
    """Fraction of the plain method's chosen edges that are among the surrogate's candidates."""
    if chosen_plain_pos.numel() == 0:
        return 1.0
    mark = torch.zeros(n_cand, dtype=torch.bool, device=cand_pos.device)
    mark[cand_pos.long()] = True
    return float(mark[chosen_plain_pos.long()].float().mean().item())


# ----------------------------------------------------------------------------- pruned sparsifier

@dataclass
class PrunedResult:
    keep: torch.Tensor            # uint8 [m]: 1 tree, 2 recovered
    fallback: bool
    reason: str
    n_cand: int                   # off-tree edges
    n_scored: int                 # edges scored exactly
    k_sel: int


def sparsify_pruned(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, x0: torch.Tensor, model,
                    sweeps: int, frac: float, cand_frac: float, storage=torch.float32) -> PrunedResult:
    """Spanning tree + top f of the off-tree edges, where only the surrogate's
    top cand_frac candidates are scored exactly.  ``model`` is a Model or a
    path; if it cannot be used the plain single-level path runs instead."""
    m = int(u.shape[0])
    try:
        mdl = load(model, u.device) if isinstance(model, str) else model
        if not bool(torch.isfinite(mdl.params).all().item()):
            raise SurrogateInvalid("surrogate parameters are not finite")
    except SurrogateInvalid as e:
        keep, rep = S.sfg_sparsify(n, u, v, w, x0, S.make_params(k=int(x0.shape[1]), sweeps=sweeps, frac=frac,
                                                                 storage=storage))
        r = rep[0]
        return PrunedResult(keep, True, str(e), int(r["n_cand"]), int(r["n_cand"]), int(r["k_sel"]))
    pp = prepare(n, u, v, w, x0[:, :mdl.kc].contiguous(), mdl.tc)
    cand_pos, _ = prune(mdl, pp, cand_frac)
    cand_e = pp.cand[cand_pos.long()].contiguous()
    X = S.sfg_smooth(pp.T, x0, sweeps, 0.5, storage=storage)
    s = S.sfg_edge_scores(X, pp.u, pp.v, pp.w32, cand=cand_e, score_dtype=torch.float32)
    n_cand = int(pp.cand.numel())
    k_sel = int(math.ceil(frac * n_cand))
    k_take = min(k_sel, int(cand_e.numel()))
    sel, _ = S.sfg_select_topk(s, k_take)
    keep = pp.tree.clone()
    keep[cand_e[sel.bool()].long()] = 2
    return PrunedResult(keep, False, "", n_cand, int(cand_e.numel()), k_take)


def sparsify_ranked(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, x0: torch.Tensor, model,
                    sweeps: int, frac: float, storage=torch.float32) -> PrunedResult:
    """Spanning tree + the top ``frac`` of the off-tree edges ranked by the
    surrogate's prediction alone: no K-vector smoothing and no exact scoring,
    only the cheap embedding, the features and one inference.
    ``model`` is a Model or a path; if it cannot be used the plain
    single-level path runs instead (``storage`` is its precision)."""
    try:
        mdl = load(model, u.device) if isinstance(model, str) else model
        if not bool(torch.isfinite(mdl.params).all().item()):
            raise SurrogateInvalid("surrogate parameters are not finite")
    except SurrogateInvalid as e:
        keep, rep = S.sfg_sparsify(n, u, v, w, x0, S.make_params(k=int(x0.shape[1]), sweeps=sweeps, frac=frac,
                                                                 storage=storage))
        r = rep[0]
        return PrunedResult(keep, True, str(e), int(r["n_cand"]), int(r["n_cand"]), int(r["k_sel"]))
    pp = prepare(n, u, v, w, x0[:, :mdl.kc].contiguous(), mdl.tc)
    pred = predict(mdl, pp)
    n_cand = int(pp.cand.numel())
    k_sel = int(math.ceil(frac * n_cand))
    sel, _ = S.sfg_select_topk(pred, k_sel)
    keep = pp.tree.clone()
    keep[pp.cand[sel.bool()].long()] = 2
    return PrunedResult(keep, False, "", n_cand, 0, k_sel)
