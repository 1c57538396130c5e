"""Python binding of libsfg (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: it allocates outputs and workspaces as torch device
tensors, passes their pointers and torch's current stream, and turns a
non-OK status into :class:`SfgError`.  If ``libsfg.so`` has not been built
the binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfg.so")

# sfg_dtype
F64, F32, F16, BF16 = 0, 1, 2, 3
_TORCH_TO_SFG = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
_SFG_TO_TORCH = {v: k for k, v in _TORCH_TO_SFG.items()}

# sfg_op
OP_LAPLACIAN_CSR, OP_SMOOTH, OP_SELECT_TOPK, OP_AFFINITY, OP_COARSEN = 0, 1, 2, 3, 4
EMBED_SPARSIFIER, EMBED_GRAPH = 0, 1

STATUS = {0: "SFG_OK", 1: "SFG_EINVAL", 2: "SFG_ENOTCONN", 3: "SFG_ENOMEM", 4: "SFG_EHIP",
          5: "SFG_EWORKSPACE", 6: "SFG_EUNSUPPORTED", 7: "SFG_ENUMERIC"}

OP_MPNN_FORWARD, OP_MPNN_TRAIN, OP_COLOR, OP_TREE_ORDER, OP_TREE_SOLVE, OP_CSR_SELECT = 5, 6, 7, 8, 9, 10
OP_MPNN_NORM, OP_SMOOTH_ORDERED = 11, 12
SMOOTH_JACOBI, SMOOTH_GAUSS_SEIDEL = 0, 1

EXPORTED = ["sfg_workspace_bytes", "sfg_last_error", "sfg_laplacian_csr", "sfg_smooth", "sfg_edge_scores",
            "sfg_select_topk", "sfg_spanning_tree", "sfg_affinity", "sfg_coarsen", "sfg_sparsify",
            "sfg_mpnn_param_count", "sfg_mpnn_features", "sfg_mpnn_forward", "sfg_mpnn_loss_grad", "sfg_mpnn_adam",
            "sfg_color", "sfg_smooth_gs", "sfg_random_block", "sfg_tree_order", "sfg_tree_solve",
            "sfg_kappa_estimate", "sfg_csr_select", "sfg_pcg", "sfg_select_topk_noalloc", "sfg_mpnn_fit_norm",
            "sfg_mpnn_standardize", "sfg_mpnn_save", "sfg_mpnn_load", "sfg_smooth_ordered"]


class SfgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class CsrStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("eid", ctypes.c_void_p),
                ("deg", ctypes.c_void_p), ("vt", ctypes.c_int)]


class KappaParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("steps", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("seed", ctypes.c_uint64), ("block", ctypes.c_uint32)]


class KappaReport(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("ritz", ctypes.c_double * 64), ("steps", ctypes.c_int32),
                ("inner_iters", ctypes.c_int64), ("max_inner", ctypes.c_int32), ("unconverged", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class TreeStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("order", ctypes.c_void_p), ("parent", ctypes.c_void_p),
                ("size", ctypes.c_void_p), ("pw", ctypes.c_void_p), ("tdown", ctypes.c_void_p),
                ("tup", ctypes.c_void_p)]


class PcgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("inner_iters", ctypes.c_int64), ("relres", ctypes.c_double),
                ("ms", ctypes.c_float), ("converged", ctypes.c_int32), ("inner_capped", ctypes.c_int32)]


class MpnnMeta(ctypes.Structure):
    _fields_ = [("kc", ctypes.c_int32), ("tc", ctypes.c_int32), ("y_mean", ctypes.c_double),
                ("y_std", ctypes.c_double)]


class SurrogateStruct(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("norm", ctypes.c_void_p), ("kc", ctypes.c_int32),
                ("tc", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("k", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("omega", ctypes.c_double), ("frac", ctypes.c_double), ("embed", ctypes.c_int32),
                ("storage", ctypes.c_int), ("final_f32", ctypes.c_int32), ("band", ctypes.c_double),
                ("rounds", ctypes.c_int32), ("smoother", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("sigma", ctypes.c_double), ("est", KappaParams), ("surrogate", ctypes.POINTER(SurrogateStruct)),
                ("cand_frac", ctypes.c_double)]


class LevelReport(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("n_cand", ctypes.c_int64),
                ("k_sel", ctypes.c_int64), ("tau", ctypes.c_double), ("band", ctypes.c_int64),
                ("band_above", ctypes.c_int64), ("band_rounds", ctypes.c_int32),
                ("ms_smooth", ctypes.c_float), ("ms_score", ctypes.c_float), ("ms_select", ctypes.c_float),
                ("ms_other", ctypes.c_float), ("cone_rows", ctypes.c_int64), ("precision_fallback", ctypes.c_int32),
                ("node_order", ctypes.c_int32), ("n_scored", ctypes.c_int64), ("surrogate_fallback", ctypes.c_int32),
                ("sweeps_per_pass", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("level", LevelReport * 16), ("n_kappa", ctypes.c_int32),
                ("kappa", ctypes.c_double * 17), ("kappa_inner_iters", ctypes.c_int64),
                ("ms_kappa", ctypes.c_float)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsfg.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2008_07633_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        S, D = ctypes.c_size_t, ctypes.c_double
        L.sfg_workspace_bytes.argtypes = [I, I64, I64, I32, I]
        L.sfg_workspace_bytes.restype = S
        L.sfg_last_error.argtypes = []
        L.sfg_last_error.restype = ctypes.c_char_p
        L.sfg_laplacian_csr.argtypes = [I64, I64, P, P, P, I, P, P, P, P, P, P, P, P, S, P]
        L.sfg_smooth.argtypes = [P, I32, I32, D, P, I, I32, P, P, S, P]
        L.sfg_smooth_ordered.argtypes = [P, P, I32, I32, D, P, I, I32, P, P, P, S, P]
        L.sfg_edge_scores.argtypes = [P, I, I64, I32, I64, P, P, P, P, I, P, I, P]
        L.sfg_select_topk.argtypes = [P, I, I64, I64, P, P, P, P, S, P]
        L.sfg_select_topk_noalloc.argtypes = [P, I, I64, I64, P, P, P, P]
        L.sfg_spanning_tree.argtypes = [I64, I64, P, P, P, I, P, P, P, P]
        L.sfg_affinity.argtypes = [P, I, I64, I32, I64, P, P, P, I, P, S, P]
        L.sfg_coarsen.argtypes = [P, I64, P, P, P, I, P, I, P, P, P, P, P, P, P, P, S, P]
        L.sfg_sparsify.argtypes = [I64, I64, P, P, P, I, P, P, P, P, P]
        L.sfg_mpnn_param_count.argtypes = []
        L.sfg_mpnn_param_count.restype = I64
        L.sfg_mpnn_features.argtypes = [P, P, P, I32, I64, P, P, P, P, P, P, P, P]
        L.sfg_mpnn_forward.argtypes = [P, P, P, I64, P, P, P, P, I, P, P, S, P]
        L.sfg_mpnn_loss_grad.argtypes = [P, P, P, I64, P, P, P, P, P, P, P, P, P, S, P]
        L.sfg_mpnn_adam.argtypes = [P, P, P, P, I64, I64, D, D, D, D, P]
        L.sfg_color.argtypes = [P, P, P, P, P, P, S, P]
        L.sfg_random_block.argtypes = [I64, I32, ctypes.c_uint64, ctypes.c_uint32, P, P]
        L.sfg_smooth_gs.argtypes = [P, P, P, I32, I32, I32, D, P, I, P, P, S, P]
        L.sfg_tree_order.argtypes = [I64, I64, P, P, P, I, P, P, P, P, P, P, P, P, S, P]
        L.sfg_tree_solve.argtypes = [P, I32, P, P, P, S, P]
        L.sfg_kappa_estimate.argtypes = [I64, I64, P, P, P, I, P, P, P, P, P, P]
        L.sfg_csr_select.argtypes = [P, P, P, P, P, P, P, P, P, S, P]
        L.sfg_pcg.argtypes = [I64, I64, P, P, P, I, P, P, P, D, I32, P, P]
        L.sfg_mpnn_fit_norm.argtypes = [I32, P, P, P, P, P, P, P, P, S, P]
        L.sfg_mpnn_standardize.argtypes = [P, I64, P, P, P]
        L.sfg_mpnn_save.argtypes = [ctypes.c_char_p, P, P, P, P]
        L.sfg_mpnn_load.argtypes = [ctypes.c_char_p, P, P, P, P]
        for name in EXPORTED:
            if name not in ("sfg_workspace_bytes", "sfg_last_error", "sfg_mpnn_param_count"):
                getattr(L, name).restype = I
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        msg = lib().sfg_last_error()
        raise SfgError(status, msg.decode() if msg else "")


_I32, _U8, _F32, _F64 = (torch.int32,), (torch.uint8,), (torch.float32,), (torch.float64,)
_W = (torch.float64, torch.float32)                        # weight / score types
_X = (torch.float64, torch.float32, torch.float16, torch.bfloat16)   # block storage types


def _chk(t: Optional[torch.Tensor], name: str = "tensor", dtypes=None, numel: Optional[int] = None,
         optional: bool = False) -> None:
    """Check what the C ABI assumes of ``t`` apart from its device: one of
    ``dtypes``, contiguous, at least ``numel`` elements."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name}: required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: holds {t.numel()} elements, the call needs {numel}")


def _ptr(t: Optional[torch.Tensor], name: str = "tensor", dtypes=None, numel: Optional[int] = None,
         optional: bool = False):
    """Device pointer of ``t`` after the checks of :func:`_chk` and a check
    that it lives on a GPU.  Every binding runs these before it calls the
    library, so a wrong tensor raises ValueError instead of letting a kernel
    read or write past its end."""
    _chk(t, name, dtypes, numel, optional)
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name}: libsfg takes device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _ptrs(*specs) -> list:
    """Pointers of several (tensor, name, dtypes, numel[, optional]) arguments:
    every one is checked by :func:`_chk` before any is checked for its device."""
    for spec in specs:
        _chk(*spec)
    return [_ptr(*spec) for spec in specs]


def _block(x: torch.Tensor, name: str, dtypes, rows: Optional[int] = None) -> tuple[int, int]:
    """(n, k) of an n-by-k row-major block, checked to be 2-D."""
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise ValueError(f"{name}: expected an n-by-k tensor")
    if rows is not None and int(x.shape[0]) != rows:
        raise ValueError(f"{name}: has {int(x.shape[0])} rows, the graph has {rows} nodes")
    _chk(x, name, dtypes)
    return int(x.shape[0]), int(x.shape[1])


def _edges(u: torch.Tensor, v: torch.Tensor, w: Optional[torch.Tensor] = None) -> int:
    """Edge count of an edge list (u, v int32 of equal length, w of F64/F32)."""
    for name, t in (("u", u), ("v", v)):
        if not isinstance(t, torch.Tensor) or t.dim() != 1:
            raise ValueError(f"{name}: expected a 1-D tensor")
    m = int(u.shape[0])
    _chk(u, "u", _I32, m)
    if int(v.shape[0]) != m:
        raise ValueError(f"v: {int(v.shape[0])} entries, u has {m}")
    _chk(v, "v", _I32, m)
    if w is not None:
        _chk(w, "w", _W, m)
        if w.numel() != m:
            raise ValueError(f"w: {w.numel()} entries, u has {m}")
    return m


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(t: torch.Tensor) -> int:
    return _TORCH_TO_SFG[t.dtype]


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sfg_workspace_bytes(op: int, n: int, m: int, k: int, dtype) -> int:
    t = dtype if isinstance(dtype, int) else _TORCH_TO_SFG[dtype]
    return int(lib().sfg_workspace_bytes(op, n, m, k, t))


@dataclass
class Csr:
    """Device CSR of the adjacency plus the degree vector (views of torch tensors)."""
    n: int
    nnz: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    eid: torch.Tensor
    deg: torch.Tensor

    def struct(self) -> CsrStruct:
        """The C view, after checking every array against n and nnz."""
        n, nnz = int(self.n), int(self.nnz)
        ptrs = _ptrs((self.rowptr, "csr.rowptr", _I32, n + 1), (self.col, "csr.col", _I32, nnz),
                     (self.val, "csr.val", _W, nnz), (self.eid, "csr.eid", _I32, nnz, True),
                     (self.deg, "csr.deg", (self.val.dtype,), n))
        return CsrStruct(n, nnz, *(None if p is None else p.value for p in ptrs), _TORCH_TO_SFG[self.val.dtype])


def sfg_laplacian_csr(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                      mask: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                      out: Optional[Csr] = None, nnz: Optional[int] = None) -> Csr:
    """CSR of A and the degrees D of the graph (L = D - A).  With ``out`` and
    ``nnz`` given nothing is allocated and the call does not synchronise."""
    m = _edges(u, v, w)
    pm = _ptr(mask, "mask", _U8, m, optional=True)
    dev = u.device
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_LAPLACIAN_CSR, n, m, 0, w.dtype), dev)
    if out is None:
        cap = 2 * m if mask is None else 2 * int(mask.sum().item())
        out = Csr(n, cap, torch.empty(n + 1, dtype=torch.int32, device=dev),
                  torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                  torch.empty(max(cap, 1), dtype=w.dtype, device=dev),
                  torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                  torch.empty(n, dtype=w.dtype, device=dev))
    # the call writes 2 x (included edges) entries
    need = int(nnz) if nnz is not None else (2 * m if mask is None else 2 * int(mask.sum().item()))
    if out.val.dtype != w.dtype:
        raise ValueError(f"out.val: dtype {out.val.dtype}, the weights are {w.dtype}")
    outs = _ptrs((out.rowptr, "out.rowptr", _I32, n + 1), (out.col, "out.col", _I32, need),
                 (out.val, "out.val", _W, need), (out.eid, "out.eid", _I32, need),
                 (out.deg, "out.deg", (w.dtype,), n))
    got = ctypes.c_int64(0)
    _check(lib().sfg_laplacian_csr(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w), pm, *outs,
                                   None if nnz is not None else ctypes.byref(got), _ptr(ws, "ws", _U8),
                                   ws.numel(), _stream()))
    out.nnz = int(nnz) if nnz is not None else int(got.value)
    return out


def sfg_csr_select(G: Csr, mask: torch.Tensor, out: Optional[Csr] = None, nnz: Optional[int] = None,
                   ws: Optional[torch.Tensor] = None) -> Csr:
    """CSR of the subgraph of the edges with mask != 0, taken from G's CSR (bit-identical to
    sfg_laplacian_csr with the mask).  With ``out`` and ``nnz`` given nothing is allocated and the
    call does not synchronise."""
    n = G.n
    dev = G.rowptr.device
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_CSR_SELECT, n, G.nnz // 2, 0, G.val.dtype), dev)
    if out is None:
        cap = G.nnz
        out = Csr(n, cap, torch.empty(n + 1, dtype=torch.int32, device=dev),
                  torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                  torch.empty(max(cap, 1), dtype=G.val.dtype, device=dev),
                  torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                  torch.empty(n, dtype=G.val.dtype, device=dev))
    got = ctypes.c_int64(0)
    gs = G.struct()
    need = int(nnz) if nnz is not None else G.nnz
    if out.val.dtype != G.val.dtype:
        raise ValueError(f"out.val: dtype {out.val.dtype}, G's values are {G.val.dtype}")
    _chk(mask, "mask", _U8, G.nnz // 2)
    outs = _ptrs((out.rowptr, "out.rowptr", _I32, n + 1), (out.col, "out.col", _I32, need),
                 (out.val, "out.val", _W, need), (out.eid, "out.eid", _I32, need),
                 (out.deg, "out.deg", (G.val.dtype,), n))
    _check(lib().sfg_csr_select(ctypes.byref(gs), _ptr(mask, "mask", _U8, G.nnz // 2), *outs,
                                None if nnz is not None else ctypes.byref(got), _ptr(ws, "ws", _U8), ws.numel(),
                                _stream()))
    out.nnz = int(nnz) if nnz is not None else int(got.value)
    return out


def sfg_smooth(H: Csr, x0: torch.Tensor, sweeps: int, omega: float = 0.5, storage=torch.float64,
               final_f32: bool = False, out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Centre the n-by-k FP64 block x0 and smooth it with damped-Jacobi sweeps on H."""
    n, k = _block(x0, "x0", _F64, rows=H.n)
    st = storage if isinstance(storage, int) else _TORCH_TO_SFG[storage]
    odt = torch.float32 if (final_f32 and st in (F16, BF16)) else _SFG_TO_TORCH[st]
    if out is None:
        out = torch.empty((n, k), dtype=odt, device=x0.device)
    _chk(out, "out", (odt,), n * k)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_SMOOTH, n, 0, k, st), x0.device)
    hs = H.struct()
    _check(lib().sfg_smooth(ctypes.byref(hs), k, sweeps, float(omega), _ptr(x0), st, int(bool(final_f32)),
                            _ptr(out, "out", (odt,), n * k), _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    return out


def sfg_smooth_ordered(H: Csr, order: torch.Tensor, x0: torch.Tensor, sweeps: int, omega: float = 0.5,
                       storage=torch.float64, final_f32: bool = False, out: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, info: Optional[dict] = None) -> torch.Tensor:
    """sfg_smooth with the rows taken in ``order`` (a permutation, e.g. a spanning tree's preorder), several
    sweeps per pass over the block where the graph allows; the same bits.  ``info["sweeps_per_pass"]``: 2 to 4,
    or 1 when the plain path ran."""
    n, k = _block(x0, "x0", _F64, rows=H.n)
    _chk(order, "order", _I32, n)
    st = storage if isinstance(storage, int) else _TORCH_TO_SFG[storage]
    odt = torch.float32 if (final_f32 and st in (F16, BF16)) else _SFG_TO_TORCH[st]
    if out is None:
        out = torch.empty((n, k), dtype=odt, device=x0.device)
    _chk(out, "out", (odt,), n * k)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_SMOOTH_ORDERED, n, 0, k, st), x0.device)
    hs = H.struct()
    per_pass = ctypes.c_int32(0)
    _check(lib().sfg_smooth_ordered(ctypes.byref(hs), _ptr(order), k, sweeps, float(omega), _ptr(x0), st,
                                    int(bool(final_f32)), _ptr(out), ctypes.byref(per_pass), _ptr(ws, "ws", _U8),
                                    ws.numel(), _stream()))
    if info is not None:
        info["sweeps_per_pass"] = int(per_pass.value)
    return out


def sfg_random_block(n: int, k: int, seed: int, block: int = 0, device="cuda",
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """n-by-k FP64 standard normals drawn on the device (Philox4x32-10, Box-Muller)."""
    if out is None:
        out = torch.empty((n, k), dtype=torch.float64, device=device)
    _check(lib().sfg_random_block(n, k, ctypes.c_uint64(seed), ctypes.c_uint32(block),
                                  _ptr(out, "out", _F64, n * k), _stream()))
    return out


def sfg_color(H: Csr, ws: Optional[torch.Tensor] = None):
    """Multicolouring for the Gauss-Seidel smoother: (color[n], class_rows[n],
    class_ptr[n+1] with the first ncolors+1 entries used, ncolors)."""
    dev = H.rowptr.device
    color = torch.empty(H.n, dtype=torch.int32, device=dev)
    rows = torch.empty(H.n, dtype=torch.int32, device=dev)
    ptr = torch.empty(H.n + 1, dtype=torch.int32, device=dev)
    nc = ctypes.c_int32(0)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_COLOR, H.n, 0, 0, F64), dev)
    hs = H.struct()
    _check(lib().sfg_color(ctypes.byref(hs), _ptr(color), _ptr(rows), _ptr(ptr), ctypes.byref(nc),
                           _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    return color, rows, ptr, int(nc.value)


def sfg_smooth_gs(H: Csr, classes, x0: torch.Tensor, sweeps: int, omega: float = 1.0, storage=torch.float64,
                  out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Centre x0 and smooth it by multicolour Gauss-Seidel sweeps (classes from sfg_color)."""
    _, rows, ptr, nc = classes
    n, k = _block(x0, "x0", _F64, rows=H.n)
    st = storage if isinstance(storage, int) else _TORCH_TO_SFG[storage]
    if out is None:
        out = torch.empty((n, k), dtype=_SFG_TO_TORCH[st], device=x0.device)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_SMOOTH, n, 0, k, st), x0.device)
    hs = H.struct()
    _check(lib().sfg_smooth_gs(ctypes.byref(hs), _ptr(rows, "class_rows", _I32, n),
                               _ptr(ptr, "class_ptr", _I32, int(nc) + 1), nc, k, sweeps, float(omega), _ptr(x0),
                               st, _ptr(out, "out", (_SFG_TO_TORCH[st],), n * k), _ptr(ws, "ws", _U8),
                               ws.numel(), _stream()))
    return out


def sfg_edge_scores(x: torch.Tensor, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                    cand: Optional[torch.Tensor] = None, score_dtype=None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """w_e * |x_u - x_v|^2 for every candidate edge (all edges if cand is None)."""
    n, k = _block(x, "x", _X)
    m = _edges(u, v, w)
    ne = int(cand.numel()) if cand is not None else m
    _chk(cand, "cand", _I32, ne, optional=True)
    sdt = score_dtype or (torch.float64 if x.dtype == torch.float64 else torch.float32)
    if out is None:
        out = torch.empty(max(ne, 1), dtype=sdt, device=x.device)[:ne]
    _chk(out, "out", _W, ne)
    _check(lib().sfg_edge_scores(_ptr(x), _dt(x), n, k, ne, _ptr(cand, optional=True), _ptr(u), _ptr(v), _ptr(w),
                                 _dt(w), _ptr(out), _TORCH_TO_SFG[out.dtype], _stream()))
    return out


def sfg_select_topk(score: torch.Tensor, k: int, sel: Optional[torch.Tensor] = None,
                    tau: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, sync: bool = True):
    """Mark the top k scores (ties: lower position first).  Returns (sel, tau)."""
    _chk(score, "score", _W)
    ne = int(score.numel())
    dev = score.device
    if sel is None:
        sel = torch.empty(max(ne, 1), dtype=torch.uint8, device=dev)[:ne]
    if tau is None:
        tau = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_SELECT_TOPK, 0, ne, 0, score.dtype), dev)
    th = ctypes.c_double(0.0)
    _chk(sel, "sel", _U8, ne)
    _chk(tau, "tau", _F64, 1)
    _check(lib().sfg_select_topk(_ptr(score), _dt(score), ne, int(k), _ptr(sel, "sel", _U8, ne),
                                 _ptr(tau, "tau", _F64, 1), ctypes.byref(th) if sync else None,
                                 _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    return sel, (th.value if sync else tau)


def sfg_select_topk_noalloc(score: torch.Tensor, k: int, sel: Optional[torch.Tensor] = None,
                            tau: Optional[torch.Tensor] = None, sync: bool = True):
    """sfg_select_topk on the library's per-device scratch array: no workspace, nothing allocated by
    the library (pass ``sel`` and ``tau`` to allocate nothing at all).  Returns (sel, tau)."""
    _chk(score, "score", _W)
    ne = int(score.numel())
    dev = score.device
    if sel is None:
        sel = torch.empty(max(ne, 1), dtype=torch.uint8, device=dev)[:ne]
    if tau is None:
        tau = torch.empty(1, dtype=torch.float64, device=dev)
    _chk(sel, "sel", _U8, ne)
    _chk(tau, "tau", _F64, 1)
    th = ctypes.c_double(0.0)
    _check(lib().sfg_select_topk_noalloc(_ptr(score), _dt(score), ne, int(k), _ptr(sel), _ptr(tau),
                                         ctypes.byref(th) if sync else None, _stream()))
    return sel, (th.value if sync else tau)


def sfg_spanning_tree(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                      allowed: Optional[torch.Tensor] = None):
    """Maximum-weight spanning forest (weight desc, edge id asc).  Returns (in_tree, n_components)."""
    m = _edges(u, v, w)
    out = torch.empty(max(m, 1), dtype=torch.uint8, device=u.device)[:m]
    nc = ctypes.c_int64(0)
    _check(lib().sfg_spanning_tree(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w),
                                   _ptr(allowed, "allowed", _U8, m, optional=True), _ptr(out), ctypes.byref(nc),
                                   _stream()))
    return out, int(nc.value)


def sfg_affinity(x: torch.Tensor, u: torch.Tensor, v: torch.Tensor, aff_dtype=None,
                 out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    n, k = _block(x, "x", _W)
    m = _edges(u, v)
    adt = aff_dtype or x.dtype
    if out is None:
        out = torch.empty(max(m, 1), dtype=adt, device=x.device)[:m]
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_AFFINITY, n, m, k, x.dtype), x.device)
    _check(lib().sfg_affinity(_ptr(x), _dt(x), n, k, m, _ptr(u), _ptr(v), _ptr(out, "out", _W, m), _dt(out),
                              _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    return out


def sfg_coarsen(G: Csr, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, aff: torch.Tensor,
                ws: Optional[torch.Tensor] = None):
    """One coarsening step.  Returns (agg, cu, cv, cw, crep) trimmed to the coarse sizes."""
    m = _edges(u, v, w)
    _chk(aff, "aff", _W, m)
    dev = u.device
    agg = torch.empty(G.n, dtype=torch.int32, device=dev)
    cu = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    cw = torch.empty(max(m, 1), dtype=w.dtype, device=dev)
    crep = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_COARSEN, G.n, m, 0, w.dtype), dev)
    nc, mc = ctypes.c_int64(0), ctypes.c_int64(0)
    gs = G.struct()
    _check(lib().sfg_coarsen(ctypes.byref(gs), m, _ptr(u), _ptr(v), _ptr(w), _dt(w), _ptr(aff), _dt(aff),
                             _ptr(agg), ctypes.byref(nc), ctypes.byref(mc), _ptr(cu), _ptr(cv), _ptr(cw),
                             _ptr(crep), _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    mc = int(mc.value)
    return agg, int(nc.value), cu[:mc], cv[:mc], cw[:mc], crep[:mc]


def make_kappa_params(k=8, steps=6, tol=1e-1, max_iter=20000, seed=0, block=0) -> KappaParams:
    return KappaParams(k, steps, tol, max_iter, seed, block)


def make_params(levels=1, k=8, sweeps=10, omega=0.5, frac=0.05, embed=EMBED_SPARSIFIER, storage=F64,
                final_f32=False, band=0.0, rounds=None, smoother=SMOOTH_JACOBI, seed=0, sigma=0.0,
                est: Optional[KappaParams] = None, surrogate=None, cand_frac=0.2) -> Params:
    """rounds: multi-round densification (default 1); with sigma > 0 the cap on batches (default 0 = 16).
    surrogate: anything with device tensors ``params`` and ``norm`` and ints ``kc``, ``tc`` (a trained
    surrogate.Model): sfg_sparsify then scores exactly only its top ``cand_frac`` of the off-tree edges."""
    if rounds is None:
        rounds = 0 if sigma > 0 else 1
    st = storage if isinstance(storage, int) else _TORCH_TO_SFG[storage]
    p = Params(levels, k, sweeps, omega, frac, embed, st, int(bool(final_f32)), band, rounds, smoother, seed,
               sigma, est if est is not None else make_kappa_params(), None, cand_frac)
    if surrogate is not None:
        sg = SurrogateStruct(_ptr(surrogate.params), _ptr(surrogate.norm), int(surrogate.kc), int(surrogate.tc))
        p.surrogate = ctypes.pointer(sg)
        p._keep = (sg, surrogate)      # the struct and the tensors it points to live as long as the params
    return p


def sfg_sparsify(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, x0: Optional[torch.Tensor],
                 params: Params, keep: Optional[torch.Tensor] = None, info: Optional[dict] = None):
    """Sparsifier keep mask (0 off, 1 base sparsifier, 2 recovered) and the per-level report.
    x0 None: the random blocks are drawn on the device from params.seed.  ``info`` (a dict)
    receives the condition-number estimates of sigma mode."""
    m = _edges(u, v, w)
    if keep is None:
        keep = torch.empty(max(m, 1), dtype=torch.uint8, device=u.device)[:m]
    # x0 holds one n-by-k block per level, per round, or per batch of sigma mode (as the library reads it)
    blocks = (params.levels if params.levels > 1 else
              (params.rounds if params.rounds > 0 else 16) if params.sigma > 0 else max(params.rounds, 1))
    _chk(x0, "x0", _F64, blocks * n * params.k, optional=True)
    _chk(keep, "keep", _U8, m)
    rep = Report()
    _check(lib().sfg_sparsify(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w), ctypes.byref(params),
                              _ptr(x0, "x0", _F64, blocks * n * params.k, optional=True),
                              _ptr(keep, "keep", _U8, m), ctypes.byref(rep), _stream()))
    levels = []
    for i in range(rep.levels):
        L = rep.level[i]
        levels.append({f: getattr(L, f) for f, _ in LevelReport._fields_})
    if info is not None:
        info["kappa"] = [float(rep.kappa[j]) for j in range(rep.n_kappa)]
        info["kappa_inner_iters"] = int(rep.kappa_inner_iters)
        info["ms_kappa"] = float(rep.ms_kappa)
    return keep, levels


# ----------------------------------------------------------------------------- sigma-driven stopping

class Tree:
    """Device arrays of sfg_tree_order (preorder layout of a spanning tree rooted at 0)."""

    def __init__(self, n, order, parent, size, pw, tdown, tup):
        self.n, self.order, self.parent, self.size = n, order, parent, size
        self.pw, self.tdown, self.tup = pw, tdown, tup

    def struct(self) -> TreeStruct:
        n = self.n
        ptrs = _ptrs((self.order, "tree.order", _I32, n), (self.parent, "tree.parent", _I32, n),
                     (self.size, "tree.size", _I32, n), (self.pw, "tree.pw", _F64, n),
                     (self.tdown, "tree.tdown", _I32, n), (self.tup, "tree.tup", _I32, n))
        return TreeStruct(n, *(p.value for p in ptrs))


def sfg_tree_order(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, keep: torch.Tensor) -> Tree:
    """Preorder layout of the spanning tree of the edges with keep == 1 (w must be float64)."""
    dev = u.device
    m = _edges(u, v, w)
    _chk(keep, "keep", _U8, m)
    arr = [torch.empty(n, dtype=torch.int32, device=dev) for _ in range(5)]
    pw = torch.empty(n, dtype=torch.float64, device=dev)
    ws = _ws(sfg_workspace_bytes(OP_TREE_ORDER, n, m, 0, F64), dev)
    order, parent, size, tdown, tup = arr
    _check(lib().sfg_tree_order(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w), _ptr(keep), _ptr(order), _ptr(parent),
                                _ptr(size), _ptr(pw), _ptr(tdown), _ptr(tup), _ptr(ws), ws.numel(), _stream()))
    return Tree(n, order, parent, size, pw, tdown, tup)


def sfg_tree_solve(tree: Tree, b: torch.Tensor, out: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = L_T^+ b per column (b: n-by-k float64, node order)."""
    if int(b.shape[0]) != tree.n:
        raise ValueError(f"b: has {int(b.shape[0])} rows, the tree has {tree.n} nodes")
    b2 = b.reshape(b.shape[0], -1)
    k = int(b2.shape[1])
    if out is None:
        out = torch.empty_like(b2)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_TREE_SOLVE, tree.n, 0, k, F64), b.device)
    ts = tree.struct()
    _check(lib().sfg_tree_solve(ctypes.byref(ts), k, _ptr(b2, "b", _F64, tree.n * k),
                                _ptr(out, "out", _F64, tree.n * k), _ptr(ws, "ws", _U8), ws.numel(), _stream()))
    return out.reshape(b.shape)


def sfg_pcg(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, keep: torch.Tensor, b: torch.Tensor,
            tol: float = 1e-3, max_iter: int = 20000, want_x: bool = True):
    """CG on L_G x = b grounded at node 0, preconditioned by the sparsifier ``keep`` (its tree marked 1).
    Returns (x or None, report dict)."""
    m = _edges(u, v, w)
    x = torch.empty(n, dtype=torch.float64, device=b.device) if want_x else None
    rep = PcgReport()
    b64 = b.to(torch.float64).contiguous()
    _check(lib().sfg_pcg(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w), _ptr(keep, "keep", _U8, m),
                         _ptr(b64, "b", _F64, n), _ptr(x, optional=True), float(tol), int(max_iter),
                         ctypes.byref(rep), _stream()))
    return x, {f: getattr(rep, f) for f, _ in PcgReport._fields_}


def sfg_kappa_estimate(n: int, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, keep: torch.Tensor,
                       params: Optional[KappaParams] = None, y0: Optional[torch.Tensor] = None):
    """Estimate of kappa(L_G, L_P) for P = edges with keep != 0 (tree edges marked 1).
    Returns (kappa, report dict)."""
    m = _edges(u, v, w)
    kp = params if params is not None else make_kappa_params()
    kap = ctypes.c_double(0.0)
    rep = KappaReport()
    kb = kp.k if kp.k > 0 else 8
    _check(lib().sfg_kappa_estimate(n, m, _ptr(u), _ptr(v), _ptr(w), _dt(w), _ptr(keep, "keep", _U8, m),
                                    ctypes.byref(kp), _ptr(y0, "y0", _F64, n * kb, optional=True),
                                    ctypes.byref(kap), ctypes.byref(rep), _stream()))
    steps = int(rep.steps)
    return float(kap.value), {"ritz": [float(rep.ritz[i]) for i in range(min(steps, 64))],
                              "inner_iters": int(rep.inner_iters), "max_inner": int(rep.max_inner),
                              "unconverged": int(rep.unconverged), "ms": float(rep.ms)}


# ----------------------------------------------------------------------------- learned surrogate

def sfg_mpnn_param_count() -> int:
    return int(lib().sfg_mpnn_param_count())


def _mpnn_args(G: Csr, params, node_feat, u, v, edge_feat, cand, ne: int) -> None:
    """Checks shared by inference and training: parameter vector, n-by-8 node and ne-by-4 edge features."""
    _chk(params, "params", _F32, sfg_mpnn_param_count())
    _chk(node_feat, "node_feat", _F32, G.n * 8)
    _chk(edge_feat, "edge_feat", _F32, ne * 4)
    m = _edges(u, v)
    _chk(cand, "cand", _I32, ne, optional=True)
    if cand is None and ne > m:
        raise ValueError(f"edge_feat: {ne} rows, the edge list has {m} edges")


def sfg_mpnn_features(G: Csr, T: Csr, xc: torch.Tensor, u: torch.Tensor, v: torch.Tensor, w32: torch.Tensor,
                      cand: Optional[torch.Tensor] = None, norm: Optional[torch.Tensor] = None):
    """Node (n x 8) and candidate-edge (ne x 4) features of the surrogate."""
    n, kc = _block(xc, "xc", _F32, rows=G.n)
    m = _edges(u, v, w32)
    if w32.dtype != torch.float32:
        raise ValueError("w32: the surrogate takes F32 weights")
    ne = int(cand.numel()) if cand is not None else m
    _chk(cand, "cand", _I32, ne, optional=True)
    _chk(norm, "norm", _F32, 24, optional=True)
    nf = torch.empty((n, 8), dtype=torch.float32, device=xc.device)
    ef = torch.empty((max(ne, 1), 4), dtype=torch.float32, device=xc.device)[:ne]
    gs, ts = G.struct(), T.struct()
    _check(lib().sfg_mpnn_features(ctypes.byref(gs), ctypes.byref(ts), _ptr(xc), kc, ne,
                                   _ptr(cand, optional=True), _ptr(u), _ptr(v), _ptr(w32),
                                   _ptr(norm, optional=True), _ptr(nf), _ptr(ef), _stream()))
    return nf, ef


def sfg_mpnn_forward(G: Csr, params: torch.Tensor, node_feat: torch.Tensor, u: torch.Tensor, v: torch.Tensor,
                     edge_feat: torch.Tensor, cand: Optional[torch.Tensor] = None, act=torch.bfloat16,
                     out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    ne = int(edge_feat.shape[0])
    _mpnn_args(G, params, node_feat, u, v, edge_feat, cand, ne)
    if out is None:
        out = torch.empty(max(ne, 1), dtype=torch.float32, device=params.device)[:ne]
    _chk(out, "out", _F32, ne)
    a = _TORCH_TO_SFG[act]
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_MPNN_FORWARD, G.n, 0, 0, a), params.device)
    gs = G.struct()
    _check(lib().sfg_mpnn_forward(ctypes.byref(gs), _ptr(params), _ptr(node_feat), ne,
                                  _ptr(cand, optional=True), _ptr(u), _ptr(v),
                                  _ptr(edge_feat), a, _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def sfg_mpnn_loss_grad(G: Csr, params: torch.Tensor, node_feat: torch.Tensor, u: torch.Tensor, v: torch.Tensor,
                       edge_feat: torch.Tensor, target: torch.Tensor, cand: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
    """FP32 forward + backward.  Returns (pred, loss (device scalar), grad)."""
    ne = int(edge_feat.shape[0])
    _mpnn_args(G, params, node_feat, u, v, edge_feat, cand, ne)
    _chk(target, "target", _F32, ne)
    if grad is not None:
        _chk(grad, "grad", _F32, sfg_mpnn_param_count())
    dev = params.device
    pred = torch.empty(ne, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    if grad is None:
        grad = torch.empty_like(params)
    if ws is None:
        ws = _ws(sfg_workspace_bytes(OP_MPNN_TRAIN, G.n, ne, 0, F32), dev)
    gs = G.struct()
    _check(lib().sfg_mpnn_loss_grad(ctypes.byref(gs), _ptr(params), _ptr(node_feat), ne,
                                    _ptr(cand, optional=True), _ptr(u), _ptr(v),
                                    _ptr(edge_feat), _ptr(target), _ptr(pred), _ptr(loss), _ptr(grad), _ptr(ws),
                                    ws.numel(), _stream()))
    return pred, loss, grad


def sfg_mpnn_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                  lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    n = params.numel()
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _chk(t, name, _F32, n)
    _check(lib().sfg_mpnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(params.numel()), int(step),
                               float(lr), float(beta1), float(beta2), float(eps), _stream()))


def sfg_mpnn_fit_norm(node_feats, edge_feats, targets):
    """Standardisation of a training set (lists of device tensors: raw n_i x 8 node features, raw e_i x 4
    edge features, e_i targets).  Returns (norm: 24 F32 in sfg_mpnn_features' layout, ystat: target mean
    and standard deviation as 2 F64), both on the device."""
    g = len(node_feats)
    if g < 1 or len(edge_feats) != g or len(targets) != g:
        raise ValueError("mpnn_fit_norm: one node, edge and target array per graph")
    for nf, ef, t in zip(node_feats, edge_feats, targets):
        if nf.dim() != 2 or int(nf.shape[1]) != 8 or ef.dim() != 2 or int(ef.shape[1]) != 4:
            raise ValueError("mpnn_fit_norm: node features are n x 8, edge features e x 4")
        _chk(nf, "node_feat", _F32)
        _chk(ef, "edge_feat", _F32)
        _chk(t, "target", _F32, int(ef.shape[0]))
    dev = node_feats[0].device
    norm = torch.empty(24, dtype=torch.float32, device=dev)
    ystat = torch.empty(2, dtype=torch.float64, device=dev)
    ws = _ws(sfg_workspace_bytes(OP_MPNN_NORM, 0, 0, 0, F64), dev)
    ptrs = (ctypes.c_void_p * g)(*[_ptr(t).value for t in node_feats])
    eptrs = (ctypes.c_void_p * g)(*[_ptr(t).value for t in edge_feats])
    tptrs = (ctypes.c_void_p * g)(*[_ptr(t).value for t in targets])
    nrows = (ctypes.c_int64 * g)(*[int(t.shape[0]) for t in node_feats])
    erows = (ctypes.c_int64 * g)(*[int(t.shape[0]) for t in edge_feats])
    _check(lib().sfg_mpnn_fit_norm(g, ptrs, nrows, eptrs, tptrs, erows, _ptr(norm), _ptr(ystat), _ptr(ws),
                                   ws.numel(), _stream()))
    return norm, ystat


def sfg_mpnn_standardize(y: torch.Tensor, ystat: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(y - mean) / std with the target statistics of sfg_mpnn_fit_norm."""
    _chk(y, "y", _F32)
    _chk(ystat, "ystat", _F64, 2)
    if out is None:
        out = torch.empty_like(y)
    _chk(out, "out", _F32, y.numel())
    _check(lib().sfg_mpnn_standardize(_ptr(y), int(y.numel()), _ptr(ystat), _ptr(out), _stream()))
    return out


def sfg_mpnn_save(path: str, params: torch.Tensor, norm: torch.Tensor, kc: int, tc: int, y_mean: float,
                  y_std: float) -> None:
    """Write a model file (the C ABI's format: versioned, shapes, FNV-1a hash)."""
    _chk(params, "params", _F32, sfg_mpnn_param_count())
    _chk(norm, "norm", _F32, 24)
    meta = MpnnMeta(int(kc), int(tc), float(y_mean), float(y_std))
    _check(lib().sfg_mpnn_save(os.fsencode(path), _ptr(params), _ptr(norm), ctypes.byref(meta), _stream()))


def sfg_mpnn_load(path: str, device="cuda"):
    """Read a model file.  Returns (params, norm) on the device and a dict with kc, tc, y_mean, y_std."""
    params = torch.empty(sfg_mpnn_param_count(), dtype=torch.float32, device=device)
    norm = torch.empty(24, dtype=torch.float32, device=device)
    meta = MpnnMeta()
    _check(lib().sfg_mpnn_load(os.fsencode(path), _ptr(params), _ptr(norm), ctypes.byref(meta), _stream()))
    return params, norm, {"kc": int(meta.kc), "tc": int(meta.tc), "y_mean": float(meta.y_mean),
                          "y_std": float(meta.y_std)}
