"""Python binding of the st-HOSVD C ABI (argument marshalling only).

Every numeric step runs in libsthosvd.so's HIP kernels; PyTorch provides
device memory and the current stream.  Tensors are column-major (the first
index fastest): ``fortran_empty`` / ``to_device`` build such tensors, and
every entry point rejects tensors with other strides.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import PREC, SOLVER, check, i32arr, i64arr, ptrarr

__all__ = [
    "fortran_empty", "to_device", "to_numpy", "Plan", "sthosvd", "gram_mode_n", "ttt_mode_n",
    "ttm_mode_n", "ttm_mode_n_noalloc", "ttm_factor_prepare", "ttm_mode_n_prepared", "eig_leading", "tucker_reconstruct", "tucker_error", "sumsq", "mode_step",
    "selector_features", "selector_predict", "mlp_forward", "mlp_loss_grad", "mlp_adam",
    "BatchPlan",
]


# ----------------------------------------------------------- tensors ----

def fortran_empty(shape, dtype=torch.float32, device="cuda") -> torch.Tensor:
    shape = tuple(int(s) for s in shape)
    t = torch.empty(shape[::-1], dtype=dtype, device=device)
    return t.permute(*range(len(shape) - 1, -1, -1))


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """numpy array -> column-major device tensor with the same shape."""
    a = np.asfortranarray(a)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.permute(*range(a.ndim - 1, -1, -1))


def to_numpy(t: torch.Tensor) -> np.ndarray:
    """column-major device tensor -> numpy (Fortran order)."""
    c = t.permute(*range(t.dim() - 1, -1, -1)).contiguous().cpu().numpy()
    return np.asfortranarray(c.T)


def _is_fortran(t: torch.Tensor) -> bool:
    s = 1
    for k in range(t.dim()):
        if t.shape[k] > 1 and t.stride(k) != s:
            return False
        s *= t.shape[k]
    return True


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.STH_F64
    if t.dtype == torch.float32:
        return _lib.STH_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _need(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not _is_fortran(t):
        raise ValueError(f"{name} must be column-major (first index fastest)")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


# --------------------------------------------------------------- plan ----

class Plan:
    """sthosvd_plan: host-side shape work, solver choice and workspace size."""

    def __init__(self, dims: Sequence[int], ranks: Sequence[int], dtype=torch.float32,
                 gram_prec="fp32", ttm_prec="fp32", solver="eig", per_mode=None,
                 mode_order=None, als_iters: int = 5, eig_max_sweeps: int = 0,
                 workspace_cap: int = 0, mlp_weights: Optional[np.ndarray] = None):
        L = _lib.load()
        self.dims = [int(d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.N = len(self.dims)
        self.dtype = dtype
        self._keep = [i64arr(self.dims), i64arr(self.ranks)]
        d = _lib.sth_desc()
        d.order = self.N
        d.dims = ctypes.cast(self._keep[0], ctypes.POINTER(ctypes.c_int64))
        d.ranks = ctypes.cast(self._keep[1], ctypes.POINTER(ctypes.c_int64))
        if mode_order is not None:
            mo = i32arr(mode_order)
            self._keep.append(mo)
            d.mode_order = ctypes.cast(mo, ctypes.POINTER(ctypes.c_int32))
        d.dtype = _lib.STH_F64 if dtype == torch.float64 else _lib.STH_F32
        d.gram_prec = _prec(gram_prec)
        d.ttm_prec = _prec(ttm_prec)
        d.solver = SOLVER[solver] if isinstance(solver, str) else int(solver)
        if per_mode is not None:
            pm = i32arr([SOLVER[s] if isinstance(s, str) else int(s) for s in per_mode])
            self._keep.append(pm)
            d.per_mode = ctypes.cast(pm, ctypes.POINTER(ctypes.c_int32))
        d.als_iters = int(als_iters)
        d.eig_max_sweeps = int(eig_max_sweeps)
        d.workspace_cap = int(workspace_cap)
        if mlp_weights is not None:
            w = np.ascontiguousarray(mlp_weights, dtype=np.float32)
            self._keep.append(w)
            d.mlp_weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._desc = d
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(L.sthosvd_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws)))
        self._h = h
        self.workspace_bytes = int(ws.value)
        out = (ctypes.c_int32 * self.N)()
        check(L.sthosvd_plan_solvers(h, out))
        self.solvers = [int(v) for v in out]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().sthosvd_plan_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def run(self, X: torch.Tensor, G: torch.Tensor, U: List[torch.Tensor],
            workspace: torch.Tensor, eigvals: Optional[List[Optional[torch.Tensor]]] = None,
            als_init: Optional[List[Optional[torch.Tensor]]] = None, seed: int = 0) -> None:
        """sthosvd_run: enqueue the decomposition on the current stream."""
        L = _lib.load()
        _need(X, "X")
        _need(G, "core")
        Up = ptrarr([u.data_ptr() for u in U])
        ep = ptrarr([e.data_ptr() if e is not None else 0 for e in eigvals]) if eigvals else None
        ap = ptrarr([a.data_ptr() if a is not None else 0 for a in als_init]) if als_init else None
        check(L.sthosvd_run(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                            Up, ep, ap, ctypes.c_uint64(seed), ctypes.c_void_p(workspace.data_ptr()),
                            ctypes.c_size_t(workspace.numel()), _stream()))

    def check(self, workspace: torch.Tensor) -> None:
        check(_lib.load().sthosvd_check(self._h, ctypes.c_void_p(workspace.data_ptr()), _stream()))


def sthosvd(X: torch.Tensor, ranks: Sequence[int], gram_prec="fp32", ttm_prec="fp32",
            solver="eig", per_mode=None, mode_order=None, als_iters: int = 5,
            als_init=None, seed: int = 0, return_eigvals: bool = False, check_numeric=True):
    """Alg. 2 on the device: returns (G, [U_n], [eigvals_n or None])."""
    _need(X, "X")
    plan = Plan(X.shape, ranks, X.dtype, gram_prec, ttm_prec, solver, per_mode, mode_order,
                als_iters)
    dev = X.device
    G = fortran_empty(plan.ranks, X.dtype, dev)
    U = [fortran_empty((X.shape[n], plan.ranks[n]), torch.float64, dev) for n in range(plan.N)]
    ev = [torch.empty(plan.ranks[n], dtype=torch.float64, device=dev) for n in range(plan.N)] \
        if return_eigvals else None
    ws = _ws(plan.workspace_bytes, dev)
    if als_init is not None:
        als_init = [a if a is None or isinstance(a, torch.Tensor) else to_device(a, dev)
                    for a in als_init]
    plan.run(X, G, U, ws, ev, als_init, seed)
    if check_numeric:
        plan.check(ws)
    if ev is not None:
        ev = [ev[n] if plan.solvers[n] == SOLVER["eig"] else None for n in range(plan.N)]
    return G, U, ev


# ------------------------------------------------------ building blocks ----

def gram_mode_n(Y: torch.Tensor, n: int, prec="fp32") -> torch.Tensor:
    """Mode-n Gram S = Y_(n) Y_(n)^T (FP64 I_n x I_n)."""
    _need(Y, "Y")
    L = _lib.load()
    dims = i64arr(Y.shape)
    S = fortran_empty((Y.shape[n], Y.shape[n]), torch.float64, Y.device)
    nb = L.gram_mode_n_workspace(Y.dim(), dims, n, 0)
    ws = _ws(nb, Y.device)
    check(L.gram_mode_n(Y.dim(), dims, n, _dtype_code(Y), _prec(prec), ctypes.c_void_p(Y.data_ptr()),
                        ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                        _stream()))
    return S


def ttt_mode_n(Y: torch.Tensor, Z: torch.Tensor, n: int, prec="fp32") -> torch.Tensor:
    """Mode-n TTT P = Y_(n) Z_(n)^T (FP64 I_n x R)."""
    _need(Y, "Y")
    _need(Z, "Z")
    R = Z.shape[n]
    for k in range(Y.dim()):
        if k != n and Y.shape[k] != Z.shape[k]:
            raise ValueError("Y and Z differ outside mode n")
    L = _lib.load()
    dims = i64arr(Y.shape)
    P = fortran_empty((Y.shape[n], R), torch.float64, Y.device)
    nb = L.gram_mode_n_workspace(Y.dim(), dims, n, R)
    ws = _ws(nb, Y.device)
    check(L.ttt_mode_n(Y.dim(), dims, n, R, _dtype_code(Y), _prec(prec), ctypes.c_void_p(Y.data_ptr()),
                       ctypes.c_void_p(Z.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return P


def ttm_mode_n(Y: torch.Tensor, U: torch.Tensor, n: int, prec="fp32",
               transpose_u: bool = False) -> torch.Tensor:
    """Z = Y x_n U^T for an I_n x R factor U (transpose_u: U is R x I_n, Z = Y x_n U)."""
    _need(Y, "Y")
    _need(U, "U")
    if U.dtype != torch.float64:
        raise TypeError("factors are FP64")
    In = Y.shape[n]
    if transpose_u:
        R, k = U.shape
    else:
        k, R = U.shape
    if k != In:
        raise ValueError("factor does not match mode n")
    L = _lib.load()
    dims = i64arr(Y.shape)
    oshape = list(Y.shape)
    oshape[n] = R
    Z = fortran_empty(oshape, Y.dtype, Y.device)
    ws = _ws(L.ttm_mode_n_workspace(In, R), Y.device)
    check(L.ttm_mode_n(Y.dim(), dims, n, R, _dtype_code(Y), _prec(prec), ctypes.c_void_p(Y.data_ptr()),
                       ctypes.c_void_p(U.data_ptr()), 1 if transpose_u else 0,
                       ctypes.c_void_p(Z.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                       _stream()))
    return Z


def ttm_mode_n_noalloc(Y: torch.Tensor, U: torch.Tensor, n: int, prec="fp32",
                       transpose_u: bool = False, out: torch.Tensor = None) -> torch.Tensor:
    """ttm_mode_n without a workspace: the library keeps the pre-split factor in
    its own per-device scratch.  `out` (column-major, the dims of Y with
    dims[n] = R) is written when given, so a caller can allocate nothing."""
    _need(Y, "Y")
    _need(U, "U")
    if U.dtype != torch.float64:
        raise TypeError("factors are FP64")
    In = Y.shape[n]
    R, k = U.shape if transpose_u else U.shape[::-1]
    if k != In:
        raise ValueError("factor does not match mode n")
    L = _lib.load()
    oshape = list(Y.shape)
    oshape[n] = R
    Z = out if out is not None else fortran_empty(oshape, Y.dtype, Y.device)
    if list(Z.shape) != oshape or Z.dtype != Y.dtype:
        raise ValueError("out has the wrong shape or dtype")
    _need(Z, "out")
    check(L.ttm_mode_n_noalloc(Y.dim(), i64arr(Y.shape), n, R, _dtype_code(Y), _prec(prec),
                               ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                               1 if transpose_u else 0, ctypes.c_void_p(Z.data_ptr()), _stream()))
    return Z


def ttm_factor_prepare(U: torch.Tensor, prec="fp32", transpose_u: bool = False) -> torch.Tensor:
    """Splits an FP64 factor once for ttm_mode_n_prepared (opaque uint8 device buffer)."""
    _need(U, "U")
    if U.dtype != torch.float64:
        raise TypeError("factors are FP64")
    R, k = U.shape if transpose_u else U.shape[::-1]
    L = _lib.load()
    nbytes = L.ttm_factor_bytes(k, R, _prec(prec))
    out = torch.empty(nbytes, dtype=torch.uint8, device=U.device)
    check(L.ttm_factor_prepare(k, R, _prec(prec), ctypes.c_void_p(U.data_ptr()), 1 if transpose_u else 0,
                               ctypes.c_void_p(out.data_ptr()), out.numel(), _stream()))
    return out


def ttm_mode_n_prepared(Y: torch.Tensor, Uprep: torch.Tensor, n: int, R: int, prec="fp32",
                        out: torch.Tensor = None) -> torch.Tensor:
    """ttm_mode_n with a factor from ttm_factor_prepare (one kernel launch).  `out`
    (column-major, the dims of Y with dims[n] = R) is written when given."""
    _need(Y, "Y")
    _need(Uprep, "Uprep")
    L = _lib.load()
    oshape = list(Y.shape)
    oshape[n] = R
    Z = out if out is not None else fortran_empty(oshape, Y.dtype, Y.device)
    if list(Z.shape) != oshape or Z.dtype != Y.dtype:
        raise ValueError("out has the wrong shape or dtype")
    _need(Z, "out")
    check(L.ttm_mode_n_prepared(Y.dim(), i64arr(Y.shape), n, R, _dtype_code(Y), _prec(prec),
                                ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(Uprep.data_ptr()),
                                Uprep.numel(), ctypes.c_void_p(Z.data_ptr()), _stream()))
    return Z


def eig_leading(S: torch.Tensor, R: int, max_sweeps: int = 0, s_unit: float = 0.0):
    """R leading eigenpairs of a symmetric FP64 matrix: (U n x R, lam R, ws).
    s_unit: unit roundoff with which S was formed (eig_leading_ex)."""
    _need(S, "S")
    L = _lib.load()
    n = S.shape[0]
    U = fortran_empty((n, R), torch.float64, S.device)
    lam = torch.empty(R, dtype=torch.float64, device=S.device)
    ws = _ws(L.eig_leading_workspace(n), S.device)
    check(L.eig_leading_ex(n, R, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                           ctypes.c_void_p(lam.data_ptr()), max_sweeps, ctypes.c_double(s_unit),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return U, lam, ws


def tucker_reconstruct(G: torch.Tensor, U: List[torch.Tensor], prec="fp32") -> torch.Tensor:
    """X^ = G x_1 U1 ... x_N UN."""
    _need(G, "G")
    L = _lib.load()
    dims = [u.shape[0] for u in U]
    ranks = list(G.shape)
    Xh = fortran_empty(dims, G.dtype, G.device)
    da, ra = i64arr(dims), i64arr(ranks)
    ws = _ws(L.tucker_reconstruct_workspace(G.dim(), da, ra, _dtype_code(G)), G.device)
    check(L.tucker_reconstruct(G.dim(), da, ra, _dtype_code(G), _prec(prec),
                               ctypes.c_void_p(G.data_ptr()), ptrarr([u.data_ptr() for u in U]),
                               ctypes.c_void_p(Xh.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream()))
    return Xh


def hooi(X: torch.Tensor, U: List[torch.Tensor], sweeps: int = 1, gram_prec="fp64", ttm_prec="fp32",
         check_flag: bool = True):
    """HOOI refinement in place: U (device FP64 I_n x R_n, orthonormal
    columns, e.g. st-HOSVD's) are updated by `sweeps` sweeps; returns the
    core X x_1 U_1^T ... x_N U_N^T (and the workspace)."""
    _need(X, "X")
    L = _lib.load()
    ranks = [int(u.shape[1]) for u in U]
    da, ra = i64arr(X.shape), i64arr(ranks)
    G = fortran_empty(ranks, X.dtype, X.device)
    ws = _ws(L.sth_hooi_workspace(X.dim(), da, ra, _dtype_code(X), _prec(ttm_prec)), X.device)
    check(L.sth_hooi(X.dim(), da, ra, _dtype_code(X), _prec(gram_prec), _prec(ttm_prec),
                     ctypes.c_void_p(X.data_ptr()), ptrarr([u.data_ptr() for u in U]),
                     ctypes.c_void_p(G.data_ptr()), sweeps, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                     _stream()))
    if check_flag:
        check(L.sth_hooi_check(ctypes.c_void_p(ws.data_ptr()), _stream()))
    return G, ws


def tucker_error(X: torch.Tensor, G: torch.Tensor, U: List[torch.Tensor], prec="fp32"):
    """(||X - X^||^2, ||X||^2) accumulated in FP64 on the device."""
    _need(X, "X")
    _need(G, "G")
    L = _lib.load()
    da, ra = i64arr(X.shape), i64arr(G.shape)
    out = torch.zeros(2, dtype=torch.float64, device=X.device)
    ws = _ws(L.tucker_error_workspace(X.dim(), da, ra, _dtype_code(X)), X.device)
    check(L.tucker_error(X.dim(), da, ra, _dtype_code(X), _prec(prec), ctypes.c_void_p(X.data_ptr()),
                         ctypes.c_void_p(G.data_ptr()), ptrarr([u.data_ptr() for u in U]),
                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                         _stream()))
    return out


def sumsq(x: torch.Tensor) -> torch.Tensor:
    """FP64 sum of squares of a device tensor (Eq. 1 squared)."""
    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    L = _lib.load()
    out = torch.zeros(1, dtype=torch.float64, device=x.device)
    ws = _ws(8 * 1024, x.device)
    check(L.sth_sumsq(_dtype_code(x), ctypes.c_void_p(x.data_ptr()), x.numel(),
                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                      _stream()))
    return out


# ---------------------------------------------------------- one mode ----

def mode_step(Y: torch.Tensor, n: int, R: int, solver="eig", gram_prec="fp32", ttm_prec="fp32",
              als_iters: int = 5, als_init=None, seed: int = 0, out=None, workspace=None):
    """One mode of Alg. 2 on Y: returns (Z, U, eigvals or None, workspace)."""
    _need(Y, "Y")
    L = _lib.load()
    dims = i64arr(Y.shape)
    sv = SOLVER[solver] if isinstance(solver, str) else int(solver)
    dt = _dtype_code(Y)
    gp, tp = _prec(gram_prec), _prec(ttm_prec)
    if dt == _lib.STH_F64:
        gp = tp = PREC["fp64"]
    nb = L.sthosvd_mode_step_workspace(Y.dim(), dims, n, R, dt, gp, tp, sv, als_iters)
    if nb == 0:
        raise _lib.SthError(_lib.STH_ERR_INVALID, L.sth_last_error().decode())
    oshape = list(Y.shape)
    oshape[n] = R
    Z = out if out is not None else fortran_empty(oshape, Y.dtype, Y.device)
    U = fortran_empty((Y.shape[n], R), torch.float64, Y.device)
    ev = torch.empty(R, dtype=torch.float64, device=Y.device) if sv == 0 else None
    ws = workspace if workspace is not None and workspace.numel() >= nb else _ws(nb, Y.device)
    ai = None
    if als_init is not None:
        ai = als_init if isinstance(als_init, torch.Tensor) else to_device(als_init, Y.device)
    check(L.sthosvd_mode_step(Y.dim(), dims, n, R, dt, gp, tp, sv, als_iters,
                              ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(Z.data_ptr()),
                              ctypes.c_void_p(U.data_ptr()),
                              ctypes.c_void_p(ev.data_ptr()) if ev is not None else None,
                              ctypes.c_void_p(ai.data_ptr()) if ai is not None else None,
                              ctypes.c_uint64(seed), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream()))
    return Z, U, ev, ws


def choose_exhaustive(X: torch.Tensor, ranks: Sequence[int], gram_prec="fp32", ttm_prec="fp32",
                      als_iters: int = 5):
    """sthosvd_choose_exhaustive: the per-mode solver by timing both steps on
    X (Sec. IV-B).  Returns (["eig" | "als"] per mode, [(eig_ms, als_ms)]
    per mode, -1 where a step did not count).  Synchronizes the stream."""
    _need(X, "X")
    L = _lib.load()
    N = X.dim()
    dims, rk = i64arr(X.shape), i64arr(ranks)
    dt = _dtype_code(X)
    gp, tp = _prec(gram_prec), _prec(ttm_prec)
    if dt == _lib.STH_F64:
        gp = tp = PREC["fp64"]
    nb = L.sthosvd_choose_exhaustive_workspace(N, dims, rk, dt, gp, tp, als_iters)
    if nb == 0:
        raise _lib.SthError(_lib.STH_ERR_INVALID, L.sth_last_error().decode())
    ws = _ws(nb, X.device)
    out = (ctypes.c_int32 * N)()
    ms = (ctypes.c_float * (2 * N))()
    check(L.sthosvd_choose_exhaustive(N, dims, rk, dt, gp, tp, als_iters, ctypes.c_void_p(X.data_ptr()), out,
                                      ms, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    names = ["eig", "als"]
    return [names[v] for v in out], [(ms[2 * n], ms[2 * n + 1]) for n in range(N)]


# -------------------------------------------------- learned selector ----

def selector_num_params() -> int:
    return int(_lib.load().sth_selector_num_params())


def selector_num_trainable() -> int:
    return int(_lib.load().sth_selector_num_trainable())


def selector_features(I: int, R: int, J: int) -> np.ndarray:
    out = np.zeros(10, dtype=np.float32)
    check(_lib.load().sth_selector_features(I, R, J, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def selector_predict(I: int, R: int, J: int, weights: Optional[np.ndarray] = None) -> np.ndarray:
    out = np.zeros(2, dtype=np.float32)
    wp = None
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.float32)
        wp = weights.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    check(_lib.load().sth_selector_predict(wp, I, R, J, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def selector_choose(I: int, R: int, J: int, weights: Optional[np.ndarray] = None) -> str:
    """The solver sthosvd_plan picks for a mode under solver="auto"."""
    out = ctypes.c_int32()
    wp = None
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.float32)
        wp = weights.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    check(_lib.load().sth_selector_choose(wp, I, R, J, ctypes.byref(out)))
    return "als" if out.value == SOLVER["als"] else "eig"


def selector_tree_choose(I: int, R: int, J: int) -> str:
    """The solver sthosvd_plan picks for a mode under solver="auto_tree"."""
    out = ctypes.c_int32()
    check(_lib.load().sth_selector_tree_choose(I, R, J, ctypes.byref(out)))
    return "als" if out.value == SOLVER["als"] else "eig"


def mlp_forward(params: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Y (2 x B) of the selector network on device features X (10 x B)."""
    L = _lib.load()
    B = X.shape[1]
    Y = torch.empty((B, 2), dtype=torch.float32, device=X.device).t()
    ws = _ws(L.sth_mlp_workspace(B), X.device)
    check(L.sth_mlp_forward(ctypes.c_void_p(params.data_ptr()), B, ctypes.c_void_p(X.data_ptr()),
                            ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream()))
    return Y


def mlp_loss_grad(params: torch.Tensor, X: torch.Tensor, T: torch.Tensor, workspace=None):
    """(loss tensor [1], grad tensor [num_params]) of 0.5/B ||Y - T||^2."""
    L = _lib.load()
    B = X.shape[1]
    grad = torch.empty_like(params)
    loss = torch.empty(4, dtype=torch.float32, device=X.device)
    nb = L.sth_mlp_workspace(B)
    ws = workspace if workspace is not None and workspace.numel() >= nb else _ws(nb, X.device)
    check(L.sth_mlp_loss_grad(ctypes.c_void_p(params.data_ptr()), B, ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream()))
    return loss[:1], grad


def mlp_adam(params, grad, m, v, count: int, lr: float, step: int, beta1=0.9, beta2=0.999,
             eps=1e-8) -> None:
    check(_lib.load().sth_mlp_adam(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                   ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), count,
                                   lr, beta1, beta2, eps, step, _stream()))


# ----------------------------------------------------------- batched ----

class BatchPlan:
    """sthosvd_plan_batched over a list of (dims, ranks) of FP32 tensors."""

    def __init__(self, shapes, gram_prec="bf16x6", ttm_prec="bf16x3", eig_max_sweeps: int = 0,
                 tiles=None):
        """tiles: None (defaults) or (gram_wg_per_cu, gram_wt_max, ttm_rows_per_wave)."""
        L = _lib.load()
        self.tiles = tuple(int(v) for v in tiles) if tiles is not None else None
        self.shapes = [([int(x) for x in d], [int(x) for x in r]) for d, r in shapes]
        self.count = len(self.shapes)
        self.N = len(self.shapes[0][0])
        self._keep = []
        descs = (_lib.sth_desc * self.count)()
        for t, (d, r) in enumerate(self.shapes):
            da, ra = i64arr(d), i64arr(r)
            self._keep += [da, ra]
            descs[t].order = len(d)
            descs[t].dims = ctypes.cast(da, ctypes.POINTER(ctypes.c_int64))
            descs[t].ranks = ctypes.cast(ra, ctypes.POINTER(ctypes.c_int64))
            descs[t].dtype = _lib.STH_F32
            descs[t].gram_prec = _prec(gram_prec)
            descs[t].ttm_prec = _prec(ttm_prec)
            descs[t].solver = SOLVER["eig"]
            descs[t].eig_max_sweeps = int(eig_max_sweeps)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        tl = None
        if self.tiles is not None:
            tl = _lib.sth_batch_tiles(*self.tiles, 0)
        check(L.sthosvd_plan_batched_tiles(descs, self.count, ctypes.byref(tl) if tl is not None else None,
                                           ctypes.byref(h), ctypes.byref(ws)))
        self._h = h
        self.workspace_bytes = int(ws.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().sthosvd_plan_batched_destroy(h)
            except Exception:
                pass
            self._h = None

    def outputs(self, device="cuda"):
        """Allocates (cores, factors, pointer arrays) for a run."""
        G = [fortran_empty(r, torch.float32, device) for _, r in self.shapes]
        U = [[fortran_empty((d[n], r[n]), torch.float64, device) for n in range(self.N)]
             for d, r in self.shapes]
        cp = torch.tensor([g.data_ptr() for g in G], dtype=torch.int64, device=device)
        up = torch.tensor([u.data_ptr() for us in U for u in us], dtype=torch.int64, device=device)
        return G, U, cp, up

    def run(self, Xptrs: torch.Tensor, Cptrs: torch.Tensor, Uptrs: torch.Tensor,
            workspace: torch.Tensor) -> None:
        check(_lib.load().sthosvd_run_batched(self._h, ctypes.c_void_p(Xptrs.data_ptr()),
                                              ctypes.c_void_p(Cptrs.data_ptr()),
                                              ctypes.c_void_p(Uptrs.data_ptr()),
                                              ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                              _stream()))

    def check(self, workspace: torch.Tensor) -> None:
        check(_lib.load().sthosvd_check_batched(self._h, ctypes.c_void_p(workspace.data_ptr()),
                                                _stream()))
