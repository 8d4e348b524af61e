"""Plain FP64 CPU oracle for st-HOSVD -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code.  The arithmetic lives in ``sthosvd_oracle.c`` (plain loops, double
precision, explicit matricization); this module only marshals numpy arrays.

Each function cites the part of the paper it follows:
  unfold / fold          Sec. II-A (mode-n matricization, tensorization)
  gram, ttt              Sec. II-A Eq. 3 (Gram = TTT(Y, Y)), Alg. 2 EIG branch
  ttm_t, ttm_tensor      Sec. II-A Eq. 2
  jacobi_eig             Alg. 2 EIG branch ("R_n leading eigenvectors")
  qr, right_solve_spd    Alg. 2 ALS branch (QR) and Alg. 3 (inverses)
  als_mode               Alg. 3 + Alg. 2 ALS branch
  sthosvd                Alg. 2 (mode-wise flexible st-HOSVD; Alg. 1 when all EIG)
  reconstruct            Sec. II-B (Tucker model)
  mlp_forward, mlp_loss_grad   the solver-selector cost model (Sec. IV analogue)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sthosvd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_numel.restype = ctypes.c_int64
        L.orc_sumsq.restype = ctypes.c_double
        L.orc_sumsq.argtypes = [ctypes.c_int64, _dp]
        L.orc_jacobi_eig.restype = ctypes.c_int
        L.orc_qr_householder.restype = ctypes.c_int
        L.orc_cholesky.restype = ctypes.c_int
        L.orc_right_solve_spd.restype = ctypes.c_int
        L.orc_als_mode.restype = ctypes.c_int
        L.orc_sthosvd.restype = ctypes.c_int
        L.orc_reconstruct.restype = ctypes.c_int
        L.orc_ttm_tensor.restype = ctypes.c_int
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and (a.flags.f_contiguous or a.ndim <= 1 or a.size <= 1)
    return a.ctypes.data_as(_dp)


def _dims(shape) -> ctypes.Array:
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def _f(a) -> np.ndarray:
    """float64, column-major copy (FP32 inputs are upcast exactly)."""
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(t: int) -> None:
    lib().orc_set_threads(ctypes.c_int(int(t)))


def sumsq(x) -> float:
    """Eq. 1 squared: sum of squares of all entries."""
    x = _f(x)
    return float(lib().orc_sumsq(ctypes.c_int64(x.size), _d(x.reshape(-1, order="F"))))


def unfold(X, n: int) -> np.ndarray:
    """Mode-n matricization (Sec. II-A); columns in Kolda order."""
    X = _f(X)
    In = X.shape[n]
    out = np.zeros((In, X.size // In), dtype=np.float64, order="F")
    lib().orc_unfold(ctypes.c_int(X.ndim), _dims(X.shape), ctypes.c_int(n), _d(X), _d(out))
    return out


def fold(Yn, shape, n: int) -> np.ndarray:
    """Tensorization, the inverse of unfold (Sec. II-A)."""
    Yn = _f(Yn)
    out = np.zeros(tuple(shape), dtype=np.float64, order="F")
    lib().orc_fold(ctypes.c_int(len(shape)), _dims(shape), ctypes.c_int(n), _d(Yn), _d(out))
    return out


def gram(Yn) -> np.ndarray:
    """S = Yn Yn^T (Alg. 2 EIG branch)."""
    Yn = _f(Yn)
    I, J = Yn.shape
    S = np.zeros((I, I), order="F")
    lib().orc_gram(ctypes.c_int64(I), ctypes.c_int64(J), _d(Yn), _d(S))
    return S


def ttt(Xn, Yn) -> np.ndarray:
    """Eq. 3 matricized: Z = X_(n) Y_(n)^T."""
    Xn, Yn = _f(Xn), _f(Yn)
    I, J = Xn.shape
    R = Yn.shape[0]
    assert Yn.shape[1] == J
    Z = np.zeros((I, R), order="F")
    lib().orc_ttt(ctypes.c_int64(I), ctypes.c_int64(R), ctypes.c_int64(J), _d(Xn), _d(Yn), _d(Z))
    return Z


def ttm_t(U, Yn) -> np.ndarray:
    """Eq. 2 matricized with the transpose of an I x R factor: U^T Yn."""
    U, Yn = _f(U), _f(Yn)
    I, R = U.shape
    J = Yn.shape[1]
    out = np.zeros((R, J), order="F")
    lib().orc_ttm_t(ctypes.c_int64(I), ctypes.c_int64(R), ctypes.c_int64(J), _d(U), _d(Yn), _d(out))
    return out


def ttm_tensor(X, A, n: int) -> np.ndarray:
    """Eq. 2 on a tensor: X x_n A with A of shape (rows, I_n)."""
    X, A = _f(X), _f(A)
    shape = list(X.shape)
    assert A.shape[1] == shape[n]
    oshape = list(shape)
    oshape[n] = A.shape[0]
    out = np.zeros(tuple(oshape), order="F")
    rc = lib().orc_ttm_tensor(ctypes.c_int(X.ndim), _dims(shape), ctypes.c_int(n),
                              ctypes.c_int64(A.shape[0]), _d(A), _d(X), _d(out))
    if rc != 0:
        raise MemoryError("oracle ttm_tensor")
    return out


def jacobi_eig(S, tol: float = 1e-15, max_sweeps: int = 50):
    """Cyclic Jacobi: (lam descending, V with the sign rule, sweeps)."""
    S = _f(S)
    n = S.shape[0]
    lam = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sw = lib().orc_jacobi_eig(ctypes.c_int64(n), _d(S), _d(lam), _d(V), ctypes.c_double(tol),
                              ctypes.c_int(max_sweeps))
    return lam, V, int(sw)


def qr(A):
    """Householder QR, diag(R) >= 0."""
    A = _f(A)
    m, n = A.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    rc = lib().orc_qr_householder(ctypes.c_int64(m), ctypes.c_int64(n), _d(A), _d(Q), _d(R))
    if rc != 0:
        raise ValueError("qr needs rows >= cols")
    return Q, R


def right_solve_spd(A, B):
    """X = B A^{-1} for SPD A (Cholesky solves)."""
    A, B = _f(A), _f(B)
    m, n = B.shape
    X = np.zeros((m, n), order="F")
    rc = lib().orc_right_solve_spd(ctypes.c_int64(m), ctypes.c_int64(n), _d(A), _d(B), _d(X))
    if rc != 0:
        raise np.linalg.LinAlgError("not SPD")
    return X


def als_mode(Yn, L0, iters: int = 5, variant: int = 0):
    """Alg. 3 + Alg. 2 ALS branch on a matricized tensor: (U, Ynew = R^ R_{k-1}^T)."""
    Yn, L0 = _f(Yn), _f(L0)
    I, J = Yn.shape
    R = L0.shape[1]
    U = np.zeros((I, R), order="F")
    Ynew = np.zeros((R, J), order="F")
    rc = lib().orc_als_mode(ctypes.c_int64(I), ctypes.c_int64(J), ctypes.c_int64(R), _d(Yn),
                            _d(L0), ctypes.c_int(iters), ctypes.c_int(variant), _d(U), _d(Ynew))
    if rc != 0:
        raise np.linalg.LinAlgError(f"oracle ALS failed ({rc})")
    return U, Ynew


def sthosvd(X, ranks, order=None, methods=None, L0=None, als_iters: int = 5,
            als_variant: int = 0, jacobi_tol: float = 1e-15, jacobi_max_sweeps: int = 50):
    """Alg. 2 in FP64.  Returns (G, [U_n], [lam_n or None])."""
    X = _f(X)
    N = X.ndim
    dims = list(X.shape)
    ranks = [int(r) for r in ranks]
    G = np.zeros(tuple(ranks), order="F")
    U = [np.zeros((dims[n], ranks[n]), order="F") for n in range(N)]
    lam = [np.zeros(dims[n]) for n in range(N)]
    Up = (_dp * N)(*[_d(u) for u in U])
    lp = (_dp * N)(*[_d(l) for l in lam])
    op = (ctypes.c_int * N)(*order) if order is not None else None
    mp = (ctypes.c_int * N)(*methods) if methods is not None else None
    if methods is not None and any(m == 1 for m in methods) and L0 is None:
        raise ValueError("ALS modes need their initial guesses L0 (Alg. 3 input)")
    if L0 is not None:
        L0 = [_f(l) if l is not None else np.zeros((dims[n], ranks[n]), order="F")
              for n, l in enumerate(L0)]
        L0p = (_dp * N)(*[_d(l) for l in L0])
    else:
        L0p = None
    rc = lib().orc_sthosvd(ctypes.c_int(N), _dims(dims), _dims(ranks), op, mp, L0p,
                           ctypes.c_int(als_iters), ctypes.c_int(als_variant), _d(X), _d(G),
                           Up, lp, ctypes.c_double(jacobi_tol), ctypes.c_int(jacobi_max_sweeps))
    if rc != 0:
        raise RuntimeError(f"oracle st-HOSVD failed ({rc})")
    meth = methods if methods is not None else [0] * N
    lam = [lam[n] if meth[n] == 0 else None for n in range(N)]
    return G, U, lam


def hooi(X, U0, sweeps: int = 1, jacobi_tol: float = 1e-15, jacobi_max_sweeps: int = 50):
    """Higher-order orthogonal iteration (De Lathauwer, De Moor and
    Vandewalle, 2000), the Tucker algorithm Sec. II-B names beside st-HOSVD
    and initializes from it.  Each sweep updates the factors in mode order:
    the tensor is projected onto the current factors of every other mode
    (Y = X x_m U_m^T, m != n, increasing m), and U_n becomes the R_n leading
    eigenvectors of the mode-n Gram of Y (the left singular vectors of
    Y_(n)), by the same cyclic Jacobi and sign rule as sthosvd.  Returns
    (G, [U_n]) with G = X x_1 U_1^T ... x_N U_N^T."""
    X = _f(X)
    N = X.ndim
    U = [_f(u).copy(order="F") for u in U0]
    for _ in range(sweeps):
        for n in range(N):
            Y = X
            for m in range(N):
                if m != n:
                    Y = ttm_tensor(Y, U[m].T, m)
            lam, V, _ = jacobi_eig(gram(unfold(Y, n)), jacobi_tol, jacobi_max_sweeps)
            U[n] = np.asfortranarray(V[:, :U[n].shape[1]])
    G = X
    for m in range(N):
        G = ttm_tensor(G, U[m].T, m)
    return G, U


def reconstruct(G, U) -> np.ndarray:
    """Tucker model X^ = G x_1 U1 ... x_N UN (Sec. II-B)."""
    G = _f(G)
    U = [_f(u) for u in U]
    N = G.ndim
    dims = [u.shape[0] for u in U]
    ranks = list(G.shape)
    Xh = np.zeros(tuple(dims), order="F")
    Up = (_dp * N)(*[_d(u) for u in U])
    rc = lib().orc_reconstruct(ctypes.c_int(N), _dims(dims), _dims(ranks), _d(G), Up, _d(Xh))
    if rc != 0:
        raise MemoryError("oracle reconstruct")
    return Xh


# ---------------------------------------------------------------- MLP ----

def _mlp_ptrs(Ws, bs):
    Ws = [_f(w) for w in Ws]
    bs = [_f(b).reshape(-1) for b in bs]
    nl = len(Ws)
    widths = [Ws[0].shape[1]] + [w.shape[0] for w in Ws]
    return Ws, bs, nl, widths


def mlp_forward(Ws, bs, X) -> np.ndarray:
    """Dense tanh MLP (linear output) on a batch X (features x B)."""
    Ws, bs, nl, widths = _mlp_ptrs(Ws, bs)
    X = _f(X)
    B = X.shape[1]
    acts = np.zeros(sum(widths[1:]) * B)
    Y = np.zeros((widths[-1], B), order="F")
    lib().orc_mlp_forward(ctypes.c_int(nl), (ctypes.c_int * (nl + 1))(*widths),
                          (_dp * nl)(*[_d(w) for w in Ws]), (_dp * nl)(*[_d(b) for b in bs]),
                          ctypes.c_int64(B), _d(X), _d(acts), _d(Y))
    return Y


def mlp_loss_grad(Ws, bs, X, T):
    """0.5/B * ||Y - T||^2 and its gradients (dW list, db list)."""
    Ws, bs, nl, widths = _mlp_ptrs(Ws, bs)
    X, T = _f(X), _f(T)
    B = X.shape[1]
    dW = [np.zeros_like(w, order="F") for w in Ws]
    db = [np.zeros_like(b) for b in bs]
    loss = lib().orc_mlp_loss_grad(ctypes.c_int(nl), (ctypes.c_int * (nl + 1))(*widths),
                                   (_dp * nl)(*[_d(w) for w in Ws]),
                                   (_dp * nl)(*[_d(b) for b in bs]), ctypes.c_int64(B), _d(X),
                                   _d(T), (_dp * nl)(*[_d(w) for w in dW]),
                                   (_dp * nl)(*[_d(b) for b in db]))
    return float(loss), dW, db
