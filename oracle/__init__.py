"""CPU float64 oracle for the sparse CG path — TEST INFRASTRUCTURE ONLY.

Thin numpy/ctypes wrapper over `oracle.c` (plain sequential C, compiled
without FMA contraction).  Only `tests/`, the package smoke check and the CPU
baseline leg of `bench.py` may import this package; the GPU library neither
imports it nor shares code with it.

Each function follows a passage of the paper (arXiv 2112.10823):
  csr_check, spmv        Section 2.3 (CSR storage) and Table "SpMV with CSR format"
  add, axpy              Table "Addition of vectors" (labelled daxpy)
  xmul                   Table "Element wise product"
  dot                    Table "Dot product" (Kahan-compensated, index order)
  cg                     Section 5.3, classical CG (Saad's textbook recurrences)
  cg(jacobi=True)        CG with diagonal preconditioning (not in the paper)
  mixed_ir               mixed-precision iterative refinement (reference cited
                         beside CG in Section 5.3)
  lanczos_extremes       extreme Ritz values from CG coefficients (Saad 6.7)
  schwarz.solve          CG under an additive Schwarz preconditioner with CG
                         subdomain solves (domain decomposition, end of
                         Section 5.3; module `oracle.schwarz`)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")  # timing build (all cores)
_libs: dict = {}

OK, EINVAL, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, -1, -4, -5, -6


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double)]


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iters: int
    outer_iters: int
    relres: float
    relres_true: float
    alpha: np.ndarray | None = None
    beta: np.ndarray | None = None
    relres_hist: np.ndarray | None = None  # ||r_k|| / ||b||, k = 0 .. iters


def _load(path: str = _LIB_PATH):
    if path not in _libs:
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_csr_check.argtypes = [i64, i64, i64, i32p, i32p]
        lib.oracle_csr_check.restype = i64
        lib.oracle_add.argtypes = [i64, f64p, f64p, f64p]
        lib.oracle_axpy.argtypes = [i64, dbl, f64p, f64p]
        lib.oracle_xmul.argtypes = [i64, f64p, f64p, f64p]
        lib.oracle_dot.argtypes = [i64, f64p, f64p]
        lib.oracle_dot.restype = dbl
        lib.oracle_dot_f32.argtypes = [i64, f32p, f32p]
        lib.oracle_dot_f32.restype = ctypes.c_float
        lib.oracle_spmv.argtypes = [i64, i32p, i32p, f64p, f64p, f64p]
        lib.oracle_spmv_f32.argtypes = [i64, i32p, i32p, f32p, f32p, f32p]
        lib.oracle_inv_diag.argtypes = [i64, i32p, i32p, f64p, f64p]
        lib.oracle_inv_diag.restype = i64
        lib.oracle_cg.argtypes = [i64, i32p, i32p, f64p, f64p, f64p, dbl, i32, i32,
                                  ctypes.POINTER(_Stats), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]
        lib.oracle_cg.restype = ctypes.c_int
        lib.oracle_mixed_ir.argtypes = [i64, i32p, i32p, f64p, f32p, f64p, f64p, dbl, dbl, i32,
                                        i32, i32, ctypes.POINTER(_Stats)]
        lib.oracle_mixed_ir.restype = ctypes.c_int
        for name, lp in (("oracle_mixed_ru", f32p), ("oracle_mixed_ru_f64", f64p)):
            fn = getattr(lib, name)
            fn.argtypes = [i64, i32p, i32p, f64p, lp, f64p, f64p, dbl, dbl, i32, i32,
                           ctypes.POINTER(_Stats), ctypes.c_void_p]
            fn.restype = ctypes.c_int
        for name, lp in (("oracle_mixed_ru_block", f32p), ("oracle_mixed_ru_block_f64", f64p)):
            fn = getattr(lib, name)
            fn.argtypes = [i64, i32p, i32p, f64p, lp, i32, f64p, f64p, dbl, dbl, i32, i32,
                           ctypes.POINTER(_Stats)]
            fn.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _libs[path] = lib
    return _libs[path]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def from_one_based(ia, ja, aa):
    """Convert the paper's 1-based CSR triple (IA, JA, AA) to 0-based arrays."""
    return (_i32(np.asarray(ia) - 1), _i32(np.asarray(ja) - 1), _f64(aa))


def csr_check(n_rows, n_cols, row_ptr, col_idx) -> int:
    """0 if (row_ptr, col_idx) is a valid 0-based CSR pattern, else nonzero."""
    row_ptr, col_idx = _i32(row_ptr), _i32(col_idx)
    if row_ptr.size != n_rows + 1:
        return -1
    nnz = int(row_ptr[-1]) if row_ptr.size else 0
    if col_idx.size < nnz:
        return -1
    return int(_load().oracle_csr_check(n_rows, n_cols, col_idx.size, row_ptr, col_idx))


def add(x, y):
    x, y = _f64(x), _f64(y)
    z = np.empty_like(x)
    _load().oracle_add(x.size, x, y, z)
    return z


def axpy(alpha, x, y):
    """Returns fma(alpha, x, y) elementwise (y is not modified)."""
    x = _f64(x)
    out = _f64(y).copy()
    _load().oracle_axpy(x.size, float(alpha), x, out)
    return out


def xmul(x, y):
    x, y = _f64(x), _f64(y)
    z = np.empty_like(x)
    _load().oracle_xmul(x.size, x, y, z)
    return z


def dot(x, y) -> float:
    x, y = _f64(x), _f64(y)
    return float(_load().oracle_dot(x.size, x, y))


def dot_f32(x, y) -> float:
    x, y = _f32(x), _f32(y)
    return float(_load().oracle_dot_f32(x.size, x, y))


def spmv(A, x):
    """y = A x for a CSR object with row_ptr / col_idx / val / n_rows."""
    x = _f64(x)
    y = np.empty(A.n_rows, np.float64)
    _load().oracle_spmv(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val), x, y)
    return y


def spmv_f32(A, val32, x32):
    x32 = _f32(x32)
    y = np.empty(A.n_rows, np.float32)
    _load().oracle_spmv_f32(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f32(val32), x32, y)
    return y


def inv_diag(A):
    d = np.empty(A.n_rows, np.float64)
    bad = _load().oracle_inv_diag(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val), d)
    if bad:
        raise ValueError(f"row {bad - 1} has no positive diagonal entry")
    return d


def timing_threads() -> int:
    """Threads of the all-cores timing build (OpenMP; OMP_NUM_THREADS applies)."""
    return int(_load(_OMP_PATH).oracle_threads())


def cg_timing(A, b, rtol=1e-8, maxit=0, jacobi=False) -> SolveResult:
    """The same CG from the all-cores timing build of oracle.c (rows and
    elements in parallel, per-thread compensated dot partials): for the CPU
    baseline's timing only, never for parity."""
    b = _f64(b)
    x = np.zeros(A.n_rows)
    st = _Stats()
    _load(_OMP_PATH).oracle_cg(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val), b, x,
                               float(rtol), int(maxit), int(bool(jacobi)), ctypes.byref(st),
                               None, None, None)
    return SolveResult(x, st.status, st.iters, 0, st.relres, st.relres_true)


def cg(A, b, x0=None, rtol=1e-8, maxit=0, jacobi=False, history=False) -> SolveResult:
    """Classical (optionally Jacobi-preconditioned) CG; see oracle.c."""
    b = _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    st = _Stats()
    cap = maxit if maxit > 0 else A.n_rows
    ah = np.zeros(max(cap, 1)) if history else None
    bh = np.zeros(max(cap, 1)) if history else None
    rh = np.full(max(cap, 1) + 1, np.nan) if history else None
    _load().oracle_cg(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val), b, x, float(rtol),
                      int(maxit), int(bool(jacobi)), ctypes.byref(st),
                      ah.ctypes.data if history else None, bh.ctypes.data if history else None,
                      rh.ctypes.data if history else None)
    res = SolveResult(x, st.status, st.iters, 0, st.relres, st.relres_true)
    if history:
        res.alpha = ah[:st.iters].copy()
        res.beta = bh[:max(st.iters - 1, 0)].copy()
        res.relres_hist = rh[:st.iters + 1].copy()
    return res


def mixed_ru(A, val32, b, x0=None, rtol=1e-10, delta=0.1, maxit=0, jacobi=False,
             history=False, inner_f64=False) -> SolveResult:
    """CG iterating in binary32 with float64 reliable updates (the true
    residual, the solution and the stopping test in float64, the Krylov space
    kept across updates); see mixed_ru.inc.  outer_iters = reliable updates.
    inner_f64: the same steps iterating in float64 (val32 ignored), for tests."""
    b = _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    st = _Stats()
    cap = maxit if maxit > 0 else A.n_rows
    rh = np.full(cap + 1, np.nan) if history else None
    lib = _load()
    if inner_f64:
        lib.oracle_mixed_ru_f64(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val),
                                _f64(A.val), b, x, float(rtol), float(delta), int(maxit),
                                int(bool(jacobi)), ctypes.byref(st),
                                rh.ctypes.data if history else None)
    else:
        lib.oracle_mixed_ru(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val),
                            _f32(val32), b, x, float(rtol), float(delta), int(maxit),
                            int(bool(jacobi)), ctypes.byref(st),
                            rh.ctypes.data if history else None)
    res = SolveResult(x, st.status, st.iters, st.outer_iters, st.relres, st.relres_true)
    if history:
        res.relres_hist = rh[:st.iters + 1].copy()
    return res


def mixed_ir(A, val32, b, x0=None, rtol=1e-10, tau=1e-3, inner_maxit=0, max_outer=50,
             jacobi=False):
    """FP64 iterative refinement around a binary32 inner CG (optionally
    Jacobi-preconditioned); see oracle.c."""
    b = _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    st = _Stats()
    _load().oracle_mixed_ir(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val), _f32(val32),
                            b, x, float(rtol), float(tau), int(inner_maxit), int(max_outer),
                            int(bool(jacobi)), ctypes.byref(st))
    return SolveResult(x, st.status, st.iters, st.outer_iters, st.relres, st.relres_true)


def mixed_ru_block(A, val32, B, X0=None, rtol=1e-10, delta=0.1, maxit=0, jacobi=False,
                   inner_f64=False):
    """mixed_ru for the k rows of B (right-hand sides of A) in step, an
    update of one taken by all (see mixed_ru_block.inc).  Returns one
    SolveResult per right-hand side (outer_iters = reliable updates)."""
    B = np.ascontiguousarray(np.atleast_2d(B), dtype=np.float64)
    k, n = B.shape
    X = np.zeros((k, n)) if X0 is None else np.ascontiguousarray(X0, dtype=np.float64).copy()
    st = (_Stats * k)()
    lib = _load()
    if inner_f64:
        lib.oracle_mixed_ru_block_f64(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val),
                                      _f64(A.val), int(k), B, X, float(rtol), float(delta),
                                      int(maxit), int(bool(jacobi)), st)
    else:
        lib.oracle_mixed_ru_block(A.n_rows, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val),
                                  _f32(val32), int(k), B, X, float(rtol), float(delta),
                                  int(maxit), int(bool(jacobi)), st)
    return [SolveResult(X[j], s.status, s.iters, s.outer_iters, s.relres, s.relres_true)
            for j, s in enumerate(st)]


def lanczos_extremes(alpha, beta):
    """Extreme eigenvalues of the Lanczos tridiagonal T_k implied by k CG steps.

    T[j, j] = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T[j, j+1] = sqrt(beta_j)/alpha_j
    (Saad, Iterative Methods for Sparse Linear Systems, Section 6.7.3).
    """
    k = len(alpha)
    if k == 0:
        return float("nan"), float("nan")
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])
