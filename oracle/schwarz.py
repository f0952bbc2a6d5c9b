"""Additive Schwarz preconditioned conjugate gradient — TEST INFRASTRUCTURE
ONLY (part of the CPU oracle; see the package docstring for who may use it).

The paper (end of Section 5.3) notes that CG runs well on the GPU under a
domain-decomposition preconditioner (Schwarz, FETI), with the outer iteration
on the host and every subdomain solved by CG on the GPU, and gives no further
algorithm.  This module writes out the classical form of that method, step by
step and without blocking or reordering, so that the GPU path can be checked
against it:

* Subdomains.  The rows are cut into `n_sub` contiguous core blocks
  [floor(i n / S), floor((i+1) n / S)); subdomain i is its core block
  extended by `overlap` rows on each side, clipped to [0, n).  For a grid in
  lexicographic order these are slabs, and `overlap` = k N^2 (N^2 rows per
  layer) overlaps k grid layers.

* Local problems.  A_i is the principal submatrix of A on subdomain i's rows
  and columns (a Dirichlet condition on the subdomain boundary); the
  restriction R_i picks the subdomain's rows of a vector.

* Preconditioner (additive Schwarz).  z = sum_i R_i^T z_i, z_i the result of
  CG on A_i z_i = R_i r from z_i = 0: to relative tolerance `inner_rtol`
  within `inner_maxit` iterations, or, for inner_rtol < 0, exactly
  `inner_maxit` iterations.  The sum runs over i in increasing order.

* Outer iteration.  The CG solve of a subdomain to a tolerance is a
  different linear map at every call, so the outer iteration is flexible CG
  (the Polak-Ribiere form of beta): with q = A p,
      alpha = (r.z) / (p.q),  x += alpha p,  r -= alpha q,
      stop when ||r|| <= rtol ||b||,
      z = M(r),  beta = z.(r_new - r_old) / (r_old.z_old) = -alpha (z.q) / rho,
      rho = r.z,  p = z + beta p.
  With exact subdomain solves it is preconditioned CG with the fixed SPD
  preconditioner sum_i R_i^T A_i^-1 R_i.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import OK, BREAKDOWN, NONFINITE, NOT_CONVERGED, axpy, cg, dot, spmv


@dataclass
class LocalCSR:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray


@dataclass
class SchwarzResult:
    x: np.ndarray
    status: int
    outer_iters: int
    inner_iters: int   # sum over outer steps of the largest subdomain iteration count
    relres: float
    history: dict = field(default_factory=dict)


def ranges(n: int, n_sub: int, overlap: int):
    """[lo, hi) of every subdomain."""
    s = [(i * n) // n_sub for i in range(n_sub + 1)]
    return [(max(0, s[i] - overlap), min(n, s[i + 1] + overlap)) for i in range(n_sub)]


def principal_submatrix(A, lo: int, hi: int) -> LocalCSR:
    """Rows and columns [lo, hi) of A, entries kept in their stored order,
    column indices shifted by -lo."""
    rp, ci, va = np.asarray(A.row_ptr), np.asarray(A.col_idx), np.asarray(A.val)
    rows, cols, vals = [0], [], []
    for g in range(lo, hi):
        c = ci[rp[g]:rp[g + 1]]
        keep = (c >= lo) & (c < hi)
        cols.append(c[keep] - lo)
        vals.append(va[rp[g]:rp[g + 1]][keep])
        rows.append(rows[-1] + int(keep.sum()))
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return LocalCSR(hi - lo, hi - lo, np.asarray(rows, np.int32), cat(cols, np.int32),
                    cat(vals, np.float64))


def local_matrices(A, n_sub: int, overlap: int):
    rg = ranges(A.n_rows, n_sub, overlap)
    return rg, [principal_submatrix(A, lo, hi) for lo, hi in rg]


def apply(rg, subs, r, inner_rtol: float, inner_maxit: int, jacobi: bool):
    """z = sum_i R_i^T CG(A_i, R_i r); returns (z, largest subdomain
    iteration count, worst status among the subdomain solves)."""
    z = np.zeros(r.size)
    its, worst = 0, OK
    fixed = inner_rtol < 0
    for (lo, hi), Ai in zip(rg, subs):
        res = cg(Ai, r[lo:hi], rtol=0.0 if fixed else inner_rtol, maxit=inner_maxit,
                 jacobi=jacobi)
        if res.status in (BREAKDOWN, NONFINITE):
            worst = res.status
        z[lo:hi] += res.x
        its = max(its, res.iters)
    return z, its, worst


def solve(A, b, x0=None, rtol=1e-8, max_outer=0, n_sub=4, overlap=0, inner_rtol=1e-2,
          inner_maxit=50, jacobi=False, history=False) -> SchwarzResult:
    """Flexible CG on A x = b preconditioned by additive Schwarz (module
    docstring).  b = 0 gives x = 0.  max_outer <= 0 means n."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = A.n_rows
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.sqrt(dot(b, b))
    if bnorm == 0.0:
        return SchwarzResult(np.zeros(n), OK, 0, 0, 0.0)
    cap = max_outer if max_outer > 0 else n
    rg, subs = local_matrices(A, n_sub, overlap)
    r = axpy(-1.0, spmv(A, x), b)               # r = b - A x
    hist = {"p": [], "q": [], "relres": []} if history else {}
    rr = dot(r, r)
    if np.sqrt(rr) <= rtol * bnorm:
        return SchwarzResult(x, OK, 0, 0, np.sqrt(rr) / bnorm, hist)
    z, inner, worst = apply(rg, subs, r, inner_rtol, inner_maxit, jacobi)
    rho = dot(r, z)
    p = z.copy()
    status, k = NOT_CONVERGED, 0
    while k < cap:
        if worst != OK or not (rho > 0.0):
            status = worst if worst != OK else BREAKDOWN
            break
        q = spmv(A, p)
        pq = dot(p, q)
        if not np.isfinite(pq):
            status = NONFINITE
            break
        if not (pq > 0.0):
            status = BREAKDOWN
            break
        if history:
            hist["p"].append(p.copy())
            hist["q"].append(q.copy())
        alpha = rho / pq
        x = axpy(alpha, p, x)
        r = axpy(-alpha, q, r)
        k += 1
        rr = dot(r, r)
        if history:
            hist["relres"].append(np.sqrt(rr) / bnorm)
        if not np.isfinite(rr):
            status = NONFINITE
            break
        if np.sqrt(rr) <= rtol * bnorm:
            status = OK
            break
        if k >= cap:
            break
        z, its, worst = apply(rg, subs, r, inner_rtol, inner_maxit, jacobi)
        inner += its
        beta = -alpha * dot(z, q) / rho
        rho = dot(r, z)
        p = axpy(beta, p, z)                     # p = z + beta p
    return SchwarzResult(x, status, k, inner, np.sqrt(rr) / bnorm, hist)
