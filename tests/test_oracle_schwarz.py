"""Pins of the additive Schwarz oracle against facts it does not produce
itself: dense slicing and dense inverses of the subdomain matrices, scipy's
preconditioned CG with the same fixed preconditioner, the Jacobi-PCG oracle
(pinned on its own) as the one-row-subdomain special case, and the local
A-conjugacy that flexible CG's beta enforces."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import schwarz


def dense(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols)).toarray()


def systems():
    return [("fd7_6", synth.fd7(6)), ("q1_5_var", synth.q1cube(5, 1.0, seed=3)),
            ("fd7var_7", synth.fd7_var(7, 1.0, seed=4))]


@pytest.mark.parametrize("n,S,o", [(10, 1, 0), (10, 3, 2), (100, 7, 14), (64, 64, 0),
                                   (65, 4, 16)])
def test_ranges_cover_and_overlap(n, S, o):
    rg = schwarz.ranges(n, S, o)
    cores = [((i * n) // S, ((i + 1) * n) // S) for i in range(S)]
    assert cores[0][0] == 0 and cores[-1][1] == n
    assert all(b - a in (n // S, -(-n // S)) for a, b in cores)
    for (lo, hi), (a, b) in zip(rg, cores):
        assert lo == max(0, a - o) and hi == min(n, b + o)


@pytest.mark.parametrize("name,A", systems())
def test_principal_submatrix_is_dense_slice(name, A):
    D = dense(A)
    for lo, hi in schwarz.ranges(A.n_rows, 5, 11):
        L = schwarz.principal_submatrix(A, lo, hi)
        assert np.array_equal(dense(L), D[lo:hi, lo:hi])


@pytest.mark.parametrize("name,A", systems())
@pytest.mark.parametrize("S,o", [(1, 0), (4, 0), (4, 9), (5, 30)])
def test_apply_with_exact_solves_is_dense_asm(name, A, S, o):
    """With subdomain CG run to 1e-14 the preconditioner is sum_i R_i^T
    A_i^-1 R_i, built here from dense inverses."""
    D = dense(A)
    n = A.n_rows
    r = synth.uniform(7, n)
    rg, subs = schwarz.local_matrices(A, S, o)
    z, _, worst = schwarz.apply(rg, subs, r, 1e-14, 0, False)
    ref = np.zeros(n)
    for lo, hi in rg:
        ref[lo:hi] += np.linalg.solve(D[lo:hi, lo:hi], r[lo:hi])
    assert worst == oracle.OK
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,A", systems())
def test_one_subdomain_solves_in_one_step(name, A):
    b = synth.uniform(8, A.n_rows)
    res = schwarz.solve(A, b, rtol=1e-10, n_sub=1, overlap=0, inner_rtol=1e-14, inner_maxit=0)
    assert res.status == oracle.OK and res.outer_iters == 1


@pytest.mark.parametrize("name,A", systems())
@pytest.mark.parametrize("S,o", [(4, 0), (3, 20)])
def test_exact_solves_match_scipy_pcg(name, A, S, o):
    """Fixed SPD preconditioner: flexible CG reduces to PCG; scipy's cg with
    the dense additive Schwarz operator takes the same iterations to the same
    answer."""
    D = dense(A)
    n = A.n_rows
    b = synth.uniform(9, n)
    rg = schwarz.ranges(n, S, o)
    Minv = np.zeros((n, n))
    for lo, hi in rg:
        Minv[lo:hi, lo:hi] += np.linalg.inv(D[lo:hi, lo:hi])
    its = []
    x_sp, info = spla.cg(sp.csr_matrix(D), b, rtol=1e-10, atol=0.0, maxiter=10 * n,
                         M=spla.LinearOperator((n, n), matvec=lambda v: Minv @ v),
                         callback=lambda xk: its.append(1))
    res = schwarz.solve(A, b, rtol=1e-10, n_sub=S, overlap=o, inner_rtol=1e-14, inner_maxit=0)
    assert info == 0 and res.status == oracle.OK
    assert abs(res.outer_iters - len(its)) <= 1
    xs = np.linalg.solve(D, b)
    assert np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)


@pytest.mark.parametrize("name,A", systems())
def test_single_row_subdomains_are_jacobi_pcg(name, A):
    """One row per subdomain and no overlap: each subdomain solve is r_i /
    a_ii, so the method is Jacobi-preconditioned CG."""
    n = A.n_rows
    b = synth.uniform(10, n)
    res = schwarz.solve(A, b, rtol=1e-10, n_sub=n, overlap=0, inner_rtol=1e-14, inner_maxit=4)
    ref = oracle.cg(A, b, rtol=1e-10, jacobi=True)
    assert res.status == oracle.OK and ref.status == oracle.OK
    assert res.outer_iters == ref.iters
    assert np.linalg.norm(res.x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("name,A", systems())
@pytest.mark.parametrize("tau,m", [(0.3, 6), (-1.0, 3)])
def test_inexact_solves_keep_local_conjugacy(name, A, tau, m):
    """With inexact subdomain solves the preconditioner changes every step;
    the flexible beta keeps consecutive directions A-conjugate, the A-norm
    of the error falls at every step, and the solve still converges."""
    D = dense(A)
    n = A.n_rows
    b = synth.uniform(11, n)
    res = schwarz.solve(A, b, rtol=1e-10, n_sub=4, overlap=n // 8, inner_rtol=tau,
                        inner_maxit=m, history=True)
    assert res.status == oracle.OK
    P, Q = res.history["p"], res.history["q"]
    for k in range(len(P) - 1):
        a = P[k + 1] @ Q[k]
        assert abs(a) <= 1e-9 * np.sqrt((P[k + 1] @ (D @ P[k + 1])) * (P[k] @ Q[k]))
    xs = np.linalg.solve(D, b)
    assert np.linalg.norm(D @ res.x - b) <= 1e-10 * np.linalg.norm(b) * 1.01 + 1e-14
    assert np.linalg.norm(res.x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_overlap_lowers_outer_iterations():
    """With exact subdomain solves, more overlap gives a better
    preconditioner (Schwarz theory); two grid layers beat none."""
    A = synth.fd7(8)
    b = synth.uniform(12, A.n_rows)
    its = [schwarz.solve(A, b, rtol=1e-10, n_sub=4, overlap=o, inner_rtol=1e-14,
                         inner_maxit=0).outer_iters for o in (0, 64, 128)]
    assert its[0] > its[1] > its[2]


def test_zero_rhs_and_initial_guess():
    A = synth.fd7(5)
    res = schwarz.solve(A, np.zeros(A.n_rows), x0=np.ones(A.n_rows), n_sub=3, overlap=5)
    assert res.status == oracle.OK and res.outer_iters == 0 and not res.x.any()
    b = synth.uniform(13, A.n_rows)
    xs = oracle.cg(A, b, rtol=1e-13).x
    res = schwarz.solve(A, b, x0=xs, rtol=1e-8, n_sub=3, overlap=5)
    assert res.status == oracle.OK and res.outer_iters == 0
