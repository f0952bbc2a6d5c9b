"""Pins of the CPU oracle against facts that do not come from the oracle itself:
the paper's worked CSR example, dense brute force, exact rational arithmetic,
IEEE-754 special cases, Krylov theory (termination, manufactured eigenvectors,
Chebyshev bound) and textbook identities (Jacobi-PCG == CG on the scaled
system, Lanczos Ritz values)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import CSR

U = 2.0 ** -53


# ------------------------------------------------------------------ helpers --

def dense_to_csr(a):
    a = np.asarray(a)
    rp, ci, v = [0], [], []
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            if a[i, j] != 0:
                ci.append(j)
                v.append(float(a[i, j]))
        rp.append(len(ci))
    return CSR(a.shape[0], a.shape[1], np.array(rp, np.int32), np.array(ci, np.int32),
               np.array(v, np.float64))


def exact(v):
    return Fraction(float(v))


def random_csr(rng, n_rows, n_cols, density, integer=False, empty_rows=()):
    a = np.zeros((n_rows, n_cols))
    mask = rng.random((n_rows, n_cols)) < density
    if integer:
        a[mask] = rng.integers(-9, 10, mask.sum())
    else:
        a[mask] = rng.uniform(-1, 1, mask.sum())
    for r in empty_rows:
        a[r, :] = 0
    return a, dense_to_csr(a)


# ------------------------------------------------- Table 1 (Section 2.3) --

def test_table1_csr_derivation_and_spmv(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table1_example.json")))
    dense = np.array(g["dense"])
    # CSR by the paper's definition (1-based) == the fixture's arrays
    A1 = dense_to_csr(dense)
    rp, ci, v = oracle.from_one_based(g["IA_1based"], g["JA_1based"], g["AA_1based"])
    assert np.array_equal(rp, A1.row_ptr) and np.array_equal(ci, A1.col_idx)
    assert np.array_equal(v, A1.val)
    assert oracle.csr_check(5, 5, rp, ci) == 0
    A = CSR(5, 5, rp, ci, v)
    assert np.array_equal(A.to_dense(), dense)
    # y = A x by integer brute force over the printed matrix
    x = g["x"]
    y_exact = [sum(int(dense[i][j]) * x[j] for j in range(5)) for i in range(5)]
    assert y_exact == [-3, 37, 32, 61, 26]
    y = oracle.spmv(A, np.array(x, float))
    assert list(y) == [float(t) for t in y_exact]


# ----------------------------------------------------------------- SpMV --

@pytest.mark.parametrize("seed", range(6))
def test_spmv_integer_bruteforce_exact(seed):
    rng = np.random.default_rng(seed)
    n_rows, n_cols = int(rng.integers(1, 65)), int(rng.integers(1, 65))
    a, A = random_csr(rng, n_rows, n_cols, 0.3, integer=True,
                      empty_rows=[0] if n_rows > 2 else [])
    x = rng.integers(-50, 51, n_cols)
    y_ref = [sum(int(a[i, j]) * int(x[j]) for j in range(n_cols)) for i in range(n_rows)]
    y = oracle.spmv(A, x.astype(float))
    assert [float(t) for t in y_ref] == list(y)
    if n_rows > 2:
        assert y[0] == 0.0 and math.copysign(1.0, y[0]) == 1.0  # empty row -> +0.0


@pytest.mark.parametrize("seed", range(6))
def test_spmv_float_within_sequential_error_bound(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 65))
    a, A = random_csr(rng, n, n, 0.4)
    x = rng.uniform(-1, 1, n)
    y = oracle.spmv(A, x)
    for i in range(n):
        terms = [exact(a[i, j]) * exact(x[j]) for j in range(n) if a[i, j] != 0]
        s = sum(terms, Fraction(0))
        absum = float(sum((abs(t) for t in terms), Fraction(0)))
        k = len(terms)
        gamma = k * U / (1 - k * U)
        assert abs(Fraction(y[i]) - s) <= Fraction(gamma * absum) + Fraction(1e-300)


def test_spmv_rejects_malformed_csr():
    rp = np.array([0, 2, 1], np.int32)
    assert oracle.csr_check(2, 3, rp, np.array([0, 1], np.int32)) != 0      # decreasing ptr
    assert oracle.csr_check(1, 3, np.array([0, 2], np.int32), np.array([0, 3], np.int32)) != 0
    assert oracle.csr_check(1, 3, np.array([0, 2], np.int32), np.array([1, 1], np.int32)) != 0
    assert oracle.csr_check(1, 3, np.array([1, 2], np.int32), np.array([1, 1], np.int32)) != 0
    assert oracle.csr_check(3, 3, np.array([0, 0, 2, 2], np.int32),
                            np.array([2, 0], np.int32)) == 0                 # empty rows, unsorted ok


# ---------------------------------------------- add / axpy / xmul (IEEE) --

def _rand_specials(rng, n):
    v = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-30, 30, n))
    v[:8] = [0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, 1e-310, 1.0, -1.0]
    return v


def test_add_xmul_match_exact_rounding():
    rng = np.random.default_rng(7)
    x, y = _rand_specials(rng, 2000), _rand_specials(rng, 2000)
    z_add, z_mul = oracle.add(x, y), oracle.xmul(x, y)
    for i in range(x.size):
        assert z_add[i] == float(exact(x[i]) + exact(y[i]))
        assert z_mul[i] == float(exact(x[i]) * exact(y[i]))


def test_axpy_is_single_rounding_fma():
    rng = np.random.default_rng(8)
    x, y = rng.uniform(-1, 1, 5000), rng.uniform(-1, 1, 5000)
    alpha = 0.7390851332151607
    z = oracle.axpy(alpha, x, y)
    two_roundings_differ = 0
    for i in range(x.size):
        e = exact(alpha) * exact(x[i]) + exact(y[i])
        assert z[i] == float(e)
        if float(e) != alpha * x[i] + y[i]:
            two_roundings_differ += 1
    assert two_roundings_differ > 50  # the cases discriminate fma from mul+add


def test_elementwise_ieee_special_values():
    inf, nan = float("inf"), float("nan")
    x = np.array([inf, inf, -inf, 0.0, -0.0, -0.0, nan, 1e308])
    y = np.array([1.0, -inf, -inf, -0.0, -0.0, 0.0, 1.0, 1e308])
    z = oracle.add(x, y)
    assert z[0] == inf and math.isnan(z[1]) and z[2] == -inf
    assert z[3] == 0 and math.copysign(1, z[3]) == 1     # +0 + -0 = +0 (round to nearest)
    assert z[4] == 0 and math.copysign(1, z[4]) == -1    # -0 + -0 = -0
    assert math.isnan(z[6]) and z[7] == inf              # overflow to +inf
    m = oracle.xmul(np.array([inf, 0.0, -0.0, 1e200, nan]), np.array([0.0, -3.0, -0.0, 1e200, 0.0]))
    assert math.isnan(m[0]) and math.copysign(1, m[1]) == -1 and math.copysign(1, m[2]) == 1
    assert m[3] == inf and math.isnan(m[4])


# ------------------------------------------------------------------ dot --

@pytest.mark.parametrize("n", [1, 17, 1000, 10000])
def test_dot_kahan_bound_vs_exact_rational(n):
    rng = np.random.default_rng(n)
    x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    s_exact = sum((exact(a) * exact(b) for a, b in zip(x, y)), Fraction(0))
    absum = float(np.sum(np.abs(x * y)))
    d = oracle.dot(x, y)
    # products rounded once (u each) + Kahan's 2u + O(n u^2) summation bound
    assert abs(Fraction(d) - s_exact) <= Fraction((3 * U + 2 * n * U * U) * absum)


def test_dot_cancellation_and_integers():
    # integer vectors with |sum| < 2^53: exact in any order
    rng = np.random.default_rng(3)
    x = rng.integers(-1000, 1000, 5000).astype(float)
    y = rng.integers(-1000, 1000, 5000).astype(float)
    assert oracle.dot(x, y) == float(int(np.dot(x.astype(np.int64), y.astype(np.int64))))
    # many tiny terms after a large one: recursive summation drops all of them,
    # the compensated sum stays within its 2u * sum|x_i y_i| bound
    x = np.array([1.0] + [1e-16] * 10000)
    y = np.ones_like(x)
    s_exact = Fraction(1) + 10000 * exact(1e-16)
    d = oracle.dot(x, y)
    assert abs(Fraction(d) - s_exact) <= Fraction(3 * U * 1.000000000001)
    assert d != 1.0


# ------------------------------------------------------------------- CG --

def fd7_eigs(N):
    th = [j * math.pi / (N + 1) for j in range(1, N + 1)]
    l1 = [4 * math.sin(t / 2) ** 2 for t in th]
    return l1


def test_cg_fd7_manufactured_eigenvector_one_iteration():
    N = 9
    A = synth.fd7(N)
    j = (2, 5, 7)
    i = np.arange(1, N + 1)
    vs = [np.sin(jj * math.pi * i / (N + 1)) for jj in j]
    v = np.einsum("k,j,i->kji", vs[2], vs[1], vs[0]).ravel()
    lam = sum(4 * math.sin(jj * math.pi / (2 * (N + 1))) ** 2 for jj in j)
    r = oracle.cg(A, lam * v, rtol=1e-12)
    assert r.status == oracle.OK and r.iters == 1
    assert np.linalg.norm(r.x - v) / np.linalg.norm(v) < 1e-13


def test_cg_q1_manufactured_eigenvector_one_iteration():
    """Constant-k Q1 on the unit cube: A = S(x)M(x)M + M(x)S(x)M + M(x)M(x)S with
    1D stiffness S = tridiag(-1,2,-1)/h and mass M = h tridiag(1,4,1)/6, whose
    sine eigenvectors give lambda = s_a m_b m_c + m_a s_b m_c + m_a m_b s_c."""
    N = 8
    A = synth.q1cube(N, sigma=0.0)
    h = 1.0 / (N + 1)
    jx, jy, jz = 1, 4, 6
    i = np.arange(1, N + 1)
    vx, vy, vz = (np.sin(j * math.pi * i / (N + 1)) for j in (jx, jy, jz))
    v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()

    def s_m(j):
        c = math.cos(j * math.pi / (N + 1))
        return (2 - 2 * c) / h, h * (4 + 2 * c) / 6

    (sx, mx), (sy, my), (sz, mz) = s_m(jx), s_m(jy), s_m(jz)
    lam = sx * my * mz + mx * sy * mz + mx * my * sz
    assert np.allclose(oracle.spmv(A, v), lam * v, rtol=0, atol=1e-14 * lam)
    r = oracle.cg(A, lam * v, rtol=1e-12)
    assert r.status == oracle.OK and r.iters == 1
    assert np.linalg.norm(r.x - v) / np.linalg.norm(v) < 1e-13


@pytest.mark.parametrize("N", [2, 3, 4])
def test_cg_terminates_within_distinct_eigenvalue_count(N):
    l1 = fd7_eigs(N)
    sums = sorted({round(a + b + c, 9) for a in l1 for b in l1 for c in l1})
    m = len(sums)
    assert m == {2: 4, 3: 7, 4: 16}[N]
    A = synth.fd7(N)
    b = synth.uniform(5, N ** 3)
    r = oracle.cg(A, b, rtol=0.0, maxit=m)
    assert r.relres_true < 1e-11
    r_short = oracle.cg(A, b, rtol=0.0, maxit=m - 1)
    assert r_short.relres_true > 1e-9  # not earlier for a generic right-hand side


@pytest.mark.parametrize("seed", range(5))
def test_cg_random_spd_matches_dense_solve(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 65))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(0, math.log(100), n))
    a = (Q * ev) @ Q.T
    a = (a + a.T) / 2
    A = dense_to_csr(a)
    b = rng.uniform(-1, 1, n)
    r = oracle.cg(A, b, rtol=1e-12, maxit=10 * n)
    kappa = ev.max() / ev.min()
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    kcheb = math.ceil(math.log(1e-12 / (2 * math.sqrt(kappa))) / math.log(rho))
    assert r.status == oracle.OK and r.iters <= kcheb
    xs = np.linalg.solve(a, b)
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 100 * 1e-12 * 10


def test_cg_fd7_16_chebyshev_bound_and_ritz_values():
    """The plain-CG configuration on the 16^3 7-point grid: x* ~ U[-1,1] (seed 0),
    b = A x*, stop at 1e-10.  Iterations obey the Chebyshev bound
    ||r_k||/||b|| <= 2 sqrt(kappa) ((sqrt(kappa)-1)/(sqrt(kappa)+1))^k, and the
    Lanczos Ritz extremes reproduce the analytic spectrum edges."""
    N = 16
    A = synth.fd7(N)
    xs = synth.uniform(synth.SEED_C1_XSTAR, N ** 3)
    b = oracle.spmv(A, xs)
    r = oracle.cg(A, b, rtol=1e-10, history=True)
    l1 = fd7_eigs(N)
    lmin, lmax = 3 * l1[0], 3 * l1[-1]
    kappa = lmax / lmin
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    kmax = math.ceil(math.log(1e-10 / (2 * math.sqrt(kappa))) / math.log(rho))
    assert r.status == oracle.OK and 0 < r.iters <= kmax
    assert r.relres_true < 2e-10
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < kappa * 1e-10
    emin, emax = oracle.lanczos_extremes(r.alpha, r.beta)
    assert abs(emin - lmin) / lmin < 1e-8 and abs(emax - lmax) / lmax < 1e-8


def test_jacobi_pcg_equals_cg_on_symmetrically_scaled_system():
    N = 6
    A = synth.q1cube(N, sigma=1.0, seed=3)
    a = A.to_dense()
    d = np.diag(a)
    s = 1 / np.sqrt(d)
    As = dense_to_csr(a * s[:, None] * s[None, :])
    b = synth.uniform(9, N ** 3)
    for k in (1, 2, 5, 12):
        rj = oracle.cg(A, b, rtol=0.0, maxit=k, jacobi=True)
        rs = oracle.cg(As, s * b, rtol=0.0, maxit=k)
        assert rj.iters == rs.iters == k
        assert np.linalg.norm(rj.x - s * rs.x) / np.linalg.norm(rj.x) < 1e-12


def test_jacobi_pcg_converges_and_helps_on_rough_coefficients():
    N = 12
    A = synth.q1cube(N, sigma=1.0, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(N, synth.SEED_C2_BLOBS)
    rp = oracle.cg(A, b, rtol=1e-8)
    rj = oracle.cg(A, b, rtol=1e-8, jacobi=True)
    assert rp.status == rj.status == oracle.OK
    assert rj.iters < rp.iters
    assert rj.relres_true < 2e-8 and rp.relres_true < 2e-8


def test_cg_status_codes():
    A = synth.fd7(3)
    n = A.n_rows
    # b = 0 -> x = 0 after 0 iterations, whatever x0
    r = oracle.cg(A, np.zeros(n), x0=np.ones(n))
    assert r.status == oracle.OK and r.iters == 0 and not r.x.any()
    # maxit too small -> NOT_CONVERGED, last iterate kept
    r = oracle.cg(A, synth.uniform(1, n), rtol=1e-14, maxit=2)
    assert r.status == oracle.NOT_CONVERGED and r.iters == 2 and r.relres_true < 1
    # indefinite matrix -> breakdown
    neg = CSR(n, n, A.row_ptr, A.col_idx, -A.val)
    r = oracle.cg(neg, synth.uniform(1, n))
    assert r.status == oracle.BREAKDOWN
    # non-finite right-hand side
    bb = synth.uniform(1, n)
    bb[3] = float("nan")
    assert oracle.cg(A, bb).status == oracle.NONFINITE
    # Jacobi with a non-positive diagonal
    bad = CSR(n, n, A.row_ptr, A.col_idx, np.where(A.col_idx == np.repeat(np.arange(n), np.diff(A.row_ptr)), 0.0, A.val))
    assert oracle.cg(bad, synth.uniform(1, n), jacobi=True).status == oracle.BREAKDOWN


# ------------------------------------------------------- mixed precision --

@pytest.mark.parametrize("jacobi", [False, True])
def test_mixed_ir_reaches_fp64_accuracy(jacobi):
    N = 14
    A = synth.q1cube(N, sigma=1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, N ** 3)
    v32 = A.val.astype(np.float32)
    tau = 1e-3
    r = oracle.mixed_ir(A, v32, b, rtol=1e-10, tau=tau, jacobi=jacobi)
    assert r.status == oracle.OK and r.relres <= 1e-10
    # each refinement step contracts by about tau (plus the binary32 floor)
    assert r.outer_iters <= 2 * math.ceil(math.log(1e-10) / math.log(tau)) + 1
    ref = oracle.cg(A, b, rtol=1e-13)
    xs = np.linalg.solve(A.to_dense(), b)
    assert np.linalg.norm(ref.x - xs) / np.linalg.norm(xs) < 1e-9
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-7


def test_f32_kernels_are_binary32():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, 3000).astype(np.float32)
    y = rng.uniform(-1, 1, 3000).astype(np.float32)
    d = oracle.dot_f32(x, y)
    s = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    absum = float(np.sum(np.abs(x.astype(float) * y.astype(float))))
    u32 = 2.0 ** -24
    assert abs(Fraction(d) - s) <= Fraction((3 * u32 + 2 * 3000 * u32 * u32) * absum)
    assert np.float32(d) == d
    A = synth.fd7(5)
    y32 = oracle.spmv_f32(A, A.val.astype(np.float32), np.ones(A.n_rows, np.float32))
    assert y32.dtype == np.float32
    assert np.array_equal(y32, oracle.spmv(A, np.ones(A.n_rows)).astype(np.float32))


def _power_of_two_diagonal(n):
    """diag(a) with a_i cycling through 1/2, 2, 8: three distinct eigenvalues,
    every entry and its reciprocal exact in binary32."""
    a = np.resize(np.array([0.5, 2.0, 8.0]), n)
    return a, CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), a.copy())


def test_mixed_ir_diagonal_closed_form():
    """Refinement on a diagonal matrix, where each step has a closed form.
    Jacobi-preconditioned, the binary32 inner CG is exact after one step
    (z = D^-1 c, q = c, alpha = 1), so one refinement step gives
    x_i = s * float(b_i / s) / a_i with s = ||b||: only the rounding of the
    scaled residual to binary32 remains, a relative residual of at most
    2^-24, and a second step squares it.  Unpreconditioned, the inner CG
    takes exactly three steps (three distinct eigenvalues, a generic
    right-hand side) whenever the inner tolerance lies above the binary32
    floor."""
    n = 300
    a, A = _power_of_two_diagonal(n)
    v32 = A.val.astype(np.float32)
    b = synth.uniform(41, n)
    s = np.linalg.norm(b)
    one = oracle.mixed_ir(A, v32, b, rtol=1e-10, tau=1e-3, max_outer=1, jacobi=True)
    assert one.status == oracle.NOT_CONVERGED and one.outer_iters == 1 and one.iters == 1
    x1 = s * (b / s).astype(np.float32).astype(np.float64) / a
    assert np.all(np.abs(one.x - x1) <= 4 * U * np.abs(x1))
    assert 0.0 < one.relres <= 2.0 ** -24 * 1.001
    full = oracle.mixed_ir(A, v32, b, rtol=1e-10, tau=1e-3, jacobi=True)
    assert full.status == oracle.OK and full.outer_iters == 2 and full.iters == 2
    assert full.relres <= 1e-14
    assert np.linalg.norm(full.x - b / a) <= 1e-14 * np.linalg.norm(b / a)
    plain = oracle.mixed_ir(A, v32, b, rtol=1e-10, tau=1e-3)
    assert plain.status == oracle.OK and 2 <= plain.outer_iters <= 3
    assert plain.iters == 3 * plain.outer_iters
    assert np.linalg.norm(plain.x - b / a) <= 1e-9 * np.linalg.norm(b / a)


def test_mixed_ir_trivial_cases():
    """A zero right-hand side gives x = 0 without a step; an exact starting
    guess gives no step and leaves x untouched."""
    a, A = _power_of_two_diagonal(30)
    v32 = A.val.astype(np.float32)
    z = oracle.mixed_ir(A, v32, np.zeros(30), x0=np.ones(30))
    assert z.status == oracle.OK and z.outer_iters == 0 and not z.x.any()
    x = synth.uniform(3, 30)
    b = a * x  # exact: every a_i is a power of two
    e = oracle.mixed_ir(A, v32, b, x0=x)
    assert e.status == oracle.OK and e.outer_iters == 0 and e.iters == 0
    assert np.array_equal(e.x, x)


def test_mixed_ir_jacobi_inner_sees_two_eigenvalues():
    """A = S B S with B block-diagonal in identical 2x2 blocks [[1, t], [t, 1]]
    (eigenvalues 1 - t and 1 + t) and S diagonal in powers of two, so that A,
    its diagonal S^2 and the scaling are exact in binary32.  Jacobi-PCG on A is
    CG on B, which ends in two steps for any right-hand side: every inner solve
    of the Jacobi refinement takes exactly two steps, while the unpreconditioned
    inner CG sees the many distinct eigenvalues of A and takes more."""
    rng = np.random.default_rng(8)
    nb, t = 200, 0.5
    s = 2.0 ** rng.integers(-2, 3, 2 * nb)
    rows, cols, vals = [], [], []
    for k in range(nb):
        i, j = 2 * k, 2 * k + 1
        for r, c, v in ((i, i, 1.0), (i, j, t), (j, i, t), (j, j, 1.0)):
            rows.append(r)
            cols.append(c)
            vals.append(s[r] * v * s[c])
    n = 2 * nb
    A = CSR(n, n, np.arange(0, 2 * n + 1, 2, dtype=np.int32), np.array(cols, np.int32),
            np.array(vals))
    assert np.array_equal(A.val.astype(np.float32).astype(np.float64), A.val)
    b = synth.uniform(77, n)
    xs = np.linalg.solve(A.to_dense(), b)
    jac = oracle.mixed_ir(A, A.val.astype(np.float32), b, rtol=1e-10, tau=1e-3, jacobi=True)
    assert jac.status == oracle.OK and 2 <= jac.outer_iters <= 3
    assert jac.iters == 2 * jac.outer_iters
    assert np.linalg.norm(jac.x - xs) <= 1e-9 * np.linalg.norm(xs)
    plain = oracle.mixed_ir(A, A.val.astype(np.float32), b, rtol=1e-10, tau=1e-3)
    assert plain.status == oracle.OK and plain.iters > 2 * plain.outer_iters


def test_rounding_is_per_operation_in_each_precision():
    """Inputs whose results follow by hand from IEEE round-to-nearest-even.
    With e = 2^-12 (binary32) or 2^-27 (float64), (1+e)^2 = 1 + 2e + e^2
    rounds to 1 + 2e, so -1 + (1+e)(1+e) is 2e; an SpMV that fuses the
    product into its sum, or a dot carried wholly in a wider type, gives
    2e + e^2.  And 1 + u + u with u half an ulp of 1 stays 1 when added in
    order (ties to even), where a wider SpMV accumulator reaches the next
    float.  (The compensated dot's own correction term is zero on these
    inputs, so how that step is rounded is left to the dot's error-bound
    pins.)"""
    for e, u, f32 in ((2.0 ** -12, 2.0 ** -24, True), (2.0 ** -27, 2.0 ** -53, False)):
        A = CSR(2, 4, np.array([0, 2, 5], np.int32), np.array([0, 1, 0, 2, 3], np.int32),
                np.array([-1.0, 1 + e, 1.0, u, u]))
        x = np.array([1.0, 1 + e, 1.0, 1.0])
        if f32:
            y = oracle.spmv_f32(A, A.val.astype(np.float32), x.astype(np.float32))
            d = oracle.dot_f32(np.array([1 + e, -1], np.float32), np.array([1 + e, 1], np.float32))
        else:
            y = oracle.spmv(A, x)
            d = oracle.dot(np.array([1 + e, -1.0]), np.array([1 + e, 1.0]))
        assert y[0] == 2 * e and y[1] == 1.0, (f32, y)
        assert d == 2 * e, (f32, d)


def test_degenerate_systems():
    """n = 0: nothing to do, OK after no iteration; an empty dot is +0.0.
    1 x 1 (4 x = 3): one step of CG, Jacobi-CG or refinement lands on 3/4,
    which every precision holds exactly."""
    A0 = CSR(0, 0, np.array([0], np.int32), np.array([], np.int32), np.array([], np.float64))
    assert oracle.spmv(A0, np.zeros(0)).size == 0
    r0 = oracle.cg(A0, np.zeros(0))
    assert r0.status == oracle.OK and r0.iters == 0 and r0.x.size == 0
    d0 = oracle.dot(np.zeros(0), np.zeros(0))
    assert d0 == 0.0 and math.copysign(1.0, d0) == 1.0
    A1 = CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    b = np.array([3.0])
    for r in (oracle.cg(A1, b, rtol=1e-14), oracle.cg(A1, b, rtol=1e-14, jacobi=True)):
        assert r.status == oracle.OK and r.iters == 1 and r.x[0] == 0.75
    ir = oracle.mixed_ir(A1, np.array([4.0], np.float32), b, rtol=1e-14)
    assert ir.status == oracle.OK and ir.outer_iters == 1 and ir.iters == 1 and ir.x[0] == 0.75


# ------------------------------------------------- CG residual history --

def _exact_cg_residuals(Ad, b, iters, jacobi):
    """CG (Saad's recurrences, the paper's cited textbook) carried out in exact
    rational arithmetic on an integer matrix: ||r_k|| / ||b|| for k = 0..iters."""
    n = len(b)
    A = [[Fraction(int(v)) for v in row] for row in Ad]
    dinv = [Fraction(1) / A[i][i] if jacobi else Fraction(1) for i in range(n)]
    r = [Fraction(int(v)) for v in b]
    z = [dinv[i] * r[i] for i in range(n)]
    p = list(z)
    rho = sum(ri * zi for ri, zi in zip(r, z))
    bb = sum(v * v for v in r)
    out = [1.0]
    for _ in range(iters):
        q = [sum(A[i][j] * p[j] for j in range(n)) for i in range(n)]
        alpha = rho / sum(pi * qi for pi, qi in zip(p, q))
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        rr = sum(v * v for v in r)
        out.append(math.sqrt(rr / bb))
        if rr == 0:
            break
        z = [dinv[i] * r[i] for i in range(n)]
        rho_new = sum(ri * zi for ri, zi in zip(r, z))
        p = [zi + (rho_new / rho) * pi for zi, pi in zip(z, p)]
        rho = rho_new
    return out


@pytest.mark.parametrize("jacobi", [False, True])
def test_cg_residual_history_exact_rational(jacobi):
    """The recorded ||r_k|| / ||b|| of every step against CG in exact rational
    arithmetic on a small integer SPD system (a well-conditioned case, so
    finite precision follows the exact iterates closely); the last entry is
    the reported relres, at or below rtol, and the one before it above."""
    rng = np.random.default_rng(11)
    n = 8
    M = rng.integers(-3, 4, (n, n))
    Ad = M @ M.T + np.diag(rng.integers(4, 12, n))
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    A = CSR(n, n, rp, ci, Ad.astype(np.float64).ravel())
    b = rng.integers(-5, 6, n).astype(np.float64)
    rtol = 1e-10
    res = oracle.cg(A, b, rtol=rtol, jacobi=jacobi, history=True)
    h = res.relres_hist
    assert res.status == oracle.OK and len(h) == res.iters + 1
    exact = _exact_cg_residuals(Ad, b, res.iters, jacobi)
    assert h[0] == 1.0
    for k in range(1, res.iters):
        assert abs(h[k] - exact[k]) <= 1e-9 * max(exact[k], 1e-6), (k, h[k], exact[k])
    assert h[-1] == res.relres and h[-1] <= rtol < h[-2]


def test_cg_residual_history_plain_matches_coefficients():
    """Plain CG: ||r_k||^2 = rho_k = rho_0 * beta_0 ... beta_{k-1} (beta_j =
    rho_{j+1} / rho_j), so the history and the coefficient record agree; the
    manufactured eigenvector's history is [1, ~0]."""
    N = 12
    A = synth.fd7(N)
    b = synth.uniform(21, A.n_rows)
    res = oracle.cg(A, b, rtol=1e-9, history=True)
    h = res.relres_hist
    prod = np.concatenate([[1.0], np.cumprod(res.beta)])
    np.testing.assert_allclose(h[:-1] ** 2, prod, rtol=1e-12)
    i = np.arange(1, N + 1)
    v = np.einsum("k,j,i->kji", *[np.sin(j * math.pi * i / (N + 1)) for j in (4, 2, 1)]).ravel()
    lam = sum(4 * math.sin(j * math.pi / (2 * (N + 1))) ** 2 for j in (1, 2, 4))
    e = oracle.cg(A, lam * v, rtol=1e-12, history=True)
    assert e.iters == 1 and e.relres_hist[0] == 1.0 and e.relres_hist[1] < 1e-13


# ---------------------------- mixed precision with reliable updates --

def _dense_of(A):
    D = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        D[i, A.col_idx[s:e]] = A.val[s:e]
    return D


@pytest.mark.parametrize("delta", [0.3, 1e-2])
@pytest.mark.parametrize("case", ["fd7_plain", "q1_jacobi", "fd7var_jacobi"])
def test_mixed_ru_float64_steps_are_cg(case, delta):
    """In exact arithmetic the reliable-update method is CG (the replaced
    residual equals the recursive one, the rescaled beta is CG's beta).  Its
    steps carried out in float64 therefore follow float64 CG: the same
    iteration count and residual history, across several updates.  (On
    well-conditioned operators: where CG's residual history is itself
    rounding-sensitive, as plain CG on the lognormal matrices, it differs from
    the oracle's own reversed-order run by tens of percent, and no history
    comparison is meaningful.)"""
    A = {"fd7_plain": lambda: synth.fd7(12), "q1_jacobi": lambda: synth.q1cube(12, 1.0, 4),
         "fd7var_jacobi": lambda: synth.fd7_var(12, 1.0, 4)}[case]()
    jacobi = case.endswith("jacobi")
    b = synth.uniform(12, A.n_rows)
    ref = oracle.cg(A, b, rtol=1e-10, jacobi=jacobi, history=True)
    ru = oracle.mixed_ru(A, None, b, rtol=1e-10, delta=delta, jacobi=jacobi, history=True,
                         inner_f64=True)
    assert ru.status == oracle.OK and ru.outer_iters >= 3
    assert ru.iters == ref.iters
    np.testing.assert_allclose(ru.relres_hist, ref.relres_hist, rtol=1e-5)
    assert np.linalg.norm(ru.x - ref.x) / np.linalg.norm(ref.x) <= 1e-9


def test_mixed_ru_diagonal_closed_form():
    """Power-of-two diagonal with Jacobi: D^-1 A = I, so each binary32 step
    solves its scaled residual up to the rounding of float(r / s) (relative
    2^-24), the recursive residual is exactly 0 and an update follows; two
    steps and two updates reach 1e-10, x = b / a."""
    n = 64
    d = 2.0 ** (np.arange(n) % 7 - 3)
    A = CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = synth.uniform(3, n)
    ru = oracle.mixed_ru(A, d.astype(np.float32), b, rtol=1e-10, delta=0.1, jacobi=True,
                         history=True)
    assert ru.status == oracle.OK and ru.iters == 2 and ru.outer_iters == 2
    assert ru.relres_hist[1] <= 2.0 ** -24
    np.testing.assert_allclose(ru.x, b / d, rtol=2.0 ** -46)


@pytest.mark.parametrize("jacobi", [False, True])
def test_mixed_ru_keeps_the_krylov_space(jacobi):
    """Binary32 iteration with float64 updates converges like float64 CG
    (within 10 % of its iterations with Jacobi, 20 % without), where
    refinement that restarts the
    inner CG at every correction needs markedly more; the solution is within
    kappa rtol of a dense solve and its true residual meets rtol."""
    A = synth.q1cube(14, 1.0, 7)
    b = synth.uniform(8, A.n_rows)
    v32 = A.val.astype(np.float32)
    ref = oracle.cg(A, b, rtol=1e-10, jacobi=jacobi)
    ru = oracle.mixed_ru(A, v32, b, rtol=1e-10, delta=0.01, jacobi=jacobi)
    ir = oracle.mixed_ir(A, v32, b, rtol=1e-10, tau=0.01, jacobi=jacobi)
    assert ru.status == oracle.OK
    assert ru.iters <= (1.1 if jacobi else 1.2) * ref.iters + 2
    assert ir.iters >= 1.15 * ru.iters
    D = _dense_of(A)
    xs = np.linalg.solve(D, b)
    ev = np.linalg.eigvalsh(D)
    assert np.linalg.norm(ru.x - xs) / np.linalg.norm(xs) <= (ev[-1] / ev[0]) * 1e-10
    assert np.linalg.norm(b - oracle.spmv(A, ru.x)) / np.linalg.norm(b) <= 1e-10
    assert ru.relres == np.linalg.norm(b - oracle.spmv(A, ru.x)) / np.linalg.norm(b) or \
        abs(ru.relres / (np.linalg.norm(b - oracle.spmv(A, ru.x)) / np.linalg.norm(b)) - 1) < 1e-6


def test_mixed_ru_status_cases():
    A = synth.fd7(6)
    v32 = A.val.astype(np.float32)
    n = A.n_rows
    z = oracle.mixed_ru(A, v32, np.zeros(n), rtol=1e-10)
    assert z.status == oracle.OK and z.iters == 0 and not z.x.any()
    xs = synth.uniform(2, n)
    e = oracle.mixed_ru(A, v32, oracle.spmv(A, xs), x0=xs, rtol=1e-10)
    assert e.status == oracle.OK and e.iters == 0
    neg = CSR(n, n, A.row_ptr, A.col_idx, -A.val)
    assert oracle.mixed_ru(neg, -v32, synth.uniform(3, n), jacobi=True).status == oracle.BREAKDOWN
    assert oracle.mixed_ru(neg, -v32, synth.uniform(3, n)).status == oracle.BREAKDOWN
    b = synth.uniform(4, n)
    cap = oracle.mixed_ru(A, v32, b, rtol=1e-14, maxit=5)
    assert cap.status == oracle.NOT_CONVERGED and cap.iters == 5
    # the correction of the unfinished cycle is kept: reported residual = true residual
    true = np.linalg.norm(b - oracle.spmv(A, cap.x)) / np.linalg.norm(b)
    assert abs(cap.relres - true) <= 1e-12 * true and true < 0.5


# ------------------------------------------- reliable updates, k in step --

@pytest.mark.parametrize("case", ["fd7_plain", "q1_jacobi", "q1s_plain"])
def test_ru_block_of_one_is_mixed_ru(case):
    """One right-hand side: the block method is the single method, bit for
    bit (iterates, counts, status), in binary32 and in float64."""
    A = {"fd7_plain": lambda: synth.fd7(9), "q1_jacobi": lambda: synth.q1cube(10, 1.0, 5),
         "q1s_plain": lambda: synth.q1cube(9, 1.5, 6)}[case]()
    jacobi = case.endswith("jacobi")
    b = synth.uniform(31, A.n_rows)
    v32 = A.val.astype(np.float32)
    for f64 in (False, True):
        one = oracle.mixed_ru(A, v32, b, rtol=1e-10, delta=0.01, jacobi=jacobi, inner_f64=f64)
        blk = oracle.mixed_ru_block(A, v32, b[None], rtol=1e-10, delta=0.01, jacobi=jacobi,
                                    inner_f64=f64)[0]
        assert (blk.status, blk.iters, blk.outer_iters) == (one.status, one.iters, one.outer_iters)
        assert np.array_equal(blk.x, one.x) and blk.relres == one.relres


@pytest.mark.parametrize("case", ["fd7_plain", "q1_jacobi", "fd7var_jacobi"])
def test_ru_block_float64_steps_are_cg(case):
    """Updates taken because another right-hand side fired are exact in
    exact arithmetic too: in float64 every right-hand side of the block
    follows float64 CG (iteration count, solution), whatever the others do."""
    A = {"fd7_plain": lambda: synth.fd7(12), "q1_jacobi": lambda: synth.q1cube(12, 1.0, 4),
         "fd7var_jacobi": lambda: synth.fd7_var(12, 1.0, 4)}[case]()
    jacobi = case.endswith("jacobi")
    B = np.stack([synth.uniform(40 + j, A.n_rows) for j in range(4)])
    B[2] *= np.linspace(0.1, 3.0, A.n_rows)  # a right-hand side of another spectrum mix
    res = oracle.mixed_ru_block(A, None, B, rtol=1e-10, delta=0.1, jacobi=jacobi,
                                inner_f64=True)
    for j, r in enumerate(res):
        ref = oracle.cg(A, B[j], rtol=1e-10, jacobi=jacobi)
        assert r.status == oracle.OK and r.outer_iters >= 3, j
        assert abs(r.iters - ref.iters) <= 1, (j, r.iters, ref.iters)
        assert np.linalg.norm(r.x - ref.x) / np.linalg.norm(ref.x) <= 1e-8, j


def test_ru_block_updates_are_shared():
    """Every active right-hand side takes every update event: those still
    running have equal counts, each at least as many as alone less rounding
    slack; duplicates of one right-hand side reproduce its solo run; a zero
    right-hand side is inert (the others equal the block without it)."""
    A = synth.q1cube(11, 1.0, 8)
    v32 = A.val.astype(np.float32)
    B = np.stack([synth.uniform(50 + j, A.n_rows) for j in range(3)])
    res = oracle.mixed_ru_block(A, v32, B, rtol=1e-10, delta=0.01, jacobi=True)
    solo = [oracle.mixed_ru(A, v32, B[j], rtol=1e-10, delta=0.01, jacobi=True) for j in range(3)]
    assert all(r.status == oracle.OK for r in res)
    last = max(r.iters for r in res)
    # the right-hand sides that ran to the end saw every event
    runners = [r for r in res if r.iters == last]
    assert len({r.outer_iters for r in runners}) == 1
    for r, s in zip(res, solo):
        assert r.outer_iters >= s.outer_iters - 1
        assert np.linalg.norm(r.x - s.x) <= 1e-8 * np.linalg.norm(s.x)
    dup = oracle.mixed_ru_block(A, v32, np.stack([B[0], B[0]]), rtol=1e-10, delta=0.01,
                                jacobi=True)
    for r in dup:
        assert (r.iters, r.outer_iters) == (solo[0].iters, solo[0].outer_iters)
        assert np.array_equal(r.x, solo[0].x)
    Bz = np.stack([B[0], np.zeros(A.n_rows), B[1]])
    rz = oracle.mixed_ru_block(A, v32, Bz, rtol=1e-10, delta=0.01, jacobi=True)
    r2 = oracle.mixed_ru_block(A, v32, np.stack([B[0], B[1]]), rtol=1e-10, delta=0.01,
                               jacobi=True)
    assert rz[1].status == oracle.OK and rz[1].iters == 0 and not rz[1].x.any()
    for a, c in zip((rz[0], rz[2]), r2):
        assert (a.iters, a.outer_iters) == (c.iters, c.outer_iters) and np.array_equal(a.x, c.x)


def test_ru_block_status_cases():
    A = synth.fd7(6)
    v32 = A.val.astype(np.float32)
    n = A.n_rows
    B = np.stack([synth.uniform(4, n), synth.uniform(5, n)])
    cap = oracle.mixed_ru_block(A, v32, B, rtol=1e-14, maxit=5)
    for j, c in enumerate(cap):
        assert c.status == oracle.NOT_CONVERGED and c.iters == 5
        true = np.linalg.norm(B[j] - oracle.spmv(A, c.x)) / np.linalg.norm(B[j])
        assert abs(c.relres - true) <= 1e-12 * true and true < 0.5
    neg = CSR(n, n, A.row_ptr, A.col_idx, -A.val)
    assert all(r.status == oracle.BREAKDOWN
               for r in oracle.mixed_ru_block(neg, -v32, B, jacobi=True))
    assert all(r.status == oracle.BREAKDOWN for r in oracle.mixed_ru_block(neg, -v32, B))


def test_ru_block_sibling_event_reaches_every_rhs():
    """A discrete eigenvector of the 7-point operator converges in one binary32
    step and fires an update there; in the block the other right-hand side
    takes that update too (its run then differs from its solo run and counts
    at least as many updates), while each lane alone keeps its solo result."""
    N = 9
    A = synth.fd7(N)
    v32 = A.val.astype(np.float32)
    i = np.arange(1, N + 1)
    vs = [np.sin(jj * math.pi * i / (N + 1)) for jj in (2, 5, 7)]
    v = np.einsum("k,j,i->kji", vs[2], vs[1], vs[0]).ravel()
    lam = sum(4 * math.sin(jj * math.pi / (2 * (N + 1))) ** 2 for jj in (2, 5, 7))
    b_eig, b_rnd = lam * v, synth.uniform(60, A.n_rows)
    solo_eig = oracle.mixed_ru(A, v32, b_eig, rtol=1e-6, delta=0.01)
    solo_rnd = oracle.mixed_ru(A, v32, b_rnd, rtol=1e-6, delta=0.01)
    assert solo_eig.iters == 1 and solo_eig.outer_iters == 1
    assert solo_rnd.iters > 3
    blk = oracle.mixed_ru_block(A, v32, np.stack([b_rnd, b_eig]), rtol=1e-6, delta=0.01)
    assert blk[1].iters == 1 and np.array_equal(blk[1].x, solo_eig.x)
    assert blk[0].status == oracle.OK and blk[0].outer_iters >= solo_rnd.outer_iters
    assert not np.array_equal(blk[0].x, solo_rnd.x)  # the update at step 1 was taken
    # capped at that step: the sibling still takes the update (then stops at
    # the cap with its correction in x), as it does when rho <= 0 would stop it
    cap = oracle.mixed_ru_block(A, v32, np.stack([b_rnd, b_eig]), rtol=1e-6, delta=0.01, maxit=1)
    assert (cap[1].status, cap[1].iters, cap[1].outer_iters) == (oracle.OK, 1, 1)
    assert (cap[0].status, cap[0].iters, cap[0].outer_iters) == (oracle.NOT_CONVERGED, 1, 1)
    alone = oracle.mixed_ru(A, v32, b_rnd, rtol=1e-6, delta=0.01, maxit=1)
    assert alone.outer_iters == 0 and np.array_equal(cap[0].x, alone.x)
