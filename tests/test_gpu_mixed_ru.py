"""GPU parity of the mixed-precision solve with reliable updates (binary32 CG
whose direction is kept across float64 updates of x, the true residual and
the stopping test) against the CPU oracle's mixed_ru.

Both sides iterate in binary32 in different summation orders, so iterates
differ at the binary32 level.  What must agree: the true residual (the
oracle's float64 SpMV on the GPU solution) below the tolerance; the solution
within the kappa * rtol bound of the float64 oracle; the step where the run
stopped inside the band of the oracle's own residual history and its
rounding sensitivity (tests/cg_gates.py); the update count within 2."""
import numpy as np
import pytest
import torch

import oracle
import synth
from cg_gates import assert_stop_in_band, residual_band
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ru(A, b, rtol=1e-10, delta=1e-2, jacobi=False, maxit=0, max_outer=0, x0=None, sell=False):
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    dx = dev(np.zeros(A.n_rows) if x0 is None else x0)
    S = cgx.SellMatrix(dA) if sell else None
    st = cgx.cg_solve(dA, dev(b), dx, cgx.make_opts(rtol=rtol, precision=cgx.PRECISION_MIXED_RU,
                                                    inner_rtol=delta, precond=int(jacobi),
                                                    maxit=maxit, max_outer=max_outer),
                      sell=S)
    return st, dx.cpu().numpy()


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


@pytest.mark.parametrize("N,jacobi,delta", [(14, False, 1e-2), (14, True, 1e-2), (30, True, 1e-2),
                                            (30, True, 0.1), (30, False, 1e-3)])
def test_mixed_ru_vs_oracle(N, jacobi, delta):
    A = synth.q1cube(N, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    v32 = A.val.astype(np.float32)
    rtol = 1e-10
    ref = oracle.mixed_ru(A, v32, b, rtol=rtol, delta=delta, jacobi=jacobi)
    ref64 = oracle.cg(A, b, rtol=1e-13, jacobi=True, maxit=20000)
    st, x = ru(A, b, rtol=rtol, delta=delta, jacobi=jacobi)
    assert st.status == cgx.OK and st.path == 6, st.as_dict()
    tr = true_relres(A, b, x)
    assert tr <= rtol
    assert abs(st.relres_true - tr) <= 1e-3 * tr + 1e-16
    assert abs(st.outer_iters - ref.outer_iters) <= 2, (st.outer_iters, ref.outer_iters)
    h, F = residual_band(A, b, rtol, solve=lambda M, v, t: oracle.mixed_ru(
        M, M.val.astype(np.float32), v, rtol=t, delta=delta, jacobi=jacobi,
        history=True).relres_hist)
    assert_stop_in_band(h, F, st.iters, rtol, (st.iters, ref.iters))
    err = np.linalg.norm(x - ref64.x) / np.linalg.norm(ref64.x)
    assert err <= 1e-6  # kappa < 1e4 here: kappa * rtol


def test_mixed_ru_keeps_krylov_space_on_gpu():
    """The GPU's binary32 iteration count stays near float64 CG's, well under
    the restarted refinement's at the same residual drop."""
    A = synth.q1cube(30, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    db = dev(b)
    x = torch.zeros_like(db)
    s64 = cgx.cg_solve(dA, db, x, cgx.make_opts(rtol=1e-10, precond=1))
    x.zero_()
    sru = cgx.cg_solve(dA, db, x, cgx.make_opts(rtol=1e-10, precond=1, inner_rtol=1e-2,
                                                precision=cgx.PRECISION_MIXED_RU))
    x.zero_()
    sir = cgx.cg_solve(dA, db, x, cgx.make_opts(rtol=1e-10, precond=1, inner_rtol=1e-2,
                                                precision=cgx.PRECISION_MIXED))
    assert s64.status == sru.status == sir.status == cgx.OK
    assert sru.iters <= 1.1 * s64.iters + 2
    assert sir.iters >= 1.15 * sru.iters


def test_mixed_ru_sell_and_kappa():
    """The same method with the binary32 SpMV on the sliced-ELL copy; its
    Ritz values (coefficients of the whole binary32 run, the betas at updates
    carried to the true residuals) lie inside the 7-point spectrum."""
    N = 20
    A = synth.fd7(N)
    b = synth.uniform(5, A.n_rows)
    st, x = ru(A, b, rtol=1e-10, sell=True)
    assert st.status == cgx.OK and st.outer_iters >= 2
    assert true_relres(A, b, x) <= 1e-10
    th = np.pi / (N + 1)
    lo, hi = 12 * np.sin(th / 2) ** 2, 12 * np.sin(N * th / 2) ** 2
    assert lo * (1 - 1e-4) <= st.ritz_min <= st.ritz_max <= hi * (1 + 1e-4)
    assert abs(st.ritz_min - lo) <= 1e-3 * lo and abs(st.ritz_max - hi) <= 1e-3 * hi


def test_mixed_ru_status_cases():
    A = synth.q1cube(12, 1.0, seed=1)
    n = A.n_rows
    st, x = ru(A, np.zeros(n), x0=np.ones(n))
    assert st.status == cgx.OK and not x.any() and st.iters == 0
    b = synth.uniform(2, n)
    st, x = ru(A, b, rtol=1e-15, maxit=7)
    assert st.status == cgx.NOT_CONVERGED and st.iters == 7
    # the correction of the unfinished cycle is kept and the residual is the true one
    tr = true_relres(A, b, x)
    assert abs(st.relres - tr) <= 1e-6 * tr and tr < 0.9
    st, _ = ru(A, b, rtol=1e-15, max_outer=2)
    assert st.status == cgx.NOT_CONVERGED and st.outer_iters == 2
    bb = synth.uniform(2, n)
    bb[5] = np.inf
    st, _ = ru(A, bb)
    assert st.status == cgx.NONFINITE
    neg = synth.CSR(n, n, A.row_ptr, A.col_idx, -A.val)
    st, _ = ru(neg, b, jacobi=True)
    assert st.status == cgx.BREAKDOWN


def test_mixed_ru_q1_192_full_size():
    """The mixed-precision configuration: Q1 192^3 (7,077,888 rows, 189,119,224
    nnz), lognormal(0, 1.5), Jacobi, to 1e-10.  Gate: the oracle's float64
    SpMV on the GPU solution; the error against the GPU's float64 Jacobi-CG
    solution at 1e-12 is reported."""
    N = 192
    A = synth.q1cube(N, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    st, x = ru(A, b, jacobi=True)
    assert st.status == cgx.OK
    tr = true_relres(A, b, x)
    assert tr <= 1e-10
    assert abs(st.relres_true - tr) <= 1e-2 * tr
