"""The allocation-free CG entry point (cgx_cg_solve_noalloc, the library's
static device scratch as workspace) against cgx_cg_solve: the same kernels in
the same order, so the same bits, iteration counts and statistics; two calls
in a row, the second on a smaller system, then a system too large for the
scratch (refused) and the same matrix without Jacobi (fits)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def both(h, A, b, **kw):
    dA = cgx.DeviceCSR.from_host(A, handle=h)
    db = dev(b)
    x_ref = torch.zeros_like(db)
    st_ref = cgx.cg_solve(dA, db, x_ref, cgx.make_opts(**kw), handle=h)
    x_na = torch.full_like(db, 7.0)
    x_na.zero_()
    st_na = cgx.cg_solve_noalloc(dA, db, x_na, cgx.make_opts(**kw), handle=h)
    return st_ref, x_ref.cpu().numpy(), st_na, x_na.cpu().numpy()


def same(st_ref, x_ref, st_na, x_na):
    assert st_na.status == st_ref.status == cgx.OK
    assert st_na.iters == st_ref.iters and st_na.path == st_ref.path
    assert np.array_equal(x_na.view(np.int64), x_ref.view(np.int64))
    assert st_na.relres == st_ref.relres
    assert st_na.kappa_est == st_ref.kappa_est


def test_noalloc_equals_cg_solve_twice_then_smaller():
    h = cgx.Handle()
    # first call: 64,000 rows, Jacobi, phase kernels
    A1 = synth.q1cube(40, 1.0, 31)
    b1 = synth.uniform(32, A1.n_rows)
    r = both(h, A1, b1, rtol=1e-10, precond=cgx.PRECOND_JACOBI)
    same(*r)
    ref = oracle.cg(A1, b1, rtol=1e-10, jacobi=True)
    assert abs(r[2].iters - ref.iters) <= 2
    assert np.linalg.norm(b1 - oracle.spmv(A1, r[3])) / np.linalg.norm(b1) <= 1.5e-10
    # second call, smaller: 4096 rows, plain CG, the single-workgroup kernel
    A2 = synth.fd7(16)
    b2 = oracle.spmv(A2, synth.uniform(synth.SEED_C1_XSTAR, A2.n_rows))
    r = both(h, A2, b2, rtol=1e-10)
    same(*r)
    assert r[2].path == 1
    ref = oracle.cg(A2, b2, rtol=1e-10)
    assert abs(r[2].iters - ref.iters) <= 2
    assert np.linalg.norm(b2 - oracle.spmv(A2, r[3])) / np.linalg.norm(b2) <= 1.5e-10


def test_noalloc_size_limit():
    """1.73 M rows: Jacobi needs more workspace than the 64 MiB scratch
    (refused before any launch, x untouched); plain CG fits and matches."""
    h = cgx.Handle()
    A = synth.fd7(120)
    dA = cgx.DeviceCSR.from_host(A, handle=h)
    b = dev(synth.uniform(33, A.n_rows))
    oj = cgx.make_opts(rtol=1e-8, precond=cgx.PRECOND_JACOBI)
    assert cgx.cg_workspace_bytes(A.n_rows, A.nnz, oj) > 64 << 20
    x = torch.full_like(b, 3.0)
    with pytest.raises(cgx.CgxError) as ei:
        cgx.cg_solve_noalloc(dA, b, x, oj, handle=h)
    assert ei.value.code == cgx.ENOMEM
    assert bool((x == 3.0).all())
    op = cgx.make_opts(rtol=1e-8)
    assert cgx.cg_workspace_bytes(A.n_rows, A.nnz, op) <= 64 << 20
    x_ref = torch.zeros_like(b)
    st_ref = cgx.cg_solve(dA, b, x_ref, op, handle=h)
    x.zero_()
    st = cgx.cg_solve_noalloc(dA, b, x, op, handle=h)
    assert st.status == st_ref.status == cgx.OK and st.iters == st_ref.iters
    assert torch.equal(x, x_ref)
    with pytest.raises(cgx.CgxError) as ei:
        cgx.cg_solve_noalloc(dA, b, x, cgx.make_opts(precision=cgx.PRECISION_MIXED), handle=h)
    assert ei.value.code == cgx.EINVAL
