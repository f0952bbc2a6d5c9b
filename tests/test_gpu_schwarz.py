"""GPU tests of the additive Schwarz solver (domain decomposition with
batched CG subdomain solves): the subdomain matrices the build writes
against the oracle's principal submatrices (bit for bit), and the solve
against the oracle's flexible CG on the same inputs.

Bars.  With a fixed number of subdomain iterations (inner_rtol < 0) nothing
inside the preconditioner depends on a tolerance test, so the two sides
differ only by the order of floating-point sums (wave-tree and blocked sums
on the GPU, compensated index-order dots in the oracle): every SpMV and dot
carries a relative error of a few units of 2^-53 times the condition of the
local problem (<= 1e3 here), and a few outer steps of a few subdomain
iterations each stay below 1e-10 of the iterate; a wrong restriction,
prolongation or coefficient changes the iterate at the first outer step by
far more.  Full solves are compared by their outer iteration counts
(exact, or +-1 where subdomain tolerances decide) and by the true residual
and the error bound rtol * cond(A) against the direct solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import oracle
import synth
from oracle import schwarz
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def true_relres(A, x, b):
    return np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)


BUILD_CASES = [
    ("fd7_6_S1", lambda: synth.fd7(6), 1, 0),
    ("fd7_6_S5_o7", lambda: synth.fd7(6), 5, 7),
    ("fd7_6_rows", lambda: synth.fd7(6), 216, 0),
    ("fd7_6_maxo", lambda: synth.fd7(6), 7, 216 // 7),
    ("q1_12_S4_layer", lambda: synth.q1cube(12, 1.0, 5), 4, 144),
    ("q1_24_S3_2layers", lambda: synth.q1cube(24, 1.0, 6), 3, 2 * 576),
    ("paper_box_S6", lambda: synth.q1box(14, 9), 6, 14 * 14),
]


@pytest.mark.parametrize("name,make,S,o", BUILD_CASES, ids=[c[0] for c in BUILD_CASES])
def test_build_matches_principal_submatrices(name, make, S, o):
    A = make()
    print(f"[schwarz build] {name} n={A.n_rows} S={S} o={o}", flush=True)
    D = cgx.SchwarzDecomposition(cgx.DeviceCSR.from_host(A), S, o)
    rg, subs = schwarz.local_matrices(A, S, o)
    assert D.local_rows == sum(hi - lo for lo, hi in rg)
    nnz_off, rp, col, val = (t.cpu().numpy() for t in D.arrays())
    assert D.local_nnz == sum(L.col_idx.size for L in subs) == nnz_off[-1]
    row0 = 0
    for i, L in enumerate(subs):
        m = L.n_rows
        assert nnz_off[i] == sum(s.col_idx.size for s in subs[:i])
        assert np.array_equal(rp[row0 + i:row0 + i + m + 1], L.row_ptr)
        a, b = nnz_off[i], nnz_off[i + 1]
        assert np.array_equal(col[a:b], L.col_idx)
        assert np.array_equal(val[a:b], L.val)
        row0 += m


SOLVE_CASES = [
    ("fd7_12_S4_layer", lambda: synth.fd7(12), 4, 144),
    ("q1_12_S5_none", lambda: synth.q1cube(12, 1.0, 7), 5, 0),
    ("fd7var_16_S7_ragged", lambda: synth.fd7_var(16, 1.0, 8), 7, 256),
    ("q1_24_S3_multitile", lambda: synth.q1cube(24, 1.0, 9), 3, 576),
]


@pytest.mark.parametrize("name,make,S,o", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
@pytest.mark.parametrize("jacobi", [False, True], ids=["plain", "jacobi"])
@pytest.mark.parametrize("outer", [1, 3])
def test_fixed_inner_iterates_match_oracle(name, make, S, o, jacobi, outer):
    A = make()
    b = synth.uniform(31, A.n_rows)
    print(f"[schwarz iterate] {name} jacobi={jacobi} outer={outer}", flush=True)
    ref = schwarz.solve(A, b, rtol=1e-14, max_outer=outer, n_sub=S, overlap=o,
                        inner_rtol=-1.0, inner_maxit=6, jacobi=jacobi)
    dA = cgx.DeviceCSR.from_host(A)
    D = cgx.SchwarzDecomposition(dA, S, o)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    opts = cgx.make_opts(rtol=1e-14, maxit=6, inner_rtol=-1.0, max_outer=outer,
                         precond=cgx.PRECOND_JACOBI if jacobi else cgx.PRECOND_NONE)
    st = cgx.schwarz_solve(dA, D, dev(b), x, opts)
    assert st.status == cgx.NOT_CONVERGED and ref.status == oracle.NOT_CONVERGED
    assert st.outer_iters == ref.outer_iters == outer
    assert st.iters == ref.inner_iters == 6 * outer
    xg = x.cpu().numpy()
    assert np.max(np.abs(xg - ref.x)) <= 1e-10 * np.max(np.abs(ref.x))


@pytest.mark.parametrize("name,make,S,o", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_full_solve_fixed_inner(name, make, S, o):
    A = make()
    b = synth.uniform(32, A.n_rows)
    print(f"[schwarz solve fixed] {name}", flush=True)
    ref = schwarz.solve(A, b, rtol=1e-10, n_sub=S, overlap=o, inner_rtol=-1.0, inner_maxit=8)
    dA = cgx.DeviceCSR.from_host(A)
    D = cgx.SchwarzDecomposition(dA, S, o)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    st = cgx.schwarz_solve(dA, D, dev(b), x,
                           cgx.make_opts(rtol=1e-10, maxit=8, inner_rtol=-1.0, true_residual=True))
    assert st.status == cgx.OK and ref.status == oracle.OK
    assert abs(st.outer_iters - ref.outer_iters) <= 1
    xg = x.cpu().numpy()
    assert true_relres(A, xg, b) <= 1.5e-10
    assert st.relres_true <= 1.5e-10
    assert np.linalg.norm(xg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("name,make,S,o", SOLVE_CASES[:3], ids=[c[0] for c in SOLVE_CASES[:3]])
@pytest.mark.parametrize("tau", [1e-1, 1e-3])
def test_full_solve_inner_tolerance(name, make, S, o, tau):
    """Subdomain solves to a tolerance: which iteration meets it can differ
    by one between the two sides, so counts agree to +-1 per outer step and
    the answers to the error bound."""
    A = make()
    b = synth.uniform(33, A.n_rows)
    print(f"[schwarz solve tau] {name} tau={tau}", flush=True)
    ref = schwarz.solve(A, b, rtol=1e-10, n_sub=S, overlap=o, inner_rtol=tau, inner_maxit=200,
                        jacobi=True)
    dA = cgx.DeviceCSR.from_host(A)
    D = cgx.SchwarzDecomposition(dA, S, o)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    st = cgx.schwarz_solve(dA, D, dev(b), x,
                           cgx.make_opts(rtol=1e-10, maxit=200, inner_rtol=tau,
                                         precond=cgx.PRECOND_JACOBI))
    assert st.status == cgx.OK and ref.status == oracle.OK
    assert abs(st.outer_iters - ref.outer_iters) <= 2
    xg = x.cpu().numpy()
    assert true_relres(A, xg, b) <= 1.5e-10
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_rows))
    xs = spla.spsolve(M.tocsc(), b)
    lam = spla.eigsh(M, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(M, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    bound = 1.5e-10 * lam / lmin
    assert np.linalg.norm(xg - xs) <= bound * np.linalg.norm(xs)


def test_edge_cases():
    A = synth.fd7(8)
    n = A.n_rows
    dA = cgx.DeviceCSR.from_host(A)
    D = cgx.SchwarzDecomposition(dA, 4, 64)
    print("[schwarz edges] zero rhs, exact x0, one subdomain", flush=True)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    st = cgx.schwarz_solve(dA, D, torch.zeros(n, dtype=torch.float64, device="cuda"), x)
    assert st.status == cgx.OK and st.outer_iters == 0 and not x.any()
    b = synth.uniform(34, n)
    xs = oracle.cg(A, b, rtol=1e-14).x
    x = dev(xs)
    st = cgx.schwarz_solve(dA, D, dev(b), x, cgx.make_opts(rtol=1e-8))
    assert st.status == cgx.OK and st.outer_iters == 0
    D1 = cgx.SchwarzDecomposition(dA, 1, 0)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = cgx.schwarz_solve(dA, D1, dev(b), x,
                           cgx.make_opts(rtol=1e-10, maxit=n, inner_rtol=1e-14))
    assert st.status == cgx.OK and st.outer_iters == 1
    assert true_relres(A, x.cpu().numpy(), b) <= 1e-10


def test_argument_errors():
    A = synth.fd7(4)
    dA = cgx.DeviceCSR.from_host(A)
    for S, o in [(0, 0), (65, 0), (4, 17), (4, -1)]:
        with pytest.raises(cgx.CgxError):
            cgx.SchwarzDecomposition(dA, S, o)
    D = cgx.SchwarzDecomposition(dA, 4, 16)
    b = torch.ones(64, dtype=torch.float64, device="cuda")
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    small = torch.empty(D.workspace_bytes() - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(cgx.CgxError):
        cgx.schwarz_solve(dA, D, b, x, workspace=small)
    with pytest.raises(cgx.CgxError):
        cgx.schwarz_solve(dA, D, b, x, cgx.make_opts(precision=cgx.PRECISION_MIXED))
    B = cgx.DeviceCSR.from_host(synth.fd7(5))
    with pytest.raises(cgx.CgxError):
        cgx.schwarz_solve(B, D, torch.ones(125, dtype=torch.float64, device="cuda"),
                          torch.zeros(125, dtype=torch.float64, device="cuda"))


def test_q1_128_full_size():
    """The Q1 128^3 system of the benchmark (lognormal(0,1), blob right-hand
    side) in 8 slabs overlapping by one grid layer, Jacobi-CG subdomain
    solves to 0.1: the oracle's SpMV of the GPU solution gives the true
    residual (the oracle's own Schwarz solve at this size takes minutes)."""
    A = synth.q1cube(128, 1.0, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(128, synth.SEED_C2_BLOBS)
    dA = cgx.DeviceCSR.from_host(A)
    D = cgx.SchwarzDecomposition(dA, 8, 128 * 128)
    assert D.local_rows == A.n_rows + 2 * 128 * 128 * 7
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    print("[schwarz] Q1 128^3 full size", flush=True)
    st = cgx.schwarz_solve(dA, D, dev(b), x,
                           cgx.make_opts(rtol=1e-8, maxit=100, inner_rtol=0.1,
                                         precond=cgx.PRECOND_JACOBI, true_residual=True))
    assert st.status == cgx.OK and 0 < st.outer_iters < 356
    rr = true_relres(A, x.cpu().numpy(), b)
    assert rr <= 1.5e-8 and abs(rr - st.relres_true) <= 1e-10
