"""GPU tests of the sliced-ELL copy (64-row slices, column-major, padded
to the slice's longest row): its layout against a numpy construction from
the definition (exact), its SpMV against the CPU oracle (same bars as the
CSR SpMV: integer cases bit for bit, else normwise <= 1e-13), and CG /
mixed refinement running their SpMV on it against the oracle and against
the CSR path."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2112_10823_amd import cgx
from synth import CSR

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def normwise(y, yref, A, x):
    absA = CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, np.abs(A.val))
    denom = max(float(np.max(oracle.spmv(absA, np.abs(x)))), 1e-300)
    return float(np.max(np.abs(y - yref))) / denom


def expected_layout(A):
    """slice_ptr, col, val of the sliced-ELL copy, written from its definition."""
    n = A.n_rows
    ns = (n + 63) // 64
    lens = np.zeros(ns * 64, np.int64)
    lens[:n] = np.diff(A.row_ptr)
    width = lens.reshape(ns, 64).max(axis=1)
    sp = np.zeros(ns + 1, np.int64)
    sp[1:] = np.cumsum(64 * width)
    col = np.full(int(sp[-1]), -1, np.int32)
    val = np.zeros(int(sp[-1]))
    for i in range(n):
        s, l = divmod(i, 64)
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            e = sp[s] + 64 * (k - A.row_ptr[i]) + l
            col[e] = A.col_idx[k]
            val[e] = A.val[k]
    return sp, col, val


def random_csr(seed, n_rows, n_cols, max_len):
    rng = np.random.default_rng(seed)
    lens = np.minimum(rng.integers(0, max_len + 1, n_rows), n_cols)
    rp = np.zeros(n_rows + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([rng.choice(n_cols, l, replace=False) for l in lens]
                        + [np.zeros(0, int)]).astype(np.int32)
    return CSR(n_rows, n_cols, rp, ci, rng.uniform(-1, 1, ci.size))


CASES = [lambda: synth.fd7(5), lambda: synth.q1cube(9, 1.0, 3),
         lambda: random_csr(1, 200, 150, 40), lambda: random_csr(2, 1, 3, 3),
         lambda: random_csr(3, 130, 5000, 900)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_layout_matches_definition(case):
    A = CASES[case]()
    S = cgx.SellMatrix(cgx.DeviceCSR.from_host(A))
    sp, col, val = expected_layout(A)
    assert S.n_slices == len(sp) - 1 and S.stored == sp[-1]
    dsp, dcol, dval = S.arrays()
    assert np.array_equal(dsp.cpu().numpy(), sp)
    assert np.array_equal(dcol.cpu().numpy(), col)
    assert np.array_equal(dval.cpu().numpy(), val)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sell_spmv_vs_oracle(case):
    A = CASES[case]()
    S = cgx.SellMatrix(cgx.DeviceCSR.from_host(A))
    x = synth.uniform(40 + case, A.n_cols)
    y = cgx.sell_spmv(S, dev(x)).cpu().numpy()
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13
    empty = np.diff(A.row_ptr) == 0
    assert np.all(y[empty] == 0) and not np.any(np.signbit(y[empty]))


def test_sell_spmv_integer_exact():
    A = synth.fd7(23)  # 12167 rows: many slices and a ragged last one
    x = np.floor(synth.uniform(3, A.n_cols) * 1000)
    S = cgx.SellMatrix(cgx.DeviceCSR.from_host(A))
    assert np.array_equal(cgx.sell_spmv(S, dev(x)).cpu().numpy(), oracle.spmv(A, x))


def test_sell_spmv_full_size_q1_128():
    A = synth.q1cube(128, 1.0, seed=synth.SEED_C2_COEFF)
    S = cgx.SellMatrix(cgx.DeviceCSR.from_host(A))
    assert S.stored >= A.nnz and S.stored <= 1.01 * A.nnz  # padding well under 1 %
    x = synth.uniform(4, A.n_cols)
    y = cgx.sell_spmv(S, dev(x)).cpu().numpy()
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13


@pytest.mark.parametrize("N", [12, 40])
def test_sell_spmv_f32(N):
    A = synth.q1cube(N, 1.0, seed=7)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    S = cgx.SellMatrix(dA)
    x32 = synth.uniform(8, A.n_cols).astype(np.float32)
    y = cgx.sell_spmv_f32(S, dev(x32)).cpu().numpy()
    v32 = A.val.astype(np.float32)
    ref = oracle.spmv_f32(A, v32, x32).astype(np.float64)
    A32 = CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, v32.astype(np.float64))
    # binary32 accumulation over <= 27 terms: a few units of 2^-24 normwise
    assert normwise(y.astype(np.float64), ref, A32, x32.astype(np.float64)) <= 64 * 2.0 ** -24


@pytest.mark.parametrize("N,jacobi", [(20, False), (40, True), (61, True)])
def test_cg_on_sell_vs_oracle_and_csr(N, jacobi):
    A = synth.q1cube(N, 1.0, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(N, synth.SEED_C2_BLOBS)
    dA = cgx.DeviceCSR.from_host(A)
    S = cgx.SellMatrix(dA)
    ref = oracle.cg(A, b, rtol=1e-8, jacobi=jacobi)
    opts = cgx.make_opts(rtol=1e-8, precond=int(jacobi), true_residual=True)
    xs = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    st = cgx.cg_solve(dA, dev(b), xs, opts, sell=S)
    xc = torch.zeros_like(xs)
    stc = cgx.cg_solve(dA, dev(b), xc, opts)
    assert st.status == cgx.OK and st.path == 0
    assert abs(st.iters - ref.iters) <= 2 and abs(st.iters - stc.iters) <= 2
    x = xs.cpu().numpy()
    tr = float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))
    assert tr <= 1.5e-8 and abs(st.relres_true - tr) <= 1e-3 * tr
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-5


def test_mixed_refinement_on_sell_vs_oracle():
    A = synth.q1cube(33, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    S = cgx.SellMatrix(dA)
    ref = oracle.mixed_ir(A, A.val.astype(np.float32), b, rtol=1e-10, tau=1e-3, jacobi=True)
    ref64 = oracle.cg(A, b, rtol=1e-13, jacobi=True, maxit=20000)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    st = cgx.cg_solve(dA, dev(b), x, cgx.make_opts(rtol=1e-10, precond=1,
                                                   precision=cgx.PRECISION_MIXED), sell=S)
    assert st.status == cgx.OK and st.path == 2
    assert abs(st.outer_iters - ref.outer_iters) <= 1
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - oracle.spmv(A, xh)) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(xh - ref64.x) / np.linalg.norm(ref64.x) <= 1e-6


def test_sell_argument_errors():
    A = synth.q1cube(10, 1.0, seed=1)
    dA = cgx.DeviceCSR.from_host(A)
    S = cgx.SellMatrix(dA)
    B = synth.q1cube(11, 1.0, seed=1)
    dB = cgx.DeviceCSR.from_host(B)
    b = torch.ones(B.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(cgx.CgxError):  # copy of another matrix
        cgx.cg_solve(dB, b, torch.zeros_like(b), cgx.make_opts(), sell=S)
    b = torch.ones(A.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(cgx.CgxError):  # mixed precision needs the binary32 values
        cgx.cg_solve(dA, b, torch.zeros_like(b),
                     cgx.make_opts(precision=cgx.PRECISION_MIXED), sell=S)
