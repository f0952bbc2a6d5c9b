"""GPU parity of CSR SpMV (float64 and float32) against the CPU oracle.

Integer-valued products are exact in any summation order, so those cases
must match bit for bit; otherwise the bar is the normwise relative error
max_i |y_i - y_ref_i| / max_i sum_j |a_ij x_j| <= 1e-13 (stencil rows cancel,
so entry-wise relative error is meaningless)."""
import json
import os

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


def absrow(A, x):
    return oracle.spmv(CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, np.abs(A.val)), np.abs(x))


def normwise(y, yref, A, x):
    denom = max(float(np.max(absrow(A, x))), 1e-300)
    return float(np.max(np.abs(y - yref))) / denom


def run(A, x):
    dA = cgx.DeviceCSR.from_host(A)
    return cgx.csr_spmv(dA, dev(x)).cpu().numpy()


def test_table1_example_bit_exact(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table1_example.json")))
    rp, ci, v = oracle.from_one_based(g["IA_1based"], g["JA_1based"], g["AA_1based"])
    A = CSR(5, 5, rp, ci, v)
    y = run(A, np.array(g["x"], float))
    assert list(y) == [-3.0, 37.0, 32.0, 61.0, 26.0]


@pytest.mark.parametrize("N", [3, 16, 41])
def test_fd7_integer_exact(N):
    A = synth.fd7(N)
    x = np.floor(synth.uniform(3, A.n_cols) * 1000)
    y = run(A, x)
    assert np.array_equal(y, oracle.spmv(A, x))


def random_csr(seed, n_rows, n_cols, max_len, integer=False):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n_rows)
    lens[rng.random(n_rows) < 0.05] = 0          # empty rows
    rp = np.zeros(n_rows + 1, np.int32)
    rp[1:] = np.cumsum(np.minimum(lens, n_cols))
    ci = np.concatenate([rng.choice(n_cols, l, replace=False) for l in np.minimum(lens, n_cols)]
                        + [np.zeros(0, int)]).astype(np.int32)
    v = (rng.integers(-9, 10, ci.size).astype(float) if integer
         else rng.uniform(-1, 1, ci.size))
    return CSR(n_rows, n_cols, rp, ci, v)


@pytest.mark.parametrize("seed,n_rows,n_cols,max_len", [
    (0, 1, 1, 1), (1, 37, 50, 9), (2, 1000, 700, 30), (3, 5003, 5003, 70),
    (4, 20000, 3000, 130), (5, 333, 100000, 3), (6, 300, 9000, 5000)])
def test_random_unsorted_rows_normwise(seed, n_rows, n_cols, max_len):
    A = random_csr(seed, n_rows, n_cols, max_len)
    assert oracle.csr_check(A.n_rows, A.n_cols, A.row_ptr, A.col_idx) == 0
    x = synth.uniform(seed + 100, n_cols)
    y = run(A, x)
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13
    empty = np.diff(A.row_ptr) == 0
    assert np.all(y[empty] == 0) and not np.any(np.signbit(y[empty]))


def test_skewed_rows_multi_chunk():
    """A few rows far longer than one staged chunk among short rows."""
    rng = np.random.default_rng(21)
    n = 8000
    lens = rng.integers(0, 12, n)
    lens[[5, 6, 1700, n - 1]] = [2500, 0, 7000, 1300]
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([rng.choice(n, l, replace=False) for l in lens]).astype(np.int32)
    A = CSR(n, n, rp, ci, rng.uniform(-1, 1, ci.size))
    x = synth.uniform(22, n)
    y = run(A, x)
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13


def test_random_integer_exact():
    A = random_csr(11, 4000, 4000, 100, integer=True)
    x = np.floor(synth.uniform(12, 4000) * 100)
    assert np.array_equal(run(A, x), oracle.spmv(A, x))


@pytest.mark.parametrize("N,sigma", [(10, 0.0), (23, 1.0), (37, 1.5)])
def test_q1_cube_normwise(N, sigma):
    A = synth.q1cube(N, sigma, seed=synth.SEED_C2_COEFF)
    x = synth.uniform(4, A.n_cols)
    y = run(A, x)
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13


def test_q1_128_full_size():
    """The SpMV of the FP64 microbenchmark: Q1 128^3, lognormal(0,1) coefficients."""
    A = synth.q1cube(128, 1.0, seed=synth.SEED_C2_COEFF)
    assert A.nnz == 55742968
    x = synth.uniform(4, A.n_cols)
    y = run(A, x)
    assert normwise(y, oracle.spmv(A, x), A, x) <= 1e-13


def test_spmv_deterministic():
    A = synth.q1cube(30, 1.0, seed=1)
    dA = cgx.DeviceCSR.from_host(A)
    dx = dev(synth.uniform(2, A.n_cols))
    ys = [cgx.csr_spmv(dA, dx).cpu().numpy() for _ in range(3)]
    assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2])


@pytest.mark.parametrize("N", [12, 50])
def test_spmv_f32(N):
    A = synth.q1cube(N, 1.0, seed=7)
    v32 = A.val.astype(np.float32)
    x32 = synth.uniform(8, A.n_cols).astype(np.float32)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    assert np.array_equal(dA.val32.cpu().numpy(), v32)
    y = cgx.csr_spmv_f32(dA, dev(x32)).cpu().numpy()
    yref = oracle.spmv_f32(A, v32, x32)
    denom = float(np.max(absrow(A, x32.astype(float))))
    assert float(np.max(np.abs(y.astype(float) - yref.astype(float)))) / denom <= 2e-6


def test_validate_rejects_malformed():
    A = synth.fd7(4)
    h = cgx.default_handle()
    good = cgx.DeviceCSR.from_host(A)
    assert cgx.csr_validate(good) == -1
    bad_ci = A.col_idx.copy()
    bad_ci[17] = A.n_cols  # out of range
    with pytest.raises(cgx.CgxError):
        cgx.DeviceCSR.from_host(CSR(A.n_rows, A.n_cols, A.row_ptr, bad_ci, A.val))
    dup = A.col_idx.copy()
    dup[A.row_ptr[5] + 1] = dup[A.row_ptr[5]]
    with pytest.raises(cgx.CgxError):
        cgx.DeviceCSR.from_host(CSR(A.n_rows, A.n_cols, A.row_ptr, dup, A.val))
    rp = A.row_ptr.copy()
    rp[10] = rp[11] + 1  # decreasing row start
    with pytest.raises(cgx.CgxError):
        cgx.DeviceCSR.from_host(CSR(A.n_rows, A.n_cols, rp, A.col_idx, A.val))
    assert h is not None


def test_out_of_range_columns_do_not_fault():
    """Kernels clamp indices: a malformed (unvalidated) matrix gives wrong
    numbers for the bad entries but no memory fault."""
    A = synth.fd7(6)
    ci = A.col_idx.copy()
    ci[::7] = 1 << 30
    dA = cgx.DeviceCSR.from_host(CSR(A.n_rows, A.n_cols, A.row_ptr, ci, A.val), validate=False)
    y = cgx.csr_spmv(dA, dev(np.ones(A.n_cols))).cpu().numpy()
    ok = ci < A.n_cols
    keep = CSR(A.n_rows, A.n_cols, A.row_ptr, np.where(ok, ci, 0), np.where(ok, A.val, 0.0))
    assert np.array_equal(y, oracle.spmv(keep, np.ones(A.n_cols)))
