"""Pins of the seeded input generators: the paper's Table 2 shape statistics,
the sizes of the standard workloads, the published SplitMix64 test vector and
structural properties of the stiffness matrices."""
import json
import os

import numpy as np
import pytest

import synth


def test_splitmix64_published_vectors():
    # Vigna's reference splitmix64.c, seed 1234567, and the seed-0 first output
    assert list(map(int, synth.splitmix64(1234567, 5))) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    assert int(synth.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_uniform_and_normal_streams():
    u = synth.uniform(42, 200000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01
    raw = synth.splitmix64(42, 3)
    assert u[0] == -1 + 2 * ((int(raw[0]) >> 11) * 2.0 ** -53)
    z = synth.normal(7, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


def test_table2_shapes_reproduced(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table2_matrices.json")))
    for row, (a, c) in zip(g["rows"], g["reading"]["a_c"]):
        h, nz, density, _bw, max_row, mean, std = row
        A = synth.q1box(a, c)
        rl = np.diff(A.row_ptr)
        n = A.n_rows
        assert n == (101568 if h == 101168 else h)
        assert A.nnz == nz == synth._load().synth_q1box_nnz(a, c)
        assert round(100.0 * nz / n ** 2, 3) == density
        assert int(rl.max()) == max_row
        assert round(float(rl.mean()), 3) == mean
        assert round(float(rl.std()), 3) == std


def test_standard_workload_sizes():
    lib = synth._load()
    assert lib.synth_fd7_nnz(16) == 27136                 # 16^3 7-point grid
    assert lib.synth_q1cube_nnz(128) == 55742968          # Q1 128^3
    assert lib.synth_q1cube_nnz(192) == 189119224         # Q1 192^3
    A = synth.fd7(16)
    assert A.n_rows == 4096 and A.nnz == 27136


@pytest.mark.parametrize("make", [lambda: synth.fd7(7), lambda: synth.q1cube(7, 1.0, 4),
                                  lambda: synth.q1box(9, 7)])
def test_structure_sorted_symmetric(make):
    A = make()
    rp, ci = A.row_ptr, A.col_idx
    for i in range(A.n_rows):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
    d = A.to_dense()
    assert np.array_equal(d, d.T)                          # bitwise symmetric
    assert np.all(np.linalg.eigvalsh(d) > 0)               # SPD


def test_q1_constant_coefficient_stencil():
    N = 6
    A = synth.q1cube(N, 0.0)
    h = 1.0 / (N + 1)
    c = (N // 2) + N * ((N // 2) + N * (N // 2))           # an interior node
    row = dict(zip(A.col_idx[A.row_ptr[c]:A.row_ptr[c + 1]], A.val[A.row_ptr[c]:A.row_ptr[c + 1]]))
    assert len(row) == 27
    assert row[c] == pytest.approx(8 * h / 3, rel=1e-15)
    assert row[c + 1] == 0.0 and row[c + N] == 0.0 and row[c + N * N] == 0.0
    assert row[c + 1 + N] == pytest.approx(-h / 6, rel=1e-15)
    assert row[c + 1 + N + N * N] == pytest.approx(-h / 12, rel=1e-15)
    assert abs(sum(row.values())) < 1e-15                  # constants are in the kernel
    F = synth.fd7(N)
    ones = np.ones(F.n_rows)
    rs = np.array([F.val[F.row_ptr[i]:F.row_ptr[i + 1]].sum() for i in range(F.n_rows)])
    assert rs[c] == 0 and rs[0] == 3                       # interior 0, corner 6-3


def test_q1_coefficients_enter_linearly():
    N = 5
    k = synth.q1_coeffs(N, 1.0, 12)
    A1 = synth.q1cube_from_coeffs(N, k)
    A2 = synth.q1cube_from_coeffs(N, 2 * k)
    assert np.array_equal(A2.val, 2 * A1.val)
    assert np.all(k > 0)


def test_blob_rhs_reproducible():
    b1 = synth.blob_rhs(10, 11)
    b2 = synth.blob_rhs(10, 11)
    assert np.array_equal(b1, b2) and np.linalg.norm(b1) > 0
    assert not np.array_equal(b1, synth.blob_rhs(10, 12))
