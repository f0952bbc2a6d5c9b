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


def _q1_element_stiffness(h, hy=None, hz=None):
    """int over [0, hx] x [0, hy] x [0, hz] of grad phi_a . grad phi_b for the
    eight trilinear basis functions (vertex a = (ax, ay, az) in {0,1}^3,
    a = ax + 2 ay + 4 az), by two-point Gauss quadrature per axis, exact for
    these integrands.  One side length gives the cube."""
    hs = (h, h if hy is None else hy, h if hz is None else hz)
    pts = [hd * (0.5 + np.array([-0.5, 0.5]) / np.sqrt(3.0)) for hd in hs]
    w = hs[0] * hs[1] * hs[2] / 8.0
    K = np.zeros((8, 8))
    for qx in pts[0]:
        for qy in pts[1]:
            for qz in pts[2]:
                q = (qx, qy, qz)
                grads = []
                for a in range(8):
                    bits = ((a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1)
                    f = [q[d] / hs[d] if bits[d] else 1.0 - q[d] / hs[d] for d in range(3)]
                    df = [(1.0 if bits[d] else -1.0) / hs[d] for d in range(3)]
                    grads.append([df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]])
                G = np.array(grads)
                K += w * G @ G.T
    return K


@pytest.mark.parametrize("elem", [(2, 1, 3), (0, 2, 4), (5, 5, 0)])
def test_q1_single_element_matches_quadrature(elem):
    """One element with coefficient 1.7, every other zero: the assembled
    matrix is 1.7 times the element stiffness matrix on the element's
    vertices that are unknowns (grid nodes 1..N; 0 and N+1 are the Dirichlet
    boundary), and zero elsewhere.  Element (ex, ey, ez) spans grid nodes
    ex..ex+1 along x (and likewise y, z) and its coefficient sits at
    ex + (N+1) (ey + (N+1) ez)."""
    N = 5
    h = 1.0 / (N + 1)
    ex, ey, ez = elem
    k = np.zeros((N + 1) ** 3)
    k[ex + (N + 1) * (ey + (N + 1) * ez)] = 1.7
    A = synth.q1cube_from_coeffs(N, k).to_dense()
    K = 1.7 * _q1_element_stiffness(h)
    expect = np.zeros_like(A)
    verts = []
    for a in range(8):
        x, y, z = ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1)
        if 1 <= x <= N and 1 <= y <= N and 1 <= z <= N:
            verts.append((a, (x - 1) + N * ((y - 1) + N * (z - 1))))
    for a, i in verts:
        for b, j in verts:
            expect[i, j] = K[a, b]
    assert len(verts) == {(2, 1, 3): 8, (0, 2, 4): 4, (5, 5, 0): 1}[elem]
    assert np.allclose(A, expect, rtol=0, atol=1e-14 * np.abs(K).max())


def test_fd7_var_face_weights_are_series_conductances():
    """The 7-point operator's node coefficients are k = exp(sigma Z) from the
    normal stream of the same seed.  A face joins two half cells in series,
    so its weight w = -a_ij lies between min(k_i, k_j) and 2 min(k_i, k_j)
    (an arithmetic mean leaves that range once the contrast exceeds 3, which
    many faces here do); each diagonal is its face weights plus k_i for every
    face on the Dirichlet boundary."""
    N, sigma, seed = 6, 1.0, 3
    A = synth.fd7_var(N, sigma, seed)
    k = np.exp(sigma * synth.normal(seed, N ** 3))
    contrast = 0
    for i in range(A.n_rows):
        cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        vals = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        off = cols != i
        w, kj = -vals[off], k[cols[off]]
        m = np.minimum(k[i], kj)
        assert np.all(w >= m * (1 - 1e-15)) and np.all(w <= 2 * m * (1 + 1e-15)), i
        contrast += int(np.sum(np.maximum(k[i], kj) > 3 * m))
        diag = vals[~off][0]
        assert diag == pytest.approx(w.sum() + k[i] * (6 - off.sum()), rel=1e-14), i
    assert contrast > 100


def test_q1box_rows_match_quadrature():
    """The paper-shape box (a x a x c nodes over 200 x 200 x 10 km): a node
    whose neighbours are all unknowns has the row the eight bricks around it
    assemble, each brick's stiffness integrated by quadrature with sides
    hx = hy = 200/(a-1), hz = 10/(c-1); Dirichlet nodes are identity rows."""
    a, c = 9, 7
    A = synth.q1box(a, c)
    hx, hz = 200.0 / (a - 1), 10.0 / (c - 1)
    K = _q1_element_stiffness(hx, hx, hz)

    def node(x, y, z):
        return x + a * (y + a * z)

    for (x, y, z) in [(2, 2, 2), (4, 3, 3), (6, 6, 4)]:
        i = node(x, y, z)
        expect = {}
        for ez in (z - 1, z):
            for ey in (y - 1, y):
                for ex in (x - 1, x):
                    la = (x - ex) + 2 * (y - ey) + 4 * (z - ez)
                    for lb in range(8):
                        j = node(ex + (lb & 1), ey + ((lb >> 1) & 1), ez + ((lb >> 2) & 1))
                        expect[j] = expect.get(j, 0.0) + K[la, lb]
        got = dict(zip(A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]].tolist(),
                       A.val[A.row_ptr[i]:A.row_ptr[i + 1]].tolist()))
        assert sorted(got) == sorted(expect)
        scale = max(abs(v) for v in expect.values())
        for j in expect:
            assert abs(got[j] - expect[j]) <= 1e-13 * scale, (x, y, z, j)
    for i in (node(0, 3, 3), node(4, 8, 2), node(5, 5, 0), node(3, 3, c - 1)):
        assert A.row_ptr[i + 1] - A.row_ptr[i] == 1
        assert A.col_idx[A.row_ptr[i]] == i and A.val[A.row_ptr[i]] == 1.0
