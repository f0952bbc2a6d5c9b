"""Host-side checks of the benchmark driver (no GPU): the byte models it
reports against counts of the arrays they stand for, the wave-tile rows it
names against the library's rule, the byte-counter lookup keyed by the
kernel sources, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("make", [lambda: synth.fd7(7), lambda: synth.q1cube(6, 1.0, 1)])
def test_byte_models_count_the_arrays(make):
    """SpMV: every stored value and column index once, the row pointers, x
    and y once.  Jacobi-CG iteration: the SpMV plus the vectors the update
    (x, r read and written, p, q, D^-1 read, z written) and the p update (z
    and p read, p written) touch."""
    A = make()
    n, nnz = A.n_rows, A.nnz
    arrays = A.val.nbytes + A.col_idx.nbytes + A.row_ptr.nbytes + 2 * 8 * n
    assert bench.spmv_bytes(n, nnz) == arrays
    assert bench.jacobi_iter_bytes(n, nnz) == arrays + 8 * n * (2 * 2 + 3 + 1) + 8 * n * 3
    assert bench.jacobi_setup_bytes(n, nnz) == arrays + 8 * n + 8 * n * 4


def test_wave_tile_rows_rule():
    """The largest power of two up to 64 whose expected entries fill at most
    97 % of 64 x 8: 16 rows for the 27-point Q1 rows, 64 for the 7-point
    rows, one row when a mean row exceeds the chunk."""
    assert bench.wave_tile_rows(2_097_152, 55_742_968) == 16
    assert bench.wave_tile_rows(4096, 27136) == 64
    assert bench.wave_tile_rows(100, 100 * 600) == 1
    for rt in (1, 2, 4, 8, 16, 32, 64):
        mean = 0.97 * 64 * 8 / rt
        assert bench.wave_tile_rows(1000, int(1000 * mean)) == rt


def test_traffic_lookup_is_keyed_by_the_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    t = bench.measured_traffic(h)
    if t is not None:  # the committed counters were taken on these sources
        alg = bench.spmv_bytes(2_097_152, 55_742_968)
        assert 0.9 * alg <= t <= 1.2 * alg
    assert bench.measured_traffic("0" * 16) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_host_residual_matches_the_oracle():
    """The residual the extras report (scipy's CSR product on the host) is
    the oracle's ||b - A x|| / ||b|| up to rounding."""
    import oracle
    A = synth.q1cube(8, 1.0, 3)
    b = synth.uniform(4, A.n_rows)
    x = oracle.cg(A, b, rtol=1e-6).x
    ref = float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))
    assert abs(bench.host_relres(A, b, x) - ref) <= 1e-9 * ref
    assert bench.host_relres(A, b, np.zeros(A.n_rows)) == 1.0


def test_only_the_cpu_baseline_uses_the_oracle():
    """Apart from the CPU baselines (one core, all cores; headline, small
    system, BLAS-1, batched and mixed-precision samples), no part of the
    benchmark imports the oracle."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    names = [a.name for a in node.names] + [getattr(node, "module", None) or ""]
                    if any(n == "oracle" or n.startswith("oracle.") for n in names):
                        users.add(fn.name)
    assert users == {"cpu_baseline", "cpu_baseline_all_cores", "cpu_baseline_batched",
                     "cpu_baseline_mixed", "cpu_baseline_small", "cpu_baseline_blas1"}


def test_batch_sample_spans_both_stencils():
    """The one-at-a-time sample of the batch holds both stencils (the stencil
    alternates with the system index) and distinct systems."""
    pick = bench.batch_sample()
    assert len(set(pick)) == len(pick) == 8 and all(0 <= s < 64 for s in pick)
    assert {s % 2 for s in pick} == {0, 1}


def test_oracle_timing_build_matches_the_oracle():
    """The all-cores timing build of oracle.c runs the same CG (rows and
    elements in parallel, dot partials per thread): the same iterates up to
    rounding; the default build stays sequential."""
    import oracle
    import synth
    assert oracle._load().oracle_threads() == 1
    assert oracle.timing_threads() >= 1
    A = synth.q1cube(14, 1.0, 3)
    b = synth.uniform(9, A.n_rows)
    ref = oracle.cg(A, b, rtol=1e-9, jacobi=True)
    tim = oracle.cg_timing(A, b, rtol=1e-9, jacobi=True)
    assert tim.status == oracle.OK and abs(tim.iters - ref.iters) <= 2
    assert np.linalg.norm(tim.x - ref.x) / np.linalg.norm(ref.x) <= 1e-7
