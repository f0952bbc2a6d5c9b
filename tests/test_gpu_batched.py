"""GPU parity of the batched solve (many systems, up to 16 right-hand sides
each, one launch per phase for the whole batch) against the CPU oracle run
on every (system, right-hand side) separately, plus the property that a
system's result is bit-identical alone and inside a batch."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_items(mats, nrhs, seed=300):
    items, hostB = [], []
    for s, (A, k) in enumerate(zip(mats, nrhs)):
        B = np.stack([synth.uniform(seed + 17 * s + j, A.n_rows) for j in range(k)])
        hostB.append(B)
        items.append((cgx.DeviceCSR.from_host(A), dev(B), torch.zeros(k, A.n_rows,
                                                                     dtype=torch.float64,
                                                                     device="cuda")))
    return items, hostB


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


MATS = [lambda: synth.fd7_var(6, 1.0, 1), lambda: synth.q1cube(9, 1.0, 2),
        lambda: synth.fd7_var(13, 1.0, 3), lambda: synth.q1cube(17, 1.0, 4),
        lambda: synth.fd7_var(30, 1.0, 5), lambda: synth.q1cube(11, 1.0, 6)]
NRHS = [1, 3, 16, 4, 2, 8]


@pytest.mark.parametrize("jacobi", [False, True])
def test_batched_vs_oracle(jacobi):
    mats = [f() for f in MATS]
    items, hostB = make_items(mats, NRHS)
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-9, precond=int(jacobi)))
    for s, (A, (dA, dB, dX)) in enumerate(zip(mats, items)):
        X = dX.cpu().numpy()
        for j in range(NRHS[s]):
            ref = oracle.cg(A, hostB[s][j], rtol=1e-9, jacobi=jacobi)
            assert st[s][j].status == cgx.OK, (s, j, st[s][j].as_dict())
            assert abs(st[s][j].iters - ref.iters) <= 2, (s, j, st[s][j].iters, ref.iters)
            assert true_relres(A, hostB[s][j], X[j]) <= 1.5e-9
            assert np.linalg.norm(X[j] - ref.x) / np.linalg.norm(ref.x) <= 1e-6


def test_batched_alone_equals_in_mix():
    mats = [f() for f in MATS]
    items, hostB = make_items(mats, NRHS, seed=900)
    opts = cgx.make_opts(rtol=1e-10, precond=1)
    st_mix = cgx.cg_solve_batched(items, opts)
    mix = [it[2].cpu().numpy().copy() for it in items]
    for s in (1, 2, 4):
        A, B, X = items[s]
        X.zero_()
        st_alone = cgx.cg_solve_batched([(A, B, X)], opts)
        alone = X.cpu().numpy()
        assert np.array_equal(alone, mix[s]), s
        assert [v.iters for v in st_alone[0]] == [v.iters for v in st_mix[s]]


def test_batched_status_isolation():
    good = synth.q1cube(10, 1.0, 7)
    bad = synth.fd7(8)
    bad = synth.CSR(bad.n_rows, bad.n_cols, bad.row_ptr, bad.col_idx, -bad.val)  # negative definite
    items, hostB = make_items([good, bad, good], [2, 1, 3])
    hostB[2][1][:] = 0.0
    items[2][1][1].zero_()            # a zero right-hand side
    items[2][2][1].fill_(5.0)         # with a nonzero initial guess
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-10))
    assert [v.status for v in st[0]] == [cgx.OK, cgx.OK]
    assert st[1][0].status == cgx.BREAKDOWN
    assert st[2][0].status == cgx.OK and st[2][1].status == cgx.OK and st[2][2].status == cgx.OK
    assert not items[2][2][1].any().item()  # b = 0 gives x = 0
    st = cgx.cg_solve_batched(items[:1], cgx.make_opts(rtol=1e-15, maxit=5))
    assert all(v.status == cgx.NOT_CONVERGED and v.iters == 5 for v in st[0])


def test_batched_schedule_reported():
    mats = [f() for f in MATS[:3]]
    items, _ = make_items(mats, NRHS[:3])
    ms = cgx.batch_schedule(items)
    for M, k in zip(ms, NRHS[:3]):
        K = 1
        while K < k:
            K *= 2
        if M < 0:  # wave tiles: a power of two of rows, at most 64 lanes per row group
            assert -M * K <= 64 and (-M & (-M - 1)) == 0
        else:
            assert M >= 1 and K * M <= 64 and K * M >= 8
    fixed = [items[0] + (-4,), items[1] + (8 // 4,), items[2]]
    ms = cgx.batch_schedule(fixed)
    assert ms[0] == -4 and ms[1] == 2


@pytest.mark.parametrize("schedule", [-16, -64, -1, 8])
def test_single_rhs_schedules_vs_oracle(schedule):
    """One right-hand side per system with each SpMM schedule forced: wave
    tiles of 16, 64 or 1 rows per wavefront and 8 lanes per row."""
    mats = [synth.q1cube(14, 1.0, 21), synth.fd7_var(19, 1.0, 22), synth.q1cube(5, 1.0, 23)]
    items, hostB = make_items(mats, [1, 1, 1], seed=700)
    items = [it + (schedule,) for it in items]
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-10, precond=1))
    for s, A in enumerate(mats):
        X = items[s][2].cpu().numpy()
        ref = oracle.cg(A, hostB[s][0], rtol=1e-10, jacobi=True)
        assert st[s][0].status == cgx.OK
        assert abs(st[s][0].iters - ref.iters) <= 2
        assert true_relres(A, hostB[s][0], X[0]) <= 1.5e-10
        assert np.linalg.norm(X[0] - ref.x) / np.linalg.norm(ref.x) <= 1e-7


def test_schedule_argument_errors():
    mats = [synth.q1cube(6, 1.0, 1)]
    items, _ = make_items(mats, [2])
    for bad in (-64, -3, -2, 3, 64):  # wave rows * K in [16, 64]; K * M in 8..64
        with pytest.raises(cgx.CgxError):
            cgx.cg_solve_batched([items[0] + (bad,)], cgx.make_opts())


@pytest.mark.parametrize("nrhs,schedule", [(16, -4), (16, -1), (8, -8), (4, -16), (2, -32),
                                           (3, -8), (16, 1)])
def test_multi_rhs_schedules_vs_oracle(nrhs, schedule):
    """Several right-hand sides with each SpMM schedule forced: wave tiles of
    64 / K rows (one lane per right-hand side and row) or fewer rows (slices
    combined by butterfly), and the vector-CSR schedule."""
    mats = [synth.q1cube(11, 1.0, 31), synth.fd7_var(15, 1.0, 32)]
    items, hostB = make_items(mats, [nrhs, nrhs], seed=710)
    items = [it + (schedule,) for it in items]
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-10, precond=1))
    for s, A in enumerate(mats):
        X = items[s][2].cpu().numpy()
        for j in range(nrhs):
            ref = oracle.cg(A, hostB[s][j], rtol=1e-10, jacobi=True)
            assert st[s][j].status == cgx.OK
            assert abs(st[s][j].iters - ref.iters) <= 2
            assert true_relres(A, hostB[s][j], X[j]) <= 1.5e-10
            assert np.linalg.norm(X[j] - ref.x) / np.linalg.norm(ref.x) <= 1e-7


def test_batched_64_systems_16_rhs_full_size():
    """The batched configuration: 64 systems, N ~ U{24..96}, 7-point FD (even
    index) and Q1 FEM (odd), lognormal(0,1), 16 right-hand sides U[-1,1] each.
    Gate on a sample of (system, right-hand side) pairs: the oracle's SpMV of
    the GPU solution."""
    mats = synth.batch_systems(64)
    items = []
    for s, A in enumerate(mats):
        B = torch.empty(16, A.n_rows, dtype=torch.float64)
        for j in range(16):
            B[j] = torch.from_numpy(synth.uniform(1000 + s * 16 + j, A.n_rows))
        items.append((cgx.DeviceCSR.from_host(A), B.cuda(),
                      torch.zeros(16, A.n_rows, dtype=torch.float64, device="cuda")))
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-8, precond=1))
    assert all(v.status == cgx.OK for row in st for v in row)
    rng = np.random.default_rng(0)
    for s in rng.choice(64, 8, replace=False):
        for j in rng.choice(16, 2, replace=False):
            b = items[s][1][j].cpu().numpy()
            x = items[s][2][j].cpu().numpy()
            assert true_relres(mats[s], b, x) <= 1.5e-8


@pytest.mark.parametrize("schedule", [2, 4])
def test_batched_graph_reused_only_for_same_layout(schedule):
    """Regression for the cached iteration graph: the same matrices, B / X
    pointers, workspace, schedule and replay length with 4 and then 16
    right-hand sides give equal tile counts but another scalar and partial
    layout, so the second solve must capture its own graph.  Both runs are
    checked against the oracle (and a rerun with 4 reuses the first layout)."""
    mats = [synth.q1cube(9, 1.0, 41), synth.fd7_var(8, 1.0, 42)]
    B16 = [np.stack([synth.uniform(5000 + 31 * s + j, A.n_rows) for j in range(16)])
           for s, A in enumerate(mats)]
    dA = [cgx.DeviceCSR.from_host(A) for A in mats]
    dB = [dev(B) for B in B16]
    dX = [torch.zeros_like(B) for B in dB]
    full = [(dA[s], dB[s], dX[s], schedule) for s in range(2)]
    ws = cgx.batch_workspace(full)
    opts = cgx.make_opts(rtol=1e-9, precond=1, check_every=4)
    for k in (4, 16, 4):
        for X in dX:
            X.zero_()
        items = [(dA[s], dB[s][:k], dX[s][:k], schedule) for s in range(2)]
        st = cgx.cg_solve_batched(items, opts, workspace=ws)
        for s, A in enumerate(mats):
            X = dX[s][:k].cpu().numpy()
            for j in range(k):
                ref = oracle.cg(A, B16[s][j], rtol=1e-9, jacobi=True)
                assert st[s][j].status == cgx.OK, (k, s, j, st[s][j].as_dict())
                assert abs(st[s][j].iters - ref.iters) <= 2, (k, s, j, st[s][j].iters, ref.iters)
                assert true_relres(A, B16[s][j], X[j]) <= 1.5e-9, (k, s, j)
