"""GPU parity of the batched reliable-update solve (binary32 CG per (system,
right-hand side) whose direction is kept across float64 updates of x, the
true residual and the stopping test, all right-hand sides advanced together,
an update of one right-hand side taken by all of its system) against the
oracle's mixed_ru_block run on each system's right-hand sides.

Bars, as for the single-system reliable-update solve: the true residual
(the oracle's float64 SpMV on the GPU solution) below the tolerance; the
solution within the kappa * rtol bound of the float64 oracle; the step where
the run stopped inside the band of the oracle's own residual history and its
rounding sensitivity (tests/cg_gates.py; in exact arithmetic the history of a
right-hand side does not depend on where updates are taken); the update
count within the slack of the oracle's own reordered run (cg_gates.
ru_block_refs) and, exactly, a strictly increasing function of the stopping
step over a system's right-hand sides (each takes every event up to its
stop); and a system's result bit-identical alone and inside the batch."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from cg_gates import assert_stop_in_band, assert_updates_shared, residual_band, ru_block_refs
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu

MATS = [lambda: synth.q1cube(12, 1.5, 21), lambda: synth.fd7_var(14, 1.0, 22),
        lambda: synth.q1cube(17, 1.0, 23), lambda: synth.fd7_var(9, 1.0, 24)]
NRHS = [3, 16, 1, 5]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ru_opts(rtol=1e-10, jacobi=True, delta=1e-2, **kw):
    return cgx.make_opts(rtol=rtol, precond=int(jacobi), precision=cgx.PRECISION_MIXED_RU,
                         inner_rtol=delta, **kw)


def make_items(mats, nrhs, seed, zero_last=False):
    items, hostB = [], []
    for s, (A, k) in enumerate(zip(mats, nrhs)):
        B = np.stack([synth.uniform(seed + 19 * s + j, A.n_rows) for j in range(k)])
        if zero_last and s == len(mats) - 1:
            B[1] = 0.0
        hostB.append(B)
        items.append((cgx.DeviceCSR.from_host(A, with_f32=True), dev(B),
                      torch.zeros(k, A.n_rows, dtype=torch.float64, device="cuda")))
    return items, hostB


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


@pytest.mark.parametrize("jacobi,delta", [(True, 1e-2), (False, 1e-2), (True, 0.1)],
                         ids=["jacobi", "plain", "jacobi_delta0.1"])
def test_batched_ru_vs_oracle(jacobi, delta):
    mats = [f() for f in MATS]
    items, hostB = make_items(mats, NRHS, seed=900, zero_last=True)
    rtol = 1e-10
    print(f"[batched ru] jacobi={jacobi} delta={delta}", flush=True)
    st = cgx.cg_solve_batched(items, ru_opts(rtol, jacobi, delta))
    for s, (A, (dA, dB, dX)) in enumerate(zip(mats, items)):
        X = dX.cpu().numpy()
        refs, slack = ru_block_refs(A, hostB[s], rtol, delta, jacobi)
        assert_updates_shared([(v.iters, v.outer_iters) for v, b in zip(st[s], hostB[s])
                               if b.any()], (s, jacobi, delta))
        for j in range(NRHS[s]):
            b = hostB[s][j]
            v = st[s][j]
            info = (s, j, v.as_dict())
            assert v.status == cgx.OK and v.path == 3, info
            if not b.any():
                assert not X[j].any() and v.iters == 0, info
                continue
            ref = refs[j]
            assert ref.status == oracle.OK
            tr = true_relres(A, b, X[j])
            assert tr <= rtol, info
            assert abs(v.relres - tr) <= 1e-3 * tr + 1e-16, info
            assert abs(v.outer_iters - ref.outer_iters) <= slack, (info, ref.outer_iters, slack)
            xs = oracle.cg(A, b, rtol=1e-13, jacobi=True, maxit=20000).x
            assert np.linalg.norm(X[j] - xs) <= 1e-6 * np.linalg.norm(xs), info
            if j == 0:  # the stopping step, gated by the oracle's own history
                h, F = residual_band(A, b, rtol, solve=lambda M, w, t: oracle.mixed_ru(
                    M, M.val.astype(np.float32), w, rtol=t, delta=delta, jacobi=jacobi,
                    history=True).relres_hist)
                assert_stop_in_band(h, F, v.iters, rtol, (v.iters, ref.iters))


@pytest.mark.parametrize("nrhs,schedule", [(16, -4), (16, -1), (8, -8), (4, -16), (1, -64),
                                           (3, -8), (16, 1)])
def test_batched_ru_schedules_vs_oracle(nrhs, schedule):
    """Reliable updates with each SpMM schedule forced (the float64 setup and
    the update residual then run on the SpMM's wave tiles of that shape, or
    on vector CSR for the positive schedule): the bars of the test above."""
    mats = [synth.q1cube(11, 1.0, 31), synth.fd7_var(15, 1.0, 32)]
    items, hostB = make_items(mats, [nrhs, nrhs], seed=720)
    items = [it + (schedule,) for it in items]
    rtol = 1e-10
    print(f"[batched ru] nrhs={nrhs} schedule={schedule}", flush=True)
    st = cgx.cg_solve_batched(items, ru_opts(rtol, True, 1e-2))
    for s, (A, it) in enumerate(zip(mats, items)):
        X = it[2].cpu().numpy()
        refs, slack = ru_block_refs(A, hostB[s], rtol, 1e-2, True)
        assert_updates_shared([(v.iters, v.outer_iters) for v in st[s]], (s, nrhs, schedule))
        for j in range(nrhs):
            v = st[s][j]
            info = (s, j, v.as_dict())
            assert v.status == cgx.OK, info
            b = hostB[s][j]
            tr = true_relres(A, b, X[j])
            assert tr <= rtol, info
            assert abs(v.relres - tr) <= 1e-3 * tr + 1e-16, info
            assert abs(v.outer_iters - refs[j].outer_iters) <= slack, (info, refs[j].outer_iters)
            xs = oracle.cg(A, b, rtol=1e-13, jacobi=True, maxit=20000).x
            assert np.linalg.norm(X[j] - xs) <= 1e-6 * np.linalg.norm(xs), info


def test_batched_ru_alone_equals_in_batch():
    mats = [f() for f in MATS]
    items, _ = make_items(mats, NRHS, seed=950)
    opts = ru_opts()
    print("[batched ru] alone vs in the batch", flush=True)
    st_mix = cgx.cg_solve_batched(items, opts)
    for s in (0, 1, 3):
        dA, dB, dX = items[s]
        X_mix = dX.clone()
        X1 = torch.zeros_like(dX)
        st1 = cgx.cg_solve_batched([(dA, dB, X1)], opts)
        assert torch.equal(X1, X_mix), s
        assert [(v.iters, v.outer_iters) for v in st1[0]] == \
            [(v.iters, v.outer_iters) for v in st_mix[s]]


def test_batched_ru_keeps_krylov_space():
    """Binary32 iterations near float64 CG's, fewer than the restarted
    refinement's at the same tolerance (over the four right-hand sides: the
    oracle's two methods differ by 17-24 % on each of them here)."""
    A = synth.q1cube(30, 1.5, seed=synth.SEED_C3_COEFF)
    B = np.stack([synth.uniform(960 + j, A.n_rows) for j in range(4)])
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    counts = {}
    for name, o in (("fp64", cgx.make_opts(rtol=1e-10, precond=1)),
                    ("ru", ru_opts()),
                    ("ir", cgx.make_opts(rtol=1e-10, precond=1, inner_rtol=1e-2,
                                         precision=cgx.PRECISION_MIXED))):
        X = torch.zeros(4, A.n_rows, dtype=torch.float64, device="cuda")
        st = cgx.cg_solve_batched([(dA, dev(B), X)], o)
        assert all(v.status == cgx.OK for v in st[0]), name
        counts[name] = [v.iters for v in st[0]]
    for j in range(4):
        assert counts["ru"][j] <= 1.1 * counts["fp64"][j] + 2, counts
    assert sum(counts["ir"]) >= 1.15 * sum(counts["ru"]), counts


def test_batched_ru_sibling_event_and_cap():
    """A discrete eigenvector of the 7-point operator converges in one binary32
    step and fires an update there: its sibling takes that update, also when
    the iteration cap stops it at that step (status, counts and the folded
    correction as in the oracle's block method)."""
    N = 9
    A = synth.fd7(N)
    i = np.arange(1, N + 1)
    vs = [np.sin(jj * math.pi * i / (N + 1)) for jj in (2, 5, 7)]
    v = np.einsum("k,j,i->kji", vs[2], vs[1], vs[0]).ravel()
    lam = sum(4 * math.sin(jj * math.pi / (2 * (N + 1))) ** 2 for jj in (2, 5, 7))
    B = np.stack([synth.uniform(60, A.n_rows), lam * v])
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    v32 = A.val.astype(np.float32)
    print("[batched ru] sibling event, uncapped and capped at it", flush=True)
    for maxit in (0, 1):
        X = torch.zeros(2, A.n_rows, dtype=torch.float64, device="cuda")
        st = cgx.cg_solve_batched([(dA, dev(B), X)], ru_opts(rtol=1e-6, jacobi=False,
                                                              maxit=maxit))[0]
        refs = oracle.mixed_ru_block(A, v32, B, rtol=1e-6, delta=1e-2, maxit=maxit)
        Xh = X.cpu().numpy()
        assert (st[1].status, st[1].iters, st[1].outer_iters) == (cgx.OK, 1, 1), st[1].as_dict()
        assert true_relres(A, B[1], Xh[1]) <= 1e-6
        if maxit == 1:
            assert (refs[0].status, refs[0].outer_iters) == (oracle.NOT_CONVERGED, 1)
            assert (st[0].status, st[0].iters, st[0].outer_iters) == \
                (cgx.NOT_CONVERGED, 1, 1), st[0].as_dict()
            tr = true_relres(A, B[0], Xh[0])
            assert abs(st[0].relres - tr) <= 1e-6 * tr
            # the step's correction is in x: the oracle's x within binary32 rounding
            assert np.linalg.norm(Xh[0] - refs[0].x) <= 1e-4 * np.linalg.norm(refs[0].x)
        else:
            assert st[0].status == cgx.OK and true_relres(A, B[0], Xh[0]) <= 1e-6
            assert st[0].outer_iters >= 2  # the event at step 1, then its own


def test_batched_ru_caps_and_errors():
    A = synth.q1cube(12, 1.0, seed=1)
    n = A.n_rows
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    B = np.stack([synth.uniform(2, n), synth.uniform(3, n)])
    print("[batched ru] caps", flush=True)
    X = torch.zeros(2, n, dtype=torch.float64, device="cuda")
    st = cgx.cg_solve_batched([(dA, dev(B), X)], ru_opts(rtol=1e-15, jacobi=False, maxit=7))
    for j in range(2):
        assert st[0][j].status == cgx.NOT_CONVERGED and st[0][j].iters == 7
        # the correction of the unfinished cycle is kept; relres is the true one
        tr = true_relres(A, B[j], X[j].cpu().numpy())
        assert abs(st[0][j].relres - tr) <= 1e-6 * tr and tr < 0.9
        ref = oracle.mixed_ru(A, A.val.astype(np.float32), B[j], rtol=1e-15, delta=1e-2,
                              maxit=7)
        assert ref.status == oracle.NOT_CONVERGED and ref.iters == 7
    X.zero_()
    st = cgx.cg_solve_batched([(dA, dev(B), X)], ru_opts(rtol=1e-15, jacobi=False,
                                                          max_outer=2))
    assert all(v.status == cgx.NOT_CONVERGED and v.outer_iters == 2 for v in st[0])
    neg = synth.CSR(n, n, A.row_ptr, A.col_idx, -A.val)
    dneg = cgx.DeviceCSR.from_host(neg, with_f32=True)
    X.zero_()
    st = cgx.cg_solve_batched([(dneg, dev(B), X)], ru_opts(jacobi=True))
    assert all(v.status == cgx.BREAKDOWN for v in st[0])
    d64 = cgx.DeviceCSR.from_host(A)  # no val32
    with pytest.raises(cgx.CgxError):
        cgx.cg_solve_batched([(d64, dev(B), X)], ru_opts(),
                             workspace=torch.empty(1 << 22, dtype=torch.uint8, device="cuda"))


def test_batched_ru_64_systems_16_rhs_full_size():
    """The batched configuration with reliable updates (binary32 Jacobi-CG,
    delta 1e-2): every (system, right-hand side) converges to 1e-8 in
    float64, gated on a sample through the oracle's SpMV of the GPU solution."""
    mats = synth.batch_systems(64)
    items = []
    for s, A in enumerate(mats):
        B = torch.empty(16, A.n_rows, dtype=torch.float64)
        for j in range(16):
            B[j] = torch.from_numpy(synth.uniform(1000 + s * 16 + j, A.n_rows))
        items.append((cgx.DeviceCSR.from_host(A, with_f32=True), B.cuda(),
                      torch.zeros(16, A.n_rows, dtype=torch.float64, device="cuda")))
    print("[batched ru] 64 x 16 full size", flush=True)
    st = cgx.cg_solve_batched(items, ru_opts(rtol=1e-8))
    assert all(v.status == cgx.OK for row in st for v in row)
    assert all(v.relres <= 1e-8 for row in st for v in row)
    rng = np.random.default_rng(2)
    for s in rng.choice(64, 8, replace=False):
        for j in rng.choice(16, 2, replace=False):
            b = items[s][1][j].cpu().numpy()
            x = items[s][2][j].cpu().numpy()
            assert true_relres(mats[s], b, x) <= 1e-8 * 1.01
