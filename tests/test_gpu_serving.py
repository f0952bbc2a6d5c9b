"""GPU tests of the continuous-batching solve server: served results against
the CPU oracle, the same bits alone and in a mix without grouping (and the
same as the batched path), grouped requests on one matrix against the
oracle and against their ungrouped results, memory admission, and requests
admitted while others run."""
import threading
import time

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


def pool(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def resident():
    mats = [synth.q1cube(N, 1.0, 2000 + i) for i, N in enumerate((12, 22, 31, 40))]
    return mats, [cgx.DeviceCSR.from_host(A) for A in mats]


def test_served_results_match_oracle(resident):
    mats, dmats = resident
    opts = cgx.make_opts(rtol=1e-8)
    with cgx.Server(pool(1 << 28), max_slots=8) as srv:
        reqs = []
        for i in range(10):
            k = i % 4
            b = synth.uniform(50 + i, mats[k].n_rows)
            x = torch.zeros(mats[k].n_rows, dtype=torch.float64, device="cuda")
            reqs.append((k, b, x, srv.submit(dmats[k], dev(b), x, opts)))
        for k, b, x, t in reqs:
            st = srv.wait(t)
            ref = oracle.cg(mats[k], b, rtol=1e-8)
            assert st.status == cgx.OK and st.path == 4
            assert abs(st.iters - ref.iters) <= 2
            assert true_relres(mats[k], b, x.cpu().numpy()) <= 1.5e-8
            assert st.latency_ms >= st.queue_ms >= 0.0


def test_alone_equals_mix_equals_batched(resident):
    mats, dmats = resident
    opts = cgx.make_opts(rtol=1e-10, precond=cgx.PRECOND_JACOBI)
    b = dev(synth.uniform(77, mats[2].n_rows))
    h = cgx.Handle()
    # alone
    x_alone = torch.zeros_like(b)
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        st_alone = srv.wait(srv.submit(dmats[2], b, x_alone, opts))
    # in a mix, arriving while others run
    x_mix = torch.zeros_like(b)
    others = []
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        for i in range(6):
            k = i % 4
            bo = dev(synth.uniform(300 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append((bo, xo, srv.submit(dmats[k], bo, xo, opts)))
        time.sleep(0.002)
        t = srv.submit(dmats[2], b, x_mix, opts)
        for i in range(4):
            k = (i + 1) % 4
            bo = dev(synth.uniform(400 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append((bo, xo, srv.submit(dmats[k], bo, xo, opts)))
        st_mix = srv.wait(t)
        for _, _, to in others:
            assert srv.wait(to).status == cgx.OK
    assert st_alone.status == st_mix.status == cgx.OK
    assert st_alone.iters == st_mix.iters
    assert torch.equal(x_alone, x_mix)
    # the batched path with one right-hand side runs the same arithmetic
    X = torch.zeros(1, b.numel(), dtype=torch.float64, device="cuda")
    st_b = cgx.cg_solve_batched([(dmats[2], b.view(1, -1), X)], opts, handle=h)
    assert st_b[0][0].iters == st_alone.iters
    assert torch.equal(X[0], x_alone)


def test_grouped_requests_match_oracle_and_alone(resident):
    """Requests on one matrix queued behind a running one are admitted as one
    slot (right-hand sides of one multi-RHS solve); each result matches the
    oracle and its ungrouped solve within the tolerance."""
    mats, dmats = resident
    big = synth.q1cube(60, 1.0, 8)
    dbig = cgx.DeviceCSR.from_host(big)
    opts = cgx.make_opts(rtol=1e-12)
    A, dA = mats[1], dmats[1]
    bs = [synth.uniform(800 + i, A.n_rows) for i in range(5)]
    xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _ in bs]
    with cgx.Server(pool(1 << 30), max_slots=1, max_group=16) as srv:
        bb = dev(synth.uniform(9, big.n_rows))
        tb = srv.submit(dbig, bb, torch.zeros_like(bb), opts)  # holds the only slot
        ts = [srv.submit(dA, dev(b), x, opts) for b, x in zip(bs, xs)]
        assert srv.wait(tb).status == cgx.OK
        sts = [srv.wait(t) for t in ts]
    assert all(st.outer_iters == 5 for st in sts)  # one group of five
    for b, x, st in zip(bs, xs, sts):
        ref = oracle.cg(A, b, rtol=1e-12)
        xg = x.cpu().numpy()
        assert st.status == cgx.OK and abs(st.iters - ref.iters) <= 2
        assert true_relres(A, b, xg) <= 1.5e-12
        assert np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x) <= 1e-8
    # ungrouped, one at a time
    with cgx.Server(pool(1 << 28), max_slots=1, max_group=1) as srv:
        for b, x in zip(bs, xs):
            xa = torch.zeros_like(x)
            st = srv.wait(srv.submit(dA, dev(b), xa, opts))
            assert st.outer_iters == 1
            assert (torch.linalg.norm(xa - x) / torch.linalg.norm(xa)).item() <= 1e-8


def test_late_requests_join_a_running_slot():
    """A request arriving while a slot on its matrix runs takes a free lane of
    that slot (started mid-solve of the others) and still matches the oracle."""
    A = synth.q1cube(44, 1.0, 12)  # 85184 rows: its slot keeps a spare lane
    dA = cgx.DeviceCSR.from_host(A)
    opts = cgx.make_opts(rtol=1e-11)
    bs = [synth.uniform(900 + i, A.n_rows) for i in range(4)]
    xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _ in bs]
    dbs = [dev(b) for b in bs]
    with cgx.Server(pool(1 << 30), max_slots=1, max_group=16) as srv:
        c0 = time.perf_counter()
        t0 = srv.submit(dA, dbs[0], xs[0], opts)
        time.sleep(0.002)  # the first request now holds the only slot (one spare lane)
        c1 = time.perf_counter()
        ts = [t0] + [srv.submit(dA, b, x, opts) for b, x in zip(dbs[1:], xs[1:])]
        sts = [srv.wait(t) for t in ts]
    if sts[0].queue_ms * 1e-3 < c1 - c0:
        # the first request was running when the others arrived (the recorded
        # times say so): the second took the spare lane of its slot, the
        # other two waited for the slot and then ran as one group
        assert sts[0].outer_iters == 1
        assert sts[1].outer_iters == 2 and sts[1].queue_ms < sts[0].latency_ms
        assert sts[2].outer_iters == sts[3].outer_iters == 2
    else:
        # admitted only while or after the others arrived: how they grouped
        # depends on that moment; each still shared a slot of at most four
        print("[serving] first request admitted late:", [st.outer_iters for st in sts],
              flush=True)
        assert all(1 <= st.outer_iters <= 4 for st in sts), [st.as_dict() for st in sts]
    for b, x, st in zip(bs, xs, sts):
        ref = oracle.cg(A, b, rtol=1e-11)
        xg = x.cpu().numpy()
        # the multi-RHS SpMM sums in another order than the oracle: where the
        # run stopped is gated by the oracle's own residual history and its
        # rounding sensitivity (tests/cg_gates.py), not by an iteration count
        h, F = residual_band(A, b, 1e-11)
        assert st.status == cgx.OK
        assert_stop_in_band(h, F, st.iters, 1e-11, st.as_dict())
        assert true_relres(A, b, xg) <= 1.5e-11
        assert np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x) <= 1e-7


def test_admission_by_memory(resident):
    mats, dmats = resident
    need = cgx.Server.request_bytes(mats[3].n_rows)
    # room for the tables plus about two of the largest requests
    with cgx.Server(pool(need * 2 + (8 << 20)), max_slots=16) as srv:
        big = synth.fd7(100)  # 1e6 rows: more than the whole pool
        dbig = cgx.DeviceCSR.from_host(big)
        with pytest.raises(cgx.CgxError) as ei:
            srv.submit(dbig, dev(np.ones(big.n_rows)), torch.zeros(big.n_rows, dtype=torch.float64,
                                                                    device="cuda"))
        assert ei.value.code == cgx.ENOMEM
        ts = []
        for i in range(8):
            b = dev(synth.uniform(500 + i, mats[3].n_rows))
            x = torch.zeros_like(b)
            ts.append((b, x, srv.submit(dmats[3], b, x, cgx.make_opts(rtol=1e-8))))
        for b, x, t in ts:
            st = srv.wait(t)
            assert st.status == cgx.OK
            assert true_relres(mats[3], b.cpu().numpy(), x.cpu().numpy()) <= 1.5e-8


def test_small_requests_overtake_a_large_one(resident):
    """Continuous batching: small requests submitted after a large one start
    while it runs and finish first."""
    mats, dmats = resident
    big = synth.q1cube(80, 1.0, 3)
    dbig = cgx.DeviceCSR.from_host(big)
    opts = cgx.make_opts(rtol=1e-10)
    with cgx.Server(pool(1 << 30), max_slots=8) as srv:
        bb = dev(synth.uniform(9, big.n_rows))
        xb = torch.zeros_like(bb)
        tb = srv.submit(dbig, bb, xb, opts)
        time.sleep(0.02)
        small = []
        for i in range(4):
            b = dev(synth.uniform(600 + i, mats[0].n_rows))
            x = torch.zeros_like(b)
            small.append((b, x, srv.submit(dmats[0], b, x, opts)))
        st_small = [srv.wait(t) for _, _, t in small]
        st_big = srv.wait(tb)
    assert st_big.status == cgx.OK and all(s.status == cgx.OK for s in st_small)
    # ordering from the recorded times: every small request finished before
    # the large one, which was submitted first (its latency spans theirs)
    assert max(s.latency_ms for s in st_small) < st_big.latency_ms
    assert all(s.queue_ms < 50.0 for s in st_small)


def test_poll_unknown_ticket_and_restart():
    h = cgx.Handle()
    srv = cgx.Server(pool(1 << 24), max_slots=2, handle=h)
    with pytest.raises(cgx.CgxError):
        srv.poll(12345)
    srv.stop()
    srv2 = cgx.Server(pool(1 << 24), max_slots=2, handle=h)
    A = synth.fd7(10)
    dA = cgx.DeviceCSR.from_host(A)
    b = dev(synth.uniform(1, A.n_rows))
    x = torch.zeros_like(b)
    assert srv2.wait(srv2.submit(dA, b, x)).status == cgx.OK
    srv2.stop()


def test_wait_returns_the_error_when_tuning_fails():
    """A tuning failure in the progress thread (forced from the host before any
    launch) wakes a thread blocked in cgx_wait with the error instead of
    leaving it blocked; later polls and the stop report it too."""
    h = cgx.Handle()
    cgx.debug_fail_tuning(1, handle=h)
    A = synth.fd7(12)
    dA = cgx.DeviceCSR.from_host(A)
    b = dev(synth.uniform(3, A.n_rows))
    x = torch.zeros_like(b)
    srv = cgx.Server(pool(1 << 26), max_slots=2, handle=h)
    t = srv.submit(dA, b, x)
    out = {}

    def waiter():
        try:
            out["st"] = srv.wait(t)
        except cgx.CgxError as e:
            out["err"] = e.code

    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    th.join(timeout=30.0)
    assert not th.is_alive(), "cgx_wait stayed blocked after the tuning failure"
    assert out.get("err") == cgx.EHIP, out
    with pytest.raises(cgx.CgxError) as ei:
        srv.stop()
    assert ei.value.code == cgx.EHIP
    # the handle serves again once the hook is spent
    with cgx.Server(pool(1 << 26), max_slots=2, handle=h) as srv2:
        assert srv2.wait(srv2.submit(dA, b, x)).status == cgx.OK


@pytest.mark.parametrize("N", [101, 159])
def test_large_request_in_a_mix(N):
    """The serving workload's range of sizes: a Q1 request of 1.03 M (N = 101)
    or 4.02 M rows (N = 159, the top of the 1e4 .. 4e6 range) served with
    small requests arriving around it.  Its true residual (oracle SpMV) meets
    the tolerance, and ungrouped (max_group 1) its result has the same bits
    alone and in the mix; the small requests match the oracle."""
    A = synth.q1cube(N, 1.0, 2100 + N)
    dA = cgx.DeviceCSR.from_host(A)
    smalls = [synth.q1cube(M, 1.0, 2200 + M) for M in (12, 17, 22)]
    dsm = [cgx.DeviceCSR.from_host(S) for S in smalls]
    opts = cgx.make_opts(rtol=1e-8)
    b = dev(synth.uniform(2300 + N, A.n_rows))
    h = cgx.Handle()
    psize = 4 * cgx.Server.request_bytes(A.n_rows) + (64 << 20)
    x_alone = torch.zeros_like(b)
    with cgx.Server(pool(psize), max_slots=8, handle=h, max_group=1) as srv:
        st_alone = srv.wait(srv.submit(dA, b, x_alone, opts))
    assert st_alone.status == cgx.OK
    x_mix = torch.zeros_like(b)
    others = []
    with cgx.Server(pool(psize), max_slots=8, handle=h, max_group=1) as srv:
        for i in range(3):
            bo = synth.uniform(2400 + i, smalls[i].n_rows)
            xo = torch.zeros(smalls[i].n_rows, dtype=torch.float64, device="cuda")
            others.append((i, bo, xo, srv.submit(dsm[i], dev(bo), xo, opts)))
        t = srv.submit(dA, b, x_mix, opts)
        time.sleep(0.005)
        for i in range(3, 9):
            k = i % 3
            bo = synth.uniform(2400 + i, smalls[k].n_rows)
            xo = torch.zeros(smalls[k].n_rows, dtype=torch.float64, device="cuda")
            others.append((k, bo, xo, srv.submit(dsm[k], dev(bo), xo, opts)))
        st_mix = srv.wait(t)
        st_others = [(k, bo, xo, srv.wait(to)) for k, bo, xo, to in others]
    assert st_mix.status == cgx.OK and st_mix.iters == st_alone.iters
    assert torch.equal(x_alone, x_mix)
    xb = x_mix.cpu().numpy()
    assert true_relres(A, b.cpu().numpy(), xb) <= 1.5e-8
    for k, bo, xo, st in st_others:
        ref = oracle.cg(smalls[k], bo, rtol=1e-8)
        assert st.status == cgx.OK and abs(st.iters - ref.iters) <= 2, (k, st.iters, ref.iters)
        assert true_relres(smalls[k], bo, xo.cpu().numpy()) <= 1.5e-8
