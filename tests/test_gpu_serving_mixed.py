"""GPU tests of binary32 requests in the solve server: restarted refinement
(MIXED: float64 residual, update and stopping test per request, binary32
inner CG of all such requests in the batched kernels) and reliable updates
(MIXED_RU: one binary32 CG per request, float64 updates inside the
iteration; bars at the end of the file).

Bars, as for the float32-refined batch: the float64 true residual (the
oracle's SpMV on the served solution) <= rtol; the solution within 1e-6 of
the float64 oracle CG; refinement steps within one of the oracle's
mixed-precision refinement (its inner sums run in another order, so an inner
solve may stop an iteration earlier or later); the same bits alone and in a
mix without grouping; caps, breakdown and argument errors as the oracle and
the header state them."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from cg_gates import assert_updates_shared, ru_block_refs
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pool(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


def mixed_opts(rtol=1e-10, jacobi=True, inner_rtol=1e-3, **kw):
    return cgx.make_opts(rtol=rtol, precond=int(jacobi), precision=cgx.PRECISION_MIXED,
                         inner_rtol=inner_rtol, **kw)


@pytest.fixture(scope="module")
def resident():
    mats = [synth.q1cube(11, 1.0, 3100), synth.fd7_var(17, 1.0, 3101),
            synth.q1cube(24, 1.0, 3102), synth.fd7_var(9, 1.0, 3103)]
    return mats, [cgx.DeviceCSR.from_host(A, with_f32=True) for A in mats]


def check_against_oracle(A, b, x, st, rtol, jacobi, inner_rtol, x0=None):
    info = st.as_dict()
    ref = oracle.mixed_ir(A, A.val.astype(np.float32), b, x0=x0, rtol=rtol, tau=inner_rtol,
                          jacobi=jacobi)
    xs = oracle.cg(A, b, rtol=1e-13, jacobi=True).x
    assert ref.status == oracle.OK
    assert st.status == cgx.OK and st.path == 4, info
    assert abs(st.outer_iters - ref.outer_iters) <= 1, (info, ref.outer_iters)
    assert true_relres(A, b, x) <= rtol * 1.01, info
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs), info
    assert st.relres <= rtol
    assert abs(st.relres - true_relres(A, b, x)) <= 1e-3 * rtol + 1e-14


@pytest.mark.parametrize("jacobi", [False, True], ids=["plain", "jacobi"])
def test_served_mixed_matches_oracle(resident, jacobi):
    mats, dmats = resident
    opts = mixed_opts(jacobi=jacobi)
    print(f"[served mixed] oracle parity jacobi={jacobi}", flush=True)
    with cgx.Server(pool(1 << 28), max_slots=6) as srv:
        reqs = []
        for i in range(8):
            k = i % 4
            b = synth.uniform(3200 + i, mats[k].n_rows)
            x = torch.zeros(mats[k].n_rows, dtype=torch.float64, device="cuda")
            reqs.append((k, b, x, srv.submit(dmats[k], dev(b), x, opts)))
        for k, b, x, t in reqs:
            st = srv.wait(t)
            check_against_oracle(mats[k], b, x.cpu().numpy(), st, 1e-10, jacobi, 1e-3)
            assert st.slot_requests >= 1 and st.latency_ms >= st.queue_ms >= 0.0


def test_served_mixed_initial_guess_and_zero_rhs(resident):
    """x holds x0 on submission; b = 0 gives x = 0 without a step."""
    mats, dmats = resident
    A, dA = mats[2], dmats[2]
    b = synth.uniform(3300, A.n_rows)
    x0 = synth.uniform(3301, A.n_rows)
    x = dev(x0)
    xz = dev(synth.uniform(3302, A.n_rows))
    with cgx.Server(pool(1 << 28), max_slots=4) as srv:
        t = srv.submit(dA, dev(b), x, mixed_opts())
        tz = srv.submit(dA, torch.zeros_like(x), xz, mixed_opts())
        st, stz = srv.wait(t), srv.wait(tz)
    check_against_oracle(A, b, x.cpu().numpy(), st, 1e-10, True, 1e-3, x0=x0)
    assert stz.status == cgx.OK and stz.outer_iters == 0 and not xz.any()


def test_served_mixed_alone_equals_mix(resident):
    """Without grouping a MIXED request gets the same bits alone and among
    float64 and MIXED requests that arrive before and after it."""
    mats, dmats = resident
    opts = mixed_opts()
    b = dev(synth.uniform(3400, mats[2].n_rows))
    h = cgx.Handle()
    x_alone = torch.zeros_like(b)
    print("[served mixed] alone", flush=True)
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        st_alone = srv.wait(srv.submit(dmats[2], b, x_alone, opts))
    x_mix = torch.zeros_like(b)
    others = []
    print("[served mixed] in a mix", flush=True)
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        for i in range(6):
            k = i % 4
            o = opts if i % 2 else cgx.make_opts(rtol=1e-10, precond=1)
            bo = dev(synth.uniform(3500 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append(srv.submit(dmats[k], bo, xo, o))
        time.sleep(0.002)
        t = srv.submit(dmats[2], b, x_mix, opts)
        for i in range(4):
            k = (i + 1) % 4
            bo = dev(synth.uniform(3600 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append(srv.submit(dmats[k], bo, xo, opts))
        st_mix = srv.wait(t)
        for to in others:
            assert srv.wait(to).status == cgx.OK
    assert st_alone.status == st_mix.status == cgx.OK
    assert (st_alone.iters, st_alone.outer_iters) == (st_mix.iters, st_mix.outer_iters)
    assert torch.equal(x_alone, x_mix)


def test_served_mixed_grouped(resident):
    """MIXED requests on one matrix queued behind a running one share a slot
    (right-hand sides of the binary32 multi-RHS solve), each with its own
    float64 steps; each matches the oracle."""
    mats, dmats = resident
    big = synth.q1cube(50, 1.0, 3700)
    dbig = cgx.DeviceCSR.from_host(big, with_f32=True)
    A, dA = mats[1], dmats[1]
    opts = mixed_opts()
    bs = [synth.uniform(3800 + i, A.n_rows) for i in range(5)]
    xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _ in bs]
    print("[served mixed] grouped", flush=True)
    with cgx.Server(pool(1 << 30), max_slots=1, max_group=16) as srv:
        bb = synth.uniform(3801, big.n_rows)
        xb = torch.zeros(big.n_rows, dtype=torch.float64, device="cuda")
        tb = srv.submit(dbig, dev(bb), xb, opts)  # holds the only slot
        ts = [srv.submit(dA, dev(b), x, opts) for b, x in zip(bs, xs)]
        stb = srv.wait(tb)
        sts = [srv.wait(t) for t in ts]
    check_against_oracle(big, bb, xb.cpu().numpy(), stb, 1e-10, True, 1e-3)
    assert stb.slot_requests == 1
    for b, x, st in zip(bs, xs, sts):
        assert st.slot_requests == 5
        check_against_oracle(A, b, x.cpu().numpy(), st, 1e-10, True, 1e-3)


def test_served_mixed_caps_and_errors(resident):
    mats, dmats = resident
    A, dA = mats[0], dmats[0]
    b = synth.uniform(3900, A.n_rows)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    print("[served mixed] outer cap", flush=True)
    with cgx.Server(pool(1 << 26), max_slots=2) as srv:
        st = srv.wait(srv.submit(dA, dev(b), x, mixed_opts(rtol=1e-14, jacobi=False,
                                                             inner_rtol=1e-2, max_outer=2)))
        assert st.status == cgx.NOT_CONVERGED and st.outer_iters == 2
        ref = oracle.mixed_ir(A, A.val.astype(np.float32), b, rtol=1e-14, tau=1e-2, max_outer=2)
        assert ref.outer_iters == 2 and ref.status == oracle.NOT_CONVERGED
        xh = x.cpu().numpy()
        assert true_relres(A, b, xh) <= 1e-3 and true_relres(A, b, ref.x) <= 1e-3
        assert abs(st.relres - true_relres(A, b, xh)) <= 1e-6
        # a nonpositive diagonal entry: Jacobi breakdown, as the oracle reports it
        Bad = synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.copy())
        r = 5
        d = [k for k in range(A.row_ptr[r], A.row_ptr[r + 1]) if A.col_idx[k] == r][0]
        Bad.val[d] = -1.0
        dBad = cgx.DeviceCSR.from_host(Bad, with_f32=True)
        xb = torch.zeros_like(x)
        stb = srv.wait(srv.submit(dBad, dev(b), xb, mixed_opts()))
        assert stb.status == cgx.BREAKDOWN
        assert oracle.mixed_ir(Bad, Bad.val.astype(np.float32), b, jacobi=True).status == \
            oracle.BREAKDOWN
        # no binary32 values: refused at submission
        d64 = cgx.DeviceCSR.from_host(A)
        with pytest.raises(cgx.CgxError):
            srv.submit(d64, dev(b), torch.zeros_like(x), mixed_opts())
        with pytest.raises(cgx.CgxError):
            srv.submit(dA, dev(b), torch.zeros_like(x), mixed_opts(inner_rtol=1.5))


def test_served_mixed_million_rows_in_a_mix():
    """A Q1 request of 1,030,301 rows (N = 101), MIXED, served with small
    float64 and MIXED requests; gated by the oracle's SpMV of the served
    solution."""
    A = synth.q1cube(101, 1.0, 4000)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    small = [synth.q1cube(16, 1.0, 4001 + i) for i in range(3)]
    dsmall = [cgx.DeviceCSR.from_host(S, with_f32=True) for S in small]
    b = synth.uniform(4010, A.n_rows)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    opts = mixed_opts(rtol=1e-8, inner_rtol=1e-2)
    print("[served mixed] 1.03M rows in a mix", flush=True)
    with cgx.Server(pool(1 << 31), max_slots=8, max_group=1) as srv:
        t = srv.submit(dA, dev(b), x, opts)
        rest = []
        for i, (S, dS) in enumerate(zip(small * 2, dsmall * 2)):
            bs = synth.uniform(4020 + i, S.n_rows)
            xs = torch.zeros(S.n_rows, dtype=torch.float64, device="cuda")
            o = opts if i % 2 else cgx.make_opts(rtol=1e-8, precond=1)
            rest.append((S, bs, xs, srv.submit(dS, dev(bs), xs, o)))
        st = srv.wait(t)
        for S, bs, xs, ts in rest:
            sts = srv.wait(ts)
            assert sts.status == cgx.OK
            assert true_relres(S, bs, xs.cpu().numpy()) <= 1e-8 * 1.01
    assert st.status == cgx.OK and st.outer_iters >= 2
    assert true_relres(A, b, x.cpu().numpy()) <= 1e-8 * 1.01


# ---------------------------------------------------------------- MIXED_RU --
# Served requests with reliable updates: ungrouped, each against the oracle's
# mixed_ru of it alone, with the bars of the single-system reliable-update
# tests (true residual, the kappa * rtol bound against float64, updates within
# 2, the stopping step in the band of the oracle's history); requests grouped
# in one slot share update events, against the oracle's mixed_ru_block.

def ru_opts(rtol=1e-10, jacobi=True, delta=1e-2, **kw):
    return cgx.make_opts(rtol=rtol, precond=int(jacobi), precision=cgx.PRECISION_MIXED_RU,
                         inner_rtol=delta, **kw)


def check_ru_against_oracle(A, b, x, st, rtol, jacobi, delta, gate_stop=False):
    info = st.as_dict()
    ref = oracle.mixed_ru(A, A.val.astype(np.float32), b, rtol=rtol, delta=delta, jacobi=jacobi)
    assert ref.status == oracle.OK
    assert st.status == cgx.OK and st.path == 4, info
    tr = true_relres(A, b, x)
    assert tr <= rtol, info
    assert abs(st.relres - tr) <= 1e-3 * tr + 1e-16, info
    assert abs(st.outer_iters - ref.outer_iters) <= 2, (info, ref.outer_iters)
    xs = oracle.cg(A, b, rtol=1e-13, jacobi=True, maxit=20000).x
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs), info
    if gate_stop:
        from cg_gates import assert_stop_in_band, residual_band
        h, F = residual_band(A, b, rtol, solve=lambda M, w, t: oracle.mixed_ru(
            M, M.val.astype(np.float32), w, rtol=t, delta=delta, jacobi=jacobi,
            history=True).relres_hist)
        assert_stop_in_band(h, F, st.iters, rtol, (st.iters, ref.iters))


@pytest.mark.parametrize("jacobi", [False, True], ids=["plain", "jacobi"])
def test_served_ru_matches_oracle(resident, jacobi):
    mats, dmats = resident
    opts = ru_opts(jacobi=jacobi)
    print(f"[served ru] oracle parity jacobi={jacobi}", flush=True)
    # ungrouped: each request alone in its slot, as the oracle runs it
    with cgx.Server(pool(1 << 28), max_slots=6, max_group=1) as srv:
        reqs = []
        for i in range(8):
            k = i % 4
            b = synth.uniform(5200 + i, mats[k].n_rows)
            x = torch.zeros(mats[k].n_rows, dtype=torch.float64, device="cuda")
            reqs.append((k, b, x, srv.submit(dmats[k], dev(b), x, opts)))
        for i, (k, b, x, t) in enumerate(reqs):
            st = srv.wait(t)
            check_ru_against_oracle(mats[k], b, x.cpu().numpy(), st, 1e-10, jacobi, 1e-2,
                                    gate_stop=i < 4)


def test_served_ru_alone_equals_mix(resident):
    """Ungrouped, a MIXED_RU request gets the same bits alone and among
    float64, MIXED and MIXED_RU requests."""
    mats, dmats = resident
    opts = ru_opts()
    b = dev(synth.uniform(5300, mats[2].n_rows))
    h = cgx.Handle()
    x_alone = torch.zeros_like(b)
    print("[served ru] alone", flush=True)
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        st_alone = srv.wait(srv.submit(dmats[2], b, x_alone, opts))
    x_mix = torch.zeros_like(b)
    others = []
    kinds = [cgx.make_opts(rtol=1e-10, precond=1), mixed_opts(), opts]
    print("[served ru] in a mix", flush=True)
    with cgx.Server(pool(1 << 28), max_slots=8, handle=h, max_group=1) as srv:
        for i in range(6):
            k = i % 4
            bo = dev(synth.uniform(5400 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append(srv.submit(dmats[k], bo, xo, kinds[i % 3]))
        time.sleep(0.002)
        t = srv.submit(dmats[2], b, x_mix, opts)
        for i in range(4):
            k = (i + 1) % 4
            bo = dev(synth.uniform(5500 + i, mats[k].n_rows))
            xo = torch.zeros_like(bo)
            others.append(srv.submit(dmats[k], bo, xo, kinds[(i + 1) % 3]))
        st_mix = srv.wait(t)
        for to in others:
            assert srv.wait(to).status == cgx.OK
    assert st_alone.status == st_mix.status == cgx.OK
    assert (st_alone.iters, st_alone.outer_iters) == (st_mix.iters, st_mix.outer_iters)
    assert torch.equal(x_alone, x_mix)


def test_served_ru_grouped_and_initial_guess(resident):
    """MIXED_RU requests on one matrix sharing a slot, one with an initial
    guess, one with b = 0."""
    mats, dmats = resident
    big = synth.q1cube(50, 1.0, 5600)
    dbig = cgx.DeviceCSR.from_host(big, with_f32=True)
    A, dA = mats[1], dmats[1]
    opts = ru_opts()
    bs = [synth.uniform(5700 + i, A.n_rows) for i in range(4)]
    x0 = synth.uniform(5710, A.n_rows)
    xs = [dev(x0)] + [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _ in bs[1:]]
    xz = dev(synth.uniform(5711, A.n_rows))
    print("[served ru] grouped", flush=True)
    with cgx.Server(pool(1 << 30), max_slots=1, max_group=16) as srv:
        bb = synth.uniform(5701, big.n_rows)
        xb = torch.zeros(big.n_rows, dtype=torch.float64, device="cuda")
        tb = srv.submit(dbig, dev(bb), xb, opts)  # holds the only slot
        ts = [srv.submit(dA, dev(b), x, opts) for b, x in zip(bs, xs)]
        tz = srv.submit(dA, torch.zeros_like(xz), xz, opts)
        stb = srv.wait(tb)
        sts = [srv.wait(t) for t in ts]
        stz = srv.wait(tz)
    check_ru_against_oracle(big, bb, xb.cpu().numpy(), stb, 1e-10, True, 1e-2)
    X0 = np.zeros((len(bs), A.n_rows))
    X0[0] = x0
    # the four requests started together: one update event serves all
    refs, slack = ru_block_refs(A, np.stack(bs), 1e-10, 1e-2, True, X0=X0)
    assert_updates_shared([(st.iters, st.outer_iters) for st in sts])
    for j, (b, x, st) in enumerate(zip(bs, xs, sts)):
        assert st.slot_requests == 5
        info = st.as_dict()
        assert st.status == cgx.OK, info
        assert true_relres(A, b, x.cpu().numpy()) <= 1e-10, info
        assert refs[j].status == oracle.OK
        assert abs(st.outer_iters - refs[j].outer_iters) <= slack, (info, refs[j].outer_iters)
    assert stz.status == cgx.OK and stz.outer_iters == 0 and not xz.any()


def test_served_ru_caps_and_errors(resident):
    mats, dmats = resident
    A, dA = mats[0], dmats[0]
    b = synth.uniform(5800, A.n_rows)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    print("[served ru] caps", flush=True)
    with cgx.Server(pool(1 << 26), max_slots=2) as srv:
        st = srv.wait(srv.submit(dA, dev(b), x, ru_opts(rtol=1e-15, jacobi=False, maxit=7)))
        assert st.status == cgx.NOT_CONVERGED and st.iters == 7, st.as_dict()
        tr = true_relres(A, b, x.cpu().numpy())
        assert abs(st.relres - tr) <= 1e-6 * tr and tr < 0.9
        x.zero_()
        st = srv.wait(srv.submit(dA, dev(b), x, ru_opts(rtol=1e-15, jacobi=False, max_outer=2)))
        assert st.status == cgx.NOT_CONVERGED and st.outer_iters == 2, st.as_dict()
        neg = synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, -A.val)
        dneg = cgx.DeviceCSR.from_host(neg, with_f32=True)
        st = srv.wait(srv.submit(dneg, dev(b), torch.zeros_like(x), ru_opts()))
        assert st.status == cgx.BREAKDOWN, st.as_dict()
        with pytest.raises(cgx.CgxError):
            srv.submit(cgx.DeviceCSR.from_host(A), dev(b), torch.zeros_like(x), ru_opts())
