"""GPU parity of the float32-refined batched solve (float64 outer residual
and update, binary32 inner batched CG, every (system, right-hand side) at
once) against the oracle's mixed-precision refinement run on each (system,
right-hand side) separately.

Bars, as for the single-system refinement: the float64 true residual (the
oracle's SpMV on the GPU result) <= rtol; the solution within 1e-6 of the
float64 oracle CG (cond(A) up to about 1e4 times rtol 1e-10); refinement
steps within one of the oracle's (the binary32 inner sums are taken in
another order, so an inner solve may stop an iteration earlier or later);
and a system's result bit-identical alone and inside the batch."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu

MATS = [lambda: synth.fd7_var(6, 1.0, 11), lambda: synth.q1cube(9, 1.0, 12),
        lambda: synth.fd7_var(13, 1.0, 13), lambda: synth.q1cube(14, 1.0, 14),
        lambda: synth.fd7(10)]
NRHS = [1, 3, 16, 2, 4]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_items(mats, nrhs, seed=500, special=True):
    items, hostB = [], []
    for s, (A, k) in enumerate(zip(mats, nrhs)):
        B = np.stack([synth.uniform(seed + 17 * s + j, A.n_rows) for j in range(k)])
        if special and s == len(mats) - 1:
            B[1] = 0.0  # a zero right-hand side: x = 0 after no step
        hostB.append(B)
        dA = cgx.DeviceCSR.from_host(A, with_f32=True)
        items.append((dA, dev(B), torch.zeros(k, A.n_rows, dtype=torch.float64, device="cuda")))
    return items, hostB


def true_relres(A, b, x):
    return float(np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b))


@pytest.mark.parametrize("jacobi", [False, True], ids=["plain", "jacobi"])
def test_refined_batch_vs_oracle(jacobi):
    mats = [f() for f in MATS]
    items, hostB = make_items(mats, NRHS)
    print(f"[batched mixed] jacobi={jacobi}", flush=True)
    opts = cgx.make_opts(rtol=1e-10, precond=int(jacobi), precision=cgx.PRECISION_MIXED,
                         inner_rtol=1e-3)
    st = cgx.cg_solve_batched(items, opts)
    for s, (A, (dA, dB, dX)) in enumerate(zip(mats, items)):
        X = dX.cpu().numpy()
        val32 = A.val.astype(np.float32)
        for j in range(NRHS[s]):
            b = hostB[s][j]
            info = (s, j, st[s][j].as_dict())
            assert st[s][j].status == cgx.OK, info
            if not b.any():
                assert not X[j].any() and st[s][j].outer_iters == 0, info
                continue
            ref = oracle.mixed_ir(A, val32, b, rtol=1e-10, tau=1e-3, jacobi=jacobi)
            xs = oracle.cg(A, b, rtol=1e-13, jacobi=True).x
            assert ref.status == oracle.OK
            assert abs(st[s][j].outer_iters - ref.outer_iters) <= 1, (info, ref.outer_iters)
            assert true_relres(A, b, X[j]) <= 1e-10 * 1.01, info
            assert np.linalg.norm(X[j] - xs) <= 1e-6 * np.linalg.norm(xs), info
            assert st[s][j].relres <= 1e-10


def test_refined_batch_alone_equals_in_mix():
    mats = [f() for f in MATS]
    items, _ = make_items(mats, NRHS, seed=700, special=False)
    opts = cgx.make_opts(rtol=1e-10, precond=1, precision=cgx.PRECISION_MIXED)
    print("[batched mixed] alone vs in the batch", flush=True)
    st_mix = cgx.cg_solve_batched(items, opts)
    for s in (0, 2, 3):
        dA, dB, dX = items[s]
        X_mix = dX.clone()
        X1 = torch.zeros_like(dX)
        st1 = cgx.cg_solve_batched([(dA, dB, X1)], opts)
        assert torch.equal(X1, X_mix), s
        assert [v.iters for v in st1[0]] == [v.iters for v in st_mix[s]]


def test_refined_batch_caps_and_errors():
    A = synth.q1cube(9, 1.0, 15)
    b = synth.uniform(16, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    X = torch.zeros(1, A.n_rows, dtype=torch.float64, device="cuda")
    print("[batched mixed] outer cap", flush=True)
    st = cgx.cg_solve_batched([(dA, dev(b[None]), X)],
                              cgx.make_opts(rtol=1e-14, precision=cgx.PRECISION_MIXED,
                                            inner_rtol=1e-2, max_outer=2))
    assert st[0][0].status == cgx.NOT_CONVERGED and st[0][0].outer_iters == 2
    ref = oracle.mixed_ir(A, A.val.astype(np.float32), b, rtol=1e-14, tau=1e-2, max_outer=2)
    assert ref.outer_iters == 2
    # two steps of a 1e-2 inner solve: both residuals near 1e-4
    x = X[0].cpu().numpy()
    assert true_relres(A, b, x) <= 1e-3 and true_relres(A, b, ref.x) <= 1e-3
    assert abs(st[0][0].relres - true_relres(A, b, x)) <= 1e-6
    dA64 = cgx.DeviceCSR.from_host(A)  # no val32
    with pytest.raises(cgx.CgxError):
        cgx.cg_solve_batched([(dA64, dev(b[None]), X)],
                             cgx.make_opts(precision=cgx.PRECISION_MIXED),
                             workspace=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))


def test_refined_64_systems_16_rhs_full_size():
    """The batched configuration float32-refined (binary32 inner Jacobi-CG to
    1e-2): every (system, right-hand side) converges to 1e-8 in float64, gated
    on a sample through the oracle's SpMV of the GPU solution."""
    mats = synth.batch_systems(64)
    items = []
    for s, A in enumerate(mats):
        B = torch.empty(16, A.n_rows, dtype=torch.float64)
        for j in range(16):
            B[j] = torch.from_numpy(synth.uniform(1000 + s * 16 + j, A.n_rows))
        items.append((cgx.DeviceCSR.from_host(A, with_f32=True), B.cuda(),
                      torch.zeros(16, A.n_rows, dtype=torch.float64, device="cuda")))
    print("[batched mixed] 64 x 16 full size", flush=True)
    st = cgx.cg_solve_batched(items, cgx.make_opts(rtol=1e-8, precond=1,
                                                   precision=cgx.PRECISION_MIXED,
                                                   inner_rtol=1e-2))
    assert all(v.status == cgx.OK for row in st for v in row)
    assert all(v.relres <= 1e-8 for row in st for v in row)
    rng = np.random.default_rng(1)
    for s in rng.choice(64, 8, replace=False):
        for j in rng.choice(16, 2, replace=False):
            b = items[s][1][j].cpu().numpy()
            x = items[s][2][j].cpu().numpy()
            assert true_relres(mats[s], b, x) <= 1e-8 * 1.01
