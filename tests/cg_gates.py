"""Gates on where a GPU CG run stopped, derived from the oracle alone.

Two correct finite-precision CG runs on the same system stop at the first
step whose own recursive residual ||r_k|| / ||b|| is at or below rtol.  Their
residual histories are not equal: each rounding order perturbs the recurrences
(CG's residual norm is not even monotone), so the crossing can move by a few
steps.  How far depends on the system, not on any kernel: the oracle measures
it by running the same CG on the reversed-order system P A P^T, P b (exact in
exact arithmetic, every sum in another order).  If the oracle's two histories
differ at the same step by at most a factor (1 + delta), a third correct run
(the GPU's) differs from the oracle's by at most F = (1 + delta)^2 (each
deviates from the exact history by up to (1 + delta)).  At the GPU's stopping
step k the oracle's residual must then satisfy h[k] <= F rtol, and at the
step before h[k - 1] > rtol / F.
"""
import numpy as np

import oracle
from synth import CSR


def reversed_system(A, b):
    """P A P^T and P b for the reversal permutation i -> n - 1 - i (rows and
    the entries inside each row in reverse order)."""
    n = A.n_rows
    rp = np.asarray(A.row_ptr, np.int64)
    lens = np.diff(rp)[::-1]
    new_rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = (n - 1 - np.asarray(A.col_idx, np.int64))[::-1].astype(np.int32)
    val = np.asarray(A.val)[::-1].copy()
    return CSR(n, n, new_rp, ci, val), np.asarray(b)[::-1].copy()


def residual_band(A, b, rtol, jacobi=False, solve=None):
    """The oracle's residual history h (run past rtol, to rtol / 100) and the
    band factor F = (1 + delta)^2 from its reversed-order run.  solve(A, b,
    rtol) -> history selects the oracle method (default: CG)."""
    if solve is None:
        def solve(M, v, t):
            return oracle.cg(M, v, rtol=t, jacobi=jacobi, history=True).relres_hist
    h = solve(A, b, rtol / 100)
    Ar, br = reversed_system(A, b)
    hr = solve(Ar, br, rtol / 100)
    m = min(len(h), len(hr))
    ratio = hr[:m] / h[:m]
    delta = float(np.max(np.maximum(ratio, 1.0 / ratio)) - 1.0)
    return h, (1.0 + delta) ** 2


def assert_stop_in_band(h, F, k, rtol, what=""):
    assert 1 <= k < len(h), (what, k, len(h))
    assert h[k] <= F * rtol, (what, k, h[k] / rtol, F)
    assert h[k - 1] > rtol / F, (what, k, h[k - 1] / rtol, F)


def ru_block_refs(A, B, rtol, delta, jacobi, X0=None):
    """The oracle's reliable-update run of the right-hand sides B (k x n) of
    A with updates shared by all of them, and the slack it implies for the
    update count of another correct run.

    An update event of the block is the union of every right-hand side's
    trigger, the final ones (each right-hand side's own convergence test)
    included, so a stopping step moved by one iteration merges or splits an
    event of every right-hand side still running: the count is far more
    sensitive to rounding than a single right-hand side's.  The oracle
    measures that sensitivity as D, the largest per-right-hand-side
    difference of the count between its run and the same run on the
    reversed-order system; a third run is allowed max(2, 2 D)."""
    v32 = np.asarray(A.val).astype(np.float32)
    refs = oracle.mixed_ru_block(A, v32, B, X0=X0, rtol=rtol, delta=delta, jacobi=jacobi)
    Ar, _ = reversed_system(A, B[0])
    Br = np.ascontiguousarray(np.asarray(B)[:, ::-1])
    X0r = None if X0 is None else np.ascontiguousarray(np.asarray(X0)[:, ::-1])
    rev = oracle.mixed_ru_block(Ar, np.asarray(Ar.val).astype(np.float32), Br, X0=X0r,
                                rtol=rtol, delta=delta, jacobi=jacobi)
    D = max(abs(a.outer_iters - b.outer_iters) for a, b in zip(refs, rev))
    return refs, max(2, 2 * D)


def assert_updates_shared(runs, what=""):
    """runs: (iters, updates) of the right-hand sides of one matrix that
    started together and converged.  With shared updates each stops at an
    event and has taken every event up to it, so the update count is a
    strictly increasing function of the stopping step."""
    runs = sorted(runs)
    for (i0, u0), (i1, u1) in zip(runs, runs[1:]):
        assert (u1 == u0) if i1 == i0 else (u1 > u0), (what, runs)
