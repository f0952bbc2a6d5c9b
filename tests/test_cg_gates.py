"""CPU checks of the stopping-step gate used by the GPU tests (cg_gates)."""
import numpy as np
import pytest

import oracle
import synth
from cg_gates import (assert_stop_in_band, assert_updates_shared, residual_band,
                      reversed_system, ru_block_refs)


def dense(A):
    D = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        D[i, A.col_idx[s:e]] = A.val[s:e]
    return D


def test_reversed_system_is_the_permuted_matrix():
    A = synth.q1cube(5, 1.0, 3)
    b = synth.uniform(4, A.n_rows)
    Ar, br = reversed_system(A, b)
    P = np.eye(A.n_rows)[::-1]
    np.testing.assert_array_equal(dense(Ar), P @ dense(A) @ P.T)
    np.testing.assert_array_equal(br, P @ b)
    # rows keep their entries, in reverse order
    r = A.n_rows - 1
    np.testing.assert_array_equal(Ar.val[Ar.row_ptr[0]:Ar.row_ptr[1]],
                                  A.val[A.row_ptr[r]:A.row_ptr[r + 1]][::-1])


def test_band_accepts_the_oracle_and_its_reversal_and_rejects_shifts():
    A = synth.q1cube(14, 1.0, 5)
    b = synth.uniform(6, A.n_rows)
    rtol = 1e-9
    h, F = residual_band(A, b, rtol)
    assert F >= 1.0
    k = oracle.cg(A, b, rtol=rtol).iters
    assert_stop_in_band(h, F, k, rtol)
    Ar, br = reversed_system(A, b)
    assert_stop_in_band(h, F, oracle.cg(Ar, br, rtol=rtol).iters, rtol)
    # a run stopping far too early or late is refused
    for bad in (k // 2, k + 40):
        try:
            assert_stop_in_band(h, F, bad, rtol)
        except AssertionError:
            continue
        raise AssertionError(f"stop at {bad} (oracle {k}) accepted")


def test_shared_update_gates_accept_the_oracle_and_reject_solo_updates():
    """The reversed-order block run is within the slack and satisfies the
    shared-update invariant; per-right-hand-side (solo) updates break it."""
    A = synth.fd7_var(10, 1.0, 7)
    B = np.stack([synth.uniform(70 + j, A.n_rows) for j in range(6)])
    refs, slack = ru_block_refs(A, B, 1e-10, 1e-2, False)
    assert 2 <= slack <= 8
    assert all(r.status == oracle.OK for r in refs)
    assert_updates_shared([(r.iters, r.outer_iters) for r in refs])
    Ar, _ = reversed_system(A, B[0])
    rev = oracle.mixed_ru_block(Ar, Ar.val.astype(np.float32), B[:, ::-1].copy(), rtol=1e-10,
                                delta=1e-2)
    assert_updates_shared([(r.iters, r.outer_iters) for r in rev])
    for a, b in zip(refs, rev):
        assert abs(a.outer_iters - b.outer_iters) <= slack
    solo = [oracle.mixed_ru(A, A.val.astype(np.float32), b, rtol=1e-10, delta=1e-2) for b in B]
    with pytest.raises(AssertionError):
        assert_updates_shared([(r.iters, r.outer_iters) for r in solo])
