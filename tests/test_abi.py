"""Host-side checks of the C ABI: the library loads, exports every function
include/cgx.h declares, and its struct layouts match the binding (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2112_10823_amd import cgx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = cgx.load_library()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), f"{name} declared in cgx.h but not exported"
    assert set(names) == set(cgx.EXPORTS)


def test_host_only_calls():
    lib = cgx.load_library()
    assert lib.cgx_version() == 100
    o = cgx.make_opts(rtol=1e-8)
    nb = cgx.cg_workspace_bytes(1000, 27000, o)
    assert nb >= 3 * 1000 * 8
    oj = cgx.make_opts(precond=cgx.PRECOND_JACOBI)
    assert cgx.cg_workspace_bytes(1000, 27000, oj) >= nb + 2 * 1000 * 8
    assert cgx.cg_workspace_bytes(-1, 0, o) == 0
    assert lib.cgx_last_error() is not None


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu\\n", sizeof(cgx_csr), offsetof(cgx_csr, row_ptr), offsetof(cgx_csr, val32), offsetof(cgx_csr, nnz));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(cgx_opts), offsetof(cgx_opts, inner_rtol), offsetof(cgx_opts, max_outer), offsetof(cgx_opts, true_residual), offsetof(cgx_opts, profile));
  printf("%zu %zu %zu %zu\\n", sizeof(cgx_stats), offsetof(cgx_stats, relres), offsetof(cgx_stats, device_ms), offsetof(cgx_stats, phase_ms));
  printf("%zu %zu %zu %zu\\n", sizeof(cgx_sell), offsetof(cgx_sell, n_slices), offsetof(cgx_sell, slice_ptr), offsetof(cgx_sell, val32));
  printf("%zu %zu %zu\\n", sizeof(cgx_system), offsetof(cgx_system, schedule), offsetof(cgx_system, X));
  printf("%zu %zu %zu %zu\\n", sizeof(cgx_schwarz), offsetof(cgx_schwarz, local_rows), offsetof(cgx_schwarz, nnz_off), offsetof(cgx_schwarz, val));
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    c = [list(map(int, l.split())) for l in out if l.strip()]
    S, O, T = cgx._Csr, cgx.Opts, cgx.Stats
    assert c[0] == [ctypes.sizeof(S), S.row_ptr.offset, S.val32.offset, S.nnz.offset]
    assert c[1] == [ctypes.sizeof(O), O.inner_rtol.offset, O.max_outer.offset, O.true_residual.offset,
                    O.profile.offset]
    assert c[2] == [ctypes.sizeof(T), T.relres.offset, T.device_ms.offset, T.phase_ms.offset]
    L, Y = cgx._Sell, cgx._System
    assert c[3] == [ctypes.sizeof(L), L.n_slices.offset, L.slice_ptr.offset, L.val32.offset]
    assert c[4] == [ctypes.sizeof(Y), Y.schedule.offset, Y.X.offset]
    W = cgx._Schwarz
    assert c[5] == [ctypes.sizeof(W), W.local_rows.offset, W.nnz_off.offset, W.val.offset]


def test_schwarz_workspace_bytes_host_only():
    """The workspace size query needs no GPU; a descriptor whose sizes do not
    add up is refused with 0."""
    W = cgx._Schwarz
    d = W(n_rows=1000, n_sub=4, overlap=50, local_rows=1000 + 2 * 50 * 3, local_nnz=0,
          nnz_off=256, row_ptr=512, col=None, val=None)
    lib = cgx.load_library()
    nb = lib.cgx_schwarz_workspace_bytes(ctypes.byref(d))
    assert nb >= (4 * 1000 + 1300) * 8
    d.local_rows = 1299
    assert lib.cgx_schwarz_workspace_bytes(ctypes.byref(d)) == 0
    d.local_rows, d.overlap = 1300 + 2 * 3 * 200, 251
    assert lib.cgx_schwarz_workspace_bytes(ctypes.byref(d)) == 0


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        cgx._dev_tensor(torch.zeros(3, dtype=torch.float64), torch.float64, "x")


def test_binding_refuses_host_workspaces(monkeypatch):
    """A host workspace or pool is refused before the library is reached: the
    vector checks are waved through here (there is no GPU), and any library
    call fails the test."""
    import torch

    def no_library(*a, **k):
        raise AssertionError("library reached with a host workspace")

    monkeypatch.setattr(cgx, "_dev_tensor", lambda t, dtype, name: t)
    monkeypatch.setattr(cgx, "load_library", no_library)

    class FakeCSR:
        n_rows = n_cols = 4
        nnz = 4

        def desc(self):
            return cgx._Csr()

    A = FakeCSR()
    v = torch.zeros(4, dtype=torch.float64)
    host_ws = torch.zeros(1024, dtype=torch.uint8)
    with pytest.raises(TypeError, match="workspace"):
        cgx.cg_solve(A, v, v.clone(), workspace=host_ws)
    with pytest.raises(TypeError, match="workspace"):
        cgx.schwarz_solve(A, None, v, v.clone(), workspace=host_ws)
    B = torch.zeros(2, 4, dtype=torch.float64)
    with pytest.raises(TypeError, match="workspace"):
        cgx.cg_solve_batched([(A, B, B.clone())], workspace=host_ws)
    with pytest.raises(TypeError, match="workspace"):
        cgx.batch_schedule([(A, B, B.clone())], workspace=host_ws)
    with pytest.raises(TypeError, match="pool"):
        cgx.Server(host_ws, handle=object())


def test_binding_checks_batch_descriptors(monkeypatch):
    """The workspace-size queries take descriptors as given; the binding
    refuses a system with no or more than 16 right-hand sides, or a
    non-square or empty matrix, before it sizes or solves the batch."""
    import torch

    def no_library(*a, **k):
        raise AssertionError("library reached with a bad batch")

    monkeypatch.setattr(cgx, "_dev_tensor", lambda t, dtype, name: t)
    monkeypatch.setattr(cgx, "load_library", no_library)

    class FakeCSR:
        def __init__(self, n_rows, n_cols):
            self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, max(n_rows, 0)

        def desc(self):
            return cgx._Csr()

    for A, k in ((FakeCSR(4, 4), 0), (FakeCSR(4, 4), 17), (FakeCSR(4, 5), 1), (FakeCSR(0, 0), 1)):
        B = torch.zeros(k, A.n_rows, dtype=torch.float64)
        with pytest.raises(ValueError):
            cgx.batch_workspace_bytes([(A, B, B.clone())])
        with pytest.raises(ValueError):
            cgx.cg_solve_batched([(A, B, B.clone())])


def test_from_host_checks_sizes_before_copying():
    """Index arrays that would wrap in the cast to 32 bits, a row-pointer
    array of the wrong length or mismatched entry arrays are refused before
    anything is copied; a valid int64 CSR converts exactly."""
    import numpy as np
    import synth

    A = synth.fd7(3)
    bad_rp = A.row_ptr.astype(np.int64)
    bad_rp[-1] = 2 ** 31
    cases = [
        synth.CSR(A.n_rows, A.n_cols, bad_rp, A.col_idx, A.val),
        synth.CSR(A.n_rows, A.n_cols, A.row_ptr[:-1], A.col_idx, A.val),
        synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val[:-1]),
        synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx.astype(np.int64) - 2 ** 32, A.val),
        synth.CSR(2 ** 31, A.n_cols, A.row_ptr, A.col_idx, A.val),
    ]
    for bad in cases:
        with pytest.raises(ValueError):
            cgx.DeviceCSR.from_host(bad, device="cpu", validate=False)
    with pytest.raises(TypeError):
        cgx.DeviceCSR.from_host(synth.CSR(A.n_rows, A.n_cols, A.row_ptr.astype(float), A.col_idx,
                                          A.val), device="cpu", validate=False)
    ok = synth.CSR(A.n_rows, A.n_cols, A.row_ptr.astype(np.int64), A.col_idx.astype(np.int64), A.val)
    d = cgx.DeviceCSR.from_host(ok, device="cpu", validate=False)
    assert np.array_equal(d.row_ptr.numpy(), A.row_ptr) and np.array_equal(d.col_idx.numpy(), A.col_idx)
