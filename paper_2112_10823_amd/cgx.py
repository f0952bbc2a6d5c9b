"""Python binding of libcgx (argument marshalling only).

Each function here forwards to the C entry point of the same name with the
`cgx_` prefix (`csr_spmv` -> `cgx_csr_spmv`, ...).  Device memory and streams
come from PyTorch (ROCm build): tensors must live on the handle's GPU; the
handle follows `torch.cuda.current_stream()` at creation.  All arithmetic runs
in the library's HIP kernels; if libcgx.so cannot be loaded every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgx.so")

OK, PENDING, EINVAL, ENOMEM, EHIP, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 1, -1, -2, -3, -4, -5, -6
PRECOND_NONE, PRECOND_JACOBI = 0, 1
PRECISION_FP64, PRECISION_MIXED, PRECISION_MIXED_RU = 0, 1, 2
STATUS_NAMES = {OK: "OK", PENDING: "PENDING", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP",
                NOT_CONVERGED: "NOT_CONVERGED", BREAKDOWN: "BREAKDOWN", NONFINITE: "NONFINITE"}


class CgxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("val32", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("true_residual", ctypes.c_int32),
                ("profile", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("path", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("phase_ms", ctypes.c_double * 3),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("kappa_est", ctypes.c_double), ("ritz_min", ctypes.c_double),
                ("ritz_max", ctypes.c_double), ("slot_requests", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        return d


class _Sell(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("n_slices", ctypes.c_int64), ("stored", ctypes.c_int64),
                ("slice_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("val32", ctypes.c_void_p)]


class _Schwarz(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_sub", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("local_rows", ctypes.c_int64), ("local_nnz", ctypes.c_int64),
                ("nnz_off", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _System(ctypes.Structure):
    _fields_ = [("A", _Csr), ("nrhs", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("B", ctypes.c_void_p), ("X", ctypes.c_void_p)]


EXPORTS = [
    "cgx_create", "cgx_destroy", "cgx_set_stream", "cgx_last_error", "cgx_version",
    "cgx_csr_validate", "cgx_csr_spmv", "cgx_csr_spmv_f32", "cgx_add", "cgx_axpy", "cgx_xmul",
    "cgx_dot", "cgx_demote", "cgx_cg_workspace_bytes", "cgx_cg_solve",
    "cgx_sell_bytes", "cgx_sell_build", "cgx_sell_spmv", "cgx_sell_spmv_f32", "cgx_cg_solve_sell",
    "cgx_batch_workspace_bytes", "cgx_cg_solve_batched", "cgx_batch_schedule",
    "cgx_serve_start", "cgx_serve_stop", "cgx_serve_request_bytes", "cgx_submit", "cgx_poll",
    "cgx_wait", "cgx_batch_mixed_workspace_bytes", "cgx_schwarz_bytes", "cgx_schwarz_build", "cgx_schwarz_workspace_bytes",
    "cgx_schwarz_solve", "cgx_dot_sync", "cgx_debug_fail_tuning",
    "cgx_cg_solve_noalloc",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcgx.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcgx.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "cgx_create": ([P(vp), ctypes.c_int, vp], ctypes.c_int),
        "cgx_destroy": ([vp], ctypes.c_int),
        "cgx_set_stream": ([vp, vp], ctypes.c_int),
        "cgx_last_error": ([], ctypes.c_char_p),
        "cgx_version": ([], ctypes.c_int),
        "cgx_csr_validate": ([vp, P(_Csr), P(i64)], ctypes.c_int),
        "cgx_csr_spmv": ([vp, P(_Csr), vp, vp], ctypes.c_int),
        "cgx_csr_spmv_f32": ([vp, P(_Csr), vp, vp], ctypes.c_int),
        "cgx_add": ([vp, i64, vp, vp, vp], ctypes.c_int),
        "cgx_axpy": ([vp, i64, dbl, vp, vp], ctypes.c_int),
        "cgx_xmul": ([vp, i64, vp, vp, vp], ctypes.c_int),
        "cgx_dot": ([vp, i64, vp, vp, vp], ctypes.c_int),
        "cgx_dot_sync": ([vp, i64, vp, vp, P(dbl)], ctypes.c_int),
        "cgx_cg_solve_noalloc": ([vp, P(_Csr), vp, vp, P(Opts), P(Stats)], ctypes.c_int),
        "cgx_debug_fail_tuning": ([vp, i32], ctypes.c_int),
        "cgx_demote": ([vp, i64, vp, vp], ctypes.c_int),
        "cgx_cg_workspace_bytes": ([i64, i64, P(Opts)], ctypes.c_size_t),
        "cgx_cg_solve": ([vp, P(_Csr), vp, vp, vp, ctypes.c_size_t, P(Opts), P(Stats)],
                         ctypes.c_int),
        "cgx_sell_bytes": ([vp, P(_Csr), P(ctypes.c_size_t)], ctypes.c_int),
        "cgx_sell_build": ([vp, P(_Csr), vp, ctypes.c_size_t, P(_Sell)], ctypes.c_int),
        "cgx_sell_spmv": ([vp, P(_Sell), vp, vp], ctypes.c_int),
        "cgx_sell_spmv_f32": ([vp, P(_Sell), vp, vp], ctypes.c_int),
        "cgx_cg_solve_sell": ([vp, P(_Csr), P(_Sell), vp, vp, vp, ctypes.c_size_t, P(Opts),
                               P(Stats)], ctypes.c_int),
        "cgx_batch_workspace_bytes": ([i32, P(_System)], ctypes.c_size_t),
        "cgx_batch_mixed_workspace_bytes": ([i32, P(_System)], ctypes.c_size_t),
        "cgx_cg_solve_batched": ([vp, i32, P(_System), vp, ctypes.c_size_t, P(Opts), P(Stats)],
                                 ctypes.c_int),
        "cgx_batch_schedule": ([vp, i32, P(_System), vp, ctypes.c_size_t, P(i32)], ctypes.c_int),
        "cgx_serve_start": ([vp, vp, ctypes.c_size_t, i32, i32], ctypes.c_int),
        "cgx_serve_stop": ([vp], ctypes.c_int),
        "cgx_serve_request_bytes": ([i64], ctypes.c_size_t),
        "cgx_submit": ([vp, P(_Csr), vp, vp, P(Opts), P(ctypes.c_uint64)], ctypes.c_int),
        "cgx_poll": ([vp, ctypes.c_uint64, P(Stats)], ctypes.c_int),
        "cgx_wait": ([vp, ctypes.c_uint64, P(Stats)], ctypes.c_int),
        "cgx_schwarz_bytes": ([vp, P(_Csr), i32, i32, P(ctypes.c_size_t)], ctypes.c_int),
        "cgx_schwarz_build": ([vp, P(_Csr), i32, i32, vp, ctypes.c_size_t, P(_Schwarz)],
                              ctypes.c_int),
        "cgx_schwarz_workspace_bytes": ([P(_Schwarz)], ctypes.c_size_t),
        "cgx_schwarz_solve": ([vp, P(_Csr), P(_Schwarz), vp, vp, vp, ctypes.c_size_t, P(Opts),
                               P(Stats)], ctypes.c_int),
    }
    for name, (argt, rest) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = argt
        fn.restype = rest
    _lib = lib
    return lib


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise CgxError(rc, _lib.cgx_last_error().decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


_I32_MAX = 2 ** 31 - 1


def _host_i32(a, name):
    """A host index array as contiguous int32, refused if an entry would not
    fit (a cast would wrap it)."""
    a = np.asarray(a)
    if not np.issubdtype(a.dtype, np.integer):
        raise TypeError(f"{name} must hold integers, got {a.dtype}")
    if a.dtype != np.int32 and a.size and (int(a.min()) < -_I32_MAX - 1 or int(a.max()) > _I32_MAX):
        raise ValueError(f"{name} has entries beyond the 32-bit range")
    if a.size > _I32_MAX:
        raise ValueError(f"{name} has more than 2^31 - 1 entries")
    return np.ascontiguousarray(a, np.int32)


def _buffer(t, name):
    """A caller-supplied workspace or pool: contiguous GPU memory of any
    dtype, passed on with its size in bytes (a host tensor would hand a host
    address to the kernels, so it is refused here)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.numel() * t.element_size()


class Handle:
    """A libcgx handle bound to a device and a stream."""

    def __init__(self, device: int | None = None, stream=None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.cgx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)))
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.cgx_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict = {}


def default_handle() -> Handle:
    dev = torch.cuda.current_device()
    s = torch.cuda.current_stream(dev)
    key = (dev, s.cuda_stream)
    h = _handles.get(key)
    if h is None:
        h = Handle(dev, s)
        _handles[key] = h
    return h


@dataclass
class DeviceCSR:
    """CSR matrix resident on the GPU (torch-owned arrays) plus its C descriptor."""

    n_rows: int
    n_cols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor | None
    val32: torch.Tensor | None = None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def desc(self) -> _Csr:
        return _Csr(self.n_rows, self.n_cols, self.nnz, self.row_ptr.data_ptr(),
                    self.col_idx.data_ptr(),
                    self.val.data_ptr() if self.val is not None else None,
                    self.val32.data_ptr() if self.val32 is not None else None)

    @classmethod
    def from_host(cls, A, device="cuda", with_f32=False, validate=True, handle=None):
        """Upload a host CSR (row_ptr, col_idx, val numpy arrays) and validate it on the GPU.
        Sizes and indices must fit the library's 32-bit CSR; they are checked
        here before anything is copied, so that no index wraps in the cast."""
        n_rows, n_cols = int(A.n_rows), int(A.n_cols)
        if not (0 <= n_rows <= _I32_MAX and 0 <= n_cols <= _I32_MAX):
            raise ValueError("n_rows and n_cols must lie in [0, 2^31 - 1]")
        rp_h = _host_i32(A.row_ptr, "row_ptr")
        ci_h = _host_i32(A.col_idx, "col_idx")
        v_h = np.ascontiguousarray(A.val, np.float64)
        if rp_h.size != n_rows + 1:
            raise ValueError("row_ptr must hold n_rows + 1 entries")
        if ci_h.size != v_h.size:
            raise ValueError("col_idx and val must have the same length")
        rp = torch.from_numpy(rp_h).to(device)
        ci = torch.from_numpy(ci_h).to(device)
        v = torch.from_numpy(v_h).to(device)
        d = cls(int(A.n_rows), int(A.n_cols), rp, ci, v)
        if with_f32:
            d.val32 = torch.empty(d.nnz, dtype=torch.float32, device=device)
            demote(v, d.val32, handle=handle)
        if validate:
            csr_validate(d, handle=handle)
        return d


class SellMatrix:
    """Sliced-ELL copy of a DeviceCSR (cgx_sell_build) in a torch-owned
    buffer; keeps the CSR alive beside it (the CG setup passes read it)."""

    def __init__(self, A: DeviceCSR, handle=None):
        d = A.desc()
        nbytes = ctypes.c_size_t()
        _check(load_library().cgx_sell_bytes(_h(handle), ctypes.byref(d), ctypes.byref(nbytes)))
        self.csr = A
        self.buffer = torch.empty(max(nbytes.value, 256), dtype=torch.uint8,
                                  device=A.row_ptr.device)
        self._desc = _Sell()
        _check(load_library().cgx_sell_build(_h(handle), ctypes.byref(d), _ptr(self.buffer),
                                             self.buffer.numel(), ctypes.byref(self._desc)))

    @property
    def n_rows(self) -> int:
        return self._desc.n_rows

    @property
    def n_slices(self) -> int:
        return self._desc.n_slices

    @property
    def stored(self) -> int:
        return self._desc.stored

    def desc(self) -> _Sell:
        return self._desc

    def arrays(self):
        """(slice_ptr int64, col int32, val float64) views of the buffer."""
        d = self._desc
        base = self.buffer.data_ptr()

        def view(ptr, count, dtype, size):
            off = ptr - base
            return self.buffer[off:off + count * size].view(dtype)

        return (view(d.slice_ptr, d.n_slices + 1, torch.int64, 8),
                view(d.col, d.stored, torch.int32, 4), view(d.val, d.stored, torch.float64, 8))


class SchwarzDecomposition:
    """Subdomain matrices of an additive Schwarz preconditioner for a
    DeviceCSR (cgx_schwarz_build: n_sub contiguous row blocks, each extended
    by `overlap` rows on both sides) in a torch-owned buffer."""

    def __init__(self, A: DeviceCSR, n_sub: int, overlap: int = 0, handle=None):
        d = A.desc()
        nbytes = ctypes.c_size_t()
        _check(load_library().cgx_schwarz_bytes(_h(handle), ctypes.byref(d), int(n_sub),
                                                int(overlap), ctypes.byref(nbytes)))
        self.csr = A
        self.buffer = torch.empty(max(nbytes.value, 256), dtype=torch.uint8,
                                  device=A.row_ptr.device)
        self._desc = _Schwarz()
        _check(load_library().cgx_schwarz_build(_h(handle), ctypes.byref(d), int(n_sub),
                                                int(overlap), _ptr(self.buffer),
                                                self.buffer.numel(), ctypes.byref(self._desc)))

    @property
    def n_sub(self) -> int:
        return self._desc.n_sub

    @property
    def overlap(self) -> int:
        return self._desc.overlap

    @property
    def local_rows(self) -> int:
        return self._desc.local_rows

    @property
    def local_nnz(self) -> int:
        return self._desc.local_nnz

    def desc(self) -> _Schwarz:
        return self._desc

    def workspace_bytes(self) -> int:
        return int(load_library().cgx_schwarz_workspace_bytes(ctypes.byref(self._desc)))

    def arrays(self):
        """(nnz_off int64, row_ptr int32, col int32, val float64) views of the buffer."""
        d = self._desc
        base = self.buffer.data_ptr()

        def view(ptr, count, dtype, size):
            off = ptr - base
            return self.buffer[off:off + count * size].view(dtype)

        return (view(d.nnz_off, d.n_sub + 1, torch.int64, 8),
                view(d.row_ptr, d.local_rows + d.n_sub, torch.int32, 4),
                view(d.col, d.local_nnz, torch.int32, 4),
                view(d.val, d.local_nnz, torch.float64, 8))


def _h(handle):
    return (handle or default_handle()).ptr


# ------------------------------------------------------------------ calls --

def csr_validate(A: DeviceCSR, handle=None) -> int:
    bad = ctypes.c_int64(-1)
    d = A.desc()
    _check(load_library().cgx_csr_validate(_h(handle), ctypes.byref(d), ctypes.byref(bad)))
    return bad.value


def csr_spmv(A: DeviceCSR, x: torch.Tensor, y: torch.Tensor | None = None, handle=None):
    _dev_tensor(x, torch.float64, "x")
    if y is None:
        y = torch.empty(A.n_rows, dtype=torch.float64, device=x.device)
    _dev_tensor(y, torch.float64, "y")
    if x.numel() != A.n_cols or y.numel() != A.n_rows:
        raise ValueError("x / y length does not match A")
    d = A.desc()
    _check(load_library().cgx_csr_spmv(_h(handle), ctypes.byref(d), _ptr(x), _ptr(y)))
    return y


def csr_spmv_f32(A: DeviceCSR, x: torch.Tensor, y: torch.Tensor | None = None, handle=None):
    _dev_tensor(x, torch.float32, "x")
    if y is None:
        y = torch.empty(A.n_rows, dtype=torch.float32, device=x.device)
    _dev_tensor(y, torch.float32, "y")
    if x.numel() != A.n_cols or y.numel() != A.n_rows:
        raise ValueError("x / y length does not match A")
    d = A.desc()
    _check(load_library().cgx_csr_spmv_f32(_h(handle), ctypes.byref(d), _ptr(x), _ptr(y)))
    return y


def sell_spmv(S: SellMatrix, x: torch.Tensor, y: torch.Tensor | None = None, handle=None):
    _dev_tensor(x, torch.float64, "x")
    d = S.desc()
    if y is None:
        y = torch.empty(d.n_rows, dtype=torch.float64, device=x.device)
    _dev_tensor(y, torch.float64, "y")
    if x.numel() != d.n_cols or y.numel() != d.n_rows:
        raise ValueError("x / y length does not match S")
    _check(load_library().cgx_sell_spmv(_h(handle), ctypes.byref(d), _ptr(x), _ptr(y)))
    return y


def sell_spmv_f32(S: SellMatrix, x: torch.Tensor, y: torch.Tensor | None = None, handle=None):
    _dev_tensor(x, torch.float32, "x")
    d = S.desc()
    if y is None:
        y = torch.empty(d.n_rows, dtype=torch.float32, device=x.device)
    _dev_tensor(y, torch.float32, "y")
    if x.numel() != d.n_cols or y.numel() != d.n_rows:
        raise ValueError("x / y length does not match S")
    _check(load_library().cgx_sell_spmv_f32(_h(handle), ctypes.byref(d), _ptr(x), _ptr(y)))
    return y


def _vec_args(x, y, z=None):
    _dev_tensor(x, torch.float64, "x")
    _dev_tensor(y, torch.float64, "y")
    if x.numel() != y.numel() or (z is not None and z.numel() != x.numel()):
        raise ValueError("length mismatch")
    if z is not None:
        _dev_tensor(z, torch.float64, "z")


def add(x, y, z=None, handle=None):
    if z is None:
        z = torch.empty_like(x)
    _vec_args(x, y, z)
    _check(load_library().cgx_add(_h(handle), x.numel(), _ptr(x), _ptr(y), _ptr(z)))
    return z


def axpy(alpha: float, x, y, handle=None):
    """y <- fma(alpha, x, y) in place; returns y."""
    _vec_args(x, y)
    _check(load_library().cgx_axpy(_h(handle), x.numel(), float(alpha), _ptr(x), _ptr(y)))
    return y


def xmul(x, y, z=None, handle=None):
    if z is None:
        z = torch.empty_like(x)
    _vec_args(x, y, z)
    _check(load_library().cgx_xmul(_h(handle), x.numel(), _ptr(x), _ptr(y), _ptr(z)))
    return z


def dot(x, y, out=None, handle=None):
    """Returns a 1-element float64 GPU tensor holding x . y (asynchronous)."""
    _vec_args(x, y)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _dev_tensor(out, torch.float64, "out")
    _check(load_library().cgx_dot(_h(handle), x.numel(), _ptr(x), _ptr(y), _ptr(out)))
    return out


def dot_sync(x, y, handle=None) -> float:
    """x . y returned to the host (cgx_dot_sync: waits for the handle's stream)."""
    _vec_args(x, y)
    out = ctypes.c_double()
    _check(load_library().cgx_dot_sync(_h(handle), x.numel(), _ptr(x), _ptr(y), ctypes.byref(out)))
    return out.value


def debug_fail_tuning(count: int, handle=None):
    """Test hook: the next `count` autotuner calls on the handle fail (cgx_debug_fail_tuning)."""
    _check(load_library().cgx_debug_fail_tuning(_h(handle), int(count)))


def demote(src, dst=None, handle=None):
    _dev_tensor(src, torch.float64, "src")
    if dst is None:
        dst = torch.empty(src.numel(), dtype=torch.float32, device=src.device)
    _dev_tensor(dst, torch.float32, "dst")
    if dst.numel() != src.numel():
        raise ValueError("length mismatch")
    _check(load_library().cgx_demote(_h(handle), src.numel(), _ptr(src), _ptr(dst)))
    return dst


def make_opts(rtol=1e-8, maxit=0, precond=PRECOND_NONE, precision=PRECISION_FP64,
              check_every=0, inner_rtol=0.0, max_outer=0, true_residual=False,
              profile=False) -> Opts:
    return Opts(float(rtol), int(maxit), int(precond), int(precision), int(check_every),
                float(inner_rtol), int(max_outer), int(bool(true_residual)), int(bool(profile)))


def cg_workspace_bytes(n_rows: int, nnz: int, opts: Opts) -> int:
    return int(load_library().cgx_cg_workspace_bytes(n_rows, nnz, ctypes.byref(opts)))


def cg_workspace(A: DeviceCSR, opts: Opts, device=None) -> torch.Tensor:
    nbytes = cg_workspace_bytes(A.n_rows, A.nnz, opts)
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or A.row_ptr.device)


def cg_solve(A: DeviceCSR, b, x, opts: Opts | None = None, workspace=None, handle=None,
             raise_on_fail=False, sell: "SellMatrix | None" = None) -> Stats:
    """Solve A x = b in place on x (x holds x0 on entry).  Returns Stats.
    With `sell` (a SellMatrix of A) the iteration's SpMV runs on it."""
    opts = opts or make_opts()
    _dev_tensor(b, torch.float64, "b")
    _dev_tensor(x, torch.float64, "x")
    if b.numel() != A.n_rows or x.numel() != A.n_rows:
        raise ValueError("b / x length does not match A")
    if workspace is None:
        workspace = cg_workspace(A, opts)
    ws_bytes = _buffer(workspace, "workspace")
    st = Stats()
    d = A.desc()
    if sell is None:
        rc = load_library().cgx_cg_solve(_h(handle), ctypes.byref(d), _ptr(b), _ptr(x),
                                         _ptr(workspace), ws_bytes, ctypes.byref(opts),
                                         ctypes.byref(st))
    else:
        rc = load_library().cgx_cg_solve_sell(_h(handle), ctypes.byref(d),
                                              ctypes.byref(sell.desc()), _ptr(b), _ptr(x),
                                              _ptr(workspace), ws_bytes,
                                              ctypes.byref(opts), ctypes.byref(st))
    if rc in (EINVAL, ENOMEM, EHIP) or (raise_on_fail and rc != OK):
        _check(rc)
    return st


def cg_solve_noalloc(A: DeviceCSR, b, x, opts: Opts | None = None, handle=None) -> Stats:
    """cgx_cg_solve_noalloc: float64 CG with the library's static device
    scratch as workspace (no allocation in the call).  Returns Stats; raises
    CgxError on argument errors and on a system too large for the scratch."""
    opts = opts or make_opts()
    _dev_tensor(b, torch.float64, "b")
    _dev_tensor(x, torch.float64, "x")
    if b.numel() != A.n_rows or x.numel() != A.n_rows:
        raise ValueError("b / x length does not match A")
    st = Stats()
    d = A.desc()
    rc = load_library().cgx_cg_solve_noalloc(_h(handle), ctypes.byref(d), _ptr(b), _ptr(x),
                                             ctypes.byref(opts), ctypes.byref(st))
    if rc in (EINVAL, ENOMEM, EHIP):
        _check(rc)
    return st


def schwarz_solve(A: DeviceCSR, D: SchwarzDecomposition, b, x, opts: Opts | None = None,
                  workspace=None, handle=None, raise_on_fail=False) -> Stats:
    """Solve A x = b in place on x by flexible CG under the additive Schwarz
    preconditioner D (cgx_schwarz_solve; subdomain CG per opts.inner_rtol,
    opts.maxit, opts.precond; outer cap opts.max_outer)."""
    opts = opts or make_opts()
    _dev_tensor(b, torch.float64, "b")
    _dev_tensor(x, torch.float64, "x")
    if b.numel() != A.n_rows or x.numel() != A.n_rows:
        raise ValueError("b / x length does not match A")
    if workspace is None:
        workspace = torch.empty(max(D.workspace_bytes(), 1), dtype=torch.uint8, device=x.device)
    ws_bytes = _buffer(workspace, "workspace")
    st = Stats()
    d = A.desc()
    rc = load_library().cgx_schwarz_solve(_h(handle), ctypes.byref(d), ctypes.byref(D.desc()),
                                          _ptr(b), _ptr(x), _ptr(workspace), ws_bytes,
                                          ctypes.byref(opts), ctypes.byref(st))
    if rc in (EINVAL, ENOMEM, EHIP) or (raise_on_fail and rc != OK):
        _check(rc)
    return st


# ---------------------------------------------------------------- batched --

def _systems(items):
    """items: list of (DeviceCSR, B, X) with B, X float64 GPU tensors of shape
    (nrhs, n) (right-hand-side major, contiguous)."""
    arr = (_System * len(items))()
    for i, item in enumerate(items):
        A, B, X = item[:3]
        arr[i].schedule = int(item[3]) if len(item) > 3 else 0
        _dev_tensor(B, torch.float64, "B")
        _dev_tensor(X, torch.float64, "X")
        if B.dim() != 2 or B.shape != X.shape or B.shape[1] != A.n_rows:
            raise ValueError("B and X must be (nrhs, n_rows)")
        if not 1 <= B.shape[0] <= 16 or A.n_rows < 1 or A.n_rows != A.n_cols:
            raise ValueError("each system needs a square matrix with n_rows >= 1 and 1 to 16 "
                             "right-hand sides")
        arr[i].A = A.desc()
        arr[i].nrhs = B.shape[0]
        arr[i].B = B.data_ptr()
        arr[i].X = X.data_ptr()
    return arr


def batch_workspace_bytes(items, opts: Opts | None = None) -> int:
    """Workspace bytes of cg_solve_batched (binary32 with float64
    refinement or reliable updates when opts.precision is PRECISION_MIXED or
    PRECISION_MIXED_RU)."""
    arr = _systems(items)
    if opts is not None and opts.precision in (PRECISION_MIXED, PRECISION_MIXED_RU):
        return int(load_library().cgx_batch_mixed_workspace_bytes(len(items), arr))
    return int(load_library().cgx_batch_workspace_bytes(len(items), arr))


def batch_workspace(items, device="cuda", opts: Opts | None = None) -> torch.Tensor:
    return torch.empty(max(batch_workspace_bytes(items, opts), 1), dtype=torch.uint8,
                       device=device)


def cg_solve_batched(items, opts: Opts | None = None, workspace=None, handle=None):
    """Solve every (system, right-hand side) of the batch in place on X.
    items: (A, B, X) or (A, B, X, schedule) tuples, B and X (nrhs, n_rows).
    Returns a list with one Stats per system, each a list over its right-hand sides."""
    opts = opts or make_opts()
    arr = _systems(items)
    if workspace is None:
        workspace = batch_workspace(items, opts=opts)
    ws_bytes = _buffer(workspace, "workspace")
    nstat = sum(int(item[1].shape[0]) for item in items)
    st = (Stats * nstat)()
    rc = load_library().cgx_cg_solve_batched(_h(handle), len(items), arr, _ptr(workspace),
                                             ws_bytes, ctypes.byref(opts), st)
    if rc in (EINVAL, ENOMEM, EHIP):
        _check(rc)
    out, k = [], 0
    for item in items:
        nr = int(item[1].shape[0])
        out.append([st[k + j] for j in range(nr)])
        k += nr
    return out


def batch_schedule(items, workspace=None, handle=None):
    """Schedule of each system: its own if fixed, else the autotuner's pick
    (M > 0 slices per right-hand side, M < 0 wave tiles of -M rows)."""
    arr = _systems(items)
    if workspace is None:
        workspace = batch_workspace(items)
    ws_bytes = _buffer(workspace, "workspace")
    m = (ctypes.c_int32 * len(items))()
    _check(load_library().cgx_batch_schedule(_h(handle), len(items), arr, _ptr(workspace),
                                             ws_bytes, m))
    return list(m)


# ---------------------------------------------------------------- serving --

class Server:
    """Continuous-batching solve server on a handle (see cgx_serve_start).

    pool: uint8 GPU tensor the server carves its tables and request vectors
    from; max_group: requests on one matrix that may share a slot as the
    right-hand sides of one solve (1: no grouping).  Matrices, right-hand
    sides and solution vectors stay owned by the caller and must outlive
    their requests."""

    def __init__(self, pool: torch.Tensor, max_slots: int = 64, handle: Handle | None = None,
                 max_group: int = 16):
        pool_bytes = _buffer(pool, "pool")
        self.handle = handle or Handle()
        self.pool = pool
        self._keep = {}
        self.running = False
        _check(load_library().cgx_serve_start(self.handle.ptr, _ptr(pool), pool_bytes,
                                              int(max_slots), int(max_group)))
        self.running = True

    @staticmethod
    def request_bytes(n_rows: int) -> int:
        return int(load_library().cgx_serve_request_bytes(int(n_rows)))

    def submit(self, A: DeviceCSR, b: torch.Tensor, x: torch.Tensor, opts: Opts | None = None) -> int:
        _dev_tensor(b, torch.float64, "b")
        _dev_tensor(x, torch.float64, "x")
        if b.numel() != A.n_rows or x.numel() != A.n_rows:
            raise ValueError("b / x length does not match A")
        opts = opts or make_opts()
        d = A.desc()
        t = ctypes.c_uint64()
        _check(load_library().cgx_submit(self.handle.ptr, ctypes.byref(d), _ptr(b), _ptr(x),
                                         ctypes.byref(opts), ctypes.byref(t)))
        self._keep[t.value] = (A, b, x)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the final Stats."""
        st = Stats()
        rc = load_library().cgx_poll(self.handle.ptr, ticket, ctypes.byref(st))
        if rc == PENDING:
            return None
        if rc in (EINVAL, ENOMEM, EHIP):
            _check(rc)
        self._keep.pop(ticket, None)
        return st

    def wait(self, ticket: int) -> Stats:
        st = Stats()
        rc = load_library().cgx_wait(self.handle.ptr, ticket, ctypes.byref(st))
        if rc in (EINVAL, ENOMEM, EHIP):
            _check(rc)
        self._keep.pop(ticket, None)
        return st

    def stop(self):
        if self.running:
            self.running = False
            _check(load_library().cgx_serve_stop(self.handle.ptr))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
