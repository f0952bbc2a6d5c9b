"""MI355X-native sparse conjugate-gradient path (HIP/gfx950) with a C ABI.

The compute lives in libcgx.so (hand-written HIP kernels); `cgx` is the thin
ctypes binding over it.  PyTorch provides device memory and streams only.
"""
from . import cgx  # noqa: F401
from .cgx import (DeviceCSR, Handle, Opts, Stats, add, axpy, cg_solve, cg_workspace,  # noqa: F401
                  cg_workspace_bytes, csr_spmv, csr_spmv_f32, csr_validate, default_handle,
                  demote, dot, load_library, make_opts, xmul)

__all__ = ["cgx", "DeviceCSR", "Handle", "Opts", "Stats", "add", "axpy", "cg_solve",
           "cg_workspace", "cg_workspace_bytes", "csr_spmv", "csr_spmv_f32", "csr_validate",
           "default_handle", "demote", "dot", "load_library", "make_opts", "xmul"]
