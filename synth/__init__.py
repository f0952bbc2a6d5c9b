"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This package generates inputs only: SplitMix64 streams, the 7-point
finite-difference and Q1 finite-element stiffness matrices in CSR form and
right-hand sides.  It contains none of the solver's arithmetic.

The paper's matrices (Section 5.1, Table "Canvas of the matrices") come from a
Q1 discretisation of the gravity Poisson problem -lap(Phi) = 4 pi G drho on a
200 x 200 x 10 km box; they are not available, so `q1box` rebuilds their
shape and `q1cube` / `fd7` give the unit-cube stand-ins the benchmarks use.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        lib.synth_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_int64, u64p]
        lib.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, f64p]
        lib.synth_normal.argtypes = [ctypes.c_uint64, ctypes.c_int64, f64p]
        lib.synth_fd7_nnz.argtypes = [ctypes.c_int]
        lib.synth_fd7_nnz.restype = ctypes.c_int64
        lib.synth_fd7.argtypes = [ctypes.c_int, i32p, i32p, f64p]
        lib.synth_fd7_var.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, i32p, i32p,
                                      f64p]
        lib.synth_q1_coeffs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, f64p]
        lib.synth_q1cube_nnz.argtypes = [ctypes.c_int]
        lib.synth_q1cube_nnz.restype = ctypes.c_int64
        lib.synth_q1cube_from_coeffs.argtypes = [ctypes.c_int, f64p, i32p, i32p, f64p]
        lib.synth_q1box_nnz.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.synth_q1box_nnz.restype = ctypes.c_int64
        lib.synth_q1box.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, i32p, i32p, f64p]
        lib.synth_blob_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, f64p]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Host CSR matrix: 0-based int32 row starts / columns, float64 values."""

    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n_rows, self.n_cols))
        for i in range(self.n_rows):
            for k in range(self.row_ptr[i], self.row_ptr[i + 1]):
                a[i, self.col_idx[k]] = self.val[k]
        return a


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, np.uint64)
    _load().synth_splitmix64(seed, n, out)
    return out


def uniform(seed: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().synth_uniform(seed, n, lo, hi, out)
    return out


def normal(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().synth_normal(seed, n, out)
    return out


def fd7(N: int) -> CSR:
    """7-point Laplacian, N^3 interior unknowns, stencil 6 / -1."""
    lib = _load()
    n = N ** 3
    nnz = lib.synth_fd7_nnz(N)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    lib.synth_fd7(N, rp, ci, v)
    return CSR(n, n, rp, ci, v, name=f"fd7_{N}")


def fd7_var(N: int, sigma: float, seed: int) -> CSR:
    """7-point -div(k grad u), node coefficients exp(sigma Z), harmonic-mean faces."""
    lib = _load()
    n = N ** 3
    nnz = lib.synth_fd7_nnz(N)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    lib.synth_fd7_var(N, sigma, seed, rp, ci, v)
    return CSR(n, n, rp, ci, v, name=f"fd7var_{N}_s{sigma:g}")


def batch_systems(count: int = 64, n_lo: int = 24, n_hi: int = 96, sigma: float = 1.0,
                  seed0: int = 1000):
    """The batched workload: `count` systems, grid size N ~ U{n_lo..n_hi} drawn
    per system from its own stream (seed0 + s), 7-point FD for even s and Q1
    FEM for odd s, lognormal(0, sigma) coefficients."""
    out = []
    for s in range(count):
        u = splitmix64(seed0 + s, 2)
        N = n_lo + int(u[0] % np.uint64(n_hi - n_lo + 1))
        if s % 2 == 0:
            out.append(fd7_var(N, sigma, int(u[1])))
        else:
            out.append(q1cube(N, sigma, int(u[1])))
    return out


def q1_coeffs(N: int, sigma: float, seed: int) -> np.ndarray:
    out = np.empty((N + 1) ** 3, np.float64)
    _load().synth_q1_coeffs(N, sigma, seed, out)
    return out


def q1cube_from_coeffs(N: int, k_e: np.ndarray) -> CSR:
    lib = _load()
    k_e = np.ascontiguousarray(k_e, dtype=np.float64)
    if k_e.size != (N + 1) ** 3:
        raise ValueError("need (N+1)^3 element coefficients")
    n = N ** 3
    nnz = lib.synth_q1cube_nnz(N)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    lib.synth_q1cube_from_coeffs(N, k_e, rp, ci, v)
    return CSR(n, n, rp, ci, v, name=f"q1cube_{N}")


def q1cube(N: int, sigma: float = 0.0, seed: int = 0) -> CSR:
    """Q1 stiffness on the unit cube, N^3 unknowns, k_e = exp(sigma*Z)."""
    a = q1cube_from_coeffs(N, q1_coeffs(N, sigma, seed))
    a.name = f"q1cube_{N}_s{sigma:g}"
    return a


def q1box(a: int, c: int, Lx: float = 200.0, Ly: float = 200.0, Lz: float = 10.0) -> CSR:
    """Paper-shape Q1 box: a x a x c nodes, Dirichlet nodes as identity rows."""
    lib = _load()
    n = a * a * c
    nnz = lib.synth_q1box_nnz(a, c)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    lib.synth_q1box(a, c, Lx, Ly, Lz, rp, ci, v)
    return CSR(n, n, rp, ci, v, name=f"q1box_{a}x{a}x{c}")


def blob_rhs(N: int, seed: int, nblobs: int = 8) -> np.ndarray:
    out = np.empty(N ** 3, np.float64)
    _load().synth_blob_rhs(N, nblobs, seed, out)
    return out


# Seeds of the standard workloads, fixed once so every consumer draws the same data.
SEED_C1_XSTAR = 0
SEED_VEC_X = 1
SEED_VEC_Y = 2
SEED_C2_COEFF = 10
SEED_C2_BLOBS = 11
SEED_C3_COEFF = 20
SEED_C3_RHS = 21
