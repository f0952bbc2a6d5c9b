#!/usr/bin/env python3
"""Benchmark of the sparse CG hot path on one MI355X.

Workload: Jacobi-preconditioned CG on the 27-point trilinear (Q1) finite
element stiffness matrix of a 128^3 grid (2,097,152 rows, 55,742,968 nnz),
per-element coefficient lognormal(0,1), right-hand side from 8 Gaussian
density blobs, stop at ||r|| <= 1e-8 ||b||.  One step = one full solve from
x0 = 0 (SpMV, fused BLAS-1 updates and dots, preconditioner apply), all in
libcgx's HIP kernels with inputs already resident in HBM.

Printed (one JSON line): achieved HBM GB/s of the solve (algorithmic bytes /
wall time), solves/s, p50/p99 latency, J/solve from the GPU energy counter,
the roofline entry of the dominant kernel (SpMV phase, timed live with HIP
events) and the CPU oracle baseline on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_GRID = 128
SIGMA = 1.0
RTOL = 1e-8


def spmv_bytes(n, nnz):
    """Algorithmic HBM bytes of y = A x: val 8 + col 4 per nonzero, row_ptr 4(n+1), x 8n, y 8n."""
    return 12 * nnz + 4 * (n + 1) + 16 * n


def jacobi_iter_bytes(n, nnz):
    """One Jacobi-CG iteration: SpMV + (x, r read-write; p, q, dinv read; z write) + (z read, p rw)."""
    return spmv_bytes(n, nnz) + 64 * n + 24 * n


def jacobi_setup_bytes(n, nnz):
    """r0 = b - A x0 with diagonal extraction: SpMV + b read + r, z, p, dinv written."""
    return spmv_bytes(n, nnz) + 8 * n + 32 * n


class EnergyMeter:
    """GPU energy through the amdsmi accumulator, sampled in the background
    (it advances about once per second on MI355X): the mean power over an
    interval comes from the counter updates inside it and their own
    timestamps, and energy = power x time."""

    def __init__(self):
        from paper_2112_10823_amd.energy import EnergySampler
        self.sampler = EnergySampler().start()

    def power(self, t0, t1):
        return self.sampler.power_between(t0, t1) if self.sampler.ok else None

    def updates_between(self, t0, t1):
        return sum(1 for u in self.sampler.updates if t0 <= u[0] <= t1)


def wave_tile_rows(n, nnz, entries_per_lane=8):
    """Rows per SpMV wave tile the library picks: the largest power of two in
    [1, 64] whose expected entries fill at most 97% of 64 * entries_per_lane."""
    mean = max(nnz / n, 1.0) if n else 1.0
    rt = 64
    while rt > 1 and rt * mean > 0.97 * 64 * entries_per_lane:
        rt //= 2
    return rt


# The sources the profiled CG SpMV kernel is built from: a change elsewhere
# (batched, serving, Schwarz code) leaves its committed byte counters valid.
SPMV_KERNEL_SOURCES = ("cg.hip", "cgx_device.h", "cgx_internal.h")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_10823_amd", "csrc")
    for f in SPMV_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per launch of the SpMV phase from the committed rocprofv3 counter
    summary, or None when absent or taken on other kernel sources."""
    p = os.path.join(ROOT, "profiles", "cg_spmv_phase_q1_128_counters.md")
    if not os.path.exists(p):
        return None
    txt = open(p).read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash:
        return None
    return float(t.group(1))


def cpu_baseline(A, b, n, nnz, iters=20):
    """The CPU oracle (plain sequential C) on a bounded sample of the same
    workload: `iters` Jacobi-CG iterations on the full matrix, reported in the
    same unit (algorithmic GB/s) with the same byte model."""
    import oracle
    t0 = time.perf_counter()
    oracle.cg(A, b, rtol=0.0, maxit=iters, jacobi=True)
    dt = time.perf_counter() - t0
    gbs = (jacobi_setup_bytes(n, nnz) + iters * jacobi_iter_bytes(n, nnz)) / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} Jacobi-CG iterations (plus setup) of the oracle on the full "
                      f"Q1 {N_GRID}^3 system, {dt:.1f} s"}


def cpu_baseline_all_cores(A, b, n, nnz, iters=20):
    """The same sample with the oracle's all-cores timing build (the same
    source compiled with -O3 -fopenmp: rows and elements in parallel,
    per-thread compensated dot partials), on every thread OpenMP is given."""
    import oracle
    threads = oracle.timing_threads()
    t0 = time.perf_counter()
    oracle.cg_timing(A, b, rtol=0.0, maxit=iters, jacobi=True)
    dt = time.perf_counter() - t0
    gbs = (jacobi_setup_bytes(n, nnz) + iters * jacobi_iter_bytes(n, nnz)) / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle (OpenMP timing build)", "nproc": os.cpu_count(),
            "sample": f"{iters} Jacobi-CG iterations (plus setup) on the full Q1 {N_GRID}^3 "
                      f"system, {dt:.1f} s on {threads} threads"}


def batch_sample():
    """Systems of the 64-system batch measured one at a time: eight, both
    stencils (the stencil alternates with the system index) and sizes across
    the range."""
    return [8 * k + (k % 2) for k in range(8)]


def cpu_baseline_batched(mats):
    """The oracle solving the batch's sample one (system, right-hand side) at
    a time, Jacobi-CG to 1e-8 from 0 on each sampled system's first
    right-hand side: solves/s of the sample, on one core (the plain C
    oracle) and on all cores (its OpenMP timing build)."""
    import oracle
    import synth
    pick = batch_sample()
    rhs = [synth.uniform(1000 + s * 16, mats[s].n_rows) for s in pick]
    desc = (f"systems {pick} of the batch (mean {np.mean([mats[s].nnz for s in pick]) / 1e6:.2f} M "
            f"nnz against {np.mean([A.nnz for A in mats]) / 1e6:.2f} M for all 64), first "
            "right-hand side each, Jacobi-CG to 1e-8 one at a time")
    out = {}
    for key, solve, cores, kind in (
            ("cpu_baseline", oracle.cg, 1, "oracle"),
            ("cpu_baseline_all_cores", oracle.cg_timing, oracle.timing_threads(),
             "oracle (OpenMP timing build)")):
        t0 = time.perf_counter()
        for s, b in zip(pick, rhs):
            solve(mats[s], b, rtol=1e-8, jacobi=True)
        dt = time.perf_counter() - t0
        out[key] = {"value": round(len(pick) / dt, 3), "unit": "solves/s", "cores": cores,
                    "kind": kind, "sample": f"{desc}, {dt:.1f} s"}
    return out


def cpu_baseline_small(A, xs, min_s=2.0):
    """The oracle's plain CG (one core) on the whole 7-point 16^3 solve to
    1e-10 (b = A x* by the oracle's SpMV), repeated for about min_s seconds:
    solves per second."""
    import oracle
    b = oracle.spmv(A, xs)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.cg(A, b, rtol=1e-10)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_s:
            break
    return {"value": round(n / dt, 1), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} whole solves, {dt:.1f} s"}


def cpu_baseline_blas1(x, y, min_s=1.0):
    """The oracle's add (24 bytes per element) and compensated dot (16) on
    one core, each repeated for about min_s seconds: GB/s."""
    import oracle
    out = {}
    for name, fn, bpe in (("add", lambda: oracle.add(x, y), 24), ("dot", lambda: oracle.dot(x, y), 16)):
        t0 = time.perf_counter()
        k = 0
        while True:
            fn()
            k += 1
            dt = time.perf_counter() - t0
            if dt >= min_s:
                break
        out[name + "_GBs"] = round(bpe * x.size * k / dt / 1e9, 2)
    return {"value": out, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"n = {x.size} float64, add then dot, about {min_s:g} s each"}


def cpu_baseline_mixed(A, b, iters=40):
    """The oracle's binary32 CG with float64 reliable updates (delta 1e-2,
    Jacobi) for `iters` iterations on the full mixed-precision system, setup
    and final residual included: binary32 iterations per second."""
    import oracle
    t0 = time.perf_counter()
    oracle.mixed_ru(A, np.asarray(A.val).astype(np.float32), b, rtol=1e-10, delta=1e-2,
                    maxit=iters, jacobi=True)
    dt = time.perf_counter() - t0
    return {"value": round(iters / dt, 3), "unit": "binary32 iterations/s", "cores": 1,
            "kind": "oracle", "sample": f"{iters} iterations of the reliable-update method "
                                       f"(setup, updates and final residual included), {dt:.1f} s"}


def calib_gather_matrix(n):
    """Permutation matrix of n rows (n a multiple of 16) moving 16-entry
    blocks of x (one 128-byte line) to a seeded random order: row i reads
    x[16 perm[i // 16] + i % 16]."""
    import synth
    nb = n // 16
    perm = np.argsort(synth.uniform(77, nb)).astype(np.int64)
    i = np.arange(n, dtype=np.int64)
    col = (16 * perm[i // 16] + i % 16).astype(np.int32)
    return synth.CSR(n, n, np.arange(n + 1, dtype=np.int32), col, np.ones(n))


def mixed_path(cgx, synth, meter, reps=3, cpu=True):
    """The mixed-precision configuration beside the headline: Q1 192^3
    (7,077,888 rows, 189,119,224 nnz), lognormal(0, 1.5), uniform RHS,
    Jacobi, to 1e-10: float64 Jacobi-CG against binary32 CG with float64
    reliable updates (delta 1e-2), wall time per solve (best of `reps`),
    J/solve from the energy counter, and the mixed solution's distance to the
    float64 one."""
    import torch
    N = 192
    A = synth.q1cube(N, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    out = {"workload": f"Q1 hex FEM {N}^3 ({A.n_rows:,} rows, {A.nnz:,} nnz), lognormal(0,1.5), "
                       "uniform RHS, Jacobi, rtol 1e-10"}
    sol = {}
    for name, o in (("fp64_jacobi", cgx.make_opts(rtol=1e-10, precond=1)),
                    ("mixed_ru", cgx.make_opts(rtol=1e-10, precond=1, inner_rtol=1e-2,
                                               precision=cgx.PRECISION_MIXED_RU))):
        ws = cgx.cg_workspace(dA, o)

        def solve():
            x.zero_()
            return cgx.cg_solve(dA, db, x, o, workspace=ws)
        st = solve()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            st = solve()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        _, j = _energy_window(solve, meter, min_s=2.0)
        sol[name] = x.clone()
        out[f"{name}_ms"] = round(best * 1e3, 2)
        out[f"{name}_iters"] = st.iters
        out[f"{name}_j_per_solve"] = round(j, 2) if j is not None else None
        out[f"{name}_relres"] = st.relres
        if name == "mixed_ru":
            out["mixed_ru_updates"] = st.outer_iters
        del ws
    out["time_ratio"] = round(out["mixed_ru_ms"] / out["fp64_jacobi_ms"], 4)
    out["mixed_ru_iters_per_s"] = round(out["mixed_ru_iters"] / (out["mixed_ru_ms"] * 1e-3), 1)
    if cpu:
        out["cpu_baseline"] = cpu_baseline_mixed(A, b)
    out["mixed_vs_fp64_rel_error"] = float(torch.linalg.norm(sol["mixed_ru"] - sol["fp64_jacobi"])
                                           / torch.linalg.norm(sol["fp64_jacobi"]))
    return out


def host_relres(A, b, x):
    """||b - A x|| / ||b|| with scipy's CSR product on the host: a library
    routine independent of the GPU library, used to check the solutions the
    extras report."""
    import scipy.sparse as sp
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
    return float(np.linalg.norm(b - M @ x) / np.linalg.norm(b))


# ------------------------------------------------------------------ extras --
# One JSON line per workload of the benchmark suite, outside the default run.

def _timeit(fn, reps=20, warm=3):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3  # s


def _energy_window(fn, meter, min_s=2.5, min_reps=1, warm_s=1.0):
    """Run fn repeatedly for at least min_s seconds and until the energy
    counter has advanced three times inside the window (at most 4 min_s);
    returns (s per call, J per call or None).  With telemetry on, fn first
    runs untimed for warm_s seconds, so that the board's power has settled
    at the workload's level (it takes about a second to move between
    levels) before the window opens."""
    import torch
    if meter.sampler.ok:
        tw = time.perf_counter()
        while time.perf_counter() - tw < warm_s:
            fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 0
    while (reps < min_reps or time.perf_counter() - t0 < min_s
           or (meter.sampler.ok and meter.updates_between(t0, time.perf_counter()) < 3
               and time.perf_counter() - t0 < 4 * min_s)):
        fn()
        reps += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = (t1 - t0) / reps
    p = meter.power(t0, t1)
    return wall, (p * wall if p is not None else None)


def extra_small_cg(cgx, synth, meter):
    """Plain CG on the 7-point 16^3 grid, b = A x*, x* ~ U[-1,1] seed 0, to
    1e-10; BLAS-1 on 4096-element vectors.  Latency-bound (0.5 MB of data)."""
    import torch
    A = synth.fd7(16)
    xs = synth.uniform(synth.SEED_C1_XSTAR, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A)
    dxs = torch.from_numpy(xs).cuda()
    db = cgx.csr_spmv(dA, dxs)
    dx = torch.zeros_like(db)
    opts = cgx.make_opts(rtol=1e-10)
    ws = cgx.cg_workspace(dA, opts)
    st = None

    def solve():
        nonlocal st
        dx.zero_()
        st = cgx.cg_solve(dA, db, dx, opts, workspace=ws)

    for _ in range(5):
        solve()
    wall, jsolve = _energy_window(solve, meter, min_s=2.0)
    err = float(torch.linalg.norm(dx - dxs) / torch.linalg.norm(dxs))
    x4 = torch.from_numpy(synth.uniform(synth.SEED_VEC_X, 4096)).cuda()
    y4 = torch.from_numpy(synth.uniform(synth.SEED_VEC_Y, 4096)).cuda()
    z4 = torch.empty_like(x4)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    t_add = _timeit(lambda: cgx.add(x4, y4, z4), reps=200)
    t_mul = _timeit(lambda: cgx.xmul(x4, y4, z4), reps=200)
    t_dot = _timeit(lambda: cgx.dot(x4, y4, out), reps=200)
    return {"workload": "plain CG, 7-point 16^3 (4096 rows, 27136 nnz), rtol 1e-10",
            "iters": st.iters, "status": st.status, "solve_us": round(wall * 1e6, 1),
            "device_us": round(st.device_ms * 1e3, 1),
            "us_per_iter": round(st.device_ms * 1e3 / max(st.iters, 1), 2),
            "solves_per_s": round(1.0 / wall, 1), "path": "single workgroup",
            "rel_err_vs_xstar": err,
            "j_per_solve": round(jsolve, 5) if jsolve is not None else None,
            "blas1_n4096_us": {"add": round(t_add * 1e6, 2), "xmul": round(t_mul * 1e6, 2),
                               "dot": round(t_dot * 1e6, 2)},
            "bound": "latency (whole problem on chip)",
            "cpu_baseline": cpu_baseline_small(A, xs)}


def extra_blas1_sweep(cgx, synth):
    """BLAS-1 GB/s for n = 2^20 .. 2^26.  Same buffers every call: sizes up to
    2^23 (<= 200 MB working set) sit in the 256 MB MALL, so those rates are
    cache-resident, not HBM."""
    import torch
    rows = []
    for lg in range(20, 27):
        n = 1 << lg
        x = torch.from_numpy(synth.uniform(synth.SEED_VEC_X, n)).cuda()
        y = torch.from_numpy(synth.uniform(synth.SEED_VEC_Y, n)).cuda()
        z = torch.empty_like(x)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        reps = max(10, min(200, (1 << 28) // n))
        t_add = _timeit(lambda: cgx.add(x, y, z), reps=reps)
        t_mul = _timeit(lambda: cgx.xmul(x, y, z), reps=reps)
        t_axpy = _timeit(lambda: cgx.axpy(0.5, x, z), reps=reps)
        t_dot = _timeit(lambda: cgx.dot(x, y, out), reps=reps)
        rows.append({"n": n, "add_GBs": round(24 * n / t_add / 1e9, 1),
                     "xmul_GBs": round(24 * n / t_mul / 1e9, 1),
                     "axpy_GBs": round(24 * n / t_axpy / 1e9, 1),
                     "dot_GBs": round(16 * n / t_dot / 1e9, 1),
                     "mall_resident": 24 * n < 256e6})
        del x, y, z
    n = 1 << 24
    cpu = cpu_baseline_blas1(synth.uniform(synth.SEED_VEC_X, n), synth.uniform(synth.SEED_VEC_Y, n))
    return {"workload": "BLAS-1 add / xmul / axpy / dot, float64 U[-1,1]", "rows": rows,
            "cpu_baseline": cpu}


def extra_spmv_and_cg(cgx, synth, meter):
    """Standalone SpMV and plain / Jacobi CG on the Q1 128^3 system."""
    import torch
    A = synth.q1cube(N_GRID, SIGMA, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(N_GRID, synth.SEED_C2_BLOBS)
    n, nnz = A.n_rows, A.nnz
    dA = cgx.DeviceCSR.from_host(A)
    xv = torch.from_numpy(synth.uniform(4, n)).cuda()
    yv = torch.empty_like(xv)
    t_sp = _timeit(lambda: cgx.csr_spmv(dA, xv, yv), reps=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = cgx.SellMatrix(dA)  # sliced-ELL copy (sync build)
    t_build = time.perf_counter() - t0
    t_sell = _timeit(lambda: cgx.sell_spmv(S, xv, yv), reps=50)
    sell_bytes = 12 * S.stored + 8 * (S.n_slices + 1) + 16 * n
    db = torch.from_numpy(b).cuda()
    res = {"workload": "Q1 128^3 lognormal(0,1), blob RHS, rtol 1e-8",
           "spmv_us": round(t_sp * 1e6, 1),
           "spmv_GBs": round(spmv_bytes(n, nnz) / t_sp / 1e9, 1),
           "sell": {"stored": S.stored, "padding": round(S.stored / nnz - 1, 5),
                    "build_ms": round(t_build * 1e3, 2), "spmv_us": round(t_sell * 1e6, 1),
                    "spmv_GBs": round(sell_bytes / t_sell / 1e9, 1),
                    "spmv_GBs_csr_bytes": round(spmv_bytes(n, nnz) / t_sell / 1e9, 1)}}
    for name, pc, sell in (("plain", 0, None), ("jacobi", 1, None), ("jacobi_sell", 1, S)):
        dx = torch.zeros_like(db)
        opts = cgx.make_opts(rtol=RTOL, precond=pc)
        ws = cgx.cg_workspace(dA, opts)
        st = cgx.cg_solve(dA, db, dx, opts, workspace=ws, sell=sell)

        def solve():
            dx.zero_()
            cgx.cg_solve(dA, db, dx, opts, workspace=ws, sell=sell)

        wall, j = _energy_window(solve, meter, min_s=2.0)
        per_it = spmv_bytes(n, nnz) + (72 * n if pc == 0 else 88 * n)
        res[name] = {"iters": st.iters, "solve_ms": round(wall * 1e3, 2),
                     "GBs": round(per_it * st.iters / wall / 1e9, 1),
                     "j_per_solve": round(j, 3) if j is not None else None}
    return res


def extra_schwarz(cgx, synth, meter):
    """Additive Schwarz (slabs of the Q1 128^3 grid, overlap in grid layers of
    N^2 rows) around flexible CG, every subdomain solved by the batched CG
    solver; against Jacobi-CG on the same system (lognormal(0,1), blob RHS,
    1e-8).  The subdomain phase's rate uses the batched model bytes per
    iteration (12 nnz_i + 4 (m_i + 1) + 88 m_i summed over the subdomains),
    with the largest subdomain iteration count of every outer step."""
    import torch
    A = synth.q1cube(N_GRID, SIGMA, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(N_GRID, synth.SEED_C2_BLOBS)
    n = A.n_rows
    layer = N_GRID * N_GRID
    dA = cgx.DeviceCSR.from_host(A)
    db = torch.from_numpy(b).cuda()
    dx = torch.zeros_like(db)
    res = {"workload": "Q1 128^3 lognormal(0,1), blob RHS, rtol 1e-8; additive Schwarz slabs "
                       "around flexible CG, subdomains by batched Jacobi-CG"}
    jopts = cgx.make_opts(rtol=RTOL, precond=cgx.PRECOND_JACOBI)
    ws = cgx.cg_workspace(dA, jopts)
    st = cgx.cg_solve(dA, db, dx, jopts, workspace=ws)

    def jsolve():
        dx.zero_()
        cgx.cg_solve(dA, db, dx, jopts, workspace=ws)

    wall, j = _energy_window(jsolve, meter, min_s=2.0)
    res["jacobi_cg"] = {"iters": st.iters, "solve_ms": round(wall * 1e3, 2),
                        "j_per_solve": round(j, 3) if j is not None else None}
    rows = []
    for S, layers, tau, m in ((8, 1, 0.1, 100), (8, 2, 0.1, 100), (32, 1, 0.1, 100),
                              (32, 1, -1.0, 8), (128, 1, 0.1, 100), (128, 1, -1.0, 8)):
        t0 = time.perf_counter()
        D = cgx.SchwarzDecomposition(dA, S, layers * layer)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        opts = cgx.make_opts(rtol=RTOL, maxit=m, inner_rtol=tau, precond=cgx.PRECOND_JACOBI)
        wsd = torch.empty(D.workspace_bytes(), dtype=torch.uint8, device="cuda")
        dx.zero_()
        st = cgx.schwarz_solve(dA, D, db, dx, opts, workspace=wsd)
        relres = host_relres(A, b, dx.cpu().numpy())

        def solve():
            dx.zero_()
            cgx.schwarz_solve(dA, D, db, dx, opts, workspace=wsd)

        wall, j = _energy_window(solve, meter, min_s=2.0)
        nnz_off = D.arrays()[0].cpu().numpy()
        lrows = D.local_rows
        # batched iteration: SpMM p, q; update r, q, r; p update p, r, x, p, x
        it_bytes = 12 * int(nnz_off[-1]) + 4 * (lrows + S) + 80 * lrows
        rows.append({"n_sub": S, "overlap_layers": layers,
                     "inner": f"tau {tau:g}, cap {m}" if tau > 0 else f"{m} iterations",
                     "status": st.status, "outer": st.outer_iters, "inner_iters": st.iters,
                     "build_ms": round(build_ms, 1), "solve_ms": round(wall * 1e3, 1),
                     "local_share": round(st.phase_ms[0] / st.device_ms, 3),
                     "local_GBs_model": round(it_bytes * st.iters / (st.phase_ms[0] * 1e-3) / 1e9, 1),
                     "j_per_solve": round(j, 3) if j is not None else None,
                     "true_relres_host_spmv": relres})
        print(f"# schwarz S={S} layers={layers} tau={tau} done", file=sys.stderr, flush=True)
        del D, wsd
    res["rows"] = rows
    return res


def extra_mixed(cgx, synth, meter):
    """Q1 192^3 lognormal(0,1.5), uniform RHS, to 1e-10: float64 CG against
    binary32-inner refinement (restarted) and binary32 CG with float64
    reliable updates, each plain and Jacobi-preconditioned."""
    import torch
    A = synth.q1cube(192, 1.5, seed=synth.SEED_C3_COEFF)
    b = synth.uniform(synth.SEED_C3_RHS, A.n_rows)
    dA = cgx.DeviceCSR.from_host(A, with_f32=True)
    db = torch.from_numpy(b).cuda()
    out = {"workload": "Q1 192^3 (7,077,888 rows, 189,119,224 nnz) lognormal(0,1.5), "
                       "uniform RHS, rtol 1e-10"}
    S = cgx.SellMatrix(dA)  # sliced-ELL copy (float64 and binary32 values)
    runs = [("fp64_plain", cgx.PRECISION_FP64, 0, 0.0, None),
            ("fp64_jacobi", cgx.PRECISION_FP64, 1, 0.0, None),
            ("mixed_plain_tau1e-3", cgx.PRECISION_MIXED, 0, 1e-3, None),
            ("mixed_jacobi_tau1e-2", cgx.PRECISION_MIXED, 1, 1e-2, None),
            ("mixed_jacobi_tau1e-3", cgx.PRECISION_MIXED, 1, 1e-3, None),
            ("mixed_jacobi_tau1e-4", cgx.PRECISION_MIXED, 1, 1e-4, None),
            ("fp64_jacobi_sell", cgx.PRECISION_FP64, 1, 0.0, S),
            ("mixed_jacobi_tau1e-2_sell", cgx.PRECISION_MIXED, 1, 1e-2, S),
            ("ru_plain_delta1e-2", cgx.PRECISION_MIXED_RU, 0, 1e-2, None),
            ("ru_jacobi_delta1e-1", cgx.PRECISION_MIXED_RU, 1, 1e-1, None),
            ("ru_jacobi_delta1e-2", cgx.PRECISION_MIXED_RU, 1, 1e-2, None),
            ("ru_jacobi_delta1e-3", cgx.PRECISION_MIXED_RU, 1, 1e-3, None),
            ("ru_jacobi_delta1e-2_sell", cgx.PRECISION_MIXED_RU, 1, 1e-2, S)]
    ref = None
    for name, prec, pc, tau, sell in runs:
        opts = cgx.make_opts(rtol=1e-10, precond=pc, precision=prec, inner_rtol=tau,
                             maxit=20000)
        ws = cgx.cg_workspace(dA, opts)
        dx = torch.zeros_like(db)
        st = None

        def solve():
            nonlocal st
            dx.zero_()
            st = cgx.cg_solve(dA, db, dx, opts, workspace=ws, sell=sell)

        solve()
        wall, j = _energy_window(solve, meter, min_s=2.0)
        x = dx.cpu().numpy()
        if ref is None:
            ref = x
        tr = host_relres(A, b, x)
        out[name] = {"status": st.status, "iters": st.iters, "outer": st.outer_iters,
                     "solve_ms": round(wall * 1e3, 1), "solves_per_s": round(1 / wall, 3),
                     "j_per_solve": round(j, 2) if j is not None else None,
                     "true_relres_host_spmv": tr, "kappa_est": round(st.kappa_est, 1),
                     "rel_diff_vs_fp64_plain": float(np.linalg.norm(x - ref) / np.linalg.norm(ref))}
        del ws
    return out


def extra_batched(cgx, synth, meter):
    """64 systems (7-point / Q1 alternating, N ~ U{24..96}, lognormal(0,1)),
    16 RHS each, Jacobi CG to 1e-8: batched against one solve at a time."""
    import torch
    mats = synth.batch_systems(64)
    items = []
    for s, A in enumerate(mats):
        B = torch.empty(16, A.n_rows, dtype=torch.float64)
        for j in range(16):
            B[j] = torch.from_numpy(synth.uniform(1000 + s * 16 + j, A.n_rows))
        items.append((cgx.DeviceCSR.from_host(A, with_f32=True), B.cuda(),
                      torch.zeros(16, A.n_rows, dtype=torch.float64, device="cuda")))
    opts = cgx.make_opts(rtol=1e-8, precond=1)
    ws = cgx.batch_workspace(items)
    st = cgx.cg_solve_batched(items, opts, workspace=ws)  # tunes + warms

    def solve():
        nonlocal st
        for _, _, X in items:
            X.zero_()
        st = cgx.cg_solve_batched(items, opts, workspace=ws)

    wall, jb = _energy_window(solve, meter, min_s=2.0)
    ok = sum(v.status == cgx.OK for row in st for v in row)
    byts = 0.0
    for (dA, B, X), row in zip(items, st):
        it = max(v.iters for v in row)
        # per iteration: the matrix; p, q (SpMM), r, q, r (update), p, r, x,
        # p, x (p update) for each of the 16 right-hand sides
        byts += it * (12 * dA.nnz + 4 * (dA.n_rows + 1) + 80 * 16 * dA.n_rows)
    sched = cgx.batch_schedule(items, workspace=ws)
    # one right-hand side at a time with the single-system solver (a sample, scaled)
    sample = batch_sample()
    t_single = 0.0
    for s in sample:
        dA, B, _ = items[s]
        x1 = torch.zeros(dA.n_rows, dtype=torch.float64, device="cuda")
        o1 = cgx.make_opts(rtol=1e-8, precond=1)
        w1 = cgx.cg_workspace(dA, o1)
        cgx.cg_solve(dA, B[0].contiguous(), x1, o1, workspace=w1)
        t1 = time.perf_counter()
        for j in range(4):
            x1.zero_()
            cgx.cg_solve(dA, B[j].contiguous(), x1, o1, workspace=w1)
        t_single += (time.perf_counter() - t1) / 4 * 16
    t_single *= 64 / len(sample)
    # the same batch float32-refined: float64 residual and update, binary32
    # inner batched Jacobi-CG to 1e-2
    mopts = cgx.make_opts(rtol=1e-8, precond=1, precision=cgx.PRECISION_MIXED, inner_rtol=1e-2)
    mws = cgx.batch_workspace(items, opts=mopts)
    for _, _, X in items:
        X.zero_()
    mst = cgx.cg_solve_batched(items, mopts, workspace=mws)
    check = []
    for s in (0, 21, 42, 63):
        dA, B, X = items[s]
        for j in (0, 15):
            b = B[j].cpu().numpy()
            x = X[j].cpu().numpy()
            check.append(host_relres(mats[s], b, x))

    def msolve():
        nonlocal mst
        for _, _, X in items:
            X.zero_()
        mst = cgx.cg_solve_batched(items, mopts, workspace=mws)

    mwall, mjb = _energy_window(msolve, meter, min_s=2.0)
    mixed = {"solves_per_s": round(1024 / mwall, 1), "batch_s": round(mwall, 3),
             "converged": sum(v.status == cgx.OK for row in mst for v in row),
             "j_per_solve": round(mjb / 1024, 4) if mjb is not None else None,
             "inner_iters_mean": round(float(np.mean([v.iters for row in mst for v in row])), 1),
             "outer_mean": round(float(np.mean([v.outer_iters for row in mst for v in row])), 2),
             "true_relres_max_sample": max(check)}
    # the same batch with binary32 CG and float64 reliable updates (delta 1e-2)
    ropts = cgx.make_opts(rtol=1e-8, precond=1, precision=cgx.PRECISION_MIXED_RU,
                          inner_rtol=1e-2)
    rst = None

    def rsolve():
        nonlocal rst
        for _, _, X in items:
            X.zero_()
        rst = cgx.cg_solve_batched(items, ropts, workspace=mws)

    rsolve()
    rcheck = []
    for s in (0, 21, 42, 63):
        dA, B, X = items[s]
        for j in (0, 15):
            rcheck.append(host_relres(mats[s], B[j].cpu().numpy(), X[j].cpu().numpy()))
    rwall, rjb = _energy_window(rsolve, meter, min_s=2.0)
    ru = {"solves_per_s": round(1024 / rwall, 1), "batch_s": round(rwall, 3),
          "converged": sum(v.status == cgx.OK for row in rst for v in row),
          "j_per_solve": round(rjb / 1024, 4) if rjb is not None else None,
          "iters_mean": round(float(np.mean([v.iters for row in rst for v in row])), 1),
          "updates_mean": round(float(np.mean([v.outer_iters for row in rst for v in row])), 2),
          "true_relres_max_sample": max(rcheck)}
    return {"workload": "64 systems N~U{24..96} 7-point/Q1 lognormal(0,1), 16 RHS each, "
                        "Jacobi CG rtol 1e-8",
            "float32_refined": mixed, "reliable_updates": ru,
            "solves": 1024, "converged": ok, "batch_s": round(wall, 3),
            "fp64_iters_mean": round(float(np.mean([v.iters for row in st for v in row])), 1),
            "solves_per_s": round(1024 / wall, 1),
            "model_GBs": round(byts / wall / 1e9, 1),
            "j_per_solve": round(jb / 1024, 4) if jb is not None else None,
            "one_at_a_time_est_s": round(t_single, 3),
            "one_at_a_time_solves_per_s": round(1024 / t_single, 1),
            "one_at_a_time_sample": sample,
            "schedule_M": {"fd7": sched[0], "q1": sched[1]},
            **cpu_baseline_batched(mats)}


def extra_serving(cgx, synth, meter, n_req=300, pool_systems=24, seed=5, full=True):
    """Poisson arrivals of solve requests on resident Q1 systems whose row
    counts follow ln(rows) ~ N(mu, sigma) truncated to [1e4, 4e6] (pool of
    `pool_systems` resident systems, bounded from the 256 of the full
    workload), lognormal(0,1), uniform RHS, rtol 1e-8.  full=False (the long
    stream) runs, for plain float64 CG, float64 Jacobi-CG and binary32
    Jacobi-CG with float64 reliable updates, the burst and one Poisson rate
    at 0.8 of it."""
    import torch
    rng = np.random.default_rng(seed)
    mu = 0.5 * (math.log(1e4) + math.log(4e6))
    sg = (math.log(4e6) - math.log(1e4)) / 4
    mats = []
    for i in range(pool_systems):
        while True:
            r = math.exp(rng.normal(mu, sg))
            if 1e4 <= r <= 4e6:
                break
        N = max(2, round(r ** (1 / 3)))
        A = synth.q1cube(N, 1.0, 2000 + i)
        mats.append((A, cgx.DeviceCSR.from_host(A, with_f32=True)))
    opts = cgx.make_opts(rtol=1e-8)
    picks = rng.integers(0, pool_systems, n_req)
    max_n = max(A.n_rows for A, _ in mats)
    pool_bytes = 48 * cgx.Server.request_bytes(max_n) + (64 << 20)
    pool_t = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    bs = [torch.from_numpy(synth.uniform(7000 + i, A.n_rows)).cuda() for i, (A, _) in enumerate(mats)]

    def run(qps, max_group=16, opts=opts):
        h = cgx.Handle()
        gaps = rng.exponential(1.0 / qps, n_req) if qps else np.zeros(n_req)
        lat, ok = [], 0
        out = [torch.zeros_like(bs[k]) for k in picks]
        with cgx.Server(pool_t, max_slots=48, handle=h, max_group=max_group) as srv:
            t0 = time.perf_counter()
            tickets = []
            nxt = t0
            for i, k in enumerate(picks):
                nxt += gaps[i]
                while time.perf_counter() < nxt:
                    pass
                tickets.append(srv.submit(mats[k][1], bs[k], out[i], opts))
                if (i + 1) % 1000 == 0:
                    print(f"# serving qps={qps:.1f}: {i + 1} of {n_req} submitted",
                          file=sys.stderr, flush=True)
            for i, t in enumerate(tickets):
                st = srv.wait(t)
                ok += st.status == cgx.OK
                lat.append(st.latency_ms)
                if (i + 1) % 1000 == 0:
                    print(f"# serving qps={qps:.1f}: {i + 1} of {n_req} done", file=sys.stderr,
                          flush=True)
            wall = time.perf_counter() - t0
        p = meter.power(t0, t0 + wall)
        lat.sort()
        return {"qps": round(qps, 2) if qps else "burst", "max_group": max_group,
                "precond": "jacobi" if opts.precond else "none",
                "precision": {cgx.PRECISION_MIXED: "mixed",
                              cgx.PRECISION_MIXED_RU: "mixed_ru"}.get(opts.precision, "fp64"),
                "solves_per_s": round(n_req / wall, 2),
                "p50_ms": round(lat[len(lat) // 2], 2),
                "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 2),
                "ok": ok, "wall_s": round(wall, 2),
                "j_per_solve": round(p * wall / n_req, 3) if p is not None else None}

    def sequential(opts=opts):
        """The same requests solved one after another with the single-system
        float64 solver (plain CG, the paper's method, unless Jacobi is asked
        for), no batching."""
        h = cgx.Handle()
        out = [torch.zeros_like(bs[k]) for k in picks]
        wss = {k: cgx.cg_workspace(mats[k][1], opts) for k in set(picks.tolist())}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok = 0
        for i, k in enumerate(picks):
            st = cgx.cg_solve(mats[k][1], bs[k], out[i], opts, workspace=wss[k], handle=h)
            ok += st.status == cgx.OK
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        p = meter.power(t0, t0 + wall)
        return {"solves_per_s": round(n_req / wall, 2), "wall_s": round(wall, 2), "ok": ok,
                "j_per_solve": round(p * wall / n_req, 3) if p is not None else None}

    jac = cgx.make_opts(rtol=1e-8, precond=cgx.PRECOND_JACOBI)
    rmix = cgx.make_opts(rtol=1e-8, precond=cgx.PRECOND_JACOBI,
                         precision=cgx.PRECISION_MIXED_RU, inner_rtol=1e-2)
    sat = run(0)  # all requests at once: saturation throughput
    if not full:
        rows = [sat, run(0.8 * sat["solves_per_s"])]
        for o in (jac, rmix):
            osat = run(0, opts=o)
            rows += [osat, run(0.8 * osat["solves_per_s"], opts=o)]
        return {"workload": f"{n_req} Poisson-arrival requests on {pool_systems} resident Q1 "
                            f"systems (rows lognormal in [1e4, 4e6]), lognormal(0,1), rtol 1e-8",
                "rows": rows, "pool_rows": sorted(A.n_rows for A, _ in mats)}
    rows = [sat, run(0, max_group=1)]
    for f in (0.5, 0.8, 0.95):
        rows.append(run(f * sat["solves_per_s"]))
    rows.append(run(0, opts=jac))
    # binary32-refined requests (float64 residual, update and stopping test;
    # binary32 inner Jacobi-CG to 1e-2), burst and Poisson at 0.8 of it
    mix = cgx.make_opts(rtol=1e-8, precond=cgx.PRECOND_JACOBI, precision=cgx.PRECISION_MIXED,
                        inner_rtol=1e-2)
    msat = run(0, opts=mix)
    rows += [msat, run(0.8 * msat["solves_per_s"], opts=mix)]
    # binary32 CG with float64 reliable updates (delta 1e-2)
    rsat = run(0, opts=rmix)
    rows += [rsat, run(0.8 * rsat["solves_per_s"], opts=rmix)]
    return {"workload": f"{n_req} Poisson-arrival requests on {pool_systems} resident Q1 systems "
                        f"(rows lognormal in [1e4, 4e6]), lognormal(0,1), rtol 1e-8",
            "rows": rows, "one_at_a_time_fp64_cg": sequential(),
            "one_at_a_time_fp64_jacobi_cg": sequential(jac),
            "pool_rows": sorted(A.n_rows for A, _ in mats)}


# The paper's seven gravity matrices, rebuilt by shape (Q1 on an a x a x c
# node grid of the 200 x 200 x 10 km box, Dirichlet nodes as identity rows):
# (a, c) and the SpMV / plain-CG times and energies the paper prints for
# its own GPU, as context.
PAPER_SHAPES = [(46, 48), (66, 68), (86, 88), (94, 96), (106, 108), (106, 118), (116, 118)]
PAPER_SPMV_MS = [0.943, 2.699, 5.963, 7.877, 11.222, 12.405, 14.661]
PAPER_SPMV_J = [0.136, 0.401, 0.891, 1.176, 1.676, 1.807, 2.165]
PAPER_CG_ITERS = [203, 299, 394, 435, 491, 538, None]
PAPER_CG_S = [0.313, 1.155, 2.460, 4.336, 6.872, 8.180, None]
PAPER_CG_J = [31.363, 142.284, 329.078, 597.618, 970.115, 1159.492, None]


def extra_paper_shapes(cgx, synth, meter):
    """SpMV and plain CG (rtol 1e-6, RHS U[-1,1] seed 7: the paper states
    neither) on the paper-shape matrices, beside the paper's own figures."""
    import torch
    rows = []
    for i, (a, c) in enumerate(PAPER_SHAPES):
        A = synth.q1box(a, c)
        n, nnz = A.n_rows, A.nnz
        dA = cgx.DeviceCSR.from_host(A)
        b = torch.from_numpy(synth.uniform(7, n)).cuda()
        y = torch.empty_like(b)
        sp_s, sp_j = _energy_window(lambda: cgx.csr_spmv(dA, b, y), meter, min_s=2.0, min_reps=50)
        S = cgx.SellMatrix(dA)
        sell_s = _timeit(lambda: cgx.sell_spmv(S, b, y), reps=50)
        opts = cgx.make_opts(rtol=1e-6)
        ws = cgx.cg_workspace(dA, opts)
        x = torch.zeros_like(b)
        st = cgx.cg_solve(dA, b, x, opts, workspace=ws)

        def solve():
            x.zero_()
            cgx.cg_solve(dA, b, x, opts, workspace=ws)

        cg_s, cg_j = _energy_window(solve, meter, min_s=2.0)
        rows.append({"a": a, "c": c, "n": n, "nnz": nnz,
                     "spmv_us": round(sp_s * 1e6, 2),
                     "spmv_GBs": round(spmv_bytes(n, nnz) / sp_s / 1e9, 1),
                     "spmv_j": round(sp_j, 5) if sp_j is not None else None,
                     "sell_spmv_us": round(sell_s * 1e6, 2),
                     "sell_spmv_GBs_csr_bytes": round(spmv_bytes(n, nnz) / sell_s / 1e9, 1),
                     "paper_spmv_ms": PAPER_SPMV_MS[i], "paper_spmv_j": PAPER_SPMV_J[i],
                     "cg_iters": st.iters, "cg_ms": round(cg_s * 1e3, 3),
                     "cg_j": round(cg_j, 4) if cg_j is not None else None,
                     "paper_cg_iters": PAPER_CG_ITERS[i], "paper_cg_s": PAPER_CG_S[i],
                     "paper_cg_j": PAPER_CG_J[i]})
        del dA, ws, S
    return {"workload": "the paper's 7 gravity-matrix shapes (Q1, a x a x c nodes, identity "
                        "Dirichlet rows); SpMV, plain CG to 1e-6", "rows": rows}


def extra_transfer(meter, sizes_mib=(1, 16, 256, 1024), min_s=2.0):
    """Host <-> device copies (the paper's transfer figure gives no numbers):
    float64 buffers of 1 MiB to 1 GiB, pinned and pageable host memory,
    each direction timed with events and its energy taken over >= min_s."""
    import torch
    rows = []
    for mib in sizes_mib:
        nel = mib * (1 << 20) // 8
        dev_buf = torch.empty(nel, dtype=torch.float64, device="cuda")
        for pinned in (True, False):
            host = torch.empty(nel, dtype=torch.float64, pin_memory=pinned)
            host.fill_(1.0)
            for direction in ("h2d", "d2h"):
                if direction == "h2d":
                    fn = lambda: dev_buf.copy_(host, non_blocking=pinned)  # noqa: E731
                else:
                    fn = lambda: host.copy_(dev_buf, non_blocking=pinned)  # noqa: E731
                t = _timeit(fn, reps=max(3, min(200, 2048 // mib)), warm=2)
                wall, j = _energy_window(fn, meter, min_s=min_s, min_reps=3)
                rows.append({"MiB": mib, "pinned": pinned, "dir": direction,
                             "ms": round(t * 1e3, 4), "GBs": round(mib * (1 << 20) / t / 1e9, 2),
                             "j_per_GB": round(j / (mib * (1 << 20) / 1e9), 3) if j else None})
            del host
        del dev_buf
    return {"workload": "host<->device copies, float64, pinned / pageable", "rows": rows}


def extra_energy_phases(cgx, synth, meter, phase_s=8.0, runs=3):
    """The paper's Section 4 analysis on this GPU's energy counter: runs of
    idle / add / xmul / axpy / dot / SpMV / Jacobi-CG / idle phases of
    phase_s seconds each on the Q1 128^3 system and vectors of its length;
    the power trace of each run is cut into phases by the variance-based
    step detector (noise from the first idle phase), the runs with the most
    common phase pattern are averaged, and the per-call energies are used to
    check the paper's composition claim for one CG iteration."""
    import torch
    from paper_2112_10823_amd.energy import (Segment, detect_steps, merge_short, most_common_pattern,
                                             noise_from_differences, phase_pattern, robust_spread,
                                             segments_of)
    A = synth.q1cube(N_GRID, SIGMA, seed=synth.SEED_C2_COEFF)
    n = A.n_rows
    dA = cgx.DeviceCSR.from_host(A)
    x = torch.from_numpy(synth.uniform(synth.SEED_VEC_X, n)).cuda()
    y = torch.from_numpy(synth.uniform(synth.SEED_VEC_Y, n)).cuda()
    z = torch.empty_like(x)
    w = y.clone()  # the axpy phase accumulates into w (|w| stays below 1e7)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    db = torch.from_numpy(synth.blob_rhs(N_GRID, synth.SEED_C2_BLOBS)).cuda()
    xs = torch.zeros_like(db)
    opts = cgx.make_opts(rtol=RTOL, precond=cgx.PRECOND_JACOBI)
    ws = cgx.cg_workspace(dA, opts)
    st = cgx.cg_solve(dA, db, xs, opts, workspace=ws)

    def solve():
        xs.zero_()
        cgx.cg_solve(dA, db, xs, opts, workspace=ws)

    ops = [("idle", None), ("add", lambda: cgx.add(x, y, z)), ("xmul", lambda: cgx.xmul(x, y, z)),
           ("axpy", lambda: cgx.axpy(0.5, x, w)), ("dot", lambda: cgx.dot(x, y, out)),
           ("spmv", lambda: cgx.csr_spmv(dA, x, z)), ("jacobi_cg", solve), ("idle_end", None)]
    per_run, phase_lists = [], []
    direct = {name: [] for name, _ in ops}
    for r in range(runs):
        torch.cuda.synchronize()
        time.sleep(2.0)  # back to idle before the run
        bounds = []
        for name, fn in ops:
            t0 = time.perf_counter()
            calls = 0
            if fn is None:
                time.sleep(phase_s)
            else:
                while time.perf_counter() - t0 < phase_s:
                    for _ in range(20):
                        fn()
                    calls += 20
                    torch.cuda.synchronize()
            t1 = time.perf_counter()
            bounds.append((name, t0, t1, calls))
            print(f"# energy run {r}: phase {name} done, {calls} calls", file=sys.stderr, flush=True)
        t, p = meter.sampler.trace()
        sel = (t >= bounds[0][1]) & (t <= bounds[-1][2])
        t, p = t[sel], p[sel]
        # the noise sample: the first idle phase past its first two seconds
        # (its spread by median absolute deviation: the last sample may reach
        # into the next phase); the estimate from the trace's own differences
        # where it is larger; at least 10 W, the drift of the board's power
        # within one steady phase, so that drift is not cut into phases
        idle = p[(t >= bounds[0][1] + 2.0) & (t <= bounds[0][2])]
        idle_sd = robust_spread(idle)
        noise = max(idle_sd, noise_from_differences(p), 10.0)
        # one counter sample spans about a second, so the sample taken across a
        # phase boundary mixes two levels: segments shorter than three samples
        # are such mixtures and join the closer neighbour
        cuts = merge_short(p, detect_steps(p, noise, min_len=1), 3)
        segs = segments_of(p, cuts)
        dt = float(np.median(np.diff(t))) if t.size > 1 else 1.0
        phase_lists.append([((sg.end - sg.start) * dt, sg.level) for sg in segs])
        for name, t0, t1, calls in bounds:
            pw = meter.power(t0 + 1.0, t1)  # the first second is the ramp
            if pw is not None:
                direct[name].append((pw, (t1 - t0) / calls if calls else None))
        per_run.append({"samples": int(p.size), "noise_W": round(noise, 2), "idle_sd_W": round(idle_sd, 2),
                        "trace_W": [round(float(v), 1) for v in p],
                        "phases": [[round(d, 1), round(lv, 1)] for d, lv in phase_lists[-1]]})
    pat, keep, phases = most_common_pattern(phase_lists)
    table = {}
    for name, vals in direct.items():
        if not vals:
            continue
        pw = float(np.mean([v[0] for v in vals]))
        per_call = [v[1] for v in vals if v[1] is not None]
        row = {"W": round(pw, 1)}
        if per_call:
            s_call = float(np.mean(per_call))
            row.update({"us_per_call": s_call, "J_per_call": pw * s_call})
        table[name] = row
    comp = None
    if all(k in table and "J_per_call" in table[k] for k in ("spmv", "dot", "axpy", "xmul", "jacobi_cg")):
        pred = (table["spmv"]["J_per_call"] + 2 * table["dot"]["J_per_call"]
                + 3 * table["axpy"]["J_per_call"] + table["xmul"]["J_per_call"])
        meas = table["jacobi_cg"]["J_per_call"] / st.iters
        comp = {"iters": st.iters, "predicted_J_per_iter": round(pred, 4),
                "measured_J_per_iter": round(meas, 4), "measured_over_predicted": round(meas / pred, 3)}
    for row in table.values():
        if "J_per_call" in row:
            row["J_per_call"] = round(row["J_per_call"], 5)
            row["us_per_call"] = round(row["us_per_call"] * 1e6, 1)
    return {"workload": f"{runs} runs of {len(ops)} phases x {phase_s:g} s; vectors of {n} float64, "
                        "Q1 128^3 SpMV and Jacobi-CG", "runs": per_run,
            "most_common_pattern": list(pat), "runs_kept": keep,
            "pattern_of_known_phases": list(phase_pattern(
                [Segment(0, 0, table[name]["W"]) for name, _ in ops if name in table])),
            "phases_W": [[round(d, 1), round(lv, 1)] for d, lv in phases],
            "per_op_known_boundaries": table, "composition": comp}


def run_extras(which):
    import numpy as _np  # noqa: F401
    import torch
    import synth
    from paper_2112_10823_amd import cgx
    torch.cuda.set_device(0)
    meter = EnergyMeter()
    table = {"small": lambda: extra_small_cg(cgx, synth, meter),
             "blas1": lambda: extra_blas1_sweep(cgx, synth),
             "q1": lambda: extra_spmv_and_cg(cgx, synth, meter),
             "mixed": lambda: extra_mixed(cgx, synth, meter),
             "schwarz": lambda: extra_schwarz(cgx, synth, meter),
             "batched": lambda: extra_batched(cgx, synth, meter),
             "serving": lambda: extra_serving(cgx, synth, meter),
             "serving10k": lambda: extra_serving(cgx, synth, meter, n_req=10000, full=False),
             "paper": lambda: extra_paper_shapes(cgx, synth, meter),
             "transfer": lambda: extra_transfer(meter),
             "energy": lambda: extra_energy_phases(cgx, synth, meter)}
    for name in which:
        print(f"# extra {name}", file=sys.stderr, flush=True)
        res = table[name]()
        print(json.dumps({"extra": name, **res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision comparison on Q1 192^3 in the default line")
    ap.add_argument("--cpu-iters", type=int, default=300,
                    help="Jacobi-CG iterations of the CPU oracle sample (about 10-15 s)")
    ap.add_argument("--profile-only", action="store_true",
                    help="warm-up plus a few solves, for profiler runs")
    ap.add_argument("--extras", default="",
                    help="comma list of extra workloads (small,blas1,q1,mixed,batched,serving,paper,"
                         "transfer,energy); "
                         "prints one JSON line each instead of the benchmark line")
    ap.add_argument("--calib", action="store_true",
                    help="with --profile-only: first run cgx_add on 2^26 float64 elements "
                         "(reads 1 GiB, writes 0.5 GiB) to calibrate byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver is measured on one GPU only; the multi-GPU path is a design "
              "(independent systems per GPU, row-slab halo exchange for one big system) "
              "and is not run. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.extras:
        run_extras([w for w in args.extras.split(",") if w])
        return

    import numpy as np
    import torch

    import synth
    from paper_2112_10823_amd import cgx

    torch.cuda.set_device(0)
    if args.calib:
        m = 1 << 26
        xa = torch.rand(m, dtype=torch.float64, device="cuda")
        ya = torch.rand(m, dtype=torch.float64, device="cuda")
        za = torch.empty_like(xa)
        for _ in range(5):
            cgx.add(xa, ya, za)
        torch.cuda.synchronize()
        del xa, ya, za
        print("# calibration adds done (5 x 2^26 elements)", file=sys.stderr, flush=True)
        # a gathering kernel of known bytes: the CSR SpMV on a permutation
        # matrix of 2^25 rows that moves whole 128-byte blocks of x (16
        # float64) to random places, so every x line is fetched once, in full,
        # by a gather: reads 12 nnz + 4 (n + 1) + 8 n, writes 8 n bytes
        P = calib_gather_matrix(1 << 25)
        dP = cgx.DeviceCSR.from_host(P, validate=False)
        xg = torch.rand(P.n_rows, dtype=torch.float64, device="cuda")
        yg = torch.empty_like(xg)
        for _ in range(5):
            cgx.csr_spmv(dP, xg, yg)
        torch.cuda.synchronize()
        del dP, xg, yg
        print("# calibration gathers done (5 x 2^25-row block permutation)", file=sys.stderr,
              flush=True)
    print(f"# building Q1 {N_GRID}^3 lognormal({SIGMA}) system", file=sys.stderr, flush=True)
    A = synth.q1cube(N_GRID, SIGMA, seed=synth.SEED_C2_COEFF)
    b = synth.blob_rhs(N_GRID, synth.SEED_C2_BLOBS)
    n, nnz = A.n_rows, A.nnz
    dA = cgx.DeviceCSR.from_host(A)
    db = torch.from_numpy(b).cuda()
    dx = torch.zeros_like(db)
    opts = cgx.make_opts(rtol=RTOL, precond=cgx.PRECOND_JACOBI)
    ws = cgx.cg_workspace(dA, opts)
    handle = cgx.default_handle()

    def step():
        dx.zero_()
        st = cgx.cg_solve(dA, db, dx, opts, workspace=ws, handle=handle)
        if st.status != cgx.OK:
            raise RuntimeError(f"solve failed: {st.as_dict()}")
        return st

    for _ in range(args.warmup):
        step()
    print("# warm-up done", file=sys.stderr, flush=True)
    if args.profile_only:
        for _ in range(max(args.steps, 1)):
            step()
        torch.cuda.synchronize()
        print("# profile steps done", file=sys.stderr, flush=True)
        return

    meter = EnergyMeter()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, iters = [], []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        st = step()
        lat.append(time.perf_counter() - s0)
        iters.append(st.iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # Energy: the mean board power while the solve runs back to back, over a
    # window that opens one second into the timed region (the board takes
    # about a second to reach the workload's level) and, when the timed
    # region is shorter than that plus two seconds or holds fewer than three
    # updates of the (about 1 Hz) energy counter, continues over untimed
    # solves of the same kind after it.  The timed region is unchanged.
    jw0 = t0 + 1.0
    extra_solves = 0
    if meter.sampler.ok:
        while ((time.perf_counter() - jw0 < 2.0
                or meter.updates_between(jw0, time.perf_counter()) < 3)
               and time.perf_counter() - jw0 < 12.0):
            step()
            extra_solves += 1
        torch.cuda.synchronize()
    jw1 = time.perf_counter()
    p_avg = meter.power(jw0, jw1)
    energy_window = {"start_s_after_timed_start": 1.0, "length_s": round(jw1 - jw0, 3),
                     "counter_updates": meter.updates_between(jw0, jw1) if meter.sampler.ok else 0,
                     "untimed_solves_after_timed_region": extra_solves,
                     "mean_power_w": round(p_avg, 1) if p_avg is not None else None}
    wall = t1 - t0
    total_bytes = sum(jacobi_setup_bytes(n, nnz) + k * jacobi_iter_bytes(n, nnz) for k in iters)
    value = total_bytes / wall / 1e9
    print(f"# timed {args.steps} solves in {wall:.3f} s, iters {iters[0]}", file=sys.stderr,
          flush=True)

    # accuracy of the last solve, checked with the library's own residual (device)
    chk = cgx.cg_solve(dA, db, dx.zero_(), cgx.make_opts(rtol=RTOL, precond=1,
                                                          true_residual=True),
                       workspace=ws, handle=handle)

    # dominant kernel: the SpMV phase (q = A p fused with p.q), mean launch
    # duration from HIP events on the solver stream, profile solve
    prof = cgx.cg_solve(dA, db, dx.zero_(), cgx.make_opts(rtol=RTOL, precond=1, profile=True),
                        workspace=ws, handle=handle)
    spmv_ms = prof.phase_ms[0]
    sp_bytes = spmv_bytes(n, nnz)
    achieved = sp_bytes / (spmv_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    traffic = measured_traffic(khash)
    print(f"# phase ms {list(prof.phase_ms)}", file=sys.stderr, flush=True)

    # the same solves with the iteration's SpMV on a sliced-ELL copy of A
    # (cgx_cg_solve_sell), built once from the resident CSR; the setup and
    # residual passes still read the CSR
    torch.cuda.synchronize()
    tb = time.perf_counter()
    sell = cgx.SellMatrix(dA, handle=handle)
    build_ms = (time.perf_counter() - tb) * 1e3
    for _ in range(2):
        cgx.cg_solve(dA, db, dx.zero_(), opts, workspace=ws, handle=handle, sell=sell)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    k_sell = 10
    for _ in range(k_sell):
        st_s = cgx.cg_solve(dA, db, dx.zero_(), opts, workspace=ws, handle=handle, sell=sell)
    torch.cuda.synchronize()
    wall_s = (time.perf_counter() - ts) / k_sell
    prof_s = cgx.cg_solve(dA, db, dx.zero_(), cgx.make_opts(rtol=RTOL, precond=1, profile=True),
                          workspace=ws, handle=handle, sell=sell)
    sell_gbs = sp_bytes / (prof_s.phase_ms[0] * 1e-3) / 1e9
    sell_path = {"kernel": "cg_sell_spmv_kernel<double> (64-row column-major slices, one lane per row)",
                 "build_ms": round(build_ms, 2), "ms_per_step": round(wall_s * 1e3, 3),
                 "solves_per_s": round(1.0 / wall_s, 3), "iters": st_s.iters,
                 "value": round((jacobi_setup_bytes(n, nnz) + st_s.iters * jacobi_iter_bytes(n, nnz))
                                / wall_s / 1e9, 2),
                 "spmv_achieved": round(sell_gbs, 1), "spmv_frac": round(sell_gbs / HBM_PEAK_GBS, 4),
                 "spmv_mean_launch_ms": round(prof_s.phase_ms[0], 5),
                 "padding": round(sell.stored / nnz - 1, 5)}
    del sell
    print(f"# sliced-ELL path {sell_path['ms_per_step']} ms per solve", file=sys.stderr, flush=True)
    del ws
    mixed = None
    if not args.no_mixed:
        mixed = mixed_path(cgx, synth, meter, cpu=not args.no_cpu_baseline)
        print(f"# mixed path {mixed['mixed_ru_ms']} ms vs float64 {mixed['fp64_jacobi_ms']} ms",
              file=sys.stderr, flush=True)

    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        print("# CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(A, b, n, nnz, args.cpu_iters)
        print("# CPU oracle sample, all cores", file=sys.stderr, flush=True)
        cpu_all = cpu_baseline_all_cores(A, b, n, nnz, args.cpu_iters)

    joules = p_avg * wall / args.steps if p_avg is not None else None
    lat_ms = sorted(1e3 * v for v in lat)
    p99 = lat_ms[min(len(lat_ms) - 1, math.ceil(0.99 * len(lat_ms)) - 1)]
    out = {
        "metric": "SpMV/CG achieved HBM GB/s, solves/s + p99 latency, J/solve at 1e-8 resid",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Jacobi-CG, Q1 hex FEM 128^3 (2,097,152 rows, 55,742,968 nnz), "
                               "lognormal(0,1) element coefficients, Gaussian-blob RHS, "
                               "rtol 1e-8, x0 = 0",
                   "n_rows": n, "nnz": nnz, "rtol": RTOL, "precond": "jacobi"},
        "solves_per_s": round(args.steps / wall, 3),
        "p50_ms": round(statistics.median(lat_ms), 3),
        "p99_ms": round(p99, 3),
        "j_per_solve": round(joules, 4) if joules is not None else None,
        "energy_window": energy_window,
        "iters": iters[0],
        "relres_true": chk.relres_true,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": f"cg_spmv_kernel<{wave_tile_rows(n, nnz)}, double> "
                               "(q = A p, one 64-lane wave tile per workgroup, fused with the "
                               "tile's p.q partial)",
                     "algorithmic_bytes": sp_bytes, "mean_launch_ms": round(spmv_ms, 5),
                     "kernel_source_hash": khash},
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "sell_path": sell_path,
        "mixed_path": mixed,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
