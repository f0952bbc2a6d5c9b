// Device building blocks for gfx950: wave64 reductions, XCD-aware block
// numbering, the deterministic grid-wide sum and the vector-CSR row body.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cgx_internal.h"

namespace cgx {

constexpr int kWave = 64;
constexpr int kXcds = 8;  // MI355X: 8 accelerator dies, each with its own L2

// Workgroups are dispatched round-robin over the XCDs (block b runs on die
// b % 8).  Renumber so that each die works on one contiguous range of logical
// blocks: neighbouring rows then share a die's L2 for the x gathers.
__device__ __forceinline__ int xcd_block(int b, int grid)
{
    const int q = grid / kXcds, r = grid % kXcds;
    const int die = b % kXcds, t = b / kXcds;
    return die * q + (die < r ? die : r) + t;
}

// Butterfly sum over the 64 lanes: every lane ends with the same bits since
// each step adds the same two operands (a + b == b + a in IEEE arithmetic).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Butterfly sum inside aligned groups of L lanes.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum NV per-thread values over the block; the result is valid in thread 0.
// `red` is __shared__ scratch of NV * (BS / 64) doubles.
template <int NV, int BS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red)
{
    constexpr int W = BS / kWave;
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (l == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) red[j * W + w] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < W; ++i) s += red[j * W + i];
            v[j] = s;
        }
}

// Deterministic grid-wide sum of NV values per thread.  Every workgroup
// stores its NV block totals at partials[j * gridDim.x + blockIdx.x] and
// takes an arrival ticket; the last workgroup to arrive adds the partials in
// index order with a fixed tree, resets the ticket and returns true with the
// totals in thread 0's `v`.  Other workgroups return false.  The partial
// exchange uses device-scope atomic loads/stores so it does not depend on the
// per-die L2s being coherent.  Must be reached by all threads of the block.
template <int NV, int BS>
__device__ __forceinline__ bool grid_sum(double (&v)[NV], double *partials, uint32_t *ticket)
{
    __shared__ double red[NV * (BS / kWave)];
    __shared__ int is_last;
    const int G = gridDim.x;
    block_sum<NV, BS>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            __hip_atomic_store(&partials[(int64_t)j * G + blockIdx.x], v[j], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = (t == (uint32_t)G - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double s[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        s[j] = 0.0;
        for (int i = threadIdx.x; i < G; i += BS)
            s[j] += __hip_atomic_load(&partials[(int64_t)j * G + i], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();  // `red` is reused
    block_sum<NV, BS>(s, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = s[j];
        *ticket = 0u;
    }
    return true;
}

// Error-free transformations (Knuth two-sum; two-product via fma).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// ------------------------------------------------------- vector CSR rows --

// One workgroup of BS threads covers GPB = BS / L row-groups of L lanes;
// for a tile starting at row0, group g handles rows row0 + g + GPB * r,
// r < R, so that at each r the groups of a wave read one contiguous stretch
// of col_idx / val.  Lane k of a group takes entries start + k, + k + L, ...
// Every index read is clamped: row_ptr values to [0, nnz], columns to
// [0, n_cols) (out-of-range columns contribute nothing).  acc[r] ends with
// the row sum in every lane of the group; with kDiag, dg[r] gets the
// diagonal entry (0 if absent).
template <int L, int R, int BS, typename T, bool kDiag>
__device__ __forceinline__ void vector_rows(int row0, int n_rows, int n_cols, int64_t nnz,
                                            const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ ci,
                                            const T *__restrict__ val, const T *__restrict__ x,
                                            T (&acc)[R], T (&dg)[R], int (&rows)[R])
{
    constexpr int GPB = BS / L;
    const int lane = threadIdx.x % L;
    const int g = threadIdx.x / L;
    int k[R], e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = row0 + g + GPB * r;
        rows[r] = row;
        int s = 0, t = 0;
        if (row < n_rows) {
            s = rp[row];
            t = rp[row + 1];
            s = s < 0 ? 0 : (s > nnz ? (int)nnz : s);
            t = t < s ? s : (t > nnz ? (int)nnz : t);
        }
        k[r] = s + lane;
        e[r] = t;
        acc[r] = T(0);
        dg[r] = T(0);
    }
    bool more = true;
    while (more) {
        int c[R];
        T a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            c[r] = -1;
            a[r] = T(0);
            if (k[r] < e[r]) {
                c[r] = ci[k[r]];
                a[r] = val[k[r]];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if ((unsigned)c[r] < (unsigned)n_cols) {
                acc[r] += a[r] * x[c[r]];
                if (kDiag && c[r] == rows[r]) dg[r] = a[r];
            }
        }
        more = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            k[r] += L;
            more |= k[r] < e[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] = group_sum<L>(acc[r]);
        if (kDiag) dg[r] = group_sum<L>(dg[r]);
    }
}

}  // namespace cgx
