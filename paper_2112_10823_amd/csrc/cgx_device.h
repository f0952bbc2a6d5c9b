// Device building blocks for gfx950: wave64 reductions, XCD-aware block
// numbering, the vector-CSR, wave-tile and sliced-ELL row bodies and the
// fixed-order sum of per-workgroup partials.
//
// Grid-wide sums never use a per-workgroup device-scope fence (on this
// multi-die part such a release writes back the die's L2 and halved the
// bandwidth of the kernels that used it): each workgroup stores a plain
// partial, and the next kernel in stream order, for which the kernel
// boundary makes the partials visible, adds them in index order.
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
// `red` is __shared__ scratch of NV * (BS / 64) values of type T.
template <int NV, int BS, typename T>
__device__ __forceinline__ void block_sum(T (&v)[NV], T *red)
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
            T s = T(0);
#pragma unroll
            for (int i = 0; i < W; ++i) s += red[j * W + i];
            v[j] = s;
        }
}

// Error-free transformations (Knuth two-sum; two-product via fma).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// ---------------------------------------------------------- wave CSR rows --

// Wave-local barrier for LDS data exchanged between the lanes of one wave:
// orders the wave's LDS accesses around it (no workgroup barrier needed).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS staging of one wave tile: a chunk of 64 * E column indices and values
// and the tile's RT + 1 row starts.
template <int E, int RT, typename T>
struct WaveSmem {
    T val[kWave * E];
    int col[kWave * E];
    int rp[RT + 1];
};

// Wave tile: one wavefront computes RT consecutive rows starting at row0.
// Phase 1 reads the tile's col_idx / val as one contiguous stream (lane l
// takes entries c0 + l + 64 j, j < E, non-temporal: each entry is used once)
// and stages them in LDS.  Phase 2 gives each row TPR = 64 / RT lanes; lane
// `sub` walks entries sub, sub + TPR, ... of its row, U at a time, gathering
// x[col].  At each step the lanes of a wave hold the same entry position of
// 64 / TPR neighbouring rows, so for banded / stencil matrices their gathers
// fall on a few cache lines instead of one line per row.  The TPR lanes then
// combine by butterfly.  A tile with more than 64 * E entries is processed in
// several chunks.  Returns the row sum in all TPR lanes of the row's group;
// `row` receives the row index (>= n_rows for idle groups).  Every index
// read is clamped: row_ptr values to [0, nnz], columns to [0, n_cols)
// (out-of-range columns contribute nothing).  Must be reached by all 64
// lanes of the wave.
// With a non-null `stop`, *stop is read together with the row starts (its
// latency hidden behind theirs); if nonzero the tile is skipped: returns 0
// with row = -1 in every lane.
// kDiag: *xdiag receives x[row] in all TPR lanes of the row, taken from the
// gather of the row's diagonal entry (no load of its own), or loaded when
// the row stores no diagonal.
// kDiagA: *adiag receives the row's stored diagonal a_ii in all TPR lanes of
// the row (0 when the row stores none).
template <int E, int RT, int U, typename T, bool kDiag = false, bool kDiagA = false>
__device__ __forceinline__ T wave_rows(int row0, int n_rows, int n_cols, int64_t nnz,
                                       const int32_t *__restrict__ rp,
                                       const int32_t *__restrict__ ci,
                                       const T *__restrict__ val, const T *__restrict__ x,
                                       WaveSmem<E, RT, T> &sm, int &row,
                                       const int *stop = nullptr, T *xdiag = nullptr,
                                       T *adiag = nullptr)
{
    constexpr int TPR = kWave / RT;
    constexpr int C = kWave * E;
    static_assert(RT >= 1 && RT <= kWave && (RT & (RT - 1)) == 0, "rows per wave tile");
    const int halt = stop != nullptr ? *stop : 0;
    const int lane = threadIdx.x % kWave;
    const int nr = min(RT, n_rows - row0);
    wave_lds_sync();  // earlier readers of sm are done
    for (int i = lane; i <= nr; i += kWave) {
        int v = rp[row0 + i];
        v = v < 0 ? 0 : (v > nnz ? (int)nnz : v);
        sm.rp[i] = v;
    }
    if (halt) {
        row = -1;
        return T(0);
    }
    wave_lds_sync();
    const int k0 = sm.rp[0];
    const int k1 = max(k0, sm.rp[nr]);
    const int g = lane / TPR, sub = lane % TPR;
    row = row0 + g;
    int s = k0, e = k0;
    if (g < nr) {
        s = max(sm.rp[g], k0);
        e = min(max(sm.rp[g + 1], s), k1);
    }
    T acc = T(0), xd = T(0), ad = T(0);
    int seen = 0;
    for (int c0 = k0; c0 < k1; c0 += C) {
        int col[E];
        T a[E];
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int k = c0 + lane + kWave * j;
            col[j] = -1;
            a[j] = T(0);
            if (k < k1) {  // streamed once: non-temporal, keeps x resident in L2
                col[j] = __builtin_nontemporal_load(&ci[k]);
                a[j] = __builtin_nontemporal_load(&val[k]);
            }
        }
        wave_lds_sync();  // the previous chunk's readers are done
#pragma unroll
        for (int j = 0; j < E; ++j) {
            sm.col[lane + kWave * j] = col[j];
            sm.val[lane + kWave * j] = a[j];
        }
        wave_lds_sync();
        const int lo = max(s, c0) - c0, hi = min(e, c0 + C) - c0;
        for (int k = lo + sub; k < hi; k += U * TPR) {
            int cc[U];
            T vv[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k + u * TPR;
                cc[u] = -1;
                vv[u] = T(0);
                if (kk < hi) {
                    cc[u] = sm.col[kk];
                    vv[u] = sm.val[kk];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = (unsigned)cc[u] < (unsigned)n_cols ? x[cc[u]] : T(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                acc += vv[u] * xv[u];
                if (kDiag && cc[u] == row) {
                    xd = xv[u];
                    seen = 1;
                }
                if (kDiagA && cc[u] == row) ad = vv[u];
            }
        }
    }
    if (kDiagA) *adiag = group_sum<TPR>(ad);  // one lane of the row holds it, the others 0
    if (kDiag) {
        // one lane of the row holds the diagonal's value, the others 0
        xd = group_sum<TPR>(xd);
        seen = group_sum<TPR>(seen);
        if (!seen && (unsigned)row < (unsigned)min(n_rows, n_cols)) xd = x[row];
        *xdiag = xd;
    }
    return group_sum<TPR>(acc);
}

// -------------------------------------------------------- sliced ELL rows --

// One wavefront computes the 64 rows of sliced-ELL slice s: lane l owns row
// 64 s + l and walks its entries k = 0 .. width - 1 at sp[s] + 64 k + l, U
// at a time (U col / val loads, then U gathers in flight); columns outside
// [0, n_cols) (the padding's -1) contribute nothing.  Returns the row sum in
// lane l; `row` receives the row index (>= n_rows past the last row).  The
// entries of a row are added in storage order.
// With a non-null `stop`, *stop is read together with the slice bounds; if
// nonzero the slice is skipped: returns 0 with row = -1 in every lane.
// kDiag: *xdiag receives x[row], taken from the gather of the row's diagonal
// entry, or loaded when the row stores no diagonal.
template <int U, typename T, bool kDiag = false>
__device__ __forceinline__ T sell_rows(int s, int n_rows, int n_cols,
                                       const int64_t *__restrict__ sp,
                                       const int32_t *__restrict__ col,
                                       const T *__restrict__ val, const T *__restrict__ x,
                                       int &row, const int *stop = nullptr, T *xdiag = nullptr)
{
    const int halt = stop != nullptr ? *stop : 0;
    const int lane = threadIdx.x % kWave;
    row = s * kWave + lane;
    const int64_t b = sp[s];
    const int w = (int)((sp[s + 1] - b) / kWave);
    if (halt) {
        row = -1;
        return T(0);
    }
    const int32_t *c = col + b + lane;
    const T *v = val + b + lane;
    T acc = T(0), xd = T(0);
    bool seen = false;
    int k = 0;
    for (; k + U <= w; k += U) {
        int cc[U];
        T vv[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {  // streamed once: non-temporal, keeps x resident in L2
            cc[u] = __builtin_nontemporal_load(c + (int64_t)(k + u) * kWave);
            vv[u] = __builtin_nontemporal_load(v + (int64_t)(k + u) * kWave);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = (unsigned)cc[u] < (unsigned)n_cols ? x[cc[u]] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc += vv[u] * xv[u];
            if (kDiag && cc[u] == row) {
                xd = xv[u];
                seen = true;
            }
        }
    }
    // the remainder with ordinary loads: measured faster than non-temporal
    // ones here, and than predicating a last batch of U
    for (; k < w; ++k) {
        const int cc = c[(int64_t)k * kWave];
        if ((unsigned)cc < (unsigned)n_cols) {
            const T xv = x[cc];
            acc += v[(int64_t)k * kWave] * xv;
            if (kDiag && cc == row) {
                xd = xv;
                seen = true;
            }
        }
    }
    if (kDiag) {
        if (!seen && (unsigned)row < (unsigned)min(n_rows, n_cols)) xd = x[row];
        *xdiag = xd;
    }
    return acc;
}

// Per-thread part of a sum of partials: thread t adds partials t, t + BS,
// t + 2 BS, ... in that order, two loads in flight at a time, for NA arrays
// of `count` partials each at once (their loads in flight together).
template <int BS, int NA, typename T>
__device__ __forceinline__ void thread_partials(const T *const (&pa)[NA], int count, T (&s)[NA])
{
#pragma unroll
    for (int k = 0; k < NA; ++k) s[k] = T(0);
    int i = threadIdx.x;
    for (; i + BS < count; i += 2 * BS) {
        T v0[NA], v1[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            v0[k] = pa[k][i];
            v1[k] = pa[k][i + BS];
        }
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            s[k] += v0[k];
            s[k] += v1[k];
        }
    }
    if (i < count)
#pragma unroll
        for (int k = 0; k < NA; ++k) s[k] += pa[k][i];
}

// The block's total of the threads' values s: a wave sum, then the waves'
// sums in wave order; every thread receives the same bits.  `red` is
// __shared__ scratch of BS / 64 values.
template <int BS, typename T>
__device__ __forceinline__ T block_total(T s, T *red)
{
    s = wave_sum(s);
    constexpr int W = BS / kWave;
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x % kWave == 0) red[w] = s;
    __syncthreads();
    T t = T(0);
#pragma unroll
    for (int i = 0; i < W; ++i) t += red[i];
    return t;
}

// Sum of `count` partials in index order (strided per thread, then a fixed
// block tree); every thread of the block receives the same bits.  `red` is
// __shared__ scratch of BS / 64 values.
template <int BS, typename T>
__device__ __forceinline__ T sum_partials(const T *partials, int count, T *red)
{
    const T *const pa[1] = {partials};
    T s[1];
    thread_partials<BS>(pa, count, s);
    return block_total<BS>(s[0], red);
}

}  // namespace cgx
