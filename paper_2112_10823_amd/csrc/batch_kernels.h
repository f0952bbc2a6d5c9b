// Device side of the batched solver (shared by the batch call and the
// solve server): system descriptors, work-table entries and the phase kernels.
#pragma once

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <type_traits>
#include <vector>

#include "cgx_device.h"

namespace cgx {

// Caller vectors of one right-hand side of a served group.
struct LanePtr {
    const double *b;
    double *x;
};

// T: the type of the values, vectors and sums (double, or float for the
// inner solves of the float32-refined batch).
template <typename T>
struct BSysT {
    const int32_t *rp;
    const int32_t *ci;
    const T *val;
    const T *B;  // caller right-hand sides, [nrhs][n] (batch call)
    T *X;        // caller solutions, [nrhs][n] (batch call)
    const LanePtr *lanes;  // served groups: per right-hand side b / x (else null)
    T *x, *r, *p, *q, *z;  // interleaved [n][K]
    T *dinv;     // [n]
    int64_t nnz;
    int n, K, nrhs, M;
    int tile0, ntiles, trows, scal0;
    int n_cols, jac;     // jac: Jacobi preconditioning for this system
    int maxit;
    int staged;          // SpMM wave tiles for K >= 8 staged per wave (batch call; see below)
    int ru;              // binary32 system of a reliable-update batch: the stopping test of
                         // R2 becomes the update test (rtol2 = delta^2, see batch_r2_kernel)
    double rtol2;        // squared relative tolerance of this system
};
using BSys = BSysT<double>;

struct BTile {
    int sys, row0, rows, tile;  // tile = index within the whole table
};

template <typename T>
struct BScalT {
    T rho, rho_used, alpha, beta, rr, bb, stop2, pq;
    int32_t iter, status, active, pad;  // pad: a diagonal entry <= 0 met at setup
    int32_t xstep;                      // x += alpha p due in this iteration's p update
    int32_t ru;                         // reliable update due after this iteration's p update
};
using BScal = BScalT<double>;

template <typename T>
struct BArgsT {
    const BSysT<T> *sys;
    const BTile *tiles;     // tiles this launch covers (one workgroup each)
    const int32_t *list;    // systems the per-system kernels cover (one workgroup each)
    BScalT<T> *scal;
    int32_t *sys_done;      // per system: 0 running; 2 all right-hand sides finished, the
                            // last x steps pending in this iteration's p update; 1 done;
                            // 3 (reliable-update batch) updates due after the p update
    T *part;                // 3 regions of part_stride values
    int64_t part_stride;    // (tiles of the whole table) * 16
    int ntiles;
    int nlist;
    int wave_lds;           // dynamic LDS bytes of the SpMM launch (wave-tile staging or 0)
};
using BArgs = BArgsT<double>;

namespace bk {
namespace {  // internal linkage: each translation unit keeps its own copy

constexpr int kBB = 256;  // threads per workgroup of the batched kernels
constexpr int kMaxK = 16;

// Sixteen bytes of an interleaved vector: V = 16 / sizeof(T) consecutive
// right-hand sides of one row.
template <typename T>
using Vec16 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;

__device__ __forceinline__ int clampk(int v, int64_t nnz)
{
    return v < 0 ? 0 : (v > nnz ? (int)nnz : v);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Per-RHS block sum: thread t holds a value for right-hand side t % K; the
// K totals (fixed order) are written to out[0..K) by threads 0..K-1.
template <typename T>
__device__ __forceinline__ void block_sum_by_rhs(T v, int K, T *red, T *out)
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < K) {
        T s = T(0);
        for (int i = threadIdx.x; i < kBB; i += K) s += red[i];
        out[threadIdx.x] = s;
    }
}

// Slices per row of the setup pass: the tuned M, or for systems whose SpMM
// runs on wave tiles (M < 0) M = max(1, 8 / K): groups of K * M <= 64 lanes
// (K <= 16), so every wave holds at least one row group.
template <typename T>
__device__ __forceinline__ int setup_m(const BSysT<T> &S) { return S.M > 0 ? S.M : max(1, 8 / S.K); }

// Row sum of one row for right-hand side j over nonzero slice m of M, using
// interleaved vector v ([n][K]); combined over the M slices by butterfly.
// Also returns the diagonal entry (summed the same way; one slice holds it).
// The nonzero loop is unrolled four ways (four col/val loads, then four
// gathers in flight per lane); the accumulation order is k, k + M, ... in
// both the unrolled and the remainder part.
template <typename T>
__device__ __forceinline__ T row_spmm(const BSysT<T> &S, int row, int j, int m, int M, T &diag,
                                      const T *v)
{
    int s = S.rp[row], e = S.rp[row + 1];
    s = clampk(s, S.nnz);
    e = clampk(e, S.nnz);
    if (e < s) e = s;
    const int K = S.K;
    T acc = T(0), dg = T(0);
    int k = s + m;
    for (; k + 3 * M < e; k += 4 * M) {
        int c[4];
        T a[4], pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = S.ci[k + u * M];
            a[u] = S.val[k + u * M];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            pv[u] = (unsigned)c[u] < (unsigned)S.n_cols ? v[(int64_t)c[u] * K + j] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if ((unsigned)c[u] < (unsigned)S.n_cols) acc += a[u] * pv[u];
            if (c[u] == row) dg = a[u];
        }
    }
    for (; k < e; k += M) {
        const int c = S.ci[k];
        const T a = S.val[k];
        if ((unsigned)c < (unsigned)S.n_cols) acc += a * v[(int64_t)c * K + j];
        if (c == row) dg = a;
    }
    const int G = K * M;
    for (int off = K; off < G; off <<= 1) {
        acc += __shfl_xor(acc, off);
        dg += __shfl_xor(dg, off);
    }
    diag = dg;
    return acc;
}

// Caller layout -> interleaved x.
template <typename T>
__global__ __launch_bounds__(kBB) void batch_in_kernel(BArgsT<T> a)
{
    const BTile t = a.tiles[blockIdx.x];
    const BSysT<T> S = a.sys[t.sys];
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        T v = T(0);
        if (j < S.nrhs) {
            if (!S.lanes)
                v = S.X[(int64_t)j * S.n + row];
            else if (S.lanes[j].x)  // a free lane of a served slot holds zeros
                v = S.lanes[j].x[row];
        }
        S.x[e] = v;
    }
}

// Block sum of one value per thread in a fixed order (wave butterflies, then
// the waves in order); the result is valid in thread 0.  `red` holds
// kBB / 64 values.
__device__ __forceinline__ double sum_partials_in_block(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBB / kWave; ++w) t += red[w];
    return t;
}

// Sum of region `reg` partials of system s for right-hand side j (fixed
// order: tile-strided per thread slice, then slices in order).
template <typename T>
__device__ __forceinline__ T sys_sum(const BArgsT<T> &a, const BSysT<T> &S, int reg, T *red)
{
    const int K = S.K;
    const int slice = threadIdx.x / K, j = threadIdx.x % K, nsl = kBB / K;
    T s = T(0);
    const T *base = a.part + reg * a.part_stride;
    // unrolled: eight loads in flight, still added one by one in tile order
#pragma unroll 8
    for (int t = S.tile0 + slice; t < S.tile0 + S.ntiles; t += nsl) s += base[(int64_t)t * kMaxK + j];
    __syncthreads();
    red[threadIdx.x] = s;
    __syncthreads();
    T tot = T(0);
    if ((int)threadIdx.x < K)
        for (int i = 0; i < nsl; ++i) tot += red[i * K + threadIdx.x];
    return tot;  // valid in threads 0..K-1
}

template <typename T>
__global__ __launch_bounds__(kBB) void batch_r0_kernel(BArgsT<T> a)
{
    __shared__ T red[kBB];
    const int sid = a.list[blockIdx.x];
    const BSysT<T> S = a.sys[sid];
    const T rr = sys_sum(a, S, 0, red);
    const T rz = sys_sum(a, S, 1, red);
    const T bb = sys_sum(a, S, 2, red);
    __shared__ int any_active;
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    if ((int)threadIdx.x < S.K) {
        const int j = threadIdx.x;
        BScalT<T> &c = a.scal[S.scal0 + j];
        const bool badd = c.pad != 0;
        c.rr = rr;
        c.bb = bb;
        c.rho = S.jac ? rz : rr;
        c.stop2 = (T)S.rtol2 * bb;
        c.iter = 0;
        int status = CGX_PENDING;
        if (j >= S.nrhs)
            status = CGX_OK;
        else if (badd)
            status = CGX_BREAKDOWN;
        else if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz))
            status = CGX_NONFINITE;
        else if (bb == T(0) || rr <= c.stop2)
            status = CGX_OK;
        else if (S.jac && !(rz > T(0)))
            status = CGX_BREAKDOWN;
        c.status = status;
        c.active = status == CGX_PENDING;
        if (c.active) atomicOr(&any_active, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.sys_done[sid] = any_active ? 0 : 1;
}

// Wave tiles for K right-hand sides: a wavefront computes RT consecutive rows
// at a time and gives each row K * T lanes (T = 64 / (RT K)), lane = g K T +
// t K + j for row g, right-hand side j and entry slice t.  Every lane walks
// its row's entries t, t + T, ... four at a time from LDS, gathering
// p[col][j] from the interleaved vector; the T slices are then combined by
// butterfly.  For K = 1 this is the single-system wave tile.  Staged (kStaged
// and K >= 8): the four waves of the workgroup take contiguous quarters of
// the work tile, and a wave reads the row starts of up to 64 of its rows at
// once and streams the col_idx / val of as many whole groups of RT rows as
// fit one 64 x 8 chunk into LDS (coalesced, non-temporal), then computes them
// group by group with eight gathers in flight, so that the dependent loads
// (row starts, then entries, then gathers) are paid once per chunk, not once
// per RT rows (RT is at most 4 there).  Otherwise the waves take groups of RT
// rows in turn, one group per chunk, four gathers in flight, so that
// neighbouring groups run at the same time and share their gathers in the
// cache.  The batch call stages (faster on its systems of up to 96^3 rows);
// the solve server does not (faster on its larger systems, whose neighbouring
// planes are further apart).  A group of RT rows longer than a chunk is
// streamed chunk by chunk.  The staging is dynamic LDS, requested
// only by launches that contain such a system, so that the vector-CSR
// schedules keep their occupancy.
constexpr int kWaveStageBytes = (kBB / kWave) * (kWave * 8 * 12 + 65 * 4 + 8);

// src: the interleaved vector multiplied (p in the SpMM phase); fin(row, j,
// sum, part, diag) consumes the sum of a (row, right-hand side) in the lane
// that holds it, part being the lane's running partial (returned at the
// end); with kDiag, diag is the row's stored diagonal (0 if it stores none),
// otherwise 0.
template <int RT, int K, typename T, bool kStaged, bool kDiag, typename Fin>
__device__ __forceinline__ T spmm_wave_tiles(const BSysT<T> &S, const BTile &t, double *lds,
                                             const T *__restrict__ src, Fin fin)
{
    using Sm = WaveSmem<8, kWave, T>;  // row starts of up to 64 rows
    static_assert((kBB / kWave) * sizeof(Sm) <= kWaveStageBytes, "wave staging");
    constexpr int TL = kWave / (RT * K);
    static_assert(TL >= 1 && RT * K * TL == kWave, "lanes per row");
    constexpr bool kContig = kStaged && K >= 8;
    constexpr int C = kWave * 8, U = kContig ? 8 : 4, NW = kBB / kWave;
    Sm &sm = reinterpret_cast<Sm *>(lds)[threadIdx.x / kWave];
    const int lane = threadIdx.x % kWave;
    const int g = lane / (K * TL), sl = (lane / K) % TL, j = lane % K;
    const int w = threadIdx.x / kWave;
    const int per = ((t.rows + NW - 1) / NW + RT - 1) / RT * RT;  // rows per wave (kContig)
    const int wr0 = kContig ? t.row0 + w * per : t.row0 + w * RT;
    const int wend = kContig ? min(t.row0 + t.rows, wr0 + per) : t.row0 + t.rows;
    const T *__restrict__ p = src;
    T ppq = T(0);

    // rows [row0 + r_lo, row0 + r_hi) of the staged range (entries [k0, k1)
    // of the current chunk c0) for this lane's (row, right-hand side, slice)
    auto walk = [&](int s, int e, int c0, T &acc, int row, T &dg) {
        const int lo = s - c0, hi = e - c0;
        for (int k = lo + sl; k < hi; k += U * TL) {
            int cc[U];
            T vv[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k + u * TL;
                cc[u] = -1;
                vv[u] = T(0);
                if (kk < hi) {
                    cc[u] = sm.col[kk];
                    vv[u] = sm.val[kk];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                xv[u] = (unsigned)cc[u] < (unsigned)S.n_cols ? p[(int64_t)cc[u] * K + j] : T(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                acc += vv[u] * xv[u];
                if (kDiag && cc[u] == row) dg = vv[u];
            }
        }
    };
    auto stage = [&](int c0, int k1) {
        int col[8];
        T a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = c0 + lane + kWave * u;
            col[u] = -1;
            a[u] = T(0);
            if (k < k1) {
                col[u] = __builtin_nontemporal_load(&S.ci[k]);
                a[u] = __builtin_nontemporal_load(&S.val[k]);
            }
        }
        wave_lds_sync();  // earlier readers of the chunk are done
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sm.col[lane + kWave * u] = col[u];
            sm.val[lane + kWave * u] = a[u];
        }
        wave_lds_sync();
    };
    auto finish = [&](int row, bool valid, T acc, T dg) {
#pragma unroll
        for (int off = TL / 2; off > 0; off >>= 1) {
            acc += __shfl_xor(acc, off * K);
            if (kDiag) dg += __shfl_xor(dg, off * K);  // one slice holds it, the others 0
        }
        if (sl == 0 && valid) fin(row, j, acc, ppq, dg);
    };

    for (int r0 = wr0; r0 < wend;) {
        const int na = min(kContig ? kWave : RT, wend - r0);
        wave_lds_sync();  // the previous range's readers of sm are done
        for (int i = lane; i <= na; i += kWave) sm.rp[i] = clampk(S.rp[r0 + i], S.nnz);
        wave_lds_sync();
        const int k0 = sm.rp[0];
        // rows to stage: the most (whole groups of RT, or all na) whose
        // entries fit one chunk; 0 if even the first group does not
        int rs = 0;
        {
            const int l = lane + 1;
            if (l <= na && (l % RT == 0 || l == na) && sm.rp[l] - k0 <= C) rs = l;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) rs = max(rs, __shfl_xor(rs, off));
        }
        if (rs > 0) {
            const int k1 = max(k0, sm.rp[rs]);
            stage(k0, k1);
            for (int g0 = 0; g0 < rs; g0 += RT) {
                const int gr = g0 + g;
                int s = k0, e = k0;
                if (gr < rs) {
                    s = max(sm.rp[gr], k0);
                    e = min(max(sm.rp[gr + 1], s), k1);
                }
                T acc = T(0), dg = T(0);
                walk(s, e, k0, acc, r0 + gr, dg);
                finish(r0 + gr, gr < rs, acc, dg);
            }
            r0 += kContig ? rs : NW * RT;
        } else {  // one group of RT rows longer than a chunk
            const int nr = min(RT, na);
            const int k1 = max(k0, sm.rp[nr]);
            int s = k0, e = k0;
            if (g < nr) {
                s = max(sm.rp[g], k0);
                e = min(max(sm.rp[g + 1], s), k1);
            }
            T acc = T(0), dg = T(0);
            for (int c0 = k0; c0 < k1; c0 += C) {
                stage(c0, k1);
                walk(max(s, c0), min(e, c0 + C), c0, acc, r0 + g, dg);
            }
            finish(r0 + g, g < nr, acc, dg);
            r0 += kContig ? nr : NW * RT;
        }
    }
    return ppq;
}

// Staged wave tiles with vector gathers (batch call, K >= 8): as the staged
// form of spmm_wave_tiles, but every lane serves V = 16 / sizeof(T)
// consecutive right-hand sides with one 16-byte gather per entry, so a wave
// covers V times the rows per pass (RT V) and keeps twice (float64) or four
// times (binary32) the bytes in flight per instruction.  Each (row, right-
// hand side) still sums its entries in the same order.  The p.q partials
// come back per lane and right-hand side: pp[v] for right-hand side
// (lane % (K / V)) V + v.
// src, kDiag and finv as for spmm_wave_tiles: finv(row, j0, sums, pp, diag)
// takes the V sums of right-hand sides j0 .. j0 + V - 1 of a row.
template <int RT, int K, typename T, bool kDiag, typename FinV>
__device__ __forceinline__ void spmm_wave_tiles_vec(const BSysT<T> &S, const BTile &t,
                                                    double *lds, T (&pp)[16 / sizeof(T)],
                                                    const T *__restrict__ src, FinV finv)
{
    constexpr int V = 16 / (int)sizeof(T), KV = K / V;
    using Sm = WaveSmem<8, kWave, T>;
    static_assert((kBB / kWave) * sizeof(Sm) <= kWaveStageBytes, "wave staging");
    constexpr int TL = kWave / (RT * K);  // entry slices per (row, right-hand side)
    constexpr int RTV = RT * V;           // rows per pass
    static_assert(TL >= 1 && RTV * KV * TL == kWave, "lanes per row");
    constexpr int C = kWave * 8, U = 8, NW = kBB / kWave;
    using VT = Vec16<T>;
    Sm &sm = reinterpret_cast<Sm *>(lds)[threadIdx.x / kWave];
    const int lane = threadIdx.x % kWave;
    const int g = lane / (KV * TL), sl = (lane / KV) % TL, j0 = (lane % KV) * V;
    const int per = ((t.rows + NW - 1) / NW + RTV - 1) / RTV * RTV;  // rows per wave
    const int wr0 = t.row0 + (threadIdx.x / kWave) * per;
    const int wend = min(t.row0 + t.rows, wr0 + per);
    const T *__restrict__ p = src;
#pragma unroll
    for (int v = 0; v < V; ++v) pp[v] = T(0);

    auto walk = [&](int s, int e, int c0, T (&acc)[V], int row, T &dg) {
        const int lo = s - c0, hi = e - c0;
        for (int k = lo + sl; k < hi; k += U * TL) {
            int cc[U];
            T vv[U];
            VT xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k + u * TL;
                cc[u] = -1;
                vv[u] = T(0);
                if (kk < hi) {
                    cc[u] = sm.col[kk];
                    vv[u] = sm.val[kk];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xv[u] = VT{};
                if ((unsigned)cc[u] < (unsigned)S.n_cols)
                    xv[u] = *reinterpret_cast<const VT *>(p + (int64_t)cc[u] * K + j0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T xs[V];
                __builtin_memcpy(xs, &xv[u], sizeof(VT));
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += vv[u] * xs[v];
                if (kDiag && cc[u] == row) dg = vv[u];
            }
        }
    };
    auto stage = [&](int c0, int k1) {
        int col[8];
        T a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = c0 + lane + kWave * u;
            col[u] = -1;
            a[u] = T(0);
            if (k < k1) {
                col[u] = __builtin_nontemporal_load(&S.ci[k]);
                a[u] = __builtin_nontemporal_load(&S.val[k]);
            }
        }
        wave_lds_sync();  // earlier readers of the chunk are done
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sm.col[lane + kWave * u] = col[u];
            sm.val[lane + kWave * u] = a[u];
        }
        wave_lds_sync();
    };
    auto finish = [&](int row, bool valid, T (&acc)[V], T dg) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int off = TL / 2; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off * KV);
        if (kDiag)
#pragma unroll
            for (int off = TL / 2; off > 0; off >>= 1) dg += __shfl_xor(dg, off * KV);
        if (sl == 0 && valid) finv(row, j0, acc, pp, dg);
    };

    for (int r0 = wr0; r0 < wend;) {
        const int na = min(kWave, wend - r0);
        wave_lds_sync();  // the previous range's readers of sm are done
        for (int i = lane; i <= na; i += kWave) sm.rp[i] = clampk(S.rp[r0 + i], S.nnz);
        wave_lds_sync();
        const int k0 = sm.rp[0];
        int rs = 0;
        {
            const int l = lane + 1;
            if (l <= na && (l % RTV == 0 || l == na) && sm.rp[l] - k0 <= C) rs = l;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) rs = max(rs, __shfl_xor(rs, off));
        }
        if (rs > 0) {
            const int k1 = max(k0, sm.rp[rs]);
            stage(k0, k1);
            for (int g0 = 0; g0 < rs; g0 += RTV) {
                const int gr = g0 + g;
                int s = k0, e = k0;
                if (gr < rs) {
                    s = max(sm.rp[gr], k0);
                    e = min(max(sm.rp[gr + 1], s), k1);
                }
                T acc[V], dg = T(0);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = T(0);
                walk(s, e, k0, acc, r0 + gr, dg);
                finish(r0 + gr, gr < rs, acc, dg);
            }
            r0 += rs;
        } else {  // one group of RTV rows longer than a chunk
            const int nr = min(RTV, na);
            const int k1 = max(k0, sm.rp[nr]);
            int s = k0, e = k0;
            if (g < nr) {
                s = max(sm.rp[g], k0);
                e = min(max(sm.rp[g + 1], s), k1);
            }
            T acc[V], dg = T(0);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = T(0);
            for (int c0 = k0; c0 < k1; c0 += C) {
                stage(c0, k1);
                walk(max(s, c0), min(e, c0 + C), c0, acc, r0 + g, dg);
            }
            finish(r0 + g, g < nr, acc, dg);
            r0 += nr;
        }
    }
}

// Wave-tile schedule (M < 0: RT = -M rows per wave tile) for K = S.K.
// Returns the number of p.q values in pp: 1 (pp[0], right-hand side
// threadIdx.x % K) or V = 16 / sizeof(T) (the vector-gather form, see
// spmm_wave_tiles_vec).  kDiag: the epilogues receive the row's stored
// diagonal.
template <typename T, bool kDiag = false, typename Fin, typename FinV>
__device__ __forceinline__ int spmm_wave_dispatch(const BSysT<T> &S, const BTile &t, double *lds,
                                                  T (&pp)[16 / sizeof(T)], const T *src, Fin fin,
                                                  FinV finv)
{
    const int rt = -S.M;
#define CGX_WT(R, KK)                                                                 \
    if (rt == R && S.K == KK) {                                                       \
        pp[0] = S.staged ? spmm_wave_tiles<R, KK, T, true, kDiag>(S, t, lds, src, fin)   \
                         : spmm_wave_tiles<R, KK, T, false, kDiag>(S, t, lds, src, fin); \
        return 1;                                                                     \
    }
#define CGX_WV(R, KK)                                                                 \
    if (rt == R && S.K == KK) {                                                       \
        if (S.staged) {                                                               \
            spmm_wave_tiles_vec<R, KK, T, kDiag>(S, t, lds, pp, src, finv);           \
            return 16 / (int)sizeof(T);                                               \
        }                                                                             \
        pp[0] = spmm_wave_tiles<R, KK, T, false, kDiag>(S, t, lds, src, fin);         \
        return 1;                                                                     \
    }
    CGX_WT(1, 1) CGX_WT(2, 1) CGX_WT(4, 1) CGX_WT(8, 1) CGX_WT(16, 1) CGX_WT(32, 1) CGX_WT(64, 1)
    CGX_WT(8, 2) CGX_WT(16, 2) CGX_WT(32, 2)
    CGX_WT(4, 4) CGX_WT(8, 4) CGX_WT(16, 4)
    CGX_WV(2, 8) CGX_WV(4, 8) CGX_WV(8, 8)
    CGX_WV(1, 16) CGX_WV(2, 16) CGX_WV(4, 16)
#undef CGX_WT
#undef CGX_WV
    pp[0] = T(0);  // not reached: schedules are validated on the host
    return 1;
}

// Per-right-hand-side sums of the wave-tile partials pp (nv values per
// thread, see spmm_wave_dispatch) into out[0..K).  With nv = V, thread t's
// value v belongs to right-hand side (t V + v) mod K: the staging LDS (free
// by then) holds them in that order, and each right-hand side's values are
// added in index order.
template <typename T>
__device__ __forceinline__ void wave_partials_out(const T (&pp)[16 / sizeof(T)], int nv, int K,
                                                  double *stage, T *red, T *out)
{
    constexpr int V = 16 / (int)sizeof(T);
    if (nv == 1) {
        block_sum_by_rhs(pp[0], K, red, out);
        return;
    }
    __syncthreads();
    T *vred = reinterpret_cast<T *>(stage);
#pragma unroll
    for (int v = 0; v < V; ++v) vred[threadIdx.x * V + v] = pp[v];
    __syncthreads();
    if ((int)threadIdx.x < K) {
        T sum = T(0);
        for (int i = threadIdx.x; i < kBB * V; i += K) sum += vred[i];
        out[threadIdx.x] = sum;
    }
}

// r0 = b - A x0, D^-1, z0, p0 and the partials of r.r, r.z, b.b.  D^-1 is
// 1 / a_ii rounded once to T from a float64 division.  On the SpMM's wave
// tiles (the stored diagonal read on the way) for systems of the batch call
// on that schedule when the launch carries the staging LDS (a.wave_lds);
// otherwise, and in the solve server, a vector-CSR pass.
template <typename T>
__global__ __launch_bounds__(kBB) void batch_init_kernel(BArgsT<T> a)
{
    __shared__ T red[kBB];
    extern __shared__ double stage[];  // a.wave_lds bytes
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    const BSysT<T> S = a.sys[t.sys];
    // the row's residual, preconditioned residual, direction and partials
    auto init_row = [&](int row, int j, T ax, T dg, T &prr, T &prz, T &pbb) {
        const int64_t e = (int64_t)row * S.K + j;
        T bi = T(0);
        if (j < S.nrhs) {
            if (!S.lanes)
                bi = S.B[(int64_t)j * S.n + row];
            else if (S.lanes[j].b)
                bi = S.lanes[j].b[row];
        }
        const T ri = bi - ax;
        T zi = ri;
        S.r[e] = ri;
        if (S.jac) {
            const T d = dg > T(0) ? dg : T(1);
            if (!(dg > T(0))) a.scal[S.scal0 + j].pad = 1;  // same value from every writer
            const T di = (T)(1.0 / (double)d);
            if (j == 0) S.dinv[row] = di;
            zi = di * ri;
            S.z[e] = zi;
        }
        S.p[e] = zi;
        prr += ri * ri;
        prz += ri * zi;
        pbb += bi * bi;
    };
    T *base = a.part + (int64_t)t.tile * kMaxK;
    if (S.M < 0 && S.staged && a.wave_lds >= kWaveStageBytes) {
        // on the SpMM's wave tiles, the stored diagonal read on the way
        constexpr int V = 16 / (int)sizeof(T);
        T prr[V], prz[V], pbb[V], pp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) prr[v] = prz[v] = pbb[v] = T(0);
        auto fin = [&](int row, int j, T acc, T &, T dg) {
            init_row(row, j, acc, dg, prr[0], prz[0], pbb[0]);
        };
        auto finv = [&](int row, int j0, T (&acc)[V], T (&)[V], T dg) {
#pragma unroll
            for (int v = 0; v < V; ++v) init_row(row, j0 + v, acc[v], dg, prr[v], prz[v], pbb[v]);
        };
        const int nv = spmm_wave_dispatch<T, true>(S, t, stage, pp, (const T *)S.x, fin, finv);
        wave_partials_out(prr, nv, S.K, stage, red, base);
        wave_partials_out(prz, nv, S.K, stage, red, base + a.part_stride);
        wave_partials_out(pbb, nv, S.K, stage, red, base + 2 * a.part_stride);
        return;
    }
    const int M = setup_m(S);
    const int G = S.K * M, gpw = kWave / G;
    if (gpw < 1) return;  // not reached: K * M <= 64 is validated on the host
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
    T prr = T(0), prz = T(0), pbb = T(0);
    for (int row = t.row0 + wave * gpw + grp; row < t.row0 + t.rows; row += (kBB / kWave) * gpw) {
        T dg;
        const T ax = row_spmm(S, row, j, m, M, dg, S.x);
        if (m == 0) init_row(row, j, ax, dg, prr, prz, pbb);
    }
    // lanes with m > 0 hold zeros; the lane of (grp, j, m = 0) is lane % K == j
    block_sum_by_rhs(prr, S.K, red, base);
    block_sum_by_rhs(prz, S.K, red, base + a.part_stride);
    block_sum_by_rhs(pbb, S.K, red, base + 2 * a.part_stride);
}

// (1) q = A p for every active system, p.q partials per right-hand side.
// Systems with M > 0 use K * M lanes per row (vector CSR over the
// interleaved vectors), systems with M < 0 wave tiles of -M rows.
template <typename T>
__global__ __launch_bounds__(kBB) void batch_spmm_kernel(BArgsT<T> a)
{
    __shared__ T red[kBB];
    extern __shared__ double stage[];  // kWaveStageBytes when a system runs on wave tiles
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys]) return;
    const BSysT<T> S = a.sys[t.sys];
    T ppq = T(0);
    if (S.M < 0) {
        constexpr int V = 16 / (int)sizeof(T);
        T pp[V];
        // q = A p and the p.q partials
        auto fin = [&](int row, int j, T acc, T &part, T) {
            const int64_t ei = (int64_t)row * S.K + j;
            S.q[ei] = acc;
            part += S.p[ei] * acc;
        };
        auto finv = [&](int row, int j0, T (&acc)[V], T (&part)[V], T) {
            using VT = Vec16<T>;
            const int64_t ei = (int64_t)row * S.K + j0;
            VT qv;
            __builtin_memcpy(&qv, acc, sizeof(VT));
            *reinterpret_cast<VT *>(S.q + ei) = qv;
            const VT pvv = *reinterpret_cast<const VT *>(S.p + ei);
            T ps[V];
            __builtin_memcpy(ps, &pvv, sizeof(VT));
#pragma unroll
            for (int v = 0; v < V; ++v) part[v] += ps[v] * acc[v];
        };
        const int nv = spmm_wave_dispatch(S, t, stage, pp, (const T *)S.p, fin, finv);
        wave_partials_out(pp, nv, S.K, stage, red, a.part + (int64_t)t.tile * kMaxK);
        return;
    } else {
        const int G = S.K * S.M, gpw = kWave / G;
        const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
        const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
        for (int row = t.row0 + wave * gpw + grp; gpw >= 1 && row < t.row0 + t.rows;
             row += (kBB / kWave) * gpw) {
            T dg;
            const T qv = row_spmm(S, row, j, m, S.M, dg, S.p);
            if (m == 0) {
                const int64_t e = (int64_t)row * S.K + j;
                S.q[e] = qv;
                ppq += S.p[e] * qv;
            }
        }
    }
    block_sum_by_rhs(ppq, S.K, red, a.part + (int64_t)t.tile * kMaxK);
}

// (R1) alpha per right-hand side; breakdown / non-finite p.q ends it.  A
// system whose last x steps were taken (state 2) becomes done (1).
template <typename T>
__global__ __launch_bounds__(kBB) void batch_r1_kernel(BArgsT<T> a)
{
    __shared__ T red[kBB];
    __shared__ int any_active;
    const int sid = a.list[blockIdx.x];
    const int done = a.sys_done[sid];
    if (done) {
        if (done == 2 && threadIdx.x == 0) a.sys_done[sid] = 1;
        return;
    }
    const BSysT<T> S = a.sys[sid];
    if (threadIdx.x == 0) any_active = 0;
    const T pq = sys_sum(a, S, 0, red);  // its barriers order any_active's reset
    if ((int)threadIdx.x < S.K) {
        BScalT<T> &c = a.scal[S.scal0 + threadIdx.x];
        c.xstep = 0;
        c.ru = 0;
        if (c.active) {
            c.pq = pq;
            if (!isfinite(pq) || !(pq > T(0))) {
                c.status = isfinite(pq) ? CGX_BREAKDOWN : CGX_NONFINITE;
                c.active = 0;
            } else {
                c.alpha = c.rho / pq;
                c.rho_used = c.rho;
                c.iter += 1;
                c.xstep = 1;
                atomicOr(&any_active, 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && !any_active) a.sys_done[sid] = 1;  // no x step left either
}

// (2) r -= alpha q, z = D^-1 r for active right-hand sides; r.r and r.z
// partials.  x += alpha p is taken in the p update (3), which reads p
// anyway, so that p is read once per iteration outside the SpMM.
// 16-byte accesses of the interleaved vectors (Vec16): V = 16 / sizeof(T)
// consecutive right-hand sides of one row per access (used when K >= V; the
// vectors start 256-byte aligned and K is a multiple of V, so every access
// is aligned).

// Per-right-hand-side sums of V values per thread: value v of thread t
// belongs to right-hand side (t V + v) mod K (K a multiple of V, K / V
// dividing kBB); each right-hand side's values are added in index order.
// `red` holds kBB * V values; the K totals go to out[0..K).
template <typename T, int V>
__device__ __forceinline__ void block_sum_by_rhs_vec(const T (&v)[V], int K, T *red, T *out)
{
    __syncthreads();
#pragma unroll
    for (int u = 0; u < V; ++u) red[threadIdx.x * V + u] = v[u];
    __syncthreads();
    if ((int)threadIdx.x < K) {
        T s = T(0);
        for (int i = threadIdx.x; i < kBB * V; i += K) s += red[i];
        out[threadIdx.x] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(kBB) void batch_update_kernel(BArgsT<T> a)
{
    constexpr int V = 16 / (int)sizeof(T);
    __shared__ T red[kBB * V];
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys]) return;
    const BSysT<T> S = a.sys[t.sys];
    T *base = a.part + (int64_t)t.tile * kMaxK;
    if (S.K >= V) {
        // thread t: right-hand sides j0 .. j0 + V - 1 of every (kBB / KV)-th row
        const int KV = S.K / V, j0 = ((int)threadIdx.x % KV) * V;
        T alpha[V], prr[V], prz[V];
        bool act[V], any = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const BScalT<T> c = a.scal[S.scal0 + j0 + v];
            alpha[v] = c.alpha;
            act[v] = c.active != 0;
            any = any || act[v];
            prr[v] = prz[v] = T(0);
        }
        if (any) {
            Vec16<T> *pr = reinterpret_cast<Vec16<T> *>(S.r);
            const Vec16<T> *pq = reinterpret_cast<const Vec16<T> *>(S.q);
            const int64_t g1 = (int64_t)(t.row0 + t.rows) * KV;
            const int drow = kBB / KV;
            int row = t.row0 + (int)threadIdx.x / KV;
#pragma unroll 2
            for (int64_t g = (int64_t)t.row0 * KV + threadIdx.x; g < g1; g += kBB, row += drow) {
                const Vec16<T> rv = pr[g], qv = pq[g];
                T rs[V], qs[V];
                __builtin_memcpy(rs, &rv, sizeof(rv));
                __builtin_memcpy(qs, &qv, sizeof(qv));
                const T di = S.jac ? S.dinv[row] : T(0);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (!act[v]) continue;
                    rs[v] = fma_t(-alpha[v], qs[v], rs[v]);
                    prr[v] += rs[v] * rs[v];
                    if (S.jac) prz[v] += rs[v] * (di * rs[v]);
                }
                Vec16<T> ro;
                __builtin_memcpy(&ro, rs, sizeof(ro));
                pr[g] = ro;
            }
        }
        block_sum_by_rhs_vec<T, V>(prr, S.K, red, base + a.part_stride);
        block_sum_by_rhs_vec<T, V>(prz, S.K, red, base + 2 * a.part_stride);
        return;
    }
    const int j = threadIdx.x % S.K;  // fixed per thread: K divides kBB
    const BScalT<T> c = a.scal[S.scal0 + j];
    T prr = T(0), prz = T(0);
    if (c.active) {
        const T alpha = c.alpha;
        const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
        // K divides kBB: the thread's row advances by kBB / K per step
        const int drow = kBB / S.K;
        int row = t.row0 + (int)threadIdx.x / S.K;
#pragma unroll 4
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB, row += drow) {
            const T ri = fma_t(-alpha, S.q[e], S.r[e]);
            S.r[e] = ri;
            prr += ri * ri;
            if (S.jac) {  // z = D^-1 r is not stored: the p update forms it again
                const T zi = S.dinv[row] * ri;
                prz += ri * zi;
            }
        }
    }
    block_sum_by_rhs(prr, S.K, red, base + a.part_stride);
    block_sum_by_rhs(prz, S.K, red, base + 2 * a.part_stride);
}

// (R2) stopping test and beta per right-hand side; when none stays active
// the system enters state 2 (its last x steps follow in the p update).
// Reliable-update systems (S.ru; binary32 iteration scaled by sigma = ||r||
// of the last float64 update, Sleijpen and van der Vorst's scheme as in
// mixed-precision CG): the test is the update test instead, ||r^||^2 <=
// stop2 (the tolerance in the scale of the last update) or ||r^||^2 <
// delta^2 max ||r^||^2 since the last update (c.bb holds that maximum); a
// right-hand side that passes it pauses (no beta, no p update; its x step
// still runs), with it every other right-hand side of the system that
// would go on, and the system enters state 3, after which the update
// kernels take over.
template <typename T>
__global__ __launch_bounds__(kBB) void batch_r2_kernel(BArgsT<T> a)
{
    __shared__ T red[kBB];
    __shared__ int any_active, any_ru;
    const int sid = a.list[blockIdx.x];
    if (a.sys_done[sid]) return;
    const BSysT<T> S = a.sys[sid];
    const T rr = sys_sum(a, S, 1, red);
    const T rz0 = sys_sum(a, S, 2, red);
    if (threadIdx.x == 0) any_active = any_ru = 0;
    __syncthreads();
    const bool mine = (int)threadIdx.x < S.K && a.scal[S.scal0 + threadIdx.x].active;
    T rz = T(0);
    int status = CGX_PENDING;
    bool pause = false;
    if (mine) {
        BScalT<T> &c = a.scal[S.scal0 + threadIdx.x];
        rz = S.jac ? rz0 : rr;
        c.rr = rr;
        if (!isfinite(rr) || !isfinite(rz)) {
            status = CGX_NONFINITE;
        } else if (S.ru) {
            if (rr > c.bb) c.bb = rr;
            pause = rr <= c.stop2 || (double)rr < S.rtol2 * (double)c.bb;
            if (!pause && !(rz > T(0)))
                status = CGX_BREAKDOWN;
            else if (!pause && c.iter >= S.maxit)
                status = CGX_NOT_CONVERGED;
        } else if (rr <= c.stop2) {
            status = CGX_OK;
        } else if (!(rz > T(0))) {
            status = CGX_BREAKDOWN;
        } else if (c.iter >= S.maxit) {
            status = CGX_NOT_CONVERGED;
        }
        if (pause) atomicOr(&any_ru, 1);
    }
    __syncthreads();
    if (mine) {
        BScalT<T> &c = a.scal[S.scal0 + threadIdx.x];
        // the float64 residual of an update is a pass over the whole system
        // for all its right-hand sides: every one still active after this
        // step takes the update too (exact in exact arithmetic, like any
        // reliable update), also one that the iteration cap or rho <= 0 would
        // stop here: the update restarts rho from the true residual and the
        // resume applies the cap; a non-finite one stops
        if (S.ru && any_ru && status != CGX_NONFINITE) pause = true;
        if (pause) {
            c.ru = 1;
            c.active = 0;
        } else if (status == CGX_PENDING) {
            c.beta = rz / c.rho_used;
            c.rho = rz;
            atomicOr(&any_active, 1);
        } else {
            c.status = status;
            c.active = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (any_ru)
            a.sys_done[sid] = 3;
        else if (!any_active)
            a.sys_done[sid] = 2;
    }
}

// (3) x += alpha p for the right-hand sides that took a step this
// iteration, then p = z + beta p for those still active, z = D^-1 r formed
// here (the same product as in the update, so the same bits) instead of
// being stored by the update and read back: D^-1 has one value per row, z
// one per (row, right-hand side).
template <typename T>
__global__ __launch_bounds__(kBB) void batch_direction_kernel(BArgsT<T> a)
{
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys] == 1) return;
    const BSysT<T> S = a.sys[t.sys];
    constexpr int V = 16 / (int)sizeof(T);
    if (S.K >= V) {  // 16-byte accesses, as in the update
        const int KV = S.K / V, j0 = ((int)threadIdx.x % KV) * V;
        T alpha[V], beta[V];
        bool xs[V], act[V], anyx = false, anyp = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const BScalT<T> c = a.scal[S.scal0 + j0 + v];
            alpha[v] = c.alpha;
            beta[v] = c.beta;
            xs[v] = c.xstep != 0;
            act[v] = xs[v] && c.active != 0;
            anyx = anyx || xs[v];
            anyp = anyp || act[v];
        }
        if (!anyx) return;
        Vec16<T> *pp = reinterpret_cast<Vec16<T> *>(S.p), *px = reinterpret_cast<Vec16<T> *>(S.x);
        const Vec16<T> *pr = reinterpret_cast<const Vec16<T> *>(S.r);
        const int64_t g1 = (int64_t)(t.row0 + t.rows) * KV;
        const int drow = kBB / KV;
        int row = t.row0 + (int)threadIdx.x / KV;
#pragma unroll 2
        for (int64_t g = (int64_t)t.row0 * KV + threadIdx.x; g < g1; g += kBB, row += drow) {
            const Vec16<T> pv = pp[g], xv = px[g];
            T ps[V], xsv[V], rs[V];
            __builtin_memcpy(ps, &pv, sizeof(pv));
            __builtin_memcpy(xsv, &xv, sizeof(xv));
            T di = T(1);
            if (anyp) {
                const Vec16<T> rv = pr[g];
                __builtin_memcpy(rs, &rv, sizeof(rv));
                if (S.jac) di = S.dinv[row];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (xs[v]) xsv[v] = fma_t(alpha[v], ps[v], xsv[v]);
                if (act[v]) ps[v] = fma_t(beta[v], ps[v], S.jac ? di * rs[v] : rs[v]);
            }
            Vec16<T> xo;
            __builtin_memcpy(&xo, xsv, sizeof(xo));
            px[g] = xo;
            if (anyp) {
                Vec16<T> po;
                __builtin_memcpy(&po, ps, sizeof(po));
                pp[g] = po;
            }
        }
        return;
    }
    const int j = threadIdx.x % S.K;
    const BScalT<T> c = a.scal[S.scal0 + j];
    if (!c.xstep) return;
    const T alpha = c.alpha, beta = c.beta;
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    if (!c.active) {  // finished in this iteration: its last x step only
#pragma unroll 4
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) S.x[e] = fma_t(alpha, S.p[e], S.x[e]);
    } else if (S.jac) {
        const int drow = kBB / S.K;
        int row = t.row0 + (int)threadIdx.x / S.K;
#pragma unroll 4
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB, row += drow) {
            const T pv = S.p[e];
            S.x[e] = fma_t(alpha, pv, S.x[e]);
            S.p[e] = fma_t(beta, pv, S.dinv[row] * S.r[e]);
        }
    } else {
#pragma unroll 4
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
            const T pv = S.p[e];
            S.x[e] = fma_t(alpha, pv, S.x[e]);
            S.p[e] = fma_t(beta, pv, S.r[e]);
        }
    }
}

// Interleaved x -> caller layout (x = 0 where b = 0).
template <typename T>
__global__ __launch_bounds__(kBB) void batch_out_kernel(BArgsT<T> a)
{
    const BTile t = a.tiles[blockIdx.x];
    const BSysT<T> S = a.sys[t.sys];
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        if (j < S.nrhs) {
            const BScalT<T> &c = a.scal[S.scal0 + j];
            S.X[(int64_t)j * S.n + row] = (c.bb == T(0) && c.status == CGX_OK) ? T(0) : S.x[e];
        }
    }
}

// Served slot: a request joins free lane j of running system `si`.  Setup of
// that lane alone, one workgroup per tile of the system (a.tiles + tile0):
// x[:, j] = caller x0, r = b - A x0 (SpMV over the caller's x0 directly), z =
// D^-1 r (dinv from the slot's setup; the lane checks its diagonal itself),
// p = z, and the tile partials of r.r, r.z, b.b for lane j.
__global__ __launch_bounds__(kBB) void lane_init_kernel(BArgs a, int si, int j)
{
    __shared__ double red[3 * (kBB / kWave)];
    const BSys S = a.sys[si];
    // tile blockIdx.x of the system: rows [b trows, (b + 1) trows), partials
    // at S.tile0 + b (the work table may hold other systems' tiles between)
    const int row0 = blockIdx.x * S.trows, row1 = min(S.n, row0 + S.trows);
    const double *x0 = S.lanes[j].x;
    const double *b = S.lanes[j].b;
    const int K = S.K;
    double part[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    for (int row = row0 + threadIdx.x; row < row1; row += kBB) {
        const int s0 = clampk(S.rp[row], S.nnz);
        const int s1 = max(s0, clampk(S.rp[row + 1], S.nnz));
        double ax = 0.0, dg = 0.0;
        for (int k = s0; k < s1; ++k) {
            const int c = S.ci[k];
            if ((unsigned)c < (unsigned)S.n_cols) ax += S.val[k] * x0[c];
            if (c == row) dg = S.val[k];
        }
        const int64_t e = (int64_t)row * K + j;
        const double bi = b[row];
        const double ri = bi - ax;
        double zi = ri;
        S.x[e] = x0[row];
        S.r[e] = ri;
        if (S.jac) {
            bad = bad || !(dg > 0.0);
            zi = S.dinv[row] * ri;
            S.z[e] = zi;
        }
        S.p[e] = zi;
        part[0] += ri * ri;
        part[1] += ri * zi;
        part[2] += bi * bi;
    }
    if (bad) a.scal[S.scal0 + j].pad = 1;  // same value from every writer
    block_sum<3, kBB>(part, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < 3; ++r)
            a.part[r * a.part_stride + (int64_t)(S.tile0 + blockIdx.x) * kMaxK + j] = part[r];
}

// One workgroup: lane j's initial state from its tile partials (tile order),
// as batch_r0_kernel does for a whole system; an active lane clears the
// system's done flag.
__global__ __launch_bounds__(kBB) void lane_r0_kernel(BArgs a, int si, int j)
{
    __shared__ double red[kBB / kWave];
    const BSys S = a.sys[si];
    double v[3];
    for (int r = 0; r < 3; ++r) {
        const double *base = a.part + r * a.part_stride;
        double s = 0.0;
        for (int q = threadIdx.x; q < S.ntiles; q += kBB) s += base[(int64_t)(S.tile0 + q) * kMaxK + j];
        v[r] = sum_partials_in_block(s, red);
    }
    if (threadIdx.x == 0) {
        BScal &c = a.scal[S.scal0 + j];
        const bool badd = c.pad != 0;
        const double rr = v[0], rz = v[1], bb = v[2];
        c.rr = rr;
        c.bb = bb;
        c.rho = S.jac ? rz : rr;
        c.stop2 = S.rtol2 * bb;
        c.iter = 0;
        int status = CGX_PENDING;
        if (badd)
            status = CGX_BREAKDOWN;
        else if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz))
            status = CGX_NONFINITE;
        else if (bb == 0.0 || rr <= S.rtol2 * bb)
            status = CGX_OK;
        else if (S.jac && !(rz > 0.0))
            status = CGX_BREAKDOWN;
        c.status = status;
        c.active = status == CGX_PENDING;
        if (c.active) a.sys_done[si] = 0;
    }
}

// Served slot: right-hand side j of system `si` (finished) -> its caller x
// (x = 0 where b = 0).
__global__ __launch_bounds__(kBB) void lane_out_kernel(const BSys *sys, int si, int j,
                                                       const BScal *scal)
{
    const BSys &S = sys[si];
    const BScal &c = scal[S.scal0 + j];
    const bool zero = c.bb == 0.0 && c.status == CGX_OK;
    double *x = S.lanes[j].x;
    const int64_t stride = (int64_t)gridDim.x * kBB;
    for (int64_t i = (int64_t)blockIdx.x * kBB + threadIdx.x; i < S.n; i += stride)
        x[i] = zero ? 0.0 : S.x[i * S.K + j];
}

template <typename T>
__global__ void batch_scal_init_kernel(BScalT<T> *scal, int64_t n, int32_t *done, int nsys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) scal[i] = BScalT<T>{};
    if (i < nsys) done[i] = 0;
}

// x[0..n) = 0 (solutions of zero right-hand sides).
__global__ void batch_zero_kernel(double *x, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

template <typename T>
void launch_batch_iteration(const BArgsT<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL((batch_spmm_kernel<T>), dim3(a.ntiles), dim3(kBB), a.wave_lds, s, a);
    hipLaunchKernelGGL((batch_r1_kernel<T>), dim3(a.nlist), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL((batch_update_kernel<T>), dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL((batch_r2_kernel<T>), dim3(a.nlist), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL((batch_direction_kernel<T>), dim3(a.ntiles), dim3(kBB), 0, s, a);
}

// ------------------------------------------- reliable-update batch --
// Binary32 CG with float64 reliable updates for every (system, right-hand
// side) of the batch (the single-system MIXED_RU method): the binary32
// plan iterates on r^ = r / sigma with d (its x) the correction in that
// scale; batch_r2_kernel pauses a right-hand side when its update test
// fires (system state 3), and these kernels, launched after the p update of
// every iteration, take the update for the paused ones: x += sigma d, d = 0
// (fold); r = b - A x in float64 (residual); sigma' = ||r||, the float64
// stopping test (norm); r^ = float(r / sigma'), z = D^-1 r^ (rescale);
// beta = (rho' / rho) (sigma' / sigma) and the right-hand side resumes
// (resume); p = z + beta p (direction).  Systems in another state return at
// once.  The tile kernels walk the binary32 work table (the batch call's
// two plans have the same tiles; the server's binary32 table holds the
// tiles of its binary32-refined slots, numbered in one space with the
// float64 ones), the per-system kernels the binary32 list.

__global__ __launch_bounds__(kBB) void ru_fold_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    const BTile t = a32.tiles[blockIdx.x];
    if (a32.sys_done[t.sys] != 3) return;
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    const int j = threadIdx.x % S.K;
    if (!a32.scal[F.scal0 + j].ru) return;
    const double sigma = sqrt(a64.scal[S.scal0 + j].rr);
    const int64_t e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = (int64_t)t.row0 * S.K + threadIdx.x; e < e1; e += kBB) {
        S.x[e] = __builtin_fma(sigma, (double)F.x[e], S.x[e]);
        F.x[e] = 0.0f;
    }
}

// The residual runs on the SpMM's wave tiles (the tile's rows times x) for
// systems of the batch call on that schedule, when the launch carries the
// staging LDS (a64.wave_lds); otherwise, and in the solve server, as a
// vector-CSR pass.
__global__ __launch_bounds__(kBB) void ru_residual_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    __shared__ double red[kBB];
    extern __shared__ double stage[];  // a64.wave_lds bytes
    const BTile t = a32.tiles[blockIdx.x];
    if (a32.sys_done[t.sys] != 3) return;
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    if (S.M < 0 && S.staged && a64.wave_lds >= kWaveStageBytes) {
        constexpr int V = 2;
        const BScalT<float> *fs = a32.scal + F.scal0;
        auto fin = [&](int row, int j, double acc, double &part, double) {
            if (!fs[j].ru) return;
            const double bi = S.lanes ? S.lanes[j].b[row] : S.B[(int64_t)j * S.n + row];
            const double ri = bi - acc;
            S.r[(int64_t)row * S.K + j] = ri;
            part += ri * ri;
        };
        auto finv = [&](int row, int j0, double (&acc)[V], double (&part)[V], double) {
#pragma unroll
            for (int v = 0; v < V; ++v) fin(row, j0 + v, acc[v], part[v], 0.0);
        };
        double pp[V];
        const int nv = spmm_wave_dispatch(S, t, stage, pp, (const double *)S.x, fin, finv);
        wave_partials_out(pp, nv, S.K, stage, red, a64.part + (int64_t)t.tile * kMaxK);
        return;
    }
    const int M = setup_m(S);
    const int G = S.K * M, gpw = kWave / G;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
    const bool on = a32.scal[F.scal0 + j].ru != 0;
    double prr = 0.0;
    for (int row = t.row0 + wave * gpw + grp; gpw >= 1 && row < t.row0 + t.rows;
         row += (kBB / kWave) * gpw) {
        double dg;
        const double ax = row_spmm(S, row, j, m, M, dg, S.x);
        if (m == 0 && on) {
            const double bi = S.lanes ? S.lanes[j].b[row] : S.B[(int64_t)j * S.n + row];
            const double ri = bi - ax;
            S.r[(int64_t)row * S.K + j] = ri;
            prr += ri * ri;
        }
    }
    block_sum_by_rhs(prr, S.K, red, a64.part + (int64_t)t.tile * kMaxK);
}

// max_updates: the update cap (0: the float64 descriptor's maxit holds it)
__global__ __launch_bounds__(kBB) void ru_norm_kernel(BArgsT<double> a64, BArgsT<float> a32,
                                                      int max_updates)
{
    __shared__ double red[kBB];
    const int sid = a32.list[blockIdx.x];
    if (a32.sys_done[sid] != 3) return;
    const BSysT<double> S = a64.sys[sid];
    const BSysT<float> F = a32.sys[sid];
    const double rr = sys_sum(a64, S, 0, red);
    if ((int)threadIdx.x < S.K) {
        BScalT<float> &c = a32.scal[F.scal0 + threadIdx.x];
        if (c.ru) {
            BScalT<double> &d = a64.scal[S.scal0 + threadIdx.x];
            d.pq = d.rr;  // sigma^2 of the previous update
            d.rr = rr;
            d.iter += 1;  // updates taken
            int status = CGX_PENDING;
            if (!isfinite(rr))
                status = CGX_NONFINITE;
            else if (rr <= d.stop2)
                status = CGX_OK;
            else if (d.iter >= (max_updates > 0 ? max_updates : S.maxit))
                status = CGX_NOT_CONVERGED;  // the update cap (x already holds d)
            if (status != CGX_PENDING) {
                d.status = status;
                c.status = status;
                c.ru = 0;
            }
        }
    }
}

__global__ __launch_bounds__(kBB) void ru_rescale_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    __shared__ float red[kBB];
    const BTile t = a32.tiles[blockIdx.x];
    if (a32.sys_done[t.sys] != 3) return;
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    const int j = threadIdx.x % S.K;
    const bool on = a32.scal[F.scal0 + j].ru != 0;
    float prz = 0.0f, prr = 0.0f;
    if (on) {
        const double sigma = sqrt(a64.scal[S.scal0 + j].rr);
        const int64_t e1 = (int64_t)(t.row0 + t.rows) * S.K;
        int row = t.row0 + (int)threadIdx.x / S.K;
        for (int64_t e = (int64_t)t.row0 * S.K + threadIdx.x; e < e1; e += kBB, row += kBB / S.K) {
            const float ci = (float)(S.r[e] / sigma);
            const float zi = F.jac ? F.dinv[row] * ci : ci;
            F.r[e] = ci;
            prz += ci * zi;
            prr += ci * ci;
        }
    }
    float *base = a32.part + (int64_t)t.tile * kMaxK;
    block_sum_by_rhs(prz, S.K, red, base);
    block_sum_by_rhs(prr, S.K, red, base + a32.part_stride);
}

__global__ __launch_bounds__(kBB) void ru_resume_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    __shared__ float red[kBB];
    __shared__ int any_active;
    const int sid = a32.list[blockIdx.x];
    if (a32.sys_done[sid] != 3) return;
    const BSysT<double> S = a64.sys[sid];
    const BSysT<float> F = a32.sys[sid];
    if (threadIdx.x == 0) any_active = 0;
    const float rz = sys_sum(a32, F, 0, red);  // its barriers order the reset above
    const float rr = sys_sum(a32, F, 1, red);
    if ((int)threadIdx.x < S.K) {
        BScalT<float> &c = a32.scal[F.scal0 + threadIdx.x];
        if (c.ru) {
            BScalT<double> &d = a64.scal[S.scal0 + threadIdx.x];
            int status = CGX_PENDING;
            if (!isfinite(rz) || !isfinite(rr))
                status = CGX_NONFINITE;
            else if (!(rz > 0.0f))
                status = CGX_BREAKDOWN;
            else if (c.iter >= F.maxit)
                status = CGX_NOT_CONVERGED;
            if (status == CGX_PENDING) {
                c.beta = (rz / c.rho) * (float)(sqrt(d.rr) / sqrt(d.pq));
                c.rho = rz;
                c.rr = rr;
                c.bb = rr;  // the maximum of ||r^||^2 restarts at the update
                c.stop2 = (float)(d.stop2 / d.rr);
                c.active = 1;
                atomicOr(&any_active, 1);
            } else {
                c.status = status;
                c.ru = 0;
                if (status != CGX_NOT_CONVERGED) d.status = status;
            }
        } else if (c.active) {
            atomicOr(&any_active, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a32.sys_done[sid] = any_active ? 0 : 1;
}

__global__ __launch_bounds__(kBB) void ru_direction_kernel(BArgsT<float> a32)
{
    const BTile t = a32.tiles[blockIdx.x];
    const BSysT<float> F = a32.sys[t.sys];
    const int j = threadIdx.x % F.K;
    const BScalT<float> c = a32.scal[F.scal0 + j];
    if (!c.ru || !c.active) return;
    const float beta = c.beta;
    const int64_t e1 = (int64_t)(t.row0 + t.rows) * F.K;
    int row = t.row0 + (int)threadIdx.x / F.K;
    for (int64_t e = (int64_t)t.row0 * F.K + threadIdx.x; e < e1; e += kBB, row += kBB / F.K)
        F.p[e] = fma_t(beta, F.p[e], F.jac ? F.dinv[row] * F.r[e] : F.r[e]);
}

// Start of the reliable-update iteration (after the first float64
// residual and the binary32 setup on float(r / sigma)): the maximum of
// ||r^||^2 starts at its first value and the stopping test moves into the
// scale sigma; right-hand sides already done in float64 stay inactive.
__global__ __launch_bounds__(kBB) void ru_start_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    __shared__ int any_active;
    const int sid = a32.list[blockIdx.x];
    const BSysT<double> S = a64.sys[sid];
    const BSysT<float> F = a32.sys[sid];
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    if ((int)threadIdx.x < S.K) {
        BScalT<float> &c = a32.scal[F.scal0 + threadIdx.x];
        const BScalT<double> &d = a64.scal[S.scal0 + threadIdx.x];
        if (d.status != CGX_PENDING) {
            c.active = 0;
            c.status = CGX_OK;
        } else if (c.active) {
            c.bb = c.rr;
            c.stop2 = (float)(d.stop2 / d.rr);
            atomicOr(&any_active, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a32.sys_done[sid] = any_active ? 0 : 1;
}

// End: x += sigma d for every right-hand side (d is 0 where the last update
// folded it; it holds the pending correction where the iteration cap or a
// breakdown stopped the binary32 iteration).
__global__ __launch_bounds__(kBB) void ru_final_fold_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    const BTile t = a32.tiles[blockIdx.x];
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    const int j = threadIdx.x % S.K;
    if (j >= S.nrhs) return;
    const double sigma = sqrt(a64.scal[S.scal0 + j].rr);
    const int64_t e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = (int64_t)t.row0 * S.K + threadIdx.x; e < e1; e += kBB)
        S.x[e] = __builtin_fma(sigma, (double)F.x[e], S.x[e]);
}

void launch_ru_iteration(const BArgsT<double> &a64, const BArgsT<float> &a32, int max_updates,
                         hipStream_t s)
{
    launch_batch_iteration(a32, s);
    const dim3 g(a32.ntiles), l(a32.nlist), b(kBB);
    hipLaunchKernelGGL(ru_fold_kernel, g, b, 0, s, a64, a32);
    hipLaunchKernelGGL(ru_residual_kernel, g, b, a64.wave_lds, s, a64, a32);
    hipLaunchKernelGGL(ru_norm_kernel, l, b, 0, s, a64, a32, max_updates);
    hipLaunchKernelGGL(ru_rescale_kernel, g, b, 0, s, a64, a32);
    hipLaunchKernelGGL(ru_resume_kernel, l, b, 0, s, a64, a32);
    hipLaunchKernelGGL(ru_direction_kernel, g, b, 0, s, a32);
}

int pad_k(int nrhs)
{
    int K = 1;
    while (K < nrhs) K *= 2;
    return K;
}

int tile_rows_for(int K, bool staged) { return staged && K >= 8 ? 4096 / K : 2048 / K; }

// Wave-tile schedules the kernels instantiate: RT rows per wave with
// RT * K <= 64 (K = 1: any power of two; K > 1: 1, 2 or 4 lanes per
// right-hand side and row).
bool wave_schedule_ok(int rt, int K)
{
    if (rt < 1 || rt > 64 || (rt & (rt - 1)) || rt * K > 64) return false;
    return K == 1 || rt * K >= 16;
}

// Candidate schedules for K right-hand sides: slice counts M > 0, groups of
// K * M lanes in {8, 16, 32, 64} (at least one lane per right-hand side), and
// wave tiles (M = -rows per wave tile): for one right-hand side the rows
// whose expected entries fill one 64 x 8 chunk and half of that, for K > 1
// one or two lanes per right-hand side and row.
std::vector<int> m_candidates(int K, int64_t n = 0, int64_t nnz = 0)
{
    std::vector<int> out;
    for (int G = 8; G <= 64; G *= 2)
        if (G >= K) out.push_back(G / K);
    if (out.empty()) out.push_back(1);
    if (n > 0) {
        if (K == 1) {
            const int rt = wave_tile_rows(n, nnz, 8);
            out.push_back(-rt);
            if (rt > 1) out.push_back(-rt / 2);
        } else {
            out.push_back(-(64 / K));
            out.push_back(-(32 / K));
        }
    }
    return out;
}

// Deterministic default before tuning: about one lane per nonzero of a row
// (half for many right-hand sides), within the candidates.
int default_m(int K, double mean_row)
{
    int best = m_candidates(K).front();
    for (int M : m_candidates(K))
        if (K * M <= std::max(8.0, mean_row * (K >= 8 ? 0.5 : 1.0))) best = M;
    return best;
}

std::tuple<int, int, int> shape_key(int K, int64_t n, int64_t nnz)
{
    const int mean = n ? (int)std::lround((double)nnz / (double)n) : 0;
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= n) ++lg;
    return std::make_tuple(K, mean, lg);
}

}  // namespace
}  // namespace bk
}  // namespace cgx
