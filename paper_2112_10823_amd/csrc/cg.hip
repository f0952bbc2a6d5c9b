// Conjugate gradient (the paper's Section 5.3: classical CG, here with an
// optional Jacobi preconditioner, and binary32-inner iterative refinement as
// in the mixed-precision reference cited beside CG) on gfx950.
//
// Each iteration is three phases whose scalars never leave the GPU:
//   (1) q = A p (one wave tile per 64-thread workgroup) fused with one p.q
//       partial per tile; for more tiles than partial slots, a small kernel
//       adds the tile partials in fixed slices
//   (2) alpha = rho / p.q, x += alpha p, r -= alpha q, [z = D^-1 r], partials
//       of r.r [and r.z]
//   (3) stopping test, beta = rho' / rho, p = z + beta p
// Every workgroup of (2) and (3) adds the previous phase's partials itself,
// in the same order, so all of them hold bit-identical scalars without any
// grid-wide synchronisation inside a kernel; workgroup 0 records the state.
// The kernels are templated on the working precision: float64 for the plain
// solve, binary32 (values, vectors and accumulation) for the inner solve of
// the refinement.  K iterations are captured once into a HIP graph and
// replayed; the host reads one status word per replay.  After convergence
// the remaining kernels of a replay see `done` and return at once.  Systems
// of at most 4096 rows whose rows fit the register slots run the whole
// float64 solve inside one 1024-thread workgroup with the matrix on chip
// (one launch, workgroup barriers between phases): at that size the cost is
// launches and grid synchronisation, not bandwidth.
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "cgx_device.h"

namespace cgx {

// Workspace of cgx_cg_solve_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes its name to a
// kernel (on the host it is only a stand-in symbol): static_scratch_address
// looks up its device address per device, and that address is what the
// launches take.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kRB = 256;             // threads per workgroup of the p.q tile-partial reduction
constexpr int kMinTilesPerRed = 512; // tile partials per reduction workgroup, at least
constexpr int kPB = 512;             // threads per workgroup of the other phase kernels
constexpr int kPhaseBlocksPerCu = 4;
constexpr int kPre = 4;              // rows per thread an elementwise phase loads before its scalar
constexpr int kMaxPhaseBlocks = 2048;
constexpr int kSmallBlock = 1024;

// Partials of the grid-wide sums, one slot per workgroup of the phase grid.
// Each producer writes its own region; consumers read regions written by
// earlier kernels only.
enum PartialRegion { kPInit = 0 /* 3 arrays */, kPPq = 3, kPRr = 4, kPRz = 5, kPAux = 6 /* 2 */,
                     kPRegions = 8 };

template <typename T>
struct CgArgs {
    int n;
    int n_cols;
    int64_t nnz;
    const int32_t *rp;
    const int32_t *ci;
    const T *val;
    const T *b;
    T *x;
    T *r;
    T *p;
    T *q;
    T *z;     // == r without preconditioner
    T *dinv;  // nullptr without preconditioner
    T *partials;  // kPRegions * kMaxPhaseBlocks values
    T *tpart;     // p.q partial of each SpMV wave tile (region kPPq itself when it fits)
    const int64_t *sell_sp;  // sliced-ELL copy of A for the SpMV phase (null: CSR wave tiles)
    const int32_t *sell_col;
    const T *sell_val;
    CgState *st;
    double *coef;         // alpha_j at 2 j, beta_j at 2 j + 1, j < kCoefRec (while st->rec)
    int ntiles;           // wave tiles of the SpMV phase (= its workgroups)
    int tiles_per_red;    // tile partials added by one reduction workgroup
    int n_pq;             // p.q partials in region kPPq
    int grid_ew;          // workgroups of the update phase
};

template <typename T>
__host__ __device__ __forceinline__ T *region(const CgArgs<T> &a, int r)
{
    return a.partials + (int64_t)r * kMaxPhaseBlocks;
}

__global__ void cg_state_init_kernel(CgState *st, int maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        CgState s = {};
        s.maxit = maxit;
        s.status = CGX_PENDING;
        s.rec = 1;
        *st = s;
    }
}

// Status after the setup pass r0 = b - A x0, z0 = D^-1 r0, p0 = z0.
__device__ void finish_init(CgState *st, double rr, double rz, double bb, double rtol2, bool jac)
{
    st->rr = rr;
    st->bb = bb;
    st->rho = jac ? rz : rr;
    st->stop2 = rtol2 * bb;
    st->iter = 0;
    int status = CGX_PENDING;
    if (st->bad)
        status = CGX_BREAKDOWN;
    else if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz))
        status = CGX_NONFINITE;
    else if (bb == 0.0 || rr <= rtol2 * bb)
        status = CGX_OK;
    else if (jac && !(rz > 0.0))
        status = CGX_BREAKDOWN;
    st->status = status;
    st->done = status != CGX_PENDING;
}

// Lane 0 of a row group: residual, preconditioner and direction of a row.
template <bool kJac>
__device__ __forceinline__ void init_row(const CgArgs<double> &a, int row, double ax, double diag,
                                         double (&part)[3])
{
    const double bi = a.b[row];
    const double ri = bi - ax;
    double zi = ri;
    a.r[row] = ri;
    if (kJac) {
        double d = diag;
        if (!(d > 0.0)) {
            a.st->bad = 1;  // every writer stores the same value
            d = 1.0;
        }
        const double di = 1.0 / d;
        a.dinv[row] = di;
        zi = di * ri;
        a.z[row] = zi;
    }
    a.p[row] = zi;
    part[0] += ri * ri;
    part[1] += ri * zi;
    part[2] += bi * bi;
}

// Row-tile range [t0, t1) of this workgroup in the SpMV-type phases; the
// tiles of one die are contiguous.
__device__ __forceinline__ void tile_range(int ntiles, int tiles_per_block, int &t0, int &t1)
{
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    t0 = lb * tiles_per_block;
    t1 = min(t0 + tiles_per_block, ntiles);
}

// ------------------------------------------------ phase kernels (large n) --

// Float64 row passes of the setup and the mixed solver's residual: the
// workgroup's contiguous range of wave tiles of RT rows (die-contiguous as
// in the phase kernels), wave w of the workgroup taking tiles w, w + W, ...
// (W waves per workgroup), each tile computed by wave_rows with the row's
// stored diagonal captured on the way.  f(row, A x row, a_ii) runs on the
// first lane of every row.  sm: the workgroup's W staging areas.
template <int RT>
using SetupSmem = WaveSmem<wave_e<double>(), RT, double>;

template <int RT, bool kDiagA, typename F>
__device__ __forceinline__ void setup_rows(int n, int n_cols, int64_t nnz,
                                           const int32_t *__restrict__ rp,
                                           const int32_t *__restrict__ ci,
                                           const double *__restrict__ val,
                                           const double *__restrict__ x, SetupSmem<RT> *sm, F f)
{
    constexpr int W = kPB / kWave;
    const int nt = (n + RT - 1) / RT;
    const int per = (nt + gridDim.x - 1) / gridDim.x;
    int t0, t1;
    tile_range(nt, per, t0, t1);
    const int w = threadIdx.x / kWave;
    for (int t = t0 + w; t < t1; t += W) {
        int row;
        double dg = 0.0;
        const double acc = wave_rows<wave_e<double>(), RT, 4, double, false, kDiagA>(
            t * RT, n, n_cols, nnz, rp, ci, val, x, sm[w], row, nullptr, nullptr, &dg);
        if (threadIdx.x % (kWave / RT) == 0 && row < n) f(row, acc, dg);
    }
}

// Setup: r0 = b - A x0 (the row's stored diagonal read on the way), z0, p0,
// and the partials of r.r, r.z, b.b.
template <int RT, bool kJac>
__global__ __launch_bounds__(kPB) void cg_init_kernel(CgArgs<double> a)
{
    __shared__ SetupSmem<RT> sm[kPB / kWave];
    double part[3] = {0.0, 0.0, 0.0};
    setup_rows<RT, kJac>(a.n, a.n_cols, a.nnz, a.rp, a.ci, a.val, a.x, sm,
                         [&](int row, double ax, double dg) { init_row<kJac>(a, row, ax, dg, part); });
    __shared__ double red[3 * (kPB / kWave)];
    block_sum<3, kPB>(part, red);
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) region(a, kPInit + j)[blockIdx.x] = part[j];
}

// One workgroup: adds the setup partials and sets the initial state.
__global__ __launch_bounds__(kPB) void cg_init_finish_kernel(CgArgs<double> a, int count,
                                                             double rtol2, int jac)
{
    __shared__ double red[kPB / kWave];
    const double rr = sum_partials<kPB>(region(a, kPInit + 0), count, red);
    const double rz = sum_partials<kPB>(region(a, kPInit + 1), count, red);
    const double bb = sum_partials<kPB>(region(a, kPInit + 2), count, red);
    if (threadIdx.x == 0) finish_init(a.st, rr, rz, bb, rtol2, jac != 0);
}

// (1) q = A p, one wave tile per workgroup, and the tile's partial of p.q.
template <int RT, typename T>
__global__ __launch_bounds__(kWave) void cg_spmv_kernel(CgArgs<T> a)
{
    // gathers in flight per lane: 8 in float64 (all of a Q1 row's share at 4
    // lanes per row), 16 in binary32 (2 lanes per row); measured in the solve
    // against 4, bit-identical
    constexpr int U = sizeof(T) == sizeof(double) ? 8 : 16;
    __shared__ WaveSmem<wave_e<T>(), RT, T> sm;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int row;
    T prow;  // p[row], from the gather of the diagonal entry
    const T acc = wave_rows<wave_e<T>(), RT, U, T, true>(tile * RT, a.n, a.n_cols, a.nnz, a.rp,
                                                         a.ci, a.val, a.p, sm, row, &a.st->done,
                                                         &prow);
    if (row < 0) return;  // the solve has stopped
    T part = T(0);
    if (threadIdx.x % (kWave / RT) == 0 && row < a.n) {
        a.q[row] = acc;
        part = prow * acc;
    }
    part = wave_sum(part);
    if (threadIdx.x == 0) a.tpart[tile] = part;
}

// (1) on a sliced-ELL copy of A: one 64-row slice per workgroup, the slice's
// partial of p.q.
template <typename T>
__global__ __launch_bounds__(kWave) void cg_sell_spmv_kernel(CgArgs<T> a)
{
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int row;
    T prow;  // p[row], from the gather of the diagonal entry
    const T acc = sell_rows<8, T, true>(tile, a.n, a.n_cols, a.sell_sp, a.sell_col, a.sell_val,
                                        a.p, row, &a.st->done, &prow);
    if (row < 0) return;  // the solve has stopped
    T part = T(0);
    if (row < a.n) {
        a.q[row] = acc;
        part = prow * acc;
    }
    part = wave_sum(part);
    if (threadIdx.x == 0) a.tpart[tile] = part;
}

// (1b) Workgroup b adds tile partials [b * tiles_per_red, ...) in index order
// into slot b of region kPPq.
// kStop: return once the solve has stopped (inside the iteration; the true
// residual pass after the solve reduces regardless).
template <typename T, bool kStop>
__global__ __launch_bounds__(kRB) void cg_pq_reduce_kernel(CgArgs<T> a)
{
    const int t0 = blockIdx.x * a.tiles_per_red;
    const int count = max(0, min(a.tiles_per_red, a.ntiles - t0));
    __shared__ T red[kRB / kWave];
    const T s = sum_partials<kRB>(a.tpart + t0, count, red);  // loads in flight with st->done's
    if (kStop && a.st->done) return;
    if (threadIdx.x == 0) region(a, kPPq)[blockIdx.x] = s;
}

// (2) alpha = rho / p.q (every workgroup adds the p.q partials in the same
// order), x += alpha p, r -= alpha q, z = D^-1 r, partials of r.r and r.z.
// Workgroup 0 records alpha, the rho in use and the iteration count.
template <bool kJac, typename T>
__global__ __launch_bounds__(kPB) void cg_update_kernel(CgArgs<T> a)
{
    CgState *st = a.st;
    T *__restrict__ x = a.x;
    T *__restrict__ r = a.r;
    T *__restrict__ z = a.z;
    const T *__restrict__ p = a.p;
    const T *__restrict__ q = a.q;
    const T *__restrict__ dinv = a.dinv;
    const int64_t i0 = (int64_t)blockIdx.x * kPB + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kPB;
    // The thread's first kPre rows are loaded before alpha is known, so that
    // their loads are in flight with those of the partials and state fields
    // (rows past the end load row n - 1, n >= 1, and are not used).
    T xv[kPre], pv[kPre], rv[kPre], qv[kPre], dv[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const int64_t i = min(i0 + u * stride, (int64_t)a.n - 1);
        xv[u] = x[i];
        pv[u] = p[i];
        rv[u] = r[i];
        qv[u] = q[i];
        dv[u] = kJac ? dinv[i] : T(0);
    }
    __shared__ T red[kPB / kWave];
    const T pq = sum_partials<kPB>(region(a, kPPq), a.n_pq, red);
    if (st->done) return;
    const T rho = (T)st->rho;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!isfinite(pq) || !(pq > T(0))) {
        if (lead) {
            st->pq = pq;
            st->status = isfinite(pq) ? CGX_BREAKDOWN : CGX_NONFINITE;
            st->done = 1;
        }
        return;
    }
    const T alpha = rho / pq;
    if (lead) {
        const int it = st->iter;
        if (st->rec && it < kCoefRec) a.coef[2 * it] = (double)alpha;
        st->pq = pq;
        st->alpha = alpha;
        st->rho_used = rho;
        st->iter = it + 1;
    }
    T part[2] = {T(0), T(0)};
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const int64_t i = i0 + u * stride;
        if (i < a.n) {
            const T xi = __builtin_fma(alpha, pv[u], xv[u]);
            const T ri = __builtin_fma(-alpha, qv[u], rv[u]);
            x[i] = xi;
            r[i] = ri;
            part[0] += ri * ri;
            if (kJac) {
                const T zi = dv[u] * ri;
                z[i] = zi;
                part[1] += ri * zi;
            }
        }
    }
#pragma unroll 4
    for (int64_t i = i0 + kPre * stride; i < a.n; i += stride) {
        const T xi = __builtin_fma(alpha, p[i], x[i]);
        const T ri = __builtin_fma(-alpha, q[i], r[i]);
        x[i] = xi;
        r[i] = ri;
        part[0] += ri * ri;
        if (kJac) {
            const T zi = dinv[i] * ri;
            z[i] = zi;
            part[1] += ri * zi;
        }
    }
    __shared__ T red2[2 * (kPB / kWave)];
    block_sum<2, kPB>(part, red2);
    if (threadIdx.x == 0) {
        region(a, kPRr)[blockIdx.x] = part[0];
        region(a, kPRz)[blockIdx.x] = part[1];
    }
}

// (3) Stopping test on r.r (every workgroup adds the partials in the same
// order); beta = rho' / rho; p = z + beta p.  Workgroup 0 records the state.
// With delta2 > 0 (the binary32 iteration of the reliable-update solve) the
// iteration also stops, for a float64 update, once r.r < delta2 * rmax2,
// rmax2 the largest r.r since the last update (delta2 = 0 elsewhere: the
// test is r.r <= stop2 alone).
template <bool kJac, typename T>
__global__ __launch_bounds__(kPB) void cg_direction_kernel(CgArgs<T> a)
{
    CgState *st = a.st;
    T *__restrict__ p = a.p;
    const T *__restrict__ z = a.z;
    const int64_t i0 = (int64_t)blockIdx.x * kPB + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kPB;
    // the thread's first kPre rows, loaded before beta is known (rows past
    // the end load row n - 1, n >= 1, and are not used)
    T pv[kPre], zv[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const int64_t i = min(i0 + u * stride, (int64_t)a.n - 1);
        pv[u] = p[i];
        zv[u] = z[i];
    }
    __shared__ T red[kPB / kWave];
    T rr, rz;
    if constexpr (kJac) {
        // the loads of both partial arrays in flight together
        const T *const pa[2] = {region(a, kPRr), region(a, kPRz)};
        T ts[2];
        thread_partials<kPB>(pa, a.grid_ew, ts);
        rr = block_total<kPB>(ts[0], red);
        rz = block_total<kPB>(ts[1], red);
    } else {
        rr = rz = sum_partials<kPB>(region(a, kPRr), a.grid_ew, red);
    }
    if (st->done) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double rmax2 = fmax(st->rmax2, (double)rr);
    int status = CGX_PENDING;
    if (!isfinite(rr) || !isfinite(rz))
        status = CGX_NONFINITE;
    else if (rr <= (T)st->stop2 || (double)rr < st->delta2 * rmax2)
        status = CGX_OK;
    else if (!(rz > T(0)))
        status = CGX_BREAKDOWN;
    else if (st->iter >= st->maxit)
        status = CGX_NOT_CONVERGED;
    if (status != CGX_PENDING) {
        if (lead) {
            st->rr = rr;
            st->status = status;
            st->done = 1;
        }
        return;
    }
    const T beta = rz / (T)st->rho_used;
    if (lead) {
        const int j = st->iter - 1;  // the iteration whose alpha the update kernel formed
        if (st->rec && j >= 0 && j < kCoefRec) a.coef[2 * j + 1] = (double)beta;
        st->rr = rr;
        st->rho = rz;
        st->beta = beta;
        st->rmax2 = rmax2;
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const int64_t i = i0 + u * stride;
        if (i < a.n) p[i] = __builtin_fma(beta, pv[u], zv[u]);
    }
#pragma unroll 4
    for (int64_t i = i0 + kPre * stride; i < a.n; i += stride)
        p[i] = __builtin_fma(beta, p[i], z[i]);
}

// ||b - A x||^2 after the solve: one partial per wave tile, written to the
// p.q tile partials (free once the iteration has stopped), reduced like p.q
// into region kPPq, then one workgroup into st->rr_true.
template <int RT>
__global__ __launch_bounds__(kWave) void cg_true_residual_kernel(CgArgs<double> a)
{
    __shared__ WaveSmem<wave_e<double>(), RT, double> sm;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int row;
    const double acc = wave_rows<wave_e<double>(), RT, 4, double>(tile * RT, a.n, a.n_cols, a.nnz,
                                                                  a.rp, a.ci, a.val, a.x, sm, row);
    double part = 0.0;
    if (threadIdx.x % (kWave / RT) == 0 && row < a.n) {
        const double d = a.b[row] - acc;
        part = d * d;
    }
    part = wave_sum(part);
    if (threadIdx.x == 0) a.tpart[tile] = part;
}

__global__ __launch_bounds__(kPB) void cg_true_residual_finish_kernel(CgArgs<double> a)
{
    __shared__ double red[kPB / kWave];
    const double rr = sum_partials<kPB>(region(a, kPPq), a.n_pq, red);
    if (threadIdx.x == 0) a.st->rr_true = rr;
}

__global__ __launch_bounds__(kBlock) void zero_kernel(int64_t n, double *x)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// Status after p.q (single-workgroup path); forms alpha.
__device__ void small_finish_pq(CgState *st, double pq, double *coef)
{
    st->pq = pq;
    if (!isfinite(pq) || !(pq > 0.0)) {
        st->status = isfinite(pq) ? CGX_BREAKDOWN : CGX_NONFINITE;
        st->done = 1;
    } else {
        st->alpha = st->rho / pq;
        if (st->rec && st->iter < kCoefRec) coef[2 * st->iter] = st->alpha;
    }
}

// Status after the update (single-workgroup path); forms beta.
__device__ void small_finish_update(CgState *st, double rr, double rz, double *coef)
{
    const int iter = st->iter + 1;
    st->iter = iter;
    st->rr = rr;
    int status = CGX_PENDING;
    if (!isfinite(rr) || !isfinite(rz))
        status = CGX_NONFINITE;
    else if (rr <= st->stop2)
        status = CGX_OK;
    else if (!(rz > 0.0))
        status = CGX_BREAKDOWN;
    else if (iter >= st->maxit)
        status = CGX_NOT_CONVERGED;
    if (status == CGX_PENDING) {
        st->beta = rz / st->rho;
        st->rho = rz;
        if (st->rec && iter - 1 < kCoefRec) coef[2 * (iter - 1) + 1] = st->beta;
    } else {
        st->status = status;
        st->done = 1;
    }
}

// ------------------------------------ matrix-resident solve (n <= 4096) --
//
// One 1024-thread workgroup holds the whole system on chip for the solve:
// thread t owns rows t + 1024 j (j < R) with their values in registers (row
// j's entries in slots j * MAXE ...) and their column indices, as uint16, in
// LDS; p lives in LDS too, and x, r, z, D^-1, q of the owned rows in
// registers, and the solver state (rho, alpha, iteration count, status) in
// LDS.  An iteration then touches no global memory: SpMV from registers and
// LDS, three workgroup reductions, the p update in LDS.  A
// system with a row longer than MAXE does not fit: the kernel stores
// kStatusRetry before touching x and the host runs the phase kernels.
// (R, MAXE) = (1, 16), (2, 8), (4, 7): at most 28 value slots per thread,
// what the 128 registers of a 1024-thread workgroup hold beside the rest.

constexpr int kStatusRetry = 2;
constexpr int kResN = 4 * kSmallBlock;

template <int R, int MAXE, bool kJac>
__global__ __launch_bounds__(kSmallBlock) void cg_res_kernel(CgArgs<double> a, double rtol2)
{
    constexpr int BS = kSmallBlock;
    __shared__ double sp[R * BS];           // x0 during the setup, then p
    __shared__ double sx[R * BS];           // x
    __shared__ uint16_t cs[R * MAXE * BS];  // column of slot (j, e) of thread t
    __shared__ double red[3 * (BS / kWave)];
    __shared__ double sh_alpha, sh_beta;
    __shared__ int sh_done;
    __shared__ CgState sst;  // the solve's state, written back to a.st at exit
    CgState *st = &sst;
    const int n = a.n, t = threadIdx.x;
    if (t == 0) sst = *a.st;
    bool too_long = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = t + BS * j;
        if (i < n) too_long |= a.rp[i + 1] - a.rp[i] > MAXE;
    }
    if (__syncthreads_or(too_long)) {
        if (t == 0) {
            a.st->status = kStatusRetry;
            a.st->done = 1;
        }
        return;
    }
    // values to registers, columns to LDS; padding and out-of-range columns
    // become (value 0, column 0), which adds 0 * p[0]
    double v[R][MAXE], r[R], dv[R], q[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = t + BS * j;
        int s0 = 0, s1 = 0;
        if (i < n) {
            s0 = a.rp[i];
            s1 = a.rp[i + 1];
            s0 = s0 < 0 ? 0 : (s0 > a.nnz ? (int)a.nnz : s0);
            s1 = s1 < s0 ? s0 : (s1 > a.nnz ? (int)a.nnz : s1);
        }
        double d = 0.0;
#pragma unroll
        for (int e = 0; e < MAXE; ++e) {
            const int k = s0 + e;
            double vv = 0.0;
            int c = 0;
            if (k < s1) {
                const int cc = a.ci[k];
                if ((unsigned)cc < (unsigned)n) {
                    vv = a.val[k];
                    c = cc;
                    if (cc == i) d = vv;
                }
            }
            v[j][e] = vv;
            cs[(j * MAXE + e) * BS + t] = (uint16_t)c;
        }
        dv[j] = d;
        const double xi = i < n ? a.x[i] : 0.0;
        sx[i] = xi;
        sp[i] = xi;
    }
    __syncthreads();
    auto spmv = [&](double (&acc)[R]) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < MAXE; ++e) {
                s += v[j][e] * sp[cs[(j * MAXE + e) * BS + t]];
            }
            acc[j] = s;
        }
    };
    // r0 = b - A x0, z0 = D^-1 r0, p0 = z0 and the sums r.r, r.z, b.b
    spmv(q);
    double p3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = t + BS * j;
        r[j] = 0.0;
        if (i < n) {
            const double bi = a.b[i];
            r[j] = bi - q[j];
            double zj = r[j];
            if (kJac) {
                double d = dv[j];
                if (!(d > 0.0)) {
                    st->bad = 1;
                    d = 1.0;
                }
                dv[j] = 1.0 / d;
                zj = dv[j] * r[j];
            }
            p3[0] += r[j] * r[j];
            p3[1] += r[j] * zj;
            p3[2] += bi * bi;
        }
    }
    __syncthreads();  // every thread is done reading x0 from sp
#pragma unroll
    for (int j = 0; j < R; ++j) sp[t + BS * j] = kJac ? dv[j] * r[j] : r[j];
    block_sum<3, BS>(p3, red);
    if (t == 0) {
        finish_init(st, p3[0], p3[1], p3[2], rtol2, kJac);
        sh_done = st->done;
    }
    __syncthreads();

    while (!sh_done) {
        // q = A p, p.q
        spmv(q);
        double p1[1] = {0.0};
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (t + BS * j < n) p1[0] += sp[t + BS * j] * q[j];
        block_sum<1, BS>(p1, red);
        if (t == 0) {
            small_finish_pq(st, p1[0], a.coef);
            sh_done = st->done;
            sh_alpha = st->alpha;
        }
        __syncthreads();
        if (sh_done) break;
        // x += alpha p, r -= alpha q, z = D^-1 r, r.r and r.z
        const double alpha = sh_alpha;
        double p2[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = t + BS * j;
            if (i < n) {
                sx[i] = __builtin_fma(alpha, sp[i], sx[i]);
                r[j] = __builtin_fma(-alpha, q[j], r[j]);
                p2[0] += r[j] * r[j];
                if (kJac) p2[1] += r[j] * (dv[j] * r[j]);
            }
        }
        block_sum<2, BS>(p2, red);
        if (t == 0) {
            small_finish_update(st, p2[0], kJac ? p2[1] : p2[0], a.coef);
            sh_done = st->done;
            sh_beta = st->beta;
        }
        __syncthreads();
        if (sh_done) break;
        // p = z + beta p (each thread rewrites only its own rows)
        const double beta = sh_beta;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = t + BS * j;
            if (i < n) sp[i] = __builtin_fma(beta, sp[i], kJac ? dv[j] * r[j] : r[j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (t + BS * j < n) a.x[t + BS * j] = sx[t + BS * j];
    if (t == 0) *a.st = sst;
}

// ------------------------------------------------ mixed-precision refinement --
//
// Outer state (a CgState): rr = ||b - A x||^2 of the current x, bb = ||b||^2,
// stop2 = rtol^2 bb, alpha = the scale s = ||r|| of the current step, iter =
// refinement steps done, maxit = their cap.

struct MxArgs {
    int n;
    int n_cols;
    int64_t nnz;
    const int32_t *rp;
    const int32_t *ci;
    const double *val;
    const double *b;
    double *x;
    double *r;         // float64 residual b - A x
    float *dinv32;     // Jacobi: (float)(1 / a_ii), written on the first step
    double *partials;  // kPRegions * kMaxPhaseBlocks doubles (shared with the inner solve)
    CgState *ost;
};

// r = b - A x in float64 and the partials of ||r||^2 (and ||b||^2 and the
// inverse diagonal on the first step).
template <int RT, bool kFirst, bool kJac>
__global__ __launch_bounds__(kPB) void mx_residual_kernel(MxArgs m)
{
    __shared__ SetupSmem<RT> sm[kPB / kWave];
    if (m.ost->done) return;
    double part[2] = {0.0, 0.0};
    setup_rows<RT, kFirst && kJac>(m.n, m.n_cols, m.nnz, m.rp, m.ci, m.val, m.x, sm,
                                   [&](int row, double ax, double dg) {
        const double bi = m.b[row];
        const double ri = bi - ax;
        m.r[row] = ri;
        part[0] += ri * ri;
        if (kFirst) {
            part[1] += bi * bi;
            if (kJac) {
                double d = dg;
                if (!(d > 0.0)) {
                    m.ost->bad = 1;
                    d = 1.0;
                }
                m.dinv32[row] = (float)(1.0 / d);
            }
        }
    });
    __shared__ double red[2 * (kPB / kWave)];
    block_sum<2, kPB>(part, red);
    if (threadIdx.x == 0) {
        m.partials[(int64_t)kPAux * kMaxPhaseBlocks + blockIdx.x] = part[0];
        m.partials[(int64_t)(kPAux + 1) * kMaxPhaseBlocks + blockIdx.x] = part[1];
    }
}

// One workgroup: outer stopping test on the residual partials.
__global__ __launch_bounds__(kPB) void mx_residual_finish_kernel(MxArgs m, int count, int first,
                                                                 double rtol2)
{
    CgState *o = m.ost;
    if (o->done) return;
    __shared__ double red[kPB / kWave];
    const double rr = sum_partials<kPB>(m.partials + (int64_t)kPAux * kMaxPhaseBlocks, count, red);
    const double bb =
        sum_partials<kPB>(m.partials + (int64_t)(kPAux + 1) * kMaxPhaseBlocks, count, red);
    if (threadIdx.x != 0) return;
    if (first) {
        o->bb = bb;
        o->stop2 = rtol2 * bb;
    }
    o->rr = rr;
    int status = CGX_PENDING;
    if (o->bad)
        status = CGX_BREAKDOWN;
    else if (!isfinite(rr) || !isfinite(o->bb))
        status = CGX_NONFINITE;
    else if (o->bb == 0.0 || rr <= o->stop2)
        status = CGX_OK;
    else if (o->iter >= o->maxit)
        status = CGX_NOT_CONVERGED;
    if (status == CGX_PENDING) {
        o->sigma_prev = o->alpha;  // the scale of the step that just ended
        o->alpha = sqrt(rr);
    } else {
        o->status = status;
        o->done = 1;
    }
}

// Inner start: c = float(r / s), d = 0, r32 = c, z = D^-1 c, p = z, and the
// partials of c.c and c.z.
template <bool kJac>
__global__ __launch_bounds__(kPB) void mx_inner_init_kernel(MxArgs m, CgArgs<float> in)
{
    if (m.ost->done) return;
    const double inv_s = 1.0 / m.ost->alpha;
    float part[2] = {0.0f, 0.0f};
    const int64_t stride = (int64_t)gridDim.x * kPB;
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < m.n; i += stride) {
        const float ci = (float)(m.r[i] * inv_s);
        const float zi = kJac ? m.dinv32[i] * ci : ci;
        in.r[i] = ci;
        in.x[i] = 0.0f;
        if (kJac) in.z[i] = zi;
        in.p[i] = zi;
        part[0] += ci * ci;
        part[1] += ci * zi;
    }
    __shared__ float red[2 * (kPB / kWave)];
    block_sum<2, kPB>(part, red);
    if (threadIdx.x == 0) {
        region(in, kPInit)[blockIdx.x] = part[0];
        region(in, kPInit + 1)[blockIdx.x] = part[1];
    }
}

// One workgroup: inner state for a new refinement step (stop at
// ||r32|| <= tau ||c||).
// Reliable updates (delta2 > 0): the binary32 iteration runs on over all
// updates; it pauses for a float64 update when c.c falls below delta2 times
// its largest value since the last update, or below (rtol ||b|| / s)^2
// (converged by the estimate), and records its coefficients throughout.
__global__ __launch_bounds__(kPB) void mx_inner_init_finish_kernel(MxArgs m, CgArgs<float> in,
                                                                   int count, float tau2,
                                                                   int inner_maxit, int jac,
                                                                   double delta2)
{
    if (m.ost->done) return;
    __shared__ float red[kPB / kWave];
    const float cc = sum_partials<kPB>(region(in, kPInit), count, red);
    const float cz = jac ? sum_partials<kPB>(region(in, kPInit + 1), count, red) : cc;
    if (threadIdx.x != 0) return;
    CgState *s = in.st;
    s->rr = cc;
    s->rho = cz;
    s->iter = 0;
    s->maxit = inner_maxit;
    s->rec = m.ost->iter == 0 ? 1 : 0;  // coefficients of the first refinement step
    s->delta2 = delta2;
    s->rmax2 = cc;
    if (delta2 > 0.0) {
        const double sg = m.ost->alpha;
        s->stop2 = m.ost->stop2 / (sg * sg);
    } else {
        s->stop2 = (double)(tau2 * cc);
    }
    const bool bad = !isfinite(cc) || !isfinite(cz) || !(cz > 0.0f);
    s->status = bad ? CGX_NONFINITE : CGX_PENDING;
    s->done = bad ? 1 : 0;
}

// x += s * double(d); one refinement step done.
__global__ __launch_bounds__(kPB) void mx_correct_kernel(MxArgs m, const float *d)
{
    if (m.ost->done) return;
    const double s = m.ost->alpha;
    const int64_t stride = (int64_t)gridDim.x * kPB;
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < m.n; i += stride)
        m.x[i] = __builtin_fma(s, (double)d[i], m.x[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) m.ost->iter += 1;
}

// Reliable update, after x += s d and the float64 residual r = b - A x with
// its new norm s' (outer alpha; the old s in sigma_prev): the binary32
// recursive residual is replaced by c = float(r / s'), d = 0, z = D^-1 c, and
// the partials of c.c and c.z go where the direction kernel reads them.
template <bool kJac>
__global__ __launch_bounds__(kPB) void mx_ru_rescale_kernel(MxArgs m, CgArgs<float> in)
{
    if (m.ost->done) return;
    const double inv_s = 1.0 / m.ost->alpha;
    float part[2] = {0.0f, 0.0f};
    const int64_t stride = (int64_t)gridDim.x * kPB;
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < m.n; i += stride) {
        const float ci = (float)(m.r[i] * inv_s);
        const float zi = kJac ? m.dinv32[i] * ci : ci;
        in.r[i] = ci;
        in.x[i] = 0.0f;
        if (kJac) in.z[i] = zi;
        part[0] += ci * ci;
        part[1] += ci * zi;
    }
    __shared__ float red[2 * (kPB / kWave)];
    block_sum<2, kPB>(part, red);
    if (threadIdx.x == 0) {
        region(in, kPRr)[blockIdx.x] = part[0];
        region(in, kPRz)[blockIdx.x] = part[1];
    }
}

// One workgroup, between the rescale and the direction kernel: the inner
// state resumes in the new scale.  The direction kernel then forms
// beta = rho' / rho_used with rho_used = rho s / s', i.e. the CG beta of the
// true residuals carried into the new scale, and p = z + beta p keeps the
// search direction.  rmax2 restarts (0: the direction kernel takes c.c).
__global__ void mx_ru_resume_kernel(MxArgs m, CgArgs<float> in)
{
    if (threadIdx.x != 0 || m.ost->done) return;
    const CgState *o = m.ost;
    CgState *s = in.st;
    const double sg = o->alpha;
    s->rho_used = (double)(float)(s->rho_used * (o->sigma_prev / sg));
    s->stop2 = o->stop2 / (sg * sg);
    s->rmax2 = 0.0;
    s->status = CGX_PENDING;
    s->done = 0;
}

// ----------------------------------------------------------------- host --

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace layout.  float64 solve: state | r p q [z dinv] | partials.
// Mixed: outer state | inner state | r64 | r32 p32 q32 [z32 dinv32] | d32 | partials.
struct Layout {
    size_t state = 0, state2 = 0, r64 = 0, r = 0, p = 0, q = 0, z = 0, dinv = 0, d = 0;
    size_t partials = 0, tpart = 0, coef = 0, total = 0;
};

// Wave tiles of the SpMV phase for a system of n rows and nnz entries.
int64_t spmv_tiles(int64_t n, int64_t nnz, bool mixed)
{
    const int rt = wave_tile_rows(n, nnz, mixed ? wave_e<float>() : wave_e<double>());
    return (n + rt - 1) / rt;
}

Layout make_layout(int64_t n, int64_t nnz, bool jac, bool mixed)
{
    Layout L;
    size_t off = 0;
    const size_t vec = align_up((size_t)n * (mixed ? sizeof(float) : sizeof(double)));
    L.state = off;
    off += align_up(sizeof(CgState));
    if (mixed) {
        L.state2 = off;
        off += align_up(sizeof(CgState));
        L.r64 = off;
        off += align_up((size_t)n * sizeof(double));
    }
    L.r = off;
    off += vec;
    L.p = off;
    off += vec;
    L.q = off;
    off += vec;
    L.z = L.r;
    if (jac) {
        L.z = off;
        off += vec;
        L.dinv = off;
        off += vec;
    }
    if (mixed) {
        L.d = off;
        off += vec;
    }
    L.partials = off;
    off += align_up((size_t)kPRegions * kMaxPhaseBlocks * sizeof(double));
    L.tpart = off;
    off += align_up((size_t)std::max<int64_t>(spmv_tiles(n, nnz, mixed), 1) * sizeof(double));
    L.coef = off;
    off += align_up((size_t)2 * kCoefRec * sizeof(double));
    L.total = off;
    return L;
}

struct Grids {
    int RT64;           // rows per wave tile of the float64 setup passes
    int RT;             // rows per wave tile of the SpMV phase
    int ntiles;         // wave tiles (= workgroups) of the SpMV phase
    int grid_red;       // workgroups of the p.q reduction, 0 when the tiles write region kPPq
    int tiles_per_red;  // tile partials per reduction workgroup
    int n_pq;           // p.q partials the update phase adds
    int grid_ew;        // workgroups of the elementwise phases
    int grid_vr;        // workgroups of the float64 setup passes
};

Grids make_grids(const Context *c, int64_t n, int64_t nnz, bool mixed, bool sell)
{
    Grids g{};
    g.RT64 = wave_tile_rows(n, nnz, wave_e<double>());
    // sliced ELL: one 64-row slice per SpMV workgroup (never more tiles than
    // the wave tiles the workspace is sized for)
    g.RT = sell ? kWave : wave_tile_rows(n, nnz, mixed ? wave_e<float>() : wave_e<double>());
    g.ntiles = (int)std::max<int64_t>(1, (n + g.RT - 1) / g.RT);
    if (g.ntiles <= kMaxPhaseBlocks) {
        g.grid_red = 0;
        g.tiles_per_red = 0;
        g.n_pq = g.ntiles;
    } else {
        const int64_t per = (g.ntiles + kMaxPhaseBlocks - 1) / kMaxPhaseBlocks;
        g.tiles_per_red = (int)std::max<int64_t>(kMinTilesPerRed, per);
        g.grid_red = (int)((g.ntiles + g.tiles_per_red - 1) / g.tiles_per_red);
        g.n_pq = g.grid_red;
    }
    const int cap = std::min(c->num_cu * kPhaseBlocksPerCu, kMaxPhaseBlocks);
    const int64_t ew_need = (n + kPB - 1) / kPB;
    g.grid_ew = (int)std::max<int64_t>(1, std::min<int64_t>(cap, ew_need));
    // at least one wave tile per wave of a setup workgroup
    const int64_t vr_tiles = (n + g.RT64 - 1) / g.RT64;
    const int64_t vr_need = (vr_tiles + kPB / kWave - 1) / (kPB / kWave);
    g.grid_vr = (int)std::max<int64_t>(1, std::min<int64_t>(cap, vr_need));
    return g;
}

// Fills the launch-shape fields of a and points tpart at the tile partials.
template <typename T>
void bind_grids(const Grids &g, CgArgs<T> &a, void *tpart_ws)
{
    a.ntiles = g.ntiles;
    a.tiles_per_red = g.tiles_per_red;
    a.n_pq = g.n_pq;
    a.grid_ew = g.grid_ew;
    a.tpart = g.grid_red > 0 ? static_cast<T *>(tpart_ws) : region(a, kPPq);
}

void launch_init(const Grids &g, bool jac, hipStream_t s, const CgArgs<double> &a, double rtol2)
{
#define CGX_INIT(LL)                                                                             \
    if (jac)                                                                                     \
        hipLaunchKernelGGL((cg_init_kernel<LL, true>), dim3(g.grid_vr), dim3(kPB), 0, s, a);      \
    else                                                                                         \
        hipLaunchKernelGGL((cg_init_kernel<LL, false>), dim3(g.grid_vr), dim3(kPB), 0, s, a)
    CGX_WRT_SWITCH(g.RT64, CGX_INIT)
#undef CGX_INIT
    hipLaunchKernelGGL(cg_init_finish_kernel, dim3(1), dim3(kPB), 0, s, a, g.grid_vr, rtol2,
                       jac ? 1 : 0);
}

template <typename T>
void launch_spmv_kernel(const Grids &g, hipStream_t s, const CgArgs<T> &a)
{
    if (a.sell_sp) {
        hipLaunchKernelGGL((cg_sell_spmv_kernel<T>), dim3(g.ntiles), dim3(kWave), 0, s, a);
        return;
    }
#define CGX_SP(RR) \
    hipLaunchKernelGGL((cg_spmv_kernel<RR, T>), dim3(g.ntiles), dim3(kWave), 0, s, a)
    CGX_WRT_SWITCH(g.RT, CGX_SP)
#undef CGX_SP
}

template <typename T>
void launch_pq_reduce(const Grids &g, hipStream_t s, const CgArgs<T> &a)
{
    if (g.grid_red > 0)
        hipLaunchKernelGGL((cg_pq_reduce_kernel<T, true>), dim3(g.grid_red), dim3(kRB), 0, s, a);
}

template <typename T>
void launch_update_phase(const Grids &g, bool jac, hipStream_t s, const CgArgs<T> &a)
{
    if (jac)
        hipLaunchKernelGGL((cg_update_kernel<true, T>), dim3(g.grid_ew), dim3(kPB), 0, s, a);
    else
        hipLaunchKernelGGL((cg_update_kernel<false, T>), dim3(g.grid_ew), dim3(kPB), 0, s, a);
}

template <typename T>
void launch_direction_phase(const Grids &g, bool jac, hipStream_t s, const CgArgs<T> &a)
{
    if (jac)
        hipLaunchKernelGGL((cg_direction_kernel<true, T>), dim3(g.grid_ew), dim3(kPB), 0, s, a);
    else
        hipLaunchKernelGGL((cg_direction_kernel<false, T>), dim3(g.grid_ew), dim3(kPB), 0, s, a);
}

template <typename T>
void launch_iteration(const Grids &g, bool jac, hipStream_t s, const CgArgs<T> &a)
{
    launch_spmv_kernel<T>(g, s, a);
    launch_pq_reduce<T>(g, s, a);
    launch_update_phase<T>(g, jac, s, a);
    launch_direction_phase<T>(g, jac, s, a);
}

void launch_true_residual(const Grids &g, hipStream_t s, const CgArgs<double> &a)
{
#define CGX_TR(RR) \
    hipLaunchKernelGGL((cg_true_residual_kernel<RR>), dim3(g.ntiles), dim3(kWave), 0, s, a)
    CGX_WRT_SWITCH(g.RT, CGX_TR)
#undef CGX_TR
    if (g.grid_red > 0)
        hipLaunchKernelGGL((cg_pq_reduce_kernel<double, false>), dim3(g.grid_red), dim3(kRB), 0, s,
                           a);
    hipLaunchKernelGGL(cg_true_residual_finish_kernel, dim3(1), dim3(kPB), 0, s, a);
}

void launch_resident(bool jac, hipStream_t s, const CgArgs<double> &a, double rtol2)
{
#define CGX_RES(RR, EE)                                                                       \
    if (jac)                                                                                  \
        hipLaunchKernelGGL((cg_res_kernel<RR, EE, true>), dim3(1), dim3(kSmallBlock), 0, s, a, \
                           rtol2);                                                            \
    else                                                                                      \
        hipLaunchKernelGGL((cg_res_kernel<RR, EE, false>), dim3(1), dim3(kSmallBlock), 0, s,   \
                           a, rtol2)
    if (a.n <= kSmallBlock) {
        CGX_RES(1, 16);
    } else if (a.n <= 2 * kSmallBlock) {
        CGX_RES(2, 8);
    } else {
        CGX_RES(4, 7);
    }
#undef CGX_RES
}

void launch_mx_residual(const Grids &g, bool first, bool jac, hipStream_t s, const MxArgs &m,
                        double rtol2)
{
#define CGX_MX(LL)                                                                             \
    if (first && jac)                                                                          \
        hipLaunchKernelGGL((mx_residual_kernel<LL, true, true>), dim3(g.grid_vr), dim3(kPB), 0, \
                           s, m);                                                              \
    else if (first)                                                                            \
        hipLaunchKernelGGL((mx_residual_kernel<LL, true, false>), dim3(g.grid_vr), dim3(kPB), 0,\
                           s, m);                                                              \
    else                                                                                       \
        hipLaunchKernelGGL((mx_residual_kernel<LL, false, false>), dim3(g.grid_vr), dim3(kPB),  \
                           0, s, m)
    CGX_WRT_SWITCH(g.RT64, CGX_MX)
#undef CGX_MX
    hipLaunchKernelGGL(mx_residual_finish_kernel, dim3(1), dim3(kPB), 0, s, m, g.grid_vr,
                       first ? 1 : 0, rtol2);
}

// Iterations per graph replay: about 2 ms of work between host checks.
int replay_iters(const cgx_opts *o, double bytes_per_iter)
{
    int K = o->check_every;
    if (K <= 0) {
        const double t_iter = bytes_per_iter / 4.0e12 + 8.0e-6;
        K = (int)(2.0e-3 / t_iter);
        K = K < 4 ? 4 : (K > 32 ? 32 : K);
    }
    return K;
}

// Capture (or reuse) a graph of K iterations and replay it until the state's
// `done` flag is set, at most max_replays times.
// Key of a graph of K iterations: every argument and launch shape the
// captured launches take.
template <typename T>
GraphKey iteration_key(int K, const Grids &g, bool jac, const CgArgs<T> &a)
{
    GraphKey k;
    k.add(sizeof(T)).add((uint64_t)K).add(jac ? 1 : 0);
    k.add((uint64_t)g.RT).add((uint64_t)g.ntiles).add((uint64_t)g.grid_red);
    k.add((uint64_t)g.tiles_per_red).add((uint64_t)g.n_pq).add((uint64_t)g.grid_ew);
    k.add((uint64_t)a.n).add((uint64_t)a.n_cols).add((uint64_t)a.nnz);
    k.ptr(a.rp).ptr(a.ci).ptr(a.val).ptr(a.b).ptr(a.x).ptr(a.r).ptr(a.p).ptr(a.q).ptr(a.z);
    k.ptr(a.dinv).ptr(a.partials).ptr(a.tpart).ptr(a.sell_sp).ptr(a.sell_col).ptr(a.sell_val);
    k.ptr(a.st).ptr(a.coef).add((uint64_t)a.ntiles).add((uint64_t)a.tiles_per_red).add((uint64_t)a.n_pq);
    k.add((uint64_t)a.grid_ew);
    return k;
}

template <typename T>
int replay_until_done(Context *c, GraphSlot &slot, int K, const Grids &g, bool jac, hipStream_t s,
                      const CgArgs<T> &a, int64_t max_replays)
{
    const GraphKey key = iteration_key<T>(K, g, jac, a);
    if (!slot.matches(key)) {
        slot.reset();
        CGX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) launch_iteration<T>(g, jac, s, a);
        hipGraph_t graph = nullptr;
        CGX_HIP_CHECK(hipStreamEndCapture(s, &graph));
        slot.graph = graph;
        CGX_HIP_CHECK(hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0));
        slot.key = key.w;
    }
    for (int64_t rep = 0; rep < max_replays; ++rep) {
        CGX_HIP_CHECK(hipGraphLaunch(slot.exec, s));
        CGX_HIP_CHECK(
            hipMemcpyAsync(c->host_state, a.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        if (c->host_state->done) break;
    }
    return CGX_OK;
}

// Records the end of a solve, waits for it and reads the state; returns the
// solve's device time in ms.
int finish_solve(Context *c, hipStream_t s, const CgState *dev_state, CgState &hs, float &ms)
{
    CGX_HIP_CHECK(hipEventRecord(c->ev1, s));
    CGX_HIP_CHECK(
        hipMemcpyAsync(c->host_state, dev_state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    hs = *c->host_state;
    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    return CGX_OK;
}

// x = 0 when b = 0; then orders the caller's stream after the solve.
int zero_if_needed(Context *c, hipStream_t s, bool zero, int64_t n, double *x)
{
    if (zero) {
        hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(kBlock), 0, s, n, x);
        CGX_HIP_CHECK(hipGetLastError());
    }
    CGX_HIP_CHECK(hipEventRecord(c->ev_out, s));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_out, 0));
    if (zero) CGX_HIP_CHECK(hipStreamSynchronize(s));  // else finish_solve has waited
    return CGX_OK;
}

// Ritz extremes and condition estimate from the first k recorded
// coefficients (k = 0: left at 0).
// beta_scale (reliable updates): the beta recorded at iteration j is in the
// scale of the new residual; the Lanczos relation takes the CG beta of the
// true residuals, that beta times s' / s.
int fill_kappa(Context *c, hipStream_t s, const double *coef_dev, int64_t iters, cgx_stats *st,
               const std::vector<std::pair<int, double>> *beta_scale = nullptr)
{
    const int k = (int)std::min<int64_t>(iters, kCoefRec);
    st->kappa_est = st->ritz_min = st->ritz_max = 0.0;
    if (k <= 0) return CGX_OK;
    double *coef = c->kappa_host.data();  // 2 k coefficients, then 3 k of bisection work
    CGX_HIP_CHECK(hipMemcpyAsync(coef, coef_dev, 2 * (size_t)k * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    if (beta_scale)
        for (const auto &f : *beta_scale)
            if (f.first >= 0 && f.first + 1 < k) coef[2 * f.first + 1] *= f.second;
    double lo = 0.0, hi = 0.0;
    if (lanczos_extremes_ws(coef, k, coef + 2 * (size_t)kCoefRec, lo, hi)) {
        st->ritz_min = lo;
        st->ritz_max = hi;
        st->kappa_est = lo > 0.0 ? hi / lo : 0.0;
    }
    return CGX_OK;
}

int begin_solve(Context *c, hipStream_t s)
{
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    return CGX_OK;
}

// Launches K iterations at a time directly on the stream (no graph) until
// the state's `done` flag is set, at most max_rounds times.
int launch_until_done(Context *c, int K, const Grids &g, bool jac, hipStream_t s,
                      const CgArgs<double> &a, int64_t max_rounds)
{
    for (int64_t rep = 0; rep < max_rounds; ++rep) {
        for (int k = 0; k < K; ++k) launch_iteration<double>(g, jac, s, a);
        CGX_HIP_CHECK(hipGetLastError());
        CGX_HIP_CHECK(
            hipMemcpyAsync(c->host_state, a.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        if (c->host_state->done) break;
    }
    return CGX_OK;
}

// direct: iterations launched one by one instead of through a captured graph
// (the allocation-free entry point).
int run_fp64(Context *c, const cgx_csr *A, const cgx_sell *S, const double *b, double *x, void *ws,
             size_t ws_bytes, const cgx_opts *o, cgx_stats *st, bool direct = false)
{
    const int64_t n = A->n_rows;
    const bool jac = o->precond == CGX_PRECOND_JACOBI;
    const Layout lay = make_layout(n, A->nnz, jac, false);
    if (ws_bytes < lay.total) {
        set_error("workspace too small: need " + std::to_string(lay.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    const Grids g = make_grids(c, n, A->nnz, false, S != nullptr);
    CgArgs<double> a{};
    a.n = (int)n;
    a.n_cols = A->n_cols;
    a.nnz = A->nnz;
    a.rp = A->row_ptr;
    a.ci = A->col_idx;
    a.val = A->val;
    a.b = b;
    a.x = x;
    a.r = reinterpret_cast<double *>(w + lay.r);
    a.p = reinterpret_cast<double *>(w + lay.p);
    a.q = reinterpret_cast<double *>(w + lay.q);
    a.z = reinterpret_cast<double *>(w + lay.z);
    a.dinv = jac ? reinterpret_cast<double *>(w + lay.dinv) : nullptr;
    a.partials = reinterpret_cast<double *>(w + lay.partials);
    a.st = reinterpret_cast<CgState *>(w + lay.state);
    a.coef = reinterpret_cast<double *>(w + lay.coef);
    if (S) {
        a.sell_sp = S->slice_ptr;
        a.sell_col = S->col;
        a.sell_val = S->val;
    }
    bind_grids(g, a, w + lay.tpart);

    const int maxit = o->maxit > 0 ? o->maxit : (int)std::min<int64_t>(n > 0 ? n : 1, 0x7fffffff);
    const double rtol2 = o->rtol * o->rtol;

    hipStream_t s = c->own_stream;
    int rc = begin_solve(c, s);
    if (rc) return rc;
    hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, s, a.st, maxit);

    bool small = n <= kResN;
    CgState hs{};
    float ms = 0.0f;
    if (small) {
        launch_resident(jac, s, a, rtol2);
        CGX_HIP_CHECK(hipGetLastError());
        if (!o->true_residual) {
            rc = finish_solve(c, s, a.st, hs, ms);
            if (rc) return rc;
        } else {
            CGX_HIP_CHECK(
                hipMemcpyAsync(c->host_state, a.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            CGX_HIP_CHECK(hipStreamSynchronize(s));
            hs = *c->host_state;
        }
        if (hs.status == kStatusRetry) {  // a row does not fit: phase kernels
            small = false;
            hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, s, a.st, maxit);
        }
    }
    if (!small) {
        launch_init(g, jac, s, a, rtol2);
        CGX_HIP_CHECK(hipGetLastError());
        if (o->profile) {
            // Phase kernels launched one by one (no graph), back to back in
            // windows of kProfWindow iterations, with events around each
            // phase: the first interval is the SpMV kernel alone, the second
            // the p.q reduction (if any) and the update, the third the p
            // update.  Only iterations that ran all phases are averaged.
            double tot[3] = {0.0, 0.0, 0.0};
            int counted = 0;
            int iters_before = 0;
            for (int64_t base = 0; base < (int64_t)maxit + 1; base += kProfWindow) {
                const int cnt = (int)std::min<int64_t>(kProfWindow, (int64_t)maxit + 1 - base);
                for (int i = 0; i < cnt; ++i) {
                    hipEvent_t *e = c->ev_phase + 4 * i;
                    CGX_HIP_CHECK(hipEventRecord(e[0], s));
                    launch_spmv_kernel<double>(g, s, a);
                    CGX_HIP_CHECK(hipEventRecord(e[1], s));
                    launch_pq_reduce<double>(g, s, a);
                    launch_update_phase<double>(g, jac, s, a);
                    CGX_HIP_CHECK(hipEventRecord(e[2], s));
                    launch_direction_phase<double>(g, jac, s, a);
                    CGX_HIP_CHECK(hipEventRecord(e[3], s));
                }
                CGX_HIP_CHECK(hipMemcpyAsync(c->host_state, a.st, sizeof(CgState),
                                             hipMemcpyDeviceToHost, s));
                CGX_HIP_CHECK(hipStreamSynchronize(s));
                const bool done = c->host_state->done != 0;
                const int ran = c->host_state->iter - iters_before;
                iters_before = c->host_state->iter;
                // the iteration that set `done` skipped part of its work
                const int full = done ? std::max(0, std::min(cnt, ran - 1)) : cnt;
                for (int i = 0; i < full; ++i)
                    for (int ph = 0; ph < 3; ++ph) {
                        float ms = 0.0f;
                        CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev_phase[4 * i + ph],
                                                          c->ev_phase[4 * i + ph + 1]));
                        tot[ph] += ms;
                    }
                counted += full;
                if (done) break;
            }
            for (int ph = 0; ph < 3; ++ph) st->phase_ms[ph] = counted ? tot[ph] / counted : 0.0;
        } else {
            const double bytes = 12.0 * (double)A->nnz + (jac ? 104.0 : 88.0) * (double)n;
            const int K = replay_iters(o, bytes);
            const int64_t max_replays = (int64_t)maxit / K + 2;
            rc = direct ? launch_until_done(c, K, g, jac, s, a, max_replays)
                        : replay_until_done<double>(c, c->graph64, K, g, jac, s, a, max_replays);
            if (rc) return rc;
        }
    }
    if (o->true_residual) {
        launch_true_residual(g, s, a);
        CGX_HIP_CHECK(hipGetLastError());
    }
    if (!small || o->true_residual) {
        rc = finish_solve(c, s, a.st, hs, ms);
        if (rc) return rc;
    }
    const bool zero_b = hs.bb == 0.0 && hs.status == CGX_OK;
    rc = zero_if_needed(c, s, zero_b, n, x);
    if (rc) return rc;

    st->status = hs.status == CGX_PENDING ? CGX_NOT_CONVERGED : hs.status;
    st->iters = hs.iter;
    st->outer_iters = 0;
    st->path = small ? 1 : 0;
    st->relres = hs.bb > 0.0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
    st->relres_true = -1.0;
    if (o->true_residual) st->relres_true = hs.bb > 0.0 ? std::sqrt(hs.rr_true / hs.bb) : 0.0;
    if (zero_b) st->relres_true = 0.0, st->relres = 0.0;
    st->device_ms = ms;
    rc = fill_kappa(c, s, a.coef, hs.iter, st);
    if (rc) return rc;
    return st->status;
}

int run_mixed(Context *c, const cgx_csr *A, const cgx_sell *S, const double *b, double *x, void *ws,
              size_t ws_bytes, const cgx_opts *o, cgx_stats *st)
{
    const int64_t n = A->n_rows;
    const bool jac = o->precond == CGX_PRECOND_JACOBI;
    const Layout lay = make_layout(n, A->nnz, jac, true);
    if (ws_bytes < lay.total) {
        set_error("workspace too small: need " + std::to_string(lay.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    const Grids g = make_grids(c, n, A->nnz, true, S != nullptr);

    MxArgs m{};
    m.n = (int)n;
    m.n_cols = A->n_cols;
    m.nnz = A->nnz;
    m.rp = A->row_ptr;
    m.ci = A->col_idx;
    m.val = A->val;
    m.b = b;
    m.x = x;
    m.r = reinterpret_cast<double *>(w + lay.r64);
    m.dinv32 = jac ? reinterpret_cast<float *>(w + lay.dinv) : nullptr;
    m.partials = reinterpret_cast<double *>(w + lay.partials);
    m.ost = reinterpret_cast<CgState *>(w + lay.state);

    CgArgs<float> in{};
    in.n = (int)n;
    in.n_cols = A->n_cols;
    in.nnz = A->nnz;
    in.rp = A->row_ptr;
    in.ci = A->col_idx;
    in.val = A->val32;
    in.b = nullptr;
    in.x = reinterpret_cast<float *>(w + lay.d);
    in.r = reinterpret_cast<float *>(w + lay.r);
    in.p = reinterpret_cast<float *>(w + lay.p);
    in.q = reinterpret_cast<float *>(w + lay.q);
    in.z = reinterpret_cast<float *>(w + lay.z);
    in.dinv = m.dinv32;
    in.partials = reinterpret_cast<float *>(w + lay.partials);
    in.st = reinterpret_cast<CgState *>(w + lay.state2);
    in.coef = reinterpret_cast<double *>(w + lay.coef);
    if (S) {
        in.sell_sp = S->slice_ptr;
        in.sell_col = S->col;
        in.sell_val = S->val32;
    }
    bind_grids(g, in, w + lay.tpart);

    // reliable updates: one binary32 CG over all float64 updates (delta: the
    // residual drop that triggers an update); else restarted refinement
    const bool ru = o->precision == CGX_PRECISION_MIXED_RU;
    const int max_outer = o->max_outer > 0 ? o->max_outer : 100;
    const int inner_maxit =
        o->maxit > 0 ? o->maxit : (int)std::min<int64_t>(n > 0 ? n : 1, 0x7fffffff);
    const double tau = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-3;
    const double delta = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-2;
    const double rtol2 = o->rtol * o->rtol;

    hipStream_t s = c->own_stream;
    int rc = begin_solve(c, s);
    if (rc) return rc;
    hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, s, m.ost, max_outer);
    hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, s, in.st, inner_maxit);
    CGX_HIP_CHECK(hipGetLastError());

    const double bytes_in = 8.0 * (double)A->nnz + (jac ? 52.0 : 44.0) * (double)n;
    const int K = replay_iters(o, bytes_in);
    int64_t inner_total = 0, first_inner = 0;
    int status = CGX_NOT_CONVERGED;
    int inner_status = CGX_OK;
    std::vector<std::pair<int, double>> beta_scale;  // (iteration, s' / s) of each update
    for (int step = 0; step <= max_outer + 1; ++step) {
        launch_mx_residual(g, step == 0, jac, s, m, rtol2);
        CGX_HIP_CHECK(hipGetLastError());
        CGX_HIP_CHECK(
            hipMemcpyAsync(c->host_state, m.ost, sizeof(CgState), hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        if (c->host_state->done) {
            status = c->host_state->status;
            break;
        }
        if (ru && inner_status != CGX_OK) {  // the binary32 iteration hit its cap
            status = inner_status;
            break;
        }
        if (!ru || step == 0) {
            if (jac)
                hipLaunchKernelGGL((mx_inner_init_kernel<true>), dim3(g.grid_ew), dim3(kPB), 0, s,
                                   m, in);
            else
                hipLaunchKernelGGL((mx_inner_init_kernel<false>), dim3(g.grid_ew), dim3(kPB), 0, s,
                                   m, in);
            hipLaunchKernelGGL(mx_inner_init_finish_kernel, dim3(1), dim3(kPB), 0, s, m, in,
                               g.grid_ew, (float)(tau * tau), inner_maxit, jac ? 1 : 0,
                               ru ? delta * delta : 0.0);
        } else {
            // reliable update: replace the binary32 residual, keep the direction
            const CgState &ho = *c->host_state;
            beta_scale.emplace_back((int)inner_total - 1, ho.alpha / ho.sigma_prev);
            if (jac)
                hipLaunchKernelGGL((mx_ru_rescale_kernel<true>), dim3(g.grid_ew), dim3(kPB), 0, s,
                                   m, in);
            else
                hipLaunchKernelGGL((mx_ru_rescale_kernel<false>), dim3(g.grid_ew), dim3(kPB), 0, s,
                                   m, in);
            hipLaunchKernelGGL(mx_ru_resume_kernel, dim3(1), dim3(64), 0, s, m, in);
            launch_direction_phase<float>(g, jac, s, in);
        }
        CGX_HIP_CHECK(hipGetLastError());
        const int64_t max_replays = (int64_t)inner_maxit / K + 2;
        rc = replay_until_done<float>(c, c->graph32, K, g, jac, s, in, max_replays);
        if (rc) return rc;
        const CgState inner = *c->host_state;
        if (step == 0) first_inner = inner.iter;
        inner_total = ru ? inner.iter : inner_total + inner.iter;
        inner_status = inner.status;
        if (inner.status == CGX_NONFINITE) {
            status = CGX_NONFINITE;
            break;
        }
        hipLaunchKernelGGL(mx_correct_kernel, dim3(g.grid_ew), dim3(kPB), 0, s, m, in.x);
        CGX_HIP_CHECK(hipGetLastError());
    }
    CgState hs{};
    float ms = 0.0f;
    rc = finish_solve(c, s, m.ost, hs, ms);
    if (rc) return rc;
    const bool zero_b = hs.bb == 0.0 && status == CGX_OK;
    rc = zero_if_needed(c, s, zero_b, n, x);
    if (rc) return rc;

    st->status = status == CGX_PENDING ? CGX_NOT_CONVERGED : status;
    st->iters = (int32_t)std::min<int64_t>(inner_total, 0x7fffffff);
    st->outer_iters = hs.iter;
    st->path = ru ? 6 : 2;
    st->relres = hs.bb > 0.0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
    st->relres_true = st->relres;
    st->device_ms = ms;
    rc = fill_kappa(c, s, in.coef, ru ? inner_total : first_inner, st, &beta_scale);
    if (rc) return rc;
    return st->status;
}

}  // namespace

// Sturm count: eigenvalues of the symmetric tridiagonal (diagonal d,
// off-diagonal squares e2) below x.
// The Sturm counts at NX points at once: the NX recurrences are independent,
// so their divisions overlap instead of waiting on one another.
template <int NX>
static void sturm_below_n(const double *d, const double *e2, int k, const double (&x)[NX],
                          double pivmin, int (&c)[NX])
{
    double q[NX];
    for (int t = 0; t < NX; ++t) {
        c[t] = 0;
        q[t] = d[0] - x[t];
    }
    for (int i = 0;; ++i) {
        for (int t = 0; t < NX; ++t) {
            if (std::fabs(q[t]) < pivmin) q[t] = -pivmin;
            if (q[t] < 0.0) ++c[t];
        }
        if (i + 1 == k) break;
        const double di = d[i + 1], ei = e2[i];
        for (int t = 0; t < NX; ++t) q[t] = di - x[t] - ei / q[t];
    }
}

bool lanczos_extremes_ws(const double *coef, int k, double *work, double &lo, double &hi)
{
    if (k <= 0) return false;
    // T[j][j] = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T[j][j+1]^2 = beta_j / alpha_j^2
    double *d = work, *e2 = work + k, *e = work + 2 * (size_t)k;
    for (int j = 0; j < k; ++j) {
        const double al = coef[2 * j];
        if (!std::isfinite(al) || !(al > 0.0)) return false;
        d[j] = 1.0 / al;
        if (j > 0) d[j] += coef[2 * (j - 1) + 1] / coef[2 * (j - 1)];
        if (j + 1 < k) {
            const double be = coef[2 * j + 1];
            if (!std::isfinite(be) || be < 0.0) return false;
            e2[j] = be / (al * al);
            e[j] = std::sqrt(e2[j]);
        }
    }
    // Gershgorin interval, then bisection on the Sturm count for the two ends
    double g0 = HUGE_VAL, g1 = -HUGE_VAL, emax2 = 0.0;
    for (int j = 0; j < k; ++j) {
        const double r = (j > 0 ? e[j - 1] : 0.0) + (j + 1 < k ? e[j] : 0.0);
        g0 = std::min(g0, d[j] - r);
        g1 = std::max(g1, d[j] + r);
        if (j + 1 < k) emax2 = std::max(emax2, e2[j]);
    }
    if (!std::isfinite(g0) || !std::isfinite(g1)) return false;
    const double span = std::max(std::fabs(g0), std::fabs(g1));
    const double pivmin = std::max(1e-300, 1e-290 * std::max(1.0, emax2));
    g0 -= 1e-15 * span + pivmin;
    g1 += 1e-15 * span + pivmin;
    // Both ends at once by quadrisection: each pass counts at the quarter
    // points of the two intervals [a, b] (Sturm count below a < target <=
    // count below b, target 1 for the smallest Ritz value, k for the
    // largest) and keeps the quarter holding the target.
    double a[2] = {g0, g0}, b[2] = {g1, g1};
    const int target[2] = {1, k};
    bool done[2] = {false, false};
    for (int pass = 0; pass < 200 && !(done[0] && done[1]); ++pass) {
        double x[6];
        for (int t = 0; t < 2; ++t)
            for (int i = 0; i < 3; ++i) x[3 * t + i] = a[t] + (b[t] - a[t]) * (0.25 * (i + 1));
        int c[6];
        sturm_below_n<6>(d, e2, k, x, pivmin, c);
        for (int t = 0; t < 2; ++t) {
            if (done[t]) continue;
            int i = 0;
            while (i < 3 && c[3 * t + i] < target[t]) ++i;
            const double na = i > 0 ? x[3 * t + i - 1] : a[t];
            const double nb = i < 3 ? x[3 * t + i] : b[t];
            if (!(na > a[t]) && !(nb < b[t])) {  // the quarter points no longer split it
                done[t] = true;
                continue;
            }
            a[t] = na;
            b[t] = nb;
            if (b[t] - a[t] <= 2e-16 * std::max(std::fabs(a[t]), std::fabs(b[t]))) done[t] = true;
        }
    }
    lo = 0.5 * (a[0] + b[0]);
    hi = 0.5 * (a[1] + b[1]);
    return std::isfinite(lo) && std::isfinite(hi);
}

bool lanczos_extremes(const double *coef, int k, double &lo, double &hi)
{
    if (k <= 0) return false;
    std::vector<double> work(3 * (size_t)k);
    return lanczos_extremes_ws(coef, k, work.data(), lo, hi);
}

size_t cg_workspace_bytes(int64_t n, int64_t nnz, const cgx_opts *o)
{
    if (n < 0) return 0;
    const bool jac = o && o->precond == CGX_PRECOND_JACOBI;
    const bool mixed = o && o->precision != CGX_PRECISION_FP64;
    return make_layout(n, nnz, jac, mixed).total;
}

int static_scratch_address(int device, void **out)
{
    static std::mutex mu;
    static std::map<int, void *> addr;  // device -> address of its copy of `scratch`
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *p = nullptr;
        CGX_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        it = addr.emplace(device, p).first;
    }
    *out = it->second;
    return CGX_OK;
}

int run_cg_noalloc(Context *c, const cgx_csr *A, const double *b, double *x, const cgx_opts *o,
                   cgx_stats *st)
{
    if (c->static_ws == nullptr) {
        set_error("static scratch not available on this device");
        return CGX_EHIP;
    }
    const size_t need = cg_workspace_bytes(A->n_rows, A->nnz, o);
    if (need > kStaticScratchBytes) {
        set_error("system needs " + std::to_string(need) +
                  " bytes of workspace; the static scratch of cgx_cg_solve_noalloc holds " +
                  std::to_string(kStaticScratchBytes));
        return CGX_ENOMEM;
    }
    return run_fp64(c, A, nullptr, b, x, c->static_ws, kStaticScratchBytes, o, st, true);
}

int run_cg(Context *c, const cgx_csr *A, const cgx_sell *S, const double *b, double *x, void *ws,
           size_t ws_bytes, const cgx_opts *o, cgx_stats *st)
{
    if (o->precision != CGX_PRECISION_FP64) return run_mixed(c, A, S, b, x, ws, ws_bytes, o, st);
    return run_fp64(c, A, S, b, x, ws, ws_bytes, o, st);
}

}  // namespace cgx
