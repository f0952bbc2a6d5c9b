// Conjugate gradient (the paper's Section 5.3: classical CG, here with an
// optional Jacobi preconditioner) on gfx950.
//
// Each iteration is three kernels whose scalars never leave the GPU:
//   (1) q = A p fused with p.q; the last workgroup forms alpha = rho / p.q
//   (2) x += alpha p, r -= alpha q, [z = D^-1 r], r.r [, r.z]; the last
//       workgroup applies the stopping test and forms beta = rho' / rho
//   (3) p = z + beta p
// K iterations are captured once into a HIP graph and replayed; the host
// reads one status word per replay.  After convergence the remaining kernels
// of a replay see `done` and return at once.  Systems of at most kSmallN rows
// run the whole solve inside one 1024-thread workgroup instead (one launch,
// workgroup barriers between phases): at that size the cost is launches and
// grid synchronisation, not bandwidth.
#include <cmath>

#include "cgx_device.h"

namespace cgx {
namespace {

constexpr int kRowsPerGroup = 4;
constexpr int kBlocksPerCu = 8;
constexpr int kMaxPhaseBlocks = 4096;
constexpr int kSmallBlock = 1024;
constexpr int kSmallRows = 2;
constexpr int64_t kSmallN = 16384;

struct CgArgs {
    int n;
    int n_cols;
    int64_t nnz;
    const int32_t *rp;
    const int32_t *ci;
    const double *val;
    const double *b;
    double *x;
    double *r;
    double *p;
    double *q;
    double *z;     // == r without preconditioner
    double *dinv;  // nullptr without preconditioner
    double *partials;
    CgState *st;
    int tiles_per_block;  // SpMV phases: row tiles per workgroup
};

__device__ __forceinline__ int load_flag(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void cg_state_init_kernel(CgState *st, int maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        CgState s = {};
        s.maxit = maxit;
        s.status = CGX_PENDING;
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
    if (load_flag(&st->bad))
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

// Status after p.q of an iteration; forms alpha.
__device__ void finish_pq(CgState *st, double pq)
{
    st->pq = pq;
    if (!isfinite(pq)) {
        st->status = CGX_NONFINITE;
        st->done = 1;
    } else if (!(pq > 0.0)) {
        st->status = CGX_BREAKDOWN;
        st->done = 1;
    } else {
        st->alpha = st->rho / pq;
    }
}

// Status after the update of an iteration; forms beta.
__device__ void finish_update(CgState *st, double rr, double rz)
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
    } else {
        st->status = status;
        st->done = 1;
    }
}

// Lane 0 of a row group: residual, preconditioner and direction of a row.
template <bool kJac>
__device__ __forceinline__ void init_row(const CgArgs &a, int row, double ax, double diag,
                                         double (&part)[3])
{
    const double bi = a.b[row];
    const double ri = bi - ax;
    double zi = ri;
    a.r[row] = ri;
    if (kJac) {
        double d = diag;
        if (!(d > 0.0)) {
            atomicOr(&a.st->bad, 1);
            __threadfence();
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

// ------------------------------------------------ phase kernels (large n) --

template <int L, bool kJac>
__global__ __launch_bounds__(kBlock) void cg_init_kernel(CgArgs a, double rtol2)
{
    constexpr int R = kRowsPerGroup, RPB = (kBlock / L) * R;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ntiles = (a.n + RPB - 1) / RPB;
    const int t0 = lb * a.tiles_per_block;
    const int t1 = min(t0 + a.tiles_per_block, ntiles);
    double part[3] = {0.0, 0.0, 0.0};
    for (int t = t0; t < t1; ++t) {
        double acc[R], dg[R];
        int rows[R];
        vector_rows<L, R, kBlock, double, kJac>(t * RPB, a.n, a.n_cols, a.nnz, a.rp, a.ci, a.val,
                                                a.x, acc, dg, rows);
        if (threadIdx.x % L == 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (rows[r] < a.n) init_row<kJac>(a, rows[r], acc[r], dg[r], part);
    }
    if (grid_sum<3, kBlock>(part, a.partials, &a.st->counter[0]) && threadIdx.x == 0)
        finish_init(a.st, part[0], part[1], part[2], rtol2, kJac);
}

template <int L>
__global__ __launch_bounds__(kBlock) void cg_spmv_kernel(CgArgs a)
{
    if (a.st->done) return;
    constexpr int R = kRowsPerGroup, RPB = (kBlock / L) * R;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ntiles = (a.n + RPB - 1) / RPB;
    const int t0 = lb * a.tiles_per_block;
    const int t1 = min(t0 + a.tiles_per_block, ntiles);
    double part[1] = {0.0};
    for (int t = t0; t < t1; ++t) {
        double acc[R], dg[R];
        int rows[R];
        vector_rows<L, R, kBlock, double, false>(t * RPB, a.n, a.n_cols, a.nnz, a.rp, a.ci, a.val,
                                                 a.p, acc, dg, rows);
        if (threadIdx.x % L == 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (rows[r] < a.n) {
                    a.q[rows[r]] = acc[r];
                    part[0] += a.p[rows[r]] * acc[r];
                }
    }
    if (grid_sum<1, kBlock>(part, a.partials, &a.st->counter[1]) && threadIdx.x == 0)
        finish_pq(a.st, part[0]);
}

template <bool kJac>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(CgArgs a)
{
    if (a.st->done) return;
    const double alpha = a.st->alpha;
    double part[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
#pragma unroll 4
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += stride) {
        const double xi = __builtin_fma(alpha, a.p[i], a.x[i]);
        const double ri = __builtin_fma(-alpha, a.q[i], a.r[i]);
        a.x[i] = xi;
        a.r[i] = ri;
        part[0] += ri * ri;
        if (kJac) {
            const double zi = a.dinv[i] * ri;
            a.z[i] = zi;
            part[1] += ri * zi;
        }
    }
    if (grid_sum<2, kBlock>(part, a.partials, &a.st->counter[2]) && threadIdx.x == 0)
        finish_update(a.st, part[0], kJac ? part[1] : part[0]);
}

__global__ __launch_bounds__(kBlock) void cg_direction_kernel(CgArgs a)
{
    if (a.st->done) return;
    const double beta = a.st->beta;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
#pragma unroll 4
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += stride)
        a.p[i] = __builtin_fma(beta, a.p[i], a.z[i]);
}

// ||b - A x||^2 into st->rr_true.
template <int L>
__global__ __launch_bounds__(kBlock) void cg_true_residual_kernel(CgArgs a)
{
    constexpr int R = kRowsPerGroup, RPB = (kBlock / L) * R;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ntiles = (a.n + RPB - 1) / RPB;
    const int t0 = lb * a.tiles_per_block;
    const int t1 = min(t0 + a.tiles_per_block, ntiles);
    double part[1] = {0.0};
    for (int t = t0; t < t1; ++t) {
        double acc[R], dg[R];
        int rows[R];
        vector_rows<L, R, kBlock, double, false>(t * RPB, a.n, a.n_cols, a.nnz, a.rp, a.ci, a.val,
                                                 a.x, acc, dg, rows);
        if (threadIdx.x % L == 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (rows[r] < a.n) {
                    const double d = a.b[rows[r]] - acc[r];
                    part[0] += d * d;
                }
    }
    if (grid_sum<1, kBlock>(part, a.partials, &a.st->counter[3]) && threadIdx.x == 0)
        a.st->rr_true = part[0];
}

__global__ __launch_bounds__(kBlock) void zero_kernel(int64_t n, double *x)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// ------------------------------------------- single-workgroup solve (small n) --

template <int L, bool kJac>
__global__ __launch_bounds__(kSmallBlock) void cg_small_kernel(CgArgs a, double rtol2)
{
    constexpr int BS = kSmallBlock, R = kSmallRows, RPB = (BS / L) * R;
    __shared__ double red[3 * (BS / kWave)];
    __shared__ double sh_alpha, sh_beta;
    __shared__ int sh_done;
    CgState *st = a.st;
    const int n = a.n;

    double p3[3] = {0.0, 0.0, 0.0};
    for (int row0 = 0; row0 < n; row0 += RPB) {
        double acc[R], dg[R];
        int rows[R];
        vector_rows<L, R, BS, double, kJac>(row0, n, a.n_cols, a.nnz, a.rp, a.ci, a.val, a.x, acc,
                                            dg, rows);
        if (threadIdx.x % L == 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (rows[r] < n) init_row<kJac>(a, rows[r], acc[r], dg[r], p3);
    }
    block_sum<3, BS>(p3, red);
    if (threadIdx.x == 0) {
        finish_init(st, p3[0], p3[1], p3[2], rtol2, kJac);
        sh_done = st->done;
    }
    __syncthreads();

    while (!sh_done) {
        // (1) q = A p, p.q
        double p1[1] = {0.0};
        for (int row0 = 0; row0 < n; row0 += RPB) {
            double acc[R], dg[R];
            int rows[R];
            vector_rows<L, R, BS, double, false>(row0, n, a.n_cols, a.nnz, a.rp, a.ci, a.val, a.p,
                                                 acc, dg, rows);
            if (threadIdx.x % L == 0)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (rows[r] < n) {
                        a.q[rows[r]] = acc[r];
                        p1[0] += a.p[rows[r]] * acc[r];
                    }
        }
        block_sum<1, BS>(p1, red);
        if (threadIdx.x == 0) {
            finish_pq(st, p1[0]);
            sh_done = st->done;
            sh_alpha = st->alpha;
        }
        __syncthreads();
        if (sh_done) break;
        // (2) x, r, z updates and r.r, r.z
        const double alpha = sh_alpha;
        double p2[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += BS) {
            const double xi = __builtin_fma(alpha, a.p[i], a.x[i]);
            const double ri = __builtin_fma(-alpha, a.q[i], a.r[i]);
            a.x[i] = xi;
            a.r[i] = ri;
            p2[0] += ri * ri;
            if (kJac) {
                const double zi = a.dinv[i] * ri;
                a.z[i] = zi;
                p2[1] += ri * zi;
            }
        }
        block_sum<2, BS>(p2, red);
        if (threadIdx.x == 0) {
            finish_update(st, p2[0], kJac ? p2[1] : p2[0]);
            sh_done = st->done;
            sh_beta = st->beta;
        }
        __syncthreads();
        if (sh_done) break;
        // (3) p = z + beta p
        const double beta = sh_beta;
        for (int i = threadIdx.x; i < n; i += BS) a.p[i] = __builtin_fma(beta, a.p[i], a.z[i]);
        __syncthreads();
    }
}

// ----------------------------------------------------------------- host --

struct Layout {
    size_t state, r, p, q, z, dinv, partials, total;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout_fp64(int64_t n, bool jac)
{
    Layout L{};
    size_t off = 0;
    const size_t vec = align_up((size_t)n * sizeof(double));
    L.state = off;
    off += align_up(sizeof(CgState));
    L.r = off;
    off += vec;
    L.p = off;
    off += vec;
    L.q = off;
    off += vec;
    L.z = L.r;
    L.dinv = 0;
    if (jac) {
        L.z = off;
        off += vec;
        L.dinv = off;
        off += vec;
    }
    L.partials = off;
    off += align_up((size_t)3 * kMaxPhaseBlocks * sizeof(double));
    L.total = off;
    return L;
}

#define CGX_LANE_SWITCH(L, EXPR_T)                                                       \
    switch (L) {                                                                         \
        case 2: EXPR_T(2); break;                                                        \
        case 4: EXPR_T(4); break;                                                        \
        case 8: EXPR_T(8); break;                                                        \
        case 16: EXPR_T(16); break;                                                      \
        case 32: EXPR_T(32); break;                                                      \
        default: EXPR_T(64); break;                                                      \
    }

void launch_init(int L, bool jac, int grid, hipStream_t s, const CgArgs &a, double rtol2)
{
#define CGX_INIT(LL)                                                                        \
    if (jac)                                                                                \
        hipLaunchKernelGGL((cg_init_kernel<LL, true>), dim3(grid), dim3(kBlock), 0, s, a,    \
                           rtol2);                                                          \
    else                                                                                    \
        hipLaunchKernelGGL((cg_init_kernel<LL, false>), dim3(grid), dim3(kBlock), 0, s, a, rtol2)
    CGX_LANE_SWITCH(L, CGX_INIT)
#undef CGX_INIT
}

void launch_spmv_phase(int L, int grid, hipStream_t s, const CgArgs &a)
{
#define CGX_SP(LL) hipLaunchKernelGGL((cg_spmv_kernel<LL>), dim3(grid), dim3(kBlock), 0, s, a)
    CGX_LANE_SWITCH(L, CGX_SP)
#undef CGX_SP
}

void launch_true_residual(int L, int grid, hipStream_t s, const CgArgs &a)
{
#define CGX_TR(LL) \
    hipLaunchKernelGGL((cg_true_residual_kernel<LL>), dim3(grid), dim3(kBlock), 0, s, a)
    CGX_LANE_SWITCH(L, CGX_TR)
#undef CGX_TR
}

void launch_small(int L, bool jac, hipStream_t s, const CgArgs &a, double rtol2)
{
#define CGX_SM(LL)                                                                            \
    if (jac)                                                                                  \
        hipLaunchKernelGGL((cg_small_kernel<LL, true>), dim3(1), dim3(kSmallBlock), 0, s, a,   \
                           rtol2);                                                            \
    else                                                                                      \
        hipLaunchKernelGGL((cg_small_kernel<LL, false>), dim3(1), dim3(kSmallBlock), 0, s, a, \
                           rtol2)
    CGX_LANE_SWITCH(L, CGX_SM)
#undef CGX_SM
}

void launch_iteration(int L, bool jac, int grid_sp, int grid_ew, hipStream_t s, const CgArgs &a)
{
    launch_spmv_phase(L, grid_sp, s, a);
    if (jac)
        hipLaunchKernelGGL((cg_update_kernel<true>), dim3(grid_ew), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((cg_update_kernel<false>), dim3(grid_ew), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(cg_direction_kernel, dim3(grid_ew), dim3(kBlock), 0, s, a);
}

}  // namespace

size_t cg_workspace_bytes(int64_t n, int64_t /*nnz*/, const cgx_opts *o)
{
    if (n < 0) return 0;
    const bool jac = o && o->precond == CGX_PRECOND_JACOBI;
    return layout_fp64(n, jac).total;
}

int run_cg(Context *c, const cgx_csr *A, const double *b, double *x, void *ws, size_t ws_bytes,
           const cgx_opts *o, cgx_stats *st)
{
    const int64_t n = A->n_rows;
    const bool jac = o->precond == CGX_PRECOND_JACOBI;
    const Layout lay = layout_fp64(n, jac);
    if (ws_bytes < lay.total) {
        set_error("workspace too small: need " + std::to_string(lay.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    CgArgs a{};
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

    const int maxit = o->maxit > 0 ? o->maxit : (int)std::min<int64_t>(n > 0 ? n : 1, 0x7fffffff);
    const double rtol2 = o->rtol * o->rtol;
    const int L = lanes_per_row(n, A->nnz);
    const int RPB = (kBlock / L) * kRowsPerGroup;
    const int64_t ntiles = (n + RPB - 1) / RPB;
    int grid_sp = c->num_cu * kBlocksPerCu;
    if (grid_sp > kMaxPhaseBlocks) grid_sp = kMaxPhaseBlocks;
    if (grid_sp > ntiles) grid_sp = (int)(ntiles > 0 ? ntiles : 1);
    a.tiles_per_block = (int)((ntiles + grid_sp - 1) / grid_sp);
    int grid_ew = c->num_cu * kBlocksPerCu;
    if (grid_ew > kMaxPhaseBlocks) grid_ew = kMaxPhaseBlocks;
    const int64_t ew_need = (n + kBlock - 1) / kBlock;
    if (grid_ew > ew_need) grid_ew = (int)(ew_need > 0 ? ew_need : 1);

    hipStream_t s = c->own_stream;
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, s, a.st, maxit);

    const bool small = n <= kSmallN;
    if (small) {
        launch_small(L, jac, s, a, rtol2);
        CGX_HIP_CHECK(hipGetLastError());
    } else {
        launch_init(L, jac, grid_sp, s, a, rtol2);
        CGX_HIP_CHECK(hipGetLastError());
        if (o->profile) {
            // One iteration at a time with events around each phase kernel;
            // only iterations that ran all three phases are averaged.
            double tot[3] = {0.0, 0.0, 0.0};
            int counted = 0;
            for (int it = 0; it < maxit + 1; ++it) {
                CGX_HIP_CHECK(hipEventRecord(c->ev_phase[0], s));
                launch_spmv_phase(L, grid_sp, s, a);
                CGX_HIP_CHECK(hipEventRecord(c->ev_phase[1], s));
                if (jac)
                    hipLaunchKernelGGL((cg_update_kernel<true>), dim3(grid_ew), dim3(kBlock), 0, s, a);
                else
                    hipLaunchKernelGGL((cg_update_kernel<false>), dim3(grid_ew), dim3(kBlock), 0, s, a);
                CGX_HIP_CHECK(hipEventRecord(c->ev_phase[2], s));
                hipLaunchKernelGGL(cg_direction_kernel, dim3(grid_ew), dim3(kBlock), 0, s, a);
                CGX_HIP_CHECK(hipEventRecord(c->ev_phase[3], s));
                CGX_HIP_CHECK(hipMemcpyAsync(c->host_state, a.st, sizeof(CgState),
                                             hipMemcpyDeviceToHost, s));
                CGX_HIP_CHECK(hipStreamSynchronize(s));
                if (c->host_state->done) break;
                for (int ph = 0; ph < 3; ++ph) {
                    float ms = 0.0f;
                    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev_phase[ph], c->ev_phase[ph + 1]));
                    tot[ph] += ms;
                }
                ++counted;
            }
            for (int ph = 0; ph < 3; ++ph) st->phase_ms[ph] = counted ? tot[ph] / counted : 0.0;
        } else {
            int K = o->check_every;
            if (K <= 0) {
                // aim at about 2 ms of work between host checks
                const double bytes = 12.0 * (double)A->nnz + (jac ? 104.0 : 88.0) * (double)n;
                const double t_iter = bytes / 4.0e12 + 8.0e-6;
                K = (int)(2.0e-3 / t_iter);
                K = K < 4 ? 4 : (K > 32 ? 32 : K);
            }
            const uint64_t key[12] = {(uint64_t)(uintptr_t)a.rp, (uint64_t)(uintptr_t)a.ci,
                                      (uint64_t)(uintptr_t)a.val, (uint64_t)(uintptr_t)b,
                                      (uint64_t)(uintptr_t)x, (uint64_t)(uintptr_t)ws,
                                      (uint64_t)n, (uint64_t)A->nnz, (uint64_t)A->n_cols,
                                      (uint64_t)(jac ? 1 : 0), (uint64_t)K,
                                      ((uint64_t)grid_sp << 32) | (uint64_t)grid_ew};
            bool hit = c->graph_exec != nullptr;
            for (int i = 0; i < 12 && hit; ++i) hit = c->graph_key[i] == key[i];
            if (!hit) {
                if (c->graph_exec) {
                    (void)hipGraphExecDestroy(c->graph_exec);
                    c->graph_exec = nullptr;
                }
                if (c->graph) {
                    (void)hipGraphDestroy(c->graph);
                    c->graph = nullptr;
                }
                CGX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < K; ++k) launch_iteration(L, jac, grid_sp, grid_ew, s, a);
                hipGraph_t g = nullptr;
                CGX_HIP_CHECK(hipStreamEndCapture(s, &g));
                c->graph = g;
                CGX_HIP_CHECK(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
                for (int i = 0; i < 12; ++i) c->graph_key[i] = key[i];
            }
            // Replays until `done`; maxit bounds the loop since the update kernel
            // sets `done` when the cap is reached.
            const int64_t max_replays = (int64_t)maxit / K + 2;
            for (int64_t rep = 0; rep < max_replays; ++rep) {
                CGX_HIP_CHECK(hipGraphLaunch(c->graph_exec, s));
                CGX_HIP_CHECK(hipMemcpyAsync(c->host_state, a.st, sizeof(CgState),
                                             hipMemcpyDeviceToHost, s));
                CGX_HIP_CHECK(hipStreamSynchronize(s));
                if (c->host_state->done) break;
            }
        }
    }
    if (o->true_residual) {
        launch_true_residual(L, grid_sp, s, a);
        CGX_HIP_CHECK(hipGetLastError());
    }
    CGX_HIP_CHECK(hipEventRecord(c->ev1, s));
    CGX_HIP_CHECK(hipMemcpyAsync(c->host_state, a.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    const CgState hs = *c->host_state;
    if (hs.bb == 0.0 && hs.status == CGX_OK) {
        hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(kBlock), 0, s, n, x);
        CGX_HIP_CHECK(hipGetLastError());
        CGX_HIP_CHECK(hipStreamSynchronize(s));
    }
    float ms = 0.0f;
    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    CGX_HIP_CHECK(hipEventRecord(c->ev_out, s));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_out, 0));

    st->status = hs.status == CGX_PENDING ? CGX_NOT_CONVERGED : hs.status;
    st->iters = hs.iter;
    st->outer_iters = 0;
    st->path = small ? 1 : 0;
    st->relres = hs.bb > 0.0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
    st->relres_true = -1.0;
    if (o->true_residual) st->relres_true = hs.bb > 0.0 ? std::sqrt(hs.rr_true / hs.bb) : 0.0;
    if (hs.bb == 0.0 && hs.status == CGX_OK) st->relres_true = 0.0, st->relres = 0.0;
    st->device_ms = ms;
    return st->status;
}

}  // namespace cgx
