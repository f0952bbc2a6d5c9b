// Batched conjugate gradient: many independent SPD systems, each with up to
// 16 right-hand sides, advanced together (the many-subdomain setting the
// paper's Section 5.3 describes for domain decomposition, where every
// subdomain problem is solved by CG on the GPU).
//
// Layout.  Each system's Krylov vectors are stored interleaved, [n][K] with
// K = the system's right-hand-side count rounded up to a power of two, so the
// SpMM gather p[col][0..K) of one nonzero reads one contiguous segment and
// the matrix is streamed once for all K right-hand sides.
//
// Schedule.  A host-built work table maps every workgroup to one row tile of
// one system; each phase of an iteration is ONE launch over all tiles of all
// systems: (1) SpMM q = A p with per-tile p.q partials, (R1) one workgroup
// per system adds them in tile order and forms alpha per right-hand side,
// (2) x/r/z updates with r.r / r.z partials, (R2) the stopping test and beta,
// (3) p = z + beta p.  A row is served by K * M lanes (lane = m * K + j:
// right-hand side j, nonzero slice m); M is picked per system by the
// autotuner.  Every reduction a system depends on runs over that system's
// own tiles in a fixed order, so a system's iterates are the same bits alone
// or in any batch (given the same schedule).  Converged right-hand sides are
// masked; a system whose right-hand sides are all done is skipped.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "cgx_device.h"

namespace cgx {

struct BSys {
    const int32_t *rp;
    const int32_t *ci;
    const double *val;
    const double *B;  // caller right-hand sides, [nrhs][n]
    double *X;        // caller solutions, [nrhs][n]
    double *x, *r, *p, *q, *z;  // interleaved [n][K]
    double *dinv;     // [n]
    int64_t nnz;
    int n, K, nrhs, M;
    int tile0, ntiles, trows, scal0;
    int n_cols, pad;
};

struct BTile {
    int sys, row0, rows, tile;  // tile = index within the whole table
};

struct BScal {
    double rho, rho_used, alpha, beta, rr, bb, stop2, pq;
    int32_t iter, status, active, pad;
};

struct BArgs {
    const BSys *sys;
    const BTile *tiles;
    BScal *scal;
    int32_t *sys_done;  // per system: all right-hand sides finished
    double *part;       // 3 regions of ntiles * 16
    int64_t part_stride;  // ntiles * 16
    int ntiles;
    int nsys;
    int maxit;
    int jac;
    double rtol2;
};

namespace {

constexpr int kBB = 256;  // threads per workgroup of the batched kernels
constexpr int kMaxK = 16;

__device__ __forceinline__ int clampk(int v, int64_t nnz)
{
    return v < 0 ? 0 : (v > nnz ? (int)nnz : v);
}

// Per-RHS block sum: thread t holds a value for right-hand side t % K; the
// K totals (fixed order) are written to out[0..K) by threads 0..K-1.
__device__ __forceinline__ void block_sum_by_rhs(double v, int K, double *red, double *out)
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int i = threadIdx.x; i < kBB; i += K) s += red[i];
        out[threadIdx.x] = s;
    }
}

// Row sum of one row for right-hand side j over nonzero slice m of M, using
// interleaved vector v ([n][K]); combined over the M slices by butterfly.
// Also returns the diagonal entry (summed the same way; one slice holds it).
__device__ __forceinline__ double row_spmm(const BSys &S, int row, int j, int m, double &diag,
                                           const double *v)
{
    int s = S.rp[row], e = S.rp[row + 1];
    s = clampk(s, S.nnz);
    e = clampk(e, S.nnz);
    if (e < s) e = s;
    double acc = 0.0, dg = 0.0;
    for (int k = s + m; k < e; k += S.M) {
        const int c = S.ci[k];
        const double a = S.val[k];
        if ((unsigned)c < (unsigned)S.n_cols) acc += a * v[(int64_t)c * S.K + j];
        if (c == row) dg = a;
    }
    const int G = S.K * S.M;
    for (int off = S.K; off < G; off <<= 1) {
        acc += __shfl_xor(acc, off);
        dg += __shfl_xor(dg, off);
    }
    diag = dg;
    return acc;
}

// Caller layout -> interleaved x.
__global__ __launch_bounds__(kBB) void batch_in_kernel(BArgs a)
{
    const BTile t = a.tiles[blockIdx.x];
    const BSys S = a.sys[t.sys];
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        S.x[e] = j < S.nrhs ? S.X[(int64_t)j * S.n + row] : 0.0;
    }
}

// r0 = b - A x0, D^-1, z0, p0 and the partials of r.r, r.z, b.b.
__global__ __launch_bounds__(kBB) void batch_init_kernel(BArgs a)
{
    __shared__ double red[kBB];
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    const BSys S = a.sys[t.sys];
    const int G = S.K * S.M, gpw = kWave / G;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
    double prr = 0.0, prz = 0.0, pbb = 0.0;
    for (int row = t.row0 + wave * gpw + grp; row < t.row0 + t.rows; row += (kBB / kWave) * gpw) {
        double dg;
        const double ax = row_spmm(S, row, j, m, dg, S.x);
        if (m == 0) {
            const int64_t e = (int64_t)row * S.K + j;
            const double bi = j < S.nrhs ? S.B[(int64_t)j * S.n + row] : 0.0;
            const double ri = bi - ax;
            double zi = ri;
            S.r[e] = ri;
            if (a.jac) {
                const double d = dg > 0.0 ? dg : 1.0;
                if (!(dg > 0.0)) a.scal[S.scal0 + j].pad = 1;  // same value from every writer
                const double di = 1.0 / d;
                if (j == 0) S.dinv[row] = di;
                zi = di * ri;
                S.z[e] = zi;
            }
            S.p[e] = zi;
            prr += ri * ri;
            prz += ri * zi;
            pbb += bi * bi;
        }
    }
    // lanes with m > 0 hold zeros; the lane of (grp, j, m = 0) is lane % K == j
    double *base = a.part + (int64_t)t.tile * kMaxK;
    block_sum_by_rhs(prr, S.K, red, base);
    block_sum_by_rhs(prz, S.K, red, base + a.part_stride);
    block_sum_by_rhs(pbb, S.K, red, base + 2 * a.part_stride);
}

// Sum of region `reg` partials of system s for right-hand side j (fixed
// order: tile-strided per thread slice, then slices in order).
__device__ __forceinline__ double sys_sum(const BArgs &a, const BSys &S, int reg, double *red)
{
    const int K = S.K;
    const int slice = threadIdx.x / K, j = threadIdx.x % K, nsl = kBB / K;
    double s = 0.0;
    const double *base = a.part + reg * a.part_stride;
    for (int t = S.tile0 + slice; t < S.tile0 + S.ntiles; t += nsl) s += base[(int64_t)t * kMaxK + j];
    __syncthreads();
    red[threadIdx.x] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x < K)
        for (int i = 0; i < nsl; ++i) tot += red[i * K + threadIdx.x];
    return tot;  // valid in threads 0..K-1
}

__global__ __launch_bounds__(kBB) void batch_r0_kernel(BArgs a)
{
    __shared__ double red[kBB];
    const BSys S = a.sys[blockIdx.x];
    const double rr = sys_sum(a, S, 0, red);
    const double rz = sys_sum(a, S, 1, red);
    const double bb = sys_sum(a, S, 2, red);
    __shared__ int any_active;
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    if (threadIdx.x < S.K) {
        const int j = threadIdx.x;
        BScal &c = a.scal[S.scal0 + j];
        const bool badd = c.pad != 0;
        c.rr = rr;
        c.bb = bb;
        c.rho = a.jac ? rz : rr;
        c.stop2 = a.rtol2 * bb;
        c.iter = 0;
        int status = CGX_PENDING;
        if (j >= S.nrhs)
            status = CGX_OK;
        else if (badd)
            status = CGX_BREAKDOWN;
        else if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz))
            status = CGX_NONFINITE;
        else if (bb == 0.0 || rr <= a.rtol2 * bb)
            status = CGX_OK;
        else if (a.jac && !(rz > 0.0))
            status = CGX_BREAKDOWN;
        c.status = status;
        c.active = status == CGX_PENDING;
        if (c.active) atomicOr(&any_active, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.sys_done[blockIdx.x] = any_active ? 0 : 1;
}

// (1) q = A p for every active system, p.q partials per right-hand side.
__global__ __launch_bounds__(kBB) void batch_spmm_kernel(BArgs a)
{
    __shared__ double red[kBB];
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys]) return;
    const BSys S = a.sys[t.sys];
    const int G = S.K * S.M, gpw = kWave / G;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
    double ppq = 0.0;
    for (int row = t.row0 + wave * gpw + grp; row < t.row0 + t.rows; row += (kBB / kWave) * gpw) {
        double dg;
        const double qv = row_spmm(S, row, j, m, dg, S.p);
        if (m == 0) {
            const int64_t e = (int64_t)row * S.K + j;
            S.q[e] = qv;
            ppq += S.p[e] * qv;
        }
    }
    block_sum_by_rhs(ppq, S.K, red, a.part + (int64_t)t.tile * kMaxK);
}

// (R1) alpha per right-hand side; breakdown / non-finite p.q ends it.
__global__ __launch_bounds__(kBB) void batch_r1_kernel(BArgs a)
{
    __shared__ double red[kBB];
    if (a.sys_done[blockIdx.x]) return;
    const BSys S = a.sys[blockIdx.x];
    const double pq = sys_sum(a, S, 0, red);
    if (threadIdx.x < S.K) {
        BScal &c = a.scal[S.scal0 + threadIdx.x];
        if (c.active) {
            c.pq = pq;
            if (!isfinite(pq) || !(pq > 0.0)) {
                c.status = isfinite(pq) ? CGX_BREAKDOWN : CGX_NONFINITE;
                c.active = 0;
            } else {
                c.alpha = c.rho / pq;
                c.rho_used = c.rho;
                c.iter += 1;
            }
        }
    }
}

// (2) x += alpha p, r -= alpha q, z = D^-1 r for active right-hand sides;
// r.r and r.z partials.
__global__ __launch_bounds__(kBB) void batch_update_kernel(BArgs a)
{
    __shared__ double red[kBB];
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys]) return;
    const BSys S = a.sys[t.sys];
    const int j = threadIdx.x % S.K;  // fixed per thread: K divides kBB
    const BScal c = a.scal[S.scal0 + j];
    double prr = 0.0, prz = 0.0;
    if (c.active) {
        const double alpha = c.alpha;
        const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
            const double xi = __builtin_fma(alpha, S.p[e], S.x[e]);
            const double ri = __builtin_fma(-alpha, S.q[e], S.r[e]);
            S.x[e] = xi;
            S.r[e] = ri;
            prr += ri * ri;
            if (a.jac) {
                const double zi = S.dinv[e / S.K] * ri;
                S.z[e] = zi;
                prz += ri * zi;
            }
        }
    }
    double *base = a.part + (int64_t)t.tile * kMaxK;
    block_sum_by_rhs(prr, S.K, red, base + a.part_stride);
    block_sum_by_rhs(prz, S.K, red, base + 2 * a.part_stride);
}

// (R2) stopping test and beta per right-hand side; system-done flag.
__global__ __launch_bounds__(kBB) void batch_r2_kernel(BArgs a)
{
    __shared__ double red[kBB];
    __shared__ int any_active;
    if (a.sys_done[blockIdx.x]) return;
    const BSys S = a.sys[blockIdx.x];
    const double rr = sys_sum(a, S, 1, red);
    const double rz0 = sys_sum(a, S, 2, red);
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    if (threadIdx.x < S.K) {
        BScal &c = a.scal[S.scal0 + threadIdx.x];
        if (c.active) {
            const double rz = a.jac ? rz0 : rr;
            c.rr = rr;
            int status = CGX_PENDING;
            if (!isfinite(rr) || !isfinite(rz))
                status = CGX_NONFINITE;
            else if (rr <= c.stop2)
                status = CGX_OK;
            else if (!(rz > 0.0))
                status = CGX_BREAKDOWN;
            else if (c.iter >= a.maxit)
                status = CGX_NOT_CONVERGED;
            if (status == CGX_PENDING) {
                c.beta = rz / c.rho_used;
                c.rho = rz;
                atomicOr(&any_active, 1);
            } else {
                c.status = status;
                c.active = 0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && !any_active) a.sys_done[blockIdx.x] = 1;
}

// (3) p = z + beta p for active right-hand sides.
__global__ __launch_bounds__(kBB) void batch_direction_kernel(BArgs a)
{
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const BTile t = a.tiles[w];
    if (a.sys_done[t.sys]) return;
    const BSys S = a.sys[t.sys];
    const int j = threadIdx.x % S.K;
    const BScal c = a.scal[S.scal0 + j];
    if (!c.active) return;
    const double beta = c.beta;
    const double *z = a.jac ? S.z : S.r;
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) S.p[e] = __builtin_fma(beta, S.p[e], z[e]);
}

// Interleaved x -> caller layout (x = 0 where b = 0).
__global__ __launch_bounds__(kBB) void batch_out_kernel(BArgs a)
{
    const BTile t = a.tiles[blockIdx.x];
    const BSys S = a.sys[t.sys];
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        if (j < S.nrhs) {
            const BScal &c = a.scal[S.scal0 + j];
            S.X[(int64_t)j * S.n + row] = (c.bb == 0.0 && c.status == CGX_OK) ? 0.0 : S.x[e];
        }
    }
}

// ----------------------------------------------------------------- host --

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int pad_k(int nrhs)
{
    int K = 1;
    while (K < nrhs) K *= 2;
    return K;
}

int tile_rows_for(int K) { return std::max(16, 2048 / K); }

struct Plan {
    std::vector<BSys> sys;
    std::vector<BTile> tiles;
    size_t off_sys = 0, off_tiles = 0, off_scal = 0, off_done = 0, off_part = 0, off_vec = 0;
    size_t total = 0;
    int64_t nscal = 0;
};

// Candidate slice counts M for K right-hand sides: groups of K * M lanes in
// {8, 16, 32, 64} (at least one lane per right-hand side).
std::vector<int> m_candidates(int K)
{
    std::vector<int> out;
    for (int G = 8; G <= 64; G *= 2)
        if (G >= K) out.push_back(G / K);
    if (out.empty()) out.push_back(1);
    return out;
}

// Deterministic default when no tuning has been done: about one lane per
// nonzero of a row over all K right-hand sides, capped at 64 lanes.
int default_m(int K, double mean_row)
{
    int best = 1;
    for (int M : m_candidates(K))
        if (K * M <= std::max(8.0, mean_row * (K >= 8 ? 0.5 : 1.0))) best = M;
    return best;
}

// Layout of the workspace and the host copies of the device tables.
int build_plan(int32_t nsys, const cgx_system *in, const int *Ms, Plan &P)
{
    P.sys.assign(nsys, BSys{});
    P.tiles.clear();
    int64_t scal = 0;
    size_t vec_bytes = 0;
    for (int s = 0; s < nsys; ++s) {
        const cgx_system &q = in[s];
        BSys &S = P.sys[s];
        S.n = q.A.n_rows;
        S.n_cols = q.A.n_cols;
        S.nnz = q.A.nnz;
        S.nrhs = q.nrhs;
        S.K = pad_k(q.nrhs);
        S.M = Ms ? Ms[s] : default_m(S.K, S.n ? (double)S.nnz / S.n : 1.0);
        S.trows = tile_rows_for(S.K);
        S.scal0 = (int)scal;
        scal += S.K;
        S.tile0 = (int)P.tiles.size();
        for (int r0 = 0; r0 < S.n; r0 += S.trows) {
            BTile t{};
            t.sys = s;
            t.row0 = r0;
            t.rows = std::min(S.trows, S.n - r0);
            t.tile = (int)P.tiles.size();
            P.tiles.push_back(t);
        }
        S.ntiles = (int)P.tiles.size() - S.tile0;
        vec_bytes += 5 * align256((size_t)S.n * S.K * sizeof(double)) +
                     align256((size_t)S.n * sizeof(double));
    }
    if (P.tiles.size() > 0x7fffffff) return CGX_EINVAL;
    P.nscal = scal;
    size_t off = 0;
    P.off_sys = off;
    off += align256(sizeof(BSys) * nsys);
    P.off_tiles = off;
    off += align256(sizeof(BTile) * std::max<size_t>(P.tiles.size(), 1));
    P.off_scal = off;
    off += align256(sizeof(BScal) * std::max<int64_t>(scal, 1));
    P.off_done = off;
    off += align256(sizeof(int32_t) * nsys);
    P.off_part = off;
    off += align256((size_t)3 * std::max<size_t>(P.tiles.size(), 1) * kMaxK * sizeof(double));
    P.off_vec = off;
    off += vec_bytes;
    P.total = off;
    return CGX_OK;
}

void bind_pointers(Plan &P, int32_t nsys, const cgx_system *in, char *ws)
{
    size_t off = P.off_vec;
    for (int s = 0; s < nsys; ++s) {
        BSys &S = P.sys[s];
        S.rp = in[s].A.row_ptr;
        S.ci = in[s].A.col_idx;
        S.val = in[s].A.val;
        S.B = in[s].B;
        S.X = in[s].X;
        const size_t vb = align256((size_t)S.n * S.K * sizeof(double));
        double **vecs[5] = {&S.x, &S.r, &S.p, &S.q, &S.z};
        for (double **v : vecs) {
            *v = reinterpret_cast<double *>(ws + off);
            off += vb;
        }
        S.dinv = reinterpret_cast<double *>(ws + off);
        off += align256((size_t)S.n * sizeof(double));
    }
}

BArgs make_args(const Plan &P, char *ws, int maxit, bool jac, double rtol)
{
    BArgs a{};
    a.sys = reinterpret_cast<const BSys *>(ws + P.off_sys);
    a.tiles = reinterpret_cast<const BTile *>(ws + P.off_tiles);
    a.scal = reinterpret_cast<BScal *>(ws + P.off_scal);
    a.sys_done = reinterpret_cast<int32_t *>(ws + P.off_done);
    a.part = reinterpret_cast<double *>(ws + P.off_part);
    a.ntiles = (int)P.tiles.size();
    a.part_stride = (int64_t)std::max<size_t>(P.tiles.size(), 1) * kMaxK;
    a.nsys = (int)P.sys.size();
    a.maxit = maxit;
    a.jac = jac ? 1 : 0;
    a.rtol2 = rtol * rtol;
    return a;
}

void launch_batch_iteration(const BArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(batch_spmm_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_r1_kernel, dim3(a.nsys), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_update_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_r2_kernel, dim3(a.nsys), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_direction_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
}

__global__ void batch_scal_init_kernel(BScal *scal, int64_t n, int32_t *done, int nsys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) scal[i] = BScal{};
    if (i < nsys) done[i] = 0;
}

// Key of a system's shape class for the autotuner cache.
std::tuple<int, int, int> shape_key(const BSys &S)
{
    const int mean = S.n ? (int)std::lround((double)S.nnz / S.n) : 0;
    int lg = 0;
    while ((1 << (lg + 1)) <= S.n) ++lg;
    return std::make_tuple(S.K, mean, lg);
}

}  // namespace

// Autotuner: per shape class, time the SpMM phase of one representative
// system for every slice count M and keep the fastest.
int batch_autotune(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                   std::vector<int> &Ms)
{
    Ms.assign(nsys, 0);
    for (int s = 0; s < nsys; ++s) {
        const int K = pad_k(in[s].nrhs);
        const double mean = in[s].A.n_rows ? (double)in[s].A.nnz / in[s].A.n_rows : 1.0;
        int lg = 0;
        while ((1 << (lg + 1)) <= in[s].A.n_rows) ++lg;
        const auto key = std::make_tuple(K, (int)std::lround(mean), lg);
        auto it = c->batch_tune.find(key);
        if (it != c->batch_tune.end()) {
            Ms[s] = it->second;
            continue;
        }
        // time this system alone with each candidate
        float best_ms = 1e30f;
        int best_m = default_m(K, mean);
        for (int M : m_candidates(K)) {
            int Mv[1] = {M};
            Plan P;
            if (build_plan(1, &in[s], Mv, P) != CGX_OK || P.total > ws_bytes) continue;
            char *w = static_cast<char *>(ws);
            bind_pointers(P, 1, &in[s], w);
            CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_sys, P.sys.data(), sizeof(BSys),
                                         hipMemcpyHostToDevice, c->own_stream));
            CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_tiles, P.tiles.data(),
                                         sizeof(BTile) * P.tiles.size(), hipMemcpyHostToDevice,
                                         c->own_stream));
            BArgs a = make_args(P, w, 1, false, 0.0);
            hipLaunchKernelGGL(batch_scal_init_kernel, dim3((unsigned)((P.nscal + 255) / 256 + 1)),
                               dim3(256), 0, c->own_stream, a.scal, P.nscal, a.sys_done, 1);
            // p = 0 content is irrelevant for timing; use the workspace as is
            for (int rep = 0; rep < 2; ++rep)
                hipLaunchKernelGGL(batch_spmm_kernel, dim3(a.ntiles), dim3(kBB), 0, c->own_stream,
                                   a);
            CGX_HIP_CHECK(hipEventRecord(c->ev0, c->own_stream));
            for (int rep = 0; rep < 5; ++rep)
                hipLaunchKernelGGL(batch_spmm_kernel, dim3(a.ntiles), dim3(kBB), 0, c->own_stream,
                                   a);
            CGX_HIP_CHECK(hipEventRecord(c->ev1, c->own_stream));
            CGX_HIP_CHECK(hipEventSynchronize(c->ev1));
            float ms = 0.0f;
            CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
            if (ms < best_ms) {
                best_ms = ms;
                best_m = M;
            }
        }
        c->batch_tune[key] = best_m;
        Ms[s] = best_m;
    }
    return CGX_OK;
}

size_t batch_workspace_bytes(int32_t nsys, const cgx_system *in)
{
    Plan P;
    if (build_plan(nsys, in, nullptr, P) != CGX_OK) return 0;
    return P.total;
}

int run_batched(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                const cgx_opts *o, cgx_stats *stats)
{
    std::vector<int> Ms;
    // the workspace of the whole batch is large enough to time any one system
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->own_stream, c->ev_in, 0));
    int rc = batch_autotune(c, nsys, in, ws, ws_bytes, Ms);
    if (rc) return rc;
    Plan P;
    rc = build_plan(nsys, in, Ms.empty() ? nullptr : Ms.data(), P);
    if (rc) {
        set_error("batch too large");
        return rc;
    }
    if (ws_bytes < P.total) {
        set_error("workspace too small: need " + std::to_string(P.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    bind_pointers(P, nsys, in, w);
    hipStream_t s = c->own_stream;
    int64_t max_n = 1;
    for (const BSys &S : P.sys) max_n = std::max<int64_t>(max_n, S.n);
    const int maxit = o->maxit > 0 ? o->maxit : (int)std::min<int64_t>(max_n, 0x7fffffff);
    const bool jac = o->precond == CGX_PRECOND_JACOBI;
    BArgs a = make_args(P, w, maxit, jac, o->rtol);

    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_sys, P.sys.data(), sizeof(BSys) * nsys,
                                 hipMemcpyHostToDevice, s));
    CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_tiles, P.tiles.data(), sizeof(BTile) * P.tiles.size(),
                                 hipMemcpyHostToDevice, s));
    const int64_t init_n = std::max<int64_t>(P.nscal, nsys);
    hipLaunchKernelGGL(batch_scal_init_kernel, dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0,
                       s, a.scal, P.nscal, a.sys_done, nsys);
    hipLaunchKernelGGL(batch_in_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_init_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL(batch_r0_kernel, dim3(nsys), dim3(kBB), 0, s, a);
    CGX_HIP_CHECK(hipGetLastError());

    // iterations per replay: about 2 ms of work between host checks
    double bytes = 0.0;
    for (const BSys &S : P.sys) bytes += 12.0 * S.nnz + 88.0 * S.K * S.n;
    int K = o->check_every;
    if (K <= 0) {
        const double t_iter = bytes / 4.0e12 + 15.0e-6;
        K = (int)(2.0e-3 / t_iter);
        K = K < 2 ? 2 : (K > 32 ? 32 : K);
    }
    uint64_t key[12] = {(uint64_t)(uintptr_t)ws, (uint64_t)nsys, (uint64_t)P.tiles.size(),
                        (uint64_t)K, (uint64_t)jac, (uint64_t)maxit,
                        (uint64_t)std::hash<double>{}(o->rtol), 0, 0, 0, 0, 0};
    for (int i = 0; i < nsys && i < 64; ++i) {
        key[7 + (i % 5)] ^= ((uint64_t)(uintptr_t)in[i].A.row_ptr * 1000003u) ^
                            ((uint64_t)(uintptr_t)in[i].X << 1) ^ ((uint64_t)P.sys[i].M << 7) ^
                            (uint64_t)i;
    }
    GraphSlot &slot = c->graph_batch;
    bool hit = slot.exec != nullptr;
    for (int i = 0; i < 12 && hit; ++i) hit = slot.key[i] == key[i];
    if (!hit) {
        slot.reset();
        CGX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) launch_batch_iteration(a, s);
        hipGraph_t g = nullptr;
        CGX_HIP_CHECK(hipStreamEndCapture(s, &g));
        slot.graph = g;
        CGX_HIP_CHECK(hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0));
        for (int i = 0; i < 12; ++i) slot.key[i] = key[i];
    }
    std::vector<int32_t> done(nsys);
    const int64_t max_replays = (int64_t)maxit / K + 2;
    for (int64_t rep = 0; rep < max_replays; ++rep) {
        CGX_HIP_CHECK(hipGraphLaunch(slot.exec, s));
        CGX_HIP_CHECK(hipMemcpyAsync(done.data(), a.sys_done, sizeof(int32_t) * nsys,
                                     hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        bool all = true;
        for (int32_t d : done) all = all && d;
        if (all) break;
    }
    hipLaunchKernelGGL(batch_out_kernel, dim3(a.ntiles), dim3(kBB), 0, s, a);
    CGX_HIP_CHECK(hipGetLastError());
    CGX_HIP_CHECK(hipEventRecord(c->ev1, s));
    std::vector<BScal> hs(P.nscal);
    CGX_HIP_CHECK(hipMemcpyAsync(hs.data(), a.scal, sizeof(BScal) * P.nscal, hipMemcpyDeviceToHost,
                                 s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.0f;
    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    CGX_HIP_CHECK(hipEventRecord(c->ev_out, s));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_out, 0));

    int worst = CGX_OK;
    int64_t k = 0;
    for (int sidx = 0; sidx < nsys; ++sidx) {
        const BSys &S = P.sys[sidx];
        for (int j = 0; j < S.nrhs; ++j, ++k) {
            const BScal &v = hs[S.scal0 + j];
            cgx_stats &st = stats[k];
            st.status = v.status == CGX_PENDING ? CGX_NOT_CONVERGED : v.status;
            st.iters = v.iter;
            st.outer_iters = 0;
            st.path = 3;
            st.relres = v.bb > 0.0 ? std::sqrt(v.rr / v.bb) : 0.0;
            st.relres_true = -1.0;
            st.device_ms = ms;
            if (st.status != CGX_OK && worst == CGX_OK) worst = st.status;
        }
    }
    return worst;
}

}  // namespace cgx
