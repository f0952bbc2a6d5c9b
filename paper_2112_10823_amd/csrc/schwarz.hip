// Additive Schwarz preconditioning with GPU conjugate-gradient subdomain
// solves (domain decomposition, end of the paper's Section 5.3: the outer
// iteration on the host, every subdomain problem solved by CG on the GPU).
//
// Subdomains.  The rows are cut into n_sub contiguous core blocks
// [floor(i n / S), floor((i+1) n / S)), each extended by `overlap` rows on
// both sides and clipped to [0, n).  overlap <= floor(n / S), so a row lies
// in its own core's subdomain and at most the two neighbouring ones.  The
// local matrix A_i is the principal submatrix of A on the subdomain's rows
// and columns, entries in stored order, columns shifted to start at 0.
//
// Build.  One pass counts each local row's kept entries, a three-kernel
// exclusive scan over all local rows (subdomain by subdomain) gives every
// local row its entry offset, and a second pass writes the per-subdomain row
// pointers (each starting at 0) and copies the entries.
//
// Solve.  Flexible CG on the host: every step is a library kernel (SpMV,
// compensated dots, axpy) or the batched CG solver, which advances all
// subdomain problems together (one work-table launch per phase for all of
// them; B_i is the subdomain's slice of r, read in place).  The local
// solutions are added back in subdomain order by the prolongation kernel.
#include <chrono>
#include <cmath>
#include <vector>

#include "cgx_device.h"

namespace cgx {
namespace {

constexpr int kSB = 256;       // threads per block of the build / vector kernels
constexpr int kScanPer = 16;   // scan elements per thread
constexpr int kScanChunk = kSB * kScanPer;

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Subdomain ranges, one definition for host and device.  Core block i is
// [blk(i), blk(i+1)) with blk(i) = floor(i n / S); with 0 <= o <= floor(n / S)
// only the outer ends need clipping: subdomain i is [blk(i) - o, blk(i+1) + o)
// except lo = 0 for i = 0 and hi = n for i = S - 1, and its rows start at
// local row sub_off(i) = blk(i) + o (2 i - 1) for 0 < i < S (0 for i = 0;
// n + 2 o (S - 1) in total).
__host__ __device__ __forceinline__ int64_t blk(int64_t i, int64_t n, int64_t S) { return i * n / S; }
__host__ __device__ __forceinline__ int64_t sub_lo(int64_t i, int64_t n, int64_t S, int64_t o)
{
    return i == 0 ? 0 : blk(i, n, S) - o;
}
__host__ __device__ __forceinline__ int64_t sub_hi(int64_t i, int64_t n, int64_t S, int64_t o)
{
    return i == S - 1 ? n : blk(i + 1, n, S) + o;
}
__host__ __device__ __forceinline__ int64_t sub_off(int64_t i, int64_t n, int64_t S, int64_t o)
{
    return i == 0 ? 0 : (i == S ? n + 2 * o * (S - 1) : blk(i, n, S) + o * (2 * i - 1));
}

// Subdomain of local row L: the largest i < S with sub_off(i) <= L.
__device__ __forceinline__ int sub_of(int64_t L, int64_t n, int S, int64_t o)
{
    int a = 0, b = S - 1;
    while (a < b) {
        const int m = (a + b + 1) / 2;
        if (sub_off(m, n, S, o) <= L) a = m; else b = m - 1;
    }
    return a;
}

__device__ __forceinline__ void row_range(const int32_t *__restrict__ rp, int64_t nnz, int g,
                                          int &a, int &b)
{
    a = rp[g];
    b = rp[g + 1];
    a = a < 0 ? 0 : (a > nnz ? (int)nnz : a);
    b = b < a ? a : (b > nnz ? (int)nnz : b);
}

// Kept entries of every local row -> cnt[L]; optionally their total.
__global__ __launch_bounds__(kSB) void sub_count_kernel(int64_t local_rows, int n, int S, int o,
                                                        int64_t nnz, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        int64_t *cnt, unsigned long long *total)
{
    const int64_t stride = (int64_t)gridDim.x * kSB;
    unsigned long long mine = 0;
    for (int64_t L = (int64_t)blockIdx.x * kSB + threadIdx.x; L < local_rows; L += stride) {
        const int i = sub_of(L, n, S, o);
        const int l = (int)sub_lo(i, n, S, o), h = (int)sub_hi(i, n, S, o);
        const int g = l + (int)(L - sub_off(i, n, S, o));
        int a, b;
        row_range(rp, nnz, g, a, b);
        int64_t k = 0;
        for (int e = a; e < b; ++e) {
            const int c = ci[e];
            k += (c >= l && c < h) ? 1 : 0;
        }
        if (cnt) cnt[L] = k;
        mine += (unsigned long long)k;
    }
    if (total) {
        mine = wave_sum(mine);
        if (threadIdx.x % kWave == 0 && mine) atomicAdd(total, mine);
    }
}

// Exclusive scan of v[0 .. m) into v, with v[m] = the total.  Pass 1: the
// sum of every chunk of kScanChunk elements.
__global__ __launch_bounds__(kSB) void scan_sums_kernel(int64_t m, const int64_t *__restrict__ v,
                                                        int64_t *sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + (int64_t)k * kSB + threadIdx.x;
        if (i < m) s += v[i];
    }
    __shared__ int64_t red[kSB / kWave];
    int64_t t[1] = {s};
    block_sum<1, kSB>(t, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = t[0];
}

// Pass 2 (one workgroup): exclusive scan of the chunk sums in place; the
// grand total goes to *total.
__global__ __launch_bounds__(1024) void scan_chunks_kernel(int64_t nchunks, int64_t *sums,
                                                           int64_t *total)
{
    __shared__ int64_t tot[1024];
    const int64_t per = (nchunks + 1023) / 1024;
    const int64_t a = threadIdx.x * per, b = min(nchunks, a + per);
    int64_t run = 0;
    for (int64_t i = a; i < b; ++i) run += sums[i];
    tot[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t x = tot[i];
            tot[i] = acc;
            acc += x;
        }
        *total = acc;
    }
    __syncthreads();
    int64_t acc = tot[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        const int64_t x = sums[i];
        sums[i] = acc;
        acc += x;
    }
}

// Pass 3: each chunk scanned in place from its offset.  Thread t owns
// elements [t * kScanPer, (t + 1) * kScanPer) of the chunk.
__global__ __launch_bounds__(kSB) void scan_apply_kernel(int64_t m, int64_t *v,
                                                         const int64_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t loc[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k;
        loc[k] = i < m ? v[i] : 0;
        s += loc[k];
    }
    __shared__ int64_t pre[kSB];
    pre[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the thread totals
    for (int off = 1; off < kSB; off <<= 1) {
        const int64_t add = (int)threadIdx.x >= off ? pre[threadIdx.x - off] : 0;
        __syncthreads();
        pre[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t acc = sums[blockIdx.x] + pre[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k;
        if (i < m) v[i] = acc;
        acc += loc[k];
    }
}

// Row pointers (per subdomain, from 0) and the kept entries of every local
// row; off[L] = the exclusive scan of the counts, off[local_rows] = total.
__global__ __launch_bounds__(kSB) void sub_fill_kernel(int64_t local_rows, int n, int S, int o,
                                                       int64_t nnz, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ val,
                                                       const int64_t *__restrict__ off,
                                                       int64_t *nnz_off, int32_t *lrp,
                                                       int32_t *lcol, double *lval)
{
    const int64_t stride = (int64_t)gridDim.x * kSB;
    for (int64_t L = (int64_t)blockIdx.x * kSB + threadIdx.x; L < local_rows; L += stride) {
        const int i = sub_of(L, n, S, o);
        const int64_t r0 = sub_off(i, n, S, o), k = L - r0;
        const int l = (int)sub_lo(i, n, S, o), h = (int)sub_hi(i, n, S, o);
        const int g = l + (int)k;
        const int64_t first = off[r0];
        int32_t *rpi = lrp + r0 + i;  // the m_i + 1 row pointers of subdomain i
        if (k == 0) {
            rpi[0] = 0;
            nnz_off[i] = first;
        }
        if (L == local_rows - 1) nnz_off[S] = off[local_rows];
        rpi[k + 1] = (int32_t)(off[L + 1] - first);
        int a, b;
        row_range(rp, nnz, g, a, b);
        int64_t e_out = off[L];
        for (int e = a; e < b; ++e) {
            const int c = ci[e];
            if (c >= l && c < h) {
                lcol[e_out] = c - l;
                lval[e_out] = val[e];
                ++e_out;
            }
        }
    }
}

// z[g] = sum over the subdomains containing g, in increasing order, of the
// subdomain solution's entry for g.  g's core block is within one of
// floor(g S / n); the blocks within two of it are checked.
__global__ __launch_bounds__(kSB) void prolong_kernel(int n, int S, int o,
                                                      const double *__restrict__ zloc,
                                                      double *__restrict__ z)
{
    const int64_t stride = (int64_t)gridDim.x * kSB;
    for (int64_t g = (int64_t)blockIdx.x * kSB + threadIdx.x; g < n; g += stride) {
        const int i0 = (int)(g * S / n);
        const int j0 = i0 >= 2 ? i0 - 2 : 0, j1 = i0 + 2 < S ? i0 + 2 : S - 1;
        double acc = 0.0;
        for (int j = j0; j <= j1; ++j) {
            const int64_t l = sub_lo(j, n, S, o);
            if (l <= g && g < sub_hi(j, n, S, o)) acc += zloc[sub_off(j, n, S, o) + (g - l)];
        }
        z[g] = acc;
    }
}

// p = fma(beta, p, z)
__global__ __launch_bounds__(kSB) void xpby_kernel(int64_t n, double beta,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ p)
{
    const int64_t stride = (int64_t)gridDim.x * kSB;
    for (int64_t i = (int64_t)blockIdx.x * kSB + threadIdx.x; i < n; i += stride)
        p[i] = __builtin_fma(beta, p[i], z[i]);
}

unsigned grid_for(int64_t n)
{
    int64_t g = (n + kSB - 1) / kSB;
    if (g > 8192) g = 8192;
    return (unsigned)(g < 1 ? 1 : g);
}

struct Ranges {
    std::vector<int64_t> lo, hi, row_off;  // row_off: S + 1 entries
};

Ranges make_ranges(int n, int S, int o)
{
    Ranges R;
    R.lo.resize(S);
    R.hi.resize(S);
    R.row_off.resize(S + 1);
    for (int i = 0; i < S; ++i) {
        R.lo[i] = sub_lo(i, n, S, o);
        R.hi[i] = sub_hi(i, n, S, o);
        R.row_off[i] = sub_off(i, n, S, o);
    }
    R.row_off[S] = sub_off(S, n, S, o);
    return R;
}

struct BuildLayout {
    size_t nnz_off, scan, sums, rp, col, val, total;
};

// Buffer of a Schwarz descriptor: nnz_off, the scan area (build only), row
// pointers, columns, values.  The parts before `col` do not depend on
// local_nnz.
BuildLayout build_layout(int S, int64_t local_rows, int64_t local_nnz)
{
    BuildLayout L{};
    size_t off = 0;
    L.nnz_off = off; off += al256(sizeof(int64_t) * (S + 1));
    L.scan = off;    off += al256(sizeof(int64_t) * (local_rows + 1));
    L.sums = off;    off += al256(sizeof(int64_t) * ((local_rows + kScanChunk - 1) / kScanChunk + 1));
    L.rp = off;      off += al256(sizeof(int32_t) * (local_rows + S));
    L.col = off;     off += al256(sizeof(int32_t) * std::max<int64_t>(local_nnz, 1));
    L.val = off;     off += al256(sizeof(double) * std::max<int64_t>(local_nnz, 1));
    L.total = off;
    return L;
}

struct SolveLayout {
    size_t r, p, q, z, zloc, scal, batch, total;
};

std::vector<cgx_system> local_systems(const cgx_schwarz *S, const Ranges &R,
                                      const std::vector<int64_t> &nnz_off, const double *r,
                                      double *zloc)
{
    std::vector<cgx_system> sys(S->n_sub);
    for (int i = 0; i < S->n_sub; ++i) {
        cgx_system &q = sys[i];
        q = cgx_system{};
        const int m = (int)(R.hi[i] - R.lo[i]);
        const bool have = !nnz_off.empty();
        q.A.n_rows = m;
        q.A.n_cols = m;
        q.A.nnz = have ? nnz_off[i + 1] - nnz_off[i] : 0;
        q.A.row_ptr = S->row_ptr + R.row_off[i] + i;
        q.A.col_idx = have ? S->col + nnz_off[i] : nullptr;
        q.A.val = have ? S->val + nnz_off[i] : nullptr;
        q.A.val32 = nullptr;
        q.nrhs = 1;
        q.schedule = 0;
        q.B = r ? r + R.lo[i] : nullptr;
        q.X = zloc ? zloc + R.row_off[i] : nullptr;
    }
    return sys;
}

SolveLayout solve_layout(const cgx_schwarz *S, const Ranges &R)
{
    SolveLayout L{};
    const size_t vb = al256((size_t)S->n_rows * sizeof(double));
    size_t off = 0;
    L.r = off;    off += vb;
    L.p = off;    off += vb;
    L.q = off;    off += vb;
    L.z = off;    off += vb;
    L.zloc = off; off += al256((size_t)std::max<int64_t>(S->local_rows, 1) * sizeof(double));
    L.scal = off; off += 256;
    L.batch = off;
    const std::vector<int64_t> none;
    const auto sys = local_systems(S, R, none, nullptr, nullptr);
    off += batch_workspace_bytes(S->n_sub, sys.data());
    L.total = off;
    return L;
}

// Device scalars -> host (sync on the caller's stream).
int read_scalars(Context *c, const double *d, double *h, int count)
{
    CGX_HIP_CHECK(hipMemcpyAsync(h, d, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    return CGX_OK;
}

}  // namespace

int schwarz_bytes(Context *c, const cgx_csr *A, int n_sub, int overlap, size_t *bytes)
{
    const int n = A->n_rows;
    const int64_t m = sub_off(n_sub, n, n_sub, overlap);
    unsigned long long *d_tot = reinterpret_cast<unsigned long long *>(c->scratch);
    const unsigned long long zero = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(d_tot, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    if (m > 0)
        hipLaunchKernelGGL(sub_count_kernel, dim3(grid_for(m)), dim3(kSB), 0, c->stream, m, n,
                           n_sub, overlap, A->nnz, A->row_ptr, A->col_idx, nullptr, d_tot);
    CGX_HIP_CHECK(hipGetLastError());
    unsigned long long tot = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(&tot, d_tot, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    *bytes = build_layout(n_sub, m, (int64_t)tot).total;
    return CGX_OK;
}

int schwarz_build(Context *c, const cgx_csr *A, int n_sub, int overlap, void *buf, size_t bytes,
                  cgx_schwarz *out)
{
    size_t need = 0;
    int rc = schwarz_bytes(c, A, n_sub, overlap, &need);
    if (rc) return rc;
    if (bytes < need) {
        set_error("Schwarz buffer too small: need " + std::to_string(need) + " bytes");
        return CGX_ENOMEM;
    }
    const int n = A->n_rows;
    const int64_t m = sub_off(n_sub, n, n_sub, overlap);
    char *w = static_cast<char *>(buf);
    BuildLayout L = build_layout(n_sub, m, 0);
    int64_t *scan = reinterpret_cast<int64_t *>(w + L.scan);
    int64_t *sums = reinterpret_cast<int64_t *>(w + L.sums);
    const int64_t nchunks = (m + kScanChunk - 1) / kScanChunk;
    if (m > 0) {
        hipLaunchKernelGGL(sub_count_kernel, dim3(grid_for(m)), dim3(kSB), 0, c->stream, m, n,
                           n_sub, overlap, A->nnz, A->row_ptr, A->col_idx, scan, nullptr);
        hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nchunks), dim3(kSB), 0, c->stream, m,
                           scan, sums);
        hipLaunchKernelGGL(scan_chunks_kernel, dim3(1), dim3(1024), 0, c->stream, nchunks, sums,
                           scan + m);
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nchunks), dim3(kSB), 0, c->stream, m,
                           scan, sums);
    }
    CGX_HIP_CHECK(hipGetLastError());
    int64_t local_nnz = 0;
    if (m > 0)
        CGX_HIP_CHECK(hipMemcpyAsync(&local_nnz, scan + m, sizeof(local_nnz),
                                     hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    L = build_layout(n_sub, m, local_nnz);
    if (L.total > bytes) {
        set_error("Schwarz buffer too small");
        return CGX_ENOMEM;
    }
    int64_t *nnz_off = reinterpret_cast<int64_t *>(w + L.nnz_off);
    int32_t *lrp = reinterpret_cast<int32_t *>(w + L.rp);
    int32_t *lcol = reinterpret_cast<int32_t *>(w + L.col);
    double *lval = reinterpret_cast<double *>(w + L.val);
    if (m > 0)
        hipLaunchKernelGGL(sub_fill_kernel, dim3(grid_for(m)), dim3(kSB), 0, c->stream, m, n,
                           n_sub, overlap, A->nnz, A->row_ptr, A->col_idx, A->val, scan, nnz_off,
                           lrp, lcol, lval);
    CGX_HIP_CHECK(hipGetLastError());
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    out->n_rows = n;
    out->n_sub = n_sub;
    out->overlap = overlap;
    out->reserved = 0;
    out->local_rows = m;
    out->local_nnz = local_nnz;
    out->nnz_off = nnz_off;
    out->row_ptr = lrp;
    out->col = lcol;
    out->val = lval;
    return CGX_OK;
}

size_t schwarz_workspace_bytes(const cgx_schwarz *S)
{
    const Ranges R = make_ranges(S->n_rows, S->n_sub, S->overlap);
    return solve_layout(S, R).total;
}

int schwarz_solve(Context *c, const cgx_csr *A, const cgx_schwarz *S, const double *b, double *x,
                  void *ws, size_t ws_bytes, const cgx_opts *o, cgx_stats *st)
{
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    const int n = A->n_rows;
    const Ranges R = make_ranges(n, S->n_sub, S->overlap);
    if (S->n_rows != n || R.row_off[S->n_sub] != S->local_rows) {
        set_error("Schwarz descriptor does not match its subdomain sizes");
        return CGX_EINVAL;
    }
    const SolveLayout L = solve_layout(S, R);
    if (ws_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    double *r = reinterpret_cast<double *>(w + L.r);
    double *p = reinterpret_cast<double *>(w + L.p);
    double *q = reinterpret_cast<double *>(w + L.q);
    double *z = reinterpret_cast<double *>(w + L.z);
    double *zloc = reinterpret_cast<double *>(w + L.zloc);
    double *d = reinterpret_cast<double *>(w + L.scal);  // device scalars
    void *bws = w + L.batch;
    const size_t bws_bytes = ws_bytes - L.batch;

    std::vector<int64_t> nnz_off(S->n_sub + 1);
    CGX_HIP_CHECK(hipMemcpyAsync(nnz_off.data(), S->nnz_off, sizeof(int64_t) * (S->n_sub + 1),
                                 hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    const auto sys = local_systems(S, R, nnz_off, r, zloc);

    cgx_opts io{};
    io.rtol = o->inner_rtol > 0.0 ? o->inner_rtol : (o->inner_rtol == 0.0 ? 1e-2 : 0.0);
    io.maxit = o->maxit > 0 ? o->maxit : 50;
    io.precond = o->precond;
    io.precision = CGX_PRECISION_FP64;
    const int64_t cap = o->max_outer > 0 ? o->max_outer : n;

    std::vector<cgx_stats> ist(S->n_sub);
    double local_ms = 0.0;
    int64_t inner = 0;
    // z = M(r): every subdomain solve from 0, then the sum of the local
    // solutions; returns the worst hard failure among the subdomain solves
    auto precondition = [&](int &hard) -> int {
        CGX_HIP_CHECK(hipMemsetAsync(zloc, 0, sizeof(double) * S->local_rows, c->stream));
        const auto t0 = clock::now();
        const int brc = run_batched(c, S->n_sub, sys.data(), bws, bws_bytes, &io, ist.data());
        if (brc != CGX_OK && brc != CGX_NOT_CONVERGED && brc != CGX_BREAKDOWN &&
            brc != CGX_NONFINITE)
            return brc;
        local_ms += std::chrono::duration<double, std::milli>(clock::now() - t0).count();
        hard = CGX_OK;
        int its = 0;
        for (const cgx_stats &s : ist) {
            if (s.status == CGX_BREAKDOWN || s.status == CGX_NONFINITE || s.status == CGX_EHIP ||
                s.status == CGX_EINVAL || s.status == CGX_ENOMEM)
                if (hard == CGX_OK) hard = s.status;
            its = std::max(its, s.iters);
        }
        inner += its;
        hipLaunchKernelGGL(prolong_kernel, dim3(grid_for(n)), dim3(kSB), 0, c->stream, n,
                           S->n_sub, S->overlap, zloc, z);
        CGX_HIP_CHECK(hipGetLastError());
        return CGX_OK;
    };

    double h[2];
    int status = CGX_NOT_CONVERGED;
    int64_t k = 0;
    double rr = 0.0;
    int rc = launch_dot(c, n, b, b, d);
    if (rc) return rc;
    rc = read_scalars(c, d, h, 1);
    if (rc) return rc;
    const double bb = h[0];
    const double bnorm = std::sqrt(bb);
    auto finish = [&](int s) {
        st->status = s;
        st->iters = (int32_t)std::min<int64_t>(inner, 0x7fffffff);
        st->outer_iters = (int32_t)k;
        st->path = 5;
        st->relres = bnorm > 0.0 ? std::sqrt(rr) / bnorm : 0.0;
        st->device_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
        st->phase_ms[0] = local_ms;
        st->phase_ms[1] = st->device_ms - local_ms;
        return s;
    };
    if (!std::isfinite(bb)) return finish(CGX_NONFINITE);
    if (bb == 0.0) {
        CGX_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
        CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
        return finish(CGX_OK);
    }
    // r = b - A x
    rc = launch_spmv(c, A, x, q);
    if (rc) return rc;
    CGX_HIP_CHECK(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    rc = launch_axpy(c, n, -1.0, q, r);
    if (rc) return rc;
    rc = launch_dot(c, n, r, r, d);
    if (rc) return rc;
    rc = read_scalars(c, d, h, 1);
    if (rc) return rc;
    rr = h[0];
    if (!std::isfinite(rr)) return finish(CGX_NONFINITE);
    if (std::sqrt(rr) <= o->rtol * bnorm) return finish(CGX_OK);
    int hard = CGX_OK;
    rc = precondition(hard);
    if (rc) return rc;
    rc = launch_dot(c, n, r, z, d);
    if (rc) return rc;
    rc = read_scalars(c, d, h, 1);
    if (rc) return rc;
    double rho = h[0];
    CGX_HIP_CHECK(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    while (k < cap) {
        if (hard != CGX_OK) {
            status = hard;
            break;
        }
        if (!(rho > 0.0)) {
            status = std::isfinite(rho) ? CGX_BREAKDOWN : CGX_NONFINITE;
            break;
        }
        rc = launch_spmv(c, A, p, q);
        if (rc) return rc;
        rc = launch_dot(c, n, p, q, d);
        if (rc) return rc;
        rc = read_scalars(c, d, h, 1);
        if (rc) return rc;
        const double pq = h[0];
        if (!std::isfinite(pq)) {
            status = CGX_NONFINITE;
            break;
        }
        if (!(pq > 0.0)) {
            status = CGX_BREAKDOWN;
            break;
        }
        const double alpha = rho / pq;
        rc = launch_axpy(c, n, alpha, p, x);
        if (rc) return rc;
        rc = launch_axpy(c, n, -alpha, q, r);
        if (rc) return rc;
        ++k;
        rc = launch_dot(c, n, r, r, d);
        if (rc) return rc;
        rc = read_scalars(c, d, h, 1);
        if (rc) return rc;
        rr = h[0];
        if (!std::isfinite(rr)) {
            status = CGX_NONFINITE;
            break;
        }
        if (std::sqrt(rr) <= o->rtol * bnorm) {
            status = CGX_OK;
            break;
        }
        if (k >= cap) break;
        rc = precondition(hard);
        if (rc) return rc;
        rc = launch_dot(c, n, z, q, d);
        if (rc) return rc;
        rc = launch_dot(c, n, r, z, d + 1);
        if (rc) return rc;
        rc = read_scalars(c, d, h, 2);
        if (rc) return rc;
        const double beta = -alpha * h[0] / rho;
        rho = h[1];
        hipLaunchKernelGGL(xpby_kernel, dim3(grid_for(n)), dim3(kSB), 0, c->stream, (int64_t)n,
                           beta, z, p);
        CGX_HIP_CHECK(hipGetLastError());
    }
    if (o->true_residual) {
        rc = launch_spmv(c, A, x, q);
        if (rc) return rc;
        CGX_HIP_CHECK(hipMemcpyAsync(z, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        rc = launch_axpy(c, n, -1.0, q, z);
        if (rc) return rc;
        rc = launch_dot(c, n, z, z, d);
        if (rc) return rc;
        rc = read_scalars(c, d, h, 1);
        if (rc) return rc;
        st->relres_true = std::sqrt(h[0]) / bnorm;
    }
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    return finish(status);
}

}  // namespace cgx
