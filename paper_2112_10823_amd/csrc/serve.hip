// Continuous-batching solve server: requests (a resident CSR matrix, a
// right-hand side and a solution vector, all device memory owned by the
// caller) are admitted while a slot and pool memory are free, and every
// admitted request advances inside one batched CG iteration sequence with
// all others (the batched kernels of batch_kernels.h).  A progress thread
// alternates: admit queued requests, run a few iterations of all active
// requests, retire the finished ones.  Requests that arrive while others are
// on the GPU join at the next cycle.
//
// Grouping: when a request is admitted, up to max_group - 1 queued requests
// on the same matrix (same arrays and options) join its slot as further
// right-hand sides, so the matrix is streamed once per iteration for all of
// them (the batched solver's multi-right-hand-side SpMM).  Each request keeps
// its own scalars and stopping test and is retired as soon as it finishes.
//
// Binary32-refined requests (MIXED) get slots of their own: float64 x and
// residual, binary32 inner vectors and D^-1.  Their inner CG iterations run
// in the batched binary32 kernels, all such slots in one launch per phase;
// the float64 step of a lane (fold the inner solution into x, r = b - A x,
// stopping test, next inner right-hand side r / ||r||) is taken at the start
// of the cycle after its inner solve ended, in one short kernel sequence per
// slot for all of its lanes that are due.  Requests with reliable updates
// (MIXED_RU) use the same slots, start and finish the same way, but take
// their float64 updates inside the iteration sequence (the update kernels of
// batch_kernels.h run after every binary32 iteration while such a slot is
// active), so between start and finish they need no host step.
//
// Device memory comes only from the caller's pool: a fixed arena (system
// tables, lane table, work tables, scalars, reduction partials) at its start
// and a first-fit heap for per-slot Krylov vectors.  A request's arithmetic
// depends only on its slot's rows, tiles, right-hand-side count and
// schedule: alone and in any mix it gets the same bits when it is served
// ungrouped (max_group = 1) and the same solution within the solve
// tolerance when grouping changes its slot's right-hand-side count.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "batch_kernels.h"

namespace cgx {

using namespace bk;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct Request {
    uint64_t ticket = 0;
    cgx_csr A{};
    const double *b = nullptr;
    double *x = nullptr;
    int jac = 0, maxit = 0;
    double rtol = 0.0;
    int mixed = 0;            // 1: restarted refinement (MIXED); 2: reliable updates (MIXED_RU)
    double inner_rtol = 0.0;  // MIXED: inner stopping tolerance; MIXED_RU: update trigger delta
    int max_outer = 0;        // MIXED: inner solves at most; MIXED_RU: updates at most
    double t_submit = 0.0;
    size_t bytes = 0;  // heap bytes: Krylov vectors plus a one-system tuning plan
};

enum LaneState : uint8_t { kLaneFree = 0, kLaneRunning = 1, kLaneJoining = 2 };

struct Slot {
    bool used = false;
    bool fresh = false;
    std::vector<Request> lane;      // K lanes; lane j serves lane[j] while not free
    std::vector<uint8_t> state;     // LaneState per lane
    std::vector<double> t_start;    // admission / join time per lane
    std::vector<int> sharing;       // per lane: requests in the slot when it started
    // MIXED slots, per lane: float64 step due at the next cycle, first step
    // (x = caller x0), step issued this cycle, inner solves started, inner
    // iterations so far; MIXED_RU lanes: the status of a stopped binary32
    // iteration (its last float64 step is due), and the update cap
    std::vector<uint8_t> need_outer, first, outer_ran, last;
    std::vector<int> outer, inner_sum, final_status;
    size_t off = 0, bytes = 0;      // heap block of the slot's vectors
    bool mixed = false;             // binary32 slot (MIXED or MIXED_RU)
    bool ru = false;                // MIXED_RU: reliable updates inside the iteration
    int M = 1;
    int K = 1;
    int ntiles = 0;
    Request key;                    // matrix and options every lane shares
    int running() const
    {
        int c = 0;
        for (uint8_t v : state) c += v != kLaneFree;
        return c;
    }
    int free_lane() const
    {
        for (size_t j = 0; j < state.size(); ++j)
            if (state[j] == kLaneFree) return (int)j;
        return -1;
    }
};

struct Result {
    bool done = false;
    cgx_stats st{};
};

struct Engine {
    Context *c = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    char *pool = nullptr;
    size_t pool_bytes = 0;
    int max_slots = 0;
    int max_group = 1;
    int64_t max_tiles = 0;
    size_t off_sys = 0, off_lanes = 0, off_list = 0, off_list2 = 0, off_scal = 0, off_done = 0,
           off_tiles = 0, off_tiles2 = 0, off_part = 0, heap0 = 0;
    // binary32 tables of the MIXED slots (indexed by slot like the float64
    // ones; the work-table entries number tiles in one space with them)
    size_t off_sys32 = 0, off_list32 = 0, off_scal32 = 0, off_done32 = 0, off_tiles32 = 0,
           off_part32 = 0, off_bad = 0;
    std::map<size_t, size_t> free_list;  // heap offset -> size
    std::vector<Slot> slots;
    std::deque<Request> queue;
    std::map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    std::thread th;
    int fail = CGX_OK;
    std::string fail_msg;
    BScal *h_scal = nullptr;
    int32_t *h_done = nullptr;
    BScalT<float> *h_scal32 = nullptr;
    double head_wait_limit = 0.25;  // s a blocked head may wait before backfilling stops
    uint64_t completed = 0;
    int active_tiles = 0;    // entries of the float64 work table (engine thread only)
    int active_tiles32 = 0;  // entries of the binary32 work table
    int nlist64 = 0, nlist32 = 0;  // float64 / MIXED slots in the per-system lists

    // --------------------------------------------------------- pool heap --
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = a256(bytes);
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_list.erase(it);
                if (rest) free_list[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = a256(bytes);
        auto it = free_list.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_list.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_list.erase(nx);
        }
        if (it != free_list.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_list.erase(it);
            }
        }
    }
    size_t heap_capacity() const { return pool_bytes - heap0; }
};

namespace {

int tiles_of(int64_t n, int nrhs)
{
    const int tr = tile_rows_for(pad_k(nrhs), false);
    return (int)((n + tr - 1) / tr);
}

// Heap bytes of a group of nrhs requests on an n-row matrix: its Krylov
// vectors, and room for the one-system plan the autotuner times in place.
size_t group_bytes(int64_t n, int nrhs)
{
    cgx_system sys{};
    sys.A.n_rows = (int32_t)n;
    sys.A.n_cols = (int32_t)n;
    sys.nrhs = nrhs;
    return batch_workspace_bytes(1, &sys);
}

size_t request_bytes(int64_t n) { return group_bytes(n, 1); }

// Requests that may share a slot: same matrix arrays and solver options.
bool same_group(const Request &a, const Request &b)
{
    return a.A.row_ptr == b.A.row_ptr && a.A.col_idx == b.A.col_idx && a.A.val == b.A.val &&
           a.A.n_rows == b.A.n_rows && a.A.nnz == b.A.nnz && a.jac == b.jac &&
           a.maxit == b.maxit && a.rtol == b.rtol && a.mixed == b.mixed &&
           (!a.mixed || (a.A.val32 == b.A.val32 && a.inner_rtol == b.inner_rtol &&
                         a.max_outer == b.max_outer));
}

// ------------------------------------------------ MIXED slot kernels --
// Float64 steps of the lanes of MIXED slot si in bit mask `mask` (lane j:
// bit j), all at once; S / F are the slot's float64 / binary32 descriptors.
// The tile kernels run a workgroup per tile of trows rows (partials at tile
// S.tile0 + blockIdx.x) and, as the batched kernels, give thread t the lane
// t % K.  A lane's arithmetic does not depend on which other lanes are in
// the mask.

// D^-1 of the slot from val32's diagonal, 1 / a_ii rounded once to binary32
// from a float64 division (as the float32-refined batch forms it); a
// diagonal entry <= 0 or missing marks the slot (Jacobi breakdown).
__global__ __launch_bounds__(kBB) void mixed_setup_kernel(const BSysT<float> *sys32, int32_t *bad,
                                                          int si)
{
    const BSysT<float> &F = sys32[si];
    const int row0 = blockIdx.x * F.trows, row1 = min(F.n, row0 + F.trows);
    bool b = false;
    for (int row = row0 + threadIdx.x; row < row1; row += kBB) {
        const int s0 = clampk(F.rp[row], F.nnz), s1 = max(s0, clampk(F.rp[row + 1], F.nnz));
        float dg = 0.0f;
        for (int k = s0; k < s1; ++k)
            if (F.ci[k] == row) dg = F.val[k];
        b = b || !(dg > 0.0f);
        F.dinv[row] = (float)(1.0 / (double)(dg > 0.0f ? dg : 1.0f));
    }
    if (b) bad[si] = 1;  // same value from every writer
}

// x[:, j] = caller x0 (lanes in `first`) or fma(||r_prev||, double(d[:, j]),
// x[:, j]): the inner solution folded into the float64 iterate.
__global__ __launch_bounds__(kBB) void mixed_x_kernel(BArgs a64, BArgsT<float> a32, int si,
                                                      uint32_t mask, uint32_t first)
{
    const BSys &S = a64.sys[si];
    const BSysT<float> &F = a32.sys[si];
    const int j = threadIdx.x % S.K;
    if (!((mask >> j) & 1u)) return;
    const bool f0 = (first >> j) & 1u;
    const double sigma = sqrt(a64.scal[S.scal0 + j].rr);
    const double *x0 = S.lanes[j].x;
    const int row0 = blockIdx.x * S.trows, row1 = min(S.n, row0 + S.trows);
    const int64_t e1 = (int64_t)row1 * S.K;
    int row = row0 + (int)threadIdx.x / S.K;
    for (int64_t e = (int64_t)row0 * S.K + threadIdx.x; e < e1; e += kBB, row += kBB / S.K)
        S.x[e] = f0 ? x0[row] : __builtin_fma(sigma, (double)F.x[e], S.x[e]);
}

// r = b - A x in float64 for the masked lanes (the row sums of the batched
// setup pass: K * M lanes per row group, all K lanes gathering each column's
// line) and the tile partials of r.r and b.b per lane.
__global__ __launch_bounds__(kBB) void mixed_residual_kernel(BArgs a64, int si, uint32_t mask)
{
    __shared__ double red[kBB];
    const BSys &S = a64.sys[si];
    const int M = setup_m(S);
    const int G = S.K * M, gpw = kWave / G;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int grp = lane / G, sub = lane % G, j = sub % S.K, m = sub / S.K;
    const bool on = (mask >> j) & 1u;
    const double *b = S.lanes[j].b;
    const int row0 = blockIdx.x * S.trows, row1 = min(S.n, row0 + S.trows);
    double prr = 0.0, pbb = 0.0;
    for (int row = row0 + wave * gpw + grp; gpw >= 1 && row < row1; row += (kBB / kWave) * gpw) {
        double dg;
        const double ax = row_spmm(S, row, j, m, M, dg, S.x);
        if (m == 0 && on) {
            const double bi = b[row];
            const double ri = bi - ax;
            S.r[(int64_t)row * S.K + j] = ri;
            prr += ri * ri;
            pbb += bi * bi;
        }
    }
    double *base = a64.part + (int64_t)(S.tile0 + blockIdx.x) * kMaxK;
    block_sum_by_rhs(prr, S.K, red, base);
    block_sum_by_rhs(pbb, S.K, red, base + a64.part_stride);
}

// One workgroup: ||r||^2 and ||b||^2 per masked lane from the tile partials
// (fixed order) and the float64 stopping test: b = 0 or ||r|| <= rtol ||b||
// ends the lane (CGX_OK), a bad Jacobi diagonal ends it (CGX_BREAKDOWN), and
// so does the step after max_outer inner solves (lanes in `last`:
// CGX_NOT_CONVERGED).
__global__ __launch_bounds__(kBB) void mixed_outer_kernel(BArgs a64, const int32_t *bad, int si,
                                                          uint32_t mask, uint32_t last)
{
    __shared__ double red[kBB];
    const BSys &S = a64.sys[si];
    const double rr = sys_sum(a64, S, 0, red);
    const double bb = sys_sum(a64, S, 1, red);
    const int j = threadIdx.x;
    if (j < S.K && ((mask >> j) & 1u)) {
        BScal &c = a64.scal[S.scal0 + j];
        c.rr = rr;
        c.bb = bb;
        c.stop2 = S.rtol2 * bb;
        int status = CGX_PENDING;
        if (!isfinite(bb) || !isfinite(rr))
            status = CGX_NONFINITE;
        else if (bb == 0.0 || rr <= S.rtol2 * bb)
            status = CGX_OK;
        else if (S.jac && bad[si])
            status = CGX_BREAKDOWN;
        else if ((last >> j) & 1u)
            status = CGX_NOT_CONVERGED;
        c.status = status;
        c.active = status == CGX_PENDING;
    }
}

// Start of the next inner solve of each masked lane whose float64 status is
// still pending: c = float(r / ||r||) is its right-hand side and, from d =
// 0, its residual; z = D^-1 c, p = z; tile partials of c.c and c.z in
// binary32.
__global__ __launch_bounds__(kBB) void mixed_start_kernel(BArgs a64, BArgsT<float> a32, int si,
                                                          uint32_t mask)
{
    __shared__ float red[kBB];
    const BSys &S = a64.sys[si];
    const BSysT<float> &F = a32.sys[si];
    const int j = threadIdx.x % S.K;
    const BScal c64 = a64.scal[S.scal0 + j];
    const bool on = ((mask >> j) & 1u) && c64.status == CGX_PENDING;
    float prr = 0.0f, prz = 0.0f;
    if (on) {
        const double sigma = sqrt(c64.rr);
        const int row0 = blockIdx.x * S.trows, row1 = min(S.n, row0 + S.trows);
        const int64_t e1 = (int64_t)row1 * S.K;
        int row = row0 + (int)threadIdx.x / S.K;
        for (int64_t e = (int64_t)row0 * S.K + threadIdx.x; e < e1; e += kBB, row += kBB / S.K) {
            const float ci = (float)(S.r[e] / sigma);
            const float zi = F.jac ? F.dinv[row] * ci : ci;
            F.r[e] = ci;
            F.x[e] = 0.0f;
            F.p[e] = zi;
            prr += ci * ci;
            prz += ci * zi;
        }
    }
    float *base = a32.part + (int64_t)(F.tile0 + blockIdx.x) * kMaxK;
    block_sum_by_rhs(prr, S.K, red, base);
    block_sum_by_rhs(prz, S.K, red, base + a32.part_stride);
}

// One workgroup: each masked lane's binary32 scalars for its next inner
// solve (or an inactive lane when its float64 status is final), as
// batch_r0_kernel sets them for a whole system: stop when ||c - A d|| <=
// inner_rtol ||c||.
__global__ __launch_bounds__(kBB) void mixed_inner_r0_kernel(BArgs a64, BArgsT<float> a32, int si,
                                                             uint32_t mask)
{
    __shared__ float red[kBB];
    const BSys &S = a64.sys[si];
    const BSysT<float> &F = a32.sys[si];
    const float rr = sys_sum(a32, F, 0, red);
    const float rz = sys_sum(a32, F, 1, red);
    const int j = threadIdx.x;
    if (j < S.K && ((mask >> j) & 1u)) {
        BScalT<float> &c = a32.scal[F.scal0 + j];
        c = BScalT<float>{};
        if (a64.scal[S.scal0 + j].status != CGX_PENDING) {
            c.status = CGX_OK;  // no inner solve: the lane is finished
            return;
        }
        const BScal &d = a64.scal[S.scal0 + j];
        c.rr = rr;
        c.bb = rr;  // reliable updates: the largest ||r^||^2 since the last update
        c.rho = F.jac ? rz : rr;
        // restarted refinement: stop at inner_rtol ||c||; reliable updates:
        // the float64 stopping test in the scale ||r|| (update when reached)
        c.stop2 = F.ru ? (float)(d.stop2 / d.rr) : (float)F.rtol2 * rr;
        int status = CGX_PENDING;
        if (!isfinite(rr) || !isfinite(rz))
            status = CGX_NONFINITE;
        else if (rr == 0.0f || (!F.ru && rr <= c.stop2))
            status = CGX_OK;
        else if (F.jac && !(rz > 0.0f))
            status = CGX_BREAKDOWN;
        c.status = status;
        c.active = status == CGX_PENDING;
        if (c.active) a32.sys_done[si] = 0;  // same value from every writer
    }
}

// Heap block of a MIXED slot: float64 x, r, then binary32 d (the inner
// solution, the binary32 system's x), r, p, q, all interleaved [n][K], and
// binary32 D^-1 [n].  No larger than the float64 slot's block (x r p q z,
// D^-1), which also holds the tuner's one-system plan.
size_t mixed_slot_bytes(int64_t n, int K)
{
    return 2 * a256((size_t)n * K * sizeof(double)) + 4 * a256((size_t)n * K * sizeof(float)) +
           a256((size_t)n * sizeof(float));
}

// Device descriptor of slot `si`: interleaved x r p q z of its K lanes and
// dinv at the start of its heap block (MIXED slot: x and r only); b / x of
// each request through the slot's lane table (null for a free lane).
BSys slot_sys(const Engine &E, int si, int tile0)
{
    const Slot &s = E.slots[si];
    const Request &q = s.key;
    BSys S{};
    S.rp = q.A.row_ptr;
    S.ci = q.A.col_idx;
    S.val = q.A.val;
    S.lanes = reinterpret_cast<const LanePtr *>(E.pool + E.off_lanes) + (size_t)si * kMaxK;
    const size_t vb = a256((size_t)q.A.n_rows * s.K * sizeof(double));
    char *base = E.pool + s.off;
    if (s.mixed) {
        S.x = reinterpret_cast<double *>(base);
        S.r = reinterpret_cast<double *>(base + vb);
    } else {
        double **vecs[5] = {&S.x, &S.r, &S.p, &S.q, &S.z};
        for (int v = 0; v < 5; ++v) *vecs[v] = reinterpret_cast<double *>(base + v * vb);
        S.dinv = reinterpret_cast<double *>(base + 5 * vb);
    }
    S.nnz = q.A.nnz;
    S.n = q.A.n_rows;
    S.n_cols = q.A.n_cols;
    S.K = s.K;
    S.nrhs = s.K;
    S.M = s.M;
    S.trows = tile_rows_for(s.K, false);
    S.tile0 = tile0;
    S.ntiles = s.ntiles;
    S.scal0 = si * kMaxK;
    S.jac = q.jac;
    S.maxit = q.mixed == 2 ? q.max_outer : q.maxit;  // MIXED_RU: the update cap
    S.rtol2 = q.rtol * q.rtol;
    return S;
}

// Binary32 descriptor of MIXED slot `si` (the inner solves): values val32,
// vectors after the float64 x and r of its heap block, tolerance inner_rtol,
// iteration cap maxit per inner solve.
BSysT<float> slot_sys32(const Engine &E, int si, int tile0)
{
    const Slot &s = E.slots[si];
    const Request &q = s.key;
    BSysT<float> F{};
    F.rp = q.A.row_ptr;
    F.ci = q.A.col_idx;
    F.val = q.A.val32;
    const size_t n = (size_t)q.A.n_rows;
    const size_t vb64 = a256(n * s.K * sizeof(double)), vb = a256(n * s.K * sizeof(float));
    char *base = E.pool + s.off + 2 * vb64;
    float **vecs[4] = {&F.x, &F.r, &F.p, &F.q};
    for (int v = 0; v < 4; ++v) *vecs[v] = reinterpret_cast<float *>(base + v * vb);
    F.dinv = reinterpret_cast<float *>(base + 4 * vb);
    F.nnz = q.A.nnz;
    F.n = q.A.n_rows;
    F.n_cols = q.A.n_cols;
    F.K = s.K;
    F.nrhs = s.K;
    F.M = s.M;
    F.trows = tile_rows_for(s.K, false);
    F.tile0 = tile0;
    F.ntiles = s.ntiles;
    F.scal0 = si * kMaxK;
    F.jac = q.jac;
    F.maxit = q.maxit;
    F.rtol2 = q.inner_rtol * q.inner_rtol;
    F.ru = q.mixed == 2;
    return F;
}

BArgsT<float> engine_args32(const Engine &E)
{
    BArgsT<float> a{};
    a.sys = reinterpret_cast<const BSysT<float> *>(E.pool + E.off_sys32);
    a.tiles = reinterpret_cast<const BTile *>(E.pool + E.off_tiles32);
    a.list = reinterpret_cast<const int32_t *>(E.pool + E.off_list32);
    a.scal = reinterpret_cast<BScalT<float> *>(E.pool + E.off_scal32);
    a.sys_done = reinterpret_cast<int32_t *>(E.pool + E.off_done32);
    a.part = reinterpret_cast<float *>(E.pool + E.off_part32);
    a.part_stride = E.max_tiles * kMaxK;
    a.ntiles = E.active_tiles32;
    a.nlist = E.nlist32;
    a.wave_lds = 0;
    for (const Slot &sl : E.slots)
        if (sl.used && sl.mixed && sl.M < 0) a.wave_lds = kWaveStageBytes;
    return a;
}

BArgs engine_args(const Engine &E, bool fresh, int ntiles, int nlist)
{
    BArgs a{};
    a.sys = reinterpret_cast<const BSys *>(E.pool + E.off_sys);
    a.tiles = reinterpret_cast<const BTile *>(E.pool + (fresh ? E.off_tiles2 : E.off_tiles));
    a.list = reinterpret_cast<const int32_t *>(E.pool + (fresh ? E.off_list2 : E.off_list));
    a.scal = reinterpret_cast<BScal *>(E.pool + E.off_scal);
    a.sys_done = reinterpret_cast<int32_t *>(E.pool + E.off_done);
    a.part = reinterpret_cast<double *>(E.pool + E.off_part);
    a.part_stride = E.max_tiles * kMaxK;
    a.ntiles = ntiles;
    a.nlist = nlist;
    a.wave_lds = 0;
    for (const Slot &sl : E.slots)
        if (sl.used && !sl.mixed && sl.M < 0) a.wave_lds = kWaveStageBytes;
    return a;
}

#define ENG_CHECK(expr)                                                          \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            E.fail = CGX_EHIP;                                                   \
            E.fail_msg = std::string(#expr " failed: ") + hipGetErrorString(e_); \
            return false;                                                        \
        }                                                                        \
    } while (0)

// One cycle's device work: rebuild tables if membership changed, initialise
// fresh slots and the lanes requests joined, take the float64 steps of the
// MIXED lanes whose inner solve ended, run `iters` iterations (float64 slots
// and binary32 inner solves), read back the slot states.  `active` receives
// every used slot.
bool device_cycle(Engine &E, bool changed, int iters, std::vector<int> &active)
{
    hipStream_t s = E.stream;
    if (changed) {
        std::vector<BSys> sys(E.max_slots);
        std::vector<BSysT<float>> sys32(E.max_slots);
        std::vector<BTile> tiles, tiles2, tiles32;
        std::vector<int32_t> list, list2, list32, fresh32;
        int next_tile = 0;  // one numbering for the tiles of both tables
        active.clear();
        for (int i = 0; i < E.max_slots; ++i) {
            const Slot &sl = E.slots[i];
            if (!sl.used) continue;
            const int tile0 = next_tile;
            next_tile += sl.ntiles;
            sys[i] = slot_sys(E, i, tile0);
            if (sl.mixed) sys32[i] = slot_sys32(E, i, tile0);
            for (int t = 0; t < sl.ntiles; ++t) {
                BTile bt{};
                bt.sys = i;
                bt.row0 = t * sys[i].trows;
                bt.rows = std::min(sys[i].trows, sys[i].n - bt.row0);
                bt.tile = tile0 + t;
                (sl.mixed ? tiles32 : tiles).push_back(bt);
                if (sl.fresh && !sl.mixed) tiles2.push_back(bt);
            }
            (sl.mixed ? list32 : list).push_back(i);
            if (sl.fresh) (sl.mixed ? fresh32 : list2).push_back(i);
            active.push_back(i);
        }
        ENG_CHECK(hipMemcpyAsync(E.pool + E.off_sys, sys.data(), sizeof(BSys) * sys.size(),
                                 hipMemcpyHostToDevice, s));
        if (!list32.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_sys32, sys32.data(),
                                     sizeof(BSysT<float>) * sys32.size(), hipMemcpyHostToDevice, s));
        if (!tiles.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_tiles, tiles.data(), sizeof(BTile) * tiles.size(),
                                     hipMemcpyHostToDevice, s));
        if (!list.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_list, list.data(), sizeof(int32_t) * list.size(),
                                     hipMemcpyHostToDevice, s));
        if (!tiles32.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_tiles32, tiles32.data(),
                                     sizeof(BTile) * tiles32.size(), hipMemcpyHostToDevice, s));
        if (!list32.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_list32, list32.data(),
                                     sizeof(int32_t) * list32.size(), hipMemcpyHostToDevice, s));
        E.active_tiles = (int)tiles.size();
        E.active_tiles32 = (int)tiles32.size();
        E.nlist64 = (int)list.size();
        E.nlist32 = (int)list32.size();
        const std::vector<BScal> zero(kMaxK);
        const std::vector<BScalT<float>> zero32(kMaxK);
        const int32_t zd = 0, one = 1;
        auto upload_lanes = [&](int i) -> bool {
            LanePtr lanes[kMaxK] = {};
            const Slot &sl = E.slots[i];
            for (int j = 0; j < sl.K; ++j)
                if (sl.state[j] != kLaneFree) lanes[j] = {sl.lane[j].b, sl.lane[j].x};
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_lanes + sizeof(LanePtr) * kMaxK * i, lanes,
                                     sizeof(lanes), hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_scal + sizeof(BScal) * kMaxK * i, zero.data(),
                                     sizeof(BScal) * kMaxK, hipMemcpyHostToDevice, s));
            return true;
        };
        if (!list2.empty()) {
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_tiles2, tiles2.data(),
                                     sizeof(BTile) * tiles2.size(), hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_list2, list2.data(),
                                     sizeof(int32_t) * list2.size(), hipMemcpyHostToDevice, s));
            for (int i : list2) {
                Slot &sl = E.slots[i];
                if (!upload_lanes(i)) return false;
                ENG_CHECK(hipMemcpyAsync(E.pool + E.off_done + sizeof(int32_t) * i, &zd,
                                         sizeof(int32_t), hipMemcpyHostToDevice, s));
                for (int j = 0; j < sl.K; ++j)
                    if (sl.state[j] == kLaneJoining) sl.state[j] = kLaneRunning;
            }
            const BArgs f = engine_args(E, true, (int)tiles2.size(), (int)list2.size());
            hipLaunchKernelGGL((batch_in_kernel<double>), dim3(f.ntiles), dim3(kBB), 0, s, f);
            hipLaunchKernelGGL((batch_init_kernel<double>), dim3(f.ntiles), dim3(kBB), 0, s, f);
            hipLaunchKernelGGL((batch_r0_kernel<double>), dim3(f.nlist), dim3(kBB), 0, s, f);
            ENG_CHECK(hipGetLastError());
            for (int i : list2) E.slots[i].fresh = false;
        }
        // fresh MIXED slots: D^-1 in binary32; every lane starts with its
        // first float64 step below
        for (int i : fresh32) {
            Slot &sl = E.slots[i];
            if (!upload_lanes(i)) return false;
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_scal32 + sizeof(BScalT<float>) * kMaxK * i,
                                     zero32.data(), sizeof(BScalT<float>) * kMaxK,
                                     hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_done32 + sizeof(int32_t) * i, &one,
                                     sizeof(int32_t), hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_bad + sizeof(int32_t) * i, &zd, sizeof(int32_t),
                                     hipMemcpyHostToDevice, s));
            if (sl.key.jac)
                hipLaunchKernelGGL(mixed_setup_kernel, dim3(sl.ntiles), dim3(kBB), 0, s,
                                   reinterpret_cast<const BSysT<float> *>(E.pool + E.off_sys32),
                                   reinterpret_cast<int32_t *>(E.pool + E.off_bad), i);
            for (int j = 0; j < sl.K; ++j)
                if (sl.state[j] == kLaneJoining) {
                    sl.state[j] = kLaneRunning;
                    sl.need_outer[j] = 1;
                    sl.first[j] = 1;
                }
            sl.fresh = false;
        }
        ENG_CHECK(hipGetLastError());
    }
    // requests that joined a free lane of a running slot: set that lane up
    const BArgs m = engine_args(E, false, E.active_tiles, E.nlist64);
    const BArgsT<float> m32 = engine_args32(E);
    for (int i : active) {
        Slot &sl = E.slots[i];
        for (int j = 0; j < sl.K; ++j) {
            if (sl.state[j] != kLaneJoining) continue;
            const LanePtr lp = {sl.lane[j].b, sl.lane[j].x};
            const BScal zero{};
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_lanes + sizeof(LanePtr) * (kMaxK * i + j), &lp,
                                     sizeof(lp), hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_scal + sizeof(BScal) * (kMaxK * i + j), &zero,
                                     sizeof(zero), hipMemcpyHostToDevice, s));
            sl.state[j] = kLaneRunning;
            if (sl.mixed) {
                sl.need_outer[j] = 1;
                sl.first[j] = 1;
                continue;
            }
            hipLaunchKernelGGL(lane_init_kernel, dim3(sl.ntiles), dim3(kBB), 0, s, m, i, j);
            hipLaunchKernelGGL(lane_r0_kernel, dim3(1), dim3(kBB), 0, s, m, i, j);
            ENG_CHECK(hipGetLastError());
        }
    }
    // float64 steps of MIXED lanes: fold d into x (or take x0), r = b - A x,
    // stopping test, next inner solve's start; one pass per slot for all of
    // its lanes whose inner solve ended
    const int32_t *bad = reinterpret_cast<const int32_t *>(E.pool + E.off_bad);
    for (int i : active) {
        Slot &sl = E.slots[i];
        if (!sl.mixed) continue;
        uint32_t mask = 0, first = 0, last = 0;
        for (int j = 0; j < sl.K; ++j) {
            if (sl.state[j] != kLaneRunning || !sl.need_outer[j]) continue;
            mask |= 1u << j;
            if (sl.first[j]) first |= 1u << j;
            if (sl.ru ? sl.last[j] != 0 : sl.outer[j] >= sl.key.max_outer) last |= 1u << j;
            sl.need_outer[j] = 0;
            sl.first[j] = 0;
            sl.outer_ran[j] = 1;
        }
        if (!mask) continue;
        const dim3 g(sl.ntiles);
        hipLaunchKernelGGL(mixed_x_kernel, g, dim3(kBB), 0, s, m, m32, i, mask, first);
        hipLaunchKernelGGL(mixed_residual_kernel, g, dim3(kBB), 0, s, m, i, mask);
        hipLaunchKernelGGL(mixed_outer_kernel, dim3(1), dim3(kBB), 0, s, m, bad, i, mask, last);
        hipLaunchKernelGGL(mixed_start_kernel, g, dim3(kBB), 0, s, m, m32, i, mask);
        hipLaunchKernelGGL(mixed_inner_r0_kernel, dim3(1), dim3(kBB), 0, s, m, m32, i, mask);
        ENG_CHECK(hipGetLastError());
    }
    if (E.nlist64 > 0 && E.active_tiles > 0)
        for (int k = 0; k < iters; ++k) launch_batch_iteration(m, s);
    if (E.nlist32 > 0 && E.active_tiles32 > 0) {
        bool any_ru = false;
        for (int i : active) any_ru = any_ru || (E.slots[i].used && E.slots[i].ru);
        for (int k = 0; k < iters; ++k) {
            if (any_ru)
                launch_ru_iteration(m, m32, 0, s);  // the update caps in the slots' descriptors
            else
                launch_batch_iteration(m32, s);
        }
    }
    ENG_CHECK(hipGetLastError());
    ENG_CHECK(hipMemcpyAsync(E.h_done, E.pool + E.off_done, sizeof(int32_t) * E.max_slots,
                             hipMemcpyDeviceToHost, s));
    ENG_CHECK(hipMemcpyAsync(E.h_scal, E.pool + E.off_scal, sizeof(BScal) * kMaxK * E.max_slots,
                             hipMemcpyDeviceToHost, s));
    if (E.nlist32 > 0)
        ENG_CHECK(hipMemcpyAsync(E.h_scal32, E.pool + E.off_scal32,
                                 sizeof(BScalT<float>) * kMaxK * E.max_slots, hipMemcpyDeviceToHost, s));
    ENG_CHECK(hipStreamSynchronize(s));
    return true;
}

// Rows from which a slot keeps one spare lane for later requests on its
// matrix: there the matrix stream dominates an iteration and a joined
// request costs little more than its own vectors.
constexpr int64_t kSpareLaneRows = 1 << 16;

// Admission.  A queued request first joins a free lane of a running slot on
// the same matrix and options (at most max_group requests per slot); the
// rest go FIFO with backfill into free slots (a head blocked longer than the
// limit stops backfilling so large requests are not starved), each taking
// queued requests on its matrix along, up to max_group, as long as the
// slot's vectors fit the heap (else the group shrinks).  Caller holds E.mu.
bool admit(Engine &E, int &ntiles_active)
{
    bool changed = false;
    const double t = now_s();
    std::vector<Request> pending(E.queue.begin(), E.queue.end());
    std::vector<uint8_t> taken(pending.size(), 0);
    bool joined = false;
    for (size_t h = 0; h < pending.size(); ++h)
        for (int i = 0; i < E.max_slots; ++i) {
            Slot &sl = E.slots[i];
            const bool finishing = sl.mixed ? sl.running() == 0 : E.h_done[i] != 0;
            if (!sl.used || sl.fresh || finishing || !same_group(sl.key, pending[h])) continue;
            const int j = sl.free_lane();
            if (j < 0 || sl.running() >= E.max_group) continue;
            sl.lane[j] = pending[h];
            sl.state[j] = kLaneJoining;
            sl.t_start[j] = t;
            sl.sharing[j] = sl.running();
            sl.need_outer[j] = sl.first[j] = sl.outer_ran[j] = sl.last[j] = 0;
            sl.outer[j] = sl.inner_sum[j] = 0;
            sl.final_status[j] = CGX_PENDING;
            taken[h] = 1;
            joined = true;
            break;
        }
    bool blocked_head = false;
    for (size_t h = 0; h < pending.size(); ++h) {
        if (taken[h]) continue;
        int free_slot = -1;
        for (int i = 0; i < E.max_slots; ++i)
            if (!E.slots[i].used) {
                free_slot = i;
                break;
            }
        if (free_slot < 0) break;
        std::vector<size_t> members{h};
        for (size_t k = h + 1; k < pending.size() && (int)members.size() < E.max_group; ++k)
            if (!taken[k] && same_group(pending[h], pending[k])) members.push_back(k);
        bool fits = false;
        size_t off = 0, bytes = 0;
        int nt = 0, K = 1;
        while (!members.empty()) {
            const int g = (int)members.size();
            const bool spare = g < E.max_group && pending[h].A.n_rows >= kSpareLaneRows;
            K = pad_k(g);
            if (K == g && spare) K = pad_k(g + 1);
            bytes = group_bytes(pending[h].A.n_rows, K);
            if (pending[h].mixed) bytes = std::max(bytes, mixed_slot_bytes(pending[h].A.n_rows, K));
            nt = tiles_of(pending[h].A.n_rows, K);
            if (ntiles_active + nt <= E.max_tiles && E.alloc(bytes, off)) {
                fits = true;
                break;
            }
            members.resize(g > 1 ? g / 2 : 0);
        }
        if (!fits) {
            if (h == 0 && t - pending[h].t_submit > E.head_wait_limit) blocked_head = true;
            if (blocked_head) break;
            continue;
        }
        Slot &sl = E.slots[free_slot];
        sl.used = true;
        sl.fresh = true;
        sl.K = K;
        sl.key = pending[h];
        sl.mixed = pending[h].mixed != 0;
        sl.ru = pending[h].mixed == 2;
        sl.lane.assign(K, Request{});
        sl.state.assign(K, kLaneFree);
        sl.t_start.assign(K, t);
        sl.sharing.assign(K, (int)members.size());
        sl.need_outer.assign(K, 0);
        sl.first.assign(K, 0);
        sl.outer_ran.assign(K, 0);
        sl.last.assign(K, 0);
        sl.outer.assign(K, 0);
        sl.inner_sum.assign(K, 0);
        sl.final_status.assign(K, CGX_PENDING);
        for (size_t q = 0; q < members.size(); ++q) {
            sl.lane[q] = pending[members[q]];
            sl.state[q] = kLaneJoining;
            taken[members[q]] = 1;
        }
        sl.off = off;
        sl.bytes = bytes;
        sl.ntiles = nt;
        ntiles_active += nt;
        changed = true;
    }
    if (changed || joined) {
        E.queue.clear();
        for (size_t k = 0; k < pending.size(); ++k)
            if (!taken[k]) E.queue.push_back(pending[k]);
    }
    return changed;
}

void engine_loop(Engine *Ep)
{
    Engine &E = *Ep;
    (void)hipSetDevice(E.device);
    std::vector<int> active;
    bool changed = false;
    int ntiles_active = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(E.mu);
            changed = admit(E, ntiles_active) || changed;
            bool any = false;
            for (const Slot &sl : E.slots) any = any || sl.used;
            if (!any) {
                if (E.stopping && E.queue.empty()) break;
                E.cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        // schedules for fresh slots (tuned once per shape class, in the handle)
        for (Slot &sl : E.slots) {
            if (!sl.used || !sl.fresh) continue;
            cgx_system sys{};
            sys.A = sl.key.A;
            sys.nrhs = sl.K;
            int M = 1;
            if (tune_one(E.c, sys, E.pool + sl.off, sl.bytes, E.stream, M) != CGX_OK) {
                // every waiter wakes and every unfinished ticket reports the failure
                std::lock_guard<std::mutex> lk(E.mu);
                E.fail = CGX_EHIP;
                E.fail_msg = "autotuning failed";
                E.cv_done.notify_all();
                return;
            }
            sl.M = M;
        }
        // iterations this cycle: about 1 ms of device work
        double bytes = 0.0;
        for (const Slot &sl : E.slots)
            if (sl.used)
                bytes += sl.mixed ? 8.0 * sl.key.A.nnz + 40.0 * sl.K * sl.key.A.n_rows
                                  : 12.0 * sl.key.A.nnz + 80.0 * sl.K * sl.key.A.n_rows;
        int iters = (int)(1.0e-3 / (bytes / 4.0e12 + 25.0e-6));
        iters = iters < 1 ? 1 : (iters > 16 ? 16 : iters);
        if (!device_cycle(E, changed, iters, active)) {
            std::lock_guard<std::mutex> lk(E.mu);
            E.cv_done.notify_all();
            return;
        }
        changed = false;
        // retire each finished request (its x copied out at once), and slots
        // whose lanes have all finished
        const double t = now_s();
        std::vector<std::pair<uint64_t, cgx_stats>> finished;
        const BSys *dsys = reinterpret_cast<const BSys *>(E.pool + E.off_sys);
        const BScal *dscal = reinterpret_cast<const BScal *>(E.pool + E.off_scal);
        auto retire = [&](int i, int j, const BScal &v, int iters, int outer) {
            Slot &sl = E.slots[i];
            const Request &q = sl.lane[j];
            cgx_stats st{};
            st.status = v.status == CGX_PENDING ? CGX_NOT_CONVERGED : v.status;
            st.iters = iters;
            st.outer_iters = outer;
            st.slot_requests = sl.sharing[j];
            st.path = 4;
            st.relres = v.bb > 0.0 ? std::sqrt(v.rr / v.bb) : 0.0;
            if (v.bb == 0.0 && v.status == CGX_OK) st.relres = 0.0;
            st.relres_true = -1.0;
            st.queue_ms = 1e3 * (sl.t_start[j] - q.t_submit);
            st.latency_ms = 1e3 * (t - q.t_submit);
            hipLaunchKernelGGL(lane_out_kernel, dim3(256), dim3(kBB), 0, E.stream, dsys, i, j, dscal);
            finished.emplace_back(q.ticket, st);
            sl.state[j] = kLaneFree;
        };
        for (int i : active) {
            Slot &sl = E.slots[i];
            if (!sl.used) continue;
            if (sl.ru) {
                // reliable updates: a lane is finished when a float64 test
                // (start, an update, or its last step) gave a final status;
                // a lane whose binary32 iteration stopped otherwise (cap,
                // breakdown) takes a last float64 step (fold, residual) first
                for (int j = 0; j < sl.K; ++j) {
                    if (sl.state[j] != kLaneRunning) continue;
                    BScal v = E.h_scal[(size_t)i * kMaxK + j];
                    const BScalT<float> &f = E.h_scal32[(size_t)i * kMaxK + j];
                    const bool ran = sl.outer_ran[j] != 0;
                    sl.outer_ran[j] = 0;
                    if (v.status != CGX_PENDING) {
                        if (sl.last[j] && v.status != CGX_OK) v.status = sl.final_status[j];
                        retire(i, j, v, sl.last[j] ? sl.inner_sum[j] : (ran ? 0 : f.iter), v.iter);
                        continue;
                    }
                    if (!ran && !f.active) {
                        sl.final_status[j] = f.status;
                        sl.inner_sum[j] = f.iter;
                        sl.last[j] = 1;
                        sl.need_outer[j] = 1;
                    }
                }
                if (sl.running() > 0) continue;
            } else if (sl.mixed) {
                // a lane whose float64 step ran this cycle is finished if its
                // status is final; a lane whose inner solve ended takes its
                // next float64 step at the next cycle
                for (int j = 0; j < sl.K; ++j) {
                    if (sl.state[j] != kLaneRunning) continue;
                    const BScal &v = E.h_scal[(size_t)i * kMaxK + j];
                    if (sl.outer_ran[j]) {
                        sl.outer_ran[j] = 0;
                        if (v.status != CGX_PENDING) {
                            retire(i, j, v, sl.inner_sum[j], sl.outer[j]);
                            continue;
                        }
                        ++sl.outer[j];
                    }
                    const BScalT<float> &f = E.h_scal32[(size_t)i * kMaxK + j];
                    if (!f.active) {
                        sl.inner_sum[j] += f.iter;
                        sl.need_outer[j] = 1;
                    }
                }
                if (sl.running() > 0) continue;
            } else {
                for (int j = 0; j < sl.K; ++j) {
                    const BScal &v = E.h_scal[(size_t)i * kMaxK + j];
                    if (sl.state[j] != kLaneRunning || (v.active && !E.h_done[i])) continue;
                    retire(i, j, v, v.iter, sl.sharing[j]);
                }
                if (!E.h_done[i]) continue;
            }
            E.release(sl.off, sl.bytes);
            ntiles_active -= sl.ntiles;
            sl.used = false;
            changed = true;
        }
        if (!finished.empty()) {
            if (hipStreamSynchronize(E.stream) != hipSuccess) {
                std::lock_guard<std::mutex> lk(E.mu);
                E.fail = CGX_EHIP;
                E.fail_msg = "stream synchronize failed";
                E.cv_done.notify_all();
                return;
            }
            std::lock_guard<std::mutex> lk(E.mu);
            for (auto &f : finished) {
                Result &r = E.results[f.first];
                r.done = true;
                r.st = f.second;
                ++E.completed;
            }
            E.cv_done.notify_all();
        }
    }
    std::lock_guard<std::mutex> lk(E.mu);
    E.cv_done.notify_all();
}

}  // namespace

int serve_start(Context *c, void *pool, size_t pool_bytes, int32_t max_slots, int32_t max_group)
{
    if (c->engine) {
        set_error("server already running on this handle");
        return CGX_EINVAL;
    }
    Engine *E = new Engine();
    E->c = c;
    E->device = c->device;
    E->pool = static_cast<char *>(pool);
    E->pool_bytes = pool_bytes;
    E->max_slots = max_slots;
    E->max_group = max_group;
    // arena: tables sized for the most tiles the heap can hold
    E->max_tiles = (int64_t)(pool_bytes / (40.0 * tile_rows_for(1, false))) + max_slots + 1;
    size_t off = 0;
    E->off_sys = off;
    off += a256(sizeof(BSys) * max_slots);
    E->off_lanes = off;
    off += a256(sizeof(LanePtr) * kMaxK * max_slots);
    E->off_list = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_list2 = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_scal = off;
    off += a256(sizeof(BScal) * kMaxK * max_slots);
    E->off_done = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_tiles = off;
    off += a256(sizeof(BTile) * E->max_tiles);
    E->off_tiles2 = off;
    off += a256(sizeof(BTile) * E->max_tiles);
    E->off_part = off;
    off += a256(sizeof(double) * 3 * E->max_tiles * kMaxK);
    E->off_sys32 = off;
    off += a256(sizeof(BSysT<float>) * max_slots);
    E->off_list32 = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_scal32 = off;
    off += a256(sizeof(BScalT<float>) * kMaxK * max_slots);
    E->off_done32 = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_bad = off;
    off += a256(sizeof(int32_t) * max_slots);
    E->off_tiles32 = off;
    off += a256(sizeof(BTile) * E->max_tiles);
    E->off_part32 = off;
    off += a256(sizeof(float) * 3 * E->max_tiles * kMaxK);
    E->heap0 = off;
    if (off >= pool_bytes) {
        delete E;
        set_error("pool too small for the server tables");
        return CGX_ENOMEM;
    }
    E->free_list[off] = (pool_bytes - off) & ~(size_t)255;
    E->slots.resize(max_slots);
    hipError_t e = hipHostMalloc(&E->h_scal, sizeof(BScal) * kMaxK * max_slots);
    if (e == hipSuccess) e = hipHostMalloc(&E->h_done, sizeof(int32_t) * max_slots);
    if (e == hipSuccess) e = hipHostMalloc(&E->h_scal32, sizeof(BScalT<float>) * kMaxK * max_slots);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (E->h_scal) (void)hipHostFree(E->h_scal);
        if (E->h_done) (void)hipHostFree(E->h_done);
        if (E->h_scal32) (void)hipHostFree(E->h_scal32);
        delete E;
        set_error(std::string("serve_start: ") + hipGetErrorString(e));
        return CGX_EHIP;
    }
    // the caller's pending work on its stream (e.g. uploads) precedes serving
    (void)hipEventRecord(c->ev_in, c->stream);
    (void)hipStreamWaitEvent(E->stream, c->ev_in, 0);
    c->engine = E;
    E->th = std::thread(engine_loop, E);
    return CGX_OK;
}

int serve_stop(Context *c)
{
    Engine *E = c->engine;
    if (!E) return CGX_OK;
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->stopping = true;
    }
    E->cv_work.notify_all();
    if (E->th.joinable()) E->th.join();
    const int fail = E->fail;
    const std::string msg = E->fail_msg;
    (void)hipStreamSynchronize(E->stream);
    (void)hipStreamDestroy(E->stream);
    (void)hipHostFree(E->h_scal);
    (void)hipHostFree(E->h_done);
    (void)hipHostFree(E->h_scal32);
    delete E;
    c->engine = nullptr;
    if (fail) {
        set_error(msg);
        return fail;
    }
    return CGX_OK;
}

size_t serve_request_bytes(int64_t n_rows) { return request_bytes(n_rows); }

int serve_submit(Context *c, const cgx_csr *A, const double *b, double *x, const cgx_opts *o,
                 uint64_t *ticket)
{
    Engine *E = c->engine;
    if (!E) {
        set_error("server not running");
        return CGX_EINVAL;
    }
    Request q;
    q.A = *A;
    q.b = b;
    q.x = x;
    q.jac = o->precond == CGX_PRECOND_JACOBI ? 1 : 0;
    q.maxit = o->maxit > 0 ? o->maxit : std::max(A->n_rows, 1);
    q.rtol = o->rtol;
    q.mixed = o->precision == CGX_PRECISION_MIXED ? 1 : o->precision == CGX_PRECISION_MIXED_RU ? 2 : 0;
    q.inner_rtol = o->inner_rtol > 0.0 ? o->inner_rtol : (q.mixed == 2 ? 1e-2 : 1e-3);
    q.max_outer = o->max_outer > 0 ? o->max_outer : 100;
    q.bytes = request_bytes(A->n_rows);
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->fail) {
        set_error(E->fail_msg);
        return E->fail;
    }
    if (E->stopping) {
        set_error("server stopping");
        return CGX_EINVAL;
    }
    if (a256(q.bytes) > E->heap_capacity() ||
        tiles_of(A->n_rows, 1) > E->max_tiles || E->max_slots < 1) {
        set_error("request larger than the server pool");
        return CGX_ENOMEM;
    }
    q.ticket = E->next_ticket++;
    q.t_submit = now_s();
    E->results[q.ticket] = Result{};
    E->queue.push_back(q);
    *ticket = q.ticket;
    E->cv_work.notify_all();
    return CGX_OK;
}

int serve_poll(Context *c, uint64_t ticket, cgx_stats *st, bool wait)
{
    Engine *E = c->engine;
    if (!E) {
        set_error("server not running");
        return CGX_EINVAL;
    }
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->results.find(ticket);
    if (it == E->results.end()) {
        set_error("unknown or already collected ticket");
        return CGX_EINVAL;
    }
    if (wait)
        E->cv_done.wait(lk, [&] { return E->results[ticket].done || E->fail; });
    it = E->results.find(ticket);
    if (!it->second.done) {
        if (E->fail) {
            set_error(E->fail_msg);
            return E->fail;
        }
        return CGX_PENDING;
    }
    if (st) *st = it->second.st;
    const int status = it->second.st.status;
    E->results.erase(it);
    return status;
}

}  // namespace cgx
