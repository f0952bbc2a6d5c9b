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
// (3) p = z + beta p.  The SpMM schedule of a system is either K * M lanes
// per row (lane = m * K + j: right-hand side j, nonzero slice m) or wave
// tiles (M < 0: -M rows per wavefront, col_idx / val staged in LDS), picked
// per shape class by the autotuner unless the system fixes it.  Every
// reduction a system depends on runs over that system's own tiles in a fixed
// order, so a system's iterates are the same bits alone or in any batch
// (given the same schedule).  Converged right-hand sides are masked; a
// system whose right-hand sides are all done is skipped.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "batch_kernels.h"

namespace cgx {

using namespace bk;

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <typename T>
struct PlanT {
    std::vector<BSysT<T>> sys;
    std::vector<BTile> tiles;
    std::vector<int32_t> list;
    size_t off_sys = 0, off_tiles = 0, off_list = 0, off_scal = 0, off_done = 0, off_part = 0,
           off_vec = 0;
    size_t total = 0;
    int64_t nscal = 0;
};
using Plan = PlanT<double>;

// Layout of the workspace and the host copies of the device tables (T: the
// type of the vectors, partials and scalars).
template <typename T>
int build_plan(int32_t nsys, const cgx_system *in, const int *Ms, const cgx_opts *o, PlanT<T> &P)
{
    P.sys.assign(nsys, BSysT<T>{});
    P.tiles.clear();
    P.list.resize(nsys);
    int64_t scal = 0;
    size_t vec_bytes = 0;
    for (int s = 0; s < nsys; ++s) {
        const cgx_system &q = in[s];
        BSysT<T> &S = P.sys[s];
        S.n = q.A.n_rows;
        S.n_cols = q.A.n_cols;
        S.nnz = q.A.nnz;
        S.nrhs = q.nrhs;
        S.K = pad_k(q.nrhs);
        S.M = Ms ? Ms[s] : default_m(S.K, S.n ? (double)S.nnz / S.n : 1.0);
        S.staged = 1;
        S.trows = tile_rows_for(S.K, true);
        S.scal0 = (int)scal;
        S.jac = o && o->precond == CGX_PRECOND_JACOBI ? 1 : 0;
        S.rtol2 = o ? o->rtol * o->rtol : 0.0;
        S.maxit = o && o->maxit > 0 ? o->maxit : std::max(S.n, 1);
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
        P.list[s] = s;
        vec_bytes += 5 * align256((size_t)S.n * S.K * sizeof(T)) + align256((size_t)S.n * sizeof(T));
    }
    if (P.tiles.size() > 0x7fffffff) return CGX_EINVAL;
    P.nscal = scal;
    size_t off = 0;
    P.off_sys = off;
    off += align256(sizeof(BSysT<T>) * nsys);
    P.off_tiles = off;
    off += align256(sizeof(BTile) * std::max<size_t>(P.tiles.size(), 1));
    P.off_list = off;
    off += align256(sizeof(int32_t) * nsys);
    P.off_scal = off;
    off += align256(sizeof(BScalT<T>) * std::max<int64_t>(scal, 1));
    P.off_done = off;
    off += align256(sizeof(int32_t) * nsys);
    P.off_part = off;
    off += align256((size_t)3 * std::max<size_t>(P.tiles.size(), 1) * kMaxK * sizeof(T));
    P.off_vec = off;
    off += vec_bytes;
    P.total = off;
    return CGX_OK;
}

// Krylov vectors of every system from the plan's vector region; matrix and
// caller vectors from `in` (float64 values and B / X).
template <typename T>
void bind_vectors(PlanT<T> &P, int32_t nsys, char *ws)
{
    size_t off = P.off_vec;
    for (int s = 0; s < nsys; ++s) {
        BSysT<T> &S = P.sys[s];
        const size_t vb = align256((size_t)S.n * S.K * sizeof(T));
        T **vecs[5] = {&S.x, &S.r, &S.p, &S.q, &S.z};
        for (T **v : vecs) {
            *v = reinterpret_cast<T *>(ws + off);
            off += vb;
        }
        S.dinv = reinterpret_cast<T *>(ws + off);
        off += align256((size_t)S.n * sizeof(T));
    }
}

void bind_pointers(Plan &P, int32_t nsys, const cgx_system *in, char *ws)
{
    for (int s = 0; s < nsys; ++s) {
        BSys &S = P.sys[s];
        S.rp = in[s].A.row_ptr;
        S.ci = in[s].A.col_idx;
        S.val = in[s].A.val;
        S.B = in[s].B;
        S.X = in[s].X;
    }
    bind_vectors(P, nsys, ws);
}

template <typename T>
BArgsT<T> make_args(const PlanT<T> &P, char *ws)
{
    BArgsT<T> a{};
    a.sys = reinterpret_cast<const BSysT<T> *>(ws + P.off_sys);
    a.tiles = reinterpret_cast<const BTile *>(ws + P.off_tiles);
    a.list = reinterpret_cast<const int32_t *>(ws + P.off_list);
    a.scal = reinterpret_cast<BScalT<T> *>(ws + P.off_scal);
    a.sys_done = reinterpret_cast<int32_t *>(ws + P.off_done);
    a.part = reinterpret_cast<T *>(ws + P.off_part);
    a.ntiles = (int)P.tiles.size();
    a.part_stride = (int64_t)std::max<size_t>(P.tiles.size(), 1) * kMaxK;
    a.nlist = (int)P.sys.size();
    a.wave_lds = 0;
    for (const BSysT<T> &S : P.sys)
        if (S.M < 0) a.wave_lds = kWaveStageBytes;
    return a;
}

template <typename T>
int upload_plan(const PlanT<T> &P, char *w, hipStream_t s)
{
    CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_sys, P.sys.data(), sizeof(BSysT<T>) * P.sys.size(),
                                 hipMemcpyHostToDevice, s));
    CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_tiles, P.tiles.data(), sizeof(BTile) * P.tiles.size(),
                                 hipMemcpyHostToDevice, s));
    CGX_HIP_CHECK(hipMemcpyAsync(w + P.off_list, P.list.data(), sizeof(int32_t) * P.list.size(),
                                 hipMemcpyHostToDevice, s));
    return CGX_OK;
}

// Float32-refined batch, start of an outer step: for every right-hand side
// j still refining (status pending after the float64 residual pass),
// s_j = ||r_j|| and c = float(r / s_j) into the inner right-hand sides
// (caller layout, b32), 0 for the others; the inner solutions are cleared.
// The tiles of the two plans are the same.
__global__ __launch_bounds__(kBB) void refine_rhs_kernel(BArgsT<double> a64, BArgsT<float> a32,
                                                         float *b32)
{
    const BTile t = a64.tiles[blockIdx.x];
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    const int64_t boff = F.B - b32;  // the system's inner right-hand sides in b32
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        if (j >= S.nrhs) continue;
        const BScalT<double> &c = a64.scal[S.scal0 + j];
        const int64_t o = (int64_t)j * S.n + row;
        b32[boff + o] = c.status == CGX_PENDING ? (float)(S.r[e] / sqrt(c.rr)) : 0.0f;
        F.X[o] = 0.0f;
    }
}

// End of an outer step: x = fma(s_j, double(d), x) for the right-hand sides
// that were refined (d: the inner solution, caller layout).
__global__ __launch_bounds__(kBB) void refine_update_kernel(BArgsT<double> a64, BArgsT<float> a32)
{
    const BTile t = a64.tiles[blockIdx.x];
    const BSysT<double> S = a64.sys[t.sys];
    const BSysT<float> F = a32.sys[t.sys];
    const int64_t e0 = (int64_t)t.row0 * S.K, e1 = (int64_t)(t.row0 + t.rows) * S.K;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBB) {
        const int row = (int)(e / S.K), j = (int)(e % S.K);
        if (j >= S.nrhs) continue;
        const BScalT<double> &c = a64.scal[S.scal0 + j];
        if (c.status != CGX_PENDING) continue;
        S.x[e] = __builtin_fma(sqrt(c.rr), (double)F.X[(int64_t)j * S.n + row], S.x[e]);
    }
}

// Workspace of the float32-refined batch: the float64 plan (outer state),
// the binary32 plan at `base32`, then the inner right-hand sides and
// solutions in caller layout (nrhs x n floats per system).
struct MixedLayout {
    Plan P64;
    PlanT<float> P32;
    size_t base32 = 0, off_b32 = 0, off_d32 = 0, total = 0;
    std::vector<size_t> sys_off;  // first float of each system in b32 / d32
};

int mixed_layout(int32_t nsys, const cgx_system *in, const int *Ms, const cgx_opts *o,
                 MixedLayout &L)
{
    cgx_opts o64{};
    o64.rtol = o ? o->rtol : 0.0;
    o64.precond = CGX_PRECOND_NONE;
    int rc = build_plan(nsys, in, Ms, &o64, L.P64);
    if (rc) return rc;
    cgx_opts o32{};
    if (o) o32 = *o;
    o32.rtol = o && o->inner_rtol > 0.0 ? o->inner_rtol : 1e-3;
    rc = build_plan(nsys, in, Ms, &o32, L.P32);
    if (rc) return rc;
    L.base32 = align256(L.P64.total);
    size_t floats = 0;
    L.sys_off.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        L.sys_off[s] = floats;
        floats += (size_t)in[s].nrhs * in[s].A.n_rows;
    }
    L.off_b32 = L.base32 + align256(L.P32.total);
    L.off_d32 = L.off_b32 + align256(floats * sizeof(float) + 4);
    L.total = L.off_d32 + align256(floats * sizeof(float) + 4);
    return CGX_OK;
}

// Key of a graph of K batched iterations: the captured launches take
// exactly the fields of `a` (grid sizes ntiles / nlist, dynamic LDS
// wave_lds), so those and K identify it; the per-system tables they read are
// uploaded before every solve.
template <typename T>
GraphKey batch_key(int K, const BArgsT<T> &a)
{
    GraphKey k;
    k.add(0x42ull).add(sizeof(T)).add((uint64_t)K);
    k.ptr(a.sys).ptr(a.tiles).ptr(a.list).ptr(a.scal).ptr(a.sys_done).ptr(a.part);
    k.add((uint64_t)a.part_stride).add((uint64_t)a.ntiles).add((uint64_t)a.nlist);
    k.add((uint64_t)a.wave_lds);
    return k;
}

// Capture K batched iterations over `a` into `slot` unless its graph was
// captured for the same key.
template <typename T>
int ensure_batch_graph(GraphSlot &slot, int K, const BArgsT<T> &a, hipStream_t s)
{
    const GraphKey key = batch_key<T>(K, a);
    if (slot.matches(key)) return CGX_OK;
    slot.reset();
    CGX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < K; ++k) launch_batch_iteration(a, s);
    hipGraph_t g = nullptr;
    CGX_HIP_CHECK(hipStreamEndCapture(s, &g));
    slot.graph = g;
    CGX_HIP_CHECK(hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0));
    slot.key = key.w;
    return CGX_OK;
}

// K reliable-update iterations captured into `slot` (the binary32 graph
// slot of the handle, keyed apart from the restarted refinement's graph).
int ensure_ru_graph(GraphSlot &slot, int K, const BArgsT<double> &a64, const BArgsT<float> &a32,
                    int max_updates, hipStream_t s)
{
    GraphKey key = batch_key<float>(K, a32);
    key.add(0x5255ull).ptr(a64.sys).ptr(a64.tiles).ptr(a64.list).ptr(a64.scal).ptr(a64.part);
    key.ptr(a64.sys_done).add((uint64_t)a64.part_stride).add((uint64_t)a64.ntiles);
    key.add((uint64_t)a64.nlist).add((uint64_t)a64.wave_lds);
    key.add((uint64_t)max_updates);
    if (slot.matches(key)) return CGX_OK;
    slot.reset();
    CGX_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < K; ++k) launch_ru_iteration(a64, a32, max_updates, s);
    hipGraph_t g = nullptr;
    CGX_HIP_CHECK(hipStreamEndCapture(s, &g));
    slot.graph = g;
    CGX_HIP_CHECK(hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0));
    slot.key = key.w;
    return CGX_OK;
}

// Two timing events destroyed on every exit path.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

bool batch_wave_schedule_ok(int rt, int K) { return wave_schedule_ok(rt, K); }

// Autotuner: per shape class (K, mean row length, log2 rows) time the SpMM
// phase of the first system of that class alone for every candidate slice
// count M and keep the fastest.  Results stay in the handle, so a class is
// tuned once and later solves (batch, single, served) use the same schedule.
int tune_one(Context *c, const cgx_system &sys, void *ws, size_t ws_bytes, hipStream_t s, int &M_out)
{
    const int K = pad_k(sys.nrhs);
    const auto key = shape_key(K, sys.A.n_rows, sys.A.nnz);
    {
        std::lock_guard<std::mutex> lk(c->tune_mu);
        if (c->fail_tune > 0) {  // test hook: fail before any launch
            --c->fail_tune;
            set_error("autotuning failed (forced)");
            return CGX_EHIP;
        }
        auto it = c->batch_tune.find(key);
        if (it != c->batch_tune.end()) {
            M_out = it->second;
            return CGX_OK;
        }
    }
    const double mean = sys.A.n_rows ? (double)sys.A.nnz / sys.A.n_rows : 1.0;
    float best_ms = 1e30f;
    int best_m = default_m(K, mean);
    EventPair ev;
    CGX_HIP_CHECK(hipEventCreate(&ev.e0));
    CGX_HIP_CHECK(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    for (int M : m_candidates(K, sys.A.n_rows, sys.A.nnz)) {
        int Mv[1] = {M};
        Plan P;
        if (build_plan(1, &sys, Mv, nullptr, P) != CGX_OK || P.total > ws_bytes) continue;
        char *w = static_cast<char *>(ws);
        bind_pointers(P, 1, &sys, w);
        int rc = upload_plan(P, w, s);
        if (rc) return rc;
        BArgs a = make_args(P, w);
        hipLaunchKernelGGL((batch_scal_init_kernel<double>), dim3((unsigned)((P.nscal + 255) / 256 + 1)),
                           dim3(256), 0, s, a.scal, P.nscal, a.sys_done, 1);
        // p holds whatever the workspace held: only the time is used
        for (int rep = 0; rep < 2; ++rep)
            hipLaunchKernelGGL((batch_spmm_kernel<double>), dim3(a.ntiles), dim3(kBB), a.wave_lds, s, a);
        CGX_HIP_CHECK(hipEventRecord(e0, s));
        for (int rep = 0; rep < 5; ++rep)
            hipLaunchKernelGGL((batch_spmm_kernel<double>), dim3(a.ntiles), dim3(kBB), a.wave_lds, s, a);
        CGX_HIP_CHECK(hipEventRecord(e1, s));
        CGX_HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CGX_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best_m = M;
        }
    }
    std::lock_guard<std::mutex> lk(c->tune_mu);
    c->batch_tune[key] = best_m;
    M_out = best_m;
    return CGX_OK;
}

int batch_autotune(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                   std::vector<int> &Ms)
{
    Ms.assign(nsys, 0);
    for (int s = 0; s < nsys; ++s) {
        if (in[s].schedule != 0) {  // fixed by the caller
            Ms[s] = in[s].schedule;
            continue;
        }
        int rc = tune_one(c, in[s], ws, ws_bytes, c->own_stream, Ms[s]);
        if (rc) return rc;
    }
    return CGX_OK;
}

size_t batch_workspace_bytes(int32_t nsys, const cgx_system *in)
{
    Plan P;
    if (build_plan(nsys, in, nullptr, nullptr, P) != CGX_OK) return 0;
    return P.total;
}

int run_batched(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                const cgx_opts *o, cgx_stats *stats)
{
    hipStream_t s = c->own_stream;
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    std::vector<int> Ms;
    int rc = batch_autotune(c, nsys, in, ws, ws_bytes, Ms);
    if (rc) return rc;
    Plan P;
    rc = build_plan(nsys, in, Ms.data(), o, P);
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
    int maxit = 1;
    for (const BSys &S : P.sys) maxit = std::max(maxit, S.maxit);
    BArgs a = make_args(P, w);

    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    rc = upload_plan(P, w, s);
    if (rc) return rc;
    const int64_t init_n = std::max<int64_t>(P.nscal, nsys);
    hipLaunchKernelGGL((batch_scal_init_kernel<double>), dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0,
                       s, a.scal, P.nscal, a.sys_done, nsys);
    hipLaunchKernelGGL((batch_in_kernel<double>), dim3(a.ntiles), dim3(kBB), 0, s, a);
    hipLaunchKernelGGL((batch_init_kernel<double>), dim3(a.ntiles), dim3(kBB), a.wave_lds, s, a);
    hipLaunchKernelGGL((batch_r0_kernel<double>), dim3(a.nlist), dim3(kBB), 0, s, a);
    CGX_HIP_CHECK(hipGetLastError());

    // iterations per replay: about 2 ms of work between host checks
    double bytes = 0.0;
    for (const BSys &S : P.sys) bytes += 12.0 * S.nnz + 80.0 * S.K * S.n;
    int K = o->check_every;
    if (K <= 0) {
        const double t_iter = bytes / 4.0e12 + 15.0e-6;
        K = (int)(2.0e-3 / t_iter);
        K = K < 2 ? 2 : (K > 32 ? 32 : K);
    }
    rc = ensure_batch_graph(c->graph_batch, K, a, s);
    if (rc) return rc;
    GraphSlot &slot = c->graph_batch;
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
    hipLaunchKernelGGL((batch_out_kernel<double>), dim3(a.ntiles), dim3(kBB), 0, s, a);
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
            st = cgx_stats{};
            st.status = v.status == CGX_PENDING ? CGX_NOT_CONVERGED : v.status;
            st.iters = v.iter;
            st.path = 3;
            st.relres = v.bb > 0.0 ? std::sqrt(v.rr / v.bb) : 0.0;
            st.relres_true = -1.0;
            st.device_ms = ms;
            if (st.status != CGX_OK && worst == CGX_OK) worst = st.status;
        }
    }
    return worst;
}

size_t batch_mixed_workspace_bytes(int32_t nsys, const cgx_system *in)
{
    MixedLayout L;
    if (mixed_layout(nsys, in, nullptr, nullptr, L) != CGX_OK) return 0;
    return L.total;
}

// Binary32 CG with float64 reliable updates for the whole batch (see the
// reliable-update kernels above): float64 r = b - A x and the stopping test
// per right-hand side, the binary32 setup on float(r / ||r||) for the
// others, then graph replays of K iterations (the binary32 phase kernels and
// the update kernels) until every system is done, a final fold of the
// pending corrections and a float64 residual pass for the statistics.
static int run_batched_ru(Context *c, int32_t nsys, const cgx_system *in, void *ws,
                          size_t ws_bytes, const cgx_opts *o_in, cgx_stats *stats)
{
    cgx_opts o = *o_in;
    if (!(o.inner_rtol > 0.0)) o.inner_rtol = 1e-2;  // delta of the update test
    hipStream_t s = c->own_stream;
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    std::vector<int> Ms;
    int rc = batch_autotune(c, nsys, in, ws, ws_bytes, Ms);
    if (rc) return rc;
    MixedLayout L;
    rc = mixed_layout(nsys, in, Ms.data(), &o, L);
    if (rc) {
        set_error("batch too large");
        return rc;
    }
    if (ws_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    char *w32 = w + L.base32;
    float *b32 = reinterpret_cast<float *>(w + L.off_b32);
    float *d32 = reinterpret_cast<float *>(w + L.off_d32);
    bind_pointers(L.P64, nsys, in, w);
    for (int i = 0; i < nsys; ++i) {
        BSysT<float> &F = L.P32.sys[i];
        F.rp = in[i].A.row_ptr;
        F.ci = in[i].A.col_idx;
        F.val = in[i].A.val32;
        F.B = b32 + L.sys_off[i];
        F.X = d32 + L.sys_off[i];
        F.ru = 1;
    }
    bind_vectors(L.P32, nsys, w32);
    const BArgsT<double> a64 = make_args(L.P64, w);
    const BArgsT<float> a32 = make_args(L.P32, w32);
    int maxit = 1;
    for (const BSysT<float> &F : L.P32.sys) maxit = std::max(maxit, F.maxit);

    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    rc = upload_plan(L.P64, w, s);
    if (rc) return rc;
    rc = upload_plan(L.P32, w32, s);
    if (rc) return rc;
    const int64_t n64 = std::max<int64_t>(L.P64.nscal, nsys);
    const int64_t n32 = std::max<int64_t>(L.P32.nscal, nsys);
    hipLaunchKernelGGL((batch_scal_init_kernel<double>), dim3((unsigned)((n64 + 255) / 256)),
                       dim3(256), 0, s, a64.scal, L.P64.nscal, a64.sys_done, nsys);
    hipLaunchKernelGGL((batch_in_kernel<double>), dim3(a64.ntiles), dim3(kBB), 0, s, a64);
    hipLaunchKernelGGL((batch_init_kernel<double>), dim3(a64.ntiles), dim3(kBB), a64.wave_lds, s,
                       a64);
    hipLaunchKernelGGL((batch_r0_kernel<double>), dim3(a64.nlist), dim3(kBB), 0, s, a64);
    hipLaunchKernelGGL(refine_rhs_kernel, dim3(a64.ntiles), dim3(kBB), 0, s, a64, a32, b32);
    hipLaunchKernelGGL((batch_scal_init_kernel<float>), dim3((unsigned)((n32 + 255) / 256)),
                       dim3(256), 0, s, a32.scal, L.P32.nscal, a32.sys_done, nsys);
    hipLaunchKernelGGL((batch_in_kernel<float>), dim3(a32.ntiles), dim3(kBB), 0, s, a32);
    hipLaunchKernelGGL((batch_init_kernel<float>), dim3(a32.ntiles), dim3(kBB), a32.wave_lds, s,
                       a32);
    hipLaunchKernelGGL((batch_r0_kernel<float>), dim3(a32.nlist), dim3(kBB), 0, s, a32);
    hipLaunchKernelGGL(ru_start_kernel, dim3(a32.nlist), dim3(kBB), 0, s, a64, a32);
    CGX_HIP_CHECK(hipGetLastError());

    // binary32 iterations per graph replay: about 2 ms of work between checks
    double bytes = 0.0;
    for (const BSysT<float> &F : L.P32.sys) bytes += 8.0 * F.nnz + 40.0 * F.K * F.n;
    int K = o.check_every;
    if (K <= 0) {
        const double t_iter = bytes / 4.0e12 + 40.0e-6;
        K = (int)(2.0e-3 / t_iter);
        K = K < 2 ? 2 : (K > 32 ? 32 : K);
    }
    const int max_updates = o.max_outer > 0 ? o.max_outer : 100;
    rc = ensure_ru_graph(c->graph_batch32, K, a64, a32, max_updates, s);
    if (rc) return rc;
    GraphSlot &slot = c->graph_batch32;
    std::vector<int32_t> done(nsys);
    const int64_t max_replays = (int64_t)maxit / K + 2;
    for (int64_t rep = 0; rep < max_replays; ++rep) {
        CGX_HIP_CHECK(hipMemcpyAsync(done.data(), a32.sys_done, sizeof(int32_t) * nsys,
                                     hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        bool all = true;
        for (int32_t d : done) all = all && d;
        if (all) break;
        CGX_HIP_CHECK(hipGraphLaunch(slot.exec, s));
    }
    hipLaunchKernelGGL(ru_final_fold_kernel, dim3(a64.ntiles), dim3(kBB), 0, s, a64, a32);
    CGX_HIP_CHECK(hipGetLastError());
    std::vector<BScalT<double>> h64(L.P64.nscal);
    std::vector<BScalT<float>> h32(L.P32.nscal);
    CGX_HIP_CHECK(hipMemcpyAsync(h64.data(), a64.scal, sizeof(BScalT<double>) * L.P64.nscal,
                                 hipMemcpyDeviceToHost, s));
    CGX_HIP_CHECK(hipMemcpyAsync(h32.data(), a32.scal, sizeof(BScalT<float>) * L.P32.nscal,
                                 hipMemcpyDeviceToHost, s));
    // float64 residual of the result for the statistics (and x = 0 where b = 0)
    hipLaunchKernelGGL((batch_init_kernel<double>), dim3(a64.ntiles), dim3(kBB), a64.wave_lds, s,
                       a64);
    hipLaunchKernelGGL((batch_r0_kernel<double>), dim3(a64.nlist), dim3(kBB), 0, s, a64);
    hipLaunchKernelGGL((batch_out_kernel<double>), dim3(a64.ntiles), dim3(kBB), 0, s, a64);
    CGX_HIP_CHECK(hipGetLastError());
    std::vector<BScalT<double>> hf(L.P64.nscal);
    CGX_HIP_CHECK(hipMemcpyAsync(hf.data(), a64.scal, sizeof(BScalT<double>) * L.P64.nscal,
                                 hipMemcpyDeviceToHost, s));
    CGX_HIP_CHECK(hipEventRecord(c->ev1, s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.0f;
    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    CGX_HIP_CHECK(hipEventRecord(c->ev_out, s));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_out, 0));

    int worst = CGX_OK;
    int64_t k = 0;
    for (int sidx = 0; sidx < nsys; ++sidx) {
        const BSysT<double> &S = L.P64.sys[sidx];
        for (int j = 0; j < S.nrhs; ++j, ++k) {
            const BScalT<double> &v = h64[S.scal0 + j];
            const BScalT<float> &f = h32[S.scal0 + j];
            const BScalT<double> &r = hf[S.scal0 + j];
            cgx_stats &st = stats[k];
            st = cgx_stats{};
            // float64 status when the float64 test ended it, else the
            // binary32 iteration's (cap, breakdown), else not converged
            st.status = v.status != CGX_PENDING ? v.status
                        : (f.status != CGX_PENDING && f.status != CGX_OK) ? f.status
                                                                          : CGX_NOT_CONVERGED;
            st.iters = f.iter;
            st.outer_iters = v.iter;
            st.path = 3;
            st.relres = r.bb > 0.0 ? std::sqrt(r.rr / r.bb) : 0.0;
            st.relres_true = st.relres;
            st.device_ms = ms;
            if (st.status != CGX_OK && worst == CGX_OK) worst = st.status;
        }
    }
    return worst;
}

// Float64 outer refinement around binary32 inner batched CG (the mixed
// precision of the single-system solve, for every (system, right-hand side)
// of the batch at once): r = b - A x in float64 with the float64 kernels;
// right-hand sides with ||r|| <= rtol ||b|| are done; for the others c =
// float(r / ||r||), d from binary32 CG (values A.val32, binary32 vectors,
// scalars and sums) from 0 to inner_rtol, then x += ||r|| d.  Every phase of
// an outer step is one launch over all systems.
int run_batched_mixed(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                      const cgx_opts *o, cgx_stats *stats)
{
    if (o->precision == CGX_PRECISION_MIXED_RU)
        return run_batched_ru(c, nsys, in, ws, ws_bytes, o, stats);
    hipStream_t s = c->own_stream;
    CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
    CGX_HIP_CHECK(hipStreamWaitEvent(s, c->ev_in, 0));
    std::vector<int> Ms;
    int rc = batch_autotune(c, nsys, in, ws, ws_bytes, Ms);
    if (rc) return rc;
    MixedLayout L;
    rc = mixed_layout(nsys, in, Ms.data(), o, L);
    if (rc) {
        set_error("batch too large");
        return rc;
    }
    if (ws_bytes < L.total) {
        set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
        return CGX_ENOMEM;
    }
    char *w = static_cast<char *>(ws);
    char *w32 = w + L.base32;
    float *b32 = reinterpret_cast<float *>(w + L.off_b32);
    float *d32 = reinterpret_cast<float *>(w + L.off_d32);
    bind_pointers(L.P64, nsys, in, w);
    for (int i = 0; i < nsys; ++i) {
        BSysT<float> &F = L.P32.sys[i];
        F.rp = in[i].A.row_ptr;
        F.ci = in[i].A.col_idx;
        F.val = in[i].A.val32;
        F.B = b32 + L.sys_off[i];
        F.X = d32 + L.sys_off[i];
    }
    bind_vectors(L.P32, nsys, w32);
    const BArgsT<double> a64 = make_args(L.P64, w);
    const BArgsT<float> a32 = make_args(L.P32, w32);
    const int max_outer = o->max_outer > 0 ? o->max_outer : 100;
    int maxit = 1;
    for (const BSysT<float> &F : L.P32.sys) maxit = std::max(maxit, F.maxit);

    CGX_HIP_CHECK(hipEventRecord(c->ev0, s));
    rc = upload_plan(L.P64, w, s);
    if (rc) return rc;
    rc = upload_plan(L.P32, w32, s);
    if (rc) return rc;
    const int64_t n64 = std::max<int64_t>(L.P64.nscal, nsys);
    hipLaunchKernelGGL((batch_scal_init_kernel<double>), dim3((unsigned)((n64 + 255) / 256)),
                       dim3(256), 0, s, a64.scal, L.P64.nscal, a64.sys_done, nsys);
    hipLaunchKernelGGL((batch_in_kernel<double>), dim3(a64.ntiles), dim3(kBB), 0, s, a64);
    CGX_HIP_CHECK(hipGetLastError());

    // binary32 iterations per graph replay: about 2 ms of work between checks
    double bytes = 0.0;
    for (const BSysT<float> &F : L.P32.sys) bytes += 8.0 * F.nnz + 40.0 * F.K * F.n;
    int K = o->check_every;
    if (K <= 0) {
        const double t_iter = bytes / 4.0e12 + 15.0e-6;
        K = (int)(2.0e-3 / t_iter);
        K = K < 2 ? 2 : (K > 32 ? 32 : K);
    }
    rc = ensure_batch_graph(c->graph_batch32, K, a32, s);
    if (rc) return rc;
    GraphSlot &slot = c->graph_batch32;

    std::vector<BScalT<double>> h64(L.P64.nscal);
    std::vector<BScalT<float>> h32(L.P32.nscal);
    std::vector<int32_t> inner(L.P64.nscal, 0), outer(L.P64.nscal, 0), done(nsys);
    const int64_t n32 = std::max<int64_t>(L.P32.nscal, nsys);
    for (int step = 0;; ++step) {
        // float64 residual r = b - A x and its norms; rr <= rtol^2 bb -> done
        hipLaunchKernelGGL((batch_init_kernel<double>), dim3(a64.ntiles), dim3(kBB), a64.wave_lds,
                           s, a64);
        hipLaunchKernelGGL((batch_r0_kernel<double>), dim3(a64.nlist), dim3(kBB), 0, s, a64);
        CGX_HIP_CHECK(hipGetLastError());
        CGX_HIP_CHECK(hipMemcpyAsync(h64.data(), a64.scal, sizeof(BScalT<double>) * L.P64.nscal,
                                     hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        bool any = false;
        for (const auto &v : h64) any = any || v.status == CGX_PENDING;
        if (!any || step >= max_outer) break;
        for (size_t k = 0; k < h64.size(); ++k) outer[k] += h64[k].status == CGX_PENDING;
        // inner binary32 solves of every refining right-hand side, together
        hipLaunchKernelGGL(refine_rhs_kernel, dim3(a64.ntiles), dim3(kBB), 0, s, a64, a32, b32);
        hipLaunchKernelGGL((batch_scal_init_kernel<float>), dim3((unsigned)((n32 + 255) / 256)),
                           dim3(256), 0, s, a32.scal, L.P32.nscal, a32.sys_done, nsys);
        hipLaunchKernelGGL((batch_in_kernel<float>), dim3(a32.ntiles), dim3(kBB), 0, s, a32);
        hipLaunchKernelGGL((batch_init_kernel<float>), dim3(a32.ntiles), dim3(kBB), a32.wave_lds,
                           s, a32);
        hipLaunchKernelGGL((batch_r0_kernel<float>), dim3(a32.nlist), dim3(kBB), 0, s, a32);
        CGX_HIP_CHECK(hipGetLastError());
        const int64_t max_replays = (int64_t)maxit / K + 2;
        for (int64_t rep = 0; rep < max_replays; ++rep) {
            CGX_HIP_CHECK(hipMemcpyAsync(done.data(), a32.sys_done, sizeof(int32_t) * nsys,
                                         hipMemcpyDeviceToHost, s));
            CGX_HIP_CHECK(hipStreamSynchronize(s));
            bool all = true;
            for (int32_t d : done) all = all && d;
            if (all) break;
            CGX_HIP_CHECK(hipGraphLaunch(slot.exec, s));
        }
        hipLaunchKernelGGL((batch_out_kernel<float>), dim3(a32.ntiles), dim3(kBB), 0, s, a32);
        hipLaunchKernelGGL(refine_update_kernel, dim3(a64.ntiles), dim3(kBB), 0, s, a64, a32);
        CGX_HIP_CHECK(hipGetLastError());
        CGX_HIP_CHECK(hipMemcpyAsync(h32.data(), a32.scal, sizeof(BScalT<float>) * L.P32.nscal,
                                     hipMemcpyDeviceToHost, s));
        CGX_HIP_CHECK(hipStreamSynchronize(s));
        for (size_t k = 0; k < h32.size(); ++k) inner[k] += h32[k].iter;
    }
    hipLaunchKernelGGL((batch_out_kernel<double>), dim3(a64.ntiles), dim3(kBB), 0, s, a64);
    CGX_HIP_CHECK(hipGetLastError());
    CGX_HIP_CHECK(hipEventRecord(c->ev1, s));
    CGX_HIP_CHECK(hipStreamSynchronize(s));
    float ms = 0.0f;
    CGX_HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    CGX_HIP_CHECK(hipEventRecord(c->ev_out, s));
    CGX_HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_out, 0));

    int worst = CGX_OK;
    int64_t k = 0;
    for (int sidx = 0; sidx < nsys; ++sidx) {
        const BSysT<double> &S = L.P64.sys[sidx];
        for (int j = 0; j < S.nrhs; ++j, ++k) {
            const BScalT<double> &v = h64[S.scal0 + j];
            cgx_stats &st = stats[k];
            st = cgx_stats{};
            st.status = v.status == CGX_PENDING ? CGX_NOT_CONVERGED : v.status;
            st.iters = inner[S.scal0 + j];
            st.outer_iters = outer[S.scal0 + j];
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
