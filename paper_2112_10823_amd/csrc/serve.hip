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
// Device memory comes only from the caller's pool: a fixed arena (system
// table, lane table, work table, scalars, reduction partials) at its start
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
    size_t off = 0, bytes = 0;      // heap block of the slot's vectors
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
    double head_wait_limit = 0.25;  // s a blocked head may wait before backfilling stops
    uint64_t completed = 0;
    int active_tiles = 0;  // entries of the device work table (engine thread only)

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
           a.maxit == b.maxit && a.rtol == b.rtol;
}

// Device descriptor of slot `si`: interleaved x r p q z of its K lanes and
// dinv at the start of its heap block; b / x of each request through the
// slot's lane table (null for a free lane).
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
    double **vecs[5] = {&S.x, &S.r, &S.p, &S.q, &S.z};
    for (int v = 0; v < 5; ++v) *vecs[v] = reinterpret_cast<double *>(base + v * vb);
    S.dinv = reinterpret_cast<double *>(base + 5 * vb);
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
    S.maxit = q.maxit;
    S.rtol2 = q.rtol * q.rtol;
    return S;
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
        if (sl.used && sl.M < 0) a.wave_lds = kWaveStageBytes;
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
// fresh slots and the lanes requests joined, run `iters` iterations, read
// back the slot states.
bool device_cycle(Engine &E, bool changed, int iters, std::vector<int> &active)
{
    hipStream_t s = E.stream;
    if (changed) {
        std::vector<BSys> sys(E.max_slots);
        std::vector<BTile> tiles, tiles2;
        std::vector<int32_t> list, list2;
        for (int i = 0; i < E.max_slots; ++i) {
            const Slot &sl = E.slots[i];
            if (!sl.used) continue;
            const int tile0 = (int)tiles.size();
            sys[i] = slot_sys(E, i, tile0);
            for (int t = 0; t < sl.ntiles; ++t) {
                BTile bt{};
                bt.sys = i;
                bt.row0 = t * sys[i].trows;
                bt.rows = std::min(sys[i].trows, sys[i].n - bt.row0);
                bt.tile = (int)tiles.size();
                tiles.push_back(bt);
                if (sl.fresh) tiles2.push_back(bt);
            }
            list.push_back(i);
            if (sl.fresh) list2.push_back(i);
        }
        ENG_CHECK(hipMemcpyAsync(E.pool + E.off_sys, sys.data(), sizeof(BSys) * sys.size(),
                                 hipMemcpyHostToDevice, s));
        if (!tiles.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_tiles, tiles.data(), sizeof(BTile) * tiles.size(),
                                     hipMemcpyHostToDevice, s));
        if (!list.empty())
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_list, list.data(), sizeof(int32_t) * list.size(),
                                     hipMemcpyHostToDevice, s));
        if (!list2.empty()) {
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_tiles2, tiles2.data(),
                                     sizeof(BTile) * tiles2.size(), hipMemcpyHostToDevice, s));
            ENG_CHECK(hipMemcpyAsync(E.pool + E.off_list2, list2.data(),
                                     sizeof(int32_t) * list2.size(), hipMemcpyHostToDevice, s));
            const std::vector<BScal> zero(kMaxK);
            const int32_t zd = 0;
            for (int i : list2) {
                LanePtr lanes[kMaxK] = {};
                Slot &sl = E.slots[i];
                for (int j = 0; j < sl.K; ++j)
                    if (sl.state[j] != kLaneFree) lanes[j] = {sl.lane[j].b, sl.lane[j].x};
                ENG_CHECK(hipMemcpyAsync(E.pool + E.off_lanes + sizeof(LanePtr) * kMaxK * i, lanes,
                                         sizeof(lanes), hipMemcpyHostToDevice, s));
                ENG_CHECK(hipMemcpyAsync(E.pool + E.off_scal + sizeof(BScal) * kMaxK * i,
                                         zero.data(), sizeof(BScal) * kMaxK,
                                         hipMemcpyHostToDevice, s));
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
        active.assign(list.begin(), list.end());
        E.active_tiles = (int)tiles.size();
    }
    // requests that joined a free lane of a running slot: set that lane up
    const BArgs m = engine_args(E, false, E.active_tiles, (int)active.size());
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
            hipLaunchKernelGGL(lane_init_kernel, dim3(sl.ntiles), dim3(kBB), 0, s, m, i, j);
            hipLaunchKernelGGL(lane_r0_kernel, dim3(1), dim3(kBB), 0, s, m, i, j);
            ENG_CHECK(hipGetLastError());
            sl.state[j] = kLaneRunning;
        }
    }
    const int ntiles = E.active_tiles;
    if (!active.empty() && ntiles > 0) {
        const BArgs a = engine_args(E, false, ntiles, (int)active.size());
        for (int k = 0; k < iters; ++k) launch_batch_iteration(a, s);
        ENG_CHECK(hipGetLastError());
    }
    ENG_CHECK(hipMemcpyAsync(E.h_done, E.pool + E.off_done, sizeof(int32_t) * E.max_slots,
                             hipMemcpyDeviceToHost, s));
    ENG_CHECK(hipMemcpyAsync(E.h_scal, E.pool + E.off_scal, sizeof(BScal) * kMaxK * E.max_slots,
                             hipMemcpyDeviceToHost, s));
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
            if (!sl.used || sl.fresh || E.h_done[i] || !same_group(sl.key, pending[h])) continue;
            const int j = sl.free_lane();
            if (j < 0 || sl.running() >= E.max_group) continue;
            sl.lane[j] = pending[h];
            sl.state[j] = kLaneJoining;
            sl.t_start[j] = t;
            sl.sharing[j] = sl.running();
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
        sl.lane.assign(K, Request{});
        sl.state.assign(K, kLaneFree);
        sl.t_start.assign(K, t);
        sl.sharing.assign(K, (int)members.size());
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
            if (sl.used) bytes += 12.0 * sl.key.A.nnz + 88.0 * sl.K * sl.key.A.n_rows;
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
        for (int i : active) {
            Slot &sl = E.slots[i];
            if (!sl.used) continue;
            for (int j = 0; j < sl.K; ++j) {
                const BScal &v = E.h_scal[(size_t)i * kMaxK + j];
                if (sl.state[j] != kLaneRunning || (v.active && !E.h_done[i])) continue;
                const Request &q = sl.lane[j];
                cgx_stats st{};
                st.status = v.status == CGX_PENDING ? CGX_NOT_CONVERGED : v.status;
                st.iters = v.iter;
                st.outer_iters = sl.sharing[j];
                st.path = 4;
                st.relres = v.bb > 0.0 ? std::sqrt(v.rr / v.bb) : 0.0;
                if (v.bb == 0.0 && v.status == CGX_OK) st.relres = 0.0;
                st.relres_true = -1.0;
                st.queue_ms = 1e3 * (sl.t_start[j] - q.t_submit);
                st.latency_ms = 1e3 * (t - q.t_submit);
                hipLaunchKernelGGL(lane_out_kernel, dim3(256), dim3(kBB), 0, E.stream, dsys, i, j,
                                   dscal);
                finished.emplace_back(q.ticket, st);
                sl.state[j] = kLaneFree;
            }
            if (!E.h_done[i]) continue;
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
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (E->h_scal) (void)hipHostFree(E->h_scal);
        if (E->h_done) (void)hipHostFree(E->h_done);
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
