// Internal declarations shared by the libcgx translation units (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cgx.h"

namespace cgx {

// ------------------------------------------------------------- errors ----

void set_error(const std::string &msg);
void clear_error();

#define CGX_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::cgx::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_));    \
            return CGX_EHIP;                                                             \
        }                                                                                \
    } while (0)

#define CGX_REQUIRE(cond, msg)                                                           \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            ::cgx::set_error(msg);                                                       \
            return CGX_EINVAL;                                                           \
        }                                                                                \
    } while (0)

// -------------------------------------------------------- launch sizes ----

constexpr int kBlock = 256;         // threads per workgroup for streaming kernels
constexpr int kReduceBlocks = 1024; // fixed grid of the standalone reductions
constexpr int kProfWindow = 32;     // profile mode: iterations launched between host checks

// Wave tiles (one wavefront per tile, 64 * E entries per chunk): E = 8
// float64 or 14 binary32 entries per lane.  14 is the fewest that hold 32
// rows of 27 entries (a Q1 tile) in one chunk; the smaller staging area
// (7.3 KB against 8.3 KB at 16) admits more waves per compute unit, which
// measured 88.2 against 91-92 us for the binary32 SpMV of the Q1 128^3
// matrix (float64 at 7 entries, 5.4 KB: no change).
template <typename T>
constexpr int wave_e() { return sizeof(T) == sizeof(double) ? 8 : 14; }

// Rows per wave tile: the largest power of two in [1, 64] whose expected
// entries fill at most 97% of one chunk of 64 * entries_per_lane entries.
int wave_tile_rows(int64_t n_rows, int64_t nnz, int entries_per_lane);

#define CGX_WRT_SWITCH(RT, EXPR_T)    \
    switch (RT) {                     \
        case 1: EXPR_T(1); break;     \
        case 2: EXPR_T(2); break;     \
        case 4: EXPR_T(4); break;     \
        case 8: EXPR_T(8); break;     \
        case 16: EXPR_T(16); break;   \
        case 32: EXPR_T(32); break;   \
        default: EXPR_T(64); break;   \
    }

// Device-side CG state, stored at the start of the solver workspace.  Its
// fields are written by thread 0 of workgroup 0 of the kernel that forms
// them (every workgroup computes the same values) and read by the following
// kernels.
struct CgState {
    double rho;    // r.z of the current iterate (r.r without preconditioner)
    double rho_used; // rho of the iteration in flight (copied by the update kernel)
    double alpha;  // rho / p.q
    double beta;   // rho_new / rho
    double pq;     // p.Ap
    double rr;     // r.r of the current iterate
    double bb;     // b.b
    double stop2;  // (rtol * ||b||)^2
    double rr_true;// ||b - A x||^2 when requested
    double rmax2;  // reliable updates: largest r.r since the last update
    double delta2; // reliable updates: pause when r.r < delta2 * rmax2 (0: never)
    double sigma_prev; // reliable updates (outer state): ||r|| of the previous update
    int32_t iter;  // completed iterations
    int32_t maxit;
    int32_t status;// CGX_* status; CGX_PENDING while iterating
    int32_t done;  // nonzero once converged or failed: later kernels return at once
    int32_t bad;   // set by any thread meeting a non-positive / missing diagonal
    int32_t rec;   // nonzero: record alpha_j, beta_j of iterations j < kCoefRec
    int32_t pad2[4];
};

// CG coefficients recorded per solve (alpha_j, beta_j of the first kCoefRec
// iterations): they define the Lanczos tridiagonal whose extreme eigenvalues
// estimate the spectrum of the (preconditioned) operator.
constexpr int kCoefRec = 4096;

// Extreme eigenvalues of the k x k Lanczos tridiagonal defined by CG
// coefficients coef[2 j] = alpha_j (j < k), coef[2 j + 1] = beta_j (j < k - 1);
// false when k = 0 or a coefficient is not finite and positive.
bool lanczos_extremes(const double *coef, int k, double &lo, double &hi);
// The same with caller storage: work holds at least 3 k doubles.
bool lanczos_extremes_ws(const double *coef, int k, double *work, double &lo, double &hi);

// Bytes of the library's static device scratch (the workspace of
// cgx_cg_solve_noalloc), one copy per GPU for the life of the process.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Device address of the static scratch on the current device (looked up once
// per device); CGX_EHIP if the lookup fails.
int static_scratch_address(int device, void **out);

// Words identifying what a captured graph bakes in: every kernel argument of
// the captured launches (pointers, sizes, offsets), the launch shapes and the
// number of captured iterations.  A cached graph is replayed only when the
// whole key matches.
struct GraphKey {
    std::vector<uint64_t> w;
    GraphKey &add(uint64_t v)
    {
        w.push_back(v);
        return *this;
    }
    GraphKey &ptr(const void *p) { return add((uint64_t)(uintptr_t)p); }
    GraphKey &f64(double v)
    {
        uint64_t b;
        std::memcpy(&b, &v, sizeof b);
        return add(b);
    }
};

// A captured and instantiated HIP graph plus the key it was built for.
struct GraphSlot {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
    bool matches(const GraphKey &k) const { return exec != nullptr && key == k.w; }
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
};

// Handle state.
struct Context {
    int device = 0;
    hipStream_t stream = nullptr;     // caller's stream: all asynchronous calls
    hipStream_t own_stream = nullptr; // solver stream (graph capture needs a non-null stream)
    int num_cu = 256;
    double *scratch = nullptr;     // device: reduction partials of the standalone calls
    CgState *host_state = nullptr; // pinned host copy of the solver state
    double *host_scalar = nullptr; // pinned host word for results returned to the host
    void *static_ws = nullptr;     // device address of the static scratch on this device
    std::vector<double> kappa_host; // host room for the recorded coefficients and the
                                    // Lanczos bisection (5 kCoefRec doubles), sized at create
    hipEvent_t ev0 = nullptr, ev1 = nullptr;      // timing of a solve
    hipEvent_t ev_in = nullptr, ev_out = nullptr; // ordering between the two streams
    hipEvent_t ev_phase[4 * kProfWindow] = {};  // profile mode: 4 per iteration of a window
    GraphSlot graph64;  // float64 CG iterations
    GraphSlot graph32;  // binary32 inner iterations of the refinement
    GraphSlot graph_batch;  // batched CG iterations
    GraphSlot graph_batch32;  // binary32 inner iterations of the refined batch
    // batched-SpMM autotuner: (K, mean row length, log2 rows) -> slice count M
    std::mutex tune_mu;
    std::map<std::tuple<int, int, int>, int> batch_tune;
    int fail_tune = 0;  // test hook: the next fail_tune tuning calls fail (under tune_mu)
    struct Engine *engine = nullptr;  // solve server, while running
};

// ----------------------------------------------------------- launchers ----

int launch_add(Context *c, int64_t n, const double *x, const double *y, double *z);
int launch_axpy(Context *c, int64_t n, double alpha, const double *x, double *y);
int launch_xmul(Context *c, int64_t n, const double *x, const double *y, double *z);
int launch_dot(Context *c, int64_t n, const double *x, const double *y, double *result);
int launch_demote(Context *c, int64_t n, const double *src, float *dst);
int launch_spmv(Context *c, const cgx_csr *A, const double *x, double *y);
int launch_spmv_f32(Context *c, const cgx_csr *A, const float *x, float *y);
int run_csr_validate(Context *c, const cgx_csr *A, int64_t *bad_row);
int sell_bytes(Context *c, const cgx_csr *A, size_t *bytes);
int sell_build(Context *c, const cgx_csr *A, void *buf, size_t bytes, cgx_sell *out);
int launch_sell_spmv(Context *c, const cgx_sell *S, const double *x, double *y);
int launch_sell_spmv_f32(Context *c, const cgx_sell *S, const float *x, float *y);
int run_cg(Context *c, const cgx_csr *A, const cgx_sell *S, const double *b, double *x, void *ws,
           size_t ws_bytes, const cgx_opts *o, cgx_stats *st);
// float64 CG with the static scratch as workspace and the iterations launched
// directly (no graph): allocates nothing.
int run_cg_noalloc(Context *c, const cgx_csr *A, const double *b, double *x, const cgx_opts *o,
                   cgx_stats *st);
size_t cg_workspace_bytes(int64_t n, int64_t nnz, const cgx_opts *o);
size_t batch_workspace_bytes(int32_t nsys, const cgx_system *in);
// Whether wave tiles of rt rows are an instantiated schedule for K = the
// right-hand-side count rounded up to a power of two.
bool batch_wave_schedule_ok(int rt, int K);
int run_batched(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                const cgx_opts *o, cgx_stats *stats);
size_t batch_mixed_workspace_bytes(int32_t nsys, const cgx_system *in);
int run_batched_mixed(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                      const cgx_opts *o, cgx_stats *stats);
int batch_autotune(Context *c, int32_t nsys, const cgx_system *in, void *ws, size_t ws_bytes,
                   std::vector<int> &Ms);
int tune_one(Context *c, const cgx_system &sys, void *ws, size_t ws_bytes, hipStream_t s,
             int &M_out);
int schwarz_bytes(Context *c, const cgx_csr *A, int n_sub, int overlap, size_t *bytes);
int schwarz_build(Context *c, const cgx_csr *A, int n_sub, int overlap, void *buf, size_t bytes,
                  cgx_schwarz *out);
size_t schwarz_workspace_bytes(const cgx_schwarz *S);
int schwarz_solve(Context *c, const cgx_csr *A, const cgx_schwarz *S, const double *b, double *x,
                  void *ws, size_t ws_bytes, const cgx_opts *o, cgx_stats *st);
int serve_start(Context *c, void *pool, size_t pool_bytes, int32_t max_slots, int32_t max_group);
int serve_stop(Context *c);
size_t serve_request_bytes(int64_t n_rows);
int serve_submit(Context *c, const cgx_csr *A, const double *b, double *x, const cgx_opts *o,
                 uint64_t *ticket);
int serve_poll(Context *c, uint64_t ticket, cgx_stats *st, bool wait);

// Lanes per row for the vector CSR kernel, from the mean row length.

}  // namespace cgx
