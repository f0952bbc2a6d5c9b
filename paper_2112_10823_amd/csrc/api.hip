// extern "C" entry points of libcgx: argument checks, handle lifetime and
// dispatch to the kernels.  No exception crosses this boundary.
#include <cstring>
#include <new>

#include "cgx_internal.h"

namespace cgx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

}  // namespace cgx

using cgx::Context;

namespace {

Context *ctx_of(cgx_handle h) { return reinterpret_cast<Context *>(h); }

bool overlaps(const void *a, size_t an, const void *b, size_t bn)
{
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + bn && y < x + an;
}

int check_csr(const cgx_csr *A, bool need_val, bool need_val32)
{
    CGX_REQUIRE(A != nullptr, "A is NULL");
    CGX_REQUIRE(A->n_rows >= 0 && A->n_cols >= 0, "negative matrix dimension");
    CGX_REQUIRE(A->nnz >= 0 && A->nnz < ((int64_t)1 << 31), "nnz must be in [0, 2^31)");
    CGX_REQUIRE(A->row_ptr != nullptr, "row_ptr is NULL");
    if (A->nnz > 0) {
        CGX_REQUIRE(A->col_idx != nullptr, "col_idx is NULL");
        if (need_val) CGX_REQUIRE(A->val != nullptr, "val is NULL");
        if (need_val32) CGX_REQUIRE(A->val32 != nullptr, "val32 is NULL");
    }
    return CGX_OK;
}

template <class F>
int guarded(F &&f)
{
    try {
        cgx::clear_error();
        return f();
    } catch (const std::bad_alloc &) {
        cgx::set_error("host allocation failed");
        return CGX_ENOMEM;
    } catch (...) {
        cgx::set_error("internal error");
        return CGX_EHIP;
    }
}

}  // namespace

extern "C" {

const char *cgx_last_error(void) { return cgx::g_last_error.c_str(); }

int cgx_version(void) { return 100; }

int cgx_create(cgx_handle *out, int device, void *stream)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        int ndev = 0;
        CGX_HIP_CHECK(hipGetDeviceCount(&ndev));
        CGX_REQUIRE(device >= 0 && device < ndev, "no such device");
        CGX_HIP_CHECK(hipSetDevice(device));
        Context *c = new Context();
        c->device = device;
        c->stream = static_cast<hipStream_t>(stream);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            c->num_cu = prop.multiProcessorCount;
        const size_t scratch_bytes = (size_t)2 * cgx::kReduceBlocks * sizeof(double) + 256;
        hipError_t e = hipMalloc(&c->scratch, scratch_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&c->host_state, sizeof(cgx::CgState));
        if (e == hipSuccess) e = hipHostMalloc(&c->host_scalar, sizeof(double));
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&c->ev0);
        if (e == hipSuccess) e = hipEventCreate(&c->ev1);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
        for (int i = 0; i < 4 * cgx::kProfWindow && e == hipSuccess; ++i)
            e = hipEventCreate(&c->ev_phase[i]);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        c->kappa_host.assign(5 * (size_t)cgx::kCoefRec, 0.0);
        if (e == hipSuccess && cgx::static_scratch_address(device, &c->static_ws) != CGX_OK) {
            const std::string msg = cgx_last_error();
            cgx_destroy(reinterpret_cast<cgx_handle>(c));
            cgx::set_error("cgx_create: " + msg);
            return CGX_EHIP;
        }
        if (e != hipSuccess) {
            cgx::set_error(std::string("cgx_create: ") + hipGetErrorString(e));
            cgx_destroy(reinterpret_cast<cgx_handle>(c));
            return CGX_EHIP;
        }
        *out = reinterpret_cast<cgx_handle>(c);
        return CGX_OK;
    });
}

int cgx_destroy(cgx_handle h)
{
    Context *c = ctx_of(h);
    if (!c) return CGX_OK;
    if (c->engine) (void)cgx::serve_stop(c);
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->own_stream) (void)hipStreamSynchronize(c->own_stream);
    c->graph64.reset();
    c->graph32.reset();
    c->graph_batch.reset();
    c->graph_batch32.reset();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (int i = 0; i < 4 * cgx::kProfWindow; ++i)
        if (c->ev_phase[i]) (void)hipEventDestroy(c->ev_phase[i]);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_scalar) (void)hipHostFree(c->host_scalar);
    if (c->scratch) (void)hipFree(c->scratch);
    delete c;
    return CGX_OK;
}

int cgx_set_stream(cgx_handle h, void *stream)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        ctx_of(h)->stream = static_cast<hipStream_t>(stream);
        return CGX_OK;
    });
}

int cgx_csr_validate(cgx_handle h, const cgx_csr *A, int64_t *bad_row)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        int rc = check_csr(A, false, false);
        if (rc) return rc;
        return cgx::run_csr_validate(ctx_of(h), A, bad_row);
    });
}

int cgx_csr_spmv(cgx_handle h, const cgx_csr *A, const double *x, double *y)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        int rc = check_csr(A, true, false);
        if (rc) return rc;
        if (A->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(y != nullptr && (x != nullptr || A->n_cols == 0), "x or y is NULL");
        CGX_REQUIRE(!overlaps(x, (size_t)A->n_cols * 8, y, (size_t)A->n_rows * 8),
                    "y overlaps x");
        return cgx::launch_spmv(ctx_of(h), A, x, y);
    });
}

int cgx_csr_spmv_f32(cgx_handle h, const cgx_csr *A, const float *x, float *y)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        int rc = check_csr(A, false, true);
        if (rc) return rc;
        if (A->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(y != nullptr && (x != nullptr || A->n_cols == 0), "x or y is NULL");
        CGX_REQUIRE(!overlaps(x, (size_t)A->n_cols * 4, y, (size_t)A->n_rows * 4),
                    "y overlaps x");
        return cgx::launch_spmv_f32(ctx_of(h), A, x, y);
    });
}

static int check_vec3(cgx_handle h, int64_t n, const void *x, const void *y, const void *z,
                      bool z_may_alias)
{
    CGX_REQUIRE(h != nullptr, "handle is NULL");
    CGX_REQUIRE(n >= 0, "negative length");
    if (n == 0) return CGX_OK;
    CGX_REQUIRE(x && y && z, "NULL vector");
    const size_t nb = (size_t)n * 8;
    if (z_may_alias) {
        CGX_REQUIRE(z == x || !overlaps(z, nb, x, nb), "z partially overlaps x");
        CGX_REQUIRE(z == y || !overlaps(z, nb, y, nb), "z partially overlaps y");
    } else {
        CGX_REQUIRE(!overlaps(x, nb, y, nb), "x and y overlap");
    }
    return CGX_OK;
}

int cgx_add(cgx_handle h, int64_t n, const double *x, const double *y, double *z)
{
    return guarded([&]() -> int {
        int rc = check_vec3(h, n, x, y, z, true);
        if (rc || n == 0) return rc;
        return cgx::launch_add(ctx_of(h), n, x, y, z);
    });
}

int cgx_axpy(cgx_handle h, int64_t n, double alpha, const double *x, double *y)
{
    return guarded([&]() -> int {
        int rc = check_vec3(h, n, x, y, y, false);
        if (rc || n == 0) return rc;
        return cgx::launch_axpy(ctx_of(h), n, alpha, x, y);
    });
}

int cgx_xmul(cgx_handle h, int64_t n, const double *x, const double *y, double *z)
{
    return guarded([&]() -> int {
        int rc = check_vec3(h, n, x, y, z, true);
        if (rc || n == 0) return rc;
        return cgx::launch_xmul(ctx_of(h), n, x, y, z);
    });
}

int cgx_dot(cgx_handle h, int64_t n, const double *x, const double *y, double *result)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(n >= 0, "negative length");
        CGX_REQUIRE(result != nullptr, "result is NULL");
        CGX_REQUIRE(n == 0 || (x && y), "NULL vector");
        return cgx::launch_dot(ctx_of(h), n, x, y, result);
    });
}

int cgx_dot_sync(cgx_handle h, int64_t n, const double *x, const double *y, double *result_host)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(n >= 0, "negative length");
        CGX_REQUIRE(result_host != nullptr, "result_host is NULL");
        CGX_REQUIRE(n == 0 || (x && y), "NULL vector");
        Context *c = ctx_of(h);
        // the result word sits after the reduction partials in the handle's scratch
        double *dres = c->scratch + 2 * cgx::kReduceBlocks;
        int rc = cgx::launch_dot(c, n, x, y, dres);
        if (rc) return rc;
        CGX_HIP_CHECK(hipMemcpyAsync(c->host_scalar, dres, sizeof(double), hipMemcpyDeviceToHost,
                                     c->stream));
        CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
        *result_host = *c->host_scalar;
        return CGX_OK;
    });
}

int cgx_demote(cgx_handle h, int64_t n, const double *src, float *dst)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(n >= 0, "negative length");
        if (n == 0) return CGX_OK;
        CGX_REQUIRE(src && dst, "NULL vector");
        CGX_REQUIRE(!overlaps(src, (size_t)n * 8, dst, (size_t)n * 4), "dst overlaps src");
        return cgx::launch_demote(ctx_of(h), n, src, dst);
    });
}

size_t cgx_cg_workspace_bytes(int64_t n_rows, int64_t nnz, const cgx_opts *opts)
{
    if (n_rows < 0 || nnz < 0 || opts == nullptr) return 0;
    try {
        return cgx::cg_workspace_bytes(n_rows, nnz, opts);
    } catch (...) {
        return 0;
    }
}

static int check_sell(const cgx_sell *S, const cgx_csr *A, bool need_val32)
{
    CGX_REQUIRE(S != nullptr, "S is NULL");
    CGX_REQUIRE(S->n_rows == A->n_rows && S->n_cols == A->n_cols,
                "sliced-ELL copy does not match A's dimensions");
    CGX_REQUIRE(S->n_slices == ((int64_t)S->n_rows + 63) / 64, "n_slices must be ceil(n_rows / 64)");
    CGX_REQUIRE(S->stored >= 0, "negative stored count");
    CGX_REQUIRE(S->slice_ptr != nullptr, "slice_ptr is NULL");
    if (S->stored > 0) {
        CGX_REQUIRE(S->col != nullptr && S->val != nullptr, "col or val is NULL");
        if (need_val32) CGX_REQUIRE(S->val32 != nullptr, "val32 is NULL");
    }
    return CGX_OK;
}

static int cg_solve_common(cgx_handle h, const cgx_csr *A, const cgx_sell *S, const double *b,
                           double *x, void *workspace, size_t workspace_bytes, const cgx_opts *opts,
                           cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(opts != nullptr && stats != nullptr, "opts or stats is NULL");
        const bool lowp = opts->precision != CGX_PRECISION_FP64;
        int rc = check_csr(A, true, lowp);
        if (rc) return rc;
        if (S) {
            rc = check_sell(S, A, lowp);
            if (rc) return rc;
        }
        CGX_REQUIRE(A->n_rows == A->n_cols, "matrix must be square");
        CGX_REQUIRE(opts->precond == CGX_PRECOND_NONE || opts->precond == CGX_PRECOND_JACOBI,
                    "unknown preconditioner");
        CGX_REQUIRE(opts->precision == CGX_PRECISION_FP64 ||
                        opts->precision == CGX_PRECISION_MIXED ||
                        opts->precision == CGX_PRECISION_MIXED_RU,
                    "unknown precision");
        CGX_REQUIRE(opts->rtol >= 0.0, "rtol must be >= 0");
        std::memset(stats, 0, sizeof(*stats));
        stats->relres_true = -1.0;
        if (A->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(b && x && workspace, "NULL b, x or workspace");
        CGX_REQUIRE(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
        const size_t nb = (size_t)A->n_rows * 8;
        CGX_REQUIRE(!overlaps(b, nb, x, nb), "x overlaps b");
        return cgx::run_cg(ctx_of(h), A, S, b, x, workspace, workspace_bytes, opts, stats);
    });
}

int cgx_cg_solve(cgx_handle h, const cgx_csr *A, const double *b, double *x, void *workspace,
                 size_t workspace_bytes, const cgx_opts *opts, cgx_stats *stats)
{
    return cg_solve_common(h, A, nullptr, b, x, workspace, workspace_bytes, opts, stats);
}

int cgx_cg_solve_noalloc(cgx_handle h, const cgx_csr *A, const double *b, double *x,
                         const cgx_opts *opts, cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(opts != nullptr && stats != nullptr, "opts or stats is NULL");
        int rc = check_csr(A, true, false);
        if (rc) return rc;
        CGX_REQUIRE(A->n_rows == A->n_cols, "matrix must be square");
        CGX_REQUIRE(opts->precond == CGX_PRECOND_NONE || opts->precond == CGX_PRECOND_JACOBI,
                    "unknown preconditioner");
        CGX_REQUIRE(opts->precision == CGX_PRECISION_FP64,
                    "cgx_cg_solve_noalloc runs float64 CG only");
        CGX_REQUIRE(opts->rtol >= 0.0, "rtol must be >= 0");
        std::memset(stats, 0, sizeof(*stats));
        stats->relres_true = -1.0;
        if (A->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(b && x, "NULL b or x");
        const size_t nb = (size_t)A->n_rows * 8;
        CGX_REQUIRE(!overlaps(b, nb, x, nb), "x overlaps b");
        return cgx::run_cg_noalloc(ctx_of(h), A, b, x, opts, stats);
    });
}

int cgx_cg_solve_sell(cgx_handle h, const cgx_csr *A, const cgx_sell *S, const double *b,
                      double *x, void *workspace, size_t workspace_bytes, const cgx_opts *opts,
                      cgx_stats *stats)
{
    if (!S) {
        cgx::set_error("S is NULL");
        return CGX_EINVAL;
    }
    return cg_solve_common(h, A, S, b, x, workspace, workspace_bytes, opts, stats);
}

int cgx_sell_bytes(cgx_handle h, const cgx_csr *A, size_t *bytes)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(bytes != nullptr, "bytes is NULL");
        int rc = check_csr(A, true, false);
        if (rc) return rc;
        return cgx::sell_bytes(ctx_of(h), A, bytes);
    });
}

int cgx_sell_build(cgx_handle h, const cgx_csr *A, void *buffer, size_t bytes, cgx_sell *out)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(out != nullptr, "out is NULL");
        int rc = check_csr(A, true, false);
        if (rc) return rc;
        CGX_REQUIRE(buffer != nullptr && ((uintptr_t)buffer & 255) == 0,
                    "buffer must be 256-byte aligned device memory");
        return cgx::sell_build(ctx_of(h), A, buffer, bytes, out);
    });
}

int cgx_sell_spmv(cgx_handle h, const cgx_sell *S, const double *x, double *y)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr && S != nullptr, "handle or S is NULL");
        CGX_REQUIRE(S->slice_ptr != nullptr && S->n_rows >= 0 && S->n_cols >= 0, "bad S");
        CGX_REQUIRE(S->stored == 0 || (S->col != nullptr && S->val != nullptr), "col or val is NULL");
        if (S->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(y != nullptr && (x != nullptr || S->n_cols == 0), "x or y is NULL");
        CGX_REQUIRE(!overlaps(x, (size_t)S->n_cols * 8, y, (size_t)S->n_rows * 8), "y overlaps x");
        return cgx::launch_sell_spmv(ctx_of(h), S, x, y);
    });
}

int cgx_sell_spmv_f32(cgx_handle h, const cgx_sell *S, const float *x, float *y)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr && S != nullptr, "handle or S is NULL");
        CGX_REQUIRE(S->slice_ptr != nullptr && S->n_rows >= 0 && S->n_cols >= 0, "bad S");
        CGX_REQUIRE(S->stored == 0 || (S->col != nullptr && S->val32 != nullptr),
                    "col or val32 is NULL");
        if (S->n_rows == 0) return CGX_OK;
        CGX_REQUIRE(y != nullptr && (x != nullptr || S->n_cols == 0), "x or y is NULL");
        CGX_REQUIRE(!overlaps(x, (size_t)S->n_cols * 4, y, (size_t)S->n_rows * 4), "y overlaps x");
        return cgx::launch_sell_spmv_f32(ctx_of(h), S, x, y);
    });
}

static int check_schwarz_shape(const cgx_csr *A, int32_t n_sub, int32_t overlap)
{
    int rc = check_csr(A, true, false);
    if (rc) return rc;
    CGX_REQUIRE(A->n_rows == A->n_cols, "matrix must be square");
    CGX_REQUIRE(n_sub >= 1 && n_sub <= A->n_rows, "n_sub must be in [1, n_rows]");
    CGX_REQUIRE(overlap >= 0 && overlap <= A->n_rows / n_sub,
                "overlap must be in [0, floor(n_rows / n_sub)]");
    return CGX_OK;
}

static bool schwarz_ok(const cgx_schwarz *S)
{
    if (!S || S->n_rows < 1 || S->n_sub < 1 || S->n_sub > S->n_rows) return false;
    if (S->overlap < 0 || S->overlap > S->n_rows / S->n_sub) return false;
    if (S->local_rows != (int64_t)S->n_rows + 2 * (int64_t)S->overlap * (S->n_sub - 1))
        return false;
    return S->local_nnz >= 0 && S->nnz_off && S->row_ptr &&
           (S->local_nnz == 0 || (S->col && S->val));
}

int cgx_schwarz_bytes(cgx_handle h, const cgx_csr *A, int32_t n_sub, int32_t overlap,
                      size_t *bytes)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(bytes != nullptr, "bytes is NULL");
        int rc = check_schwarz_shape(A, n_sub, overlap);
        if (rc) return rc;
        return cgx::schwarz_bytes(ctx_of(h), A, n_sub, overlap, bytes);
    });
}

int cgx_schwarz_build(cgx_handle h, const cgx_csr *A, int32_t n_sub, int32_t overlap,
                      void *buffer, size_t bytes, cgx_schwarz *out)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(out != nullptr, "out is NULL");
        int rc = check_schwarz_shape(A, n_sub, overlap);
        if (rc) return rc;
        CGX_REQUIRE(buffer != nullptr && ((uintptr_t)buffer & 255) == 0,
                    "buffer must be 256-byte aligned device memory");
        return cgx::schwarz_build(ctx_of(h), A, n_sub, overlap, buffer, bytes, out);
    });
}

size_t cgx_schwarz_workspace_bytes(const cgx_schwarz *S)
{
    if (!schwarz_ok(S)) return 0;
    try {
        return cgx::schwarz_workspace_bytes(S);
    } catch (...) {
        return 0;
    }
}

int cgx_schwarz_solve(cgx_handle h, const cgx_csr *A, const cgx_schwarz *S, const double *b,
                      double *x, void *workspace, size_t workspace_bytes, const cgx_opts *opts,
                      cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(opts != nullptr && stats != nullptr, "opts or stats is NULL");
        int rc = check_csr(A, true, false);
        if (rc) return rc;
        CGX_REQUIRE(A->n_rows == A->n_cols, "matrix must be square");
        CGX_REQUIRE(schwarz_ok(S), "bad Schwarz descriptor");
        CGX_REQUIRE(S->n_rows == A->n_rows, "Schwarz descriptor does not match A");
        CGX_REQUIRE(opts->precond == CGX_PRECOND_NONE || opts->precond == CGX_PRECOND_JACOBI,
                    "unknown preconditioner");
        CGX_REQUIRE(opts->precision == CGX_PRECISION_FP64, "Schwarz solve is float64");
        CGX_REQUIRE(opts->rtol >= 0.0, "rtol must be >= 0");
        std::memset(stats, 0, sizeof(*stats));
        stats->relres_true = -1.0;
        CGX_REQUIRE(b && x && workspace, "NULL b, x or workspace");
        CGX_REQUIRE(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
        const size_t nb = (size_t)A->n_rows * 8;
        CGX_REQUIRE(!overlaps(b, nb, x, nb), "x overlaps b");
        return cgx::schwarz_solve(ctx_of(h), A, S, b, x, workspace, workspace_bytes, opts, stats);
    });
}

// The sizes and schedules of a batch's descriptors (what the workspace
// layout follows); pointers are checked by check_batch.
static int check_batch_shapes(int32_t nsys, const cgx_system *systems)
{
    CGX_REQUIRE(nsys >= 1 && systems != nullptr, "empty batch");
    for (int32_t s = 0; s < nsys; ++s) {
        const cgx_system &q = systems[s];
        CGX_REQUIRE(q.A.n_rows >= 1, "empty system in batch");
        CGX_REQUIRE(q.A.n_rows == q.A.n_cols, "batched matrices must be square");
        CGX_REQUIRE(q.A.nnz >= 0 && q.A.nnz < ((int64_t)1 << 31), "nnz must be in [0, 2^31)");
        CGX_REQUIRE(q.nrhs >= 1 && q.nrhs <= 16, "nrhs must be in [1, 16]");
    }
    return CGX_OK;
}

static int check_batch(cgx_handle h, int32_t nsys, const cgx_system *systems,
                       bool need_val32 = false)
{
    CGX_REQUIRE(h != nullptr, "handle is NULL");
    int rc = check_batch_shapes(nsys, systems);
    if (rc) return rc;
    for (int32_t s = 0; s < nsys; ++s) {
        const cgx_system &q = systems[s];
        rc = check_csr(&q.A, true, need_val32);
        if (rc) return rc;
        CGX_REQUIRE(q.B != nullptr && q.X != nullptr, "NULL B or X");
        const size_t nb = (size_t)q.A.n_rows * q.nrhs * 8;
        CGX_REQUIRE(!overlaps(q.B, nb, q.X, nb), "X overlaps B");
        if (q.schedule > 0) {
            int K = 1;
            while (K < q.nrhs) K *= 2;
            const int64_t G = (int64_t)K * q.schedule;
            CGX_REQUIRE(G == 8 || G == 16 || G == 32 || G == 64,
                        "schedule M: K * M must be 8, 16, 32 or 64");
        } else if (q.schedule < 0) {
            int K = 1;
            while (K < q.nrhs) K *= 2;
            CGX_REQUIRE(q.schedule >= -64 && cgx::batch_wave_schedule_ok(-q.schedule, K),
                        "wave-tile schedule: -M must be a power of two <= 64 with -M * K "
                        "<= 64, and -M * K >= 16 for several right-hand sides");
        }
    }
    return CGX_OK;
}

size_t cgx_batch_workspace_bytes(int32_t nsys, const cgx_system *systems)
{
    if (check_batch_shapes(nsys, systems) != CGX_OK) return 0;
    try {
        return cgx::batch_workspace_bytes(nsys, systems);
    } catch (...) {
        return 0;
    }
}

size_t cgx_batch_mixed_workspace_bytes(int32_t nsys, const cgx_system *systems)
{
    if (check_batch_shapes(nsys, systems) != CGX_OK) return 0;
    try {
        return cgx::batch_mixed_workspace_bytes(nsys, systems);
    } catch (...) {
        return 0;
    }
}

int cgx_cg_solve_batched(cgx_handle h, int32_t nsys, const cgx_system *systems, void *workspace,
                         size_t workspace_bytes, const cgx_opts *opts, cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(opts != nullptr && stats != nullptr, "opts or stats is NULL");
        CGX_REQUIRE(opts->precision == CGX_PRECISION_FP64 ||
                        opts->precision == CGX_PRECISION_MIXED ||
                        opts->precision == CGX_PRECISION_MIXED_RU,
                    "unknown precision");
        const bool mixed = opts->precision != CGX_PRECISION_FP64;
        int rc = check_batch(h, nsys, systems, mixed);
        if (rc) return rc;
        CGX_REQUIRE(opts->precond == CGX_PRECOND_NONE || opts->precond == CGX_PRECOND_JACOBI,
                    "unknown preconditioner");
        CGX_REQUIRE(opts->rtol >= 0.0, "rtol must be >= 0");
        CGX_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
                    "workspace must be 256-byte aligned");
        if (mixed)
            return cgx::run_batched_mixed(ctx_of(h), nsys, systems, workspace, workspace_bytes,
                                          opts, stats);
        return cgx::run_batched(ctx_of(h), nsys, systems, workspace, workspace_bytes, opts, stats);
    });
}

int cgx_batch_schedule(cgx_handle h, int32_t nsys, const cgx_system *systems, void *workspace,
                       size_t workspace_bytes, int32_t *M_out)
{
    return guarded([&]() -> int {
        int rc = check_batch(h, nsys, systems);
        if (rc) return rc;
        CGX_REQUIRE(M_out != nullptr, "M_out is NULL");
        CGX_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
                    "workspace must be 256-byte aligned");
        CGX_REQUIRE(workspace_bytes >= cgx::batch_workspace_bytes(nsys, systems),
                    "workspace too small");
        std::vector<int> Ms;
        Context *c = ctx_of(h);
        CGX_HIP_CHECK(hipEventRecord(c->ev_in, c->stream));
        CGX_HIP_CHECK(hipStreamWaitEvent(c->own_stream, c->ev_in, 0));
        rc = cgx::batch_autotune(c, nsys, systems, workspace, workspace_bytes, Ms);
        if (rc) return rc;
        for (int32_t s = 0; s < nsys; ++s) M_out[s] = Ms[s];
        CGX_HIP_CHECK(hipStreamSynchronize(c->own_stream));
        return CGX_OK;
    });
}

int cgx_serve_start(cgx_handle h, void *pool, size_t pool_bytes, int32_t max_slots,
                    int32_t max_group)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(pool != nullptr && ((uintptr_t)pool & 255) == 0,
                    "pool must be 256-byte aligned device memory");
        CGX_REQUIRE(max_slots >= 1 && max_slots <= 4096, "max_slots must be in [1, 4096]");
        CGX_REQUIRE(max_group >= 1 && max_group <= 16, "max_group must be in [1, 16]");
        return cgx::serve_start(ctx_of(h), pool, pool_bytes, max_slots, max_group);
    });
}

int cgx_serve_stop(cgx_handle h)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        return cgx::serve_stop(ctx_of(h));
    });
}

size_t cgx_serve_request_bytes(int64_t n_rows)
{
    if (n_rows < 1 || n_rows > 0x7fffffff) return 0;
    try {
        return cgx::serve_request_bytes(n_rows);
    } catch (...) {
        return 0;
    }
}

int cgx_submit(cgx_handle h, const cgx_csr *A, const double *b, double *x, const cgx_opts *opts,
               uint64_t *ticket)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(opts != nullptr && ticket != nullptr, "opts or ticket is NULL");
        CGX_REQUIRE(opts->precision == CGX_PRECISION_FP64 || opts->precision == CGX_PRECISION_MIXED ||
                        opts->precision == CGX_PRECISION_MIXED_RU,
                    "served solves are float64, MIXED or MIXED_RU");
        const bool mixed = opts->precision != CGX_PRECISION_FP64;
        int rc = check_csr(A, true, mixed);
        if (rc) return rc;
        CGX_REQUIRE(A->n_rows == A->n_cols && A->n_rows >= 1, "matrix must be square, n >= 1");
        CGX_REQUIRE(b != nullptr && x != nullptr, "NULL b or x");
        const size_t nb = (size_t)A->n_rows * 8;
        CGX_REQUIRE(!overlaps(b, nb, x, nb), "x overlaps b");
        CGX_REQUIRE(opts->precond == CGX_PRECOND_NONE || opts->precond == CGX_PRECOND_JACOBI,
                    "unknown preconditioner");
        CGX_REQUIRE(opts->rtol >= 0.0, "rtol must be >= 0");
        CGX_REQUIRE(!mixed || opts->inner_rtol < 1.0, "inner_rtol must be < 1");
        return cgx::serve_submit(ctx_of(h), A, b, x, opts, ticket);
    });
}

int cgx_poll(cgx_handle h, uint64_t ticket, cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        return cgx::serve_poll(ctx_of(h), ticket, stats, false);
    });
}

int cgx_wait(cgx_handle h, uint64_t ticket, cgx_stats *stats)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        return cgx::serve_poll(ctx_of(h), ticket, stats, true);
    });
}

int cgx_debug_fail_tuning(cgx_handle h, int32_t count)
{
    return guarded([&]() -> int {
        CGX_REQUIRE(h != nullptr, "handle is NULL");
        CGX_REQUIRE(count >= 0, "count must be >= 0");
        Context *c = ctx_of(h);
        std::lock_guard<std::mutex> lk(c->tune_mu);
        c->fail_tune = count;
        return CGX_OK;
    });
}

}  // extern "C"
