// CSR sparse matrix-vector product (the paper's Section 5.2, table "SpMV
// with CSR format", storage of Section 2.3) for gfx950, float64 and float32,
// plus the structural validation kernel.
//
// Vector-CSR layout: a row is owned by a group of L lanes (L = next power of
// two >= mean row length, 2..64), so the L lanes read one contiguous stretch
// of col_idx / val per row; R rows per group are in flight together to keep
// enough loads outstanding per wave.  Workgroups are renumbered per die
// (xcd_block) so the x gathers of neighbouring rows hit the same L2.
#include "cgx_device.h"

namespace cgx {
namespace {

constexpr int kRowsPerGroup = 4;

template <int L, typename T>
__global__ __launch_bounds__(kBlock) void spmv_vector_kernel(int n_rows, int n_cols, int64_t nnz,
                                                             const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const T *__restrict__ val,
                                                             const T *__restrict__ x,
                                                             T *__restrict__ y)
{
    constexpr int R = kRowsPerGroup;
    constexpr int rows_per_block = (kBlock / L) * R;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    T acc[R], dg[R];
    int rows[R];
    vector_rows<L, R, kBlock, T, false>(tile * rows_per_block, n_rows, n_cols, nnz, rp, ci, val, x,
                                        acc, dg, rows);
    if (threadIdx.x % L == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (rows[r] < n_rows) y[rows[r]] = acc[r];
    }
}

template <typename T>
int launch_spmv_t(Context *c, const cgx_csr *A, const T *val, const T *x, T *y)
{
    if (A->n_rows == 0) return CGX_OK;
    const int L = lanes_per_row(A->n_rows, A->nnz);
    const int64_t rows_per_block = (int64_t)(kBlock / L) * kRowsPerGroup;
    const int64_t grid = (A->n_rows + rows_per_block - 1) / rows_per_block;
#define CGX_SPMV_CASE(LL)                                                                     \
    case LL:                                                                                  \
        hipLaunchKernelGGL((spmv_vector_kernel<LL, T>), dim3((unsigned)grid), dim3(kBlock), 0, \
                           c->stream, A->n_rows, A->n_cols, A->nnz, A->row_ptr, A->col_idx,   \
                           val, x, y);                                                        \
        break;
    switch (L) {
        CGX_SPMV_CASE(2)
        CGX_SPMV_CASE(4)
        CGX_SPMV_CASE(8)
        CGX_SPMV_CASE(16)
        CGX_SPMV_CASE(32)
        CGX_SPMV_CASE(64)
        default:
            set_error("internal: bad lanes per row");
            return CGX_EINVAL;
    }
#undef CGX_SPMV_CASE
    CGX_HIP_CHECK(hipGetLastError());
    return CGX_OK;
}

// One thread per row: row_ptr ordering and bounds, columns in range, no
// duplicate column in the row (quadratic scan: validation only).  The first
// offending row is kept with an atomic minimum.
__global__ __launch_bounds__(kBlock) void csr_validate_kernel(int n_rows, int n_cols, int64_t nnz,
                                                              const int32_t *rp,
                                                              const int32_t *ci,
                                                              unsigned long long *first_bad)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row > n_rows) return;
    bool bad = false;
    if (row == 0 && rp[0] != 0) bad = true;
    if (row == n_rows) {
        if ((int64_t)rp[n_rows] != nnz) bad = true;
    } else {
        const int s = rp[row], e = rp[row + 1];
        if (s < 0 || e < s || (int64_t)e > nnz) {
            bad = true;
        } else {
            for (int k = s; k < e && !bad; ++k) {
                const int col = ci[k];
                if (col < 0 || col >= n_cols) bad = true;
                for (int j = s; j < k && !bad; ++j)
                    if (ci[j] == col) bad = true;
            }
        }
    }
    if (bad) atomicMin(first_bad, (unsigned long long)row);
}

}  // namespace

int lanes_per_row(int64_t n_rows, int64_t nnz)
{
    const double mean = n_rows > 0 ? (double)nnz / (double)n_rows : 1.0;
    int L = 2;
    while (L < 64 && L < mean) L *= 2;
    return L;
}

int launch_spmv(Context *c, const cgx_csr *A, const double *x, double *y)
{
    return launch_spmv_t<double>(c, A, A->val, x, y);
}

int launch_spmv_f32(Context *c, const cgx_csr *A, const float *x, float *y)
{
    return launch_spmv_t<float>(c, A, A->val32, x, y);
}

int run_csr_validate(Context *c, const cgx_csr *A, int64_t *bad_row)
{
    unsigned long long *d_bad = reinterpret_cast<unsigned long long *>(c->scratch);
    const unsigned long long init = ~0ull;
    CGX_HIP_CHECK(hipMemcpyAsync(d_bad, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    const int64_t grid = ((int64_t)A->n_rows + 1 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(csr_validate_kernel, dim3((unsigned)grid), dim3(kBlock), 0, c->stream,
                       A->n_rows, A->n_cols, A->nnz, A->row_ptr, A->col_idx, d_bad);
    CGX_HIP_CHECK(hipGetLastError());
    unsigned long long h_bad = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(&h_bad, d_bad, sizeof(h_bad), hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (bad_row) *bad_row = h_bad == ~0ull ? -1 : (int64_t)h_bad;
    if (h_bad != ~0ull) {
        set_error("CSR structure invalid at row " + std::to_string(h_bad));
        return CGX_EINVAL;
    }
    return CGX_OK;
}

}  // namespace cgx
