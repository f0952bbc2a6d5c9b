// CSR sparse matrix-vector product (the paper's Section 5.2, table "SpMV
// with CSR format", storage of Section 2.3) for gfx950, float64 and float32,
// plus the structural validation kernel.
//
// Wave-tile layout: each 64-thread workgroup (one wavefront) owns a tile of
// RT consecutive rows, RT from the mean row length so that a tile's entries
// fill one chunk of 64 x 8 float64 (64 x 14 binary32) entries.  The tile's
// col_idx / val are read as one contiguous stream with eight (fourteen)
// independent coalesced non-temporal loads per lane and staged in LDS; then
// 64 / RT lanes per row walk the row's entries in step, so that the x gathers
// of neighbouring rows coalesce.  One tile per workgroup and many small
// workgroups (the hardware keeps the waves of a die in dispatch order, a
// compact moving front over x) measured faster than persistent workgroups
// looping over tiles and than 256-thread tiles gathering in entry order.
// Workgroups are renumbered per die (xcd_block) so the x gathers of
// neighbouring rows hit the same L2.
#include "cgx_device.h"

namespace cgx {
namespace {

template <int RT, typename T>
__global__ __launch_bounds__(kWave) void spmv_wave_kernel(int n_rows, int n_cols, int64_t nnz,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const T *__restrict__ val,
                                                          const T *__restrict__ x,
                                                          T *__restrict__ y)
{
    // gathers in flight per lane: 4 in float64, 16 in binary32, measured on
    // the Q1 128^3 matrix (float64 at 8: 138.2 against 135.5 us; binary32 at
    // 16: 91.6 against 100.4 us at 4)
    constexpr int U = sizeof(T) == sizeof(double) ? 4 : 16;
    __shared__ WaveSmem<wave_e<T>(), RT, T> sm;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    int row;
    const T acc = wave_rows<wave_e<T>(), RT, U, T>(tile * RT, n_rows, n_cols, nnz, rp, ci, val, x,
                                                   sm, row);
    if (threadIdx.x % (kWave / RT) == 0 && row < n_rows) y[row] = acc;
}

template <typename T>
int launch_spmv_t(Context *c, const cgx_csr *A, const T *val, const T *x, T *y)
{
    if (A->n_rows == 0) return CGX_OK;
    const int RT = wave_tile_rows(A->n_rows, A->nnz, wave_e<T>());
    const int64_t grid = (A->n_rows + RT - 1) / RT;
#define CGX_SPMV_CASE(RR)                                                                    \
    hipLaunchKernelGGL((spmv_wave_kernel<RR, T>), dim3((unsigned)grid), dim3(kWave), 0,       \
                       c->stream, A->n_rows, A->n_cols, A->nnz, A->row_ptr, A->col_idx, val, x, \
                       y)
    CGX_WRT_SWITCH(RT, CGX_SPMV_CASE)
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

int wave_tile_rows(int64_t n_rows, int64_t nnz, int entries_per_lane)
{
    const double mean = n_rows > 0 ? (double)nnz / (double)n_rows : 1.0;
    const double budget = 0.97 * kWave * entries_per_lane;
    int rt = kWave;
    while (rt > 1 && rt * (mean > 1.0 ? mean : 1.0) > budget) rt /= 2;
    return rt;
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
