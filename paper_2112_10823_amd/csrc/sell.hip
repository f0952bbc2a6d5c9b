// Sliced ELLPACK copy of a CSR matrix and its SpMV (the paper's Section 2.3
// names ELL beside CSR; its measurements use CSR).  Slices of 64 rows, one
// wavefront each, stored column-major with the width of the slice's longest
// row: entry k of row 64 s + l sits at slice_ptr[s] + 64 k + l, padding
// entries have column -1 and value 0.  Lane l of the slice's wavefront owns
// row 64 s + l: every load of col / val is one contiguous 64-entry segment,
// and at step k the lanes gather x for the k-th entries of 64 neighbouring
// rows, a few cache lines for stencil matrices, with no LDS staging and no
// row-pointer pass.  Rows are not reordered, so x keeps its locality and y
// is written in place.
#include "cgx_device.h"

namespace cgx {
namespace {

constexpr int kSellU = 8;  // entries per lane in flight

// One wavefront per slice: the width of slice s (its longest row, row
// pointers clamped as everywhere) times 64, stored at slice_ptr[s + 1];
// optionally added to *total (exact integer atomics: the order is free).
__global__ __launch_bounds__(kWave) void sell_width_kernel(int n_rows, int64_t nnz,
                                                           const int32_t *__restrict__ rp,
                                                           int64_t n_slices, int64_t *slice_ptr,
                                                           unsigned long long *total)
{
    const int64_t s = blockIdx.x;
    if (s >= n_slices) return;
    const int64_t row = s * kWave + threadIdx.x;
    int len = 0;
    if (row < n_rows) {
        int a = rp[row], b = rp[row + 1];
        a = a < 0 ? 0 : (a > nnz ? (int)nnz : a);
        b = b < a ? a : (b > nnz ? (int)nnz : b);
        len = b - a;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off));
    if (threadIdx.x == 0) {
        if (slice_ptr) slice_ptr[s + 1] = (int64_t)len * kWave;
        if (total) atomicAdd(total, (unsigned long long)len * kWave);
    }
}

// Exclusive prefix sum in place over slice_ptr[1 .. n_slices] (slice_ptr[0]
// = 0), one workgroup: each thread scans a contiguous run, then the run
// totals are scanned in the workgroup.
__global__ __launch_bounds__(1024) void sell_scan_kernel(int64_t n_slices, int64_t *slice_ptr)
{
    __shared__ int64_t tot[1024];
    const int64_t per = (n_slices + 1023) / 1024;
    const int64_t a = 1 + threadIdx.x * per, b = min(n_slices + 1, a + per);
    int64_t run = 0;
    for (int64_t i = a; i < b; ++i) run += slice_ptr[i];
    tot[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = tot[i];
            tot[i] = acc;
            acc += v;
        }
        slice_ptr[0] = 0;
    }
    __syncthreads();
    int64_t acc = tot[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        acc += slice_ptr[i];
        slice_ptr[i] = acc;
    }
}

// One wavefront per slice: lane l copies row 64 s + l into the slice's
// columns and pads up to the slice width.
__global__ __launch_bounds__(kWave) void sell_fill_kernel(int n_rows, int64_t nnz,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double *__restrict__ val,
                                                          const float *__restrict__ val32,
                                                          int64_t n_slices,
                                                          const int64_t *__restrict__ slice_ptr,
                                                          int32_t *col, double *sval, float *sval32)
{
    const int64_t s = blockIdx.x;
    if (s >= n_slices) return;
    const int64_t base = slice_ptr[s];
    const int w = (int)((slice_ptr[s + 1] - base) / kWave);
    const int64_t row = s * kWave + threadIdx.x;
    int a = 0, b = 0;
    if (row < n_rows) {
        a = rp[row];
        b = rp[row + 1];
        a = a < 0 ? 0 : (a > nnz ? (int)nnz : a);
        b = b < a ? a : (b > nnz ? (int)nnz : b);
    }
    for (int k = 0; k < w; ++k) {
        const int64_t e = base + (int64_t)k * kWave + threadIdx.x;
        const bool on = a + k < b;
        col[e] = on ? ci[a + k] : -1;
        sval[e] = on ? val[a + k] : 0.0;
        if (sval32) sval32[e] = on ? val32[a + k] : 0.0f;
    }
}

template <typename T>
__global__ __launch_bounds__(kWave) void sell_spmv_kernel(int n_rows, int n_cols,
                                                          const int64_t *__restrict__ sp,
                                                          const int32_t *__restrict__ col,
                                                          const T *__restrict__ val,
                                                          const T *__restrict__ x,
                                                          T *__restrict__ y)
{
    const int s = xcd_block(blockIdx.x, gridDim.x);
    int row;
    const T acc = sell_rows<kSellU, T>(s, n_rows, n_cols, sp, col, val, x, row);
    if (row < n_rows) y[row] = acc;
}

size_t sell_layout(int64_t n_slices, int64_t stored, bool f32, size_t *off_col, size_t *off_val,
                   size_t *off_val32)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = al((size_t)(n_slices + 1) * sizeof(int64_t));
    *off_col = off;
    off += al((size_t)stored * sizeof(int32_t));
    *off_val = off;
    off += al((size_t)stored * sizeof(double));
    *off_val32 = off;
    if (f32) off += al((size_t)stored * sizeof(float));
    return off;
}

template <typename T>
int launch_sell_spmv_t(Context *c, const cgx_sell *S, const T *val, const T *x, T *y)
{
    if (S->n_rows == 0) return CGX_OK;
    hipLaunchKernelGGL((sell_spmv_kernel<T>), dim3((unsigned)S->n_slices), dim3(kWave), 0,
                       c->stream, S->n_rows, S->n_cols, S->slice_ptr, S->col, val, x, y);
    CGX_HIP_CHECK(hipGetLastError());
    return CGX_OK;
}

}  // namespace

int sell_bytes(Context *c, const cgx_csr *A, size_t *bytes)
{
    const int64_t ns = ((int64_t)A->n_rows + kWave - 1) / kWave;
    unsigned long long *d_tot = reinterpret_cast<unsigned long long *>(c->scratch);
    const unsigned long long zero = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(d_tot, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    if (ns > 0)
        hipLaunchKernelGGL(sell_width_kernel, dim3((unsigned)ns), dim3(kWave), 0, c->stream,
                           A->n_rows, A->nnz, A->row_ptr, ns, nullptr, d_tot);
    CGX_HIP_CHECK(hipGetLastError());
    unsigned long long tot = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(&tot, d_tot, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    size_t a, b, d;
    *bytes = sell_layout(ns, (int64_t)tot, A->val32 != nullptr, &a, &b, &d);
    return CGX_OK;
}

int sell_build(Context *c, const cgx_csr *A, void *buf, size_t bytes, cgx_sell *out)
{
    size_t need = 0;
    int rc = sell_bytes(c, A, &need);
    if (rc) return rc;
    if (bytes < need) {
        set_error("SELL buffer too small: need " + std::to_string(need) + " bytes");
        return CGX_ENOMEM;
    }
    const int64_t ns = ((int64_t)A->n_rows + kWave - 1) / kWave;
    char *w = static_cast<char *>(buf);
    int64_t *sp = reinterpret_cast<int64_t *>(w);
    const int64_t zero = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(sp, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    if (ns > 0) {
        hipLaunchKernelGGL(sell_width_kernel, dim3((unsigned)ns), dim3(kWave), 0, c->stream,
                           A->n_rows, A->nnz, A->row_ptr, ns, sp, nullptr);
        hipLaunchKernelGGL(sell_scan_kernel, dim3(1), dim3(1024), 0, c->stream, ns, sp);
    }
    CGX_HIP_CHECK(hipGetLastError());
    int64_t stored = 0;
    CGX_HIP_CHECK(hipMemcpyAsync(&stored, sp + ns, sizeof(stored), hipMemcpyDeviceToHost, c->stream));
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    size_t oc, ov, ov32;
    const bool f32 = A->val32 != nullptr;
    sell_layout(ns, stored, f32, &oc, &ov, &ov32);
    int32_t *col = reinterpret_cast<int32_t *>(w + oc);
    double *val = reinterpret_cast<double *>(w + ov);
    float *val32 = f32 ? reinterpret_cast<float *>(w + ov32) : nullptr;
    if (ns > 0)
        hipLaunchKernelGGL(sell_fill_kernel, dim3((unsigned)ns), dim3(kWave), 0, c->stream,
                           A->n_rows, A->nnz, A->row_ptr, A->col_idx, A->val, A->val32, ns, sp,
                           col, val, val32);
    CGX_HIP_CHECK(hipGetLastError());
    CGX_HIP_CHECK(hipStreamSynchronize(c->stream));
    out->n_rows = A->n_rows;
    out->n_cols = A->n_cols;
    out->n_slices = ns;
    out->stored = stored;
    out->slice_ptr = sp;
    out->col = col;
    out->val = val;
    out->val32 = val32;
    return CGX_OK;
}

int launch_sell_spmv(Context *c, const cgx_sell *S, const double *x, double *y)
{
    return launch_sell_spmv_t<double>(c, S, S->val, x, y);
}

int launch_sell_spmv_f32(Context *c, const cgx_sell *S, const float *x, float *y)
{
    return launch_sell_spmv_t<float>(c, S, S->val32, x, y);
}

}  // namespace cgx
