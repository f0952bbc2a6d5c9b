// BLAS-1 kernels of the paper's Section 5.2 for gfx950: addition of vectors,
// daxpy, element-wise product, dot product, plus float64 -> float32 demotion.
//
// The elementwise kernels are HBM-bound streams (24 bytes per element for
// add/xmul/axpy).  Each thread moves four 16-byte pairs per trip so a wave
// keeps several dwordx4 loads in flight; scalar code handles unaligned
// pointers and the odd tail.  The dot product accumulates with error-free
// transformations; a second one-workgroup kernel adds the per-workgroup
// partials in index order.
#include "cgx_device.h"

namespace cgx {
namespace {

constexpr int kUnroll = 4;  // double2 per thread per trip

struct AddOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct MulOp {
    __device__ double operator()(double a, double b) const { return a * b; }
};
struct AxpyOp {  // op(x, y) = fma(alpha, x, y)
    double alpha;
    __device__ double operator()(double a, double b) const { return __builtin_fma(alpha, a, b); }
};

// z[i] = op(x[i], y[i]) over pairs; x, y, z 16-byte aligned.  z may be x or
// y (each element is read before it is written, by the same thread).
template <class Op>
__global__ __launch_bounds__(kBlock) void ew_pairs_kernel(int64_t npairs, const double2 *x, const double2 *y,
                                                          double2 *z, Op op)
{
    const int64_t base = (int64_t)blockIdx.x * kBlock * kUnroll + threadIdx.x;
    double2 a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kBlock;
        if (i < npairs) {
            a[u] = x[i];
            b[u] = y[i];
        }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kBlock;
        if (i < npairs) z[i] = make_double2(op(a[u].x, b[u].x), op(a[u].y, b[u].y));
    }
}

// Scalar version for unaligned pointers and the tail element.
template <class Op>
__global__ __launch_bounds__(kBlock) void ew_scalar_kernel(int64_t n, const double *x, const double *y,
                                                           double *z, Op op)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        z[i] = op(x[i], y[i]);
}

template <class Op>
int launch_ew(Context *c, int64_t n, const double *x, const double *y, double *z, Op op)
{
    if (n == 0) return CGX_OK;
    const bool aligned = ((((uintptr_t)x) | ((uintptr_t)y) | ((uintptr_t)z)) & 15) == 0;
    int64_t done = 0;
    if (aligned && n >= 2) {
        const int64_t npairs = n / 2;
        const int64_t per_block = (int64_t)kBlock * kUnroll;
        const int64_t grid = (npairs + per_block - 1) / per_block;
        if (grid > 0x7fffffff) {
            set_error("vector too long");
            return CGX_EINVAL;
        }
        hipLaunchKernelGGL(ew_pairs_kernel<Op>, dim3((unsigned)grid), dim3(kBlock), 0, c->stream,
                           npairs, (const double2 *)x, (const double2 *)y, (double2 *)z, op);
        done = npairs * 2;
    }
    if (done < n) {
        const int64_t rest = n - done;
        int64_t grid = (rest + kBlock - 1) / kBlock;
        if (grid > 4096) grid = 4096;
        hipLaunchKernelGGL(ew_scalar_kernel<Op>, dim3((unsigned)grid), dim3(kBlock), 0, c->stream,
                           rest, x + done, y + done, z + done, op);
    }
    CGX_HIP_CHECK(hipGetLastError());
    return CGX_OK;
}

// Dot product, pass 1: each thread accumulates (s, e) with two-product /
// two-sum over a grid-stride walk; each workgroup stores its block totals of
// s and e as plain partials.
__global__ __launch_bounds__(kBlock) void dot_partials_kernel(int64_t n,
                                                              const double *__restrict__ x,
                                                              const double *__restrict__ y,
                                                              double *partials)
{
#pragma clang fp contract(off)
    double s = 0.0, e = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = x[i + u * stride];
            b[u] = y[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double p = a[u] * b[u];
            const double pe = __builtin_fma(a[u], b[u], -p);
            double t, te;
            two_sum(s, p, t, te);
            s = t;
            e += pe + te;
        }
    }
    for (; i < n; i += stride) {
        const double p = x[i] * y[i];
        const double pe = __builtin_fma(x[i], y[i], -p);
        double t, te;
        two_sum(s, p, t, te);
        s = t;
        e += pe + te;
    }
    __shared__ double red[2 * (kBlock / kWave)];
    double v[2] = {s, e};
    block_sum<2, kBlock>(v, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = v[0];
        partials[gridDim.x + blockIdx.x] = v[1];
    }
}

// Dot product, pass 2 (one workgroup): the s and e partials in index order.
__global__ __launch_bounds__(kBlock) void dot_finish_kernel(const double *partials, int count,
                                                            double *result)
{
    __shared__ double red[kBlock / kWave];
    const double s = sum_partials<kBlock>(partials, count, red);
    const double e = sum_partials<kBlock>(partials + count, count, red);
    if (threadIdx.x == 0) *result = s + e;
}

__global__ __launch_bounds__(kBlock) void demote_kernel(int64_t n, const double *__restrict__ src,
                                                        float *__restrict__ dst)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = (float)src[i];
}

}  // namespace

int launch_add(Context *c, int64_t n, const double *x, const double *y, double *z)
{
    return launch_ew(c, n, x, y, z, AddOp{});
}

int launch_xmul(Context *c, int64_t n, const double *x, const double *y, double *z)
{
    return launch_ew(c, n, x, y, z, MulOp{});
}

int launch_axpy(Context *c, int64_t n, double alpha, const double *x, double *y)
{
    return launch_ew(c, n, x, y, y, AxpyOp{alpha});
}

int launch_dot(Context *c, int64_t n, const double *x, const double *y, double *result)
{
    int grid = kReduceBlocks;
    const int64_t need = (n + kBlock - 1) / kBlock;
    if (need < grid) grid = need > 0 ? (int)need : 1;
    hipLaunchKernelGGL(dot_partials_kernel, dim3(grid), dim3(kBlock), 0, c->stream, n, x, y,
                       c->scratch);
    hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(kBlock), 0, c->stream, c->scratch, grid,
                       result);
    CGX_HIP_CHECK(hipGetLastError());
    return CGX_OK;
}

int launch_demote(Context *c, int64_t n, const double *src, float *dst)
{
    if (n == 0) return CGX_OK;
    int64_t grid = (n + kBlock - 1) / kBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(demote_kernel, dim3((unsigned)grid), dim3(kBlock), 0, c->stream, n, src, dst);
    CGX_HIP_CHECK(hipGetLastError());
    return CGX_OK;
}

}  // namespace cgx
