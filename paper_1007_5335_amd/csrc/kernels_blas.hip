// kernels_blas.hip -- tall-skinny FP64 kernels for GMRES (deterministic reductions).
#include "yk_internal.h"

namespace yk {

namespace {

constexpr int kRedBlock = 256;
constexpr int kMaxChunks = 64;

__device__ __forceinline__ double block_sum(double v, double *sh) {
    // wavefront reduction (64 lanes) then across the block's waves, fixed order
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    }
    __syncthreads();
    return s;
}

// partial[v * nchunk + c] = sum over chunk c of V[v*ld + i] * x[i]
__global__ __launch_bounds__(kRedBlock) void k_multi_dot(int64_t n, const double *__restrict__ V,
                                                         int64_t ld, const double *__restrict__ x,
                                                         double *__restrict__ partial) {
    __shared__ double sh[kRedBlock / 64];
    const int v = blockIdx.y, c = blockIdx.x, nchunk = gridDim.x;
    const double *row = V + (int64_t)v * ld;
    double acc = 0.0;
    for (int64_t i = (int64_t)c * kRedBlock + threadIdx.x; i < n; i += (int64_t)nchunk * kRedBlock)
        acc += row[i] * x[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)v * nchunk + c] = s;
}

__global__ void k_reduce_rows2(int nv, int nchunk, const double *__restrict__ partial,
                               double *__restrict__ h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)v * nchunk + c];
    h[v] = s;
}

__global__ void k_multi_axpy(int64_t n, int nv, const double *__restrict__ V, int64_t ld,
                             const double *__restrict__ h, double sign, double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = x[i];
    for (int k = 0; k < nv; ++k) acc += sign * h[k] * V[(int64_t)k * ld + i];
    x[i] = acc;
}

__global__ void k_scale_div(int64_t n, const double *__restrict__ x, const double *__restrict__ s,
                            double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = x[i] / s[0];
}

__global__ __launch_bounds__(kRedBlock) void k_nonfinite(int64_t n, const double *__restrict__ x,
                                                         double *__restrict__ flag) {
    __shared__ double sh[kRedBlock / 64];
    double bad = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kRedBlock)
        if (!isfinite(x[i])) bad = 1.0;
    const double s = block_sum(bad, sh);
    if (threadIdx.x == 0) flag[0] = s > 0.0 ? 1.0 : 0.0;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_multi_dot(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                      const double *x, double *h) {
    int nchunk = (int)std::min<int64_t>(kMaxChunks, (n + 4 * kRedBlock - 1) / (4 * kRedBlock));
    if (nchunk < 1) nchunk = 1;
    double *part = ctx.partial.ensure((size_t)kMaxChunks * 128);
    hipLaunchKernelGGL(k_multi_dot, dim3(nchunk, nv), dim3(kRedBlock), 0, ctx.stream, n, V, ld, x,
                       part);
    check_launch(ctx, "k_multi_dot");
    hipLaunchKernelGGL(k_reduce_rows2, dim3(nblk(nv, 64)), dim3(64), 0, ctx.stream, nv, nchunk, part,
                       h);
    check_launch(ctx, "k_reduce_rows");
}

void launch_multi_axpy(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                       const double *h, double *x) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, nv, V, ld, h,
                       -1.0, x);
    check_launch(ctx, "k_multi_axpy");
}

void launch_add_combination(Context &ctx, int64_t n, int nv, const double *V, int64_t ld,
                            const double *y, double *x) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, nv, V, ld, y,
                       1.0, x);
    check_launch(ctx, "k_add_combination");
}

void launch_scale_div(Context &ctx, int64_t n, const double *x, const double *s, double *y) {
    hipLaunchKernelGGL(k_scale_div, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, x, s, y);
    check_launch(ctx, "k_scale_div");
}

void launch_nonfinite(Context &ctx, int64_t n, const double *x, double *flag) {
    hipLaunchKernelGGL(k_nonfinite, dim3(1), dim3(kRedBlock), 0, ctx.stream, n, x, flag);
    check_launch(ctx, "k_nonfinite");
}

}  // namespace yk
