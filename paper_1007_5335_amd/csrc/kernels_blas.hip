// kernels_blas.hip -- tall-skinny FP64 kernels for GMRES (deterministic reductions).
#include "yk_internal.h"

namespace yk {

namespace {

constexpr int kRedBlock = 256;
constexpr int kMaxChunks = 64;
constexpr int kArnMaxRows = 128;

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

// partial[v * nchunk + c] = sum over chunk c of x_v[i]^2 for v = 0, 1, 2 (a
// null vector gives zeros); the chunks are those of k_multi_dot
__global__ __launch_bounds__(kRedBlock) void k_sumsq3(int64_t n, const double *__restrict__ x0,
                                                      const double *__restrict__ x1,
                                                      const double *__restrict__ x2,
                                                      double *__restrict__ partial) {
    __shared__ double sh[kRedBlock / 64];
    const int v = blockIdx.y, c = blockIdx.x, nchunk = gridDim.x;
    const double *x = v == 0 ? x0 : v == 1 ? x1 : x2;
    double acc = 0.0;
    if (x)
        for (int64_t i = (int64_t)c * kRedBlock + threadIdx.x; i < n; i += (int64_t)nchunk * kRedBlock)
            acc += x[i] * x[i];
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

// Arnoldi step in passes over w, each a kernel of nchunk blocks.  Block c
// takes the 512-element segments c, c + nchunk, ... and leaves one partial
// per dot product; the next kernel sums the partials of the one before in
// every block, in one fixed order (lane-strided, then a wavefront tree), so
// all blocks hold identical sums and the result is deterministic without
// any cross-block synchronisation inside a kernel.
constexpr int kArnE = 2;                    // elements per thread per segment
constexpr int kArnSeg = kRedBlock * kArnE;  // elements per segment
constexpr int kArnMaxChunks = 256;
constexpr int kArnRU = 8;                   // basis vectors whose loads are issued together

inline int arn_chunks(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kArnMaxChunks, (n + kArnSeg - 1) / kArnSeg));
}

// out[r] = sum_c p[r * nchunk + c] for r < nrows (one wavefront per row)
__device__ __forceinline__ void sum_partials(const double *__restrict__ p, int nrows, int nchunk,
                                             double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r = wave; r < nrows; r += nw) {
        double t = 0.0;
        for (int c = lane; c < nchunk; c += 64) t += p[(int64_t)r * nchunk + c];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) out[r] = t;
    }
}

// w -= sum_{v < nsub} h_v V_v, h summed from the partials psub (block 0 also
// stores h to hsub_out); then the partials of V_r . w for r < nd and, with
// self, of w . w, into pout
__global__ __launch_bounds__(kRedBlock) void k_arnoldi_pass(
    int64_t n, const double *__restrict__ V, int64_t ld, double *__restrict__ w, int nsub,
    const double *__restrict__ psub, double *__restrict__ hsub_out, int nd, int self,
    double *__restrict__ pout) {
    __shared__ double hs[kArnMaxRows];
    __shared__ double sh[(kArnMaxRows + 1) * 4];
    const int c = blockIdx.x, nchunk = gridDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nrows = nd + (self ? 1 : 0);
    if (nsub > 0) sum_partials(psub, nsub, nchunk, hs);
    for (int r = tid; r < nrows * 4; r += kRedBlock) sh[r] = 0.0;
    __syncthreads();
    if (c == 0)
        for (int r = tid; r < nsub; r += kRedBlock) hsub_out[r] = hs[r];
    for (int64_t seg = c; seg * kArnSeg < n; seg += nchunk) {
        // element e of this thread: index ix[e] (clamped into range; ok[e]
        // false past the end), so every load below is unconditional
        int64_t ix[kArnE];
        bool ok[kArnE];
        double x[kArnE];
#pragma unroll
        for (int e = 0; e < kArnE; ++e) {
            const int64_t i = seg * kArnSeg + tid + e * kRedBlock;
            ok[e] = i < n;
            ix[e] = ok[e] ? i : n - 1;
            x[e] = ok[e] ? w[ix[e]] : 0.0;
        }
        if (nsub > 0) {
            // in increasing v
            for (int v0 = 0; v0 < nsub; v0 += kArnRU) {
                double a[kArnRU][kArnE];
#pragma unroll
                for (int u = 0; u < kArnRU; ++u) {
                    const double *row = V + (int64_t)min(v0 + u, nsub - 1) * ld;
#pragma unroll
                    for (int e = 0; e < kArnE; ++e) a[u][e] = row[ix[e]];
                }
#pragma unroll
                for (int u = 0; u < kArnRU; ++u) {
                    if (v0 + u < nsub) {
                        const double hv = hs[v0 + u];
#pragma unroll
                        for (int e = 0; e < kArnE; ++e) x[e] -= hv * a[u][e];
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < kArnE; ++e)
                if (ok[e]) w[ix[e]] = x[e];
        }
        double xm[kArnE];   // x masked to the range
#pragma unroll
        for (int e = 0; e < kArnE; ++e) xm[e] = ok[e] ? x[e] : 0.0;
        for (int r0 = 0; r0 < nd; r0 += kArnRU) {
            double acc[kArnRU];
#pragma unroll
            for (int u = 0; u < kArnRU; ++u) {
                const double *row = V + (int64_t)min(r0 + u, nd - 1) * ld;
                acc[u] = 0.0;
#pragma unroll
                for (int e = 0; e < kArnE; ++e) acc[u] += row[ix[e]] * xm[e];
            }
#pragma unroll
            for (int u = 0; u < kArnRU; ++u)
                for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_down(acc[u], off, 64);
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < kArnRU; ++u)
                    if (r0 + u < nd) sh[(r0 + u) * 4 + wave] += acc[u];
            }
        }
        if (self) {
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < kArnE; ++e) acc += xm[e] * xm[e];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if (lane == 0) sh[nd * 4 + wave] += acc;
        }
    }
    __syncthreads();
    for (int r = tid; r < nrows; r += kRedBlock)
        pout[(int64_t)r * nchunk + c] = (sh[r * 4] + sh[r * 4 + 1]) + (sh[r * 4 + 2] + sh[r * 4 + 3]);
}

// Second subtraction and normalisation of a CGS2 step, from the partials p of
// the previous pass (rows 0..nsub-1: h2 = V^T w; row nsub: |w|^2):
//   y = (w - sum_v h2_v V_v) / |.|,  |.|^2 = |w|^2 - |h2|^2
// (V orthonormal, so the norm of the result follows from the partials and no
// further pass over the vector is needed; a negative value from rounding is
// taken as zero, and y is then zero).  Block 0 stores h2 to h2_out and the
// squared norm to nrm2_out, and hands the column to the host:
// host_dst[0..128) = h1[0..128), host_dst[128 + v] = h2_v, host_dst[256] = |.|^2.
__global__ __launch_bounds__(256) void k_arnoldi_finish(
    int64_t n, const double *__restrict__ V, int64_t ld, const double *__restrict__ w, int nsub,
    const double *__restrict__ p, int nchunk, double *__restrict__ h2_out, double *__restrict__ nrm2_out,
    double *__restrict__ y, const double *__restrict__ h1, double *__restrict__ host_dst) {
    __shared__ double hs[kArnMaxRows + 1];
    __shared__ double nrm;
    sum_partials(p, nsub + 1, nchunk, hs);
    __syncthreads();
    if (threadIdx.x == 0) {
        double s2 = 0.0;
        for (int v = 0; v < nsub; ++v) s2 += hs[v] * hs[v];
        nrm = fmax(hs[nsub] - s2, 0.0);
    }
    __syncthreads();
    const double nrm2 = nrm;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double x = w[i];
        for (int v = 0; v < nsub; ++v) x -= hs[v] * V[(int64_t)v * ld + i];
        y[i] = nrm2 > 0.0 ? (1.0 / sqrt(nrm2)) * x : 0.0;
    }
    if (blockIdx.x == 0) {
        for (int t = threadIdx.x; t < nsub; t += blockDim.x) h2_out[t] = hs[t];
        if (threadIdx.x == 0) nrm2_out[0] = nrm2;
        if (host_dst) {
            const int t = threadIdx.x;
            if (t < 128) host_dst[t] = h1[t];
            else if (t - 128 < nsub) host_dst[t] = hs[t - 128];
            if (t == 0) host_dst[256] = nrm2;
        }
    }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_arnoldi_pass(Context &ctx, int64_t n, const double *V, int64_t ld, double *w, int nsub,
                         const double *psub, double *hsub_out, int nd, bool self, double *pout) {
    if (nd + (self ? 1 : 0) > kArnMaxRows + 1 || nsub > kArnMaxRows)
        throw Error{YK_ERR_INTERNAL, "Arnoldi pass: too many basis vectors"};
    hipLaunchKernelGGL(k_arnoldi_pass, dim3(arn_chunks(n)), dim3(kRedBlock), 0, ctx.stream, n, V, ld, w,
                       nsub, psub, hsub_out, nd, self ? 1 : 0, pout);
    check_launch(ctx, "k_arnoldi_pass");
}

void launch_arnoldi_finish(Context &ctx, int64_t n, const double *V, int64_t ld, const double *w, int nsub,
                           const double *p, double *h2_out, double *nrm2_out, double *y, const double *h1,
                           double *host_dst) {
    if (nsub > kArnMaxRows) throw Error{YK_ERR_INTERNAL, "Arnoldi finish: too many basis vectors"};
    hipLaunchKernelGGL(k_arnoldi_finish, dim3(std::max(1u, nblk(n, 256))), dim3(256), 0, ctx.stream, n, V, ld,
                       w, nsub, p, arn_chunks(n), h2_out, nrm2_out, y, h1, host_dst);
    check_launch(ctx, "k_arnoldi_finish");
}

double *arnoldi_partials(Context &ctx, int which) {
    const size_t one = (size_t)kArnMaxChunks * (kArnMaxRows + 1);
    return ctx.arn_partial.ensure(3 * one) + (size_t)which * one;
}

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

void launch_sumsq3(Context &ctx, int64_t n, const double *x0, const double *x1, const double *x2, double *h) {
    int nchunk = (int)std::min<int64_t>(kMaxChunks, (n + 4 * kRedBlock - 1) / (4 * kRedBlock));
    if (nchunk < 1) nchunk = 1;
    double *part = ctx.partial.ensure((size_t)kMaxChunks * 128);
    hipLaunchKernelGGL(k_sumsq3, dim3(nchunk, 3), dim3(kRedBlock), 0, ctx.stream, n, x0, x1, x2, part);
    check_launch(ctx, "k_sumsq3");
    hipLaunchKernelGGL(k_reduce_rows2, dim3(1), dim3(64), 0, ctx.stream, 3, nchunk, part, h);
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
