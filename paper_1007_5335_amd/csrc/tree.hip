// tree.hip -- Morton keys and a stable LSD radix sort on the GPU; the sorted
// keys then define the quadtree (fmm_plan.cpp).
//
// Sort key (32 bits): point-set id (2 bits) above the 30-bit Morton code of
// the point's cell at level 15 of the bounding square.  Sorting groups each
// set into one block, Morton-ordered inside, so every box of every level owns
// one contiguous range per set.
#include <chrono>
#include <cmath>

#include "fmm.h"

namespace yk {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ __launch_bounds__(256) void k_bbox(int64_t n, const double *__restrict__ xy,
                                              double *__restrict__ part) {
    __shared__ double s[4][256];
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double x = xy[2 * i], y = xy[2 * i + 1];
        mnx = fmin(mnx, x); mxx = fmax(mxx, x);
        mny = fmin(mny, y); mxy = fmax(mxy, y);
    }
    s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mny; s[2][threadIdx.x] = mxx; s[3][threadIdx.x] = mxy;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + off]);
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + off]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + off]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread15(uint32_t v) {
    v &= 0x7fff;
    v = (v | (v << 8)) & 0x00ff00ff;
    v = (v | (v << 4)) & 0x0f0f0f0f;
    v = (v | (v << 2)) & 0x33333333;
    v = (v | (v << 1)) & 0x55555555;
    return v;
}

__global__ void k_morton(int64_t n, const double *__restrict__ xy, double x0, double y0,
                         double inv_cell, uint32_t set, uint32_t gbase, uint32_t *__restrict__ key,
                         uint32_t *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double fx = (xy[2 * i] - x0) * inv_cell, fy = (xy[2 * i + 1] - y0) * inv_cell;
    int ix = (int)floor(fx), iy = (int)floor(fy);
    ix = min(max(ix, 0), (1 << kMaxLevel) - 1);
    iy = min(max(iy, 0), (1 << kMaxLevel) - 1);
    key[i] = (set << 30) | spread15((uint32_t)ix) | (spread15((uint32_t)iy) << 1);
    val[i] = gbase + (uint32_t)i;
}

// hist[d * nblk + b] = number of keys of block b with digit d
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                             int64_t n, int shift,
                                                             uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of 1024-element segments; segment totals to sums[]
__global__ __launch_bounds__(1024) void k_scan_seg(uint32_t *__restrict__ a, int64_t n,
                                                   uint32_t *__restrict__ sums) {
    __shared__ uint32_t s[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = i < n ? a[i] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) a[i] = s[threadIdx.x] - v;
    if (threadIdx.x == 1023) sums[blockIdx.x] = s[1023];
}

// sequential exclusive scan of the segment totals (one block, chunks of 1024)
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ sums, int64_t m) {
    __shared__ uint32_t s[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < m; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t v = i < m ? sums[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < m) sums[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += s[1023];
        __syncthreads();
    }
}

__global__ void k_scan_add(uint32_t *__restrict__ a, int64_t n, const uint32_t *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) a[i] += sums[blockIdx.x];
}

// Stable scatter: keys are ranked round by round (256 at a time, in input
// order); inside a wavefront equal digits are matched with 8 ballots.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offs) {
    __shared__ uint32_t base_d[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = gridDim.x;
    base_d[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            mask &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(mask & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            const uint32_t pos = base_d[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][tid];
        base_d[tid] += add;
        __syncthreads();
    }
}

// Sorted coordinates and, per sorted position, the index within its own set.
__global__ void k_gather_points(int64_t n, const uint32_t *__restrict__ keys,
                                const uint32_t *__restrict__ vals, const double *__restrict__ xy0,
                                const double *__restrict__ xy1, const double *__restrict__ xy2,
                                int64_t g1, int64_t g2, double *__restrict__ px,
                                double *__restrict__ py, int32_t *__restrict__ perm) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t set = keys[k] >> 30;
    const int64_t g = vals[k];
    const double *src = set == 0 ? xy0 : (set == 1 ? xy1 : xy2);
    const int64_t i = g - (set == 0 ? 0 : (set == 1 ? g1 : g2));
    px[k] = src[2 * i];
    py[k] = src[2 * i + 1];
    perm[k] = (int32_t)i;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void exclusive_scan(Context &ctx, uint32_t *a, int64_t n, DevBuf<uint32_t> &tmp) {
    const int64_t nseg = (n + 1023) / 1024;
    uint32_t *sums = tmp.ensure(nseg);
    hipLaunchKernelGGL(k_scan_seg, dim3(nseg), dim3(1024), 0, ctx.stream, a, n, sums);
    check_launch(ctx, "k_scan_seg");
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, ctx.stream, sums, nseg);
    check_launch(ctx, "k_scan_sums");
    hipLaunchKernelGGL(k_scan_add, dim3(nseg), dim3(1024), 0, ctx.stream, a, n, sums);
    check_launch(ctx, "k_scan_add");
}

}  // namespace

// Stable sort of (key, value) pairs by the low `bits` bits of the key.
void radix_sort_pairs(Context &ctx, uint32_t *&keys, uint32_t *&vals, uint32_t *&ktmp,
                      uint32_t *&vtmp, int64_t n, int bits) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    DevBuf<uint32_t> hist, scan_tmp;
    uint32_t *h = hist.ensure(256 * nb);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, ctx.stream, keys, n, shift, h);
        check_launch(ctx, "k_radix_hist");
        exclusive_scan(ctx, h, 256 * nb, scan_tmp);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, ctx.stream, keys, vals,
                           ktmp, vtmp, n, shift, h);
        check_launch(ctx, "k_radix_scatter");
        std::swap(keys, ktmp);
        std::swap(vals, vtmp);
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));   // hist/scan_tmp are freed on return
}

void build_tree(Context &ctx, FmmPlan &pl, const SumProblem &pb) {
    auto t0 = std::chrono::steady_clock::now();
    int64_t N = pb.n[0] + pb.n[1] + pb.n[2];
    YK_REQUIRE(N > 0 && N < ((int64_t)1 << 31), "point count out of range for the tree");
    pl.N = N;
    // bounding square
    double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
    {
        const int nbk = 256;
        DevBuf<double> part;
        double *dp = part.ensure(4 * nbk);
        std::vector<double> h(4 * nbk);
        for (int s = 0; s < 3; ++s) {
            if (pb.n[s] == 0) continue;
            hipLaunchKernelGGL(k_bbox, dim3(nbk), dim3(256), 0, ctx.stream, pb.n[s], pb.xy[s], dp);
            check_launch(ctx, "k_bbox");
            YK_HIP(hipMemcpyAsync(h.data(), dp, 4 * nbk * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
            YK_HIP(hipStreamSynchronize(ctx.stream));
            for (int b = 0; b < nbk; ++b) {
                mn[0] = std::fmin(mn[0], h[4 * b]); mn[1] = std::fmin(mn[1], h[4 * b + 1]);
                mx[0] = std::fmax(mx[0], h[4 * b + 2]); mx[1] = std::fmax(mx[1], h[4 * b + 3]);
            }
        }
    }
    YK_REQUIRE(std::isfinite(mn[0]) && std::isfinite(mn[1]) && std::isfinite(mx[0]) && std::isfinite(mx[1]),
               "point coordinates are not finite");
    if (pb.square) {
        YK_REQUIRE(pb.square[2] > 0.0 && mn[0] >= pb.square[0] && mn[1] >= pb.square[1] &&
                       mx[0] < pb.square[0] + pb.square[2] && mx[1] < pb.square[1] + pb.square[2],
                   "points outside the given bounding square");
        pl.x0 = pb.square[0];
        pl.y0 = pb.square[1];
        pl.size = pb.square[2];
    } else {
        double ext = std::fmax(mx[0] - mn[0], mx[1] - mn[1]);
        if (ext <= 0) ext = 1e-6 * std::fmax(1.0, std::fabs(mn[0]) + std::fabs(mn[1]));
        pl.size = ext * (1.0 + 1e-9);
        const double cxm = 0.5 * (mn[0] + mx[0]), cym = 0.5 * (mn[1] + mx[1]);
        pl.x0 = cxm - 0.5 * pl.size;
        pl.y0 = cym - 0.5 * pl.size;
    }
    const double inv_cell = (double)(1 << kMaxLevel) / pl.size;

    // keys
    DevBuf<uint32_t> kA, vA, kB, vB;
    uint32_t *keys = kA.ensure(N), *vals = vA.ensure(N), *kt = kB.ensure(N), *vt = vB.ensure(N);
    int64_t g = 0;
    for (int s = 0; s < 3; ++s) {
        if (pb.n[s] > 0) {
            hipLaunchKernelGGL(k_morton, dim3(nblk(pb.n[s], 256)), dim3(256), 0, ctx.stream, pb.n[s],
                               pb.xy[s], pl.x0, pl.y0, inv_cell, (uint32_t)s, (uint32_t)g, keys + g, vals + g);
            check_launch(ctx, "k_morton");
        }
        pl.toff[s] = g;
        g += pb.n[s];
    }
    pl.toff[3] = g;
    radix_sort_pairs(ctx, keys, vals, kt, vt, N, 32);
    pl.px.ensure(N);
    pl.py.ensure(N);
    pl.perm.ensure(N);
    hipLaunchKernelGGL(k_gather_points, dim3(nblk(N, 256)), dim3(256), 0, ctx.stream, N, keys, vals,
                       pb.xy[0], pb.xy[1], pb.xy[2], pl.toff[1], pl.toff[2], pl.px.p, pl.py.p, pl.perm.p);
    check_launch(ctx, "k_gather_points");
    std::vector<uint32_t> hkeys(N);
    YK_HIP(hipMemcpyAsync(hkeys.data(), keys, N * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    pl.adaptive = pl.opt_tree == 1;
    if (!pl.adaptive && !build_lists(ctx, pl, hkeys, keys)) pl.adaptive = true;
    if (pl.adaptive) build_lists_adaptive(ctx, pl, hkeys, keys);
    build_tables(ctx, pl, pl.opt_p > 0 ? supported_order(pl.opt_p) : choose_order(pl.opt_tol));
    pl.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace yk
