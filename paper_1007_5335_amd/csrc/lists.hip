// lists.hip -- interaction lists of the quadtree built on the GPU from the
// sorted keys (the quad-tree of Sec. 3.1 with the classical FMM lists):
//   * per sorted point: its leaf, and per (leaf, point set) the range of
//     sorted positions the leaf owns;
//   * U list of each leaf: the non-empty leaves of its 3 x 3 neighbourhood
//     (itself included), in row order (dy outer, dx inner);
//   * V list of each box: 27 slots, the children of the parent's neighbours
//     that are not adjacent, in the order of the box's parity class (the
//     slot -> offset table of the plan), -1 where the box is absent.
// Every lookup is a binary search in the sorted codes of one level, one
// thread per leaf or box; nothing is accumulated, so the lists are exact.
#include <algorithm>
#include <numeric>

#include "fmm.h"

namespace yk {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ uint32_t spread15d(uint32_t v) {
    v &= 0x7fff;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
__device__ __forceinline__ uint32_t compact15d(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

// index of c in the sorted a[0, n), or -1
__device__ __forceinline__ int64_t find_sorted(const uint32_t *__restrict__ a, int64_t n, uint32_t c) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && a[lo] == c) ? lo : -1;
}

// pleaf[k] = leaf of sorted point k; lrange[leaf][2 s], [2 s + 1] = first and
// one-past-last sorted position of set s in the leaf (zero-initialised)
__global__ void k_point_leaves(int64_t n, const uint32_t *__restrict__ keys, int shift,
                               const uint32_t *__restrict__ leaf_codes, int64_t nleaf,
                               int32_t *__restrict__ pleaf, int32_t *__restrict__ lrange) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    constexpr uint32_t kMask = 0x3fffffffu;
    const uint32_t key = keys[k];
    const uint32_t s = key >> 30, lc = (key & kMask) >> shift;
    const int64_t li = find_sorted(leaf_codes, nleaf, lc);
    if (li < 0) return;   // (cannot happen: the leaf codes are these points' own)
    pleaf[k] = (int32_t)li;
    auto same_run = [&](uint32_t other) { return (other >> 30) == s && ((other & kMask) >> shift) == lc; };
    if (k == 0 || !same_run(keys[k - 1])) lrange[li * 6 + 2 * s] = (int32_t)k;
    if (k == n - 1 || !same_run(keys[k + 1])) lrange[li * 6 + 2 * s + 1] = (int32_t)(k + 1);
}

// U lists: the non-empty leaves among the 3 x 3 neighbourhood; count (out ==
// nullptr) or fill from offsets uoff
__global__ void k_ulist(int64_t nleaf, const uint32_t *__restrict__ leaf_codes, int L,
                        const int32_t *__restrict__ uoff, int32_t *__restrict__ cnt_or_out) {
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const uint32_t c = leaf_codes[li];
    const int64_t ix = compact15d(c), iy = compact15d(c >> 1), ns = (int64_t)1 << L;
    int32_t k = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int64_t jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jy < 0 || jx >= ns || jy >= ns) continue;
            const int64_t j = find_sorted(leaf_codes, nleaf, spread15d((uint32_t)jx) | (spread15d((uint32_t)jy) << 1));
            if (j < 0) continue;
            if (uoff) cnt_or_out[uoff[li] + k] = (int32_t)j;
            ++k;
        }
    if (!uoff) cnt_or_out[li] = k;
}

// V lists of the boxes of one level (global indices begin .. begin + nb)
__global__ void k_vlist(int64_t begin, int64_t nb, const uint32_t *__restrict__ code, int l,
                        int32_t *__restrict__ vl) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const uint32_t c = code[begin + k];
    const int64_t ix = compact15d(c), iy = compact15d(c >> 1), ns = (int64_t)1 << l;
    const int cxs = (int)(ix & 1), cys = (int)(iy & 1);
    int slot = 0;
    for (int dy = -2 - cys; dy <= 3 - cys; ++dy)
        for (int dx = -2 - cxs; dx <= 3 - cxs; ++dx) {
            if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
            const int64_t jx = ix + dx, jy = iy + dy;
            int32_t src = -1;
            if (jx >= 0 && jy >= 0 && jx < ns && jy < ns) {
                const int64_t j = find_sorted(code + begin, nb,
                                              spread15d((uint32_t)jx) | (spread15d((uint32_t)jy) << 1));
                if (j >= 0) src = (int32_t)(begin + j);
            }
            vl[(begin + k) * kNumV + slot] = src;
            ++slot;
        }
}

// number of non-empty V-list slots of the listed boxes, one partial count per
// block (summed on the host)
__global__ __launch_bounds__(256) void k_count_slots(int64_t n, const int32_t *__restrict__ boxes,
                                                     const int32_t *__restrict__ vl,
                                                     unsigned int *__restrict__ part) {
    __shared__ unsigned int s[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned int c = 0;
    if (i < n) {
        const int32_t *v = vl + (int64_t)boxes[i] * kNumV;
        for (int k = 0; k < kNumV; ++k) c += v[k] >= 0 ? 1u : 0u;
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

}  // namespace

void gpu_point_leaves(Context &ctx, FmmPlan &pl, const uint32_t *dkeys, const uint32_t *dleaf_codes) {
    const int64_t N = pl.N, nleaf = pl.nleaf;
    int32_t *lr = pl.lrange.ensure((size_t)nleaf * 6);
    YK_HIP(hipMemsetAsync(lr, 0, (size_t)nleaf * 6 * sizeof(int32_t), ctx.stream));
    int32_t *pleaf = pl.pleaf.ensure((size_t)N);
    hipLaunchKernelGGL(k_point_leaves, dim3(nblk(N, 256)), dim3(256), 0, ctx.stream, N, dkeys,
                       2 * (kMaxLevel - pl.L), dleaf_codes, nleaf, pleaf, lr);
    check_launch(ctx, "k_point_leaves");
    pl.h_lrange.resize((size_t)nleaf * 6);
    YK_HIP(hipMemcpyAsync(pl.h_lrange.data(), lr, (size_t)nleaf * 6 * sizeof(int32_t), hipMemcpyDeviceToHost,
                          ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void gpu_ulists(Context &ctx, FmmPlan &pl, const uint32_t *dleaf_codes) {
    const int64_t nleaf = pl.nleaf;
    DevBuf<int32_t> cnt;
    int32_t *dc = cnt.ensure((size_t)nleaf);
    hipLaunchKernelGGL(k_ulist, dim3(nblk(nleaf, 256)), dim3(256), 0, ctx.stream, nleaf, dleaf_codes, pl.L,
                       (const int32_t *)nullptr, dc);
    check_launch(ctx, "k_ulist");
    std::vector<int32_t> hc((size_t)nleaf), uoff((size_t)nleaf + 1, 0);
    YK_HIP(hipMemcpyAsync(hc.data(), dc, (size_t)nleaf * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    for (int64_t i = 0; i < nleaf; ++i) uoff[i + 1] = uoff[i] + hc[i];
    int32_t *doff = pl.ulist_off.ensure((size_t)nleaf + 1);
    YK_HIP(hipMemcpyAsync(doff, uoff.data(), uoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
    int32_t *dul = pl.ulist.ensure(std::max<size_t>(1, (size_t)uoff[nleaf]));
    hipLaunchKernelGGL(k_ulist, dim3(nblk(nleaf, 256)), dim3(256), 0, ctx.stream, nleaf, dleaf_codes, pl.L, doff,
                       dul);
    check_launch(ctx, "k_ulist");
    pl.n_ulist = uoff[nleaf];
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void gpu_vlists(Context &ctx, FmmPlan &pl) {
    int32_t *vl = pl.vlist.ensure((size_t)pl.nbox * kNumV);
    YK_HIP(hipMemsetAsync(vl, 0xff, (size_t)pl.nbox * kNumV * sizeof(int32_t), ctx.stream));   // all -1
    for (int l = std::max(pl.lmin, 2); l <= pl.L; ++l) {
        const int64_t b0 = pl.lev[l].begin, nb = pl.lev[l].end - pl.lev[l].begin;
        if (nb <= 0) continue;
        hipLaunchKernelGGL(k_vlist, dim3(nblk(nb, 256)), dim3(256), 0, ctx.stream, b0, nb, pl.bcode.p, l, vl);
        check_launch(ctx, "k_vlist");
    }
}

int64_t gpu_count_slots(Context &ctx, FmmPlan &pl, const int32_t *dboxes, int64_t n) {
    if (n <= 0) return 0;
    const unsigned nb = nblk(n, 256);
    DevBuf<unsigned int> part;
    unsigned int *d = part.ensure(nb);
    hipLaunchKernelGGL(k_count_slots, dim3(nb), dim3(256), 0, ctx.stream, n, dboxes, pl.vlist.p, d);
    check_launch(ctx, "k_count_slots");
    std::vector<unsigned int> h(nb);
    YK_HIP(hipMemcpyAsync(h.data(), d, nb * sizeof(unsigned int), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    int64_t t = 0;
    for (unsigned int v : h) t += v;
    return t;
}

}  // namespace yk
