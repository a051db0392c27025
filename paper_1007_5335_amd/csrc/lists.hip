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

// ------------------------------------------------------ adaptive tree ---
// Boxes are compared in level-15 cells: a box of level l with code c covers
// [x0, x0 + 2^(15-l)] x [y0, y0 + 2^(15-l)], x0 = cx 2^(15-l), y0 = cy 2^(15-l)
// (closed squares: "touch" includes corners).
struct Sq { int64_t x0, y0, sz; };
__device__ __forceinline__ Sq box_sq(uint32_t code, int l) {
    const int k = kMaxLevel - l;
    return Sq{(int64_t)compact15d(code) << k, (int64_t)compact15d(code >> 1) << k, (int64_t)1 << k};
}
__device__ __forceinline__ bool sq_touch(const Sq &a, const Sq &b) {
    return a.x0 <= b.x0 + b.sz && b.x0 <= a.x0 + a.sz && a.y0 <= b.y0 + b.sz && b.y0 <= a.y0 + a.sz;
}

// pleaf[k] = the leaf holding sorted point k: the last leaf whose first
// level-15 cell is not above the point's (leaves are disjoint and cover every
// point); lrange as in k_point_leaves
__global__ void k_point_leaves_ad(int64_t n, const uint32_t *__restrict__ keys,
                                  const uint32_t *__restrict__ leaf_start, int64_t nleaf,
                                  int32_t *__restrict__ pleaf, int32_t *__restrict__ lrange) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    constexpr uint32_t kMask = 0x3fffffffu;
    const uint32_t key = keys[k], s = key >> 30, c = key & kMask;
    int64_t lo = 0, hi = nleaf;   // first leaf starting above c
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (leaf_start[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    const int64_t li = lo - 1;
    if (li < 0) return;   // (cannot happen: leaf 0 starts at the first point's cell or below)
    pleaf[k] = (int32_t)li;
    const uint32_t first = leaf_start[li], next = li + 1 < nleaf ? leaf_start[li + 1] : 0xffffffffu;
    auto same_run = [&](uint32_t other) {
        const uint32_t oc = other & kMask;
        return (other >> 30) == s && oc >= first && oc < next;
    };
    if (k == 0 || !same_run(keys[k - 1])) lrange[li * 6 + 2 * s] = (int32_t)k;
    if (k == n - 1 || !same_run(keys[k + 1])) lrange[li * 6 + 2 * s + 1] = (int32_t)(k + 1);
}

constexpr int kAdStack = 64;   // depth-first stack of the list walks
constexpr int kMaxU = 16;      // U-list capacity (2:1 balance gives at most 13)

__device__ __forceinline__ void sort_slice(int32_t *a, int n) {
    for (int i = 1; i < n; ++i) {
        const int32_t v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
}

// U lists of the adaptive tree: the leaves touching each leaf, itself
// included, in increasing leaf index.  Each of the 8 neighbouring cells of
// the leaf's level is looked up: an existing leaf there is taken; a split box
// is walked depth first for the leaves among its descendants that touch the
// leaf; an absent cell is looked up at coarser levels, where the first box
// found holds it (taken if it is a leaf; if split, the cell is empty).
// count mode (out == nullptr): cnt_or_out[li] = the count; a count beyond the
// capacity sets *flag.
__global__ void k_ulist_ad(int64_t nleaf, const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ blevel,
                           const uint32_t *__restrict__ bcode, const int64_t *__restrict__ lev_begin,
                           const int32_t *__restrict__ box_leaf, const int32_t *__restrict__ fchild,
                           const int32_t *__restrict__ nchild, const int32_t *__restrict__ uoff,
                           int32_t *__restrict__ cnt_or_out, int *__restrict__ flag) {
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const int32_t b = leaf_box[li];
    const int l = blevel[b];
    const uint32_t code = bcode[b];
    const Sq sb = box_sq(code, l);
    const int64_t ix = compact15d(code), iy = compact15d(code >> 1), ns = (int64_t)1 << l;
    int32_t buf[kMaxU];
    int n = 0;
    bool over = false;
    auto add = [&](int32_t v, bool dedupe) {
        if (dedupe)
            for (int i = 0; i < n; ++i)
                if (buf[i] == v) return;
        if (n < kMaxU) buf[n] = v;
        else over = true;
        ++n;
    };
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) {
                add((int32_t)li, false);
                continue;
            }
            const int64_t jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jy < 0 || jx >= ns || jy >= ns) continue;
            const uint32_t c = spread15d((uint32_t)jx) | (spread15d((uint32_t)jy) << 1);
            const int64_t j = find_sorted(bcode + lev_begin[l], lev_begin[l + 1] - lev_begin[l], c);
            if (j >= 0) {
                const int32_t q = (int32_t)(lev_begin[l] + j);
                if (box_leaf[q] >= 0) {
                    add(box_leaf[q], false);
                    continue;
                }
                int32_t st[kAdStack];
                int top = 0;
                st[top++] = q;
                while (top > 0) {
                    const int32_t e = st[--top];
                    for (int32_t ch = fchild[e]; ch < fchild[e] + nchild[e]; ++ch) {
                        if (!sq_touch(box_sq(bcode[ch], blevel[ch]), sb)) continue;
                        if (box_leaf[ch] >= 0) add(box_leaf[ch], false);
                        else if (top < kAdStack) st[top++] = ch;
                        else over = true;
                    }
                }
            } else {
                for (int lc = l - 1; lc >= 0; --lc) {
                    const uint32_t cc = c >> (2 * (l - lc));
                    const int64_t jc = find_sorted(bcode + lev_begin[lc], lev_begin[lc + 1] - lev_begin[lc], cc);
                    if (jc < 0) continue;
                    const int32_t q = (int32_t)(lev_begin[lc] + jc);
                    if (box_leaf[q] >= 0) add(box_leaf[q], true);
                    break;
                }
            }
        }
    if (over) {
        atomicOr(flag, 1);
        return;
    }
    if (!uoff) {
        cnt_or_out[li] = n;
        return;
    }
    sort_slice(buf, n);
    for (int i = 0; i < n; ++i) cnt_or_out[uoff[li] + i] = buf[i];
}

// W lists: the boxes of levels >= lmin, finer than the leaf, whose parent
// touches the leaf and which do not touch it: a depth-first walk of the split
// colleagues' subtrees through the boxes that touch the leaf.  Increasing box
// index per leaf; count mode as above.
__global__ void k_wlist(int64_t nleaf, const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ blevel,
                        const uint32_t *__restrict__ bcode, const int64_t *__restrict__ lev_begin,
                        const int32_t *__restrict__ fchild, const int32_t *__restrict__ nchild, int lmin,
                        const int32_t *__restrict__ woff, int32_t *__restrict__ cnt_or_out, int *__restrict__ flag) {
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const int32_t b = leaf_box[li];
    const int l = blevel[b];
    const uint32_t code = bcode[b];
    const Sq sb = box_sq(code, l);
    const int64_t ix = compact15d(code), iy = compact15d(code >> 1), ns = (int64_t)1 << l;
    int32_t *out = woff ? cnt_or_out + woff[li] : nullptr;
    int n = 0;
    bool over = false;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int64_t jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jy < 0 || jx >= ns || jy >= ns) continue;
            const uint32_t c = spread15d((uint32_t)jx) | (spread15d((uint32_t)jy) << 1);
            const int64_t j = find_sorted(bcode + lev_begin[l], lev_begin[l + 1] - lev_begin[l], c);
            if (j < 0) continue;
            int32_t st[kAdStack];
            int top = 0;
            st[top++] = (int32_t)(lev_begin[l] + j);
            while (top > 0) {
                const int32_t e = st[--top];
                for (int32_t ch = fchild[e]; ch < fchild[e] + nchild[e]; ++ch) {
                    const int lc = blevel[ch];
                    if (sq_touch(box_sq(bcode[ch], lc), sb)) {
                        if (nchild[ch] > 0) {
                            if (top < kAdStack) st[top++] = ch;
                            else over = true;
                        }
                    } else if (lc >= lmin) {
                        if (out) out[n] = ch;
                        ++n;
                    }
                }
            }
        }
    if (over) {
        atomicOr(flag, 1);
        return;
    }
    if (!out) cnt_or_out[li] = n;
    else sort_slice(out, n);
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

namespace yk {

namespace {
// exclusive prefix sum of per-item counts, uploaded as CSR offsets
int64_t offsets_from_counts(Context &ctx, const int32_t *dcnt, int64_t n, DevBuf<int32_t> &off,
                            std::vector<int32_t> &hoff) {
    std::vector<int32_t> hc((size_t)n);
    if (n > 0) YK_HIP(hipMemcpyAsync(hc.data(), dcnt, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    hoff.assign((size_t)n + 1, 0);
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) {
        tot += hc[i];
        YK_REQUIRE(tot < ((int64_t)1 << 31), "interaction list too long");
        hoff[i + 1] = (int32_t)tot;
    }
    int32_t *d = off.ensure((size_t)n + 1);
    YK_HIP(hipMemcpyAsync(d, hoff.data(), hoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
    return tot;
}

int read_flag(Context &ctx, const int *dflag) {
    int h = 0;
    YK_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    return h;
}

DevBuf<int64_t> &level_begins(Context &ctx, FmmPlan &pl, DevBuf<int64_t> &buf) {
    std::vector<int64_t> lb(pl.L + 2);
    for (int l = 0; l <= pl.L; ++l) lb[l] = pl.lev[l].begin;
    lb[pl.L + 1] = pl.nbox;
    YK_HIP(hipMemcpyAsync(buf.ensure(lb.size()), lb.data(), lb.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx.stream));
    return buf;
}
}  // namespace

void gpu_point_leaves_adaptive(Context &ctx, FmmPlan &pl, const uint32_t *dkeys) {
    const int64_t N = pl.N, nleaf = pl.nleaf;
    int32_t *lr = pl.lrange.ensure((size_t)nleaf * 6);
    YK_HIP(hipMemsetAsync(lr, 0, (size_t)nleaf * 6 * sizeof(int32_t), ctx.stream));
    int32_t *pleaf = pl.pleaf.ensure((size_t)N);
    hipLaunchKernelGGL(k_point_leaves_ad, dim3(nblk(N, 256)), dim3(256), 0, ctx.stream, N, dkeys, pl.leaf_start.p,
                       nleaf, pleaf, lr);
    check_launch(ctx, "k_point_leaves_ad");
    pl.h_lrange.resize((size_t)nleaf * 6);
    YK_HIP(hipMemcpyAsync(pl.h_lrange.data(), lr, (size_t)nleaf * 6 * sizeof(int32_t), hipMemcpyDeviceToHost,
                          ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void gpu_ulists_adaptive(Context &ctx, FmmPlan &pl) {
    const int64_t nleaf = pl.nleaf;
    DevBuf<int64_t> lbuf;
    const int64_t *lb = level_begins(ctx, pl, lbuf).p;
    DevBuf<int32_t> cnt;
    DevBuf<int> flag;
    int *df = flag.ensure(1);
    YK_HIP(hipMemsetAsync(df, 0, sizeof(int), ctx.stream));
    int32_t *dc = cnt.ensure((size_t)nleaf);
    hipLaunchKernelGGL(k_ulist_ad, dim3(nblk(nleaf, 128)), dim3(128), 0, ctx.stream, nleaf, pl.leaf_box.p,
                       pl.blevel.p, pl.bcode.p, lb, pl.box_leaf.p, pl.fchild.p, pl.nchild.p,
                       (const int32_t *)nullptr, dc, df);
    check_launch(ctx, "k_ulist_ad");
    YK_REQUIRE(read_flag(ctx, df) == 0, "adaptive tree: a U list exceeds its capacity");
    std::vector<int32_t> hoff;
    const int64_t tot = offsets_from_counts(ctx, dc, nleaf, pl.ulist_off, hoff);
    int mu = 0;
    for (int64_t i = 0; i < nleaf; ++i) mu = std::max(mu, hoff[i + 1] - hoff[i]);
    pl.max_u = mu;
    int32_t *dul = pl.ulist.ensure(std::max<size_t>(1, (size_t)tot));
    hipLaunchKernelGGL(k_ulist_ad, dim3(nblk(nleaf, 128)), dim3(128), 0, ctx.stream, nleaf, pl.leaf_box.p,
                       pl.blevel.p, pl.bcode.p, lb, pl.box_leaf.p, pl.fchild.p, pl.nchild.p, pl.ulist_off.p, dul,
                       df);
    check_launch(ctx, "k_ulist_ad");
    pl.n_ulist = tot;
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void gpu_wlists(Context &ctx, FmmPlan &pl, std::vector<int32_t> &woff, std::vector<int32_t> &wl) {
    const int64_t nleaf = pl.nleaf;
    DevBuf<int64_t> lbuf;
    const int64_t *lb = level_begins(ctx, pl, lbuf).p;
    DevBuf<int32_t> cnt;
    DevBuf<int> flag;
    int *df = flag.ensure(1);
    YK_HIP(hipMemsetAsync(df, 0, sizeof(int), ctx.stream));
    int32_t *dc = cnt.ensure((size_t)nleaf);
    hipLaunchKernelGGL(k_wlist, dim3(nblk(nleaf, 128)), dim3(128), 0, ctx.stream, nleaf, pl.leaf_box.p,
                       pl.blevel.p, pl.bcode.p, lb, pl.fchild.p, pl.nchild.p, pl.lmin, (const int32_t *)nullptr, dc,
                       df);
    check_launch(ctx, "k_wlist");
    YK_REQUIRE(read_flag(ctx, df) == 0, "adaptive tree: a W-list walk exceeds its stack");
    const int64_t tot = offsets_from_counts(ctx, dc, nleaf, pl.woff, woff);
    int32_t *dwl = pl.wl.ensure(std::max<size_t>(1, (size_t)tot));
    if (tot > 0) {
        hipLaunchKernelGGL(k_wlist, dim3(nblk(nleaf, 128)), dim3(128), 0, ctx.stream, nleaf, pl.leaf_box.p,
                           pl.blevel.p, pl.bcode.p, lb, pl.fchild.p, pl.nchild.p, pl.lmin, pl.woff.p, dwl, df);
        check_launch(ctx, "k_wlist");
    }
    pl.n_wl = tot;
    wl.resize((size_t)tot);
    if (tot > 0)
        YK_HIP(hipMemcpyAsync(wl.data(), dwl, (size_t)tot * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

}  // namespace yk
