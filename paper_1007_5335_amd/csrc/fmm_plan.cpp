// fmm_plan.cpp -- quadtree, interaction lists and translation operators on the host.
//
// The tree has uniform depth L (every leaf at level L) but stores only
// non-empty boxes, so clustered boundary nodes cost nothing where there are
// none.  Lists: U (the non-empty leaves among a leaf's 3x3 neighbourhood,
// itself included: near field by direct summation) and V (the children of the
// parent's neighbours that are not adjacent: far field by M2L), the classical
// lists of the FMM the paper relies on (Sec. 3, with the quadtree of Sec. 3.1).
// Levels whose boxes are wider than 40 alpha get no M2L: across such a gap
// the kernel is below K0(40) ~ 1e-18.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <thread>

#include "fmm.h"
#include "yk_bessel.h"

namespace yk {

using ld = long double;
using cld = std::complex<long double>;

namespace {

constexpr double kFarCut = 40.0;

inline uint32_t compact15(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}
inline uint32_t spread(uint32_t v) {
    v &= 0x7fff;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
inline uint32_t encode(uint32_t ix, uint32_t iy) { return spread(ix) | (spread(iy) << 1); }
inline void decode(uint32_t c, uint32_t &ix, uint32_t &iy) {
    ix = compact15(c);
    iy = compact15(c >> 1);
}

// F_n(y) = sum_k y^k / (k! (n+1)_k), so that I_n(x) = (x/2)^n / n! F_n(x^2/4).
ld F_series(int n, ld y) {
    ld t = 1, s = 1;
    for (int k = 1; k < 20000; ++k) {
        t *= y / ((ld)k * (ld)(n + k));
        s += t;
        if (t < 1e-22L * s) break;
    }
    return s;
}

// I_0..I_nmax at x (x >= 0) in extended precision
std::vector<ld> I_seq(ld x, int nmax) {
    std::vector<ld> I(nmax + 1);
    const ld y = 0.25L * x * x;
    ld pref = 1;                           // (x/2)^n / n!
    for (int n = 0; n <= nmax; ++n) {
        if (n > 0) pref *= (0.5L * x) / (ld)n;
        I[n] = pref * F_series(n, y);
    }
    return I;
}

// K_0..K_nmax at x > 0: K0, K1 from the library's own evaluation, then the
// forward recurrence K_{n+1} = K_{n-1} + (2n/x) K_n (stable upwards).
std::vector<ld> K_seq(double x, int nmax) {
    std::vector<ld> K(nmax + 1);
    K[0] = (ld)yk::k0(x);
    if (nmax >= 1) K[1] = (ld)yk::k1(x);
    for (int n = 1; n < nmax; ++n) K[n + 1] = K[n - 1] + (2.0L * n / (ld)x) * K[n];
    return K;
}

// Real form of out_k = sum_{n=-p..p} C[k][n] v_n (k = 0..p) for v_{-n} = conj(v_n):
// vectors are [Re v_0, Re v_1, Im v_1, ...]; the Pp x Pp result is column-major.
void to_real(const std::vector<cld> &C, int p, int Pp, double *out) {
    auto c = [&](int k, int n) { return C[(size_t)k * (2 * p + 1) + (n + p)]; };
    std::fill(out, out + (size_t)Pp * Pp, 0.0);
    auto put = [&](int row, int col, ld v) { out[(size_t)col * Pp + row] = (double)v; };
    for (int k = 0; k <= p; ++k) {
        const int rr = k == 0 ? 0 : 2 * k - 1, ri = 2 * k;
        // column of v_0
        put(rr, 0, c(k, 0).real());
        if (k > 0) put(ri, 0, c(k, 0).imag());
        for (int n = 1; n <= p; ++n) {
            const cld sp = c(k, n) + c(k, -n), sm = c(k, n) - c(k, -n);
            put(rr, 2 * n - 1, sp.real());
            put(rr, 2 * n, -sm.imag());
            if (k > 0) {
                put(ri, 2 * n - 1, sp.imag());
                put(ri, 2 * n, sm.real());
            }
        }
    }
}

inline cld cis(ld phi, int m) { return std::polar((ld)1, phi * (ld)m); }

// f(i0, i1) on contiguous chunks of [0, n) on up to 16 host threads
template <typename F>
void parallel_for(int64_t n, F f) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                (n + 65535) / 65536}));
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    const int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nt && t * per < n; ++t) pool.emplace_back(f, t * per, std::min(n, (t + 1) * per));
    for (auto &th : pool) th.join();
}

}  // namespace

int supported_order(int p) {
    // the orders the expansion kernels are instantiated for (P = 2p + 1 real
    // coefficients padded to 16, 32, 48 or 64)
    for (int q : kOrders)
        if (p <= q) return q;
    return kOrders[kNumOrders - 1];
}

int choose_order(double tol) {
    // Measured on uniform and clustered point sets: the relative error of the
    // sums behaves like 0.0123 * 0.44^p; take the smallest p with half the
    // tolerance to spare.
    int p = (int)std::ceil(std::log(0.5 * tol / 0.0123) / std::log(0.44));
    return supported_order(std::max(1, p));
}

// the level-15 Morton codes of all points in one sorted sequence (each set's
// block of the sorted keys is sorted)
std::vector<uint32_t> merged_codes(const FmmPlan &pl, const std::vector<uint32_t> &keys) {
    const uint32_t kMask = 0x3fffffffu;
    std::vector<uint32_t> merged;
    merged.reserve(pl.N);
    std::vector<uint32_t> a, b;
    for (int s = 0; s < 3; ++s) {
        if (pl.toff[s + 1] == pl.toff[s]) continue;
        b.resize(pl.toff[s + 1] - pl.toff[s]);
        for (int64_t k = pl.toff[s]; k < pl.toff[s + 1]; ++k) b[k - pl.toff[s]] = keys[k] & kMask;
        a.swap(merged);
        merged.resize(a.size() + b.size());
        std::merge(a.begin(), a.end(), b.begin(), b.end(), merged.begin());
    }
    return merged;
}

// boxes of levels 0..L from the sorted codes of each level: level ranges,
// codes, parents (by a merge of consecutive levels) and centres
void boxes_from_codes(FmmPlan &pl, const std::vector<std::vector<uint32_t>> &codes, std::vector<double> &cx,
                      std::vector<double> &cy) {
    const int L = pl.L;
    pl.lev.assign(L + 1, LevelInfo{});
    int64_t nb = 0;
    for (int l = 0; l <= L; ++l) {
        pl.lev[l].begin = nb;
        nb += (int64_t)codes[l].size();
        pl.lev[l].end = nb;
        pl.lev[l].side = pl.size / (double)(1u << l);
        pl.lev[l].R = pl.lev[l].side * 0.70710678118654752440 / pl.alpha;
    }
    pl.nbox = nb;
    pl.hcode.resize(nb);
    pl.hparent.assign(nb, -1);
    cx.resize(nb);
    cy.resize(nb);
    for (int l = 0; l <= L; ++l) {
        int64_t pi = 0;
        for (size_t k = 0; k < codes[l].size(); ++k) {
            const int64_t gidx = pl.lev[l].begin + (int64_t)k;
            pl.hcode[gidx] = codes[l][k];
            uint32_t ix, iy;
            decode(codes[l][k], ix, iy);
            cx[gidx] = pl.x0 + (ix + 0.5) * pl.lev[l].side;
            cy[gidx] = pl.y0 + (iy + 0.5) * pl.lev[l].side;
            if (l > 0) {
                while (codes[l - 1][pi] != (codes[l][k] >> 2)) ++pi;
                pl.hparent[gidx] = (int32_t)(pl.lev[l - 1].begin + pi);
            }
        }
    }
}

void finish_tree(Context &ctx, FmmPlan &pl, const std::vector<double> &cx, const std::vector<double> &cy,
                 const uint32_t *dkeys);

std::vector<long double> bessel_i_seq(long double x, int nmax) { return I_seq(x, nmax); }

int near_series_terms(double tmax) {
    const double tt = std::min(1.0, tmax);
    const double weight = 0.5 * std::fabs(std::log(tt)) + 3.0;
    const double k0min = std::max(0.11, -0.5 * std::log(tt) - 0.58);
    int k = 1;
    double term = 1;
    for (; k < YK_NSER64; ++k) {
        term *= tt / ((double)k * (double)k);
        if (term * weight < 0x1p-54 * k0min) break;
    }
    return std::min(YK_NSER64, k);
}

bool build_lists(Context &ctx, FmmPlan &pl, const std::vector<uint32_t> &keys, const uint32_t *dkeys) {
    const int64_t N = pl.N;
    // ---- merged Morton codes (each set's block is sorted) ----
    std::vector<uint32_t> merged = merged_codes(pl, keys);
    // ---- leaf level: smallest level whose point-weighted occupancy
    //      sum_i n_i^2 / N (the leaf size seen by an average point, which sets
    //      the near-field work per target) is <= leaf_size ----
    std::vector<uint32_t> uniq15;
    std::vector<int64_t> cnt15;
    uniq15.reserve(N);
    cnt15.reserve(N);
    for (int64_t k = 0; k < N; ++k) {
        if (k == 0 || merged[k] != merged[k - 1]) {
            uniq15.push_back(merged[k]);
            cnt15.push_back(0);
        }
        cnt15.back()++;
    }
    std::vector<std::vector<uint32_t>> codes(kMaxLevel + 1);
    std::vector<double> occ(kMaxLevel + 1, 0.0);
    {
        // coarsen the (code, count) runs in place, level by level
        std::vector<uint32_t> &c = uniq15;
        std::vector<int64_t> &n = cnt15;
        for (int l = kMaxLevel; l >= 0; --l) {
            double s2 = 0;
            for (int64_t v : n) s2 += (double)v * (double)v;
            occ[l] = s2 / (double)N;
            if (l == 0) break;
            size_t m = 0;
            for (size_t k = 0; k < c.size(); ++k) {
                const uint32_t v = c[k] >> 2;
                if (m > 0 && c[m - 1] == v) {
                    n[m - 1] += n[k];
                } else {
                    c[m] = v;
                    n[m] = n[k];
                    ++m;
                }
            }
            c.resize(m);
            n.resize(m);
        }
    }
    int L = kMaxLevel;
    for (int l = 0; l <= kMaxLevel; ++l) {
        if (occ[l] <= (double)pl.opt_leaf) {
            L = l;
            break;
        }
    }
    pl.L = L;
    codes.resize(L + 1);
    // codes at levels <= L come from level L's prefixes
    codes[L].clear();
    for (int64_t k = 0; k < N; ++k) {
        const uint32_t v = merged[k] >> (2 * (kMaxLevel - L));
        if (codes[L].empty() || codes[L].back() != v) codes[L].push_back(v);
    }
    // automatic form: points so clustered that the uniform tree's leaves are
    // mostly near-empty (more than six times N / leaf_size of them; a uniform
    // random set stays below four) take the adaptive tree instead
    if (pl.opt_tree == 2 && (double)codes[L].size() > 6.0 * (double)N / (double)pl.opt_leaf) return false;
    for (int l = L - 1; l >= 0; --l) {
        codes[l].clear();
        for (uint32_t v : codes[l + 1])
            if (codes[l].empty() || codes[l].back() != (v >> 2)) codes[l].push_back(v >> 2);
    }
    // ---- boxes ----
    std::vector<double> cx, cy;
    boxes_from_codes(pl, codes, cx, cy);
    pl.nleaf = (int64_t)codes[L].size();
    pl.near_tmax = 2.0 * pl.lev[L].side * pl.lev[L].side / (pl.alpha * pl.alpha);
    // ---- M2L levels ----
    int lmin = 2;
    while (lmin <= L && pl.lev[lmin].side >= kFarCut * pl.alpha) ++lmin;
    pl.lmin = lmin;
    auto up = [&](auto &buf, const auto &vec) {
        using T = typename std::decay_t<decltype(vec)>::value_type;
        T *d = buf.ensure(vec.size());
        YK_HIP(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    };
    up(pl.bcode, pl.hcode);
    const uint32_t *dleaf_codes = pl.bcode.p + pl.lev[L].begin;
    // ---- on the GPU: each point's leaf and the leaves' ranges per set, the
    //      U lists of the leaves and the V lists of every box (lists.hip) ----
    gpu_point_leaves(ctx, pl, dkeys, dleaf_codes);
    gpu_ulists(ctx, pl, dleaf_codes);
    gpu_vlists(ctx, pl);
    finish_tree(ctx, pl, cx, cy, dkeys);
    return true;
}

// The adaptive tree (Sec. 3.1's quad-tree refined box by box): a box is split
// while it holds more than leaf_size / 2 points (down to level 15); then, until
// nothing changes, a leaf touched by an existing box two levels finer is split
// (2:1 balance, so that touching leaves differ by at most one level and a U
// list holds at most 13 leaves).  Leaves are numbered in Morton order of their
// first level-15 cell; the U and W lists are built on the GPU (lists.hip), X
// is the transpose of W.
void build_lists_adaptive(Context &ctx, FmmPlan &pl, const std::vector<uint32_t> &keys, const uint32_t *dkeys) {
    // split above half the leaf size: the leaves then hold about as many
    // points on average as the uniform tree's (measured fastest on clustered
    // sets: a split box's children hold a quarter of it each)
    const int64_t N = pl.N, s = std::max(1, pl.opt_leaf / 2);
    std::vector<uint32_t> merged = merged_codes(pl, keys);
    // Boxes are built top down: a box of level l with code c holds the points
    // whose level-15 codes lie in [c 4^(15-l), (c + 1) 4^(15-l)), a range of
    // the sorted codes found by binary search; only boxes of the tree are
    // ever formed.  Per level: codes (Morton order), point ranges, leaf flag.
    struct Lev {
        std::vector<uint32_t> code;
        std::vector<int64_t> a, e;
        std::vector<char> leaf;
    };
    std::vector<Lev> tl(kMaxLevel + 1);
    auto lower = [&](uint64_t c) -> int64_t {
        return (int64_t)(std::lower_bound(merged.begin(), merged.end(), (uint32_t)std::min<uint64_t>(c, 0xffffffffu)) -
                         merged.begin());
    };
    // the non-empty children of box (l, c) with points [a, e), appended to level l + 1
    auto children = [&](int l, uint32_t c, int64_t a, int64_t e, std::vector<uint32_t> &cc,
                        std::vector<int64_t> &ca, std::vector<int64_t> &ce) {
        const int sh = 2 * (kMaxLevel - l - 1);
        int64_t lo = a;
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t ch = (c << 2) | q;
            const int64_t hi = q == 3 ? e : std::max(lo, std::min(e, lower((uint64_t)(ch + 1) << sh)));
            if (hi > lo) {
                cc.push_back(ch);
                ca.push_back(lo);
                ce.push_back(hi);
            }
            lo = hi;
        }
    };
    tl[0].code = {0};
    tl[0].a = {0};
    tl[0].e = {N};
    tl[0].leaf = {0};
    for (int l = 0; l <= kMaxLevel; ++l) {
        Lev &L0 = tl[l];
        L0.leaf.assign(L0.code.size(), 1);
        if (l == kMaxLevel) break;
        Lev &L1 = tl[l + 1];
        for (size_t k = 0; k < L0.code.size(); ++k)
            if (L0.e[k] - L0.a[k] > s) {
                L0.leaf[k] = 0;
                children(l, L0.code[k], L0.a[k], L0.e[k], L1.code, L1.a, L1.e);
            }
        if (L1.code.empty()) break;
    }
    // 2:1 balance: the 20 cells two levels finer that ring a leaf touch it;
    // a leaf with a box of the tree among them is split (its children hold
    // at most its points: leaves), until nothing changes
    for (bool changed = true; changed;) {
        changed = false;
        for (int l = 0; l + 2 <= kMaxLevel; ++l) {
            const std::vector<uint32_t> &ex = tl[l + 2].code;
            if (ex.empty() || tl[l].code.empty()) continue;
            const int64_t nl = (int64_t)tl[l].code.size();
            std::vector<char> hit((size_t)nl, 0);
            const int64_t ns = (int64_t)1 << (l + 2);
            parallel_for(nl, [&](int64_t i0, int64_t i1) {
                for (int64_t k = i0; k < i1; ++k) {
                    if (!tl[l].leaf[k]) continue;
                    uint32_t bx, by;
                    decode(tl[l].code[k], bx, by);
                    for (int j = -1; j <= 4 && !hit[k]; ++j)
                        for (int i = -1; i <= 4; ++i) {
                            if (i >= 0 && i <= 3 && j >= 0 && j <= 3) continue;
                            const int64_t X = 4 * (int64_t)bx + i, Y = 4 * (int64_t)by + j;
                            if (X < 0 || Y < 0 || X >= ns || Y >= ns) continue;
                            if (std::binary_search(ex.begin(), ex.end(), encode((uint32_t)X, (uint32_t)Y))) {
                                hit[k] = 1;
                                break;
                            }
                        }
                }
            });
            std::vector<uint32_t> nc;
            std::vector<int64_t> na, ne;
            for (int64_t k = 0; k < nl; ++k) {
                if (!hit[k]) continue;
                changed = true;
                tl[l].leaf[k] = 0;
                children(l, tl[l].code[k], tl[l].a[k], tl[l].e[k], nc, na, ne);
            }
            if (nc.empty()) continue;
            // merge the new leaves into the next level (both sorted)
            Lev &L1 = tl[l + 1];
            Lev m;
            const size_t n1 = L1.code.size(), n2 = nc.size();
            m.code.reserve(n1 + n2);
            size_t x = 0, y = 0;
            while (x < n1 || y < n2) {
                if (y == n2 || (x < n1 && L1.code[x] < nc[y])) {
                    m.code.push_back(L1.code[x]);
                    m.a.push_back(L1.a[x]);
                    m.e.push_back(L1.e[x]);
                    m.leaf.push_back(L1.leaf[x]);
                    ++x;
                } else {
                    m.code.push_back(nc[y]);
                    m.a.push_back(na[y]);
                    m.e.push_back(ne[y]);
                    m.leaf.push_back(1);
                    ++y;
                }
            }
            L1 = std::move(m);
        }
    }
    int L = 0;
    for (int l = 0; l <= kMaxLevel; ++l)
        if (!tl[l].code.empty()) L = l;
    pl.L = L;
    std::vector<std::vector<uint32_t>> codes(L + 1);
    std::vector<std::vector<int8_t>> lst(L + 1);
    for (int l = 0; l <= L; ++l) {
        codes[l] = std::move(tl[l].code);
        lst[l].resize(codes[l].size());
        for (size_t k = 0; k < codes[l].size(); ++k) lst[l][k] = tl[l].leaf[k] ? 1 : 2;
    }
    tl.clear();
    merged.clear();
    merged.shrink_to_fit();
    enum : int8_t { kLeafBox = 1 };
    std::vector<double> cx, cy;
    boxes_from_codes(pl, codes, cx, cy);
    const int64_t nb = pl.nbox;
    // leaves in Morton order of their first level-15 cell
    pl.h_blevel.assign(nb, 0);
    pl.h_box_leaf.assign(nb, -1);
    std::vector<std::pair<uint32_t, int32_t>> lv;
    for (int l = 0; l <= L; ++l)
        for (int64_t b = pl.lev[l].begin; b < pl.lev[l].end; ++b) {
            pl.h_blevel[b] = l;
            if (lst[l][b - pl.lev[l].begin] == kLeafBox)
                lv.push_back({pl.hcode[b] << (2 * (kMaxLevel - l)), (int32_t)b});
        }
    std::sort(lv.begin(), lv.end());
    pl.nleaf = (int64_t)lv.size();
    pl.h_leaf_box.resize(lv.size());
    std::vector<uint32_t> lstart(lv.size());
    std::vector<int32_t> llev(lv.size());
    for (size_t k = 0; k < lv.size(); ++k) {
        pl.h_leaf_box[k] = lv[k].second;
        pl.h_box_leaf[lv[k].second] = (int32_t)k;
        lstart[k] = lv[k].first;
        llev[k] = pl.h_blevel[lv[k].second];
    }
    int lmin = 2;
    while (lmin <= L && pl.lev[lmin].side >= kFarCut * pl.alpha) ++lmin;
    pl.lmin = lmin;
    auto up = [&](auto &buf, const auto &vec) {
        using T = typename std::decay_t<decltype(vec)>::value_type;
        T *d = buf.ensure(std::max<size_t>(vec.size(), 1));
        if (!vec.empty())
            YK_HIP(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    };
    up(pl.bcode, pl.hcode);
    up(pl.blevel, pl.h_blevel);
    up(pl.leaf_box, pl.h_leaf_box);
    up(pl.box_leaf, pl.h_box_leaf);
    up(pl.leaf_start, lstart);
    up(pl.leaf_lev, llev);
    finish_tree(ctx, pl, cx, cy, dkeys);   // children (the list walks need them)
    // ---- on the GPU: each point's leaf and the ranges, U and W lists, V lists ----
    gpu_point_leaves_adaptive(ctx, pl, dkeys);
    gpu_ulists_adaptive(ctx, pl);
    gpu_vlists(ctx, pl);
    std::vector<int32_t> woff, wl;
    gpu_wlists(ctx, pl, woff, wl);
    // ---- X lists: the transpose of W (source leaves in increasing index) ----
    {
        std::vector<int32_t> xc(nb, 0);
        for (int32_t d : wl) xc[d]++;
        std::vector<int32_t> xbox, xoff, xpos(nb, -1);
        xoff.push_back(0);
        for (int64_t d = 0; d < nb; ++d)
            if (xc[d] > 0) {
                xpos[d] = (int32_t)xbox.size();
                xbox.push_back((int32_t)d);
                xoff.push_back(xoff.back() + xc[d]);
            }
        std::vector<int32_t> xl(wl.size()), fill(xbox.size(), 0);
        std::vector<int32_t> wleaves;
        for (int64_t li = 0; li < pl.nleaf; ++li) {
            if (woff[li + 1] > woff[li]) wleaves.push_back((int32_t)li);
            for (int32_t k = woff[li]; k < woff[li + 1]; ++k) {
                const int32_t x = xpos[wl[k]];
                xl[xoff[x] + fill[x]++] = (int32_t)li;
            }
        }
        pl.n_xbox = (int64_t)xbox.size();
        pl.n_xl = (int64_t)xl.size();
        pl.h_xbox = xbox;
        pl.h_xoff = xoff;
        pl.h_xl = xl;
        pl.n_wleaves = (int64_t)wleaves.size();
        up(pl.xbox, xbox);
        up(pl.xoff, xoff);
        up(pl.xl, xl);
        up(pl.wleaves, wleaves);
    }
    // ---- leaf ranges by box (P2M launches per level), leaves per level ----
    {
        std::vector<int32_t> alr((size_t)nb * 6, 0);
        for (int64_t li = 0; li < pl.nleaf; ++li)
            for (int j = 0; j < 6; ++j) alr[(size_t)pl.h_leaf_box[li] * 6 + j] = pl.h_lrange[(size_t)li * 6 + j];
        up(pl.alr, alr);
        std::vector<int32_t> pls;
        pl.p2m_off.assign(L + 2, 0);
        for (int l = 0; l <= L; ++l) {
            pl.p2m_off[l] = (int64_t)pls.size();
            if (l < lmin) continue;
            for (int64_t b = pl.lev[l].begin; b < pl.lev[l].end; ++b)
                if (pl.h_box_leaf[b] >= 0) pls.push_back((int32_t)(b - pl.lev[l].begin));
        }
        pl.p2m_off[L + 1] = (int64_t)pls.size();
        up(pl.p2m_list, pls);
    }
    // near field: t = r^2 / (4 alpha^2) of a U-list pair is at most 2 s^2 / alpha^2
    // for the side s of the coarser leaf
    {
        int lc = L;
        for (int32_t v : llev) lc = std::min(lc, v);
        pl.near_tmax = 2.0 * pl.lev[lc].side * pl.lev[lc].side / (pl.alpha * pl.alpha);
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

// children, M2M tiles (over the split boxes), the slot -> offset table, and
// the uploads common to both tree forms
void finish_tree(Context &ctx, FmmPlan &pl, const std::vector<double> &cx, const std::vector<double> &cy,
                 const uint32_t *dkeys) {
    const int64_t N = pl.N, nb = pl.nbox;
    const int L = pl.L, lmin = pl.lmin;
    auto up = [&](auto &buf, const auto &vec) {
        using T = typename std::decay_t<decltype(vec)>::value_type;
        T *d = buf.ensure(std::max<size_t>(vec.size(), 1));
        if (!vec.empty())
            YK_HIP(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    };
    // ---- children (contiguous at the next level because codes are sorted) ----
    std::vector<int32_t> fch(nb, -1), nch(nb, 0);
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t pa = pl.hparent[b];
        if (pa < 0) continue;
        if (fch[pa] < 0) fch[pa] = (int32_t)b;
        nch[pa]++;
    }
    // ---- children by position, and M2M tiles (64 parents of one level) ----
    std::vector<int32_t> ch4((size_t)nb * 4, -1);
    for (int64_t b = 0; b < nb; ++b)
        if (pl.hparent[b] >= 0) ch4[(size_t)pl.hparent[b] * 4 + (pl.hcode[b] & 3u)] = (int32_t)b;
    std::vector<int4> utiles;
    std::vector<int32_t> uboxes;
    pl.up_tile_begin.assign(L + 1, 0);
    pl.up_tile_count.assign(L + 1, 0);
    pl.up_off.assign(L + 1, 0);
    pl.up_n.assign(L + 1, 0);
    for (int l = lmin; l < L; ++l) {
        // the boxes with children (all of them in the uniform tree)
        std::vector<int32_t> par;
        for (int64_t b = pl.lev[l].begin; b < pl.lev[l].end; ++b)
            if (nch[b] > 0) par.push_back((int32_t)b);
        pl.up_tile_begin[l] = (int)utiles.size();
        pl.up_off[l] = (int64_t)uboxes.size();
        pl.up_n[l] = (int64_t)par.size();
        for (size_t k0 = 0; k0 < par.size(); k0 += 64) {
            const int cnt = (int)std::min<size_t>(64, par.size() - k0);
            utiles.push_back(make_int4(l, 0, (int)uboxes.size(), cnt));
            for (int k = 0; k < cnt; ++k) uboxes.push_back(par[k0 + k]);
        }
        pl.up_tile_count[l] = (int)utiles.size() - pl.up_tile_begin[l];
    }
    const std::vector<int32_t> iota4 = {0, 1, 2, 3};
    // ---- slot -> offset id for the 4 parity classes ----
    std::vector<int32_t> soid(4 * kNumV);
    for (int cls = 0; cls < 4; ++cls) {
        const int cxs = cls & 1, cys = cls >> 1;
        int slot = 0;
        for (int dy = -2 - cys; dy <= 3 - cys; ++dy)
            for (int dx = -2 - cxs; dx <= 3 - cxs; ++dx) {
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                int oid = 0, found = -1;
                for (int ey = -3; ey <= 3; ++ey)
                    for (int ex = -3; ex <= 3; ++ex) {
                        if (std::abs(ex) <= 1 && std::abs(ey) <= 1) continue;
                        if (ex == dx && ey == dy) found = oid;
                        ++oid;
                    }
                soid[cls * kNumV + slot] = found;
                ++slot;
            }
    }
    // ---- upload tree ----
    up(pl.bcx, cx);
    up(pl.bcy, cy);
    up(pl.bparent, pl.hparent);
    up(pl.fchild, fch);
    up(pl.nchild, nch);
    up(pl.slot_oid, soid);
    up(pl.child4, ch4);
    up(pl.iota4, iota4);
    {
        std::vector<int32_t> iota40(kNumOff);
        for (int k = 0; k < kNumOff; ++k) iota40[k] = k;
        up(pl.iota40, iota40);
    }
    pl.h_soid = soid;
    if (!utiles.empty()) {
        up(pl.up_tiles, utiles);
        up(pl.up_boxes, uboxes);
    }
    if (!pl.adaptive) {
        std::vector<int32_t> dl;
        for (int64_t li = 0; li < pl.nleaf; ++li)
            if (pl.h_lrange[(size_t)li * 6 + 3] > pl.h_lrange[(size_t)li * 6 + 2]) dl.push_back((int32_t)li);
        pl.n_dleaves = (int64_t)dl.size();
        if (!dl.empty()) up(pl.dleaves, dl);
    }
    // the sorted keys (kept for introspection)
    YK_HIP(hipMemcpyAsync(pl.skeys.ensure(N), dkeys, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void build_tables(Context &ctx, FmmPlan &pl, int p) {
    const auto t_start = std::chrono::steady_clock::now();
    const int L = pl.L, lmin = pl.lmin;
    const int64_t nb = pl.nbox;
    auto up = [&](auto &buf, const auto &vec) {
        using T = typename std::decay_t<decltype(vec)>::value_type;
        T *d = buf.ensure(vec.size());
        YK_HIP(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    };
    // (state that depends on the order: cached P2M rows, kept multipoles)
    pl.p2m_rows_built = false;
    pl.p2m_rq.release();
    pl.p2m_rd.release();
    pl.mq_kept = false;
    pl.p = p;
    pl.P = 2 * p + 1;
    pl.Pp = (pl.P + 15) / 16 * 16;
    const int Pp = pl.Pp, nL = L + 1;
    const double alpha = pl.alpha;
    // per-level scale data
    std::vector<double> invFY((size_t)nL * (p + 2)), da((size_t)nL * (p + 2)), db((size_t)nL * (p + 2));
    std::vector<std::vector<ld>> IR(nL);
    for (int l = std::min(lmin, L); l <= L; ++l) {
        const ld R = pl.lev[l].R;
        IR[l] = I_seq(R, 2 * p + 4);
        for (int n = 0; n <= p + 1; ++n) {
            invFY[(size_t)l * (p + 2) + n] = (double)(1.0L / F_series(n, 0.25L * R * R));
            da[(size_t)l * (p + 2) + n] = (double)(IR[l][n + 1] / IR[l][n]);
            db[(size_t)l * (p + 2) + n] = (double)((n == 0 ? IR[l][1] : IR[l][n - 1]) / IR[l][n]);
        }
    }
    std::vector<double> cnn(p + 4);
    for (int n = 0; n < p + 4; ++n) cnn[n] = 1.0 / ((double)(n + 1) * (double)(n + 2));
    up(pl.invFY, invFY);
    up(pl.dipa, da);
    up(pl.dipb, db);
    up(pl.cnn, cnn);
    // series length for F_{p+1}, F_{p+2} at level l (leaf level of a uniform
    // tree; every level from lmin on in an adaptive one)
    auto series_len = [&](int l) {
        const ld Y = 0.25L * pl.lev[l].R * pl.lev[l].R * 1.0001L;
        ld t = 1;
        int k = 1;
        for (; k < 200; ++k) {
            t *= Y / ((ld)k * (ld)(p + 1 + k));
            if (t < 1e-19L) break;
        }
        return k + 1;
    };
    auto series_coef = [&](int ns, double *sc) {
        for (int w = 0; w < 2; ++w) {
            const int n = p + 1 + w;
            ld c = 1;
            for (int kk = 0; kk < ns; ++kk) {
                if (kk > 0) c /= (ld)kk * (ld)(n + kk);
                sc[w * ns + kk] = (double)c;
            }
        }
    };
    {
        pl.nser = series_len(L);
        std::vector<double> sc(2 * pl.nser);
        series_coef(pl.nser, sc.data());
        up(pl.serc, sc);
    }
    if (pl.adaptive && lmin <= L) {
        pl.nser_lv.assign(nL, 0);
        pl.nser_stride = 0;
        for (int l = lmin; l <= L; ++l) {
            pl.nser_lv[l] = series_len(l);
            pl.nser_stride = std::max(pl.nser_stride, pl.nser_lv[l]);
        }
        std::vector<double> sc((size_t)nL * 2 * pl.nser_stride, 0.0), invR(nL, 0.0);
        std::vector<double> ri((size_t)nL * (p + 3), 0.0);
        for (int l = lmin; l <= L; ++l) {
            series_coef(pl.nser_lv[l], &sc[(size_t)l * 2 * pl.nser_stride]);
            invR[l] = 1.0 / pl.lev[l].R;
            // I_0(R_l), then the ratios I_n(R_l) / I_{n-1}(R_l): the products
            // I_n(R) K_n(rho) of M2P and P2L are built from them and from the
            // ratios of K, which keeps every factor in range
            ri[(size_t)l * (p + 3)] = (double)IR[l][0];
            for (int n = 1; n <= p + 2; ++n) ri[(size_t)l * (p + 3) + n] = (double)(IR[l][n] / IR[l][n - 1]);
        }
        up(pl.serc_lv, sc);
        up(pl.invR_lv, invR);
        up(pl.rI, ri);
        up(pl.nser_dev, pl.nser_lv);
    }
    // near-field series length: t = r^2/(4 alpha^2) over U-list pairs is at most
    // (2 sqrt(2) side_L)^2 / (4 alpha^2); when it exceeds 1 the large-argument
    // branch is used too.  The series are cut at the first power whose term,
    // weighted by the largest factor it meets ((1/2)|ln t| for A, about 3 for
    // the digamma weights of B and D), is below half an ulp of the smallest
    // K0 on the range (K0(z) > -(1/2) ln t - 0.58, and K0(2) > 0.11).
    pl.near_terms = near_series_terms(pl.near_tmax);

    const int nC = 2 * p + 1;
    std::vector<cld> C((size_t)(p + 1) * nC);
    // M2M and L2L for parent levels lmin..L-1 (also below lmin: unused)
    std::vector<double> m2m((size_t)nL * 4 * Pp * Pp, 0.0), l2l((size_t)nL * 4 * Pp * Pp, 0.0);
    for (int l = std::max(lmin, 0); l < L; ++l) {
        const ld Rp = pl.lev[l].R, Rc = pl.lev[l + 1].R;
        const auto &Ip = IR[l], &Ic = IR[l + 1];
        for (int c = 0; c < 4; ++c) {
            const int bx = c & 1, by = (c >> 1) & 1;
            const ld ex = (bx - 0.5L) * pl.lev[l + 1].side / alpha;
            const ld ey = (by - 0.5L) * pl.lev[l + 1].side / alpha;
            const ld re = std::sqrt(ex * ex + ey * ey), phi = std::atan2(ey, ex);
            const std::vector<ld> Ie = I_seq(re, 2 * p + 2);
            // M2M: S[k][n] = I_|n|(Rc) F^I_{n-k}(e) / I_k(Rp)
            for (int k = 0; k <= p; ++k)
                for (int n = -p; n <= p; ++n)
                    C[(size_t)k * nC + n + p] = Ic[std::abs(n)] * Ie[std::abs(n - k)] * cis(phi, n - k) / Ip[k];
            to_real(C, p, Pp, &m2m[((size_t)l * 4 + c) * Pp * Pp]);
            // L2L: E[k][m] = F^I_{m-k}(e) I_k(Rc) / I_|m|(Rp)
            for (int k = 0; k <= p; ++k)
                for (int m = -p; m <= p; ++m)
                    C[(size_t)k * nC + m + p] = Ie[std::abs(m - k)] * cis(phi, m - k) * Ic[k] / Ip[std::abs(m)];
            to_real(C, p, Pp, &l2l[((size_t)l * 4 + c) * Pp * Pp]);
        }
    }
    // M2L for levels lmin..L, 40 offsets (dy outer, dx inner over [-3,3]^2
    // minus [-1,1]^2); the (level, offset) operators are independent and are
    // computed on several host threads
    std::vector<double> m2l((size_t)nL * kNumOff * Pp * Pp, 0.0);
    {
        std::vector<std::array<int, 4>> tasks;   // level, dx, dy, offset id
        for (int l = lmin; l <= L; ++l) {
            int oid = 0;
            for (int dy = -3; dy <= 3; ++dy)
                for (int dx = -3; dx <= 3; ++dx) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                    tasks.push_back({l, dx, dy, oid++});
                }
        }
        auto work = [&](size_t t0, size_t t1) {
            std::vector<cld> Ct((size_t)(p + 1) * nC);
            for (size_t t = t0; t < t1; ++t) {
                const int l = tasks[t][0], dx = tasks[t][1], dy = tasks[t][2], oid = tasks[t][3];
                const auto &I = IR[l];
                // d = (c_t - c_s)/alpha with the source at offset (dx, dy)
                const double ddx = -dx * pl.lev[l].side / alpha, ddy = -dy * pl.lev[l].side / alpha;
                const double dd = std::sqrt(ddx * ddx + ddy * ddy);
                const ld phi = std::atan2((ld)ddy, (ld)ddx);
                const std::vector<ld> K = K_seq(dd, 2 * p + 1);
                for (int m = 0; m <= p; ++m)
                    for (int n = -p; n <= p; ++n) {
                        const ld sgn = (m & 1) ? -1.0L : 1.0L;
                        Ct[(size_t)m * nC + n + p] = sgn * I[m] * I[std::abs(n)] * K[std::abs(n - m)] * cis(phi, n - m);
                    }
                to_real(Ct, p, Pp, &m2l[((size_t)l * kNumOff + oid) * Pp * Pp]);
            }
        };
        const size_t nt = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
        const size_t per = (tasks.size() + nt - 1) / nt;
        std::vector<std::thread> pool;
        for (size_t i = 0; i < nt && i * per < tasks.size(); ++i)
            pool.emplace_back(work, i * per, std::min(tasks.size(), (i + 1) * per));
        for (auto &th : pool) th.join();
    }
    up(pl.m2m, m2m);
    up(pl.l2l, l2l);
    up(pl.m2l, m2l);
    {
        std::vector<float> f(m2l.begin(), m2l.end());
        up(pl.m2lf, f);
        std::vector<float> g(l2l.begin(), l2l.end());
        up(pl.l2lf, g);
    }
    pl.M.ensure((size_t)nb * Pp);
    pl.Lc.ensure((size_t)nb * Pp);
    YK_HIP(hipStreamSynchronize(ctx.stream));
    pl.tables_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
}

FmmPlan *plan_in_slot(Context &ctx, int slot) {
    switch (slot) {
        case 0: return ctx.plan_vol.get();
        case 1: return ctx.plan_bnd.get();
        case 2: return ctx.plan_misc.get();
        case 3: return ctx.plan_near.get();
        case 4: return ctx.plan_nearc.get();
        default: return nullptr;
    }
}

void ensure_near_layout(Context &ctx, FmmPlan &pl, ActiveSet &as_ref) {
    if (as_ref.layout) return;
    ActiveSet *as = &as_ref;
    const int L = pl.L, mask = as->mask;
    const std::vector<int32_t> &uoff = as->h_uoff, &ul = as->h_ul;
    const std::vector<int64_t> &sq_leaf = as->h_sq, &sd_leaf = as->h_sd;
    const std::vector<int2> &items = as->h_items;
    auto tcnt = [&](int64_t li) { return as->h_tcnt[li]; };
    {
        // symmetric charge values
        const int64_t n0 = pl.toff[1] - pl.toff[0];
        // charges among the targets, at most 64 per leaf (so that they all
        // fall in the leaf's first item, which they lead), and a far field
        // (k_l2p adds the incoming slots)
        auto n0_of = [&](int64_t li) -> int64_t { return pl.h_lrange[(size_t)li * 6 + 1] - pl.h_lrange[(size_t)li * 6]; };
        bool sym = (mask & 1) && n0 > 0 && pl.lmin <= L && !(ctx.opt.debug_flags & 16);
        for (int64_t li = 0; li < pl.nleaf && sym; ++li)
            if (n0_of(li) > 64) sym = false;
        if (sym) {
            // incoming slots of leaf B: one per U-list neighbour A < B with
            // charges, in B's U-list order, each n0(B) entries; the writer is
            // A's U-list entry that names B
            std::vector<int64_t> dst(ul.size(), -1), ibase(pl.nleaf, 0);
            std::vector<int32_t> icnt(pl.nleaf, 0);
            // (three passes: slots per leaf, their offsets, then each writer's
            // destination; every entry of dst has exactly one writer)
            parallel_for(pl.nleaf, [&](int64_t b0, int64_t b1) {
                for (int64_t b = b0; b < b1; ++b) {
                    int k = 0;
                    for (int32_t u = uoff[b]; u < uoff[b + 1]; ++u)
                        if (ul[u] < b && n0_of(ul[u]) > 0) ++k;
                    icnt[b] = k;
                }
            });
            int64_t off = 0;
            for (int64_t b = 0; b < pl.nleaf; ++b) {
                ibase[b] = off;
                off += (int64_t)icnt[b] * n0_of(b);
            }
            std::atomic<bool> asym{false};
            parallel_for(pl.nleaf, [&](int64_t b0, int64_t b1) {
                for (int64_t b = b0; b < b1; ++b) {
                    int k = 0;
                    for (int32_t u = uoff[b]; u < uoff[b + 1]; ++u) {
                        const int32_t a = ul[u];
                        if (a >= b || n0_of(a) == 0) continue;
                        int32_t ua = uoff[a];
                        while (ua < uoff[a + 1] && ul[ua] != b) ++ua;
                        if (ua == uoff[a + 1]) {
                            asym = true;
                            return;
                        }
                        dst[ua] = ibase[b] + (int64_t)k * n0_of(b);
                        ++k;
                    }
                }
            });
            if (asym) throw Error{YK_ERR_INTERNAL, "U-lists are not symmetric"};
            as->inc_len = off;
            int64_t *db = as->inc_base.ensure(ibase.size());
            int32_t *dc = as->inc_cnt.ensure(icnt.size());
            YK_HIP(hipMemcpyAsync(db, ibase.data(), ibase.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
            YK_HIP(hipMemcpyAsync(dc, icnt.data(), icnt.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
            as->inc.ensure(std::max<int64_t>(off, 1));
            // per-item descriptors (layout: kItemDesc in the near-field kernels)
            constexpr int kDesc = 52;
            const int q_on = 1, d_on = (pl.toff[2] > pl.toff[1]) ? 1 : 0;
            std::vector<int32_t> desc(items.size() * kDesc, 0);
            std::vector<int64_t> ddst(items.size() * 9, -1);
            parallel_for((int64_t)items.size(), [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const int32_t li = items[i].x;
                int32_t *d = desc.data() + i * kDesc;
                const int32_t u0 = uoff[li], nu = uoff[li + 1] - u0;
                for (int u = 0; u < 9 && u < nu; ++u) {
                    const int32_t b = ul[u0 + u];
                    const int32_t *r = pl.h_lrange.data() + (size_t)b * 6;
                    d[u] = r[0];
                    d[9 + u] = q_on ? r[1] - r[0] : 0;
                    d[18 + u] = (q_on && b >= li) ? r[1] - r[0] : 0;
                    d[27 + u] = r[2];
                    d[36 + u] = d_on ? r[3] - r[2] : 0;
                    ddst[i * 9 + u] = dst[u0 + u];
                }
                const int32_t *r = pl.h_lrange.data() + (size_t)li * 6;
                for (int st = 0; st < 3; ++st) {
                    d[45 + st] = r[2 * st];
                    d[48 + st] = (mask >> st) & 1 ? r[2 * st + 1] : r[2 * st];
                }
                d[51] = items[i].y;
            }
            });
            int32_t *dde = as->sym_desc.ensure(desc.size());
            int64_t *ddd = as->sym_desc_dst.ensure(ddst.size());
            YK_HIP(hipMemcpyAsync(dde, desc.data(), desc.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
            YK_HIP(hipMemcpyAsync(ddd, ddst.data(), ddst.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
            YK_HIP(hipStreamSynchronize(ctx.stream));
            as->near_sym = true;
        }
        // entry offsets of the cached near field, item by item
        std::vector<int64_t> qoff(items.size()), doff(items.size());
        // per item: its charge entries (stored, and without padding) and
        // dipole pairs; then their offsets in order
        std::vector<int64_t> qlen(items.size()), qval(items.size()), dlen(items.size());
        parallel_for((int64_t)items.size(), [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const int li = items[i].x;
                const int64_t c = std::min<int64_t>(64, tcnt(li) - items[i].y);
                if (sym) {
                    // the leaf's charges against the owned neighbours' charges,
                    // its other targets against all neighbouring charges
                    int64_t own = 0;
                    for (int32_t u = uoff[li]; u < uoff[li + 1]; ++u)
                        if (ul[u] >= li) own += n0_of(ul[u]);
                    const int64_t na = items[i].y == 0 ? n0_of(li) : 0;
                    qlen[i] = ((na + 3) & ~(int64_t)3) * own + (c - na) * sq_leaf[li];
                    qval[i] = na * own + (c - na) * sq_leaf[li];
                } else {
                    qlen[i] = qval[i] = c * sq_leaf[li];
                }
                dlen[i] = c * sd_leaf[li];
            }
        });
        int64_t oq = 0, od = 0, vq = 0;   // (vq: charge values without the padding)
        for (size_t i = 0; i < items.size(); ++i) {
            if (sym) oq = (oq + 3) & ~(int64_t)3;   // (vector reads of four values)
            qoff[i] = oq;
            doff[i] = od;
            oq += qlen[i];
            vq += qval[i];
            od += dlen[i];
        }
        as->near_q_len = oq;
        as->near_q_vals = vq;
        as->near_d_len = od;
        if (!items.empty()) {
            int64_t *dq = as->item_qoff.ensure(items.size());
            int64_t *dd = as->item_doff.ensure(items.size());
            YK_HIP(hipMemcpyAsync(dq, qoff.data(), qoff.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
            YK_HIP(hipMemcpyAsync(dd, doff.data(), doff.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
            YK_HIP(hipStreamSynchronize(ctx.stream));
        }
    }
    as->layout = true;
}

ActiveSet &get_active(Context &ctx, FmmPlan &pl, int mask) {
    auto it = pl.active.find(mask);
    if (it != pl.active.end()) return *it->second;
    auto as = std::make_unique<ActiveSet>();
    const int L = pl.L;
    // the box of leaf li (uniform tree: the li-th box of the leaf level)
    auto leaf_gbox = [&](int64_t li) -> int64_t {
        return pl.adaptive ? (int64_t)pl.h_leaf_box[li] : pl.lev[L].begin + li;
    };
    std::vector<int64_t> cnt(pl.nbox, 0);
    for (int64_t li = 0; li < pl.nleaf; ++li) {
        int64_t c = 0;
        for (int s = 0; s < 3; ++s)
            if (mask & (1 << s)) c += pl.h_lrange[li * 6 + 2 * s + 1] - pl.h_lrange[li * 6 + 2 * s];
        cnt[leaf_gbox(li)] = c;
    }
    for (int64_t b = pl.nbox - 1; b >= 0; --b)
        if (pl.hparent[b] >= 0) cnt[pl.hparent[b]] += cnt[b];
    std::vector<int32_t> leaves;
    std::vector<int2> items;
    for (int64_t li = 0; li < pl.nleaf; ++li) {
        const int64_t c = cnt[leaf_gbox(li)];
        if (c > 0) leaves.push_back((int32_t)li);
        for (int64_t tb = 0; tb < c; tb += 64) items.push_back(make_int2((int)li, (int)tb));
    }
    // near-field pair counts over the U-lists of the active leaves
    {
        std::vector<int32_t> uoff(pl.nleaf + 1), ul;
        // recompute the U-lists from the uploaded copies
        YK_HIP(hipMemcpyAsync(uoff.data(), pl.ulist_off.p, uoff.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        ul.resize(uoff[pl.nleaf]);
        YK_HIP(hipMemcpyAsync(ul.data(), pl.ulist.p, ul.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        std::vector<int64_t> sq_leaf(pl.nleaf, 0), sd_leaf(pl.nleaf, 0);
        parallel_for(pl.nleaf, [&](int64_t i0, int64_t i1) {
            for (int64_t li = i0; li < i1; ++li) {
                int64_t sq = 0, sd = 0;
                for (int32_t u = uoff[li]; u < uoff[li + 1]; ++u) {
                    sq += pl.h_lrange[(size_t)ul[u] * 6 + 1] - pl.h_lrange[(size_t)ul[u] * 6];
                    sd += pl.h_lrange[(size_t)ul[u] * 6 + 3] - pl.h_lrange[(size_t)ul[u] * 6 + 2];
                }
                sq_leaf[li] = sq;
                sd_leaf[li] = sd;
            }
        });
        for (int32_t li : leaves) {
            const int64_t nt = cnt[leaf_gbox(li)];
            as->pairs_q += nt * sq_leaf[li];
            as->pairs_d += nt * sd_leaf[li];
            as->l2p_points += nt;
        }
        as->h_sq = std::move(sq_leaf);
        as->h_sd = std::move(sd_leaf);
        as->h_uoff = std::move(uoff);
        as->h_ul = std::move(ul);
    }
    // adaptive tree: the items grouped (stably) by their leaf's level and by
    // whether a coarser leaf touches it, class 2 l + coarser, so that each
    // class's near field runs with the series its pair distances need
    as->item_lev_begin.assign(2 * (L + 1) + 1, 0);
    if (pl.adaptive) {
        std::vector<std::vector<int2>> by(2 * (L + 1));
        for (const int2 &it : items) {
            const int l = pl.h_blevel[pl.h_leaf_box[it.x]];
            int coarser = 0;
            for (int32_t u = as->h_uoff[it.x]; u < as->h_uoff[it.x + 1]; ++u)
                if (pl.h_blevel[pl.h_leaf_box[as->h_ul[u]]] < l) coarser = 1;
            by[2 * l + coarser].push_back(it);
        }
        items.clear();
        for (int k = 0; k < 2 * (L + 1); ++k) {
            as->item_lev_begin[k] = (int64_t)items.size();
            items.insert(items.end(), by[k].begin(), by[k].end());
        }
        as->item_lev_begin[2 * (L + 1)] = (int64_t)items.size();
    }
    as->h_items = items;
    as->h_tcnt.assign(pl.nleaf, 0);
    for (int64_t li = 0; li < pl.nleaf; ++li) as->h_tcnt[li] = cnt[leaf_gbox(li)];
    as->mask = mask;
    // M2L tiles: active boxes of levels lmin..L grouped by (level, class).
    // The V lists come to the host only for small trees (the sparse form's
    // buckets); a large tree's translations are counted on the GPU.
    constexpr int kTile = 64;
    const bool small_tree = pl.nleaf < 8192;
    std::vector<int32_t> vl_host;
    if (pl.lmin <= L && small_tree) {
        vl_host.resize((size_t)pl.nbox * kNumV);
        YK_HIP(hipMemcpyAsync(vl_host.data(), pl.vlist.p, vl_host.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
    }
    // Within a level the tiles of the four classes are interleaved: the k-th
    // tiles of the classes hold the children at the four positions of (about)
    // the same parents, so their V lists draw on the same source boxes, and
    // consecutive tiles run on one XCD at about the same time (the launch
    // maps consecutive tiles to one XCD), where the sources stay in its L2.
    std::vector<int32_t> mb;
    std::vector<int4> tiles, wtiles;
    for (int l = pl.lmin; l <= L; ++l) {
        std::vector<int4> ct[4], cw[4];
        for (int cls = 0; cls < 4; ++cls) {
            const int64_t start = (int64_t)mb.size();
            for (int64_t b = pl.lev[l].begin; b < pl.lev[l].end; ++b) {
                if (cnt[b] == 0) continue;
                uint32_t ix, iy;
                decode(pl.hcode[b], ix, iy);
                if ((int)((ix & 1) | ((iy & 1) << 1)) == cls) {
                    mb.push_back((int32_t)b);
                    if (small_tree)
                        for (int k = 0; k < kNumV; ++k) as->m2l_trans += vl_host[(size_t)b * kNumV + k] >= 0;
                }
            }
            for (int64_t s = start; s < (int64_t)mb.size(); s += kTile)
                ct[cls].push_back(make_int4(l, cls, (int)s, (int)std::min<int64_t>(kTile, (int64_t)mb.size() - s)));
            for (int64_t s = start; s < (int64_t)mb.size(); s += 2 * kTile)
                cw[cls].push_back(make_int4(l, cls, (int)s, (int)std::min<int64_t>(2 * kTile, (int64_t)mb.size() - s)));
        }
        for (size_t k = 0;; ++k) {
            bool any = false;
            for (int cls = 0; cls < 4; ++cls)
                if (k < ct[cls].size()) {
                    tiles.push_back(ct[cls][k]);
                    any = true;
                }
            if (!any) break;
        }
        for (size_t k = 0;; ++k) {
            bool any = false;
            for (int cls = 0; cls < 4; ++cls)
                if (k < cw[cls].size()) {
                    wtiles.push_back(cw[cls][k]);
                    any = true;
                }
            if (!any) break;
        }
    }
    // sparse M2L when fewer than half of the V-list slots of the active boxes
    // hold a source (on a small tree, where the dense tiles' empty slots cost
    // whole operator loads)
    std::vector<int4> ptiles;
    std::vector<int32_t> ptgt, psrc;
    if (small_tree && !mb.empty() && 2 * as->m2l_trans < (int64_t)mb.size() * kNumV) {
        as->m2l_sparse = true;
        for (int l = pl.lmin; l <= L; ++l) {
            std::vector<std::vector<std::pair<int32_t, int32_t>>> bucket(kNumOff);
            for (int32_t b : mb) {
                if (b < pl.lev[l].begin || b >= pl.lev[l].end) continue;
                uint32_t ix, iy;
                decode(pl.hcode[b], ix, iy);
                const int cls = (int)((ix & 1) | ((iy & 1) << 1));
                for (int k = 0; k < kNumV; ++k) {
                    const int32_t src = vl_host[(size_t)b * kNumV + k];
                    if (src >= 0) bucket[pl.h_soid[cls * kNumV + k]].push_back({b, src});
                }
            }
            for (int oid = 0; oid < kNumOff; ++oid) {
                const auto &v = bucket[oid];
                for (size_t s0 = 0; s0 < v.size(); s0 += kTile) {
                    const int cnt = (int)std::min<size_t>(kTile, v.size() - s0);
                    ptiles.push_back(make_int4(l, oid, (int)ptgt.size(), cnt));
                    for (int k = 0; k < cnt; ++k) {
                        ptgt.push_back(v[s0 + k].first);
                        psrc.push_back(v[s0 + k].second);
                    }
                }
            }
        }
    }
    as->tile_begin.assign(L + 1, 0);
    as->tile_count.assign(L + 1, 0);
    for (size_t t = 0; t < tiles.size(); ++t) {
        const int l = tiles[t].x;
        if (as->tile_count[l] == 0) as->tile_begin[l] = (int)t;
        as->tile_count[l]++;
    }
    std::vector<int32_t> l2lb;
    as->l2l_begin.assign(L + 1, 0);
    as->l2l_count.assign(L + 1, 0);
    for (int l = pl.lmin + 1; l <= L; ++l) {
        as->l2l_begin[l] = (int64_t)l2lb.size();
        for (int64_t b = pl.lev[l].begin; b < pl.lev[l].end; ++b)
            if (cnt[b] > 0) l2lb.push_back((int32_t)b);
        as->l2l_count[l] = (int64_t)l2lb.size() - as->l2l_begin[l];
    }
    auto up = [&](auto &buf, const auto &vec) {
        using T = typename std::decay_t<decltype(vec)>::value_type;
        T *d = buf.ensure(vec.size());
        if (!vec.empty())
            YK_HIP(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    };
    up(as->m2l_boxes, mb);
    if (!small_tree && !mb.empty()) as->m2l_trans = gpu_count_slots(ctx, pl, as->m2l_boxes.p, (int64_t)mb.size());
    up(as->m2l_tiles, tiles);
    up(as->m2l_tiles_w, wtiles);
    if (as->m2l_sparse) {
        std::vector<int32_t> piota(ptgt.size());
        for (size_t k = 0; k < piota.size(); ++k) piota[k] = (int32_t)k;
        up(as->m2l_ptiles, ptiles);
        up(as->m2l_ptgt, ptgt);
        up(as->m2l_psrc, psrc);
        up(as->m2l_piota, piota);
        as->n_ptiles = (int)ptiles.size();
        // the translations of each target box, in increasing index (the
        // fixed order of their sum)
        std::vector<int32_t> order(ptgt.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ptgt[a] < ptgt[b]; });
        std::vector<int32_t> ctgt, coff;
        for (size_t k = 0; k < order.size(); ++k) {
            if (k == 0 || ptgt[order[k]] != ptgt[order[k - 1]]) {
                ctgt.push_back(ptgt[order[k]]);
                coff.push_back((int32_t)k);
            }
        }
        coff.push_back((int32_t)order.size());
        up(as->csr_tgt, ctgt);
        up(as->csr_off, coff);
        up(as->csr_rows, order);
        as->n_csr_tgt = (int64_t)ctgt.size();
        as->n_ptrans = (int64_t)ptgt.size();
    }
    up(as->l2l_boxes, l2lb);
    up(as->leaves, leaves);
    up(as->leaf_items, items);
    as->n_items = (int64_t)items.size();
    as->n_tiles = (int)tiles.size();
    as->n_tiles_w = (int)wtiles.size();
    as->n_leaves = (int64_t)leaves.size();
    as->n_m2l_boxes = (int64_t)mb.size();
    YK_HIP(hipStreamSynchronize(ctx.stream));
    auto &ref = *as;
    pl.active[mask] = std::move(as);
    return ref;
}

}  // namespace yk
