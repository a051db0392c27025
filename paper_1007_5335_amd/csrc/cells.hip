// cells.hip -- U^p at the boundary nodes when the volume points are the
// centres of square cells (yk_heat_step flags bit0).
//
// V[q] at a node is a point sum over the cells; a cell whose centre lies
// close to the node (closer than a few of its sides) is badly represented by
// its point value (the kernel's logarithmic singularity: the error grows
// like log(h / d)), and for cells larger than alpha the point value misses
// the kernel's mass altogether.  Such cells (centre within two sides of the
// node) enter instead with the integral of the kernel over their square:
//   V(node) += B_j [ (1/2pi) int_cell_j K0(|y - x|/alpha) dA - w_j K0(d_j/alpha)/(2pi) ]
// (the point term only when d_j > 0, as the sums skip coincident pairs).
// The square is the signed sum of the four triangles with apex x and one
// edge each; over a triangle the radial integral is
// F(R) = alpha^2 - alpha R K1(R/alpha), and along the edge, at the foot
// distance q, R = q cosh s and dtheta = ds / cosh s: Gauss-Legendre in s on
// unit panels.  The (node, cell) pairs depend on the geometry only and are
// found once per (points, weights, boundary), on the host, by sorting each
// cell size's centres into buckets of two sides.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <unordered_set>
#include <vector>

#include "yk_bessel.h"
#include "yk_internal.h"

namespace yk {

struct CellNodePlan {
    const double *xy = nullptr, *w = nullptr;
    int64_t n = 0;
    uint64_t bnd_gen = 0;
    int64_t n_pairs = 0;
    DevBuf<int64_t> node_off;   // [nb + 1]
    DevBuf<int32_t> cell;       // [n_pairs], grouped by node, cells ascending
    DevBuf<double> wt;          // [n_pairs]: cell integral - point value, for alpha_wt
    double alpha_wt = 0.0;
    double setup_ms = 0;
};

void CellNodePlanDeleter::operator()(CellNodePlan *p) const { delete p; }

namespace {

constexpr double kCellReach = 2.0;   // pairs: node within this many sides of the centre

__constant__ double c_cgl_x[32];
__constant__ double c_cgl_w[32];

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// 32-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_32)
void gauss_legendre_32(double *x, double *w) {
    const int n = 32;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            const double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// (1/2pi) int over the square of side h centred at (cx, cy) of K0(|y - p|/alpha) dA
__device__ double cell_k0_integral(double px, double py, double cx, double cy, double h, double alpha) {
    const double hx[4] = {-0.5, 0.5, 0.5, -0.5}, hy[4] = {-0.5, -0.5, 0.5, 0.5};
    double total = 0.0;
    for (int e = 0; e < 4; ++e) {
        const double ax = cx + hx[e] * h, ay = cy + hy[e] * h;
        const double ex = hx[(e + 1) & 3] - hx[e], ey = hy[(e + 1) & 3] - hy[e];   // unit edge direction
        const double q = (ax - px) * ey - (ay - py) * ex;                          // signed foot distance
        const double aq = fabs(q);
        if (!(aq > 1e-300)) continue;   // apex on the edge's line: the triangle is empty
        const double ta = (ax - px) * ex + (ay - py) * ey;
        const double sa = asinh(ta / aq), sb = asinh((ta + h) / aq);
        const int npan = max(1, (int)ceil(sb - sa));
        const double len = (sb - sa) / npan;
        double acc = 0.0;
        for (int pn = 0; pn < npan; ++pn) {
            const double mid = sa + (pn + 0.5) * len, half = 0.5 * len;
            for (int k = 0; k < 32; ++k) {
                const double s = mid + half * c_cgl_x[k];
                const double ch = cosh(s), R = aq * ch;
                const double F = alpha * alpha - alpha * R * k1(R / alpha);
                acc += half * c_cgl_w[k] * F / ch;
            }
        }
        total += (q > 0.0 ? 1.0 : -1.0) * acc;
    }
    return total * kInv2Pi;
}

// per (node, cell) pair: the cell integral minus the point value (geometry and alpha only)
__global__ void k_node_cell_weights(int64_t nb, const double *__restrict__ bxy, const int64_t *__restrict__ off,
                                    const int32_t *__restrict__ cell, const double *__restrict__ vxy,
                                    const double *__restrict__ vw, double alpha, double *__restrict__ wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const double px = bxy[2 * i], py = bxy[2 * i + 1];
    for (int64_t k = off[i]; k < off[i + 1]; ++k) {
        const int64_t j = cell[k];
        const double cx = vxy[2 * j], cy = vxy[2 * j + 1], w = vw[j];
        const double dx = px - cx, dy = py - cy, d = sqrt(dx * dx + dy * dy);
        const double point = d > 0.0 ? w * k0(d / alpha) * kInv2Pi : 0.0;
        wt[k] = cell_k0_integral(px, py, cx, cy, sqrt(w), alpha) - point;
    }
}

// vb[i] += sum over the node's cells of wt B_j (in a fixed order)
__global__ void k_node_cells(int64_t nb, const int64_t *__restrict__ off, const int32_t *__restrict__ cell,
                             const double *__restrict__ wt, const double *__restrict__ B, double *__restrict__ vb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double acc = 0.0;
    for (int64_t k = off[i]; k < off[i + 1]; ++k) acc += wt[k] * B[cell[k]];
    vb[i] += acc;
}

}  // namespace

CellNodePlan &cells_prepare(Context &ctx, BoundaryData &bd, int64_t n, const double *vol_xy, const double *vol_w) {
    CellNodePlan *cur = ctx.cell_nodes.get();
    if (cur && cur->xy == vol_xy && cur->w == vol_w && cur->n == n && cur->bnd_gen == bd.gen) return *cur;
    const auto t0 = std::chrono::steady_clock::now();
    ctx.cell_nodes.reset();
    CellNodePtr cp(new CellNodePlan());
    cp->xy = vol_xy;
    cp->w = vol_w;
    cp->n = n;
    cp->bnd_gen = bd.gen;
    const int64_t nb = bd.n;
    std::vector<double> hv(2 * n), hw(n), hb(2 * nb);
    YK_HIP(hipMemcpyAsync(hv.data(), vol_xy, 2 * n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipMemcpyAsync(hw.data(), vol_w, n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipMemcpyAsync(hb.data(), bd.xy, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    // cells grouped by size; per size, (bucket key, cell) sorted, buckets of kCellReach sides
    std::vector<double> sizes;
    {
        std::unordered_set<uint64_t> seen;
        for (int64_t j = 0; j < n; ++j) {
            uint64_t bits;
            std::memcpy(&bits, &hw[j], sizeof(bits));
            if (seen.insert(bits).second) {
                YK_REQUIRE(seen.size() <= 65535, "cell centres (flags bit0) need at most 65535 distinct cell areas");
                sizes.push_back(hw[j]);
            }
        }
        std::sort(sizes.begin(), sizes.end());
    }
    YK_REQUIRE(sizes.size() <= 65535, "cell centres (flags bit0) need at most 65535 distinct cell areas");
    double x0 = INFINITY, y0 = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
        x0 = std::min(x0, hv[2 * j]);
        y0 = std::min(y0, hv[2 * j + 1]);
    }
    for (int64_t i = 0; i < nb; ++i) {
        x0 = std::min(x0, hb[2 * i]);
        y0 = std::min(y0, hb[2 * i + 1]);
    }
    const int nl = (int)sizes.size();
    std::vector<double> bsz(nl);
    for (int l = 0; l < nl; ++l) bsz[l] = kCellReach * std::sqrt(sizes[l]);
    struct KC {
        uint64_t key;
        int32_t cell;
    };
    std::vector<std::vector<KC>> lev(nl);
    auto key_of = [&](double x, double y, double b) -> uint64_t {
        const uint64_t ix = (uint64_t)std::max(0.0, std::floor((x - x0) / b) + 1.0);
        const uint64_t iy = (uint64_t)std::max(0.0, std::floor((y - y0) / b) + 1.0);
        return (iy << 32) | (ix & 0xffffffffull);
    };
    for (int64_t j = 0; j < n; ++j) {
        const int l = (int)(std::lower_bound(sizes.begin(), sizes.end(), hw[j]) - sizes.begin());
        lev[l].push_back({key_of(hv[2 * j], hv[2 * j + 1], bsz[l]), (int32_t)j});
    }
    for (auto &v : lev)
        std::sort(v.begin(), v.end(), [](const KC &a, const KC &b) { return a.key != b.key ? a.key < b.key : a.cell < b.cell; });
    // per node (threads over node ranges): the cells within reach, ascending
    const int nthr = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::vector<int32_t>> part_cells(nthr);
    std::vector<std::vector<int64_t>> part_cnt(nthr);
    auto work = [&](int t) {
        const int64_t i0 = nb * t / nthr, i1 = nb * (t + 1) / nthr;
        std::vector<int32_t> &pc = part_cells[t];
        std::vector<int64_t> &cnt = part_cnt[t];
        std::vector<int32_t> mine;
        for (int64_t i = i0; i < i1; ++i) {
            const double px = hb[2 * i], py = hb[2 * i + 1];
            mine.clear();
            for (int l = 0; l < nl; ++l) {
                if (lev[l].empty()) continue;
                const double b = bsz[l], r2 = b * b;
                const int64_t ix = (int64_t)std::floor((px - x0) / b) + 1, iy = (int64_t)std::floor((py - y0) / b) + 1;
                for (int64_t dy = -1; dy <= 1; ++dy)
                    for (int64_t dx = -1; dx <= 1; ++dx) {
                        if (ix + dx < 0 || iy + dy < 0) continue;
                        const uint64_t key = ((uint64_t)(iy + dy) << 32) | ((uint64_t)(ix + dx) & 0xffffffffull);
                        auto it = std::lower_bound(lev[l].begin(), lev[l].end(), key,
                                                   [](const KC &a, uint64_t k) { return a.key < k; });
                        for (; it != lev[l].end() && it->key == key; ++it) {
                            const int64_t j = it->cell;
                            const double ddx = px - hv[2 * j], ddy = py - hv[2 * j + 1];
                            if (ddx * ddx + ddy * ddy < r2) mine.push_back(it->cell);
                        }
                    }
            }
            std::sort(mine.begin(), mine.end());
            pc.insert(pc.end(), mine.begin(), mine.end());
            cnt.push_back((int64_t)mine.size());
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthr; ++t) th.emplace_back(work, t);
    for (auto &x : th) x.join();
    std::vector<int64_t> off(nb + 1, 0);
    std::vector<int32_t> cells;
    int64_t i = 0;
    for (int t = 0; t < nthr; ++t) {
        for (int64_t c : part_cnt[t]) {
            off[i + 1] = off[i] + c;
            ++i;
        }
        cells.insert(cells.end(), part_cells[t].begin(), part_cells[t].end());
    }
    cp->n_pairs = (int64_t)cells.size();
    YK_HIP(hipMemcpyAsync(cp->node_off.ensure(nb + 1), off.data(), (nb + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, ctx.stream));
    if (!cells.empty())
        YK_HIP(hipMemcpyAsync(cp->cell.ensure(cells.size()), cells.data(), cells.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    cp->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ctx.cell_nodes = std::move(cp);
    return *ctx.cell_nodes;
}

void cells_correct_nodes(Context &ctx, CellNodePlan &cp, BoundaryData &bd, const double *vol_xy, const double *vol_w,
                         const double *B, double alpha, double *vb) {
    if (cp.n_pairs == 0) return;
    struct GL {
        double x[32], w[32];
        GL() { gauss_legendre_32(x, w); }
    };
    static const GL gl;   // initialised once, thread-safe
    if (cp.alpha_wt != alpha || !cp.wt.p) {
        YK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_cgl_x), gl.x, sizeof(gl.x), 0, hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_cgl_w), gl.w, sizeof(gl.w), 0, hipMemcpyHostToDevice, ctx.stream));
        hipLaunchKernelGGL(k_node_cell_weights, dim3(nblk(bd.n, 64)), dim3(64), 0, ctx.stream, bd.n, bd.xy,
                           cp.node_off.p, cp.cell.p, vol_xy, vol_w, alpha, cp.wt.ensure(cp.n_pairs));
        check_launch(ctx, "k_node_cell_weights");
        cp.alpha_wt = alpha;
    }
    hipLaunchKernelGGL(k_node_cells, dim3(nblk(bd.n, 256)), dim3(256), 0, ctx.stream, bd.n, cp.node_off.p, cp.cell.p,
                       cp.wt.p, B, vb);
    check_launch(ctx, "k_node_cells");
}

int64_t cells_pair_count(const CellNodePlan &cp) { return cp.n_pairs; }

}  // namespace yk
