// box.hip -- the box code of Sec. 3.1 (eq. volume_potential) on a uniform grid.
//
// The grid's cells are grouped into leaves of 4 x 4 cells.  On each leaf the
// density is the least-squares cubic through its 16 cell values, in the
// leaf's scaled coordinates (u, v) = (y - c) / (2h) (ten monomials 1, u, v,
// u^2, uv, v^2, u^3, u^2 v, u v^2, v^3), and the volume potential of that
// piecewise-cubic density is evaluated at every cell:
//   * near field (a leaf and its 3 x 3 neighbourhood): tables of the integrals
//     of K0(|x - y|/alpha)/(2 pi) times each monomial over a leaf, for the 16
//     cells of a leaf at each of the 9 offsets -- exact for the cubics up to
//     quadrature error (the cell holding the target by polar integration
//     about it, the logarithm taken out with the closed form
//     int_0^R K0(r/alpha) r dr = alpha^2 - alpha R K1(R/alpha));
//   * far field: the multipole expansion of each leaf's polynomial density,
//     M = Q^T c with Q the monomials' moments against conj(F^I_n), then the
//     FMM's M2M, M2L and L2L on a uniform tree whose leaf boxes are exactly
//     the grid's leaves, and the local expansions at the 16 cells by a table.
// U^p at points inside the grid (the boundary nodes) is the leaf polynomial
// fitted to the cell values of U^p (Sec. 3.1, the polynomials C^i_j).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <thread>
#include <vector>

#include "fmm.h"
#include "yk_bessel.h"

namespace yk {

namespace {

constexpr int kNB = 10;   // monomials of degree <= 3
constexpr int kNC = 16;   // cells of a leaf
constexpr int kNOff = 9;  // leaf offsets of the near field

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__host__ __device__ inline void monomials(double u, double v, double m[kNB]) {
    m[0] = 1.0;
    m[1] = u;
    m[2] = v;
    m[3] = u * u;
    m[4] = u * v;
    m[5] = v * v;
    m[6] = u * u * u;
    m[7] = u * u * v;
    m[8] = u * v * v;
    m[9] = v * v * v;
}

// coef[g][k] = sum_t pinv[k][t] vals(cell t of leaf g), leaf g = I + J nlx,
// cell t = jj 4 + ii at (4I + ii, 4J + jj)
__global__ void k_box_fit(int64_t nlx, int64_t nleaf, int64_t nx, const double *__restrict__ vals,
                          const double *__restrict__ pinv, double *__restrict__ coef) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nleaf) return;
    const int64_t I = g % nlx, J = g / nlx;
    double v[kNC];
#pragma unroll
    for (int t = 0; t < kNC; ++t) v[t] = vals[(4 * J + (t >> 2)) * nx + 4 * I + (t & 3)];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < kNC; ++t) s = __builtin_fma(pinv[k * kNC + t], v[t], s);
        coef[g * kNB + k] = s;
    }
}

// multipoles of 16 consecutive grid leaves g per workgroup of Pp lanes (lane
// = coefficient o): M[tree leaf of g][o] = sum_k coef[g][k] Q[k][o]
constexpr int kP2MLeaves = 16;
__global__ void k_box_p2m(int64_t nl, int64_t leaf_base, const int32_t *__restrict__ g2l,
                          const double *__restrict__ coef, const double *__restrict__ Q, int Pp,
                          double *__restrict__ M) {
    const int o = threadIdx.x;
    double q[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) q[k] = Q[k * Pp + o];
    const int64_t g0 = (int64_t)blockIdx.x * kP2MLeaves;
#pragma unroll
    for (int i = 0; i < kP2MLeaves; ++i) {
        const int64_t g = g0 + i;
        if (g < nl) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kNB; ++k) s = __builtin_fma(coef[g * kNB + k], q[k], s);
            M[(leaf_base + g2l[g]) * Pp + o] = s;
        }
    }
}

// V at the 16 cells of every leaf.  Per leaf this is one small dense product,
//   V[t] = sum_o E[t][o] L[o] / (2 pi) + sum_(offset, k) A[offset][t][k] c_nb(offset)[k],
// the far field from the leaf's local expansion L and the near field from the
// cubics c of the leaf and its 3 x 3 neighbours (zero outside the grid), so
// it runs on the FP64 matrix cores: a wavefront owns 16 leaves of one grid
// row (the columns of a 16 x 16 output tile, the rows being the 16 cells),
// and contracts over the PP far and 90 near terms in steps of four.  Lane l
// (leaf or cell l % 16, group gq = l / 16) supplies, in far step s, term
// gq FS + s of the local expansion (a contiguous run per lane), and in near
// step s, term gq kNearSteps + s of the 90 near terms (offset, monomial) in
// that order, padded with zeros to 92.  W holds the matching operator
// fragments in lane order, W[step][lane].  The output tile's row r of lane
// group gq is cell gq + 4 r: row r of the leaf's cells at column gq, so each
// store instruction writes 64 consecutive cells of one grid row.
constexpr int kNearSteps = 23;   // ceil(90 / 4)
typedef double box_d4 __attribute__((ext_vector_type(4)));

constexpr int kLeafTiles = 4;    // tiles per wavefront (the operator fragments stay in registers)

template <int PP>   // PP = 0: no far field
__global__ __launch_bounds__(256) void k_box_leaf(
    int64_t nlx, int64_t nly, int64_t nx, int64_t tiles_row, const int32_t *__restrict__ g2l, int64_t leaf_base,
    const double *__restrict__ coef, const double *__restrict__ W, const double *__restrict__ Lc,
    double *__restrict__ V) {
    constexpr int FS = PP / 4, S = FS + kNearSteps;
    const int lane = threadIdx.x & 63, j = lane & 15, gq = lane >> 4;
    const int64_t ntiles = tiles_row * nly;
    const int64_t tile0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kLeafTiles;
    if (tile0 >= ntiles) return;   // (no barriers in this kernel)
    double w[S];
#pragma unroll
    for (int s = 0; s < S; ++s) w[s] = W[s * 64 + lane];
    for (int64_t tile = tile0; tile < tile0 + kLeafTiles && tile < ntiles; ++tile) {
        const int64_t J = tile / tiles_row, I = (tile % tiles_row) * 16 + j;
        const bool ok = I < nlx;
        box_d4 accn = {0.0, 0.0, 0.0, 0.0}, accf = {0.0, 0.0, 0.0, 0.0};
        if constexpr (PP > 0) {
            const double *lp = Lc + (leaf_base + (ok ? g2l[J * nlx + I] : 0)) * PP + gq * FS;
            double bf[FS];
#pragma unroll
            for (int s = 0; s < FS; ++s) bf[s] = ok ? lp[s] : 0.0;
#pragma unroll
            for (int s = 0; s < FS; ++s) accf = __builtin_amdgcn_mfma_f64_16x16x4f64(w[s], bf[s], accf, 0, 0, 0);
        }
        double bn[kNearSteps];
#pragma unroll
        for (int s = 0; s < kNearSteps; ++s) {
            const int f = gq * kNearSteps + s, off = f / kNB, k = f - off * kNB;
            const int64_t In = I + off % 3 - 1, Jn = J + off / 3 - 1;
            const bool in = ok && f < kNOff * kNB && In >= 0 && In < nlx && Jn >= 0 && Jn < nly;
            bn[s] = in ? coef[(Jn * nlx + In) * kNB + k] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < kNearSteps; ++s)
            accn = __builtin_amdgcn_mfma_f64_16x16x4f64(w[FS + s], bn[s], accn, 0, 0, 0);
        if (ok) {
            double *out = V + 4 * J * nx + 4 * I + gq;
#pragma unroll
            for (int r = 0; r < 4; ++r) out[r * nx] = accn[r] + accf[r] * kInv2Pi;
        }
    }
}

// g2l[g] = the tree leaf whose single point is the centre of grid leaf g
__global__ void k_box_g2l(int64_t nl, const int32_t *__restrict__ lrange, const int32_t *__restrict__ perm,
                          int32_t *__restrict__ g2l) {
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (li < nl) g2l[perm[lrange[li * 6]]] = (int32_t)li;
}

// the leaf polynomial of the leaf holding each point
__global__ void k_box_eval(int64_t n, const double *__restrict__ xy, double gx0, double gy0, double h, int64_t nlx,
                           int64_t nly, const double *__restrict__ coef, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = xy[2 * i], y = xy[2 * i + 1];
    const int64_t I = min(max((int64_t)floor((x - gx0) / (4.0 * h)), (int64_t)0), nlx - 1);
    const int64_t J = min(max((int64_t)floor((y - gy0) / (4.0 * h)), (int64_t)0), nly - 1);
    const double cx = gx0 + (4 * I + 2) * h, cy = gy0 + (4 * J + 2) * h;
    double m[kNB];
    monomials((x - cx) / (2.0 * h), (y - cy) / (2.0 * h), m);
    const double *c = coef + (J * nlx + I) * kNB;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kNB; ++k) s = __builtin_fma(c[k], m[k], s);
    out[i] = s;
}

__global__ void k_box_centres(int64_t nlx, int64_t nleaf, double gx0, double gy0, double h, double *__restrict__ xy) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nleaf) return;
    xy[2 * g] = gx0 + (4 * (g % nlx) + 2) * h;
    xy[2 * g + 1] = gy0 + (4 * (g / nlx) + 2) * h;
}

// ---- adaptive leaves ----
__global__ void k_boxa_fit(int64_t n, const double *__restrict__ vals, const double *__restrict__ pinv,
                           double *__restrict__ coef) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double v[kNC];
#pragma unroll
    for (int t = 0; t < kNC; ++t) v[t] = vals[g * kNC + t];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < kNC; ++t) s = __builtin_fma(pinv[k * kNC + t], v[t], s);
        coef[g * kNB + k] = s;
    }
}

// multipole of each tree leaf at a level with M2L: M = Q_level^T coef (Pp lanes)
__global__ void k_boxa_p2m(const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ leaf_lev, int lmin,
                           const int32_t *__restrict__ tin, const double *__restrict__ coef,
                           const double *__restrict__ qlv, int Pp, double *__restrict__ M) {
    const int64_t li = blockIdx.x;
    const int l = leaf_lev[li];
    if (l < lmin) return;
    const int o = threadIdx.x;
    const double *c = coef + (int64_t)tin[li] * kNB;
    const double *q = qlv + (size_t)l * kNB * Pp;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kNB; ++k) s = __builtin_fma(c[k], q[k * Pp + o], s);
    M[(int64_t)leaf_box[li] * Pp + o] = s;
}

// near field at every sorted point: its leaf's U list, each entry's table row
// of the point's cell (cell t = the point's index within its input leaf)
__global__ void k_boxa_near(int64_t n, const int32_t *__restrict__ pleaf, const int32_t *__restrict__ perm,
                            const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist,
                            const int32_t *__restrict__ utab, const int32_t *__restrict__ tin,
                            const double *__restrict__ tabs, const double *__restrict__ coef,
                            double *__restrict__ outs) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t li = pleaf[j];
    const int t = perm[j] & (kNC - 1);
    double acc = 0.0;
    for (int32_t u = uoff[li]; u < uoff[li + 1]; ++u) {
        const double *a = tabs + ((size_t)utab[u] * kNC + t) * kNB;
        const double *c = coef + (int64_t)tin[ulist[u]] * kNB;
#pragma unroll
        for (int k = 0; k < kNB; ++k) acc = __builtin_fma(a[k], c[k], acc);
    }
    outs[j] = acc;
}

// X lists: the coarser leaves' polynomials into the box's local expansion
// (Pp lanes per box; its entries in list order)
__global__ void k_boxa_p2l(const int32_t *__restrict__ xbox, const int32_t *__restrict__ xoff,
                           const int32_t *__restrict__ xl, const int32_t *__restrict__ xtab,
                           const int32_t *__restrict__ tin, const double *__restrict__ coef,
                           const double *__restrict__ T, int Pp, double *__restrict__ Lc) {
    const int64_t b = blockIdx.x;
    const int o = threadIdx.x;
    double s = 0.0;
    for (int32_t e = xoff[b]; e < xoff[b + 1]; ++e) {
        const double *c = coef + (int64_t)tin[xl[e]] * kNB;
        const double *tb = T + (size_t)xtab[e] * kNB * Pp;
#pragma unroll
        for (int k = 0; k < kNB; ++k) s = __builtin_fma(c[k], tb[k * Pp + o], s);
    }
    Lc[(int64_t)xbox[b] * Pp + o] += s;
}

// the leaf polynomial (coefficients of leaf pleaf[i]) at scaled coordinates uv[i]
__global__ void k_boxa_eval(int64_t n, const int32_t *__restrict__ pleaf, const double *__restrict__ uv,
                            const double *__restrict__ coef, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m[kNB];
    monomials(uv[2 * i], uv[2 * i + 1], m);
    const double *c = coef + (int64_t)pleaf[i] * kNB;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kNB; ++k) s = __builtin_fma(c[k], m[k], s);
    out[i] = s;
}

// Sec. 3.1's refinement test: the cubic fitted to a leaf's 16 cell values
// against the values at its children's 64 cell centres (child q = qy 2 + qx)
__global__ void k_box_refine(int64_t n, const double *__restrict__ v16, const double *__restrict__ v64,
                             const double *__restrict__ pinv, double tol, int32_t *__restrict__ flags,
                             double *__restrict__ err) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double c[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        double s = 0.0;
        for (int t = 0; t < kNC; ++t) s = __builtin_fma(pinv[k * kNC + t], v16[g * kNC + t], s);
        c[k] = s;
    }
    double e = 0.0, m[kNB];
    for (int q = 0; q < 4; ++q)
        for (int t = 0; t < kNC; ++t) {
            const double u = -1.0 + ((q & 1) * 4 + (t & 3) + 0.5) * 0.25;
            const double v = -1.0 + ((q >> 1) * 4 + (t >> 2) + 0.5) * 0.25;
            monomials(u, v, m);
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kNB; ++k) s = __builtin_fma(c[k], m[k], s);
            e = fmax(e, fabs(s - v64[g * 64 + q * kNC + t]));
        }
    flags[g] = e > tol ? 1 : 0;
    if (err) err[g] = e;
}

// f(i0, i1) on contiguous chunks of [0, n) on up to 16 host threads
template <typename F>
void host_parallel(int64_t n, F f) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({16, n, (int64_t)std::thread::hardware_concurrency()}));
    const int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> pool;
    for (int64_t i = 0; i < nt && i * per < n; ++i) pool.emplace_back(f, i * per, std::min(n, (i + 1) * per));
    for (auto &th : pool) th.join();
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n)
void gauss01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(3.14159265358979323846L * (i + 0.75L) / (n + 0.5L)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        x[i] = (double)(0.5L * (1 - z));
        w[i] = (double)(1.0L / ((1 - z * z) * dp * dp));   // = 2/((1-z^2) P'^2) / 2
    }
}

}  // namespace

struct BoxPlan {
    double gx0 = 0, gy0 = 0, h = 0, alpha = 0;
    int64_t nx = 0, ny = 0, nlx = 0, nly = 0, nleaf = 0;
    double square[3] = {0, 0, 0};
    PlanPtr fmm;
    int Pp = 0;
    bool far = false;
    DevBuf<double> centres, pinv, A, Q, E, coef;
    DevBuf<double> W;         // the leaf kernel's operator fragments in lane order
    DevBuf<int32_t> g2l;      // grid leaf -> tree leaf
    // adaptive leaves: the leaf set (level, ix, iy) over the root square; the
    // tree over the leaves' cell centres; per U-list entry and per X-list entry
    // the index of its table; per tree leaf its input leaf; P2M tables by level
    bool adaptive = false;
    std::vector<int32_t> lev, ix, iy;
    DevBuf<double> cells, qlv, near_tab, p2l_tab;
    DevBuf<int32_t> tin, u_tab, x_tab;
    // points evaluated through the leaf polynomials (the boundary nodes):
    // their leaf and their scaled coordinates in it, for one point array
    const double *pts_key = nullptr;
    int64_t pts_n = 0;
    uint64_t pts_gen = 0;
    DevBuf<int32_t> pts_leaf;
    DevBuf<double> pts_uv;
};

void BoxPlanDeleter::operator()(BoxPlan *p) const { delete p; }

namespace {

// the least-squares fit: pinv = (V^T V)^{-1} V^T, V[t][k] = m_k at cell t
std::vector<double> fit_matrix() {
    static const double off[4] = {-0.75, -0.25, 0.25, 0.75};
    long double VtV[kNB][kNB] = {}, inv[kNB][kNB] = {};
    double Vm[kNC][kNB];
    for (int t = 0; t < kNC; ++t) monomials(off[t & 3], off[t >> 2], Vm[t]);
    for (int a = 0; a < kNB; ++a)
        for (int b = 0; b < kNB; ++b) {
            for (int t = 0; t < kNC; ++t) VtV[a][b] += (long double)Vm[t][a] * Vm[t][b];
            inv[a][b] = a == b;
        }
    for (int c = 0; c < kNB; ++c) {   // Gauss-Jordan with partial pivoting
        int piv = c;
        for (int r = c + 1; r < kNB; ++r)
            if (std::fabs((double)VtV[r][c]) > std::fabs((double)VtV[piv][c])) piv = r;
        for (int k = 0; k < kNB; ++k) {
            std::swap(VtV[c][k], VtV[piv][k]);
            std::swap(inv[c][k], inv[piv][k]);
        }
        const long double d = VtV[c][c];
        for (int k = 0; k < kNB; ++k) {
            VtV[c][k] /= d;
            inv[c][k] /= d;
        }
        for (int r = 0; r < kNB; ++r) {
            if (r == c) continue;
            const long double f = VtV[r][c];
            for (int k = 0; k < kNB; ++k) {
                VtV[r][k] -= f * VtV[c][k];
                inv[r][k] -= f * inv[c][k];
            }
        }
    }
    std::vector<double> pv(kNB * kNC);
    for (int k = 0; k < kNB; ++k)
        for (int t = 0; t < kNC; ++t) {
            long double s = 0;
            for (int b = 0; b < kNB; ++b) s += inv[k][b] * Vm[t][b];
            pv[k * kNC + t] = (double)s;
        }
    return pv;
}

// out[t][k] = (1/2pi) int over the leaf [-Hs, Hs]^2 of K0(|x_t - y|/alpha)
// m_k(y / Hs) dy for 16 targets x_t given relative to the leaf's centre.  Per
// cell of the leaf (side Hs/2): tensor Gauss-Legendre, except for a cell
// centred on the target, taken in polar form about it (per edge, the angles
// within pi/4 of its normal, R = (h/2)/cos; the radial integral of K0 r in
// closed form, the rest m(x_t + r e) - m(x_t) = O(r) with r = R s^2)
struct GLRule {
    std::vector<double> x, w;
    explicit GLRule(int n) { gauss01(n, x, w); }
};

void near_table(const double *tx, const double *ty, double Hs, double al, double *out) {
    static const GLRule g20(20), g32(32);   // (initialised once, thread-safe)
    const std::vector<double> &gx = g20.x, &gw = g20.w, &px = g32.x, &pw = g32.w;
    const double h = 0.5 * Hs;   // cell side
    for (int t = 0; t < kNC; ++t) {
        long double acc[kNB] = {};
        double m[kNB], mt[kNB];
        monomials(tx[t] / Hs, ty[t] / Hs, mt);
        for (int cj = 0; cj < 4; ++cj)
            for (int ci = 0; ci < 4; ++ci) {
                const double ccx = (ci - 1.5) * h, ccy = (cj - 1.5) * h;
                if (std::fabs(tx[t] - ccx) < 1e-9 * h && std::fabs(ty[t] - ccy) < 1e-9 * h) {
                    for (int e = 0; e < 4; ++e) {
                        const double thn = e * 0.5 * kPi;
                        for (int a = 0; a < (int)px.size(); ++a) {
                            const double th = thn + (px[a] - 0.5) * 0.5 * kPi, wth = pw[a] * 0.5 * kPi;
                            const double R = 0.5 * h / std::cos(th - thn);
                            const double c = std::cos(th), sn = std::sin(th);
                            const double base = al * al - al * R * k1(R / al);
                            for (int k = 0; k < kNB; ++k) acc[k] += (long double)wth * mt[k] * base;
                            for (int b = 0; b < (int)px.size(); ++b) {
                                const double sr = px[b], r = R * sr * sr, jac = 2.0 * R * sr;
                                monomials((tx[t] + r * c) / Hs, (ty[t] + r * sn) / Hs, m);
                                const double f = wth * pw[b] * k0(r / al) * r * jac;
                                for (int k = 0; k < kNB; ++k) acc[k] += (long double)f * (m[k] - mt[k]);
                            }
                        }
                    }
                } else {
                    for (int a = 0; a < (int)gx.size(); ++a)
                        for (int b = 0; b < (int)gx.size(); ++b) {
                            const double yx = ccx + (gx[a] - 0.5) * h, yy = ccy + (gx[b] - 0.5) * h;
                            const double f = gw[a] * gw[b] * h * h * k0(std::hypot(tx[t] - yx, ty[t] - yy) / al);
                            monomials(yx / Hs, yy / Hs, m);
                            for (int k = 0; k < kNB; ++k) acc[k] += (long double)f * m[k];
                        }
                }
            }
        for (int k = 0; k < kNB; ++k) out[t * kNB + k] = (double)(acc[k] * kInv2Pi);
    }
}

// Q[k][o]: the leaf's ([-Hs, Hs]^2) monomial moments against
// conj(F^I_n(y/alpha)) / I_n(R), in the multipoles' real layout
void moments(double Hs, long double R, double al, int p, int Pp, double *Q) {
    const std::vector<long double> IR = bessel_i_seq(R, p + 1);
    std::vector<double> gx, gw;
    gauss01(24, gx, gw);
    std::vector<long double> Ql((size_t)kNB * Pp, 0.0L);
    double m[kNB];
    for (int a = 0; a < (int)gx.size(); ++a)
        for (int b = 0; b < (int)gx.size(); ++b) {
            const double yx = (2.0 * gx[a] - 1.0) * Hs, yy = (2.0 * gx[b] - 1.0) * Hs;
            const long double wq = (long double)gw[a] * gw[b] * 4.0L * Hs * Hs;
            monomials(yx / Hs, yy / Hs, m);
            const long double rho = std::hypot((long double)yx, (long double)yy) / al;
            const long double phi = std::atan2((long double)yy, (long double)yx);
            const std::vector<long double> Ir = bessel_i_seq(rho, p + 1);
            for (int n = 0; n <= p; ++n) {
                const long double g = wq * Ir[n] / IR[n];
                const long double cr = g * std::cos(n * phi), ci = -g * std::sin(n * phi);
                for (int k = 0; k < kNB; ++k) {
                    if (n == 0) {
                        Ql[(size_t)k * Pp] += cr * m[k];
                    } else {
                        Ql[(size_t)k * Pp + 2 * n - 1] += cr * m[k];
                        Ql[(size_t)k * Pp + 2 * n] += ci * m[k];
                    }
                }
            }
        }
    for (size_t i = 0; i < Ql.size(); ++i) Q[i] = (double)Ql[i];
}

// T[k][o]: P2L of the monomials of a leaf ([-Hs, Hs]^2 about (sx, sy), given
// relative to the box centre) into the box's stored local coefficients
// (Lh_m = L_m I_m(R), L_m = int m_k K_m(rho) e^{-i m theta}, (rho, theta) of
// (y - c_box)/alpha), in the real layout
void p2l_table(double sx, double sy, double Hs, long double R, double al, int p, int Pp, double *T) {
    const std::vector<long double> IR = bessel_i_seq(R, p + 1);
    std::vector<double> gx, gw;
    gauss01(24, gx, gw);
    std::vector<long double> Tl((size_t)kNB * Pp, 0.0L), K(p + 2);
    double m[kNB];
    for (int a = 0; a < (int)gx.size(); ++a)
        for (int b = 0; b < (int)gx.size(); ++b) {
            const double ux = (2.0 * gx[a] - 1.0) * Hs, uy = (2.0 * gx[b] - 1.0) * Hs;
            const long double wq = (long double)gw[a] * gw[b] * 4.0L * Hs * Hs;
            monomials(ux / Hs, uy / Hs, m);
            const double wx = (sx + ux) / al, wy = (sy + uy) / al;
            const double rho = std::hypot(wx, wy);
            const long double th = std::atan2((long double)wy, (long double)wx);
            K[0] = k0(rho);
            K[1] = k1(rho);
            for (int n = 1; n <= p; ++n) K[n + 1] = K[n - 1] + (2.0L * n / rho) * K[n];
            for (int n = 0; n <= p; ++n) {
                const long double g = wq * K[n] * IR[n];
                const long double cr = g * std::cos(n * th), ci = -g * std::sin(n * th);
                for (int k = 0; k < kNB; ++k) {
                    if (n == 0) {
                        Tl[(size_t)k * Pp] += cr * m[k];
                    } else {
                        Tl[(size_t)k * Pp + 2 * n - 1] += cr * m[k];
                        Tl[(size_t)k * Pp + 2 * n] += ci * m[k];
                    }
                }
            }
        }
    for (size_t i = 0; i < Tl.size(); ++i) T[i] = (double)Tl[i];
}

// host tables of a uniform box plan: the fit, the near-field integrals, the
// leaf moments and the local-expansion weights at the cells
void box_tables(Context &ctx, BoxPlan &bp) {
    const double h = bp.h, al = bp.alpha, H = 2.0 * h;
    {
        const std::vector<double> pv = fit_matrix();
        YK_HIP(hipMemcpyAsync(bp.pinv.ensure(pv.size()), pv.data(), pv.size() * sizeof(double),
                              hipMemcpyHostToDevice, ctx.stream));
    }
    // near field: A[off][t][k] for the 16 cells of a leaf at each of the 9 offsets
    std::vector<double> A((size_t)kNOff * kNC * kNB, 0.0), E;
    {
        host_parallel(kNOff, [&](int64_t i0, int64_t i1) {
            for (int64_t off = i0; off < i1; ++off) {
                const int dI = (int)(off % 3) - 1, dJ = (int)(off / 3) - 1;
                double tx[kNC], ty[kNC];
                for (int t = 0; t < kNC; ++t) {   // target relative to the source leaf's centre
                    tx[t] = -4.0 * h * dI + ((t & 3) - 1.5) * h;
                    ty[t] = -4.0 * h * dJ + ((t >> 2) - 1.5) * h;
                }
                near_table(tx, ty, H, al, &A[(size_t)off * kNC * kNB]);
            }
        });
        YK_HIP(hipMemcpyAsync(bp.A.ensure(A.size()), A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
    }
    if (bp.far) {
        const FmmPlan &pl = *bp.fmm;
        const int p = pl.p, Pp = pl.Pp;
        const long double R = pl.lev[pl.L].R;
        const std::vector<long double> IR = bessel_i_seq(R, p + 1);
        std::vector<double> Q((size_t)kNB * Pp, 0.0);
        E.assign((size_t)kNC * Pp, 0.0);
        moments(H, R, al, p, Pp, Q.data());
        // E[t][o]: the weights of the stored local coefficients in the value at cell t
        for (int t = 0; t < kNC; ++t) {
            const long double x = ((t & 3) - 1.5L) * h / al, y = ((t >> 2) - 1.5L) * h / al;
            const long double rho = std::hypot(x, y), th = std::atan2(y, x);
            const std::vector<long double> Ir = bessel_i_seq(rho, p + 1);
            E[(size_t)t * Pp] = (double)(Ir[0] / IR[0]);
            for (int n = 1; n <= p; ++n) {
                const long double g = 2.0L * Ir[n] / IR[n];
                E[(size_t)t * Pp + 2 * n - 1] = (double)(g * std::cos(n * th));
                E[(size_t)t * Pp + 2 * n] = (double)(-g * std::sin(n * th));
            }
        }
        YK_HIP(hipMemcpyAsync(bp.Q.ensure(Q.size()), Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
        YK_HIP(hipMemcpyAsync(bp.E.ensure(E.size()), E.data(), E.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
    }
    // the uniform leaf kernel's operator fragments W[step][lane] (the term
    // order of k_box_leaf): cell t = lane % 16, lane group gq = lane / 16
    if (!bp.adaptive) {
        const int FS = bp.far ? bp.Pp / 4 : 0, S = FS + kNearSteps;
        std::vector<double> W((size_t)S * 64, 0.0);
        for (int st = 0; st < S; ++st)
            for (int l = 0; l < 64; ++l) {
                const int t = l & 15, gq = l >> 4;
                double v = 0.0;
                if (st < FS) {
                    v = E[(size_t)t * bp.Pp + gq * FS + st];
                } else {
                    const int f = gq * kNearSteps + (st - FS);
                    if (f < kNOff * kNB) v = A[((size_t)(f / kNB) * kNC + t) * kNB + f % kNB];
                }
                W[(size_t)st * 64 + l] = v;
            }
        YK_HIP(hipMemcpyAsync(bp.W.ensure(W.size()), W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

BoxPlan &box_plan(Context &ctx, const yk_grid &g, double alpha) {
    if (ctx.box && !ctx.box->adaptive && ctx.box->gx0 == g.x0 && ctx.box->gy0 == g.y0 && ctx.box->h == g.h &&
        ctx.box->nx == g.nx &&
        ctx.box->ny == g.ny && ctx.box->alpha == alpha)
        return *ctx.box;
    YK_REQUIRE(g.nx % 4 == 0 && g.ny % 4 == 0, "the box code needs grid sides that are multiples of 4 cells");
    ctx.box.reset();
    BoxPtr bp(new BoxPlan());
    bp->gx0 = g.x0;
    bp->gy0 = g.y0;
    bp->h = g.h;
    bp->nx = g.nx;
    bp->ny = g.ny;
    bp->alpha = alpha;
    bp->nlx = g.nx / 4;
    bp->nly = g.ny / 4;
    bp->nleaf = bp->nlx * bp->nly;
    int Lb = 0;
    while (((int64_t)1 << Lb) < std::max(bp->nlx, bp->nly)) ++Lb;
    YK_REQUIRE(Lb <= kMaxLevel, "grid too large for the box code's tree");
    bp->square[0] = g.x0;
    bp->square[1] = g.y0;
    bp->square[2] = std::ldexp(4.0 * g.h, Lb);
    double *cxy = bp->centres.ensure(2 * bp->nleaf);
    hipLaunchKernelGGL(k_box_centres, dim3(nblk(bp->nleaf, 256)), dim3(256), 0, ctx.stream, bp->nlx, bp->nleaf,
                       g.x0, g.y0, g.h, cxy);
    check_launch(ctx, "k_box_centres");
    // the tree over the leaves: one point (the centre) per leaf box
    PlanPtr fp(new FmmPlan());
    fp->key_n[0] = bp->nleaf;
    fp->key_xy[0] = cxy;
    fp->alpha = alpha;
    fp->opt_p = 31;
    fp->opt_leaf = 1;
    fp->opt_tol = 1e-10;
    fp->opt_tree = 0;
    SumProblem pb;
    pb.n[0] = bp->nleaf;
    pb.xy[0] = cxy;
    pb.alpha = alpha;
    pb.square = bp->square;
    build_tree(ctx, *fp, pb);
    YK_REQUIRE(fp->L == Lb && fp->nleaf == bp->nleaf, "box code: the tree's leaves are not the grid's leaves");
    bp->far = fp->lmin <= fp->L;
    bp->Pp = fp->Pp;
    bp->fmm = std::move(fp);
    hipLaunchKernelGGL(k_box_g2l, dim3(nblk(bp->nleaf, 256)), dim3(256), 0, ctx.stream, bp->nleaf,
                       bp->fmm->lrange.p, bp->fmm->perm.p, bp->g2l.ensure(bp->nleaf));
    check_launch(ctx, "k_box_g2l");
    box_tables(ctx, *bp);
    ctx.box = std::move(bp);
    return *ctx.box;
}

}  // namespace

void box_potential(Context &ctx, const yk_grid &g, const double *B, double alpha, double *V) {
    BoxPlan &bp = box_plan(ctx, g, alpha);
    FmmPlan &pl = *bp.fmm;
    double *coef = bp.coef.ensure(bp.nleaf * kNB);
    hipLaunchKernelGGL(k_box_fit, dim3(nblk(bp.nleaf, 128)), dim3(128), 0, ctx.stream, bp.nlx, bp.nleaf, bp.nx, B,
                       bp.pinv.p, coef);
    check_launch(ctx, "k_box_fit");
    ActiveSet &as = get_active(ctx, pl, 1);
    const int64_t leaf_base = pl.lev[pl.L].begin;
    if (bp.far) {
        {
            StageTimer tm(ctx, YK_STAGE_P2M);
            hipLaunchKernelGGL(k_box_p2m, dim3(nblk(bp.nleaf, kP2MLeaves)), dim3(pl.Pp), 0, ctx.stream, bp.nleaf,
                               leaf_base, bp.g2l.p, coef, bp.Q.p, pl.Pp, pl.M.p);
            check_launch(ctx, "k_box_p2m");
        }
        fmm_m2m(ctx, pl);
        launch_fill(ctx, (int64_t)pl.nbox * pl.Pp, 0.0, pl.Lc.p);
        fmm_m2l(ctx, pl, as, false);
        fmm_l2l(ctx, pl, as, false);
    }
    StageTimer tl(ctx, YK_STAGE_LEAF);
    const int64_t tiles_row = (bp.nlx + 15) / 16;
    const unsigned nb = nblk(tiles_row * bp.nly, 4 * kLeafTiles);
    const int pp = bp.far ? pl.Pp : 0;
#define YK_BOX_LEAF(PPV)                                                                                   \
    case PPV:                                                                                              \
        hipLaunchKernelGGL(k_box_leaf<PPV>, dim3(nb), dim3(256), 0, ctx.stream, bp.nlx, bp.nly, bp.nx, tiles_row, \
                           bp.g2l.p, leaf_base, coef, bp.W.p, pl.Lc.p, V);                                \
        break;
    switch (pp) {
        YK_BOX_LEAF(0)
        YK_BOX_LEAF(16)
        YK_BOX_LEAF(32)
        YK_BOX_LEAF(48)
        YK_BOX_LEAF(64)
        default:
            throw Error{YK_ERR_INTERNAL, "no box leaf kernel for this padded order"};
    }
#undef YK_BOX_LEAF
    check_launch(ctx, "k_box_leaf");
}

namespace {

// level-15 cell coordinates of a box from its Morton code
inline void box_xy(uint32_t code, int64_t &ix, int64_t &iy) {
    auto compact = [](uint32_t v) {
        v &= 0x55555555u;
        v = (v | (v >> 1)) & 0x33333333u;
        v = (v | (v >> 2)) & 0x0f0f0f0fu;
        v = (v | (v >> 4)) & 0x00ff00ffu;
        v = (v | (v >> 8)) & 0x0000ffffu;
        return v;
    };
    ix = compact(code);
    iy = compact(code >> 1);
}

BoxPlan &box_plan_adaptive(Context &ctx, const double root[3], int64_t n, const int32_t *lev, const int32_t *ix,
                           const int32_t *iy, double alpha) {
    if (ctx.box && ctx.box->adaptive && ctx.box->alpha == alpha && ctx.box->square[0] == root[0] &&
        ctx.box->square[1] == root[1] && ctx.box->square[2] == root[2] && (int64_t)ctx.box->lev.size() == n &&
        std::equal(lev, lev + n, ctx.box->lev.begin()) && std::equal(ix, ix + n, ctx.box->ix.begin()) &&
        std::equal(iy, iy + n, ctx.box->iy.begin()))
        return *ctx.box;
    ctx.box.reset();
    // the volume trees and near-boundary sets keyed by the cells' buffer are
    // stale: a new plan may reuse its address for other cells
    ctx.plan_vol.reset();
    ctx.plan_near.reset();
    ctx.plan_nearc.reset();
    ctx.near.reset();
    BoxPtr bp(new BoxPlan());
    bp->adaptive = true;
    bp->alpha = alpha;
    for (int k = 0; k < 3; ++k) bp->square[k] = root[k];
    bp->lev.assign(lev, lev + n);
    bp->ix.assign(ix, ix + n);
    bp->iy.assign(iy, iy + n);
    bp->nleaf = n;
    for (int64_t k = 0; k < n; ++k)
        YK_REQUIRE(lev[k] >= 0 && lev[k] <= kMaxLevel - 2 && ix[k] >= 0 && iy[k] >= 0 &&
                       ix[k] < (1 << lev[k]) && iy[k] < (1 << lev[k]),
                   "leaf levels must be 0 .. 13 and positions inside the square");
    // the leaves' cell centres: the tree's points (cell t of leaf k is point 16 k + t)
    std::vector<double> cells((size_t)n * kNC * 2);
    for (int64_t k = 0; k < n; ++k) {
        const double sl = root[2] / (double)(1 << lev[k]);
        for (int t = 0; t < kNC; ++t) {
            cells[(k * kNC + t) * 2] = root[0] + (ix[k] + ((t & 3) + 0.5) / 4.0) * sl;
            cells[(k * kNC + t) * 2 + 1] = root[1] + (iy[k] + ((t >> 2) + 0.5) / 4.0) * sl;
        }
    }
    double *dcells = bp->cells.ensure(cells.size());
    YK_HIP(hipMemcpyAsync(dcells, cells.data(), cells.size() * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
    // the adaptive tree over the cells, split above 16 points: its leaves are
    // the given leaves when these tile without overlap and are 2:1 balanced
    PlanPtr fp(new FmmPlan());
    fp->key_n[0] = n * kNC;
    fp->key_xy[0] = dcells;
    fp->alpha = alpha;
    fp->opt_p = 31;
    fp->opt_leaf = 2 * kNC;
    fp->opt_tol = 1e-10;
    fp->opt_tree = 1;
    SumProblem pb;
    pb.n[0] = n * kNC;
    pb.xy[0] = dcells;
    pb.alpha = alpha;
    pb.square = root;
    build_tree(ctx, *fp, pb);
    FmmPlan &pl = *fp;
    bool ok = pl.nleaf == n;
    for (int64_t li = 0; ok && li < pl.nleaf; ++li)
        ok = pl.h_lrange[li * 6 + 1] - pl.h_lrange[li * 6] == kNC;
    YK_REQUIRE(ok, "the leaves must not overlap and must be 2:1 balanced (touching leaves one level apart)");
    // tree leaf -> input leaf
    std::vector<int32_t> perm(pl.N);
    YK_HIP(hipMemcpyAsync(perm.data(), pl.perm.p, pl.N * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    std::vector<int32_t> tin(n);
    for (int64_t li = 0; li < n; ++li) tin[li] = perm[pl.h_lrange[li * 6]] / kNC;
    bp->far = pl.lmin <= pl.L;
    bp->Pp = pl.Pp;
    const int p = pl.p, Pp = pl.Pp;
    {
        const std::vector<double> pv = fit_matrix();
        YK_HIP(hipMemcpyAsync(bp->pinv.ensure(pv.size()), pv.data(), pv.size() * sizeof(double),
                              hipMemcpyHostToDevice, ctx.stream));
    }
    // leaf centres in units of a quarter of the finer side: exact integers
    auto unit_centre = [&](int64_t k, int lref, int64_t &ux, int64_t &uy) {
        const int sh = lref + 2 - lev[k];   // >= 1 for leaves at most one level finer than lref
        ux = (2 * (int64_t)ix[k] + 1) << (sh - 1);
        uy = (2 * (int64_t)iy[k] + 1) << (sh - 1);
    };
    // near tables, one per distinct (target level, source level, offset)
    {
        std::vector<int32_t> uoff(n + 1), ul(pl.n_ulist);
        YK_HIP(hipMemcpyAsync(uoff.data(), pl.ulist_off.p, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                              ctx.stream));
        YK_HIP(hipMemcpyAsync(ul.data(), pl.ulist.p, pl.n_ulist * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        std::map<std::array<int64_t, 4>, int32_t> keys;
        std::vector<std::array<int64_t, 4>> klist;
        std::vector<int32_t> utab(pl.n_ulist);
        for (int64_t li = 0; li < n; ++li) {
            const int64_t kt = tin[li];
            for (int32_t u = uoff[li]; u < uoff[li + 1]; ++u) {
                const int64_t ks = tin[ul[u]];
                YK_REQUIRE(std::abs(lev[ks] - lev[kt]) <= 1, "touching leaves more than one level apart");
                const int lref = std::max(lev[kt], lev[ks]);
                int64_t tx, ty, sx, sy;
                unit_centre(kt, lref, tx, ty);
                unit_centre(ks, lref, sx, sy);
                const std::array<int64_t, 4> key = {lev[kt], lev[ks], sx - tx, sy - ty};
                auto it = keys.find(key);
                if (it == keys.end()) {
                    it = keys.emplace(key, (int32_t)klist.size()).first;
                    klist.push_back(key);
                }
                utab[u] = it->second;
            }
        }
        std::vector<double> tabs(klist.size() * kNC * kNB);
        host_parallel((int64_t)klist.size(), [&](int64_t i0, int64_t i1) {
            for (int64_t q = i0; q < i1; ++q) {
                const auto &key = klist[q];
                const int lt = (int)key[0], ls = (int)key[1];
                const double st = root[2] / (double)(1 << lt), ss = root[2] / (double)(1 << ls);
                const double unit = root[2] / (double)(1ll << (std::max(lt, ls) + 2));
                double tx[kNC], ty[kNC];
                for (int t = 0; t < kNC; ++t) {   // target cells relative to the source centre
                    tx[t] = -key[2] * unit + ((t & 3) - 1.5) * 0.25 * st;
                    ty[t] = -key[3] * unit + ((t >> 2) - 1.5) * 0.25 * st;
                }
                near_table(tx, ty, 0.5 * ss, alpha, &tabs[(size_t)q * kNC * kNB]);
            }
        });
        YK_HIP(hipMemcpyAsync(bp->near_tab.ensure(std::max<size_t>(tabs.size(), 1)), tabs.data(),
                              tabs.size() * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyAsync(bp->u_tab.ensure(std::max<size_t>(utab.size(), 1)), utab.data(),
                              utab.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
    }
    if (bp->far) {
        // P2M tables of every level from lmin on
        std::vector<double> q((size_t)(pl.L + 1) * kNB * Pp, 0.0);
        host_parallel(pl.L + 1 - pl.lmin, [&](int64_t i0, int64_t i1) {
            for (int64_t k = i0; k < i1; ++k) {
                const int l = pl.lmin + (int)k;
                moments(0.5 * root[2] / (double)(1 << l), pl.lev[l].R, alpha, p, Pp, &q[(size_t)l * kNB * Pp]);
            }
        });
        YK_HIP(hipMemcpyAsync(bp->qlv.ensure(q.size()), q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
        // X tables, one per distinct (box level, leaf level, offset)
        std::map<std::array<int64_t, 4>, int32_t> keys;
        std::vector<std::array<int64_t, 4>> klist;
        std::vector<int32_t> xtab(pl.h_xl.size());
        for (size_t b = 0; b < pl.h_xbox.size(); ++b) {
            const int32_t box = pl.h_xbox[b];
            const int lb = pl.h_blevel[box];
            int64_t bx, by;
            box_xy(pl.hcode[box], bx, by);
            for (int32_t e = pl.h_xoff[b]; e < pl.h_xoff[b + 1]; ++e) {
                const int64_t kc = tin[pl.h_xl[e]];
                YK_REQUIRE(lev[kc] < lb, "an X-list leaf must be coarser than its box");
                int64_t sx, sy;
                unit_centre(kc, lb, sx, sy);
                const std::array<int64_t, 4> key = {lb, lev[kc], sx - (4 * bx + 2), sy - (4 * by + 2)};
                auto it = keys.find(key);
                if (it == keys.end()) {
                    it = keys.emplace(key, (int32_t)klist.size()).first;
                    klist.push_back(key);
                }
                xtab[e] = it->second;
            }
        }
        std::vector<double> T(klist.size() * kNB * Pp, 0.0);
        host_parallel((int64_t)klist.size(), [&](int64_t i0, int64_t i1) {
            for (int64_t q2 = i0; q2 < i1; ++q2) {
                const auto &key = klist[q2];
                const int lb = (int)key[0], lc = (int)key[1];
                const double unit = root[2] / (double)(1ll << (lb + 2));
                p2l_table(key[2] * unit, key[3] * unit, 0.5 * root[2] / (double)(1 << lc), pl.lev[lb].R, alpha, p,
                          Pp, &T[(size_t)q2 * kNB * Pp]);
            }
        });
        YK_HIP(hipMemcpyAsync(bp->p2l_tab.ensure(std::max<size_t>(T.size(), 1)), T.data(), T.size() * sizeof(double),
                              hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyAsync(bp->x_tab.ensure(std::max<size_t>(xtab.size(), 1)), xtab.data(),
                              xtab.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
    }
    YK_HIP(hipMemcpyAsync(bp->tin.ensure(n), tin.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    bp->fmm = std::move(fp);
    ctx.box = std::move(bp);
    return *ctx.box;
}

}  // namespace

void box_potential_adaptive(Context &ctx, const double root[3], int64_t n, const int32_t *lev, const int32_t *ix,
                            const int32_t *iy, const double *vals, double alpha, double *V) {
    BoxPlan &bp = box_plan_adaptive(ctx, root, n, lev, ix, iy, alpha);
    FmmPlan &pl = *bp.fmm;
    double *coef = bp.coef.ensure(n * kNB);
    hipLaunchKernelGGL(k_boxa_fit, dim3(nblk(n, 128)), dim3(128), 0, ctx.stream, n, vals, bp.pinv.p, coef);
    check_launch(ctx, "k_boxa_fit");
    ActiveSet &as = get_active(ctx, pl, 1);
    if (bp.far) {
        {
            StageTimer tm(ctx, YK_STAGE_P2M);
            hipLaunchKernelGGL(k_boxa_p2m, dim3((unsigned)pl.nleaf), dim3(pl.Pp), 0, ctx.stream, pl.leaf_box.p,
                               pl.leaf_lev.p, pl.lmin, bp.tin.p, coef, bp.qlv.p, pl.Pp, pl.M.p);
            check_launch(ctx, "k_boxa_p2m");
        }
        fmm_m2m(ctx, pl);
        launch_fill(ctx, (int64_t)pl.nbox * pl.Pp, 0.0, pl.Lc.p);
        fmm_m2l(ctx, pl, as, false);
        if (pl.n_xbox > 0) {
            StageTimer tx(ctx, YK_STAGE_M2L);
            hipLaunchKernelGGL(k_boxa_p2l, dim3((unsigned)pl.n_xbox), dim3(pl.Pp), 0, ctx.stream, pl.xbox.p,
                               pl.xoff.p, pl.xl.p, bp.x_tab.p, bp.tin.p, coef, bp.p2l_tab.p, pl.Pp, pl.Lc.p);
            check_launch(ctx, "k_boxa_p2l");
        }
        fmm_l2l(ctx, pl, as, false);
    }
    double *outs = pl.outs.ensure(pl.N);
    {
        StageTimer tl(ctx, YK_STAGE_LEAF);
        hipLaunchKernelGGL(k_boxa_near, dim3(nblk(pl.N, 256)), dim3(256), 0, ctx.stream, pl.N, pl.pleaf.p,
                           pl.perm.p, pl.ulist_off.p, pl.ulist.p, bp.u_tab.p, bp.tin.p, bp.near_tab.p, coef, outs);
        check_launch(ctx, "k_boxa_near");
    }
    double *out3[3] = {V, nullptr, nullptr};
    fmm_adaptive_finish(ctx, pl, 1, outs, out3);
}

const double *box_cells(Context &ctx) {
    YK_REQUIRE(ctx.box && ctx.box->adaptive, "no adaptive box plan");
    return ctx.box->cells.p;
}

void box_leaves_eval(Context &ctx, const double *vals, int64_t n, const double *xy, uint64_t gen, double *out) {
    YK_REQUIRE(ctx.box && ctx.box->adaptive, "the leaf polynomials need the adaptive box plan (the potential first)");
    BoxPlan &bp = *ctx.box;
    const int64_t nl = bp.nleaf;
    if (bp.pts_key != xy || bp.pts_n != n || bp.pts_gen != gen || gen == 0) {
        // each point's leaf: the level-l box holding it, looked up from the
        // coarsest level down among the leaves
        std::vector<double> hxy(2 * n);
        if (n > 0)
            YK_HIP(hipMemcpyAsync(hxy.data(), xy, 2 * n * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        std::map<std::array<int64_t, 3>, int32_t> where;
        int lmax = 0;
        for (int64_t k = 0; k < nl; ++k) {
            where[{bp.lev[k], bp.ix[k], bp.iy[k]}] = (int32_t)k;
            lmax = std::max(lmax, bp.lev[k]);
        }
        std::vector<int32_t> pl(n);
        std::vector<double> uv(2 * n);
        for (int64_t i = 0; i < n; ++i) {
            const double x = (hxy[2 * i] - bp.square[0]) / bp.square[2], y = (hxy[2 * i + 1] - bp.square[1]) / bp.square[2];
            YK_REQUIRE(x >= 0.0 && x < 1.0 && y >= 0.0 && y < 1.0, "a point lies outside the leaves' square");
            int32_t found = -1;
            for (int l = 0; l <= lmax && found < 0; ++l) {
                const int64_t cx = (int64_t)std::floor(std::ldexp(x, l)), cy = (int64_t)std::floor(std::ldexp(y, l));
                auto it = where.find({l, cx, cy});
                if (it != where.end()) found = it->second;
            }
            YK_REQUIRE(found >= 0, "a point lies in no leaf");
            pl[i] = found;
            const double s = std::ldexp(1.0, -bp.lev[found]);
            uv[2 * i] = (x - (bp.ix[found] + 0.5) * s) / (0.5 * s);
            uv[2 * i + 1] = (y - (bp.iy[found] + 0.5) * s) / (0.5 * s);
        }
        YK_HIP(hipMemcpyAsync(bp.pts_leaf.ensure(std::max<int64_t>(n, 1)), pl.data(), n * sizeof(int32_t),
                              hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyAsync(bp.pts_uv.ensure(std::max<int64_t>(2 * n, 1)), uv.data(), 2 * n * sizeof(double),
                              hipMemcpyHostToDevice, ctx.stream));
        bp.pts_key = xy;
        bp.pts_n = n;
        bp.pts_gen = gen;
    }
    DevBuf<double> cbuf;
    double *coef = cbuf.ensure(nl * kNB);
    hipLaunchKernelGGL(k_boxa_fit, dim3(nblk(nl, 128)), dim3(128), 0, ctx.stream, nl, vals, bp.pinv.p, coef);
    check_launch(ctx, "k_boxa_fit");
    if (n > 0) {
        hipLaunchKernelGGL(k_boxa_eval, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, bp.pts_leaf.p, bp.pts_uv.p,
                           coef, out);
        check_launch(ctx, "k_boxa_eval");
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void box_refine(Context &ctx, int64_t n, const double *v16, const double *v64, double tol, int32_t *flags,
                double *err) {
    DevBuf<double> pv;
    const std::vector<double> h = fit_matrix();
    double *d = pv.ensure(h.size());
    YK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
    if (n > 0) {
        hipLaunchKernelGGL(k_box_refine, dim3(nblk(n, 128)), dim3(128), 0, ctx.stream, n, v16, v64, d, tol, flags,
                           err);
        check_launch(ctx, "k_box_refine");
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void box_leaf_eval(Context &ctx, const yk_grid &g, const double *vals, int64_t n, const double *xy, double *out) {
    YK_REQUIRE(g.nx % 4 == 0 && g.ny % 4 == 0, "the box code needs grid sides that are multiples of 4 cells");
    const int64_t nlx = g.nx / 4, nly = g.ny / 4, nleaf = nlx * nly;
    // (the fit matrix comes with the box plan of this grid)
    YK_REQUIRE(ctx.box && !ctx.box->adaptive && ctx.box->nx == g.nx && ctx.box->ny == g.ny && ctx.box->h == g.h &&
                   ctx.box->gx0 == g.x0 &&
                   ctx.box->gy0 == g.y0,
               "the leaf polynomials need the box plan of this grid (the box potential first)");
    BoxPlan &bp = *ctx.box;
    DevBuf<double> cbuf;
    double *coef = cbuf.ensure(nleaf * kNB);
    hipLaunchKernelGGL(k_box_fit, dim3(nblk(nleaf, 128)), dim3(128), 0, ctx.stream, nlx, nleaf, g.nx, vals,
                       bp.pinv.p, coef);
    check_launch(ctx, "k_box_fit");
    if (n > 0) {
        hipLaunchKernelGGL(k_box_eval, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, xy, g.x0, g.y0, g.h, nlx,
                           nly, coef, out);
        check_launch(ctx, "k_box_eval");
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

}  // namespace yk
