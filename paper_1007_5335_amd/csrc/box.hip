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
#include <cmath>
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

// multipole of leaf box li (its single point is the centre of grid leaf
// perm[lrange[li][0]]): M[o] = sum_k coef[k] Q[k][o]; one workgroup of Pp lanes
__global__ void k_box_p2m(int64_t leaf_base, const int32_t *__restrict__ lrange, const int32_t *__restrict__ perm,
                          const double *__restrict__ coef, const double *__restrict__ Q, int Pp,
                          double *__restrict__ M) {
    const int64_t li = blockIdx.x;
    const int o = threadIdx.x;
    const int64_t g = perm[lrange[li * 6]];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kNB; ++k) s = __builtin_fma(coef[g * kNB + k], Q[k * Pp + o], s);
    M[(leaf_base + li) * Pp + o] = s;
}

// V at the 16 cells of every leaf: near field from the U list (the leaf and
// its existing neighbours) by the tables A[offset][cell][k], far field from
// the leaf's local expansion by E[cell][o]; 4 leaves per 64-lane workgroup
__global__ __launch_bounds__(64) void k_box_leaf(
    int64_t nl, int64_t leaf_base, const int32_t *__restrict__ lrange, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist, int64_t nlx, int64_t nx,
    const double *__restrict__ coef, const double *__restrict__ A, const double *__restrict__ E,
    const double *__restrict__ Lc, int Pp, int far, double *__restrict__ V) {
    const int64_t li = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 4);
    const int t = threadIdx.x & 15;
    if (li >= nl) return;
    const int64_t g = perm[lrange[li * 6]];
    const int64_t I = g % nlx, J = g / nlx;
    double acc = 0.0;
    for (int32_t u = uoff[li]; u < uoff[li + 1]; ++u) {
        const int64_t gs = perm[lrange[(int64_t)ulist[u] * 6]];
        const int dI = (int)(gs % nlx - I), dJ = (int)(gs / nlx - J);
        const double *a = A + ((size_t)((dJ + 1) * 3 + dI + 1) * kNC + t) * kNB;
        const double *c = coef + gs * kNB;
#pragma unroll
        for (int k = 0; k < kNB; ++k) acc = __builtin_fma(a[k], c[k], acc);
    }
    if (far) {
        const double *Lb = Lc + (leaf_base + li) * Pp;
        const double *e = E + (size_t)t * Pp;
        double s = 0.0;
        for (int o = 0; o < Pp; ++o) s = __builtin_fma(e[o], Lb[o], s);
        acc += s * kInv2Pi;
    }
    V[(4 * J + (t >> 2)) * nx + 4 * I + (t & 3)] = acc;
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
};

void BoxPlanDeleter::operator()(BoxPlan *p) const { delete p; }

namespace {

// host tables of a box plan: the fit, the near-field integrals, the leaf
// moments and the local-expansion evaluation at the cells
void box_tables(Context &ctx, BoxPlan &bp) {
    const double h = bp.h, al = bp.alpha, H = 2.0 * h;
    // least-squares fit: pinv = (V^T V)^{-1} V^T, V[t][k] = m_k at cell t
    {
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
        YK_HIP(hipMemcpyAsync(bp.pinv.ensure(pv.size()), pv.data(), pv.size() * sizeof(double),
                              hipMemcpyHostToDevice, ctx.stream));
    }
    // near field: A[off][t][k] = (1/2pi) int_source-leaf K0(|x_t - y|/alpha) m_k((y - c)/H) dy
    {
        std::vector<double> gx, gw, px, pw;
        gauss01(16, gx, gw);
        gauss01(32, px, pw);
        std::vector<double> A((size_t)kNOff * kNC * kNB, 0.0);
        host_parallel(kNOff * kNC, [&](int64_t i0, int64_t i1) {
            for (int64_t job = i0; job < i1; ++job) {
                const int off = (int)(job / kNC), t = (int)(job % kNC);
                const int dI = off % 3 - 1, dJ = off / 3 - 1;
                // target relative to the source leaf's centre
                const double tx = -4.0 * h * dI + ((t & 3) - 1.5) * h;
                const double ty = -4.0 * h * dJ + ((t >> 2) - 1.5) * h;
                long double acc[kNB] = {};
                double m[kNB], mt[kNB];
                monomials(tx / H, ty / H, mt);
                for (int cj = 0; cj < 4; ++cj)
                    for (int ci = 0; ci < 4; ++ci) {
                        const double ccx = (ci - 1.5) * h, ccy = (cj - 1.5) * h;
                        if (off == 4 && ci == (t & 3) && cj == (t >> 2)) {
                            // the target's own cell, about its centre: per edge
                            // (distance h/2) the angles within pi/4 of its normal
                            for (int e = 0; e < 4; ++e) {
                                const double thn = e * 0.5 * kPi;
                                for (int a = 0; a < (int)px.size(); ++a) {
                                    const double th = thn + (px[a] - 0.5) * 0.5 * kPi, wth = pw[a] * 0.5 * kPi;
                                    const double R = 0.5 * h / std::cos(th - thn);
                                    const double c = std::cos(th), sn = std::sin(th);
                                    const double base = al * al - al * R * k1(R / al);
                                    for (int k = 0; k < kNB; ++k) acc[k] += (long double)wth * mt[k] * base;
                                    // the rest, m(x_t + r e) - m(x_t) = O(r): r = R s^2
                                    for (int b = 0; b < (int)px.size(); ++b) {
                                        const double sr = px[b], r = R * sr * sr, jac = 2.0 * R * sr;
                                        monomials((tx + r * c) / H, (ty + r * sn) / H, m);
                                        const double f = wth * pw[b] * k0(r / al) * r * jac;
                                        for (int k = 0; k < kNB; ++k) acc[k] += (long double)f * (m[k] - mt[k]);
                                    }
                                }
                            }
                        } else {
                            for (int a = 0; a < (int)gx.size(); ++a)
                                for (int b = 0; b < (int)gx.size(); ++b) {
                                    const double yx = ccx + (gx[a] - 0.5) * h, yy = ccy + (gx[b] - 0.5) * h;
                                    const double f = gw[a] * gw[b] * h * h * k0(std::hypot(tx - yx, ty - yy) / al);
                                    monomials(yx / H, yy / H, m);
                                    for (int k = 0; k < kNB; ++k) acc[k] += (long double)f * m[k];
                                }
                        }
                    }
                for (int k = 0; k < kNB; ++k) A[((size_t)off * kNC + t) * kNB + k] = (double)(acc[k] * kInv2Pi);
            }
        });
        YK_HIP(hipMemcpyAsync(bp.A.ensure(A.size()), A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
    }
    // far field: Q[k][o], the leaf's monomial moments against
    // conj(F^I_n(y/alpha)) / I_n(R) in the real layout of the multipoles, and
    // E[t][o], the weights of the stored local coefficients (Lh_m = L_m I_m(R))
    // in the local expansion's value at cell t
    if (bp.far) {
        const FmmPlan &pl = *bp.fmm;
        const int p = pl.p, Pp = pl.Pp;
        const long double R = pl.lev[pl.L].R;
        const std::vector<long double> IR = bessel_i_seq(R, p + 1);
        std::vector<double> gx, gw;
        gauss01(24, gx, gw);
        std::vector<double> Q((size_t)kNB * Pp, 0.0), E((size_t)kNC * Pp, 0.0);
        std::vector<long double> Ql((size_t)kNB * Pp, 0.0L);
        double m[kNB];
        for (int a = 0; a < (int)gx.size(); ++a)
            for (int b = 0; b < (int)gx.size(); ++b) {
                const double yx = (2.0 * gx[a] - 1.0) * H, yy = (2.0 * gx[b] - 1.0) * H;
                const long double wq = (long double)gw[a] * gw[b] * 4.0L * H * H;
                monomials(yx / H, yy / H, m);
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
        for (size_t i = 0; i < Q.size(); ++i) Q[i] = (double)Ql[i];
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
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

BoxPlan &box_plan(Context &ctx, const yk_grid &g, double alpha) {
    if (ctx.box && ctx.box->gx0 == g.x0 && ctx.box->gy0 == g.y0 && ctx.box->h == g.h && ctx.box->nx == g.nx &&
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
            hipLaunchKernelGGL(k_box_p2m, dim3((unsigned)pl.nleaf), dim3(pl.Pp), 0, ctx.stream, leaf_base,
                               pl.lrange.p, pl.perm.p, coef, bp.Q.p, pl.Pp, pl.M.p);
            check_launch(ctx, "k_box_p2m");
        }
        fmm_m2m(ctx, pl);
        launch_fill(ctx, (int64_t)pl.nbox * pl.Pp, 0.0, pl.Lc.p);
        fmm_m2l(ctx, pl, as, false);
        fmm_l2l(ctx, pl, as, false);
    }
    StageTimer tl(ctx, YK_STAGE_LEAF);
    hipLaunchKernelGGL(k_box_leaf, dim3(nblk(pl.nleaf, 4)), dim3(64), 0, ctx.stream, pl.nleaf, leaf_base,
                       pl.lrange.p, pl.perm.p, pl.ulist_off.p, pl.ulist.p, bp.nlx, bp.nx, coef, bp.A.p,
                       bp.far ? bp.E.p : nullptr, pl.Lc.p, pl.Pp, bp.far ? 1 : 0, V);
    check_launch(ctx, "k_box_leaf");
}

void box_leaf_eval(Context &ctx, const yk_grid &g, const double *vals, int64_t n, const double *xy, double *out) {
    YK_REQUIRE(g.nx % 4 == 0 && g.ny % 4 == 0, "the box code needs grid sides that are multiples of 4 cells");
    const int64_t nlx = g.nx / 4, nly = g.ny / 4, nleaf = nlx * nly;
    // (the fit matrix comes with the box plan of this grid)
    YK_REQUIRE(ctx.box && ctx.box->nx == g.nx && ctx.box->ny == g.ny && ctx.box->h == g.h && ctx.box->gx0 == g.x0 &&
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
