// kernels_elem.hip -- direct sums and elementwise kernels (FP64).
#include <algorithm>

#include "yk_bessel.h"
#include "yk_internal.h"

namespace yk {

namespace {

constexpr int kDirectBlock = 256;

// All-pairs sum: one target per thread, sources staged through LDS in tiles.
// Charges contribute q K0(z)/(2pi); dipoles contribute (x - y).dn K1(z)/(alpha^2 z)/(2pi),
// z = r/alpha.  Pairs at distance zero are skipped (self pairs included).
// With gridDim.y > 1 the sources are split into gridDim.y contiguous chunks
// (one per blockIdx.y) and each chunk's raw sum goes to part[chunk][target],
// for k_direct_reduce to add in chunk order (few targets, many sources).
__global__ __launch_bounds__(kDirectBlock) void k_direct(
    int64_t nt, const double *__restrict__ txy, int64_t ns, const double *__restrict__ sxy,
    const double *__restrict__ q, int64_t nb, const double *__restrict__ bxy,
    const double *__restrict__ dn, double inv4a2, double inva2, double *__restrict__ out,
    int accumulate, double *__restrict__ part) {
    __shared__ double sx[kDirectBlock], sy[kDirectBlock], sq[kDirectBlock], sn[kDirectBlock];
    const int64_t i = (int64_t)blockIdx.x * kDirectBlock + threadIdx.x;
    const bool live = i < nt;
    const double x = live ? txy[2 * i] : 0.0;
    const double y = live ? txy[2 * i + 1] : 0.0;
    const int64_t c = blockIdx.y, nc = gridDim.y;
    const int64_t qs0 = c * ns / nc, qs1 = (c + 1) * ns / nc;
    const int64_t bs0 = c * nb / nc, bs1 = (c + 1) * nb / nc;
    double acc = 0.0;
    for (int64_t s0 = qs0; s0 < qs1; s0 += kDirectBlock) {
        const int64_t j = s0 + threadIdx.x;
        if (j < qs1) {
            sx[threadIdx.x] = sxy[2 * j];
            sy[threadIdx.x] = sxy[2 * j + 1];
            sq[threadIdx.x] = q[j];
        }
        __syncthreads();
        const int cnt = (int)min<int64_t>(kDirectBlock, qs1 - s0);
        for (int k = 0; k < cnt; ++k) {
            const double dx = x - sx[k], dy = y - sy[k];
            const double r2 = dx * dx + dy * dy;
            if (r2 > 0.0) acc += sq[k] * k0_of_t(r2 * inv4a2);
        }
        __syncthreads();
    }
    for (int64_t s0 = bs0; s0 < bs1; s0 += kDirectBlock) {
        const int64_t j = s0 + threadIdx.x;
        if (j < bs1) {
            sx[threadIdx.x] = bxy[2 * j];
            sy[threadIdx.x] = bxy[2 * j + 1];
            sq[threadIdx.x] = dn[2 * j];
            sn[threadIdx.x] = dn[2 * j + 1];
        }
        __syncthreads();
        const int cnt = (int)min<int64_t>(kDirectBlock, bs1 - s0);
        for (int k = 0; k < cnt; ++k) {
            const double dx = x - sx[k], dy = y - sy[k];
            const double r2 = dx * dx + dy * dy;
            if (r2 > 0.0) acc += (dx * sq[k] + dy * sn[k]) * inva2 * k1oz_of_t(r2 * inv4a2);
        }
        __syncthreads();
    }
    if (live) {
        if (part) {
            part[c * nt + i] = acc;
        } else {
            const double v = acc * kInv2Pi;
            out[i] = accumulate ? out[i] + v : v;
        }
    }
}

__global__ void k_direct_reduce(int64_t nt, int nchunk, const double *__restrict__ part, double *__restrict__ out,
                                int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * nt + i];
    const double v = acc * kInv2Pi;
    out[i] = accumulate ? out[i] + v : v;
}

__global__ void k_dipole_vectors(int64_t n, const double *__restrict__ w,
                                 const double *__restrict__ sigma,
                                 const double *__restrict__ normal, double scale,
                                 double *__restrict__ dn) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = scale * (w ? w[i] : 1.0) * sigma[i];
    dn[2 * i] = s * normal[2 * i];
    dn[2 * i + 1] = s * normal[2 * i + 1];
}

__global__ void k_dl_diagonal(int64_t n, const double *__restrict__ w,
                              const double *__restrict__ kappa, double inv_a2, const double *__restrict__ sigma,
                              double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] += dl_diag_weight(w[i], kappa[i], inv_a2) * sigma[i];
}

__global__ void k_bie_combine(int64_t n, const double *__restrict__ x,
                              const double *__restrict__ dl, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = x[i] - 2.0 * dl[i];
}

// y = x - 2 (dl + diagonal x): the corrected diagonal and the combination of
// the second-kind operator in one pass
__global__ void k_bie_finish(int64_t n, const double *__restrict__ w, const double *__restrict__ kappa,
                             double inv_a2, const double *__restrict__ x, const double *__restrict__ dl,
                             double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = x[i] - 2.0 * (dl[i] + dl_diag_weight(w[i], kappa[i], inv_a2) * x[i]);
}

__global__ void k_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    o[i] = a[i] * b[i];
}

__global__ void k_axpby(int64_t n, double ca, const double *__restrict__ a, double cb,
                        const double *__restrict__ b, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    o[i] = b ? ca * a[i] + cb * b[i] : ca * a[i];
}

// 32-point Gauss-Legendre rule on [-1, 1] (nodes and weights filled on the host).
__constant__ double c_gl_x[32];
__constant__ double c_gl_w[32];

// out[i] = scale * (out[i] + B[i] * c(h_i)), where
// c(h) = (1/2pi) * 8 * int_0^{pi/4} (alpha^2 - alpha R K1(R/alpha)) dtheta,
// R = (h/2)/cos(theta), h = sqrt(vol_w[i]): the kernel integrated over the
// target's own square cell (8 right triangles with apex at the centre).  When
// all points of a wavefront share one cell size (a uniform grid) the 32 nodes
// of the rule are spread over the lanes and c(h) is formed once per wavefront.
// The own-cell weight w0 of a grid point (U^p = (V + B w0) / alpha^2): the
// weight that makes the lattice rule exact for constant B, the kernel
// K0 / (2 pi alpha^2) integrating to 1 over the plane:
//   w0 = alpha^2 - (h^2 / 2 pi) sum_{j != 0} K0(|j| eps),  eps = h / alpha,
// the sum over the nonzero points of the square lattice with |j| eps <= 40
// (the rest is below 1e-17 of it), taken by the lattice's eight-fold
// symmetry.  Below eps = 0.005 (more than 10^7 terms) its expansion is used:
// the cell integral plus kappa h^2.  Near the target the kernel is
// -(1/2pi) log|x| times a smooth factor psi; the punctured lattice sum of
// log|x| psi misses h^2 psi(0) (log h + Z'(0)/2) (generalised Euler-Maclaurin
// expansion of lattice sums; Z(s) = 4 zeta(s) beta(s) is the Epstein zeta
// function of the square lattice, Z'(0)/2 = log(4 pi)/2 - 2 log Gamma(1/4)),
// while the cell integral supplies h^2 psi(0) (log h + c_cell) with
// c_cell = (pi/2 - 3 - log 2) / 2, so kappa = (c_cell - Z'(0)/2) / (2 pi).
// The expansion's relative error is about 0.04 eps^2.
constexpr double kLatticeSelf = 0.039686478567495465;
constexpr double kSelfSeriesBelow = 0.005;
constexpr double kLatticeReach = 40.0;

__device__ __forceinline__ double self_cell_node(int k, double h, double alpha) {
    const double th = (c_gl_x[k] + 1.0) * (kPi / 8.0);
    const double R = 0.5 * h / cos(th);
    return c_gl_w[k] * (alpha * alpha - alpha * R * k1(R / alpha));
}

// one block of 256 per cell size: w0[d] for the squared side h2[d]
__global__ __launch_bounds__(256) void k_self_weights(int nd, const double *__restrict__ h2, double alpha,
                                                      double *__restrict__ w0) {
    __shared__ double red[256];
    const int d = blockIdx.x;
    if (d >= nd) return;
    const double h = sqrt(h2[d]), eps = h / alpha;
    double s = 0.0;
    if (eps < kSelfSeriesBelow) {
        if (threadIdx.x < 32) s = self_cell_node(threadIdx.x, h, alpha);
    } else {
        const int64_t A = (int64_t)floor(kLatticeReach / eps);
        for (int64_t a = 1 + threadIdx.x; a <= A; a += blockDim.x) {
            const double ra = (double)a * eps;
            double t = 4.0 * k0(ra);
            const double rd = 1.4142135623730951 * ra;
            if (rd <= kLatticeReach) t += 4.0 * k0(rd);
            for (int64_t b = 1; b < a; ++b) {
                const double r = sqrt((double)(a * a + b * b)) * eps;
                if (r > kLatticeReach) break;
                t += 8.0 * k0(r);
            }
            s += t;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (eps < kSelfSeriesBelow)
            w0[d] = (8.0 * (kPi / 8.0) * kInv2Pi) * red[0] + kLatticeSelf * h2[d];
        else
            w0[d] = alpha * alpha - h2[d] * kInv2Pi * red[0];
    }
}

// out = scale (out + B w0[idx]) (idx NULL: one size, w0[0])
__global__ void k_self_cell(int64_t n, const uint16_t *__restrict__ idx, const double *__restrict__ w0,
                            const double *__restrict__ B, double scale, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = scale * (out[i] + B[i] * w0[idx ? idx[i] : 0]);
}

__global__ void k_grid_points(int64_t n, double x0, double y0, double h, int64_t nx, double *__restrict__ xy) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t j = k / nx, i = k - j * nx;
    xy[2 * k] = x0 + ((double)i + 0.5) * h;
    xy[2 * k + 1] = y0 + ((double)j + 0.5) * h;
}

// cubic Lagrange weights on the nodes -1, 0, 1, 2 at t in [0, 1)
__device__ __forceinline__ void cubic_weights(double t, double w[4]) {
    w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
    w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
    w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
    w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

// tensor cubic interpolation of cell-centre values: for a coordinate x the
// stencil is the centres i0 - 1 .. i0 + 2, i0 = floor((x - x0)/h - 1/2)
// (the host checks that every stencil lies inside the grid; indices are
// clamped all the same)
__global__ void k_bicubic(int64_t n, const double *__restrict__ xy, double x0, double y0, double h, int64_t nx,
                          int64_t ny, const double *__restrict__ V, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double sx = (xy[2 * k] - x0) / h - 0.5, sy = (xy[2 * k + 1] - y0) / h - 0.5;
    const double fx = floor(sx), fy = floor(sy);
    double wx[4], wy[4];
    cubic_weights(sx - fx, wx);
    cubic_weights(sy - fy, wy);
    const int64_t ix = (int64_t)fx, iy = (int64_t)fy;
    double acc = 0.0;
    for (int b = 0; b < 4; ++b) {
        const int64_t r = min(max(iy + b - 1, (int64_t)0), ny - 1);
        double row = 0.0;
        for (int a = 0; a < 4; ++a) {
            const int64_t cidx = min(max(ix + a - 1, (int64_t)0), nx - 1);
            row += wx[a] * V[r * nx + cidx];
        }
        acc += wy[b] * row;
    }
    out[k] = acc;
}

__global__ void k_rhs_be(int64_t n, const double *__restrict__ u, const double *__restrict__ F,
                         const int32_t *__restrict__ region, int n_const,
                         const double *__restrict__ c, double dt, double *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = region[i];
    if (r < 0)
        B[i] = u[i] + (F ? dt * F[i] : 0.0);
    else
        B[i] = (r < n_const) ? c[r] : 0.0;
}

// B of the linearly implicit schemes (Sec. 2): with ub the extended u (u inside
// the domain, the enclosing curve's constant elsewhere) and f = F + R(ub),
//   Euler: B = ub + dt f
//   Gear:  B = 4/3 ub - 1/3 ub' + dt (4/3 f - 2/3 f')   (primes: step N - 1)
// R = u (1 - u^2) for the Allen-Cahn reaction, else 0.
__global__ void k_rhs_imex(int64_t n, int gear, int allen_cahn, const double *__restrict__ u,
                           const double *__restrict__ up, const double *__restrict__ F,
                           const double *__restrict__ Fp, const int32_t *__restrict__ region, int n_const,
                           const double *__restrict__ c, double dt, double *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = region[i];
    const double cr = (r >= 0 && r < n_const) ? c[r] : 0.0;
    const double u0 = r < 0 ? u[i] : cr;
    const double f0 = (F ? F[i] : 0.0) + (allen_cahn ? u0 * (1.0 - u0 * u0) : 0.0);
    if (!gear) {
        B[i] = u0 + dt * f0;
        return;
    }
    const double u1 = r < 0 ? up[i] : cr;
    const double f1 = (Fp ? Fp[i] : 0.0) + (allen_cahn ? u1 * (1.0 - u1 * u1) : 0.0);
    B[i] = (4.0 / 3.0) * u0 - (1.0 / 3.0) * u1 + dt * ((4.0 / 3.0) * f0 - (2.0 / 3.0) * f1);
}

__global__ void k_boundary_prep(int64_t n, int n_curves, const int64_t *__restrict__ off,
                                const double *__restrict__ speed, double *__restrict__ w,
                                int32_t *__restrict__ curve, int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_curves - 1;
    while (lo < hi) {   // last curve k with off[k] <= i
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int64_t nk = off[lo + 1] - off[lo];
    w[i] = (2.0 * kPi / (double)nk) * speed[i];
    curve[i] = lo;
    idx[i] = (int32_t)(i - off[lo]);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_direct(Context &ctx, int64_t nt, const double *txy, int64_t ns, const double *sxy,
                   const double *q, int64_t nb, const double *bxy, const double *dn, double alpha,
                   double *out, bool accumulate) {
    if (nt <= 0) return;
    const double inv4a2 = 1.0 / (4.0 * alpha * alpha), inva2 = 1.0 / (alpha * alpha);
    // few targets against many sources (sampled checks): the sources are
    // split into chunks of at least 8192 so the launch fills the GPU, and the
    // chunks' sums are added in a fixed order.  (Square problems, such as the
    // density operator with the nodes as targets and sources, keep one chunk.)
    const int64_t nsrc = ns + nb;
    int nchunk = 1;
    if (nt <= 4096 && nsrc >= 65536) nchunk = (int)std::min<int64_t>(512, nsrc / 8192);
    if (nchunk > 1) {
        double *part = ctx.direct_part.ensure((size_t)nchunk * nt);
        hipLaunchKernelGGL(k_direct, dim3(nblk(nt, kDirectBlock), nchunk), dim3(kDirectBlock), 0, ctx.stream, nt,
                           txy, ns, sxy, q, nb, bxy, dn, inv4a2, inva2, out, 0, part);
        check_launch(ctx, "k_direct");
        hipLaunchKernelGGL(k_direct_reduce, dim3(nblk(nt, 256)), dim3(256), 0, ctx.stream, nt, nchunk, part, out,
                           accumulate ? 1 : 0);
        check_launch(ctx, "k_direct_reduce");
        return;
    }
    hipLaunchKernelGGL(k_direct, dim3(nblk(nt, kDirectBlock)), dim3(kDirectBlock), 0, ctx.stream,
                       nt, txy, ns, sxy, q, nb, bxy, dn, inv4a2, inva2, out, accumulate ? 1 : 0, (double *)nullptr);
    check_launch(ctx, "k_direct");
}

void launch_dipole_vectors(Context &ctx, int64_t n, const double *w, const double *sigma,
                           const double *normal, double scale, double *dn) {
    hipLaunchKernelGGL(k_dipole_vectors, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, w, sigma,
                       normal, scale, dn);
    check_launch(ctx, "k_dipole_vectors");
}

void launch_dl_diagonal(Context &ctx, int64_t n, const double *w, const double *kappa, double alpha,
                        const double *sigma, double *out) {
    hipLaunchKernelGGL(k_dl_diagonal, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, w, kappa,
                       1.0 / (alpha * alpha), sigma, out);
    check_launch(ctx, "k_dl_diagonal");
}

void launch_bie_combine(Context &ctx, int64_t n, const double *x, const double *dl, double *y) {
    hipLaunchKernelGGL(k_bie_combine, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, x, dl, y);
    check_launch(ctx, "k_bie_combine");
}

void launch_bie_finish(Context &ctx, int64_t n, const double *w, const double *kappa, double alpha,
                       const double *x, const double *dl, double *y) {
    hipLaunchKernelGGL(k_bie_finish, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, w, kappa,
                       1.0 / (alpha * alpha), x, dl, y);
    check_launch(ctx, "k_bie_finish");
}

void launch_mul(Context &ctx, int64_t n, const double *a, const double *b, double *out) {
    hipLaunchKernelGGL(k_mul, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, a, b, out);
    check_launch(ctx, "k_mul");
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

void launch_fill(Context &ctx, int64_t n, double v, double *out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, v, out);
    check_launch(ctx, "k_fill");
}

__global__ void k_differs(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                          int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && __double_as_longlong(a[i]) != __double_as_longlong(b[i])) *flag = 1;
}

void launch_differs(Context &ctx, int64_t n, const double *a, const double *b, int *flag) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_differs, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, a, b, flag);
    check_launch(ctx, "k_differs");
}

void launch_axpby(Context &ctx, int64_t n, double ca, const double *a, double cb, const double *b,
                  double *out) {
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, ca, a, cb, b, out);
    check_launch(ctx, "k_axpby");
}

static void gauss_legendre32(double *x, double *w) {
    // Newton iteration on P_32 from the asymptotic initial guesses.
    const int n = 32;
    for (int i = 0; i < n; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
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
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

void launch_grid_points(Context &ctx, int64_t n, double x0, double y0, double h, int64_t nx, double *xy) {
    hipLaunchKernelGGL(k_grid_points, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, x0, y0, h, nx, xy);
    check_launch(ctx, "k_grid_points");
}

void launch_bicubic(Context &ctx, int64_t n, const double *xy, double x0, double y0, double h, int64_t nx,
                    int64_t ny, const double *V, double *out) {
    hipLaunchKernelGGL(k_bicubic, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, xy, x0, y0, h, nx, ny, V, out);
    check_launch(ctx, "k_bicubic");
}

void launch_self_weights(Context &ctx, int nd, const double *h2, double alpha, double *w0) {
    static bool ready = false;
    static double gx[32], gw[32];
    if (!ready) {
        gauss_legendre32(gx, gw);
        ready = true;
    }
    YK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_gl_x), gx, sizeof(gx), 0, hipMemcpyHostToDevice, ctx.stream));
    YK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_gl_w), gw, sizeof(gw), 0, hipMemcpyHostToDevice, ctx.stream));
    hipLaunchKernelGGL(k_self_weights, dim3(nd), dim3(256), 0, ctx.stream, nd, h2, alpha, w0);
    check_launch(ctx, "k_self_weights");
}

void launch_self_cell(Context &ctx, int64_t n, const uint16_t *idx, const double *w0, const double *B, double scale,
                      double *out_accum) {
    hipLaunchKernelGGL(k_self_cell, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, idx, w0, B, scale, out_accum);
    check_launch(ctx, "k_self_cell");
}

void launch_rhs_be(Context &ctx, int64_t n, const double *u, const double *F, const int32_t *region,
                   int n_const, const double *c_dev, double dt, double *B) {
    hipLaunchKernelGGL(k_rhs_be, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, u, F, region,
                       n_const, c_dev, dt, B);
    check_launch(ctx, "k_rhs_be");
}

void launch_rhs_imex(Context &ctx, int64_t n, bool gear, bool allen_cahn, const double *u, const double *up,
                     const double *F, const double *Fp, const int32_t *region, int n_const, const double *c_dev,
                     double dt, double *B) {
    hipLaunchKernelGGL(k_rhs_imex, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, gear ? 1 : 0,
                       allen_cahn ? 1 : 0, u, up, F, Fp, region, n_const, c_dev, dt, B);
    check_launch(ctx, "k_rhs_imex");
}

void launch_boundary_prep(Context &ctx, int64_t n, int n_curves, const int64_t *off_dev,
                          const double *speed, double *w, int32_t *curve, int32_t *idx) {
    hipLaunchKernelGGL(k_boundary_prep, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, n_curves,
                       off_dev, speed, w, curve, idx);
    check_launch(ctx, "k_boundary_prep");
}

}  // namespace yk
