// near.hip -- the double layer at targets near the boundary.
//
// The trapezoid rule of Sec. 3.2 evaluates U^h = DL[w sigma] / alpha^2 to full
// accuracy only at targets farther from a curve than a few node spacings (its
// error decays like exp(-2 pi d / spacing)).  Closer targets are evaluated
// from the curve's trigonometric interpolant (Sec. 3.2 interpolates sigma in
// Fourier space):
//   * the target is projected onto the interpolated curve (Newton on
//     (y(theta) - p) . y'(theta) = 0 from the nearest node), giving theta*,
//     the distance d and the local node spacing s = |y'(theta*)| 2 pi / N;
//   * U^h is evaluated at K check points y(theta*) - k s n(theta*), k = 1..K,
//     along the inward normal, with the trapezoid rule on kNearM times as many
//     nodes (positions, normals and sigma interpolated), accurate there;
//   * the interior limit of U^h on the curve is g(theta*), the boundary
//     condition the integral equation imposes;
//   * the target's U^h is the degree-K polynomial in d / s through the K + 1
//     values at 0, 1, .., K.
// A target is treated this way when it lies on the domain side of the curve
// within kNearBand local spacings; candidates are the targets within
// kNearReach spacings of their nearest node.  The set, the projections, the
// check points and the finer nodes depend on the geometry only and are built
// once per (boundary, target set); each step costs two small DFTs per curve,
// an FMM from the finer nodes to the check points and one pass over the
// near targets.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "sums.h"
#include "yk_internal.h"

namespace yk {

constexpr int kNearK = 6;          // check points at 1..K spacings
constexpr int kNearM = 8;          // finer nodes per node
constexpr double kNearBand = 4.0;  // near targets: closer than this many spacings
constexpr double kNearReach = 5.0; // candidates: within this many spacings of their nearest node
constexpr double kTwoPi = 2.0 * kPi;

struct NearPlan {
    uint64_t bnd_gen = 0;
    const double *tgt = nullptr;
    int64_t n_tgt = 0;
    int64_t nb = 0;
    int n_curves = 0;
    std::vector<int64_t> off;
    DevBuf<int64_t> doff;            // node offsets per curve
    DevBuf<double> geo;              // [nb][4]: Fourier coefficients of x and y (re, im), per curve
    DevBuf<double> csign;            // [n_curves]: orientation of (y', -x') against the given normals
    int64_t n_fine = 0;
    DevBuf<double> fxy, fnrm, fw;    // finer nodes, curve by curve (offsets kNearM * off)
    int64_t n_near = 0;
    DevBuf<int64_t> idx;             // target index
    DevBuf<int32_t> cur;             // curve
    DevBuf<double> th, d, sp;        // theta*, distance, local spacing
    DevBuf<double> chk;              // [n_near * K][2]
    DevBuf<double> nxy;              // [n_near][2] target positions
    // per step
    DevBuf<double> scoef, gcoef;     // [nb][2]
    DevBuf<double> fdn;              // [n_fine][2]
    DevBuf<double> chk_val;          // [n_near * K]
    DevBuf<double> coarse;           // [n_near]
    DevBuf<double> gstar;            // [n_near] g(theta*)
    // curves whose node count is a power of two up to 2^kFftMaxLog take the
    // LDS FFTs, grouped by size; the others the direct sums (flag 1 = skip there)
    struct FftGroup {
        int logn = 0;
        int count = 0;
        DevBuf<int32_t> ids;
    };
    std::vector<std::unique_ptr<FftGroup>> fft;
    DevBuf<int8_t> fft_curve;        // [n_curves]: 1 when the curve takes the FFTs
    DevBuf<double> tw;               // [kTwHalf][2] butterfly factors
    bool any_direct = false;
    double setup_ms = 0;
};

void NearPlanDeleter::operator()(NearPlan *p) const { delete p; }

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ int find_curve(const int64_t *__restrict__ off, int n_curves, int64_t i, int64_t scale) {
    int lo = 0, hi = n_curves - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (scale * off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// c_k = (1/N) sum_j v_j exp(-2 pi i j k / N) for the node's own curve, k its
// index in the curve; v read with a stride, coefficients written at
// coef[i * cs + 2 * cc + {0, 1}]
__global__ void k_curve_dft(int64_t nb, int n_curves, const int64_t *__restrict__ off, const double *__restrict__ v,
                            int vs, int vc, double *__restrict__ coef, int cs, int cc,
                            const int8_t *__restrict__ skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int c = find_curve(off, n_curves, i, 1);
    if (skip && skip[c]) return;
    const int64_t base = off[c], N = off[c + 1] - base, k = i - base;
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        const int64_t m = (j * k) % N;
        double s, co;
        sincospi(-2.0 * (double)m / (double)N, &s, &co);
        const double x = v[(base + j) * vs + vc];
        re += x * co;
        im += x * s;
    }
    coef[i * cs + 2 * cc] = re / (double)N;
    coef[i * cs + 2 * cc + 1] = im / (double)N;
}

// Value and first two derivatives in theta of the real trigonometric
// interpolants whose coefficients are c[k * cs + 2 f + {0, 1}] for the NF
// fields f: c_0 + 2 sum_{0<k<N/2} Re(c_k e^{ik theta}) + [N even] c_{N/2} cos(N theta / 2).
// e^{ik theta} by complex recurrence, re-seeded from sincos every 32 modes.
template <int NF>
__device__ void series_eval(const double *__restrict__ c, int cs, int64_t N, double th, double (&v)[NF],
                            double (&d1)[NF], double (&d2)[NF]) {
    for (int f = 0; f < NF; ++f) {
        v[f] = c[2 * f];
        d1[f] = 0.0;
        d2[f] = 0.0;
    }
    const int64_t kmax = (N - 1) / 2;
    double s1, c1;
    sincos(th, &s1, &c1);
    double er = 1.0, ei = 0.0;   // e^{i k theta}, k = 0
    for (int64_t k = 1; k <= kmax; ++k) {
        if ((k & 31) == 0) {
            sincos((double)k * th, &ei, &er);
        } else {
            const double nr = er * c1 - ei * s1;
            ei = er * s1 + ei * c1;
            er = nr;
        }
        const double kk = (double)k;
        const double *ck = c + k * cs;
        for (int f = 0; f < NF; ++f) {
            const double a = ck[2 * f] * er - ck[2 * f + 1] * ei;   // Re(c_k e^{ik theta})
            const double b = ck[2 * f] * ei + ck[2 * f + 1] * er;   // Im(c_k e^{ik theta})
            v[f] += 2.0 * a;
            d1[f] -= 2.0 * kk * b;
            d2[f] -= 2.0 * kk * kk * a;
        }
    }
    if ((N & 1) == 0) {
        const double h = 0.5 * (double)N;
        double sh, ch;
        sincos(h * th, &sh, &ch);
        const double *cn = c + (N / 2) * cs;
        for (int f = 0; f < NF; ++f) {
            v[f] += cn[2 * f] * ch;
            d1[f] -= h * cn[2 * f] * sh;
            d2[f] -= h * h * cn[2 * f] * ch;
        }
    }
}

// per node: n_j . (y'_j, -x'_j) (the orientation of the parametrisation)
__global__ void k_orientation(int64_t nb, int n_curves, const int64_t *__restrict__ off,
                              const double *__restrict__ geo, const double *__restrict__ normal,
                              double *__restrict__ dot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int c = find_curve(off, n_curves, i, 1);
    const int64_t base = off[c], N = off[c + 1] - base;
    double v[2], d1[2], d2[2];
    series_eval<2>(geo + base * 4, 4, N, kTwoPi * (double)(i - base) / (double)N, v, d1, d2);
    dot[i] = normal[2 * i] * d1[1] - normal[2 * i + 1] * d1[0];
}

// Newton projection of candidate points onto their nearest node's curve
__global__ void k_project(int64_t nc, const int64_t *__restrict__ cpt, const int32_t *__restrict__ cnode,
                          const double *__restrict__ tgt, int n_curves, const int64_t *__restrict__ off,
                          const double *__restrict__ geo, const double *__restrict__ csign, double band,
                          double *__restrict__ th_out, double *__restrict__ d_out, double *__restrict__ sp_out,
                          int32_t *__restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int64_t p = cpt[i];
    const double px = tgt[2 * p], py = tgt[2 * p + 1];
    const int64_t j = cnode[i];
    const int c = find_curve(off, n_curves, j, 1);
    const int64_t base = off[c], N = off[c + 1] - base;
    const double *cf = geo + base * 4;
    double th = kTwoPi * (double)(j - base) / (double)N;
    double v[2], d1[2], d2[2];
    for (int it = 0; it < 40; ++it) {
        series_eval<2>(cf, 4, N, th, v, d1, d2);
        const double rx = v[0] - px, ry = v[1] - py;
        const double f = rx * d1[0] + ry * d1[1];
        const double fp = d1[0] * d1[0] + d1[1] * d1[1] + rx * d2[0] + ry * d2[1];
        const double step = f / fp;
        th -= step;
        if (fabs(step) < 1e-15) break;
    }
    th = fmod(th, kTwoPi);
    if (th < 0.0) th += kTwoPi;
    series_eval<2>(cf, 4, N, th, v, d1, d2);
    const double rx = px - v[0], ry = py - v[1];
    const double speed = sqrt(d1[0] * d1[0] + d1[1] * d1[1]);
    const double nx = csign[c] * d1[1] / speed, ny = -csign[c] * d1[0] / speed;
    const double d = sqrt(rx * rx + ry * ry);
    const double sp = speed * kTwoPi / (double)N;
    th_out[i] = th;
    d_out[i] = d;
    sp_out[i] = sp;
    // domain side (points on the curve count as inside) and within the band
    keep[i] = ((rx * nx + ry * ny <= 0.0 || d <= 1e-9 * sp) && d < band * sp) ? 1 : 0;
}

// finer nodes: position, outward normal and trapezoid weight
__global__ void k_fine_geometry(int64_t nf, int n_curves, const int64_t *__restrict__ off,
                                const double *__restrict__ geo, const double *__restrict__ csign,
                                double *__restrict__ fxy, double *__restrict__ fnrm, double *__restrict__ fw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int c = find_curve(off, n_curves, i, kNearM);
    const int64_t base = off[c], N = off[c + 1] - base, M = kNearM * N, k = i - kNearM * base;
    double v[2], d1[2], d2[2];
    series_eval<2>(geo + base * 4, 4, N, kTwoPi * (double)k / (double)M, v, d1, d2);
    const double speed = sqrt(d1[0] * d1[0] + d1[1] * d1[1]);
    fxy[2 * i] = v[0];
    fxy[2 * i + 1] = v[1];
    fnrm[2 * i] = csign[c] * d1[1] / speed;
    fnrm[2 * i + 1] = -csign[c] * d1[0] / speed;
    fw[i] = speed * kTwoPi / (double)M;
}

// check points y(theta*) - k s n(theta*), k = 1..K, and the target positions
__global__ void k_check_points(int64_t nn, const int64_t *__restrict__ idx, const int32_t *__restrict__ cur,
                               const double *__restrict__ th, const double *__restrict__ sp,
                               const double *__restrict__ tgt, const int64_t *__restrict__ off,
                               const double *__restrict__ geo, const double *__restrict__ csign,
                               double *__restrict__ chk, double *__restrict__ nxy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const int c = cur[i];
    const int64_t base = off[c], N = off[c + 1] - base;
    double v[2], d1[2], d2[2];
    series_eval<2>(geo + base * 4, 4, N, th[i], v, d1, d2);
    const double speed = sqrt(d1[0] * d1[0] + d1[1] * d1[1]);
    const double nx = csign[c] * d1[1] / speed, ny = -csign[c] * d1[0] / speed;
    for (int k = 1; k <= kNearK; ++k) {
        chk[2 * (i * kNearK + k - 1)] = v[0] - k * sp[i] * nx;
        chk[2 * (i * kNearK + k - 1) + 1] = v[1] - k * sp[i] * ny;
    }
    nxy[2 * i] = tgt[2 * idx[i]];
    nxy[2 * i + 1] = tgt[2 * idx[i] + 1];
}

// dipole vectors of the finer rule: w sigma(theta) n, sigma interpolated
__global__ void k_fine_dipoles(int64_t nf, int n_curves, const int64_t *__restrict__ off,
                               const double *__restrict__ scoef, const double *__restrict__ fnrm,
                               const double *__restrict__ fw, double *__restrict__ fdn,
                               const int8_t *__restrict__ skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int c = find_curve(off, n_curves, i, kNearM);
    if (skip && skip[c]) return;
    const int64_t base = off[c], N = off[c + 1] - base, M = kNearM * N, k = i - kNearM * base;
    double v[1], d1[1], d2[1];
    series_eval<1>(scoef + base * 2, 2, N, kTwoPi * (double)k / (double)M, v, d1, d2);
    const double s = fw[i] * v[0];
    fdn[2 * i] = s * fnrm[2 * i];
    fdn[2 * i + 1] = s * fnrm[2 * i + 1];
}

constexpr int kFftMinLog = 4, kFftMaxLog = 13;
constexpr int kTwHalf = 1 << (kFftMaxLog - 1);   // twiddles of the largest transform

// tw[k] = (cos, sin)(pi k / kTwHalf), k < kTwHalf: the butterflies' factors
// for every size, e^{-+ i pi k / half} = tw[k kTwHalf / half] (read, not
// recomputed per butterfly: an FP64 sincos costs far more than the butterfly)
__global__ void k_fft_twiddles(double *__restrict__ tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kTwHalf) return;
    double sn, cs;
    sincospi((double)k / (double)kTwHalf, &sn, &cs);
    tw[2 * k] = cs;
    tw[2 * k + 1] = sn;
}

// threads per workgroup of the LDS FFTs: the large transforms are the few
// long ones (one workgroup per curve), so they take more threads per stage
constexpr int fft_threads(int logn) { return logn >= 11 ? 1024 : 256; }

// The radix-2 stages of an in-place FFT of N = 2^LOGN points in LDS (input in
// bit-reversed order, decimation in time) by NT threads, factors
// e^{SIGN i pi k / half} from tw; each thread issues the loads of its
// butterflies' factors of a stage together, before their LDS work
template <int LOGN, int SIGN>
__device__ __forceinline__ void fft_stages(double *re, double *im, const double *__restrict__ tw) {
    constexpr int NT = fft_threads(LOGN), NBF = (1 << LOGN) / 2, BPT = (NBF + NT - 1) / NT;
    for (int s = 1; s <= LOGN; ++s) {
        const int half = 1 << (s - 1);
        double cs[BPT], sn[BPT];
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            // (k < half, so e < kTwHalf for every thread)
            const int e = ((threadIdx.x + NT * u) & (half - 1)) << (kFftMaxLog - s);
            cs[u] = tw[2 * e];
            sn[u] = SIGN * tw[2 * e + 1];
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int t = threadIdx.x + NT * u;
            if (NBF % NT == 0 || t < NBF) {
                const int k = t & (half - 1), i = ((t >> (s - 1)) << s) + k, j = i + half;
                const double tr = re[j] * cs[u] - im[j] * sn[u], ti = re[j] * sn[u] + im[j] * cs[u];
                re[j] = re[i] - tr;
                im[j] = im[i] - ti;
                re[i] += tr;
                im[i] += ti;
            }
        }
        __syncthreads();
    }
}

// Fourier coefficients c_k = (1/N) sum_j v_j e^{-2 pi i j k / N} of a curve
// whose N = 2^LOGN, by an in-place radix-2 FFT in LDS (input in bit-reversed
// order, decimation in time); one workgroup per (curve, field)
template <int LOGN>
__global__ __launch_bounds__(1024) void k_fft_coef(const int32_t *__restrict__ curves, const int64_t *__restrict__ off,
                                                  const double *__restrict__ v0, const double *__restrict__ v1,
                                                  const double *__restrict__ tw, double *__restrict__ c0,
                                                  double *__restrict__ c1) {
    constexpr int N = 1 << LOGN;
    __shared__ double re[N], im[N];
    const int64_t base = off[curves[blockIdx.x]];
    const double *v = blockIdx.y ? v1 : v0;
    double *cf = blockIdx.y ? c1 : c0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int j = (int)(__brev((unsigned)i) >> (32 - LOGN));
        re[j] = v[base + i];
        im[j] = 0.0;
    }
    __syncthreads();
    fft_stages<LOGN, -1>(re, im, tw);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        cf[2 * (base + i)] = re[i] * (1.0 / N);
        cf[2 * (base + i) + 1] = im[i] * (1.0 / N);
    }
}

// The interpolant at the finer nodes theta = 2 pi (m j + r) / (m N) as m
// inverse FFTs of size N of the shifted coefficients c_k e^{i kk phi},
// phi = 2 pi r / (m N), kk the signed mode (the Nyquist mode of an even N
// contributes c_{N/2} cos(N theta / 2)); one workgroup per (curve, r); writes
// the finer rule's dipole vectors w sigma n
template <int LOGN>
__global__ __launch_bounds__(1024) void k_fft_fine(const int32_t *__restrict__ curves, const int64_t *__restrict__ off,
                                                  const double *__restrict__ coef, const double *__restrict__ fnrm,
                                                  const double *__restrict__ fw, const double *__restrict__ tw,
                                                  double *__restrict__ fdn) {
    constexpr int N = 1 << LOGN;
    constexpr int M = kNearM * N;
    __shared__ double re[N], im[N];
    const int cidx = blockIdx.x / kNearM, r = blockIdx.x - cidx * kNearM;
    const int64_t base = off[curves[cidx]];
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const int j = (int)(__brev((unsigned)k) >> (32 - LOGN));
        const double a = coef[2 * (base + k)], b = coef[2 * (base + k) + 1];
        if (2 * k == N) {
            re[j] = a * cospi((double)r / kNearM);
            im[j] = 0.0;
        } else {
            const int kk = 2 * k < N ? k : k - N;
            double sn, cs;
            sincospi(2.0 * (double)kk * (double)r / (double)M, &sn, &cs);
            re[j] = a * cs - b * sn;
            im[j] = a * sn + b * cs;
        }
    }
    __syncthreads();
    fft_stages<LOGN, 1>(re, im, tw);
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const int64_t f = kNearM * base + (int64_t)kNearM * j + r;
        const double sgm = fw[f] * re[j];
        fdn[2 * f] = sgm * fnrm[2 * f];
        fdn[2 * f + 1] = sgm * fnrm[2 * f + 1];
    }
}

// g(theta*) at the near targets, one wavefront per target: lane l takes the
// modes k = 1 + l + 64 m (consecutive lanes read consecutive coefficients),
// e^{ik theta} by the recurrence of stride 64 re-seeded every 16 of a lane's
// modes, and the partial sums meet in a fixed shuffle tree
__global__ __launch_bounds__(256) void k_near_g(int64_t nn, const int32_t *__restrict__ cur,
                                                const double *__restrict__ th, const int64_t *__restrict__ off,
                                                const double *__restrict__ gcoef, double *__restrict__ gstar) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= nn) return;   // whole wavefronts leave together
    const int c = cur[w];
    const int64_t base = off[c], N = off[c + 1] - base, kmax = (N - 1) / 2;
    const double t = th[w];
    const double *cf = gcoef + 2 * base;
    double acc = 0.0;
    if (1 + lane <= kmax) {
        double s64, c64, ei = 0.0, er = 1.0;
        sincos(64.0 * t, &s64, &c64);
        int m = 0;
        for (int64_t k = 1 + lane; k <= kmax; k += 64, ++m) {
            if ((m & 15) == 0) {
                sincos((double)k * t, &ei, &er);
            } else {
                const double nr = er * c64 - ei * s64;
                ei = er * s64 + ei * c64;
                er = nr;
            }
            acc += 2.0 * (cf[2 * k] * er - cf[2 * k + 1] * ei);
        }
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) {
        double v = cf[0] + acc;
        if ((N & 1) == 0) v += cf[2 * (N / 2)] * cos(0.5 * (double)N * t);
        gstar[w] = v;
    }
}

// U^h at the near targets from the polynomial through (0, g(theta*)) and the
// check points, then out[idx] = (base[idx] or out[idx] - coarse / alpha^2) + U^h
__global__ void k_near_finish(int64_t nn, const int64_t *__restrict__ idx, const double *__restrict__ d,
                              const double *__restrict__ sp, const double *__restrict__ gstar,
                              const double *__restrict__ chk_val, const double *__restrict__ coarse,
                              const double *__restrict__ base_vals, double inv_a2, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double vals[kNearK + 1];
    vals[0] = gstar[i];
    for (int k = 1; k <= kNearK; ++k) vals[k] = chk_val[i * kNearK + k - 1] * inv_a2;
    const double t = d[i] / sp[i];
    double uh = 0.0;
    for (int k = 0; k <= kNearK; ++k) {
        double l = 1.0;
        for (int m = 0; m <= kNearK; ++m)
            if (m != k) l *= (t - (double)m) / (double)(k - m);
        uh += l * vals[k];
    }
    const int64_t p = idx[i];
    const double basev = base_vals ? base_vals[p] : out[p] - coarse[i] * inv_a2;
    out[p] = basev + uh;
}

using FftCoefKernel = void (*)(const int32_t *, const int64_t *, const double *, const double *, const double *,
                               double *, double *);
using FftFineKernel = void (*)(const int32_t *, const int64_t *, const double *, const double *, const double *,
                               const double *, double *);

FftCoefKernel fft_coef_kernel(int logn) {
    switch (logn) {
        case 4: return k_fft_coef<4>;
        case 5: return k_fft_coef<5>;
        case 6: return k_fft_coef<6>;
        case 7: return k_fft_coef<7>;
        case 8: return k_fft_coef<8>;
        case 9: return k_fft_coef<9>;
        case 10: return k_fft_coef<10>;
        case 11: return k_fft_coef<11>;
        case 12: return k_fft_coef<12>;
        default: return k_fft_coef<13>;
    }
}

FftFineKernel fft_fine_kernel(int logn) {
    switch (logn) {
        case 4: return k_fft_fine<4>;
        case 5: return k_fft_fine<5>;
        case 6: return k_fft_fine<6>;
        case 7: return k_fft_fine<7>;
        case 8: return k_fft_fine<8>;
        case 9: return k_fft_fine<9>;
        case 10: return k_fft_fine<10>;
        case 11: return k_fft_fine<11>;
        case 12: return k_fft_fine<12>;
        default: return k_fft_fine<13>;
    }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

int64_t near_count(const NearPlan &np) { return np.n_near; }
double near_setup_ms(const NearPlan &np) { return np.setup_ms; }

NearPlan &near_prepare(Context &ctx, BoundaryData &bd, int64_t n_tgt, const double *tgt) {
    NearPlan *cur = ctx.near.get();
    if (cur && cur->bnd_gen == bd.gen && cur->tgt == tgt && cur->n_tgt == n_tgt) return *cur;
    const auto t0 = std::chrono::steady_clock::now();
    ctx.near.reset();
    ctx.plan_near.reset();
    ctx.plan_nearc.reset();
    NearPtr np(new NearPlan());
    np->bnd_gen = bd.gen;
    np->tgt = tgt;
    np->n_tgt = n_tgt;
    np->nb = bd.n;
    np->n_curves = bd.n_curves;
    np->off = bd.offset;
    const int64_t nb = bd.n;
    const int nc = bd.n_curves;
    int64_t *doff = np->doff.ensure(nc + 1);
    YK_HIP(hipMemcpyAsync(doff, np->off.data(), (nc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
    // Fourier coefficients of the node positions and the orientation
    double *geo = np->geo.ensure((size_t)nb * 4);
    for (int comp = 0; comp < 2; ++comp) {
        hipLaunchKernelGGL(k_curve_dft, dim3(nblk(nb, 128)), dim3(128), 0, ctx.stream, nb, nc, doff, bd.xy, 2,
                           comp, geo, 4, comp, (const int8_t *)nullptr);
        check_launch(ctx, "k_curve_dft");
    }
    DevBuf<double> ddot;
    hipLaunchKernelGGL(k_orientation, dim3(nblk(nb, 128)), dim3(128), 0, ctx.stream, nb, nc, doff, geo,
                       bd.normal, ddot.ensure(nb));
    check_launch(ctx, "k_orientation");
    std::vector<double> hdot(nb), hxy(2 * nb), hw(nb), htgt(2 * n_tgt);
    YK_HIP(hipMemcpyAsync(hdot.data(), ddot.p, nb * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipMemcpyAsync(hxy.data(), bd.xy, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipMemcpyAsync(hw.data(), bd.w.p, nb * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipMemcpyAsync(htgt.data(), tgt, 2 * n_tgt * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    std::vector<double> sign(nc);
    for (int c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int64_t j = np->off[c]; j < np->off[c + 1]; ++j) s += hdot[j];
        sign[c] = s >= 0.0 ? 1.0 : -1.0;
    }
    double *dsign = np->csign.ensure(nc);
    YK_HIP(hipMemcpyAsync(dsign, sign.data(), nc * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
    // candidates: targets whose nearest node j (lowest index among equally
    // near ones) is closer than kNearReach w_j.  Targets and nodes are binned
    // in cells of the largest reach; each node records the targets within its
    // own reach, and a target's nearest recorded node is kept only when no
    // node at all is nearer (such a node would be outside its own reach).
    double wmax = 0.0, bx0 = INFINITY, by0 = INFINITY, bx1 = -INFINITY, by1 = -INFINITY;
    for (int64_t j = 0; j < nb; ++j) {
        wmax = std::max(wmax, hw[j]);
        bx0 = std::min(bx0, hxy[2 * j]);
        bx1 = std::max(bx1, hxy[2 * j]);
        by0 = std::min(by0, hxy[2 * j + 1]);
        by1 = std::max(by1, hxy[2 * j + 1]);
    }
    const double R = kNearReach * wmax;
    bx0 -= R; by0 -= R; bx1 += R; by1 += R;
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(2048, (int64_t)std::ceil((bx1 - bx0) / R)));
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(2048, (int64_t)std::ceil((by1 - by0) / R)));
    const double cw = (bx1 - bx0) / (double)gx, ch = (by1 - by0) / (double)gy;
    auto cell_of = [&](double x, double y, int64_t &ix, int64_t &iy) {
        ix = std::min<int64_t>(gx - 1, std::max<int64_t>(0, (int64_t)std::floor((x - bx0) / cw)));
        iy = std::min<int64_t>(gy - 1, std::max<int64_t>(0, (int64_t)std::floor((y - by0) / ch)));
    };
    auto bin = [&](const std::vector<double> &xy, int64_t n, std::vector<int64_t> &start, std::vector<int64_t> &items) {
        start.assign((size_t)(gx * gy + 1), 0);
        std::vector<int64_t> cell_id;
        std::vector<int64_t> ids;
        for (int64_t p = 0; p < n; ++p) {
            const double x = xy[2 * p], y = xy[2 * p + 1];
            if (!(x >= bx0 && x <= bx1 && y >= by0 && y <= by1)) continue;
            int64_t ix, iy;
            cell_of(x, y, ix, iy);
            ++start[iy * gx + ix + 1];
            ids.push_back(p);
            cell_id.push_back(iy * gx + ix);
        }
        for (int64_t k = 0; k < gx * gy; ++k) start[k + 1] += start[k];
        items.resize(ids.size());
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (size_t k = 0; k < ids.size(); ++k) items[fill[cell_id[k]]++] = ids[k];
    };
    std::vector<int64_t> pstart, pcell, nstart, ncell;
    bin(htgt, n_tgt, pstart, pcell);
    bin(hxy, nb, nstart, ncell);
    struct Hit {
        int64_t p;
        double d2;
        int32_t j;
    };
    std::vector<Hit> hits;
    for (int64_t j = 0; j < nb; ++j) {
        const double x = hxy[2 * j], y = hxy[2 * j + 1], rj = kNearReach * hw[j], rj2 = rj * rj;
        int64_t ix0, iy0, ix1, iy1;
        cell_of(x - rj, y - rj, ix0, iy0);
        cell_of(x + rj, y + rj, ix1, iy1);
        for (int64_t iy = iy0; iy <= iy1; ++iy)
            for (int64_t ix = ix0; ix <= ix1; ++ix)
                for (int64_t k = pstart[iy * gx + ix]; k < pstart[iy * gx + ix + 1]; ++k) {
                    const int64_t p = pcell[k];
                    const double dx = htgt[2 * p] - x, dy = htgt[2 * p + 1] - y;
                    const double d2 = dx * dx + dy * dy;
                    if (d2 < rj2) hits.push_back({p, d2, (int32_t)j});
                }
    }
    std::sort(hits.begin(), hits.end(), [](const Hit &a, const Hit &b) {
        if (a.p != b.p) return a.p < b.p;
        if (a.d2 != b.d2) return a.d2 < b.d2;
        return a.j < b.j;
    });
    std::vector<int64_t> cpt;
    std::vector<int32_t> cnode;
    for (size_t k = 0; k < hits.size(); ++k) {
        if (k > 0 && hits[k].p == hits[k - 1].p) continue;
        const int64_t p = hits[k].p;
        const double px = htgt[2 * p], py = htgt[2 * p + 1], d2 = hits[k].d2, d = std::sqrt(d2);
        bool nearest = true;
        int64_t ix0, iy0, ix1, iy1;
        cell_of(px - d, py - d, ix0, iy0);
        cell_of(px + d, py + d, ix1, iy1);
        for (int64_t iy = iy0; iy <= iy1 && nearest; ++iy)
            for (int64_t ix = ix0; ix <= ix1 && nearest; ++ix)
                for (int64_t q = nstart[iy * gx + ix]; q < nstart[iy * gx + ix + 1]; ++q) {
                    const int64_t m = ncell[q];
                    const double dx = px - hxy[2 * m], dy = py - hxy[2 * m + 1];
                    const double e2 = dx * dx + dy * dy;
                    if (e2 < d2 || (e2 == d2 && m < hits[k].j)) {
                        nearest = false;
                        break;
                    }
                }
        if (nearest) {
            cpt.push_back(p);
            cnode.push_back(hits[k].j);
        }
    }
    const int64_t ncand = (int64_t)cpt.size();
    std::vector<int64_t> hidx;
    std::vector<int32_t> hcur;
    std::vector<double> hth, hd, hsp;
    if (ncand > 0) {
        DevBuf<int64_t> dcpt;
        DevBuf<int32_t> dcnode, dkeep;
        DevBuf<double> dth, dd, dsp;
        YK_HIP(hipMemcpyAsync(dcpt.ensure(ncand), cpt.data(), ncand * sizeof(int64_t), hipMemcpyHostToDevice,
                              ctx.stream));
        YK_HIP(hipMemcpyAsync(dcnode.ensure(ncand), cnode.data(), ncand * sizeof(int32_t), hipMemcpyHostToDevice,
                              ctx.stream));
        hipLaunchKernelGGL(k_project, dim3(nblk(ncand, 64)), dim3(64), 0, ctx.stream, ncand, dcpt.p, dcnode.p, tgt,
                           nc, doff, geo, dsign, kNearBand, dth.ensure(ncand), dd.ensure(ncand),
                           dsp.ensure(ncand), dkeep.ensure(ncand));
        check_launch(ctx, "k_project");
        std::vector<double> pth(ncand), pd(ncand), psp(ncand);
        std::vector<int32_t> pkeep(ncand);
        YK_HIP(hipMemcpyAsync(pth.data(), dth.p, ncand * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipMemcpyAsync(pd.data(), dd.p, ncand * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipMemcpyAsync(psp.data(), dsp.p, ncand * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipMemcpyAsync(pkeep.data(), dkeep.p, ncand * sizeof(int32_t), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
        std::vector<int32_t> node_curve(nb);
        for (int c = 0; c < nc; ++c)
            for (int64_t j = np->off[c]; j < np->off[c + 1]; ++j) node_curve[j] = c;
        for (int64_t k = 0; k < ncand; ++k)
            if (pkeep[k]) {
                hidx.push_back(cpt[k]);
                hcur.push_back(node_curve[cnode[k]]);
                hth.push_back(pth[k]);
                hd.push_back(pd[k]);
                hsp.push_back(psp[k]);
            }
    }
    const int64_t nn = (int64_t)hidx.size();
    np->n_near = nn;
    if (nn > 0) {
        YK_HIP(hipMemcpyAsync(np->idx.ensure(nn), hidx.data(), nn * sizeof(int64_t), hipMemcpyHostToDevice,
                              ctx.stream));
        YK_HIP(hipMemcpyAsync(np->cur.ensure(nn), hcur.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice,
                              ctx.stream));
        YK_HIP(hipMemcpyAsync(np->th.ensure(nn), hth.data(), nn * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyAsync(np->d.ensure(nn), hd.data(), nn * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
        YK_HIP(hipMemcpyAsync(np->sp.ensure(nn), hsp.data(), nn * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
        hipLaunchKernelGGL(k_check_points, dim3(nblk(nn, 128)), dim3(128), 0, ctx.stream, nn, np->idx.p, np->cur.p,
                           np->th.p, np->sp.p, tgt, doff, geo, dsign, np->chk.ensure((size_t)nn * kNearK * 2),
                           np->nxy.ensure((size_t)nn * 2));
        check_launch(ctx, "k_check_points");
        np->n_fine = (int64_t)kNearM * nb;
        hipLaunchKernelGGL(k_fine_geometry, dim3(nblk(np->n_fine, 128)), dim3(128), 0, ctx.stream, np->n_fine, nc,
                           doff, geo, dsign, np->fxy.ensure((size_t)np->n_fine * 2),
                           np->fnrm.ensure((size_t)np->n_fine * 2), np->fw.ensure(np->n_fine));
        check_launch(ctx, "k_fine_geometry");
    }
    // curves for the LDS FFTs, by size
    {
        std::vector<int8_t> flag(nc, 0);
        std::vector<std::vector<int32_t>> by(kFftMaxLog + 1);
        for (int c = 0; c < nc; ++c) {
            const int64_t N = np->off[c + 1] - np->off[c];
            int lg = 0;
            while (((int64_t)1 << lg) < N) ++lg;
            if (((int64_t)1 << lg) == N && lg >= kFftMinLog && lg <= kFftMaxLog) {
                by[lg].push_back(c);
                flag[c] = 1;
            } else {
                np->any_direct = true;
            }
        }
        for (int lg = kFftMinLog; lg <= kFftMaxLog; ++lg) {
            if (by[lg].empty()) continue;
            auto gr = std::make_unique<NearPlan::FftGroup>();
            gr->logn = lg;
            gr->count = (int)by[lg].size();
            YK_HIP(hipMemcpyAsync(gr->ids.ensure(gr->count), by[lg].data(), gr->count * sizeof(int32_t),
                                  hipMemcpyHostToDevice, ctx.stream));
            np->fft.push_back(std::move(gr));
        }
        YK_HIP(hipMemcpyAsync(np->fft_curve.ensure(nc), flag.data(), nc, hipMemcpyHostToDevice, ctx.stream));
        if (!np->fft.empty()) {
            hipLaunchKernelGGL(k_fft_twiddles, dim3(nblk(kTwHalf, 256)), dim3(256), 0, ctx.stream,
                               np->tw.ensure(2 * (size_t)kTwHalf));
            check_launch(ctx, "k_fft_twiddles");
        }
    }
    YK_HIP(hipStreamSynchronize(ctx.stream));
    np->setup_ms = ms_since(t0);
    ctx.near = std::move(np);
    return *ctx.near;
}

void near_apply(Context &ctx, NearPlan &np, BoundaryData &bd, double alpha, const double *sigma, const double *g,
                const double *base, double *out) {
    const int64_t nn = np.n_near, nb = np.nb;
    if (nn == 0) return;
    const int nc = np.n_curves;
    double *sc = np.scoef.ensure((size_t)nb * 2), *gc = np.gcoef.ensure((size_t)nb * 2);
    double *fdn = np.fdn.ensure((size_t)np.n_fine * 2);
    // Fourier coefficients of sigma and g, and sigma's finer-rule dipoles:
    // LDS FFTs for power-of-two curves, direct sums for the others
    for (const auto &gp : np.fft) {
        const NearPlan::FftGroup &gr = *gp;
        hipLaunchKernelGGL(fft_coef_kernel(gr.logn), dim3(gr.count, 2), dim3(fft_threads(gr.logn)), 0, ctx.stream,
                           gr.ids.p, np.doff.p, sigma, g, np.tw.p, sc, gc);
        check_launch(ctx, "k_fft_coef");
        hipLaunchKernelGGL(fft_fine_kernel(gr.logn), dim3(gr.count * kNearM), dim3(fft_threads(gr.logn)), 0,
                           ctx.stream, gr.ids.p, np.doff.p, sc, np.fnrm.p, np.fw.p, np.tw.p, fdn);
        check_launch(ctx, "k_fft_fine");
    }
    if (np.any_direct) {
        const int8_t *skip = np.fft_curve.p;
        hipLaunchKernelGGL(k_curve_dft, dim3(nblk(nb, 128)), dim3(128), 0, ctx.stream, nb, nc, np.doff.p, sigma, 1,
                           0, sc, 2, 0, skip);
        check_launch(ctx, "k_curve_dft");
        hipLaunchKernelGGL(k_curve_dft, dim3(nblk(nb, 128)), dim3(128), 0, ctx.stream, nb, nc, np.doff.p, g, 1, 0,
                           gc, 2, 0, skip);
        check_launch(ctx, "k_curve_dft");
        hipLaunchKernelGGL(k_fine_dipoles, dim3(nblk(np.n_fine, 128)), dim3(128), 0, ctx.stream, np.n_fine, nc,
                           np.doff.p, sc, np.fnrm.p, np.fw.p, fdn, skip);
        check_launch(ctx, "k_fine_dipoles");
    }
    double *gs = np.gstar.ensure(nn);
    hipLaunchKernelGGL(k_near_g, dim3(nblk(nn * 64, 256)), dim3(256), 0, ctx.stream, nn, np.cur.p, np.th.p,
                       np.doff.p, gc, gs);
    check_launch(ctx, "k_near_g");
    // U^h (without 1/alpha^2) at the check points from the finer rule
    double *cv = np.chk_val.ensure((size_t)nn * kNearK);
    {
        SumProblem pb;
        pb.n[1] = np.n_fine;
        pb.xy[1] = np.fxy.p;
        pb.normal = np.fnrm.p;
        pb.n[2] = nn * kNearK;
        pb.xy[2] = np.chk.p;
        pb.alpha = alpha;
        double *outs[3] = {nullptr, nullptr, cv};
        evaluate_sums(ctx, SLOT_NEAR, pb, nullptr, fdn, outs, SUM_FP64);
    }
    // the coarse rule's value at the targets, to be replaced
    double *coarse = nullptr;
    if (!base) {
        coarse = np.coarse.ensure(nn);
        double *dn = ctx.dn.ensure(2 * nb);
        launch_dipole_vectors(ctx, nb, bd.w.p, sigma, bd.normal, 1.0, dn);
        SumProblem pb;
        pb.n[1] = nb;
        pb.xy[1] = bd.xy;
        pb.normal = bd.normal;
        pb.n[2] = nn;
        pb.xy[2] = np.nxy.p;
        pb.alpha = alpha;
        double *outs[3] = {nullptr, nullptr, coarse};
        evaluate_sums(ctx, SLOT_NEARC, pb, nullptr, dn, outs, SUM_FP64);
    }
    hipLaunchKernelGGL(k_near_finish, dim3(nblk(nn, 128)), dim3(128), 0, ctx.stream, nn, np.idx.p, np.d.p,
                       np.sp.p, gs, cv, coarse, base, 1.0 / (alpha * alpha), out);
    check_launch(ctx, "k_near_finish");
}

}  // namespace yk
