// fmm_kernels.hip -- upward pass, M2L, downward pass and near field of the
// modified-Helmholtz FMM (expansion conventions in fmm.h), FP64.
#include <climits>
#include <type_traits>

#include "fmm.h"
#include "yk_bessel.h"

namespace yk {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Consecutive workgroups are dealt round-robin to the 8 XCDs, each with its
// own L2.  Remapping block b so that every XCD walks one contiguous range of
// the (Morton-ordered) work list keeps neighbouring boxes' data in one L2.
// The map is a bijection on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, i = b / kXcd;
    const int q = n / kXcd, r = n % kXcd;
    return x * q + min(x, r) + i;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- gathers --
__global__ void k_gather_q(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ q,
                           double *__restrict__ qs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) qs[k] = q[perm[k]];
}

__global__ void k_gather_dn(int64_t off, int64_t n, const int32_t *__restrict__ perm,
                            const double *__restrict__ dn, double *__restrict__ dns) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = perm[off + k];
    dns[2 * k] = dn[2 * i];
    dns[2 * k + 1] = dn[2 * i + 1];
}

// the same with the dipole vectors formed on the way: dn_i = w_i sigma_i n_i
__global__ void k_gather_dn_form(int64_t off, int64_t n, const int32_t *__restrict__ perm,
                                 const double *__restrict__ w, const double *__restrict__ sigma,
                                 const double *__restrict__ normal, double *__restrict__ dns) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = perm[off + k];
    const double s = 1.0 * (w ? w[i] : 1.0) * sigma[i];
    dns[2 * k] = s * normal[2 * i];
    dns[2 * k + 1] = s * normal[2 * i + 1];
}

__global__ void k_scatter_out(int64_t off, int64_t n, const int32_t *__restrict__ perm,
                              const double *__restrict__ outs, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[perm[off + k]] = outs[off + k];
}

// ------------------------------------------------------------ F_n helpers --
// F_n(y) = sum_k y^k/(k!(n+1)_k): the two starting values F_{p+1}, F_{p+2} by
// their series; below that, F_n = F_{n+1} + y F_{n+2} / ((n+1)(n+2)) (the
// three-term recurrence of I_n, stable downwards).
__device__ __forceinline__ void f_start(double y, const double *__restrict__ sc, int nser,
                                        double &Fn1, double &Fn2) {
    double a = sc[nser - 1], b = sc[2 * nser - 1];
    for (int k = nser - 2; k >= 0; --k) {
        a = a * y + sc[k];
        b = b * y + sc[nser + k];
    }
    Fn1 = a;   // F_{p+1}
    Fn2 = b;   // F_{p+2}
}

// ------------------------------------------------------------------- P2M ---
// One wavefront serves four leaves, 16 lanes (one DPP row) each; lanes over
// source points.  Each lane builds G_n = F_n(y)/F_n(Y) for n = 0..p+1 in its
// own LDS column (downwards), then the terms of every order are summed over
// the row with DPP (no LDS round trip); the lane whose index matches the
// output's position mod 16 stores the batch sum, and the batch sums are then
// accumulated in registers, output o = lane + 16 k.  The level's tables
// (F-series coefficients, recurrence factors, normalisations, dipole weights)
// are staged in LDS so the order loops read no scalar memory.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// sum over the 16 lanes of a row, in every lane of the row
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
    return v;
}

constexpr int kP2MSlots = 8;   // outputs per lane: Pp <= 128

// NMAX > 0: orders known to be at most NMAX - 1 (Pp <= 2 NMAX), so G_n lives
// in registers and the order loops unroll; NMAX = 0: G_n in LDS, any order.
template <int NMAX>
__global__ __launch_bounds__(64) void k_p2m(
    int64_t leaf_base, int64_t nleaf, const int32_t *__restrict__ lrange,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ qs, const double *__restrict__ dns,
    int64_t off1, int has_q, int has_d, double inv_alpha, double invR,
    const double *__restrict__ invFY, const double *__restrict__ da, const double *__restrict__ db,
    const double *__restrict__ cnn, const double *__restrict__ sc, int nser, int p, int Pp,
    double *__restrict__ M) {
    constexpr bool kReg = NMAX > 0;
    extern __shared__ double smem[];
    double *G = smem;                                  // [(p+2)][64] (LDS form only)
    double *s_out = G + (kReg ? 0 : (p + 2) * 64);     // [4][Pp] row sums of one batch
    double *t_sc = s_out + 4 * Pp;                     // [2 nser] F_{p+1}, F_{p+2} series
    double *t_cnn = t_sc + 2 * nser;                   // [p+2]
    double *t_ify = t_cnn + (p + 2);                   // [p+2]
    double *t_da = t_ify + (p + 2);                    // [p+1]
    double *t_db = t_da + (p + 1);                     // [p+1]
    const int lane = threadIdx.x, grp = lane >> 4, gl = lane & 15;
    const int64_t li = (int64_t)blockIdx.x * 4 + grp;
    const bool leaf_ok = li < nleaf;
    const int64_t b = leaf_base + (leaf_ok ? li : 0);
    const int P = 2 * p + 1, nk = Pp >> 4;
    for (int k = lane; k < 2 * nser; k += 64) t_sc[k] = sc[k];
    for (int k = lane; k < p + 2; k += 64) {
        t_cnn[k] = cnn[k];
        t_ify[k] = invFY[k];
    }
    if (has_d)
        for (int k = lane; k < p + 1; k += 64) {
            t_da[k] = da[k];
            t_db[k] = db[k];
        }
    double *So = s_out + grp * Pp;
    double macc[kP2MSlots];
#pragma unroll
    for (int k = 0; k < kP2MSlots; ++k) macc[k] = 0.0;
    double Gr[kReg ? NMAX + 2 : 1];
    __syncthreads();
    const double cx = bcx[b], cy = bcy[b];
    // G_n of this lane's point, register or LDS form
    auto gget = [&](int n) -> double {
        if constexpr (kReg) return Gr[n];
        else return G[n * 64 + lane];
    };
    for (int set = 0; set < 2; ++set) {
        if ((set == 0 && !has_q) || (set == 1 && !has_d)) continue;
        const int s0 = leaf_ok ? lrange[li * 6 + 2 * set] : 0;
        const int e0 = leaf_ok ? lrange[li * 6 + 2 * set + 1] : 0;
        // uniform trip count over the four groups
        int nmax = e0 - s0;
        nmax = max(nmax, __shfl_xor(nmax, 16, 64));
        nmax = max(nmax, __shfl_xor(nmax, 32, 64));
        for (int base = 0; base < nmax; base += 16) {
            const int j = s0 + base + gl;
            const bool valid = j < e0;
            const int jc = valid ? j : (e0 > s0 ? s0 : (set == 0 ? 0 : (int)off1));   // weight 0 below
            const double wx = valid ? (px[jc] - cx) * inv_alpha : 0.0;
            const double wy = valid ? (py[jc] - cy) * inv_alpha : 0.0;
            const double y = 0.25 * (wx * wx + wy * wy);
            const double zx = wx * invR, zy = -wy * invR;   // conj(w)/R
            double F1, F2;
            f_start(y, t_sc, nser, F1, F2);
            if constexpr (kReg) {
#pragma unroll
                for (int n = NMAX + 1; n >= 0; --n) {
                    if (n > p + 1) continue;
                    if (n == p + 1) {
                        Gr[n] = F1 * t_ify[n];
                    } else {
                        const double F0 = F1 + y * F2 * t_cnn[n];
                        Gr[n] = F0 * t_ify[n];
                        F2 = F1;
                        F1 = F0;
                    }
                }
            } else {
                G[(p + 1) * 64 + lane] = F1 * t_ify[p + 1];
                for (int n = p; n >= 0; --n) {
                    const double F0 = F1 + y * F2 * t_cnn[n];
                    G[n * 64 + lane] = F0 * t_ify[n];
                    F2 = F1;
                    F1 = F0;
                }
            }
            // the row sum of order n goes to output 2n-1 (real) and 2n (imaginary)
            auto emit = [&](int n, double tr, double ti) {
                tr = row16_sum(tr);
                ti = row16_sum(ti);
                const int orr = n == 0 ? 0 : 2 * n - 1;
                if (gl == (orr & 15)) So[orr] = tr;
                if (n > 0 && gl == ((2 * n) & 15)) So[2 * n] = ti;
            };
            if (set == 0) {
                const double q = valid ? qs[jc] : 0.0;
                double pr = 1.0, pi = 0.0;     // conj(z)^n
                auto body = [&](int n) {
                    const double g = q * gget(n);
                    emit(n, g * pr, g * pi);
                    const double nr = pr * zx - pi * zy;
                    pi = pr * zy + pi * zx;
                    pr = nr;
                };
                if constexpr (kReg) {
#pragma unroll
                    for (int n = 0; n < NMAX; ++n)
                        if (n <= p) body(n);
                } else {
                    for (int n = 0; n <= p; ++n) body(n);
                }
            } else {
                const double Dx = valid ? dns[2 * (jc - off1)] : 0.0;
                const double Dy = valid ? dns[2 * (jc - off1) + 1] : 0.0;
                const double h = 0.5 * inv_alpha;
                // window Psi_{n-1}, Psi_n, Psi_{n+1};  Psi_k = G_k conj(z)^k
                double pr = zx, pi = zy;                       // conj(z)^1
                const double g1 = gget(1);
                double c_r = gget(0), c_i = 0.0;               // Psi_0
                double n_r = g1 * pr, n_i = g1 * pi;           // Psi_1
                double m_r = n_r, m_i = -n_i;                  // Psi_{-1} = conj(Psi_1)
                auto body = [&](int n) {
                    // term_n = h [a_n D Psi_{n+1} + b_n conj(D) Psi_{n-1}]
                    const double an = t_da[n], bn = t_db[n];
                    const double t1r = Dx * n_r - Dy * n_i, t1i = Dx * n_i + Dy * n_r;
                    const double t2r = Dx * m_r + Dy * m_i, t2i = Dx * m_i - Dy * m_r;
                    emit(n, h * (an * t1r + bn * t2r), h * (an * t1i + bn * t2i));
                    m_r = c_r; m_i = c_i;
                    c_r = n_r; c_i = n_i;
                    const double nr = pr * zx - pi * zy;
                    pi = pr * zy + pi * zx;
                    pr = nr;
                    if (n + 2 <= p + 1) {
                        const double g = gget(n + 2);
                        n_r = g * pr; n_i = g * pi;
                    } else {
                        n_r = 0.0; n_i = 0.0;
                    }
                };
                if constexpr (kReg) {
#pragma unroll
                    for (int n = 0; n < NMAX; ++n)
                        if (n <= p) body(n);
                } else {
                    for (int n = 0; n <= p; ++n) body(n);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kP2MSlots; ++k)
                if (k < nk && gl + 16 * k < P) macc[k] += So[gl + 16 * k];
            __syncthreads();
        }
    }
    if (leaf_ok)
#pragma unroll
        for (int k = 0; k < kP2MSlots; ++k)
            if (k < nk) M[b * Pp + gl + 16 * k] = gl + 16 * k < P ? macc[k] : 0.0;
}

// P2M with LPL lanes per leaf (4: a DPP quad; 32: half a wavefront) for a compile-time
// order PO: each lane takes every LPL-th point of its leaf and accumulates all
// 2p+1 outputs in registers; the lanes' partial sums are combined at the end
// (DPP steps for a quad, shuffles otherwise).  Per point: F_n downwards
// (G_n = F_n(y)/F_n(Y) in registers), then the terms with the powers of
// conj(z) upwards.
template <int PO, int LPL>
__global__ __launch_bounds__(64) void k_p2m_quad(
    int64_t leaf_base, int64_t nleaf, const int32_t *__restrict__ lrange,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ qs, const double *__restrict__ dns,
    int64_t off1, int has_q, int has_d, double inv_alpha, double invR,
    const double *__restrict__ invFY, const double *__restrict__ da, const double *__restrict__ db,
    const double *__restrict__ cnn, const double *__restrict__ sc, int nser, int /*p*/, int Pp,
    double *__restrict__ M, const int32_t *__restrict__ leaf_list, int accumulate) {
    constexpr int p = PO, P = 2 * PO + 1;
    extern __shared__ double smem[];
    double *t_sc = smem;                   // [2 nser] F_{p+1}, F_{p+2} series
    double *t_cnn = t_sc + 2 * nser;       // [p+2]
    double *t_ify = t_cnn + (p + 2);       // [p+2]
    double *t_da = t_ify + (p + 2);        // [p+1]
    double *t_db = t_da + (p + 1);         // [p+1]
    constexpr int LPB = 64 / LPL;           // leaves per block
    const int lane = threadIdx.x, q4 = lane % LPL;
    // leaf_list (optional): the leaves to serve, nleaf of them
    const int64_t lidx = (int64_t)blockIdx.x * LPB + lane / LPL;
    const bool leaf_ok = lidx < nleaf;
    const int64_t li = leaf_ok ? (leaf_list ? (int64_t)leaf_list[lidx] : lidx) : 0;
    const int64_t b = leaf_base + li;
    for (int k = lane; k < 2 * nser; k += 64) t_sc[k] = sc[k];
    for (int k = lane; k < p + 2; k += 64) {
        t_cnn[k] = cnn[k];
        t_ify[k] = invFY[k];
    }
    if (has_d)
        for (int k = lane; k < p + 1; k += 64) {
            t_da[k] = da[k];
            t_db[k] = db[k];
        }
    double acc[P];
#pragma unroll
    for (int o = 0; o < P; ++o) acc[o] = 0.0;
    double G[p + 2];
    __syncthreads();
    const double cx = bcx[b], cy = bcy[b];
    for (int set = 0; set < 2; ++set) {
        if ((set == 0 && !has_q) || (set == 1 && !has_d)) continue;
        const int s0 = leaf_ok ? lrange[li * 6 + 2 * set] : 0;
        const int e0 = leaf_ok ? lrange[li * 6 + 2 * set + 1] : 0;
        // a lane without a point reads a point of its own set (weight 0
        // below): the leaf's first, else the set's first (index 0 or off1)
        auto clamp_j = [&](int j) { return j < e0 ? j : (e0 > s0 ? s0 : (set == 0 ? 0 : (int)off1)); };
        // the next point's coordinates are loaded one iteration ahead
        int jn = clamp_j(s0 + q4);
        double nx = px[jn], ny = py[jn];
        for (int j0 = s0;; j0 += LPL) {
            const int j = j0 + q4;
            const bool valid = j < e0;
            if (!__any(valid)) break;
            const int jc = jn;
            const double cxp = nx, cyp = ny;
            jn = clamp_j(j + LPL);
            nx = px[jn];
            ny = py[jn];
            const double wx = (cxp - cx) * inv_alpha, wy = (cyp - cy) * inv_alpha;
            const double y = 0.25 * (wx * wx + wy * wy);
            const double zx = wx * invR, zy = -wy * invR;   // conj(w)/R
            double F1, F2;
            f_start(y, t_sc, nser, F1, F2);
            // G_n for n = 0..p+1 (n = p+1 only for the dipole window)
            G[p + 1] = F1 * t_ify[p + 1];
#pragma unroll
            for (int n = p; n >= 0; --n) {
                const double F0 = F1 + y * F2 * t_cnn[n];
                G[n] = F0 * t_ify[n];
                F2 = F1;
                F1 = F0;
            }
            if (set == 0) {
                const double qv = valid ? qs[jc] : 0.0;
                double pr = 1.0, pi = 0.0;     // conj(z)^n
#pragma unroll
                for (int n = 0; n <= p; ++n) {
                    const double g = qv * G[n];
                    if (n == 0) {
                        acc[0] += g;
                    } else {
                        acc[2 * n - 1] = __builtin_fma(g, pr, acc[2 * n - 1]);
                        acc[2 * n] = __builtin_fma(g, pi, acc[2 * n]);
                    }
                    const double nr = pr * zx - pi * zy;
                    pi = pr * zy + pi * zx;
                    pr = nr;
                }
            } else {
                const double h = valid ? 0.5 * inv_alpha : 0.0;
                const double Dx = h * dns[2 * (jc - off1)], Dy = h * dns[2 * (jc - off1) + 1];
                // window Psi_{n-1}, Psi_n, Psi_{n+1};  Psi_k = G_k conj(z)^k
                double pr = zx, pi = zy;                       // conj(z)^1
                double c_r = G[0], c_i = 0.0;                  // Psi_0
                double n_r = G[1] * pr, n_i = G[1] * pi;       // Psi_1
                double m_r = n_r, m_i = -n_i;                  // Psi_{-1} = conj(Psi_1)
#pragma unroll
                for (int n = 0; n <= p; ++n) {
                    // term_n = h [a_n D Psi_{n+1} + b_n conj(D) Psi_{n-1}]  (h folded into D)
                    const double an = t_da[n], bn = t_db[n];
                    const double t1r = Dx * n_r - Dy * n_i, t1i = Dx * n_i + Dy * n_r;
                    const double t2r = Dx * m_r + Dy * m_i, t2i = Dx * m_i - Dy * m_r;
                    if (n == 0) {
                        acc[0] += an * t1r + bn * t2r;
                    } else {
                        acc[2 * n - 1] += an * t1r + bn * t2r;
                        acc[2 * n] += an * t1i + bn * t2i;
                    }
                    m_r = c_r; m_i = c_i;
                    c_r = n_r; c_i = n_i;
                    const double nr = pr * zx - pi * zy;
                    pi = pr * zy + pi * zx;
                    pr = nr;
                    if (n + 2 <= p + 1) {
                        n_r = G[n + 2] * pr; n_i = G[n + 2] * pi;
                    } else {
                        n_r = 0.0; n_i = 0.0;
                    }
                }
            }
        }
    }
    // sums over the leaf's lanes; lane q4 writes outputs q4, q4 + LPL, ...
#pragma unroll
    for (int o = 0; o < P; ++o) {
        double v = acc[o];
        if constexpr (LPL == 4) {
            v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
            v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
        } else {
#pragma unroll
            for (int m = LPL / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, LPL);
        }
        if (leaf_ok && o % LPL == q4) M[b * Pp + o] = accumulate ? M[b * Pp + o] + v : v;
    }
    if (leaf_ok && !accumulate)
        for (int o = P + q4; o < Pp; o += LPL) M[b * Pp + o] = 0.0;
}

// Charges-only P2M in two halves of the orders: blockIdx.y = 0 takes orders
// 0..NS-1, blockIdx.y = 1 orders NS..p (NS = (p+1)/2), so each wavefront holds
// half the accumulators and half the G_n and more wavefronts fit a SIMD.  As
// in k_p2m_quad, four lanes per leaf over its points and DPP quad sums.  The
// upper half starts its powers at conj(z)^NS by repeated squaring and stops
// its downward F recurrence at NS.  Writes every entry of the leaves'
// multipoles (padding included); dipoles are added afterwards.  The blocks
// also clear zero[0..nzero) on the side (the local expansions, so that no
// launch of its own is needed).
constexpr int kP2MStage = 384;   // charges staged in LDS per block and round

template <int PO, int H>
__device__ __forceinline__ void p2m_half_body(
    int64_t leaf_base, int64_t nleaf, const int32_t *__restrict__ lrange,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ qs, int has_q, double inv_alpha,
    double invR, const double *t_ify, const double *t_cnn, const double *t_sc, int nser, int Pp,
    double *__restrict__ M, double *sx, double *sy, double *sq, int skip_d) {
    constexpr int p = PO, NS = (PO + 1) / 2;
    constexpr int N0 = H == 0 ? 0 : NS, N1 = H == 0 ? NS - 1 : p;   // orders of this half
    constexpr int O0 = H == 0 ? 0 : 2 * NS - 1;                      // its first output
    constexpr int NA = H == 0 ? 2 * NS - 1 : 2 * (p - NS + 1);       // its outputs
    constexpr int NG = N1 - N0 + 1;
    const int lane = threadIdx.x, q4 = lane & 3;
    const int64_t l0 = (int64_t)blockIdx.x * 16;
    const int64_t li = l0 + (lane >> 2);
    // (with skip_d, leaves that hold dipoles are left to the dipole pass)
    const bool leaf_ok = li < nleaf && !(skip_d && lrange[li * 6 + 3] > lrange[li * 6 + 2]);
    const int64_t b = leaf_base + (leaf_ok ? li : 0);
    double acc[NA];
#pragma unroll
    for (int o = 0; o < NA; ++o) acc[o] = 0.0;
    double G[NG];
    const double cx = bcx[b], cy = bcy[b];
    const int s0 = leaf_ok ? lrange[li * 6] : 0;
    const int e0 = (leaf_ok && has_q) ? lrange[li * 6 + 1] : s0;
    // the charges of the block's leaves (consecutive in Morton order, so one
    // run, up to the charges of leaves left to the dipole pass) are staged in
    // LDS in rounds of kP2MStage: one memory round trip per round, not per
    // point.  The run's ends come from the leaves that hold charges (an empty
    // range carries no position).
    int pbeg = e0 > s0 ? s0 : INT_MAX, pend = e0 > s0 ? e0 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        pbeg = min(pbeg, __shfl_xor(pbeg, m, 64));
        pend = max(pend, __shfl_xor(pend, m, 64));
    }
    for (int cs = pbeg; cs < pend; cs += kP2MStage) {
        const int cn = min(kP2MStage, pend - cs);
        __syncthreads();
        for (int k = lane; k < cn; k += 64) {
            sx[k] = px[cs + k];
            sy[k] = py[cs + k];
            sq[k] = qs[cs + k];
        }
        __syncthreads();
        // this lane's points j = s0 + q4 + 4k that fall in [cs, cs + cn)
        int j = s0 + q4;
        if (j < cs) j += (cs - j + 3) / 4 * 4;
        for (;; j += 4) {
            const bool valid = j < e0 && j < cs + cn;
            if (!__any(valid)) break;
            const int jl = valid ? j - cs : 0;
            const double qv = valid ? sq[jl] : 0.0;
            const double wx = (sx[jl] - cx) * inv_alpha, wy = (sy[jl] - cy) * inv_alpha;
            const double y = 0.25 * (wx * wx + wy * wy);
            const double zx = wx * invR, zy = -wy * invR;   // conj(w)/R
            double F1, F2;
            f_start(y, t_sc, nser, F1, F2);
#pragma unroll
            for (int n = p; n >= N0; --n) {
                const double F0 = F1 + y * F2 * t_cnn[n];
                if (n <= N1) G[n - N0] = F0 * t_ify[n];
                F2 = F1;
                F1 = F0;
            }
            // conj(z)^N0
            double pr = 1.0, pi = 0.0;
            {
                double br = zx, bi = zy;
#pragma unroll
                for (int bit = 0; bit < 6; ++bit) {
                    if ((N0 >> bit) & 1) {
                        const double nr = pr * br - pi * bi;
                        pi = pr * bi + pi * br;
                        pr = nr;
                    }
                    if ((N0 >> (bit + 1)) != 0) {
                        const double nr = br * br - bi * bi;
                        bi = 2.0 * br * bi;
                        br = nr;
                    }
                }
            }
#pragma unroll
            for (int n = N0; n <= N1; ++n) {
                const double g = qv * G[n - N0];
                if (n == 0) {
                    acc[0] += g;
                } else {
                    acc[2 * n - 1 - O0] = __builtin_fma(g, pr, acc[2 * n - 1 - O0]);
                    acc[2 * n - O0] = __builtin_fma(g, pi, acc[2 * n - O0]);
                }
                const double nr = pr * zx - pi * zy;
                pi = pr * zy + pi * zx;
                pr = nr;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < NA; ++o) {
        double v = acc[o];
        v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
        v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
        if (leaf_ok && (o & 3) == q4) M[b * Pp + O0 + o] = v;
    }
    if (H == 1 && leaf_ok)
        for (int o = 2 * p + 1 + q4; o < Pp; o += 4) M[b * Pp + o] = 0.0;
}

template <int PO>
__global__ __launch_bounds__(64) void k_p2m_half(
    int64_t leaf_base, int64_t nleaf, const int32_t *__restrict__ lrange,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ qs, int has_q, double inv_alpha,
    double invR, const double *__restrict__ invFY, const double *__restrict__ cnn,
    const double *__restrict__ sc, int nser, int Pp, double *__restrict__ M, int skip_d,
    double *__restrict__ zero, int64_t nzero) {
    constexpr int p = PO;
    extern __shared__ double smem[];
    {
        const int64_t nthr = (int64_t)gridDim.x * gridDim.y * 64;
        for (int64_t e = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 64 + threadIdx.x; e < nzero; e += nthr)
            zero[e] = 0.0;
    }
    double *t_sc = smem;                   // [2 nser] F_{p+1}, F_{p+2} series
    double *t_cnn = t_sc + 2 * nser;       // [p+2]
    double *t_ify = t_cnn + (p + 2);       // [p+2]
    for (int k = threadIdx.x; k < 2 * nser; k += 64) t_sc[k] = sc[k];
    for (int k = threadIdx.x; k < p + 2; k += 64) {
        t_cnn[k] = cnn[k];
        t_ify[k] = invFY[k];
    }
    __syncthreads();
    __shared__ double sx[kP2MStage], sy[kP2MStage], sq[kP2MStage];
    if (blockIdx.y == 0)
        p2m_half_body<PO, 0>(leaf_base, nleaf, lrange, bcx, bcy, px, py, qs, has_q, inv_alpha, invR, t_ify,
                             t_cnn, t_sc, nser, Pp, M, sx, sy, sq, skip_d);
    else
        p2m_half_body<PO, 1>(leaf_base, nleaf, lrange, bcx, bcy, px, py, qs, has_q, inv_alpha, invR, t_ify,
                             t_cnn, t_sc, nser, Pp, M, sx, sy, sq, skip_d);
}

// Cached P2M: the map from a point's strength to its leaf's multipole depends
// on the point and the tree only.  k_p2m_rows writes, per sorted point, the
// Pp coefficients it contributes per unit charge (charges) or per unit dipole
// component (dipoles: one row for each of d.n's two components); k_p2m_apply
// then forms every leaf's multipole as a sum of rows (one wavefront per leaf,
// lane = coefficient, contiguous loads).  Padding entries are zero.
__global__ __launch_bounds__(256) void k_p2m_rows(
    int64_t n0, int64_t n1, int64_t off1, const int32_t *__restrict__ pleaf, int64_t leaf_base,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, double inv_alpha, double invR, const double *__restrict__ invFY,
    const double *__restrict__ da, const double *__restrict__ db, const double *__restrict__ cnn,
    const double *__restrict__ sc, int nser, int p, int Pp, double *__restrict__ rq,
    double *__restrict__ rd, double *__restrict__ Gs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0 + n1) return;
    const bool dip = i >= n0;
    const int64_t j = dip ? off1 + (i - n0) : i;   // sorted point index
    const int64_t b = leaf_base + pleaf[j];
    const double wx = (px[j] - bcx[b]) * inv_alpha, wy = (py[j] - bcy[b]) * inv_alpha;
    const double y = 0.25 * (wx * wx + wy * wy);
    const double zx = wx * invR, zy = -wy * invR;   // conj(w)/R
    // G_n = F_n(y)/F_n(Y), n = 0..p+1, in this thread's scratch row of Gs
    double *G = Gs + i * (int64_t)(p + 2);
    double F1, F2;
    f_start(y, sc, nser, F1, F2);
    G[p + 1] = F1 * invFY[p + 1];
    for (int n = p; n >= 0; --n) {
        const double F0 = F1 + y * F2 * cnn[n];
        G[n] = F0 * invFY[n];
        F2 = F1;
        F1 = F0;
    }
    if (!dip) {
        double *row = rq + i * (int64_t)Pp;
        double pr = 1.0, pi = 0.0;     // conj(z)^n
        for (int n = 0; n <= p; ++n) {
            if (n == 0) {
                row[0] = G[0];
            } else {
                row[2 * n - 1] = G[n] * pr;
                row[2 * n] = G[n] * pi;
            }
            const double nr = pr * zx - pi * zy;
            pi = pr * zy + pi * zx;
            pr = nr;
        }
        for (int o = 2 * p + 1; o < Pp; ++o) row[o] = 0.0;
    } else {
        // term_n = h [a_n D Psi_{n+1} + b_n conj(D) Psi_{n-1}], D = Dx + i Dy:
        // the rows hold the coefficients of Dx and of Dy
        double *rx = rd + (i - n0) * 2 * (int64_t)Pp, *ry = rx + Pp;
        const double h = 0.5 * inv_alpha;
        double pr = zx, pi = zy;                       // conj(z)^1
        double c_r = G[0], c_i = 0.0;                  // Psi_0
        double n_r = G[1] * pr, n_i = G[1] * pi;       // Psi_1
        double m_r = n_r, m_i = -n_i;                  // Psi_{-1} = conj(Psi_1)
        for (int n = 0; n <= p; ++n) {
            const double an = h * da[n], bn = h * db[n];
            const double xr = an * n_r + bn * m_r, yr = -an * n_i + bn * m_i;
            const double xi = an * n_i + bn * m_i, yi = an * n_r - bn * m_r;
            if (n == 0) {
                rx[0] = xr;
                ry[0] = yr;
            } else {
                rx[2 * n - 1] = xr; ry[2 * n - 1] = yr;
                rx[2 * n] = xi;     ry[2 * n] = yi;
            }
            m_r = c_r; m_i = c_i;
            c_r = n_r; c_i = n_i;
            const double nr = pr * zx - pi * zy;
            pi = pr * zy + pi * zx;
            pr = nr;
            if (n + 2 <= p + 1) {
                n_r = G[n + 2] * pr; n_i = G[n + 2] * pi;
            } else {
                n_r = 0.0; n_i = 0.0;
            }
        }
        for (int o = 2 * p + 1; o < Pp; ++o) rx[o] = ry[o] = 0.0;
    }
}

// one block of four wavefronts per leaf, lanes over coefficients: wavefront w
// sums the leaf's points w, w + 4, ... (two chains per lane) and the four
// partial rows are added through LDS; the blocks also clear zero[0..nzero)
__global__ __launch_bounds__(256) void k_p2m_apply(
    int64_t leaf_base, int64_t nleaf, const int32_t *__restrict__ lrange, int64_t off1, int has_q,
    int has_d, const double *__restrict__ qs, const double *__restrict__ dns,
    const double *__restrict__ rq, const double *__restrict__ rd, int P, int Pp, double *__restrict__ M,
    double *__restrict__ zero, int64_t nzero) {
    __shared__ double part[4][64];
    // zero[0..nzero) = 0 on the side (the local expansions, cleared here
    // rather than by a launch of their own)
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nzero; e += (int64_t)gridDim.x * 256)
        zero[e] = 0.0;
    const int64_t li = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = leaf_base + li;
    const int s0 = lrange[li * 6], e0 = has_q ? lrange[li * 6 + 1] : s0;
    const int s1 = lrange[li * 6 + 2], e1 = has_d ? lrange[li * 6 + 3] : s1;
    for (int ob = 0; ob < Pp; ob += 64) {
        const int o = ob + lane;
        double a0 = 0.0, a1 = 0.0;
        if (o < Pp) {
            for (int j = s0 + w; j < e0; j += 8) {
                a0 = __builtin_fma(rq[(int64_t)j * Pp + o], qs[j], a0);
                if (j + 4 < e0) a1 = __builtin_fma(rq[(int64_t)(j + 4) * Pp + o], qs[j + 4], a1);
            }
            for (int j = s1 + w; j < e1; j += 8) {
                const int64_t jd = j - off1;
                const double *r = rd + jd * 2 * (int64_t)Pp + o;
                a0 = __builtin_fma(r[0], dns[2 * jd], __builtin_fma(r[Pp], dns[2 * jd + 1], a0));
                if (j + 4 < e1) {
                    const double *r4 = r + 8 * (int64_t)Pp;
                    a1 = __builtin_fma(r4[0], dns[2 * jd + 8], __builtin_fma(r4[Pp], dns[2 * jd + 9], a1));
                }
            }
        }
        part[w][lane] = a0 + a1;
        __syncthreads();
        if (w == 0 && o < Pp)
            M[b * Pp + o] = o < P ? (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]) : 0.0;
        __syncthreads();
    }
}

// ------------------------------------------------------------- M2L (MFMA) --
// Matrix-core version: one workgroup (4 wavefronts) per tile of up to 64
// target boxes of one level and parity class.  C (Pp x 64 local
// coefficients) stays in accumulation registers for all 27 offsets; for each
// offset the Pp x Pp operator is double-buffered in LDS (prefetched into
// registers during the previous offset's MFMAs) and the gathered multipoles
// of the 16 boxes of a wavefront are read straight into B fragments.
//   v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and
//                          C rows l/16 + 4r, column l%16 (r = 0..3);
//   v_mfma_f32_16x16x4f32: same A, B; C rows 4(l/16) + r.
typedef double yk_d4 __attribute__((ext_vector_type(4)));
typedef float yk_f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc = yk_d4;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    using acc = yk_f4;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Generic form used for M2L (27 V-list slots per box), M2M (4 child slots per
// parent) and L2L (1 parent slot per child):
//   out[box] (+)= sum_s Op[level + level_shift][slot_op[cls][s]] * X[src[box][s]]
// Every box of a tile has the same level and parity class (so the same
// operator per slot).  X is read in its own type TS and converted to T.
//
// A workgroup owns 64 boxes (4 wavefronts x 16 columns) and walks the slots;
// the slot's Pp x Pp operator is double-buffered in LDS and the gathered
// source coefficients of the next slot are loaded while the current slot runs.
// With P = 16 NB + 1 real coefficients (p a multiple of 8), the last index
// SP = 16 NB is split off: the matrix cores take the 16 NB x 16 NB block of
// indices 0..SP-1 and the vector units add row SP and column SP (a padded
// 16 (NB+1) product would spend 40% more matrix-core work on padding).
//
// Contraction order: lane group g (lane / 16) supplies, in the two matrix-core
// steps of pair kp, the contraction indices 8 kp + 2 g and 8 kp + 2 g + 1, so
// each lane loads its source coefficients as aligned pairs; the operator
// fragments read from LDS follow the same order.
typedef double yk_dpair __attribute__((ext_vector_type(2)));
typedef float yk_fpair __attribute__((ext_vector_type(2)));
template <typename TS> struct Pair2;
template <> struct Pair2<double> { using type = yk_dpair; };
template <> struct Pair2<float> { using type = yk_fpair; };

template <typename T, typename TS, int PP, bool SPLIT_REQ, int CB>
__global__ __launch_bounds__(256) void k_tile_gemm(const int4 *__restrict__ tiles, int tile0,
                                                   const int32_t *__restrict__ boxes, int nslot,
                                                   const int32_t *__restrict__ src,
                                                   const int32_t *__restrict__ slot_op,
                                                   const T *__restrict__ Op, int64_t op_stride,
                                                   int level_shift, const TS *__restrict__ X,
                                                   int assign, int nparts, double *__restrict__ out,
                                                   const int32_t *__restrict__ tgt, double *__restrict__ slab) {
    constexpr bool SPLIT = SPLIT_REQ && PP > 16;   // (the host never asks for PP = 16)
    constexpr int NB = SPLIT ? PP / 16 - 1 : PP / 16;   // 16-row blocks on the matrix cores
    constexpr int SP = 16 * NB;                         // split-off index (SPLIT only)
    constexpr int NKP = 2 * NB;                         // contraction pairs
    // LDS copy of the operator: the NCOL columns used, each LDA rows (with the
    // split, 49 x 52 instead of 64 x 64 for p = 24: less LDS, so three
    // workgroups fit a compute unit, and a column stride off the bank period)
    constexpr int NCOL = SPLIT ? SP + 1 : PP;
    constexpr int LDA = SPLIT ? ((SP + 1 + 3) & ~3) : PP;
    constexpr int kPairs = NCOL * LDA / 2;              // operator pairs per slot
    constexpr int NL2 = (kPairs + 255) / 256;           // pairs per thread
    constexpr int kMaxSlot = 27;
    constexpr int NC = 64 * CB;                         // boxes (columns) per workgroup
    using V2 = typename Pair2<TS>::type;
    using T2 = typename Pair2<T>::type;
    __shared__ T As[2][NCOL * LDA];
    __shared__ int32_t s_src[kMaxSlot * NC];
    using MF = Mfma<T>;
    // nparts > 1 (few tiles): the slots of a tile are shared among nparts
    // workgroups (assign must be 0).  With tgt (sparse M2L) the tile's
    // entries are translation indices: the source is src[entry], the target
    // is row tgt[entry].  In both cases several workgroups contribute to one
    // output row, so each stores its result in a row of its own of slab
    // (translation `entry`, or column j of workgroup bid: row bid * NC + j),
    // which k_slab_reduce_* then add to the outputs in a fixed order: the
    // sums do not depend on the order the workgroups run in.
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int part = bid % nparts;
    const int4 tl = tiles[tile0 + bid / nparts];
    const int level = tl.x, cls = tl.y, start = tl.z, count = tl.w;
    const int sl0 = part * nslot / nparts, sl1 = (part + 1) * nslot / nparts;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4;
    // column block c of this wavefront: columns 16 (CB w + c) + lane % 16
    int jb[CB];
    bool colvalid[CB];
    int64_t boxj[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        jb[c] = 16 * (CB * w + c) + (lane & 15);
        colvalid[c] = jb[c] < count;
        boxj[c] = colvalid[c] ? (tgt ? tgt[boxes[start + jb[c]]] : boxes[start + jb[c]]) : -1;
    }
    // source box of every (slot, column) of the tile, -1 where empty
    for (int e = sl0 * NC + tid; e < sl1 * NC; e += 256) {
        const int sl = e / NC, j = e % NC;
        s_src[e] = j < count ? src[(int64_t)boxes[start + j] * nslot + sl] : -1;
    }
    typename MF::acc acc[CB][NB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int r = 0; r < NB; ++r) acc[c][r] = typename MF::acc{0, 0, 0, 0};
    T rowacc[CB], colacc[CB][NB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        rowacc[c] = T(0);
#pragma unroll
        for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) colacc[c][r][q] = T(0);
    }
    const T *Olev = Op + (int64_t)(level + level_shift) * op_stride;
    auto op_of = [&](int sl) -> const T2 * {
        return reinterpret_cast<const T2 *>(Olev + (size_t)slot_op[cls * nslot + sl] * PP * PP);
    };
    // global pair of LDS pair e (column-major, PP rows per column in memory)
    auto gpair = [&](int e) { return (e / (LDA / 2)) * (PP / 2) + e % (LDA / 2); };
    // B fragment of a slot: unconditional loads (row 0 stands in for an empty
    // slot) and the empty slot's zeros selected when the fragment is consumed,
    // so the loads of the next slot stay in flight during the current one (a
    // select, not a product, so whatever row 0 holds never reaches the sums)
    V2 braw[CB][NKP];
    TS bsraw[CB];
    bool bvalid[CB];
    T bcur[CB][2 * NKP], bs[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        bsraw[c] = TS(0);
        bvalid[c] = false;
        bs[c] = T(0);
    }
    T2 pre[NL2];
    auto load_b = [&](int sl) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int32_t sj = s_src[sl * NC + jb[c]];
            const TS *row = X + (int64_t)(sj >= 0 ? sj : 0) * PP;
            const V2 *row2 = reinterpret_cast<const V2 *>(row) + g;
#pragma unroll
            for (int kp = 0; kp < NKP; ++kp) braw[c][kp] = row2[4 * kp];
            if constexpr (SPLIT) bsraw[c] = row[SP];
            bvalid[c] = sj >= 0;
        }
    };
    auto take_b = [&]() {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
#pragma unroll
            for (int kp = 0; kp < NKP; ++kp) {
                bcur[c][2 * kp] = bvalid[c] ? (T)braw[c][kp].x : T(0);
                bcur[c][2 * kp + 1] = bvalid[c] ? (T)braw[c][kp].y : T(0);
            }
            if constexpr (SPLIT) bs[c] = bvalid[c] ? (T)bsraw[c] : T(0);
        }
    };
    __syncthreads();
    load_b(sl0);
    {
        const T2 *Tg = op_of(sl0);
        T2 *Ad = reinterpret_cast<T2 *>(As[0]);
#pragma unroll
        for (int e = 0; e < NL2; ++e)
            if (kPairs >= 256 * NL2 || tid + 256 * e < kPairs) Ad[tid + 256 * e] = Tg[gpair(tid + 256 * e)];
    }
    take_b();
    __syncthreads();
    for (int slot = sl0; slot < sl1; ++slot) {
        const int cur = (slot - sl0) & 1;
        const bool more = slot + 1 < sl1;
        if (more) {
            load_b(slot + 1);
            const T2 *Tg = op_of(slot + 1);
#pragma unroll
            for (int e = 0; e < NL2; ++e)
                if (kPairs >= 256 * NL2 || tid + 256 * e < kPairs) pre[e] = Tg[gpair(tid + 256 * e)];
        }
        // operator column-major: A[i][k] = As[k * LDA + i]; step (kp, e) takes
        // contraction index 8 kp + 2 g + e in lane group g; each operator
        // fragment read from LDS serves the CB column blocks
        // (the fragments of step s are read two steps ahead, into a ring of
        // three, so the matrix cores do not wait on LDS between steps)
        const T *Ac = As[cur] + 2 * g * LDA + (lane & 15);
        constexpr int NS = 2 * NKP;   // steps; step s = 2 kp + e
        T afr[3][NB];
        auto read_a = [&](int st, T *dst) {
#pragma unroll
            for (int rt = 0; rt < NB; ++rt) dst[rt] = Ac[(8 * (st >> 1) + (st & 1)) * LDA + 16 * rt];
        };
        read_a(0, afr[0]);
        if (NS > 1) read_a(1, afr[1]);
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            if (st + 2 < NS) read_a(st + 2, afr[(st + 2) % 3]);
#pragma unroll
            for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[c][rt] = MF::step(afr[st % 3][rt], bcur[c][st], acc[c][rt]);
        }
        if constexpr (SPLIT) {
            const T *A = As[cur];
            // row SP: this lane's share of sum_k A[SP][k] b[k]; column SP into
            // the rows this lane holds of the matrix-core result
#pragma unroll
            for (int kp = 0; kp < NKP; ++kp)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const T a = A[(8 * kp + 2 * g + e) * LDA + SP];
#pragma unroll
                    for (int c = 0; c < CB; ++c) rowacc[c] += a * bcur[c][2 * kp + e];
                }
            if (g == 0) {
                const T a = A[SP * LDA + SP];
#pragma unroll
                for (int c = 0; c < CB; ++c) rowacc[c] += a * bs[c];
            }
#pragma unroll
            for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T a = A[SP * LDA + 16 * rt + MF::row(lane, q)];
#pragma unroll
                    for (int c = 0; c < CB; ++c) colacc[c][rt][q] += a * bs[c];
                }
        }
        if (more) {
            T2 *Ad = reinterpret_cast<T2 *>(As[cur ^ 1]);
#pragma unroll
            for (int e = 0; e < NL2; ++e)
                if (kPairs >= 256 * NL2 || tid + 256 * e < kPairs) Ad[tid + 256 * e] = pre[e];
            take_b();
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        if constexpr (SPLIT) {
            rowacc[c] += __shfl_xor(rowacc[c], 16, 64);
            rowacc[c] += __shfl_xor(rowacc[c], 32, 64);
        }
        if (colvalid[c]) {
            const bool to_slab = slab != nullptr;
            const int store = to_slab || assign;
            double *o = to_slab ? slab + (tgt ? (int64_t)boxes[start + jb[c]] : (int64_t)bid * NC + jb[c]) * PP
                                : out + boxj[c] * PP;
#pragma unroll
            for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 16 * rt + MF::row(lane, q);
                    const double v = SPLIT ? (double)acc[c][rt][q] + (double)colacc[c][rt][q] : (double)acc[c][rt][q];
                    o[i] = store ? v : o[i] + v;
                }
            if constexpr (SPLIT) {
                if (g == 0) o[SP] = store ? (double)rowacc[c] : o[SP] + (double)rowacc[c];
                // padding entries SP + 1 .. PP - 1 stay zero for later readers
                if (store)
                    for (int i = SP + 1 + g; i < PP; i += 4) o[i] = 0.0;
            }
        }
    }
}

// Persistent M2L for 64 padded coefficients without the split (p = 31), FP64,
// on trees with at least as many tiles as the launch has workgroups.  The
// launch is one resident round (three workgroups per compute unit: the slot's
// operator is staged in LDS in two halves of 32 contraction columns, double
// buffered at half-slot steps, 32 KB); workgroup b takes the contiguous run
// [U b / G, U (b + 1) / G) of the U = 54 ntiles (tile, slot, half) units in
// the tiles' order and keeps the tile's results in its accumulators across
// the slots, so no compute unit idles while another finishes a last round of
// whole tiles.  A run is at least 54 units long, so a tile is shared by at
// most two workgroups; those add into the local expansions, which are zero
// before M2L, with atomic adds, and with two addends into zero the sum does
// not depend on their order.  A tile that lies within one run is added
// without atomics.  The matrix-core steps and fragment layout are those of
// k_tile_gemm.
__global__ __launch_bounds__(256) void k_m2l_persist(const int4 *__restrict__ tiles, int ntiles,
                                                     const int32_t *__restrict__ boxes,
                                                     const int32_t *__restrict__ src,
                                                     const int32_t *__restrict__ slot_op,
                                                     const double *__restrict__ Op, int64_t op_stride,
                                                     const double *__restrict__ X, double *__restrict__ out) {
    constexpr int PP = 64, NB = 4, LDA = 64, NCOLH = 32, NSH = 8, kSlots = 27, NH = 2;
    constexpr int kPairs = NCOLH * LDA / 2;   // operator pairs per half
    constexpr int NL2 = kPairs / 256;         // pairs per thread
    __shared__ double As[2][NCOLH * LDA];
    using MF = Mfma<double>;
    const int G = gridDim.x;
    const int bid = xcd_remap(blockIdx.x, G);
    const int64_t U = (int64_t)ntiles * kSlots * NH;
    const int64_t u0 = U * bid / G, u1 = U * (bid + 1) / G;
    if (u0 >= u1) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4;
    const int jb = 16 * w + (lane & 15);
    // current tile
    int4 tl = tiles[(int)(u0 / (kSlots * NH))];
    bool colvalid = jb < tl.w;
    int64_t boxj = colvalid ? boxes[tl.z + jb] : -1;
    yk_d4 acc[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) acc[r] = yk_d4{0, 0, 0, 0};
    yk_dpair braw[8];
    bool bvalid = false;
    double bcur[16];
    yk_dpair pre[NL2];
    auto load_b = [&](const int4 &t, int sl) {
        int32_t sj = -1;
        if (jb < t.w) sj = src[(int64_t)boxes[t.z + jb] * kSlots + sl];
        const yk_dpair *row2 = reinterpret_cast<const yk_dpair *>(X + (int64_t)(sj >= 0 ? sj : 0) * PP) + g;
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) braw[kp] = row2[4 * kp];
        bvalid = sj >= 0;
    };
    auto take_b = [&]() {
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) {
            bcur[2 * kp] = bvalid ? braw[kp].x : 0.0;
            bcur[2 * kp + 1] = bvalid ? braw[kp].y : 0.0;
        }
    };
    auto op_half = [&](const int4 &t, int sl, int h) -> const yk_dpair * {
        return reinterpret_cast<const yk_dpair *>(Op + (int64_t)t.x * op_stride +
                                                  (size_t)slot_op[t.y * kSlots + sl] * PP * PP) +
               (size_t)h * NCOLH * (PP / 2);
    };
    {
        const int sl = (int)((u0 / NH) % kSlots), h = (int)(u0 % NH);
        load_b(tl, sl);
        const yk_dpair *Tg = op_half(tl, sl, h);
        yk_dpair *Ad = reinterpret_cast<yk_dpair *>(As[0]);
#pragma unroll
        for (int e = 0; e < NL2; ++e) Ad[tid + 256 * e] = Tg[tid + 256 * e];
        take_b();
    }
    __syncthreads();
    int64_t tile_first = (u0 / (kSlots * NH)) * (kSlots * NH);
    for (int64_t u = u0; u < u1; ++u) {
        const int cur = (int)((u - u0) & 1);
        const int h = (int)(u % NH), sl = (int)((u / NH) % kSlots);
        const bool more = u + 1 < u1;
        const int64_t un = u + 1;
        const int hn = (int)(un % NH), sln = (int)((un / NH) % kSlots);
        const bool new_tile = more && sln == 0 && hn == 0;
        int4 tn = tl;
        if (more) {
            if (new_tile) tn = tiles[(int)(un / (kSlots * NH))];
            if (hn == 0) load_b(tn, sln);
            const yk_dpair *Tg = op_half(tn, sln, hn);
#pragma unroll
            for (int e = 0; e < NL2; ++e) pre[e] = Tg[tid + 256 * e];
        }
        // this half's B values (a select: bcur is never indexed at run time)
        double bp[NSH];
#pragma unroll
        for (int st = 0; st < NSH; ++st) bp[st] = h ? bcur[NSH + st] : bcur[st];
        const double *Ac = As[cur] + 2 * g * LDA + (lane & 15);
        double afr[3][NB];
        auto read_a = [&](int st, double *dst) {
#pragma unroll
            for (int rt = 0; rt < NB; ++rt) dst[rt] = Ac[(8 * (st >> 1) + (st & 1)) * LDA + 16 * rt];
        };
        read_a(0, afr[0]);
        read_a(1, afr[1]);
#pragma unroll
        for (int st = 0; st < NSH; ++st) {
            if (st + 2 < NSH) read_a(st + 2, afr[(st + 2) % 3]);
#pragma unroll
            for (int rt = 0; rt < NB; ++rt) acc[rt] = MF::step(afr[st % 3][rt], bp[st], acc[rt]);
        }
        // the tile's last unit, or the run's: add the results (a run may end,
        // or start, between the two halves of a slot)
        if ((h == NH - 1 && sl == kSlots - 1) || !more) {
            const bool whole = tile_first >= u0 && tile_first + kSlots * NH <= u1;
            if (colvalid) {
                double *o = out + boxj * PP;
#pragma unroll
                for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = 16 * rt + MF::row(lane, q);
                        if (whole) o[i] += acc[rt][q];
                        else atomicAdd(o + i, acc[rt][q]);
                    }
            }
#pragma unroll
            for (int r = 0; r < NB; ++r) acc[r] = yk_d4{0, 0, 0, 0};
        }
        if (more) {
            yk_dpair *Ad = reinterpret_cast<yk_dpair *>(As[cur ^ 1]);
#pragma unroll
            for (int e = 0; e < NL2; ++e) Ad[tid + 256 * e] = pre[e];
            if (hn == 0) take_b();
            if (new_tile) {
                tl = tn;
                tile_first = un;
                colvalid = jb < tl.w;
                boxj = colvalid ? boxes[tl.z + jb] : -1;
            }
        }
        __syncthreads();
    }
}

// Fixed-order sums of the slab rows of k_tile_gemm into the outputs.
// Sparse M2L: target box t of the list gets rows[off[t] .. off[t+1]) (its
// translations in increasing index), one wavefront per target.
__global__ __launch_bounds__(256) void k_slab_reduce_csr(int64_t ntgt, const int32_t *__restrict__ tgt,
                                                         const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ rows,
                                                         const double *__restrict__ slab, int PP,
                                                         double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int i = threadIdx.x & 63;
    if (t >= ntgt || i >= PP) return;
    double acc = 0.0;
    for (int k = off[t]; k < off[t + 1]; ++k) acc += slab[(int64_t)rows[k] * PP + i];
    double *o = out + (int64_t)tgt[t] * PP + i;
    *o += acc;
}

// Split slots: column j of tile t gets the rows of its nparts workgroups in
// part order; one workgroup per tile.
__global__ __launch_bounds__(256) void k_slab_reduce_parts(const int4 *__restrict__ tiles, int tile0,
                                                           const int32_t *__restrict__ boxes, int nparts, int NC,
                                                           const double *__restrict__ slab, int PP,
                                                           double *__restrict__ out) {
    const int t = blockIdx.x;
    const int4 tl = tiles[tile0 + t];
    for (int e = threadIdx.x; e < tl.w * PP; e += 256) {
        const int j = e / PP, i = e % PP;
        double acc = 0.0;
        for (int part = 0; part < nparts; ++part)
            acc += slab[((int64_t)(t * nparts + part) * NC + j) * PP + i];
        out[(int64_t)boxes[tl.z + j] * PP + i] += acc;
    }
}

// Where the partial rows of a launch whose workgroups share output rows go,
// and (sparse M2L) the fixed order in which they are summed.
struct SlabPlan {
    DevBuf<double> *buf = nullptr;
    int64_t ntgt = 0;                           // sparse: targets with translations
    const int32_t *tgt = nullptr, *off = nullptr, *rows = nullptr;
};

template <typename T, typename TS, int CB = 1>
void launch_tile_gemm(Context &ctx, int P, int Pp, int ntiles, const int4 *tiles, int tile0,
                      const int32_t *boxes, int nslot, const int32_t *src, const int32_t *slot_op,
                      const T *Op, int64_t op_stride, int level_shift, const TS *X, int assign,
                      double *out, const int32_t *tgt = nullptr, const SlabPlan *slab = nullptr,
                      int64_t ntrans = 0) {
    if (ntiles <= 0) return;
    if (nslot < 1 || nslot > 27) throw Error{YK_ERR_INTERNAL, "tile GEMM supports 1..27 slots"};
    const bool split = Pp >= 32 && P == Pp - 15;
    // fewer tiles than compute units: share each tile's slots among up to 7
    // workgroups (about 4 slots each), whose partial rows are summed after
    const int nparts = (!assign && slab && nslot >= 8 && ntiles < 256) ? std::min(7, (512 + ntiles - 1) / ntiles) : 1;
    const unsigned grid = (unsigned)ntiles * (unsigned)nparts;
    if (tgt && !slab) throw Error{YK_ERR_INTERNAL, "sparse tile GEMM needs a slab"};
    constexpr int NC = 64 * CB;
    double *sl = nullptr;
    if (tgt) sl = slab->buf->ensure((size_t)std::max<int64_t>(ntrans, 1) * Pp);
    else if (nparts > 1) sl = slab->buf->ensure((size_t)grid * NC * Pp);
#define YK_TILE_CASE(PPV)                                                                          \
    case PPV:                                                                                      \
        if (split)                                                                                 \
            hipLaunchKernelGGL((k_tile_gemm<T, TS, PPV, true, CB>), dim3(grid), dim3(256), 0,     \
                               ctx.stream, tiles, tile0, boxes, nslot, src, slot_op, Op, op_stride, \
                               level_shift, X, assign, nparts, out, tgt, sl);                     \
        else                                                                                       \
            hipLaunchKernelGGL((k_tile_gemm<T, TS, PPV, false, CB>), dim3(grid), dim3(256), 0,    \
                               ctx.stream, tiles, tile0, boxes, nslot, src, slot_op, Op, op_stride, \
                               level_shift, X, assign, nparts, out, tgt, sl);                     \
        break;
    switch (Pp) {
        YK_TILE_CASE(16)
        YK_TILE_CASE(32)
        YK_TILE_CASE(48)
        YK_TILE_CASE(64)
        default:
            throw Error{YK_ERR_INTERNAL, "no matrix-core kernel for this padded order"};
    }
#undef YK_TILE_CASE
    check_launch(ctx, "k_tile_gemm");
    if (tgt) {
        if (slab->ntgt > 0)
            hipLaunchKernelGGL(k_slab_reduce_csr, dim3((unsigned)((slab->ntgt + 3) / 4)), dim3(256), 0, ctx.stream,
                               slab->ntgt, slab->tgt, slab->off, slab->rows, sl, Pp, out);
        check_launch(ctx, "k_slab_reduce_csr");
    } else if (nparts > 1) {
        hipLaunchKernelGGL(k_slab_reduce_parts, dim3((unsigned)ntiles), dim3(256), 0, ctx.stream, tiles, tile0, boxes,
                           nparts, NC, sl, Pp, out);
        check_launch(ctx, "k_slab_reduce_parts");
    }
}

// Small levels of M2M (4 child slots) and L2L (1 parent slot): one block of
// four wavefronts per box.  The (slot, column) pairs of the product are split
// into four equal runs, one per wavefront (M2M: a child slot each; L2L: a
// quarter of the columns each), so each lane's chain of operator loads is a
// quarter as long; the four partial rows are summed through LDS.  (The tile
// GEMM chains one memory round trip per slot, which dominates when a level
// has few boxes.)  Padding rows and columns of the operators and of the
// coefficient vectors are zero.
template <int PP, int NS>
__global__ __launch_bounds__(256) void k_small_gemv(
    const int32_t *__restrict__ boxes, int64_t box0, const int32_t *__restrict__ src,
    const uint32_t *__restrict__ bcode, const double *__restrict__ Op, const double *__restrict__ X,
    int P, int assign, double *__restrict__ out) {
    constexpr int KW = NS * PP / 4;          // (slot, column) pairs per wavefront
    constexpr int BT = KW < 16 ? KW : 16;    // operator loads issued together
    __shared__ double xs[NS * PP];
    __shared__ double red[4][PP];
    const int64_t box = boxes ? (int64_t)boxes[blockIdx.x] : box0 + blockIdx.x;
    const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
    for (int f = threadIdx.x; f < NS * PP; f += 256) {
        const int sj = src[box * NS + f / PP];
        xs[f] = sj >= 0 ? X[(int64_t)sj * PP + f % PP] : 0.0;
    }
    const int s = NS == 1 ? 0 : w;           // this wavefront's slot
    const int k0 = NS == 1 ? w * KW : 0;     // and its first column
    const bool live = src[box * NS + s] >= 0;
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < PP && live) {
        const double *A = Op + (size_t)(NS == 1 ? (int)(bcode[box] & 3u) : s) * PP * PP +
                          (size_t)k0 * PP + i;
        const double *x = xs + s * PP + k0;
#pragma unroll
        for (int kb = 0; kb < KW; kb += BT) {
            double a[BT];
#pragma unroll
            for (int u = 0; u < BT; ++u) a[u] = A[(size_t)(kb + u) * PP];
#pragma unroll
            for (int u = 0; u < BT; ++u) acc[u & 3] = __builtin_fma(a[u], x[kb + u], acc[u & 3]);
        }
    }
    if (i < PP) red[w][i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (w == 0 && i < PP) {
        const double v = i < P ? (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]) : 0.0;
        double *o = out + box * PP + i;
        *o = assign ? v : *o + v;
    }
}

void launch_small_gemv(Context &ctx, int Pp, int ns, int64_t nbox, const int32_t *boxes, int64_t box0,
                       const int32_t *src, const uint32_t *bcode, const double *Op, const double *X,
                       int P, int assign, double *out) {
    if (nbox <= 0) return;
#define YK_SMALL_CASE(PPV)                                                                         \
    case PPV:                                                                                      \
        if (ns == 1)                                                                               \
            hipLaunchKernelGGL((k_small_gemv<PPV, 1>), dim3((unsigned)nbox), dim3(256), 0, ctx.stream, \
                               boxes, box0, src, bcode, Op, X, P, assign, out);                    \
        else                                                                                       \
            hipLaunchKernelGGL((k_small_gemv<PPV, 4>), dim3((unsigned)nbox), dim3(256), 0, ctx.stream, \
                               boxes, box0, src, bcode, Op, X, P, assign, out);                    \
        break;
    switch (Pp) {
        YK_SMALL_CASE(16)
        YK_SMALL_CASE(32)
        YK_SMALL_CASE(48)
        YK_SMALL_CASE(64)
        default:
            throw Error{YK_ERR_INTERNAL, "no small-level kernel for this padded order"};
    }
#undef YK_SMALL_CASE
    check_launch(ctx, "k_small_gemv");
}

// levels with at most this many boxes take k_small_gemv for M2M (4 operators
// per box: beyond ~1000 boxes the tile GEMM's shared operators win) and L2L
constexpr int64_t kSmallLevelM2M = 1024, kSmallLevelL2L = 4096;

__global__ void k_to_float(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ----------------------------------------------------------- leaf kernel ---
// Near field in scaled coordinates: separations are multiplied by 1/(2 alpha),
// so the squared scaled separation is t = r^2/(4 alpha^2) itself and
//     K0(r/alpha)            = h(t) A(t) + B(t),           h = -(1/2) ln t,
//     4 K1(r/alpha)/(r/alpha) = 1/t - 2 h(t) C(t) - D(t)
// for t <= 1 (series in bessel_tables.h); larger t use the Chebyshev forms.
template <int NT, typename T>
__device__ __forceinline__ T horner_n(const T (&c)[YK_NSER64], T t) {
    T s = c[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) s = __builtin_fma(s, t, c[k]);
    return s;
}

// h(t) = -(1/2) ln t for a positive normal t.  With t = m 2^e, m in [1/2, 1),
// piece i of [1/2, 1) is given by the top eight fraction bits of m; the table
// holds rc_i ~ 1/c_i (c_i the piece's centre) and (1/2) ln rc_i, and
// -(1/2) ln m = (1/2) ln rc_i - (1/2) log1p(m rc_i - 1) with |m rc_i - 1| < 2^-9,
// where five terms of the log1p series leave an error below r^6/12 < 2^-57.
// ln 2 is split so that e * ln2_hi is exact.
__device__ __forceinline__ double neg_half_log(double t, const double2 *__restrict__ tab) {
    const int e = __builtin_amdgcn_frexp_exp(t);
    const double m = __builtin_amdgcn_frexp_mant(t);
    const int i = (__double2hiint(m) >> 12) & (YK_LOG_TAB - 1);
    const double2 c = tab[i];
    const double r = __builtin_fma(m, c.x, -1.0);
    double s = __builtin_fma(r, -0.1, 0.125);
    s = __builtin_fma(s, r, -1.0 / 6.0);
    s = __builtin_fma(s, r, 0.25);
    s = __builtin_fma(s, r, -0.5);
    const double de = (double)e;
    constexpr double h2_hi = -0.5 * 6.93147180369123816490e-01;   // -(1/2) 0x3FE62E42FEE00000
    constexpr double h2_lo = -0.5 * 1.90821492927058770002e-10;
    return __builtin_fma(de, h2_hi, c.y + __builtin_fma(de, h2_lo, s * r));
}

template <int NT, bool kSmallOnly>
__device__ __forceinline__ double near_k0(double t, const double2 *__restrict__ tab) {
    if (kSmallOnly || t <= 1.0)
        return __builtin_fma(neg_half_log(t, tab), horner_n<NT>(yk_ser_A, t), horner_n<NT>(yk_ser_B, t));
    return k0_large(2.0 * sqrt(t));
}
// 4 K1(z)/z with t = z^2/4
template <int NT, bool kSmallOnly>
__device__ __forceinline__ double near_k1oz4(double t, const double2 *__restrict__ tab) {
    if (kSmallOnly || t <= 1.0) {
        const double h2 = 2.0 * neg_half_log(t, tab);
        return fast_rcp(t) - __builtin_fma(h2, horner_n<NT>(yk_ser_C, t), horner_n<NT>(yk_ser_D, t));
    }
    const double z = 2.0 * sqrt(t);
    return 4.0 * k1_large(z) / z;
}

template <int NT>
__device__ __forceinline__ float horner_nf(const float (&c)[YK_NSER32], float t) {
    float s = c[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) s = s * t + c[k];
    return s;
}
template <bool kSmallOnly>
__device__ __forceinline__ float near_k0_f(float t) {
    if (kSmallOnly || t <= 1.0f) {
        const float lt = __logf(t);
        return -0.5f * lt * horner_nf<YK_NSER32>(yk_ser_A_f, t) + horner_nf<YK_NSER32>(yk_ser_B_f, t);
    }
    return k0_large_f(2.0f * sqrtf(t));
}
template <bool kSmallOnly>
__device__ __forceinline__ float near_k1oz4_f(float t) {
    if (kSmallOnly || t <= 1.0f) {
        const float lt = __logf(t);
        return 1.0f / t + lt * horner_nf<YK_NSER32>(yk_ser_C_f, t) - horner_nf<YK_NSER32>(yk_ser_D_f, t);
    }
    const float z = 2.0f * sqrtf(t);
    return 4.0f * k1_large_f(z) / z;
}

// Near-field accumulation policy: FP64 (series and sums in double) or FP32
// (separations and the dipole dot product in double, the Bessel series, the
// logarithm and the accumulation in float).
template <int NT, bool kSmallOnly, bool kF32>
struct Near {
    using acc_t = typename std::conditional<kF32, float, double>::type;
    static __device__ __forceinline__ acc_t charge(double q, double t, const double2 *tab) {
        if constexpr (kF32) return (float)q * near_k0_f<kSmallOnly>((float)t);
        else return q * near_k0<NT, kSmallOnly>(t, tab);
    }
    // dot = (x - y).(d n_y) in scaled coordinates; the caller multiplies the
    // sum by 1/(2 alpha), which turns dot * 4K1(z)/z into (1/alpha) K1(z) (x-y).(d n)/r
    static __device__ __forceinline__ acc_t dipole(double dot, double t, const double2 *tab) {
        if constexpr (kF32) return (float)dot * near_k1oz4_f<kSmallOnly>((float)t);
        else return dot * near_k1oz4<NT, kSmallOnly>(t, tab);
    }
};

// One wavefront per item: up to 64 targets of one leaf.  With c targets, the
// 64 lanes form g = floor(64/c) groups of c lanes; lane l serves target l mod c
// and walks every g-th source of the leaf's U list, so at most c - 1 lanes
// idle.  U-list sources are staged into LDS (scaled coordinates and strengths)
// in chunks of kLeafStage; the group partial sums are combined through LDS at
// the end.  The result is the near field alone (k_l2p adds the far field).
constexpr int kLeafStage = 192;

// MU: the longest U list (9 in a uniform tree; 16 for the adaptive one, whose
// 2:1 balance bounds it by 13)
template <int NT, bool kSmallOnly, bool kF32 = false, int MU = 9>
__global__ __launch_bounds__(64) void k_leaf(
    const int2 *__restrict__ items, int64_t leaf_base, const int32_t *__restrict__ lrange,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist,
    const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ qs,
    const double *__restrict__ dns, int64_t off1, int has_q, int has_d, int mask, double inv2a,
    double dip_scale, double *__restrict__ outs) {
    __shared__ double s_x[kLeafStage], s_y[kLeafStage], s_a[kLeafStage], s_b[kLeafStage];
    __shared__ double2 s_log[YK_LOG_TAB];
    __shared__ int qa[MU], qn[MU], da[MU], dn_[MU];
    const int2 item = items[xcd_remap(blockIdx.x, gridDim.x)];
    const int li = item.x;
    const int lane = threadIdx.x;
    if constexpr (!kF32)
        for (int i = lane; i < YK_LOG_TAB; i += 64) s_log[i] = make_double2(yk_log_tab[2 * i], yk_log_tab[2 * i + 1]);
    int rs[3], re[3], ntot = 0;
    for (int s = 0; s < 3; ++s) {
        rs[s] = lrange[li * 6 + 2 * s];
        re[s] = (mask >> s) & 1 ? lrange[li * 6 + 2 * s + 1] : rs[s];
        ntot += re[s] - rs[s];
    }
    const int u0 = uoff[li], nu = uoff[li + 1] - u0;
    // U-list source ranges (at most MU leaves) of the two source sets, in
    // LDS (indexed per lane below; a private array would live in scratch)
    if (lane < MU) {
        const int u = lane;
        int a = 0, an = 0, b2 = 0, bn = 0;
        if (u < nu) {
            const int ul = ulist[u0 + u];
            a = lrange[ul * 6];
            an = has_q ? lrange[ul * 6 + 1] - a : 0;
            b2 = lrange[ul * 6 + 2];
            bn = has_d ? lrange[ul * 6 + 3] - b2 : 0;
        }
        qa[u] = a; qn[u] = an; da[u] = b2; dn_[u] = bn;
    }
    __syncthreads();
    int nq = 0, nd = 0;
    for (int u = 0; u < MU; ++u) {
        nq += qn[u];
        nd += dn_[u];
    }
    const int tb = item.y;
    const int c = min(64, ntot - tb);          // >= 1 by construction of the items
    const int g = 64 / c;
    const int ti = lane % c, sub = lane / c;
    const bool valid = sub < g;
    int k = tb + ti, t = -1;
    for (int s = 0; s < 3; ++s) {
        const int n = re[s] - rs[s];
        if (t < 0 && k < n) t = rs[s] + k;
        k -= n;
    }
    // separations are formed from the unscaled coordinates and then scaled:
    // the difference of two nearby coordinates is exact, whereas scaling
    // first would round each coordinate, which costs digits in (x - y).n for
    // the nearly tangential pairs of densely sampled, tightly curved curves
    const double xs = px[t], ys = py[t];
    using NearT = Near<NT, kSmallOnly, kF32>;
    typename NearT::acc_t near_q = 0, near_d = 0;
    for (int set = 0; set < 2; ++set) {
        const int ntot_s = set == 0 ? nq : nd;
        for (int c0 = 0; c0 < ntot_s; c0 += kLeafStage) {
            const int cn = min(kLeafStage, ntot_s - c0);
            __syncthreads();
            // cooperative gather of flat source indices [c0, c0 + cn) into LDS
            for (int f = lane; f < cn; f += 64) {
                int r = c0 + f, u = 0;
                const int *cnt = set == 0 ? qn : dn_;
                while (u < MU - 1 && r >= cnt[u]) { r -= cnt[u]; ++u; }
                const int j = (set == 0 ? qa[u] : da[u]) + r;
                s_x[f] = px[j];
                s_y[f] = py[j];
                if (set == 0) {
                    s_a[f] = qs[j];
                } else {
                    const int64_t jd = j - off1;
                    s_a[f] = dns[2 * jd];
                    s_b[f] = dns[2 * jd + 1];
                }
            }
            __syncthreads();
            if (valid) {
                // full passes (every lane's source index in range), then the tail
                const int nfull = cn - cn % g;
                if (set == 0) {
                    auto pair = [&](int j) {
                        const double dx = (xs - s_x[j]) * inv2a, dy = (ys - s_y[j]) * inv2a;
                        const double tt = __builtin_fma(dx, dx, dy * dy);
                        if (tt > 0.0) near_q += NearT::charge(s_a[j], tt, s_log);
                    };
#pragma unroll 2
                    for (int jj = 0; jj < nfull; jj += g) pair(jj + sub);
                    if (nfull + sub < cn) pair(nfull + sub);
                } else {
                    auto pair = [&](int j) {
                        const double dx = (xs - s_x[j]) * inv2a, dy = (ys - s_y[j]) * inv2a;
                        const double tt = __builtin_fma(dx, dx, dy * dy);
                        if (tt > 0.0) near_d += NearT::dipole(__builtin_fma(dx, s_a[j], dy * s_b[j]), tt, s_log);
                    };
#pragma unroll 2
                    for (int jj = 0; jj < nfull; jj += g) pair(jj + sub);
                    if (nfull + sub < cn) pair(nfull + sub);
                }
            }
        }
    }
    __syncthreads();
    s_x[lane] = valid ? (double)near_q + dip_scale * (double)near_d : 0.0;
    __syncthreads();
    if (sub == 0) {
        double tot = 0.0;
        for (int gi = 0; gi < g; ++gi) tot += s_x[ti + gi * c];
        outs[t] = tot * kInv2Pi;
    }
}

// ------------------------------------------------- cached near field ---
// The near-field values depend on the points and alpha only, so a tree can
// keep them: k_near_build writes them once per target set, k_near_apply then
// forms the sums from them (an HBM-bound pass instead of Bessel series).
// Both walk the items exactly as k_leaf does; entries are source-major and
// target-minor per item, so a wavefront's loads are contiguous.
struct ItemSetup {
    int c, g, ti, sub, t, nq, nd;
    bool valid;
};

// Leaf ranges and U-list source ranges of an item (into the LDS arrays qa, qn,
// da, dn_, one entry per neighbour), and this lane's target.  q_on / d_on
// select which source sets are counted; NTB threads share the item.
template <int NTB = 64>
__device__ __forceinline__ ItemSetup item_setup(int2 item, const int32_t *__restrict__ lrange,
                                                const int32_t *__restrict__ uoff,
                                                const int32_t *__restrict__ ulist, int q_on, int d_on,
                                                int mask, int *qa, int *qn, int *da, int *dn_) {
    const int li = item.x, lane = threadIdx.x;
    int rs[3], re[3], ntot = 0;
    for (int s = 0; s < 3; ++s) {
        rs[s] = lrange[li * 6 + 2 * s];
        re[s] = (mask >> s) & 1 ? lrange[li * 6 + 2 * s + 1] : rs[s];
        ntot += re[s] - rs[s];
    }
    const int u0 = uoff[li], nu = uoff[li + 1] - u0;
    if (lane < 9) {
        const int u = lane;
        int a = 0, an = 0, b2 = 0, bn = 0;
        if (u < nu) {
            const int ul = ulist[u0 + u];
            a = lrange[ul * 6];
            an = q_on ? lrange[ul * 6 + 1] - a : 0;
            b2 = lrange[ul * 6 + 2];
            bn = d_on ? lrange[ul * 6 + 3] - b2 : 0;
        }
        qa[u] = a; qn[u] = an; da[u] = b2; dn_[u] = bn;
    }
    __syncthreads();
    ItemSetup r;
    r.nq = 0;
    r.nd = 0;
    for (int u = 0; u < 9; ++u) {
        r.nq += qn[u];
        r.nd += dn_[u];
    }
    r.c = min(64, ntot - item.y);
    r.g = NTB / r.c;
    r.ti = lane % r.c;
    r.sub = lane / r.c;
    r.valid = r.sub < r.g;
    int k = item.y + r.ti;
    r.t = -1;
    for (int s = 0; s < 3; ++s) {
        const int n = re[s] - rs[s];
        if (r.t < 0 && k < n) r.t = rs[s] + k;
        k -= n;
    }
    return r;
}

// sorted index of flat U-list source f of a set (counts cnt, starts st)
__device__ __forceinline__ int flat_source(int f, const int *cnt, const int *st) {
    int u = 0;
    while (u < 8 && f >= cnt[u]) { f -= cnt[u]; ++u; }
    return st[u] + f;
}

template <int NT, bool kSmallOnly, bool kF32>
__global__ __launch_bounds__(64) void k_near_build(
    const int2 *__restrict__ items, const int32_t *__restrict__ lrange,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist,
    const double *__restrict__ px, const double *__restrict__ py, int q_on, int d_on, int mask,
    double inv2a, const int64_t *__restrict__ qoff, const int64_t *__restrict__ doff,
    typename std::conditional<kF32, float, double>::type *__restrict__ Mq,
    typename std::conditional<kF32, float, double>::type *__restrict__ Md) {
    using VT = typename std::conditional<kF32, float, double>::type;
    __shared__ double s_x[kLeafStage], s_y[kLeafStage];
    __shared__ double2 s_log[YK_LOG_TAB];
    __shared__ int qa[9], qn[9], da[9], dn_[9];
    const int ib = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if constexpr (!kF32)
        for (int i = lane; i < YK_LOG_TAB; i += 64) s_log[i] = make_double2(yk_log_tab[2 * i], yk_log_tab[2 * i + 1]);
    const ItemSetup it = item_setup(items[ib], lrange, uoff, ulist, q_on, d_on, mask, qa, qn, da, dn_);
    const double xs = px[it.t], ys = py[it.t];   // unscaled: see k_leaf
    for (int set = 0; set < 2; ++set) {
        const int ntot_s = set == 0 ? it.nq : it.nd;
        VT *Mb = set == 0 ? Mq + qoff[ib] : Md + 2 * doff[ib];
        for (int c0 = 0; c0 < ntot_s; c0 += kLeafStage) {
            const int cn = min(kLeafStage, ntot_s - c0);
            __syncthreads();
            for (int f = lane; f < cn; f += 64) {
                const int j = flat_source(c0 + f, set == 0 ? qn : dn_, set == 0 ? qa : da);
                s_x[f] = px[j];
                s_y[f] = py[j];
            }
            __syncthreads();
            if (!it.valid) continue;
            for (int j = it.sub; j < cn; j += it.g) {
                const double dx = (xs - s_x[j]) * inv2a, dy = (ys - s_y[j]) * inv2a;
                const double tt = __builtin_fma(dx, dx, dy * dy);
                const int64_t e = (int64_t)(c0 + j) * it.c + it.ti;
                if (set == 0) {
                    double v = 0.0;
                    if (tt > 0.0) {
                        if constexpr (kF32) v = (double)near_k0_f<kSmallOnly>((float)tt);
                        else v = near_k0<NT, kSmallOnly>(tt, s_log);
                    }
                    Mb[e] = (VT)v;
                } else {
                    double k = 0.0;
                    if (tt > 0.0) {
                        if constexpr (kF32) k = (double)near_k1oz4_f<kSmallOnly>((float)tt);
                        else k = near_k1oz4<NT, kSmallOnly>(tt, s_log);
                    }
                    Mb[2 * e] = (VT)(dx * k);
                    Mb[2 * e + 1] = (VT)(dy * k);
                }
            }
        }
    }
}

// NTB = 64, or 256 for trees with too few items to fill the GPU (the layout
// of the values does not depend on how many lanes share a target)
template <typename VT, int NTB>
__global__ __launch_bounds__(NTB) void k_near_apply(
    const int2 *__restrict__ items, const int32_t *__restrict__ lrange,
    const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist,
    const double *__restrict__ qs, const double *__restrict__ dns, int64_t off1, int q_on, int d_on,
    int has_q, int has_d, int mask, const int64_t *__restrict__ qoff, const int64_t *__restrict__ doff,
    const VT *__restrict__ Mq, const VT *__restrict__ Md, double dip_scale, double *__restrict__ outs) {
    __shared__ double s_a[NTB > kLeafStage ? NTB : kLeafStage], s_b[kLeafStage];
    __shared__ int qa[9], qn[9], da[9], dn_[9];
    const int ib = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const ItemSetup it = item_setup<NTB>(items[ib], lrange, uoff, ulist, q_on, d_on, mask, qa, qn, da, dn_);
    double near_q = 0.0, near_d = 0.0;
    for (int set = 0; set < 2; ++set) {
        if ((set == 0 && !has_q) || (set == 1 && !has_d)) continue;
        const int ntot_s = set == 0 ? it.nq : it.nd;
        for (int c0 = 0; c0 < ntot_s; c0 += kLeafStage) {
            const int cn = min(kLeafStage, ntot_s - c0);
            __syncthreads();
            for (int f = lane; f < cn; f += NTB) {
                const int j = flat_source(c0 + f, set == 0 ? qn : dn_, set == 0 ? qa : da);
                if (set == 0) {
                    s_a[f] = qs[j];
                } else {
                    const int64_t jd = j - off1;
                    s_a[f] = dns[2 * jd];
                    s_b[f] = dns[2 * jd + 1];
                }
            }
            __syncthreads();
            if (!it.valid) continue;
            // the values are read once per pass: eight loads in flight per lane
            // (explicitly, the trip count is data dependent), non-temporal
            const int gs = it.g;
            const int64_t cs = (int64_t)it.c * gs;   // element stride of one pass
            if (set == 0) {
                const VT *Mb = Mq + qoff[ib] + (int64_t)c0 * it.c + it.ti + (int64_t)it.sub * it.c;
                int j = it.sub;
                for (; j + 7 * gs < cn; j += 8 * gs, Mb += 8 * cs) {
                    VT m[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) m[u] = __builtin_nontemporal_load(Mb + u * cs);
#pragma unroll
                    for (int u = 0; u < 8; ++u) near_q = __builtin_fma((double)m[u], s_a[j + u * gs], near_q);
                }
                for (; j < cn; j += gs, Mb += cs) near_q = __builtin_fma((double)__builtin_nontemporal_load(Mb), s_a[j], near_q);
            } else {
                const VT *Mb = Md + 2 * (doff[ib] + (int64_t)c0 * it.c + it.ti + (int64_t)it.sub * it.c);
                int j = it.sub;
                for (; j + 3 * gs < cn; j += 4 * gs, Mb += 8 * cs) {
                    VT mx[4], my[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        mx[u] = __builtin_nontemporal_load(Mb + 2 * u * cs);
                        my[u] = __builtin_nontemporal_load(Mb + 2 * u * cs + 1);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        near_d = __builtin_fma((double)mx[u], s_a[j + u * gs],
                                               __builtin_fma((double)my[u], s_b[j + u * gs], near_d));
                }
                for (; j < cn; j += gs, Mb += 2 * cs)
                    near_d = __builtin_fma((double)__builtin_nontemporal_load(Mb), s_a[j],
                                           __builtin_fma((double)__builtin_nontemporal_load(Mb + 1), s_b[j], near_d));
            }
        }
    }
    __syncthreads();
    s_a[lane] = it.valid ? near_q + dip_scale * near_d : 0.0;
    __syncthreads();
    if (it.sub == 0) {
        double tot = 0.0;
        for (int gi = 0; gi < it.g; ++gi) tot += s_a[it.ti + gi * it.c];
        outs[it.t] = tot * kInv2Pi;
    }
}

// ---------------------------------------------------- symmetric near field --
// The charge-to-charge values K0(|x - y|/alpha) are symmetric in the two
// points.  When no leaf holds more than 64 charges (and the charges are among
// the targets), the block of each unordered pair of neighbouring leaves {A, B}
// is stored once, with the leaf of smaller index
// (its owner), and the owner's item applies it both ways: to its own charges
// (a sum over B's charges) and, transposed, to B's charges (a sum over its
// own), the latter written to B's incoming slot, which k_l2p adds.  A leaf's
// own block is stored whole.  A leaf's charges lead its targets, so they all
// fall in its first item.  Per item (starting at a
// multiple of four entries) the charge values are, source major and target
// minor: (1) the item's charges as targets against the charges of the owned
// neighbours (the leaf itself and those of larger index, in U-list order),
// each source's row padded with zeros to a multiple of four targets, (2) its
// other targets against the charges of all neighbours.  The dipole values keep
// the layout of k_near_build.
//
// owned charge count of each U-list entry (lanes < 9; published by the
// barrier in item_setup)
__device__ __forceinline__ void owned_counts(int li, const int32_t *__restrict__ lrange,
                                             const int32_t *__restrict__ uoff, const int32_t *__restrict__ ulist,
                                             int *qo) {
    const int lane = threadIdx.x;
    if (lane < 9) {
        const int u0 = uoff[li], nu = uoff[li + 1] - u0;
        int o = 0;
        if (lane < nu) {
            const int ul = ulist[u0 + lane];
            if (ul >= li) o = lrange[ul * 6 + 1] - lrange[ul * 6];
        }
        qo[lane] = o;
    }
}

// sorted index of the k-th target of a leaf (sets in order, those of the mask)
__device__ __forceinline__ int item_target(int li, int k, const int32_t *__restrict__ lrange, int mask) {
    for (int s = 0; s < 3; ++s) {
        const int rs = lrange[li * 6 + 2 * s], n = (mask >> s) & 1 ? lrange[li * 6 + 2 * s + 1] - rs : 0;
        if (k < n) return rs + k;
        k -= n;
    }
    return -1;
}

template <int NT, bool kSmallOnly, bool kF32>
__global__ __launch_bounds__(64) void k_near_build_sym(
    const int2 *__restrict__ items, const int32_t *__restrict__ lrange, const int32_t *__restrict__ uoff,
    const int32_t *__restrict__ ulist, const double *__restrict__ px, const double *__restrict__ py, int mask,
    double inv2a, const int64_t *__restrict__ qoff,
    typename std::conditional<kF32, float, double>::type *__restrict__ Mq) {
    using VT = typename std::conditional<kF32, float, double>::type;
    __shared__ double2 s_log[YK_LOG_TAB];
    __shared__ int qa[9], qn[9], da[9], dn_[9], qo[9];
    const int ib = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    if constexpr (!kF32)
        for (int i = lane; i < YK_LOG_TAB; i += 64) s_log[i] = make_double2(yk_log_tab[2 * i], yk_log_tab[2 * i + 1]);
    const int2 item = items[ib];
    const int li = item.x;
    owned_counts(li, lrange, uoff, ulist, qo);
    const ItemSetup it = item_setup(item, lrange, uoff, ulist, 1, 0, mask, qa, qn, da, dn_);
    int nown = 0;
    for (int u = 0; u < 9; ++u) nown += qo[u];
    // (the mask has the charges; they lead a leaf's targets, all in its first item)
    const int rs0 = lrange[li * 6], nA0 = item.y == 0 ? lrange[li * 6 + 1] - rs0 : 0;
    const int cB = it.c - nA0;
    auto value = [&](int t, int j) -> VT {
        const double dx = (px[t] - px[j]) * inv2a, dy = (py[t] - py[j]) * inv2a;
        const double tt = __builtin_fma(dx, dx, dy * dy);
        double v = 0.0;
        if (tt > 0.0) {
            if constexpr (kF32) v = (double)near_k0_f<kSmallOnly>((float)tt);
            else v = near_k0<NT, kSmallOnly>(tt, s_log);
        }
        return (VT)v;
    };
    VT *M1 = Mq + qoff[ib];
    const int cA4 = (nA0 + 3) & ~3;
    const int64_t n1 = (int64_t)cA4 * nown;
    for (int64_t e = lane; e < n1; e += 64) {
        const int f = (int)(e / cA4), t = (int)(e % cA4);
        M1[e] = t < nA0 ? value(rs0 + t, flat_source(f, qo, qa)) : (VT)0;
    }
    VT *M2 = M1 + n1;
    const int64_t n2 = (int64_t)cB * it.nq;
    for (int64_t e = lane; e < n2; e += 64) {
        const int f = (int)(e / cB), k = (int)(e % cB);
        M2[e] = value(item_target(li, item.y + nA0 + k, lrange, mask), flat_source(f, qn, qa));
    }
}

// Per-item descriptor of the symmetric near field (built with the plan): for
// the nine U-list entries the first charge, the charge count, the owned charge
// count, the first dipole and the dipole count (entries 0-44), the item's
// target ranges per set, empty for sets outside the mask (45-47 first, 48-50
// end), its first target (51); and per entry the incoming slot it writes.
constexpr int kItemDesc = 52;

template <int NTB>
__device__ __forceinline__ ItemSetup setup_from_desc(const int *d) {
    const int lane = threadIdx.x;
    ItemSetup r;
    r.nq = 0;
    r.nd = 0;
    for (int u = 0; u < 9; ++u) {
        r.nq += d[9 + u];
        r.nd += d[36 + u];
    }
    int ntot = 0;
    for (int s = 0; s < 3; ++s) ntot += d[48 + s] - d[45 + s];
    const int y = d[51];
    r.c = min(64, ntot - y);
    r.g = NTB / r.c;
    r.ti = lane % r.c;
    r.sub = lane / r.c;
    r.valid = r.sub < r.g;
    int k = y + r.ti;
    r.t = -1;
    for (int s = 0; s < 3; ++s) {
        const int n = d[48 + s] - d[45 + s];
        if (r.t < 0 && k < n) r.t = d[45 + s] + k;
        k -= n;
    }
    return r;
}

// Sources per lane and batch in the owned charge block (each lane has this
// many quarter rows of four values in flight).
constexpr int kSymRounds = 4;

// four consecutive values (16-byte aligned for float, 32 for double), read once
__device__ __forceinline__ void load4(const double *p, double (&o)[4]) {
    const yk_dpair a = __builtin_nontemporal_load(reinterpret_cast<const yk_dpair *>(p));
    const yk_dpair b = __builtin_nontemporal_load(reinterpret_cast<const yk_dpair *>(p) + 1);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void load4(const float *p, double (&o)[4]) {
    const yk_f4 a = __builtin_nontemporal_load(reinterpret_cast<const yk_f4 *>(p));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}

template <typename VT, int NTB>
__global__ __launch_bounds__(NTB) __attribute__((amdgpu_waves_per_eu(5))) void k_near_apply_sym(
    const int32_t *__restrict__ desc, const int64_t *__restrict__ desc_dst, const double *__restrict__ qs,
    const double *__restrict__ dns, int64_t off1, int has_q, int has_d, const int64_t *__restrict__ qoff, const int64_t *__restrict__ doff, const VT *__restrict__ Mq,
    const VT *__restrict__ Md, double dip_scale, double *__restrict__ outs, double *__restrict__ inc) {
    __shared__ double s_a[NTB > kLeafStage ? NTB : kLeafStage], s_b[kLeafStage];
    __shared__ double s_res[64];
    __shared__ double s_p[4 * NTB];   // direct sums of part (1), four targets per lane
    __shared__ int s_d[kItemDesc], s_pre[9];
    __shared__ int64_t s_dst[9];
    const int ib = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    // the item's descriptor: one round trip instead of the chain leaf -> U list -> ranges
    if (lane < kItemDesc) s_d[lane] = desc[(int64_t)ib * kItemDesc + lane];
    if (lane < 9) s_dst[lane] = desc_dst[(int64_t)ib * 9 + lane];
    if (lane < 64) s_res[lane] = 0.0;
    __syncthreads();
    const int *qa = s_d, *qn = s_d + 9, *qo = s_d + 18, *da = s_d + 27, *dn_ = s_d + 36;
    const ItemSetup it = setup_from_desc<NTB>(s_d);
    // first owned source of each U-list entry (published by part (1)'s barriers)
    if (lane < 9) {
        int a = 0;
        for (int u = 0; u < lane; ++u) a += qo[u];
        s_pre[lane] = a;
    }
    const int c = it.c;
    // the leaf's charges (at most 64) lead its targets, all in its first item
    const int rs0 = s_d[45], nA0 = s_d[51] == 0 ? s_d[48] - rs0 : 0;
    int nown = 0;
    for (int u = 0; u < 9; ++u) nown += qo[u];
    // (1) the item's charges against the owned charges, both ways.  A lane
    // takes four consecutive targets (one quarter row) of four sources per
    // batch, read as vectors; it sums the direct products over its sources in
    // registers for the whole block and the transposed ones over its targets,
    // then over the tb lanes that share the sources (shuffles within a
    // wavefront: the lanes of a source never straddle one).
    if (has_q && nA0 > 0) {
        const int cA = nA0, cA4 = (cA + 3) & ~3, tb = cA4 >> 2;
        const int nf = 64 / tb, nfb = (NTB / 64) * nf;
        const int wl = lane & 63, lt = wl % tb;
        const int fs = (lane >> 6) * nf + wl / tb;
        const bool vA = wl / tb < nf;
        double qa4[4], y4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 4 * lt + i;
            qa4[i] = (vA && t < cA) ? qs[rs0 + t] : 0.0;
            y4[i] = 0.0;
        }
        const VT *Mb = Mq + qoff[ib] + 4 * lt;
        for (int c0 = 0; c0 < nown; c0 += kLeafStage) {
            const int cn = min(kLeafStage, nown - c0);
            double w[kSymRounds][4];
            // rounds of a batch that hold sources (the same for all lanes)
            int nr = 0;
            auto load_batch = [&](int r0) {
                nr = min(kSymRounds, (cn - r0 + nfb - 1) / nfb);
#pragma unroll
                for (int j = 0; j < kSymRounds; ++j) {
                    const int f = r0 + j * nfb + fs;
                    if (j < nr && vA && f < cn) {
                        load4(Mb + (int64_t)(c0 + f) * cA4, w[j]);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) w[j][i] = 0.0;
                    }
                }
            };
            // the first batch is in flight while the sources' charges are staged
            load_batch(0);
            __syncthreads();
            for (int f = lane; f < cn; f += NTB) s_a[f] = qs[flat_source(c0 + f, qo, qa)];
            __syncthreads();
            for (int r0 = 0; r0 < cn; r0 += kSymRounds * nfb) {
                if (r0 > 0) load_batch(r0);
                double z[kSymRounds];
#pragma unroll
                for (int j = 0; j < kSymRounds; ++j) {
                    z[j] = 0.0;
                    if (j >= nr) continue;
                    const int f = r0 + j * nfb + fs;
                    const double qb = (vA && f < cn) ? s_a[f] : 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        y4[i] = __builtin_fma(w[j][i], qb, y4[i]);
                        z[j] = __builtin_fma(w[j][i], qa4[i], z[j]);
                    }
                }
                for (int k = 1; k < tb; k <<= 1) {
                    const bool in = lt + k < tb;
#pragma unroll
                    for (int j = 0; j < kSymRounds; ++j) {
                        if (j >= nr) continue;
                        const double o = __shfl_down(z[j], k, 64);
                        z[j] += in ? o : 0.0;
                    }
                }
                if (vA && lt == 0) {
#pragma unroll
                    for (int j = 0; j < kSymRounds; ++j) {
                        const int f = r0 + j * nfb + fs;
                        if (f >= cn) break;
                        // the U-list entry of owned source c0 + f: the last one
                        // starting at or before it (empty entries share the
                        // next one's start)
                        const int ff = c0 + f;
                        int u = 0;
#pragma unroll
                        for (int k = 1; k < 9; ++k) u += ff >= s_pre[k] ? 1 : 0;
                        const int64_t d = s_dst[u];
                        if (d >= 0) inc[d + ff - s_pre[u]] = z[j] * kInv2Pi;
                    }
                }
            }
        }
        // the direct sums over the source slots: lane (slot, lt) holds targets 4 lt .. 4 lt + 3
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) s_p[4 * lane + i] = vA ? y4[i] : 0.0;
        __syncthreads();
        if (lane < cA) {
            double tot = 0.0;
            for (int q = 0; q < nfb; ++q) {
                const int ln = (q / nf) * 64 + (q % nf) * tb + (lane >> 2);
                tot += s_p[4 * ln + (lane & 3)];
            }
            s_res[lane] += tot;
        }
    }
    // (2) the item's other targets against all neighbouring charges
    const int cB = c - nA0;
    if (has_q && cB > 0 && it.nq > 0) {
        const int gB = NTB / cB, tiB = lane % cB, subB = lane / cB;
        const bool vB = subB < gB;
        const VT *Mb = Mq + qoff[ib] + (int64_t)((nA0 + 3) & ~3) * nown;
        double acc = 0.0;
        for (int c0 = 0; c0 < it.nq; c0 += kLeafStage) {
            const int cn = min(kLeafStage, it.nq - c0);
            __syncthreads();
            for (int f = lane; f < cn; f += NTB) s_a[f] = qs[flat_source(c0 + f, qn, qa)];
            __syncthreads();
            if (!vB) continue;
            const VT *Mr = Mb + (int64_t)c0 * cB + tiB + (int64_t)subB * cB;
            const int64_t cs = (int64_t)cB * gB;
            int j = subB;
            for (; j + 7 * gB < cn; j += 8 * gB, Mr += 8 * cs) {
                VT m[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) m[u] = __builtin_nontemporal_load(Mr + u * cs);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = __builtin_fma((double)m[u], s_a[j + u * gB], acc);
            }
            for (; j < cn; j += gB, Mr += cs) acc = __builtin_fma((double)__builtin_nontemporal_load(Mr), s_a[j], acc);
        }
        __syncthreads();
        s_a[lane] = vB ? acc : 0.0;
        __syncthreads();
        if (lane < cB) {
            double tot = 0.0;
            for (int s = 0; s < gB; ++s) tot += s_a[s * cB + lane];
            s_res[nA0 + lane] += tot;
        }
    }
    // (3) every target against the dipoles (layout of k_near_build)
    if (has_d && it.nd > 0) {
        double acc = 0.0;
        for (int c0 = 0; c0 < it.nd; c0 += kLeafStage) {
            const int cn = min(kLeafStage, it.nd - c0);
            __syncthreads();
            for (int f = lane; f < cn; f += NTB) {
                const int64_t jd = flat_source(c0 + f, dn_, da) - off1;
                s_a[f] = dns[2 * jd];
                s_b[f] = dns[2 * jd + 1];
            }
            __syncthreads();
            if (!it.valid) continue;
            const int gs = it.g;
            const int64_t cs = (int64_t)c * gs;
            const VT *Mr = Md + 2 * (doff[ib] + (int64_t)c0 * c + it.ti + (int64_t)it.sub * c);
            int j = it.sub;
            for (; j + 3 * gs < cn; j += 4 * gs, Mr += 8 * cs) {
                VT mx[4], my[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    mx[u] = __builtin_nontemporal_load(Mr + 2 * u * cs);
                    my[u] = __builtin_nontemporal_load(Mr + 2 * u * cs + 1);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc = __builtin_fma((double)mx[u], s_a[j + u * gs], __builtin_fma((double)my[u], s_b[j + u * gs], acc));
            }
            for (; j < cn; j += gs, Mr += 2 * cs)
                acc = __builtin_fma((double)__builtin_nontemporal_load(Mr), s_a[j],
                                    __builtin_fma((double)__builtin_nontemporal_load(Mr + 1), s_b[j], acc));
        }
        __syncthreads();
        s_a[lane] = it.valid ? acc : 0.0;
        __syncthreads();
        if (lane < c) {
            double tot = 0.0;
            for (int s = 0; s < it.g; ++s) tot += s_a[s * c + lane];
            s_res[lane] += dip_scale * tot;
        }
    }
    __syncthreads();
    if (lane < c) outs[it.t] = s_res[lane] * kInv2Pi;
}

using NearBuild64 = void (*)(const int2 *, const int32_t *, const int32_t *, const int32_t *,
                             const double *, const double *, int, int, int, double, const int64_t *,
                             const int64_t *, double *, double *);
using NearBuild32 = void (*)(const int2 *, const int32_t *, const int32_t *, const int32_t *,
                             const double *, const double *, int, int, int, double, const int64_t *,
                             const int64_t *, float *, float *);

NearBuild64 pick_near_build64(int nt, bool small_only) {
    if (small_only) {
        if (nt <= 5) return k_near_build<5, true, false>;
        if (nt <= 6) return k_near_build<6, true, false>;
        if (nt <= 8) return k_near_build<8, true, false>;
        if (nt <= 10) return k_near_build<10, true, false>;
        return k_near_build<14, true, false>;
    }
    return k_near_build<14, false, false>;
}
NearBuild32 pick_near_build32(bool small_only) {
    return small_only ? k_near_build<8, true, true> : k_near_build<8, false, true>;
}
using NearBuildSym64 = void (*)(const int2 *, const int32_t *, const int32_t *, const int32_t *,
                                const double *, const double *, int, double, const int64_t *, double *);
using NearBuildSym32 = void (*)(const int2 *, const int32_t *, const int32_t *, const int32_t *,
                                const double *, const double *, int, double, const int64_t *, float *);
NearBuildSym64 pick_near_build_sym64(int nt, bool small_only) {
    if (small_only) {
        if (nt <= 5) return k_near_build_sym<5, true, false>;
        if (nt <= 6) return k_near_build_sym<6, true, false>;
        if (nt <= 8) return k_near_build_sym<8, true, false>;
        if (nt <= 10) return k_near_build_sym<10, true, false>;
        return k_near_build_sym<14, true, false>;
    }
    return k_near_build_sym<14, false, false>;
}
NearBuildSym32 pick_near_build_sym32(bool small_only) {
    return small_only ? k_near_build_sym<8, true, true> : k_near_build_sym<8, false, true>;
}

using LeafKernel = void (*)(const int2 *, int64_t, const int32_t *, const int32_t *,
                            const int32_t *, const double *, const double *, const double *,
                            const double *, int64_t, int, int, int, double, double, double *);

// L2P: one thread per target point, adding the local expansion of the
// point's leaf (Horner in z with G_m = F_m(y)/F_m(Y), F_m downwards) to the
// near-field sum already in outs.  The level's tables are staged in LDS.
__global__ __launch_bounds__(256) void k_l2p(
    int64_t n, int64_t toff1, int64_t toff2, int mask, const int32_t *__restrict__ pleaf,
    int64_t leaf_base, const double *__restrict__ bcx, const double *__restrict__ bcy,
    const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ Lc,
    double inv_alpha, double invR, const double *__restrict__ invFY, const double *__restrict__ cnn,
    const double *__restrict__ sc, int nser, int p, int Pp, const double *__restrict__ outs,
    const int32_t *__restrict__ perm, double *__restrict__ out0, double *__restrict__ out1,
    double *__restrict__ out2, const double *__restrict__ bw, const double *__restrict__ bk,
    const double *__restrict__ bx, const double *__restrict__ inc, const int64_t *__restrict__ inc_base,
    const int32_t *__restrict__ inc_cnt, const int32_t *__restrict__ lrange) {
    extern __shared__ double dyn[];
    double *t_cnn = dyn;               // [p+1]
    double *t_ify = t_cnn + p + 1;     // [p+1]
    double *t_sc = t_ify + p + 1;      // [2 nser]
    for (int i = threadIdx.x; i < p + 1; i += blockDim.x) {
        t_cnn[i] = cnn[i];
        t_ify[i] = invFY[i];
    }
    for (int i = threadIdx.x; i < 2 * nser; i += blockDim.x) t_sc[i] = sc[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int set = (t >= toff1) + (t >= toff2);
    if (!((mask >> set) & 1)) return;
    const int32_t lb = pleaf[t];
    const int64_t b = leaf_base + lb;
    const double *Lb = Lc + b * Pp;
    // the incoming slots of the symmetric near field (charge targets): their
    // indices are read before the series, which hides the loads behind it
    int32_t n_in = 0, n0 = 0;
    int64_t in_base = 0;
    if (set == 0 && inc) {
        const int32_t s0 = lrange[lb * 6];
        n0 = lrange[lb * 6 + 1] - s0;
        in_base = inc_base[lb] + (t - s0);
        n_in = inc_cnt[lb];
    }
    const double wx = (px[t] - bcx[b]) * inv_alpha, wy = (py[t] - bcy[b]) * inv_alpha;
    const double yv = 0.25 * (wx * wx + wy * wy);
    const double zx = wx * invR, zy = wy * invR;
    double F1, F2;
    f_start(yv, t_sc, nser, F1, F2);
    double sr = 0.0, si = 0.0;
#pragma unroll 4
    for (int m = p; m >= 1; --m) {
        const double F0 = F1 + yv * F2 * t_cnn[m];
        const double gm = F0 * t_ify[m];
        const double cr = Lb[2 * m - 1] * gm, ci = Lb[2 * m] * gm;
        const double nr = sr * zx - si * zy + cr;
        si = sr * zy + si * zx + ci;
        sr = nr;
        F2 = F1;
        F1 = F0;
    }
    const double F0 = F1 + yv * F2 * t_cnn[0];
    // near field + far field, written straight to the caller's array of the set
    double v = outs[t] + (Lb[0] * F0 * t_ify[0] + 2.0 * (sr * zx - si * zy)) * kInv2Pi;
    // symmetric near field: the charges of the neighbours that own the pair
    // blocks with this leaf, one incoming slot per owner
    for (int k = 0; k < n_in; ++k) v += inc[in_base + (int64_t)k * n0];
    double *o = set == 0 ? out0 : set == 1 ? out1 : out2;
    const int32_t i = perm[t];
    if (set == 1 && bx)   // double-layer operator: x - 2 (DL + corrected diagonal)
        o[i] = bx[i] - 2.0 * (v + dl_diag_weight(bw[i], bk[i], inv_alpha * inv_alpha) * bx[i]);
    else
        o[i] = v;
}

// ------------------------------------------------------- adaptive tree ---
// beyond this scaled distance K_0 < 1e-250: the pair is dropped (also keeps
// K_0 and the ratio K_1/K_0 away from underflow)
constexpr double kFarRho = 600.0;
// The products I_n(R_l) K_n(rho) of the W and X translations, from I_0(R_l)
// K_0(rho) by the ratios of I (a per-level table, rI[l] = {I_0(R_l),
// I_n(R_l)/I_{n-1}(R_l)}) and of K (the upward recurrence K_{n+1} = K_{n-1} +
// (2n/rho) K_n, stable for K, run on the ratios), so that no factor leaves
// the range of doubles however small the box.

// W list (M2P): the multipole of every box of the leaf's W list evaluated at
// the leaf's targets, phi(x) = sum_n M_n F^K_n((x - c)/alpha) =
// M_0 K_0 + 2 sum_{n>=1} Re(M_n e^{in theta}) K_n, added to the near-field
// sums in outs.  One wavefront per leaf, a lane per target; each target sums
// its boxes in list order (deterministic, no atomics).
__global__ __launch_bounds__(64) void k_ad_m2p(
    const int32_t *__restrict__ wleaves, const int32_t *__restrict__ woff, const int32_t *__restrict__ wl,
    const int32_t *__restrict__ lrange, int mask, const int32_t *__restrict__ blevel,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ M, const double *__restrict__ rI, int p, int Pp,
    double inv_alpha, double *__restrict__ outs) {
    const int li = wleaves[blockIdx.x];
    const int w0 = woff[li], w1 = woff[li + 1];
    int rs[3], rn[3], ntot = 0;
    for (int st = 0; st < 3; ++st) {
        rs[st] = lrange[li * 6 + 2 * st];
        rn[st] = (mask >> st) & 1 ? lrange[li * 6 + 2 * st + 1] - rs[st] : 0;
        ntot += rn[st];
    }
    // a leaf with few targets (at most 16 or 32) splits its W list among 4 or
    // 2 lane groups, whose partial sums meet in a fixed shuffle order
    const int G = ntot <= 16 ? 4 : ntot <= 32 ? 2 : 1, T = 64 / G;
    const int g = threadIdx.x / T, kl = threadIdx.x - g * T;
    for (int kb = 0; kb < ntot; kb += T) {
        const int k = kb + kl;
        int t = -1;
        double acc = 0.0;
        if (k < ntot) {
            int r = k;
            for (int st = 0; st < 3; ++st) {
                if (t < 0 && r < rn[st]) t = rs[st] + r;
                r -= rn[st];
            }
            const double x = px[t], y = py[t];
            for (int w = w0 + g; w < w1; w += G) {
                const int32_t d = wl[w];
                const double *Md = M + (int64_t)d * Pp;
                const double *ri = rI + (int64_t)blevel[d] * (p + 3);
                const double wx = (x - bcx[d]) * inv_alpha, wy = (y - bcy[d]) * inv_alpha;
                const double rho = sqrt(wx * wx + wy * wy), ir = 1.0 / rho;
                if (rho > kFarRho) continue;          // below 1e-250 of the box's sources
                const double c = wx * ir, sn = wy * ir;
                const double k0v = k0(rho);
                double rk = k1(rho) / k0v;            // K_1 / K_0
                double T0 = ri[0] * k0v;              // I_0(R) K_0(rho)
                double sum = Md[0] * T0;
                double er = c, ei = sn;               // e^{i n theta}
                for (int n = 1; n <= p; ++n) {
                    T0 *= ri[n] * rk;                 // I_n(R) K_n(rho)
                    sum += 2.0 * T0 * (Md[2 * n - 1] * er - Md[2 * n] * ei);
                    rk = 1.0 / rk + 2.0 * n * ir;     // K_{n+1} / K_n
                    const double nr = er * c - ei * sn;
                    ei = er * sn + ei * c;
                    er = nr;
                }
                acc += sum;
            }
        }
        if (G == 4) acc += __shfl_xor(acc, 16, 64);
        if (G >= 2) acc += __shfl_xor(acc, 32, 64);
        if (t >= 0 && g == 0) outs[t] += acc * kInv2Pi;
    }
}

// X list (P2L): the sources of every leaf of the box's X list into the box's
// local expansion (scaled, Lh_m = L_m I_m(R_l)).  By Graf's addition theorem a
// charge q at w = (y - c)/alpha contributes L_m = q K_m(|w|) e^{-i m theta};
// a dipole D = d (n_x + i n_y), the normal derivative at y of that,
// L_m = -(1/(2 alpha)) [conj(D) K_{|m-1|} e^{-i(m-1) theta} + D K_{m+1}
// e^{-i(m+1) theta}].  One wavefront per box: per batch of 64 sources each
// lane writes its source's P terms to LDS, then lane o adds up output o over
// the batch (a fixed order); the box's row is added once at the end.
constexpr int kP2LStride = 65;   // LDS row stride (doubles): conflict-free transposed reads

__global__ __launch_bounds__(64) void k_ad_p2l(
    const int32_t *__restrict__ xbox, const int32_t *__restrict__ xoff, const int32_t *__restrict__ xl,
    const int32_t *__restrict__ lrange, int has_q, int has_d, const int32_t *__restrict__ blevel,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ qs, const double *__restrict__ dns, int64_t off1,
    const double *__restrict__ rI, int p, int Pp, double inv_alpha, double *__restrict__ Lc) {
    extern __shared__ double sh[];   // [Pp][kP2LStride]
    const int lane = threadIdx.x;
    const int32_t d = xbox[blockIdx.x];
    const double *ri = rI + (int64_t)blevel[d] * (p + 3);
    const double cx = bcx[d], cy = bcy[d], h = 0.5 * inv_alpha;
    const int P = 2 * p + 1;
    double acc = 0.0;
    for (int xi = xoff[blockIdx.x]; xi < xoff[blockIdx.x + 1]; ++xi) {
        const int32_t c = xl[xi];
        for (int set = 0; set < 2; ++set) {
            if ((set == 0 && !has_q) || (set == 1 && !has_d)) continue;
            const int a = lrange[c * 6 + 2 * set], e = lrange[c * 6 + 2 * set + 1];
            for (int base = a; base < e; base += 64) {
                const int j = base + lane;
                double *col = sh + lane;
                const double wx = j < e ? (px[j] - cx) * inv_alpha : 0.0;
                const double wy = j < e ? (py[j] - cy) * inv_alpha : 0.0;
                const double rho = sqrt(wx * wx + wy * wy);
                if (j < e && rho <= kFarRho) {
                    const double ir = 1.0 / rho;
                    const double co = wx * ir, sn = wy * ir;
                    const double k0v = k0(rho);
                    double rk = k1(rho) / k0v;
                    double T = ri[0] * k0v;                    // T_0 = I_0 K_0
                    if (set == 0) {
                        const double q = qs[j];
                        col[0] = q * T;
                        double er = co, ei = sn;
                        for (int m = 1; m <= p; ++m) {
                            T *= ri[m] * rk;                   // T_m
                            rk = 1.0 / rk + 2.0 * m * ir;
                            col[(2 * m - 1) * kP2LStride] = q * T * er;
                            col[(2 * m) * kP2LStride] = -q * T * ei;
                            const double nr = er * co - ei * sn;
                            ei = er * sn + ei * co;
                            er = nr;
                        }
                    } else {
                        const double Dx = dns[2 * (j - off1)], Dy = dns[2 * (j - off1) + 1];
                        // T_m and T_{m+1} side by side: A_m = K_{|m-1|} I_m, B_m = K_{m+1} I_m
                        double Tn = T * ri[1] * rk;            // T_1
                        rk = 1.0 / rk + 2.0 * ir;              // K_2 / K_1
                        double Tp = T;                         // T_{m-1} (unused at m = 0)
                        // m = 0: A_0 = B_0 = K_1 I_0 = T_1 / (I_1/I_0)
                        const double B0 = Tn / ri[1];
                        col[0] = -2.0 * h * B0 * (Dx * co + Dy * sn);
                        double ur = 1.0, ui = 0.0;             // e^{i(m-1) theta} at m = 1
                        double vr = co * co - sn * sn, vi = 2.0 * co * sn;   // e^{i(m+1) theta} at m = 1
                        double Tm = Tn;                        // T_m at m = 1
                        for (int m = 1; m <= p; ++m) {
                            Tn = Tm * ri[m + 1] * rk;          // T_{m+1}
                            rk = 1.0 / rk + 2.0 * (m + 1) * ir;
                            const double A = Tp * ri[m];       // K_{m-1} I_m
                            const double B = Tn / ri[m + 1];   // K_{m+1} I_m
                            const double re = -h * (A * (Dx * ur - Dy * ui) + B * (Dx * vr + Dy * vi));
                            const double im = -h * (-A * (Dx * ui + Dy * ur) + B * (Dy * vr - Dx * vi));
                            col[(2 * m - 1) * kP2LStride] = re;
                            col[(2 * m) * kP2LStride] = im;
                            Tp = Tm;
                            Tm = Tn;
                            double t2 = ur * co - ui * sn;
                            ui = ur * sn + ui * co;
                            ur = t2;
                            t2 = vr * co - vi * sn;
                            vi = vr * sn + vi * co;
                            vr = t2;
                        }
                    }
                } else {
                    for (int o = 0; o < P; ++o) col[o * kP2LStride] = 0.0;
                }
                __syncthreads();
                if (lane < P) {
                    const double *row = sh + lane * kP2LStride;
                    double s0 = 0.0, s1 = 0.0;
                    for (int k = 0; k < 64; k += 2) {
                        s0 += row[k];
                        s1 += row[k + 1];
                    }
                    acc += s0 + s1;
                }
                __syncthreads();
            }
        }
    }
    if (lane < P) Lc[(int64_t)d * Pp + lane] += acc;
}

// L2P of the adaptive tree: as k_l2p, with the leaf's level (and its tables)
// per point; leaves coarser than lmin have no local expansion.
__global__ __launch_bounds__(256) void k_ad_l2p(
    int64_t n, int64_t toff1, int64_t toff2, int mask, const int32_t *__restrict__ pleaf,
    const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ leaf_lev, int lmin,
    const double *__restrict__ bcx, const double *__restrict__ bcy, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ Lc, double inv_alpha,
    const double *__restrict__ invR_lv, const double *__restrict__ invFY, const double *__restrict__ cnn,
    const double *__restrict__ serc_lv, const int32_t *__restrict__ nser_lv, int nser_stride, int p, int Pp,
    const double *__restrict__ outs, const int32_t *__restrict__ perm, double *__restrict__ out0,
    double *__restrict__ out1, double *__restrict__ out2, const double *__restrict__ bw,
    const double *__restrict__ bk, const double *__restrict__ bx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int set = (t >= toff1) + (t >= toff2);
    if (!((mask >> set) & 1)) return;
    const int32_t li = pleaf[t];
    const int l = leaf_lev[li];
    double v = outs[t];
    if (l >= lmin) {
        const int64_t b = leaf_box[li];
        const double *Lb = Lc + b * Pp;
        const double *ify = invFY + (int64_t)l * (p + 2);
        const double invR = invR_lv[l];
        const double wx = (px[t] - bcx[b]) * inv_alpha, wy = (py[t] - bcy[b]) * inv_alpha;
        const double yv = 0.25 * (wx * wx + wy * wy);
        const double zx = wx * invR, zy = wy * invR;
        double F1, F2;
        f_start(yv, serc_lv + (int64_t)l * 2 * nser_stride, nser_lv[l], F1, F2);
        double sr = 0.0, si = 0.0;
        for (int m = p; m >= 1; --m) {
            const double F0 = F1 + yv * F2 * cnn[m];
            const double gm = F0 * ify[m];
            const double cr = Lb[2 * m - 1] * gm, ci = Lb[2 * m] * gm;
            const double nr = sr * zx - si * zy + cr;
            si = sr * zy + si * zx + ci;
            sr = nr;
            F2 = F1;
            F1 = F0;
        }
        const double F0 = F1 + yv * F2 * cnn[0];
        v += (Lb[0] * F0 * ify[0] + 2.0 * (sr * zx - si * zy)) * kInv2Pi;
    }
    double *o = set == 0 ? out0 : set == 1 ? out1 : out2;
    const int32_t i = perm[t];
    if (set == 1 && bx)   // double-layer operator: x - 2 (DL + corrected diagonal)
        o[i] = bx[i] - 2.0 * (v + dl_diag_weight(bw[i], bk[i], inv_alpha * inv_alpha) * bx[i]);
    else
        o[i] = v;
}

LeafKernel pick_leaf_kernel(int nt, bool small_only, bool f32, bool adaptive) {
    if (adaptive) {
        if (f32) return small_only ? k_leaf<8, true, true, 16> : k_leaf<8, false, true, 16>;
        if (small_only) {
            if (nt <= 5) return k_leaf<5, true, false, 16>;
            if (nt <= 6) return k_leaf<6, true, false, 16>;
            if (nt <= 8) return k_leaf<8, true, false, 16>;
            if (nt <= 10) return k_leaf<10, true, false, 16>;
            return k_leaf<14, true, false, 16>;
        }
        return k_leaf<14, false, false, 16>;
    }
    if (f32) return small_only ? k_leaf<8, true, true> : k_leaf<8, false, true>;
    if (small_only) {
        if (nt <= 5) return k_leaf<5, true>;
        if (nt <= 6) return k_leaf<6, true>;
        if (nt <= 8) return k_leaf<8, true>;
        if (nt <= 10) return k_leaf<10, true>;
        return k_leaf<14, true>;
    }
    return k_leaf<14, false>;
}

}  // namespace

// one resident round of the persistent M2L: three workgroups per compute unit
int m2l_persist_grid(Context &ctx) {
    static int cus = 0;
    if (cus == 0) {
        int n = 0;
        YK_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx.device));
        cus = n > 0 ? n : 256;
    }
    return 3 * cus;
}

// M2M over levels L-1 .. lmin: each parent box from its children (the
// adaptive tree's split boxes only: a leaf keeps its own multipole)
void fmm_m2m(Context &ctx, FmmPlan &pl) {
    const int L = pl.L, P = pl.P, Pp = pl.Pp;
    {
        StageTimer tmm(ctx, YK_STAGE_M2M);
        for (int l = L - 1; l >= pl.lmin; --l) {
            const int64_t nbl = pl.lev[l].end - pl.lev[l].begin;
            if (pl.adaptive) {
                // the split boxes only (a leaf keeps its P2M multipole)
                if (pl.up_n[l] <= kSmallLevelM2M)
                    launch_small_gemv(ctx, Pp, 4, pl.up_n[l], pl.up_boxes.p + pl.up_off[l], 0, pl.child4.p,
                                      pl.bcode.p, pl.m2m.p + (size_t)l * 4 * Pp * Pp, pl.M.p, P, 1, pl.M.p);
                else
                    launch_tile_gemm<double, double>(ctx, P, Pp, pl.up_tile_count[l], pl.up_tiles.p,
                                                     pl.up_tile_begin[l], pl.up_boxes.p, 4, pl.child4.p,
                                                     pl.iota4.p, pl.m2m.p, (int64_t)4 * Pp * Pp, 0, pl.M.p,
                                                     1, pl.M.p);
            } else if (nbl <= kSmallLevelM2M) {
                launch_small_gemv(ctx, Pp, 4, nbl, nullptr, pl.lev[l].begin, pl.child4.p, pl.bcode.p,
                                  pl.m2m.p + (size_t)l * 4 * Pp * Pp, pl.M.p, P, 1, pl.M.p);
            } else {
                // M2M on matrix cores: 4 child slots, operators S[l][position]
                launch_tile_gemm<double, double>(ctx, P, Pp, pl.up_tile_count[l], pl.up_tiles.p,
                                                 pl.up_tile_begin[l], pl.up_boxes.p, 4, pl.child4.p,
                                                 pl.iota4.p, pl.m2m.p, (int64_t)4 * Pp * Pp, 0, pl.M.p,
                                                 1, pl.M.p);
            }
        }
    }
}

// M2L of every level at once into the zeroed local expansions
void fmm_m2l(Context &ctx, FmmPlan &pl, ActiveSet &as, bool f32) {
    const int P = pl.P, Pp = pl.Pp;
    {
        // M2L of every level at once (levels are independent given the multipoles)
        StageTimer tl(ctx, YK_STAGE_M2L);
        // (FP32: 128-box tiles, two column blocks per wavefront, so each
        // operator fragment feeds two matrix-core steps)
        SlabPlan slab;
        slab.buf = &as.m2l_slab;
        slab.ntgt = as.n_csr_tgt;
        slab.tgt = as.csr_tgt.p;
        slab.off = as.csr_off.p;
        slab.rows = as.csr_rows.p;
        if (as.m2l_sparse && f32)
            launch_tile_gemm<float, float>(ctx, P, Pp, as.n_ptiles, as.m2l_ptiles.p, 0, as.m2l_piota.p,
                                           1, as.m2l_psrc.p, pl.iota40.p, pl.m2lf.p,
                                           (int64_t)kNumOff * Pp * Pp, 0, pl.Mf.p, 0, pl.Lc.p,
                                           as.m2l_ptgt.p, &slab, as.n_ptrans);
        else if (as.m2l_sparse)
            launch_tile_gemm<double, double>(ctx, P, Pp, as.n_ptiles, as.m2l_ptiles.p, 0,
                                             as.m2l_piota.p, 1, as.m2l_psrc.p, pl.iota40.p, pl.m2l.p,
                                             (int64_t)kNumOff * Pp * Pp, 0, pl.M.p, 0, pl.Lc.p,
                                             as.m2l_ptgt.p, &slab, as.n_ptrans);
        else if (f32)
            launch_tile_gemm<float, float, 2>(ctx, P, Pp, as.n_tiles_w, as.m2l_tiles_w.p, 0,
                                              as.m2l_boxes.p, kNumV, pl.vlist.p, pl.slot_oid.p,
                                              pl.m2lf.p, (int64_t)kNumOff * Pp * Pp, 0, pl.Mf.p, 0,
                                              pl.Lc.p, nullptr, &slab);
        else if (Pp == 64 && P == 63 && as.n_tiles >= m2l_persist_grid(ctx)) {
            hipLaunchKernelGGL(k_m2l_persist, dim3(m2l_persist_grid(ctx)), dim3(256), 0, ctx.stream,
                               as.m2l_tiles.p, as.n_tiles, as.m2l_boxes.p, pl.vlist.p, pl.slot_oid.p,
                               pl.m2l.p, (int64_t)kNumOff * Pp * Pp, pl.M.p, pl.Lc.p);
            check_launch(ctx, "k_m2l_persist");
        } else
            launch_tile_gemm<double, double, 1>(ctx, P, Pp, as.n_tiles, as.m2l_tiles.p, 0,
                                                as.m2l_boxes.p, kNumV, pl.vlist.p, pl.slot_oid.p, pl.m2l.p,
                                                (int64_t)kNumOff * Pp * Pp, 0, pl.M.p, 0, pl.Lc.p, nullptr,
                                                &slab);
    }
}

// L2L top-down over levels lmin+1 .. L (each box pulls its parent's expansion)
void fmm_l2l(Context &ctx, FmmPlan &pl, ActiveSet &as, bool f32) {
    const int L = pl.L, P = pl.P, Pp = pl.Pp;
    StageTimer tl2(ctx, YK_STAGE_L2L);
    for (int l = pl.lmin + 1; l <= L; ++l) {
        // L2L top-down: one parent slot, operator E[l-1][position]
        if (as.l2l_count[l] <= kSmallLevelL2L) {
            launch_small_gemv(ctx, Pp, 1, as.l2l_count[l], as.l2l_boxes.p + as.l2l_begin[l], 0,
                              pl.bparent.p, pl.bcode.p, pl.l2l.p + (size_t)(l - 1) * 4 * Pp * Pp,
                              pl.Lc.p, P, 0, pl.Lc.p);
        } else if (f32)
            launch_tile_gemm<float, double>(ctx, P, Pp, as.tile_count[l], as.m2l_tiles.p,
                                            as.tile_begin[l], as.m2l_boxes.p, 1, pl.bparent.p,
                                            pl.iota4.p, pl.l2lf.p, (int64_t)4 * Pp * Pp, -1, pl.Lc.p,
                                            0, pl.Lc.p);
        else
            launch_tile_gemm<double, double>(ctx, P, Pp, as.tile_count[l], as.m2l_tiles.p,
                                             as.tile_begin[l], as.m2l_boxes.p, 1, pl.bparent.p,
                                             pl.iota4.p, pl.l2l.p, (int64_t)4 * Pp * Pp, -1, pl.Lc.p,
                                             0, pl.Lc.p);
    }
}

void fmm_adaptive_finish(Context &ctx, FmmPlan &pl, int mask, double *outs, double *const out[3]) {
    const int p = pl.p, Pp = pl.Pp;
    const double inv_alpha = 1.0 / pl.alpha;
    StageTimer tl(ctx, YK_STAGE_L2P);
    if (pl.n_wleaves > 0 && pl.lmin <= pl.L) {
        hipLaunchKernelGGL(k_ad_m2p, dim3((unsigned)pl.n_wleaves), dim3(64), 0, ctx.stream, pl.wleaves.p, pl.woff.p,
                           pl.wl.p, pl.lrange.p, mask, pl.blevel.p, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p, pl.M.p,
                           pl.rI.p, p, Pp, inv_alpha, outs);
        check_launch(ctx, "k_ad_m2p");
    }
    hipLaunchKernelGGL(k_ad_l2p, dim3(nblk(pl.N, 256)), dim3(256), 0, ctx.stream, pl.N, pl.toff[1], pl.toff[2], mask,
                       pl.pleaf.p, pl.leaf_box.p, pl.leaf_lev.p, pl.lmin, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p,
                       pl.Lc.p, inv_alpha, pl.invR_lv.p, pl.invFY.p, pl.cnn.p, pl.serc_lv.p, pl.nser_dev.p,
                       pl.nser_stride, p, Pp, outs, pl.perm.p, out[0], out[1], out[2], (const double *)nullptr,
                       (const double *)nullptr, (const double *)nullptr);
    check_launch(ctx, "k_ad_l2p");
}

void fmm_run(Context &ctx, FmmPlan &pl, const double *q, const double *dn, double *const out[3],
             SumPrec prec, const BieFuse *bie, int keep_charge_m, int parts) {
    int mask = 0;
    for (int s = 0; s < 3; ++s)
        if (out[s] && pl.toff[s + 1] > pl.toff[s]) mask |= 1 << s;
    if (!mask) return;
    const int64_t n0 = pl.toff[1] - pl.toff[0], n1 = pl.toff[2] - pl.toff[1];
    if (bie && !bie->sigma) bie = nullptr;
    // The charges' leaf multipoles of a charges-only pass stay in M for a
    // later pass with the same charges (keep_charge_m 1, then 2); any other
    // pass may overwrite them, and the reusing pass adds the dipoles to them.
    if (keep_charge_m != 2) pl.mq_kept = false;
    const int has_q = (q && n0 > 0) ? 1 : 0, has_d = ((dn || bie) && n1 > 0) ? 1 : 0;
    const int L = pl.L, p = pl.p, P = pl.P, Pp = pl.Pp;
    const double inv_alpha = 1.0 / pl.alpha;
    double *qs = pl.qs.ensure(n0 > 0 ? n0 : 1);
    double *dns = pl.dns.ensure(n1 > 0 ? 2 * n1 : 1);
    double *outs = pl.outs.ensure(pl.N);
    pl.last_mask = mask;
    pl.last_has_q = has_q;
    pl.last_has_d = has_d;
    {
    StageTimer tg(ctx, YK_STAGE_GATHER);
    if (has_q) {
        hipLaunchKernelGGL(k_gather_q, dim3(nblk(n0, 256)), dim3(256), 0, ctx.stream, n0, pl.perm.p, q, qs);
        check_launch(ctx, "k_gather_q");
    }
    if (has_d && bie) {
        hipLaunchKernelGGL(k_gather_dn_form, dim3(nblk(n1, 256)), dim3(256), 0, ctx.stream, pl.toff[1], n1,
                           pl.perm.p, bie->w, bie->sigma, bie->normal, dns);
        check_launch(ctx, "k_gather_dn_form");
    } else if (has_d) {
        hipLaunchKernelGGL(k_gather_dn, dim3(nblk(n1, 256)), dim3(256), 0, ctx.stream, pl.toff[1], n1,
                           pl.perm.p, dn, dns);
        check_launch(ctx, "k_gather_dn");
    }
    }
    ActiveSet &as = get_active(ctx, pl, mask);
    // parts: bit 0 the near field, bit 1 the far field (the order check
    // evaluates them apart; the near field alone is then evaluated on the fly)
    const bool far = pl.lmin <= L && (has_q || has_d) && (parts & 2);
    const bool near_on = (parts & 1) != 0;
    const int64_t leaf_base = pl.lev[L].begin;

    // near field: independent of the far field until L2P, so it runs on the
    // side stream while M2M, M2L and L2L run on the main one (forked after P2M,
    // which would otherwise be starved of compute units)
    // (only for small trees: with a large one both streams fill the GPU and
    // sharing it was measured slower than running the stages in turn)
    const bool overlap = !(ctx.opt.debug_flags & 2) && pl.nleaf < 8192 && near_on;
    bool near_done = false;
    const double *sym_inc = nullptr;   // incoming slots of the symmetric near field (for k_l2p)
    auto launch_near = [&]() {
        near_done = true;
        if (!near_on) {   // far field alone: L2P adds it to zeros
            launch_fill(ctx, pl.N, 0.0, outs);
            return;
        }
        if (overlap) {
            ensure_side_stream(ctx);
            YK_HIP(hipEventRecord(ctx.ev_fork, ctx.stream));
            YK_HIP(hipStreamWaitEvent(ctx.side, ctx.ev_fork, 0));
        }
        hipStream_t near_stream = overlap ? ctx.side : ctx.stream;
        if (as.n_leaves > 0) {
            const bool f32 = prec == SUM_FP32, small_only = pl.near_tmax <= 1.0;
            const int q_on = n0 > 0 ? 1 : 0, d_on = n1 > 0 ? 1 : 0;
            // (the near field alone, without the far field's L2P, cannot use the
            // symmetric cache's incoming slots: it is evaluated on the fly)
            // (the adaptive tree's near field is evaluated on the fly)
            const bool want_cache = ctx.opt.near_cache_mb > 0 && (parts & 2) && !pl.adaptive;
            if (want_cache) ensure_near_layout(ctx, pl, as);
            const int64_t entries = as.near_q_len + 2 * as.near_d_len;
            const int64_t bytes = entries * (f32 ? 4 : 8);
            const bool cache = want_cache && bytes <= ((int64_t)ctx.opt.near_cache_mb << 20);
            if (cache) {
                bool &built = f32 ? as.near32 : as.near64;
                if (!built && as.near_sym) {
                    // charge values in the symmetric layout, dipole values as below
                    StageTimer tb(ctx, YK_STAGE_NEAR_BUILD, near_stream);
                    if (f32) {
                        float *mq = as.nq32.ensure(std::max<int64_t>(as.near_q_len, 1));
                        float *md = as.nd32.ensure(std::max<int64_t>(2 * as.near_d_len, 1));
                        hipLaunchKernelGGL(pick_near_build_sym32(small_only), dim3(as.n_items), dim3(64), 0,
                                           near_stream, as.leaf_items.p, pl.lrange.p, pl.ulist_off.p,
                                           pl.ulist.p, pl.px.p, pl.py.p, mask, 0.5 * inv_alpha, as.item_qoff.p,
                                           mq);
                        if (d_on)
                            hipLaunchKernelGGL(pick_near_build32(small_only), dim3(as.n_items), dim3(64), 0,
                                               near_stream, as.leaf_items.p, pl.lrange.p, pl.ulist_off.p,
                                               pl.ulist.p, pl.px.p, pl.py.p, 0, d_on, mask, 0.5 * inv_alpha,
                                               as.item_qoff.p, as.item_doff.p, mq, md);
                    } else {
                        double *mq = as.nq64.ensure(std::max<int64_t>(as.near_q_len, 1));
                        double *md = as.nd64.ensure(std::max<int64_t>(2 * as.near_d_len, 1));
                        hipLaunchKernelGGL(pick_near_build_sym64(pl.near_terms, small_only), dim3(as.n_items),
                                           dim3(64), 0, near_stream, as.leaf_items.p, pl.lrange.p,
                                           pl.ulist_off.p, pl.ulist.p, pl.px.p, pl.py.p, mask, 0.5 * inv_alpha,
                                           as.item_qoff.p, mq);
                        if (d_on)
                            hipLaunchKernelGGL(pick_near_build64(pl.near_terms, small_only), dim3(as.n_items),
                                               dim3(64), 0, near_stream, as.leaf_items.p, pl.lrange.p,
                                               pl.ulist_off.p, pl.ulist.p, pl.px.p, pl.py.p, 0, d_on, mask,
                                               0.5 * inv_alpha, as.item_qoff.p, as.item_doff.p, mq, md);
                    }
                    check_launch(ctx, "k_near_build_sym");
                    built = true;
                }
                if (!built) {
                    StageTimer tb(ctx, YK_STAGE_NEAR_BUILD, near_stream);
                    if (f32) {
                        float *mq = as.nq32.ensure(std::max<int64_t>(as.near_q_len, 1));
                        float *md = as.nd32.ensure(std::max<int64_t>(2 * as.near_d_len, 1));
                        hipLaunchKernelGGL(pick_near_build32(small_only), dim3(as.n_items), dim3(64), 0,
                                           near_stream, as.leaf_items.p, pl.lrange.p, pl.ulist_off.p,
                                           pl.ulist.p, pl.px.p, pl.py.p, q_on, d_on, mask, 0.5 * inv_alpha,
                                           as.item_qoff.p, as.item_doff.p, mq, md);
                    } else {
                        double *mq = as.nq64.ensure(std::max<int64_t>(as.near_q_len, 1));
                        double *md = as.nd64.ensure(std::max<int64_t>(2 * as.near_d_len, 1));
                        hipLaunchKernelGGL(pick_near_build64(pl.near_terms, small_only), dim3(as.n_items),
                                           dim3(64), 0, near_stream, as.leaf_items.p, pl.lrange.p,
                                           pl.ulist_off.p, pl.ulist.p, pl.px.p, pl.py.p, q_on, d_on, mask,
                                           0.5 * inv_alpha, as.item_qoff.p, as.item_doff.p, mq, md);
                    }
                    check_launch(ctx, "k_near_build");
                    built = true;
                }
                StageTimer tl(ctx, YK_STAGE_LEAF, near_stream);
                // four wavefronts per item when the items alone would leave
                // the GPU with under about eight wavefronts per CU
                const bool wide = as.n_items < 2048;
                const dim3 blk(wide ? 256 : 64);
                if (as.near_sym) {
                    double *inc = has_q ? as.inc.ensure(std::max<int64_t>(as.inc_len, 1)) : nullptr;
                    if (f32) {
                        auto kern = wide ? k_near_apply_sym<float, 256> : k_near_apply_sym<float, 64>;
                        hipLaunchKernelGGL(kern, dim3(as.n_items), blk, 0, near_stream, as.sym_desc.p,
                                           as.sym_desc_dst.p, qs, dns, pl.toff[1], has_q, has_d,
                                           as.item_qoff.p, as.item_doff.p, as.nq32.p, as.nd32.p, 0.5 * inv_alpha, outs,
                                           inc);
                    } else {
                        auto kern = wide ? k_near_apply_sym<double, 256> : k_near_apply_sym<double, 64>;
                        hipLaunchKernelGGL(kern, dim3(as.n_items), blk, 0, near_stream, as.sym_desc.p,
                                           as.sym_desc_dst.p, qs, dns, pl.toff[1], has_q, has_d,
                                           as.item_qoff.p, as.item_doff.p, as.nq64.p, as.nd64.p, 0.5 * inv_alpha, outs,
                                           inc);
                    }
                    sym_inc = inc;
                } else if (f32) {
                    auto kern = wide ? k_near_apply<float, 256> : k_near_apply<float, 64>;
                    hipLaunchKernelGGL(kern, dim3(as.n_items), blk, 0, near_stream,
                                       as.leaf_items.p, pl.lrange.p, pl.ulist_off.p, pl.ulist.p, qs, dns,
                                       pl.toff[1], q_on, d_on, has_q, has_d, mask, as.item_qoff.p,
                                       as.item_doff.p, as.nq32.p, as.nd32.p, 0.5 * inv_alpha, outs);
                } else {
                    auto kern = wide ? k_near_apply<double, 256> : k_near_apply<double, 64>;
                    hipLaunchKernelGGL(kern, dim3(as.n_items), blk, 0, near_stream,
                                       as.leaf_items.p, pl.lrange.p, pl.ulist_off.p, pl.ulist.p, qs, dns,
                                       pl.toff[1], q_on, d_on, has_q, has_d, mask, as.item_qoff.p,
                                       as.item_doff.p, as.nq64.p, as.nd64.p, 0.5 * inv_alpha, outs);
                }
                check_launch(ctx, "k_near_apply");
            } else if (pl.adaptive) {
                // one launch per item class: a leaf of side s meets pairs with
                // t = r^2/(4 alpha^2) <= 2 s^2/alpha^2 among leaves of its size
                // or finer, 4.5 s^2/alpha^2 with a coarser one (at a corner);
                // the fine levels take short series
                StageTimer tl(ctx, YK_STAGE_LEAF, near_stream);
                for (int k = 0; k < 2 * (L + 1); ++k) {
                    const int64_t i0 = as.item_lev_begin[k], ni = as.item_lev_begin[k + 1] - i0;
                    if (ni == 0) continue;
                    const int l = k >> 1;
                    const double tl_max = ((k & 1) ? 4.5 : 2.0) * pl.lev[l].side * pl.lev[l].side * inv_alpha *
                                          inv_alpha;
                    LeafKernel kern = pick_leaf_kernel(near_series_terms(tl_max), tl_max <= 1.0, f32, true);
                    hipLaunchKernelGGL(kern, dim3((unsigned)ni), dim3(64), 0, near_stream, as.leaf_items.p + i0,
                                       leaf_base, pl.lrange.p, pl.ulist_off.p, pl.ulist.p, pl.px.p, pl.py.p, qs,
                                       dns, pl.toff[1], has_q, has_d, mask, 0.5 * inv_alpha, 0.5 * inv_alpha, outs);
                    check_launch(ctx, "k_leaf");
                }
            } else {
                LeafKernel kern = pick_leaf_kernel(pl.near_terms, small_only, f32, pl.adaptive);
                StageTimer tl(ctx, YK_STAGE_LEAF, near_stream);
                hipLaunchKernelGGL(kern, dim3(as.n_items), dim3(64), 0, near_stream, as.leaf_items.p,
                                   leaf_base, pl.lrange.p, pl.ulist_off.p, pl.ulist.p, pl.px.p, pl.py.p, qs,
                                   dns, pl.toff[1], has_q, has_d, mask, 0.5 * inv_alpha, 0.5 * inv_alpha, outs);
                check_launch(ctx, "k_leaf");
            }
        }
        if (overlap) YK_HIP(hipEventRecord(ctx.ev_join, ctx.side));
    };
    const size_t lvl = (size_t)(p + 2);
    bool lc_clear = false;   // Lc already cleared (by the cached P2M kernel)
    if (far && pl.adaptive) {
        // P2M at the leaves of every level from lmin on (one launch per level,
        // the level's tables; leaves coarser than lmin need no multipole)
        StageTimer tm(ctx, YK_STAGE_P2M);
        pl.mq_kept = false;
        auto quad4 = p == 8 ? k_p2m_quad<8, 4> : p == 12 ? k_p2m_quad<12, 4> : p == 16 ? k_p2m_quad<16, 4>
                   : p == 20 ? k_p2m_quad<20, 4> : p == 24 ? k_p2m_quad<24, 4> : p == 28 ? k_p2m_quad<28, 4>
                   : p == 31 ? k_p2m_quad<31, 4> : nullptr;
        YK_REQUIRE(quad4 != nullptr, "no P2M kernel for this order");
        for (int l = pl.lmin; l <= L; ++l) {
            const int64_t nl = pl.p2m_off[l + 1] - pl.p2m_off[l];
            if (nl == 0) continue;
            const int ns = pl.nser_lv[l];
            const size_t tabs = (2 * (size_t)ns + 4 * (size_t)(p + 2)) * sizeof(double);
            hipLaunchKernelGGL(quad4, dim3((unsigned)((nl + 15) / 16)), dim3(64), tabs, ctx.stream,
                               pl.lev[l].begin, nl, pl.alr.p + pl.lev[l].begin * 6, pl.bcx.p, pl.bcy.p, pl.px.p,
                               pl.py.p, qs, dns, pl.toff[1], has_q, has_d, inv_alpha, 1.0 / pl.lev[l].R,
                               pl.invFY.p + l * lvl, pl.dipa.p + l * lvl, pl.dipb.p + l * lvl, pl.cnn.p,
                               pl.serc_lv.p + (size_t)l * 2 * pl.nser_stride, ns, p, Pp, pl.M.p,
                               pl.p2m_list.p + pl.p2m_off[l], 0);
            check_launch(ctx, "k_p2m_quad");
        }
    }
    if (far) {
        // upward pass
        if (!pl.adaptive) {
        // cached rows for small trees (there the compute kernel's chains are
        // latency-bound; for large ones it beats reading the rows) when they
        // fit the cache budget (built on first use)
        const int64_t rows_bytes = (n0 + 2 * n1) * (int64_t)Pp * (int64_t)sizeof(double);
        const bool p2m_cache = ctx.opt.near_cache_mb > 0 && pl.nleaf < 8192 && !pl.adaptive &&
                               rows_bytes <= ((int64_t)ctx.opt.near_cache_mb << 20);
        if (p2m_cache && !pl.p2m_rows_built) {
            StageTimer tb(ctx, YK_STAGE_NEAR_BUILD);
            double *rq = pl.p2m_rq.ensure(std::max<int64_t>(n0 * Pp, 1));
            double *rd = pl.p2m_rd.ensure(std::max<int64_t>(2 * n1 * Pp, 1));
            double *gs = pl.p2m_gs.ensure(std::max<int64_t>((n0 + n1) * (p + 2), 1));
            hipLaunchKernelGGL(k_p2m_rows, dim3(nblk(n0 + n1, 256)), dim3(256), 0, ctx.stream, n0, n1,
                               pl.toff[1], pl.pleaf.p, leaf_base, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p,
                               inv_alpha, 1.0 / pl.lev[L].R, pl.invFY.p + L * lvl, pl.dipa.p + L * lvl,
                               pl.dipb.p + L * lvl, pl.cnn.p, pl.serc.p, pl.nser, p, Pp, rq, rd, gs);
            check_launch(ctx, "k_p2m_rows");
            YK_HIP(hipStreamSynchronize(ctx.stream));
            pl.p2m_gs.release();
            pl.p2m_rows_built = true;
        }
        StageTimer tm(ctx, YK_STAGE_P2M);
        if (p2m_cache) {
            hipLaunchKernelGGL(k_p2m_apply, dim3((unsigned)pl.nleaf), dim3(256), 0, ctx.stream,
                               leaf_base, pl.nleaf, pl.lrange.p, pl.toff[1], has_q, has_d, qs, dns,
                               pl.p2m_rq.p, pl.p2m_rd.p, P, Pp, pl.M.p, pl.Lc.p, (int64_t)pl.nbox * Pp);
            check_launch(ctx, "k_p2m_apply");
            lc_clear = true;
        } else {
        const size_t tabs = (2 * (size_t)pl.nser + 4 * (size_t)(p + 2)) * sizeof(double);
        // four lanes per leaf for many leaves; sixteen (more parallelism per
        // leaf, shorter chains) when the leaves are too few to fill the GPU
        auto quad = pl.nleaf < 8192 ? nullptr
                  : p == 8 ? k_p2m_quad<8, 4> : p == 12 ? k_p2m_quad<12, 4> : p == 16 ? k_p2m_quad<16, 4>
                  : p == 20 ? k_p2m_quad<20, 4> : p == 24 ? k_p2m_quad<24, 4> : p == 28 ? k_p2m_quad<28, 4>
                  : p == 31 ? k_p2m_quad<31, 4> : nullptr;
        auto row = p == 8 ? k_p2m_quad<8, 32> : p == 12 ? k_p2m_quad<12, 32> : p == 16 ? k_p2m_quad<16, 32>
                 : p == 20 ? k_p2m_quad<20, 32> : p == 24 ? k_p2m_quad<24, 32> : p == 28 ? k_p2m_quad<28, 32>
                 : p == 31 ? k_p2m_quad<31, 32> : nullptr;
        auto half = p == 8 ? k_p2m_half<8> : p == 12 ? k_p2m_half<12> : p == 16 ? k_p2m_half<16>
                  : p == 20 ? k_p2m_half<20> : p == 24 ? k_p2m_half<24> : p == 28 ? k_p2m_half<28>
                  : p == 31 ? k_p2m_half<31> : nullptr;
        // the leaves that hold dipoles (few, but their points are dense along
        // the curves): 32 lanes per leaf; charges too unless add_only
        auto dipole_leaves = [&](int with_q, int add_only, hipStream_t st) {
            hipLaunchKernelGGL(row, dim3((unsigned)((pl.n_dleaves + 1) / 2)), dim3(64), tabs, st,
                               leaf_base, pl.n_dleaves, pl.lrange.p, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p, qs,
                               dns, pl.toff[1], with_q, 1, inv_alpha, 1.0 / pl.lev[L].R, pl.invFY.p + L * lvl,
                               pl.dipa.p + L * lvl, pl.dipb.p + L * lvl, pl.cnn.p, pl.serc.p, pl.nser, p, Pp,
                               pl.M.p, pl.dleaves.p, add_only);
        };
        if (quad && half && keep_charge_m == 2 && pl.mq_kept && has_q) {
            // the charges' leaf multipoles of the keeping pass are still in M:
            // the dipoles are added to them
            if (has_d && pl.n_dleaves > 0) dipole_leaves(0, 1, ctx.stream);
            pl.mq_kept = false;
        } else if (quad && half) {
            // charges in two halves of the orders on the leaves without
            // dipoles (all leaves when there are none), then the leaves with
            // dipoles, charges and dipoles together
            const int split_d = has_d && pl.n_dleaves > 0;
            // (the two kernels write disjoint leaves, but running the dipole
            // leaves' one on a second stream was measured no faster: the
            // other fills the GPU)
            const size_t tabh = (2 * (size_t)pl.nser + 2 * (size_t)(p + 2)) * sizeof(double);
            hipLaunchKernelGGL(half, dim3((unsigned)((pl.nleaf + 15) / 16), 2), dim3(64), tabh, ctx.stream,
                               leaf_base, pl.nleaf, pl.lrange.p, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p, qs,
                               has_q, inv_alpha, 1.0 / pl.lev[L].R, pl.invFY.p + L * lvl, pl.cnn.p, pl.serc.p,
                               pl.nser, Pp, pl.M.p, split_d, pl.Lc.p, (int64_t)pl.nbox * Pp);
            lc_clear = true;
            if (keep_charge_m == 1 && has_q && !has_d) pl.mq_kept = true;
            if (split_d) dipole_leaves(has_q, 0, ctx.stream);
        } else if (quad) {
            hipLaunchKernelGGL(quad, dim3((unsigned)((pl.nleaf + 15) / 16)), dim3(64), tabs, ctx.stream,
                               leaf_base, pl.nleaf, pl.lrange.p, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p, qs,
                               dns, pl.toff[1], has_q, has_d, inv_alpha, 1.0 / pl.lev[L].R,
                               pl.invFY.p + L * lvl, pl.dipa.p + L * lvl, pl.dipb.p + L * lvl, pl.cnn.p,
                               pl.serc.p, pl.nser, p, Pp, pl.M.p, (const int32_t *)nullptr, 0);
        } else {
            const size_t shp = ((size_t)(p + 2) * 64 + 4 * Pp) * sizeof(double) + tabs;
            hipLaunchKernelGGL(k_p2m<0>, dim3((unsigned)((pl.nleaf + 3) / 4)), dim3(64), shp, ctx.stream,
                               leaf_base, pl.nleaf, pl.lrange.p, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p, qs,
                               dns, pl.toff[1], has_q, has_d, inv_alpha, 1.0 / pl.lev[L].R,
                               pl.invFY.p + L * lvl, pl.dipa.p + L * lvl, pl.dipb.p + L * lvl, pl.cnn.p,
                               pl.serc.p, pl.nser, p, Pp, pl.M.p);
        }
        check_launch(ctx, "k_p2m");
        }
        }
        launch_near();
        fmm_m2m(ctx, pl);
        const bool f32 = prec == SUM_FP32;
        if (f32) {
            const int64_t nm = pl.nbox * (int64_t)Pp;
            float *mf = pl.Mf.ensure(nm);
            hipLaunchKernelGGL(k_to_float, dim3(nblk(nm, 256)), dim3(256), 0, ctx.stream, nm, pl.M.p, mf);
            check_launch(ctx, "k_to_float");
        }
        // downward pass
        // a fill kernel rather than a memset node: this pass may be captured in a graph
        if (!lc_clear) launch_fill(ctx, (int64_t)pl.nbox * Pp, 0.0, pl.Lc.p);
        {
            fmm_m2l(ctx, pl, as, f32);
            if (pl.adaptive && pl.n_xbox > 0) {
                // X lists: coarser leaves' sources straight into the local
                // expansions (before L2L passes them down)
                StageTimer tx(ctx, YK_STAGE_M2L);
                hipLaunchKernelGGL(k_ad_p2l, dim3((unsigned)pl.n_xbox), dim3(64),
                                   (size_t)Pp * kP2LStride * sizeof(double), ctx.stream, pl.xbox.p, pl.xoff.p,
                                   pl.xl.p, pl.lrange.p, has_q, has_d, pl.blevel.p, pl.bcx.p, pl.bcy.p, pl.px.p,
                                   pl.py.p, qs, dns, pl.toff[1], pl.rI.p, p, Pp, inv_alpha, pl.Lc.p);
                check_launch(ctx, "k_ad_p2l");
            }
            fmm_l2l(ctx, pl, as, f32);
        }
    }
    if (!near_done) launch_near();
    if (overlap) YK_HIP(hipStreamWaitEvent(ctx.stream, ctx.ev_join, 0));
    if (far && pl.adaptive && as.n_leaves > 0) {
        StageTimer tl(ctx, YK_STAGE_L2P);
        if (pl.n_wleaves > 0) {
            // W lists: finer boxes' multipoles at the leaves' targets
            hipLaunchKernelGGL(k_ad_m2p, dim3((unsigned)pl.n_wleaves), dim3(64), 0, ctx.stream, pl.wleaves.p,
                               pl.woff.p, pl.wl.p, pl.lrange.p, mask, pl.blevel.p, pl.bcx.p, pl.bcy.p, pl.px.p,
                               pl.py.p, pl.M.p, pl.rI.p, p, Pp, inv_alpha, outs);
            check_launch(ctx, "k_ad_m2p");
        }
        hipLaunchKernelGGL(k_ad_l2p, dim3(nblk(pl.N, 256)), dim3(256), 0, ctx.stream, pl.N, pl.toff[1], pl.toff[2],
                           mask, pl.pleaf.p, pl.leaf_box.p, pl.leaf_lev.p, pl.lmin, pl.bcx.p, pl.bcy.p, pl.px.p,
                           pl.py.p, pl.Lc.p, inv_alpha, pl.invR_lv.p, pl.invFY.p, pl.cnn.p, pl.serc_lv.p,
                           pl.nser_dev.p, pl.nser_stride, p, Pp, outs, pl.perm.p, out[0], out[1], out[2],
                           bie ? bie->w : nullptr, bie ? bie->kappa : nullptr,
                           (bie && bie->kappa) ? bie->sigma : nullptr);
        check_launch(ctx, "k_ad_l2p");
        return;   // L2P wrote the outputs
    }
    if (far && as.n_leaves > 0) {
        StageTimer tl(ctx, YK_STAGE_L2P);
        const size_t lsh = (size_t)(2 * (p + 1) + 2 * pl.nser) * sizeof(double);
        hipLaunchKernelGGL(k_l2p, dim3(nblk(pl.N, 256)), dim3(256), lsh, ctx.stream, pl.N, pl.toff[1],
                           pl.toff[2], mask, pl.pleaf.p, leaf_base, pl.bcx.p, pl.bcy.p, pl.px.p, pl.py.p,
                           pl.Lc.p, inv_alpha, 1.0 / pl.lev[L].R, pl.invFY.p + L * lvl, pl.cnn.p,
                           pl.serc.p, pl.nser, p, Pp, outs, pl.perm.p, out[0], out[1], out[2],
                           bie ? bie->w : nullptr, bie ? bie->kappa : nullptr,
                           (bie && bie->kappa) ? bie->sigma : nullptr, sym_inc, as.inc_base.p, as.inc_cnt.p,
                           pl.lrange.p);
        check_launch(ctx, "k_l2p");
        return;   // L2P wrote the outputs
    }
    StageTimer tsc(ctx, YK_STAGE_SCATTER);
    for (int s = 0; s < 3; ++s) {
        if (!((mask >> s) & 1)) continue;
        const int64_t n = pl.toff[s + 1] - pl.toff[s];
        hipLaunchKernelGGL(k_scatter_out, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, pl.toff[s], n,
                           pl.perm.p, outs, out[s]);
        check_launch(ctx, "k_scatter_out");
        if (s == 1 && bie && bie->kappa)
            launch_bie_finish(ctx, n, bie->w, bie->kappa, pl.alpha, bie->sigma, out[1], out[1]);
    }
}

}  // namespace yk
