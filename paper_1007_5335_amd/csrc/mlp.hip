// mlp.hip -- learned warm start for the density solve.
//
// A small per-node network predicts the next step's double-layer density from
// the last two densities and the boundary data; it only seeds GMRES.  The
// previous-step density is the fallback, and the residual of the second-kind
// system decides which of the two seeds is used, so every step still reaches
// the same tolerance.
//
// Network: x (F features, zero-padded to Fp) -> tanh(W1 x + b1) (H) ->
// tanh(W2 h + b2) (H) -> w3 . h + b3, FP32, trained with Adam on the mean
// squared error.  Features of node j on curve k, at curve offsets
// o in {0, +-1, +-2, +-4, +-8, +-16, +-32} (periodic within the curve):
//   sigma^N, sigma^N - sigma^{N-1}, g^{N+1} - g^N, g^N - g^{N-1}, kappa,
// each divided by its RMS over the training set.  Target: the correction to
// linear extrapolation, sigma^{N+1} - (2 sigma^N - sigma^{N-1}).
// Scaling is per step, so that one network serves early transients and later
// slow decay alike: sigma^N over its RMS, the density difference over its RMS
// r_s, both boundary-data differences over the RMS r_g of g^{N+1} - g^N (their
// ratio is kept), kappa over its RMS; the target is in units of r_s.  Two
// more features carry the step's scales: r_g / r_s and
// rms(g^N - g^{N-1}) / r_g.
#include <cmath>
#include <random>

#include "mlp.h"

namespace yk {

namespace {

constexpr int kOffsets[13] = {0, 1, -1, 2, -2, 4, -4, 8, -8, 16, -16, 32, -32};
constexpr int kChannels = 5;
constexpr int kFeat = kChannels * 13 + 2;

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef float f4v __attribute__((ext_vector_type(4)));

// Workgroups are dispatched to the 8 XCDs in turn; map the b-th of n to a
// tile so that each XCD serves one contiguous run of tiles (neighbouring
// tiles share operand rows, which then stay in one XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, i = b / kXcd;
    const int q = n / kXcd, r = n % kXcd;
    return x * q + min(x, r) + i;
}

// ------------------------------------------------------------------ GEMM ---
// C[z][m][n] = sum_{k in chunk z} A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn].  64 x 64 tiles, 4 wavefronts each owning a
// 32 x 32 quarter (2 x 2 tiles of v_mfma_f32_16x16x4f32), K staged in LDS in
// steps of KS (16 for a tall output with many tiles, 32 for a split K); the
// next step's global loads are issued before the current step's matrix-core
// work, so they are in flight during it.  gridDim.z > 1
// splits K; the partial sums are added afterwards in a fixed order.  With tb
// (one split only) the result is tanh(C + tb[n]).
constexpr int kLdsPad = 80;   // row stride of the LDS tiles (keeps the four lane groups on distinct banks)
constexpr int kGemmKSplit = 32;   // K per LDS step when K is split

template <int KS>
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, const float *__restrict__ A,
                                               int64_t sam, int64_t sak, const float *__restrict__ B,
                                               int64_t sbk, int64_t sbn, float *__restrict__ C,
                                               int64_t ldc, int64_t ldz, int kchunk,
                                               const float *__restrict__ tb) {
    constexpr int NE = 64 * KS / 256;   // elements per thread per operand and step
    __shared__ float As[KS][kLdsPad];
    __shared__ float Bs[KS][kLdsPad];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    // tile (tx, ty, tz) of this workgroup, XCD-aware: the column tiles of one
    // row of tiles (which read the same rows of A) run on one XCD
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = xcd_tile(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int tx = t % gx, ty = (t / gx) % gy, tz = t / (gx * gy);
    const int m0 = ty * 64, n0 = tx * 64;
    const int kbeg = tz * kchunk, kend = min(K, kbeg + kchunk);
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f4v acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const bool a_kfast = sak == 1, b_nfast = sbn == 1;
    // element e of this thread in a step: A tile (mm, kk), B tile (kb, nn)
    auto a_idx = [&](int e, int &mm, int &kk) {
        const int idx = tid + 256 * e;
        if (a_kfast) { mm = idx / KS; kk = idx % KS; } else { kk = idx >> 6; mm = idx & 63; }
    };
    auto b_idx = [&](int e, int &kb, int &nn) {
        const int idx = tid + 256 * e;
        if (b_nfast) { kb = idx >> 6; nn = idx & 63; } else { nn = idx / KS; kb = idx % KS; }
    };
    float ra[NE], rb[NE];
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int mm, kk, kb, nn;
            a_idx(e, mm, kk);
            b_idx(e, kb, nn);
            const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
            ra[e] = (gm < M && gk < kend) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.f;
            rb[e] = (gn < N && gkb < kend) ? B[(int64_t)gkb * sbk + (int64_t)gn * sbn] : 0.f;
        }
    };
    if (kbeg < kend) gload(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += KS) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int mm, kk, kb, nn;
            a_idx(e, mm, kk);
            b_idx(e, kb, nn);
            As[kk][mm] = ra[e];
            Bs[kb][nn] = rb[e];
        }
        __syncthreads();
        if (k0 + KS < kend) gload(k0 + KS);
#pragma unroll
        for (int kq = 0; kq < KS / 4; ++kq) {
            const int kk = 4 * kq + (lane >> 4);
            const float a0 = As[kk][wm + (lane & 15)], a1 = As[kk][wm + 16 + (lane & 15)];
            const float b0 = Bs[kk][wn + (lane & 15)], b1 = Bs[kk][wn + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    float *Cz = C + (int64_t)tz * ldz;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < M && gn < N)
                    Cz[(int64_t)gm * ldc + gn] = tb ? tanhf(acc[i][j][r] + tb[gn]) : acc[i][j][r];
            }
}

__global__ void k_sum_partials(int64_t n, int nz, const float *__restrict__ part, int64_t ldz,
                               float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
#pragma unroll 8
    for (int z = 0; z < nz; ++z) s += part[z * ldz + i];
    out[i] = s;
}

// H = tanh(Z + b[col]) in place
__global__ void k_bias_tanh(int64_t rows, int cols, float *__restrict__ Z, const float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    Z[i] = tanhf(Z[i] + b[i % cols]);
}

// y[r] = sum_c H[r][c] w[c] + b0   (one wavefront per row)
__global__ void k_rowdot(int64_t rows, int cols, const float *__restrict__ H, const float *__restrict__ w,
                         const float *__restrict__ b0, float *__restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;
    float s = 0.f;
    for (int c = lane; c < cols; c += 64) s += H[r * cols + c] * w[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[r] = s + b0[0];
}

// dy = 2 (y - t) / n ; partial loss sums per block (fixed-order reduction later)
__global__ __launch_bounds__(256) void k_mse(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                                             float *__restrict__ dy, float *__restrict__ part) {
    __shared__ float sh[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e = 0.f;
    if (i < n) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d / (float)n;
        e = d * d;
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// D[r][c] = dy[r] * w[c] * (1 - H[r][c]^2)
__global__ void k_back_out(int64_t rows, int cols, const float *__restrict__ dy, const float *__restrict__ w,
                           const float *__restrict__ H, float *__restrict__ D) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const float h = H[i];
    D[i] = dy[i / cols] * w[i % cols] * (1.f - h * h);
}

// D *= (1 - H^2)
__global__ void k_back_tanh(int64_t n, const float *__restrict__ H, float *__restrict__ D) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float h = H[i];
    D[i] *= 1.f - h * h;
}

// column sums over row blocks: part[blk][c] (one thread per column, eight
// rows' loads in flight, rows taken in increasing order)
__global__ void k_colsum_part(int64_t rows, int cols, const float *__restrict__ D, int rows_per_blk,
                              float *__restrict__ part) {
    const int c = threadIdx.x + blockIdx.y * blockDim.x;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min<int64_t>(rows, r0 + rows_per_blk);
    float s = 0.f;
    int64_t r = r0;
    for (; r + 8 <= r1; r += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = D[(r + u) * cols + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < r1; ++r) s += D[r * cols + c];
    part[(int64_t)blockIdx.x * cols + c] = s;
}

// out[c] = sum_b part[b][c] over nb row blocks: 64 columns per block, four
// wavefronts taking the row blocks b = w (mod 4), then the four sums in order
__global__ __launch_bounds__(256) void k_colsum_final(int nb, int cols, const float *__restrict__ part,
                                                      float *__restrict__ out) {
    __shared__ float sh[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (c < cols) {
        int b = w;
        for (; b + 12 < nb; b += 16) {
            const float v0 = part[(int64_t)b * cols + c], v1 = part[(int64_t)(b + 4) * cols + c];
            const float v2 = part[(int64_t)(b + 8) * cols + c], v3 = part[(int64_t)(b + 12) * cols + c];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < nb; b += 4) s += part[(int64_t)b * cols + c];
    }
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && c < cols) out[c] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Sums of squares of s0, s0 - sm1, gp1 - g0, g0 - gm1 and kappa: partials
// part[q * 256 + block] (256 blocks)
__global__ __launch_bounds__(256) void k_sumsq5(int64_t n, const double *__restrict__ sm1,
                                                const double *__restrict__ s0, const double *__restrict__ gm1,
                                                const double *__restrict__ g0, const double *__restrict__ gp1,
                                                const double *__restrict__ kappa, double *__restrict__ part) {
    __shared__ double sh[5][256];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v0 = s0[i], v1 = s0[i] - sm1[i], v2 = gp1[i] - g0[i], v3 = g0[i] - gm1[i], v4 = kappa[i];
        a[0] += v0 * v0;
        a[1] += v1 * v1;
        a[2] += v2 * v2;
        a[3] += v3 * v3;
        a[4] += v4 * v4;
    }
    for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 5) part[threadIdx.x * 256 + blockIdx.x] = sh[threadIdx.x][0];
}

// The step's scales from the partials (one block, fixed order): RMS values
// r0 = rms(s0), r_s = rms(s0 - sm1), r_g = rms(gp1 - g0), r_g0 = rms(g0 - gm1),
// r_k = rms(kappa) (the first three and r_k floored at a tiny positive value);
// fs = {1/r0, 1/r_s, 1/r_g, 1/r_k, ln(r_g/r_s), r_g0/r_g, r_s}
__global__ void k_feature_scales(int64_t n, const double *__restrict__ part, double *__restrict__ fs) {
    __shared__ double r[5];
    if (threadIdx.x < 5) {
        double t = 0.0;
        for (int b = 0; b < 256; ++b) t += part[threadIdx.x * 256 + b];
        r[threadIdx.x] = sqrt(t / (double)(n > 0 ? n : 1));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tiny = 1e-300;
        const double r0 = fmax(tiny, r[0]), rs = fmax(tiny, r[1]), rg = fmax(tiny, r[2]), rk = fmax(tiny, r[4]);
        fs[0] = 1.0 / r0;
        fs[1] = 1.0 / rs;
        fs[2] = 1.0 / rg;
        fs[3] = 1.0 / rk;
        fs[4] = log(rg / rs);
        fs[5] = r[3] / rg;
        fs[6] = rs;
    }
}

// Features of every node for one (N-1, N, N+1) triple; fs holds the per-step
// scales written by k_feature_scales.  A block builds the rows of 64 nodes in
// LDS (four thread groups over the 13 offsets) and stores them as one
// contiguous run of 64 Fp floats.
constexpr int kFp = (kFeat + 15) / 16 * 16;   // padded feature count
__global__ __launch_bounds__(256) void k_features(
    int64_t n, const double *__restrict__ sm1, const double *__restrict__ s0,
    const double *__restrict__ gm1, const double *__restrict__ g0, const double *__restrict__ gp1,
    const double *__restrict__ kappa, const int32_t *__restrict__ curve, const int32_t *__restrict__ idx,
    const int64_t *__restrict__ off, const double *__restrict__ fs, float *__restrict__ X) {
    __shared__ float rows[64 * kFp];
    const int r = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t j0 = (int64_t)blockIdx.x * 64, j = j0 + r;
    const int nrow = (int)min<int64_t>(64, n - j0);
    if (j < n) {
        const float sc0 = (float)fs[0], sc1 = (float)fs[1], sc2 = (float)fs[2], sc4 = (float)fs[3];
        const int k = curve[j];
        const int64_t base = off[k], nk = off[k + 1] - off[k];
        const int64_t jl = idx[j];
        float *row = rows + r * kFp;
        for (int o = grp; o < 13; o += 4) {
            int64_t q = (jl + kOffsets[o]) % nk;
            if (q < 0) q += nk;
            const int64_t jj = base + q;
            row[0 * 13 + o] = (float)(s0[jj] * sc0);
            row[1 * 13 + o] = (float)((s0[jj] - sm1[jj]) * sc1);
            row[2 * 13 + o] = (float)((gp1[jj] - g0[jj]) * sc2);
            row[3 * 13 + o] = (float)((g0[jj] - gm1[jj]) * sc2);
            row[4 * 13 + o] = (float)(kappa[jj] * sc4);
        }
        if (grp == 3) {
            row[65] = (float)fs[4];
            row[66] = (float)fs[5];
            for (int f = kFeat; f < kFp; ++f) row[f] = 0.f;
        }
    }
    __syncthreads();
    float *dst = X + j0 * kFp;
    for (int e = threadIdx.x; e < nrow * kFp; e += 256) dst[e] = rows[e];
}

// target (sigma^{N+1} - 2 sigma^N + sigma^{N-1}) / r_s, r_s = fs[6]
__global__ void k_target(int64_t n, const double *__restrict__ sm1, const double *__restrict__ s0,
                         const double *__restrict__ sp1, const double *__restrict__ fs, float *__restrict__ t) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float inv_sy = (float)(1.0 / fs[6]);
    t[j] = (float)((sp1[j] - 2.0 * s0[j] + sm1[j]) * inv_sy);
}

// sigma = 2 sigma^N - sigma^{N-1} + r_s * y, r_s = fs[6]
__global__ void k_apply_pred(int64_t n, const double *__restrict__ sm1, const double *__restrict__ s0,
                             const float *__restrict__ y, const double *__restrict__ fs,
                             double *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[j] = 2.0 * s0[j] - sm1[j] + fs[6] * (double)y[j];
}

__global__ void k_gather_rows(int64_t nb, int Fp, const int32_t *__restrict__ rows,
                              const float *__restrict__ X, const float *__restrict__ T,
                              float *__restrict__ Xb, float *__restrict__ Tb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb * Fp) return;
    const int64_t r = i / Fp, f = i - r * Fp;
    const int64_t src = rows[r];
    Xb[i] = X[src * Fp + f];
    if (f == 0) Tb[r] = T[src];
}

// ------------------------------------------------------- fused inference --
// Inference over many rows: a workgroup of four wavefronts takes kPredRows rows
// through both hidden layers on the matrix cores and writes one output per
// row; the first layer's activations stay in LDS.  Wavefront w owns columns
// 64 w .. 64 w + 63 of both layers.  Weights are read transposed (WT[k][col],
// so a fragment's sixteen columns are contiguous).
//   v_mfma_f32_16x16x4f32: lane l holds A[l%16][l/16], B[l/16][l%16];
//   C rows 4(l/16) + r, column l%16.
// LDS row strides are 4 more than a multiple of 64 words, so the sixteen rows
// and four k of a fragment read fall on distinct banks.
constexpr int kPredRows = 32;

template <int FP, int H>
__global__ __launch_bounds__(256) void k_mlp_predict(int64_t rows, const float *__restrict__ X,
                                                     const float *__restrict__ W1T, const float *__restrict__ b1,
                                                     const float *__restrict__ W2T, const float *__restrict__ b2,
                                                     const float *__restrict__ w3, const float *__restrict__ b3,
                                                     float *__restrict__ y) {
    static_assert(H == 256 && FP % 4 == 0, "four wavefronts of 64 columns");
    constexpr int SX = (FP + 59) / 64 * 64 + 4, SH = H + 4;
    constexpr int RT = kPredRows / 16;
    __shared__ float xs[kPredRows * SX];
    __shared__ float hs[kPredRows * SH];
    __shared__ float ys[4][kPredRows];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * kPredRows;
    for (int e = tid; e < kPredRows * FP; e += 256) {
        const int r = e / FP, k = e % FP;
        xs[r * SX + k] = r0 + r < rows ? X[(r0 + r) * FP + k] : 0.f;
    }
    __syncthreads();
    const int c0 = 64 * w;
    f4v acc[RT][4];
    auto clear = [&]() {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    };
    // acc += A[rows][k] WT[k][cols] over k < K, A in LDS with row stride S
    auto layer = [&](const float *As, int S, const float *WT, int K) {
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk;
            float a[RT], b[4];
#pragma unroll
            for (int i = 0; i < RT; ++i) a[i] = As[(16 * i + lr) * S + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = WT[(int64_t)k * H + c0 + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
    clear();
    layer(xs, SX, W1T, FP);
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = c0 + 16 * j + lr;
            const float bb = b1[col];
#pragma unroll
            for (int r = 0; r < 4; ++r) hs[(16 * i + 4 * lk + r) * SH + col] = tanhf(acc[i][j][r] + bb);
        }
    __syncthreads();
    clear();
    layer(hs, SH, W2T, H);
    // this wavefront's share of sum_col tanh(z + b2[col]) w3[col], then the
    // sixteen lanes of each row group and the four wavefronts
    float part[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float sacc = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = c0 + 16 * j + lr;
                sacc += tanhf(acc[i][j][r] + b2[col]) * w3[col];
            }
#pragma unroll
            for (int m = 8; m >= 1; m >>= 1) sacc += __shfl_xor(sacc, m, 16);
            part[i][r] = sacc;
        }
    if (lr == 0)
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) ys[w][16 * i + 4 * lk + r] = part[i][r];
    __syncthreads();
    if (tid < kPredRows && r0 + tid < rows) y[r0 + tid] = ((ys[0][tid] + ys[1][tid]) + (ys[2][tid] + ys[3][tid])) + b3[0];
}

// WT[k][col] = W[col][k] for a [cols][K] block (column-major weights)
__global__ void k_transpose_w(int cols, int K, const float *__restrict__ W, float *__restrict__ WT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)cols * K) return;
    const int k = (int)(e / cols), col = (int)(e % cols);
    WT[e] = W[(int64_t)col * K + k];
}

}  // namespace

// --------------------------------------------------------------- host side --
void sgemm(Context &ctx, int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *B,
           int64_t sbk, int64_t sbn, float *C, int64_t ldc, DevBuf<float> &part, const float *tanh_bias) {
    if (M <= 0 || N <= 0) return;
    const int gm = (M + 63) / 64, gn = (N + 63) / 64;
    // split K when the output has few tiles and K is long
    int nz = 1;
    if ((int64_t)gm * gn < 256 && K > 1024) nz = (int)std::min<int64_t>(64, std::max<int64_t>(1, 512 / ((int64_t)gm * gn)));
    int kchunk = (K + nz - 1) / nz;
    kchunk = (kchunk + kGemmKSplit - 1) / kGemmKSplit * kGemmKSplit;
    nz = (K + kchunk - 1) / kchunk;
    if (nz <= 1) {
        hipLaunchKernelGGL(k_sgemm<16>, dim3(gn, gm, 1), dim3(256), 0, ctx.stream, M, N, K, A, sam, sak, B, sbk,
                           sbn, C, ldc, (int64_t)0, K, tanh_bias);
        check_launch(ctx, "k_sgemm");
        return;
    }
    const int64_t ldz = (int64_t)M * ldc;
    float *p = part.ensure((size_t)nz * ldz);
    hipLaunchKernelGGL(k_sgemm<kGemmKSplit>, dim3(gn, gm, nz), dim3(256), 0, ctx.stream, M, N, K, A, sam, sak, B,
                       sbk, sbn, p, ldc, ldz, kchunk, (const float *)nullptr);
    check_launch(ctx, "k_sgemm");
    hipLaunchKernelGGL(k_sum_partials, dim3(nblk(ldz, 256)), dim3(256), 0, ctx.stream, ldz, nz, p, ldz, C);
    check_launch(ctx, "k_sum_partials");
    if (tanh_bias) {
        if (ldc != N) throw Error{YK_ERR_INTERNAL, "sgemm: bias epilogue needs ldc == N"};
        hipLaunchKernelGGL(k_bias_tanh, dim3(nblk((int64_t)M * N, 256)), dim3(256), 0, ctx.stream, (int64_t)M, N,
                           C, tanh_bias);
        check_launch(ctx, "k_bias_tanh");
    }
}

WarmStart::WarmStart(Context &c, BoundaryData &b, const yk_ws_options &o) : ctx(c), opt(o) {
    n = b.n;
    H = o.hidden;
    Fp = (kFeat + 15) / 16 * 16;
    offsets = b.offset;
    int64_t *d = off.ensure(offsets.size());
    YK_HIP(hipMemcpyAsync(d, offsets.data(), offsets.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
    curve = curve_buf.ensure(n);
    idx = idx_buf.ensure(n);
    YK_HIP(hipMemcpyAsync(curve_buf.p, b.curve.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx.stream));
    YK_HIP(hipMemcpyAsync(idx_buf.p, b.idx.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx.stream));
    kappa = b.curvature;
    xy = b.xy;
    // parameters: W1 [H x Fp], b1 [H], W2 [H x H], b2 [H], w3 [H], b3 [1]
    o_W1 = 0;
    o_b1 = o_W1 + (int64_t)H * Fp;
    o_W2 = o_b1 + H;
    o_b2 = o_W2 + (int64_t)H * H;
    o_w3 = o_b2 + H;
    o_b3 = o_w3 + H;
    n_params = o_b3 + 1;
    std::vector<float> p(n_params, 0.f);
    std::mt19937_64 rng(o.seed);
    auto fill = [&](int64_t o0, int64_t cnt, int fan_in, int fan_out, float gain) {
        const float a = gain * std::sqrt(6.f / (float)(fan_in + fan_out));
        std::uniform_real_distribution<float> u(-a, a);
        for (int64_t i = 0; i < cnt; ++i) p[o0 + i] = u(rng);
    };
    fill(o_W1, (int64_t)H * Fp, kFeat, H, 1.f);
    for (int r = 0; r < H; ++r)
        for (int f = kFeat; f < Fp; ++f) p[o_W1 + (int64_t)r * Fp + f] = 0.f;
    fill(o_W2, (int64_t)H * H, H, H, 1.f);
    fill(o_w3, H, H, 1, 0.1f);
    float *dp = params.ensure(n_params);
    YK_HIP(hipMemcpyAsync(dp, p.data(), n_params * sizeof(float), hipMemcpyHostToDevice, ctx.stream));
    YK_HIP(hipMemsetAsync(adam_m.ensure(n_params), 0, n_params * sizeof(float), ctx.stream));
    YK_HIP(hipMemsetAsync(adam_v.ensure(n_params), 0, n_params * sizeof(float), ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
}

void WarmStart::observe(const double *g, const double *sigma) {
    auto slot = std::make_unique<Obs>();
    YK_HIP(hipMemcpyAsync(slot->g.ensure(n), g, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    YK_HIP(hipMemcpyAsync(slot->s.ensure(n), sigma, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    obs.push_back(std::move(slot));
    // bounded history: the oldest observation is dropped beyond max_obs
    if ((int)obs.size() > opt.max_obs) obs.erase(obs.begin());
}

void WarmStart::features(const double *sm1, const double *s0, const double *gm1, const double *g0,
                         const double *gp1, float *X, double *fs) {
    double *part = scal.ensure(5 * 256);
    hipLaunchKernelGGL(k_sumsq5, dim3(256), dim3(256), 0, ctx.stream, n, sm1, s0, gm1, g0, gp1, kappa, part);
    check_launch(ctx, "k_sumsq5");
    hipLaunchKernelGGL(k_feature_scales, dim3(1), dim3(64), 0, ctx.stream, n, part, fs);
    check_launch(ctx, "k_feature_scales");
    if (Fp != kFp) throw Error{YK_ERR_INTERNAL, "feature width mismatch"};
    hipLaunchKernelGGL(k_features, dim3(nblk(n, 64)), dim3(256), 0, ctx.stream, n, sm1, s0, gm1, g0, gp1,
                       kappa, curve, idx, off.p, fs, X);
    check_launch(ctx, "k_features");
}

void WarmStart::forward(int64_t rows, const float *X, float *y) {
    float *P = params.p;
    float *H1 = h1.ensure((size_t)rows * H), *H2 = h2.ensure((size_t)rows * H);
    // hidden layers with the bias and tanh applied as the products are stored
    sgemm(ctx, (int)rows, H, Fp, X, Fp, 1, P + o_W1, 1, Fp, H1, H, part, P + o_b1);
    sgemm(ctx, (int)rows, H, H, H1, H, 1, P + o_W2, 1, H, H2, H, part, P + o_b2);
    hipLaunchKernelGGL(k_rowdot, dim3(nblk(rows, 4)), dim3(256), 0, ctx.stream, rows, H, H2, P + o_w3, P + o_b3, y);
    check_launch(ctx, "k_rowdot");
}

void WarmStart::forward_fused(int64_t rows, const float *X, float *y) {
    if (H != 256 || Fp != kFp) {   // (other widths: the layer-by-layer products)
        forward(rows, X, y);
        return;
    }
    const float *P = params.p;
    float *W1T = wt.ensure((size_t)H * Fp + (size_t)H * H), *W2T = W1T + (size_t)H * Fp;
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk((int64_t)H * Fp, 256)), dim3(256), 0, ctx.stream, H, Fp, P + o_W1,
                       W1T);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk((int64_t)H * H, 256)), dim3(256), 0, ctx.stream, H, H, P + o_W2,
                       W2T);
    check_launch(ctx, "k_transpose_w");
    hipLaunchKernelGGL((k_mlp_predict<kFp, 256>), dim3(nblk(rows, kPredRows)), dim3(256), 0, ctx.stream, rows, X,
                       W1T, P + o_b1, W2T, P + o_b2, P + o_w3, P + o_b3, y);
    check_launch(ctx, "k_mlp_predict");
}

double WarmStart::loss_grad(int64_t rows, const float *X, const float *T, float *G) {
    float *P = params.p;
    float *y = yb.ensure(rows), *dy = dyb.ensure(rows);
    forward(rows, X, y);
    const int nb = (int)nblk(rows, 256);
    float *lp = lpart.ensure(nb);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, ctx.stream, rows, y, T, dy, lp);
    check_launch(ctx, "k_mse");
    float *H1 = h1.p, *H2 = h2.p;
    float *D2 = d2.ensure((size_t)rows * H), *D1 = d1.ensure((size_t)rows * H);
    // output layer: g_w3 = H2^T dy (1 x H), g_b3 = sum dy
    sgemm(ctx, 1, H, (int)rows, dy, 0, 1, H2, H, 1, G + o_w3, H, part);
    // D2 = dy w3^T (1 - H2^2)
    hipLaunchKernelGGL(k_back_out, dim3(nblk(rows * H, 256)), dim3(256), 0, ctx.stream, rows, H, dy, P + o_w3, H2, D2);
    check_launch(ctx, "k_back_out");
    // g_W2 = D2^T H1 (H x H);  D1 = (D2 W2) (1 - H1^2);  g_W1 = D1^T X (H x Fp)
    sgemm(ctx, H, H, (int)rows, D2, 1, H, H1, H, 1, G + o_W2, H, part);
    sgemm(ctx, (int)rows, H, H, D2, H, 1, P + o_W2, H, 1, D1, H, part);
    hipLaunchKernelGGL(k_back_tanh, dim3(nblk(rows * H, 256)), dim3(256), 0, ctx.stream, rows * H, H1, D1);
    check_launch(ctx, "k_back_tanh");
    sgemm(ctx, H, Fp, (int)rows, D1, 1, H, X, Fp, 1, G + o_W1, Fp, part);
    // bias gradients: column sums of D1, D2 and of dy
    colsum(rows, H, D1, G + o_b1);
    colsum(rows, H, D2, G + o_b2);
    colsum(rows, 1, dy, G + o_b3);
    std::vector<float> hl(nb);
    YK_HIP(hipMemcpyAsync(hl.data(), lp, nb * sizeof(float), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    double s = 0;
    for (float v : hl) s += v;
    return s / (double)rows;
}

void WarmStart::colsum(int64_t rows, int cols, const float *D, float *out) {
    const int rpb = 128;
    const int nbr = (int)nblk(rows, rpb);
    float *p = cpart.ensure((size_t)nbr * cols);
    hipLaunchKernelGGL(k_colsum_part, dim3(nbr, nblk(cols, 256)), dim3(256), 0, ctx.stream, rows, cols, D, rpb, p);
    check_launch(ctx, "k_colsum_part");
    // fixed-order reduction of the row-block partials
    hipLaunchKernelGGL(k_colsum_final, dim3(nblk(cols, 64)), dim3(256), 0, ctx.stream, nbr, cols, p, out);
    check_launch(ctx, "k_colsum_final");
}

double WarmStart::train() {
    const int ns = (int)obs.size() - 2;   // (N-1, N, N+1) triples
    if (ns < 1) throw Error{YK_ERR_ARG, "warm start needs at least three observed steps to train"};
    // features and targets of every triple (per-step scaling)
    const int64_t rows = (int64_t)ns * n;
    float *X = Xall.ensure((size_t)rows * Fp), *T = Tall.ensure(rows);
    double *fs = fscale.ensure(8);
    for (int s = 0; s < ns; ++s) {
        features(obs[s]->s.p, obs[s + 1]->s.p, obs[s]->g.p, obs[s + 1]->g.p, obs[s + 2]->g.p,
                 X + (int64_t)s * n * Fp, fs);
        hipLaunchKernelGGL(k_target, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, obs[s]->s.p,
                           obs[s + 1]->s.p, obs[s + 2]->s.p, fs, T + (int64_t)s * n);
        check_launch(ctx, "k_target");
    }
    // Adam on shuffled mini-batches
    const int64_t B = std::min<int64_t>(opt.batch, rows);
    float *Xb = Xbat.ensure((size_t)B * Fp), *Tb = Tbat.ensure(B), *G = grad.ensure(n_params);
    int32_t *rowsd = brows.ensure(B);
    std::mt19937_64 rng(opt.seed ^ 0x9e3779b97f4a7c15ull);
    std::vector<int32_t> perm(rows);
    for (int64_t i = 0; i < rows; ++i) perm[i] = (int32_t)i;
    int64_t pos = rows;
    double loss = 0;
    for (int it = 0; it < opt.steps; ++it) {
        if (pos + B > rows) {
            std::shuffle(perm.begin(), perm.end(), rng);
            pos = 0;
        }
        YK_HIP(hipMemcpyAsync(rowsd, perm.data() + pos, B * sizeof(int32_t), hipMemcpyHostToDevice, ctx.stream));
        pos += B;
        hipLaunchKernelGGL(k_gather_rows, dim3(nblk(B * Fp, 256)), dim3(256), 0, ctx.stream, B, Fp, rowsd, X, T,
                           Xb, Tb);
        check_launch(ctx, "k_gather_rows");
        loss = loss_grad(B, Xb, Tb, G);
        adam_step(G);
    }
    trained = true;
    return loss;
}

void WarmStart::adam_step(const float *G) {
    // Adam (Kingma & Ba): moments with decay b1, b2 and bias corrections
    // 1 / (1 - b^t) for the step count t
    const float b1 = 0.9f, b2 = 0.999f;
    ++adam_t;
    const float c1 = 1.f / (1.f - std::pow(b1, (float)adam_t)), c2 = 1.f / (1.f - std::pow(b2, (float)adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n_params, 256)), dim3(256), 0, ctx.stream, n_params, params.p, G,
                       adam_m.p, adam_v.p, (float)opt.lr, b1, b2, 1e-8f, c1, c2);
    check_launch(ctx, "k_adam");
}

void WarmStart::predict(const double *g_next, double *out) {
    if (obs.size() < 2) throw Error{YK_ERR_ARG, "warm start needs two observed steps to predict"};
    const Obs &a = *obs[obs.size() - 2], &b = *obs[obs.size() - 1];
    float *X = Xbat.ensure((size_t)std::max<int64_t>(n, (int64_t)opt.batch) * Fp);
    double *fs = fscale.ensure(8);
    features(a.s.p, b.s.p, a.g.p, b.g.p, g_next, X, fs);
    float *y = yb.ensure(std::max<int64_t>(n, (int64_t)opt.batch));
    if (ctx.opt.debug_flags & 32) forward(n, X, y);
    else forward_fused(n, X, y);
    hipLaunchKernelGGL(k_apply_pred, dim3(nblk(n, 256)), dim3(256), 0, ctx.stream, n, a.s.p, b.s.p, y, fs, out);
    check_launch(ctx, "k_apply_pred");
}

}  // namespace yk
