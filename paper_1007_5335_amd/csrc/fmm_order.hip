// fmm_order.hip -- choice of the expansion order under error control.
//
// The truncation error of the K_n / I_n expansions (Graf's addition theorem)
// depends on the geometry in ways a fitted formula misses: along a curve the
// double-layer kernel between nodes is small (the normal is nearly
// perpendicular to the chord, (x - y).n ~ kappa r^2 / 2), while the truncation
// error of its expansion is not, so dense dipoles on a tightly curved hole
// lose digits relative to their own potential.  When the order is derived from
// fmm_tol, the plan therefore checks itself once, at build time: one FMM pass
// with probe strengths (unit charges; dipoles of random sign along the
// caller's normals) against direct sums at sampled points of every set, and
// the order is raised along the instantiated orders until every sampled
// output is within half the tolerance of the direct sum, relative to its own
// size (floored at a tenth of the samples' RMS, where a random-sign sum
// cancels).  The probe depends on the points only, so the order is a property
// of the tree, like its depth.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "fmm.h"

namespace yk {

namespace {

constexpr int kSamplesPerSet = 128;

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer finaliser (xorshift-multiply), a fixed sign pattern per index
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void k_probe_charges(int64_t n, double *__restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = 1.0;
}

// dn_j = s_j n_j with s_j = +-1; without normals a direction of its own per node
__global__ void k_probe_dipoles(int64_t n, const double *__restrict__ normal, double *__restrict__ dn) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t h = mix32((uint32_t)i * 2654435761u + 12345u);
    if (normal) {
        const double s = (h & 1u) ? 1.0 : -1.0;
        dn[2 * i] = s * normal[2 * i];
        dn[2 * i + 1] = s * normal[2 * i + 1];
    } else {
        const double th = 6.283185307179586 * (double)(h >> 8) * (1.0 / 16777216.0);
        dn[2 * i] = cos(th);
        dn[2 * i + 1] = sin(th);
    }
}

// out[k] = v[idx[k]] (stride 1) or the point idx[k] of an [n][2] array (stride 2)
__global__ void k_take(int64_t k, const int64_t *__restrict__ idx, const double *__restrict__ v, int stride,
                       double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    for (int c = 0; c < stride; ++c) out[stride * t + c] = v[stride * idx[t] + c];
}

}  // namespace

void calibrate_order(Context &ctx, FmmPlan &pl, const SumProblem &pb) {
    const auto t_start = std::chrono::steady_clock::now();
    struct Done {   // records the check's time however it ends
        FmmPlan &pl;
        std::chrono::steady_clock::time_point t0;
        ~Done() { pl.check_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); }
    } done{pl, t_start};
    pl.calib_err = -1.0;
    pl.calib_p0 = pl.p;
    if (pl.opt_p > 0 || pl.lmin > pl.L) return;   // order given, or no far field
    const int64_t n0 = pb.n[0], n1 = pb.n[1];
    // sampled points: a fixed stride through each set in the caller's order
    std::vector<int64_t> hidx;
    int64_t kcount[3] = {0, 0, 0}, kbase[3] = {0, 0, 0};
    for (int s = 0; s < 3; ++s) {
        kbase[s] = (int64_t)hidx.size();
        const int64_t n = pb.n[s];
        const int64_t k = std::min<int64_t>(n, kSamplesPerSet);
        for (int64_t t = 0; t < k; ++t) hidx.push_back((2 * t + 1) * n / (2 * k));
        kcount[s] = k;
    }
    const int64_t K = (int64_t)hidx.size();
    if (K == 0) return;
    DevBuf<int64_t> didx;
    DevBuf<double> txy, ref, got, probe_q, probe_dn;
    DevBuf<double> outbuf[3];
    YK_HIP(hipMemcpyAsync(didx.ensure(K), hidx.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, ctx.stream));
    double *dtxy = txy.ensure(2 * K);
    for (int s = 0; s < 3; ++s)
        if (kcount[s] > 0)
            hipLaunchKernelGGL(k_take, dim3(nblk(kcount[s], 256)), dim3(256), 0, ctx.stream, kcount[s],
                               didx.p + kbase[s], pb.xy[s], 2, dtxy + 2 * kbase[s]);
    check_launch(ctx, "k_take");
    double *q = n0 > 0 ? probe_q.ensure(n0) : nullptr;
    double *dn = n1 > 0 ? probe_dn.ensure(2 * n1) : nullptr;
    if (q) hipLaunchKernelGGL(k_probe_charges, dim3(nblk(n0, 256)), dim3(256), 0, ctx.stream, n0, q);
    const double *normal = pb.normal ? pb.normal : (pb.bie ? pb.bie->normal : nullptr);
    if (dn) hipLaunchKernelGGL(k_probe_dipoles, dim3(nblk(n1, 256)), dim3(256), 0, ctx.stream, n1, normal, dn);
    check_launch(ctx, "k_probe");
    double *outs[3] = {nullptr, nullptr, nullptr};
    for (int s = 0; s < 3; ++s)
        if (pb.n[s] > 0) outs[s] = outbuf[s].ensure(pb.n[s]);
    double *dref = ref.ensure(2 * K), *dgot = got.ensure(K);
    std::vector<double> href(2 * K), hnear(2 * K), hfar(K);
    // the probes run without the near-field cache (evaluated on the fly, so
    // no cache is built for a target set later calls may never use); their
    // work lists (every set a target) stay for later calls with that mask
    const int cache_mb = ctx.opt.near_cache_mb;
    ctx.opt.near_cache_mb = 0;
    // probe 0: charges alone; probe 1: dipoles alone.  The direct sums and
    // the near field do not depend on the order: they are evaluated once;
    // each order tried evaluates the far field alone.
    auto sample = [&](double *dst_host) {
        for (int s = 0; s < 3; ++s)
            if (kcount[s] > 0)
                hipLaunchKernelGGL(k_take, dim3(nblk(kcount[s], 256)), dim3(256), 0, ctx.stream, kcount[s],
                                   didx.p + kbase[s], outs[s], 1, dgot + kbase[s]);
        check_launch(ctx, "k_take");
        YK_HIP(hipMemcpyAsync(dst_host, dgot, K * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
        YK_HIP(hipStreamSynchronize(ctx.stream));
    };
    bool present[2] = {q != nullptr, dn != nullptr};
    for (int probe = 0; probe < 2; ++probe) {
        if (!present[probe]) continue;
        const double *pq = probe == 0 ? q : nullptr;
        const double *pd = probe == 1 ? dn : nullptr;
        launch_direct(ctx, K, dtxy, pq ? n0 : 0, pb.xy[0], pq, pd ? n1 : 0, pb.xy[1], pd, pl.alpha,
                      dref + probe * K, false);
        YK_HIP(hipMemcpyAsync(href.data() + probe * K, dref + probe * K, K * sizeof(double),
                              hipMemcpyDeviceToHost, ctx.stream));
        fmm_run(ctx, pl, pq, pd, outs, SUM_FP64, nullptr, 0, 1);
        sample(hnear.data() + probe * K);
    }
    auto measure = [&](int probe) -> double {
        if (!present[probe]) return 0.0;
        const double *pq = probe == 0 ? q : nullptr;
        const double *pd = probe == 1 ? dn : nullptr;
        fmm_run(ctx, pl, pq, pd, outs, SUM_FP64, nullptr, 0, 2);
        sample(hfar.data());
        const double *rf = href.data() + probe * K, *nr = hnear.data() + probe * K;
        double ss = 0.0;
        for (int64_t k = 0; k < K; ++k) ss += rf[k] * rf[k];
        const double floor = 0.1 * std::sqrt(ss / (double)K);
        double worst = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double den = std::max(std::fabs(rf[k]), floor);
            const double d = std::fabs(nr[k] + hfar[k] - rf[k]);
            const double e = den > 0.0 ? d / den : d;
            if (!std::isfinite(e)) return INFINITY;
            worst = std::max(worst, e);
        }
        return worst;
    };
    try {
        while (true) {
            const double err = std::max(measure(0), measure(1));
            pl.calib_err = err;
            if (err <= 0.5 * pl.opt_tol || pl.p >= kMaxOrder) break;
            // next order whose padded width buys more terms (28 costs what 31 does)
            int next = kMaxOrder;
            for (int q2 : kOrders)
                if (q2 > pl.p && q2 != 28) {
                    next = q2;
                    break;
                }
            build_tables(ctx, pl, next);
        }
    } catch (...) {
        ctx.opt.near_cache_mb = cache_mb;
        throw;
    }
    ctx.opt.near_cache_mb = cache_mb;
    pl.mq_kept = false;
}

}  // namespace yk
