// gmres.cpp -- restarted GMRES (Saad) with classical Gram-Schmidt applied
// twice (CGS2) in FP64 (the norm after the second projection taken as
// |w|^2 - |h2|^2, which V's orthonormality makes exact up to rounding).  The Krylov basis, the operator and all vector work
// stay on the device; only the k+2 projection scalars per iteration come back
// to the host, where the Givens rotations and the small triangular solve run.
#include <algorithm>
#include <cmath>

#include "yk_internal.h"

namespace yk {

namespace {

double dot_host(Context &ctx, int64_t n, const double *a, const double *b, double *dscal) {
    launch_multi_dot(ctx, n, 1, a, n, b, dscal);
    double v = 0.0;
    YK_HIP(hipMemcpyAsync(&v, dscal, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    YK_HIP(hipStreamSynchronize(ctx.stream));
    return v;
}

}  // namespace

double *pinned_scalars(Context &ctx) {
    if (ctx.noalloc) {   // (ordinary host memory, filled by stream-ordered copies)
        if (ctx.host_scal.size() < 512) ctx.host_scal.resize(512);
        return ctx.host_scal.data();
    }
    if (!ctx.gm_host) YK_HIP(hipHostMalloc((void **)&ctx.gm_host, 512 * sizeof(double), hipHostMallocDefault));
    return ctx.gm_host;
}

GmresResult gmres(Context &ctx, const Apply &A, int64_t n, const double *b, double *x,
                  bool zero_guess, double tol, int max_iter, int m, const double *r0, double r0_norm2,
                  double b_norm2) {
    GmresResult res;
    if (m < 1) m = 1;
    if (m > 120) m = 120;
    if (max_iter < 1) max_iter = 1;
    double *V = ctx.krylov.ensure((size_t)(m + 1) * n);
    double *w = ctx.gm_w.ensure(n);   // reserved for GMRES; operators never touch them
    double *r = ctx.gm_r.ensure(n);
    double *dscal = ctx.scal.ensure(512);   // [0,128) h1, [128,256) h2, 256 norm^2, [300,...) y
    double *host = pinned_scalars(ctx);
    double *P0 = arnoldi_partials(ctx, 0), *P1 = arnoldi_partials(ctx, 1);

    const double bnorm2 = b_norm2 >= 0.0 ? b_norm2 : dot_host(ctx, n, b, b, dscal);
    if (!std::isfinite(bnorm2)) throw Error{YK_ERR_NONFINITE, "right-hand side is not finite"};
    const double bnorm = std::sqrt(bnorm2);
    if (bnorm == 0.0) {
        YK_HIP(hipMemsetAsync(x, 0, n * sizeof(double), ctx.stream));
        res.converged = true;
        return res;
    }
    if (zero_guess) {
        YK_HIP(hipMemsetAsync(x, 0, n * sizeof(double), ctx.stream));
        YK_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    } else if (r0) {
        YK_HIP(hipMemcpyAsync(r, r0, n * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    } else {
        A(x, w);
        res.matvecs++;
        launch_axpby(ctx, n, 1.0, b, -1.0, w, r);
    }
    double beta = std::sqrt(zero_guess ? bnorm2
                            : (r0 && r0_norm2 >= 0.0) ? r0_norm2
                            : dot_host(ctx, n, r, r, dscal));
    if (!std::isfinite(beta)) throw Error{YK_ERR_NONFINITE, "initial residual is not finite"};
    res.res0 = beta / bnorm;

    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hs(2 * 128 + 1);
    if (!ctx.ev_col && !ctx.noalloc) YK_HIP(hipEventCreateWithFlags(&ctx.ev_col, hipEventDisableTiming));
    while (true) {
        if (beta <= tol * bnorm) {
            res.converged = true;
            break;
        }
        if (res.iters >= max_iter) break;
        launch_axpby(ctx, n, 1.0 / beta, r, 0.0, nullptr, V);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool breakdown = false;
        bool issued = false;   // the apply of V[k] is already on the stream
        double rho = 0.25;     // residual reduction per iteration, as last seen
        for (; k < m && res.iters < max_iter; ++k) {
            double *vk = V + (int64_t)k * n;
            if (!issued) {
                A(vk, w);
                res.matvecs++;
            }
            issued = false;
            // CGS2 in three passes over w: partials of V^T w; h1 = V^T w,
            // w -= V h1, partials of V^T w and |w|^2; h2, w - V h2 and its
            // norm (|w|^2 - |h2|^2, V being orthonormal), the next basis
            // vector and the column to the host.  The basis vector is formed
            // before the host sees the column; it is used only if the
            // iteration goes on.
            launch_arnoldi_pass(ctx, n, V, n, w, 0, nullptr, nullptr, k + 1, false, P0);
            launch_arnoldi_pass(ctx, n, V, n, w, k + 1, P0, dscal, k + 1, true, P1);
            launch_arnoldi_finish(ctx, n, V, n, w, k + 1, P1, dscal + 128, dscal + 256, V + (int64_t)(k + 1) * n,
                                  dscal, ctx.noalloc ? nullptr : host);
            if (ctx.noalloc) {
                // no pinned memory or event: copy the column (h1 at 0, h2 at
                // 128, the squared norm at 256) and wait for the stream
                YK_HIP(hipMemcpyAsync(host, dscal, (2 * 128 + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                      ctx.stream));
                YK_HIP(hipStreamSynchronize(ctx.stream));
            } else {
                YK_HIP(hipEventRecord(ctx.ev_col, ctx.stream));
            }
            // The next basis vector is already formed on the device, so its
            // apply goes on the stream before the host waits for the column:
            // the host's rotations then overlap the GPU's work instead of
            // leaving it idle.  Skipped when, at the last seen rate, this
            // column should meet the tolerance (a wasted apply costs more
            // than the wait it hides).
            if (!ctx.noalloc && k + 1 < m && res.iters + 1 < max_iter && rho * std::fabs(g[k]) > 2.0 * tol * bnorm) {
                A(V + (int64_t)(k + 1) * n, w);
                res.matvecs++;
                issued = true;
            }
            if (!ctx.noalloc) YK_HIP(hipEventSynchronize(ctx.ev_col));
            std::copy(host, host + 2 * 128 + 1, hs.begin());
            double *col = &H[(size_t)k * (m + 1)];
            for (int i = 0; i <= k; ++i) col[i] = hs[i] + hs[128 + i];
            const double hk1 = std::sqrt(hs[256]);
            col[k + 1] = hk1;
            for (int i = 0; i <= k + 1; ++i)
                if (!std::isfinite(col[i])) throw Error{YK_ERR_NONFINITE, "Arnoldi produced a non-finite value"};
            res.iters++;
            // apply the previous rotations to the new column, then make a new one
            for (int i = 0; i < k; ++i) {
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const double den = std::hypot(col[k], col[k + 1]);
            cs[k] = den > 0 ? col[k] / den : 1.0;
            sn[k] = den > 0 ? col[k + 1] / den : 0.0;
            col[k] = den;
            col[k + 1] = 0.0;
            const double gprev = std::fabs(g[k]);
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (gprev > 0.0) rho = std::min(1.0, std::fabs(g[k + 1]) / gprev);
            if (hk1 <= 1e-300 * bnorm) {   // lucky breakdown: exact in this space
                breakdown = true;
                ++k;
                break;
            }
            if (std::fabs(g[k + 1]) <= tol * bnorm) {
                ++k;
                break;
            }
        }
        // y = R^{-1} g  (upper triangular k x k)
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[(size_t)j * (m + 1) + i] * y[j];
            y[i] = s / H[(size_t)i * (m + 1) + i];
        }
        YK_HIP(hipMemcpyAsync(dscal + 300, y.data(), k * sizeof(double), hipMemcpyHostToDevice,
                              ctx.stream));
        launch_add_combination(ctx, n, k, V, n, dscal + 300, x);
        // true residual
        A(x, w);
        res.matvecs++;
        launch_axpby(ctx, n, 1.0, b, -1.0, w, r);
        beta = std::sqrt(dot_host(ctx, n, r, r, dscal));
        if (!std::isfinite(beta)) throw Error{YK_ERR_NONFINITE, "residual is not finite"};
        (void)breakdown;
        if (beta <= tol * bnorm) {
            res.converged = true;
            break;
        }
        if (res.iters >= max_iter) break;
    }
    res.res_final = beta / bnorm;
    return res;
}

}  // namespace yk
