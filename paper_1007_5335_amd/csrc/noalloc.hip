// noalloc.hip -- the density solve with direct sums for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Every device buffer of the solve (Krylov basis, GMRES vectors, reduction
// partials, dipole vectors, the boundary's weights and curve indices) is a
// window into one file-scope device array, `scratch`, of kScratchDoubles
// doubles (32 MiB), which each GPU holds for the life of the process.  Its
// device address is taken once per device with hipGetSymbolAddress (at
// yk_create, with that device current) and kept per device; host code uses
// only that address, never the array's name.  Every call on a device uses
// the same array and leaves its contents behind; the solve initialises
// everything it reads, and calls that overlap on one GPU race.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "sums.h"
#include "yk_internal.h"

namespace yk {

namespace {

constexpr int64_t kScratchDoubles = (int64_t)1 << 22;   // 32 MiB

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mutex;
std::unordered_map<int, double *> g_scratch;   // device -> address of its copy of scratch

constexpr int64_t kAlign = 32;   // doubles (256 bytes)
inline int64_t up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Fixed part of the layout (doubles): device scalars, Arnoldi partials
// (three blocks of 256 chunks x 129 rows), dot-product partials (64 x 128)
constexpr int64_t kScal = 512;
constexpr int64_t kArn = 3 * 256 * 129;
constexpr int64_t kPart = 64 * 128;

}  // namespace

void noalloc_init_device(int device) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch.count(device)) return;
    double *ptr = nullptr;
    YK_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error{YK_ERR_HIP, "hipGetSymbolAddress returned a null address for the workspace array"};
    g_scratch[device] = ptr;
}

static double *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = g_scratch.find(device);
    return it == g_scratch.end() ? nullptr : it->second;
}

// Doubles the solve needs for n nodes, n_curves curves and Krylov dimension m.
int64_t noalloc_need(int64_t n, int n_curves, int m) {
    const int64_t fixed = up(kScal) + up(kArn) + up(kPart) + up(n_curves + 1);
    // per node: w, curve + idx (two int32), b, GMRES w and r, operator
    // output, dipole vectors (2), and the m + 1 basis vectors
    return fixed + 6 * up(n) + up(2 * n) + up((int64_t)(m + 1) * n);
}

// The operator and GMRES of solve_density (capi.cpp), run with a context
// whose buffers are all borrowed from the array.
GmresResult solve_density_direct(Context &ctx, BoundaryData &bd, double alpha, const double *b, double *sigma,
                                 bool zero_guess, double tol, int max_iter);

}  // namespace yk

using namespace yk;

extern "C" yk_status yk_gmres_density_noalloc(yk_ctx ctx, const yk_boundary *bnd, double alpha, const double *g,
                                              const double *sigma0, double tol, int max_iter, double *sigma,
                                              yk_stats *stats) {
    if (!ctx) return YK_ERR_ARG;
    Context &c = ctx->c;
    try {
        YK_REQUIRE(g && sigma, "g/sigma are NULL");
        YK_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        YK_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
        YK_REQUIRE(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        YK_REQUIRE(bnd != nullptr && bnd->n_curves >= 1 && bnd->offset != nullptr, "invalid boundary");
        YK_REQUIRE(bnd->xy && bnd->normal && bnd->speed && bnd->curvature, "a boundary array is NULL");
        YK_REQUIRE(bnd->offset[0] == 0, "boundary offset[0] must be 0");
        for (int k = 0; k < bnd->n_curves; ++k)
            YK_REQUIRE(bnd->offset[k + 1] > bnd->offset[k], "boundary offsets must increase strictly");
        const int64_t n = bnd->offset[bnd->n_curves];
        const int m = std::max(1, std::min(120, c.opt.gmres_m));
        const int64_t need = noalloc_need(n, bnd->n_curves, m);
        if (need > kScratchDoubles)
            throw Error{YK_ERR_ARG, "the allocation-free solve holds (gmres_m + 9) x N doubles plus a fixed part in "
                                    "its 32 MiB array: " + std::to_string(n) + " nodes need " +
                                    std::to_string(need) + " of " + std::to_string(kScratchDoubles)};
        double *base = scratch_of(c.device);
        if (!base) throw Error{YK_ERR_HIP, "the workspace array's address was not taken on this device"};
        if (stats) std::memset(stats, 0, sizeof(*stats));

        // a context of the caller's stream and options, direct sums, whose
        // every device buffer is a window of the array
        Context lc;
        lc.opt = c.opt;
        lc.opt.direct = 1;
        lc.opt.precision = YK_PREC_FP64;
        lc.opt.debug_flags = c.opt.debug_flags & 1;
        lc.stream = c.stream;
        lc.device = c.device;
        lc.noalloc = true;
        int64_t at = 0;
        auto take = [&](int64_t count) {
            double *p = base + at;
            at += up(count);
            return p;
        };
        lc.scal.borrow(take(kScal), kScal);
        lc.arn_partial.borrow(take(kArn), kArn);
        lc.partial.borrow(take(kPart), kPart);
        int64_t *doff = reinterpret_cast<int64_t *>(take(bnd->n_curves + 1));
        BoundaryData bd;
        bd.xy = bnd->xy;
        bd.n = n;
        bd.n_curves = bnd->n_curves;
        bd.offset.assign(bnd->offset, bnd->offset + bnd->n_curves + 1);
        bd.normal = bnd->normal;
        bd.curvature = bnd->curvature;
        bd.speed = bnd->speed;
        bd.w.borrow(take(n), n);
        int32_t *ci = reinterpret_cast<int32_t *>(take(n));   // curve ids, then node indices
        bd.curve.borrow(ci, n);
        bd.idx.borrow(ci + n, n);
        double *b = take(n);
        lc.gm_w.borrow(take(n), n);
        lc.gm_r.borrow(take(n), n);
        lc.ws_a.borrow(take(n), n);
        lc.dn.borrow(take(2 * n), 2 * n);
        lc.krylov.borrow(take((int64_t)(m + 1) * n), (size_t)(m + 1) * n);
        if (at > kScratchDoubles) throw Error{YK_ERR_INTERNAL, "allocation-free layout overruns its array"};

        YK_HIP(hipMemcpyAsync(doff, bd.offset.data(), (bnd->n_curves + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                              lc.stream));
        launch_boundary_prep(lc, n, bnd->n_curves, doff, bnd->speed, bd.w.p, bd.curve.p, bd.idx.p);
        launch_axpby(lc, n, -2.0 * alpha * alpha, g, 0.0, nullptr, b);
        if (sigma0 && sigma0 != sigma)
            YK_HIP(hipMemcpyAsync(sigma, sigma0, n * sizeof(double), hipMemcpyDeviceToDevice, lc.stream));
        const auto t0 = std::chrono::steady_clock::now();
        GmresResult r = solve_density_direct(lc, bd, alpha, b, sigma, sigma0 == nullptr, tol, max_iter);
        YK_HIP(hipStreamSynchronize(lc.stream));
        if (stats) {
            stats->iters = r.iters;
            stats->guess_used = sigma0 ? 1 : 0;
            stats->matvecs = r.matvecs;
            stats->res0 = r.res0;
            stats->res_final = r.res_final;
            stats->ms[2] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        c.last_error.clear();
        if (!r.converged) {
            c.last_error = "GMRES did not reach the tolerance within max_iter";
            return YK_ERR_NOCONV;
        }
        return YK_OK;
    } catch (const Error &e) {
        c.last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        c.last_error = "host allocation failed";
        return YK_ERR_NOMEM;
    } catch (const std::exception &e) {
        c.last_error = e.what();
        return YK_ERR_INTERNAL;
    } catch (...) {
        c.last_error = "unknown internal error";
        return YK_ERR_INTERNAL;
    }
}
