// mlp.h -- learned warm start for the density solve (see mlp.hip).
#pragma once

#include <memory>
#include <vector>

#include "yk_internal.h"

namespace yk {

// C = A B (FP32 matrix cores); with tanh_bias, C = tanh(A B + tanh_bias[col])
void sgemm(Context &ctx, int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *B,
           int64_t sbk, int64_t sbn, float *C, int64_t ldc, DevBuf<float> &part,
           const float *tanh_bias = nullptr);

struct WarmStart {
    struct Obs {
        DevBuf<double> g, s;   // Dirichlet data g and density sigma of one solved step
    };
    Context &ctx;
    yk_ws_options opt;
    int64_t n = 0;
    int H = 0, Fp = 0;
    std::vector<int64_t> offsets;
    DevBuf<int64_t> off;
    DevBuf<int32_t> curve_buf, idx_buf;   // private copies of the boundary's curve ids and indices
    const int32_t *curve = nullptr, *idx = nullptr;
    const double *kappa = nullptr;
    const double *xy = nullptr;           // the boundary's node array (identifies it)
    int64_t o_W1 = 0, o_b1 = 0, o_W2 = 0, o_b2 = 0, o_w3 = 0, o_b3 = 0, n_params = 0;
    DevBuf<float> params, adam_m, adam_v, grad;
    int64_t adam_t = 0;
    DevBuf<float> Xall, Tall, Xbat, Tbat, h1, h2, d1, d2, yb, dyb, part, cpart, lpart;
    DevBuf<float> wt;                     // transposed hidden-layer weights for the fused inference
    DevBuf<int32_t> brows;
    DevBuf<double> scal, dtmp, fscale;
    std::vector<std::unique_ptr<Obs>> obs;
    bool trained = false;

    WarmStart(Context &c, BoundaryData &b, const yk_ws_options &o);
    void observe(const double *g, const double *sigma);
    double train();
    void predict(const double *g_next, double *out);
    void forward(int64_t rows, const float *X, float *y);
    // the same outputs without activation arrays: both hidden layers of a
    // block of rows in one kernel (when the sizes are the default ones)
    void forward_fused(int64_t rows, const float *X, float *y);
    double loss_grad(int64_t rows, const float *X, const float *T, float *G);
    // one Adam step of the parameters on the gradient G [n_params]
    void adam_step(const float *G);

  private:
    // writes the features of one step into X and the step's scales into fs
    // (device memory; fs[6] is the density scale r_s)
    void features(const double *sm1, const double *s0, const double *gm1, const double *g0,
                  const double *gp1, float *X, double *fs);
    void colsum(int64_t rows, int cols, const float *D, float *out);
};

}  // namespace yk

struct yk_ws_s {
    yk_ctx owner;
    std::unique_ptr<yk::WarmStart> w;
};
