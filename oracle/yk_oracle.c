/*
 * yk_oracle.c -- CPU FP64 oracle for the Yukawa (modified Helmholtz) heat step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; it shares no code, header, table or constant with the GPU
 * path.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.
 *
 * What it computes (Kropinski & Quaife, arXiv 1007.5335):
 *   - K0, K1 from their definitions: the ascending power series (Abramowitz &
 *     Stegun 9.6.10-9.6.13) for z <= 2 and the integral representation
 *     K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt (A&S 9.6.24), summed by
 *     the trapezoid rule, for z > 2;
 *   - the free-space kernel of Sec. 2 without its 1/alpha^2 factor,
 *     K0(|x-y|/alpha)/(2 pi), summed directly over all sources (volume
 *     potential, eq. vol_potential, as a weighted point sum);
 *   - the double-layer kernel d/dnu_y K0(|y-x|/alpha)
 *       = (1/alpha) K1(r/alpha) (x-y).n_y / r          (Sec. 2, double layer;
 *     the sign follows the jump relation and eq. dirichlet:inteqn), with the
 *     on-curve limit -kappa/2 (Sec. 2, continuity of the kernel on Gamma);
 *   - the dense matrix of the discretised second-kind equation (Sec. 3.2,
 *     eq. discrete_sys, trapezoid rule with the diagonal limit):
 *       A = I - 2 [ w_n D(y_j, y_n) / (2 pi) ]_{jn}.
 *
 * Everything is O(N_t N_s), double precision, no blocking or reordering
 * beyond an OpenMP split over targets.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define YKO_PI 3.14159265358979323846
#define YKO_EULER_GAMMA 0.57721566490153286061

/* ------------------------------------------------------------------------ */
/* Modified Bessel functions                                                */
/* ------------------------------------------------------------------------ */

/* I0, I1 by the ascending series (A&S 9.6.10), any z >= 0. */
double yko_i0(double z) {
    double t = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= t / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

double yko_i1(double z) {
    double t = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= t / ((double)k * (double)(k + 1));
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return 0.5 * z * sum;
}

/* K0 by A&S 9.6.13:
 *   K0(z) = -(ln(z/2) + gamma) I0(z) + sum_{k>=1} (z^2/4)^k / (k!)^2 * H_k,
 * H_k = 1 + 1/2 + ... + 1/k. */
static double k0_series(double z) {
    double t = 0.25 * z * z;
    double term = 1.0, i0 = 1.0, s = 0.0, hk = 0.0;
    for (int k = 1; k < 200; ++k) {
        term *= t / ((double)k * (double)k);
        hk += 1.0 / (double)k;
        i0 += term;
        s += term * hk;
        if (term * (hk + 1.0) < 1e-18 * (i0 + s)) break;
    }
    return -(log(0.5 * z) + YKO_EULER_GAMMA) * i0 + s;
}

/* K1 by A&S 9.6.11 with n = 1:
 *   K1(z) = 1/z + ln(z/2) I1(z)
 *           - (z/4) sum_{k>=0} [psi(k+1) + psi(k+2)] (z^2/4)^k / (k! (k+1)!),
 * psi(k+1) = -gamma + H_k. */
static double k1_series(double z) {
    double t = 0.25 * z * z;
    double term = 1.0;                 /* (z^2/4)^k / (k! (k+1)!) */
    double i1s = 1.0;                  /* I1(z) / (z/2) */
    double hk = 0.0;                   /* H_k */
    double s = (-YKO_EULER_GAMMA) + (-YKO_EULER_GAMMA + 1.0); /* k = 0 */
    for (int k = 1; k < 200; ++k) {
        term *= t / ((double)k * (double)(k + 1));
        hk += 1.0 / (double)k;
        double psi_sum = (-YKO_EULER_GAMMA + hk) + (-YKO_EULER_GAMMA + hk + 1.0 / (double)(k + 1));
        i1s += term;
        s += term * psi_sum;
        if (fabs(term * psi_sum) < 1e-18 * fabs(s) && term < 1e-18 * i1s) break;
    }
    return 1.0 / z + log(0.5 * z) * (0.5 * z * i1s) - 0.25 * z * s;
}

/* e^z K_nu(z) = int_0^inf exp(-z (cosh t - 1)) cosh(nu t) dt, trapezoid rule.
 * The integrand is analytic and even; the step is scaled with 1/sqrt(z) so the
 * discretisation error stays far below double precision for every z > 0. */
static double kv_scaled_integral(double nu, double z) {
    double h = 0.2 / sqrt(z);
    if (h > 0.1) h = 0.1;
    double sum = 0.5;                  /* t = 0 term, halved */
    for (int k = 1; k < 100000; ++k) {
        double t = k * h;
        double e = z * (cosh(t) - 1.0);
        double f = exp(-e) * cosh(nu * t);
        sum += f;
        if (e > 50.0 && f < 1e-20 * sum) break;
    }
    return h * sum;
}

double yko_k0(double z) {
    if (z <= 2.0) return k0_series(z);
    return exp(-z) * kv_scaled_integral(0.0, z);
}

double yko_k1(double z) {
    if (z <= 2.0) return k1_series(z);
    return exp(-z) * kv_scaled_integral(1.0, z);
}

/* ------------------------------------------------------------------------ */
/* Direct sums                                                              */
/* ------------------------------------------------------------------------ */

/* out[i] = sum_j q[j] K0(|t_i - s_j| / alpha) / (2 pi)
 * The pair i == j is skipped when `same` is set (targets are the sources);
 * any pair at distance exactly zero is skipped. */
void yko_volume_sum(int64_t nt, const double *txy, int64_t ns, const double *sxy,
                    const double *q, double alpha, int same, double *out) {
    const double inv2pi = 1.0 / (2.0 * YKO_PI);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double xi = txy[2 * i], yi = txy[2 * i + 1], acc = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            if (same && i == j) continue;
            double dx = xi - sxy[2 * j], dy = yi - sxy[2 * j + 1];
            double r = sqrt(dx * dx + dy * dy);
            if (r == 0.0) continue;
            acc += q[j] * yko_k0(r / alpha);
        }
        out[i] = acc * inv2pi;
    }
}

/* D(x, y) = d/dnu_y K0(|x - y|/alpha) = (1/alpha) K1(r/alpha) (x - y).n_y / r */
static double dl_kernel(double xx, double xy, double yx, double yy,
                        double nx, double ny, double alpha) {
    double dx = xx - yx, dy = xy - yy;
    double r = sqrt(dx * dx + dy * dy);
    return yko_k1(r / alpha) / alpha * (dx * nx + dy * ny) / r;
}

double yko_dl_kernel(double xx, double xy, double yx, double yy,
                     double nx, double ny, double alpha) {
    return dl_kernel(xx, xy, yx, yy, nx, ny, alpha);
}

/* out[i] = sum_j d[j] D(t_i, y_j) / (2 pi), pairs at distance zero skipped. */
void yko_dl_sum(int64_t nt, const double *txy, int64_t nb, const double *bxy,
                const double *bn, const double *d, double alpha, double *out) {
    const double inv2pi = 1.0 / (2.0 * YKO_PI);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < nb; ++j) {
            double dx = txy[2 * i] - bxy[2 * j], dy = txy[2 * i + 1] - bxy[2 * j + 1];
            if (dx == 0.0 && dy == 0.0) continue;
            acc += d[j] * dl_kernel(txy[2 * i], txy[2 * i + 1], bxy[2 * j], bxy[2 * j + 1],
                                    bn[2 * j], bn[2 * j + 1], alpha);
        }
        out[i] = acc * inv2pi;
    }
}

/* Diagonal value of the corrected trapezoid rule for the on-curve kernel.
 * Along the curve the kernel is smooth except for a term
 * -(kappa_j |y'_j|^2 / (4 alpha^2)) t^2 log|t| (t the parameter offset), which
 * comes from the (z^2/2) log z term of z K1(z) (Sec. 2: K0 behaves like -log).
 * The punctured trapezoid rule with spacing h integrates t^2 log|t| g(t) with
 * the error -2 zeta'(-2) h^3 g(0) (generalised Euler-Maclaurin expansion,
 * Navot), and zeta'(-2) = -zeta(3) / (4 pi^2); adding the error back at the
 * node makes the rule fifth order.  With w_j = |y'_j| h the kernel's diagonal
 * value becomes -kappa_j / 2 + zeta(3) kappa_j w_j^2 / (8 pi^2 alpha^2). */
double yko_dl_diag(double w, double kappa, double alpha) {
    const double zeta3 = 1.2020569031595942854;
    return kappa * (-0.5 + zeta3 * w * w / (8.0 * YKO_PI * YKO_PI * alpha * alpha));
}

/* Dense matrix of eq. discrete_sys with the corrected trapezoid rule
 * (row-major, nb x nb):
 *   A[j][n] = delta_jn - 2 w_n D(y_j, y_n) / (2 pi),  D(y_j, y_j) = yko_dl_diag. */
void yko_dl_matrix(int64_t nb, const double *bxy, const double *bn, const double *w,
                   const double *kappa, double alpha, double *A) {
    const double c = 2.0 / (2.0 * YKO_PI);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < nb; ++j) {
        for (int64_t n = 0; n < nb; ++n) {
            double dv = (j == n) ? yko_dl_diag(w[j], kappa[j], alpha)
                                 : dl_kernel(bxy[2 * j], bxy[2 * j + 1], bxy[2 * n], bxy[2 * n + 1],
                                             bn[2 * n], bn[2 * n + 1], alpha);
            A[j * nb + n] = (j == n ? 1.0 : 0.0) - c * w[n] * dv;
        }
    }
}

/* S(eps) = sum over the nonzero points j of the square lattice with
 * |j| eps <= 40 of K0(|j| eps) (the terms beyond are below 1e-17 of the
 * sum), by the eight-fold symmetry of the lattice: the axes (4 each), the
 * diagonals (4 each) and the points a > b >= 1 (8 each). */
double yko_lattice_k0_sum(double eps) {
    const double rmax = 40.0;
    const long A = (long)floor(rmax / eps);
    double s = 0.0;
    for (long a = 1; a <= A; ++a) {
        const double ra = (double)a * eps;
        s += 4.0 * yko_k0(ra);
        const double rd = sqrt(2.0) * ra;
        if (rd <= rmax) s += 4.0 * yko_k0(rd);
        for (long b = 1; b < a; ++b) {
            const double r = sqrt((double)(a * a + b * b)) * eps;
            if (r > rmax) break;
            s += 8.0 * yko_k0(r);
        }
    }
    return s;
}

/* Vectorised helpers so tests can evaluate the oracle's special functions. */
void yko_k0_vec(int64_t n, const double *z, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = yko_k0(z[i]);
}
void yko_k1_vec(int64_t n, const double *z, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = yko_k1(z[i]);
}
void yko_i0_vec(int64_t n, const double *z, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = yko_i0(z[i]);
}
void yko_i1_vec(int64_t n, const double *z, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = yko_i1(z[i]);
}

/* Thread count of the OpenMP loops (the CPU baseline is also timed on one core). */
void yko_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
int yko_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
