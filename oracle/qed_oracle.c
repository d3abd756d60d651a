/*
 * qed_oracle.c -- the FP64 CPU oracle for the Monte-Carlo QED module.
 *
 * TEST INFRASTRUCTURE ONLY (see pic_oracle.c): used by the test-suite, the
 * smoke entry and the benchmark's CPU-baseline leg, never by the HIP library.
 *
 * Sec. IV: nonlinear Compton photon emission (Eq. 23) and nonlinear
 * Breit-Wheeler pair production (Eq. 24), sampled with Monte-Carlo Method I
 * (total probability, then the photon energy from the inverse cumulative
 * spectrum) written in optical-depth form.
 *
 * Rates per unit normalized time (1/w_r), with A = alpha/(sqrt(3) pi) and
 * R = m c^2 / (hbar w_r):
 *   W_rad  = A R F_rad(chi_e) / gamma,
 *   F_rad  = int_0^1 [ (u^2-2u+2)/(1-u) K_{2/3}(y) - int_y^inf K_{1/3} ] du,
 *            y = 2u / (3 (1-u) chi_e),  u = eps_gamma / eps_e;
 *   W_pair = A R F_pair(chi_g) / eps_gamma,
 *   F_pair = int_0^1 [ (x^2+(1-x)^2)/(x(1-x)) K_{2/3}(y) + int_y^inf K_{1/3} ] dx,
 *            y = 2 / (3 chi_g x (1-x)),  x = eps_+ / eps_gamma.
 * Bessel functions come from their integral representations
 *   K_nu(y) = int_0^inf exp(-y cosh t) cosh(nu t) dt,
 *   int_y^inf K_{1/3}(s) ds = int_0^inf exp(-y cosh t) cosh(t/3) / cosh t dt,
 * evaluated with the trapezoidal rule (exponentially convergent for these
 * doubly-exponentially decaying analytic integrands).  Outer integrals use
 * adaptive Gauss-Legendre with nodes found by Newton iteration.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------- Bessel */

static double trap_integral(double y, double nu, int mode) {
    /* mode 0: cosh(nu t);  mode 1: cosh(t/3)/cosh(t) */
    const double h = 1.0 / 64.0;
    double sum = 0.0;
    for (int64_t k = 0;; ++k) {
        double t = (double)k * h;
        double ch = cosh(t);
        double e = exp(-y * ch);
        double term = mode == 0 ? e * cosh(nu * t) : e * cosh(t / 3.0) / ch;
        sum += (k == 0 ? 0.5 : 1.0) * term;
        /* past the maximum of the integrand and negligible */
        if (y * sinh(t) > nu + 1.0 && term < 1e-18 * sum) break;
        if (k > 2000000) break;
    }
    return sum * h;
}

/* Modified Bessel function of the second kind K_nu(y), y > 0. */
double orc_bessel_k(double nu, double y) { return trap_integral(y, nu, 0); }

/* int_y^inf K_{1/3}(s) ds, y > 0. */
double orc_int_k13(double y) { return trap_integral(y, 0.0, 1); }

/* ------------------------------------------------ Gauss-Legendre on [a,b] */

#define GL_N 12
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static void gl_init(void) {
    if (gl_ready) return;
    /* Roots of P_n by Newton from the Chebyshev guess; weights 2/((1-x^2) P_n'^2). */
    for (int i = 0; i < GL_N; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (GL_N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_N; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= GL_N; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

typedef double (*orc_fn)(double, const double *);

static double gl_panel(orc_fn f, const double *par, double a, double b) {
    double m = 0.5 * (a + b), r = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < GL_N; ++i) s += gl_w[i] * f(m + r * gl_x[i], par);
    return s * r;
}

static double gl_adapt(orc_fn f, const double *par, double a, double b, double whole, double tol,
                       int depth) {
    double m = 0.5 * (a + b);
    double l = gl_panel(f, par, a, m), r = gl_panel(f, par, m, b);
    /* accept at the tolerance, or once the difference is at round-off level */
    if (depth > 48 || fabs(l + r - whole) <= tol || fabs(l + r - whole) <= 1e-15 * fabs(l + r))
        return l + r;
    return gl_adapt(f, par, a, m, l, 0.5 * tol, depth + 1) +
           gl_adapt(f, par, m, b, r, 0.5 * tol, depth + 1);
}

/* Adaptive Gauss-Legendre integral of f over [a,b]; `tol` absolute. */
double orc_integrate(orc_fn f, const double *par, double a, double b, double tol) {
    gl_init();
    return gl_adapt(f, par, a, b, gl_panel(f, par, a, b), tol, 0);
}

/* -------------------------------------------------- Compton spectrum (23) */

/* Bracket of Eq. 23 at photon energy fraction u, chi_e = par[0]. */
double orc_compton_bracket(double u, double chi) {
    if (u <= 0.0 || u >= 1.0) return 0.0;
    double y = 2.0 * u / (3.0 * (1.0 - u) * chi);
    if (y > 700.0) return 0.0;
    return (u * u - 2.0 * u + 2.0) / (1.0 - u) * orc_bessel_k(2.0 / 3.0, y) - orc_int_k13(y);
}

/* Integrand in s = u^(1/3) (removes the u^(-2/3) endpoint behaviour). */
static double compton_s(double s, const double *par) {
    return 3.0 * s * s * orc_compton_bracket(s * s * s, par[0]);
}

/* int_0^{u0} bracket(u) du */
double orc_compton_cum(double chi, double u0) {
    if (u0 <= 0.0) return 0.0;
    if (u0 > 1.0) u0 = 1.0;
    double par[1] = {chi};
    double s0 = cbrt(u0);
    /* scale the absolute tolerance with the classical magnitude of F */
    double scale = chi < 1.0 ? 2.5 * ORC_PI * chi : 8.0 * cbrt(chi * chi);
    /* For small chi the spectrum lives at u of order chi (y = 2u/(3(1-u) chi)
     * of order 1), i.e. at s of order chi^(1/3): panels [0, b], [b, 2b], ...
     * with b = chi^(1/3)/4 keep the rule from stepping over it. */
    double b = 0.25 * cbrt(chi), lo = 0.0, sum = 0.0;
    while (b < s0 && b < 0.5) {
        sum += orc_integrate(compton_s, par, lo, b, 1e-13 * scale);
        lo = b;
        b *= 2.0;
    }
    return sum + orc_integrate(compton_s, par, lo, s0, 1e-13 * scale);
}

double orc_frad(double chi) { return orc_compton_cum(chi, 1.0); }

/* --------------------------------------------- Breit-Wheeler spectrum (24) */

double orc_pair_bracket(double x, double chi) {
    if (x <= 0.0 || x >= 1.0) return 0.0;
    double y = 2.0 / (3.0 * chi * x * (1.0 - x));
    if (y > 700.0) return 0.0;
    return (x * x + (1.0 - x) * (1.0 - x)) / (x * (1.0 - x)) * orc_bessel_k(2.0 / 3.0, y) +
           orc_int_k13(y);
}

static double pair_x(double x, const double *par) { return orc_pair_bracket(x, par[0]); }

/* int_0^{x0} bracket(x) dx */
double orc_pair_cum(double chi, double x0) {
    if (x0 <= 0.0) return 0.0;
    if (x0 > 1.0) x0 = 1.0;
    double par[1] = {chi};
    double scale = chi < 1.0 ? 3.0 * chi * exp(-8.0 / (3.0 * chi)) + 1e-300 : 3.0 * cbrt(chi * chi);
    /* split at the symmetric centre, where the spectrum peaks for small chi */
    if (x0 <= 0.5) return orc_integrate(pair_x, par, 0.0, x0, 1e-13 * scale);
    double half = orc_integrate(pair_x, par, 0.0, 0.5, 1e-13 * scale);
    return half + orc_integrate(pair_x, par, 0.5, x0, 1e-13 * scale);
}

double orc_fpair(double chi) { return 2.0 * orc_pair_cum(chi, 0.5); }

/* ------------------------------------------------ inverse CDF (Method I) */

/* Photon energy fraction u0 with int_0^{u0} dW = r W (Method I of Sec. IV;
 * the low-energy cutoff is zero, the u^(-2/3) singularity being integrable).
 * Bisection on the cumulative integral. */
double orc_compton_inverse(double chi, double r) {
    double total = orc_frad(chi);
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_compton_cum(chi, mid) < r * total) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Positron energy fraction x0 with int_0^{x0} dW = r W (Eq. 24). */
double orc_pair_inverse(double chi, double r) {
    double total = orc_fpair(chi);
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_pair_cum(chi, mid) < r * total) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------ Philox4x32 */

/*
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
 *   (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,
 *   c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
 * with the key bumped by the Weyl constants between rounds.
 */
void orc_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += W0;
        k1 += W1;
    }
    memcpy(out, c, sizeof(c));
}

/* Uniform double in the open interval (0,1) from two 32-bit words: the top 52
 * bits v give (v + 1/2) / 2^52, exactly representable, never 0 or 1. */
double orc_u01(uint32_t hi, uint32_t lo) {
    uint64_t v = (((uint64_t)hi << 32) | lo) >> 12;
    return ((double)v + 0.5) * (1.0 / 4503599627370496.0);
}

/*
 * Random stream of the QED module: for particle `id` at step `step` the
 * counter is (id_lo, id_hi, step, stream) with key (seed_lo, seed_hi).
 * Outputs a, b in (0,1) from words (0,1) and (2,3).
 */
void orc_qed_uniforms(uint64_t seed, uint64_t id, uint32_t step, uint32_t stream, double *a,
                      double *b) {
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    *a = orc_u01(out[0], out[1]);
    *b = orc_u01(out[2], out[3]);
}

/* ------------------------------------------------------ quantum parameters */

/* chi = (hbar w_r / m c^2) sqrt((g E + u x B)^2 - (u . E)^2) for a lepton of
 * Lorentz factor g and momentum u; for a photon pass g = eps_gamma, u = k. */
double orc_chi(double hbar_w_mc2, double g, const double *u, const double *E, const double *B) {
    double f[3] = {g * E[0] + u[1] * B[2] - u[2] * B[1], g * E[1] + u[2] * B[0] - u[0] * B[2],
                   g * E[2] + u[0] * B[1] - u[1] * B[0]};
    double ue = u[0] * E[0] + u[1] * E[1] + u[2] * E[2];
    double s = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] - ue * ue;
    return hbar_w_mc2 * sqrt(s > 0.0 ? s : 0.0);
}
