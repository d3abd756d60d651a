// beam.hip -- self-fields of a relativistic bi-Gaussian bunch (Sec. III(c)):
// Poisson's equation solved in the bunch's rest frame, then the Lorentz
// transformation of its field to the laboratory frame.
//
// Rest frame (primes): the bunch moves along +x with Lorentz factor gamma,
// so at rest it is gamma times longer along x, sigma' = (gamma sigma_x,
// sigma_y, sigma_z), with the same total charge Q = q n_b (2 pi)^{D/2}
// prod sigma (D = 3; D = 2 in a 2D box, the bunch uniform along z).  The
// free-space solution of lap phi' = -rho' (div E = rho in these units) comes
// from writing the Green's function as an integral of heat kernels over a
// diffusion time s: a heat kernel of time s is a Gaussian of variance 2 s per
// axis, so its convolution with the bunch is a Gaussian of variances
// v_b(s) = sigma_b'^2 + 2 s and
//   E'_a(p) = Q Int_0^inf (p_a / v_a(s)) prod_b N(p_b; v_b(s)) ds,
//   N(x; v) = exp(-x^2 / (2 v)) / sqrt(2 pi v).
// The integral is taken by the trapezoidal rule in tau = ln s; the integrand
// is analytic in a strip of half-width pi/2 around the real tau axis, so the
// rule's error falls like exp(-pi^2 / h) (about 1e-17 at the step h = 1/4
// used here), and the bounds leave out 1e-13 of the integral at either end.
// Lab frame, at the call's time: x' = gamma (x - x_c); E_x = E'_x,
// E_perp = gamma E'_perp, B = beta x^ x E (the rest-frame B' is zero).
//
// One thread per cell; each evaluates the five nonzero components at their
// own Yee positions (E_x at (i+1/2, j, k), E_y (i, j+1/2, k), E_z
// (i, j, k+1/2), B_y (i+1/2, j, k+1/2), B_z (i+1/2, j+1/2, k)).  The
// quadrature weights, which do not depend on the point, sit in LDS.
#include <math.h>

#include "pic_internal.h"

namespace pic {

constexpr int BEAM_MAXQ = 512;  // quadrature nodes at most

struct BeamArgs {
    double Q;          // total charge
    double c[3];       // centre
    double s2[3];      // rest-frame variances
    double gamma, beta;
    double d[3];
    int n[3];
    double tau0, htau;
    int nq;
};

template <typename R, int DIM>
__global__ void __launch_bounds__(256) beam_field_kernel(BeamArgs b, R *Ex, R *Ey, R *Ez, R *By, R *Bz) {
    // per node m: w = h s prod_b (2 pi v_b)^(-1/2), and 1/v_b
    __shared__ double wq[BEAM_MAXQ];
    __shared__ double iv[3][BEAM_MAXQ];
    for (int m = threadIdx.x; m < b.nq; m += blockDim.x) {
        const double s = exp(b.tau0 + m * b.htau);
        double w = b.htau * s;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = b.s2[a] + 2.0 * s;
            iv[a][m] = 1.0 / v;
            if (a < DIM) w /= sqrt(2.0 * 3.14159265358979323846 * v);
        }
        wq[m] = w;
    }
    __syncthreads();
    const int64_t ncell = (int64_t)b.n[0] * b.n[1] * b.n[2];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int i = (int)(c % b.n[0]);
    const int j = (int)((c / b.n[0]) % b.n[1]);
    const int k = (int)(c / ((int64_t)b.n[0] * b.n[1]));
    // rest-frame component a at the lab point of the cell shifted by (ox, oy, oz) cells
    auto rest = [&](int a, double ox, double oy, double oz) {
        const double q0 = b.gamma * ((i + ox) * b.d[0] - b.c[0]);
        const double q1 = (j + oy) * b.d[1] - b.c[1];
        const double q2 = DIM == 3 ? (k + oz) * b.d[2] - b.c[2] : 0.0;
        const double qa = a == 0 ? q0 : (a == 1 ? q1 : q2);
        double acc = 0.0;
        for (int m = 0; m < b.nq; ++m) {
            double ex = q0 * q0 * iv[0][m] + q1 * q1 * iv[1][m];
            if (DIM == 3) ex += q2 * q2 * iv[2][m];
            acc += wq[m] * iv[a][m] * exp(-0.5 * ex);
        }
        return b.Q * qa * acc;
    };
    const double g = b.gamma;
    Ex[c] += (R)rest(0, 0.5, 0.0, 0.0);
    Ey[c] += (R)(g * rest(1, 0.0, 0.5, 0.0));
    Bz[c] += (R)(b.beta * g * rest(1, 0.5, 0.5, 0.0));
    if (DIM == 3) {
        Ez[c] += (R)(g * rest(2, 0.0, 0.0, 0.5));
        By[c] += (R)(-b.beta * g * rest(2, 0.5, 0.0, 0.5));
    }
}

hipError_t launch_beam_fields(Ctx *ctx, const pic_beam *beam, const pic_fields *f, hipStream_t s) {
    const pic_config &cfg = ctx->cfg;
    const int dim = ctx->dim;
    BeamArgs b{};
    const double g = beam->gamma;
    b.gamma = g;
    b.beta = sqrt(fmax(0.0, 1.0 - 1.0 / (g * g)));
    double prod = 1.0;
    for (int a = 0; a < 3; ++a) {
        b.c[a] = a < dim ? beam->center[a] : 0.0;
        b.d[a] = cfg.d[a];
        b.n[a] = (int)cfg.n[a];
        const double sl = a < dim ? beam->sigma[a] : 1.0;
        if (a < dim) prod *= sl;
        b.s2[a] = (a == 0 ? g * sl : sl) * (a == 0 ? g * sl : sl);
    }
    b.Q = beam->charge * beam->density * pow(2.0 * 3.14159265358979323846, 0.5 * dim) * prod;
    // bounds of s: 1e-13 of the smallest variance, 1e14 of the largest
    // squared rest-frame distance to a node (plus the largest variance)
    double vmin = b.s2[0], vmax = b.s2[0], r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        vmin = fmin(vmin, b.s2[a]);
        vmax = fmax(vmax, b.s2[a]);
        const double ext = fmax(fabs(-b.c[a]), fabs((double)cfg.n[a] * cfg.d[a] - b.c[a]));
        r2 += (a == 0 ? g * g : 1.0) * ext * ext;
    }
    const double tau0 = log(vmin) - 30.0, tau1 = log(vmax + r2) + 32.3;
    b.htau = 0.25;
    b.nq = (int)ceil((tau1 - tau0) / b.htau) + 1;
    if (b.nq > BEAM_MAXQ) {  // extreme aspect ratios: a wider step, still well inside the strip
        b.nq = BEAM_MAXQ;
        b.htau = (tau1 - tau0) / (BEAM_MAXQ - 1);
    }
    b.tau0 = tau0;
    const int64_t ncell = cfg.n[0] * cfg.n[1] * cfg.n[2];
    const unsigned blocks = (unsigned)((ncell + 255) / 256);
    if (cfg.precision == PIC_FP64_PLAIN) {
        double *E[3] = {(double *)f->E[0], (double *)f->E[1], (double *)f->E[2]};
        double *B[3] = {(double *)f->B[0], (double *)f->B[1], (double *)f->B[2]};
        if (dim == 3) beam_field_kernel<double, 3><<<blocks, 256, 0, s>>>(b, E[0], E[1], E[2], B[1], B[2]);
        else beam_field_kernel<double, 2><<<blocks, 256, 0, s>>>(b, E[0], E[1], E[2], B[1], B[2]);
    } else {
        float *E[3] = {(float *)f->E[0], (float *)f->E[1], (float *)f->E[2]};
        float *B[3] = {(float *)f->B[0], (float *)f->B[1], (float *)f->B[2]};
        if (dim == 3) beam_field_kernel<float, 3><<<blocks, 256, 0, s>>>(b, E[0], E[1], E[2], B[1], B[2]);
        else beam_field_kernel<float, 2><<<blocks, 256, 0, s>>>(b, E[0], E[1], E[2], B[1], B[2]);
    }
    return hipGetLastError();
}

}  // namespace pic
