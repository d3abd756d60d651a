// diag.hip -- charge density on the nodes and the Gauss residual (Sec. II.B).
//
// The divergence equations (Eqs. 1-2) are not solved: they hold by
// themselves once they hold initially and the current conserves charge
// (Eq. 5), which the Esirkepov deposit does (Sec. II.E).  The residual
// div E - rho on the nodes must therefore stay at its initial value from step
// to step, up to rounding; these kernels measure it on diagnostic steps.
//   rho(i) += q w prod_a W(i_a - xi_a): the integer-node shape weights of
//   Sec. II.D at the particle's position in cell units, taken at the half
//   step x^n + dt u^n / (2 gamma^n) (the time of E after the first half field
//   update) or at x^n; FP64 accumulation in global memory.
//   div E(i) = sum_a (E_a(i) - E_a(i - e_a)) / d_a (E_a sits half a cell up
//   axis a from node i), in FP64 from the FP32 or FP64 planes.
#include <algorithm>

#include "device_common.h"
#include "pic_internal.h"

namespace pic {

struct RhoArgs {
    // FP32 layout
    const int32_t *cell;
    const float *off[3];
    const float *uf[3];
    const float *wf;
    // FP64 layout
    const double *x[3];
    const double *ud[3];
    const double *wd;
    int64_t n;
    double w0, q;
    int ng[3];
    int bx, by;
    double hdt_d[3];  // dt / (2 d), 0 for positions at x^n
    double inv_d[3];
    double *rho;
};

// nodes of every axis wrap periodically: the density of the whole domain,
// also with absorbing x faces (a particle there sits inside [0, n-1])
template <int DIM, int ORDER, bool FP64>
__global__ void __launch_bounds__(256) rho_kernel(RhoArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    int base[3] = {0, 0, 0};
    double xi[3] = {0.0, 0.0, 0.0}, w;
    double u[3];
    if constexpr (FP64) {
        for (int d = 0; d < 3; ++d) u[d] = a.ud[d][p];
        w = a.wd ? a.wd[p] : a.w0;
    } else {
        for (int d = 0; d < 3; ++d) u[d] = (double)a.uf[d][p];
        w = a.wf ? (double)a.wf[p] : a.w0;
    }
    const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if constexpr (FP64) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = a.x[d][p] * a.inv_d[d] + a.hdt_d[d] * u[d] * ig;
    } else {
        const int32_t c = a.cell[p];
        const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
        base[0] = c & mx;
        base[1] = (c >> a.bx) & my;
        base[2] = DIM == 3 ? (c >> (a.bx + a.by)) : 0;
        // offsets are positions relative to the cell (no loss of resolution)
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = (double)a.off[d][p] + a.hdt_d[d] * u[d] * ig;
    }
    int i0[3] = {0, 0, 0};
    double wt[3][ORDER + 1];
#pragma unroll
    for (int d = 0; d < DIM; ++d) shape_weights<ORDER>(xi[d], i0[d], wt[d]);
    const double qw = a.q * w;
#pragma unroll
    for (int kk = 0; kk < (DIM == 3 ? ORDER + 1 : 1); ++kk) {
        const int64_t gk = DIM == 3 ? (int64_t)wrap_index(base[2] + i0[2] + kk, a.ng[2]) : 0;
        const double wk = DIM == 3 ? wt[2][kk] : 1.0;
#pragma unroll
        for (int jj = 0; jj <= ORDER; ++jj) {
            const int64_t gj = wrap_index(base[1] + i0[1] + jj, a.ng[1]);
#pragma unroll
            for (int ii = 0; ii <= ORDER; ++ii) {
                const int64_t gi = wrap_index(base[0] + i0[0] + ii, a.ng[0]);
                atomicAdd(&a.rho[gi + (int64_t)a.ng[0] * (gj + (int64_t)a.ng[1] * gk)],
                          qw * wk * wt[1][jj] * wt[0][ii]);
            }
        }
    }
}

constexpr int GAUSS_BLOCKS = GAUSS_PART;

// residual(i) = div E(i) - rho(i); per-block maxima of |residual|
template <typename T>
__global__ void __launch_bounds__(256) gauss_kernel(const T *E0, const T *E1, const T *E2, const double *rho,
                                                    int dim, int n0, int n1, int n2, double id0, double id1,
                                                    double id2, double *res, double *part) {
    const int64_t nc = (int64_t)n0 * n1 * n2;
    double m = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % n0);
        const int j = (int)((c / n0) % n1);
        const int k = (int)(c / ((int64_t)n0 * n1));
        const int64_t cx = c - i + (i == 0 ? n0 - 1 : i - 1);
        const int64_t cy = c + (int64_t)n0 * ((j == 0 ? n1 - 1 : j - 1) - j);
        double s = ((double)E0[c] - (double)E0[cx]) * id0 + ((double)E1[c] - (double)E1[cy]) * id1;
        if (dim == 3) {
            const int64_t cz = c + (int64_t)n0 * n1 * ((k == 0 ? n2 - 1 : k - 1) - k);
            s += ((double)E2[c] - (double)E2[cz]) * id2;
        }
        const double r = s - rho[c];
        if (res) res[c] = r;
        m = fmax(m, fabs(r));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    __shared__ double wm[4];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
}

// diag[3] = max(diag[3], max of the block maxima)
__global__ void __launch_bounds__(256) gauss_max_kernel(const double *part, int nblocks, double *diag) {
    double m = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmax(m, part[b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    __shared__ double wm[4];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) diag[3] = fmax(diag[3], fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3])));
}

template <bool FP64>
static void launch_rho_t(int key, const RhoArgs &a, hipStream_t s) {
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    switch (key) {
        case 21: rho_kernel<2, 1, FP64><<<nb, 256, 0, s>>>(a); break;
        case 22: rho_kernel<2, 2, FP64><<<nb, 256, 0, s>>>(a); break;
        case 24: rho_kernel<2, 4, FP64><<<nb, 256, 0, s>>>(a); break;
        case 31: rho_kernel<3, 1, FP64><<<nb, 256, 0, s>>>(a); break;
        case 32: rho_kernel<3, 2, FP64><<<nb, 256, 0, s>>>(a); break;
        case 34: rho_kernel<3, 4, FP64><<<nb, 256, 0, s>>>(a); break;
    }
}

hipError_t launch_rho(Ctx *c, const pic_species *sp, const pic_particles *p, int at_half, double *rho,
                      hipStream_t s) {
    const pic_config &cfg = c->cfg;
    if (p->n == 0) return hipSuccess;
    RhoArgs a{};
    a.n = p->n;
    a.q = sp->q;
    a.w0 = sp->w0;
    a.rho = rho;
    a.bx = c->bits[0];
    a.by = c->bits[1];
    for (int d = 0; d < 3; ++d) {
        a.ng[d] = (int)cfg.n[d];
        a.inv_d[d] = 1.0 / cfg.d[d];
        a.hdt_d[d] = at_half ? 0.5 * cfg.dt / cfg.d[d] : 0.0;
    }
    const int key = c->dim * 10 + cfg.order;
    if (cfg.precision == PIC_FP64_PLAIN) {
        for (int d = 0; d < 3; ++d) {
            a.x[d] = p->x[d];
            a.ud[d] = (const double *)p->u[d];
        }
        a.wd = (const double *)p->w;
        launch_rho_t<true>(key, a, s);
    } else {
        a.cell = p->cell;
        for (int d = 0; d < 3; ++d) {
            a.off[d] = p->off[d];
            a.uf[d] = (const float *)p->u[d];
        }
        a.wf = (const float *)p->w;
        launch_rho_t<false>(key, a, s);
    }
    return hipGetLastError();
}

hipError_t launch_gauss(Ctx *c, const pic_fields *f, const double *rho, double *res, double *diag,
                        hipStream_t s) {
    const pic_config &cfg = c->cfg;
    const int64_t nc = cfg.n[0] * cfg.n[1] * cfg.n[2];
    const int nb = (int)std::min<int64_t>(GAUSS_BLOCKS, (nc + 255) / 256);
    const double id0 = 1.0 / cfg.d[0], id1 = 1.0 / cfg.d[1], id2 = c->dim == 3 ? 1.0 / cfg.d[2] : 0.0;
    const int n0 = (int)cfg.n[0], n1 = (int)cfg.n[1], n2 = (int)cfg.n[2];
    if (cfg.precision == PIC_FP64_PLAIN)
        gauss_kernel<double><<<nb, 256, 0, s>>>((const double *)f->E[0], (const double *)f->E[1],
                                                (const double *)f->E[2], rho, c->dim, n0, n1, n2, id0, id1, id2,
                                                res, c->gauss_part);
    else
        gauss_kernel<float><<<nb, 256, 0, s>>>((const float *)f->E[0], (const float *)f->E[1],
                                               (const float *)f->E[2], rho, c->dim, n0, n1, n2, id0, id1, id2,
                                               res, c->gauss_part);
    if (diag) gauss_max_kernel<<<1, 256, 0, s>>>(c->gauss_part, nb, diag);
    return hipGetLastError();
}

}  // namespace pic
