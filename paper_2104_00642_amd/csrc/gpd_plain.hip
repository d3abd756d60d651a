// gpd_plain.hip -- plain FP64 gather + Boris push + Esirkepov deposit.
//
// One thread per particle, absolute FP64 positions, fields read straight from
// global memory, current deposited with global FP64 atomics.  This is the
// precision bridge and speed baseline for the tiled FP32 kernel: the same
// method (Secs. II.C-E in the step arrangement of Sec. II.F) without LDS
// staging or reduced precision.
#include "device_common.h"
#include "pic_internal.h"

namespace pic {

struct PlainArgs {
    int64_t n;
    double *x[3];
    double *u[3];
    double *w;          // written only to absorb particles at absorbing x faces
    double w0;
    float *chi;
    double chi_scale;
    const double *F[6];
    double *J[3];
    int ng[3];
    double inv_d[3];
    double L[3];
    double dt;
    double qm_half_dt;  // q/m * dt/2
    double jfac[3];     // q * d_a / dt (times w)
    double q;
    double mdV, qdV;    // m dV, q dV for the diagnostics
    double *partials;   // [2 * nblocks]
    uint32_t *status;
    int absorb_x;       // absorbing x faces: no field from, no current to x nodes beyond
                        // [0, n), and a particle leaving [0, (n-1) d) is absorbed (weight 0)
};

template <int DIM>
__device__ __forceinline__ int64_t gidx(const int *ng, int i, int j, int k) {
    i = wrap_index(i, ng[0]);
    j = wrap_index(j, ng[1]);
    if constexpr (DIM == 3) {
        k = wrap_index(k, ng[2]);
        return (int64_t)i + (int64_t)ng[0] * ((int64_t)j + (int64_t)ng[1] * k);
    } else {
        return (int64_t)i + (int64_t)ng[0] * j;
    }
}

template <int DIM>
__device__ __forceinline__ double fld(const PlainArgs &a, int c, int i, int j, int k) {
    if (a.absorb_x && (unsigned)i >= (unsigned)a.ng[0]) return 0.0;
    return a.F[c][gidx<DIM>(a.ng, i, j, k)];
}

template <int DIM>
__device__ __forceinline__ void jadd(const PlainArgs &a, int c, int i, int j, int k, double v) {
    if (a.absorb_x && (unsigned)i >= (unsigned)a.ng[0]) return;
    atomicAdd(&a.J[c][gidx<DIM>(a.ng, i, j, k)], v);
}

template <int DIM, int ORDER, int PUSH>
__global__ void __launch_bounds__(256) gpd_plain_kernel(PlainArgs a) {
    constexpr int NW = ORDER + 1;
    constexpr int L = ORDER + 2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double kin = 0.0, chg = 0.0;
    if (p < a.n) {
        double x[3] = {a.x[0][p], a.x[1][p], DIM == 3 ? a.x[2][p] : 0.0};
        double u[3] = {a.u[0][p], a.u[1][p], a.u[2][p]};
        const double w = a.w ? a.w[p] : a.w0;
        if (!isfinite(u[0] + u[1] + u[2] + x[0] + x[1] + x[2])) atomicOr(a.status, PIC_F_NONFINITE);
        const double ig0 = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double xh[3], xi_h[3];  // half-step position, absolute and in cell units
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            xh[d] = x[d] + 0.5 * a.dt * u[d] * ig0;
            xi_h[d] = xh[d] * a.inv_d[d];
        }

        // ---- gather (Eq. 19): per-axis weights for integer and half nodes
        int i0[2][3];
        double wt[2][3][NW];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            shape_weights<ORDER>(xi_h[d], i0[0][d], wt[0][d]);
            shape_weights<ORDER>(xi_h[d] - 0.5, i0[1][d], wt[1][d]);
        }
        double EB[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const int sx = stag(c, 0), sy = stag(c, 1), sz = DIM == 3 ? stag(c, 2) : 0;
            double acc = 0.0;
            if constexpr (DIM == 2) {
#pragma unroll
                for (int jj = 0; jj < NW; ++jj) {
                    double r = 0.0;
#pragma unroll
                    for (int ii = 0; ii < NW; ++ii)
                        r += wt[sx][0][ii] * fld<2>(a, c, i0[sx][0] + ii, i0[sy][1] + jj, 0);
                    acc += wt[sy][1][jj] * r;
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < NW; ++kk) {
                    double s = 0.0;
#pragma unroll
                    for (int jj = 0; jj < NW; ++jj) {
                        double r = 0.0;
#pragma unroll
                        for (int ii = 0; ii < NW; ++ii)
                            r += wt[sx][0][ii] *
                                 fld<3>(a, c, i0[sx][0] + ii, i0[sy][1] + jj, i0[sz][2] + kk);
                        s += wt[sy][1][jj] * r;
                    }
                    acc += wt[sz][2][kk] * s;
                }
            }
            EB[c] = acc;
        }

        // ---- Boris (Eqs. 13-16) or Vay
        const double u_old[3] = {u[0], u[1], u[2]};
        push_u<PUSH, double>(a.qm_half_dt, EB, EB + 3, u);
        const double g1 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const double ig1 = 1.0 / g1;
        double v[3] = {u[0] * ig1, u[1] * ig1, u[2] * ig1};

        // ---- Esirkepov deposit of x_h -> x_h + dt v (Eqs. 20-22)
        int base[3] = {0, 0, 0};
        double S0[3][L], DS[3][L];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            esirkepov_axis<ORDER>(xi_h[d], (xh[d] + a.dt * v[d]) * a.inv_d[d], base[d], S0[d], DS[d]);
        const double jx = a.jfac[0] * w, jy = a.jfac[1] * w;
        if constexpr (DIM == 2) {
#pragma unroll
            for (int jj = 0; jj < L; ++jj) {
                const double ty = S0[1][jj] + 0.5 * DS[1][jj];
                double acc = 0.0;
#pragma unroll
                for (int ii = 0; ii < L - 1; ++ii) {
                    acc -= jx * DS[0][ii] * ty;
                    jadd<2>(a, 0, base[0] + ii, base[1] + jj, 0, acc);
                }
            }
#pragma unroll
            for (int ii = 0; ii < L; ++ii) {
                const double tx = S0[0][ii] + 0.5 * DS[0][ii];
                double acc = 0.0;
#pragma unroll
                for (int jj = 0; jj < L - 1; ++jj) {
                    acc -= jy * tx * DS[1][jj];
                    jadd<2>(a, 1, base[0] + ii, base[1] + jj, 0, acc);
                }
            }
            const double qv = a.q * w * v[2];
#pragma unroll
            for (int jj = 0; jj < L; ++jj)
#pragma unroll
                for (int ii = 0; ii < L; ++ii) {
                    const double wz = S0[0][ii] * S0[1][jj] + 0.5 * DS[0][ii] * S0[1][jj] +
                                      0.5 * S0[0][ii] * DS[1][jj] +
                                      (1.0 / 3.0) * DS[0][ii] * DS[1][jj];
                    jadd<2>(a, 2, base[0] + ii, base[1] + jj, 0, qv * wz);
                }
        } else {
            const double jz = a.jfac[2] * w;
#pragma unroll
            for (int kk = 0; kk < L; ++kk)
#pragma unroll
                for (int jj = 0; jj < L; ++jj) {
                    const double t = S0[1][jj] * S0[2][kk] + 0.5 * DS[1][jj] * S0[2][kk] +
                                     0.5 * S0[1][jj] * DS[2][kk] +
                                     (1.0 / 3.0) * DS[1][jj] * DS[2][kk];
                    double acc = 0.0;
#pragma unroll
                    for (int ii = 0; ii < L - 1; ++ii) {
                        acc -= jx * DS[0][ii] * t;
                        jadd<3>(a, 0, base[0] + ii, base[1] + jj, base[2] + kk, acc);
                    }
                }
#pragma unroll
            for (int kk = 0; kk < L; ++kk)
#pragma unroll
                for (int ii = 0; ii < L; ++ii) {
                    const double t = S0[0][ii] * S0[2][kk] + 0.5 * DS[0][ii] * S0[2][kk] +
                                     0.5 * S0[0][ii] * DS[2][kk] +
                                     (1.0 / 3.0) * DS[0][ii] * DS[2][kk];
                    double acc = 0.0;
#pragma unroll
                    for (int jj = 0; jj < L - 1; ++jj) {
                        acc -= jy * DS[1][jj] * t;
                        jadd<3>(a, 1, base[0] + ii, base[1] + jj, base[2] + kk, acc);
                    }
                }
#pragma unroll
            for (int jj = 0; jj < L; ++jj)
#pragma unroll
                for (int ii = 0; ii < L; ++ii) {
                    const double t = S0[0][ii] * S0[1][jj] + 0.5 * DS[0][ii] * S0[1][jj] +
                                     0.5 * S0[0][ii] * DS[1][jj] +
                                     (1.0 / 3.0) * DS[0][ii] * DS[1][jj];
                    double acc = 0.0;
#pragma unroll
                    for (int kk = 0; kk < L - 1; ++kk) {
                        acc -= jz * DS[2][kk] * t;
                        jadd<3>(a, 2, base[0] + ii, base[1] + jj, base[2] + kk, acc);
                    }
                }
        }

        // ---- full-step position x^{n+1} = x_h + dt v / 2, periodic wrap
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double xn = xh[d] + 0.5 * a.dt * v[d];
            if (d == 0 && a.absorb_x && (xn < 0.0 || xn >= (double)(a.ng[0] - 1) / a.inv_d[0])) a.w[p] = 0.0;
            if (xn < 0.0) xn += a.L[d];
            else if (xn >= a.L[d]) xn -= a.L[d];
            if (xn >= a.L[d]) xn = 0.0;  // a tiny negative value rounded up to L
            a.x[d][p] = xn;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) a.u[d][p] = u[d];

        if (a.chi) {
            // chi_e of Sec. IV with the fields at x_h and u^{n+1/2}
            double uh[3] = {0.5 * (u_old[0] + u[0]), 0.5 * (u_old[1] + u[1]), 0.5 * (u_old[2] + u[2])};
            double gh = sqrt(1.0 + uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]);
            double f0 = gh * EB[0] + uh[1] * EB[5] - uh[2] * EB[4];
            double f1 = gh * EB[1] + uh[2] * EB[3] - uh[0] * EB[5];
            double f2 = gh * EB[2] + uh[0] * EB[4] - uh[1] * EB[3];
            double ue = uh[0] * EB[0] + uh[1] * EB[1] + uh[2] * EB[2];
            double s2 = f0 * f0 + f1 * f1 + f2 * f2 - ue * ue;
            a.chi[p] = (float)(a.chi_scale * sqrt(s2 > 0.0 ? s2 : 0.0));
        }
        kin = w * (g1 - 1.0);
        chg = w;
    }
    // ---- fixed-order block reduction of the diagnostics (FP64)
    __shared__ double sk[256], sq[256];
    sk[threadIdx.x] = kin;
    sq[threadIdx.x] = chg;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sk[threadIdx.x] += sk[threadIdx.x + s];
            sq[threadIdx.x] += sq[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partials[2 * blockIdx.x] = sk[0] * a.mdV;
        a.partials[2 * blockIdx.x + 1] = sq[0] * a.qdV;
    }
}

// Sum `nval` interleaved FP64 partials over `nblocks` blocks in a fixed order
// and add scale * sum to diag[off + v].
template <int DIM, int ORDER>
static void launch_plain(const PlainArgs &a, int pusher, dim3 grid, dim3 block, hipStream_t s) {
    if (pusher == PIC_PUSH_VAY) gpd_plain_kernel<DIM, ORDER, PIC_PUSH_VAY><<<grid, block, 0, s>>>(a);
    else gpd_plain_kernel<DIM, ORDER, PIC_PUSH_BORIS><<<grid, block, 0, s>>>(a);
}

__global__ void __launch_bounds__(256) finalize_kernel(const double *partials, int64_t nblocks,
                                                       int nval, double *diag, int off,
                                                       double scale) {
    __shared__ double s[256];
    for (int v = 0; v < nval; ++v) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partials[b * nval + v];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) diag[off + v] += scale * s[0];
        __syncthreads();
    }
}

hipError_t launch_finalize(const double *partials, int64_t nblocks, int nval, double *diag,
                           int off, double scale, hipStream_t s) {
    finalize_kernel<<<1, 256, 0, s>>>(partials, nblocks, nval, diag, off, scale);
    return hipGetLastError();
}

size_t push_partials_plain(int64_t n) { return 2 * (size_t)((n + 255) / 256); }

hipError_t launch_gpd_plain(Ctx *c, const pic_species *sp, const pic_particles *p,
                            const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps) {
    const pic_config &cfg = c->cfg;
    PlainArgs a{};
    a.n = p->n;
    for (int d = 0; d < 3; ++d) {
        a.x[d] = p->x[d];
        a.u[d] = (double *)p->u[d];
        a.J[d] = (double *)f->J[d];
        a.F[d] = (const double *)f->E[d];
        a.F[3 + d] = (const double *)f->B[d];
        a.ng[d] = (int)cfg.n[d];
        a.inv_d[d] = 1.0 / cfg.d[d];
        a.L[d] = (double)cfg.n[d] * cfg.d[d];
        a.jfac[d] = sp->q * cfg.d[d] / cfg.dt;
    }
    a.w = (double *)p->w;
    a.absorb_x = absorbing_x(cfg);
    a.w0 = sp->w0;
    a.chi = cfg.hbar_omega_mc2 > 0.0 ? p->chi : nullptr;
    a.chi_scale = cfg.hbar_omega_mc2;
    a.dt = cfg.dt;
    a.qm_half_dt = 0.5 * sp->q / sp->m * cfg.dt;
    a.q = sp->q;
    double dV = cfg.d[0] * cfg.d[1] * (c->dim == 3 ? cfg.d[2] : 1.0);
    a.mdV = sp->m * dV;
    a.qdV = sp->q * dV;
    a.status = c->status;
    const int64_t nblocks = (p->n + 255) / 256;
    if (nblocks == 0) return hipSuccess;
    if (ps) {
        a.partials = ps->partials;
    } else {
        if (ensure_partials(c, push_partials_plain(p->n)) != PIC_OK) return hipErrorOutOfMemory;
        a.partials = c->partials;
    }
    dim3 grid((unsigned)nblocks), block(256);
    const int key = c->dim * 10 + cfg.order;
    switch (key) {
        case 21: launch_plain<2, 1>(a, cfg.pusher, grid, block, s); break;
        case 22: launch_plain<2, 2>(a, cfg.pusher, grid, block, s); break;
        case 31: launch_plain<3, 1>(a, cfg.pusher, grid, block, s); break;
        case 32: launch_plain<3, 2>(a, cfg.pusher, grid, block, s); break;
        case 24: launch_plain<2, 4>(a, cfg.pusher, grid, block, s); break;
        case 34: launch_plain<3, 4>(a, cfg.pusher, grid, block, s); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !diag) return e;
    return launch_finalize(a.partials, nblocks, 2, diag, 0, 1.0, s);
}

}  // namespace pic
