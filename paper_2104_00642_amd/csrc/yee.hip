// yee.hip -- half-step Yee FDTD update (Sec. II.B Eqs. 9-10, split in halves as
// in Sec. II.F) and the FP64 field-energy reduction.
//
// Bandwidth-bound stencil: one thread per cell, x-fastest so that every
// wavefront reads and writes contiguous 256-byte rows; the -1/+1 neighbours
// along y/z come from rows the neighbouring wavefronts already pulled into L2.
// Periodic in every axis, or along x absorbing: the domain is x in
// [0, (n-1) dx]; E_y, E_z on its two faces follow Mur's rule over each half
// step h (G. Mur, IEEE Trans. EMC 23, 377 (1981)), applied at x = 0 to
// E - E_inc of the injected pulse.  With node 0 on the face, node 1 inside,
// k = (h - dx)/(h + dx) and levels m-1, m, m+1 a half step apart:
//   first order (PIC_BC_ABSORB):  E_0^{m+1} = E_1^m + k (E_1^{m+1} - E_0^m)
//   second order (PIC_BC_ABSORB2, Engquist-Majda E_xt - E_tt + (E_yy+E_zz)/2 = 0):
//     E_0^{m+1} = -E_1^{m-1} + k (E_1^{m+1} + E_0^{m-1}) + 2dx/(h+dx) (E_0^m + E_1^m)
//                 + h^2 dx/(2(h+dx)) (D E_0^m + D E_1^m),  D the periodic
//     second difference over y (and z) on the face planes.
// The E kernel saves the face values on entry (level m); the second-order
// rule also keeps the previous call's (level m-1) in the context, and its
// first call after pic_init runs the first-order rule.  E_x, B_y, B_z half a
// cell beyond the far face stay 0.
#include "device_common.h"
#include "pic_internal.h"

namespace pic {

template <typename R>
struct YeeArgs {
    R *E[3];
    R *B[3];
    const R *J[3];
    int n[3];
    R h;          // dt / 2
    R inv_d[3];   // 1/d (0 for z in 2D)
    int absorb;   // absorbing x faces
    R *old;       // [x node 0, 1, n-2, n-1][E_y, E_z][j + n1 k]: face values before the E update
    R *hist;      // the same on entry to the previous E update (second-order rule)
};

// the pulse injected through x = 0 (pic_laser), evaluated in FP64
struct LaserArgs {
    double a0, waist, tau, t0;
    int circular;
    double d[3], yc, zc;
    int dim;
};

// E_y (comp 1) or E_z (comp 2) of the injected pulse at (x, y, z), time t
// (laser units): a0 exp(-r^2/w^2) S((t - t0 - x)/tau) sin(x - t [+ pi/2]),
// S(s) = sin^2(pi s) on [0, 1]
__device__ double incident(const LaserArgs &L, int comp, double x, double y, double z, double t) {
    if (L.a0 == 0.0 || (comp == 2 && !L.circular)) return 0.0;
    const double s = (t - L.t0 - x) / L.tau;
    if (s <= 0.0 || s >= 1.0) return 0.0;
    const double r2 = (y - L.yc) * (y - L.yc) + (L.dim == 3 ? (z - L.zc) * (z - L.zc) : 0.0);
    const double env = sin(3.14159265358979323846 * s);
    return L.a0 * exp(-r2 / (L.waist * L.waist)) * env * env *
           sin(x - t + (comp == 2 ? 1.57079632679489661923 : 0.0));
}

// E += (dt/2)(curl B - J)
template <typename R, int DIM>
__global__ void __launch_bounds__(256) yee_e_kernel(YeeArgs<R> a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n[0]) return;
    const int j = blockIdx.y;
    const int k = DIM == 3 ? (int)blockIdx.z : 0;
    const int64_t sx = 1, sy = a.n[0], sz = (int64_t)a.n[0] * a.n[1];
    const int64_t c = i + sy * j + sz * k;
    const int64_t cim = c + (i == 0 ? (a.n[0] - 1) * sx : -sx);
    const int64_t cjm = c + (j == 0 ? (int64_t)(a.n[1] - 1) * sy : -sy);
    const R *Bx = a.B[0], *By = a.B[1], *Bz = a.B[2];
    const R bx = Bx[c], by = By[c], bz = Bz[c];
    R cx = (bz - Bz[cjm]) * a.inv_d[1];
    R cy = -(bz - Bz[cim]) * a.inv_d[0];
    R cz = (by - By[cim]) * a.inv_d[0] - (bx - Bx[cjm]) * a.inv_d[1];
    if constexpr (DIM == 3) {
        const int64_t ckm = c + (k == 0 ? (int64_t)(a.n[2] - 1) * sz : -sz);
        cx -= (by - By[ckm]) * a.inv_d[2];
        cy += (bx - Bx[ckm]) * a.inv_d[2];
    }
    if (a.absorb) {
        const int n0 = a.n[0];
        const int f = i == 0 ? 0 : i == 1 ? 1 : i == n0 - 2 ? 2 : i == n0 - 1 ? 3 : -1;
        if (f >= 0) {
            const int64_t nyz = (int64_t)a.n[1] * a.n[2], q = j + (int64_t)a.n[1] * k;
            a.old[(2 * f) * nyz + q] = a.E[1][c];
            a.old[(2 * f + 1) * nyz + q] = a.E[2][c];
        }
        a.E[0][c] = i == n0 - 1 ? R(0) : a.E[0][c] + a.h * (cx - a.J[0][c]);
        if (i != 0 && i != n0 - 1) {
            a.E[1][c] += a.h * (cy - a.J[1][c]);
            a.E[2][c] += a.h * (cz - a.J[2][c]);
        }
        return;
    }
    a.E[0][c] += a.h * (cx - a.J[0][c]);
    a.E[1][c] += a.h * (cy - a.J[1][c]);
    a.E[2][c] += a.h * (cz - a.J[2][c]);
}

// Mur's rule on the two x faces after an E half step from time t; one
// thread per (j, k) line.  `second`: the second-order rule (a.hist holds the
// face values of the previous call); the second-order runs then copy this
// call's entry values into a.hist (each thread its own line, while the
// neighbours' lines are read from a.old only).
template <typename R>
__global__ void __launch_bounds__(256) yee_mur_kernel(YeeArgs<R> a, LaserArgs L, double t, double km, int second,
                                                      int keep) {
    const int64_t nyz = (int64_t)a.n[1] * a.n[2];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nyz) return;
    const int n1 = a.n[1], n2 = a.n[2];
    const int j = (int)(q % n1), k = (int)(q / n1);
    const int n0 = a.n[0];
    const int64_t row = (int64_t)n0 * q;
    const double h = (double)a.h, dx = L.d[0];
    // neighbours along y and z on the face planes (periodic)
    const int64_t qyp = (j + 1 == n1 ? 0 : j + 1) + (int64_t)n1 * k, qym = (j == 0 ? n1 - 1 : j - 1) + (int64_t)n1 * k;
    const int64_t qzp = j + (int64_t)n1 * (k + 1 == n2 ? 0 : k + 1), qzm = j + (int64_t)n1 * (k == 0 ? n2 - 1 : k - 1);
    const double iy2 = 1.0 / (L.d[1] * L.d[1]), iz2 = L.dim == 3 ? 1.0 / (L.d[2] * L.d[2]) : 0.0;
    const double c2 = h * h * dx / (2.0 * (h + dx)), c1 = 2.0 * dx / (h + dx);
#pragma unroll
    for (int cmp = 0; cmp < 2; ++cmp) {
        const int comp = 1 + cmp;
        R *E = a.E[comp];
        const double sy = comp == 1 ? 0.5 : 0.0, sz = comp == 2 ? 0.5 : 0.0;
        const double y = (j + sy) * L.d[1];
        const double z = L.dim == 3 ? (k + sz) * L.d[2] : 0.0;
        // positions of the periodic neighbours (the pulse is evaluated where each value sits)
        const double yp = ((j + 1 == n1 ? 0 : j + 1) + sy) * L.d[1], ym = ((j == 0 ? n1 - 1 : j - 1) + sy) * L.d[1];
        const double zp = L.dim == 3 ? ((k + 1 == n2 ? 0 : k + 1) + sz) * L.d[2] : 0.0;
        const double zm = L.dim == 3 ? ((k == 0 ? n2 - 1 : k - 1) + sz) * L.d[2] : 0.0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            // face node f0 and its neighbour f1 (entries of a.old / a.hist); x = 0 carries the pulse
            const int f0 = side == 0 ? 0 : 3, f1 = side == 0 ? 1 : 2;
            const int64_t i0 = side == 0 ? 0 : n0 - 1, i1 = side == 0 ? 1 : n0 - 2;
            const R *o0 = a.old + (2 * f0 + cmp) * nyz, *o1 = a.old + (2 * f1 + cmp) * nyz;
            auto inc = [&](double xx, double yy, double zz, double tt) {
                return side == 0 ? incident(L, comp, xx, yy, zz, tt) : 0.0;
            };
            const double u0 = (double)o0[q] - inc(0.0, y, z, t), u1 = (double)o1[q] - inc(dx, y, z, t);
            const double u1n = (double)E[row + i1] - inc(dx, y, z, t + h);
            double u0n;
            if (!second) {
                u0n = u1 + km * (u1n - u0);
            } else {
                const R *p0 = a.hist + (2 * f0 + cmp) * nyz, *p1 = a.hist + (2 * f1 + cmp) * nyz;
                const double u0m = (double)p0[q] - inc(0.0, y, z, t - h);
                const double u1m = (double)p1[q] - inc(dx, y, z, t - h);
                double lap = 0.0;
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    const R *o = f == 0 ? o0 : o1;
                    const double xx = f == 0 ? 0.0 : dx, uc = f == 0 ? u0 : u1;
                    lap += ((double)o[qyp] - inc(xx, yp, z, t) + (double)o[qym] - inc(xx, ym, z, t) - 2.0 * uc) * iy2;
                    if (L.dim == 3)
                        lap += ((double)o[qzp] - inc(xx, y, zp, t) + (double)o[qzm] - inc(xx, y, zm, t) - 2.0 * uc) *
                               iz2;
                }
                u0n = -u1m + km * (u1n + u0m) + c1 * (u0 + u1) + c2 * lap;
            }
            E[row + i0] = (R)(inc(0.0, y, z, t + h) + u0n);
        }
    }
    if (keep) {
#pragma unroll
        for (int f = 0; f < 8; ++f) a.hist[f * nyz + q] = a.old[f * nyz + q];
    }
}

// B -= (dt/2) curl E
template <typename R, int DIM>
__global__ void __launch_bounds__(256) yee_b_kernel(YeeArgs<R> a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n[0]) return;
    const int j = blockIdx.y;
    const int k = DIM == 3 ? (int)blockIdx.z : 0;
    const int64_t sx = 1, sy = a.n[0], sz = (int64_t)a.n[0] * a.n[1];
    const int64_t c = i + sy * j + sz * k;
    const int64_t cip = c + (i == a.n[0] - 1 ? -(int64_t)(a.n[0] - 1) * sx : sx);
    const int64_t cjp = c + (j == a.n[1] - 1 ? -(int64_t)(a.n[1] - 1) * sy : sy);
    const R *Ex = a.E[0], *Ey = a.E[1], *Ez = a.E[2];
    const R ex = Ex[c], ey = Ey[c], ez = Ez[c];
    R cx = (Ez[cjp] - ez) * a.inv_d[1];
    R cy = -(Ez[cip] - ez) * a.inv_d[0];
    R cz = (Ey[cip] - ey) * a.inv_d[0] - (Ex[cjp] - ex) * a.inv_d[1];
    if constexpr (DIM == 3) {
        const int64_t ckp = c + (k == a.n[2] - 1 ? -(int64_t)(a.n[2] - 1) * sz : sz);
        cx -= (Ey[ckp] - ey) * a.inv_d[2];
        cy += (Ex[ckp] - ex) * a.inv_d[2];
    }
    a.B[0][c] -= a.h * cx;
    if (a.absorb && i == a.n[0] - 1) {  // half a cell beyond the far face
        a.B[1][c] = R(0);
        a.B[2][c] = R(0);
        return;
    }
    a.B[1][c] -= a.h * cy;
    a.B[2][c] -= a.h * cz;
}

// Per-block FP64 sums of E^2 + B^2 in a fixed order (grid of `nblocks`
// blocks, each covering ITEMS consecutive cells).
template <typename R>
struct Planes6 {
    const R *p[6];
};

template <typename R>
__global__ void __launch_bounds__(256) field_energy_kernel(Planes6<R> F, int64_t ncell, int items,
                                                           double *partials) {
    __shared__ double s[256];
    const int64_t start = (int64_t)blockIdx.x * items;
    double acc = 0.0;
    for (int m = threadIdx.x; m < items; m += blockDim.x) {
        const int64_t c = start + m;
        if (c < ncell) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double v = (double)F.p[q][c];
                acc += v * v;
            }
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

template <typename R>
static hipError_t yee_typed(Ctx *c, int half, const pic_fields *f, double *diag, hipStream_t s) {
    const pic_config &cfg = c->cfg;
    YeeArgs<R> a{};
    for (int d = 0; d < 3; ++d) {
        a.E[d] = (R *)f->E[d];
        a.B[d] = (R *)f->B[d];
        a.J[d] = (const R *)f->J[d];
        a.n[d] = (int)cfg.n[d];
        a.inv_d[d] = d < c->dim ? (R)(1.0 / cfg.d[d]) : R(0);
    }
    a.h = (R)(0.5 * cfg.dt);
    a.absorb = absorbing_x(cfg);
    a.old = (R *)c->mur_old;
    a.hist = (R *)c->mur_hist;
    LaserArgs las{};
    las.a0 = c->laser.a0;
    las.waist = c->laser.waist;
    las.tau = c->laser.duration;
    las.t0 = c->laser.t0;
    las.circular = c->laser.circular;
    for (int d = 0; d < 3; ++d) las.d[d] = cfg.d[d];
    las.yc = 0.5 * (double)cfg.n[1] * cfg.d[1];
    las.zc = 0.5 * (double)cfg.n[2] * cfg.d[2];
    las.dim = c->dim;
    const double hh = 0.5 * cfg.dt, km = (hh - cfg.d[0]) / (hh + cfg.d[0]);
    const int64_t nyz = cfg.n[1] * cfg.n[2];
    dim3 block(256), grid((unsigned)((cfg.n[0] + 255) / 256), (unsigned)cfg.n[1],
                          (unsigned)cfg.n[2]);
    // time of E on entry: t_n for the first half, t_n + dt/2 for the second
    const double t_e = c->time + (half == 1 ? 0.0 : hh);
    auto e_step = [&]() {
        if (c->dim == 3) yee_e_kernel<R, 3><<<grid, block, 0, s>>>(a);
        else yee_e_kernel<R, 2><<<grid, block, 0, s>>>(a);
        if (a.absorb) {
            const int keep = cfg.bc[0] == PIC_BC_ABSORB2;
            yee_mur_kernel<R><<<(unsigned)((nyz + 255) / 256), 256, 0, s>>>(a, las, t_e, km,
                                                                              keep && c->mur_valid, keep);
            c->mur_valid = keep;
        }
    };
    auto b_step = [&]() {
        if (c->dim == 3) yee_b_kernel<R, 3><<<grid, block, 0, s>>>(a);
        else yee_b_kernel<R, 2><<<grid, block, 0, s>>>(a);
    };
    if (half == 1) {
        e_step();
        b_step();
    } else {
        b_step();
        e_step();
        c->time += cfg.dt;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !diag || half != 2) return e;

    const int64_t ncell = cfg.n[0] * cfg.n[1] * cfg.n[2];
    const int items = 256 * 16;
    const int64_t nblocks = (ncell + items - 1) / items;
    if (ensure_partials(c, (size_t)nblocks) != PIC_OK) return hipErrorOutOfMemory;
    Planes6<R> planes{{a.E[0], a.E[1], a.E[2], a.B[0], a.B[1], a.B[2]}};
    field_energy_kernel<R><<<(unsigned)nblocks, 256, 0, s>>>(planes, ncell, items, c->partials);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // diag[2] += dV/2 * (fixed-order total)
    const double dV = cfg.d[0] * cfg.d[1] * (c->dim == 3 ? cfg.d[2] : 1.0);
    return launch_finalize(c->partials, nblocks, 1, diag, 2, 0.5 * dV, s);
}

hipError_t launch_yee(Ctx *c, int half, const pic_fields *f, double *diag, hipStream_t s) {
    if (c->cfg.precision == PIC_FP64_PLAIN) return yee_typed<double>(c, half, f, diag, s);
    return yee_typed<float>(c, half, f, diag, s);
}

}  // namespace pic
