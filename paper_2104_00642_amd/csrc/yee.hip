// yee.hip -- half-step Yee FDTD update (Sec. II.B Eqs. 9-10, split in halves as
// in Sec. II.F) and the FP64 field-energy reduction.
//
// Bandwidth-bound stencil: one thread per cell, x-fastest so that every
// wavefront reads and writes contiguous 256-byte rows; the -1/+1 neighbours
// along y/z come from rows the neighbouring wavefronts already pulled into L2.
// Periodic in every axis.
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
};

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
    a.E[0][c] += a.h * (cx - a.J[0][c]);
    a.E[1][c] += a.h * (cy - a.J[1][c]);
    a.E[2][c] += a.h * (cz - a.J[2][c]);
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
    dim3 block(256), grid((unsigned)((cfg.n[0] + 255) / 256), (unsigned)cfg.n[1],
                          (unsigned)cfg.n[2]);
    auto e_step = [&]() {
        if (c->dim == 3) yee_e_kernel<R, 3><<<grid, block, 0, s>>>(a);
        else yee_e_kernel<R, 2><<<grid, block, 0, s>>>(a);
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
