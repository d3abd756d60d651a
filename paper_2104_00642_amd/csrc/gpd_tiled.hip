// gpd_tiled.hip -- mixed-precision gather + Boris push + Esirkepov deposit on
// tile-binned particles (the FP32 hot path).
//
// One workgroup per grid tile.  The workgroup
//   1. stages the E/B window of its tile (tile + reach + drift guard cells, all
//      six components, periodic wrap) from HBM into LDS,
//   2. pushes the tile's particles (contiguous after pic_sort, with
//      consecutive particles in distinct cells so that the LDS traffic of a
//      wavefront spreads over distinct addresses): gather from LDS (Eq. 19),
//      Boris (Eqs. 13-16), move (Eq. 12), Esirkepov current (Eqs. 20-22)
//      accumulated in an int64 fixed-point J window with LDS integer atomics,
//   3. adds its J window to global J with one pass of coalesced global float
//      atomics (neighbouring windows overlap in their guard cells).
// The current window is integer because LDS float atomics (ds_add_f32) run an
// order of magnitude slower than integer ones on gfx950.  Every contribution
// is an FP32 value bounded by B = |q| w_max max(1, d/dt) (the running sums of
// the Esirkepov weights stay within [-1, 1]); scaled by the power of two
// S = 2^30 / B it converts exactly to an int32, and the int64 sums are exact
// and independent of the order of the atomics.  The flush divides by S.
// Particles are an int32 packed cell plus FP32 in-cell offsets, so every
// weight is computed from a number in (-1.5, 2.5) and keeps full FP32
// resolution regardless of the grid size.  A particle that has wandered more
// than `drift` cells out of its tile since the last sort takes the same code
// path with global-memory accessors and is counted as a straggler.
// Blocks are remapped so that each XCD (own L2) works on a contiguous run of
// tiles: neighbouring tiles share guard rows in the same L2.
#include "device_common.h"
#include "pic_internal.h"

namespace pic {

extern __shared__ float pic_smem[];

struct TiledArgs {
    int32_t *cell;
    float *off[3];
    float *u[3];
    const float *w;
    float w0;
    float *chi;
    float chi_scale;
    const int64_t *tile_start;
    int ntiles;
    int chunk;          // tiles per XCD run
    const float *F[6];
    float *J[3];
    int ng[3];
    int bx, by;         // packed-cell field widths
    int tile[3];
    int ntile_axis[3];
    int drift;
    int win[3];
    float hdt_d[3];     // dt / (2 d)
    float dt_d[3];      // dt / d
    float qm_h;         // q/m dt/2
    float jfac[3];      // q d / dt
    float q;
    float jmax;         // max(1, d/dt) over the axes
    double mdV, qdV;
    double *partials;
    uint32_t *status;
    unsigned long long *stragglers;
};

// Accessor of the LDS window: coordinates local to the window origin.  Fields
// are the first 6*wn floats of the dynamic LDS, the fixed-point current the
// following 3*wn int64 words.
struct LdsAcc {
    int wx, wxy, wn;
    float scale;  // S of the fixed-point current
    __device__ __forceinline__ int idx(int i, int j, int k) const { return i + wx * j + wxy * k; }
    __device__ __forceinline__ float f(int c, int i, int j, int k) const {
        return pic_smem[c * wn + idx(i, j, k)];
    }
    // v is already in fixed-point units (the prefactors carry S), |v| <= 2^30
    __device__ __forceinline__ void add(int c, int i, int j, int k, float v) const {
        unsigned long long *jw = (unsigned long long *)(pic_smem + 6 * wn);
        atomicAdd(&jw[c * wn + idx(i, j, k)], (unsigned long long)(long long)(int)v);
    }
};

// Accessor of global memory: absolute cell coordinates, periodic wrap.
struct GlobAcc {
    const float *F[6];
    float *J[3];
    int ng[3];
    float scale;  // 1: values arrive in physical units
    __device__ __forceinline__ int64_t idx(int i, int j, int k) const {
        i = wrap_index(i, ng[0]);
        j = wrap_index(j, ng[1]);
        k = wrap_index(k, ng[2]);
        return (int64_t)i + (int64_t)ng[0] * ((int64_t)j + (int64_t)ng[1] * k);
    }
    __device__ __forceinline__ float f(int c, int i, int j, int k) const { return F[c][idx(i, j, k)]; }
    __device__ __forceinline__ void add(int c, int i, int j, int k, float v) const {
        atomicAdd(&J[c][idx(i, j, k)], v);
    }
};

// Push one particle whose cell origin is at o[] in the accessor's coordinates.
// f[] in-cell offsets, u[] momentum (updated); returns the cell displacement
// in dc[] and the new offsets in f[]; EB[] receives the gathered fields.
template <int DIM, int ORDER, class Acc>
__device__ __forceinline__ void push_one(const Acc &acc, const TiledArgs &a, const int *o, float *f,
                                         float *u, float w, int *dc, float *EB) {
    constexpr int NW = ORDER + 1;
    constexpr int L = ORDER + 2;
    const float ig0 = rsqrt_r(1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    float dh[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) dh[d] = f[d] + a.hdt_d[d] * u[d] * ig0;

    // gather (Eq. 19) with integer-node and half-node weights per axis
    int i0[2][3] = {{0, 0, 0}, {0, 0, 0}};
    float wt[2][3][NW];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        shape_weights<ORDER>(dh[d], i0[0][d], wt[0][d]);
        shape_weights<ORDER>(dh[d] - 0.5f, i0[1][d], wt[1][d]);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int sx = stag(c, 0), sy = stag(c, 1), sz = DIM == 3 ? stag(c, 2) : 0;
        float acc_v = 0.0f;
        if constexpr (DIM == 2) {
#pragma unroll
            for (int jj = 0; jj < NW; ++jj) {
                float r = 0.0f;
#pragma unroll
                for (int ii = 0; ii < NW; ++ii)
                    r += wt[sx][0][ii] * acc.f(c, o[0] + i0[sx][0] + ii, o[1] + i0[sy][1] + jj, 0);
                acc_v += wt[sy][1][jj] * r;
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < NW; ++kk) {
                float s = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NW; ++jj) {
                    float r = 0.0f;
#pragma unroll
                    for (int ii = 0; ii < NW; ++ii)
                        r += wt[sx][0][ii] * acc.f(c, o[0] + i0[sx][0] + ii, o[1] + i0[sy][1] + jj,
                                                   o[2] + i0[sz][2] + kk);
                    s += wt[sy][1][jj] * r;
                }
                acc_v += wt[sz][2][kk] * s;
            }
        }
        EB[c] = acc_v;
    }

    boris<float>(a.qm_h, EB, EB + 3, u);
    const float ig1 = rsqrt_r(1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const float v[3] = {u[0] * ig1, u[1] * ig1, u[2] * ig1};

    // Esirkepov (Eqs. 20-22) for the move dh -> dh + dt v / d
    int base[3] = {0, 0, 0};
    float S0[3][L], DS[3][L];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
        esirkepov_axis_from<ORDER>(i0[0][d], wt[0][d], dh[d] + a.dt_d[d] * v[d], base[d], S0[d], DS[d]);
    const int b0 = o[0] + base[0], b1 = o[1] + base[1];
    const float ws = w * acc.scale;  // fixed-point units in the LDS window
    const float jx = a.jfac[0] * ws, jy = a.jfac[1] * ws;
    if constexpr (DIM == 2) {
#pragma unroll
        for (int jj = 0; jj < L; ++jj) {
            const float ty = jx * (S0[1][jj] + 0.5f * DS[1][jj]);
            float run = 0.0f;
#pragma unroll
            for (int ii = 0; ii < L - 1; ++ii) {
                run -= DS[0][ii] * ty;
                acc.add(0, b0 + ii, b1 + jj, 0, run);
            }
        }
#pragma unroll
        for (int ii = 0; ii < L; ++ii) {
            const float tx = jy * (S0[0][ii] + 0.5f * DS[0][ii]);
            float run = 0.0f;
#pragma unroll
            for (int jj = 0; jj < L - 1; ++jj) {
                run -= DS[1][jj] * tx;
                acc.add(1, b0 + ii, b1 + jj, 0, run);
            }
        }
        const float qv = a.q * ws * v[2];
#pragma unroll
        for (int jj = 0; jj < L; ++jj) {
            const float a0 = qv * (S0[1][jj] + 0.5f * DS[1][jj]);
            const float a1 = qv * (0.5f * S0[1][jj] + (1.0f / 3.0f) * DS[1][jj]);
#pragma unroll
            for (int ii = 0; ii < L; ++ii) acc.add(2, b0 + ii, b1 + jj, 0, S0[0][ii] * a0 + DS[0][ii] * a1);
        }
    } else {
        const int b2 = o[2] + base[2];
        const float jz = a.jfac[2] * ws;
        // W_x = DS_x (S0y S0z + DSy S0z/2 + S0y DSz/2 + DSy DSz/3), etc.
#pragma unroll
        for (int kk = 0; kk < L; ++kk)
#pragma unroll
            for (int jj = 0; jj < L; ++jj) {
                const float t = jx * (S0[1][jj] * (S0[2][kk] + 0.5f * DS[2][kk]) +
                                      DS[1][jj] * (0.5f * S0[2][kk] + (1.0f / 3.0f) * DS[2][kk]));
                float run = 0.0f;
#pragma unroll
                for (int ii = 0; ii < L - 1; ++ii) {
                    run -= DS[0][ii] * t;
                    acc.add(0, b0 + ii, b1 + jj, b2 + kk, run);
                }
            }
#pragma unroll
        for (int kk = 0; kk < L; ++kk)
#pragma unroll
            for (int ii = 0; ii < L; ++ii) {
                const float t = jy * (S0[0][ii] * (S0[2][kk] + 0.5f * DS[2][kk]) +
                                      DS[0][ii] * (0.5f * S0[2][kk] + (1.0f / 3.0f) * DS[2][kk]));
                float run = 0.0f;
#pragma unroll
                for (int jj = 0; jj < L - 1; ++jj) {
                    run -= DS[1][jj] * t;
                    acc.add(1, b0 + ii, b1 + jj, b2 + kk, run);
                }
            }
#pragma unroll
        for (int jj = 0; jj < L; ++jj)
#pragma unroll
            for (int ii = 0; ii < L; ++ii) {
                const float t = jz * (S0[0][ii] * (S0[1][jj] + 0.5f * DS[1][jj]) +
                                      DS[0][ii] * (0.5f * S0[1][jj] + (1.0f / 3.0f) * DS[1][jj]));
                float run = 0.0f;
#pragma unroll
                for (int kk = 0; kk < L - 1; ++kk) {
                    run -= DS[2][kk] * t;
                    acc.add(2, b0 + ii, b1 + jj, b2 + kk, run);
                }
            }
    }

    // full-step position: offset relative to the old cell, then re-index
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const float dn = dh[d] + a.hdt_d[d] * v[d];
        const float fl = floorf(dn);
        float fr = dn - fl;
        int di = (int)fl;
        if (fr >= 1.0f) {  // dn just below an integer rounded the offset up to 1
            fr = 0.0f;
            di += 1;
        }
        f[d] = fr;
        dc[d] = di;
    }
}

template <int DIM, int ORDER>
__global__ void __launch_bounds__(256) gpd_tiled_kernel(TiledArgs a) {
    const int b = blockIdx.x;
    const int t = (b & 7) * a.chunk + (b >> 3);  // XCD-contiguous tile runs
    if (t >= a.ntiles) return;
    const int64_t pbeg = a.tile_start[t], pend = a.tile_start[t + 1];
    __shared__ double red_k[256], red_q[256];
    __shared__ unsigned int nstray;
    __shared__ float wmax_s[256];
    if (pbeg >= pend) {
        if (threadIdx.x == 0) {
            a.partials[2 * t] = 0.0;
            a.partials[2 * t + 1] = 0.0;
        }
        return;
    }
    const int tx = t % a.ntile_axis[0];
    const int ty = (t / a.ntile_axis[0]) % a.ntile_axis[1];
    const int tz = DIM == 3 ? t / (a.ntile_axis[0] * a.ntile_axis[1]) : 0;
    const int g = a.drift + 2;
    int org[3] = {tx * a.tile[0] - g, ty * a.tile[1] - g, DIM == 3 ? tz * a.tile[2] - g : 0};
    LdsAcc lds{a.win[0], a.win[0] * a.win[1], a.win[0] * a.win[1] * a.win[2], 0.0f};
    const int wn = lds.wn;
    unsigned long long *jwin = (unsigned long long *)(pic_smem + 6 * wn);

    // 1. stage E/B window, zero the J window, bound the weights of the tile
    for (int e = threadIdx.x; e < 6 * wn; e += blockDim.x) {
        const int c = e / wn;
        const int r = e - c * wn;
        const int k = r / lds.wxy;
        const int r2 = r - k * lds.wxy;
        const int j = r2 / a.win[0];
        const int i = r2 - j * a.win[0];
        const int gi = wrap_index(org[0] + i, a.ng[0]);
        const int gj = wrap_index(org[1] + j, a.ng[1]);
        const int gk = DIM == 3 ? wrap_index(org[2] + k, a.ng[2]) : 0;
        pic_smem[e] = a.F[c][(int64_t)gi + (int64_t)a.ng[0] * ((int64_t)gj + (int64_t)a.ng[1] * gk)];
    }
    for (int e = threadIdx.x; e < 3 * wn; e += blockDim.x) jwin[e] = 0ull;
    float wm = fabsf(a.w0);
    if (a.w) {
        wm = 0.0f;
        for (int64_t p = pbeg + threadIdx.x; p < pend; p += blockDim.x) wm = fmaxf(wm, fabsf(a.w[p]));
    }
    wmax_s[threadIdx.x] = wm;
    if (threadIdx.x == 0) nstray = 0;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) wmax_s[threadIdx.x] = fmaxf(wmax_s[threadIdx.x], wmax_s[threadIdx.x + h]);
        __syncthreads();
    }
    {
        // S = 2^(30 - ceil(log2 B)), B = |q| w_max max(1, d/dt): |contribution| * S <= 2^30
        const float B = fabsf(a.q) * wmax_s[0] * a.jmax;
        int ex = 0;
        frexpf(B > 0.0f ? B : 1.0f, &ex);  // B < 2^ex
        lds.scale = ldexpf(1.0f, 30 - ex);
    }

    // 2. particles of the tile, next particle prefetched while one is pushed
    const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
    const int hi[3] = {a.win[0] - 4, a.win[1] - 4, a.win[2] - 4};
    double kin = 0.0, chg = 0.0;
    GlobAcc glob{{a.F[0], a.F[1], a.F[2], a.F[3], a.F[4], a.F[5]},
                 {a.J[0], a.J[1], a.J[2]},
                 {a.ng[0], a.ng[1], a.ng[2]}, 1.0f};
    int64_t p = pbeg + threadIdx.x;
    int32_t n_cell = 0;
    float n_f[3] = {0.0f, 0.0f, 0.0f}, n_u[3] = {0.0f, 0.0f, 0.0f}, n_w = a.w0;
    if (p < pend) {
        n_cell = a.cell[p];
#pragma unroll
        for (int d = 0; d < DIM; ++d) n_f[d] = a.off[d][p];
#pragma unroll
        for (int d = 0; d < 3; ++d) n_u[d] = a.u[d][p];
        if (a.w) n_w = a.w[p];
    }
    for (; p < pend; p += blockDim.x) {
        const int32_t cell = n_cell;
        float f[3] = {n_f[0], n_f[1], n_f[2]};
        float u[3] = {n_u[0], n_u[1], n_u[2]};
        const float w = n_w;
        const int64_t pn = p + blockDim.x;
        if (pn < pend) {
            n_cell = a.cell[pn];
#pragma unroll
            for (int d = 0; d < DIM; ++d) n_f[d] = a.off[d][pn];
#pragma unroll
            for (int d = 0; d < 3; ++d) n_u[d] = a.u[d][pn];
            if (a.w) n_w = a.w[pn];
        }
        int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        bool bad = false;
#pragma unroll
        for (int d = 0; d < DIM; ++d) bad |= !(f[d] >= 0.0f && f[d] < 1.0f) || cc[d] >= a.ng[d];
        if (bad) atomicOr(a.status, PIC_F_OFFSET);
        if (!isfinite(u[0] + u[1] + u[2])) atomicOr(a.status, PIC_F_NONFINITE);
        // local cell in the window (one periodic unwrap)
        int lc[3];
        bool inside = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int l = cc[d] - org[d];
            l = l < 0 ? l + a.ng[d] : (l >= a.ng[d] ? l - a.ng[d] : l);
            lc[d] = l;
            inside &= (l >= 2) && (l <= hi[d]);
        }
        if (DIM == 2) lc[2] = 0;
        const float u_old[3] = {u[0], u[1], u[2]};
        float EB[6];
        int dc[3] = {0, 0, 0};
        if (inside) {
            push_one<DIM, ORDER>(lds, a, lc, f, u, w, dc, EB);
        } else {
            push_one<DIM, ORDER>(glob, a, cc, f, u, w, dc, EB);
            atomicAdd(&nstray, 1u);
        }
        int packed = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int nc = cc[d] + dc[d];
            nc = nc < 0 ? nc + a.ng[d] : (nc >= a.ng[d] ? nc - a.ng[d] : nc);
            packed |= nc << (d == 0 ? 0 : (d == 1 ? a.bx : a.bx + a.by));
        }
        a.cell[p] = packed;
#pragma unroll
        for (int d = 0; d < DIM; ++d) a.off[d][p] = f[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) a.u[d][p] = u[d];
        const float g1 = sqrtf(1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (a.chi) {
            // chi_e (Sec. IV) at the fields of x_h and u^{n+1/2}
            const float uh0 = 0.5f * (u_old[0] + u[0]), uh1 = 0.5f * (u_old[1] + u[1]),
                        uh2 = 0.5f * (u_old[2] + u[2]);
            const float gh = sqrtf(1.0f + uh0 * uh0 + uh1 * uh1 + uh2 * uh2);
            const float f0 = gh * EB[0] + uh1 * EB[5] - uh2 * EB[4];
            const float f1 = gh * EB[1] + uh2 * EB[3] - uh0 * EB[5];
            const float f2 = gh * EB[2] + uh0 * EB[4] - uh1 * EB[3];
            const float ue = uh0 * EB[0] + uh1 * EB[1] + uh2 * EB[2];
            const float s2 = f0 * f0 + f1 * f1 + f2 * f2 - ue * ue;
            a.chi[p] = a.chi_scale * sqrtf(fmaxf(s2, 0.0f));
        }
        kin += (double)w * (double)(g1 - 1.0f);
        chg += (double)w;
    }
    __syncthreads();

    // 3. flush the J window into global J (periodic wrap), skip exact zeros
    const double inv_scale = 1.0 / (double)lds.scale;
    for (int e = threadIdx.x; e < 3 * wn; e += blockDim.x) {
        const long long q = (long long)jwin[e];
        if (q != 0) {
            const float v = (float)((double)q * inv_scale);
            const int c = e / wn;
            const int r = e - c * wn;
            const int k = r / lds.wxy;
            const int r2 = r - k * lds.wxy;
            const int j = r2 / a.win[0];
            const int i = r2 - j * a.win[0];
            const int gi = wrap_index(org[0] + i, a.ng[0]);
            const int gj = wrap_index(org[1] + j, a.ng[1]);
            const int gk = DIM == 3 ? wrap_index(org[2] + k, a.ng[2]) : 0;
            atomicAdd(&a.J[c][(int64_t)gi + (int64_t)a.ng[0] * ((int64_t)gj + (int64_t)a.ng[1] * gk)], v);
        }
    }
    // 4. fixed-order FP64 reduction of the diagnostics
    red_k[threadIdx.x] = kin;
    red_q[threadIdx.x] = chg;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red_k[threadIdx.x] += red_k[threadIdx.x + h];
            red_q[threadIdx.x] += red_q[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partials[2 * t] = red_k[0] * a.mdV;
        a.partials[2 * t + 1] = red_q[0] * a.qdV;
        if (nstray) {
            atomicOr(a.status, PIC_F_STRAGGLER);
            atomicAdd(a.stragglers, (unsigned long long)nstray);
        }
    }
}

// Particles after the last tile (created since the last sort, e.g. by the QED
// step) take the global-memory path; a fixed grid strides over them.
constexpr int TAIL_BLOCKS = 256;

template <int DIM, int ORDER>
__global__ void __launch_bounds__(256) gpd_tail_kernel(TiledArgs a, int64_t n) {
    const int64_t first = a.tile_start[a.ntiles];
    __shared__ double red_k[256], red_q[256];
    double kin = 0.0, chg = 0.0;
    GlobAcc glob{{a.F[0], a.F[1], a.F[2], a.F[3], a.F[4], a.F[5]},
                 {a.J[0], a.J[1], a.J[2]},
                 {a.ng[0], a.ng[1], a.ng[2]}, 1.0f};
    const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
    for (int64_t p = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t cell = a.cell[p];
        int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        float f[3] = {a.off[0][p], a.off[1][p], DIM == 3 ? a.off[2][p] : 0.0f};
        float u[3] = {a.u[0][p], a.u[1][p], a.u[2][p]};
        const float w = a.w ? a.w[p] : a.w0;
        const float u_old[3] = {u[0], u[1], u[2]};
        float EB[6];
        int dc[3] = {0, 0, 0};
        push_one<DIM, ORDER>(glob, a, cc, f, u, w, dc, EB);
        int packed = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int nc = cc[d] + dc[d];
            nc = nc < 0 ? nc + a.ng[d] : (nc >= a.ng[d] ? nc - a.ng[d] : nc);
            packed |= nc << (d == 0 ? 0 : (d == 1 ? a.bx : a.bx + a.by));
            a.off[d][p] = f[d];
        }
        a.cell[p] = packed;
#pragma unroll
        for (int d = 0; d < 3; ++d) a.u[d][p] = u[d];
        if (a.chi) {
            const float uh0 = 0.5f * (u_old[0] + u[0]), uh1 = 0.5f * (u_old[1] + u[1]),
                        uh2 = 0.5f * (u_old[2] + u[2]);
            const float gh = sqrtf(1.0f + uh0 * uh0 + uh1 * uh1 + uh2 * uh2);
            const float f0 = gh * EB[0] + uh1 * EB[5] - uh2 * EB[4];
            const float f1 = gh * EB[1] + uh2 * EB[3] - uh0 * EB[5];
            const float f2 = gh * EB[2] + uh0 * EB[4] - uh1 * EB[3];
            const float ue = uh0 * EB[0] + uh1 * EB[1] + uh2 * EB[2];
            a.chi[p] = a.chi_scale * sqrtf(fmaxf(f0 * f0 + f1 * f1 + f2 * f2 - ue * ue, 0.0f));
        }
        const float g1 = sqrtf(1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        kin += (double)w * (double)(g1 - 1.0f);
        chg += (double)w;
    }
    red_k[threadIdx.x] = kin;
    red_q[threadIdx.x] = chg;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red_k[threadIdx.x] += red_k[threadIdx.x + h];
            red_q[threadIdx.x] += red_q[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partials[2 * (a.ntiles + blockIdx.x)] = red_k[0] * a.mdV;
        a.partials[2 * (a.ntiles + blockIdx.x) + 1] = red_q[0] * a.qdV;
    }
}

hipError_t launch_gpd_tiled(Ctx *c, const pic_species *sp, const pic_particles *p,
                            const pic_fields *f, double *diag, hipStream_t s) {
    const pic_config &cfg = c->cfg;
    TiledArgs a{};
    a.cell = p->cell;
    for (int d = 0; d < 3; ++d) {
        a.off[d] = p->off[d];
        a.u[d] = (float *)p->u[d];
        a.F[d] = (const float *)f->E[d];
        a.F[3 + d] = (const float *)f->B[d];
        a.J[d] = (float *)f->J[d];
        a.ng[d] = (int)cfg.n[d];
        a.tile[d] = c->tile[d];
        a.ntile_axis[d] = c->ntile_axis[d];
        a.win[d] = c->win[d];
        a.hdt_d[d] = (float)(0.5 * cfg.dt / cfg.d[d]);
        a.dt_d[d] = (float)(cfg.dt / cfg.d[d]);
        a.jfac[d] = (float)(sp->q * cfg.d[d] / cfg.dt);
    }
    a.w = (const float *)p->w;
    a.w0 = (float)sp->w0;
    a.chi = cfg.hbar_omega_mc2 > 0.0 ? p->chi : nullptr;
    a.chi_scale = (float)cfg.hbar_omega_mc2;
    a.tile_start = p->tile_start;
    a.ntiles = (int)c->ntiles;
    a.chunk = (int)((c->ntiles + 7) / 8);
    a.bx = c->bits[0];
    a.by = c->bits[1];
    a.drift = c->drift;
    a.qm_h = (float)(0.5 * sp->q / sp->m * cfg.dt);
    a.q = (float)sp->q;
    double jm = 1.0;
    for (int d = 0; d < c->dim; ++d) jm = fmax(jm, cfg.d[d] / cfg.dt);
    a.jmax = (float)jm;
    const double dV = cfg.d[0] * cfg.d[1] * (c->dim == 3 ? cfg.d[2] : 1.0);
    a.mdV = sp->m * dV;
    a.qdV = sp->q * dV;
    a.status = c->status;
    a.stragglers = (unsigned long long *)(c->status + 2);
    if (ensure_partials(c, 2 * ((size_t)c->ntiles + TAIL_BLOCKS)) != PIC_OK) return hipErrorOutOfMemory;
    a.partials = c->partials;
    dim3 grid((unsigned)(8 * a.chunk)), block(256), tgrid(TAIL_BLOCKS);
    const size_t lds = c->lds_bytes;
    const int key = c->dim * 10 + cfg.order;
    const int64_t n = p->n;
    switch (key) {
        case 21:
            gpd_tiled_kernel<2, 1><<<grid, block, lds, s>>>(a);
            gpd_tail_kernel<2, 1><<<tgrid, block, 0, s>>>(a, n);
            break;
        case 22:
            gpd_tiled_kernel<2, 2><<<grid, block, lds, s>>>(a);
            gpd_tail_kernel<2, 2><<<tgrid, block, 0, s>>>(a, n);
            break;
        case 31:
            gpd_tiled_kernel<3, 1><<<grid, block, lds, s>>>(a);
            gpd_tail_kernel<3, 1><<<tgrid, block, 0, s>>>(a, n);
            break;
        case 32:
            gpd_tiled_kernel<3, 2><<<grid, block, lds, s>>>(a);
            gpd_tail_kernel<3, 2><<<tgrid, block, 0, s>>>(a, n);
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !diag) return e;
    return launch_finalize(c->partials, c->ntiles + TAIL_BLOCKS, 2, diag, 0, 1.0, s);
}

hipError_t set_tiled_lds_limit(size_t bytes) {
    hipError_t e;
    e = hipFuncSetAttribute((const void *)gpd_tiled_kernel<2, 1>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gpd_tiled_kernel<2, 2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gpd_tiled_kernel<3, 1>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)gpd_tiled_kernel<3, 2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace pic
