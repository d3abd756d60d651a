// gpd_tiled.hip -- mixed-precision gather + Boris push + Esirkepov deposit on
// tile-binned particles (the FP32 hot path).
//
// One workgroup per grid tile.  The workgroup
//   1. stages the E/B window of its tile (tile + reach + drift guard cells, all
//      six components, periodic wrap) from HBM into LDS; the reach is
//      [c-2, c+3] around a particle's cell c for CIC and quadratic weights,
//      [c-3, c+4] for quartic ones,
//   2. pushes the tile's particles (contiguous after pic_sort, with
//      consecutive particles in distinct cells so that the LDS traffic of a
//      wavefront spreads over distinct addresses): gather from LDS (Eq. 19),
//      Boris (Eqs. 13-16) or Vay, move (Eq. 12), Esirkepov current (Eqs. 20-22)
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
// resolution regardless of the grid size.
// A particle that has wandered more than `drift` cells out of its tile since
// the last sort (or whose offset is not in [0,1)) is not pushed here: its
// index goes to a list that gpd_global_kernel works through afterwards with
// global-memory accessors, together with particles appended after the last
// tile.  The tile kernel therefore holds only the LDS path.
// Blocks are remapped so that each XCD (own L2) works on a contiguous run of
// tiles: neighbouring tiles share guard rows in the same L2.
#include <type_traits>

#include "device_common.h"
#include "pic_internal.h"

namespace pic {

extern __shared__ float pic_smem[];

#ifndef PIC_TILED_THREADS_2D
#define PIC_TILED_THREADS_2D 256
#endif
#ifndef PIC_TILED_THREADS_3D
#define PIC_TILED_THREADS_3D 1024
#endif

struct TiledArgs {
    int32_t *cell;
    float *off[3];
    float *u[3];
    float *w;           // written only to absorb particles at absorbing x faces
    float w0;
    float *chi;
    float chi_scale;
    const int64_t *tile_start;
    int64_t n;
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
    // sorted pass: the stragglers of tile t are strag_list[tile_start[t] ..
    // + strag_tile[t]); binned pass: strag_list[0 .. strag_count)
    int32_t *strag_list;   // capacity n
    uint32_t *strag_tile;  // ntiles
    uint32_t *strag_count;
    // binned second pass: particles of tile t are bin_list[bin_start[t] ..
    // bin_start[t+1]); bin_count/bin_rank build it
    int32_t *bin_list;
    int64_t *bin_start;    // ntiles + 1
    uint32_t *bin_wmax;    // ntiles: max |q| w over each tile's bin, as float bits (binning)
    uint32_t *bin_count;   // ntiles
    uint32_t *bin_rank;    // per entry of the straggler list and tail (capacity n)
    int part_off;          // first partial slot (doubles) of the launch
    int absorb_x;          // absorbing x faces: nothing is gathered from or deposited
                           // beyond x nodes [0, n), and a particle whose new position
                           // leaves [0, (n-1) dx] gets weight 0
};

// Accessor of the LDS window: coordinates local to the window origin.  Fields
// are the first 6*wn floats of the dynamic LDS, the fixed-point current the
// following 3*wn int64 words.  WX, WY, WZ > 0 fix the window shape at compile
// time (the default tiles), so that every stencil node of a particle is an
// immediate offset from one base address; 0 takes the shape at run time.
// PAIR (2D): E_x and B_y share the stagger (1/2, 0), E_y and B_x (0, 1/2), so
// each pair is interleaved node by node (one 8-byte LDS read serves both, and
// a stencil's nodes lie within the reach of the paired-read offsets); E_z and
// B_z keep planes of their own.  Otherwise one plane per component.
template <int WX, int WY, int WZ, bool PAIR>
struct LdsAcc {
    int wx_, wxy_, wn_;
    float scale;  // S of the fixed-point current
    __device__ __forceinline__ int wx() const { return WX > 0 ? WX : wx_; }
    __device__ __forceinline__ int wxy() const { return WX > 0 ? WX * WY : wxy_; }
    __device__ __forceinline__ int wn() const { return WX > 0 ? WX * WY * WZ : wn_; }
    // linear index of a stencil base (window coordinates are small, so the
    // 24-bit multiplies run at full rate); a node is then base + ii + jj wx +
    // kk wxy, a compile-time offset when the shape is fixed
    __device__ __forceinline__ int lin(int i, int j, int k) const {
        return i + __mul24(wx(), j) + __mul24(wxy(), k);
    }
    // float index of component c at window node r
    __device__ __forceinline__ int slot(int c, int r) const {
        if constexpr (PAIR) {
            // c: 0 E_x, 1 E_y, 2 E_z, 3 B_x, 4 B_y, 5 B_z
            const int plane = c == 0 || c == 4 ? 0 : (c == 1 || c == 3 ? 2 * wn() : (c == 2 ? 4 * wn() : 5 * wn()));
            const int lane = c == 4 || c == 3 ? 1 : 0;
            const int step = c == 2 || c == 5 ? 1 : 2;
            return plane + step * r + lane;
        } else {
            return c * wn() + r;
        }
    }
    __device__ __forceinline__ float f(int c, int bi, int bj, int bk, int ii, int jj, int kk) const {
        return pic_smem[slot(c, lin(bi, bj, bk) + ii + wx() * jj + wxy() * kk)];
    }
    // (PAIR) views of the window from a stencil base (bi, bj): the base
    // address is formed once per particle and plane, and the nodes (ii, jj)
    // are immediate offsets of paired reads from it.  The empty asm takes the
    // formed address as an opaque register value, so the compiler cannot fold
    // the plane offset (too large for a paired read's immediate) back into
    // every node's address.
    typedef float vec2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const vec2 lds_float2;
    typedef __attribute__((address_space(3))) const float lds_float;
    // pair p (0: E_x, B_y; 1: E_y, B_x): both components of a node in one
    // 8-byte read
    struct PairView {
        const lds_float2 *p0;
        int wx;
        __device__ __forceinline__ float2 operator()(int ii, int jj) const {
            const vec2 v = p0[ii + wx * jj];
            return make_float2(v.x, v.y);
        }
    };
    __device__ __forceinline__ PairView pair_view(int p, int bi, int bj) const {
        const lds_float2 *q = (const lds_float2 *)(const vec2 *)pic_smem + p * wn() + lin(bi, bj, 0);
        uint32_t addr = (uint32_t)(uintptr_t)q;
        asm volatile("" : "+v"(addr));
        return PairView{(const lds_float2 *)(uintptr_t)addr, wx()};
    }
    // the E_z (c = 2) or B_z (c = 5) plane
    struct PlaneView {
        const lds_float *p0;
        int wx;
        __device__ __forceinline__ float operator()(int ii, int jj) const { return p0[ii + wx * jj]; }
    };
    __device__ __forceinline__ PlaneView plane_view(int c, int bi, int bj) const {
        const lds_float *q = (const lds_float *)(const float *)pic_smem + slot(c, lin(bi, bj, 0));
        uint32_t addr = (uint32_t)(uintptr_t)q;
        asm volatile("" : "+v"(addr));
        return PlaneView{(const lds_float *)(uintptr_t)addr, wx()};
    }
    // v is already in fixed-point units (the prefactors carry S), |v| <= 2^30
    __device__ __forceinline__ void add(int c, int bi, int bj, int bk, int ii, int jj, int kk, float v) const {
        unsigned long long *jw = (unsigned long long *)(pic_smem + 6 * wn());
        atomicAdd(&jw[c * wn() + lin(bi, bj, bk) + ii + wx() * jj + wxy() * kk],
                  (unsigned long long)(long long)(int)v);
    }
    // the int64 current window: its first float of the dynamic LDS, its
    // length, and the entry of component c at window node r
    __device__ __forceinline__ int jbase() const { return 6 * wn(); }
    __device__ __forceinline__ int jcount() const { return 3 * wn(); }
    __device__ __forceinline__ int jslot(int c, int r) const { return c * wn() + r; }
    // (2D) current view from an Esirkepov stencil base: node (ii, jj) of
    // component c at base + c wn + ii + jj wx
    struct JView {
        unsigned long long *jw;
        int base, wx, wn;
        __device__ __forceinline__ void add(int c, int ii, int jj, float v) const {
            atomicAdd(&jw[c * wn + base + ii + wx * jj], (unsigned long long)(long long)(int)v);
        }
    };
    __device__ __forceinline__ JView jview(int bi, int bj) const {
        return JView{(unsigned long long *)(pic_smem + 6 * wn()), lin(bi, bj, 0), wx(), wn()};
    }
};

// 2D window in x-parity planes.  Consecutive lanes of a wavefront push
// particles in cells two apart along x (one parity class of the tile per
// wavefront), so with nodes stored row by row their addresses all have one
// parity and use half the LDS banks.  Here the nodes of even x and of odd x
// sit in separate planes: node (x, y) is at (x & 1) P + (x >> 1) + WP y, the
// lanes of a row of cells hit consecutive words, and the row stride WP
// (12 = 4 mod 8 in 8-byte words) puts the four rows of cells of a
// half-wavefront on four disjoint groups of eight banks.  P (the odd plane's
// start, 289 = 1 mod 32) was chosen by a model of the bank conflicts of
// random stencil shifts.  A stencil that starts at x = b has its even-offset
// nodes in b's plane at columns (b >> 1) + ii/2 and its odd-offset nodes in
// the other plane, so a view keeps two base addresses and every node is an
// immediate offset from one of them.  Plane groups of GS = 2P elements:
// (E_x, B_y) and (E_y, B_x) interleaved node by node (8-byte elements),
// E_z, B_z (4 bytes), then the int64 current window, three groups.  Built
// for the 23 x 23 window (16 x 16 tiles, drift 1, reach [c-2, c+3]).
template <int WX, int WY>
struct LdsSplit2 {
    static_assert(WX == 23 && WY == 23, "x-parity layout built for the 23 x 23 window");
    static constexpr int WP = 12, P = 289, GS = 2 * P;
    float scale;
    __device__ __forceinline__ int wx() const { return WX; }
    __device__ __forceinline__ int wxy() const { return WX * WY; }
    __device__ __forceinline__ int wn() const { return WX * WY; }
    static __device__ __forceinline__ int idx(int x, int y) { return (x & 1) * P + (x >> 1) + WP * y; }
    // index in a plane group of window node r (row-major r = x + WX y)
    static __device__ __forceinline__ int idx_r(int r) {
        const int y = r / WX;
        return idx(r - WX * y, y);
    }
    __device__ __forceinline__ int slot(int c, int r) const {
        const int n = idx_r(r);
        const int grp = c == 0 || c == 4 ? 0 : (c == 1 || c == 3 ? 2 * GS : (c == 2 ? 4 * GS : 5 * GS));
        const int lane = c == 4 || c == 3 ? 1 : 0;
        const int step = c == 2 || c == 5 ? 1 : 2;
        return grp + step * n + lane;
    }
    __device__ __forceinline__ int jbase() const { return 6 * GS; }
    __device__ __forceinline__ int jcount() const { return 3 * GS; }
    __device__ __forceinline__ int jslot(int c, int r) const { return c * GS + idx_r(r); }
    // the two base addresses of a stencil starting at window node (bi, bj):
    // first = its own node, second = node (bi + 1, bj)
    static __device__ __forceinline__ void bases(int bi, int bj, int &first, int &second) {
        const int e = bi & 1;
        first = (bi >> 1) + WP * bj + (e ? P : 0);
        second = first + (e ? 1 - P : P);
    }
    typedef float vec2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const vec2 lds_float2;
    typedef __attribute__((address_space(3))) const float lds_float;
    template <typename T>
    static __device__ __forceinline__ const T *opaque(const T *q) {
        uint32_t addr = (uint32_t)(uintptr_t)q;
        asm volatile("" : "+v"(addr));
        return (const T *)(uintptr_t)addr;
    }
    struct PairView {
        const lds_float2 *p0, *p1;
        __device__ __forceinline__ float2 operator()(int ii, int jj) const {
            const vec2 v = (ii & 1 ? p1 : p0)[(ii >> 1) + WP * jj];
            return make_float2(v.x, v.y);
        }
    };
    __device__ __forceinline__ PairView pair_view(int p, int bi, int bj) const {
        int f, g;
        bases(bi, bj, f, g);
        const lds_float2 *q = (const lds_float2 *)(const vec2 *)pic_smem + p * GS;
        return PairView{opaque(q + f), opaque(q + g)};
    }
    struct PlaneView {
        const lds_float *p0, *p1;
        __device__ __forceinline__ float operator()(int ii, int jj) const {
            return (ii & 1 ? p1 : p0)[(ii >> 1) + WP * jj];
        }
    };
    __device__ __forceinline__ PlaneView plane_view(int c, int bi, int bj) const {
        int f, g;
        bases(bi, bj, f, g);
        const lds_float *q = (const lds_float *)(const float *)pic_smem + (c == 2 ? 4 * GS : 5 * GS);
        return PlaneView{opaque(q + f), opaque(q + g)};
    }
    struct JView {
        unsigned long long *j0, *j1;
        __device__ __forceinline__ void add(int c, int ii, int jj, float v) const {
            atomicAdd(&(ii & 1 ? j1 : j0)[c * GS + (ii >> 1) + WP * jj], (unsigned long long)(long long)(int)v);
        }
    };
    __device__ __forceinline__ JView jview(int bi, int bj) const {
        int f, g;
        bases(bi, bj, f, g);
        unsigned long long *jw = (unsigned long long *)(pic_smem + 6 * GS);
        return JView{jw + f, jw + g};
    }
    static constexpr size_t bytes() { return (size_t)GS * (6 * sizeof(float) + 3 * sizeof(int64_t)); }
};

// Accessor of global memory: absolute cell coordinates, periodic wrap.
struct GlobAcc {
    const float *F[6];
    float *J[3];
    int ng[3];
    float scale;  // 1: values arrive in physical units
    int absorb_x;  // no field from, no current to x nodes beyond [0, ng[0])
    __device__ __forceinline__ int64_t idx(int i, int j, int k) const {
        i = wrap_index(i, ng[0]);
        j = wrap_index(j, ng[1]);
        k = wrap_index(k, ng[2]);
        return (int64_t)i + (int64_t)ng[0] * ((int64_t)j + (int64_t)ng[1] * k);
    }
    __device__ __forceinline__ float f(int c, int bi, int bj, int bk, int ii, int jj, int kk) const {
        if (absorb_x && (unsigned)(bi + ii) >= (unsigned)ng[0]) return 0.0f;
        return F[c][idx(bi + ii, bj + jj, bk + kk)];
    }
    struct PairView {
        const GlobAcc *g;
        int p, bi, bj;
        __device__ __forceinline__ float2 operator()(int ii, int jj) const {
            return make_float2(g->f(p == 0 ? 0 : 1, bi, bj, 0, ii, jj, 0), g->f(p == 0 ? 4 : 3, bi, bj, 0, ii, jj, 0));
        }
    };
    __device__ __forceinline__ PairView pair_view(int p, int bi, int bj) const { return PairView{this, p, bi, bj}; }
    struct PlaneView {
        const GlobAcc *g;
        int c, bi, bj;
        __device__ __forceinline__ float operator()(int ii, int jj) const { return g->f(c, bi, bj, 0, ii, jj, 0); }
    };
    __device__ __forceinline__ PlaneView plane_view(int c, int bi, int bj) const { return PlaneView{this, c, bi, bj}; }
    __device__ __forceinline__ void add(int c, int bi, int bj, int bk, int ii, int jj, int kk, float v) const {
        if (absorb_x && (unsigned)(bi + ii) >= (unsigned)ng[0]) return;
        atomicAdd(&J[c][idx(bi + ii, bj + jj, bk + kk)], v);
    }
    struct JView {
        const GlobAcc *g;
        int bi, bj;
        __device__ __forceinline__ void add(int c, int ii, int jj, float v) const { g->add(c, bi, bj, 0, ii, jj, 0, v); }
    };
    __device__ __forceinline__ JView jview(int bi, int bj) const { return JView{this, bi, bj}; }
};

// Push one particle whose cell origin is at o[] in the accessor's coordinates.
// f[] in-cell offsets, u[] momentum (updated); returns the cell displacement
// in dc[] and the new offsets in f[]; EB[] receives the gathered fields and
// gm1 = gamma^{n+1} - 1, formed as |u|^2 / (gamma + 1) (no cancellation).
template <int DIM, int ORDER, int PUSH, class Acc>
__device__ __forceinline__ void push_one(const Acc &acc, const TiledArgs &a, const int *o, float *f,
                                         float *u, float w, int *dc, float *EB, float &gm1) {
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
    if constexpr (DIM == 2) {
        // (E_x, B_y) share the stagger (1/2, 0) and (E_y, B_x) (0, 1/2): one
        // node read serves both members of a pair
        auto gather_pair = [&](int p, int sx, int sy, float &ra, float &rb) {
            const auto pv = acc.pair_view(p, o[0] + i0[sx][0], o[1] + i0[sy][1]);
            ra = 0.0f;
            rb = 0.0f;
#pragma unroll
            for (int jj = 0; jj < NW; ++jj) {
                float sa = 0.0f, sb = 0.0f;
#pragma unroll
                for (int ii = 0; ii < NW; ++ii) {
                    const float2 v = pv(ii, jj);
                    sa += wt[sx][0][ii] * v.x;
                    sb += wt[sx][0][ii] * v.y;
                }
                ra += wt[sy][1][jj] * sa;
                rb += wt[sy][1][jj] * sb;
            }
        };
        gather_pair(0, 1, 0, EB[0], EB[4]);
        gather_pair(1, 0, 1, EB[1], EB[3]);
        // E_z at (0, 0), B_z at (1/2, 1/2)
        auto gather_one = [&](int c, int sx, int sy) {
            const auto pv = acc.plane_view(c, o[0] + i0[sx][0], o[1] + i0[sy][1]);
            float r = 0.0f;
#pragma unroll
            for (int jj = 0; jj < NW; ++jj) {
                float t = 0.0f;
#pragma unroll
                for (int ii = 0; ii < NW; ++ii) t += wt[sx][0][ii] * pv(ii, jj);
                r += wt[sy][1][jj] * t;
            }
            return r;
        };
        EB[2] = gather_one(2, 0, 0);
        EB[5] = gather_one(5, 1, 1);
    } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int sx = stag(c, 0), sy = stag(c, 1), sz = stag(c, 2);
        float acc_v = 0.0f;
        {
#pragma unroll
            for (int kk = 0; kk < NW; ++kk) {
                float s = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NW; ++jj) {
                    float r = 0.0f;
#pragma unroll
                    for (int ii = 0; ii < NW; ++ii)
                        r += wt[sx][0][ii] * acc.f(c, o[0] + i0[sx][0], o[1] + i0[sy][1], o[2] + i0[sz][2],
                                                   ii, jj, kk);
                    s += wt[sy][1][jj] * r;
                }
                acc_v += wt[sz][2][kk] * s;
            }
        }
        EB[c] = acc_v;
    }
    }

    push_u<PUSH, float>(a.qm_h, EB, EB + 3, u);
    const float us = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float ig1 = rsqrt_r(1.0f + us);
    gm1 = us * ig1 * rcp_r(1.0f + ig1);
    const float v[3] = {u[0] * ig1, u[1] * ig1, u[2] * ig1};

    // Esirkepov (Eqs. 20-22) for the move dh -> dh + dt v / d.  Along an axis
    // the particle does not cross (start and end supports equal), the last
    // stencil node and the last running-sum node carry exactly zero: those
    // lanes sit out the atomics (fewer LDS lane operations).
    int base[3] = {0, 0, 0};
    bool cr[3] = {false, false, false};
    float S0[3][L], DS[3][L];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
        esirkepov_axis_from<ORDER>(i0[0][d], wt[0][d], dh[d] + a.dt_d[d] * v[d], base[d], S0[d], DS[d], cr[d]);
    // node k of a weight along axis d / of a running sum along d is nonzero
    auto wnode = [&](int d, int k) { return k <= ORDER || cr[d]; };
    auto rnode = [&](int d, int k) { return k < ORDER || cr[d]; };
    const int b0 = o[0] + base[0], b1 = o[1] + base[1];
    const float ws = w * acc.scale;  // fixed-point units in the LDS window
    const float jx = a.jfac[0] * ws, jy = a.jfac[1] * ws;
    if constexpr (DIM == 2) {
        const auto jv = acc.jview(b0, b1);
#pragma unroll
        for (int jj = 0; jj < L; ++jj) {
            const float ty = jx * (S0[1][jj] + 0.5f * DS[1][jj]);
            float run = 0.0f;
#pragma unroll
            for (int ii = 0; ii < L - 1; ++ii) {
                run -= DS[0][ii] * ty;
                if (rnode(0, ii) && wnode(1, jj)) jv.add(0, ii, jj, run);
            }
        }
#pragma unroll
        for (int ii = 0; ii < L; ++ii) {
            const float tx = jy * (S0[0][ii] + 0.5f * DS[0][ii]);
            float run = 0.0f;
#pragma unroll
            for (int jj = 0; jj < L - 1; ++jj) {
                run -= DS[1][jj] * tx;
                if (rnode(1, jj) && wnode(0, ii)) jv.add(1, ii, jj, run);
            }
        }
        const float qv = a.q * ws * v[2];
#pragma unroll
        for (int jj = 0; jj < L; ++jj) {
            const float a0 = qv * (S0[1][jj] + 0.5f * DS[1][jj]);
            const float a1 = qv * (0.5f * S0[1][jj] + (1.0f / 3.0f) * DS[1][jj]);
#pragma unroll
            for (int ii = 0; ii < L; ++ii)
                if (wnode(0, ii) && wnode(1, jj)) jv.add(2, ii, jj, S0[0][ii] * a0 + DS[0][ii] * a1);
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
                    if (rnode(0, ii) && wnode(1, jj) && wnode(2, kk)) acc.add(0, b0, b1, b2, ii, jj, kk, run);
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
                    if (rnode(1, jj) && wnode(0, ii) && wnode(2, kk)) acc.add(1, b0, b1, b2, ii, jj, kk, run);
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
                    if (rnode(2, kk) && wnode(0, ii) && wnode(1, jj)) acc.add(2, b0, b1, b2, ii, jj, kk, run);
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

// chi_e (Sec. IV) at the gathered fields of x_h and u^{n+1/2} = (u^n + u^{n+1})/2
__device__ __forceinline__ float chi_of(const float *u0, const float *u1, const float *EB) {
    const float uh0 = 0.5f * (u0[0] + u1[0]), uh1 = 0.5f * (u0[1] + u1[1]), uh2 = 0.5f * (u0[2] + u1[2]);
    const float gh = sqrtf(1.0f + uh0 * uh0 + uh1 * uh1 + uh2 * uh2);
    const float f0 = gh * EB[0] + uh1 * EB[5] - uh2 * EB[4];
    const float f1 = gh * EB[1] + uh2 * EB[3] - uh0 * EB[5];
    const float f2 = gh * EB[2] + uh0 * EB[4] - uh1 * EB[3];
    const float ue = uh0 * EB[0] + uh1 * EB[1] + uh2 * EB[2];
    return sqrtf(fmaxf(f0 * f0 + f1 * f1 + f2 * f2 - ue * ue, 0.0f));
}

// element at byte offset `bo` of a per-tile base pointer: one 32-bit VGPR
// offset against a wave-uniform base for every particle array
template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t bo) {
    return *(const T *)((const char *)base + bo);
}
template <typename T>
__device__ __forceinline__ void st(T *base, uint32_t bo, T v) {
    *(T *)((char *)base + bo) = v;
}

// sum of a double over the workgroup in a fixed order (wave butterflies, then
// the waves in order); `red` holds NT/64 doubles; result valid in thread 0
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) t += red[k];
    return t;
}

template <class Lds>
__device__ __forceinline__ Lds make_lds(const TiledArgs &a) {
    if constexpr (std::is_same<Lds, LdsSplit2<23, 23>>::value) {
        return Lds{0.0f};
    } else {
        return Lds{a.win[0], a.win[0] * a.win[1], a.win[0] * a.win[1] * a.win[2], 0.0f};
    }
}

// Byte offset of a particle's elements: 32-bit against per-tile bases in the
// sorted (contiguous) pass, 64-bit against the array bases in the binned pass.
template <bool LIST>
struct POff {
    typedef uint32_t type;
};
template <>
struct POff<true> {
    typedef uint64_t type;
};

// Species pushed in one pass over the tiles: each tile stages its field
// window once, and the species' currents share its fixed-point window (the
// scale bounds every species' contributions).  Grid, fields and window come
// from sp[0]; particles, charge, mass and scratch from each sp[k].
template <int NSP>
struct TiledSet {
    TiledArgs sp[NSP];
    int nsp;
};

// LIST = false: the tile's particles are [tile_start[t], tile_start[t+1]) of
// the sorted arrays.  LIST = true: they are bin_list[bin_start[t] ..
// bin_start[t+1]) (the stragglers and appended particles binned by the tile
// that holds them now).
template <int DIM, int ORDER, int PUSH, int NT, int WX, int WY, int WZ, bool LIST, bool SPLIT = false, int NSP = 1>
__global__ void __launch_bounds__(NT) gpd_tiled_kernel(TiledSet<NSP> S) {
    typedef typename POff<LIST>::type off_t;
    const TiledArgs &a0 = S.sp[0];
    const int nsp = NSP == 1 ? 1 : S.nsp;
    const int b = blockIdx.x;
    const int t = (b & 7) * a0.chunk + (b >> 3);  // XCD-contiguous tile runs
    if (t >= a0.ntiles) return;
    // particles of a species in this tile: [beg, end) of its sorted or binned order
    auto range = [&](const TiledArgs &a, int64_t &beg, int64_t &end) {
        const int64_t *start = LIST ? a.bin_start : a.tile_start;
        beg = min(start[t], a.n);
        end = min(start[t + 1], a.n);
    };
    __shared__ double red_k[NT / 64], red_q[NT / 64];
    __shared__ float wmax_s[NT / 64];
    __shared__ uint32_t nstray;
    bool any = false;
    for (int k = 0; k < nsp; ++k) {
        int64_t pb, pe;
        range(S.sp[k], pb, pe);
        any |= pb < pe;
    }
    if (!any) {
        if (threadIdx.x == 0) {
            for (int k = 0; k < nsp; ++k) {
                const TiledArgs &a = S.sp[k];
                double *part = a.partials + a.part_off;
                part[2 * t] = 0.0;
                part[2 * t + 1] = 0.0;
                if (!LIST) a.strag_tile[t] = 0u;
            }
        }
        return;
    }
    if (threadIdx.x == 0) nstray = 0u;
    const int tx = t % a0.ntile_axis[0];
    const int ty = (t / a0.ntile_axis[0]) % a0.ntile_axis[1];
    const int tz = DIM == 3 ? t / (a0.ntile_axis[0] * a0.ntile_axis[1]) : 0;
    // stencil reach around a particle's cell c: [c - RLO, c + RHI]
    constexpr int RLO = ORDER == 4 ? 3 : 2, RHI = ORDER == 4 ? 4 : 3;
    const int g = a0.drift + RLO;
    const int org[3] = {tx * a0.tile[0] - g, ty * a0.tile[1] - g, DIM == 3 ? tz * a0.tile[2] - g : 0};
    typedef typename std::conditional<SPLIT, LdsSplit2<WX, WY>, LdsAcc<WX, WY, WZ, DIM == 2>>::type Lds;
    Lds lds = make_lds<Lds>(a0);
    const int wn = lds.wn();
    const int wx = lds.wx(), wxy = lds.wxy();
    unsigned long long *jwin = (unsigned long long *)(pic_smem + lds.jbase());
    // element offsets: sorted pass, bases moved to the tile's first particle
    // and one 32-bit offset per particle; binned pass, offsets of the listed
    // particles against the array bases
    auto poff_of = [&](const int32_t *plist, uint32_t i) -> off_t {
        return LIST ? (off_t)4 * (off_t)(uint32_t)plist[i] : (off_t)(4u * i);
    };

    // 1. stage the E/B window, zero the J window (window index decoded once
    //    per cell), bound the weights of the tile.  With the window shape
    //    compiled in, every load of a thread's cells is issued before the
    //    first store, so the staging waits for one memory latency, not one
    //    per cell (it matters where one workgroup has the CU to itself).
    auto cell_src = [&](int r, int64_t &gidx, bool &beyond) {
        const int k = DIM == 3 ? r / wxy : 0;
        const int r2 = r - k * wxy;
        const int j = r2 / wx;
        const int i = r2 - j * wx;
        const int gi = wrap_index(org[0] + i, a0.ng[0]);
        const int gj = wrap_index(org[1] + j, a0.ng[1]);
        const int gk = DIM == 3 ? wrap_index(org[2] + k, a0.ng[2]) : 0;
        gidx = (int64_t)gi + (int64_t)a0.ng[0] * ((int64_t)gj + (int64_t)a0.ng[1] * gk);
        beyond = a0.absorb_x && (unsigned)(org[0] + i) >= (unsigned)a0.ng[0];
    };
    constexpr int SITER = WX > 0 ? (WX * WY * WZ + NT - 1) / NT : 0;
    if constexpr (SITER > 0 && SITER <= 4) {
        float v[SITER][6];
#pragma unroll
        for (int s = 0; s < SITER; ++s) {
            const int r = (int)threadIdx.x + s * NT;
            if (r < wn) {
                int64_t gidx;
                bool beyond;
                cell_src(r, gidx, beyond);
#pragma unroll
                for (int c = 0; c < 6; ++c) v[s][c] = beyond ? 0.0f : a0.F[c][gidx];
            }
        }
#pragma unroll
        for (int s = 0; s < SITER; ++s) {
            const int r = (int)threadIdx.x + s * NT;
            if (r < wn) {
#pragma unroll
                for (int c = 0; c < 6; ++c) pic_smem[lds.slot(c, r)] = v[s][c];
            }
        }
    } else {
        for (int r = threadIdx.x; r < wn; r += NT) {
            int64_t gidx;
            bool beyond;
            cell_src(r, gidx, beyond);
#pragma unroll
            for (int c = 0; c < 6; ++c) pic_smem[lds.slot(c, r)] = beyond ? 0.0f : a0.F[c][gidx];
        }
    }
    for (int r = threadIdx.x; r < lds.jcount(); r += NT) jwin[r] = 0ull;
    // bound of |q| |w| over the tile's particles of every species: the
    // binning's per-bin bound in the binned pass, else the per-particle
    // weights read with four loads in flight per round
    float wm = 0.0f;
    if constexpr (LIST) {
        for (int k = 0; k < nsp; ++k) wm = fmaxf(wm, __uint_as_float(S.sp[k].bin_wmax[t]));
    } else {
        for (int k = 0; k < nsp; ++k) {
            const TiledArgs &a = S.sp[k];
            int64_t pbeg, pend;
            range(a, pbeg, pend);
            if (pbeg >= pend) continue;
            const float aq = fabsf(a.q);
            if (!a.w) {
                wm = fmaxf(wm, aq * fabsf(a.w0));
                continue;
            }
            const uint32_t np = (uint32_t)(pend - pbeg);
            const float *wT = a.w + pbeg;
            for (uint32_t i = threadIdx.x; i < np; i += 4 * NT) {
                float x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = i + q * NT < np ? fabsf(ld(wT, 4u * (i + q * NT))) : 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) wm = fmaxf(wm, aq * x[q]);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wm = fmaxf(wm, __shfl_xor(wm, o));
    if ((threadIdx.x & 63) == 0) wmax_s[threadIdx.x >> 6] = wm;
    __syncthreads();
    {
        float qwmax = 0.0f;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) qwmax = fmaxf(qwmax, wmax_s[k]);
        // S = 2^(30 - ceil(log2 B)), B = max |q| w max(1, d/dt): |contribution| * S <= 2^30
        const float B = qwmax * a0.jmax;
        int ex = 0;
        frexpf(B > 0.0f ? B : 1.0f, &ex);  // B < 2^ex
        lds.scale = ldexpf(1.0f, 30 - ex);
    }

    // 2. particles of the tile, species after species, next particle
    //    prefetched while one is pushed
    const int mx = (1 << a0.bx) - 1, my = (1 << a0.by) - 1;
    const int hi[3] = {wx - RHI - 1, (DIM >= 2 ? wxy / wx : 1) - RHI - 1, (DIM == 3 ? wn / wxy : 1) - RHI - 1};
    // WRAP: the window crosses the periodic seam (or an absorbing face) along
    // some axis.  Otherwise a cell's window coordinate is its offset from the
    // origin, and a pushed particle (it stays within the window's reach)
    // cannot leave [0, n): neither needs the unwrap.
    bool wraps = false;
    const int wext[3] = {wx, DIM >= 2 ? wxy / wx : 1, DIM == 3 ? wn / wxy : 1};
#pragma unroll
    for (int d = 0; d < DIM; ++d) wraps |= org[d] < 0 || org[d] + wext[d] > a0.ng[d];
    for (int k = 0; k < nsp; ++k) {
    const TiledArgs &a = S.sp[k];
    int64_t pbeg, pend;
    range(a, pbeg, pend);
    double kin = 0.0, chg = 0.0;
    if (pbeg < pend) {
    const uint32_t np = (uint32_t)(pend - pbeg);
    const int64_t rebase = LIST ? 0 : pbeg;
    const int32_t *plist = a.bin_list + pbeg;
    auto poff = [&](uint32_t i) -> off_t { return poff_of(plist, i); };
    auto pidx = [&](uint32_t i) -> int64_t { return LIST ? (int64_t)plist[i] : pbeg + i; };
    int32_t *cellT = a.cell + rebase;
    float *offT[3], *uT[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        offT[d] = a.off[d] + rebase;
        uT[d] = a.u[d] + rebase;
    }
    const float *wT = a.w ? a.w + rebase : nullptr;
    float *wW = a.w ? a.w + rebase : nullptr;  // absorption (weights are required with absorbing faces)
    float *chiT = a.chi ? a.chi + rebase : nullptr;
    auto particles = [&](auto wrap_c) {
    constexpr bool WRAP = decltype(wrap_c)::value;
    uint32_t i = threadIdx.x;
    int32_t n_cell = 0;
    float n_f[3] = {0.0f, 0.0f, 0.0f}, n_u[3] = {0.0f, 0.0f, 0.0f}, n_w = a.w0;
    if (i < np) {
        const off_t bo = poff(i);
        n_cell = ld(cellT, bo);
#pragma unroll
        for (int d = 0; d < DIM; ++d) n_f[d] = ld(offT[d], bo);
#pragma unroll
        for (int d = 0; d < 3; ++d) n_u[d] = ld(uT[d], bo);
        if (wT) n_w = ld(wT, bo);
    }
    for (; i < np; i += NT) {
        const off_t bo = poff(i);
        const int32_t cell = n_cell;
        float f[3] = {n_f[0], n_f[1], n_f[2]};
        float u[3] = {n_u[0], n_u[1], n_u[2]};
        const float w = n_w;
        if (i + NT < np) {
            const off_t bn = LIST ? poff(i + NT) : bo + (off_t)(4u * NT);
            n_cell = ld(cellT, bn);
#pragma unroll
            for (int d = 0; d < DIM; ++d) n_f[d] = ld(offT[d], bn);
#pragma unroll
            for (int d = 0; d < 3; ++d) n_u[d] = ld(uT[d], bn);
            if (wT) n_w = ld(wT, bn);
        }
        const int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        if (!isfinite(u[0] + u[1] + u[2])) atomicOr(a.status, PIC_F_NONFINITE);
        // local cell in the window (one periodic unwrap); the particle stays
        // here only if the whole stencil lies in the window and its offsets
        // are in [0,1) (as bit patterns: 0 <= bits < bits(1.0f))
        int lc[3] = {0, 0, 0};
        bool inside = DIM == 3 || (cell >> (a.bx + a.by)) == 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            // no periodic image across an absorbing face: a particle on the
            // far side of the domain is not in this window
            const int l = WRAP && !(d == 0 && a.absorb_x) ? wrap_index(cc[d] - org[d], a.ng[d]) : cc[d] - org[d];
            lc[d] = l;
            inside &= (unsigned)(l - RLO) <= (unsigned)(hi[d] - RLO) && (unsigned)cc[d] < (unsigned)a.ng[d];
            inside &= __float_as_uint(f[d]) < 0x3f800000u;
        }
        if (!inside) {
            // sorted pass: into the tile's own slice of the list (LDS counter);
            // binned pass (rare): appended to the shared list
            const uint32_t slot = LIST ? atomicAdd(a.strag_count, 1u) : (uint32_t)pbeg + atomicAdd(&nstray, 1u);
            a.strag_list[slot] = (int32_t)pidx(i);
            continue;
        }
        const float u_old[3] = {u[0], u[1], u[2]};
        float EB[6];
        int dc[3] = {0, 0, 0};
        float gm1;
        push_one<DIM, ORDER, PUSH>(lds, a, lc, f, u, w, dc, EB, gm1);
        int packed = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            packed |= (WRAP ? wrap_index(cc[d] + dc[d], a.ng[d]) : cc[d] + dc[d])
                      << (d == 0 ? 0 : (d == 1 ? a.bx : a.bx + a.by));
        st(cellT, bo, packed);
        // absorbing x faces: x nodes of the domain are [0, n-1], so a new
        // cell outside [0, n-2] (before the wrap) is a position beyond a face
        if (a.absorb_x && (unsigned)(cc[0] + dc[0]) >= (unsigned)(a.ng[0] - 1)) st(wW, bo, 0.0f);
#pragma unroll
        for (int d = 0; d < DIM; ++d) st(offT[d], bo, f[d]);
#pragma unroll
        for (int d = 0; d < 3; ++d) st(uT[d], bo, u[d]);
        if (chiT) st(chiT, bo, a.chi_scale * chi_of(u_old, u, EB));
        kin += (double)w * (double)gm1;
        chg += (double)w;
    }
    };
    if (wraps) particles(std::integral_constant<bool, true>{});
    else particles(std::integral_constant<bool, false>{});
    }
    // fixed-order FP64 reduction of the species' diagnostics (its barrier
    // also ends the species' LDS atomics and straggler count)
    const double sk = block_sum<NT>(kin, red_k);
    const double sq = block_sum<NT>(chg, red_q);
    if (threadIdx.x == 0) {
        double *part = a.partials + a.part_off;
        part[2 * t] = sk * a.mdV;
        part[2 * t + 1] = sq * a.qdV;
        if (!LIST) a.strag_tile[t] = nstray;
        nstray = 0u;
    }
    if (NSP > 1) __syncthreads();  // red_k, red_q and nstray are reused by the next species
    }
    __syncthreads();

    // 3. flush the J window into global J (periodic wrap), skip exact zeros
    const double inv_scale = 1.0 / (double)lds.scale;
    for (int r = threadIdx.x; r < wn; r += NT) {
        const int k = DIM == 3 ? r / wxy : 0;
        const int r2 = r - k * wxy;
        const int j = r2 / wx;
        const int ii = r2 - j * wx;
        const int gi = wrap_index(org[0] + ii, a0.ng[0]);
        const int gj = wrap_index(org[1] + j, a0.ng[1]);
        const int gk = DIM == 3 ? wrap_index(org[2] + k, a0.ng[2]) : 0;
        const int64_t gidx = (int64_t)gi + (int64_t)a0.ng[0] * ((int64_t)gj + (int64_t)a0.ng[1] * gk);
        if (a0.absorb_x && (unsigned)(org[0] + ii) >= (unsigned)a0.ng[0]) continue;  // beyond a face
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long q = (long long)jwin[lds.jslot(c, r)];
            if (q != 0) atomicAdd(&a0.J[c][gidx], (float)((double)q * inv_scale));
        }
    }
}

// Clears the bin counters, the bins' weight bounds and the straggler count
// before the sorted pass.
__global__ void gpd_prep_kernel(uint32_t *bin_count, uint32_t *bin_wmax, int ntiles, uint32_t *strag_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntiles) {
        bin_count[i] = 0u;
        bin_wmax[i] = 0u;
    }
    if (i == 0) *strag_count = 0u;
}

__global__ void gpd_reset_kernel(uint32_t *count) { *count = 0u; }

__device__ __forceinline__ int tile_of(const TiledArgs &a, int dim, int32_t cell) {
    const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
    const int ix = cell & mx, iy = (cell >> a.bx) & my, iz = dim == 3 ? (cell >> (a.bx + a.by)) : 0;
    return ix / a.tile[0] + a.ntile_axis[0] * (iy / a.tile[1] + a.ntile_axis[1] * (iz / a.tile[2]));
}

constexpr uint32_t BIN_SKIP = 0xFFFFFFFFu;
constexpr int TAIL_BLOCKS = 256;
constexpr int BIN_REACH = 2;                      // neighbour tiles counted in LDS: +-2 per axis
constexpr int BIN_SLOTS = 125;                    // (2 BIN_REACH + 1)^3

// Work item of the binning kernels: block b < ntiles takes the stragglers of
// tile b (strag_list[tile_start[b] .. + strag_tile[b])); the last
// TAIL_BLOCKS blocks stride over the particles appended after the last tile.
// *pos is the entry's slot in bin_rank (its list position, or the particle
// index for the tail: the two ranges are disjoint).
struct BinItems {
    int64_t lo, hi, stride;
    bool tail;
};
__device__ __forceinline__ BinItems bin_items(const TiledArgs &a) {
    BinItems it;
    const int b = blockIdx.x;
    if (b < a.ntiles) {
        it.lo = min(a.tile_start[b], a.n);
        it.hi = min(it.lo + (int64_t)a.strag_tile[b], a.n);
        it.stride = blockDim.x;
        it.tail = false;
        it.lo += threadIdx.x;
    } else {
        const int64_t first = min(a.tile_start[a.ntiles], a.n);
        it.lo = first + (int64_t)(b - a.ntiles) * blockDim.x + threadIdx.x;
        it.hi = a.n;
        it.stride = (int64_t)TAIL_BLOCKS * blockDim.x;
        it.tail = true;
    }
    return it;
}

// slot of destination tile `dt` among the neighbours of tile `st` (periodic),
// or -1 when it lies further than BIN_REACH tiles along some axis
template <int DIM>
__device__ __forceinline__ int neighbour_slot(const TiledArgs &a, int st, int dt) {
    int slot = 0, mul = 1;
    int sc[3] = {st % a.ntile_axis[0], (st / a.ntile_axis[0]) % a.ntile_axis[1], st / (a.ntile_axis[0] * a.ntile_axis[1])};
    int dc[3] = {dt % a.ntile_axis[0], (dt / a.ntile_axis[0]) % a.ntile_axis[1], dt / (a.ntile_axis[0] * a.ntile_axis[1])};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int nt = a.ntile_axis[d];
        int o = dc[d] - sc[d];
        if (2 * o >= nt) o -= nt;      // nearest periodic image
        if (2 * o < -nt) o += nt;
        if (o < -BIN_REACH || o > BIN_REACH) return -1;
        slot += (o + BIN_REACH) * mul;
        mul *= 2 * BIN_REACH + 1;
    }
    return slot;
}

// Bins the stragglers of the sorted pass and the appended particles by the
// tile that holds them now.  A block counts the destinations that neighbour
// its tile in LDS and reserves each neighbour's share with one global atomic;
// farther destinations (and the tail) reserve one by one.  A particle with an
// offset outside [0,1) or a cell off the grid is flagged PIC_F_OFFSET and left
// unchanged (never pushed).
// (The straggler flag and count are left to the bin scan, which reads every
// tile's count anyway: one atomic per block on one shared address serialized
// the blocks once most tiles had stragglers.)
// It also bounds |q| w over each destination tile's bin (bin_wmax, the
// float's bits: for values >= 0 the unsigned order is the float order; a NaN
// weight is left out, as the tile kernel's fmaxf leaves it out), so that the
// binned pass reads its fixed-point scale instead of a pass over its
// particles' weights.
template <int DIM>
__global__ void __launch_bounds__(256) gpd_bin_count_kernel(TiledArgs a) {
    __shared__ uint32_t lcnt[BIN_SLOTS], gbase[BIN_SLOTS], lwmax[BIN_SLOTS];
    for (int k = threadIdx.x; k < BIN_SLOTS; k += blockDim.x) {
        lcnt[k] = 0u;
        lwmax[k] = 0u;
    }
    __syncthreads();
    const float aq = fabsf(a.q);
    const BinItems it = bin_items(a);
    int found = 0;
    const int st = blockIdx.x;
    const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
    for (int64_t k = it.lo; k < it.hi; k += it.stride) {
        const int64_t p = it.tail ? k : (int64_t)a.strag_list[k];
        const int32_t cell = a.cell[p];
        const int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        // the bits above x and y hold z in 3D and must be zero in 2D
        bool ok = (unsigned)(cell >> (a.bx + a.by)) < (unsigned)(DIM == 3 ? a.ng[2] : 1);
        float fs = 0.0f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const float f = a.off[d][p];
            fs += f;
            ok &= f >= 0.0f && f < 1.0f && (unsigned)cc[d] < (unsigned)a.ng[d];
        }
        // (the sorted pass has checked the stragglers' momenta already; the
        // particles appended after the last tile it never saw)
        if ((it.tail && !isfinite(a.u[0][p] + a.u[1][p] + a.u[2][p])) || !isfinite(fs))
            atomicOr(a.status, PIC_F_NONFINITE);
        if (!ok) {
            atomicOr(a.status, PIC_F_OFFSET);
            a.bin_rank[k] = BIN_SKIP;
            continue;
        }
        const int dt = tile_of(a, DIM, cell);
        const int slot = it.tail ? -1 : neighbour_slot<DIM>(a, st, dt);
        const float qw = aq * fabsf(a.w ? a.w[p] : a.w0);
        const uint32_t qwb = qw == qw ? __float_as_uint(qw) : 0u;
        // neighbour: rank inside the block's share (top bit marks it);
        // otherwise the final rank straight from the global counter
        if (slot >= 0) {
            a.bin_rank[k] = 0x80000000u | atomicAdd(&lcnt[slot], 1u);
            atomicMax(&lwmax[slot], qwb);
        } else {
            a.bin_rank[k] = atomicAdd(&a.bin_count[dt], 1u);
            atomicMax(&a.bin_wmax[dt], qwb);
        }
        found = 1;
    }
    if (!__syncthreads_or(found) || it.tail) return;
    // reserve each neighbour's share, then turn local ranks into final ones
    const int sc[3] = {st % a.ntile_axis[0], (st / a.ntile_axis[0]) % a.ntile_axis[1],
                       st / (a.ntile_axis[0] * a.ntile_axis[1])};
    for (int k = threadIdx.x; k < BIN_SLOTS; k += blockDim.x) {
        if (lcnt[k] == 0u) continue;
        int dc[3] = {0, 0, 0}, r = k;
        for (int d = 0; d < DIM; ++d) {
            const int o = r % (2 * BIN_REACH + 1) - BIN_REACH;
            r /= 2 * BIN_REACH + 1;
            dc[d] = ((sc[d] + o) % a.ntile_axis[d] + a.ntile_axis[d]) % a.ntile_axis[d];
        }
        const int dt = dc[0] + a.ntile_axis[0] * (dc[1] + a.ntile_axis[1] * dc[2]);
        gbase[k] = atomicAdd(&a.bin_count[dt], lcnt[k]);
        atomicMax(&a.bin_wmax[dt], lwmax[k]);
    }
    __syncthreads();
    for (int64_t k = it.lo; k < it.hi; k += it.stride) {
        const uint32_t r = a.bin_rank[k];
        if (r == BIN_SKIP || !(r & 0x80000000u)) continue;
        const int32_t cell = a.cell[a.strag_list[k]];
        a.bin_rank[k] = gbase[neighbour_slot<DIM>(a, st, tile_of(a, DIM, cell))] + (r & 0x7FFFFFFFu);
    }
}

// bin_start = exclusive scan of bin_count (one workgroup, in order): chunks
// of 1024 x 8 counts, each thread taking 8 consecutive ones (independent
// loads, one memory latency per chunk), wavefront prefix sums by shuffles,
// then the 16 wavefront totals.  It also sums the sorted pass's straggler
// counts per tile (strag_tile) and, when there are any, raises
// PIC_F_STRAGGLER and adds them to the run's count: one atomic per call.
__global__ void __launch_bounds__(1024) gpd_bin_scan_kernel(const uint32_t *count, const uint32_t *strag_tile,
                                                            int ntiles, int64_t *bstart, uint32_t *status,
                                                            unsigned long long *stragglers) {
    constexpr int PER = 8;
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    __shared__ unsigned long long nsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    unsigned long long ns = 0;
    for (int base = 0; base < ntiles; base += 1024 * PER) {
        const int lo = base + (int)threadIdx.x * PER;
        uint32_t v[PER], g[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            v[k] = lo + k < ntiles ? count[lo + k] : 0u;
            g[k] = lo + k < ntiles ? strag_tile[lo + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) ns += g[k];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) s += v[k];
        // inclusive prefix of the thread totals within the wavefront
        int64_t x = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int64_t before = carry_s;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        int64_t run = before + x - s;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (lo + k < ntiles) bstart[lo + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = run;  // the last thread's running sum is the chunk's end
        __syncthreads();
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ns += __shfl_xor(ns, o);
    if (lane == 0) nsum[wave] = ns;
    __syncthreads();
    if (threadIdx.x == 0) {
        bstart[ntiles] = carry_s;
        unsigned long long tot = 0;
        for (int w = 0; w < 16; ++w) tot += nsum[w];
        if (tot > 0) {
            atomicOr(status, PIC_F_STRAGGLER);
            atomicAdd(stragglers, tot);
        }
    }
}

template <int DIM>
__global__ void __launch_bounds__(256) gpd_bin_scatter_kernel(TiledArgs a) {
    const BinItems it = bin_items(a);
    for (int64_t k = it.lo; k < it.hi; k += it.stride) {
        const uint32_t r = a.bin_rank[k];
        if (r == BIN_SKIP) continue;
        const int64_t p = it.tail ? k : (int64_t)a.strag_list[k];
        a.bin_list[a.bin_start[tile_of(a, DIM, a.cell[p])] + r] = (int32_t)p;
    }
}

// Global-memory path for what the binned pass could not place in a window
// (normally nothing: a binned particle sits in its own tile).  Same checks as
// the binning: invalid particles are flagged and left unchanged.
constexpr int GLOBAL_BLOCKS = 256;

template <int DIM, int ORDER, int PUSH>
__global__ void __launch_bounds__(256) gpd_global_kernel(TiledArgs a) {
    const int64_t total = (int64_t)*a.strag_count;
    __shared__ double red_k[4], red_q[4];
    double kin = 0.0, chg = 0.0;
    GlobAcc glob{{a.F[0], a.F[1], a.F[2], a.F[3], a.F[4], a.F[5]},
                 {a.J[0], a.J[1], a.J[2]},
                 {a.ng[0], a.ng[1], a.ng[2]}, 1.0f, a.absorb_x};
    const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = a.strag_list[k];
        const int32_t cell = a.cell[p];
        const int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        float f[3] = {a.off[0][p], a.off[1][p], DIM == 3 ? a.off[2][p] : 0.0f};
        float u[3] = {a.u[0][p], a.u[1][p], a.u[2][p]};
        const float w = a.w ? a.w[p] : a.w0;
        // the bits above x and y hold z in 3D and must be zero in 2D
        bool ok = (unsigned)(cell >> (a.bx + a.by)) < (unsigned)(DIM == 3 ? a.ng[2] : 1);
#pragma unroll
        for (int d = 0; d < DIM; ++d) ok &= f[d] >= 0.0f && f[d] < 1.0f && (unsigned)cc[d] < (unsigned)a.ng[d];
        if (!ok) {
            atomicOr(a.status, PIC_F_OFFSET);
            continue;
        }
        const float u_old[3] = {u[0], u[1], u[2]};
        float EB[6];
        int dc[3] = {0, 0, 0};
        float gm1;
        push_one<DIM, ORDER, PUSH>(glob, a, cc, f, u, w, dc, EB, gm1);
        int packed = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            packed |= wrap_index(cc[d] + dc[d], a.ng[d]) << (d == 0 ? 0 : (d == 1 ? a.bx : a.bx + a.by));
            a.off[d][p] = f[d];
        }
        a.cell[p] = packed;
        if (a.absorb_x && (unsigned)(cc[0] + dc[0]) >= (unsigned)(a.ng[0] - 1)) a.w[p] = 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) a.u[d][p] = u[d];
        if (a.chi) a.chi[p] = a.chi_scale * chi_of(u_old, u, EB);
        kin += (double)w * (double)gm1;
        chg += (double)w;
    }
    const double sk = block_sum<256>(kin, red_k);
    const double sq = block_sum<256>(chg, red_q);
    if (threadIdx.x == 0) {
        a.partials[a.part_off + 2 * blockIdx.x] = sk * a.mdV;
        a.partials[a.part_off + 2 * blockIdx.x + 1] = sq * a.qdV;
    }
}

// window shapes with a compiled kernel: 16x16 tiles with drift 2 in 2D
// (25 cells wide, 27 for quartic weights) and with drift 1 (23 wide, in the
// x-parity layout: measured 7% faster than drift 2's row-major window right
// after a sort, but at 24 steps between sorts drift 1 leaves three times the
// stragglers of drift 2, so 2D runs default to drift 2; the same layout at
// 25 x 25 needs a row stride of 20 and costs two workgroups per CU, which
// measured no faster), 8x8x4 tiles in 3D with drift 1
// (drift 0 for quartic weights): 15 x 15 x 11, and with drift 0 for
// quadratic weights: 13 x 13 x 9; others use the run-time shape
constexpr int W2X = 16 + 2 * 2 + 5, W2X4 = 16 + 2 * 2 + 7, W3X = 8 + 2 * 1 + 5, W3Z = 4 + 2 * 1 + 5;
constexpr int W2S = 16 + 2 * 1 + 5;
constexpr int W3X0 = 8 + 5, W3Z0 = 4 + 5;
// 8 x 8 x 8 tiles with drift 0 (quadratic): 13 x 13 x 13
constexpr int W3C0 = 8 + 5;

// One push of NSP species (one when NSP = 1, S.nsp of them otherwise):
//   prep (zero bin counters) -> sorted pass (stragglers listed) -> bin count
//   -> bin scan -> bin scatter -> reset of the list -> binned pass -> global
//   pass over whatever the binned pass listed.  The two tile passes take
//   every species at once; the binning and global kernels go species by
//   species.  Partials per species: [sorted pass: 2 ntiles][binned pass:
//   2 ntiles][global: 2 x 256].
template <int DIM, int ORDER, int PUSH, int NT, int WX, int WY, int WZ, bool SPLIT = false, int NSP = 1>
static void launch_passes(TiledSet<NSP> S, size_t lds, hipStream_t s) {
    const int nsp = NSP == 1 ? 1 : S.nsp;
    const int ntiles = S.sp[0].ntiles;
    const dim3 tiles((unsigned)(8 * S.sp[0].chunk)), block(NT), gb(GLOBAL_BLOCKS), b256(256);
    for (int k = 0; k < nsp; ++k) {
        TiledArgs &a = S.sp[k];
        gpd_prep_kernel<<<(unsigned)((ntiles + 255) / 256), 256, 0, s>>>(a.bin_count, a.bin_wmax, ntiles,
                                                                         a.strag_count);
        a.part_off = 0;
    }
    gpd_tiled_kernel<DIM, ORDER, PUSH, NT, WX, WY, WZ, false, SPLIT, NSP><<<tiles, block, lds, s>>>(S);
    const dim3 bins((unsigned)(ntiles + TAIL_BLOCKS));
    for (int k = 0; k < nsp; ++k) {
        TiledArgs &a = S.sp[k];
        gpd_bin_count_kernel<DIM><<<bins, b256, 0, s>>>(a);
        gpd_bin_scan_kernel<<<1, 1024, 0, s>>>(a.bin_count, a.strag_tile, ntiles, a.bin_start, a.status,
                                               a.stragglers);
        gpd_bin_scatter_kernel<DIM><<<bins, b256, 0, s>>>(a);
        gpd_reset_kernel<<<1, 1, 0, s>>>(a.strag_count);
        a.part_off = 2 * ntiles;
    }
    gpd_tiled_kernel<DIM, ORDER, PUSH, NT, WX, WY, WZ, true, SPLIT, NSP><<<tiles, block, lds, s>>>(S);
    for (int k = 0; k < nsp; ++k) {
        TiledArgs &a = S.sp[k];
        a.part_off = 4 * ntiles;
        gpd_global_kernel<DIM, ORDER, PUSH><<<gb, b256, 0, s>>>(a);
    }
}

template <int DIM, int ORDER, int PUSH, int NSP>
static void launch_tiled(const TiledSet<NSP> &S, size_t lds, hipStream_t s) {
    const TiledArgs &a = S.sp[0];
    if constexpr (DIM == 2) {
        if constexpr (ORDER != 4) {
            // 16 x 16 tiles with drift 1: the x-parity window layout
            if (a.win[0] == W2S && a.win[1] == W2S) {
                launch_passes<2, ORDER, PUSH, PIC_TILED_THREADS_2D, W2S, W2S, 1, true, NSP>(
                    S, LdsSplit2<W2S, W2S>::bytes(), s);
                return;
            }
        }
        constexpr int WX = ORDER == 4 ? W2X4 : W2X;
        if (a.win[0] == WX && a.win[1] == WX)
            launch_passes<2, ORDER, PUSH, PIC_TILED_THREADS_2D, WX, WX, 1, false, NSP>(S, lds, s);
        else
            launch_passes<2, ORDER, PUSH, PIC_TILED_THREADS_2D, 0, 0, 0, false, NSP>(S, lds, s);
    } else {
        if (a.win[0] == W3X && a.win[1] == W3X && a.win[2] == W3Z) {
            launch_passes<3, ORDER, PUSH, PIC_TILED_THREADS_3D, W3X, W3X, W3Z, false, NSP>(S, lds, s);
            return;
        }
        if constexpr (ORDER == 2) {
            if (a.win[0] == W3C0 && a.win[1] == W3C0 && a.win[2] == W3C0) {
                launch_passes<3, ORDER, PUSH, PIC_TILED_THREADS_3D, W3C0, W3C0, W3C0, false, NSP>(S, lds, s);
                return;
            }
            if (a.win[0] == W3X0 && a.win[1] == W3X0 && a.win[2] == W3Z0) {
                launch_passes<3, ORDER, PUSH, PIC_TILED_THREADS_3D, W3X0, W3X0, W3Z0, false, NSP>(S, lds, s);
                return;
            }
        }
        launch_passes<3, ORDER, PUSH, PIC_TILED_THREADS_3D, 0, 0, 0, false, NSP>(S, lds, s);
    }
}

template <int DIM, int ORDER, int NSP>
static void launch_pusher(const TiledSet<NSP> &S, int pusher, size_t lds, hipStream_t s) {
    if (pusher == PIC_PUSH_VAY) launch_tiled<DIM, ORDER, PIC_PUSH_VAY, NSP>(S, lds, s);
    else launch_tiled<DIM, ORDER, PIC_PUSH_BORIS, NSP>(S, lds, s);
}

template <int NSP>
static hipError_t launch_set(Ctx *c, const TiledSet<NSP> &S, size_t lds, hipStream_t s) {
    switch (c->dim * 10 + c->cfg.order) {
        case 21: launch_pusher<2, 1, NSP>(S, c->cfg.pusher, lds, s); break;
        case 22: launch_pusher<2, 2, NSP>(S, c->cfg.pusher, lds, s); break;
        case 31: launch_pusher<3, 1, NSP>(S, c->cfg.pusher, lds, s); break;
        case 32: launch_pusher<3, 2, NSP>(S, c->cfg.pusher, lds, s); break;
        case 24: launch_pusher<2, 4, NSP>(S, c->cfg.pusher, lds, s); break;
        case 34: launch_pusher<3, 4, NSP>(S, c->cfg.pusher, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t push_partials_tiled(int64_t ntiles) { return 2 * (2 * (size_t)ntiles + GLOBAL_BLOCKS); }

// Arguments of one species' push; scratch from ps, or the context's own
static TiledArgs tiled_args(Ctx *c, const pic_species *sp, const pic_particles *p, const pic_fields *f,
                            const PushScratch &ps) {
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
    a.w = (float *)p->w;
    a.absorb_x = absorbing_x(cfg);
    a.w0 = (float)sp->w0;
    a.chi = cfg.hbar_omega_mc2 > 0.0 ? p->chi : nullptr;
    a.chi_scale = (float)cfg.hbar_omega_mc2;
    a.tile_start = p->tile_start;
    a.n = p->n;
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
    a.strag_count = ps.strag_count ? ps.strag_count : c->status + 4;
    a.partials = ps.partials;
    a.strag_list = ps.strag_list;
    a.strag_tile = ps.strag_tile;
    a.bin_list = ps.bin_list;
    a.bin_rank = ps.bin_rank;
    a.bin_start = ps.bin_start;
    a.bin_count = ps.bin_count;
    a.bin_wmax = ps.bin_wmax;
    return a;
}

hipError_t launch_gpd_tiled(Ctx *c, const pic_species *sp, const pic_particles *p,
                            const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps) {
    const size_t nblocks = 2 * (size_t)c->ntiles + GLOBAL_BLOCKS;
    PushScratch own;
    if (!ps) {
        if (ensure_partials(c, push_partials_tiled(c->ntiles)) != PIC_OK) return hipErrorOutOfMemory;
        if (ensure_strag_list(c, p->n) != PIC_OK) return hipErrorOutOfMemory;
        own.partials = c->partials;
        own.strag_list = c->strag_list;
        own.strag_tile = c->strag_tile;
        own.bin_list = c->bin_list;
        own.bin_rank = c->bin_rank;
        own.bin_start = c->bin_start;
        own.bin_count = c->bin_count;
        own.bin_wmax = c->bin_wmax;
        ps = &own;
    }
    TiledSet<1> S;
    S.sp[0] = tiled_args(c, sp, p, f, *ps);
    S.nsp = 1;
    hipError_t e = launch_set<1>(c, S, c->lds_bytes, s);
    if (e != hipSuccess || !diag) return e;
    return launch_finalize(S.sp[0].partials, (int64_t)nblocks, 2, diag, 0, 1.0, s);
}

hipError_t launch_gpd_tiled_multi(Ctx *c, int nsp, const pic_species *sp, const pic_particles *const *p,
                                  const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps) {
    if (nsp < 1 || nsp > PIC_MAX_SPECIES) return hipErrorInvalidValue;
    const size_t nblocks = 2 * (size_t)c->ntiles + GLOBAL_BLOCKS;
    TiledSet<PIC_MAX_SPECIES> S{};
    for (int k = 0; k < nsp; ++k) S.sp[k] = tiled_args(c, &sp[k], p[k], f, ps[k]);
    S.nsp = nsp;
    hipError_t e = launch_set<PIC_MAX_SPECIES>(c, S, c->lds_bytes, s);
    for (int k = 0; k < nsp && e == hipSuccess && diag; ++k)
        e = launch_finalize(S.sp[k].partials, (int64_t)nblocks, 2, diag, 0, 1.0, s);
    return e;
}

template <int DIM, int ORDER, int PUSH, int NT, int WX, int WY, int WZ, int NSP>
static hipError_t set_lds_n(size_t bytes) {
    hipError_t e =
        hipFuncSetAttribute((const void *)gpd_tiled_kernel<DIM, ORDER, PUSH, NT, WX, WY, WZ, false, false, NSP>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)gpd_tiled_kernel<DIM, ORDER, PUSH, NT, WX, WY, WZ, true, false, NSP>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int DIM, int ORDER, int PUSH, int NT, int WX, int WY, int WZ>
static hipError_t set_lds_p(size_t bytes) {
    hipError_t e = set_lds_n<DIM, ORDER, PUSH, NT, WX, WY, WZ, 1>(bytes);
    if (e != hipSuccess) return e;
    return set_lds_n<DIM, ORDER, PUSH, NT, WX, WY, WZ, PIC_MAX_SPECIES>(bytes);
}

template <int DIM, int ORDER, int NT, int WX, int WY, int WZ>
static hipError_t set_lds(size_t bytes) {
    hipError_t e = set_lds_p<DIM, ORDER, PIC_PUSH_BORIS, NT, WX, WY, WZ>(bytes);
    if (e != hipSuccess) return e;
    return set_lds_p<DIM, ORDER, PIC_PUSH_VAY, NT, WX, WY, WZ>(bytes);
}

hipError_t set_tiled_lds_limit(size_t bytes) {
    hipError_t e = set_lds<2, 1, PIC_TILED_THREADS_2D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<2, 2, PIC_TILED_THREADS_2D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<3, 1, PIC_TILED_THREADS_3D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<3, 2, PIC_TILED_THREADS_3D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<2, 4, PIC_TILED_THREADS_2D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<3, 4, PIC_TILED_THREADS_3D, 0, 0, 0>(bytes);
    if (e == hipSuccess) e = set_lds<2, 4, PIC_TILED_THREADS_2D, W2X4, W2X4, 1>(bytes);
    if (e == hipSuccess) e = set_lds<3, 4, PIC_TILED_THREADS_3D, W3X, W3X, W3Z>(bytes);
    if (e == hipSuccess) e = set_lds<2, 1, PIC_TILED_THREADS_2D, W2X, W2X, 1>(bytes);
    if (e == hipSuccess) e = set_lds<2, 2, PIC_TILED_THREADS_2D, W2X, W2X, 1>(bytes);
    if (e == hipSuccess) e = set_lds<3, 1, PIC_TILED_THREADS_3D, W3X, W3X, W3Z>(bytes);
    if (e == hipSuccess) e = set_lds<3, 2, PIC_TILED_THREADS_3D, W3X, W3X, W3Z>(bytes);
    if (e == hipSuccess) e = set_lds<3, 2, PIC_TILED_THREADS_3D, W3X0, W3X0, W3Z0>(bytes);
    if (e == hipSuccess) e = set_lds<3, 2, PIC_TILED_THREADS_3D, W3C0, W3C0, W3C0>(bytes);
    return e;
}

}  // namespace pic
