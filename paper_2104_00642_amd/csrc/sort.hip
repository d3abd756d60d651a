// sort.hip -- tile binning of the FP32 particles (pic_sort).
//
// Order produced: (tile, rank of the particle among those of its cell in the
// source order, key of the cell within the tile; see local_key).  Steps:
//   1. key = tile id of the particle's cell;
//   2. stable LSD radix sort of the tile keys (8-bit digits: per-block digit
//      histograms, one device-wide exclusive scan, stable scatter with ranks
//      inside a wavefront from 8 ballots and across wavefronts from an LDS
//      prefix).  Input that is already tile-ordered (every sort after the
//      first) keeps long runs, so the scatter stays coalesced;
//   3. tile_start from the key boundaries;
//   4. one workgroup per tile: counts per cell, stable rank of each particle
//      within its cell (same ballot ranking, in source order), then layer r of
//      the r-th particles of every populated cell, cells ascending, gathering
//      every particle array straight into the destination.
// All integer work: the permutation is deterministic and bit-exact.
#include <algorithm>

#include "device_common.h"
#include "pic_internal.h"

namespace pic {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 16;
constexpr int SORT_ITEMS = SORT_THREADS * SORT_ROUNDS;  // keys per block

struct SortGeom {
    int dim;
    int bx, by;
    int tile[3];
    int ntile_axis[3];
    int ct;            // cells per tile
    int cls_start[8];  // first key of each parity class of cells
};

// Key of a cell inside its tile (li, lj, lk tile-local): cells are grouped by
// the parities of their coordinates, classes taken in an order where
// consecutive classes differ in as many parities as possible, and by the
// coarse position (li/2, lj/2, lk/2) inside a class.  Two cells of one class
// are at least two cells apart along some axis, so the stencils of particles
// that share a wavefront seldom start on the same node and their LDS current
// atomics seldom hit the same address.
__device__ __forceinline__ uint32_t local_key(int li, int lj, int lk, const SortGeom &g) {
    const int px = li & 1, py = lj & 1, pz = lk & 1;
    const int nx = (g.tile[0] + 1 - px) >> 1;  // cells of parity px along x
    const int ny = (g.tile[1] + 1 - py) >> 1;
    return (uint32_t)(g.cls_start[px | (py << 1) | (pz << 2)] + (li >> 1) + nx * ((lj >> 1) + ny * (lk >> 1)));
}

__device__ __forceinline__ void decode_cell(int32_t c, const SortGeom &g, int &ix, int &iy, int &iz) {
    const int mx = (1 << g.bx) - 1, my = (1 << g.by) - 1;
    ix = c & mx;
    iy = (c >> g.bx) & my;
    iz = g.dim == 3 ? (c >> (g.bx + g.by)) : 0;
}

// A packed cell off the grid (x or y field beyond the cell count, or bits
// above y that are not a z inside the grid: any in 2D, a negative cell) gets
// the key ntiles: such particles follow the last tile in source order, where
// the push flags them and leaves them unchanged.
__device__ __forceinline__ uint32_t tile_key(int32_t c, const SortGeom &g) {
    int ix, iy, iz;
    decode_cell(c, g, ix, iy, iz);
    const uint32_t above = (uint32_t)(c >> (g.bx + g.by));
    const bool ok = (unsigned)ix < (unsigned)(g.tile[0] * g.ntile_axis[0]) &&
                    (unsigned)iy < (unsigned)(g.tile[1] * g.ntile_axis[1]) &&
                    above < (uint32_t)(g.dim == 3 ? g.tile[2] * g.ntile_axis[2] : 1);
    const int tx = ix / g.tile[0], ty = iy / g.tile[1], tz = g.dim == 3 ? (int)above / g.tile[2] : 0;
    return ok ? (uint32_t)(tx + g.ntile_axis[0] * (ty + g.ntile_axis[1] * tz))
              : (uint32_t)(g.ntile_axis[0] * g.ntile_axis[1] * g.ntile_axis[2]);
}

__global__ void __launch_bounds__(256) sort_keys_kernel(const int32_t *cell, int64_t n, SortGeom g,
                                                        uint32_t *keys) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    keys[p] = tile_key(cell[p], g);
}

// Digit histogram of keys [lo, hi) into the LDS counters h (one call per
// block; lo and hi are uniform over the block).
__device__ __forceinline__ void radix_hist_range(const uint32_t *keys, int64_t lo, int64_t hi, int shift,
                                                 uint32_t *h) {
    const int lane = threadIdx.x & 63;
    for (int64_t b0 = lo; b0 < hi; b0 += SORT_THREADS) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t d = i < hi ? (keys[i] >> shift) & 255u : 0u;
        bool pending = i < hi;
        // The keys arrive nearly sorted (particles rarely change tiles between
        // sorts), so a wavefront holds few distinct digits, and LDS atomics on
        // one address serialize: lanes with equal digits add once per group.
        // After four groups the remaining lanes add one by one.
        for (int k = 0; k < 4; ++k) {
            const uint64_t act = __ballot(pending);
            if (act == 0) break;
            const int lead = __ffsll((unsigned long long)act) - 1;
            const uint32_t d0 = (uint32_t)__shfl((int)d, lead);
            const uint64_t same = __ballot(pending && d == d0);
            if (lane == lead) atomicAdd(&h[d0], (uint32_t)__popcll(same));
            if (d == d0) pending = false;
        }
        if (pending) atomicAdd(&h[d], 1u);
    }
}

// Share of block b of a grid over a count held on the device: consecutive
// ranges, a multiple of SORT_THREADS long.
__device__ __forceinline__ void device_share(const uint32_t *count, int64_t &lo, int64_t &hi) {
    const int64_t n = *count;
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    per = (per + SORT_THREADS - 1) / SORT_THREADS * SORT_THREADS;
    lo = min((int64_t)blockIdx.x * per, n);
    hi = min(lo + per, n);
}

// KIN_DEV = false: block b takes keys [b SORT_ITEMS, (b+1) SORT_ITEMS) of n;
// true: its share of the count *count.  hist is digit-major: hist[d G + b].
template <bool KIN_DEV>
__global__ void __launch_bounds__(SORT_THREADS) radix_hist_kernel(const uint32_t *keys, int64_t n,
                                                                  const uint32_t *count, int shift,
                                                                  uint32_t *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t lo, hi;
    if (KIN_DEV) {
        device_share(count, lo, hi);
    } else {
        lo = (int64_t)blockIdx.x * SORT_ITEMS;
        hi = min(lo + SORT_ITEMS, n);
    }
    radix_hist_range(keys, lo, hi, shift, h);
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// ---- device-wide exclusive scan of uint32 (chunks of SORT_ITEMS) --------

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t &total) {
    // tmp: 256 entries
    const int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t add = t >= off ? tmp[t - off] : 0u;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    total = tmp[255];
    uint32_t incl = tmp[t];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(256) scan_sums_kernel(const uint32_t *a, int64_t n, uint32_t *sums) {
    __shared__ uint32_t tmp[256];
    const int64_t start = (int64_t)blockIdx.x * SORT_ITEMS;
    uint32_t s = 0;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t i = start + (int64_t)threadIdx.x * SORT_ROUNDS + r;
        if (i < n) s += a[i];
    }
    uint32_t total;
    block_exclusive_scan(s, tmp, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of `m` chunk sums in place
__global__ void __launch_bounds__(256) scan_top_kernel(uint32_t *sums, int64_t m) {
    __shared__ uint32_t tmp[256];
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += 256) {
        const int64_t i = base + threadIdx.x;
        uint32_t v = i < m ? sums[i] : 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(v, tmp, total);
        if (i < m) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(256) scan_apply_kernel(uint32_t *a, int64_t n, const uint32_t *sums) {
    __shared__ uint32_t tmp[256];
    const int64_t start = (int64_t)blockIdx.x * SORT_ITEMS;
    uint32_t v[SORT_ROUNDS];
    uint32_t s = 0;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t i = start + (int64_t)threadIdx.x * SORT_ROUNDS + r;
        v[r] = i < n ? a[i] : 0u;
        s += v[r];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan(s, tmp, total) + sums[blockIdx.x];
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t i = start + (int64_t)threadIdx.x * SORT_ROUNDS + r;
        if (i < n) a[i] = ex;
        ex += v[r];
    }
}

static hipError_t exclusive_scan(Ctx *c, uint32_t *a, int64_t n, uint32_t *sums, hipStream_t s) {
    const int64_t nb = (n + SORT_ITEMS - 1) / SORT_ITEMS;
    scan_sums_kernel<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
    scan_top_kernel<<<1, 256, 0, s>>>(sums, nb);
    scan_apply_kernel<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
    (void)c;
    return hipGetLastError();
}

// ---- stable scatter ------------------------------------------------------

template <bool KIN_DEV>
__global__ void __launch_bounds__(SORT_THREADS) radix_scatter_kernel(
    const uint32_t *kin, const uint32_t *vin, int64_t n, const uint32_t *count, int shift,
    const uint32_t *offs, uint32_t *kout, uint32_t *vout) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[SORT_THREADS / 64][256];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    base[t] = offs[(int64_t)t * gridDim.x + blockIdx.x];
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t lo, hi;
    if (KIN_DEV) {
        device_share(count, lo, hi);
    } else {
        lo = (int64_t)blockIdx.x * SORT_ITEMS;
        hi = min(lo + SORT_ITEMS, n);
    }
    for (int64_t b0 = lo; b0 < hi; b0 += SORT_THREADS) {
        const int64_t i = b0 + t;
        const bool valid = i < hi;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < SORT_THREADS / 64; ++w) wcnt[w][t] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        if (valid && rank == 0) wcnt[wave][d] = cnt;
        __syncthreads();
        {
            uint32_t run = base[t];
#pragma unroll
            for (int w = 0; w < SORT_THREADS / 64; ++w) {
                const uint32_t c = wcnt[w][t];
                wcnt[w][t] = run;
                run += c;
            }
            base[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wave][d] + rank;
            kout[pos] = key;
            vout[pos] = vin ? vin[i] : (uint32_t)i;
        }
        __syncthreads();
    }
}

// ---- tile boundaries -----------------------------------------------------

__global__ void __launch_bounds__(256) tile_bounds_kernel(const uint32_t *keys, int64_t n,
                                                          int64_t ntiles, int64_t *tile_start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    // keys are at most ntiles (off-grid particles); the clamps keep every
    // write inside the ntiles + 1 entries whatever the keys hold
    const int64_t tprev = i == 0 ? -1 : min((int64_t)keys[i - 1], ntiles);
    const int64_t tcur = i == n ? ntiles : min((int64_t)keys[i], ntiles);
    for (int64_t t = tprev + 1; t <= tcur; ++t) tile_start[t] = i;
}

// ---- per tile: stable in-cell ranks, layer order, gather into dst --------

// Particle arrays moved by the sort as 32-bit columns: a 4-byte array is one
// column (stride 1), an 8-byte array two (stride 2, word 0 and word 1).
constexpr int SORT_MAX_COLS = 16;
struct PermArgs {
    const int32_t *cell_in;
    const uint32_t *src[SORT_MAX_COLS];
    uint32_t *dst[SORT_MAX_COLS];
    int stride[SORT_MAX_COLS];
    int ncol;
};

// Off-grid particles [tile_start[ntiles], n) (key ntiles): copied in the
// order of the sorted keys, which the stable radix sort left in source order
// (vals: source indices).  Normally there are none.
__global__ void __launch_bounds__(256) tail_copy_kernel(const uint32_t *vals, const int64_t *tile_start,
                                                        int64_t ntiles, int64_t n, PermArgs pa) {
    const int64_t first = min(tile_start[ntiles], n);
    for (int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = vals[i];
        for (int col = 0; col < pa.ncol; ++col) {
            const int sd = pa.stride[col];
            pa.dst[col][i * sd] = pa.src[col][v * sd];
        }
    }
}

// phases A and D issue the loads of SORT_AHEAD rounds before using them
constexpr int SORT_AHEAD = 4;
// entries per thread that phase D keeps in registers for a one-stage tile
constexpr int PERM_REG = 12;
// entries per thread of the two-columns-per-round path
constexpr int PAIR_REG = 6;

// Layers of phase C handled per pass: R layers x (cells/64) group counters
// stay within 16 KB of LDS.
__host__ __device__ inline int sort_layer_chunk(int ct) {
    const int ng = (ct + 63) / 64;
    const int r = 4096 / ng;
    return r < 1 ? 1 : (r > 256 ? 256 : r);
}

constexpr int ORDER_THREADS = 1024;  // one workgroup per tile
constexpr int ORDER_WAVES = ORDER_THREADS / 64;

// wavefronts that rank particles in phase A: their per-cell counters take
// at most 64 KB
__host__ __device__ inline int sort_rank_waves(int ct) {
    const int w = 16384 / ct;
    return w < 1 ? 1 : (w > ORDER_WAVES ? ORDER_WAVES : w);
}

static size_t sort_lds_words_abc(int ct) {
    const int ng = (ct + 63) / 64;
    return (size_t)(sort_rank_waves(ct) + 2) * ct + (size_t)sort_layer_chunk(ct) * ng + 256 + 64;
}

// particles per LDS stage of phase D: the largest multiple of 1024 that keeps
// the workgroup within 80 KB (two workgroups per CU; at least 1024)
static int sort_stage_len(int ct) {
    const long words = 80 * 1024 / 4 - (long)sort_lds_words_abc(ct);
    long seg = words;
    seg -= seg % 1024;
    return (int)(seg < 1024 ? 1024 : (seg > 16384 ? 16384 : seg));
}

size_t sort_lds_bytes(int ct) {
    return sizeof(uint32_t) * (sort_lds_words_abc(ct) + (size_t)sort_stage_len(ct));
}

// exclusive scan over the ORDER_THREADS threads (wave prefix by shuffles,
// then the wave totals); `wt` holds ORDER_WAVES + 1 words of LDS
__device__ __forceinline__ uint32_t order_exscan(uint32_t v, uint32_t *wt, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wt[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < ORDER_WAVES; ++w) {
            const uint32_t c = wt[w];
            wt[w] = run;
            run += c;
        }
        wt[ORDER_WAVES] = run;
    }
    __syncthreads();
    total = wt[ORDER_WAVES];
    const uint32_t r = wt[wave] + x - v;
    __syncthreads();
    return r;
}

// Per-entry scratch of tile_order_kernel: the cell key and in-cell rank of
// every entry of the tile (the rank later replaced by the final position),
// and the final position of every cell-order slot.  In global memory
// (indexed like the sorted arrays), or, for a tile of at most
// order_lds_entries(seg) entries, as 16-bit words in LDS indexed from the
// tile's first entry: the ranks after the fixed arrays, then the cell keys
// and slot positions, whose space later stages the columns.
template <bool LDS>
struct OrderScratch;
template <>
struct OrderScratch<false> {
    uint32_t *lcell, *lrank, *posmap;
    int64_t ts;
    __device__ __forceinline__ uint32_t cell(int64_t i) const { return lcell[i]; }
    __device__ __forceinline__ void set_cell(int64_t i, uint32_t v) const { lcell[i] = v; }
    __device__ __forceinline__ uint32_t rank(int64_t i) const { return lrank[i]; }
    __device__ __forceinline__ void set_rank(int64_t i, uint32_t v) const { lrank[i] = v; }
    __device__ __forceinline__ uint32_t pos(uint32_t slot) const { return posmap[ts + slot]; }
    __device__ __forceinline__ void set_pos(uint32_t slot, uint32_t v) const { posmap[ts + slot] = v; }
};
template <>
struct OrderScratch<true> {
    uint16_t *lk, *lr, *pm;
    int64_t ts;
    __device__ __forceinline__ uint32_t cell(int64_t i) const { return lk[i - ts]; }
    __device__ __forceinline__ void set_cell(int64_t i, uint32_t v) const { lk[i - ts] = (uint16_t)v; }
    __device__ __forceinline__ uint32_t rank(int64_t i) const { return lr[i - ts]; }
    __device__ __forceinline__ void set_rank(int64_t i, uint32_t v) const { lr[i - ts] = (uint16_t)v; }
    __device__ __forceinline__ uint32_t pos(uint32_t slot) const { return pm[slot]; }
    __device__ __forceinline__ void set_pos(uint32_t slot, uint32_t v) const { pm[slot] = (uint16_t)v; }
};

// entries of a tile whose scratch fits the LDS stage of `seg` words: 16-bit
// ranks (half a word each) plus 16-bit keys and slot positions (a word per
// entry, later the staged column); a multiple of 64, below 2^16
__host__ __device__ inline int order_lds_entries(int seg) {
    const int e = (2 * seg / 3) & ~63;
    return e < 65536 ? e : 65472;
}

// One workgroup of ORDER_THREADS per tile.
//   A. each of the first RW wavefronts ranks the particles of its contiguous
//      share of the tile within their cells (8 ballots match equal cells; the
//      wavefront keeps private per-cell counters, so no barrier is needed);
//   B. per cell: count, base of each wavefront's share, first slot in cell
//      order;
//   C. layer r holds the r-th particle of every cell with more than r, cells
//      in key order: its start is the number of particles in earlier layers,
//      and a cell's place in it the number of populated cells before it,
//      both from ballots over groups of 64 cells; the final position of each
//      cell-order slot goes to posmap;
//   D. final position of every particle, then the particle arrays one
//      column at a time: read in source order (the radix sort is stable, so
//      a tile's sources ascend and the reads are nearly sequential), placed
//      at their final position in LDS, written out contiguously.
// Loads of SORT_AHEAD rounds are issued before they are used.
template <bool LDS>
__device__ __forceinline__ void order_tile(const uint32_t *vals, int64_t ts, int64_t te, const SortGeom &g, int lbits,
                                           int seg, uint32_t *lcell, uint32_t *lrank, uint32_t *posmap,
                                           const PermArgs &pa, uint32_t *sm, uint32_t &maxc_s) {
    const int ct = g.ct;
    const int ng = (ct + 63) >> 6;
    const int R = sort_layer_chunk(ct);
    const int RW = sort_rank_waves(ct);
    uint32_t *wcnt = sm;              // RW x ct: per-wavefront counts, then bases
    uint32_t *cnt = sm + RW * ct;     // ct: particles per cell
    uint32_t *cst = cnt + ct;         // ct: first cell-order slot of each cell
    uint32_t *gc = cst + ct;          // R x ng: populated cells per group and layer, then offsets
    uint32_t *lb = gc + R * ng;       // R: first position of each layer of the pass
    uint32_t *wt = lb + 256;          // ORDER_WAVES + 1: scan of wave totals
    uint32_t *stage = wt + 64;        // seg: a staged column
    OrderScratch<LDS> sc;
    if constexpr (LDS) {
        const int ne = order_lds_entries(seg);
        sc.lr = (uint16_t *)stage;
        sc.lk = (uint16_t *)(stage + ne / 2);
        sc.pm = sc.lk + ne;
        stage += ne / 2;  // the keys' and slot positions' space, once they are used
    } else {
        sc.lcell = lcell;
        sc.lrank = lrank;
        sc.posmap = posmap;
    }
    sc.ts = ts;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t n_t = te - ts;
    const int64_t cw = ((n_t + 64 * RW - 1) / (64 * RW)) * 64;  // share of one ranking wavefront
    const int64_t c0 = ts + wave * cw, c1 = wave < RW ? min(c0 + cw, te) : c0;
    for (int e = threadIdx.x; e < RW * ct; e += ORDER_THREADS) wcnt[e] = 0;
    if (threadIdx.x == 0) maxc_s = 0;
    __syncthreads();

    // A. rank within the cell inside the wavefront's share (source order)
    if (wave < RW) {
        uint32_t *wc = wcnt + wave * ct;
        for (int64_t base = c0; base < c1; base += 64 * SORT_AHEAD) {
            uint32_t lk[SORT_AHEAD];
            int32_t ce[SORT_AHEAD];
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q) {
                const int64_t i = base + q * 64 + lane;
                ce[q] = i < c1 ? pa.cell_in[vals[i]] : 0;
            }
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q) {
                int ix, iy, iz;
                decode_cell(ce[q], g, ix, iy, iz);
                lk[q] = local_key(ix % g.tile[0], iy % g.tile[1], iz % g.tile[2], g);
            }
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q) {
                const int64_t i = base + q * 64 + lane;
                const bool valid = i < c1;
                const uint32_t l = lk[q];
                uint64_t peers = __ballot(valid);
                for (int b = 0; b < lbits; ++b) {
                    const uint64_t m = __ballot((l >> b) & 1u);
                    peers &= ((l >> b) & 1u) ? m : ~m;
                }
                const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
                uint32_t prev = 0;
                if (valid) prev = wc[l];
                // every lane has read its cell's counter before the first lane
                // of each group of equal cells advances it (LDS keeps a
                // wavefront's order)
                __builtin_amdgcn_wave_barrier();
                if (valid && rank == 0) wc[l] = prev + (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
                if (valid) {
                    sc.set_cell(i, l);
                    sc.set_rank(i, prev + rank);
                }
            }
        }
    }
    __syncthreads();

    // B. counts, wavefront bases, cell-order slots
    const int per = (ct + ORDER_THREADS - 1) / ORDER_THREADS;
    uint32_t loc = 0, mx = 0;
    for (int q = 0; q < per; ++q) {
        const int l = threadIdx.x * per + q;
        if (l < ct) {
            uint32_t run = 0;
            for (int w = 0; w < RW; ++w) {
                const uint32_t c = wcnt[w * ct + l];
                wcnt[w * ct + l] = run;
                run += c;
            }
            cnt[l] = run;
            loc += run;
            mx = max(mx, run);
        }
    }
    atomicMax(&maxc_s, mx);
    uint32_t total;
    uint32_t ex = order_exscan(loc, wt, total);
    for (int q = 0; q < per; ++q) {
        const int l = threadIdx.x * per + q;
        if (l < ct) {
            cst[l] = ex;
            ex += cnt[l];
        }
    }
    __syncthreads();

    // C. layers, R at a time
    const uint32_t maxc = maxc_s;
    uint32_t lcarry = 0;
    for (uint32_t r0 = 0; r0 < maxc; r0 += (uint32_t)R) {
        const uint32_t rr = min((uint32_t)R, maxc - r0);
        for (int gi = wave; gi < ng; gi += ORDER_WAVES) {
            const int l = gi * 64 + lane;
            const uint32_t c = l < ct ? cnt[l] : 0u;
            for (uint32_t r = 0; r < rr; ++r) {
                const uint64_t b = __ballot(c > r0 + r);
                if (lane == 0) gc[r * ng + gi] = (uint32_t)__popcll(b);
            }
        }
        __syncthreads();
        uint32_t tot = 0;
        if (threadIdx.x < rr) {
            uint32_t run = 0;
            for (int gi = 0; gi < ng; ++gi) {
                const uint32_t c = gc[threadIdx.x * ng + gi];
                gc[threadIdx.x * ng + gi] = run;
                run += c;
            }
            tot = run;
        }
        uint32_t all;
        const uint32_t lex = order_exscan(tot, wt, all);
        if (threadIdx.x < rr) lb[threadIdx.x] = lcarry + lex;
        lcarry += all;
        __syncthreads();
        for (int gi = wave; gi < ng; gi += ORDER_WAVES) {
            const int l = gi * 64 + lane;
            const uint32_t c = l < ct ? cnt[l] : 0u;
            for (uint32_t r = 0; r < rr; ++r) {
                const bool has = c > r0 + r;
                const uint64_t b = __ballot(has);
                if (has) sc.set_pos(cst[l] + r0 + r, lb[r] + gc[r * ng + gi] + (uint32_t)__popcll(b & lt_mask));
            }
        }
        __syncthreads();
    }

    // D. final position of each particle (in place of its in-cell rank)
    if (wave < RW) {
        for (int64_t i0 = c0 + lane; i0 < c1; i0 += 64 * SORT_AHEAD) {
            uint32_t slot[SORT_AHEAD], pos[SORT_AHEAD];
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q) {
                const int64_t i = i0 + q * 64;
                if (i < c1) {
                    const uint32_t l = sc.cell(i);
                    slot[q] = cst[l] + wcnt[wave * ct + l] + sc.rank(i);
                }
            }
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q)
                if (i0 + q * 64 < c1) pos[q] = sc.pos(slot[q]);
#pragma unroll
            for (int q = 0; q < SORT_AHEAD; ++q)
                if (i0 + q * 64 < c1) sc.set_rank(i0 + q * 64, pos[q]);
        }
    }
    __syncthreads();
    //    columns through LDS.  A tile that fits one stage and PERM_REG
    //    entries per thread keeps its entries' final positions and sources
    //    in registers across the columns (read once, not once per column);
    //    larger tiles go `seg` final positions at a time.  A tile of at most
    //    PAIR_REG entries per thread (the 3D tiles) moves two columns per
    //    round: the second stages in the per-wavefront counters' space, free
    //    once the positions are known, so each round has twice the loads in
    //    flight and the rounds of barriers and write-outs halve.
    if (n_t <= (int64_t)seg && n_t <= (int64_t)PAIR_REG * ORDER_THREADS && n_t <= (int64_t)RW * ct) {
        uint32_t *stage2 = wcnt;
        uint32_t pos[PAIR_REG], v[PAIR_REG];
#pragma unroll
        for (int u = 0; u < PAIR_REG; ++u) {
            const int64_t i = ts + threadIdx.x + (int64_t)u * ORDER_THREADS;
            pos[u] = i < te ? sc.rank(i) : 0xFFFFFFFFu;
            v[u] = i < te ? vals[i] : 0u;
        }
        for (int col = 0; col < pa.ncol; col += 2) {
            const bool two = col + 1 < pa.ncol;
            const uint32_t *src0 = pa.src[col], *src1 = pa.src[two ? col + 1 : col];
            const int sd0 = pa.stride[col], sd1 = pa.stride[two ? col + 1 : col];
            uint32_t x0[PAIR_REG], x1[PAIR_REG];
#pragma unroll
            for (int u = 0; u < PAIR_REG; ++u)
                if (pos[u] != 0xFFFFFFFFu) {
                    x0[u] = src0[(int64_t)v[u] * sd0];
                    if (two) x1[u] = src1[(int64_t)v[u] * sd1];
                }
#pragma unroll
            for (int u = 0; u < PAIR_REG; ++u)
                if (pos[u] != 0xFFFFFFFFu) {
                    stage[pos[u]] = x0[u];
                    if (two) stage2[pos[u]] = x1[u];
                }
            __syncthreads();
            uint32_t *d0 = pa.dst[col] + ts * sd0;
            for (uint32_t j = threadIdx.x; j < (uint32_t)n_t; j += ORDER_THREADS) d0[(int64_t)j * sd0] = stage[j];
            if (two) {
                uint32_t *d1 = pa.dst[col + 1] + ts * sd1;
                for (uint32_t j = threadIdx.x; j < (uint32_t)n_t; j += ORDER_THREADS) d1[(int64_t)j * sd1] = stage2[j];
            }
            __syncthreads();
        }
        return;
    }
    if (n_t <= (int64_t)seg && n_t <= (int64_t)PERM_REG * ORDER_THREADS) {
        uint32_t pos[PERM_REG], v[PERM_REG];
#pragma unroll
        for (int u = 0; u < PERM_REG; ++u) {
            const int64_t i = ts + threadIdx.x + (int64_t)u * ORDER_THREADS;
            pos[u] = i < te ? sc.rank(i) : 0xFFFFFFFFu;
            v[u] = i < te ? vals[i] : 0u;
        }
        for (int col = 0; col < pa.ncol; ++col) {
            const uint32_t *src = pa.src[col];
            const int sd = pa.stride[col];
            uint32_t x[PERM_REG];
#pragma unroll
            for (int u = 0; u < PERM_REG; ++u)
                if (pos[u] != 0xFFFFFFFFu) x[u] = src[(int64_t)v[u] * sd];
#pragma unroll
            for (int u = 0; u < PERM_REG; ++u)
                if (pos[u] != 0xFFFFFFFFu) stage[pos[u]] = x[u];
            __syncthreads();
            uint32_t *d = pa.dst[col] + ts * sd;
            for (uint32_t j = threadIdx.x; j < (uint32_t)n_t; j += ORDER_THREADS) d[(int64_t)j * sd] = stage[j];
            __syncthreads();
        }
        return;
    }
    for (int64_t s0 = 0; s0 < n_t; s0 += seg) {
        const uint32_t len = (uint32_t)min((int64_t)seg, n_t - s0);
        for (int col = 0; col < pa.ncol; ++col) {
            const uint32_t *src = pa.src[col];
            const int sd = pa.stride[col];
            for (int64_t i0 = ts + threadIdx.x; i0 < te; i0 += SORT_AHEAD * ORDER_THREADS) {
                uint32_t pos[SORT_AHEAD], v[SORT_AHEAD], x[SORT_AHEAD];
#pragma unroll
                for (int u = 0; u < SORT_AHEAD; ++u) {
                    const int64_t i = i0 + u * ORDER_THREADS;
                    pos[u] = i < te ? sc.rank(i) - (uint32_t)s0 : 0xFFFFFFFFu;
                    v[u] = i < te ? vals[i] : 0u;
                }
#pragma unroll
                for (int u = 0; u < SORT_AHEAD; ++u)
                    if (pos[u] < len) x[u] = src[(int64_t)v[u] * sd];
#pragma unroll
                for (int u = 0; u < SORT_AHEAD; ++u)
                    if (pos[u] < len) stage[pos[u]] = x[u];
            }
            __syncthreads();
            uint32_t *d = pa.dst[col] + (ts + s0) * sd;
            for (uint32_t j = threadIdx.x; j < len; j += ORDER_THREADS) d[(int64_t)j * sd] = stage[j];
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(ORDER_THREADS, 8) tile_order_kernel(const uint32_t *vals, const int64_t *tile_start,
                                                                   SortGeom g, int lbits, int seg, uint32_t *lcell,
                                                                   uint32_t *lrank, uint32_t *posmap, PermArgs pa) {
    extern __shared__ uint32_t sm[];
    __shared__ uint32_t maxc_s;
    const int t = blockIdx.x;
    const int64_t ts = tile_start[t], te = tile_start[t + 1];
    if (ts == te) return;
    if (te - ts <= order_lds_entries(seg))
        order_tile<true>(vals, ts, te, g, lbits, seg, lcell, lrank, posmap, pa, sm, maxc_s);
    else
        order_tile<false>(vals, ts, te, g, lbits, seg, lcell, lrank, posmap, pa, sm, maxc_s);
}

// ---- re-binning from the source's own tile offsets ----------------------
//
// Between sorts few particles change tiles.  When src->tile_start holds a
// partition of the source into tile segments (the offsets written by the
// sort that produced the source), a particle of segment t whose key is t
// "stays"; every other particle (another key, off the grid, outside every
// segment) "moves".  In the sorted order tile t holds, by ascending source
// index, the movers into t from before segment t, the stayers of t, then the
// movers into t from after it.  So the positions follow from the stayer
// counts and the movers sorted by (key, source index): one stable radix sort
// of the movers instead of one of every key, with the same result.  A hint
// that is not a partition (decreasing, negative, beyond n) makes every
// particle a mover: the result is still the same.

// blocks that take the particles before the first segment, and those after
// the last one
constexpr int INC_LOOSE = 256;

struct IncRange {
    int64_t lo, hi;
    int64_t seg;  // tile of the segment, -1 outside the segments
};

// Work unit u: INC_LOOSE shares of [0, h[0]), the ntiles segments, INC_LOOSE
// shares of [h[ntiles], n).  Without a valid hint the first run is [0, n).
__device__ __forceinline__ IncRange inc_range(int64_t u, const int64_t *h, int64_t ntiles, int64_t n, bool ok) {
    IncRange r;
    if (u >= INC_LOOSE && u < INC_LOOSE + ntiles) {
        const int64_t t = u - INC_LOOSE;
        r.lo = ok ? h[t] : 0;
        r.hi = ok ? h[t + 1] : 0;
        r.seg = t;
        return r;
    }
    const bool head = u < INC_LOOSE;
    const int64_t a = head ? 0 : (ok ? h[ntiles] : n);
    const int64_t b = head ? (ok ? h[0] : n) : n;
    const int64_t k = head ? u : u - INC_LOOSE - ntiles;
    int64_t per = (b - a + INC_LOOSE - 1) / INC_LOOSE;
    per = (per + SORT_THREADS - 1) / SORT_THREADS * SORT_THREADS;
    r.lo = min(a + k * per, b);
    r.hi = min(r.lo + per, b);
    r.seg = -1;
    return r;
}

// rank of a flagged thread among the flagged threads of the block (thread
// order) and their number; wt: SORT_THREADS/64 words of LDS
__device__ __forceinline__ uint32_t block_flag_rank(bool f, uint32_t *wt, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t b = __ballot(f);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) wt[wave] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < SORT_THREADS / 64; ++w) {
        const uint32_t c = wt[w];
        before += w < wave ? c : 0u;
        total += c;
    }
    __syncthreads();
    return before + (uint32_t)__popcll(b & lt);
}

// rounds of SORT_THREADS particles whose cells are loaded together
constexpr int INC_AHEAD = 8;

// flag = 1 when h is non-decreasing with h[0] >= 0 and h[ntiles] <= n
__global__ void __launch_bounds__(1024) inc_check_kernel(const int64_t *h, int64_t ntiles, int64_t n,
                                                         uint32_t *flag) {
    int bad = 0;
    for (int64_t i = threadIdx.x; i < ntiles; i += blockDim.x) bad |= h[i] > h[i + 1];
    if (threadIdx.x == 0) bad |= h[0] < 0 || h[ntiles] > n;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *flag = bad ? 0u : 1u;
}

// Per unit: stayers (into stay[t]) and movers, the movers' keys and sources
// written in source order at the start of the unit's own range of tk / ti.
__global__ void __launch_bounds__(SORT_THREADS) inc_count_kernel(const int32_t *cell, SortGeom g, const int64_t *h,
                                                                 int64_t ntiles, int64_t n, const uint32_t *flag,
                                                                 uint32_t *stay, uint32_t *mcount, uint32_t *tk,
                                                                 uint32_t *ti) {
    __shared__ uint32_t wt[SORT_THREADS / 64];
    const IncRange r = inc_range(blockIdx.x, h, ntiles, n, *flag != 0u);
    uint32_t carry = 0, nstay = 0;
    for (int64_t b0 = r.lo; b0 < r.hi; b0 += INC_AHEAD * SORT_THREADS) {
        int32_t ce[INC_AHEAD];
#pragma unroll
        for (int q = 0; q < INC_AHEAD; ++q) {
            const int64_t p = b0 + q * SORT_THREADS + threadIdx.x;
            ce[q] = p < r.hi ? cell[p] : 0;
        }
#pragma unroll
        for (int q = 0; q < INC_AHEAD; ++q) {
            const int64_t p0 = b0 + q * SORT_THREADS;
            if (p0 >= r.hi) break;  // uniform over the block
            const int64_t p = p0 + threadIdx.x;
            const bool valid = p < r.hi;
            const uint32_t key = tile_key(ce[q], g);
            const bool mv = valid && (int64_t)key != r.seg;
            uint32_t tot;
            const uint32_t rk = block_flag_rank(mv, wt, tot);
            if (mv) {
                tk[r.lo + carry + rk] = key;
                ti[r.lo + carry + rk] = (uint32_t)p;
            }
            carry += tot;
            nstay += (uint32_t)min((int64_t)SORT_THREADS, r.hi - p0) - tot;
        }
    }
    if (threadIdx.x == 0) {
        mcount[blockIdx.x] = carry;
        if (r.seg >= 0) stay[r.seg] = nstay;
        if (blockIdx.x == 0) mcount[gridDim.x] = 0u;  // the scan's last entry: the mover total
    }
}

// movers of each unit to their place in the list (moff: exclusive scan of
// the units' counts)
__global__ void __launch_bounds__(SORT_THREADS) inc_compact_kernel(const int64_t *h, int64_t ntiles, int64_t n,
                                                                   const uint32_t *flag, const uint32_t *moff,
                                                                   const uint32_t *tk, const uint32_t *ti,
                                                                   uint32_t *lk, uint32_t *li) {
    const IncRange r = inc_range(blockIdx.x, h, ntiles, n, *flag != 0u);
    const uint32_t o = moff[blockIdx.x], m = moff[blockIdx.x + 1] - o;
    for (uint32_t j = threadIdx.x; j < m; j += SORT_THREADS) {
        lk[o + j] = tk[r.lo + j];
        li[o + j] = ti[r.lo + j];
    }
}

// mstart[t] = first sorted mover with key >= t, t in [0, ntiles + 1]
__global__ void __launch_bounds__(256) inc_bounds_kernel(const uint32_t *mk, const uint32_t *count, int64_t ntiles,
                                                         uint32_t *mstart) {
    const int64_t m = *count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tprev = i == 0 ? -1 : min((int64_t)mk[i - 1], ntiles);
        const int64_t tcur = i == m ? ntiles + 1 : min((int64_t)mk[i], ntiles);
        for (int64_t t = tprev + 1; t <= tcur; ++t) mstart[t] = (uint32_t)i;
    }
}

// tile_start of the result: exclusive scan of stayers + movers per tile (one
// workgroup, chunks of 1024 x 8 tiles, in order)
__global__ void __launch_bounds__(1024) inc_tiles_kernel(const uint32_t *stay, const uint32_t *mstart,
                                                         int64_t ntiles, int64_t *ts) {
    constexpr int PER = 8;
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += 1024 * PER) {
        const int64_t lo = base + (int64_t)threadIdx.x * PER;
        int64_t v[PER];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t t = lo + k;
            v[k] = t < ntiles ? (int64_t)stay[t] + (int64_t)(mstart[t + 1] - mstart[t]) : 0;
            sum += v[k];
        }
        int64_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int64_t before = carry_s, total = carry_s;
        for (int w = 0; w < 16; ++w) {
            before += w < wave ? wsum[w] : 0;
            total += wsum[w];
        }
        int64_t run = before + x - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (lo + k < ntiles) ts[lo + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s = total;
        __syncthreads();
    }
    if (threadIdx.x == 0) ts[ntiles] = carry_s;
}

// Stayers of segment t to ts[t] + (movers into t from before the segment) +
// their rank among the segment's stayers.  mi: sorted movers' sources.
__global__ void __launch_bounds__(SORT_THREADS) inc_stayers_kernel(const int32_t *cell, SortGeom g, const int64_t *h,
                                                                   int64_t ntiles, const uint32_t *flag,
                                                                   const uint32_t *stay, const uint32_t *mstart,
                                                                   const uint32_t *mi, const int64_t *ts,
                                                                   uint32_t *vals) {
    __shared__ uint32_t wt[SORT_THREADS / 64];
    __shared__ int64_t out_s;
    const int64_t t = blockIdx.x;
    if (*flag == 0u || stay[t] == 0u) return;
    const int64_t lo = h[t], hi = h[t + 1];
    if (threadIdx.x == 0) {
        // movers into t are sorted by source: those before the segment first
        uint32_t a = mstart[t], b = mstart[t + 1];
        while (a < b) {
            const uint32_t mid = a + (b - a) / 2;
            if ((int64_t)mi[mid] < lo) a = mid + 1;
            else b = mid;
        }
        out_s = ts[t] + (int64_t)(a - mstart[t]);
    }
    __syncthreads();
    const int64_t out = out_s;
    uint32_t carry = 0;
    for (int64_t b0 = lo; b0 < hi; b0 += INC_AHEAD * SORT_THREADS) {
        int32_t ce[INC_AHEAD];
#pragma unroll
        for (int q = 0; q < INC_AHEAD; ++q) {
            const int64_t p = b0 + q * SORT_THREADS + threadIdx.x;
            ce[q] = p < hi ? cell[p] : 0;
        }
#pragma unroll
        for (int q = 0; q < INC_AHEAD; ++q) {
            const int64_t p0 = b0 + q * SORT_THREADS;
            if (p0 >= hi) break;  // uniform over the block
            const int64_t p = p0 + threadIdx.x;
            const bool st = p < hi && (int64_t)tile_key(ce[q], g) == t;
            uint32_t tot;
            const uint32_t rk = block_flag_rank(st, wt, tot);
            if (st) vals[out + carry + rk] = (uint32_t)p;
            carry += tot;
        }
    }
}

// Movers to ts[t] + their rank among the movers into t, after the stayers
// when they come from after the segment.
__global__ void __launch_bounds__(256) inc_movers_kernel(const uint32_t *mk, const uint32_t *mi, const uint32_t *count,
                                                         const uint32_t *mstart, const int64_t *ts,
                                                         const uint32_t *stay, const int64_t *h, int64_t ntiles,
                                                         const uint32_t *flag, uint32_t *vals) {
    const int64_t m = *count;
    const bool ok = *flag != 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = min((int64_t)mk[i], ntiles);
        const uint32_t src = mi[i];
        int64_t pos = ts[t] + (i - (int64_t)mstart[t]);
        if (ok && t < ntiles && (int64_t)src >= h[t]) pos += stay[t];
        vals[pos] = src;
    }
}

pic_status ensure_sort_scratch(Ctx *c, int64_t n);

// words of Ctx::inc for a grid of ntiles tiles
size_t inc_scratch_words(int64_t ntiles) {
    const int64_t units = 2 * INC_LOOSE + ntiles;
    return (size_t)(16 + ntiles + (units + 1) + ((units + 1 + SORT_ITEMS - 1) / SORT_ITEMS + 16) + (ntiles + 2) + 16);
}

// Source order (vals[cur]) and dst->tile_start from the source's tile offsets
// (see inc_range): stayer counts, the movers listed in source order and
// sorted by key, then both placed.
static hipError_t rebin_from_hint(Ctx *c, const pic_particles *src, const pic_particles *dst, const SortGeom &g,
                                  hipStream_t s, int &cur) {
    const int64_t n = src->n, nt = c->ntiles;
    const int64_t units = 2 * INC_LOOSE + nt;
    uint32_t *flag = c->inc;
    uint32_t *stay = c->inc + 16;                                  // nt
    uint32_t *mcount = stay + nt;                                  // units + 1, then their exclusive scan
    uint32_t *msums = mcount + units + 1;
    uint32_t *mstart = msums + (units + 1 + SORT_ITEMS - 1) / SORT_ITEMS + 16;  // nt + 2
    const int64_t *h = src->tile_start;
    inc_check_kernel<<<1, 1024, 0, s>>>(h, nt, n, flag);
    inc_count_kernel<<<(unsigned)units, SORT_THREADS, 0, s>>>(src->cell, g, h, nt, n, flag, stay, mcount,
                                                              c->keys[0], c->vals[0]);
    hipError_t e = exclusive_scan(c, mcount, units + 1, msums, s);
    if (e != hipSuccess) return e;
    inc_compact_kernel<<<(unsigned)units, SORT_THREADS, 0, s>>>(h, nt, n, flag, mcount, c->keys[0], c->vals[0],
                                                                c->keys[1], c->vals[1]);
    const uint32_t *m_dev = mcount + units;  // number of movers
    int bits = 0;
    while ((1ll << bits) <= nt) ++bits;
    const int passes = bits == 0 ? 1 : (bits + 7) / 8;
    const int64_t G = std::min<int64_t>((n + SORT_ITEMS - 1) / SORT_ITEMS, 4096);
    int in = 1;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        radix_hist_kernel<true><<<(unsigned)G, SORT_THREADS, 0, s>>>(c->keys[in], 0, m_dev, shift, c->hist);
        e = exclusive_scan(c, c->hist, 256 * G, c->hist + 256 * G, s);
        if (e != hipSuccess) return e;
        radix_scatter_kernel<true><<<(unsigned)G, SORT_THREADS, 0, s>>>(c->keys[in], c->vals[in], 0, m_dev, shift,
                                                                        c->hist, c->keys[in ^ 1], c->vals[in ^ 1]);
        in ^= 1;
    }
    const unsigned gb = (unsigned)std::min<int64_t>((n + 1 + 255) / 256, 2048);
    inc_bounds_kernel<<<gb, 256, 0, s>>>(c->keys[in], m_dev, nt, mstart);
    inc_tiles_kernel<<<1, 1024, 0, s>>>(stay, mstart, nt, dst->tile_start);
    inc_stayers_kernel<<<(unsigned)nt, SORT_THREADS, 0, s>>>(src->cell, g, h, nt, flag, stay, mstart, c->vals[in],
                                                             dst->tile_start, c->vals[in ^ 1]);
    inc_movers_kernel<<<gb, 256, 0, s>>>(c->keys[in], c->vals[in], m_dev, mstart, dst->tile_start, stay, h, nt, flag,
                                        c->vals[in ^ 1]);
    cur = in ^ 1;
    return hipGetLastError();
}

hipError_t launch_sort(Ctx *c, const pic_particles *src, const pic_particles *dst, hipStream_t s) {
    const int64_t n = src->n;
    SortGeom g{};
    g.dim = c->dim;
    g.bx = c->bits[0];
    g.by = c->bits[1];
    for (int d = 0; d < 3; ++d) {
        g.tile[d] = c->tile[d];
        g.ntile_axis[d] = c->ntile_axis[d];
    }
    g.ct = c->tile[0] * c->tile[1] * c->tile[2];
    {
        // parity classes in the order (000 111 001 110 010 101 100 011) of
        // (x | y<<1 | z<<2); in 2D the z-odd classes are empty
        static const int order[8] = {0, 7, 1, 6, 2, 5, 4, 3};
        static const int order2[4] = {0, 3, 1, 2};
        int next = 0;
        for (int q = 0; q < 8; ++q) g.cls_start[q] = 0;
        const int ncls = c->dim == 3 ? 8 : 4;
        for (int q = 0; q < ncls; ++q) {
            const int cls = c->dim == 3 ? order[q] : order2[q];
            int size = 1;
            for (int d = 0; d < 3; ++d) size *= (c->tile[d] + 1 - ((cls >> d) & 1)) >> 1;
            g.cls_start[cls] = next;
            next += size;
        }
    }
    if (n == 0) {
        tile_bounds_kernel<<<1, 256, 0, s>>>(c->keys[0], 0, c->ntiles, dst->tile_start);
        return hipGetLastError();
    }
    int cur = 0;
    if (src->tile_start && src->tile_start != dst->tile_start) {
        hipError_t e = rebin_from_hint(c, src, dst, g, s, cur);
        if (e != hipSuccess) return e;
    } else {
        sort_keys_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src->cell, n, g, c->keys[0]);
        // keys run up to ntiles (the off-grid key)
        int bits = 0;
        while ((1ll << bits) <= c->ntiles) ++bits;
        const int passes = bits == 0 ? 1 : (bits + 7) / 8;
        const int64_t nblocks = (n + SORT_ITEMS - 1) / SORT_ITEMS;
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = 8 * pass;
            radix_hist_kernel<false><<<(unsigned)nblocks, SORT_THREADS, 0, s>>>(c->keys[cur], n, nullptr, shift,
                                                                                c->hist);
            hipError_t e = exclusive_scan(c, c->hist, 256 * nblocks, c->hist + 256 * nblocks, s);
            if (e != hipSuccess) return e;
            radix_scatter_kernel<false><<<(unsigned)nblocks, SORT_THREADS, 0, s>>>(
                c->keys[cur], pass == 0 ? nullptr : c->vals[cur], n, nullptr, shift, c->hist, c->keys[cur ^ 1],
                c->vals[cur ^ 1]);
            cur ^= 1;
        }
        tile_bounds_kernel<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(c->keys[cur], n, c->ntiles,
                                                                           dst->tile_start);
    }
    PermArgs pa{};
    pa.cell_in = src->cell;
    int nc = 0;
    auto col4 = [&](const void *a, void *b) {
        pa.src[nc] = (const uint32_t *)a;
        pa.dst[nc] = (uint32_t *)b;
        pa.stride[nc++] = 1;
    };
    auto col8 = [&](const void *a, void *b) {
        for (int w = 0; w < 2; ++w) {
            pa.src[nc] = (const uint32_t *)a + w;
            pa.dst[nc] = (uint32_t *)b + w;
            pa.stride[nc++] = 2;
        }
    };
    col4(src->cell, dst->cell);
    for (int d = 0; d < c->dim; ++d) col4(src->off[d], dst->off[d]);
    for (int d = 0; d < 3; ++d) col4(src->u[d], dst->u[d]);
    if (src->w) col4(src->w, dst->w);
    if (src->chi) col4(src->chi, dst->chi);
    if (src->tau_thr) col4(src->tau_thr, dst->tau_thr);
    if (src->tau) col8(src->tau, dst->tau);
    if (src->id) col8(src->id, dst->id);
    pa.ncol = nc;
    int lbits = 0;
    while ((1 << lbits) < g.ct) ++lbits;
    // scratch: keys[cur^1] (key of the cell within the tile), vals[cur^1]
    // (rank within the cell in the wavefront's share, then final position),
    // final_perm (final position of each cell-order slot)
    tile_order_kernel<<<(unsigned)c->ntiles, ORDER_THREADS, sort_lds_bytes(g.ct), s>>>(
        c->vals[cur], dst->tile_start, g, lbits, sort_stage_len(g.ct), c->keys[cur ^ 1], c->vals[cur ^ 1],
        c->final_perm, pa);
    tail_copy_kernel<<<64, 256, 0, s>>>(c->vals[cur], dst->tile_start, c->ntiles, n, pa);
    return hipGetLastError();
}

hipError_t set_sort_lds_limit(size_t bytes) {
    return hipFuncSetAttribute((const void *)tile_order_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace pic
