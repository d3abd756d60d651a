// mlp.hip -- the 4 -> 64 -> 64 -> 2 surrogate of the QED rates and inverse
// spectra (Sec. IV, Eqs. 23-24), trained and evaluated with BF16 matrix cores
// (v_mfma_f32_16x16x16_bf16 and v_mfma_f32_16x16x32_bf16, FP32 accumulate)
// on gfx950.
//
// Network: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3.
// Weights are BF16 pairs, biases FP32.  Each weight is stored as two BF16
// terms, hi = bf16(w) and lo = bf16(w - hi) (about 16 significant bits), and
// in the forward pass every activation enters the MFMAs as two BF16 terms
// too; a product takes w_hi a_hi + w_hi a_lo + w_lo a_hi (the lo x lo term
// is below 2^-16 of it).  With single BF16 weights the rates stalled near
// 1e-3 relative error: gradient steps below half a BF16 unit do not change
// the rounded weights, so training cannot polish them.  The backward pass
// uses single BF16 terms (hi only).
// Training objective: sum over rows and outputs of w_o (y_o - t_o)^2 / (2 n)
// with w = (MLP_RATE_WEIGHT, 1): the rate output carries the 1e-3 accuracy
// target, the sampled fraction only enters a Monte-Carlo draw.
// Inputs:  x0 = (log10 chi - c_p) / h_p over the process's chi range,
//          x1 = 2 rho(r) - 1 (r the level of the inverse CDF, rho the table's
//          level coordinate), x2 = [photon emission], x3 = [pair creation].
// Outputs: y0 = g of the rate tables (ln(F/chi) for emission,
//          ln F + 8/(3 chi) for pairs); y1 = u^(1/3) (emission) or x (pairs).
// Every matrix product is a sum of 16x16x16 tiles in the MFMA lane layout
// (A: lane l holds row l%16, k = 4(l/16)+i; B: column l%16, k = 4(l/16)+i;
// C: column l%16, rows 4(l/16)+i).  Inference keeps the weight fragments in
// registers, chains the layers without leaving registers and runs 64 samples
// per wavefront round; training runs 16 samples per round with fragments read
// from LDS and memory.
#include "device_common.h"
#include "pic_internal.h"
#include "qed_internal.h"

namespace pic {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }

// acc += sum over k0 of A(m, k) B(k, n) for one 16x16 tile, K a multiple of 16
template <class FA, class FB>
__device__ __forceinline__ f32x4 tile_mma(FA A, FB B, int K, f32x4 acc) {
    const int l = threadIdx.x & 63;
    const int rc = l & 15, kq = 4 * (l >> 4);
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = f2bf(A(rc, k0 + kq + i));
            b[i] = f2bf(B(k0 + kq + i, rc));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// acc += A B for one 16x16 tile with A split into hi + lo BF16 terms
template <class FA, class FB>
__device__ __forceinline__ f32x4 tile_mma_split(FA A, FB B, int K, f32x4 acc) {
    const int l = threadIdx.x & 63;
    const int rc = l & 15, kq = 4 * (l >> 4);
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 ah, al, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float x = A(rc, k0 + kq + i);
            ah[i] = f2bf(x);
            al[i] = f2bf(x - bf2f(ah[i]));
            b[i] = f2bf(B(k0 + kq + i, rc));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, b, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, b, acc, 0, 0, 0);
    }
    return acc;
}

// acc += A B for one 16x16 tile, A split into hi + lo BF16 terms and B given
// as its hi and lo BF16 terms: A_hi B_hi + A_lo B_hi + A_hi B_lo
template <class FA, class FB, class FBL>
__device__ __forceinline__ f32x4 tile_mma_split2(FA A, FB Bh, FBL Bl, int K, f32x4 acc) {
    const int l = threadIdx.x & 63;
    const int rc = l & 15, kq = 4 * (l >> 4);
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 ah, al, bh, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float x = A(rc, k0 + kq + i);
            ah[i] = f2bf(x);
            al[i] = f2bf(x - bf2f(ah[i]));
            bh[i] = Bh(k0 + kq + i, rc);
            bl[i] = Bl(k0 + kq + i, rc);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    }
    return acc;
}

constexpr float MLP_RATE_WEIGHT = 10.0f;

// tanh from the hardware exponential and reciprocal: 1 - 2 / (1 + 2^{2x log2 e})
// (saturates to +-1, absolute error about 1e-7)
__device__ __forceinline__ float tanh_f(float x) {
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(2.8853900817779268f * x)), 1.0f);
}

struct MlpView {
    const short *W1, *W2, *W3;  // [4][64], [64][64], [64][2] BF16 hi terms
    const float *b1, *b2, *b3;
    const short *L1, *L2, *L3;  // their BF16 lo terms
};

__device__ __forceinline__ MlpView mlp_view(const void *m) {
    const char *p = (const char *)m;
    return MlpView{(const short *)(p + PIC_MLP_OFF_W1), (const short *)(p + PIC_MLP_OFF_W2),
                   (const short *)(p + PIC_MLP_OFF_W3), (const float *)(p + PIC_MLP_OFF_B1),
                   (const float *)(p + PIC_MLP_OFF_B2), (const float *)(p + PIC_MLP_OFF_B3),
                   (const short *)(p + PIC_MLP_OFF_W1_LO), (const short *)(p + PIC_MLP_OFF_W2_LO),
                   (const short *)(p + PIC_MLP_OFF_W3_LO)};
}

// a weight's hi and lo BF16 terms
__device__ __forceinline__ void bf_split(float p, short &hi, short &lo) {
    hi = f2bf(p);
    lo = f2bf(p - bf2f(hi));
}

struct WaveLds {
    float X[16][4];
    float H1[16][64];
    float H2[16][64];
    float D[16][64];   // dZ2 then dZ1
    float Y[16][2];
};

// forward of 16 samples held in L.X; leaves H1, H2 (tanh outputs) and Y
__device__ void mlp_forward16(const MlpView &w, WaveLds &L) {
    const int l = threadIdx.x & 63;
    const int col = l & 15, r4 = 4 * (l >> 4);
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = tile_mma_split2([&](int m, int k) { return k < 4 ? L.X[m][k] : 0.0f; },
                              [&](int k, int n) { return k < 4 ? w.W1[k * 64 + 16 * nt + n] : (short)0; },
                              [&](int k, int n) { return k < 4 ? w.L1[k * 64 + 16 * nt + n] : (short)0; }, 16, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) L.H1[r4 + i][16 * nt + col] = tanh_f(acc[i] + w.b1[16 * nt + col]);
    }
    __syncthreads();
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = tile_mma_split2([&](int m, int k) { return L.H1[m][k]; },
                              [&](int k, int n) { return w.W2[k * 64 + 16 * nt + n]; },
                              [&](int k, int n) { return w.L2[k * 64 + 16 * nt + n]; }, 64, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) L.H2[r4 + i][16 * nt + col] = tanh_f(acc[i] + w.b2[16 * nt + col]);
    }
    __syncthreads();
    {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = tile_mma_split2([&](int m, int k) { return L.H2[m][k]; },
                              [&](int k, int n) { return n < 2 ? w.W3[k * 2 + n] : (short)0; },
                              [&](int k, int n) { return n < 2 ? w.L3[k * 2 + n] : (short)0; }, 64, acc);
        if (col < 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) L.Y[r4 + i][col] = acc[i] + w.b3[col];
        }
    }
    __syncthreads();
}

// ---- inputs and outputs of the QED surrogate ------------------------------

__device__ __forceinline__ void mlp_chi_range(int proc, float &c, float &h) {
    const float lo = proc == QED_COMPTON ? (float)QED_LOG_CHI_MIN_C : (float)QED_LOG_CHI_MIN_P;
    const float hi = (float)QED_LOG_CHI_MAX;
    c = 0.5f * (lo + hi);
    h = 0.5f * (hi - lo);
}

__device__ __forceinline__ void mlp_inputs(int proc, float chi, float r, float *x) {
    float c, h;
    mlp_chi_range(proc, c, h);
    x[0] = (log10f(chi) - c) / h;
    x[1] = 2.0f * qed_rho_of_r(proc, r) - 1.0f;
    x[2] = proc == QED_COMPTON ? 1.0f : 0.0f;
    x[3] = proc == QED_PAIR ? 1.0f : 0.0f;
}

// rate F and sampled energy fraction from the outputs
__device__ __forceinline__ void mlp_decode(int proc, float chi, const float *y, float &F, float &smp) {
    if (proc == QED_COMPTON) {
        F = chi * expf(y[0]);
        const float s = fminf(fmaxf(y[1], 0.0f), 1.0f);
        smp = s * s * s;
    } else {
        F = expf(y[0] - 8.0f / (3.0f * chi));
        smp = fminf(fmaxf(y[1], 0.0f), 1.0f);
    }
}

// ---- inference: weights held in registers --------------------------------
// The weights are the A operand and the activations the B operand (outputs
// as rows, samples as columns), so the C fragment one layer produces (lane l:
// rows 4(l/16)+i of a 16-row output block, column l%16 = sample) already is
// the B fragment of the next layer and activations never leave registers.
// Layers 2 and 3 contract 32 features per v_mfma_f32_16x16x32_bf16 in the
// slot order k(g, i) = 32 j + (i < 4 ? 4 g + i : 12 + 4 g + i), g = l/16,
// i = 0..7: the lane's values of output blocks 2j and 2j+1.  Any order of
// the contraction is the same sum, provided the weights' A fragments use it
// too.  Layer 1 (v_mfma_f32_16x16x16_bf16, k = 4 g + i) takes the inputs'
// hi terms against W1's hi terms in g = 0, their lo terms against W1's hi
// terms in g = 1, the bias as three BF16 terms against constant ones in
// g = 2 and the inputs' hi terms against W1's lo terms in g = 3.  Layers 2
// and 3 add a third MFMA per k-step, the weights' lo terms against the hi
// activations.  Per 16-sample tile: 4 + 24 + 6 MFMAs, 32 tanh and 32 hi/lo
// splits per lane.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v4 __attribute__((ext_vector_type(4)));

struct MlpFrags {
    bf16x4 w1[4];     // [output block]
    bf16x8 w2[4][2];  // [output block][k-step], hi terms
    bf16x8 l2[4][2];  // lo terms
    bf16x8 w3[2];     // [k-step]; rows 0, 1 are the two outputs; hi terms
    bf16x8 l3[2];     // lo terms
    f32x4 b2[4];      // bias of rows 4g+i of each output block
    f32x4 b3;
};

// feature of slot i of lane group g in k-step j (layers 2 and 3)
__device__ __forceinline__ int mlp_slot_feature(int j, int g, int i) { return 32 * j + (i < 4 ? 4 * g + i : 12 + 4 * g + i); }

__device__ __forceinline__ short bf_bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ __forceinline__ void mlp_load_frags(const MlpView &w, MlpFrags &F) {
    const int l = threadIdx.x & 63;
    const int m = l & 15, g = l >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int o = 16 * nt + m;
        const float b = w.b1[o];
        const float t0 = (float)(__bf16)b, t1 = (float)(__bf16)(b - t0), t2 = (float)(__bf16)(b - t0 - t1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            short v = 0;
            if (g < 2) v = w.W1[i * 64 + o];
            else if (g == 2) v = bf_bits(i == 0 ? t0 : i == 1 ? t1 : i == 2 ? t2 : 0.0f);
            else v = w.L1[i * 64 + o];
            F.w1[nt][i] = v;
            F.b2[nt][i] = w.b2[16 * nt + 4 * g + i];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                F.w2[nt][j][i] = __builtin_bit_cast(__bf16, w.W2[mlp_slot_feature(j, g, i) * 64 + o]);
                F.l2[nt][j][i] = __builtin_bit_cast(__bf16, w.L2[mlp_slot_feature(j, g, i) * 64 + o]);
            }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            F.w3[j][i] = __builtin_bit_cast(__bf16, m < 2 ? w.W3[mlp_slot_feature(j, g, i) * 2 + m] : (short)0);
            F.l3[j][i] = __builtin_bit_cast(__bf16, m < 2 ? w.L3[mlp_slot_feature(j, g, i) * 2 + m] : (short)0);
        }
#pragma unroll
    for (int i = 0; i < 4; ++i) F.b3[i] = g == 0 && i < 2 ? w.b3[i] : 0.0f;
}

typedef float f32x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// hi and lo BF16 terms of eight values: one rounding conversion per pair,
// the hi values read back from the packed pair by shift and mask
__device__ __forceinline__ void split8(const f32x8 &h, bf16x8 &hi, bf16x8 &lo) {
    u32x4 ph, pl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x2 v = {h[2 * q], h[2 * q + 1]};
        const uint32_t u = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
        const f32x2 r = {v[0] - __uint_as_float(u << 16), v[1] - __uint_as_float(u & 0xFFFF0000u)};
        ph[q] = u;
        pl[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
    }
    hi = __builtin_bit_cast(bf16x8, ph);
    lo = __builtin_bit_cast(bf16x8, pl);
}

// tanh of C blocks 2j, 2j+1 as the hi and lo B fragments of k-step j
__device__ __forceinline__ void mlp_act_frags(const f32x4 &c0, const f32x4 &c1, bf16x8 &hi, bf16x8 &lo) {
    f32x8 h;
#pragma unroll
    for (int i = 0; i < 8; ++i) h[i] = tanh_f(i < 4 ? c0[i] : c1[i - 4]);
    split8(h, hi, lo);
}

// per-wavefront LDS of the inference: 64 samples' inputs and outputs
struct InferLds {
    float X[64][4];
    float Y[64][2];
};

// outputs Y[16t .. 16t+15] from inputs X[16t ..]
__device__ __forceinline__ void mlp_infer_tile(const MlpFrags &F, InferLds &L, int t) {
    const int l = threadIdx.x & 63;
    const int g = l >> 4, s = 16 * t + (l & 15);
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    // lane group g: 0 hi terms, 1 lo terms, 2 the ones against the bias
    // terms, 3 hi terms against the weights' lo terms
    const f32x4 x = *(const f32x4 *)L.X[s];
    const bf16v4 xh = __builtin_convertvector(x, bf16v4);
    const bf16v4 xl = __builtin_convertvector(x - __builtin_convertvector(xh, f32x4), bf16v4);
    const bf16v4 one = {(__bf16)1.0f, (__bf16)1.0f, (__bf16)1.0f, (__bf16)0.0f};
    const bf16x4 xb = __builtin_bit_cast(bf16x4, g == 1 ? xl : g == 2 ? one : xh);
    f32x4 c1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) c1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F.w1[nt], xb, z, 0, 0, 0);
    bf16x8 hh[2], hl[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) mlp_act_frags(c1[2 * j], c1[2 * j + 1], hh[j], hl[j]);
    f32x4 c2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = F.b2[nt];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[nt][j], hh[j], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w2[nt][j], hl[j], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.l2[nt][j], hh[j], acc, 0, 0, 0);
        }
        c2[nt] = acc;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) mlp_act_frags(c2[2 * j], c2[2 * j + 1], hh[j], hl[j]);
    f32x4 c3 = F.b3;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[j], hh[j], c3, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.w3[j], hl[j], c3, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.l3[j], hh[j], c3, 0, 0, 0);
    }
    if (g == 0) {
        L.Y[s][0] = c3[0];
        L.Y[s][1] = c3[1];
    }
}

constexpr int INFER_THREADS = 256;

// the network answers inside its training range less this margin (decades
// of chi) at both ends, where its fit is least constrained; the tables
// answer elsewhere
constexpr float MLP_EDGE = 0.1f;

// network inference for the QED step: one output pair (F, sample) per
// particle; the level r is the uniform the particle uses if its event fires
// this step.  chi outside the trained range less MLP_EDGE falls back to the
// tables.  Each
// wavefront prepares 64 particles' inputs (one per lane), runs four tiles,
// and decodes one output per lane.
__global__ void __launch_bounds__(INFER_THREADS, 4) mlp_qed_kernel(const void *mlp, const float *tab, QedSpeciesView v,
                                                                int proc, float *out) {
    __shared__ InferLds Ls[INFER_THREADS / 64];
    InferLds &L = Ls[threadIdx.x >> 6];
    MlpFrags F;
    mlp_load_frags(mlp_view(mlp), F);
    const int l = threadIdx.x & 63;
    const float lo = proc == QED_COMPTON ? (float)QED_LOG_CHI_MIN_C : (float)QED_LOG_CHI_MIN_P;
    const int64_t nw = (int64_t)gridDim.x * (INFER_THREADS / 64);
    for (int64_t base = ((int64_t)blockIdx.x * (INFER_THREADS / 64) + (threadIdx.x >> 6)) * 64; base < v.n;
         base += nw * 64) {
        const int64_t p = base + l;
        float chi = 0.0f, r = 0.5f;
        float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (p < v.n) {
            chi = v.chi[p];
            double ru, rt;
            qed_uniforms(v.seed, v.id[p], v.step, 0u, ru, rt);
            r = (float)ru;
            mlp_inputs(proc, fmaxf(chi, 1e-30f), r, x);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) L.X[l][k] = x[k];
        __builtin_amdgcn_wave_barrier();
        for (int t = 0; t < 4; ++t) mlp_infer_tile(F, L, t);
        __builtin_amdgcn_wave_barrier();
        if (p < v.n) {
            const float lc = chi > 0.0f ? log10f(chi) : -100.0f;
            float F_, smp;
            if (lc >= lo + MLP_EDGE && lc <= (float)QED_LOG_CHI_MAX - MLP_EDGE) {
                const float y[2] = {L.Y[l][0], L.Y[l][1]};
                mlp_decode(proc, chi, y, F_, smp);
            } else {
                F_ = qed_rate_F(tab, proc, chi);
                smp = qed_inverse(tab, proc, chi, r);
            }
            out[2 * p] = F_;
            out[2 * p + 1] = smp;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

static unsigned infer_blocks(int64_t n) {
    const int64_t waves = (n + 63) / 64;
    const int64_t blocks = (waves + INFER_THREADS / 64 - 1) / (INFER_THREADS / 64);
    return (unsigned)(blocks < 2048 ? blocks : 2048);
}

hipError_t launch_mlp_for_qed(Ctx *c, const void *mlp, const QedSpeciesView &v, int proc, float *out,
                              hipStream_t s) {
    if (v.n <= 0) return hipSuccess;
    mlp_qed_kernel<<<infer_blocks(v.n), INFER_THREADS, 0, s>>>(mlp, c->qed.dev, v, proc, out);
    return hipGetLastError();
}

// plain forward: x [n][4] -> y [n][2]
__global__ void __launch_bounds__(INFER_THREADS, 4) mlp_forward_kernel(const void *mlp, const float *x, int64_t n,
                                                                    float *y) {
    __shared__ InferLds Ls[INFER_THREADS / 64];
    InferLds &L = Ls[threadIdx.x >> 6];
    MlpFrags F;
    mlp_load_frags(mlp_view(mlp), F);
    const int l = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (INFER_THREADS / 64);
    for (int64_t base = ((int64_t)blockIdx.x * (INFER_THREADS / 64) + (threadIdx.x >> 6)) * 64; base < n;
         base += nw * 64) {
        const int64_t p = base + l;
#pragma unroll
        for (int k = 0; k < 4; ++k) L.X[l][k] = p < n ? x[p * 4 + k] : 0.0f;
        __builtin_amdgcn_wave_barrier();
        for (int t = 0; t < 4; ++t) mlp_infer_tile(F, L, t);
        __builtin_amdgcn_wave_barrier();
        if (p < n) {
            y[p * 2] = L.Y[l][0];
            y[p * 2 + 1] = L.Y[l][1];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---- training -----------------------------------------------------------
// flat FP32 parameter order (also of the gradient): W1[4][64], b1[64],
// W2[64][64], b2[64], W3[64][2], b3[2]
constexpr int P_W1 = 0, P_B1 = 256, P_W2 = 320, P_B2 = 4416, P_W3 = 4480, P_B3 = 4608;

// gradient of sum_rows sum_o w_o (y - t)^2 / (2 n_total) over the rows
// [r0, r0 + rows) assigned to this wave, added to grad[]; loss sum too
__global__ void __launch_bounds__(64) mlp_grad_kernel(const void *mlp, const float *x, const float *t, int64_t r0,
                                                      int64_t rows, int64_t n_total, int rows_per_wave,
                                                      float *grad, float *loss) {
    __shared__ WaveLds L;
    const MlpView w = mlp_view(mlp);
    const int l = threadIdx.x;
    const int col = l & 15, r4 = 4 * (l >> 4);
    f32x4 g2[4][4], g1[4], g3[4];
    for (int a = 0; a < 4; ++a) {
        g1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        g3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 4; ++b) g2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, lsum = 0.f;
    const float inv_n = 1.0f / (float)n_total;
    const int64_t w0 = (int64_t)blockIdx.x * rows_per_wave;
    for (int64_t base = w0; base < w0 + rows_per_wave && base < rows; base += 16) {
        const int64_t row = r0 + base + (l & 15);
        const bool ok = base + (l & 15) < rows;
        if (l < 16) {
            for (int k = 0; k < 4; ++k) L.X[l][k] = ok ? x[row * 4 + k] : 0.0f;
        }
        __syncthreads();
        mlp_forward16(w, L);
        // dY = (Y - T) / n on valid rows (lanes 0..31: row = l/2, output l%2)
        float dy = 0.0f;
        if (l < 32) {
            const int rr = l >> 1, o = l & 1;
            const bool ok2 = base + rr < rows;
            if (ok2) {
                const float d = L.Y[rr][o] - t[(r0 + base + rr) * 2 + o];
                const float wo = o == 0 ? MLP_RATE_WEIGHT : 1.0f;
                lsum += wo * d * d;
                dy = wo * d * inv_n;
            }
        }
        __syncthreads();
        if (l < 32) L.Y[l >> 1][l & 1] = dy;
        __syncthreads();
        // gW3 += H2^T dY ; gb3
        for (int mt = 0; mt < 4; ++mt)
            g3[mt] = tile_mma([&](int m, int k) { return L.H2[k][16 * mt + m]; },
                              [&](int k, int n) { return n < 2 ? L.Y[k][n] : 0.0f; }, 16, g3[mt]);
        if (l < 2)
            for (int s = 0; s < 16; ++s) gb3 += L.Y[s][l];
        // dZ2 = (dY W3^T) (1 - H2^2): lane = hidden unit
        {
            const float w30 = bf2f(w.W3[l * 2]), w31 = bf2f(w.W3[l * 2 + 1]);
            for (int s = 0; s < 16; ++s) {
                const float h = L.H2[s][l];
                L.D[s][l] = (L.Y[s][0] * w30 + L.Y[s][1] * w31) * (1.0f - h * h);
            }
        }
        __syncthreads();
        // gW2 += H1^T dZ2 ; gb2
        for (int mt = 0; mt < 4; ++mt)
            for (int nt = 0; nt < 4; ++nt)
                g2[mt][nt] = tile_mma([&](int m, int k) { return L.H1[k][16 * mt + m]; },
                                      [&](int k, int n) { return L.D[k][16 * nt + n]; }, 16, g2[mt][nt]);
        for (int s = 0; s < 16; ++s) gb2 += L.D[s][l];
        // dZ1 = (dZ2 W2^T) (1 - H1^2)
        f32x4 dh1[4];
        for (int nt = 0; nt < 4; ++nt) {
            dh1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
            dh1[nt] = tile_mma([&](int m, int k) { return L.D[m][k]; },
                               [&](int k, int n) { return bf2f(w.W2[(16 * nt + n) * 64 + k]); }, 64, dh1[nt]);
        }
        __syncthreads();
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h = L.H1[r4 + i][16 * nt + col];
                L.D[r4 + i][16 * nt + col] = dh1[nt][i] * (1.0f - h * h);
            }
        __syncthreads();
        // gW1 += X^T dZ1 ; gb1
        for (int nt = 0; nt < 4; ++nt)
            g1[nt] = tile_mma([&](int m, int k) { return m < 4 ? L.X[k][m] : 0.0f; },
                              [&](int k, int n) { return L.D[k][16 * nt + n]; }, 16, g1[nt]);
        for (int s = 0; s < 16; ++s) gb1 += L.D[s][l];
        __syncthreads();
    }
    // add this wave's gradient into the global one
    for (int mt = 0; mt < 4; ++mt)
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) atomicAdd(&grad[P_W2 + (16 * mt + r4 + i) * 64 + 16 * nt + col], g2[mt][nt][i]);
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (r4 + i < 4) atomicAdd(&grad[P_W1 + (r4 + i) * 64 + 16 * nt + col], g1[nt][i]);
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (col < 2) atomicAdd(&grad[P_W3 + (16 * mt + r4 + i) * 2 + col], g3[mt][i]);
    atomicAdd(&grad[P_B1 + l], gb1);
    atomicAdd(&grad[P_B2 + l], gb2);
    if (l < 2) atomicAdd(&grad[P_B3 + l], gb3);
    if (loss) {
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off);
        if (l == 0) atomicAdd(loss, 0.5f * lsum * inv_n);
    }
}

// parameter i (flat order) into the network: weights as hi and lo BF16 terms
__device__ __forceinline__ void mlp_store_param(char *net, int i, float p) {
    short hi, lo;
    bf_split(p, hi, lo);
    if (i < P_B1) {
        ((short *)(net + PIC_MLP_OFF_W1))[i - P_W1] = hi;
        ((short *)(net + PIC_MLP_OFF_W1_LO))[i - P_W1] = lo;
    } else if (i < P_W2) {
        ((float *)(net + PIC_MLP_OFF_B1))[i - P_B1] = p;
    } else if (i < P_B2) {
        ((short *)(net + PIC_MLP_OFF_W2))[i - P_W2] = hi;
        ((short *)(net + PIC_MLP_OFF_W2_LO))[i - P_W2] = lo;
    } else if (i < P_W3) {
        ((float *)(net + PIC_MLP_OFF_B2))[i - P_B2] = p;
    } else if (i < P_B3) {
        ((short *)(net + PIC_MLP_OFF_W3))[i - P_W3] = hi;
        ((short *)(net + PIC_MLP_OFF_W3_LO))[i - P_W3] = lo;
    } else {
        ((float *)(net + PIC_MLP_OFF_B3))[i - P_B3] = p;
    }
}

// Adam step on the FP32 master parameters, then the BF16/FP32 network copy;
// clears the gradient.  state: [params | m | v | grad] floats, then step count.
__global__ void __launch_bounds__(256) mlp_adam_kernel(float *state, float lr, void *mlp) {
    float *prm = state, *m = state + PIC_MLP_NPARAM, *v = state + 2 * PIC_MLP_NPARAM,
          *g = state + 3 * PIC_MLP_NPARAM;
    float *tstep = state + 4 * PIC_MLP_NPARAM;
    const float t = tstep[0] + 1.0f;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    char *net = (char *)mlp;
    for (int i = threadIdx.x; i < PIC_MLP_NPARAM; i += blockDim.x) {
        const float gi = g[i];
        m[i] = b1 * m[i] + (1.0f - b1) * gi;
        v[i] = b2 * v[i] + (1.0f - b2) * gi * gi;
        prm[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + 1e-8f);
        g[i] = 0.0f;
        const float p = prm[i];
        mlp_store_param(net, i, p);
    }
    __syncthreads();
    if (threadIdx.x == 0) tstep[0] = t;
}

// copy the master parameters into the network (BF16 weights) without a step
__global__ void mlp_export_kernel(const float *prm, void *mlp) {
    char *net = (char *)mlp;
    for (int i = threadIdx.x; i < PIC_MLP_NPARAM; i += blockDim.x) {
        const float p = prm[i];
        mlp_store_param(net, i, p);
    }
}

__global__ void zero_kernel(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// training samples from the library's tables: row i uses process i & 1,
// log10 chi uniform over the process's range and r uniform, both from
// Philox at counter (i_lo, i_hi, 0, 7) with key = seed
__global__ void mlp_data_kernel(const float *tab, int64_t n, uint64_t seed, float *x, float *t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int proc = (int)(i & 1);
    uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 7u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double a = u01_pair(c[0], c[1]), b = u01_pair(c[2], c[3]);
    const float lo = proc == QED_COMPTON ? (float)QED_LOG_CHI_MIN_C : (float)QED_LOG_CHI_MIN_P;
    const float lc = lo + (float)a * ((float)QED_LOG_CHI_MAX - lo);
    const float chi = exp10f(lc);
    const float r = (float)b;
    float xi[4];
    mlp_inputs(proc, chi, r, xi);
    for (int k = 0; k < 4; ++k) x[i * 4 + k] = xi[k];
    t[i * 2] = qed_rate_g(tab, proc, chi);
    const float smp = qed_inverse(tab, proc, chi, r);
    t[i * 2 + 1] = proc == QED_COMPTON ? cbrtf(smp) : smp;
}

hipError_t launch_mlp_forward(const void *mlp, const float *x, int64_t n, float *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    mlp_forward_kernel<<<infer_blocks(n), INFER_THREADS, 0, s>>>(mlp, x, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const void *mlp, const float *x, const float *t, int64_t n, float *grad, float *loss,
                           hipStream_t s) {
    const int rpw = 256;
    const int64_t waves = (n + rpw - 1) / rpw;
    mlp_grad_kernel<<<(unsigned)waves, 64, 0, s>>>(mlp, x, t, 0, n, n, rpw, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float *state, void *mlp, const float *x, const float *t, int64_t n, int batch,
                            int iters, float lr, float *loss, hipStream_t s) {
    float *grad = state + 3 * PIC_MLP_NPARAM;
    const int rpw = 128;
    mlp_export_kernel<<<1, 256, 0, s>>>(state, mlp);
    for (int it = 0; it < iters; ++it) {
        // cosine decay of the step size from lr to 0 over the run
        const float lr_it = 0.5f * lr * (1.0f + cosf(3.14159265f * (float)it / (float)iters));
        const int64_t r0 = ((int64_t)it * batch) % n;
        const int64_t rows = r0 + batch <= n ? batch : n - r0;
        const int64_t waves = (rows + rpw - 1) / rpw;
        mlp_grad_kernel<<<(unsigned)waves, 64, 0, s>>>(mlp, x, t, r0, rows, rows, rpw, grad,
                                                       it == iters - 1 ? loss : nullptr);
        mlp_adam_kernel<<<1, 256, 0, s>>>(state, lr_it, mlp);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_data(Ctx *c, int64_t n, uint64_t seed, float *x, float *t, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    mlp_data_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c->qed.dev, n, seed, x, t);
    return hipGetLastError();
}

}  // namespace pic
