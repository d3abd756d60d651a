// qed_internal.h -- table layout, lookups and the counter-based generator of
// the QED module (Sec. IV of the paper).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

enum { QED_COMPTON = 0, QED_PAIR = 1 };

constexpr int QED_NCHI = 256;   // chi points (log-uniform)
constexpr int QED_NR = 1024;    // inverse-CDF points in the transformed level rho
constexpr int QED_NV = 16384;   // quadrature nodes of the table build
constexpr double QED_LOG_CHI_MIN_C = -4.0;
constexpr double QED_LOG_CHI_MIN_P = -1.7;  // W_pair ~ exp(-8/(3 chi)) is below 1e-50 under chi = 0.02
constexpr double QED_LOG_CHI_MAX = 3.0;
constexpr int QED_OFF_RATE_C = 0;
constexpr int QED_OFF_RATE_P = QED_NCHI;
constexpr int QED_OFF_INV_C = 2 * QED_NCHI;
constexpr int QED_OFF_INV_P = 2 * QED_NCHI + QED_NCHI * QED_NR;
// Method II: the normalized differential spectrum p(chi, sigma) (density of
// s = u^(1/3) for emission, of x for pairs; integral over sigma in [0,1] is 1)
// at sigma = (1 - cos(pi v))/2, v uniform: nodes cluster at both ends, where
// the spectra have their narrow features (the hard cut-off next to u = 1 at
// large chi, the soft peak next to s = 0 at small chi)
constexpr int QED_NS = 1025;
constexpr int QED_OFF_DEN_C = 2 * QED_NCHI + 2 * QED_NCHI * QED_NR;
constexpr int QED_OFF_DEN_P = QED_OFF_DEN_C + QED_NCHI * QED_NS;
constexpr int QED_TABLE_FLOATS = QED_OFF_DEN_P + QED_NCHI * QED_NS;

struct QedTables {
    float *dev = nullptr;
};

// what the network inference of the QED step reads per particle
struct QedSpeciesView {
    const float *chi;
    const uint64_t *id;
    const float *w;
    int64_t n;
    uint64_t seed;
    uint32_t step;
};

hipError_t build_qed_tables(QedTables *t, hipStream_t s);

// Level r of the inverse CDF as a function of the uniform table coordinate
// rho in [0,1]: denser near r = 1 for photon emission (long hard tail), near
// both ends for pairs (symmetric spectrum).
__host__ __device__ inline double qed_r_of_rho(int proc, double rho) {
    if (proc == QED_COMPTON) return 1.0 - (1.0 - rho) * (1.0 - rho);
    return 0.5 * (1.0 - cos(3.14159265358979323846 * rho));
}
__device__ __forceinline__ float qed_rho_of_r(int proc, float r) {
    if (proc == QED_COMPTON) return 1.0f - sqrtf(fmaxf(1.0f - r, 0.0f));
    return acosf(fminf(fmaxf(1.0f - 2.0f * r, -1.0f), 1.0f)) * 0.318309886183790672f;
}

__device__ __forceinline__ float qed_log_chi_min(int proc) {
    return proc == QED_COMPTON ? (float)QED_LOG_CHI_MIN_C : (float)QED_LOG_CHI_MIN_P;
}

// Tabulated g (Catmull-Rom in log10 chi) for chi inside the table; above the
// table linear extrapolation of g in log chi.
__device__ inline float qed_rate_g(const float *tab, int proc, float chi) {
    const float lmin = qed_log_chi_min(proc), lmax = (float)QED_LOG_CHI_MAX;
    const float lc = log10f(chi);
    const float *g = tab + (proc == QED_COMPTON ? QED_OFF_RATE_C : QED_OFF_RATE_P);
    const float x = fmaxf((lc - lmin) / (lmax - lmin) * (QED_NCHI - 1), 0.0f);
    float gv;
    if (x >= QED_NCHI - 1) {
        const float slope = g[QED_NCHI - 1] - g[QED_NCHI - 2];
        gv = g[QED_NCHI - 1] + slope * (x - (QED_NCHI - 1));
    } else {
        const int i = (int)x;
        const float t = x - i;
        const float p1 = g[i], p2 = g[i + 1];
        const float p0 = i > 0 ? g[i - 1] : 2.0f * p1 - p2;
        const float p3 = i + 2 < QED_NCHI ? g[i + 2] : 2.0f * p2 - p1;
        gv = p1 + 0.5f * t * (p2 - p0 + t * (2.0f * p0 - 5.0f * p1 + 4.0f * p2 - p3 +
                                             t * (3.0f * (p1 - p2) + p3 - p0)));
    }
    return gv;
}

// F(chi) from g.  Compton below the table: classical limit 5 pi chi / 2;
// pairs below the table: 0 (W_pair < e^-133 there).
__device__ inline float qed_rate_F(const float *tab, int proc, float chi) {
    if (!(chi > 0.0f)) return 0.0f;
    if (log10f(chi) < qed_log_chi_min(proc)) return proc == QED_COMPTON ? 7.85398163397448f * chi : 0.0f;
    const float gv = qed_rate_g(tab, proc, chi);
    return proc == QED_COMPTON ? chi * expf(gv) : expf(gv - 8.0f / (3.0f * chi));
}

// Inverse CDF: photon energy fraction u (Compton) or positron fraction x
// (pairs) at level r: linear in rho, Catmull-Rom in log10 chi (at small chi
// the fractions scale as powers of chi, u^(1/3) ~ chi^(1/3) and
// x - 1/2 ~ chi^(1/2), curved in log chi enough that linear interpolation
// would move the level by a few 1e-5); chi clamped to the table.
__device__ inline float qed_inverse(const float *tab, int proc, float chi, float r) {
    const float lmin = qed_log_chi_min(proc), lmax = (float)QED_LOG_CHI_MAX;
    float x = (log10f(fmaxf(chi, 1e-30f)) - lmin) / (lmax - lmin) * (QED_NCHI - 1);
    x = fminf(fmaxf(x, 0.0f), (float)(QED_NCHI - 1) - 1e-3f);
    const int i = (int)x;
    const float t = x - i;
    float y = qed_rho_of_r(proc, r) * (QED_NR - 1);
    y = fminf(fmaxf(y, 0.0f), (float)(QED_NR - 1) - 1e-3f);
    const int k = (int)y;
    const float ty = y - k;
    const float *T = tab + (proc == QED_COMPTON ? QED_OFF_INV_C : QED_OFF_INV_P);
    auto row = [&](int ii) { return T[ii * QED_NR + k] * (1.0f - ty) + T[ii * QED_NR + k + 1] * ty; };
    const float p1 = row(i), p2 = row(i + 1);
    const float p0 = i > 0 ? row(i - 1) : 2.0f * p1 - p2;
    const float p3 = i + 2 < QED_NCHI ? row(i + 2) : 2.0f * p2 - p1;
    const float v = p1 + 0.5f * t * (p2 - p0 + t * (2.0f * p0 - 5.0f * p1 + 4.0f * p2 - p3 +
                                                    t * (3.0f * (p1 - p2) + p3 - p0)));
    return proc == QED_COMPTON ? v * v * v : v;
}

// Method II density p(chi, sigma), bilinear in (log10 chi, v) with
// v = acos(1 - 2 sigma)/pi; chi clamped to the table (outside it the shape of
// the nearest tabulated chi, as the inverse spectra do).
__device__ inline float qed_density(const float *tab, int proc, float chi, float sig) {
    const float lmin = qed_log_chi_min(proc), lmax = (float)QED_LOG_CHI_MAX;
    float x = (log10f(fmaxf(chi, 1e-30f)) - lmin) / (lmax - lmin) * (QED_NCHI - 1);
    x = fminf(fmaxf(x, 0.0f), (float)(QED_NCHI - 1) - 1e-3f);
    const int i = (int)x;
    const float tx = x - i;
    float y = acosf(fminf(fmaxf(1.0f - 2.0f * sig, -1.0f), 1.0f)) * 0.318309886183790672f * (QED_NS - 1);
    y = fminf(fmaxf(y, 0.0f), (float)(QED_NS - 1) - 1e-3f);
    const int k = (int)y;
    const float ty = y - k;
    const float *T = tab + (proc == QED_COMPTON ? QED_OFF_DEN_C : QED_OFF_DEN_P);
    const float a = T[i * QED_NS + k] * (1.0f - ty) + T[i * QED_NS + k + 1] * ty;
    const float b = T[(i + 1) * QED_NS + k] * (1.0f - ty) + T[(i + 1) * QED_NS + k + 1] * ty;
    return a * (1.0f - tx) + b * tx;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// (v + 1/2) / 2^52 from the top 52 bits of (hi, lo): open interval (0,1)
__device__ __forceinline__ double u01_pair(uint32_t hi, uint32_t lo) {
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 12;
    return ((double)v + 0.5) * (1.0 / 4503599627370496.0);
}

// Two uniforms of particle `id` at `step`, stream `stream` (counter
// (id_lo, id_hi, step, stream), key = seed).
__device__ __forceinline__ void qed_uniforms(uint64_t seed, uint64_t id, uint32_t step, uint32_t stream,
                                             double &a, double &b) {
    uint32_t c[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, stream};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    a = u01_pair(c[0], c[1]);
    b = u01_pair(c[2], c[3]);
}

// Identifier of a particle created from `parent` at `step` (tag 1 photon,
// 2 positron, 3 electron): the first 64 bits of Philox at counter
// (parent_lo, parent_hi, step, 0x80000000 | tag).
__device__ __forceinline__ uint64_t qed_child_id(uint64_t seed, uint64_t parent, uint32_t step, uint32_t tag) {
    uint32_t c[4] = {(uint32_t)parent, (uint32_t)(parent >> 32), step, 0x80000000u | tag};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ((uint64_t)c[1] << 32) | c[0];
}

}  // namespace pic
