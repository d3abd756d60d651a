// qed.hip -- Monte-Carlo nonlinear Compton and Breit-Wheeler step (Sec. IV),
// Method I in optical-depth form: every lepton and photon carries an FP64
// optical depth tau and a threshold tau_thr = -ln r; tau += W dt each step
// (W the total rate of Eq. 23 or 24); when tau reaches tau_thr the event
// happens, its energy is drawn from the inverse cumulative spectrum with a
// second uniform, and tau restarts from 0 with a fresh threshold.
//   leptons: photon of energy u gamma along u (recoil u <- u (1 - eps/|u|));
//            photons under `photon_min_energy` are not created;
//   photons: move ballistically, chi_gamma from the fields at their position;
//            above 2 m c^2 decay into e+ (x eps) and e- ((1-x) eps) along k.
// Method II (rejection, PIC_QED_METHOD2): each step the uniforms (r1, r2)
// propose u0 = r1^3 (emission) or x0 = r1 (pairs), and the event happens
// when the step's probability density at the proposal, W dt p(chi, r1) with
// p the normalized spectrum in s = u^(1/3) or x, exceeds r2; tau is not used.
// An acceptance above 1 is flagged (the step is too long for the rate).
// Created particles are appended with an atomic counter (dropped and flagged
// beyond capacity); their identifiers derive from the parent's, so every
// random number depends only on (seed, identifier, step).
#include "device_common.h"
#include "pic_internal.h"
#include "qed_internal.h"

namespace pic {

constexpr double QED_ALPHA = 1.0 / 137.035999084;
constexpr double QED_A = QED_ALPHA / (1.7320508075688772 * 3.14159265358979323846);

struct QedSpecies {
    int32_t *cell;
    float *off[3];
    float *u[3];
    float *w;
    float *chi;
    double *tau;
    float *tau_thr;
    uint64_t *id;
    int64_t n;
    int64_t capacity;
    unsigned long long *n_dev;
};

struct QedArgs {
    QedSpecies sp[3];  // electrons, positrons, photons
    int has[3];
    const float *F[6];
    const float *tab;
    const float *mlp_out;  // per particle (F, sample) from the network, or NULL
    int ng[3];
    int bx, by, dim, order;
    float inv_d[3];
    float dt;
    double rate_scale;     // alpha/(sqrt3 pi) * m c^2/(hbar w_r)
    float hbar_w;
    float emin;
    uint64_t seed;
    uint32_t step;
    int method2;
    int absorb_x;          // absorbing x faces (photons leave through them)
    uint32_t *status;
};

// one particle per thread; large workgroups make fewer reservations on the
// shared append counters (photons: 512, which leaves the 3D quartic gather
// its registers)
constexpr int QED_THREADS = 1024;
constexpr int QED_PHOTON_THREADS = 512;

// Slots for the particles a workgroup appends to species counter `counter`:
// every thread of the group calls this (uniform control flow) with want =
// whether it appends one particle; ranks come from a ballot per wavefront,
// one LDS atomic per wavefront and one global atomic per workgroup, so the
// shared counter is not serialized per particle.  The group's appends are
// slots base + rank (rank < count, in wavefront then lane order); slots at
// or beyond `cap` are dropped: the counter is brought back to cap and
// PIC_F_CAPACITY set.  base and count are the same in every thread.
__device__ void group_slots(bool want, unsigned long long *counter, int64_t cap, uint32_t *status,
                            unsigned long long &base, unsigned &count, unsigned &rank) {
    __shared__ unsigned s_cnt, s_total;
    __shared__ unsigned long long s_base;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const unsigned long long mask = __ballot(want);
    const int lane = threadIdx.x & 63;
    const int leader = mask ? __ffsll(mask) - 1 : 0;
    unsigned wbase = 0;
    if (mask && lane == leader) wbase = atomicAdd(&s_cnt, (unsigned)__popcll(mask));
    wbase = __shfl(wbase, leader);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned cnt = s_cnt;
        unsigned long long b = 0;
        if (cnt) {
            b = atomicAdd(counter, (unsigned long long)cnt);
            const unsigned long long end = b + cnt, c = (unsigned long long)cap;
            if (end > c) {
                atomicAdd(counter, 0ull - (end - (b > c ? b : c)));
                atomicOr(status, PIC_F_CAPACITY);
            }
        }
        s_base = b;
        s_total = cnt;  // s_cnt is cleared by the next call before its first barrier
    }
    __syncthreads();
    base = s_base;
    count = s_total;
    rank = wbase + (unsigned)__popcll(mask & ((1ull << lane) - 1));
}

// The slot of the calling thread's append, or -1 (none, or beyond cap).
__device__ int64_t group_reserve(bool want, unsigned long long *counter, int64_t cap, uint32_t *status) {
    unsigned long long base;
    unsigned count, rank;
    group_slots(want, counter, cap, status, base, count, rank);
    if (!want) return -1;
    const int64_t slot = (int64_t)(base + rank);
    return slot < cap ? slot : -1;
}

// a created particle at slot idx of species s
__device__ void qed_write(const QedArgs &a, int s, int64_t idx, int32_t cell, const float *off, const float *u,
                          float w, uint64_t id) {
    const QedSpecies &d = a.sp[s];
    d.cell[idx] = cell;
    for (int k = 0; k < a.dim; ++k) d.off[k][idx] = off[k];
    for (int k = 0; k < 3; ++k) d.u[k][idx] = u[k];
    if (d.w) d.w[idx] = w;
    if (d.chi) d.chi[idx] = 0.0f;
    d.tau[idx] = 0.0;
    double r0, r1;  // first threshold, so that the particle can enter Method I
    qed_uniforms(a.seed, id, a.step, 1u, r0, r1);
    d.tau_thr[idx] = (float)(-log(r0));
    d.id[idx] = id;
}

// one thread per lepton of species s (0 electrons, 1 positrons); the photon
// of an event has energy fraction uf along u and the lepton recoils
// collinearly.  Every per-lepton input is loaded in one round (one memory
// latency instead of a chain of them: weight, then momentum and chi, then
// the optical depth).
__global__ void __launch_bounds__(QED_THREADS) qed_lepton_kernel(QedArgs a, int s) {
    const QedSpecies &L = a.sp[s];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < L.n;
    float w = 0.0f, chi = 0.0f, thr = 0.0f, net_F = 0.0f, net_uf = 0.0f;
    float u[3] = {0.0f, 0.0f, 0.0f};
    double tau = 0.0;
    uint64_t id = 0;
    if (in) {
        w = L.w ? L.w[p] : 1.0f;
        u[0] = L.u[0][p];
        u[1] = L.u[1][p];
        u[2] = L.u[2][p];
        chi = L.chi[p];
        id = L.id[p];
        if (!a.method2) {
            tau = L.tau[p];
            thr = L.tau_thr[p];
        }
        if (a.mlp_out) {
            net_F = a.mlp_out[2 * p];
            net_uf = a.mlp_out[2 * p + 1];
        }
    }
    bool fire = false;
    float pu2 = 0.0f, gam = 1.0f, uf = 0.0f;
    if (in && w != 0.0f) {
        pu2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        gam = sqrtf(1.0f + pu2);
        if (a.method2) {
            if (chi > 0.0f) {
                double r1, r2;
                qed_uniforms(a.seed, id, a.step, 0u, r1, r2);
                const float F = qed_rate_F(a.tab, QED_COMPTON, chi);
                const double acc = a.rate_scale * (double)F / (double)gam * (double)a.dt *
                                   (double)qed_density(a.tab, QED_COMPTON, chi, (float)r1);
                if (acc > 1.0) atomicOr(a.status, PIC_F_QED_SATURATED);
                fire = acc > r2;
                uf = (float)(r1 * r1 * r1);
            }
        } else {
            const float F = a.mlp_out ? net_F : qed_rate_F(a.tab, QED_COMPTON, chi);
            tau += a.rate_scale * (double)F / (double)gam * (double)a.dt;
            if (tau >= (double)thr && chi > 0.0f) {
                double ru, rt;
                qed_uniforms(a.seed, id, a.step, 0u, ru, rt);
                uf = a.mlp_out ? net_uf : qed_inverse(a.tab, QED_COMPTON, chi, (float)ru);
                fire = true;
                tau = 0.0;
                L.tau_thr[p] = (float)(-log(rt));
            }
            L.tau[p] = tau;
        }
    }
    const float pm = sqrtf(pu2);
    fire = fire && pm > 0.0f;
    const float eps = fminf(fmaxf(uf, 0.0f), 1.0f) * gam;
    const float k[3] = {eps * u[0] / pm, eps * u[1] / pm, eps * u[2] / pm};
    if (fire) {
        const float f = fmaxf(0.0f, 1.0f - eps / pm);
        for (int c = 0; c < 3; ++c) L.u[c][p] = u[c] * f;
    }
    if (a.has[2]) {  // uniform over the grid
        // A few percent of the leptons emit, so most wavefronts hold one or
        // two: the emitters leave their photon in LDS at their rank among
        // the group's appends, and the first `count` threads write the
        // photons (the same slots, by few full wavefronts instead of many
        // nearly empty ones)
        __shared__ uint32_t e_src[QED_THREADS];
        __shared__ float e_k[3][QED_THREADS], e_w[QED_THREADS];
        __shared__ uint64_t e_id[QED_THREADS];
        const bool emit = fire && eps >= a.emin;
        unsigned long long base;
        unsigned count, rank;
        group_slots(emit, a.sp[2].n_dev, a.sp[2].capacity, a.status, base, count, rank);
        if (emit) {
            e_src[rank] = threadIdx.x;
            for (int c = 0; c < 3; ++c) e_k[c][rank] = k[c];
            e_w[rank] = w;
            e_id[rank] = id;
        }
        __syncthreads();
        const int64_t slot = (int64_t)(base + threadIdx.x);
        if (threadIdx.x < count && slot < a.sp[2].capacity) {
            const int64_t q = (int64_t)blockIdx.x * blockDim.x + e_src[threadIdx.x];
            const float off[3] = {L.off[0][q], L.off[1][q], a.dim == 3 ? L.off[2][q] : 0.0f};
            const float kq[3] = {e_k[0][threadIdx.x], e_k[1][threadIdx.x], e_k[2][threadIdx.x]};
            qed_write(a, 2, slot, L.cell[q], off, kq, e_w[threadIdx.x],
                      qed_child_id(a.seed, e_id[threadIdx.x], a.step, 1u));
        }
    }
}

// Photon step phases.  The tables (and Method II) take every step of a photon
// in one pass; the network needs chi_gamma at the moved photon before it can
// answer, so network mode runs the move and chi_gamma first (PH_MOVE, which
// writes chi), then the network on those chi, then the decays (PH_DECAY).
enum { PH_ALL = 0, PH_MOVE = 1, PH_DECAY = 2 };

// photons: ballistic move, chi_gamma at the new position, pair creation.
// With absorbing x faces a photon whose new position leaves [0, (n-1) dx]
// is absorbed (weight 0, chi 0, no decay), and no field is gathered from x
// nodes beyond [0, n).
template <int DIM, int ORDER, int PHASE>
__global__ void __launch_bounds__(QED_PHOTON_THREADS) qed_photon_kernel(QedArgs a) {
    const QedSpecies &P = a.sp[2];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float x = -1.0f;  // positron fraction if the photon decays this step
    float w = 0.0f, eps = 1.0f, k[3] = {0.0f, 0.0f, 0.0f}, f[3] = {0.0f, 0.0f, 0.0f};
    int packed = 0;
    uint64_t id = 0;
    do {  // every thread reaches the appends below
    if (p >= P.n) break;
    w = P.w[p];
    if (w == 0.0f) break;
    k[0] = P.u[0][p];
    k[1] = P.u[1][p];
    k[2] = P.u[2][p];
    eps = sqrtf(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    if (!(eps > 0.0f)) break;
    float chi;
    if constexpr (PHASE == PH_DECAY) {
        // moved, and chi_gamma written, by the PH_MOVE pass
        packed = P.cell[p];
        f[0] = P.off[0][p];
        f[1] = P.off[1][p];
        f[2] = DIM == 3 ? P.off[2][p] : 0.0f;
        chi = P.chi[p];
    } else {
        const int mx = (1 << a.bx) - 1, my = (1 << a.by) - 1;
        const int32_t cell = P.cell[p];
        int cc[3] = {cell & mx, (cell >> a.bx) & my, DIM == 3 ? (cell >> (a.bx + a.by)) : 0};
        f[0] = P.off[0][p];
        f[1] = P.off[1][p];
        f[2] = DIM == 3 ? P.off[2][p] : 0.0f;
        bool gone = false;
        // move at c along k
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const float xn = f[d] + a.dt * a.inv_d[d] * k[d] / eps;
            const float fl = floorf(xn);
            float fr = xn - fl;
            int di = (int)fl;
            if (fr >= 1.0f) {
                fr = 0.0f;
                ++di;
            }
            int nc = cc[d] + di;
            // x nodes of the domain are [0, n-1]: a new cell outside [0, n-2]
            // (before the wrap) is a position beyond a face
            if (d == 0 && a.absorb_x) gone = nc < 0 || nc >= a.ng[0] - 1;
            nc = ((nc % a.ng[d]) + a.ng[d]) % a.ng[d];
            cc[d] = nc;
            f[d] = fr;
            P.off[d][p] = fr;
            packed |= nc << (d == 0 ? 0 : (d == 1 ? a.bx : a.bx + a.by));
        }
        P.cell[p] = packed;
        if (gone) {
            P.w[p] = 0.0f;
            if (P.chi) P.chi[p] = 0.0f;
            w = 0.0f;
            break;
        }
        // fields at the photon (Eq. 19 with the push's weights)
        constexpr int NW = ORDER + 1;
        int i0[2][3] = {{0, 0, 0}, {0, 0, 0}};
        float wt[2][3][NW];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            shape_weights<ORDER>(f[d], i0[0][d], wt[0][d]);
            shape_weights<ORDER>(f[d] - 0.5f, i0[1][d], wt[1][d]);
        }
        float EB[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const int sx = stag(c, 0), sy = stag(c, 1), sz = DIM == 3 ? stag(c, 2) : 0;
            float acc = 0.0f;
#pragma unroll
            for (int kk = 0; kk < (DIM == 3 ? NW : 1); ++kk)
#pragma unroll
                for (int jj = 0; jj < NW; ++jj)
#pragma unroll
                    for (int ii = 0; ii < NW; ++ii) {
                        const int ui = cc[0] + i0[sx][0] + ii;
                        if (a.absorb_x && (unsigned)ui >= (unsigned)a.ng[0]) continue;  // beyond a face
                        const int gi = wrap_index(ui, a.ng[0]);
                        const int gj = wrap_index(cc[1] + i0[sy][1] + jj, a.ng[1]);
                        const int gk = DIM == 3 ? wrap_index(cc[2] + i0[sz][2] + kk, a.ng[2]) : 0;
                        const float wk = DIM == 3 ? wt[sz][2][kk] : 1.0f;
                        acc += wt[sx][0][ii] * wt[sy][1][jj] * wk *
                               a.F[c][(int64_t)gi + (int64_t)a.ng[0] * ((int64_t)gj + (int64_t)a.ng[1] * gk)];
                    }
            EB[c] = acc;
        }
        const float f0 = eps * EB[0] + k[1] * EB[5] - k[2] * EB[4];
        const float f1 = eps * EB[1] + k[2] * EB[3] - k[0] * EB[5];
        const float f2 = eps * EB[2] + k[0] * EB[4] - k[1] * EB[3];
        const float ke = k[0] * EB[0] + k[1] * EB[1] + k[2] * EB[2];
        chi = a.hbar_w * sqrtf(fmaxf(f0 * f0 + f1 * f1 + f2 * f2 - ke * ke, 0.0f));
        if (P.chi) P.chi[p] = chi;
        if constexpr (PHASE == PH_MOVE) break;
    }
    double tau = 0.0;
    id = P.id[p];
    if (a.method2) {
        if (eps > 2.0f && chi > 0.0f) {
            double r1, r2;
            qed_uniforms(a.seed, id, a.step, 0u, r1, r2);
            const double acc = a.rate_scale * (double)qed_rate_F(a.tab, QED_PAIR, chi) / (double)eps *
                               (double)a.dt * (double)qed_density(a.tab, QED_PAIR, chi, (float)r1);
            if (acc > 1.0) atomicOr(a.status, PIC_F_QED_SATURATED);
            if (acc > r2) x = (float)r1;
        }
    } else {
        const float F = a.mlp_out ? a.mlp_out[2 * p] : qed_rate_F(a.tab, QED_PAIR, chi);
        tau = P.tau[p] + a.rate_scale * (double)F / (double)eps * (double)a.dt;
        if (tau >= (double)P.tau_thr[p] && eps > 2.0f && chi > 0.0f) {
            double rx, rn;
            qed_uniforms(a.seed, id, a.step, 0u, rx, rn);
            x = a.mlp_out ? a.mlp_out[2 * p + 1] : qed_inverse(a.tab, QED_PAIR, chi, (float)rx);
            tau = 0.0;
        }
    }
    if (x >= 0.0f) P.w[p] = 0.0f;  // the photon is gone
    if (!a.method2) P.tau[p] = tau;
    } while (false);
    if constexpr (PHASE == PH_MOVE) return;  // uniform: no appends in this pass
    const bool decay = x >= 0.0f;
    const float xs = fminf(fmaxf(x, 0.0f), 1.0f);
    const float ep = xs * eps, em = (1.0f - xs) * eps;
    const float np_ = sqrtf(fmaxf(ep * ep - 1.0f, 0.0f)) / eps, nm = sqrtf(fmaxf(em * em - 1.0f, 0.0f)) / eps;
    if (a.has[0] || a.has[1]) {  // uniform over the grid
        // as in the lepton kernel: the decaying photons leave their pair in
        // LDS at their rank among the group's decays (the same in both
        // reservations), and the first `count` threads write the positrons
        // and electrons
        __shared__ int32_t d_cell[QED_PHOTON_THREADS];
        __shared__ float d_f[3][QED_PHOTON_THREADS], d_k[3][QED_PHOTON_THREADS];
        __shared__ float d_n[2][QED_PHOTON_THREADS], d_w[QED_PHOTON_THREADS];
        __shared__ uint64_t d_id[QED_PHOTON_THREADS];
        unsigned long long base[2] = {0ull, 0ull};
        unsigned count = 0, rank = 0;
        if (a.has[1]) group_slots(decay, a.sp[1].n_dev, a.sp[1].capacity, a.status, base[1], count, rank);
        if (a.has[0]) group_slots(decay, a.sp[0].n_dev, a.sp[0].capacity, a.status, base[0], count, rank);
        if (decay) {
            d_cell[rank] = packed;
            for (int c = 0; c < 3; ++c) {
                d_f[c][rank] = f[c];
                d_k[c][rank] = k[c];
            }
            d_n[0][rank] = nm;   // electron
            d_n[1][rank] = np_;  // positron
            d_w[rank] = w;
            d_id[rank] = id;
        }
        __syncthreads();
        const unsigned t = threadIdx.x;
        if (t < count) {
            const float ft[3] = {d_f[0][t], d_f[1][t], d_f[2][t]};
            for (int s2 = 1; s2 >= 0; --s2) {  // positron (tag 2), electron (tag 3)
                const int64_t slot = (int64_t)(base[s2] + t);
                if (!a.has[s2] || slot >= a.sp[s2].capacity) continue;
                const float n = d_n[s2][t];
                const float us[3] = {n * d_k[0][t], n * d_k[1][t], n * d_k[2][t]};
                qed_write(a, s2, slot, d_cell[t], ft, us, d_w[t], qed_child_id(a.seed, d_id[t], a.step, 3u - s2));
            }
        }
    }
}

template <int PHASE>
static void launch_photons(const QedArgs &ap, int key, unsigned nb, hipStream_t s) {
    switch (key) {
        case 21: qed_photon_kernel<2, 1, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
        case 22: qed_photon_kernel<2, 2, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
        case 31: qed_photon_kernel<3, 1, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
        case 32: qed_photon_kernel<3, 2, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
        case 24: qed_photon_kernel<2, 4, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
        case 34: qed_photon_kernel<3, 4, PHASE><<<nb, QED_PHOTON_THREADS, 0, s>>>(ap); break;
    }
}

hipError_t launch_mlp_for_qed(Ctx *c, const void *mlp, const QedSpeciesView &v, int proc, float *out,
                              hipStream_t s);

static QedSpecies view_of(const pic_particles *p, int dim) {
    QedSpecies q{};
    q.cell = p->cell;
    for (int d = 0; d < 3; ++d) {
        q.off[d] = p->off[d];
        q.u[d] = (float *)p->u[d];
    }
    q.w = (float *)p->w;
    q.chi = p->chi;
    q.tau = p->tau;
    q.tau_thr = p->tau_thr;
    q.id = p->id;
    q.n = p->n;
    q.capacity = p->capacity;
    q.n_dev = (unsigned long long *)p->n_dev;
    (void)dim;
    return q;
}

hipError_t launch_qed(Ctx *c, const pic_qed_args *qa, hipStream_t s) {
    const pic_config &cfg = c->cfg;
    QedArgs a{};
    const pic_particles *sp[3] = {qa->electrons, qa->positrons, qa->photons};
    for (int k = 0; k < 3; ++k) {
        a.has[k] = sp[k] != nullptr;
        if (sp[k]) a.sp[k] = view_of(sp[k], c->dim);
    }
    for (int d = 0; d < 3; ++d) {
        a.F[d] = (const float *)qa->fields->E[d];
        a.F[3 + d] = (const float *)qa->fields->B[d];
        a.ng[d] = (int)cfg.n[d];
        a.inv_d[d] = (float)(1.0 / cfg.d[d]);
    }
    a.tab = c->qed.dev;
    a.bx = c->bits[0];
    a.by = c->bits[1];
    a.dim = c->dim;
    a.order = cfg.order;
    a.dt = (float)cfg.dt;
    a.rate_scale = QED_A / cfg.hbar_omega_mc2;
    a.hbar_w = (float)cfg.hbar_omega_mc2;
    a.emin = (float)qa->photon_min_energy;
    a.seed = cfg.seed;
    a.step = qa->step;
    a.method2 = qa->mode == PIC_QED_METHOD2;
    a.absorb_x = absorbing_x(cfg);
    a.status = c->status;
    // photons first (their pairs are created from this step's photons only),
    // then the leptons that existed at the start of the step
    if (sp[2] && sp[2]->n > 0) {
        QedArgs ap = a;
        const unsigned nb = (unsigned)((sp[2]->n + QED_PHOTON_THREADS - 1) / QED_PHOTON_THREADS);
        const int key = c->dim * 10 + cfg.order;
        if (qa->mode == PIC_QED_MLP) {
            // move and chi_gamma first: the network answers at this step's chi
            launch_photons<PH_MOVE>(ap, key, nb, s);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            QedSpeciesView v{sp[2]->chi, sp[2]->id, (const float *)sp[2]->w, sp[2]->n, cfg.seed, qa->step};
            e = launch_mlp_for_qed(c, qa->mlp, v, QED_PAIR, c->mlp_scratch, s);
            if (e != hipSuccess) return e;
            ap.mlp_out = c->mlp_scratch;
            launch_photons<PH_DECAY>(ap, key, nb, s);
        } else {
            launch_photons<PH_ALL>(ap, key, nb, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int k = 0; k < 2; ++k) {
        if (!sp[k] || sp[k]->n == 0) continue;
        QedArgs al = a;
        if (qa->mode == PIC_QED_MLP) {
            QedSpeciesView v{sp[k]->chi, sp[k]->id, (const float *)sp[k]->w, sp[k]->n, cfg.seed, qa->step};
            hipError_t e = launch_mlp_for_qed(c, qa->mlp, v, QED_COMPTON, c->mlp_scratch, s);
            if (e != hipSuccess) return e;
            al.mlp_out = c->mlp_scratch;
        }
        qed_lepton_kernel<<<(unsigned)((sp[k]->n + QED_THREADS - 1) / QED_THREADS), QED_THREADS, 0, s>>>(al, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// table lookups exposed for the tests (one thread per query)
__global__ void qed_lookup_kernel(const float *tab, int proc, int what, const float *chi, const float *r,
                                  int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = what == 0 ? qed_rate_F(tab, proc, chi[i]) : qed_inverse(tab, proc, chi[i], r[i]);
}

hipError_t launch_qed_lookup(Ctx *c, int proc, int what, const float *chi, const float *r, int64_t n,
                             float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    qed_lookup_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c->qed.dev, proc, what, chi, r, n, out);
    return hipGetLastError();
}

}  // namespace pic
