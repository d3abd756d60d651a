// abi.hip -- the extern "C" entry points of libpic: argument validation,
// context lifetime, scratch management, launch dispatch.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "pic_internal.h"

namespace pic {

static thread_local std::string g_init_error;

pic_status fail(Ctx *c, pic_status s, const std::string &msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return s;
}

static pic_status hip_fail(Ctx *c, hipError_t e, const char *what) {
    return fail(c, PIC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Scratch that an enqueueing call outgrows is not freed there: work already
// queued (on any stream) may still use it, and a free would have to wait for
// the whole device.  The old buffer is retired and released by the next
// pic_reserve or by pic_destroy, which synchronize anyway.
static void retire(Ctx *c, void *p) {
    if (p) c->retired.push_back(p);
}

static void release_retired(Ctx *c) {
    if (c->retired.empty()) return;
    hipDeviceSynchronize();
    for (void *p : c->retired) hipFree(p);
    c->retired.clear();
}

pic_status ensure_partials(Ctx *c, size_t n) {
    if (n <= c->partials_cap) return PIC_OK;
    retire(c, c->partials);
    c->partials = nullptr;
    c->partials_cap = 0;
    size_t cap = n + n / 4 + 64;
    if (hipMalloc(&c->partials, cap * sizeof(double)) != hipSuccess) {
        c->partials = nullptr;
        return fail(c, PIC_E_NOMEM, "cannot allocate reduction partials");
    }
    c->partials_cap = cap;
    return PIC_OK;
}

pic_status ensure_strag_list(Ctx *c, int64_t n) {
    if (!c->bin_count) {
        if (hipMalloc(&c->bin_count, sizeof(uint32_t) * (size_t)c->ntiles) != hipSuccess ||
            hipMalloc(&c->bin_wmax, sizeof(uint32_t) * (size_t)c->ntiles) != hipSuccess ||
            hipMalloc(&c->strag_tile, sizeof(uint32_t) * (size_t)c->ntiles) != hipSuccess ||
            hipMalloc(&c->bin_start, sizeof(int64_t) * ((size_t)c->ntiles + 1)) != hipSuccess)
            return fail(c, PIC_E_NOMEM, "cannot allocate the tile bins");
    }
    if ((size_t)n <= c->strag_cap) return PIC_OK;
    retire(c, c->strag_list);
    retire(c, c->bin_list);
    retire(c, c->bin_rank);
    c->strag_list = c->bin_list = nullptr;
    c->bin_rank = nullptr;
    c->strag_cap = 0;
    const size_t cap = (size_t)n + (size_t)n / 8 + 1024;
    if (hipMalloc(&c->strag_list, cap * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->bin_list, cap * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->bin_rank, cap * sizeof(uint32_t)) != hipSuccess)
        return fail(c, PIC_E_NOMEM, "cannot allocate the straggler lists");
    c->strag_cap = cap;
    return PIC_OK;
}

pic_status ensure_sort_scratch(Ctx *c, int64_t n) {
    const int64_t items = 256 * 16;
    const int64_t nblocks = (n + items - 1) / items;
    const size_t hist_need = (size_t)(256 * nblocks + (256 * nblocks + items - 1) / items + 16);
    if (!c->inc && hipMalloc(&c->inc, inc_scratch_words(c->ntiles) * 4) != hipSuccess) {
        c->inc = nullptr;
        return fail(c, PIC_E_NOMEM, "cannot allocate sort scratch");
    }
    if ((size_t)n <= c->sort_cap && hist_need <= c->hist_cap) return PIC_OK;
    for (int b = 0; b < 2; ++b) {
        retire(c, c->keys[b]);
        retire(c, c->vals[b]);
        c->keys[b] = c->vals[b] = nullptr;
    }
    retire(c, c->hist);
    retire(c, c->final_perm);
    c->hist = c->final_perm = nullptr;
    c->sort_cap = c->hist_cap = 0;
    size_t cap = (size_t)n + (size_t)n / 8 + 1024;
    size_t hcap = hist_need + hist_need / 8 + 1024;
    bool ok = true;
    for (int b = 0; b < 2; ++b) {
        ok &= hipMalloc(&c->keys[b], cap * 4) == hipSuccess;
        ok &= hipMalloc(&c->vals[b], cap * 4) == hipSuccess;
    }
    ok &= hipMalloc(&c->hist, hcap * 4) == hipSuccess;
    ok &= hipMalloc(&c->final_perm, cap * 4) == hipSuccess;
    if (!ok) return fail(c, PIC_E_NOMEM, "cannot allocate sort scratch");
    c->sort_cap = cap;
    c->hist_cap = hcap;
    return PIC_OK;
}

pic_status ensure_mlp_scratch(Ctx *c, int64_t nmax) {
    if ((size_t)(2 * nmax) <= c->mlp_scratch_cap) return PIC_OK;
    retire(c, c->mlp_scratch);
    c->mlp_scratch = nullptr;
    c->mlp_scratch_cap = 0;
    const size_t cap = (size_t)(2 * nmax) + (size_t)nmax / 2 + 1024;
    if (hipMalloc(&c->mlp_scratch, cap * sizeof(float)) != hipSuccess) {
        c->mlp_scratch = nullptr;
        return fail(c, PIC_E_NOMEM, "cannot allocate network outputs");
    }
    c->mlp_scratch_cap = cap;
    return PIC_OK;
}

pic_status reserve(Ctx *c, int64_t n) {
    pic_status st = ensure_strag_list(c, n);
    if (st == PIC_OK && c->cfg.precision == PIC_FP32_MIXED) st = ensure_sort_scratch(c, n);
    if (st == PIC_OK && c->qed.dev) st = ensure_mlp_scratch(c, n);
    release_retired(c);
    return st;
}

hipError_t set_tiled_lds_limit(size_t bytes);
hipError_t set_sort_lds_limit(size_t bytes);

}  // namespace pic

using namespace pic;

static int ceil_log2(int64_t v) {
    int b = 0;
    while ((1ll << b) < v) ++b;
    return b;
}

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

extern "C" void pic_destroy(void *ctx);

extern "C" pic_status pic_init(const pic_config *cfg, void **out) {
    if (!out) return fail(nullptr, PIC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, PIC_E_ARG, "config is NULL");
    if (cfg->dim != 2 && cfg->dim != 3)
        return fail(nullptr, PIC_E_UNSUPPORTED, "dim must be 2 (2D3V) or 3 (3D3V)");
    if (cfg->order != 1 && cfg->order != 2 && cfg->order != 4)
        return fail(nullptr, PIC_E_UNSUPPORTED, "order must be 1 (CIC), 2 (quadratic) or 4 (quartic)");
    if (cfg->precision != PIC_FP32_MIXED && cfg->precision != PIC_FP64_PLAIN)
        return fail(nullptr, PIC_E_UNSUPPORTED, "precision must be PIC_FP32_MIXED or PIC_FP64_PLAIN");
    const int dim = cfg->dim;
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            if (cfg->n[a] < 8 || cfg->n[a] > (1 << 20))
                return fail(nullptr, PIC_E_ARG, "cells per axis must be in [8, 2^20]");
            if (!finite_pos(cfg->d[a])) return fail(nullptr, PIC_E_ARG, "cell sizes must be > 0");
            s += 1.0 / (cfg->d[a] * cfg->d[a]);
            if (cfg->bc[a] != PIC_BC_PERIODIC && !(a == 0 && absorbing_x(*cfg)))
                return fail(nullptr, PIC_E_UNSUPPORTED, "boundaries: periodic, or absorbing along x");
        } else if (cfg->n[a] != 1) {
            return fail(nullptr, PIC_E_ARG, "n[2] must be 1 in 2D");
        }
    }
    if (!finite_pos(cfg->dt)) return fail(nullptr, PIC_E_ARG, "dt must be > 0");
    if (cfg->dt * sqrt(s) > 1.0 + 1e-12)
        return fail(nullptr, PIC_E_CFL, "dt exceeds the Courant limit 1/sqrt(sum 1/d^2)");
    // the deposit stencils assume a move shorter than one cell per axis with margin
    for (int a = 0; a < dim; ++a)
        if (cfg->dt / cfg->d[a] > 0.999)
            return fail(nullptr, PIC_E_CFL, "dt / d above 0.999 on one axis (extreme cell aspect ratio)");
    if (!(cfg->hbar_omega_mc2 >= 0.0) || !isfinite(cfg->hbar_omega_mc2))
        return fail(nullptr, PIC_E_ARG, "hbar_omega_mc2 must be >= 0");
    if (cfg->pusher != PIC_PUSH_BORIS && cfg->pusher != PIC_PUSH_VAY)
        return fail(nullptr, PIC_E_ARG, "pusher must be PIC_PUSH_BORIS or PIC_PUSH_VAY");
    if (cfg->drift < 0 || cfg->drift > 4) return fail(nullptr, PIC_E_ARG, "drift must be in [0, 4]");

    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return fail(nullptr, PIC_E_NOMEM, "cannot allocate context");
    c->cfg = *cfg;
    c->dim = dim;
    c->drift = cfg->drift;
    int64_t ncell = cfg->n[0] * cfg->n[1] * cfg->n[2];
    int total_bits = 0;
    for (int a = 0; a < 3; ++a) {
        c->bits[a] = a < dim ? ceil_log2(cfg->n[a]) : 0;
        total_bits += c->bits[a];
    }
    if (cfg->precision == PIC_FP32_MIXED && total_bits > 31) {
        delete c;
        return fail(nullptr, PIC_E_UNSUPPORTED, "packed cell index needs more than 31 bits");
    }
    if (ncell > (int64_t)1 << 31) {
        delete c;
        return fail(nullptr, PIC_E_UNSUPPORTED, "more than 2^31 cells");
    }
    c->ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        int t = cfg->tile[a];
        if (a >= dim) t = 1;
        else if (t == 0) t = dim == 2 ? 16 : (a == 2 ? 4 : 8);
        if (t < 1 || cfg->n[a] % t != 0) {
            delete c;
            return fail(nullptr, PIC_E_ARG, "tile size must divide the cell count on every axis");
        }
        c->tile[a] = t;
        c->ntile_axis[a] = (int)(cfg->n[a] / t);
        c->ntiles *= c->ntile_axis[a];
        // window: tile, drift, and the stencil reach [c-2, c+3] ([c-3, c+4] quartic)
        c->win[a] = a < dim ? t + 2 * c->drift + (cfg->order == 4 ? 7 : 5) : 1;
        if (a < dim && c->win[a] > cfg->n[a] && cfg->precision == PIC_FP32_MIXED) {
            delete c;
            return fail(nullptr, PIC_E_UNSUPPORTED, "grid smaller than one tile window (tile + 2 drift + stencil reach)");
        }
    }
    if (c->tile[0] * c->tile[1] * c->tile[2] > 4096) {
        delete c;
        return fail(nullptr, PIC_E_UNSUPPORTED, "more than 4096 cells per tile");
    }
    // fields: 6 float planes; current: 3 int64 planes (fixed point); the
    // push kernel's own static LDS (its reduction slots) takes under 1 KB
    c->lds_bytes = (size_t)c->win[0] * c->win[1] * c->win[2] * (6 * sizeof(float) + 3 * sizeof(int64_t));
    if (cfg->precision == PIC_FP32_MIXED && c->lds_bytes + 1024 > 160 * 1024) {
        delete c;
        return fail(nullptr, PIC_E_UNSUPPORTED, "tile window does not fit in 160 KB of LDS");
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->status, 32);
    if (e == hipSuccess) e = hipMemset(c->status, 0, 32);
    if (e == hipSuccess && cfg->precision == PIC_FP32_MIXED && c->lds_bytes > 64 * 1024)
        e = set_tiled_lds_limit(c->lds_bytes);
    const size_t sort_lds = sort_lds_bytes(c->tile[0] * c->tile[1] * c->tile[2]);
    if (e == hipSuccess && cfg->precision == PIC_FP32_MIXED && sort_lds > 64 * 1024)
        e = set_sort_lds_limit(sort_lds);
    if (e != hipSuccess) {
        pic_status st = hip_fail(nullptr, e, "pic_init");
        if (c->status) hipFree(c->status);
        delete c;
        return st;
    }
    if (e == hipSuccess && absorbing_x(*cfg))
        e = hipMalloc(&c->mur_old, sizeof(double) * 8 * (size_t)cfg->n[1] * (size_t)cfg->n[2]);
    if (e == hipSuccess && cfg->bc[0] == PIC_BC_ABSORB2)
        e = hipMalloc(&c->mur_hist, sizeof(double) * 8 * (size_t)cfg->n[1] * (size_t)cfg->n[2]);
    if (e != hipSuccess) {
        pic_status st = hip_fail(nullptr, e, "pic_init");
        pic_destroy(c);
        return st;
    }
    if (hipMalloc(&c->gauss_part, sizeof(double) * GAUSS_PART) != hipSuccess) {
        pic_destroy(c);
        return fail(nullptr, PIC_E_NOMEM, "cannot allocate the residual partials");
    }
    // device address of the static scratch of pic_gather_push_deposit_noalloc
    // on this device (looked up once per device)
    e = noalloc_scratch_init(&c->noalloc_scratch);
    if (e != hipSuccess) {
        pic_status st = hip_fail(nullptr, e, "pic_init: no-allocation scratch address");
        pic_destroy(c);
        return st;
    }
    if (ensure_partials(c, 2 * (size_t)c->ntiles + 1024) != PIC_OK) {
        g_init_error = c->err;
        pic_destroy(c);
        return PIC_E_NOMEM;
    }
    if (cfg->hbar_omega_mc2 > 0.0) {
        e = build_qed_tables(&c->qed, nullptr);
        if (e != hipSuccess) {
            pic_status st = hip_fail(nullptr, e, "pic_init: QED tables");
            pic_destroy(c);
            return st;
        }
    }
    *out = c;
    return PIC_OK;
}

extern "C" void pic_destroy(void *ctx) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    hipFree(c->status);
    hipFree(c->partials);
    hipFree(c->strag_list);
    hipFree(c->bin_list);
    hipFree(c->bin_rank);
    hipFree(c->bin_count);
    hipFree(c->bin_wmax);
    hipFree(c->strag_tile);
    hipFree(c->bin_start);
    for (int b = 0; b < 2; ++b) {
        hipFree(c->keys[b]);
        hipFree(c->vals[b]);
    }
    hipFree(c->hist);
    hipFree(c->final_perm);
    hipFree(c->inc);
    hipFree(c->multi_scratch);
    hipFree(c->qed.dev);
    hipFree(c->mlp_scratch);
    hipFree(c->mur_old);
    hipFree(c->mur_hist);
    hipFree(c->gauss_part);
    for (void *p : c->retired) hipFree(p);
    delete c;
}

extern "C" pic_status pic_reserve(void *ctx, int64_t particles) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (particles < 0 || particles >= ((int64_t)1 << 31)) return fail(c, PIC_E_ARG, "particles must be in [0, 2^31)");
    hipSetDevice(c->device);
    return reserve(c, particles);
}

extern "C" pic_status pic_set_laser(void *ctx, const pic_laser *laser, double t) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!laser || !isfinite(t)) return fail(c, PIC_E_ARG, "null laser or non-finite time");
    if (!absorbing_x(c->cfg)) return fail(c, PIC_E_ARG, "injection needs absorbing x faces");
    if (!isfinite(laser->a0) || !isfinite(laser->t0) ||
        (laser->a0 != 0.0 && !(laser->waist > 0.0 && laser->duration > 0.0)))
        return fail(c, PIC_E_ARG, "laser: finite a0 and t0, positive waist and duration");
    c->laser = *laser;
    c->time = t;
    return PIC_OK;
}

extern "C" const char *pic_last_error(const void *ctx) {
    const Ctx *c = (const Ctx *)ctx;
    return c ? c->err.c_str() : g_init_error.c_str();
}

extern "C" pic_status pic_get_layout(const void *ctx, int32_t bits[3], int32_t tile[3], int64_t *ntiles) {
    const Ctx *c = (const Ctx *)ctx;
    if (!c) return PIC_E_ARG;
    for (int a = 0; a < 3; ++a) {
        if (bits) bits[a] = c->bits[a];
        if (tile) tile[a] = c->tile[a];
    }
    if (ntiles) *ntiles = c->ntiles;
    return PIC_OK;
}

static pic_status check_fields(Ctx *c, const pic_fields *f) {
    if (!f) return fail(c, PIC_E_ARG, "fields is NULL");
    for (int a = 0; a < 3; ++a)
        if (!f->E[a] || !f->B[a] || !f->J[a]) return fail(c, PIC_E_ARG, "a field plane is NULL");
    return PIC_OK;
}

// checks shared by the push entry points; PIC_OK with p->n == 0 means a no-op
pic_status pic::validate_push_args(Ctx *c, const pic_species *sp, const pic_particles *p,
                                   const pic_fields *fields) {
    if (!sp || !p) return fail(c, PIC_E_ARG, "species or particles is NULL");
    if (!(sp->m > 0.0) || !isfinite(sp->q) || !isfinite(sp->w0))
        return fail(c, PIC_E_ARG, "species mass must be > 0 and charge/weight finite");
    if (p->n < 0) return fail(c, PIC_E_ARG, "negative particle count");
    pic_status st = check_fields(c, fields);
    if (st != PIC_OK) return st;
    if (p->n == 0) return PIC_OK;  // nothing to push; the arrays may be NULL
    for (int a = 0; a < 3; ++a)
        if (!p->u[a]) return fail(c, PIC_E_ARG, "momentum array is NULL");
    if (absorbing_x(c->cfg) && !p->w)
        return fail(c, PIC_E_ARG, "absorbing x faces need per-particle weights (absorbed particles get w = 0)");
    if (c->cfg.precision == PIC_FP32_MIXED) {
        if (!p->cell || !p->tile_start) return fail(c, PIC_E_ARG, "cell or tile_start is NULL");
        for (int a = 0; a < c->dim; ++a)
            if (!p->off[a]) return fail(c, PIC_E_ARG, "offset array is NULL");
        if (p->n >= ((int64_t)1 << 31)) return fail(c, PIC_E_UNSUPPORTED, "more than 2^31 particles");
    } else {
        for (int a = 0; a < c->dim; ++a)
            if (!p->x[a]) return fail(c, PIC_E_ARG, "position array is NULL");
    }
    return PIC_OK;
}

extern "C" pic_status pic_gather_push_deposit(void *ctx, const pic_species *sp, const pic_particles *p,
                                              const pic_fields *fields, double *diag, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    pic_status st = validate_push_args(c, sp, p, fields);
    if (st != PIC_OK || p->n == 0) return st;
    hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = c->cfg.precision == PIC_FP32_MIXED ? launch_gpd_tiled(c, sp, p, fields, diag, s)
                                                      : launch_gpd_plain(c, sp, p, fields, diag, s);
    if (e != hipSuccess) return hip_fail(c, e, "pic_gather_push_deposit");
    return PIC_OK;
}

extern "C" pic_status pic_gather_push_deposit_multi(void *ctx, int32_t nsp, const pic_species *sp,
                                                    const pic_particles *const *p, const pic_fields *fields,
                                                    double *diag, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (nsp < 1 || nsp > PIC_MAX_SPECIES) return fail(c, PIC_E_ARG, "nsp must be in [1, PIC_MAX_SPECIES]");
    if (!sp || !p) return fail(c, PIC_E_ARG, "species or particles is NULL");
    int64_t total = 0;
    for (int k = 0; k < nsp; ++k) {
        pic_status st = validate_push_args(c, &sp[k], p[k], fields);
        if (st != PIC_OK) return st;
        total += p[k]->n;
        for (int j = 0; j < k; ++j)
            if (p[j]->n > 0 && p[k]->n > 0 && p[j]->cell == p[k]->cell && p[j]->u[0] == p[k]->u[0])
                return fail(c, PIC_E_ARG, "a species is listed twice");
    }
    if (total == 0) return PIC_OK;
    hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (c->cfg.precision != PIC_FP32_MIXED) {
        // the plain FP64 path has no tiles to share: one species after another
        for (int k = 0; k < nsp && e == hipSuccess; ++k)
            if (p[k]->n > 0) e = launch_gpd_plain(c, &sp[k], p[k], fields, diag, s);
    } else {
        // species with particles only (an empty one may have no arrays at all)
        pic_species spk[PIC_MAX_SPECIES];
        const pic_particles *pk[PIC_MAX_SPECIES];
        int m = 0;
        for (int k = 0; k < nsp; ++k)
            if (p[k]->n > 0) {
                spk[m] = sp[k];
                pk[m++] = p[k];
            }
        PushScratch ps[PIC_MAX_SPECIES];
        size_t need = 0;
        for (int k = 0; k < m; ++k) need += carve_push_scratch(c, pk[k]->n, nullptr, ps[k]);
        if (need > c->multi_cap) {
            retire(c, c->multi_scratch);
            c->multi_scratch = nullptr;
            c->multi_cap = 0;
            const size_t cap = need + need / 8 + 4096;
            if (hipMalloc(&c->multi_scratch, cap) != hipSuccess) {
                c->multi_scratch = nullptr;
                return fail(c, PIC_E_NOMEM, "cannot allocate the several-species push scratch");
            }
            c->multi_cap = cap;
        }
        size_t off = 0;
        for (int k = 0; k < m; ++k) off += carve_push_scratch(c, pk[k]->n, c->multi_scratch + off, ps[k]);
        e = launch_gpd_tiled_multi(c, m, spk, pk, fields, diag, s, ps);
    }
    if (e != hipSuccess) return hip_fail(c, e, "pic_gather_push_deposit_multi");
    return PIC_OK;
}

extern "C" pic_status pic_yee_step(void *ctx, int32_t half, const pic_fields *fields, double *diag,
                                   void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (half != 1 && half != 2) return fail(c, PIC_E_ARG, "half must be 1 or 2");
    pic_status st = check_fields(c, fields);
    if (st != PIC_OK) return st;
    hipSetDevice(c->device);
    hipError_t e = launch_yee(c, half, fields, diag, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_yee_step");
    return PIC_OK;
}

static pic_status check_particles_layout(Ctx *c, const pic_particles *p) {
    for (int a = 0; a < 3; ++a)
        if (!p->u[a]) return fail(c, PIC_E_ARG, "momentum array is NULL");
    if (c->cfg.precision == PIC_FP32_MIXED) {
        if (!p->cell) return fail(c, PIC_E_ARG, "cell array is NULL");
        for (int a = 0; a < c->dim; ++a)
            if (!p->off[a]) return fail(c, PIC_E_ARG, "offset array is NULL");
    } else {
        for (int a = 0; a < c->dim; ++a)
            if (!p->x[a]) return fail(c, PIC_E_ARG, "position array is NULL");
    }
    return PIC_OK;
}

extern "C" pic_status pic_deposit_rho(void *ctx, const pic_species *sp, const pic_particles *p, int32_t at_half,
                                      double *rho, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!sp || !p || !rho) return fail(c, PIC_E_ARG, "species, particles or rho is NULL");
    if (!isfinite(sp->q) || !isfinite(sp->w0)) return fail(c, PIC_E_ARG, "charge and weight must be finite");
    if (at_half != 0 && at_half != 1) return fail(c, PIC_E_ARG, "at_half must be 0 or 1");
    if (p->n < 0) return fail(c, PIC_E_ARG, "negative particle count");
    if (p->n == 0) return PIC_OK;
    pic_status st = check_particles_layout(c, p);
    if (st != PIC_OK) return st;
    hipSetDevice(c->device);
    hipError_t e = launch_rho(c, sp, p, at_half, rho, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_deposit_rho");
    return PIC_OK;
}

extern "C" pic_status pic_gauss_residual(void *ctx, const pic_fields *fields, const double *rho,
                                         double *residual, double *diag, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!fields || !rho) return fail(c, PIC_E_ARG, "fields or rho is NULL");
    for (int a = 0; a < c->dim; ++a)
        if (!fields->E[a]) return fail(c, PIC_E_ARG, "an E plane is NULL");
    hipSetDevice(c->device);
    hipError_t e = launch_gauss(c, fields, rho, residual, diag, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_gauss_residual");
    return PIC_OK;
}

extern "C" pic_status pic_beam_fields(void *ctx, const pic_beam *beam, const pic_fields *fields, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!beam || !fields) return fail(c, PIC_E_ARG, "beam or fields is NULL");
    // written: E_x, E_y, B_z, and in 3D E_z, B_y
    if (!fields->E[0] || !fields->E[1] || !fields->B[2] || (c->dim == 3 && (!fields->E[2] || !fields->B[1])))
        return fail(c, PIC_E_ARG, "an E or B plane is NULL");
    if (!(beam->gamma >= 1.0) || !isfinite(beam->gamma) || !isfinite(beam->charge) || !isfinite(beam->density))
        return fail(c, PIC_E_ARG, "beam: gamma >= 1, finite charge and density");
    for (int a = 0; a < c->dim; ++a)
        if (!finite_pos(beam->sigma[a]) || !isfinite(beam->center[a]))
            return fail(c, PIC_E_ARG, "beam: sigmas > 0 and a finite centre");
    hipSetDevice(c->device);
    hipError_t e = launch_beam_fields(c, beam, fields, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_beam_fields");
    return PIC_OK;
}

extern "C" pic_status pic_sort(void *ctx, const pic_particles *src, const pic_particles *dst,
                               void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (c->cfg.precision != PIC_FP32_MIXED)
        return fail(c, PIC_E_UNSUPPORTED, "pic_sort works on the FP32 particle layout");
    if (!src || !dst) return fail(c, PIC_E_ARG, "src or dst is NULL");
    if (src->n < 0 || src->n >= ((int64_t)1 << 31)) return fail(c, PIC_E_ARG, "bad particle count");
    if (!dst->tile_start) return fail(c, PIC_E_ARG, "dst->tile_start is NULL");
    if (src->n > 0) {
        if (!src->cell || !dst->cell) return fail(c, PIC_E_ARG, "cell array is NULL");
        if (src->cell == dst->cell) return fail(c, PIC_E_ARG, "src and dst alias");
        for (int a = 0; a < c->dim; ++a)
            if (!src->off[a] || !dst->off[a]) return fail(c, PIC_E_ARG, "offset array is NULL");
        for (int a = 0; a < 3; ++a)
            if (!src->u[a] || !dst->u[a]) return fail(c, PIC_E_ARG, "momentum array is NULL");
        if ((src->w != nullptr) != (dst->w != nullptr) && src->w)
            return fail(c, PIC_E_ARG, "src has weights but dst has none");
        if (src->chi && !dst->chi) return fail(c, PIC_E_ARG, "src has chi but dst has none");
        if ((src->tau && !dst->tau) || (src->tau_thr && !dst->tau_thr) || (src->id && !dst->id))
            return fail(c, PIC_E_ARG, "src has QED arrays that dst lacks");
    }
    hipSetDevice(c->device);
    if (src->n > 0) {
        pic_status st = ensure_sort_scratch(c, src->n);
        if (st != PIC_OK) return st;
    }
    hipError_t e = launch_sort(c, src, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_sort");
    return PIC_OK;
}

extern "C" pic_status pic_check(void *ctx, void *stream, uint32_t *flags, uint64_t *stragglers) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_check: stream synchronize");
    uint32_t h[4] = {0, 0, 0, 0};
    e = hipMemcpy(h, c->status, 16, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(c->status, 0, 16);
    if (e != hipSuccess) return hip_fail(c, e, "pic_check: status word");
    if (flags) *flags = h[0];
    if (stragglers) *stragglers = (uint64_t)h[2] | ((uint64_t)h[3] << 32);
    if (h[0] & PIC_F_CAPACITY) return fail(c, PIC_E_CAPACITY, "particle creation hit capacity");
    if (h[0] & (PIC_F_NONFINITE | PIC_F_OFFSET))
        return fail(c, PIC_E_STATE, "non-finite momentum or offset outside [0,1) seen");
    return PIC_OK;
}

static pic_status check_qed_species(Ctx *c, const pic_particles *p, const char *name) {
    if (!p) return PIC_OK;
    if (p->n < 0 || p->n > p->capacity)
        return fail(c, PIC_E_ARG, std::string(name) + ": need 0 <= n <= capacity");
    if (p->n == 0 && p->capacity == 0) return PIC_OK;
    if (!p->cell || !p->u[0] || !p->u[1] || !p->u[2] || !p->tau || !p->tau_thr || !p->id || !p->n_dev)
        return fail(c, PIC_E_ARG, std::string(name) + ": cell, u, tau, tau_thr, id and n_dev are required");
    for (int a = 0; a < c->dim; ++a)
        if (!p->off[a]) return fail(c, PIC_E_ARG, std::string(name) + ": offset array is NULL");
    return PIC_OK;
}

extern "C" pic_status pic_qed_step(void *ctx, const pic_qed_args *qa, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!qa) return fail(c, PIC_E_ARG, "args is NULL");
    if (c->cfg.precision != PIC_FP32_MIXED)
        return fail(c, PIC_E_UNSUPPORTED, "pic_qed_step works on the FP32 particle layout");
    if (!(c->cfg.hbar_omega_mc2 > 0.0) || !c->qed.dev)
        return fail(c, PIC_E_ARG, "QED needs hbar_omega_mc2 > 0 at pic_init");
    if (qa->mode != PIC_QED_TABLE && qa->mode != PIC_QED_MLP && qa->mode != PIC_QED_METHOD2)
        return fail(c, PIC_E_ARG, "bad mode");
    if (qa->mode == PIC_QED_MLP && !qa->mlp) return fail(c, PIC_E_ARG, "PIC_QED_MLP needs a network");
    pic_status st = check_fields(c, qa->fields);
    if (st != PIC_OK) return st;
    const pic_particles *sp[3] = {qa->electrons, qa->positrons, qa->photons};
    const char *names[3] = {"electrons", "positrons", "photons"};
    int64_t nmax = 0;
    for (int k = 0; k < 3; ++k) {
        st = check_qed_species(c, sp[k], names[k]);
        if (st != PIC_OK) return st;
        if (sp[k] && k < 2 && sp[k]->n > 0 && !sp[k]->chi)
            return fail(c, PIC_E_ARG, "leptons need the chi array written by the push");
        // a decayed photon is removed through its weight
        if (sp[k] && k == 2 && (sp[k]->n > 0 || sp[k]->capacity > 0) && !sp[k]->w)
            return fail(c, PIC_E_ARG, "photons need per-particle weights (a decayed photon gets w = 0)");
        // the network reads chi_gamma, which the photon step writes there first
        if (sp[k] && k == 2 && sp[k]->n > 0 && qa->mode == PIC_QED_MLP && !sp[k]->chi)
            return fail(c, PIC_E_ARG, "PIC_QED_MLP needs the photons' chi array");
        if (sp[k] && sp[k]->n > nmax) nmax = sp[k]->n;
    }
    hipSetDevice(c->device);
    if (qa->mode == PIC_QED_MLP) {
        st = ensure_mlp_scratch(c, nmax);
        if (st != PIC_OK) return st;
    }
    hipError_t e = launch_qed(c, qa, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_qed_step");
    return PIC_OK;
}

extern "C" pic_status pic_mlp_forward(void *ctx, const void *mlp, const float *x, int64_t n, float *y,
                                      void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!mlp || (n > 0 && (!x || !y)) || n < 0) return fail(c, PIC_E_ARG, "null or bad argument");
    hipSetDevice(c->device);
    hipError_t e = launch_mlp_forward(mlp, x, n, y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_mlp_forward");
    return PIC_OK;
}

extern "C" pic_status pic_mlp_grad(void *ctx, const void *mlp, const float *x, const float *t, int64_t n,
                                   float *grad, float *loss, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!mlp || !x || !t || !grad || n <= 0) return fail(c, PIC_E_ARG, "null or bad argument");
    hipSetDevice(c->device);
    hipError_t e = launch_mlp_grad(mlp, x, t, n, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_mlp_grad");
    return PIC_OK;
}

extern "C" pic_status pic_mlp_train(void *ctx, float *state, void *mlp, const float *x, const float *t,
                                    int64_t n, int32_t batch, int32_t iters, float lr, float *loss,
                                    void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!state || !mlp || !x || !t || n <= 0 || batch <= 0 || iters < 0 || !(lr > 0.0f))
        return fail(c, PIC_E_ARG, "null or bad argument");
    hipSetDevice(c->device);
    hipError_t e = launch_mlp_train(state, mlp, x, t, n, batch, iters, lr, loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_mlp_train");
    return PIC_OK;
}

extern "C" pic_status pic_qed_training_data(void *ctx, int64_t n, uint64_t seed, float *x, float *t,
                                            void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!c->qed.dev) return fail(c, PIC_E_ARG, "QED needs hbar_omega_mc2 > 0 at pic_init");
    if (n < 0 || (n > 0 && (!x || !t))) return fail(c, PIC_E_ARG, "null or bad argument");
    hipSetDevice(c->device);
    hipError_t e = launch_mlp_data(c, n, seed, x, t, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_qed_training_data");
    return PIC_OK;
}

extern "C" pic_status pic_qed_table_lookup(void *ctx, int32_t proc, int32_t what, const float *chi,
                                           const float *r, int64_t n, float *out, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    if (!c->qed.dev) return fail(c, PIC_E_ARG, "QED needs hbar_omega_mc2 > 0 at pic_init");
    if ((proc != 0 && proc != 1) || (what != 0 && what != 1) || n < 0 ||
        (n > 0 && (!chi || !out || (what == 1 && !r))))
        return fail(c, PIC_E_ARG, "null or bad argument");
    hipSetDevice(c->device);
    hipError_t e = launch_qed_lookup(c, proc, what, chi, r, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pic_qed_table_lookup");
    return PIC_OK;
}
