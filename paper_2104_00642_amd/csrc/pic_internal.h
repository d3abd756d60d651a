// pic_internal.h -- context structure and launcher declarations of libpic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pic.h"
#include "qed_internal.h"

namespace pic {

struct Ctx {
    pic_config cfg;
    int dim = 2;
    int bits[3] = {0, 0, 0};     // packed-cell field widths
    int tile[3] = {1, 1, 1};     // tile size (cells)
    int ntile_axis[3] = {1, 1, 1};
    int64_t ntiles = 1;
    int win[3] = {1, 1, 1};      // LDS window (cells) of the FP32 push
    int drift = 2;
    size_t lds_bytes = 0;
    int device = 0;
    // device status: [0] flags, [2..3] straggler count (uint64 at byte 8),
    // [4] length of the straggler list of the current push
    uint32_t *status = nullptr;
    // push scratch: stragglers of the sorted pass, their bin ranks and the
    // binned list (capacity strag_cap entries each), bin counters and starts
    int32_t *strag_list = nullptr;
    int32_t *bin_list = nullptr;
    uint32_t *bin_rank = nullptr;
    size_t strag_cap = 0;        // entries
    uint32_t *bin_count = nullptr;  // ntiles
    uint32_t *bin_wmax = nullptr;   // ntiles: bound of |q| w of each tile's bin (float bits)
    uint32_t *strag_tile = nullptr; // ntiles
    int64_t *bin_start = nullptr;   // ntiles + 1
    // FP64 block partials of the diagnostics reductions
    double *partials = nullptr;
    size_t partials_cap = 0;     // in doubles
    // sort scratch (grown on demand)
    uint32_t *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    uint32_t *hist = nullptr;
    uint32_t *final_perm = nullptr;
    size_t sort_cap = 0;         // elements
    size_t hist_cap = 0;         // entries
    // re-binning from the source's tile offsets: hint check, stayer and
    // mover counts per tile (inc_scratch_words(ntiles) words)
    uint32_t *inc = nullptr;
    // QED tables (built at init when hbar_omega_mc2 > 0) and network outputs
    QedTables qed;
    float *mlp_scratch = nullptr;
    size_t mlp_scratch_cap = 0;  // floats
    // absorbing x faces: face values of E_y, E_z saved by the E half step
    // (8 x n1 x n2 reals), for the second-order rule those of the previous
    // half step and whether they are there yet, the injected pulse and the
    // field clock
    void *mur_old = nullptr;
    void *mur_hist = nullptr;
    int mur_valid = 0;
    pic_laser laser{};
    double time = 0.0;
    // block maxima of the Gauss residual (GAUSS_PART doubles)
    double *gauss_part = nullptr;
    // device address of the library's static no-allocation scratch on this
    // context's device
    void *noalloc_scratch = nullptr;
    // scratch of the several-species push (every species' lists and
    // counters, carved like the no-allocation scratch)
    unsigned char *multi_scratch = nullptr;
    size_t multi_cap = 0;        // bytes
    // scratch outgrown by an enqueueing call, freed by pic_reserve / pic_destroy
    std::vector<void *> retired;
    std::string err;
};

// absorbing x faces (either order of the field rule)
inline bool absorbing_x(const pic_config &cfg) {
    return cfg.bc[0] == PIC_BC_ABSORB || cfg.bc[0] == PIC_BC_ABSORB2;
}

hipError_t launch_beam_fields(Ctx *c, const pic_beam *beam, const pic_fields *f, hipStream_t s);

// error helpers
pic_status fail(Ctx *c, pic_status s, const std::string &msg);
pic_status ensure_partials(Ctx *c, size_t n);
pic_status ensure_strag_list(Ctx *c, int64_t n);
pic_status ensure_sort_scratch(Ctx *c, int64_t n);
pic_status ensure_mlp_scratch(Ctx *c, int64_t nmax);

// Scratch of one push: FP64 block partials of the diagnostics, the straggler
// list, the bin list and ranks (n entries each), per-tile counters and bin
// starts.  The context's own buffers, or carved from a caller's region.
struct PushScratch {
    double *partials = nullptr;
    int32_t *strag_list = nullptr;
    int32_t *bin_list = nullptr;
    uint32_t *bin_rank = nullptr;
    uint32_t *bin_count = nullptr;   // ntiles
    uint32_t *bin_wmax = nullptr;    // ntiles
    uint32_t *strag_tile = nullptr;  // ntiles
    int64_t *bin_start = nullptr;    // ntiles + 1
    uint32_t *strag_count = nullptr; // length of the binned pass's own list (NULL: the context's)
};
// doubles of FP64 partials one push writes (FP32 tiled path, FP64 plain path)
size_t push_partials_tiled(int64_t ntiles);
size_t push_partials_plain(int64_t n);

// launchers (return hipError_t of the launch); ps = nullptr: the context's
// scratch, grown as needed
hipError_t launch_gpd_plain(Ctx *c, const pic_species *sp, const pic_particles *p,
                            const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps = nullptr);
hipError_t launch_gpd_tiled(Ctx *c, const pic_species *sp, const pic_particles *p,
                            const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps = nullptr);
// several species in one pass over the tiles; ps[k]: scratch of species k
hipError_t launch_gpd_tiled_multi(Ctx *c, int nsp, const pic_species *sp, const pic_particles *const *p,
                                  const pic_fields *f, double *diag, hipStream_t s, const PushScratch *ps);
// carves one push's scratch (FP32 tiled or FP64 plain path, n particles)
// from base; returns the bytes it takes (base = nullptr: only counts)
size_t carve_push_scratch(Ctx *c, int64_t n, unsigned char *base, PushScratch &ps);
pic_status validate_push_args(Ctx *c, const pic_species *sp, const pic_particles *p, const pic_fields *fields);
hipError_t noalloc_scratch_init(void **ptr);
hipError_t launch_yee(Ctx *c, int half, const pic_fields *f, double *diag, hipStream_t s);
hipError_t launch_sort(Ctx *c, const pic_particles *src, const pic_particles *dst,
                       hipStream_t s);
hipError_t launch_qed(Ctx *c, const pic_qed_args *qa, hipStream_t s);
hipError_t launch_qed_lookup(Ctx *c, int proc, int what, const float *chi, const float *r, int64_t n,
                             float *out, hipStream_t s);
hipError_t launch_mlp_forward(const void *mlp, const float *x, int64_t n, float *y, hipStream_t s);
hipError_t launch_mlp_grad(const void *mlp, const float *x, const float *t, int64_t n, float *grad, float *loss,
                           hipStream_t s);
hipError_t launch_mlp_train(float *state, void *mlp, const float *x, const float *t, int64_t n, int batch,
                            int iters, float lr, float *loss, hipStream_t s);
hipError_t launch_mlp_data(Ctx *c, int64_t n, uint64_t seed, float *x, float *t, hipStream_t s);
hipError_t launch_rho(Ctx *c, const pic_species *sp, const pic_particles *p, int at_half, double *rho,
                      hipStream_t s);
hipError_t launch_gauss(Ctx *c, const pic_fields *f, const double *rho, double *res, double *diag,
                        hipStream_t s);
constexpr int GAUSS_PART = 1024;
size_t sort_lds_bytes(int cells_per_tile);
size_t inc_scratch_words(int64_t ntiles);
hipError_t launch_finalize(const double *partials, int64_t nblocks, int nval, double *diag,
                           int diag_offset, double scale, hipStream_t s);

}  // namespace pic
