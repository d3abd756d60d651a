// noalloc.hip -- the push without any allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).
//
// Every scratch buffer of one push (FP64 partials, straggler and bin lists,
// per-tile counters and bin starts) is carved from `scratch`, a static device
// array of NOALLOC_BYTES that each GPU the library runs on holds until the
// process ends.  In host code the array's name only stands for the symbol:
// its device address on the current device comes from hipGetSymbolAddress,
// taken once per device at pic_init and kept per device; kernels and copies
// get that address, never the name.  Every call on a device shares the array
// and leaves its contents behind: the counters that must start at zero are
// cleared by the push's own first kernel, and calls that overlap in time on
// one device race.
#include <mutex>

#include "pic_internal.h"

namespace pic {

constexpr size_t NOALLOC_BYTES = (size_t)PIC_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mutex;

// device address of `scratch` on the current device (looked up once per device)
hipError_t noalloc_scratch_init(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

// Carves the push's buffers from `base`; returns the bytes they take.  With
// base = nullptr only counts.
size_t carve_push_scratch(Ctx *c, int64_t n, unsigned char *base, PushScratch &ps) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        unsigned char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    if (c->cfg.precision == PIC_FP64_PLAIN) {
        ps.partials = (double *)take(sizeof(double) * push_partials_plain(n));
        return off;
    }
    const size_t nt = (size_t)c->ntiles;
    ps.partials = (double *)take(sizeof(double) * push_partials_tiled(c->ntiles));
    ps.bin_count = (uint32_t *)take(sizeof(uint32_t) * nt);
    ps.bin_wmax = (uint32_t *)take(sizeof(uint32_t) * nt);
    ps.strag_tile = (uint32_t *)take(sizeof(uint32_t) * nt);
    ps.bin_start = (int64_t *)take(sizeof(int64_t) * (nt + 1));
    ps.strag_list = (int32_t *)take(sizeof(int32_t) * (size_t)n);
    ps.bin_list = (int32_t *)take(sizeof(int32_t) * (size_t)n);
    ps.bin_rank = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    ps.strag_count = (uint32_t *)take(sizeof(uint32_t));
    return off;
}

}  // namespace pic

using namespace pic;

extern "C" pic_status pic_gather_push_deposit_noalloc(void *ctx, const pic_species *sp, const pic_particles *p,
                                                      const pic_fields *fields, double *diag, void *stream) {
    Ctx *c = (Ctx *)ctx;
    if (!c) return fail(nullptr, PIC_E_ARG, "context is NULL");
    pic_status st = validate_push_args(c, sp, p, fields);
    if (st != PIC_OK || p->n == 0) return st;
    if (!c->noalloc_scratch) return fail(c, PIC_E_HIP, "no-allocation scratch has no device address");
    PushScratch ps;
    const size_t need = carve_push_scratch(c, p->n, nullptr, ps);
    if (need > NOALLOC_BYTES)
        return fail(c, PIC_E_ARG, "push needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                      std::to_string(NOALLOC_BYTES) + " of the no-allocation entry point");
    carve_push_scratch(c, p->n, (unsigned char *)c->noalloc_scratch, ps);
    hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = c->cfg.precision == PIC_FP32_MIXED ? launch_gpd_tiled(c, sp, p, fields, diag, s, &ps)
                                                      : launch_gpd_plain(c, sp, p, fields, diag, s, &ps);
    if (e != hipSuccess) return fail(c, PIC_E_HIP, std::string("pic_gather_push_deposit_noalloc: ") +
                                                       hipGetErrorString(e));
    return PIC_OK;
}
