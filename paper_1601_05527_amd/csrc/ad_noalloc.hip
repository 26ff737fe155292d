// ad_noalloc.hip -- ad_edge_dist for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// hipMalloc): the distance pass's launch plan lives in one fixed device
// array per GPU instead of a caller workspace.
//
// The array is a file-scope __device__ object.  Its host-side name only
// stands for the symbol; the device address comes from hipGetSymbolAddress,
// looked up once per device with that device current and kept per device,
// and only that address is handed to kernels.
#include "ad_internal.h"

#include <mutex>

namespace ad {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

struct ScratchSlot {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
};
static ScratchSlot scratch_slots[MAX_DEVICES];

// Device address of this device's copy of `scratch` (looked up on the first
// call made on the device).
static ad_status scratch_address(void **out) {
    int dev = 0;
    AD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(AD_ERR_UNSUPPORTED, "device index beyond the library's table");
    ScratchSlot &slot = scratch_slots[dev];
    std::call_once(slot.once, [&slot]() {
        void *p = nullptr;
        slot.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (slot.err == hipSuccess) slot.ptr = p;
    });
    if (slot.err != hipSuccess) return hip_fail(slot.err, "hipGetSymbolAddress(scratch)");
    *out = slot.ptr;
    return AD_OK;
}

}  // namespace ad

using namespace ad;

extern "C" size_t ad_edge_dist_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" ad_status ad_edge_dist_noalloc(const ad_graph *g, int32_t R, ad_dtype x_dtype, const void *x,
                                          const double *minmax, ad_dtype rho_dtype, void *rho,
                                          hipStream_t stream) {
    ad_status s = check_graph_args(g);
    if (s != AD_OK) return s;
    if (R < 1 || R > 64) return fail(AD_ERR_INVALID_ARG, "R must be in [1, 64]");
    if (x_dtype != AD_F32 && x_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "x must be F32 or F64");
    if (rho_dtype != AD_F32 && rho_dtype != AD_F64) return fail(AD_ERR_INVALID_ARG, "rho must be F32 or F64");
    if (rho_dtype == AD_F64 && x_dtype != AD_F64) return fail(AD_ERR_UNSUPPORTED, "FP64 rho needs FP64 x");
    if (g->m > 0 && (!x || !minmax || !rho)) return fail(AD_ERR_INVALID_ARG, "x, minmax or rho is NULL");
    const size_t need = edge_dist_segs_workspace(g, Segs());
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(AD_ERR_UNSUPPORTED, "the graph's distance plan needs " + std::to_string(need) +
                                             " bytes; the fixed scratch array holds " +
                                             std::to_string(NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    s = scratch_address(&ws);
    if (s != AD_OK) return s;
    return edge_dist_segs(g, R, x_dtype, x, minmax, rho_dtype, rho, ws, NOALLOC_SCRATCH_BYTES, Segs(), stream);
}
