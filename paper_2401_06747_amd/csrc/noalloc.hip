// inpaint_solve for callers that cannot allocate: the workspace is a
// file-scope device array of fixed size instead of a caller buffer.
//
// Each GPU the library runs on holds its own copy of `scratch` from the first
// call on that GPU until the process ends. In host code the name `scratch` is
// only a host-side handle, so its device address is looked up once per device
// with hipGetSymbolAddress and every launch gets that address. A per-device
// lock serialises the calls of this process on one GPU, because they all share
// the array; a call leaves its contents behind, and the solve writes every
// workspace byte it reads before reading it.
#include <mutex>

#include "hdi_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)HDI_NOALLOC_SCRATCH_MB << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct DeviceScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;   // device address of this GPU's `scratch`
    std::mutex busy;       // held for the whole of a call on this GPU
};
DeviceScratch g_dev[MAX_DEVICES];

// The device address of the current device's array (set-up on first use).
DeviceScratch *scratch_for(int dev) {
    DeviceScratch &d = g_dev[dev];
    std::call_once(d.once, [&d] {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (d.err == hipSuccess && p == nullptr) d.err = hipErrorInvalidSymbol;
        d.ptr = d.err == hipSuccess ? p : nullptr;
    });
    return &d;
}

}  // namespace

using namespace hdi;

extern "C" {

size_t hdi_noalloc_scratch_bytes(void) { return SCRATCH_BYTES; }

int32_t inpaint_solve_noalloc(hdi_image img, const uint8_t *mask, const float *f, double *u, const double *u0,
                              const hdi_solve_params *params, hdi_solve_report *report, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !f || !u) {
        set_error("mask, f and u must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    const size_t need = hdi_inpaint_workspace_bytes(img);
    if (need > SCRATCH_BYTES) {
        set_error("a %dx%dx%d image needs %zu bytes of scratch; the no-allocation solve holds %zu "
                  "(use inpaint_solve with a workspace)", img.width, img.height, img.channels, need,
                  SCRATCH_BYTES);
        return HDI_ERR_WORKSPACE;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_error("hipGetDevice: %s (device %d)", hipGetErrorString(e), dev);
        return HDI_ERR_HIP;
    }
    DeviceScratch *d = scratch_for(dev);
    if (d->err != hipSuccess) {
        set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(d->err));
        return HDI_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(d->busy);
    NoAllocScope no_alloc;
    return inpaint_solve(img, mask, f, u, u0, d->ptr, SCRATCH_BYTES, params, report, stream);
}

}  // extern "C"
