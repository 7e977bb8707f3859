// dsm_forward for callers that cannot allocate device memory: the forward's
// temporaries live in one file-scope device array per GPU instead of a
// caller scratch buffer.  Nothing here calls hipMalloc or hipFree.
#include <mutex>

#include "plan.h"

namespace {

// Each GPU the library runs on holds its own copy of this array from the
// time the code object is loaded until the process ends.  In host code its
// name is only a stand-in for the symbol; the device address of each GPU's
// copy comes from hipGetSymbolAddress and is the only form passed to kernels.
static __device__ __align__(256) unsigned char scratch[DSM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch_dev[kMaxDevices] = {};   // address of `scratch` on each device, looked up once

// Device address of the current device's copy of `scratch`: looked up on the
// first call on that device (with that device current), cached afterwards.
dsm_status static_scratch(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return DSM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DSM_ERR_HIP;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return DSM_OK;
}

}  // namespace

extern "C" dsm_status dsm_forward_static_scratch(dsm_plan *p, const float *verts, const float *lparams,
                                                 const float *albedo, void *saved, size_t saved_bytes,
                                                 float *images, dsm_stream stream) {
    if (!p) return DSM_ERR_INVALID_ARG;
    if (p->sc_fwd_end > DSM_STATIC_SCRATCH_BYTES) return DSM_ERR_WORKSPACE_TOO_SMALL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DSM_ERR_NO_DEVICE;
    if (dev != p->device) return DSM_ERR_INVALID_ARG;
    void *buf = nullptr;
    const dsm_status st = static_scratch(dev, &buf);
    if (st != DSM_OK) return st;
    return dsm::forward_in_scratch(p, verts, lparams, albedo, saved, saved_bytes, buf, DSM_STATIC_SCRATCH_BYTES,
                                   images, (hipStream_t)stream);
}
