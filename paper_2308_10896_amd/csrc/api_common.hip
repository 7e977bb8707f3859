// C ABI entry points that need no plan: version, status strings, and the
// stand-alone moment filter.
#include <string.h>

#include "dsm_internal.h"

using namespace dsm;

extern "C" const char *dsm_version(void) { return "dsm 0.1.0 (gfx950, HIP)"; }

extern "C" const char *dsm_status_string(dsm_status status) {
    switch (status) {
        case DSM_OK: return "ok";
        case DSM_ERR_INVALID_ARG: return "invalid argument";
        case DSM_ERR_OUT_OF_MEMORY: return "out of device memory";
        case DSM_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case DSM_ERR_UNSUPPORTED: return "unsupported";
        case DSM_ERR_NO_DEVICE: return "no HIP device";
        case DSM_ERR_HIP: return "HIP runtime error";
        case DSM_ERR_DEVICE_FAULT: return "device-side fault";
    }
    return "unknown status";
}

namespace dsm {
bool valid_filter(int S, int filter, int k) {
    return (filter == DSM_FILTER_BOX || filter == DSM_FILTER_GAUSSIAN) && k >= 1 && k <= DSM_MAX_KERNEL &&
           (k & 1) == 1 && S >= 1 && S <= DSM_MAX_RESOLUTION && k <= S;
}
}  // namespace dsm

extern "C" dsm_status dsm_filter_moments(int32_t S, int32_t n_maps, int32_t filter, int32_t k, float sigma,
                                         const float *in_dev, float *out_dev, int32_t adjoint,
                                         dsm_stream stream) {
    if (!valid_filter(S, filter, k) || n_maps < 0 || n_maps > 65535) return DSM_ERR_INVALID_ARG;
    if (n_maps == 0) return DSM_OK;
    if (!in_dev || !out_dev || in_dev == out_dev) return DSM_ERR_INVALID_ARG;
    const size_t bytes = (size_t)n_maps * 2 * (size_t)S * S * sizeof(float);
    const char *a = (const char *)in_dev, *b = (const char *)out_dev;
    if (a < b + bytes && b < a + bytes) return DSM_ERR_INVALID_ARG;
    BlurJob job;
    memset(&job, 0, sizeof(job));
    job.S = S;
    job.k = k;
    filter_taps_host(filter, k, sigma, job.w);
    hipError_t e = launch_blur_uniform(job, n_maps, in_dev, out_dev, adjoint != 0, (hipStream_t)stream);
    return e == hipSuccess ? DSM_OK : DSM_ERR_HIP;
}
