// Tile-size / bin-depth autotuner.  For a batch description it times a
// forward + backward pass for every candidate (raster tile side, bin
// capacity scale) on the caller's inputs and returns the fastest, keeping
// the decision in an optional text cache keyed by the batch's shape and the
// device, so later plans of the same shape skip the timing.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "dsm_internal.h"

namespace {

constexpr int kTiles[] = {8, 16, 32};
constexpr int kScales[] = {8, 32};

struct Fnv {
    unsigned long long h = 1469598103934665603ULL;
    void bytes(const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ULL;
        }
    }
    template <class T>
    void pod(const T &v) { bytes(&v, sizeof(v)); }
};

// Shape of the batch as far as it matters for speed: counts, mesh sizes,
// map and image sizes, filters, smoothing switches, and the device.
unsigned long long shape_key(const dsm_batch_desc *d) {
    Fnv f;
    f.pod(DSM_ABI_VERSION);
    f.pod(d->num_scenes);
    f.pod(d->num_lights);
    f.pod(d->num_cameras);
    f.pod(d->num_renders);
    f.pod(d->channels);
    f.pod(d->camera_antialias);
    f.bytes(d->vert_offsets, sizeof(int32_t) * ((size_t)d->num_scenes + 1));
    f.bytes(d->face_offsets, sizeof(int32_t) * ((size_t)d->num_scenes + 1));
    for (int l = 0; l < d->num_lights; ++l) {
        const dsm_light_desc &x = d->lights[l];
        f.pod(x.type);
        f.pod(x.scene);
        f.pod(x.resolution);
        f.pod(x.filter);
        f.pod(x.k);
        f.pod(x.antialias);
    }
    for (int c = 0; c < d->num_cameras; ++c) {
        f.pod(d->cameras[c].width);
        f.pod(d->cameras[c].height);
        f.pod(d->cameras[c].scene);
    }
    for (int r = 0; r < d->num_renders; ++r) {
        f.pod(d->renders[r].camera);
        f.pod(d->renders[r].light_count);
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        f.bytes(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
        f.pod(prop.multiProcessorCount);
    }
    return f.h;
}

bool cache_lookup(const char *path, unsigned long long key, int *tile, int *scale, float *ms) {
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    bool found = false;
    char line[256];
    while (fgets(line, sizeof(line), fp)) {
        unsigned long long k;
        int t, sc;
        float m;
        if (sscanf(line, "%llx %d %d %f", &k, &t, &sc, &m) == 4 && k == key) {
            bool ok = false;
            for (int c : kTiles) ok = ok || c == t;
            if (ok && sc >= 1 && sc <= 1024) {
                *tile = t;
                *scale = sc;
                *ms = m;
                found = true;       // the last matching line wins
            }
        }
    }
    fclose(fp);
    return found;
}

void cache_store(const char *path, unsigned long long key, int tile, int scale, float ms) {
    FILE *fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "%016llx %d %d %.6f\n", key, tile, scale, ms);
    fclose(fp);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t n) { return hipMalloc(&p, n < 256 ? 256 : n) == hipSuccess; }
};

// Mean ms of one forward + backward for one candidate; < 0 on failure.
dsm_status time_candidate(const dsm_batch_desc *d, int tile, int scale, const float *verts, const float *lparams,
                          const float *albedo, const float *gimg, int reps, hipStream_t s, float *ms) {
    dsm_plan *plan = nullptr;
    dsm_status st = dsm_plan_create(d, tile, scale, &plan);
    if (st != DSM_OK) return st;
    dsm_plan_info info;
    dsm_plan_info_get(plan, &info);
    DevBuf saved, scratch, images, gv, gl, ga;
    const size_t L = (size_t)d->num_lights;
    if (!saved.alloc((size_t)info.saved_bytes) || !scratch.alloc((size_t)info.scratch_bytes) ||
        !images.alloc(4 * (size_t)info.image_floats) || !gv.alloc(12 * (size_t)info.total_vertices) ||
        !gl.alloc(12 * L) || !ga.alloc(4 * (size_t)d->channels * (size_t)info.total_faces)) {
        dsm_plan_destroy(plan);
        return DSM_ERR_OUT_OF_MEMORY;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = DSM_ERR_HIP;
    auto step = [&]() {
        dsm_status r = dsm_forward(plan, verts, lparams, albedo, saved.p, (size_t)info.saved_bytes, scratch.p,
                                   (size_t)info.scratch_bytes, (float *)images.p, s);
        if (r == DSM_OK)
            r = dsm_backward(plan, verts, lparams, albedo, saved.p, (size_t)info.saved_bytes, scratch.p,
                             (size_t)info.scratch_bytes, gimg, (float *)gv.p, (float *)gl.p, (float *)ga.p, s);
        return r;
    };
    if (st == DSM_OK) st = step();                                   // warm-up
    if (st == DSM_OK && hipEventRecord(e0, s) != hipSuccess) st = DSM_ERR_HIP;
    for (int i = 0; i < reps && st == DSM_OK; ++i) st = step();
    if (st == DSM_OK && hipEventRecord(e1, s) != hipSuccess) st = DSM_ERR_HIP;
    if (st == DSM_OK && hipStreamSynchronize(s) != hipSuccess) st = DSM_ERR_HIP;
    float t = 0.f;
    if (st == DSM_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = DSM_ERR_HIP;
    if (st == DSM_OK) *ms = t / (float)reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);           // nothing of this candidate may be in flight when buffers are freed
    dsm_plan_destroy(plan);
    return st;
}

}  // namespace

extern "C" dsm_status dsm_autotune(const dsm_batch_desc *desc, const float *verts_dev, const float *light_params_dev,
                                   const float *albedo_dev, const float *grad_images_dev, int32_t reps,
                                   const char *cache_path, dsm_stream stream, int32_t *tile_size_out,
                                   int32_t *bin_capacity_scale_out, float *ms_out) {
    if (!desc || !tile_size_out || !bin_capacity_scale_out || reps < 1 || reps > DSM_MAX_TIMING_REPS)
        return DSM_ERR_INVALID_ARG;
    if (!desc->vert_offsets || !desc->face_offsets || desc->num_scenes < 1 || desc->num_lights < 0 ||
        desc->num_cameras < 0 || desc->num_renders < 0 || (desc->num_lights > 0 && !desc->lights) ||
        (desc->num_cameras > 0 && !desc->cameras) || (desc->num_renders > 0 && !desc->renders))
        return DSM_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return DSM_ERR_NO_DEVICE;
    const unsigned long long key = shape_key(desc);
    int tile = 0, scale = 0;
    float best = 0.f;
    if (cache_path && cache_lookup(cache_path, key, &tile, &scale, &best)) {
        *tile_size_out = tile;
        *bin_capacity_scale_out = scale;
        if (ms_out) *ms_out = best;
        return DSM_OK;
    }
    const hipStream_t s = (hipStream_t)stream;
    dsm_status last = DSM_ERR_INVALID_ARG;
    bool any = false;
    for (int t : kTiles)
        for (int sc : kScales) {
            float ms = 0.f;
            const dsm_status st = time_candidate(desc, t, sc, verts_dev, light_params_dev, albedo_dev,
                                                 grad_images_dev, reps, s, &ms);
            if (st != DSM_OK) {
                last = st;
                if (st == DSM_ERR_INVALID_ARG || st == DSM_ERR_HIP) return st;
                continue;                      // e.g. a candidate too large for memory
            }
            if (!any || ms < best) {
                best = ms;
                tile = t;
                scale = sc;
                any = true;
            }
        }
    if (!any) return last;
    if (cache_path) cache_store(cache_path, key, tile, scale, best);
    *tile_size_out = tile;
    *bin_capacity_scale_out = scale;
    if (ms_out) *ms_out = best;
    return DSM_OK;
}
