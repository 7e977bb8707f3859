// Internal layout shared by the HIP translation units of the library.
// Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsm.h"

namespace dsm {

constexpr int kSub = 256;              // 8 sub-pixel bits of the fixed-point grid
constexpr float kGuard = 32768.0f;     // |screen coordinate| limit in pixels
constexpr uint64_t kBgKey = ~0ull;     // background key (no triangle)
constexpr int kMaxTaps = 32;

enum ViewKind { kDirectional = 0, kPoint = 1, kSpot = 2, kCamera = 3, kCubeFace = 4 };

// One view: a light camera (views [0, L)) or a viewer camera (views [L, L+Cm)).
// Light views get M / pos / dir rewritten on the device by every forward.
struct ViewConst {
    float M[16];        // row-major view-projection, clip = M [x, 1]
    float pos[3];       // point/spot: position; directional: eye
    float dir[3];       // directional: unit travel direction; spot: cone axis
    float zfar;         // distance normalization
    float cos_half;     // spot cone
    float intensity;
    float min_var;
    int kind;
    int scene;
    int W, H;
    int vert_off, nverts;
    int face_off, nfaces;
    int clip_off;       // first vertex of this view in the clip / gclip arrays
    int setup_off;      // first triangle of this view in the per-(view, triangle) arrays
    long long pix_off;  // first sample of this view in the key array
    int tile_off;       // first tile of this view in the global tile list
    int tiles_x, tiles_y;
    int antialias;
    long long map_off;  // light views: first texel of the 2-channel maps (plane stride S*S)
    int part_off;       // light views: first per-tile slot of the backward light-frame partials
    int part_gm_off;    // light views: first per-vertex-block slot of the dL/dM partials
    int cube_face;      // cube-face lights: face 0..5 (+x, -x, +y, -y, +z, -z)
    float warp_c;       // light views: exponential maps store exp(c z), exp(2 c z); 0 = plain z, z^2
    float bleed;        // light views: light-bleeding reduction amount
    long long fmap_off; // light views: first texel of the filtered maps (and their gradient), side W + 2 fpad
    long long pad_off;  // cube faces: first texel of the padded unfiltered maps in the smoothed-map buffers
    int fpad;           // cube faces: texels of padding sampled from the neighbouring faces; else 0
    int cube_nb[4];     // cube faces, per map edge (left, right, top, bottom): neighbour face
                        // | its edge << 3 | (indices along the edge reversed) << 5
    int ring_off;       // cube faces: first CubeTap of this face's padding (4 P S entries)
    float zc;           // light views: reference depth; maps hold moments of z - zc (see light_depth)
};

// One padded texel of a cube face beyond one of its edges: the bilinear
// sample of the neighbouring face g along the direction the padded texel
// centre looks along.  Entries of a face run over edge e (left, right, top,
// bottom), depth k = 1..P beyond it, and position t = 0..S-1 along it.
struct CubeTap {
    int g;                        // neighbouring face 0..5
    int o[4];                     // texel indices j * S + i of the taps in g's map
    float w[4];                   // bilinear weights (clamp-to-edge taps)
};

// Receiver depth as the lookup compares it, and the variance floor:
// exponential maps compare exp(c z) and floor sigma^2 at min_var (c exp(c z))^2
// (the floor follows the warp's slope); plain maps use z and min_var.
__device__ __forceinline__ void warp_receiver(const ViewConst &l, float zz, float &zw, float &floor_v) {
    if (l.warp_c > 0.f) {
        zw = expf(l.warp_c * zz);
        const float s = l.warp_c * zw;
        floor_v = l.min_var * (s * s);
    } else {
        zw = zz;
        floor_v = l.min_var;
    }
}

// Light-bleeding reduction: v -> clamp((v - a) / (1 - a), 0, 1) for a > 0.
__device__ __forceinline__ float bleed_reduce(const ViewConst &l, float v) {
    return l.bleed > 0.f ? fminf(fmaxf((v - l.bleed) / (1.f - l.bleed), 0.f), 1.f) : v;
}

// Cube face owning the direction d from an omnidirectional light: the axis of
// the largest |d_a| (the first one on ties) and its sign, face 2a (+) or
// 2a + 1 (-).
__device__ __forceinline__ int cube_face_of(float dx, float dy, float dz) {
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int a = 0;
    float m = ax, s = dx;
    if (ay > m) { a = 1; m = ay; s = dy; }
    if (az > m) { a = 2; s = dz; }
    return 2 * a + (s < 0.f ? 1 : 0);
}

struct RenderConst {
    int camera_view;    // view index of the camera
    int light_begin;    // range into the device list of light view indices
    int light_count;
    int W, H;
    int part_off;       // first float of this render's per-(light, tile) backward partials
    long long img_off;  // first float of the [H,W,C] image
    long long pix_off;  // camera view's first sample (keys)
};

// Per (view, triangle) fixed-point setup, written by the setup kernel.
struct TriSetup {
    long long A;                 // doubled area, > 0 when valid
    int X[3], Y[3];              // oriented fixed-point screen coordinates
    float z[3];                  // oriented z01
    unsigned short bx0, by0, bx1, by1;  // inclusive pixel bbox, clipped to the view
    signed char facing;          // +1 / -1 orientation before re-orienting, 0 if not rasterized
    unsigned char swapped;       // 2nd and 3rd vertex exchanged
    unsigned char sil;           // unused (the silhouette mask lives in its own byte array)
    unsigned char pad1;
    int pad2[2];
};
static_assert(sizeof(TriSetup) == 64, "TriSetup must stay 64 bytes");

// Workgroups per light in the first pass of the light-gradient reduction.
constexpr int kGlightBlocks = 16;

struct BlurJob {
    int S;
    int k;
    long long in_off;            // first float of the 2-channel input map
    long long out_off;
    int tile_off;                // first tile of this job
    int tiles_x;
    float w[kMaxTaps];
};

// Counters written by the device, read by dsm_get_stats.
struct DevCounters {
    unsigned long long culled;
    unsigned long long pairs;
    unsigned long long overflow;
    unsigned long long bad_indices;
    unsigned int overflow_list_len;
    unsigned int big_bin_len;        // triangles binned a workgroup each
    unsigned int pad[6];
};

// ----------------------------------------------------------------------------- helpers

// Sum over the 64 lanes of a wave, returned to every lane.  DPP moves inside
// each 16-lane row (quad swaps, then rotations by 4 and 8), then the four row
// sums are read out with v_readlane.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x124>(v);   // row_ror:4
    v += dpp_mov<0x128>(v);   // row_ror:8
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Wave-wide sums of N <= 32 values at once by recursive halving: at each
// butterfly step every lane keeps half of its remaining values and receives
// its partner's copy of that half, so the 64 lanes end up each holding one
// total.  Lane l returns the total of value (l >> 1) (0 for (l >> 1) >= N).
// About 4 instructions per value instead of 11 for N separate wave_sum calls.
// All 64 lanes must be active.
template <int N>
__device__ __forceinline__ float wave_sum_multi(const float (&v)[N]) {
    static_assert(N >= 1 && N <= 32, "wave_sum_multi handles up to 32 values");
    const int lane = (int)(threadIdx.x & 63);
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    float a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {            // partner lane ^ 32
        const float lo = j < N ? v[j] : 0.f, hi = j + 16 < N ? v[j + 16] : 0.f;
        a[j] = (b5 ? hi : lo) + __shfl_xor(b5 ? lo : hi, 32, 64);
    }
    float b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)               // partner lane ^ 16
        b[j] = (b4 ? a[j + 8] : a[j]) + __shfl_xor(b4 ? a[j] : a[j + 8], 16, 64);
    float c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)               // partner lane ^ 8: row_ror:8 within 16-lane rows
        c[j] = (b3 ? b[j + 4] : b[j]) + dpp_mov<0x128>(b3 ? b[j] : b[j + 4]);
    float d[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {             // partner lane ^ 4: from lane + 4 (row_ror:12) or lane - 4 (row_ror:4)
        const float send = b2 ? c[j] : c[j + 2];
        const float up = dpp_mov<0x12C>(send), down = dpp_mov<0x124>(send);
        d[j] = (b2 ? c[j + 2] : c[j]) + (b2 ? down : up);
    }
    float e = (b1 ? d[1] : d[0]) + dpp_mov<0x4E>(b1 ? d[0] : d[1]);   // partner lane ^ 2
    e += dpp_mov<0xB1>(e);                                              // partner lane ^ 1: plain sum
    return e;
}

template <int CTRL>
__device__ __forceinline__ int dpp_movi(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
// Minimum over the 64 lanes of a wave, returned to every lane.  All lanes active.
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_movi<0xB1>(v));
    v = min(v, dpp_movi<0x4E>(v));
    v = min(v, dpp_movi<0x124>(v));
    v = min(v, dpp_movi<0x128>(v));
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return min(min(r0, r1), min(r2, r3));
}
// Maximum over the 64 lanes of a wave, returned to every lane.  All lanes active.
__device__ __forceinline__ int wave_max(int v) {
    v = max(v, dpp_movi<0xB1>(v));
    v = max(v, dpp_movi<0x4E>(v));
    v = max(v, dpp_movi<0x124>(v));
    v = max(v, dpp_movi<0x128>(v));
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each
// XCD has its own L2.  These renumber a grid so that each XCD takes a
// contiguous range of work items: neighbouring tiles and rows, which share
// cache lines and halos, then share an L2.  Both are bijections, so any
// dispatch order stays correct.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int kXcd = 8;
    const int xcd = b % kXcd, idx = b / kXcd;
    const int per = n / kXcd, rem = n % kXcd;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

struct Blk {
    int x, y;
};
__device__ __forceinline__ Blk xcd_block2() {
    const int gx = (int)gridDim.x;
    const int lin = xcd_remap((int)blockIdx.x + (int)blockIdx.y * gx, gx * (int)gridDim.y);
    return Blk{lin % gx, lin / gx};
}

// Clip coordinates M [x, 1] in the fixed operation order every kernel uses
// (no contraction), so that recomputing them anywhere is bit-identical.
__device__ __forceinline__ float4 clip_of(const float *M, float x, float y, float z) {
    float4 c;
    c.x = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    c.y = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    c.z = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    c.w = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
    return c;
}

// World positions of a triangle's three corners, packed as three float4
// (x0 y0 z0 x1 | y1 z1 x2 y2 | z2 - - -), one record per face of the batch.
struct TriVerts {
    float4 a, b, c;     // x0 y0 z0 x1 | y1 z1 x2 y2 | z2 albedo[0..2]
};

__device__ __forceinline__ void atomic_add_f32(float *p, float v) {
    if (v != 0.0f) atomicAdd(p, v);
}

}  // namespace dsm

// Host-side launchers implemented per translation unit.
namespace dsm {
hipError_t launch_blur(const BlurJob *jobs_dev, int njobs, int total_tiles, const float *in, float *out,
                       bool adjoint, int rmax, hipStream_t s);
int blur_tile_height(int rmax);
hipError_t launch_blur_uniform(const BlurJob &job, int n_maps, const float *in, float *out, bool adjoint,
                               hipStream_t s);
int blur_tiles(int S, int rmax);
int blur_tiles_x(int S);
bool valid_filter(int S, int filter, int k);

struct CamStatic;
// Jacobian of a light frame (M[16], pos[3], dir[3]) w.r.t. its three parameter components, [22][3].
constexpr int kJac = 66;
// Also clears bytes1 at z1 and bytes2 at z2 (multiples of 4) in the same launch.
hipError_t launch_light_frames(ViewConst *views, const CamStatic *cams, const float *params, int L, float *jac,
                               float *zc_out, void *z1, size_t bytes1, void *z2, size_t bytes2, hipStream_t s);
hipError_t launch_transform(const ViewConst *views, int nviews, int max_verts, const float *verts, float4 *clip,
                            hipStream_t s);
hipError_t launch_silhouettes(const ViewConst *views, int nviews, int max_faces, const int *adj,
                              const signed char *facing8, unsigned char *silm, hipStream_t s);
hipError_t launch_setup(const ViewConst *views, int nviews, int max_faces, const int *faces, const float4 *clip,
                        TriSetup *setup, signed char *facing8, unsigned *pair_count, int tile, DevCounters *counters,
                        hipStream_t s);
int scan_scratch_words(int n);
hipError_t launch_scan(const unsigned *in, unsigned *out, unsigned *scratch, int n, hipStream_t s);
hipError_t launch_binning(const ViewConst *views, const TriSetup *setup, const unsigned *pair_off, int ntri,
                          unsigned capacity, int tile, unsigned *tile_count, unsigned *tile_start,
                          unsigned *pair_slot, unsigned *scan_scratch, int ntiles, unsigned *bins,
                          unsigned *bin_pair, unsigned *overflow_list, unsigned *big_list, DevCounters *counters,
                          hipStream_t s);
hipError_t launch_raster(const ViewConst *views, const int *tile_view, int ntiles, int tile, const TriSetup *setup,
                         const unsigned *tile_start, const unsigned *bins, const unsigned *overflow_list,
                         const DevCounters *counters_ro, DevCounters *counters, unsigned long long *keys,
                         hipStream_t s);
hipError_t launch_cube_pad(const ViewConst *views, int L, int max_padded, const CubeTap *taps, float *F1,
                           hipStream_t s);
hipError_t launch_cube_pad_transpose(const ViewConst *views, int L, int max_texels, int max_ring,
                                     const CubeTap *taps, float *gF1, hipStream_t s);
hipError_t launch_resolve(const ViewConst *views, int L, int max_texels, const TriVerts *tv,
                          const unsigned long long *keys, float *F0, hipStream_t s);
hipError_t launch_aa_forward(bool light, const ViewConst *views, const RenderConst *renders, int n, int max_pix,
                             const TriSetup *setup, const int *faces, const unsigned char *silm, const float *verts,
                             const unsigned long long *keys, const float *src, float *dst, int C, uint2 *list,
                             unsigned *count, unsigned char *aa_flag, hipStream_t s);
hipError_t launch_lookup(const ViewConst *views, const RenderConst *renders, int R, int max_pix,
                         const int *render_lights, const TriVerts *tv, const float *albedo,
                         const unsigned long long *keys, const float *maps, float *img0, int C, hipStream_t s);
hipError_t launch_tri_verts(const int *scene_vert_off, const int *scene_face_off, int B, int max_faces,
                            const int *faces, const float *verts, const float *albedo, int C, TriVerts *tv,
                            hipStream_t s);
// backward
hipError_t launch_aa_camera_backward(const ViewConst *views, const RenderConst *renders, int R, int max_pix,
                                     const TriSetup *setup, const int *faces, const unsigned char *silm, const float *verts,
                                     const unsigned long long *keys, const unsigned char *aa_flag, const float *img0,
                                     const float *gimg, float *gimg0, float4 *gclip, int C, hipStream_t s);
hipError_t launch_lookup_backward(int tile, const ViewConst *views, int L, int Cm, int max_tiles, int max_lights,
                                  const RenderConst *renders, const int *cam_renders_off, const int *cam_renders,
                                  const int *render_lights, const int *faces, const float *verts, const float *albedo,
                                  const TriVerts *tv, const unsigned long long *keys, const float *maps,
                                  const float *gimg0, float *gmaps, const TriSetup *setup, const unsigned *tile_start,
                                  const unsigned *bins, const unsigned *bin_pair, unsigned char *pair_flag,
                                  float *pair_sums, float *gtri, float *part_render, int C, const float *jac,
                                  const unsigned *pair_off, unsigned capacity, hipStream_t s);
hipError_t launch_light_backward(int tile, const ViewConst *views, int L, int max_tiles, const TriSetup *setup,
                                 const int *faces, const unsigned char *silm, const float *verts, const TriVerts *tv,
                                 const unsigned long long *keys, const unsigned char *aa_flag, const float *F0, const float *gF1, float4 *gclip,
                                 const unsigned *tile_start, const unsigned *bins, const unsigned *bin_pair,
                                 unsigned char *pair_flag, float *pair_sums, float *gtri, float *part_light,
                                 const float *jac, const unsigned *pair_off, unsigned capacity, hipStream_t s);
hipError_t launch_vertex_gradients(const ViewConst *views, int L, int B, int max_verts, int max_faces, int ntri,
                                   unsigned capacity, const int *scene_vert_off, const int *scene_face_off,
                                   const int *scene_views_off, const int *scene_views, const int *vc_off,
                                   const int *vc_list, const unsigned *pair_off, const unsigned char *pair_flag,
                                   const float *pair_sums, float *gtri, const float *zero_rec,
                                   unsigned *big_list, unsigned *big_count, const float *verts, const float4 *gclip,
                                   float *gverts, float *part_gm, float *galbedo, int C, const float *jac, hipStream_t s);
hipError_t launch_overflow_rows_zero(const unsigned *list, const DevCounters *counters, float *gtri, hipStream_t s);
hipError_t launch_glight_reduce(const ViewConst *views, int L, const RenderConst *renders,
                                const int *light_renders_off, const int *light_renders, const float *part_gm,
                                const float *part_light, const float *part_render, float *gl_part, float *gparams,
                                hipStream_t s);
hipError_t launch_pose(const int *scene_vert_off, const int *pose_counts, const float *pose_centers, int B,
                       int max_verts, const float *local, const float *poses, float *world, hipStream_t s);
hipError_t launch_pose_backward(const int *scene_vert_off, const int *pose_counts, int B, int max_verts,
                                const float *local, const float *poses, const float *gworld, float *gposes,
                                hipStream_t s);
void filter_taps_host(int filter, int k, float sigma, float *w);
}  // namespace dsm
