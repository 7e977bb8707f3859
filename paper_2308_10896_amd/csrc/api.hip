// C ABI: plans, forward / backward passes, pose, graphs, stage getters.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "aa.h"
#include "dsm_internal.h"
#include "frames.h"
#include "plan.h"

using namespace dsm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Frame of cube face f as integer vectors: viewing axis a = (-1)^s e_k for
// f = 2k + s, up +z for the y faces and +y otherwise, right = a x up and the
// camera's up u = right x a (the light camera's look-at frame).
void cube_frame(int f, int a[3], int r[3], int u[3]) {
    const int k = f >> 1;
    int up[3] = {0, 0, 0};
    up[k == 1 ? 2 : 1] = 1;
    for (int i = 0; i < 3; ++i) a[i] = i == k ? ((f & 1) ? -1 : 1) : 0;
    r[0] = a[1] * up[2] - a[2] * up[1];
    r[1] = a[2] * up[0] - a[0] * up[2];
    r[2] = a[0] * up[1] - a[1] * up[0];
    u[0] = r[1] * a[2] - r[2] * a[1];
    u[1] = r[2] * a[0] - r[0] * a[2];
    u[2] = r[0] * a[1] - r[1] * a[0];
}

int dot3i(const int x[3], const int y[3]) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; }

// Bilinear taps for the padding of cube face f (side S, P texels): for edge
// e, depth k = 1..P beyond it and position t along it, the padded texel
// centre's direction a + u r + v up (u, v its NDC continued past +-1) is
// projected into the neighbouring face g and sampled there with
// clamp-to-edge, in double precision.
void cube_ring_taps(int f, int S, int P, const int nb[4], std::vector<CubeTap> &out) {
    int a[3], r[3], u[3];
    cube_frame(f, a, r, u);
    for (int e = 0; e < 4; ++e)
        for (int k = 1; k <= P; ++k)
            for (int t = 0; t < S; ++t) {
                const int i = e == 0 ? -k : e == 1 ? S - 1 + k : t;
                const int j = e == 2 ? -k : e == 3 ? S - 1 + k : t;
                const double un = (double)(2 * i + 1) / S - 1.0, vn = 1.0 - (double)(2 * j + 1) / S;
                double d[3];
                for (int c = 0; c < 3; ++c) d[c] = a[c] + un * r[c] + vn * u[c];
                CubeTap tp;
                tp.g = nb[e] & 7;
                int ag[3], rg[3], ug[3];
                cube_frame(tp.g, ag, rg, ug);
                const double da = d[0] * ag[0] + d[1] * ag[1] + d[2] * ag[2];
                const double gu = (d[0] * rg[0] + d[1] * rg[1] + d[2] * rg[2]) / da;
                const double gv = (d[0] * ug[0] + d[1] * ug[1] + d[2] * ug[2]) / da;
                const double sx = (gu + 1.0) * S / 2.0 - 0.5, sy = (1.0 - gv) * S / 2.0 - 0.5;
                const double x0 = floor(sx), y0 = floor(sy), fx = sx - x0, fy = sy - y0;
                const int xs[2] = {std::min(std::max((int)x0, 0), S - 1), std::min(std::max((int)x0 + 1, 0), S - 1)};
                const int ys[2] = {std::min(std::max((int)y0, 0), S - 1), std::min(std::max((int)y0 + 1, 0), S - 1)};
                tp.o[0] = ys[0] * S + xs[0];
                tp.o[1] = ys[0] * S + xs[1];
                tp.o[2] = ys[1] * S + xs[0];
                tp.o[3] = ys[1] * S + xs[1];
                tp.w[0] = (float)((1.0 - fx) * (1.0 - fy));
                tp.w[1] = (float)(fx * (1.0 - fy));
                tp.w[2] = (float)((1.0 - fx) * fy);
                tp.w[3] = (float)(fx * fy);
                out.push_back(tp);
            }
}

// The face across edge e (0 left, 1 right, 2 top, 3 bottom of the map) of
// cube face f, the edge of that face's map on the same cube edge, and whether
// texel indices along the edge run in opposite directions: packed as
// g | e' << 3 | reversed << 5.  Two points of the edge, at along-coordinates
// -1/2 and +1/2 (scaled by 2 to stay integer), are expressed in g's frame.
int cube_edge_neighbour(int f, int e) {
    int a[3], r[3], u[3];
    cube_frame(f, a, r, u);
    int out[3], along[3];
    for (int i = 0; i < 3; ++i) {
        out[i] = e == 0 ? -r[i] : e == 1 ? r[i] : e == 2 ? u[i] : -u[i];
        along[i] = e < 2 ? u[i] : r[i];
    }
    int g = 0;
    for (int i = 0; i < 3; ++i)
        if (out[i] != 0) g = 2 * i + (out[i] < 0 ? 1 : 0);
    int ag[3], rg[3], ug[3];
    cube_frame(g, ag, rg, ug);
    int pm[3], pp[3];                     // 2 x the two edge points
    for (int i = 0; i < 3; ++i) {
        pm[i] = 2 * a[i] + 2 * out[i] - along[i];
        pp[i] = 2 * a[i] + 2 * out[i] + along[i];
    }
    // in g's map (NDC x2): the edge coordinate is +-2 at both points
    int e2, dg;
    if (dot3i(pm, rg) == dot3i(pp, rg)) {
        e2 = dot3i(pm, rg) < 0 ? 0 : 1;
        dg = -(dot3i(pp, ug) - dot3i(pm, ug));        // index runs against v
    } else {
        e2 = dot3i(pm, ug) > 0 ? 2 : 3;
        dg = dot3i(pp, rg) - dot3i(pm, rg);           // index runs with u
    }
    const int df = e < 2 ? -1 : 1;                    // f: along is v for left/right, u for top/bottom
    const bool reversed = (df > 0) != (dg > 0);
    return g | (e2 << 3) | ((reversed ? 1 : 0) << 5);
}

__global__ void zero_kernel(unsigned *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// A light's maps as the getter hands them out: two planes of S x S texels
// holding (f, f^2) of z = d / zfar (or exp(c z), exp(2 c z)).  The library
// stores moments of z - zc (zc: the light's reference depth, kept in saved),
// which an affine map turns back: f = f' + zc, f^2 = f^2' + zc (2 f' + zc),
// or for exponential maps f = f' e^{c zc}, f^2 = f^2' e^{2 c zc}.  Filtered
// maps are stored (m1, m2) interleaved per texel with side S + 2P (the face
// at offset P); the others are planar with side S.
__global__ void light_maps_out_kernel(const float *src, int S, int sp, int P, bool interleaved, const float *zc_p,
                                      float warp_c, float *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * S) return;
    const float zc = *zc_p;
    float a, b;
    if (interleaved) {
        const long long q = 2 * ((long long)(t / S + P) * sp + (t % S + P));
        a = src[q];
        b = src[q + 1];
    } else {
        a = src[t];
        b = src[(long long)S * S + t];
    }
    if (warp_c > 0.f) {
        const float e = expf(warp_c * zc);
        a *= e;
        b *= e * e;
    } else {
        b = b + zc * (2.f * a + zc);
        a = a + zc;
    }
    out[t] = a;
    out[(long long)S * S + t] = b;
}

hipError_t zero_async(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned *)p, n);
    return hipGetLastError();
}

template <class T>
dsm_status upload(T **dst, const T *src, size_t n) {
    *dst = nullptr;
    if (n == 0) return DSM_OK;
    if (hipMalloc((void **)dst, n * sizeof(T)) != hipSuccess) return DSM_ERR_OUT_OF_MEMORY;
    if (hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return DSM_ERR_HIP;
    return DSM_OK;
}

bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Edge adjacency of one scene: for face f and original edge k (opposite
// vertex k) the face across the undirected edge; -1 boundary, -2 shared by
// more than two faces.
void build_adjacency(const int *faces, int F, int V, int *adj) {
    std::vector<std::pair<long long, int>> e;
    e.reserve(3 * (size_t)F);
    for (int f = 0; f < F; ++f)
        for (int k = 0; k < 3; ++k) {
            const long long a = faces[3 * f + (k + 1) % 3], b = faces[3 * f + (k + 2) % 3];
            e.push_back({std::min(a, b) * (long long)V + std::max(a, b), 3 * f + k});
        }
    std::sort(e.begin(), e.end());
    size_t i = 0;
    while (i < e.size()) {
        size_t j = i;
        while (j < e.size() && e[j].first == e[i].first) ++j;
        const size_t n = j - i;
        for (size_t q = i; q < j; ++q) {
            int v = -1;
            if (n == 2) v = e[q == i ? i + 1 : i].second / 3;
            else if (n > 2) v = -2;
            adj[e[q].second] = v;
        }
        i = j;
    }
}

bool layout_ok(long long x) { return x >= 0 && x < (1LL << 31); }

}  // namespace

extern "C" dsm_status dsm_plan_create(const dsm_batch_desc *d, int32_t tile_size, int32_t bin_capacity_scale,
                                      dsm_plan **out_plan) {
    if (!d || !out_plan) return DSM_ERR_INVALID_ARG;
    *out_plan = nullptr;
    if (tile_size == 0) tile_size = 8;
    if (tile_size != 8 && tile_size != 16 && tile_size != 32) return DSM_ERR_INVALID_ARG;
    if (bin_capacity_scale == 0) bin_capacity_scale = 32;
    if (bin_capacity_scale < 0 || bin_capacity_scale > 1024) return DSM_ERR_INVALID_ARG;
    const int B = d->num_scenes, L = d->num_lights, Cm = d->num_cameras, R = d->num_renders;
    if (B < 1 || L < 0 || Cm < 0 || R < 0 || !d->vert_offsets || !d->face_offsets) return DSM_ERR_INVALID_ARG;
    if ((L > 0 && !d->lights) || (Cm > 0 && !d->cameras) || (R > 0 && (!d->renders || !d->render_light_list)))
        return DSM_ERR_INVALID_ARG;
    if (d->channels != 1 && d->channels != 3) return DSM_ERR_INVALID_ARG;
    if (d->vert_offsets[0] != 0 || d->face_offsets[0] != 0) return DSM_ERR_INVALID_ARG;
    for (int b = 0; b < B; ++b)
        if (d->vert_offsets[b + 1] < d->vert_offsets[b] || d->face_offsets[b + 1] < d->face_offsets[b])
            return DSM_ERR_INVALID_ARG;
    const long long Vt = d->vert_offsets[B], Ft = d->face_offsets[B];
    if (!layout_ok(3 * Vt) || !layout_ok(3 * Ft) || (Ft > 0 && !d->faces)) return DSM_ERR_INVALID_ARG;
    for (int b = 0; b < B; ++b) {
        const int nv = d->vert_offsets[b + 1] - d->vert_offsets[b];
        for (long long f = d->face_offsets[b]; f < d->face_offsets[b + 1]; ++f)
            for (int k = 0; k < 3; ++k)
                if (d->faces[3 * f + k] < 0 || d->faces[3 * f + k] >= nv) return DSM_ERR_INVALID_ARG;
        if (d->pose_counts && (d->pose_counts[b] < 0 || d->pose_counts[b] > nv)) return DSM_ERR_INVALID_ARG;
    }
    for (int l = 0; l < L; ++l) {
        const dsm_light_desc &x = d->lights[l];
        if (x.type < 0 || x.type > DSM_LIGHT_CUBE_FACE || x.scene < 0 || x.scene >= B) return DSM_ERR_INVALID_ARG;
        if (x.type == DSM_LIGHT_CUBE_FACE) {
            // the six faces of one cube light are consecutive lights, faces 0..5
            // in order, with one scene, map size and filter
            if (x.cube_face < 0 || x.cube_face > 5 || l - x.cube_face < 0 || l - x.cube_face + 5 >= L)
                return DSM_ERR_INVALID_ARG;
            for (int g = 0; g < 6; ++g) {
                const dsm_light_desc &y = d->lights[l - x.cube_face + g];
                if (y.type != DSM_LIGHT_CUBE_FACE || y.cube_face != g || y.scene != x.scene ||
                    y.resolution != x.resolution || y.k != x.k || y.filter != x.filter || y.sigma != x.sigma)
                    return DSM_ERR_INVALID_ARG;
            }
        }
        if (!(x.warp_exponent >= 0.f && x.warp_exponent <= 40.f) ||
            !(x.bleed_reduction >= 0.f && x.bleed_reduction < 1.f))
            return DSM_ERR_INVALID_ARG;
        if (!valid_filter(x.resolution, x.filter, x.k)) return DSM_ERR_INVALID_ARG;
        if (!(x.znear > 0 && x.zfar > x.znear) || !std::isfinite(x.zfar)) return DSM_ERR_INVALID_ARG;
        if (x.type == DSM_LIGHT_DIRECTIONAL && !(x.ortho_half > 0 && x.dir_distance > 0)) return DSM_ERR_INVALID_ARG;
        if ((x.type == DSM_LIGHT_POINT || x.type == DSM_LIGHT_SPOT) && !(x.fov_deg > 0 && x.fov_deg < 180))
            return DSM_ERR_INVALID_ARG;
        if (!finite3(x.target) || !finite3(x.up) || !(x.min_variance >= 0) || !std::isfinite(x.intensity))
            return DSM_ERR_INVALID_ARG;
    }
    for (int c = 0; c < Cm; ++c) {
        const dsm_camera_desc &x = d->cameras[c];
        if (x.width < 1 || x.height < 1 || x.width > DSM_MAX_RESOLUTION || x.height > DSM_MAX_RESOLUTION)
            return DSM_ERR_INVALID_ARG;
        if (x.scene < 0 || x.scene >= B || !(x.fov_deg > 0 && x.fov_deg < 180) || !(x.znear > 0 && x.zfar > x.znear))
            return DSM_ERR_INVALID_ARG;
        if (!finite3(x.eye) || !finite3(x.target) || !finite3(x.up)) return DSM_ERR_INVALID_ARG;
    }
    long long list_len = 0;
    for (int r = 0; r < R; ++r) {
        const dsm_render_desc &x = d->renders[r];
        if (x.camera < 0 || x.camera >= Cm || x.light_begin < 0 || x.light_count < 0 ||
            x.light_count > DSM_MAX_LIGHTS_PER_RENDER)
            return DSM_ERR_INVALID_ARG;
        list_len = std::max<long long>(list_len, (long long)x.light_begin + x.light_count);
        for (int q = 0; q < x.light_count; ++q) {
            const int l = d->render_light_list[x.light_begin + q];
            if (l < 0 || l >= L || d->lights[l].scene != d->cameras[x.camera].scene) return DSM_ERR_INVALID_ARG;
        }
    }

    int ndev = 0, dev = -1;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return DSM_ERR_NO_DEVICE;
    if (hipGetDevice(&dev) != hipSuccess) return DSM_ERR_HIP;
    dsm_plan *p = new (std::nothrow) dsm_plan();
    if (!p) return DSM_ERR_OUT_OF_MEMORY;
    p->device = dev;
    p->B = B; p->L = L; p->Cm = Cm; p->R = R; p->C = d->channels; p->nviews = L + Cm;
    p->camera_antialias = d->camera_antialias != 0;
    p->V_total = Vt; p->F_total = Ft;
    p->tile = tile_size;
    p->bin_scale = bin_capacity_scale;
    p->vert_off.assign(d->vert_offsets, d->vert_offsets + B + 1);
    p->face_off.assign(d->face_offsets, d->face_offsets + B + 1);
    p->pose_counts.assign(B, 0);
    p->pose_centers.assign(3 * (size_t)B, 0.f);
    if (d->pose_counts) p->pose_counts.assign(d->pose_counts, d->pose_counts + B);
    if (d->pose_centers) p->pose_centers.assign(d->pose_centers, d->pose_centers + 3 * (size_t)B);
    for (int b = 0; b < B; ++b) {
        p->max_pose_verts = std::max(p->max_pose_verts, p->pose_counts[b]);
        p->max_scene_verts = std::max(p->max_scene_verts, p->vert_off[b + 1] - p->vert_off[b]);
        p->max_scene_faces = std::max(p->max_scene_faces, p->face_off[b + 1] - p->face_off[b]);
    }

    // views: lights then cameras
    long long clip = 0, tri = 0, pix = 0, maps = 0, tiles = 0, part_light = 0, part_gm = 0, part_render = 0;
    long long fmaps = 0, padmaps = 0;
    auto add_view = [&](ViewConst &v, int scene, int W, int H) {
        v.scene = scene;
        v.W = W;
        v.H = H;
        v.vert_off = p->vert_off[scene];
        v.nverts = p->vert_off[scene + 1] - p->vert_off[scene];
        v.face_off = p->face_off[scene];
        v.nfaces = p->face_off[scene + 1] - p->face_off[scene];
        v.clip_off = (int)clip;
        v.setup_off = (int)tri;
        v.pix_off = pix;
        v.tile_off = (int)tiles;
        v.tiles_x = (W + tile_size - 1) / tile_size;
        v.tiles_y = (H + tile_size - 1) / tile_size;
        clip += v.nverts;
        tri += v.nfaces;
        pix += (long long)W * H;
        tiles += (long long)v.tiles_x * v.tiles_y;
        p->max_verts = std::max(p->max_verts, v.nverts);
        p->max_faces = std::max(p->max_faces, v.nfaces);
    };
    p->views_h.resize(p->nviews);
    p->light_cams_h.resize(L);
    for (int l = 0; l < L; ++l) {
        const dsm_light_desc &x = d->lights[l];
        ViewConst v;
        memset(&v, 0, sizeof(v));
        v.kind = x.type == DSM_LIGHT_DIRECTIONAL ? kDirectional
                 : x.type == DSM_LIGHT_POINT   ? kPoint
                 : x.type == DSM_LIGHT_SPOT    ? kSpot
                                               : kCubeFace;
        v.cube_face = v.kind == kCubeFace ? x.cube_face : 0;
        v.warp_c = x.warp_exponent;
        v.bleed = x.bleed_reduction;
        v.zfar = x.zfar;
        v.cos_half = (float)cos((double)x.fov_deg * (M_PI / 180.0) / 2.0);
        v.intensity = x.intensity;
        v.min_var = x.min_variance;
        v.antialias = x.antialias != 0;
        add_view(v, x.scene, x.resolution, x.resolution);
        v.map_off = maps;
        maps += 2LL * x.resolution * x.resolution;
        // filtered maps of a cube face keep (k - 1) / 2 + 1 texels of its
        // neighbours around it: enough for the filter to reach across the seam
        // and for the bilinear fetch to take one texel beyond the face
        v.fpad = v.kind == kCubeFace ? (x.k - 1) / 2 + 1 : 0;
        v.fmap_off = fmaps;
        {
            const long long sp = x.resolution + 2LL * v.fpad;
            fmaps += 2 * sp * sp;
            if (v.kind == kCubeFace) {
                v.pad_off = padmaps;          // relative; moved past the unpadded maps below
                padmaps += 2 * sp * sp;
                p->has_cube = true;
                p->max_cube_padded = std::max(p->max_cube_padded, (int)(sp * sp));
                p->max_cube_texels = std::max(p->max_cube_texels, x.resolution * x.resolution);
                for (int e = 0; e < 4; ++e) v.cube_nb[e] = cube_edge_neighbour(x.cube_face, e);
                v.ring_off = (int)p->cube_taps_h.size();
                cube_ring_taps(x.cube_face, x.resolution, v.fpad, v.cube_nb, p->cube_taps_h);
                p->max_cube_ring = std::max(p->max_cube_ring, 4 * v.fpad * x.resolution);
            }
        }
        v.part_off = (int)part_light;
        part_light += (long long)v.tiles_x * v.tiles_y;
        v.part_gm_off = (int)part_gm;
        part_gm += (v.nverts + 255) / 256;
        p->max_light_texels = std::max(p->max_light_texels, x.resolution * x.resolution);
        p->max_light_tiles = std::max(p->max_light_tiles, v.tiles_x * v.tiles_y);
        p->views_h[l] = v;
        CamStatic &cs = p->light_cams_h[l];
        memset(&cs, 0, sizeof(cs));
        cs.kind = v.kind;
        for (int i = 0; i < 3; ++i) { cs.target[i] = x.target[i]; cs.up[i] = x.up[i]; }
        cs.focal = 1.0 / tan((double)x.fov_deg * (M_PI / 180.0) / 2.0);
        if (v.kind == kCubeFace) {
            // face f = 2a + s views along (-1)^s e_a; up is +z for the y faces, +y otherwise
            const int a = x.cube_face >> 1;
            for (int i = 0; i < 3; ++i) {
                cs.target[i] = i == a ? ((x.cube_face & 1) ? -1.0 : 1.0) : 0.0;
                cs.up[i] = i == (a == 1 ? 2 : 1) ? 1.0 : 0.0;
            }
            cs.focal = 1.0;
        }
        cs.aspect = 1.0;
        cs.znear = x.znear;
        cs.zfar = x.zfar;
        cs.dir_distance = x.dir_distance;
        cs.ortho_half = x.ortho_half;
    }
    for (int c = 0; c < Cm; ++c) {
        const dsm_camera_desc &x = d->cameras[c];
        ViewConst v;
        memset(&v, 0, sizeof(v));
        v.kind = kCamera;
        v.zfar = x.zfar;
        v.antialias = p->camera_antialias;
        add_view(v, x.scene, x.width, x.height);
        CamStatic cs;
        memset(&cs, 0, sizeof(cs));
        cs.kind = kCamera;
        for (int i = 0; i < 3; ++i) cs.up[i] = x.up[i];
        cs.focal = 1.0 / tan((double)x.fov_deg * (M_PI / 180.0) / 2.0);
        cs.aspect = (double)x.width / (double)x.height;
        cs.znear = x.znear;
        cs.zfar = x.zfar;
        const Vec3<double> eye{x.eye[0], x.eye[1], x.eye[2]}, tg{x.target[0], x.target[1], x.target[2]};
        double M[16];
        view_projection<double>(cs, eye, tg, M);
        for (int i = 0; i < 16; ++i) v.M[i] = (float)M[i];
        p->max_cam_pix = std::max(p->max_cam_pix, x.width * x.height);
        p->max_cam_tiles = std::max(p->max_cam_tiles, v.tiles_x * v.tiles_y);
        p->views_h[L + c] = v;
    }
    long long img = 0;
    p->renders_h.resize(R);
    for (int r = 0; r < R; ++r) {
        const dsm_render_desc &x = d->renders[r];
        RenderConst rc;
        memset(&rc, 0, sizeof(rc));
        rc.camera_view = L + x.camera;
        rc.light_begin = x.light_begin;
        rc.light_count = x.light_count;
        p->max_lights_per_render = std::max(p->max_lights_per_render, x.light_count);
        rc.W = d->cameras[x.camera].width;
        rc.H = d->cameras[x.camera].height;
        rc.img_off = img;
        rc.pix_off = p->views_h[L + x.camera].pix_off;
        rc.part_off = (int)part_render;
        part_render += 3LL * x.light_count * p->views_h[L + x.camera].tiles_x * p->views_h[L + x.camera].tiles_y;
        img += (long long)rc.W * rc.H * p->C;
        p->renders_h[r] = rc;
    }
    p->render_lights_h.assign(d->render_light_list, d->render_light_list + list_len);
    p->nclip = (int)clip;
    p->ntri = (int)tri;
    p->ntiles = (int)tiles;
    p->key_count = pix;
    p->map_floats = maps;
    for (int l = 0; l < L; ++l)
        if (p->views_h[l].fpad) p->views_h[l].pad_off += maps;
    p->image_floats = img;
    if (!layout_ok(clip) || !layout_ok(tri) || !layout_ok(tiles) || !layout_ok(pix) || !layout_ok(maps) ||
        !layout_ok(img) || !layout_ok((long long)bin_capacity_scale * (tri + tiles) / 4)) {
        delete p;
        return DSM_ERR_INVALID_ARG;
    }
    // pair rows are addressed with 32-bit offsets (pair * 21 + value)
    p->capacity = (unsigned)std::min<long long>((long long)bin_capacity_scale * (tri + tiles) / 4,
                                                (long long)(0xFFFFFFFFu / 21u));

    // blur jobs over all light maps, grouped by filter radius (one launch per radius)
    {
        std::vector<int> order(L);
        for (int l = 0; l < L; ++l) order[l] = l;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return d->lights[x].k < d->lights[y].k; });
        for (int q = 0; q < L; ++q) {
            const int l = order[q];
            const dsm_light_desc &x = d->lights[l];
            const int R = (x.k - 1) / 2;
            if (p->blur_groups.empty() || p->blur_groups.back().R != R)
                p->blur_groups.push_back(dsm_plan::BlurGroup{R, q, 0, 0});
            dsm_plan::BlurGroup &g = p->blur_groups.back();
            // forward: smoothed maps (cube faces: their padded copies) -> filtered maps
            const ViewConst &v = p->views_h[l];
            const int sp = x.resolution + 2 * v.fpad;
            BlurJob j;
            memset(&j, 0, sizeof(j));
            j.S = sp;
            j.k = x.k;
            j.in_off = v.fpad ? v.pad_off : v.map_off;
            j.out_off = v.fmap_off;
            j.tile_off = g.tiles;
            j.tiles_x = blur_tiles_x(sp);
            filter_taps_host(x.filter, x.k, x.sigma, j.w);
            g.tiles += blur_tiles(sp, R);
            g.n += 1;
            p->blur_jobs_h.push_back(j);
        }
        // transpose: the same jobs reading the filtered side, writing the smoothed side
        for (int q = 0; q < L; ++q) {
            BlurJob j = p->blur_jobs_h[q];
            std::swap(j.in_off, j.out_off);
            p->blur_jobs_h.push_back(j);
        }
    }

    // saved layout
    size_t o = 0;
    p->sv_counters = o; o = align_up(o + sizeof(DevCounters));
    p->sv_zero_end = o;
    p->sv_keys = o; o = align_up(o + 8 * (size_t)pix);
    p->sv_clip = o; o = align_up(o + 16 * (size_t)clip);
    p->sv_setup = o; o = align_up(o + sizeof(TriSetup) * (size_t)tri);
    p->sv_sil = o; o = align_up(o + (size_t)tri);
    p->sv_tv = o; o = align_up(o + sizeof(TriVerts) * (size_t)std::max<long long>(Ft, 1));
    p->sv_F0 = o; o = align_up(o + 4 * (size_t)maps);
    p->sv_M = o; o = align_up(o + 4 * (size_t)fmaps);
    p->sv_img0 = o; o = align_up(o + 4 * (size_t)img);
    p->sv_pair_off = o; o = align_up(o + 4 * ((size_t)tri + 1));
    p->sv_tile_start = o; o = align_up(o + 4 * ((size_t)tiles + 1));
    p->sv_bins = o; o = align_up(o + 4 * (size_t)p->capacity);
    p->sv_bin_pair = o; o = align_up(o + 4 * (size_t)p->capacity);
    p->sv_overflow = o; o = align_up(o + 4 * ((size_t)tri + 1));
    p->sv_zc = o; o = align_up(o + 4 * (size_t)std::max(L, 1));
    p->sv_aa_flag = o; o = align_up(o + (size_t)pix);        // per sample: it has candidate smoothing pairs
    p->saved_bytes = std::max<size_t>(o, kAlign);
    // scratch layout
    o = 0;
    p->sc_tile_cnt = o; o = align_up(o + 4 * ((size_t)tiles + 1));
    p->sc_aa_count = o; o = align_up(o + 4 * (size_t)kAaSegments);      // light smoothing list counters
    p->sc_zero_fwd_end = o;
    p->sc_pair_cnt = o; o = align_up(o + 4 * ((size_t)tri + 1));
    p->sc_scan = o; o = align_up(o + 4 * (size_t)std::max(scan_scratch_words((int)tri), scan_scratch_words((int)tiles)) + 64);
    p->sc_facing = o; o = align_up(o + (size_t)tri + 1);
    p->sc_pair_slot = o; o = align_up(o + 4 * (size_t)p->capacity);    // each pair's slot in its tile's bin
    p->sc_big_bin = o; o = align_up(o + 4 * ((size_t)tri + 1));       // triangles binned a workgroup each
    // light-map samples whose smoothing has candidate pairs: the segmented list of the light smoothing
    // grid (launch_aa_forward cuts it the same way)
    {
        const AaList ll = aa_list_for(nullptr, nullptr, (long long)((p->max_light_texels + 255) / 256) * L);
        p->sc_aa_list = o; o = align_up(o + 8 * (size_t)ll.nseg * ll.segcap + 8);
    }
    p->sc_F1 = o; o = align_up(o + 4 * (size_t)(maps + padmaps));
    p->sc_fwd_end = o;                 // the forward touches nothing past this
    p->sc_pair_flag = o; o = align_up(o + (size_t)p->capacity);
    p->sc_gimg0 = o; o = align_up(o + 4 * (size_t)img);
    p->sc_bigcount = o; o = align_up(o + 64);
    p->sc_zero_rec = o; o = align_up(o + 32);          // an all-zero corner record for the vertex gather
    p->sc_gM = o; o = align_up(o + 4 * (size_t)fmaps);
    p->sc_gclip = o; o = align_up(o + 16 * (size_t)clip);
    p->sc_zero_bwd_end = o;
    p->sc_glight = o; o = align_up(o + 4 * 3 * (size_t)kGlightBlocks * (size_t)std::max(L, 1));
    p->sc_gF1 = o; o = align_up(o + 4 * (size_t)(maps + padmaps));
    p->sc_pair_sums = o; o = align_up(o + 4 * 21 * (size_t)p->capacity);
    p->sc_gtri = o; o = align_up(o + 4 * 24 * ((size_t)tri + 1));       // three 8-float corner records per triangle
    p->sc_biglist = o; o = align_up(o + 4 * ((size_t)tri + 1));
    p->sc_part_light = o; o = align_up(o + 4 * 3 * (size_t)(part_light + 1));
    p->sc_part_gm = o; o = align_up(o + 4 * 3 * (size_t)(part_gm + 1));
    p->sc_jac = o; o = align_up(o + 4 * (size_t)kJac * (size_t)std::max(L, 1));
    p->sc_part_render = o; o = align_up(o + 4 * (size_t)(part_render + 1));
    p->scratch_bytes = o;

    // device uploads
    std::vector<int> adj(3 * (size_t)Ft, -1);
    for (int b = 0; b < B; ++b)
        build_adjacency(d->faces + 3 * (size_t)p->face_off[b], p->face_off[b + 1] - p->face_off[b],
                        p->vert_off[b + 1] - p->vert_off[b], adj.data() + 3 * (size_t)p->face_off[b]);
    std::vector<int> tile_view((size_t)tiles);
    for (int v = 0; v < p->nviews; ++v) {
        const ViewConst &x = p->views_h[v];
        for (int t = 0; t < x.tiles_x * x.tiles_y; ++t) tile_view[x.tile_off + t] = v;
    }
    // backward gather lists
    std::vector<int> cam_off(Cm + 1, 0), cam_list;
    for (int c = 0; c < Cm; ++c) {
        for (int r = 0; r < R; ++r)
            if (d->renders[r].camera == c) cam_list.push_back(r);
        cam_off[c + 1] = (int)cam_list.size();
    }
    std::vector<int> sv_off(B + 1, 0), sv_list;
    for (int b = 0; b < B; ++b) {
        for (int v = 0; v < p->nviews; ++v)
            if (p->views_h[v].scene == b) sv_list.push_back(v);
        sv_off[b + 1] = (int)sv_list.size();
    }
    std::vector<int> vc_off(Vt + 1, 0), vc_list(3 * (size_t)Ft);
    for (int b = 0; b < B; ++b)
        for (long long f = p->face_off[b]; f < p->face_off[b + 1]; ++f)
            for (int k = 0; k < 3; ++k) vc_off[p->vert_off[b] + d->faces[3 * f + k] + 1]++;
    for (long long v = 0; v < Vt; ++v) vc_off[v + 1] += vc_off[v];
    {
        std::vector<int> fill(vc_off.begin(), vc_off.end() - 1);
        for (int b = 0; b < B; ++b)
            for (long long f = p->face_off[b]; f < p->face_off[b + 1]; ++f)
                for (int k = 0; k < 3; ++k) {
                    const long long gv = p->vert_off[b] + d->faces[3 * f + k];
                    vc_list[fill[gv]++] = (int)((f - p->face_off[b]) << 2) | k;
                }
    }
    std::vector<int> lr_off(L + 1, 0), lr_list;
    for (int l = 0; l < L; ++l) {
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < d->renders[r].light_count; ++q)
                if (d->render_light_list[d->renders[r].light_begin + q] == l) lr_list.push_back((r << 5) | q);
        lr_off[l + 1] = (int)lr_list.size();
    }
    dsm_status st = DSM_OK;
    if (st == DSM_OK) st = upload(&p->cam_renders_off_d, cam_off.data(), cam_off.size());
    if (st == DSM_OK) st = upload(&p->cam_renders_d, cam_list.data(), cam_list.size());
    if (st == DSM_OK) st = upload(&p->scene_views_off_d, sv_off.data(), sv_off.size());
    if (st == DSM_OK) st = upload(&p->scene_views_d, sv_list.data(), sv_list.size());
    if (st == DSM_OK) st = upload(&p->vc_off_d, vc_off.data(), vc_off.size());
    if (st == DSM_OK) st = upload(&p->vc_list_d, vc_list.data(), vc_list.size());
    if (st == DSM_OK) st = upload(&p->light_renders_off_d, lr_off.data(), lr_off.size());
    if (st == DSM_OK) st = upload(&p->light_renders_d, lr_list.data(), lr_list.size());
    if (st == DSM_OK) st = upload(&p->scene_face_off_d, p->face_off.data(), p->face_off.size());
    if (st == DSM_OK) st = upload(&p->views_d, p->views_h.data(), p->views_h.size());
    if (st == DSM_OK) st = upload(&p->light_cams_d, p->light_cams_h.data(), p->light_cams_h.size());
    if (st == DSM_OK) st = upload(&p->renders_d, p->renders_h.data(), p->renders_h.size());
    if (st == DSM_OK) st = upload(&p->render_lights_d, p->render_lights_h.data(), p->render_lights_h.size());
    if (st == DSM_OK) st = upload(&p->faces_d, d->faces, 3 * (size_t)Ft);
    if (st == DSM_OK) st = upload(&p->adj_d, adj.data(), adj.size());
    if (st == DSM_OK) st = upload(&p->tile_view_d, tile_view.data(), tile_view.size());
    if (st == DSM_OK) st = upload(&p->blur_jobs_d, p->blur_jobs_h.data(), p->blur_jobs_h.size());
    if (st == DSM_OK && !p->cube_taps_h.empty())
        st = upload(&p->cube_taps_d, p->cube_taps_h.data(), p->cube_taps_h.size());
    if (st == DSM_OK) st = upload(&p->scene_vert_off_d, p->vert_off.data(), p->vert_off.size());
    if (st == DSM_OK) st = upload(&p->pose_counts_d, p->pose_counts.data(), p->pose_counts.size());
    if (st == DSM_OK) st = upload(&p->pose_centers_d, p->pose_centers.data(), p->pose_centers.size());
    if (st != DSM_OK) {
        dsm_plan_destroy(p);
        return st;
    }
    *out_plan = p;
    return DSM_OK;
}

extern "C" void dsm_plan_destroy(dsm_plan *p) {
    if (!p) return;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void *bufs[] = {p->views_d, p->light_cams_d, p->renders_d, p->render_lights_d, p->faces_d, p->adj_d,
                    p->tile_view_d, p->blur_jobs_d, p->cube_taps_d, p->scene_vert_off_d, p->pose_counts_d, p->pose_centers_d,
                    p->cam_renders_off_d, p->cam_renders_d, p->scene_views_off_d, p->scene_views_d, p->vc_off_d,
                    p->vc_list_d, p->light_renders_off_d, p->light_renders_d, p->scene_face_off_d};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

extern "C" dsm_status dsm_plan_info_get(const dsm_plan *p, dsm_plan_info *out) {
    if (!p || !out) return DSM_ERR_INVALID_ARG;
    out->total_vertices = p->V_total;
    out->total_faces = p->F_total;
    out->image_floats = p->image_floats;
    out->saved_bytes = (int64_t)p->saved_bytes;
    out->scratch_bytes = (int64_t)p->scratch_bytes;
    out->forward_scratch_bytes = (int64_t)p->sc_fwd_end;
    out->map_floats = p->map_floats;
    out->tile_size = p->tile;
    out->bin_capacity_scale = p->bin_scale;
    return DSM_OK;
}

#define DSM_TRY(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return DSM_ERR_HIP;   \
    } while (0)

namespace {

template <class T>
T *at(void *base, size_t off) { return (T *)((char *)base + off); }
template <class T>
const T *at(const void *base, size_t off) { return (const T *)((const char *)base + off); }

// Stage timing (nullable): ev[2i] opens stage i, ev[2i + 1] closes it.  With
// a flush buffer, flush_bytes of it are overwritten after a stage closes
// and before the next one opens, so every stage starts with cold caches.
struct StageMarks {
    hipEvent_t *ev;
    void *flush;
    size_t flush_bytes;
};
dsm_status stage_mark(const StageMarks *m, int i, hipStream_t s) {
    if (!m) return DSM_OK;
    if (i > 0) DSM_TRY(hipEventRecord(m->ev[2 * (i - 1) + 1], s));
    if (i < DSM_STAGE_COUNT) {
        if (m->flush) DSM_TRY(zero_async(m->flush, m->flush_bytes, s));
        DSM_TRY(hipEventRecord(m->ev[2 * i], s));
    }
    return DSM_OK;
}
#define DSM_MARK(i)                                                      \
    do {                                                                 \
        const dsm_status mark_st_ = stage_mark(marks, (i), s);          \
        if (mark_st_ != DSM_OK) return mark_st_;                        \
    } while (0)

dsm_status enqueue_forward(dsm_plan *p, const float *verts, const float *lparams, const float *albedo, void *saved,
                           void *scratch, float *images, hipStream_t s, const StageMarks *marks = nullptr) {
    DevCounters *cnt = at<DevCounters>(saved, p->sv_counters);
    unsigned *tile_cnt = at<unsigned>(scratch, p->sc_tile_cnt);
    unsigned *pair_slot = at<unsigned>(scratch, p->sc_pair_slot);
    uint2 *aa_list = at<uint2>(scratch, p->sc_aa_list);
    unsigned *aa_count = at<unsigned>(scratch, p->sc_aa_count);
    unsigned *pair_cnt = at<unsigned>(scratch, p->sc_pair_cnt);
    unsigned *pair_off = at<unsigned>(saved, p->sv_pair_off);
    unsigned *scan = at<unsigned>(scratch, p->sc_scan);
    unsigned *tile_start = at<unsigned>(saved, p->sv_tile_start);
    unsigned *bins = at<unsigned>(saved, p->sv_bins);
    unsigned *bin_pair = at<unsigned>(saved, p->sv_bin_pair);
    unsigned *overflow = at<unsigned>(saved, p->sv_overflow);
    float *F1 = at<float>(scratch, p->sc_F1);
    unsigned long long *keys = at<unsigned long long>(saved, p->sv_keys);
    unsigned char *aa_flag = at<unsigned char>(saved, p->sv_aa_flag);
    float4 *clip = at<float4>(saved, p->sv_clip);
    TriSetup *setup = at<TriSetup>(saved, p->sv_setup);
    unsigned char *silm = at<unsigned char>(saved, p->sv_sil);
    TriVerts *tv = at<TriVerts>(saved, p->sv_tv);
    float *F0 = at<float>(saved, p->sv_F0);
    float *Mm = at<float>(saved, p->sv_M);
    float *img0 = at<float>(saved, p->sv_img0);

    DSM_MARK(DSM_STAGE_SETUP);
    // with the light frames, the counters (saved) and the tile counts (scratch) are cleared
    DSM_TRY(launch_light_frames(p->views_d, p->light_cams_d, lparams, p->L, nullptr, at<float>(saved, p->sv_zc), saved,
                                p->sv_zero_end, scratch, p->sc_zero_fwd_end, s));
    DSM_TRY(launch_transform(p->views_d, p->nviews, p->max_verts, verts, clip, s));
    DSM_TRY(launch_tri_verts(p->scene_vert_off_d, p->scene_face_off_d, p->B, p->max_scene_faces, p->faces_d, verts,
                             albedo, p->C, tv, s));
    signed char *facing8 = at<signed char>(scratch, p->sc_facing);
    DSM_TRY(launch_setup(p->views_d, p->nviews, p->max_faces, p->faces_d, clip, setup, facing8, pair_cnt, p->tile,
                         cnt, s));
    DSM_TRY(launch_silhouettes(p->views_d, p->nviews, p->max_faces, p->adj_d, facing8, silm, s));
    DSM_MARK(DSM_STAGE_BIN);
    DSM_TRY(launch_scan(pair_cnt, pair_off, scan, p->ntri, s));
    DSM_TRY(launch_binning(p->views_d, setup, pair_off, p->ntri, p->capacity, p->tile, tile_cnt, tile_start,
                           pair_slot, scan, p->ntiles, bins, bin_pair, overflow, at<unsigned>(scratch, p->sc_big_bin), cnt,
                           s));
    DSM_MARK(DSM_STAGE_RASTER);
    DSM_TRY(launch_raster(p->views_d, p->tile_view_d, p->ntiles, p->tile, setup, tile_start, bins, overflow, cnt, cnt,
                          keys, s));
    DSM_MARK(DSM_STAGE_RESOLVE);
    DSM_TRY(launch_resolve(p->views_d, p->L, p->max_light_texels, tv, keys, F0, s));
    DSM_MARK(DSM_STAGE_LIGHT_AA);
    DSM_TRY(launch_aa_forward(true, p->views_d, p->renders_d, p->L, p->max_light_texels, setup, p->faces_d, silm,
                              verts, keys, F0, F1, 2, aa_list, aa_count, aa_flag, s));
    DSM_MARK(DSM_STAGE_FILTER);
    if (p->has_cube) DSM_TRY(launch_cube_pad(p->views_d, p->L, p->max_cube_padded, p->cube_taps_d, F1, s));
    for (const auto &g : p->blur_groups)
        DSM_TRY(launch_blur(p->blur_jobs_d + g.first, g.n, g.tiles, F1, Mm, false, g.R, s));
    DSM_MARK(DSM_STAGE_LOOKUP);
    DSM_TRY(launch_lookup(p->views_d, p->renders_d, p->R, p->max_cam_pix, p->render_lights_d, tv, albedo, keys, Mm,
                          img0, p->C, s));
    DSM_MARK(DSM_STAGE_CAMERA_AA);
    DSM_TRY(launch_aa_forward(false, p->views_d, p->renders_d, p->R, p->max_cam_pix, setup, p->faces_d, silm,
                              verts, keys, img0, images, p->C, nullptr, nullptr, aa_flag, s));
    return DSM_OK;
}

dsm_status enqueue_backward(dsm_plan *p, const float *verts, const float *lparams, const float *albedo,
                            const void *saved, void *scratch, const float *gimg, float *gverts, float *glparams,
                            float *galbedo, hipStream_t s, const StageMarks *marks = nullptr) {
    const unsigned long long *keys = at<unsigned long long>(saved, p->sv_keys);
    const unsigned char *aa_flag = at<unsigned char>(saved, p->sv_aa_flag);
    const float4 *clip = at<float4>(saved, p->sv_clip);
    const TriSetup *setup = at<TriSetup>(saved, p->sv_setup);
    const unsigned char *silm = at<unsigned char>(saved, p->sv_sil);
    const TriVerts *tv = at<TriVerts>(saved, p->sv_tv);
    const float *F0 = at<float>(saved, p->sv_F0);
    const float *Mm = at<float>(saved, p->sv_M);
    const float *img0 = at<float>(saved, p->sv_img0);
    const DevCounters *cnt = at<DevCounters>(saved, p->sv_counters);
    const unsigned *pair_off = at<unsigned>(saved, p->sv_pair_off);
    const unsigned *tile_start = at<unsigned>(saved, p->sv_tile_start);
    const unsigned *bins = at<unsigned>(saved, p->sv_bins);
    const unsigned *bin_pair = at<unsigned>(saved, p->sv_bin_pair);
    unsigned char *pair_flag = at<unsigned char>(scratch, p->sc_pair_flag);
    const unsigned *overflow = at<unsigned>(saved, p->sv_overflow);
    float *gimg0 = at<float>(scratch, p->sc_gimg0);
    unsigned *big_count = at<unsigned>(scratch, p->sc_bigcount);
    float *gM = at<float>(scratch, p->sc_gM);
    float4 *gclip = at<float4>(scratch, p->sc_gclip);
    float *gF1 = at<float>(scratch, p->sc_gF1);
    float *pair_sums = at<float>(scratch, p->sc_pair_sums);
    float *gtri = at<float>(scratch, p->sc_gtri);
    unsigned *big_list = at<unsigned>(scratch, p->sc_biglist);
    float *part_light = at<float>(scratch, p->sc_part_light);
    float *part_gm = at<float>(scratch, p->sc_part_gm);
    float *part_render = at<float>(scratch, p->sc_part_render);
    float *jac = at<float>(scratch, p->sc_jac);

    DSM_MARK(DSM_STAGE_BWD_SETUP);
    // with the light frames and their Jacobian: big count, zero corner record, gM, silhouette
    // gclip; and the pair flags (the 8x8 tile walks set only the flags of pairs that got a sum)
    DSM_TRY(launch_light_frames(p->views_d, p->light_cams_d, lparams, p->L, jac, nullptr, big_count,
                                p->sc_zero_bwd_end - p->sc_bigcount, pair_flag, ((size_t)p->capacity + 3) & ~(size_t)3,
                                s));
    DSM_TRY(launch_overflow_rows_zero(overflow, cnt, gtri, s));
    DSM_MARK(DSM_STAGE_CAMERA_AA_ADJ);
    DSM_TRY(launch_aa_camera_backward(p->views_d, p->renders_d, p->R, p->max_cam_pix, setup, p->faces_d, silm,
                                      verts, keys, aa_flag, img0, gimg, gimg0, gclip, p->C, s));
    DSM_MARK(DSM_STAGE_LOOKUP_ADJ);
    DSM_TRY(launch_lookup_backward(p->tile, p->views_d, p->L, p->Cm, p->max_cam_tiles, p->max_lights_per_render,
                                   p->renders_d, p->cam_renders_off_d, p->cam_renders_d, p->render_lights_d,
                                   p->faces_d, verts, albedo, tv, keys, Mm, gimg0, gM, setup, tile_start, bins,
                                   bin_pair, pair_flag, pair_sums, gtri, part_render, p->C, jac, pair_off,
                                   p->capacity, s));
    DSM_MARK(DSM_STAGE_FILTER_ADJ);
    for (const auto &g : p->blur_groups)
        DSM_TRY(launch_blur(p->blur_jobs_d + p->L + g.first, g.n, g.tiles, gM, gF1, true, g.R, s));
    if (p->has_cube)
        DSM_TRY(launch_cube_pad_transpose(p->views_d, p->L, p->max_cube_texels, p->max_cube_ring, p->cube_taps_d,
                                          gF1, s));
    DSM_MARK(DSM_STAGE_LIGHT_ADJ);
    DSM_TRY(launch_light_backward(p->tile, p->views_d, p->L, p->max_light_tiles, setup, p->faces_d, silm, verts,
                                  tv, keys, aa_flag, F0, gF1, gclip, tile_start, bins, bin_pair, pair_flag, pair_sums,
                                  gtri, part_light, jac, pair_off, p->capacity, s));
    DSM_MARK(DSM_STAGE_VERTEX_GRAD);
    DSM_TRY(launch_vertex_gradients(p->views_d, p->L, p->B, p->max_scene_verts, p->max_scene_faces, p->ntri,
                                    p->capacity, p->scene_vert_off_d, p->scene_face_off_d, p->scene_views_off_d,
                                    p->scene_views_d, p->vc_off_d, p->vc_list_d, pair_off, pair_flag, pair_sums, gtri,
                                    at<float>(scratch, p->sc_zero_rec), big_list,
                                    big_count, verts, gclip, gverts, part_gm, galbedo, p->C, jac, s));
    DSM_MARK(DSM_STAGE_LIGHT_GRAD);
    DSM_TRY(launch_glight_reduce(p->views_d, p->L, p->renders_d, p->light_renders_off_d, p->light_renders_d, part_gm,
                                 part_light, part_render, at<float>(scratch, p->sc_glight), glparams, s));
    DSM_MARK(DSM_STAGE_COUNT);
    return DSM_OK;
}

bool buffers_ok(const dsm_plan *p, const void *saved, size_t saved_bytes, const void *scratch, size_t scratch_bytes,
                dsm_status *st) {
    if (!saved || !scratch) { *st = DSM_ERR_INVALID_ARG; return false; }
    if (saved_bytes < p->saved_bytes || scratch_bytes < p->scratch_bytes) { *st = DSM_ERR_WORKSPACE_TOO_SMALL; return false; }
    if (((uintptr_t)saved & 255) || ((uintptr_t)scratch & 255)) { *st = DSM_ERR_INVALID_ARG; return false; }
    return true;
}

}  // namespace

extern "C" dsm_status dsm_forward(dsm_plan *p, const float *verts, const float *lparams, const float *albedo,
                                  void *saved, size_t saved_bytes, void *scratch, size_t scratch_bytes,
                                  float *images, dsm_stream stream) {
    if (!p) return DSM_ERR_INVALID_ARG;
    dsm_status st;
    if (!buffers_ok(p, saved, saved_bytes, scratch, scratch_bytes, &st)) return st;
    if ((p->V_total > 0 && !verts) || (p->L > 0 && !lparams) || (p->F_total > 0 && !albedo) ||
        (p->image_floats > 0 && !images))
        return DSM_ERR_INVALID_ARG;
    return enqueue_forward(p, verts, lparams, albedo, saved, scratch, images, (hipStream_t)stream);
}

namespace dsm {
dsm_status forward_in_scratch(dsm_plan *p, const float *verts, const float *lparams, const float *albedo, void *saved,
                              size_t saved_bytes, void *scratch, size_t scratch_bytes, float *images,
                              hipStream_t stream) {
    if (!p || !saved || !scratch) return DSM_ERR_INVALID_ARG;
    if (saved_bytes < p->saved_bytes || scratch_bytes < p->sc_fwd_end) return DSM_ERR_WORKSPACE_TOO_SMALL;
    if (((uintptr_t)saved & 255) || ((uintptr_t)scratch & 255)) return DSM_ERR_INVALID_ARG;
    if ((p->V_total > 0 && !verts) || (p->L > 0 && !lparams) || (p->F_total > 0 && !albedo) ||
        (p->image_floats > 0 && !images))
        return DSM_ERR_INVALID_ARG;
    return enqueue_forward(p, verts, lparams, albedo, saved, scratch, images, stream);
}
}  // namespace dsm

extern "C" dsm_status dsm_backward(dsm_plan *p, const float *verts, const float *lparams, const float *albedo,
                                   const void *saved, size_t saved_bytes, void *scratch, size_t scratch_bytes,
                                   const float *gimg, float *gverts, float *glparams, float *galbedo,
                                   dsm_stream stream) {
    if (!p) return DSM_ERR_INVALID_ARG;
    dsm_status st;
    if (!buffers_ok(p, saved, saved_bytes, scratch, scratch_bytes, &st)) return st;
    if ((p->V_total > 0 && (!verts || !gverts)) || (p->L > 0 && (!lparams || !glparams)) ||
        (p->F_total > 0 && !albedo) || (p->image_floats > 0 && !gimg))
        return DSM_ERR_INVALID_ARG;
    return enqueue_backward(p, verts, lparams, albedo, saved, scratch, gimg, gverts, glparams, galbedo,
                            (hipStream_t)stream);
}

extern "C" dsm_status dsm_time_stages(dsm_plan *p, const float *verts, const float *lparams, const float *albedo,
                                      void *saved, size_t saved_bytes, void *scratch, size_t scratch_bytes,
                                      float *images, const float *gimg, float *gverts, float *glparams,
                                      float *galbedo, int32_t reps, void *flush, size_t flush_bytes, float *ms_out,
                                      dsm_stream stream) {
    if (!p || !ms_out || reps < 1 || reps > DSM_MAX_TIMING_REPS || !stream) return DSM_ERR_INVALID_ARG;
    if (flush && (flush_bytes < 4 || ((uintptr_t)flush & 3))) return DSM_ERR_INVALID_ARG;
    dsm_status st;
    if (!buffers_ok(p, saved, saved_bytes, scratch, scratch_bytes, &st)) return st;
    if ((p->V_total > 0 && (!verts || !gverts)) || (p->L > 0 && (!lparams || !glparams)) ||
        (p->F_total > 0 && !albedo) || (p->image_floats > 0 && (!images || !gimg)))
        return DSM_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    constexpr int NE = 2 * DSM_STAGE_COUNT;
    std::vector<hipEvent_t> ev((size_t)reps * NE, nullptr);
    dsm_status r = DSM_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) { e = nullptr; r = DSM_ERR_HIP; break; }
    for (int i = 0; i < reps && r == DSM_OK; ++i) {
        const StageMarks m{ev.data() + (size_t)i * NE, flush, flush ? flush_bytes : 0};
        r = enqueue_forward(p, verts, lparams, albedo, saved, scratch, images, s, &m);
        if (r == DSM_OK)
            r = enqueue_backward(p, verts, lparams, albedo, saved, scratch, gimg, gverts, glparams, galbedo, s, &m);
    }
    if (r == DSM_OK && hipStreamSynchronize(s) != hipSuccess) r = DSM_ERR_HIP;
    for (int k = 0; k < DSM_STAGE_COUNT; ++k) ms_out[k] = 0.f;
    for (int i = 0; i < reps && r == DSM_OK; ++i)
        for (int k = 0; k < DSM_STAGE_COUNT; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[(size_t)i * NE + 2 * k], ev[(size_t)i * NE + 2 * k + 1]) != hipSuccess) {
                r = DSM_ERR_HIP;
                break;
            }
            ms_out[k] += ms / (float)reps;
        }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return r;
}

extern "C" dsm_status dsm_pose_forward(dsm_plan *p, const float *local, const float *poses, float *world,
                                       dsm_stream stream) {
    if (!p || (p->V_total > 0 && (!local || !world)) || !poses) return DSM_ERR_INVALID_ARG;
    if (local == world) return DSM_ERR_INVALID_ARG;
    DSM_TRY(launch_pose(p->scene_vert_off_d, p->pose_counts_d, p->pose_centers_d, p->B,
                        std::max(p->max_verts, 1), local, poses, world, (hipStream_t)stream));
    return DSM_OK;
}

extern "C" dsm_status dsm_pose_backward(dsm_plan *p, const float *local, const float *poses, const float *gworld,
                                        float *gposes, dsm_stream stream) {
    if (!p || (p->V_total > 0 && (!local || !gworld)) || !poses || !gposes) return DSM_ERR_INVALID_ARG;
    DSM_TRY(zero_async(gposes, 4 * 6 * (size_t)p->B, (hipStream_t)stream));
    DSM_TRY(launch_pose_backward(p->scene_vert_off_d, p->pose_counts_d, p->B, std::max(p->max_pose_verts, 1), local,
                                 poses, gworld, gposes, (hipStream_t)stream));
    return DSM_OK;
}

extern "C" dsm_status dsm_graph_capture(dsm_plan *p, const float *local, const float *poses, float *verts,
                                        const float *lparams, const float *albedo, void *saved, size_t saved_bytes,
                                        void *scratch, size_t scratch_bytes, float *images, const float *gimg,
                                        float *gverts, float *glparams, float *galbedo, float *gposes,
                                        dsm_stream stream) {
    if (!p || !stream) return DSM_ERR_INVALID_ARG;
    dsm_status st;
    if (!buffers_ok(p, saved, saved_bytes, scratch, scratch_bytes, &st)) return st;
    if (!verts || !lparams || !albedo || !images || !gimg || !gverts || !glparams) return DSM_ERR_INVALID_ARG;
    if (poses && (!local || !gposes)) return DSM_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    DSM_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    dsm_status r = DSM_OK;
    if (poses) r = dsm_pose_forward(p, local, poses, verts, stream);
    if (r == DSM_OK) r = enqueue_forward(p, verts, lparams, albedo, saved, scratch, images, s);
    if (r == DSM_OK)
        r = enqueue_backward(p, verts, lparams, albedo, saved, scratch, gimg, gverts, glparams, galbedo, s);
    if (r == DSM_OK && poses) r = dsm_pose_backward(p, local, poses, gverts, gposes, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (r != DSM_OK) { if (g) (void)hipGraphDestroy(g); return r; }
    if (e != hipSuccess || !g) return DSM_ERR_HIP;
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) { (void)hipGraphDestroy(g); return DSM_ERR_HIP; }
    p->graph = g;
    p->graph_exec = x;
    return DSM_OK;
}

extern "C" dsm_status dsm_graph_launch(dsm_plan *p, dsm_stream stream) {
    if (!p || !p->graph_exec) return DSM_ERR_INVALID_ARG;
    DSM_TRY(hipGraphLaunch(p->graph_exec, (hipStream_t)stream));
    return DSM_OK;
}

extern "C" dsm_status dsm_get_view_keys(const dsm_plan *p, const void *saved, int32_t view, uint64_t *out,
                                        dsm_stream stream) {
    if (!p || !saved || !out || view < 0 || view >= p->nviews) return DSM_ERR_INVALID_ARG;
    const ViewConst &v = p->views_h[view];
    DSM_TRY(hipMemcpyAsync(out, at<char>(saved, p->sv_keys + 8 * (size_t)v.pix_off), 8 * (size_t)v.W * v.H,
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return DSM_OK;
}

extern "C" dsm_status dsm_get_light_maps(const dsm_plan *p, const void *saved, const void *scratch, int32_t light,
                                         int32_t which, float *out, dsm_stream stream) {
    if (!p || !out || light < 0 || light >= p->L || which < 0 || which > 2) return DSM_ERR_INVALID_ARG;
    if ((which != 1 && !saved) || (which == 1 && !scratch)) return DSM_ERR_INVALID_ARG;
    const ViewConst &v = p->views_h[light];
    const size_t base = which == 0 ? p->sv_F0 : which == 1 ? p->sc_F1 : p->sv_M;
    const void *src = which == 1 ? scratch : saved;
    if (!saved) return DSM_ERR_INVALID_ARG;       // holds the light's reference depth
    const bool il = which == 2;
    // filtered maps: the face itself, without the texels sampled from cube neighbours
    hipLaunchKernelGGL(light_maps_out_kernel, dim3((v.W * v.W + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       at<float>(src, base + 4 * (size_t)(il ? v.fmap_off : v.map_off)), v.W,
                       il ? v.W + 2 * v.fpad : v.W, il ? v.fpad : 0, il, at<float>(saved, p->sv_zc + 4 * (size_t)light), v.warp_c, out);
    DSM_TRY(hipGetLastError());
    return DSM_OK;
}

extern "C" dsm_status dsm_get_render_image0(const dsm_plan *p, const void *saved, int32_t render, float *out,
                                            dsm_stream stream) {
    if (!p || !saved || !out || render < 0 || render >= p->R) return DSM_ERR_INVALID_ARG;
    const RenderConst &r = p->renders_h[render];
    DSM_TRY(hipMemcpyAsync(out, at<char>(saved, p->sv_img0 + 4 * (size_t)r.img_off),
                           4 * (size_t)r.W * r.H * p->C, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return DSM_OK;
}

extern "C" dsm_status dsm_get_stats(const dsm_plan *p, const void *saved, dsm_stats *out, dsm_stream stream) {
    if (!p || !saved || !out) return DSM_ERR_INVALID_ARG;
    DevCounters c;
    DSM_TRY(hipMemcpyAsync(&c, at<char>(saved, p->sv_counters), sizeof(c), hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
    DSM_TRY(hipStreamSynchronize((hipStream_t)stream));
    out->culled_triangles = c.culled;
    out->binned_pairs = c.pairs;
    out->overflow_triangles = c.overflow;
    out->bad_indices = c.bad_indices;
    return DSM_OK;
}
