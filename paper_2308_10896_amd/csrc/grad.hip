// Reverse-mode kernels (Sec. 4: the gradient of the loss w.r.t. the scene
// parameters flows through the visibility v, the filtered moments
// m1 = G f~, m2 = G f^2~ and the smoothed shadow map; the Jacobians are never
// formed, Sec. 5).  Every kernel is the hand-written adjoint of its forward
// counterpart in shade.hip / raster.hip:
//
//   camera smoothing^T    : dL/dimage -> dL/dimage0, dL/d(clip of edge ends)
//   lookup^T              : dL/dimage0 -> dL/d(m1, m2) scattered bilinearly,
//                           dL/dvertices, dL/d(camera clip), dL/d(light frame),
//                           dL/dalbedo.  For d > mu:
//                           dv/dmu = 2 s^2 (d-mu) / (s^2+(d-mu)^2)^2 = -dv/dd
//                           (the paper's derivative, s^2 held fixed), and
//                           dv/ds^2 = (d-mu)^2 / (s^2+(d-mu)^2)^2 with
//                           s^2 = m2 - m1^2 (zero where the floor is active).
//   filter^T              : blur.hip (adjoint mode)
//   light smoothing^T + resolve^T (fused per texel)
//   transform^T           : dL/dclip -> dL/dvertices (M^T) and dL/dM
//
// Vertex-indexed gradients are scattered with atomics after a wavefront
// reduction over lanes that share a triangle (most lanes of a wave do), so a
// ground plane covered by two triangles costs one atomic per wave, not 64.
#include "aa.h"
#include "dsm_internal.h"
#include "frames.h"

namespace dsm {

// Scatter N values per lane to addresses that depend only on (key, i): lanes
// with equal keys are summed across the wave first.  All 64 lanes must call.
template <int N, class Addr>
__device__ __forceinline__ void scatter_by_key(bool active, int key, const float (&val)[N], Addr addr) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int k = __shfl(key, leader, 64);
        const bool mine = active && key == k;
        const unsigned long long m = __ballot(mine);
        pending &= ~m;
        if (__popcll(m) >= 4) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float s = wave_sum(mine ? val[i] : 0.f);
                if (lane == leader) atomic_add_f32(addr(k, i), s);
            }
        } else if (mine) {
#pragma unroll
            for (int i = 0; i < N; ++i) atomic_add_f32(addr(k, i), val[i]);
        }
    }
}

// Wave-sum N values and add them at dst (lane 0).  All 64 lanes must call.
template <int N>
__device__ __forceinline__ void wave_add(const float (&val)[N], float *dst) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float s = wave_sum(val[i]);
        if ((threadIdx.x & 63) == 0) atomic_add_f32(dst + i, s);
    }
}

__device__ __forceinline__ float ndc_c(int i, int n) { return (float)(2 * i + 1) / (float)n - 1.0f; }

struct BaryFull {
    float a0x, a0y, a1x, a1y, a2x, a2y, k0, k1, k2, s, b0, b1, b2;
};

__device__ __forceinline__ BaryFull bary_full(float4 c0, float4 c1, float4 c2, float px, float py) {
    BaryFull r;
    r.a0x = c0.x - px * c0.w; r.a0y = c0.y - py * c0.w;
    r.a1x = c1.x - px * c1.w; r.a1y = c1.y - py * c1.w;
    r.a2x = c2.x - px * c2.w; r.a2y = c2.y - py * c2.w;
    r.k0 = r.a1x * r.a2y - r.a1y * r.a2x;
    r.k1 = r.a2x * r.a0y - r.a2y * r.a0x;
    r.k2 = r.a0x * r.a1y - r.a0y * r.a1x;
    r.s = r.k0 + r.k1 + r.k2;
    r.b0 = r.k0 / r.s; r.b1 = r.k1 / r.s; r.b2 = r.k2 / r.s;
    return r;
}

// gb (d loss / d barycentrics) -> gradient w.r.t. clip (x, y, w) of the 3 corners: out[3*i + {0,1,2}]
__device__ __forceinline__ void bary_backward(const BaryFull &b, float px, float py, float gb0, float gb1, float gb2,
                                              float out[9]) {
    const float dotg = (gb0 * b.b0 + gb1 * b.b1) + gb2 * b.b2;
    const float gk0 = (gb0 - dotg) / b.s, gk1 = (gb1 - dotg) / b.s, gk2 = (gb2 - dotg) / b.s;
    const float ga0x = -gk1 * b.a2y + gk2 * b.a1y, ga0y = gk1 * b.a2x - gk2 * b.a1x;
    const float ga1x = gk0 * b.a2y - gk2 * b.a0y, ga1y = -gk0 * b.a2x + gk2 * b.a0x;
    const float ga2x = -gk0 * b.a1y + gk1 * b.a0y, ga2y = gk0 * b.a1x - gk1 * b.a0x;
    out[0] = ga0x; out[1] = ga0y; out[2] = -px * ga0x - py * ga0y;
    out[3] = ga1x; out[4] = ga1y; out[5] = -px * ga1x - py * ga1y;
    out[6] = ga2x; out[7] = ga2y; out[8] = -px * ga2x - py * ga2y;
}

// ----------------------------------------------------------------------------- camera smoothing^T

__global__ __launch_bounds__(256) void aa_camera_backward_kernel(
    const ViewConst *__restrict__ views, const RenderConst *__restrict__ renders, const TriSetup *__restrict__ setup,
    const int *__restrict__ faces, const int *__restrict__ adj, const float *__restrict__ verts,
    const unsigned long long *__restrict__ keys, const float *__restrict__ img0, const float *__restrict__ gimg,
    float *__restrict__ gimg0, float4 *__restrict__ gclip, int C) {
    const RenderConst &R = renders[blockIdx.y];
    const ViewConst &v = views[R.camera_view];
    const int W = v.W, H = v.H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= W * H) return;
    const float *c0 = img0 + R.img_off;
    const float *g = gimg + R.img_off;
    float acc[3];
    for (int c = 0; c < C; ++c) acc[c] = g[(long long)p * C + c];
    if (v.antialias) {
        const int i = p % W, j = p / W;
        const unsigned long long *kv = keys + v.pix_off;
        const unsigned long long ks = kv[p];
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
        for (int d = 0; d < 4; ++d) {
            const int in_ = i + di[d], jn = j + dj[d];
            if (in_ < 0 || in_ >= W || jn < 0 || jn >= H) continue;
            const int q = jn * W + in_;
            const unsigned long long kn = kv[q];
            if ((unsigned)kn == (unsigned)ks) continue;
            bool self_front;
            AAPair pr;
            if (!aa_eval<true>(v, setup, faces, adj, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
            const bool self_recv = (pr.recv == 1) != self_front;
            if (self_recv) {
                double galpha = 0;
                for (int c = 0; c < C; ++c) {
                    const float gs = g[(long long)p * C + c];
                    acc[c] -= pr.w * gs;
                    galpha += (double)gs * (c0[(long long)q * C + c] - c0[(long long)p * C + c]);
                }
                galpha *= pr.recv == 1 ? 1.0 : -1.0;      // w = alpha - 1/2 or 1/2 - alpha
                float4 *ga = gclip + v.clip_off + pr.va;
                float4 *gb = gclip + v.clip_off + pr.vb;
                atomic_add_f32(&ga->x, (float)(galpha * pr.dax));
                atomic_add_f32(&ga->y, (float)(galpha * pr.day));
                atomic_add_f32(&ga->w, (float)(galpha * pr.daw));
                atomic_add_f32(&gb->x, (float)(galpha * pr.dbx));
                atomic_add_f32(&gb->y, (float)(galpha * pr.dby));
                atomic_add_f32(&gb->w, (float)(galpha * pr.dbw));
            } else {
                for (int c = 0; c < C; ++c) acc[c] += pr.w * g[(long long)q * C + c];
            }
        }
    }
    for (int c = 0; c < C; ++c) gimg0[R.img_off + (long long)p * C + c] = acc[c];
}

// ----------------------------------------------------------------------------- lookup^T

__global__ __launch_bounds__(256) void lookup_backward_kernel(
    const ViewConst *__restrict__ views, const RenderConst *__restrict__ renders,
    const int *__restrict__ render_lights, const int *__restrict__ faces, const float *__restrict__ verts,
    const float *__restrict__ albedo, const float4 *__restrict__ clip, const unsigned long long *__restrict__ keys,
    const float *__restrict__ maps, const float *__restrict__ gimg0, float *__restrict__ gmaps,
    float *__restrict__ gverts, float4 *__restrict__ gclip, float *__restrict__ glight, float *__restrict__ galbedo,
    int C) {
    const RenderConst &R = renders[blockIdx.y];
    const ViewConst &cv = views[R.camera_view];
    const int W = cv.W, H = cv.H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool inimg = p < W * H;
    const unsigned long long key = inimg ? keys[cv.pix_off + p] : kBgKey;
    float g[3] = {0.f, 0.f, 0.f};
    if (inimg)
        for (int c = 0; c < C; ++c) g[c] = gimg0[R.img_off + (long long)p * C + c];
    bool active = key != kBgKey && (g[0] != 0.f || g[1] != 0.f || g[2] != 0.f);
    const int tri = active ? (int)(unsigned)key : 0;
    const int *f = faces + 3 * (size_t)(cv.face_off + tri);
    const int i = inimg ? p % W : 0, j = inimg ? p / W : 0;
    const float px = ndc_c(i, W), py = -ndc_c(j, H);
    float4 c0 = make_float4(0, 0, 0, 1), c1 = c0, c2 = c0;
    float v0[3] = {0, 0, 0}, v1[3] = {0, 0, 0}, v2[3] = {0, 0, 0};
    if (active) {
        c0 = clip[cv.clip_off + f[0]]; c1 = clip[cv.clip_off + f[1]]; c2 = clip[cv.clip_off + f[2]];
        for (int k = 0; k < 3; ++k) {
            v0[k] = verts[3 * (size_t)(cv.vert_off + f[0]) + k];
            v1[k] = verts[3 * (size_t)(cv.vert_off + f[1]) + k];
            v2[k] = verts[3 * (size_t)(cv.vert_off + f[2]) + k];
        }
    } else {
        c0 = make_float4(1, 0, 0, 1); c1 = make_float4(0, 1, 0, 1); c2 = make_float4(0, 0, 0, 1);
        v1[0] = 1.f; v2[1] = 1.f;
    }
    const BaryFull b = bary_full(c0, c1, c2, px, py);
    const float x = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
    const float y = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
    const float z = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
    const float e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e1z = v1[2] - v0[2];
    const float e2x = v2[0] - v0[0], e2y = v2[1] - v0[1], e2z = v2[2] - v0[2];
    const float crx = e1y * e2z - e1z * e2y, cry = e1z * e2x - e1x * e2z, crz = e1x * e2y - e1y * e2x;
    const float nn = sqrtf((crx * crx + cry * cry) + crz * crz);
    const float nx = crx / nn, ny = cry / nn, nz = crz / nn;
    float rho[3] = {0.f, 0.f, 0.f};
    if (active)
        for (int c = 0; c < C; ++c) rho[c] = albedo[(size_t)(cv.face_off + tri) * C + c];
    float srho = 0.f;
    for (int c = 0; c < C; ++c) srho += g[c] * rho[c];
    float gx[3] = {0, 0, 0}, gn[3] = {0, 0, 0};
    float shade = 0.f;
    for (int q = 0; q < R.light_count; ++q) {
        const int lidx = render_lights[R.light_begin + q];
        const ViewConst &l = views[lidx];
        const float *M = l.M;
        const float cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
        const float cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
        const float cw = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
        const float ux = cx / cw, uy = cy / cw;
        const bool inside = cw > 0.f && fabsf(ux) <= 1.f && fabsf(uy) <= 1.f;
        float vis = 1.f, zz = 0.f, m1 = 0.f, m2 = 0.f, var = 0.f, dd = 0.f, fx = 0.f, fy = 0.f;
        int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
        const int S = l.W;
        const float *ma = maps + l.map_off, *mb = maps + l.map_off + (long long)S * S;
        if (inside) {
            const float sx = (ux + 1.f) * (0.5f * S) - 0.5f;
            const float sy = (1.f - uy) * (0.5f * S) - 0.5f;
            const float fx0 = floorf(sx), fy0 = floorf(sy);
            fx = sx - fx0;
            fy = sy - fy0;
            const int ix = (int)fx0, iy = (int)fy0;
            x0 = min(max(ix, 0), S - 1); x1 = min(max(ix + 1, 0), S - 1);
            y0 = min(max(iy, 0), S - 1); y1 = min(max(iy + 1, 0), S - 1);
            const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
            const long long o00 = (long long)y0 * S + x0, o01 = (long long)y0 * S + x1;
            const long long o10 = (long long)y1 * S + x0, o11 = (long long)y1 * S + x1;
            m1 = ((w00 * ma[o00] + w01 * ma[o01]) + w10 * ma[o10]) + w11 * ma[o11];
            m2 = ((w00 * mb[o00] + w01 * mb[o01]) + w10 * mb[o10]) + w11 * mb[o11];
            float depth;
            if (l.kind == kDirectional)
                depth = ((x - l.pos[0]) * l.dir[0] + (y - l.pos[1]) * l.dir[1]) + (z - l.pos[2]) * l.dir[2];
            else {
                const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
                depth = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
            }
            zz = depth / l.zfar;
            var = fmaxf(m2 - m1 * m1, l.min_var);
            dd = zz - m1;
            vis = (zz <= m1) ? 1.f : var / (var + dd * dd);
        }
        float ox, oy, oz, olen = 1.f;
        if (l.kind == kDirectional) {
            ox = -l.dir[0]; oy = -l.dir[1]; oz = -l.dir[2];
        } else {
            ox = l.pos[0] - x; oy = l.pos[1] - y; oz = l.pos[2] - z;
            olen = sqrtf((ox * ox + oy * oy) + oz * oz);
            ox /= olen; oy /= olen; oz /= olen;
        }
        const float ndo = (nx * ox + ny * oy) + nz * oz;
        const float lam = fmaxf(ndo, 0.f);
        float cone = 1.f;
        if (l.kind == kSpot) {
            const float ca = -((ox * l.dir[0] + oy * l.dir[1]) + oz * l.dir[2]);
            cone = ca >= l.cos_half ? 1.f : 0.f;
        }
        shade += lam * vis * l.intensity * cone;
        const float gvis = active ? srho * lam * l.intensity * cone : 0.f;
        const float glam = active ? srho * vis * l.intensity * cone : 0.f;
        const float gndo = ndo > 0.f ? glam : 0.f;
        gn[0] += gndo * ox; gn[1] += gndo * oy; gn[2] += gndo * oz;
        const float gox = gndo * nx, goy = gndo * ny, goz = gndo * nz;
        float gl[22];
        for (int k = 0; k < 22; ++k) gl[k] = 0.f;   // M[16], pos[3], dir[3]
        if (l.kind == kDirectional) {
            gl[19] -= gox; gl[20] -= goy; gl[21] -= goz;
        } else {
            const float od = (ox * gox + oy * goy) + oz * goz;
            const float gpx = (gox - ox * od) / olen, gpy = (goy - oy * od) / olen, gpz = (goz - oz * od) / olen;
            gl[16] += gpx; gl[17] += gpy; gl[18] += gpz;
            gx[0] -= gpx; gx[1] -= gpy; gx[2] -= gpz;
        }
        if (inside && gvis != 0.f && zz > m1) {
            const float qd = var + dd * dd;
            const float dv_dmu = 2.f * var * dd / (qd * qd);
            const bool clamped = m2 - m1 * m1 < l.min_var;
            const float dv_dvar = clamped ? 0.f : dd * dd / (qd * qd);
            const float gm1 = gvis * (dv_dmu - 2.f * m1 * dv_dvar);
            const float gm2 = gvis * dv_dvar;
            const float gz = -gvis * dv_dmu;
            const float gdepth = gz / l.zfar;
            if (l.kind == kDirectional) {
                gx[0] += gdepth * l.dir[0]; gx[1] += gdepth * l.dir[1]; gx[2] += gdepth * l.dir[2];
                gl[16] -= gdepth * l.dir[0]; gl[17] -= gdepth * l.dir[1]; gl[18] -= gdepth * l.dir[2];
                gl[19] += gdepth * (x - l.pos[0]); gl[20] += gdepth * (y - l.pos[1]); gl[21] += gdepth * (z - l.pos[2]);
            } else {
                const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
                const float dl = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
                const float ux_ = ddx / dl, uy_ = ddy / dl, uz_ = ddz / dl;
                gx[0] += gdepth * ux_; gx[1] += gdepth * uy_; gx[2] += gdepth * uz_;
                gl[16] -= gdepth * ux_; gl[17] -= gdepth * uy_; gl[18] -= gdepth * uz_;
            }
            // bilinear scatter to the moment maps
            float *ga = gmaps + l.map_off, *gb = gmaps + l.map_off + (long long)S * S;
            const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
            const long long o00 = (long long)y0 * S + x0, o01 = (long long)y0 * S + x1;
            const long long o10 = (long long)y1 * S + x0, o11 = (long long)y1 * S + x1;
            atomic_add_f32(ga + o00, gm1 * w00); atomic_add_f32(ga + o01, gm1 * w01);
            atomic_add_f32(ga + o10, gm1 * w10); atomic_add_f32(ga + o11, gm1 * w11);
            atomic_add_f32(gb + o00, gm2 * w00); atomic_add_f32(gb + o01, gm2 * w01);
            atomic_add_f32(gb + o10, gm2 * w10); atomic_add_f32(gb + o11, gm2 * w11);
            // position in the map moves with x and with the light camera
            const float dm1fx = (1.f - fy) * (ma[o01] - ma[o00]) + fy * (ma[o11] - ma[o10]);
            const float dm1fy = (1.f - fx) * (ma[o10] - ma[o00]) + fx * (ma[o11] - ma[o01]);
            const float dm2fx = (1.f - fy) * (mb[o01] - mb[o00]) + fy * (mb[o11] - mb[o10]);
            const float dm2fy = (1.f - fx) * (mb[o10] - mb[o00]) + fx * (mb[o11] - mb[o01]);
            const float gsx = gm1 * dm1fx + gm2 * dm2fx;
            const float gsy = gm1 * dm1fy + gm2 * dm2fy;
            const float hs = 0.5f * S;
            const float gcx = gsx * hs / cw, gcy = -gsy * hs / cw;
            const float gcw = (-gsx * hs * cx + gsy * hs * cy) / (cw * cw);
            const float xh[4] = {x, y, z, 1.f};
            for (int k = 0; k < 4; ++k) {
                gl[k] += gcx * xh[k];
                gl[4 + k] += gcy * xh[k];
                gl[12 + k] += gcw * xh[k];
            }
            for (int k = 0; k < 3; ++k) gx[k] += (M[k] * gcx + M[4 + k] * gcy) + M[12 + k] * gcw;
        }
        wave_add(gl, glight + 24 * lidx);
    }
    // albedo
    float ga3[3];
    for (int c = 0; c < 3; ++c) ga3[c] = c < C ? g[c] * shade : 0.f;
    scatter_by_key(active, tri, ga3, [&](int k, int c) { return galbedo + (size_t)(cv.face_off + k) * C + (c < C ? c : 0); });
    // normal: n = cr / |cr|, cr = e1 x e2
    const float ndg = (nx * gn[0] + ny * gn[1]) + nz * gn[2];
    const float gcr[3] = {(gn[0] - nx * ndg) / nn, (gn[1] - ny * ndg) / nn, (gn[2] - nz * ndg) / nn};
    const float ge1[3] = {e2y * gcr[2] - e2z * gcr[1], e2z * gcr[0] - e2x * gcr[2], e2x * gcr[1] - e2y * gcr[0]};
    const float ge2[3] = {gcr[1] * e1z - gcr[2] * e1y, gcr[2] * e1x - gcr[0] * e1z, gcr[0] * e1y - gcr[1] * e1x};
    // x = sum b_i v_i
    float gv[9];
    for (int k = 0; k < 3; ++k) {
        gv[k] = b.b0 * gx[k] - ge1[k] - ge2[k];
        gv[3 + k] = b.b1 * gx[k] + ge1[k];
        gv[6 + k] = b.b2 * gx[k] + ge2[k];
    }
    const float gb0 = (gx[0] * v0[0] + gx[1] * v0[1]) + gx[2] * v0[2];
    const float gb1 = (gx[0] * v1[0] + gx[1] * v1[1]) + gx[2] * v1[2];
    const float gb2 = (gx[0] * v2[0] + gx[1] * v2[1]) + gx[2] * v2[2];
    float gc[9];
    bary_backward(b, px, py, gb0, gb1, gb2, gc);
    const int vo = cv.vert_off, co = cv.clip_off, fo = cv.face_off;
    scatter_by_key(active, tri, gv, [&](int k, int e) {
        return gverts + 3 * (size_t)(vo + faces[3 * (size_t)(fo + k) + e / 3]) + (e % 3);
    });
    scatter_by_key(active, tri, gc, [&](int k, int e) {
        float4 *t = gclip + co + faces[3 * (size_t)(fo + k) + e / 3];
        const int comp = e % 3;
        return comp == 0 ? &t->x : (comp == 1 ? &t->y : &t->w);
    });
}

// ----------------------------------------------------------------------------- light smoothing^T + resolve^T

__global__ __launch_bounds__(256) void light_backward_kernel(
    const ViewConst *__restrict__ views, const TriSetup *__restrict__ setup, const int *__restrict__ faces,
    const int *__restrict__ adj, const float *__restrict__ verts, const float4 *__restrict__ clip,
    const unsigned long long *__restrict__ keys, const float *__restrict__ F0, const float *__restrict__ gF1,
    float *__restrict__ gverts, float4 *__restrict__ gclip, float *__restrict__ glight) {
    const int lidx = blockIdx.y;
    const ViewConst &l = views[lidx];
    const int S = l.W;
    const long long plane = (long long)S * S;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < S * S;
    const int pp = in ? p : 0;
    const int i = pp % S, j = pp / S;
    const unsigned long long *kv = keys + l.pix_off;
    const unsigned long long ks = kv[pp];
    const float *f0a = F0 + l.map_off, *f0b = F0 + l.map_off + plane;
    const float *ga = gF1 + l.map_off, *gbp = gF1 + l.map_off + plane;
    float g0 = in ? ga[pp] : 0.f, g1 = in ? gbp[pp] : 0.f;
    if (in && l.antialias) {
        const float gs0 = g0, gs1 = g1;
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
        for (int d = 0; d < 4; ++d) {
            const int in_ = i + di[d], jn = j + dj[d];
            if (in_ < 0 || in_ >= S || jn < 0 || jn >= S) continue;
            const int q = jn * S + in_;
            const unsigned long long kn = kv[q];
            if ((unsigned)kn == (unsigned)ks) continue;
            bool self_front;
            AAPair pr;
            if (!aa_eval<true>(l, setup, faces, adj, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
            const bool self_recv = (pr.recv == 1) != self_front;
            if (self_recv) {
                g0 -= pr.w * gs0;
                g1 -= pr.w * gs1;
                double galpha = (double)gs0 * (f0a[q] - f0a[pp]) + (double)gs1 * (f0b[q] - f0b[pp]);
                galpha *= pr.recv == 1 ? 1.0 : -1.0;
                float4 *gpa = gclip + l.clip_off + pr.va;
                float4 *gpb = gclip + l.clip_off + pr.vb;
                atomic_add_f32(&gpa->x, (float)(galpha * pr.dax));
                atomic_add_f32(&gpa->y, (float)(galpha * pr.day));
                atomic_add_f32(&gpa->w, (float)(galpha * pr.daw));
                atomic_add_f32(&gpb->x, (float)(galpha * pr.dbx));
                atomic_add_f32(&gpb->y, (float)(galpha * pr.dby));
                atomic_add_f32(&gpb->w, (float)(galpha * pr.dbw));
            } else {
                g0 += pr.w * ga[q];
                g1 += pr.w * gbp[q];
            }
        }
    }
    // resolve^T: F0 = (z, z^2), z = d(x) / far
    const bool active = in && ks != kBgKey && (g0 != 0.f || g1 != 0.f);
    const int tri = active ? (int)(unsigned)ks : 0;
    const int *f = faces + 3 * (size_t)(l.face_off + tri);
    float4 c0 = make_float4(1, 0, 0, 1), c1 = make_float4(0, 1, 0, 1), c2 = make_float4(0, 0, 0, 1);
    float v0[3] = {0, 0, 0}, v1[3] = {1, 0, 0}, v2[3] = {0, 1, 0};
    if (active) {
        c0 = clip[l.clip_off + f[0]]; c1 = clip[l.clip_off + f[1]]; c2 = clip[l.clip_off + f[2]];
        for (int k = 0; k < 3; ++k) {
            v0[k] = verts[3 * (size_t)(l.vert_off + f[0]) + k];
            v1[k] = verts[3 * (size_t)(l.vert_off + f[1]) + k];
            v2[k] = verts[3 * (size_t)(l.vert_off + f[2]) + k];
        }
    }
    const float px = ndc_c(i, S), py = -ndc_c(j, S);
    const BaryFull b = bary_full(c0, c1, c2, px, py);
    const float x = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
    const float y = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
    const float z = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
    const float zval = active ? f0a[pp] : 0.f;
    const float gz = active ? g0 + 2.f * zval * g1 : 0.f;
    const float gdepth = gz / l.zfar;
    float gx[3], gl[6];
    if (l.kind == kDirectional) {
        gx[0] = gdepth * l.dir[0]; gx[1] = gdepth * l.dir[1]; gx[2] = gdepth * l.dir[2];
        gl[0] = -gx[0]; gl[1] = -gx[1]; gl[2] = -gx[2];
        gl[3] = gdepth * (x - l.pos[0]); gl[4] = gdepth * (y - l.pos[1]); gl[5] = gdepth * (z - l.pos[2]);
    } else {
        const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
        const float dl = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
        const float inv = active ? gdepth / dl : 0.f;
        gx[0] = ddx * inv; gx[1] = ddy * inv; gx[2] = ddz * inv;
        gl[0] = -gx[0]; gl[1] = -gx[1]; gl[2] = -gx[2];
        gl[3] = gl[4] = gl[5] = 0.f;
    }
    wave_add(gl, glight + 24 * lidx + 16);
    float gv[9];
    for (int k = 0; k < 3; ++k) {
        gv[k] = b.b0 * gx[k];
        gv[3 + k] = b.b1 * gx[k];
        gv[6 + k] = b.b2 * gx[k];
    }
    const float gb0 = (gx[0] * v0[0] + gx[1] * v0[1]) + gx[2] * v0[2];
    const float gb1 = (gx[0] * v1[0] + gx[1] * v1[1]) + gx[2] * v1[2];
    const float gb2 = (gx[0] * v2[0] + gx[1] * v2[1]) + gx[2] * v2[2];
    float gc[9];
    bary_backward(b, px, py, gb0, gb1, gb2, gc);
    const int vo = l.vert_off, co = l.clip_off, fo = l.face_off;
    scatter_by_key(active, tri, gv, [&](int k, int e) {
        return gverts + 3 * (size_t)(vo + faces[3 * (size_t)(fo + k) + e / 3]) + (e % 3);
    });
    scatter_by_key(active, tri, gc, [&](int k, int e) {
        float4 *t = gclip + co + faces[3 * (size_t)(fo + k) + e / 3];
        const int comp = e % 3;
        return comp == 0 ? &t->x : (comp == 1 ? &t->y : &t->w);
    });
}

// ----------------------------------------------------------------------------- transform^T

__global__ __launch_bounds__(256) void transform_backward_kernel(const ViewConst *__restrict__ views, int L,
                                                                 const float *__restrict__ verts,
                                                                 const float4 *__restrict__ gclip,
                                                                 float *__restrict__ gverts,
                                                                 float *__restrict__ glight) {
    const int view = blockIdx.y;
    const ViewConst &v = views[view];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < v.nverts;
    const float4 g = in ? gclip[v.clip_off + i] : make_float4(0, 0, 0, 0);
    const float *M = v.M;
    if (in && (g.x != 0.f || g.y != 0.f || g.w != 0.f)) {
        float *dst = gverts + 3 * (size_t)(v.vert_off + i);
        for (int k = 0; k < 3; ++k) atomic_add_f32(dst + k, (M[k] * g.x + M[4 + k] * g.y) + M[12 + k] * g.w);
    }
    if (view < L) {
        float xh[4] = {0, 0, 0, 0};
        if (in) {
            const float *p = verts + 3 * (size_t)(v.vert_off + i);
            xh[0] = p[0]; xh[1] = p[1]; xh[2] = p[2]; xh[3] = 1.f;
        }
        float gm[16];
        for (int k = 0; k < 4; ++k) {
            gm[k] = g.x * xh[k];
            gm[4 + k] = g.y * xh[k];
            gm[8 + k] = 0.f;
            gm[12 + k] = g.w * xh[k];
        }
        // one atomic set per workgroup: wave sums then LDS
        __shared__ float part[4][16];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        for (int k = 0; k < 16; ++k) {
            const float s = wave_sum(gm[k]);
            if (lane == 0) part[wid][k] = s;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            const float s = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
            atomic_add_f32(glight + 24 * view + threadIdx.x, s);
        }
    }
}

// ----------------------------------------------------------------------------- pose

__host__ __device__ inline Dual3 dsin(const Dual3 &a) {
    const double s = sin(a.v), c = cos(a.v);
    return Dual3{s, {c * a.d[0], c * a.d[1], c * a.d[2]}};
}
__host__ __device__ inline Dual3 dcos(const Dual3 &a) {
    const double s = sin(a.v), c = cos(a.v);
    return Dual3{c, {-s * a.d[0], -s * a.d[1], -s * a.d[2]}};
}
__host__ __device__ inline double dsin(double a) { return sin(a); }
__host__ __device__ inline double dcos(double a) { return cos(a); }

// Rotation matrix of an axis-angle vector (Rodrigues): I + sin(t)/t K + (1-cos t)/t^2 K^2.
template <class T>
__device__ inline void rodrigues(const T r[3], T Rm[9]) {
    const T th2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    const T zero = mkT<T>(0.0);
    const T K[9] = {zero, -r[2], r[1], r[2], zero, -r[0], -r[1], r[0], zero};
    T K2[9];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            T s = zero;
            for (int k = 0; k < 3; ++k) s = s + K[3 * a + k] * K[3 * k + c];
            K2[3 * a + c] = s;
        }
    const bool small = val(th2) < 1e-24;
    for (int k = 0; k < 9; ++k) Rm[k] = K[k];
    if (!small) {
        const T th = dsqrt(th2);
        const T A = dsin(th) / th;
        const T Bc = (mkT<T>(1.0) - dcos(th)) / th2;
        for (int k = 0; k < 9; ++k) Rm[k] = A * K[k] + Bc * K2[k];
    }
    Rm[0] = Rm[0] + mkT<T>(1.0);
    Rm[4] = Rm[4] + mkT<T>(1.0);
    Rm[8] = Rm[8] + mkT<T>(1.0);
}

__global__ void pose_kernel(const int *__restrict__ vert_off, const int *__restrict__ pose_counts,
                            const float *__restrict__ centers, const float *__restrict__ local,
                            const float *__restrict__ poses, float *__restrict__ world) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nv = vert_off[b + 1] - vert_off[b];
    if (i >= nv) return;
    const size_t gi = (size_t)(vert_off[b] + i);
    const float *src = local + 3 * gi;
    float *dst = world + 3 * gi;
    if (i >= pose_counts[b]) {
        dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2];
        return;
    }
    const double r[3] = {poses[6 * b], poses[6 * b + 1], poses[6 * b + 2]};
    double Rm[9];
    rodrigues<double>(r, Rm);
    for (int a = 0; a < 3; ++a) {
        const double acc = ((Rm[3 * a] * src[0] + Rm[3 * a + 1] * src[1]) + Rm[3 * a + 2] * src[2]) +
                           (double)centers[3 * b + a] + (double)poses[6 * b + 3 + a];
        dst[a] = (float)acc;
    }
}

__global__ __launch_bounds__(256) void pose_backward_kernel(const int *__restrict__ vert_off,
                                                            const int *__restrict__ pose_counts,
                                                            const float *__restrict__ local,
                                                            const float *__restrict__ poses,
                                                            const float *__restrict__ gworld,
                                                            float *__restrict__ gposes) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x * blockDim.x >= (unsigned)pose_counts[b]) return;     // whole workgroup idle
    const bool in = i < pose_counts[b];
    Dual3 r[3];
    for (int k = 0; k < 3; ++k) {
        r[k].v = poses[6 * b + k];
        for (int q = 0; q < 3; ++q) r[k].d[q] = k == q ? 1.0 : 0.0;
    }
    Dual3 Rm[9];
    rodrigues<Dual3>(r, Rm);
    float out[6] = {0, 0, 0, 0, 0, 0};
    if (in) {
        const size_t gi = (size_t)(vert_off[b] + i);
        const float *v = local + 3 * gi;
        const float *g = gworld + 3 * gi;
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int a = 0; a < 3; ++a)
                acc += g[a] * ((Rm[3 * a].d[q] * v[0] + Rm[3 * a + 1].d[q] * v[1]) + Rm[3 * a + 2].d[q] * v[2]);
            out[q] = (float)acc;
        }
        out[3] = g[0]; out[4] = g[1]; out[5] = g[2];
    }
    __shared__ float part[4][6];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 6; ++k) {
        const float s = wave_sum(out[k]);
        if (lane == 0) part[wid][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const float s = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
        atomic_add_f32(gposes + 6 * b + threadIdx.x, s);
    }
}

// ----------------------------------------------------------------------------- launchers

hipError_t launch_aa_camera_backward(const ViewConst *views, const RenderConst *renders, int R, int max_pix,
                                     const TriSetup *setup, const int *faces, const int *adj, const float *verts,
                                     const unsigned long long *keys, const float *img0, const float *gimg,
                                     float *gimg0, float4 *gclip, int C, hipStream_t s) {
    if (R == 0) return hipSuccess;
    hipLaunchKernelGGL(aa_camera_backward_kernel, dim3((max_pix + 255) / 256, R), dim3(256), 0, s, views, renders,
                       setup, faces, adj, verts, keys, img0, gimg, gimg0, gclip, C);
    return hipGetLastError();
}

hipError_t launch_lookup_backward(const ViewConst *views, const RenderConst *renders, int R, int max_pix,
                                  const int *render_lights, const int *faces, const float *verts,
                                  const float *albedo, const float4 *clip, const unsigned long long *keys,
                                  const float *maps, const float *gimg0, float *gmaps, float *gverts,
                                  float4 *gclip, float *glight, float *galbedo, int C, hipStream_t s) {
    if (R == 0) return hipSuccess;
    hipLaunchKernelGGL(lookup_backward_kernel, dim3((max_pix + 255) / 256, R), dim3(256), 0, s, views, renders,
                       render_lights, faces, verts, albedo, clip, keys, maps, gimg0, gmaps, gverts, gclip, glight,
                       galbedo, C);
    return hipGetLastError();
}

hipError_t launch_light_backward(const ViewConst *views, int L, int max_texels, const TriSetup *setup,
                                 const int *faces, const int *adj, const float *verts, const float4 *clip,
                                 const unsigned long long *keys, const float *F0, const float *gF1, float *gverts,
                                 float4 *gclip, float *glight, hipStream_t s) {
    if (L == 0) return hipSuccess;
    hipLaunchKernelGGL(light_backward_kernel, dim3((max_texels + 255) / 256, L), dim3(256), 0, s, views, setup,
                       faces, adj, verts, clip, keys, F0, gF1, gverts, gclip, glight);
    return hipGetLastError();
}

hipError_t launch_transform_backward(const ViewConst *views, int nviews, int L, int max_verts, const float *verts,
                                     const float4 *gclip, float *gverts, float *glight, hipStream_t s) {
    if (nviews == 0 || max_verts == 0) return hipSuccess;
    hipLaunchKernelGGL(transform_backward_kernel, dim3((max_verts + 255) / 256, nviews), dim3(256), 0, s, views, L,
                       verts, gclip, gverts, glight);
    return hipGetLastError();
}

hipError_t launch_pose(const int *scene_vert_off, const int *pose_counts, const float *pose_centers, int B,
                       int max_verts, const float *local, const float *poses, float *world, hipStream_t s) {
    hipLaunchKernelGGL(pose_kernel, dim3((max_verts + 255) / 256, B), dim3(256), 0, s, scene_vert_off, pose_counts,
                       pose_centers, local, poses, world);
    return hipGetLastError();
}

hipError_t launch_pose_backward(const int *scene_vert_off, const int *pose_counts, int B, int max_verts,
                                const float *local, const float *poses, const float *gworld, float *gposes,
                                hipStream_t s) {
    hipLaunchKernelGGL(pose_backward_kernel, dim3((max_verts + 255) / 256, B), dim3(256), 0, s, scene_vert_off,
                       pose_counts, local, poses, gworld, gposes);
    return hipGetLastError();
}

}  // namespace dsm
