// Forward shading kernels: moment resolve of the light views, edge smoothing
// (light maps and camera images), and the deferred Chebyshev + Lambert pass.
//
// Moment resolve (Alg. 1, RenderScene): for each shadow-map texel the world
// point x on the nearest triangle is recovered from perspective-correct
// barycentrics (the point of the triangle that projects to the texel
// centre), its distance d(x) to the light (Sec. 3: Euclidean for point and
// spot lights, from a plane outside the scene for directional lights) is
// normalized, z = d / far, and (z, z^2) is written; texels without a triangle
// hold the far value (1, 1).
//
// Lookup (Alg. 2, ComputeVisibility, and Lambert shading summed over lights):
// per camera pixel the world point x and face normal n are recovered the same
// way; per light u = L(x), (m1, m2) is fetched bilinearly (clamp-to-edge),
// sigma^2 = max(m2 - m1^2, min_variance), v = 1 if z <= m1 else
// sigma^2 / (sigma^2 + (z - m1)^2) (one-sided Chebyshev, Sec. 3); points outside
// the light frustum count as lit; colour = albedo * sum_l max(0, n.omega_l)
// v_l I_l cone_l.
#include "aa.h"
#include "dsm_internal.h"

namespace dsm {

// Pixels per thread of the lookup (latency hiding; see lookup_kernel).
constexpr int kLookupPixelsPerThread = 2;

struct Bary {
    float b0, b1, b2;
};

// Barycentrics of the point of triangle (c0, c1, c2) that projects to NDC
// (px, py): sum b_i (x_i - px w_i) = 0, sum b_i (y_i - py w_i) = 0, sum b_i = 1,
// through the hardware reciprocal of the sum (about one ulp; the resolve, the
// lookup and their adjoints all form them this way).
__device__ __forceinline__ Bary persp_bary_rcp(float4 c0, float4 c1, float4 c2, float px, float py) {
    const float a0x = c0.x - px * c0.w, a0y = c0.y - py * c0.w;
    const float a1x = c1.x - px * c1.w, a1y = c1.y - py * c1.w;
    const float a2x = c2.x - px * c2.w, a2y = c2.y - py * c2.w;
    const float k0 = a1x * a2y - a1y * a2x;
    const float k1 = a2x * a0y - a2y * a0x;
    const float k2 = a0x * a1y - a0y * a1x;
    const float rs = __builtin_amdgcn_rcpf(k0 + k1 + k2);
    return Bary{k0 * rs, k1 * rs, k2 * rs};
}

// The resolve and the lookup form their quotients through the hardware
// reciprocal (about 1 ulp), where the raster setup, whose coverage and depth
// keys are integer results, keeps the correctly rounded division.  The
// lookup's adjoint forms every value with the same expressions (the map
// position, which picks the bilinear cell and the inside test, among them),
// so the two passes take the same decisions.
__device__ __forceinline__ float ndc_centre(int i, int n) {
    return (float)(2 * i + 1) * __builtin_amdgcn_rcpf((float)n) - 1.0f;
}

__device__ __forceinline__ float light_depth(const ViewConst &l, float x, float y, float z) {
    float d;
    if (l.kind == kDirectional) {
        d = ((x - l.pos[0]) * l.dir[0] + (y - l.pos[1]) * l.dir[1]) + (z - l.pos[2]) * l.dir[2];
    } else {
        const float dx = x - l.pos[0], dy = y - l.pos[1], dz = z - l.pos[2];
        d = sqrtf((dx * dx + dy * dy) + dz * dz);
    }
    return d * __builtin_amdgcn_rcpf(l.zfar) - l.zc;
}

// ----------------------------------------------------------------------------- resolve

// Texels per thread of the resolve (256 apart): their keys, then their face
// records, in flight together (the chain key -> record -> store is the
// kernel's latency; 80 -> 62 -> 55 us for 1, 2, 4 on 64 512^2 maps).
constexpr int kResolvePerThread = 4;

__global__ __launch_bounds__(256) void resolve_kernel(const ViewConst *__restrict__ views,
                                                      const TriVerts *__restrict__ tv,
                                                      const unsigned long long *__restrict__ keys,
                                                      float *__restrict__ F0) {
    constexpr int PPT = kResolvePerThread;
    const ViewConst &l = views[blockIdx.y];
    const int S = l.W, P = S * S;
    const int t0 = blockIdx.x * (256 * PPT) + (int)threadIdx.x;
    if (t0 >= P) return;
    unsigned long long key[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int t = t0 + 256 * k;
        key[k] = t < P ? keys[l.pix_off + t] : kBgKey;
    }
    TriVerts r[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (key[k] != kBgKey) r[k] = tv[l.face_off + (int)(unsigned)key[k]];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int t = t0 + 256 * k;
        if (t >= P) break;
        float z = 1.0f - l.zc;          // background: the far plane
        if (key[k] != kBgKey) {
            const float v0[3] = {r[k].a.x, r[k].a.y, r[k].a.z}, v1[3] = {r[k].a.w, r[k].b.x, r[k].b.y},
                        v2[3] = {r[k].b.z, r[k].b.w, r[k].c.x};
            const int i = t % S, j = t / S;
            const float px = ndc_centre(i, S), py = -ndc_centre(j, S);
            const float4 c0 = clip_of(l.M, v0[0], v0[1], v0[2]), c1 = clip_of(l.M, v1[0], v1[1], v1[2]),
                         c2 = clip_of(l.M, v2[0], v2[1], v2[2]);
            const Bary b = persp_bary_rcp(c0, c1, c2, px, py);
            const float x = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
            const float y = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
            const float zz = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
            z = light_depth(l, x, y, zz);
        }
        if (l.warp_c > 0.f) z = expf(l.warp_c * z);     // exponential maps
        F0[l.map_off + t] = z;
        F0[l.map_off + (long long)P + t] = z * z;
    }
}

// ----------------------------------------------------------------------------- smoothing forward

// Light maps: planar 2-channel; grid.y = light view.  Camera images:
// interleaved C channels; grid.y = render (view = that render's camera).
// C is a template parameter so that the per-channel values stay in registers.
//
// Light maps: two passes.  A sample changes only through a pair whose front
// triangle has a silhouette edge (a candidate, AANeighbours), which is rare
// in a shadow map, while testing a candidate waits for three more dependent
// loads (the triangle's record, then its vertices).  The first pass therefore copies every
// sample without candidates and lists the others (AaList, one atomic per
// wave on one of many counters); the second pass evaluates only the listed
// samples, so no wave of the first waits for them.

// The smoothed value of sample p (all of its candidate pairs evaluated).
template <bool LIGHT, int C>
__device__ __forceinline__ void aa_forward_sample(const ViewConst &v, long long base, const TriSetup *__restrict__ setup,
                                                  const int *__restrict__ faces, const unsigned char *__restrict__ silm,
                                                  const float *__restrict__ verts,
                                                  const unsigned long long *__restrict__ kv,
                                                  const float *__restrict__ src, float *__restrict__ dst, int p) {
    const int W = v.W;
    const long long cstride = LIGHT ? (long long)W * v.H : 1;
    const int pstride = LIGHT ? 1 : C;
    const int i = p % W, j = p / W;
    const unsigned long long ks = kv[p];
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) acc[c] = src[base + (long long)p * pstride + c * cstride];
    const float self[3] = {acc[0], acc[1], acc[2]};
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    const AANeighbours nb = aa_neighbours(v, kv, silm, ks, i, j);
    // values of the candidate neighbours, fetched before the pair tests
    // so that they arrive with the triangle records
    float nv[4][3];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            nv[d][c] = (nb.cand[d] && c < C) ? src[base + (long long)nb.q[d] * pstride + c * cstride] : 0.f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (!nb.cand[d]) continue;
        const int in_ = i + di[d], jn = j + dj[d];
        const unsigned long long kn = nb.kn[d];
        bool self_front;
        AAPair pr;
        if (!aa_eval<false>(v, setup, faces, silm, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
        const bool self_recv = (pr.recv == 1) != self_front;   // receiver: other when recv==1
        if (!self_recv) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c < C) acc[c] += pr.w * (nv[d][c] - self[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) dst[base + (long long)p * pstride + c * cstride] = acc[c];
}

// First pass: copy samples without candidates, list the others.  Each
// thread takes kAaFirstPassPerThread samples 256 apart, with all of their
// neighbour keys in flight together and one wave vote on whether any
// silhouette byte is needed; list segments are assigned per 256-sample
// chunk (chunk index gxv * row + column), as if each chunk were a
// workgroup, so the list sizing does not depend on it.  Samples run in row
// order: this pass streams, and has no candidate tests to concentrate.
constexpr int kAaFirstPassPerThread = 2;

template <bool LIGHT, int C>
__global__ __launch_bounds__(256) void aa_forward_kernel(const ViewConst *__restrict__ views,
                                                         const RenderConst *__restrict__ renders,
                                                         const unsigned char *__restrict__ silm,
                                                         const unsigned long long *__restrict__ keys,
                                                         const float *__restrict__ src, float *__restrict__ dst,
                                                         AaList list, unsigned char *__restrict__ flag, int gxv) {
    constexpr int PPT = kAaFirstPassPerThread;
    const Blk blk = xcd_block2();
    const ViewConst &v = LIGHT ? views[blk.y] : views[renders[blk.y].camera_view];
    const int W = v.W, H = v.H, P = W * H;
    const int p0 = blk.x * (256 * PPT) + (int)threadIdx.x;
    if (p0 >= P) return;
    int ps[PPT];
    bool live[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        ps[k] = p0 + 256 * k;
        live[k] = ps[k] < P;
    }
    const long long base = LIGHT ? v.map_off : renders[blk.y].img_off;
    const long long cstride = LIGHT ? (long long)P : 1;
    const int pstride = LIGHT ? 1 : C;
    const unsigned long long *kv = keys + v.pix_off;
    float val[PPT][3];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = ps[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) val[k][c] = (live[k] && c < C) ? src[base + (long long)p * pstride + c * cstride] : 0.f;
    }
    bool cand[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) cand[k] = false;
    if (v.antialias && v.nfaces > 0) {
        // every neighbour key of every sample first, then the differing pairs
        unsigned long long ks[PPT], kn[PPT][4];
        bool differ[PPT][4];
        bool any = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = live[k] ? ps[k] : ps[0];
            const int i = p % W, j = p / W;
            ks[k] = kv[p];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int in_ = i + (d == 0 ? -1 : d == 1 ? 1 : 0), jn = j + (d == 2 ? -1 : d == 3 ? 1 : 0);
                const bool inb = in_ >= 0 && in_ < W && jn >= 0 && jn < H;
                kn[k][d] = kv[inb ? jn * W + in_ : p];
                differ[k][d] = inb;
            }
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                differ[k][d] = live[k] && differ[k][d] && (unsigned)kn[k][d] != (unsigned)ks[k];
                any = any || differ[k][d];
            }
        if (__ballot(any) != 0ull) {
#pragma unroll
            for (int k = 0; k < PPT; ++k)
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const unsigned front = ks[k] < kn[k][d] ? (unsigned)ks[k] : (unsigned)kn[k][d];
                    const unsigned char sil = differ[k][d] ? silm[v.setup_off + front] : (unsigned char)0;
                    cand[k] = cand[k] || (differ[k][d] && sil != 0);
                }
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = ps[k];
        if (live[k]) flag[v.pix_off + p] = cand[k] ? 1 : 0;
        wave_append(cand[k], make_uint2((unsigned)blk.y, (unsigned)p), list,
                    (long long)blk.y * gxv + (long long)blk.x * PPT + k);
        if (live[k] && !cand[k]) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (c < C) dst[base + (long long)p * pstride + c * cstride] = val[k][c];
        }
    }
}

// One pass over every sample (camera images: their candidates are too
// frequent for a second pass to pay off).
template <bool LIGHT, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void aa_forward_direct_kernel(const ViewConst *__restrict__ views, const RenderConst *__restrict__ renders,
                                  const TriSetup *__restrict__ setup, const int *__restrict__ faces,
                                  const unsigned char *__restrict__ silm, const float *__restrict__ verts,
                                  const unsigned long long *__restrict__ keys, const float *__restrict__ src,
                                  float *__restrict__ dst,
                                  unsigned char *__restrict__ flag) {
    const Blk blk = xcd_block2();
    const ViewConst &v = LIGHT ? views[blk.y] : views[renders[blk.y].camera_view];
    const int W = v.W, H = v.H;
    const int p = aa_sample_index(blk.x, (int)threadIdx.x, W, H);
    if (blk.x * 256 >= W * H || p >= W * H) return;
    const long long base = LIGHT ? v.map_off : renders[blk.y].img_off;
    const long long cstride = LIGHT ? (long long)W * H : 1;
    const int pstride = LIGHT ? 1 : C;
    const int i = p % W, j = p / W;
    const unsigned long long *kv = keys + v.pix_off;
    const unsigned long long ks = kv[p];
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) acc[c] = src[base + (long long)p * pstride + c * cstride];
    const float self[3] = {acc[0], acc[1], acc[2]};
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    bool any = false;
    if (v.antialias && v.nfaces > 0) {
        const AANeighbours nb = aa_neighbours(v, kv, silm, ks, i, j);
        any = nb.cand[0] || nb.cand[1] || nb.cand[2] || nb.cand[3];
        // values of the candidate neighbours, fetched before the pair tests
        // so that they arrive with the triangle records
        float nv[4][3];
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                nv[d][c] = (nb.cand[d] && c < C) ? src[base + (long long)nb.q[d] * pstride + c * cstride] : 0.f;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (!nb.cand[d]) continue;
            const int in_ = i + di[d], jn = j + dj[d];
            const unsigned long long kn = nb.kn[d];
            bool self_front;
            AAPair pr;
            if (!aa_eval<false>(v, setup, faces, silm, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
            const bool self_recv = (pr.recv == 1) != self_front;   // receiver: other when recv==1
            if (!self_recv) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (c < C) acc[c] += pr.w * (nv[d][c] - self[c]);
        }
    }
    flag[v.pix_off + p] = any ? 1 : 0;      // for the adjoint: this sample has candidate pairs
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) dst[base + (long long)p * pstride + c * cstride] = acc[c];
}

// Second pass: one workgroup per list segment.
template <bool LIGHT, int C>
__global__ __launch_bounds__(256) void aa_forward_list_kernel(
    const ViewConst *__restrict__ views, const RenderConst *__restrict__ renders, const TriSetup *__restrict__ setup,
    const int *__restrict__ faces, const unsigned char *__restrict__ silm, const float *__restrict__ verts,
    const unsigned long long *__restrict__ keys, const float *__restrict__ src, float *__restrict__ dst,
    AaList list) {
    const unsigned seg = blockIdx.x, n = list.counts[seg];
    for (unsigned e = threadIdx.x; e < n; e += blockDim.x) {
        const uint2 it = list.items[(size_t)seg * list.segcap + e];
        const ViewConst &v = LIGHT ? views[it.x] : views[renders[it.x].camera_view];
        const long long base = LIGHT ? v.map_off : renders[it.x].img_off;
        aa_forward_sample<LIGHT, C>(v, base, setup, faces, silm, verts, keys + v.pix_off, src, dst, (int)it.y);
    }
}

// ----------------------------------------------------------------------------- lookup + shade

// PPT pixels per thread, PPT * 256 contiguous pixels per workgroup (pixel
// k of a thread at k * 256 + its lane, so every load stays coalesced).  The
// three dependent gathers of a pixel (its depth|id key, its triangle's
// record, its map taps) are issued for all PPT pixels before any of them is
// used, so a thread waits for three round trips per PPT pixels instead of
// three per pixel.  Each pixel's arithmetic is the one-pixel form, unchanged.
template <int PPT>
__global__ __launch_bounds__(256) void lookup_kernel(const ViewConst *__restrict__ views,
                                                     const RenderConst *__restrict__ renders,
                                                     const int *__restrict__ render_lights,
                                                     const TriVerts *__restrict__ tv, const float *__restrict__ albedo,
                                                     const unsigned long long *__restrict__ keys,
                                                     const float *__restrict__ maps, float *__restrict__ img0, int C) {
    const RenderConst &R = renders[blockIdx.y];
    const ViewConst &cv = views[R.camera_view];
    const int W = cv.W, H = cv.H, P = W * H;
    const int p0 = blockIdx.x * (256 * PPT) + (int)threadIdx.x;
    if (p0 >= P) return;
    unsigned long long key[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = p0 + 256 * k;
        key[k] = p < P ? keys[cv.pix_off + p] : kBgKey;
    }
    TriVerts r[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (key[k] != kBgKey) r[k] = tv[cv.face_off + (int)(unsigned)key[k]];
    float x[PPT], y[PPT], z[PPT], nx[PPT], ny[PPT], nz[PPT], shade[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        shade[k] = 0.f;
        x[k] = y[k] = z[k] = nx[k] = ny[k] = nz[k] = 0.f;
        if (key[k] == kBgKey) continue;
        const float v0[3] = {r[k].a.x, r[k].a.y, r[k].a.z}, v1[3] = {r[k].a.w, r[k].b.x, r[k].b.y},
                    v2[3] = {r[k].b.z, r[k].b.w, r[k].c.x};
        const int p = p0 + 256 * k;
        const int i = p % W, j = p / W;
        const float px = ndc_centre(i, W), py = -ndc_centre(j, H);
        const float4 c0 = clip_of(cv.M, v0[0], v0[1], v0[2]), c1 = clip_of(cv.M, v1[0], v1[1], v1[2]),
                     c2 = clip_of(cv.M, v2[0], v2[1], v2[2]);
        const Bary b = persp_bary_rcp(c0, c1, c2, px, py);
        x[k] = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
        y[k] = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
        z[k] = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
        const float e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e1z = v1[2] - v0[2];
        const float e2x = v2[0] - v0[0], e2y = v2[1] - v0[1], e2z = v2[2] - v0[2];
        float cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
        const float rn = __builtin_amdgcn_rsqf((cx * cx + cy * cy) + cz * cz);
        nx[k] = cx * rn;
        ny[k] = cy * rn;
        nz[k] = cz * rn;
    }
    for (int q = 0; q < R.light_count; ++q) {
        const ViewConst &l = views[render_lights[R.light_begin + q]];
        const int S = l.W, Sp = S + 2 * l.fpad;
        const float2 *mm = (const float2 *)(maps + l.fmap_off);     // (m1, m2) interleaved per texel
        bool inside[PPT];
        float fx[PPT], fy[PPT];
        int o00[PPT], o01[PPT], o10[PPT], o11[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            inside[k] = false;
            fx[k] = fy[k] = 0.f;
            o00[k] = o01[k] = o10[k] = o11[k] = 0;
            if (key[k] == kBgKey) continue;
            // a cube face lights only the directions it owns: no fetch elsewhere
            if (l.kind == kCubeFace &&
                cube_face_of(x[k] - l.pos[0], y[k] - l.pos[1], z[k] - l.pos[2]) != l.cube_face)
                continue;
            const float *M = l.M;
            const float cx = ((M[0] * x[k] + M[1] * y[k]) + M[2] * z[k]) + M[3];
            const float cy = ((M[4] * x[k] + M[5] * y[k]) + M[6] * z[k]) + M[7];
            const float cw = ((M[12] * x[k] + M[13] * y[k]) + M[14] * z[k]) + M[15];
            const float rcw = __builtin_amdgcn_rcpf(cw);
            const float ux = cx * rcw, uy = cy * rcw;
            inside[k] = cw > 0.f && fabsf(ux) <= 1.f && fabsf(uy) <= 1.f;
            if (!inside[k]) continue;
            const float sx = (ux + 1.f) * (0.5f * S) - 0.5f;
            const float sy = (1.f - uy) * (0.5f * S) - 0.5f;
            const float fx0 = floorf(sx), fy0 = floorf(sy);
            fx[k] = sx - fx0;
            fy[k] = sy - fy0;
            const int ix = (int)fx0 + l.fpad, iy = (int)fy0 + l.fpad;
            const int x0 = min(max(ix, 0), Sp - 1), x1 = min(max(ix + 1, 0), Sp - 1);
            const int y0 = min(max(iy, 0), Sp - 1), y1 = min(max(iy + 1, 0), Sp - 1);
            o00[k] = y0 * Sp + x0; o01[k] = y0 * Sp + x1;
            o10[k] = y1 * Sp + x0; o11[k] = y1 * Sp + x1;
        }
        float2 t00[PPT], t01[PPT], t10[PPT], t11[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            // offsets of pixels without a fetch are 0, a texel of this map
            t00[k] = mm[o00[k]]; t01[k] = mm[o01[k]]; t10[k] = mm[o10[k]]; t11[k] = mm[o11[k]];
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (key[k] == kBgKey) continue;
            if (l.kind == kCubeFace &&
                cube_face_of(x[k] - l.pos[0], y[k] - l.pos[1], z[k] - l.pos[2]) != l.cube_face)
                continue;
            float vis = 1.f;
            if (inside[k]) {
                const float w00 = (1.f - fx[k]) * (1.f - fy[k]), w01 = fx[k] * (1.f - fy[k]);
                const float w10 = (1.f - fx[k]) * fy[k], w11 = fx[k] * fy[k];
                const float m1 = ((w00 * t00[k].x + w01 * t01[k].x) + w10 * t10[k].x) + w11 * t11[k].x;
                const float m2 = ((w00 * t00[k].y + w01 * t01[k].y) + w10 * t10[k].y) + w11 * t11[k].y;
                float zw, floor_v;
                warp_receiver(l, light_depth(l, x[k], y[k], z[k]), zw, floor_v);
                const float var = fmaxf(m2 - m1 * m1, floor_v);
                const float dd = zw - m1;
                vis = bleed_reduce(l, (zw <= m1) ? 1.f : var * __builtin_amdgcn_rcpf(var + dd * dd));
            }
            float ox, oy, oz;
            if (l.kind == kDirectional) {
                ox = -l.dir[0];
                oy = -l.dir[1];
                oz = -l.dir[2];
            } else {
                ox = l.pos[0] - x[k];
                oy = l.pos[1] - y[k];
                oz = l.pos[2] - z[k];
                const float ron = __builtin_amdgcn_rsqf((ox * ox + oy * oy) + oz * oz);
                ox *= ron;
                oy *= ron;
                oz *= ron;
            }
            const float lam = fmaxf((nx[k] * ox + ny[k] * oy) + nz[k] * oz, 0.f);
            float cone = 1.f;
            if (l.kind == kSpot) {
                // cos of the angle between x - p and the axis: (-omega) . axis
                const float ca = -((ox * l.dir[0] + oy * l.dir[1]) + oz * l.dir[2]);
                cone = ca >= l.cos_half ? 1.f : 0.f;
            }
            shade[k] += lam * vis * l.intensity * cone;
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = p0 + 256 * k;
        if (p >= P) continue;
        float *out = img0 + R.img_off + (long long)p * C;
        const float rho[3] = {r[k].c.y, r[k].c.z, r[k].c.w};    // albedo, carried in the face record
        for (int c = 0; c < C; ++c) out[c] = key[k] == kBgKey ? 0.f : rho[c] * shade[k];
    }
}

// ----------------------------------------------------------------------------- launchers

hipError_t launch_resolve(const ViewConst *views, int L, int max_texels, const TriVerts *tv,
                          const unsigned long long *keys, float *F0, hipStream_t s) {
    if (L == 0) return hipSuccess;
    hipLaunchKernelGGL(resolve_kernel, dim3((max_texels + 256 * kResolvePerThread - 1) / (256 * kResolvePerThread), L),
                       dim3(256), 0, s, views, tv, keys, F0);
    return hipGetLastError();
}

hipError_t launch_aa_forward(bool light, const ViewConst *views, const RenderConst *renders, int n, int max_pix,
                             const TriSetup *setup, const int *faces, const unsigned char *silm, const float *verts,
                             const unsigned long long *keys, const float *src, float *dst, int C, uint2 *list,
                             unsigned *counts, unsigned char *aa_flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 grid((max_pix + 255) / 256, n);
    const AaList l = aa_list_for(list, counts, (long long)grid.x * grid.y);
    constexpr int P1 = kAaFirstPassPerThread;
    const dim3 grid1((max_pix + 256 * P1 - 1) / (256 * P1), n);
#define DSM_AAF(LL, CC)                                                                                          \
    do {                                                                                                         \
        hipLaunchKernelGGL((aa_forward_kernel<LL, CC>), grid1, dim3(256), 0, s, views, renders, silm, keys, src, \
                           dst, l, aa_flag, (int)grid.x);                                                        \
        hipLaunchKernelGGL((aa_forward_list_kernel<LL, CC>), dim3(l.nseg), dim3(256), 0, s, views, renders,      \
                           setup, faces, silm, verts, keys, src, dst, l);                                        \
    } while (0)
    // light maps in two passes (a sample with candidate pairs is rare there); camera images in one
    if (light) {
        DSM_AAF(true, 2);
    } else if (C == 1) {
        hipLaunchKernelGGL((aa_forward_direct_kernel<false, 1>), grid, dim3(256), 0, s, views, renders, setup, faces,
                           silm, verts, keys, src, dst, aa_flag);
    } else {
        hipLaunchKernelGGL((aa_forward_direct_kernel<false, 3>), grid, dim3(256), 0, s, views, renders, setup, faces,
                           silm, verts, keys, src, dst, aa_flag);
    }
#undef DSM_AAF
    return hipGetLastError();
}

hipError_t launch_lookup(const ViewConst *views, const RenderConst *renders, int R, int max_pix,
                         const int *render_lights, const TriVerts *tv, const float *albedo,
                         const unsigned long long *keys, const float *maps, float *img0, int C, hipStream_t s) {
    if (R == 0) return hipSuccess;
    constexpr int PPT = kLookupPixelsPerThread;
    hipLaunchKernelGGL(lookup_kernel<PPT>, dim3((max_pix + 256 * PPT - 1) / (256 * PPT), R), dim3(256), 0, s, views,
                       renders, render_lights, tv, albedo, keys, maps, img0, C);
    return hipGetLastError();
}

}  // namespace dsm
