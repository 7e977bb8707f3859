// Rasterization of every view of a batch (light views into shadow maps, Eq. 1;
// camera views for deferred shading): vertex transform, fixed-point triangle
// setup, tile binning, and a tile rasterizer producing a 64-bit
// depth|triangle-id visibility buffer (the nearest surface per sample, ties
// to the lower triangle index).
//
// Coverage conventions (shared with no other code; stated here in full):
//  * clip = M [x,1] per row as ((m0*x + m1*y) + m2*z) + m3 in float32 (the
//    library is built without contraction, so no fused multiply-add);
//  * sx = (x/w + 1) * (W/2), sy = (1 - y/w) * (H/2); X = rint(256 sx),
//    Y = rint(256 sy); pixel (i,j) is sampled at (256 i + 128, 256 j + 128);
//  * a triangle is culled when a vertex has w <= 0, z/w < -1, or a screen
//    coordinate outside (-32768, 32768); it is re-oriented to positive doubled
//    area A (2nd and 3rd vertex swapped when A < 0), A == 0 is skipped;
//  * edge e is opposite vertex e, E_e = dx (py - ya) - dy (px - xa) for the
//    directed edge a -> b; a sample on an edge belongs to the triangle only
//    for top (dy == 0, dx > 0) or left (dy < 0) edges;
//  * z01 = 0.5 z/w + 0.5 per vertex, interpolated (z0 + b1 (z1-z0)) + b2 (z2-z0)
//    with b_e = f32(E_e) / f32(A); samples with z01 outside [0,1] are dropped;
//  * key = bits(z01) << 32 | local triangle index, minimum wins.
#include "dsm_internal.h"
#include "frames.h"

namespace dsm {

// ----------------------------------------------------------------------------- light frames

// The Jacobian of (M[16], pos[3], dir[3]) with respect to the three
// parameter components (forward-mode dual numbers), [22][3] per light: the
// reverse pass pulls every light-frame gradient back to the parameter as
// soon as it is formed.
__device__ void light_jacobian(const CamStatic &cam, const float *param, float *J) {
    Dual3 pd[3];
    for (int i = 0; i < 3; ++i) {
        pd[i].v = param[i];
        for (int j = 0; j < 3; ++j) pd[i].d[j] = (i == j) ? 1.0 : 0.0;
    }
    Dual3 Md[16], posd[3], dird[3];
    light_frame<Dual3>(cam, pd, Md, posd, dird);
    for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 16; ++i) J[3 * i + j] = (float)Md[i].d[j];
        for (int i = 0; i < 3; ++i) {
            J[3 * (16 + i) + j] = (float)posd[i].d[j];
            J[3 * (19 + i) + j] = (float)dird[i].d[j];
        }
    }
}

// One thread per light: the light camera from its float32 parameter, in
// float64, rounded to float32 for the rest of the pipeline; with jac, also
// the frame's Jacobian.  Workgroups from nf on clear the words z1[0, n1) and
// z2[0, n2) instead (the pass's counters and accumulators: one launch for
// all of it).
__global__ void light_frames_kernel(ViewConst *views, const CamStatic *cams, const float *params, int L,
                                    float *zc_out, float *jac, int nf, unsigned *z1, size_t n1, unsigned *z2,
                                    size_t n2) {
    if ((int)blockIdx.x >= nf) {
        const size_t stride = (size_t)(gridDim.x - nf) * blockDim.x;
        for (size_t i = (size_t)(blockIdx.x - nf) * blockDim.x + threadIdx.x; i < n1 + n2; i += stride) {
            if (i < n1) z1[i] = 0u;
            else z2[i - n1] = 0u;
        }
        return;
    }
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    const double p[3] = {params[3 * l], params[3 * l + 1], params[3 * l + 2]};
    double M[16], pos[3], dir[3];
    light_frame<double>(cams[l], p, M, pos, dir);
    ViewConst &v = views[l];
    for (int i = 0; i < 16; ++i) v.M[i] = (float)M[i];
    for (int i = 0; i < 3; ++i) {
        v.pos[i] = (float)pos[i];
        v.dir[i] = (float)dir[i];
    }
    v.zc = (float)light_reference_depth(cams[l], p);
    if (zc_out) zc_out[l] = v.zc;
    if (jac) light_jacobian(cams[l], params + 3 * l, jac + (size_t)kJac * l);
}

// ----------------------------------------------------------------------------- transform

__global__ void transform_kernel(const ViewConst *__restrict__ views, const float *__restrict__ verts,
                                 float4 *__restrict__ clip) {
    const ViewConst &v = views[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.nverts) return;
    const float *p = verts + 3 * (size_t)(v.vert_off + i);
    const float x = p[0], y = p[1], z = p[2];
    clip[v.clip_off + i] = clip_of(v.M, x, y, z);
}

// One TriVerts record per face: the corners' world positions gathered once,
// so that per-pixel passes fetch one record instead of face -> vertices.
__global__ void tri_verts_kernel(const int *__restrict__ scene_vert_off, const int *__restrict__ scene_face_off,
                                 const int *__restrict__ faces, const float *__restrict__ verts,
                                 const float *__restrict__ albedo, int C, TriVerts *__restrict__ tv) {
    const int b = blockIdx.y;
    const int f = scene_face_off[b] + blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= scene_face_off[b + 1]) return;
    const float *v0 = verts + 3 * (size_t)(scene_vert_off[b] + faces[3 * (size_t)f]);
    const float *v1 = verts + 3 * (size_t)(scene_vert_off[b] + faces[3 * (size_t)f + 1]);
    const float *v2 = verts + 3 * (size_t)(scene_vert_off[b] + faces[3 * (size_t)f + 2]);
    TriVerts r;
    r.a = make_float4(v0[0], v0[1], v0[2], v1[0]);
    r.b = make_float4(v1[1], v1[2], v2[0], v2[1]);
    // the face's albedo rides in the record's spare words: the lookups read it
    // with the corners instead of with a load of its own
    const float *rho = albedo + (size_t)f * C;
    r.c = make_float4(v2[2], rho[0], C > 1 ? rho[1] : 0.f, C > 2 ? rho[2] : 0.f);
    tv[f] = r;
}

hipError_t launch_tri_verts(const int *scene_vert_off, const int *scene_face_off, int B, int max_faces,
                            const int *faces, const float *verts, const float *albedo, int C, TriVerts *tv,
                            hipStream_t s) {
    if (B == 0 || max_faces == 0) return hipSuccess;
    hipLaunchKernelGGL(tri_verts_kernel, dim3((max_faces + 255) / 256, B), dim3(256), 0, s, scene_vert_off,
                       scene_face_off, faces, verts, albedo, C, tv);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- setup

__device__ __forceinline__ int floor_div256(int a) { return a >= 0 ? (a >> 8) : -((-a + 255) >> 8); }

__global__ void setup_kernel(const ViewConst *__restrict__ views, const int *__restrict__ faces,
                             const float4 *__restrict__ clip, TriSetup *__restrict__ setup,
                             signed char *__restrict__ facing8, unsigned *__restrict__ pair_count, int tile,
                             DevCounters *counters) {
    const int view = blockIdx.y;
    const ViewConst &v = views[view];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= v.nfaces) return;
    const int *f = faces + 3 * (size_t)(v.face_off + t);
    int idx[3] = {f[0], f[1], f[2]};
    bool bad = false;
    for (int k = 0; k < 3; ++k)
        if (idx[k] < 0 || idx[k] >= v.nverts) { bad = true; idx[k] = 0; }
    int X[3], Y[3];
    float z[3];
    bool ok = !bad;
    const float hw = 0.5f * (float)v.W, hh = 0.5f * (float)v.H;
    for (int k = 0; k < 3; ++k) {
        const float4 c = clip[v.clip_off + idx[k]];
        const float nx = c.x / c.w, ny = c.y / c.w, nz = c.z / c.w;
        const float sx = (nx + 1.0f) * hw;
        const float sy = (1.0f - ny) * hh;
        const bool okv = (c.w > 0.0f) && (nz >= -1.0f) && (fabsf(sx) < kGuard) && (fabsf(sy) < kGuard);
        ok = ok && okv;
        X[k] = okv ? (int)rintf(sx * 256.0f) : 0;
        Y[k] = okv ? (int)rintf(sy * 256.0f) : 0;
        z[k] = 0.5f * nz + 0.5f;
    }
    long long A = (long long)(X[1] - X[0]) * (Y[2] - Y[0]) - (long long)(Y[1] - Y[0]) * (X[2] - X[0]);
    const bool swapped = A < 0;
    if (swapped) {
        int ti = X[1]; X[1] = X[2]; X[2] = ti;
        ti = Y[1]; Y[1] = Y[2]; Y[2] = ti;
        float tz = z[1]; z[1] = z[2]; z[2] = tz;
        A = -A;
    }
    const bool valid = ok && A > 0;
    TriSetup s;
    s.A = A;
    for (int k = 0; k < 3; ++k) { s.X[k] = X[k]; s.Y[k] = Y[k]; s.z[k] = z[k]; }
    s.facing = valid ? (swapped ? -1 : 1) : 0;
    s.swapped = swapped ? 1 : 0;
    s.sil = 0;
    s.pad1 = 0;
    s.pad2[0] = view;
    s.pad2[1] = 0;
    unsigned npairs = 0;
    int i0 = 1, i1 = 0, j0 = 1, j1 = 0;
    if (valid) {
        const int mnx = min(X[0], min(X[1], X[2])), mxx = max(X[0], max(X[1], X[2]));
        const int mny = min(Y[0], min(Y[1], Y[2])), mxy = max(Y[0], max(Y[1], Y[2]));
        // pixel centres 256 i + 128 inside [mnx, mxx]
        i0 = max(floor_div256(mnx - 128 + 255), 0);
        i1 = min(floor_div256(mxx - 128), v.W - 1);
        j0 = max(floor_div256(mny - 128 + 255), 0);
        j1 = min(floor_div256(mxy - 128), v.H - 1);
        if (i0 <= i1 && j0 <= j1) npairs = (unsigned)((i1 / tile - i0 / tile + 1) * (j1 / tile - j0 / tile + 1));
    }
    if (!(i0 <= i1 && j0 <= j1)) { i0 = 1; i1 = 0; j0 = 1; j1 = 0; }
    s.bx0 = (unsigned short)i0;
    s.bx1 = (unsigned short)i1;
    s.by0 = (unsigned short)j0;
    s.by1 = (unsigned short)j1;
    setup[v.setup_off + t] = s;
    facing8[v.setup_off + t] = s.facing;
    pair_count[v.setup_off + t] = npairs;
    const unsigned long long nc = __popcll(__ballot(!ok && !bad));
    const unsigned long long nb = __popcll(__ballot(bad));
    if ((threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(1)) - 1) {
        if (nc) atomicAdd(&counters->culled, nc);
        if (nb) atomicAdd(&counters->bad_indices, nb);
    }
}

// Silhouette mask per (view, triangle): oriented edge e is a silhouette when
// no triangle or more than one other triangle shares it, or when the
// neighbour across it faces the other way in this view.
__global__ void silhouette_kernel(const ViewConst *__restrict__ views, const int *__restrict__ adj,
                                  const signed char *__restrict__ facing8, unsigned char *__restrict__ silm) {
    const ViewConst &v = views[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= v.nfaces) return;
    const int facing = facing8[v.setup_off + t];
    if (facing == 0) {
        silm[v.setup_off + t] = 0;
        return;
    }
    const bool sw = facing < 0;        // second and third vertex were exchanged
    unsigned mask = 0;
    for (int e = 0; e < 3; ++e) {
        const int a = (e + 1) % 3, b = (e + 2) % 3;
        const int oa = sw ? (a == 0 ? 0 : 3 - a) : a, ob = sw ? (b == 0 ? 0 : 3 - b) : b;
        const int nb = adj[3 * (size_t)(v.face_off + t) + (3 - oa - ob)];
        if (nb < 0 || facing8[v.setup_off + nb] != facing) mask |= 1u << e;
    }
    silm[v.setup_off + t] = (unsigned char)mask;
}

// ----------------------------------------------------------------------------- scan (exclusive, uint32)

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned *total) {
    __shared__ unsigned wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    unsigned base = 0, all = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) base += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return base + x - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(const unsigned *in, unsigned *out,
                                                                   unsigned *block_sums, int n) {
    const long long base = (long long)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    unsigned vals[kScanPer];
    unsigned sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        vals[k] = (base + k < n) ? in[base + k] : 0u;
        sum += vals[k];
    }
    unsigned total;
    unsigned off = block_exclusive_scan(sum, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = off;
        off += vals[k];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup per scan block: its offset is the sum of the block sums
// before it (nb <= kScanBlock, so each thread adds at most kScanPer of
// them), added to the block's kScanBlock outputs.  The last block also
// writes the grand total to out[n]; with n = 0 one workgroup writes 0.
__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(unsigned *out, const unsigned *block_sums, int n,
                                                                int nb) {
    const int b = blockIdx.x;
    unsigned part = 0;
    for (int k = threadIdx.x; k < b; k += kScanThreads) part += block_sums[k];
    unsigned off;
    block_exclusive_scan(part, &off);
    const long long base = (long long)b * kScanBlock;
    for (int k = threadIdx.x; k < kScanBlock; k += kScanThreads)
        if (base + k < n) out[base + k] += off;
    if (threadIdx.x == 0) {
        if (nb == 0) out[0] = 0u;
        else if (b == nb - 1) out[n] = off + block_sums[b];
    }
}

// Exclusive scan of n values in place-capable form: out[0..n] (out[n] = total).
// scratch: at least scan_scratch_words(n) words.
int scan_scratch_words(int n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan(const unsigned *in, unsigned *out, unsigned *scratch, int n, hipStream_t s) {
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb > kScanBlock) return hipErrorInvalidValue;
    if (nb > 0) hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, out, scratch, n);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb > 0 ? nb : 1), dim3(kScanThreads), 0, s, out, scratch, n, nb);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- binning

// Pairs of triangle i are the tiles of its bounding box in row-major order,
// numbered pair_off[i] .. pair_off[i+1]-1.  FILL = false counts pairs per
// tile and records each pair's slot in its tile (pair_slot, indexed by
// pair); FILL = true scatters (triangle, pair) to tile_start[tile] + slot,
// with no atomics.  Pairs q0, q0 + step, ... of the triangle are handled by
// the calling thread.
template <bool FILL>
__device__ __forceinline__ void bin_pairs(const ViewConst *__restrict__ views, const TriSetup &s, int i, unsigned a,
                                          unsigned b, int tile, unsigned q0, unsigned step,
                                          unsigned *__restrict__ tile_count, unsigned *__restrict__ pair_slot,
                                          const unsigned *__restrict__ tile_start, unsigned *__restrict__ bins,
                                          unsigned *__restrict__ bin_pair) {
    const ViewConst &v = views[s.pad2[0]];
    const int tx0 = s.bx0 / tile, tx1 = s.bx1 / tile, ty0 = s.by0 / tile;
    const int ntx = tx1 - tx0 + 1;
    for (unsigned q = q0; q < b - a; q += step) {
        const int tx = tx0 + (int)(q % ntx), ty = ty0 + (int)(q / ntx);
        const int gt = v.tile_off + ty * v.tiles_x + tx;
        if (!FILL) {
            pair_slot[a + q] = atomicAdd(&tile_count[gt], 1u);
        } else {
            const unsigned pos = tile_start[gt] + pair_slot[a + q];
            bins[pos] = (unsigned)i;
            bin_pair[pos] = a + q;
        }
    }
}

// Add each active lane's 1 to cnt[g], one atomic per distinct g in the wave
// (neighbouring triangles of a mesh mostly share tiles), and return the
// lane's slot: the old count plus its rank among the lanes with the same g.
// All leaders' atomics are issued together, so the wave waits for one round
// trip.  Uniform call (all 64 lanes).
__device__ __forceinline__ unsigned wave_aggregated_slot(bool has, int g, unsigned *__restrict__ cnt) {
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long pending = __ballot(has);
    int leader_of = lane;
    unsigned rank = 0, size = 0;
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int gg = __builtin_amdgcn_readlane(g, leader);
        const bool mine = has && g == gg;
        const unsigned long long m = __ballot(mine);
        pending &= ~m;
        if (mine) {
            leader_of = leader;
            rank = (unsigned)__popcll(m & ((1ull << lane) - 1ull));
            if (lane == leader) size = (unsigned)__popcll(m);
        }
    }
    unsigned base = 0;
    if (size) base = atomicAdd(&cnt[g], size);
    base = (unsigned)__shfl((int)base, leader_of, 64);
    return base + rank;
}

// Triangles with at most kBigBin pairs: one thread each.  Larger ones are
// listed (count pass) and handled a workgroup each, by bin_big_kernel in the
// count pass and by the fill pass's workgroups past nsmall.
// Triangles whose pair range does not fit the bin capacity go to the
// overflow path instead (decided per triangle, so never split).
constexpr unsigned kBigBin = 32;

template <bool FILL>
__global__ void bin_small_kernel(const ViewConst *__restrict__ views, const TriSetup *__restrict__ setup,
                                 const unsigned *__restrict__ pair_off, int ntri, unsigned capacity, int tile,
                                 unsigned *__restrict__ tile_count, unsigned *__restrict__ pair_slot,
                                 const unsigned *__restrict__ tile_start, unsigned *__restrict__ bins,
                                 unsigned *__restrict__ bin_pair, unsigned *__restrict__ big_list,
                                 unsigned *__restrict__ overflow_list, DevCounters *counters, int nsmall) {
    if (FILL && (int)blockIdx.x >= nsmall) {
        // workgroups past the triangles' own: the listed large triangles, a
        // workgroup each (their list is complete after the count pass)
        const unsigned n = counters->big_bin_len;
        for (unsigned o = blockIdx.x - nsmall; o < n; o += gridDim.x - nsmall) {
            const int t = (int)big_list[o];
            bin_pairs<true>(views, setup[t], t, pair_off[t], pair_off[t + 1], tile, threadIdx.x, blockDim.x, tile_count,
                            pair_slot, tile_start, bins, bin_pair);
        }
        return;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (!FILL && i == 0) counters->pairs = pair_off[ntri];   // total pairs, for the plan's statistics
    unsigned a = 0, b = 0;
    if (i < ntri) {
        a = pair_off[i];
        b = pair_off[i + 1];
        if (b > capacity) {                                // overflow path (listed by the count pass)
            if (!FILL && b > a) overflow_list[atomicAdd(&counters->overflow_list_len, 1u)] = (unsigned)i;
            b = a;
        }
        if (b - a > kBigBin) {
            if (!FILL) big_list[atomicAdd(&counters->big_bin_len, 1u)] = (unsigned)i;
            b = a;
        }
    }
    const unsigned cnt = b - a;
    if (__ballot(cnt > 0) == 0) return;                    // whole wave idle
    TriSetup st{};
    int tx0 = 0, ty0 = 0, ntx = 1, toff = 0, tiles_x = 0;
    if (cnt > 0) {
        st = setup[i];
        const ViewConst &v = views[st.pad2[0]];
        tx0 = st.bx0 / tile;
        ty0 = st.by0 / tile;
        ntx = st.bx1 / tile - tx0 + 1;
        toff = v.tile_off;
        tiles_x = v.tiles_x;
    }
    if (!FILL) {
        for (unsigned q = 0; __ballot(q < cnt) != 0; ++q) {   // uniform loop: the wave's largest count
            const bool has = q < cnt;
            const int gt = has ? toff + (ty0 + (int)(q / ntx)) * tiles_x + tx0 + (int)(q % ntx) : 0;
            const unsigned slot = wave_aggregated_slot(has, gt, tile_count);
            if (has) pair_slot[a + q] = slot;
        }
    } else {
        for (unsigned q = 0; q < cnt; ++q) {
            const int gt = toff + (ty0 + (int)(q / ntx)) * tiles_x + tx0 + (int)(q % ntx);
            const unsigned pos = tile_start[gt] + pair_slot[a + q];
            bins[pos] = (unsigned)i;
            bin_pair[pos] = a + q;
        }
    }
}

template <bool FILL>
__global__ void bin_big_kernel(const ViewConst *__restrict__ views, const TriSetup *__restrict__ setup,
                               const unsigned *__restrict__ pair_off, int tile, unsigned *__restrict__ tile_count,
                               unsigned *__restrict__ pair_slot, const unsigned *__restrict__ tile_start,
                               unsigned *__restrict__ bins, unsigned *__restrict__ bin_pair,
                               const unsigned *__restrict__ big_list, const DevCounters *counters) {
    const unsigned n = counters->big_bin_len;
    for (unsigned o = blockIdx.x; o < n; o += gridDim.x) {
        const int i = (int)big_list[o];
        bin_pairs<FILL>(views, setup[i], i, pair_off[i], pair_off[i + 1], tile, threadIdx.x, blockDim.x, tile_count,
                        pair_slot, tile_start, bins, bin_pair);
    }
}


// ----------------------------------------------------------------------------- raster

// A triangle as the tile raster tests it: each edge function in plane form,
// E_e(px, py) = a px + b py + c with a = -dy, b = dx, c = dy xa - dx ya for
// the directed edge a -> b opposite vertex e.  With fixed-point coordinates
// below 2^23 and differences below 2^24 every term and every partial sum is
// an integer below 2^49, so float64 holds the coefficients and evaluates
// E_e exactly with two fused multiply-adds: the same value, and the same
// inside / top-left / depth results, as the 64-bit integer form.  a and b
// (below 2^24) are kept as int32 to keep the LDS record small.
struct RasterTri {
    double c[3];
    int a[3], b[3];
    float z0, dz1, dz2;     // z0, z1 - z0, z2 - z0
    float rA;           // correctly rounded float32 1 / A
    unsigned short bx0, by0, bx1, by1;
    unsigned tri;
    int top_left;       // bit e: edge e is a top or left edge
};

__device__ __forceinline__ bool top_left(int xa, int ya, int xb, int yb) {
    const int dx = xb - xa, dy = yb - ya;
    return dy < 0 || (dy == 0 && dx > 0);
}

__device__ __forceinline__ RasterTri load_raster_tri(const TriSetup &s, unsigned local) {
    RasterTri r;
    r.top_left = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int ia = (e + 1) % 3, ib = (e + 2) % 3;
        const int xa = s.X[ia], ya = s.Y[ia], dx = s.X[ib] - xa, dy = s.Y[ib] - ya;
        r.a[e] = -dy;
        r.b[e] = dx;
        r.c[e] = (double)((long long)dy * xa - (long long)dx * ya);
        r.top_left |= top_left(xa, ya, s.X[ib], s.Y[ib]) ? 1 << e : 0;
    }
    r.z0 = s.z[0];
    r.dz1 = s.z[1] - s.z[0];
    r.dz2 = s.z[2] - s.z[0];
    r.rA = 1.0f / (float)(double)s.A;
    r.bx0 = s.bx0; r.by0 = s.by0; r.bx1 = s.bx1; r.by1 = s.by1;
    r.tri = local;
    return r;
}

// Key of triangle r at pixel (i, j), or kBgKey when not covered.
__device__ __forceinline__ unsigned long long sample_key(const RasterTri &r, int i, int j) {
    if (i < r.bx0 || i > r.bx1 || j < r.by0 || j > r.by1) return kBgKey;
    const double px = (double)(i * kSub + kSub / 2), py = (double)(j * kSub + kSub / 2);
    const double e0 = fma((double)r.a[0], px, fma((double)r.b[0], py, r.c[0]));
    const double e1 = fma((double)r.a[1], px, fma((double)r.b[1], py, r.c[1]));
    const double e2 = fma((double)r.a[2], px, fma((double)r.b[2], py, r.c[2]));
    const bool in0 = e0 > 0.0 || (e0 == 0.0 && (r.top_left & 1));
    const bool in1 = e1 > 0.0 || (e1 == 0.0 && (r.top_left & 2));
    const bool in2 = e2 > 0.0 || (e2 == 0.0 && (r.top_left & 4));
    if (!(in0 && in1 && in2)) return kBgKey;
    // b_e = f32(E_e) * (1 / A): one reciprocal per triangle, one product per sample
    const float b1 = (float)e1 * r.rA;
    const float b2 = (float)e2 * r.rA;
    const float z = (r.z0 + b1 * r.dz1) + b2 * r.dz2;
    if (!(z >= 0.0f && z <= 1.0f)) return kBgKey;
    const unsigned bits = __float_as_uint(z) & 0x7FFFFFFFu;
    return ((unsigned long long)bits << 32) | r.tri;
}

constexpr int kRasterThreads = 256;

// One workgroup per tile; each thread owns T*T/256 (or one) pixels and keeps
// the minimum key in registers while the tile's bin streams through LDS.
template <int T>
__global__ __launch_bounds__(kRasterThreads) void raster_kernel(
    const ViewConst *__restrict__ views, const int *__restrict__ tile_view, const TriSetup *__restrict__ setup,
    const unsigned *__restrict__ tile_start, const unsigned *__restrict__ bins,
    unsigned long long *__restrict__ keys) {
    constexpr int NPIX = T * T;
    constexpr int NT = NPIX < kRasterThreads ? NPIX : kRasterThreads;
    constexpr int PPT = NPIX / NT;
    __shared__ RasterTri tris[NT];
    const int gt = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int view = tile_view[gt];
    const ViewConst &v = views[view];
    const int lt = gt - v.tile_off;
    const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
    const int tid = threadIdx.x;
    if (tid >= NT) return;
    int pi[PPT], pj[PPT];
    unsigned long long best[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int l = tid + k * NT;
        pi[k] = tx * T + (l % T);
        pj[k] = ty * T + (l / T);
        best[k] = kBgKey;
    }
    const unsigned b0 = tile_start[gt], b1 = tile_start[gt + 1];
    for (unsigned c = b0; c < b1; c += NT) {
        const unsigned n = min((unsigned)NT, b1 - c);
        __syncthreads();
        if ((unsigned)tid < n) {
            const unsigned si = bins[c + tid];
            tris[tid] = load_raster_tri(setup[si], si - (unsigned)v.setup_off);
        }
        __syncthreads();
        // four entries per step: their independent edge-function / depth
        // chains interleave, which hides latency at a given occupancy
        unsigned q = 0;
        for (; q + 4 <= n; q += 4) {
            const RasterTri &r0 = tris[q], &r1 = tris[q + 1], &r2 = tris[q + 2], &r3 = tris[q + 3];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const unsigned long long k0 = sample_key(r0, pi[k], pj[k]);
                const unsigned long long k1 = sample_key(r1, pi[k], pj[k]);
                const unsigned long long k2 = sample_key(r2, pi[k], pj[k]);
                const unsigned long long k3 = sample_key(r3, pi[k], pj[k]);
                const unsigned long long a01 = k0 < k1 ? k0 : k1, a23 = k2 < k3 ? k2 : k3;
                const unsigned long long a = a01 < a23 ? a01 : a23;
                best[k] = a < best[k] ? a : best[k];
            }
        }
        for (; q < n; ++q) {
            const RasterTri &r = tris[q];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const unsigned long long key = sample_key(r, pi[k], pj[k]);
                best[k] = key < best[k] ? key : best[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (pi[k] < v.W && pj[k] < v.H) keys[v.pix_off + (long long)pj[k] * v.W + pi[k]] = best[k];
}

// Triangles that did not fit the bins: one workgroup per listed triangle at
// a time, atomic minimum over its bounding box.  The first thread also adds
// the list's length to the overflow count.
__global__ void overflow_raster_kernel(const ViewConst *__restrict__ views, const TriSetup *__restrict__ setup,
                                       const unsigned *__restrict__ list, DevCounters *counters,
                                       unsigned long long *__restrict__ keys) {
    const unsigned n = counters->overflow_list_len;
    if (blockIdx.x == 0 && threadIdx.x == 0) counters->overflow += n;
    for (unsigned o = blockIdx.x; o < n; o += gridDim.x) {
        const unsigned si = list[o];
        const TriSetup &s = setup[si];
        const ViewConst &v = views[s.pad2[0]];
        const RasterTri r = load_raster_tri(s, si - (unsigned)v.setup_off);
        const int w = r.bx1 - r.bx0 + 1, h = r.by1 - r.by0 + 1;
        if (w <= 0 || h <= 0) continue;
        const long long npix = (long long)w * h;
        for (long long q = threadIdx.x; q < npix; q += blockDim.x) {
            const int i = r.bx0 + (int)(q % w), j = r.by0 + (int)(q / w);
            const unsigned long long key = sample_key(r, i, j);
            if (key != kBgKey) atomicMin(&keys[v.pix_off + (long long)j * v.W + i], key);
        }
    }
}

// ----------------------------------------------------------------------------- host launchers

hipError_t launch_light_frames(ViewConst *views, const CamStatic *cams, const float *params, int L, float *jac,
                               float *zc_out, void *z1, size_t bytes1, void *z2, size_t bytes2, hipStream_t s) {
    const int nf = (L + 63) / 64;
    const size_t n1 = bytes1 / 4, n2 = bytes2 / 4;
    const size_t nz = std::min<size_t>((n1 + n2 + 255) / 256, 16384);
    if (nf + nz == 0) return hipSuccess;
    hipLaunchKernelGGL(light_frames_kernel, dim3((unsigned)(nf + nz)), dim3(64), 0, s, views, cams, params, L, zc_out,
                       jac, nf, (unsigned *)z1, n1, (unsigned *)z2, n2);
    return hipGetLastError();
}

hipError_t launch_transform(const ViewConst *views, int nviews, int max_verts, const float *verts, float4 *clip,
                            hipStream_t s) {
    if (nviews == 0 || max_verts == 0) return hipSuccess;
    hipLaunchKernelGGL(transform_kernel, dim3((max_verts + 255) / 256, nviews), dim3(256), 0, s, views, verts, clip);
    return hipGetLastError();
}

hipError_t launch_silhouettes(const ViewConst *views, int nviews, int max_faces, const int *adj,
                              const signed char *facing8, unsigned char *silm, hipStream_t s) {
    if (nviews == 0 || max_faces == 0) return hipSuccess;
    hipLaunchKernelGGL(silhouette_kernel, dim3((max_faces + 255) / 256, nviews), dim3(256), 0, s, views, adj, facing8, silm);
    return hipGetLastError();
}

hipError_t launch_setup(const ViewConst *views, int nviews, int max_faces, const int *faces, const float4 *clip,
                        TriSetup *setup, signed char *facing8, unsigned *pair_count, int tile, DevCounters *counters,
                        hipStream_t s) {
    if (nviews == 0 || max_faces == 0) return hipSuccess;
    hipLaunchKernelGGL(setup_kernel, dim3((max_faces + 255) / 256, nviews), dim3(256), 0, s, views, faces, clip,
                       setup, facing8, pair_count, tile, counters);
    return hipGetLastError();
}

hipError_t launch_binning(const ViewConst *views, const TriSetup *setup, const unsigned *pair_off, int ntri,
                          unsigned capacity, int tile, unsigned *tile_count, unsigned *tile_start,
                          unsigned *pair_slot, unsigned *scan_scratch, int ntiles, unsigned *bins,
                          unsigned *bin_pair, unsigned *overflow_list, unsigned *big_list, DevCounters *counters,
                          hipStream_t s) {
    const dim3 tgrid((ntri + 255) / 256);
    const dim3 bgrid(1024);
    if (ntri > 0) {
        hipLaunchKernelGGL(bin_small_kernel<false>, tgrid, dim3(256), 0, s, views, setup, pair_off, ntri, capacity, tile,
                           tile_count, pair_slot, (const unsigned *)nullptr, (unsigned *)nullptr, (unsigned *)nullptr,
                           big_list, overflow_list, counters, (int)tgrid.x);
        hipLaunchKernelGGL(bin_big_kernel<false>, bgrid, dim3(256), 0, s, views, setup, pair_off, tile, tile_count,
                           pair_slot, (const unsigned *)nullptr, (unsigned *)nullptr, (unsigned *)nullptr,
                           (const unsigned *)big_list, (const DevCounters *)counters);
    }
    hipError_t e = launch_scan(tile_count, tile_start, scan_scratch, ntiles, s);
    if (e != hipSuccess) return e;
    if (ntri > 0) {
        // the fill pass and the large triangles' fill in one launch (bgrid.x extra workgroups)
        hipLaunchKernelGGL(bin_small_kernel<true>, dim3(tgrid.x + bgrid.x), dim3(256), 0, s, views, setup, pair_off,
                           ntri, capacity, tile, (unsigned *)nullptr, pair_slot, (const unsigned *)tile_start, bins,
                           bin_pair, big_list, overflow_list, counters, (int)tgrid.x);
    }
    return hipGetLastError();
}

hipError_t launch_raster(const ViewConst *views, const int *tile_view, int ntiles, int tile, const TriSetup *setup,
                         const unsigned *tile_start, const unsigned *bins, const unsigned *overflow_list,
                         const DevCounters *counters_ro, DevCounters *counters, unsigned long long *keys,
                         hipStream_t s) {
    if (ntiles > 0) {
        if (tile == 8)
            hipLaunchKernelGGL(raster_kernel<8>, dim3(ntiles), dim3(64), 0, s, views, tile_view, setup, tile_start,
                               bins, keys);
        else if (tile == 16)
            hipLaunchKernelGGL(raster_kernel<16>, dim3(ntiles), dim3(256), 0, s, views, tile_view, setup, tile_start,
                               bins, keys);
        else
            hipLaunchKernelGGL(raster_kernel<32>, dim3(ntiles), dim3(256), 0, s, views, tile_view, setup, tile_start,
                               bins, keys);
    }
    hipLaunchKernelGGL(overflow_raster_kernel, dim3(512), dim3(256), 0, s, views, setup, overflow_list, counters,
                       keys);
    return hipGetLastError();
}

}  // namespace dsm
