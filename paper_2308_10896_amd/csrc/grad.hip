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
// Vertex-indexed gradients are reduced per (tile, triangle) before they reach
// global memory (see "tile accumulation" below).
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
        const int k = __builtin_amdgcn_readlane(key, leader);
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

// Reciprocal (about one ulp) for gradient terms and for the shading values
// the adjoints recompute exactly as the forward kernels form them (the map
// position, which picks the bilinear cell, among them: both passes take that
// decision from the same float32 value).  The correctly rounded division,
// which the raster setup keeps for its integer results, costs about ten
// instructions, this one.
__device__ __forceinline__ float grcp(float x) { return __builtin_amdgcn_rcpf(x); }

// NDC of pixel centre i of n, as the forward resolve and lookup form it.
__device__ __forceinline__ float ndc_c(int i, int n) { return (float)(2 * i + 1) * grcp((float)n) - 1.0f; }

// Barycentrics through the hardware reciprocal of their sum (about one ulp):
// the forward lookup forms the world point the same way, so the reverse pass
// recomputes its values, and its decisions, bit for bit.
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
    const float rs = __builtin_amdgcn_rcpf(r.s);
    r.b0 = r.k0 * rs; r.b1 = r.k1 * rs; r.b2 = r.k2 * rs;
    return r;
}

// gb (d loss / d barycentrics) -> gradient w.r.t. clip (x, y, w) of the 3 corners: out[3*i + {0,1,2}]
__device__ __forceinline__ void bary_backward(const BaryFull &b, float px, float py, float gb0, float gb1, float gb2,
                                              float out[9]) {
    // adjoint only: fused multiply-adds
    const float dotg = fmaf(gb2, b.b2, fmaf(gb1, b.b1, gb0 * b.b0));
    const float rs = grcp(b.s);
    const float gk0 = (gb0 - dotg) * rs, gk1 = (gb1 - dotg) * rs, gk2 = (gb2 - dotg) * rs;
    const float ga0x = fmaf(gk2, b.a1y, -gk1 * b.a2y), ga0y = fmaf(gk1, b.a2x, -gk2 * b.a1x);
    const float ga1x = fmaf(gk0, b.a2y, -gk2 * b.a0y), ga1y = fmaf(gk2, b.a0x, -gk0 * b.a2x);
    const float ga2x = fmaf(gk1, b.a0y, -gk0 * b.a1y), ga2y = fmaf(gk0, b.a1x, -gk1 * b.a0x);
    out[0] = ga0x; out[1] = ga0y; out[2] = -fmaf(px, ga0x, py * ga0y);
    out[3] = ga1x; out[4] = ga1y; out[5] = -fmaf(px, ga1x, py * ga1y);
    out[6] = ga2x; out[7] = ga2y; out[8] = -fmaf(px, ga2x, py * ga2y);
}

// ----------------------------------------------------------------------------- camera smoothing^T

template <int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void aa_camera_backward_kernel(
    const ViewConst *__restrict__ views, const RenderConst *__restrict__ renders, const TriSetup *__restrict__ setup,
    const int *__restrict__ faces, const unsigned char *__restrict__ silm, const float *__restrict__ verts,
    const unsigned long long *__restrict__ keys, const unsigned char *__restrict__ aa_flag,
    const float *__restrict__ img0, const float *__restrict__ gimg,
    float *__restrict__ gimg0, float4 *__restrict__ gclip) {
    const Blk blk = xcd_block2();
    const RenderConst &R = renders[blk.y];
    const ViewConst &v = views[R.camera_view];
    const int W = v.W, H = v.H;
    const int p = aa_sample_index(blk.x, (int)threadIdx.x, W, H);
    if (blk.x * 256 >= W * H || p >= W * H) return;
    const float *c0 = img0 + R.img_off;
    const float *g = gimg + R.img_off;
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) acc[c] = g[(long long)p * C + c];
    const float gself[3] = {acc[0], acc[1], acc[2]};
    // samples the forward found without candidate pairs pass the gradient through
    if (v.antialias && v.nfaces > 0 && aa_flag[v.pix_off + p]) {
        const int i = p % W, j = p / W;
        const unsigned long long *kv = keys + v.pix_off;
        const unsigned long long ks = kv[p];
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
        const AANeighbours nb = aa_neighbours(v, kv, silm, ks, i, j);
        // image values and upstream gradients of this sample and the
        // candidate neighbours, fetched before the pair tests so that they
        // arrive with the triangle records
        const bool any = nb.cand[0] || nb.cand[1] || nb.cand[2] || nb.cand[3];
        float cself[3], cn[4][3], gn[4][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) cself[c] = (any && c < C) ? c0[(long long)p * C + c] : 0.f;
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const bool ld = nb.cand[d] && c < C;
                cn[d][c] = ld ? c0[(long long)nb.q[d] * C + c] : 0.f;
                gn[d][c] = ld ? g[(long long)nb.q[d] * C + c] : 0.f;
            }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (!nb.cand[d]) continue;
            const int in_ = i + di[d], jn = j + dj[d];
            const unsigned long long kn = nb.kn[d];
            bool self_front;
            AAPair pr;
            if (!aa_eval<true>(v, setup, faces, silm, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
            const bool self_recv = (pr.recv == 1) != self_front;
            if (self_recv) {
                double galpha = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (c >= C) continue;
                    const float gs = gself[c];
                    acc[c] -= pr.w * gs;
                    galpha += (double)gs * (cn[d][c] - cself[c]);
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
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (c < C) acc[c] += pr.w * gn[d][c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (c < C) gimg0[R.img_off + (long long)p * C + c] = acc[c];
}

// ----------------------------------------------------------------------------- reduction by (triangle, tile)

// Float atomics on this GPU are performed at the memory side, so many
// workgroups adding into the same few addresses (the two triangles of a
// ground plane, a light's frame gradient) serialize.  The backward kernels
// therefore avoid hot atomics altogether: they walk the same tiles as the
// rasterizer and, for every triangle binned to a tile, write the sum of that
// triangle's per-pixel gradient terms over the tile's pixels into the
// triangle's slot for that tile (the binning already gave every (triangle,
// tile) pair a unique index).  Later gathers sum those slots per triangle,
// then per vertex (through the vertex -> triangle-corner lists), with plain
// stores.  Per-light terms are written per tile and summed per light the
// same way.  Only triangles that overflowed the bins, the sparse silhouette
// terms and the bilinear moment-map scatter use atomics.
constexpr int kNV = 21;   // per pair: 9 world-position terms, 9 clip (x, y, w) terms, 3 albedo terms

// Per-triangle gradient rows (gtri) hold the same 21 values as three 8-float
// corner records, [world x y z | clip x y w | albedo term of channel c | 0]
// for corner c, so that the per-vertex gather reads one aligned 32-byte
// sector per incident corner.  gtri_slot maps value index i (the pair-row
// order above) to its place in the row.
constexpr int kGtriStride = 24;
__host__ __device__ constexpr int gtri_slot(int i) {
    return i < 9 ? (i / 3) * 8 + i % 3 : i < 18 ? ((i - 9) / 3) * 8 + 3 + (i - 9) % 3 : (i - 18) * 8 + 6;
}

template <int T>
struct TileShape {
    static constexpr int NPIX = T * T;
    static constexpr int NT = NPIX < 256 ? NPIX : 256;
    static constexpr int PPT = NPIX / NT;
    static constexpr int NW = NT / 64;
};

// Per-workgroup sum of N per-thread values, written to dst[0..N) by threads < N.  Uniform call.
struct IdentitySlot {
    __device__ int operator()(int i) const { return i; }
};

// Workgroup sums of N values; value i is stored at dst[slot(i)].
template <int NW, int N, class Slot = IdentitySlot>
__device__ __forceinline__ void block_sum_store(const float (&val)[N], float *dst, Slot slot = Slot()) {
    __shared__ float part[NW][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    const float t = wave_sum_multi(val);      // lane 2i holds the wave's total of value i
    const int i = lane >> 1;
    if (NW == 1) {
        if ((lane & 1) == 0 && i < N) dst[slot(i)] = t;
        return;
    }
    if ((lane & 1) == 0 && i < N) part[w][i] = t;
    __syncthreads();
    if (threadIdx.x < N) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < NW; ++q) s += part[q][threadIdx.x];
        dst[slot(threadIdx.x)] = s;
    }
}

// For every triangle binned to tile gt: sum of val over the tile's active
// pixels it owns -> pair_sums[pair index][0..N), zeros when it owns none.
// Marks the pixels whose triangle was found.  Uniform call.
//
// The bin is walked in chunks of 64 entries (triangle and pair index, both
// written by the binning pass).  Each pixel finds the entry of its triangle
// (a broadcast LDS scan of the chunk) and adds its N values into that
// entry's LDS row with LDS atomics.  Every entry's pair_flag byte is written
// (1: the row holds a sum, 0: the triangle owns no active pixel here), and
// only flagged rows are stored.  Cost per pixel is N LDS adds however many
// triangles share the tile, so dense meshes (about one triangle per pixel)
// stay cheap.
// The tile's bin range and this thread's entry of its first chunk, loaded
// at the start of a tile kernel so that these dependent loads overlap the
// per-pixel work instead of following it.  Loads are unconditional (clamped
// indices) so that nothing waits for them before their use.
struct BinHead {
    unsigned b0, b1, si, pair;
};
__device__ __forceinline__ BinHead bin_head(int gt, int tid, const unsigned *__restrict__ tile_start,
                                            const unsigned *__restrict__ bins,
                                            const unsigned *__restrict__ bin_pair) {
    BinHead h;
    h.b0 = tile_start[gt];
    h.b1 = tile_start[gt + 1];
    const unsigned c = h.b1 > h.b0 ? min(h.b0 + (unsigned)tid, h.b1 - 1) : 0u;
    h.si = bins[c];
    h.pair = bin_pair[c];
    return h;
}

template <int T, int N>
__device__ __forceinline__ void tile_pair_sums(const ViewConst &v, const BinHead &head,
                                               const unsigned *__restrict__ bins,
                                               const unsigned *__restrict__ bin_pair,
                                               const int (&key)[TileShape<T>::PPT],
                                               const float (&val)[TileShape<T>::PPT][N],
                                               const bool (&act)[TileShape<T>::PPT],
                                               bool (&matched)[TileShape<T>::PPT],
                                               unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums) {
    using TS = TileShape<T>;
    constexpr int CH = 64;
    __shared__ float part[CH * N];
    __shared__ __align__(16) int ent[CH];
    __shared__ unsigned slot[CH];
    __shared__ int hit[CH];
    const int tid = threadIdx.x;
    const unsigned b0 = head.b0, b1 = head.b1;
    bool mine = false;
#pragma unroll
    for (int k = 0; k < TS::PPT; ++k) mine = mine || act[k];
    const bool any = __syncthreads_or(mine) != 0;
    for (unsigned c0 = b0; c0 < b1; c0 += CH) {
        const int n = (int)min((unsigned)CH, b1 - c0);
        if (tid < CH) {
            const bool first = c0 == b0;
            // unused entries hold -2, which matches no key (background is -1)
            ent[tid] = tid < n ? (int)((first ? head.si : bins[c0 + tid]) - (unsigned)v.setup_off) : -2;
            slot[tid] = tid < n ? (first ? head.pair : bin_pair[c0 + tid]) : 0u;
            hit[tid] = 0;
        }
        if (any)
            for (int f = tid; f < n * N; f += TS::NT) part[f] = 0.f;
        __syncthreads();
        if (any) {
            int idx[TS::PPT];
#pragma unroll
            for (int k = 0; k < TS::PPT; ++k) idx[k] = -1;
            // fixed-length scan, four entries per LDS read, all reads in flight together
            const int4 *ent4 = reinterpret_cast<const int4 *>(ent);
#pragma unroll
            for (int e4 = 0; e4 < CH / 4; ++e4) {
                const int4 t = ent4[e4];
#pragma unroll
                for (int k = 0; k < TS::PPT; ++k) {
                    idx[k] = key[k] == t.x ? 4 * e4 : idx[k];
                    idx[k] = key[k] == t.y ? 4 * e4 + 1 : idx[k];
                    idx[k] = key[k] == t.z ? 4 * e4 + 2 : idx[k];
                    idx[k] = key[k] == t.w ? 4 * e4 + 3 : idx[k];
                }
            }
            const int lane = tid & 63;
#pragma unroll
            for (int k = 0; k < TS::PPT; ++k) {
                if (idx[k] >= 0) matched[k] = true;
                bool todo = idx[k] >= 0 && act[k];
                // A triangle owning many of the wave's pixels (a large ground
                // polygon) is summed with one multi-value wave reduction; LDS
                // atomics from that many lanes into one row would serialize.
                for (int round = 0; round < 2; ++round) {
                    const unsigned long long m = __ballot(todo);
                    if (m == 0) break;
                    const int leader = __ffsll(m) - 1;
                    const int kk = __builtin_amdgcn_readlane(key[k], leader);
                    const bool in = todo && key[k] == kk;
                    if (__popcll(__ballot(in)) < 16) break;
                    float masked[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) masked[i] = in ? val[k][i] : 0.f;
                    const float t = wave_sum_multi(masked);
                    const int e = __builtin_amdgcn_readlane(idx[k], leader);
                    if ((lane & 1) == 0 && (lane >> 1) < N) atomicAdd(part + e * N + (lane >> 1), t);
                    if (lane == leader) hit[e] = 1;
                    todo = todo && !in;
                }
                if (todo) {
                    hit[idx[k]] = 1;
                    float *row = part + idx[k] * N;
#pragma unroll
                    for (int i = 0; i < N; ++i)
                        if (val[k][i] != 0.f) atomicAdd(row + i, val[k][i]);
                }
            }
            __syncthreads();
        }
        if (tid < n) pair_flag[slot[tid]] = (unsigned char)hit[tid];
        if (any) {
            constexpr int G = 4;                          // LDS reads of G iterations in flight together
            const int iters = (n * N + TS::NT - 1) / TS::NT;
#pragma unroll 1
            for (int it0 = 0; it0 < iters; it0 += G) {
                float pv[G];
                unsigned dst[G];
                bool wr[G];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int f = tid + (it0 + g) * TS::NT;
                    const int e = min(f / N, CH - 1), i = f - (f / N) * N;
                    wr[g] = f < n * N && hit[e] != 0;
                    dst[g] = slot[e] * (unsigned)kNV + (unsigned)i;
                    pv[g] = part[min(f, CH * N - 1)];
                }
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (wr[g]) pair_sums[dst[g]] = pv[g];
            }
        }
        __syncthreads();
    }
}

// Pixels of triangles that overflowed the bins: straight to their rows of gtri.  Uniform call.
template <int PPT, int N>
__device__ __forceinline__ void overflow_rows(const ViewConst &v, const int (&key)[PPT], const float (&val)[PPT][N],
                                              const bool (&active)[PPT], const bool (&matched)[PPT],
                                              float *__restrict__ gtri) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const bool a = active[k] && !matched[k];
        if (__ballot(a))
            scatter_by_key(a, key[k], val[k],
                           [&](int t, int i) { return gtri + (size_t)(v.setup_off + t) * kGtriStride + gtri_slot(i); });
    }
}

// Per-(triangle, tile) sums of one 8x8 tile held by one wave, without walking
// the tile's bin: the pairs of triangle t are the tiles of its bounding box
// in row-major order, numbered from pair_off[t] as the binning numbers them,
// so a pixel finds its row from its triangle's setup record.  Lanes holding
// the same triangle are grouped by a leader loop (one iteration per distinct
// triangle in the wave); a group of 16 or more lanes (a large ground
// polygon) is summed with one multi-value wave reduction, the others with
// LDS atomics into the row of their leader (the group's lowest lane), which
// then stores the row and flags the pair.  Pair flags start at zero (the
// backward clears them), so pairs without a pixel keep flag 0.  Pixels of
// triangles that overflowed the bins stay unmatched for overflow_rows.
// Uniform call (all 64 lanes).
template <int T, int N>
__device__ __forceinline__ void wave_pair_sums(const ViewConst &v, int tx, int ty, int key, const float (&val)[N],
                                               bool act, bool &matched, const TriSetup *__restrict__ setup,
                                               const unsigned *__restrict__ pair_off, unsigned capacity,
                                               unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums) {
    __shared__ float part[64 * N];
    const int lane = (int)(threadIdx.x & 63);
    unsigned slot = 0;
    bool mine = false;
    if (act && key >= 0) {
        const int si = v.setup_off + key;
        const unsigned a = pair_off[si], b = pair_off[si + 1];
        if (!(b > capacity && b > a)) {                  // else: the overflow path
            const TriSetup &st = setup[si];
            const int tx0 = st.bx0 / T, ty0 = st.by0 / T, ntx = st.bx1 / T - tx0 + 1;
            slot = a + (unsigned)((ty - ty0) * ntx + (tx - tx0));
            mine = true;
        }
    }
    matched = mine;
    // leader of every lane's group; groups of 16 or more lanes go to the wave reduction
    int leader = lane;
    unsigned long long pending = __ballot(mine), big = 0ull;
    while (pending) {
        const int l = __ffsll(pending) - 1;
        const int kk = __builtin_amdgcn_readlane(key, l);
        const bool in = mine && key == kk;
        const unsigned long long m = __ballot(in);
        pending &= ~m;
        if (in) leader = l;
        if (__popcll(m) >= 16) big |= m;
    }
    while (big) {
        const int l = __ffsll(big) - 1;
        const int kk = __builtin_amdgcn_readlane(key, l);
        const bool in = mine && key == kk;
        big &= ~__ballot(in);
        float masked[N];
#pragma unroll
        for (int i = 0; i < N; ++i) masked[i] = in ? val[i] : 0.f;
        const float t = wave_sum_multi(masked);          // lane 2i: the group's total of value i
        const unsigned sl = (unsigned)__builtin_amdgcn_readlane((int)slot, l);
        if ((lane & 1) == 0 && (lane >> 1) < N) pair_sums[(size_t)sl * kNV + (lane >> 1)] = t;
        if (lane == l) pair_flag[sl] = 1;
        mine = mine && !in;
    }
    const bool lead = mine && leader == lane;
    if (lead) {
#pragma unroll
        for (int i = 0; i < N; ++i) part[lane * N + i] = val[i];
    }
    __syncthreads();
    if (mine && !lead) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (val[i] != 0.f) atomicAdd(part + leader * N + i, val[i]);
    }
    __syncthreads();
    if (lead) {
#pragma unroll
        for (int i = 0; i < N; ++i) pair_sums[(size_t)slot * kNV + i] = part[lane * N + i];
        pair_flag[slot] = 1;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------- lookup^T

// Gradient contributions of one camera pixel: vertex terms (gv[9] for the
// 3 corners' world positions, gc[9] for their clip (x, y, w)), albedo terms,
// and per-light frame terms added into accl.
// Where one pixel's gradient lands in a light's moment maps: the bilinear
// taps around texel coordinate (ix + fx, iy + fy), weights for (gm1, gm2).
struct MapHit {
    int ix, iy;
    float fx, fy, gm1, gm2;
};

template <int MAXL, bool DIRECT>
__device__ __forceinline__ void lookup_pixel_grad(const ViewConst &cv, const RenderConst &R,
                                                  const ViewConst *__restrict__ views,
                                                  const int *__restrict__ render_lights,
                                                  const TriVerts *__restrict__ tv, const float *__restrict__ albedo,
                                                  const float *__restrict__ maps,
                                                  float *__restrict__ gmaps, int i, int j, int tri, const float g[3],
                                                  int C, float (&vals)[21], float (&accl)[MAXL][3],
                                                  MapHit (&hits)[MAXL], const float *__restrict__ jac) {
    const TriVerts r = tv[cv.face_off + tri];
    const float v0[3] = {r.a.x, r.a.y, r.a.z}, v1[3] = {r.a.w, r.b.x, r.b.y}, v2[3] = {r.b.z, r.b.w, r.c.x};
    const float px = ndc_c(i, cv.W), py = -ndc_c(j, cv.H);
    const float4 c0 = clip_of(cv.M, v0[0], v0[1], v0[2]), c1 = clip_of(cv.M, v1[0], v1[1], v1[2]),
                 c2 = clip_of(cv.M, v2[0], v2[1], v2[2]);
    const BaryFull b = bary_full(c0, c1, c2, px, py);
    const float x = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
    const float y = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
    const float z = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
    const float e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e1z = v1[2] - v0[2];
    const float e2x = v2[0] - v0[0], e2y = v2[1] - v0[1], e2z = v2[2] - v0[2];
    const float crx = e1y * e2z - e1z * e2y, cry = e1z * e2x - e1x * e2z, crz = e1x * e2y - e1y * e2x;
    const float rn0 = __builtin_amdgcn_rsqf((crx * crx + cry * cry) + crz * crz);
    const float nx = crx * rn0, ny = cry * rn0, nz = crz * rn0;
    float rho[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < C; ++c) rho[c] = c == 0 ? r.c.y : c == 1 ? r.c.z : r.c.w;   // from the face record
    float srho = 0.f;
    for (int c = 0; c < C; ++c) srho += g[c] * rho[c];
    float gx[3] = {0, 0, 0}, gn[3] = {0, 0, 0};
    float shade = 0.f;
#pragma unroll
    for (int q = 0; q < MAXL; ++q) {
        if (q >= R.light_count) break;
        const ViewConst &l = views[render_lights[R.light_begin + q]];
        const float *M = l.M;
        const float cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
        const float cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
        const float cw = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
        const float rcw = __builtin_amdgcn_rcpf(cw);
        const float ux = cx * rcw, uy = cy * rcw;
        const bool inside = cw > 0.f && fabsf(ux) <= 1.f && fabsf(uy) <= 1.f;
        float vis = 1.f, visr = 1.f, zz = 0.f, zw = 0.f, floor_v = 0.f, m1 = 0.f, m2 = 0.f, var = 0.f, dd = 0.f,
              fx = 0.f, fy = 0.f;
        long long o00 = 0, o01 = 0, o10 = 0, o11 = 0;
        int ixs = 0, iys = 0;
        hits[q].gm1 = 0.f;
        hits[q].gm2 = 0.f;
        // outside its own directions a cube face adds nothing, nor any gradient
        if (l.kind == kCubeFace && cube_face_of(x - l.pos[0], y - l.pos[1], z - l.pos[2]) != l.cube_face) continue;
        const int S = l.W;
        // filtered maps are stored with side Sp; cube faces keep P texels of
        // their neighbours around the face, so taps may cross the seam
        const int P = l.fpad, Sp = S + 2 * P;
        // filtered maps hold (m1, m2) interleaved per texel
        const float2 *mm = (const float2 *)(maps + l.fmap_off);
        float2 t00 = make_float2(0.f, 0.f), t01 = t00, t10 = t00, t11 = t00;
        if (inside) {
            const float sx = (ux + 1.f) * (0.5f * S) - 0.5f;
            const float sy = (1.f - uy) * (0.5f * S) - 0.5f;
            const float fx0 = floorf(sx), fy0 = floorf(sy);
            fx = sx - fx0;
            fy = sy - fy0;
            const int ix = (int)fx0 + P, iy = (int)fy0 + P;
            ixs = ix;
            iys = iy;
            const int x0 = min(max(ix, 0), Sp - 1), x1 = min(max(ix + 1, 0), Sp - 1);
            const int y0 = min(max(iy, 0), Sp - 1), y1 = min(max(iy + 1, 0), Sp - 1);
            const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
            o00 = (long long)y0 * Sp + x0; o01 = (long long)y0 * Sp + x1;
            o10 = (long long)y1 * Sp + x0; o11 = (long long)y1 * Sp + x1;
            t00 = mm[o00]; t01 = mm[o01]; t10 = mm[o10]; t11 = mm[o11];
            m1 = ((w00 * t00.x + w01 * t01.x) + w10 * t10.x) + w11 * t11.x;
            m2 = ((w00 * t00.y + w01 * t01.y) + w10 * t10.y) + w11 * t11.y;
            float depth;
            if (l.kind == kDirectional)
                depth = ((x - l.pos[0]) * l.dir[0] + (y - l.pos[1]) * l.dir[1]) + (z - l.pos[2]) * l.dir[2];
            else {
                const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
                depth = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
            }
            zz = depth * grcp(l.zfar) - l.zc;
            warp_receiver(l, zz, zw, floor_v);
            var = fmaxf(m2 - m1 * m1, floor_v);
            dd = zw - m1;
            visr = (zw <= m1) ? 1.f : var * grcp(var + dd * dd);
            vis = bleed_reduce(l, visr);
        }
        float ox, oy, oz, olen = 1.f;
        if (l.kind == kDirectional) {
            ox = -l.dir[0]; oy = -l.dir[1]; oz = -l.dir[2];
        } else {
            ox = l.pos[0] - x; oy = l.pos[1] - y; oz = l.pos[2] - z;
            olen = sqrtf((ox * ox + oy * oy) + oz * oz);
            const float rol = grcp(olen);
            ox *= rol; oy *= rol; oz *= rol;
        }
        const float ndo = (nx * ox + ny * oy) + nz * oz;
        const float lam = fmaxf(ndo, 0.f);
        float cone = 1.f;
        if (l.kind == kSpot) {
            const float ca = -((ox * l.dir[0] + oy * l.dir[1]) + oz * l.dir[2]);
            cone = ca >= l.cos_half ? 1.f : 0.f;
        }
        shade += lam * vis * l.intensity * cone;
        const float gvis = srho * lam * l.intensity * cone;
        const float glam = srho * vis * l.intensity * cone;
        const float gndo = ndo > 0.f ? glam : 0.f;
        // from here on only gradient terms are formed: fused multiply-adds
        // (nothing below feeds a forward value or a decision)
        gn[0] = fmaf(gndo, ox, gn[0]); gn[1] = fmaf(gndo, oy, gn[1]); gn[2] = fmaf(gndo, oz, gn[2]);
        const float gox = gndo * nx, goy = gndo * ny, goz = gndo * nz;
        // this pixel's gradient w.r.t. the light frame (M, pos, dir), pulled
        // back to the light parameter through the frame's Jacobian at the end
        float gpos[3] = {0.f, 0.f, 0.f}, gdir[3] = {0.f, 0.f, 0.f};
        float gcx = 0.f, gcy = 0.f, gcw = 0.f;
        if (l.kind == kDirectional) {
            gdir[0] -= gox; gdir[1] -= goy; gdir[2] -= goz;
        } else {
            const float od = fmaf(oz, goz, fmaf(oy, goy, ox * gox));
            const float rl = grcp(olen);
            const float gpx = fmaf(-ox, od, gox) * rl, gpy = fmaf(-oy, od, goy) * rl, gpz = fmaf(-oz, od, goz) * rl;
            gpos[0] += gpx; gpos[1] += gpy; gpos[2] += gpz;
            gx[0] -= gpx; gx[1] -= gpy; gx[2] -= gpz;
        }
        // through the bleeding reduction: slope 1 / (1 - a) on [a, 1], else 0
        const float gvr = l.bleed > 0.f ? (visr >= l.bleed ? gvis / (1.f - l.bleed) : 0.f) : gvis;
        if (inside && gvr != 0.f && zw > m1) {
            const float qd = var + dd * dd;
            float dv_dmu, dv_dvar_raw;
            if (l.warp_c > 0.f) {
                // exponential maps: the squares of var and dd overflow float32
                const float rq = grcp(qd);
                const float tv = var * rq, td = dd * rq;
                dv_dmu = 2.f * tv * td;
                dv_dvar_raw = td * td;
            } else {
                const float rq2 = grcp(qd * qd);
                dv_dmu = 2.f * var * dd * rq2;
                dv_dvar_raw = dd * dd * rq2;
            }
            const bool clamped = m2 - m1 * m1 < floor_v;
            const float dv_dvar = clamped ? 0.f : dv_dvar_raw;
            const float gm1 = gvr * fmaf(-2.f * m1, dv_dvar, dv_dmu);
            const float gm2 = gvr * dv_dvar;
            // d v / d (receiver depth): through d - mu, through the floor when
            // it binds and follows the warp, and through the warp itself
            float dv_dzw = -dv_dmu;
            if (l.warp_c > 0.f) {
                if (clamped) dv_dzw = fmaf(dv_dvar_raw, 2.f * l.min_var * l.warp_c * l.warp_c * zw, dv_dzw);
                dv_dzw *= l.warp_c * zw;
            }
            const float gdepth = gvr * dv_dzw * grcp(l.zfar);
            if (l.kind == kDirectional) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gx[k] = fmaf(gdepth, l.dir[k], gx[k]);
                    gpos[k] = fmaf(-gdepth, l.dir[k], gpos[k]);
                }
                gdir[0] = fmaf(gdepth, x - l.pos[0], gdir[0]);
                gdir[1] = fmaf(gdepth, y - l.pos[1], gdir[1]);
                gdir[2] = fmaf(gdepth, z - l.pos[2], gdir[2]);
            } else {
                const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
                const float dl = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
                const float rd = grcp(dl);
                const float ux_ = ddx * rd, uy_ = ddy * rd, uz_ = ddz * rd;
                gx[0] = fmaf(gdepth, ux_, gx[0]); gx[1] = fmaf(gdepth, uy_, gx[1]); gx[2] = fmaf(gdepth, uz_, gx[2]);
                gpos[0] = fmaf(-gdepth, ux_, gpos[0]); gpos[1] = fmaf(-gdepth, uy_, gpos[1]);
                gpos[2] = fmaf(-gdepth, uz_, gpos[2]);
            }
            // bilinear scatter to the moment maps
            if (DIRECT) {
                float *ga = gmaps + l.fmap_off, *gb = gmaps + l.fmap_off + 1;      // interleaved: texel o at 2 o
                o00 *= 2; o01 *= 2; o10 *= 2; o11 *= 2;
                const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
                atomic_add_f32(ga + o00, gm1 * w00); atomic_add_f32(ga + o01, gm1 * w01);
                atomic_add_f32(ga + o10, gm1 * w10); atomic_add_f32(ga + o11, gm1 * w11);
                atomic_add_f32(gb + o00, gm2 * w00); atomic_add_f32(gb + o01, gm2 * w01);
                atomic_add_f32(gb + o10, gm2 * w10); atomic_add_f32(gb + o11, gm2 * w11);
            } else {
                hits[q] = MapHit{ixs, iys, fx, fy, gm1, gm2};
            }
            // the map position moves with x and with the light camera
            // d m / d(fx, fy): each a lerp of two texel differences
            const float a1 = t01.x - t00.x, b1 = t11.x - t10.x, c1 = t10.x - t00.x, d1 = t11.x - t01.x;
            const float a2 = t01.y - t00.y, b2 = t11.y - t10.y, c2 = t10.y - t00.y, d2 = t11.y - t01.y;
            const float dm1fx = fmaf(fy, b1 - a1, a1), dm1fy = fmaf(fx, d1 - c1, c1);
            const float dm2fx = fmaf(fy, b2 - a2, a2), dm2fy = fmaf(fx, d2 - c2, c2);
            const float hs = 0.5f * S;
            const float gsx = fmaf(gm2, dm2fx, gm1 * dm1fx) * hs;
            const float gsy = fmaf(gm2, dm2fy, gm1 * dm1fy) * hs;
            const float rw = grcp(cw);
            gcx = gsx * rw;
            gcy = -gsy * rw;
            gcw = fmaf(-gsx, cx, gsy * cy) * (rw * rw);
#pragma unroll
            for (int k = 0; k < 3; ++k) gx[k] = fmaf(M[12 + k], gcw, fmaf(M[4 + k], gcy, fmaf(M[k], gcx, gx[k])));
        }
        // dL/dM = (gcx, gcy, 0, gcw) outer [x, 1]; with dL/dpos, dL/ddir through J
        const float *J = jac + (size_t)kJac * render_lights[R.light_begin + q];
        const float xh[4] = {x, y, z, 1.f};
        // per parameter j: sum over rows r in (x, y, w) of g_r (J_r(j) . [x, 1]),
        // plus the position and direction terms
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float u[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int row = r == 0 ? 0 : r == 1 ? 4 : 12;
                u[r] = fmaf(xh[2], J[3 * (row + 2) + j],
                            fmaf(xh[1], J[3 * (row + 1) + j], fmaf(xh[0], J[3 * row + j], J[3 * (row + 3) + j])));
            }
            float a = fmaf(gcw, u[2], fmaf(gcy, u[1], fmaf(gcx, u[0], accl[q][j])));
#pragma unroll
            for (int i = 0; i < 3; ++i) a = fmaf(gdir[i], J[3 * (19 + i) + j], fmaf(gpos[i], J[3 * (16 + i) + j], a));
            accl[q][j] = a;
        }
    }
    // albedo
    for (int c = 0; c < 3; ++c) vals[18 + c] = c < C ? g[c] * shade : 0.f;
    // normal: n = cr / |cr|, cr = e1 x e2
    const float ndg = fmaf(nz, gn[2], fmaf(ny, gn[1], nx * gn[0]));
    const float rn = rn0;
    const float gcr[3] = {fmaf(-nx, ndg, gn[0]) * rn, fmaf(-ny, ndg, gn[1]) * rn, fmaf(-nz, ndg, gn[2]) * rn};
    const float ge1[3] = {fmaf(e2y, gcr[2], -e2z * gcr[1]), fmaf(e2z, gcr[0], -e2x * gcr[2]),
                          fmaf(e2x, gcr[1], -e2y * gcr[0])};
    const float ge2[3] = {fmaf(gcr[1], e1z, -gcr[2] * e1y), fmaf(gcr[2], e1x, -gcr[0] * e1z),
                          fmaf(gcr[0], e1y, -gcr[1] * e1x)};
    // x = sum b_i v_i
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vals[k] = fmaf(b.b0, gx[k], -ge1[k]) - ge2[k];
        vals[3 + k] = fmaf(b.b1, gx[k], ge1[k]);
        vals[6 + k] = fmaf(b.b2, gx[k], ge2[k]);
    }
    const float gb0 = fmaf(gx[2], v0[2], fmaf(gx[1], v0[1], gx[0] * v0[0]));
    const float gb1 = fmaf(gx[2], v1[2], fmaf(gx[1], v1[1], gx[0] * v1[0]));
    const float gb2 = fmaf(gx[2], v2[2], fmaf(gx[1], v2[1], gx[0] * v2[0]));
    float gc[9];
    bary_backward(b, px, py, gb0, gb1, gb2, gc);
#pragma unroll
    for (int k = 0; k < 9; ++k) vals[9 + k] = gc[k];
}

// Bilinear scatter of one light's moment-map gradient from the pixels of a
// tile.  Each wave adds its taps into an LDS window of WIN x WIN texels
// anchored at the smallest tap it touches, then adds the non-zero values of
// the texels its taps can reach (the taps' bounding box, clipped to the
// window) to global memory: lit pixels carry no map gradient, so most
// windows hold a few texels, not WIN x WIN.  Taps outside the window go to
// global memory directly.  Uniform call.
template <int NW, int PPT, int WIN>
__device__ __forceinline__ void map_window_scatter(const MapHit (&hit)[PPT], int S, float *__restrict__ gmap) {
    __shared__ float win[NW][2][WIN * WIN];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int mx = 0x7fffffff, my = 0x7fffffff, Mx = -1, My = -1;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (hit[k].gm1 != 0.f || hit[k].gm2 != 0.f) {
            mx = min(mx, min(max(hit[k].ix, 0), S - 1));
            my = min(my, min(max(hit[k].iy, 0), S - 1));
            Mx = max(Mx, min(max(hit[k].ix + 1, 0), S - 1));
            My = max(My, min(max(hit[k].iy + 1, 0), S - 1));
        }
    mx = wave_min(mx);
    my = wave_min(my);
    Mx = wave_max(Mx);
    My = wave_max(My);
    const bool any = mx != 0x7fffffff;
    // every tap that lands in the window lies in the bounding box
    const int bw = any ? min(Mx - mx + 1, WIN) : 0, bh = any ? min(My - my + 1, WIN) : 0;
    for (int e = lane; e < bw * bh; e += 64) {
        const int o = (e / bw) * WIN + e % bw;
        win[w][0][o] = 0.f;
        win[w][1][o] = 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const MapHit &h = hit[k];
        if (h.gm1 == 0.f && h.gm2 == 0.f) continue;
        const int x0 = min(max(h.ix, 0), S - 1), x1 = min(max(h.ix + 1, 0), S - 1);
        const int y0 = min(max(h.iy, 0), S - 1), y1 = min(max(h.iy + 1, 0), S - 1);
        const float w00 = (1.f - h.fx) * (1.f - h.fy), w01 = h.fx * (1.f - h.fy);
        const float w10 = (1.f - h.fx) * h.fy, w11 = h.fx * h.fy;
        if (x1 - mx < WIN && y1 - my < WIN) {
            float *a = win[w][0], *b = win[w][1];
            const int o00 = (y0 - my) * WIN + (x0 - mx), o01 = (y0 - my) * WIN + (x1 - mx);
            const int o10 = (y1 - my) * WIN + (x0 - mx), o11 = (y1 - my) * WIN + (x1 - mx);
            atomicAdd(a + o00, h.gm1 * w00); atomicAdd(a + o01, h.gm1 * w01);
            atomicAdd(a + o10, h.gm1 * w10); atomicAdd(a + o11, h.gm1 * w11);
            atomicAdd(b + o00, h.gm2 * w00); atomicAdd(b + o01, h.gm2 * w01);
            atomicAdd(b + o10, h.gm2 * w10); atomicAdd(b + o11, h.gm2 * w11);
        } else {
            float *a = gmap, *b = gmap + 1;          // interleaved (m1, m2): texel o at 2 o
            const long long o00 = 2 * ((long long)y0 * S + x0), o01 = 2 * ((long long)y0 * S + x1);
            const long long o10 = 2 * ((long long)y1 * S + x0), o11 = 2 * ((long long)y1 * S + x1);
            atomic_add_f32(a + o00, h.gm1 * w00); atomic_add_f32(a + o01, h.gm1 * w01);
            atomic_add_f32(a + o10, h.gm1 * w10); atomic_add_f32(a + o11, h.gm1 * w11);
            atomic_add_f32(b + o00, h.gm2 * w00); atomic_add_f32(b + o01, h.gm2 * w01);
            atomic_add_f32(b + o10, h.gm2 * w10); atomic_add_f32(b + o11, h.gm2 * w11);
        }
    }
    __syncthreads();
    if (any) {
        for (int e = lane; e < bw * bh; e += 64) {
            const int ex = e % bw, ey = e / bw;
            const long long o = 2 * ((long long)(my + ey) * S + (mx + ex));
            const float a = win[w][0][ey * WIN + ex], b = win[w][1][ey * WIN + ex];
            if (a != 0.f) atomic_add_f32(gmap + o, a);
            if (b != 0.f) atomic_add_f32(gmap + o + 1, b);
        }
    }
    __syncthreads();
}

template <int T, int MAXL>
__device__ __forceinline__ void lookup_backward_body(
    const ViewConst *__restrict__ views, int L, const RenderConst *__restrict__ renders,
    const int *__restrict__ cam_renders_off, const int *__restrict__ cam_renders,
    const int *__restrict__ render_lights, const int *__restrict__ faces, const float *__restrict__ verts,
    const float *__restrict__ albedo, const TriVerts *__restrict__ tv, const unsigned long long *__restrict__ keys,
    const float *__restrict__ maps, const float *__restrict__ gimg0, float *__restrict__ gmaps,
    const TriSetup *__restrict__ setup, const unsigned *__restrict__ tile_start, const unsigned *__restrict__ bins,
    const unsigned *__restrict__ bin_pair, unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums,
    float *__restrict__ gtri, float *__restrict__ part_render, int C, const float *__restrict__ jac,
    const unsigned *__restrict__ pair_off, unsigned capacity) {
    using TS = TileShape<T>;
    // one wave per 8x8 tile: pair rows found from the setup records (wave_pair_sums)
    constexpr bool kWavePairs = T == 8;
    const Blk blk = xcd_block2();
    const int cam = blk.y;
    const ViewConst &cv = views[L + cam];
    const int lt = blk.x;
    if (lt >= cv.tiles_x * cv.tiles_y) return;     // whole workgroup
    const int gt = cv.tile_off + lt;
    BinHead head{};
    if (!kWavePairs) head = bin_head(gt, (int)threadIdx.x, tile_start, bins, bin_pair);
    const int tx = lt % cv.tiles_x, ty = lt / cv.tiles_x;
    const int tid = threadIdx.x;
    int key[TS::PPT], pi[TS::PPT], pj[TS::PPT];
    bool act[TS::PPT], matched[TS::PPT];
    float val[TS::PPT][kNV];
#pragma unroll
    for (int k = 0; k < TS::PPT; ++k) {
        const int l = tid + k * TS::NT;
        pi[k] = tx * T + (l % T);
        pj[k] = ty * T + (l / T);
        const bool in = pi[k] < cv.W && pj[k] < cv.H;
        const unsigned long long kk = in ? keys[cv.pix_off + (long long)pj[k] * cv.W + pi[k]] : kBgKey;
        key[k] = kk == kBgKey ? -1 : (int)(unsigned)kk;
        act[k] = false;
        matched[k] = false;
#pragma unroll
        for (int i = 0; i < kNV; ++i) val[k][i] = 0.f;
    }
    for (int rr = cam_renders_off[cam]; rr < cam_renders_off[cam + 1]; ++rr) {
        const int r = cam_renders[rr];
        const RenderConst &R = renders[r];
        float accl[MAXL][3];
#pragma unroll
        for (int q = 0; q < MAXL; ++q)
#pragma unroll
            for (int i = 0; i < 3; ++i) accl[q][i] = 0.f;
        constexpr bool kDirect = TS::PPT * MAXL > 4;     // register budget for deferred map taps
        MapHit hits[TS::PPT][MAXL];
#pragma unroll
        for (int k = 0; k < TS::PPT; ++k) {
#pragma unroll
            for (int q = 0; q < MAXL; ++q) hits[k][q] = MapHit{0, 0, 0.f, 0.f, 0.f, 0.f};
            if (key[k] < 0) continue;
            const long long p = (long long)pj[k] * cv.W + pi[k];
            float g[3] = {0.f, 0.f, 0.f};
            for (int c = 0; c < C; ++c) g[c] = gimg0[R.img_off + p * C + c];
            if (g[0] == 0.f && g[1] == 0.f && g[2] == 0.f) continue;
            float tmp[kNV];
            lookup_pixel_grad<MAXL, kDirect>(cv, R, views, render_lights, tv, albedo, maps, gmaps,
                                             pi[k], pj[k], key[k], g, C, tmp, accl, hits[k], jac);
            act[k] = true;
#pragma unroll
            for (int i = 0; i < kNV; ++i) val[k][i] += tmp[i];
        }
        if (!kDirect) {
#pragma unroll
            for (int q = 0; q < MAXL; ++q) {
                if (q >= R.light_count) break;
                const ViewConst &l = views[render_lights[R.light_begin + q]];
                MapHit hq[TS::PPT];
#pragma unroll
                for (int k = 0; k < TS::PPT; ++k) hq[k] = hits[k][q];
                map_window_scatter<TS::NW, TS::PPT, (T == 32 ? 32 : 16)>(hq, l.W + 2 * l.fpad, gmaps + l.fmap_off);
            }
        }
        const int ntiles = cv.tiles_x * cv.tiles_y;
#pragma unroll
        for (int q = 0; q < MAXL; ++q) {
            if (q >= R.light_count) break;
            block_sum_store<TS::NW>(accl[q], part_render + R.part_off + ((long long)q * ntiles + lt) * 3);
        }
    }
    if constexpr (kWavePairs)
        wave_pair_sums<T, kNV>(cv, tx, ty, key[0], val[0], act[0], matched[0], setup, pair_off, capacity, pair_flag,
                               pair_sums);
    else
        tile_pair_sums<T, kNV>(cv, head, bins, bin_pair, key, val, act, matched, pair_flag, pair_sums);
    overflow_rows(cv, key, val, act, matched, gtri);
}

template <int T, int MAXL>
__global__ __launch_bounds__(256) void lookup_backward_kernel(
    const ViewConst *__restrict__ views, int L, const RenderConst *__restrict__ renders,
    const int *__restrict__ cam_renders_off, const int *__restrict__ cam_renders,
    const int *__restrict__ render_lights, const int *__restrict__ faces, const float *__restrict__ verts,
    const float *__restrict__ albedo, const TriVerts *__restrict__ tv, const unsigned long long *__restrict__ keys,
    const float *__restrict__ maps, const float *__restrict__ gimg0, float *__restrict__ gmaps,
    const TriSetup *__restrict__ setup, const unsigned *__restrict__ tile_start, const unsigned *__restrict__ bins,
    const unsigned *__restrict__ bin_pair, unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums,
    float *__restrict__ gtri, float *__restrict__ part_render, int C, const float *__restrict__ jac,
    const unsigned *__restrict__ pair_off, unsigned capacity) {
    lookup_backward_body<T, MAXL>(views, L, renders, cam_renders_off, cam_renders, render_lights, faces, verts, albedo, tv, keys, maps, gimg0, gmaps, setup, tile_start, bins, bin_pair, pair_flag, pair_sums, gtri, part_render, C, jac, pair_off, capacity);
}

// One light per render at 8x8 or 16x16 tiles: capped at 128 VGPRs (4 waves
// per SIMD instead of 3) at the cost of a few spilled dwords.
template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void lookup_backward_kernel_1l(
    const ViewConst *__restrict__ views, int L, const RenderConst *__restrict__ renders,
    const int *__restrict__ cam_renders_off, const int *__restrict__ cam_renders,
    const int *__restrict__ render_lights, const int *__restrict__ faces, const float *__restrict__ verts,
    const float *__restrict__ albedo, const TriVerts *__restrict__ tv, const unsigned long long *__restrict__ keys,
    const float *__restrict__ maps, const float *__restrict__ gimg0, float *__restrict__ gmaps,
    const TriSetup *__restrict__ setup, const unsigned *__restrict__ tile_start, const unsigned *__restrict__ bins,
    const unsigned *__restrict__ bin_pair, unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums,
    float *__restrict__ gtri, float *__restrict__ part_render, int C, const float *__restrict__ jac,
    const unsigned *__restrict__ pair_off, unsigned capacity) {
    lookup_backward_body<T, 1>(views, L, renders, cam_renders_off, cam_renders, render_lights, faces, verts, albedo, tv, keys, maps, gimg0, gmaps, setup, tile_start, bins, bin_pair, pair_flag, pair_sums, gtri, part_render, C, jac, pair_off, capacity);
}

// ----------------------------------------------------------------------------- light smoothing^T + resolve^T

template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void light_backward_kernel(
    const ViewConst *__restrict__ views, const TriSetup *__restrict__ setup, const int *__restrict__ faces,
    const unsigned char *__restrict__ silm, const float *__restrict__ verts, const TriVerts *__restrict__ tv,
    const unsigned long long *__restrict__ keys, const unsigned char *__restrict__ aa_flag,
    const float *__restrict__ F0, const float *__restrict__ gF1, float4 *__restrict__ gclip, const unsigned *__restrict__ tile_start, const unsigned *__restrict__ bins,
    const unsigned *__restrict__ bin_pair, unsigned char *__restrict__ pair_flag, float *__restrict__ pair_sums,
    float *__restrict__ gtri, float *__restrict__ part_light, const float *__restrict__ jac,
    const unsigned *__restrict__ pair_off, unsigned capacity) {
    using TS = TileShape<T>;
    // one wave per 8x8 tile: pair rows found from the setup records (wave_pair_sums)
    constexpr bool kWavePairs = T == 8;
    const Blk blk = xcd_block2();
    const int lidx = blk.y;
    const ViewConst &l = views[lidx];
    const int S = l.W;
    const long long plane = (long long)S * S;
    const int lt = blk.x;
    if (lt >= l.tiles_x * l.tiles_y) return;     // whole workgroup
    const int gt = l.tile_off + lt;
    BinHead head{};
    if (!kWavePairs) head = bin_head(gt, (int)threadIdx.x, tile_start, bins, bin_pair);
    const int tx = lt % l.tiles_x, ty = lt / l.tiles_x;
    const unsigned long long *kv = keys + l.pix_off;
    const float *f0a = F0 + l.map_off, *f0b = F0 + l.map_off + plane;
    const float *ga = gF1 + l.map_off, *gbp = gF1 + l.map_off + plane;
    float accl[6] = {0, 0, 0, 0, 0, 0};
    int key[TS::PPT];
    bool act[TS::PPT], matched[TS::PPT];
    float val[TS::PPT][18];
#pragma unroll
    for (int k = 0; k < TS::PPT; ++k) {
        const int lix = threadIdx.x + k * TS::NT;
        const int i = tx * T + (lix % T), j = ty * T + (lix / T);
        const bool in = i < S && j < S;
        const int pp = in ? j * S + i : 0;
        const unsigned long long ks = kv[pp];
        key[k] = (in && ks != kBgKey) ? (int)(unsigned)ks : -1;
        matched[k] = false;
#pragma unroll
        for (int q = 0; q < 18; ++q) val[k][q] = 0.f;
        float g0 = in ? ga[pp] : 0.f, g1 = in ? gbp[pp] : 0.f;
        // texels the forward found without candidate pairs skip the smoothing terms
        if (in && l.antialias && l.nfaces > 0 && aa_flag[l.pix_off + pp]) {
            const float gs0 = g0, gs1 = g1;
            const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
            // the four neighbour keys, then their silhouette bytes, each batch
            // loaded together; a candidate neighbour's map values and
            // gradients are requested with its triangle's records
            const AANeighbours nb = aa_neighbours(l, kv, silm, ks, i, j);
            const bool any = nb.cand[0] || nb.cand[1] || nb.cand[2] || nb.cand[3];
            const float fs0 = any ? f0a[pp] : 0.f, fs1 = any ? f0b[pp] : 0.f;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if (!nb.cand[d]) continue;
                const int q = nb.q[d];
                const float fn0 = f0a[q], fn1 = f0b[q], gn0 = ga[q], gn1 = gbp[q];
                const int in_ = i + di[d], jn = j + dj[d];
                const unsigned long long kn = nb.kn[d];
                bool self_front;
                AAPair pr;
                if (!aa_eval<true>(l, setup, faces, silm, verts, ks, kn, i, j, in_, jn, d < 2, self_front, pr)) continue;
                const bool self_recv = (pr.recv == 1) != self_front;
                if (self_recv) {
                    g0 -= pr.w * gs0;
                    g1 -= pr.w * gs1;
                    double galpha = (double)gs0 * (fn0 - fs0) + (double)gs1 * (fn1 - fs1);
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
                    g0 += pr.w * gn0;
                    g1 += pr.w * gn1;
                }
            }
        }
        // resolve^T: F0 = (z, z^2), z = d(x) / far
        act[k] = key[k] >= 0 && (g0 != 0.f || g1 != 0.f);
        if (act[k]) {
            const TriVerts r = tv[l.face_off + key[k]];
            const float v0[3] = {r.a.x, r.a.y, r.a.z}, v1[3] = {r.a.w, r.b.x, r.b.y}, v2[3] = {r.b.z, r.b.w, r.c.x};
            const float4 c0 = clip_of(l.M, v0[0], v0[1], v0[2]), c1 = clip_of(l.M, v1[0], v1[1], v1[2]),
                         c2 = clip_of(l.M, v2[0], v2[1], v2[2]);
            const float px = ndc_c(i, S), py = -ndc_c(j, S);
            const BaryFull b = bary_full(c0, c1, c2, px, py);
            const float x = (b.b0 * v0[0] + b.b1 * v1[0]) + b.b2 * v2[0];
            const float y = (b.b0 * v0[1] + b.b1 * v1[1]) + b.b2 * v2[1];
            const float z = (b.b0 * v0[2] + b.b1 * v1[2]) + b.b2 * v2[2];
            // F0 = (f, f^2), f = z, or exp(c z) for exponential maps
            const float gz = l.warp_c > 0.f ? l.warp_c * f0a[pp] * (g0 + 2.f * f0a[pp] * g1) : g0 + 2.f * f0a[pp] * g1;
            const float gdepth = gz * grcp(l.zfar);
            float gx[3];
            if (l.kind == kDirectional) {
                gx[0] = gdepth * l.dir[0]; gx[1] = gdepth * l.dir[1]; gx[2] = gdepth * l.dir[2];
                accl[0] -= gx[0]; accl[1] -= gx[1]; accl[2] -= gx[2];
                accl[3] += gdepth * (x - l.pos[0]); accl[4] += gdepth * (y - l.pos[1]); accl[5] += gdepth * (z - l.pos[2]);
            } else {
                const float ddx = x - l.pos[0], ddy = y - l.pos[1], ddz = z - l.pos[2];
                const float dl = sqrtf((ddx * ddx + ddy * ddy) + ddz * ddz);
                const float inv = gdepth * grcp(dl);
                gx[0] = ddx * inv; gx[1] = ddy * inv; gx[2] = ddz * inv;
                accl[0] -= gx[0]; accl[1] -= gx[1]; accl[2] -= gx[2];
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                val[k][q] = b.b0 * gx[q];
                val[k][3 + q] = b.b1 * gx[q];
                val[k][6 + q] = b.b2 * gx[q];
            }
            const float gb0 = (gx[0] * v0[0] + gx[1] * v0[1]) + gx[2] * v0[2];
            const float gb1 = (gx[0] * v1[0] + gx[1] * v1[1]) + gx[2] * v1[2];
            const float gb2 = (gx[0] * v2[0] + gx[1] * v2[1]) + gx[2] * v2[2];
            float gc[9];
            bary_backward(b, px, py, gb0, gb1, gb2, gc);
#pragma unroll
            for (int q = 0; q < 9; ++q) val[k][9 + q] = gc[q];
        }
    }
    // (pos, dir) terms pulled back to the light parameter
    const float *J = jac + (size_t)kJac * lidx;
    float gpar[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) a += accl[i] * J[3 * (16 + i) + j] + accl[3 + i] * J[3 * (19 + i) + j];
        gpar[j] = a;
    }
    block_sum_store<TS::NW>(gpar, part_light + ((long long)l.part_off + lt) * 3);
    if constexpr (kWavePairs)
        wave_pair_sums<T, 18>(l, tx, ty, key[0], val[0], act[0], matched[0], setup, pair_off, capacity, pair_flag,
                              pair_sums);
    else
        tile_pair_sums<T, 18>(l, head, bins, bin_pair, key, val, act, matched, pair_flag, pair_sums);
    overflow_rows(l, key, val, act, matched, gtri);
}

// ----------------------------------------------------------------------------- gathers

// Zero the gtri rows of triangles that overflowed the bins (their pixels are
// added there with atomics) and reset the big-triangle list.
__global__ void overflow_rows_zero_kernel(const unsigned *__restrict__ list, const DevCounters *counters,
                                          float *__restrict__ gtri) {
    const unsigned n = counters->overflow_list_len;
    for (unsigned o = blockIdx.x; o < n; o += gridDim.x)
        for (int i = threadIdx.x; i < kGtriStride; i += blockDim.x) gtri[(size_t)list[o] * kGtriStride + i] = 0.f;
}

constexpr unsigned kBigPairs = 16;

// gtri[i] = sum of triangle i's pair slots (triangles with many pairs are listed for the big pass).
__global__ void pair_reduce_kernel(const unsigned *__restrict__ pair_off, int ntri, unsigned capacity,
                                   const unsigned char *__restrict__ pair_flag,
                                   const float *__restrict__ pair_sums, float *__restrict__ gtri,
                                   unsigned *__restrict__ big_list, unsigned *__restrict__ big_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntri) return;
    const unsigned a = pair_off[i], b = pair_off[i + 1];
    if (b > capacity && b > a) return;            // overflowed: rows filled by atomics
    if (b - a > kBigPairs) {
        big_list[atomicAdd(big_count, 1u)] = (unsigned)i;
        return;
    }
    float acc[kNV];
#pragma unroll
    for (int q = 0; q < kNV; ++q) acc[q] = 0.f;
    for (unsigned p = a; p < b; ++p)
        if (pair_flag[p])
#pragma unroll
            for (int q = 0; q < kNV; ++q) acc[q] += pair_sums[(size_t)p * kNV + q];
#pragma unroll
    for (int q = 0; q < kNV; ++q) gtri[(size_t)i * kGtriStride + gtri_slot(q)] = acc[q];
}

__global__ __launch_bounds__(256) void big_pair_reduce_kernel(const unsigned *__restrict__ pair_off,
                                                              const unsigned char *__restrict__ pair_flag,
                                                              const float *__restrict__ pair_sums,
                                                              float *__restrict__ gtri,
                                                              const unsigned *__restrict__ big_list,
                                                              const unsigned *__restrict__ big_count) {
    const unsigned n = *big_count;
    for (unsigned o = blockIdx.x; o < n; o += gridDim.x) {
        const unsigned i = big_list[o];
        const unsigned a = pair_off[i], b = pair_off[i + 1];
        float acc[kNV];
#pragma unroll
        for (int q = 0; q < kNV; ++q) acc[q] = 0.f;
        for (unsigned p = a + threadIdx.x; p < b; p += blockDim.x)
            if (pair_flag[p])
#pragma unroll
                for (int q = 0; q < kNV; ++q) acc[q] += pair_sums[(size_t)p * kNV + q];
        block_sum_store<4>(acc, gtri + (size_t)i * kGtriStride, [](int q) { return gtri_slot(q); });
        __syncthreads();
    }
}

// Albedo gradient per face: sum over the camera views of its scene.  Run by
// the workgroups of the vertex gather's launch past its vertex blocks
// (column bx of scene b).
__device__ __forceinline__ void albedo_gather_block(const ViewConst *__restrict__ views, int L, int b, int bx,
                                                    const int *__restrict__ scene_face_off,
                                                    const int *__restrict__ scene_views_off,
                                                    const int *__restrict__ scene_views,
                                                    const float *__restrict__ gtri, float *__restrict__ galbedo,
                                                    int C) {
    const int fl = bx * blockDim.x + threadIdx.x;
    if (fl >= scene_face_off[b + 1] - scene_face_off[b]) return;
    float acc[3] = {0, 0, 0};
    for (int s = scene_views_off[b]; s < scene_views_off[b + 1]; ++s) {
        const int vi = scene_views[s];
        if (vi < L) continue;
        const float *row = gtri + (size_t)(views[vi].setup_off + fl) * kGtriStride;
        for (int c = 0; c < C; ++c) acc[c] += row[gtri_slot(18 + c)];
    }
    for (int c = 0; c < C; ++c) galbedo[(size_t)(scene_face_off[b] + fl) * C + c] = acc[c];
}

// Per vertex: sum its triangle corners' terms over every view of its scene,
// add the silhouette clip terms, map clip terms through M^T; per light view
// the workgroup's share of dL/dM is written for glight_reduce.
__global__ __launch_bounds__(256) void vertex_gather_kernel(
    const ViewConst *__restrict__ views, int L, const int *__restrict__ scene_vert_off,
    const int *__restrict__ scene_views_off, const int *__restrict__ scene_views, const int *__restrict__ vc_off,
    const int *__restrict__ vc_list, const float *__restrict__ verts, const float *__restrict__ gtri,
    const float *__restrict__ zero_rec, const float4 *__restrict__ gclip, float *__restrict__ gverts,
    float *__restrict__ part_gm, const float *__restrict__ jac, int vx, const int *__restrict__ scene_face_off,
    float *__restrict__ galbedo, int C) {
    const int b = blockIdx.y;
    if ((int)blockIdx.x >= vx) {                               // the albedo gather's workgroups
        albedo_gather_block(views, L, b, (int)blockIdx.x - vx, scene_face_off, scene_views_off, scene_views, gtri,
                            galbedo, C);
        return;
    }
    const int nv = scene_vert_off[b + 1] - scene_vert_off[b];
    if ((int)(blockIdx.x * blockDim.x) >= nv) return;        // whole workgroup
    const int vl = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = vl < nv;
    const int gv_idx = scene_vert_off[b] + (in ? vl : 0);
    float x[3] = {0, 0, 0};
    if (in)
        for (int k = 0; k < 3; ++k) x[k] = verts[3 * (size_t)gv_idx + k];
    float gv[3] = {0, 0, 0};
    const int c0 = in ? vc_off[gv_idx] : 0, c1 = in ? vc_off[gv_idx + 1] : 0;
    // the first eight corners' indices, loaded once for every view (a vertex
    // of a closed mesh has about six)
    constexpr int kHeld = 8;
    int eh[kHeld];
#pragma unroll
    for (int k = 0; k < kHeld; ++k) eh[k] = c0 + k < c1 ? vc_list[c0 + k] : -1;
    for (int s = scene_views_off[b]; s < scene_views_off[b + 1]; ++s) {
        const int vi = scene_views[s];
        const ViewConst &v = views[vi];
        const int soff = v.setup_off;
        float gc[3] = {0, 0, 0};
        // Every slot loads a record, absent corners an all-zero one
        // (zero_rec), so that no load sits behind a branch and the sums add
        // the same terms in the same order.  Corners past the held ones go
        // sixteen at a time, the next sixteen indices loaded with the current
        // records: a vertex of high valence (the pole of a UV sphere has one
        // corner per longitude) waits for one load per sixteen corners.
        constexpr int kChunk = 16;
        const float4 ga = gclip[v.clip_off + (in ? vl : 0)];     // silhouette terms, issued early
        int e[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) e[k] = c0 + kHeld + k < c1 ? vc_list[c0 + kHeld + k] : -1;
        {
            // the held corners' records: eight loads in flight
            float4 a[kHeld];
            float2 bb[kHeld];
#pragma unroll
            for (int k = 0; k < kHeld; ++k) {
                // the corner's record: world x y z, clip x | clip y w
                const float *rec =
                    eh[k] >= 0 ? gtri + (size_t)(soff + (eh[k] >> 2)) * kGtriStride + (eh[k] & 3) * 8 : zero_rec;
                a[k] = *(const float4 *)rec;
                bb[k] = *(const float2 *)(rec + 4);
            }
#pragma unroll
            for (int k = 0; k < kHeld; ++k) {
                gv[0] += a[k].x; gv[1] += a[k].y; gv[2] += a[k].z;
                gc[0] += a[k].w; gc[1] += bb[k].x; gc[2] += bb[k].y;
            }
        }
        for (int c = c0 + kHeld; c < c1; c += kChunk) {
            float4 a[kChunk];
            float2 b[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                const float *rec =
                    e[k] >= 0 ? gtri + (size_t)(soff + (e[k] >> 2)) * kGtriStride + (e[k] & 3) * 8 : zero_rec;
                a[k] = *(const float4 *)rec;
                b[k] = *(const float2 *)(rec + 4);
            }
#pragma unroll
            for (int k = 0; k < kChunk; ++k) e[k] = c + kChunk + k < c1 ? vc_list[c + kChunk + k] : -1;
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                gv[0] += a[k].x; gv[1] += a[k].y; gv[2] += a[k].z;
                gc[0] += a[k].w; gc[1] += b[k].x; gc[2] += b[k].y;
            }
        }
        if (in) {
            gc[0] += ga.x; gc[1] += ga.y; gc[2] += ga.w;
        }
        const float *M = v.M;
#pragma unroll
        for (int k = 0; k < 3; ++k) gv[k] += (M[k] * gc[0] + M[4 + k] * gc[1]) + M[12 + k] * gc[2];
        if (vi < L) {
            // dL/dM = (gc_x, gc_y, 0, gc_w) outer [x, 1], pulled back to the light parameter
            const float xh[4] = {x[0], x[1], x[2], in ? 1.f : 0.f};
            const float *J = jac + (size_t)kJac * vi;
            float gp[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float a = 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    a += xh[k] * ((gc[0] * J[3 * k + j] + gc[1] * J[3 * (4 + k) + j]) + gc[2] * J[3 * (12 + k) + j]);
                gp[j] = a;
            }
            block_sum_store<4>(gp, part_gm + ((long long)v.part_gm_off + blockIdx.x) * 3);
        }
    }
    if (in)
        for (int k = 0; k < 3; ++k) gverts[3 * (size_t)gv_idx + k] = gv[k];
}

// glight[l] = sum of every partial written for light l (vertex blocks, light
// tiles, and the tiles of each render that uses it), in two passes so that a
// few lights with many partials still fill the GPU: kGlightBlocks workgroups
// per light each sum a strided share, then one thread per light adds their
// results in a fixed order (deterministic, no atomics).
__global__ __launch_bounds__(256) void glight_partial_kernel(const ViewConst *__restrict__ views,
                                                             const RenderConst *__restrict__ renders,
                                                             const int *__restrict__ light_renders_off,
                                                             const int *__restrict__ light_renders,
                                                             const float *__restrict__ part_gm,
                                                             const float *__restrict__ part_light,
                                                             const float *__restrict__ part_render,
                                                             float *__restrict__ gl_part) {
    const int l = blockIdx.y;
    const ViewConst &v = views[l];
    const int first = blockIdx.x * blockDim.x + threadIdx.x, step = kGlightBlocks * blockDim.x;
    float acc[3] = {0.f, 0.f, 0.f};
    const int nvb = (v.nverts + 255) / 256;
    for (int q = first; q < nvb; q += step)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += part_gm[((long long)v.part_gm_off + q) * 3 + k];
    const int nlt = v.tiles_x * v.tiles_y;
    for (int q = first; q < nlt; q += step)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += part_light[((long long)v.part_off + q) * 3 + k];
    for (int e = light_renders_off[l]; e < light_renders_off[l + 1]; ++e) {
        const int r = light_renders[e] >> 5, slot = light_renders[e] & 31;
        const RenderConst &R = renders[r];
        const ViewConst &cv = views[R.camera_view];
        const int nct = cv.tiles_x * cv.tiles_y;
        for (int q = first; q < nct; q += step)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k] += part_render[R.part_off + ((long long)slot * nct + q) * 3 + k];
    }
    block_sum_store<4>(acc, gl_part + ((long long)l * kGlightBlocks + blockIdx.x) * 3);
}

__global__ void glight_final_kernel(const float *__restrict__ gl_part, int L, float *__restrict__ gparams) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * L) return;
    const int l = t / 3, k = t % 3;
    float a = 0.f;
    for (int b = 0; b < kGlightBlocks; ++b) a += gl_part[((long long)l * kGlightBlocks + b) * 3 + k];
    gparams[t] = a;
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
                                     const TriSetup *setup, const int *faces, const unsigned char *silm, const float *verts,
                                     const unsigned long long *keys, const unsigned char *aa_flag, const float *img0,
                                     const float *gimg, float *gimg0, float4 *gclip, int C, hipStream_t s) {
    if (R == 0) return hipSuccess;
    const dim3 grid((max_pix + 255) / 256, R);
    if (C == 1)
        hipLaunchKernelGGL(aa_camera_backward_kernel<1>, grid, dim3(256), 0, s, views, renders, setup, faces, silm,
                           verts, keys, aa_flag, img0, gimg, gimg0, gclip);
    else
        hipLaunchKernelGGL(aa_camera_backward_kernel<3>, grid, dim3(256), 0, s, views, renders, setup, faces, silm,
                           verts, keys, aa_flag, img0, gimg, gimg0, gclip);
    return hipGetLastError();
}

hipError_t launch_lookup_backward(int tile, const ViewConst *views, int L, int Cm, int max_tiles, int max_lights,
                                  const RenderConst *renders, const int *cam_renders_off, const int *cam_renders,
                                  const int *render_lights, const int *faces, const float *verts, const float *albedo,
                                  const TriVerts *tv, const unsigned long long *keys, const float *maps,
                                  const float *gimg0, float *gmaps, const TriSetup *setup, const unsigned *tile_start,
                                  const unsigned *bins, const unsigned *bin_pair, unsigned char *pair_flag,
                                  float *pair_sums, float *gtri, float *part_render, int C, const float *jac,
                                  const unsigned *pair_off, unsigned capacity, hipStream_t s) {
    if (Cm == 0 || max_tiles == 0) return hipSuccess;
    const dim3 grid(max_tiles, Cm);
#define DSM_LB1(TT)                                                                                                 \
    hipLaunchKernelGGL((lookup_backward_kernel_1l<TT>), grid, dim3(TileShape<TT>::NT), 0, s, views, L, renders,     \
                       cam_renders_off, cam_renders, render_lights, faces, verts, albedo, tv, keys, maps, gimg0,     \
                       gmaps, setup, tile_start, bins, bin_pair, pair_flag, pair_sums, gtri, part_render, C, jac, \
                       pair_off, capacity)
#define DSM_LB(TT, ML)                                                                                              \
    hipLaunchKernelGGL((lookup_backward_kernel<TT, ML>), grid, dim3(TileShape<TT>::NT), 0, s, views, L, renders,   \
                       cam_renders_off, cam_renders, render_lights, faces, verts, albedo, tv, keys, maps, gimg0,     \
                       gmaps, setup, tile_start, bins, bin_pair, pair_flag, pair_sums, gtri, part_render, C, jac, \
                       pair_off, capacity)
#define DSM_LB_T(TT)                                                  \
    if (max_lights <= 1 && TT <= 16) DSM_LB1(TT);                     \
    else if (max_lights <= 1) DSM_LB(TT, 1);                          \
    else if (max_lights <= 4) DSM_LB(TT, 4);                          \
    else DSM_LB(TT, DSM_MAX_LIGHTS_PER_RENDER)
    if (tile == 8) { DSM_LB_T(8); }
    else if (tile == 16) { DSM_LB_T(16); }
    else { DSM_LB_T(32); }
#undef DSM_LB_T
#undef DSM_LB
#undef DSM_LB1
    return hipGetLastError();
}

hipError_t launch_light_backward(int tile, const ViewConst *views, int L, int max_tiles, const TriSetup *setup,
                                 const int *faces, const unsigned char *silm, const float *verts, const TriVerts *tv,
                                 const unsigned long long *keys, const unsigned char *aa_flag, const float *F0, const float *gF1,
                                 float4 *gclip,
                                 const unsigned *tile_start, const unsigned *bins, const unsigned *bin_pair,
                                 unsigned char *pair_flag, float *pair_sums, float *gtri, float *part_light,
                                 const float *jac, const unsigned *pair_off, unsigned capacity, hipStream_t s) {
    if (L == 0 || max_tiles == 0) return hipSuccess;
    const dim3 grid(max_tiles, L);
#define DSM_LIB(TT)                                                                                                  \
    hipLaunchKernelGGL((light_backward_kernel<TT>), grid, dim3(TileShape<TT>::NT), 0, s, views, setup, faces, silm,  \
                       verts, tv, keys, aa_flag, F0, gF1, gclip, tile_start, bins, bin_pair, pair_flag, pair_sums, \
                       gtri, part_light, jac, pair_off, capacity)
    if (tile == 8) DSM_LIB(8);
    else if (tile == 16) DSM_LIB(16);
    else DSM_LIB(32);
#undef DSM_LIB
    return hipGetLastError();
}

hipError_t launch_vertex_gradients(const ViewConst *views, int L, int B, int max_verts, int max_faces, int ntri,
                                   unsigned capacity, const int *scene_vert_off, const int *scene_face_off,
                                   const int *scene_views_off, const int *scene_views, const int *vc_off,
                                   const int *vc_list, const unsigned *pair_off, const unsigned char *pair_flag,
                                   const float *pair_sums, float *gtri, const float *zero_rec,
                                   unsigned *big_list, unsigned *big_count, const float *verts, const float4 *gclip,
                                   float *gverts, float *part_gm, float *galbedo, int C, const float *jac, hipStream_t s) {
    if (ntri > 0) {
        hipLaunchKernelGGL(pair_reduce_kernel, dim3((ntri + 255) / 256), dim3(256), 0, s, pair_off, ntri, capacity,
                           pair_flag, pair_sums, gtri, big_list, big_count);
        hipLaunchKernelGGL(big_pair_reduce_kernel, dim3(512), dim3(256), 0, s, pair_off, pair_flag, pair_sums, gtri,
                           big_list,
                           (const unsigned *)big_count);
    }
    // one launch: the vertex gather's workgroups, then the albedo gather's
    const int vx = (max_verts + 255) / 256, fx = (galbedo && max_faces > 0) ? (max_faces + 255) / 256 : 0;
    if (B > 0 && vx + fx > 0)
        hipLaunchKernelGGL(vertex_gather_kernel, dim3(vx + fx, B), dim3(256), 0, s, views, L, scene_vert_off,
                           scene_views_off, scene_views, vc_off, vc_list, verts, gtri, zero_rec, gclip, gverts,
                           part_gm, jac, vx, scene_face_off, galbedo, C);
    return hipGetLastError();
}

hipError_t launch_overflow_rows_zero(const unsigned *list, const DevCounters *counters, float *gtri, hipStream_t s) {
    hipLaunchKernelGGL(overflow_rows_zero_kernel, dim3(256), dim3(64), 0, s, list, counters, gtri);
    return hipGetLastError();
}

hipError_t launch_glight_reduce(const ViewConst *views, int L, const RenderConst *renders,
                                const int *light_renders_off, const int *light_renders, const float *part_gm,
                                const float *part_light, const float *part_render, float *gl_part, float *gparams,
                                hipStream_t s) {
    if (L == 0) return hipSuccess;
    hipLaunchKernelGGL(glight_partial_kernel, dim3(kGlightBlocks, L), dim3(256), 0, s, views, renders,
                       light_renders_off, light_renders, part_gm, part_light, part_render, gl_part);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(glight_final_kernel, dim3((3 * L + 255) / 256), dim3(256), 0, s, gl_part, L, gparams);
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
