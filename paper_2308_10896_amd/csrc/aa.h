// Edge antialiasing at primitive borders, shared by the light view (the
// smoothed shadow map f~, f^2~ of Sec. 4, which Alg. 1 filters) and the
// camera view (the shaded image).
//
// For two horizontally or vertically adjacent samples owned by different
// triangles: the sample with the smaller depth|id key is the front sample F,
// the other O.  The front triangle's edges whose edge function is negative at
// O are exit edges; the first one crossed on the way F -> O (smallest
// float32 ratio E(F) / (E(F) - E(O)), lower edge index on ties) is taken.
// The pair is smoothed only if that edge is a silhouette in the view
// (boundary, non-manifold, or neighbour of opposite facing; precomputed per
// triangle as TriSetup::sil) and, so that
// each edge is handled in one direction only, |dY| > |dX| for horizontal
// pairs and |dY| <= |dX| for vertical ones.  The continuous crossing
// alpha = E(F) / (E(F) - E(O)) is computed from the unsnapped vertex
// positions (float64): alpha > 1/2 moves O toward F by (alpha - 1/2),
// otherwise F moves toward O by (1/2 - alpha).  Deltas use pre-smoothing
// values; every sample gathers the deltas of its four pairs.
#pragma once

#include "dsm_internal.h"

namespace dsm {

__device__ __forceinline__ long long aa_edge_fn(int xa, int ya, int xb, int yb, int px, int py) {
    return (long long)(xb - xa) * (py - ya) - (long long)(yb - ya) * (px - xa);
}

struct AAPair {
    int recv;          // 0: receiver is the front sample, 1: the other sample
    float w;           // blend weight |alpha - 1/2|
    int va, vb;        // scene-local vertex indices of the chosen edge
    double alpha;      // continuous crossing
    // partial derivatives of alpha w.r.t. the clip coordinates (x, y, w) of va and vb
    double dax, day, daw, dbx, dby, dbw;
};

__device__ __forceinline__ int orig_slot(int s, bool swapped) { return swapped ? (s == 0 ? 0 : 3 - s) : s; }

__device__ __forceinline__ void clip_f64(const float *M, const float *p, double c[4]) {
    const double x = p[0], y = p[1], z = p[2];
    for (int r = 0; r < 4; ++r) c[r] = ((double)M[4 * r] * x + (double)M[4 * r + 1] * y) + (double)M[4 * r + 2] * z +
                                     (double)M[4 * r + 3];
}

// Evaluate the pair (self sample s, neighbour sample n).  Returns false when
// the pair is not smoothed.  keys: this view's key array base.
template <bool WANT_GRAD>
__device__ __forceinline__ bool aa_eval(const ViewConst &v, const TriSetup *__restrict__ setup,
                                        const int *__restrict__ faces, const unsigned char *__restrict__ silm,
                                        const float *__restrict__ verts, unsigned long long ks,
                                        unsigned long long kn, int is, int js, int in_, int jn, bool horiz,
                                        bool &self_is_front, AAPair &out) {
    const unsigned ts = (unsigned)ks, tn = (unsigned)kn;
    if (ts == tn) return false;
    self_is_front = ks < kn;
    const unsigned t = self_is_front ? ts : tn;
    const int fi = self_is_front ? is : in_, fj = self_is_front ? js : jn;
    const int oi = self_is_front ? in_ : is, oj = self_is_front ? jn : js;
    const unsigned sm = silm[v.setup_off + t];
    if (sm == 0) return false;                       // no silhouette edge to cross
    const TriSetup &S = setup[v.setup_off + t];
    // the triangle's three vertex indices, loaded with its setup record so
    // that the vertex fetch below is the only load that waits on the edge choice
    const size_t fidx = (size_t)(v.face_off + (int)t);
    const int fv[3] = {faces[3 * fidx], faces[3 * fidx + 1], faces[3 * fidx + 2]};
    const int fX = fi * kSub + kSub / 2, fY = fj * kSub + kSub / 2;
    const int oX = oi * kSub + kSub / 2, oY = oj * kSub + kSub / 2;
    float best = 0.f;
    int ebest = -1;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int a = (e + 1) % 3, b = (e + 2) % 3;
        const long long eo = aa_edge_fn(S.X[a], S.Y[a], S.X[b], S.Y[b], oX, oY);
        if (eo < 0) {
            const long long ef = aa_edge_fn(S.X[a], S.Y[a], S.X[b], S.Y[b], fX, fY);
            const float r = (float)(double)ef / (float)(double)(ef - eo);
            if (ebest < 0 || r < best) { best = r; ebest = e; }
        }
    }
    if (ebest < 0) return false;
    const int a = (ebest + 1) % 3, b = (ebest + 2) % 3;
    const int dX = S.X[b] - S.X[a], dY = S.Y[b] - S.Y[a];
    const bool dir_ok = horiz ? (abs(dY) > abs(dX)) : (abs(dY) <= abs(dX));
    if (!dir_ok) return false;
    if (!((sm >> ebest) & 1)) return false;
    const bool sw = S.swapped != 0;
    const int oa = orig_slot(a, sw), ob = orig_slot(b, sw);
    out.va = oa == 0 ? fv[0] : oa == 1 ? fv[1] : fv[2];
    out.vb = ob == 0 ? fv[0] : ob == 1 ? fv[1] : fv[2];
    double ca[4], cb[4];
    clip_f64(v.M, verts + 3 * (size_t)(v.vert_off + out.va), ca);
    clip_f64(v.M, verts + 3 * (size_t)(v.vert_off + out.vb), cb);
    const double hw = 0.5 * v.W, hh = 0.5 * v.H;
    const double xa = (ca[0] / ca[3] + 1.0) * hw, ya = (1.0 - ca[1] / ca[3]) * hh;
    const double xb = (cb[0] / cb[3] + 1.0) * hw, yb = (1.0 - cb[1] / cb[3]) * hh;
    const double pfx = fi + 0.5, pfy = fj + 0.5, pox = oi + 0.5, poy = oj + 0.5;
    const double eF = (xb - xa) * (pfy - ya) - (yb - ya) * (pfx - xa);
    const double eO = (xb - xa) * (poy - ya) - (yb - ya) * (pox - xa);
    const double D = eF - eO;
    const double alpha = eF / D;
    out.alpha = alpha;
    if (alpha > 0.5) {
        out.recv = 1;
        out.w = (float)(alpha - 0.5);
    } else {
        out.recv = 0;
        out.w = (float)(0.5 - alpha);
    }
    if (WANT_GRAD) {
        const double dF = -eO / (D * D), dO = eF / (D * D);    // d alpha / d eF, d alpha / d eO
        // d E(p) / d (xa, ya, xb, yb)
        const double gxa = dF * (yb - pfy) + dO * (yb - poy);
        const double gya = dF * (pfx - xb) + dO * (pox - xb);
        const double gxb = dF * (pfy - ya) + dO * (poy - ya);
        const double gyb = -dF * (pfx - xa) - dO * (pox - xa);
        // screen coordinates to clip (x, y, w)
        out.dax = gxa * hw / ca[3];
        out.day = -gya * hh / ca[3];
        out.daw = -gxa * hw * ca[0] / (ca[3] * ca[3]) + gya * hh * ca[1] / (ca[3] * ca[3]);
        out.dbx = gxb * hw / cb[3];
        out.dby = -gyb * hh / cb[3];
        out.dbw = -gxb * hw * cb[0] / (cb[3] * cb[3]) + gyb * hh * cb[1] / (cb[3] * cb[3]);
    }
    return true;
}

// The four neighbours of sample (i, j) (order -x, +x, -y, +y) and which of
// the pairs can be smoothed at all: different triangles and a front
// triangle with a silhouette edge in this view.  All neighbour keys are
// loaded together, then all silhouette bytes, so a sample waits for two
// dependent loads instead of two per neighbour (one when no lane of its
// wave has a differing neighbour).  The view must have faces.
struct AANeighbours {
    unsigned long long kn[4];
    int q[4];
    bool cand[4];
};

__device__ __forceinline__ AANeighbours aa_neighbours(const ViewConst &v, const unsigned long long *__restrict__ kv,
                                                      const unsigned char *__restrict__ silm, unsigned long long ks,
                                                      int i, int j) {
    AANeighbours n;
    bool inb[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int in_ = i + (d == 0 ? -1 : d == 1 ? 1 : 0), jn = j + (d == 2 ? -1 : d == 3 ? 1 : 0);
        inb[d] = in_ >= 0 && in_ < v.W && jn >= 0 && jn < v.H;
        n.q[d] = inb[d] ? jn * v.W + in_ : j * v.W + i;
        n.kn[d] = kv[n.q[d]];
    }
    bool differ[4], any = false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        differ[d] = inb[d] && (unsigned)n.kn[d] != (unsigned)ks;
        any = any || differ[d];
        n.cand[d] = false;
    }
    // a wave inside one triangle (most of a ground plane) waits for no
    // silhouette byte at all
    if (__ballot(any) != 0ull) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const unsigned front = ks < n.kn[d] ? (unsigned)ks : (unsigned)n.kn[d];
            const unsigned char sil = differ[d] ? silm[v.setup_off + front] : (unsigned char)0;
            n.cand[d] = differ[d] && sil != 0;
        }
    }
    return n;
}

// Sample of thread t of workgroup b (256 threads) in a W x H view.  When
// the view is a whole number of 32 x 8 regions, each workgroup takes one
// region and each wave one 8 x 8 tile of it, so that a silhouette touches
// fewer waves than with row segments of 64 samples (a wave with one
// candidate pair waits for the pair tests' loads on all of its lanes);
// otherwise samples run in row order.  Either way the workgroups cover the
// view's W * H samples exactly once.
__device__ __forceinline__ int aa_sample_index(int b, int t, int W, int H) {
    if ((W & 31) == 0 && (H & 7) == 0) {
        const int rx = b % (W >> 5), ry = b / (W >> 5);
        const int w = t >> 6, l = t & 63;
        return (ry * 8 + (l >> 3)) * W + rx * 32 + w * 8 + (l & 7);
    }
    return b * 256 + t;
}

// Samples listed for the second pass of the smoothing kernels.  The list is
// cut into segments, each with its own counter, so that the appends of
// different workgroups do not contend for one address: workgroup b of the
// first pass (b counted over the whole grid) appends to segment
// b % kAaSegments, which holds every sample of the workgroups that map to
// it and so cannot overflow.  The second pass runs one workgroup per
// segment.
constexpr int kAaSegments = 4096;

struct AaList {
    uint2 *items;
    unsigned *counts;        // kAaSegments counters, zero before the first pass
    unsigned nseg, segcap;   // segments in use, items per segment
};

__host__ __device__ inline AaList aa_list_for(uint2 *items, unsigned *counts, long long blocks) {
    AaList l;
    l.items = items;
    l.counts = counts;
    l.nseg = (unsigned)(blocks < kAaSegments ? blocks : kAaSegments);
    l.segcap = l.nseg ? (unsigned)(((blocks + l.nseg - 1) / l.nseg) * 256) : 0u;
    return l;
}

// Append the active lanes' items to the segment of this workgroup (one
// atomic per wave).  lin: the workgroup's index over the whole grid.
__device__ __forceinline__ void wave_append(bool mine, uint2 item, const AaList &l, long long lin) {
    const unsigned long long m = __ballot(mine);
    if (m == 0ull) return;
    const unsigned seg = (unsigned)(lin % l.nseg);
    const int lane = (int)(threadIdx.x & 63), leader = __ffsll(m) - 1;
    unsigned first = 0;
    if (lane == leader) first = atomicAdd(l.counts + seg, (unsigned)__popcll(m));
    first = (unsigned)__shfl((int)first, leader, 64);
    if (mine) l.items[(size_t)seg * l.segcap + first + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = item;
}

}  // namespace dsm
