// Cube shadow maps across their seams.  The six faces of an omnidirectional
// light are consecutive light views.  Before the moment filter every face's
// smoothed map is copied into a map padded by P texels whose border comes
// from the neighbouring faces: the k-th texel beyond an edge takes the
// neighbour's texel at depth k - 1 from the shared cube edge, at the same
// place along the edge; the corner blocks, which no face covers, repeat the
// face's corner texel.  The filter then runs over the padded map, so it and
// the bilinear fetch continue across the seams (Sec. 3 lets the rays of a
// light be parameterized over several planes arranged as a box).  The
// transpose gathers, for every texel, the gradient of each padded copy.
#include "dsm_internal.h"

namespace dsm {

// Texel of the six-face group that padded position (pi, pj) of face f copies:
// returns the face (0..5) and writes the texel index j * S + i.
__device__ __forceinline__ int cube_pad_source(const ViewConst &v, int S, int pi, int pj, int &texel) {
    const int P = v.fpad;
    const int i = pi - P, j = pj - P;
    const bool in_i = i >= 0 && i < S, in_j = j >= 0 && j < S;
    if (in_i && in_j) {
        texel = j * S + i;
        return v.cube_face;
    }
    if (!in_i && !in_j) {
        texel = min(max(j, 0), S - 1) * S + min(max(i, 0), S - 1);
        return v.cube_face;
    }
    int e, k, t;
    if (i < 0) { e = 0; k = -i; t = j; }
    else if (i >= S) { e = 1; k = i - S + 1; t = j; }
    else if (j < 0) { e = 2; k = -j; t = i; }
    else { e = 3; k = j - S + 1; t = i; }
    const int nb = v.cube_nb[e];
    const int g = nb & 7, e2 = (nb >> 3) & 3;
    const int t2 = ((nb >> 5) & 1) ? S - 1 - t : t;
    const int d = k - 1;
    int ii, jj;
    if (e2 == 0) { ii = d; jj = t2; }
    else if (e2 == 1) { ii = S - 1 - d; jj = t2; }
    else if (e2 == 2) { ii = t2; jj = d; }
    else { ii = t2; jj = S - 1 - d; }
    texel = jj * S + ii;
    return g;
}

__global__ void cube_pad_kernel(const ViewConst *__restrict__ views, float *__restrict__ F1) {
    const ViewConst &v = views[blockIdx.y];
    if (v.fpad == 0) return;
    const int S = v.W, Sp = S + 2 * v.fpad;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Sp * Sp) return;
    int texel;
    const int g = cube_pad_source(v, S, t % Sp, t / Sp, texel);
    const ViewConst &src = views[blockIdx.y - v.cube_face + g];
    const long long plane = (long long)S * S, pplane = (long long)Sp * Sp;
    F1[v.pad_off + t] = F1[src.map_off + texel];
    F1[v.pad_off + pplane + t] = F1[src.map_off + plane + texel];
}

// gF1 of a face texel = the gradient of its own padded copy, of the copies in
// the neighbours' borders (one per edge it is within P of) and, for a corner
// texel, of the face's corner block.
__global__ void cube_pad_transpose_kernel(const ViewConst *__restrict__ views, float *__restrict__ gF1) {
    const ViewConst &v = views[blockIdx.y];
    if (v.fpad == 0) return;
    const int S = v.W, P = v.fpad, Sp = S + 2 * P;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * S) return;
    const int i = t % S, j = t / S;
    const long long plane = (long long)S * S, pplane = (long long)Sp * Sp;
    const float *gp = gF1 + v.pad_off;
    float a0 = gp[(long long)(j + P) * Sp + (i + P)], a1 = gp[pplane + (long long)(j + P) * Sp + (i + P)];
    if ((i == 0 || i == S - 1) && (j == 0 || j == S - 1)) {
        const int bx = i == 0 ? 0 : P + S, by = j == 0 ? 0 : P + S;
        for (int y = by; y < by + P; ++y)
            for (int x = bx; x < bx + P; ++x) {
                a0 += gp[(long long)y * Sp + x];
                a1 += gp[pplane + (long long)y * Sp + x];
            }
    }
    for (int e = 0; e < 4; ++e) {
        const int m = e == 0 ? i : e == 1 ? S - 1 - i : e == 2 ? j : S - 1 - j;
        if (m >= P) continue;
        const int along = e < 2 ? j : i;
        const int nb = v.cube_nb[e];
        const int g = nb & 7, e2 = (nb >> 3) & 3;
        const int tg = ((nb >> 5) & 1) ? S - 1 - along : along;
        const int k = m + 1;
        int pi, pj;
        if (e2 == 0) { pi = P - k; pj = tg + P; }
        else if (e2 == 1) { pi = P + S - 1 + k; pj = tg + P; }
        else if (e2 == 2) { pi = tg + P; pj = P - k; }
        else { pi = tg + P; pj = P + S - 1 + k; }
        const float *gq = gF1 + views[blockIdx.y - v.cube_face + g].pad_off;
        a0 += gq[(long long)pj * Sp + pi];
        a1 += gq[pplane + (long long)pj * Sp + pi];
    }
    gF1[v.map_off + t] = a0;
    gF1[v.map_off + plane + t] = a1;
}

hipError_t launch_cube_pad(const ViewConst *views, int L, int max_padded, float *F1, hipStream_t s) {
    if (L == 0 || max_padded == 0) return hipSuccess;
    hipLaunchKernelGGL(cube_pad_kernel, dim3((max_padded + 255) / 256, L), dim3(256), 0, s, views, F1);
    return hipGetLastError();
}

hipError_t launch_cube_pad_transpose(const ViewConst *views, int L, int max_texels, float *gF1, hipStream_t s) {
    if (L == 0 || max_texels == 0) return hipSuccess;
    hipLaunchKernelGGL(cube_pad_transpose_kernel, dim3((max_texels + 255) / 256, L), dim3(256), 0, s, views, gF1);
    return hipGetLastError();
}

}  // namespace dsm
