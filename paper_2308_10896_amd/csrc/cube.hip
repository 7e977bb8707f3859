// Cube shadow maps across their seams.  The six faces of an omnidirectional
// light are consecutive light views.  Before the moment filter every face's
// smoothed map is copied into a map padded by P texels: beyond each edge,
// the padded texel takes the bilinear sample of the neighbouring face along
// the direction its centre looks along when the face's plane is continued
// across the edge (taps precomputed per plan); the corner blocks, which no
// face covers, repeat the face's corner texel.  The filter then runs over the
// padded map, so it and the bilinear fetch continue across the seams (Sec. 3
// lets the rays of a light be parameterized over several planes arranged as
// a box).  The transpose returns each padded texel's gradient to the texels
// it was sampled from.
#include "dsm_internal.h"

namespace dsm {

// Edge block of a padded position outside exactly one side of the face:
// edge e (0 left, 1 right, 2 top, 3 bottom), depth k >= 1, position t.
__device__ __forceinline__ int cube_ring_entry(int S, int P, int i, int j) {
    int e, k, t;
    if (i < 0) { e = 0; k = -i; t = j; }
    else if (i >= S) { e = 1; k = i - S + 1; t = j; }
    else if (j < 0) { e = 2; k = -j; t = i; }
    else { e = 3; k = j - S + 1; t = i; }
    return (e * P + (k - 1)) * S + t;
}

__global__ void cube_pad_kernel(const ViewConst *__restrict__ views, const CubeTap *__restrict__ taps,
                                float *__restrict__ F1) {
    const int l = blockIdx.y;
    const ViewConst &v = views[l];
    if (v.fpad == 0) return;
    const int S = v.W, P = v.fpad, Sp = S + 2 * P;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Sp * Sp) return;
    const int i = t % Sp - P, j = t / Sp - P;
    const bool in_i = i >= 0 && i < S, in_j = j >= 0 && j < S;
    const long long plane = (long long)S * S, pplane = (long long)Sp * Sp;
    float a0, a1;
    if (in_i == in_j) {               // inside, or a corner block: the face's own (corner) texel
        const long long q = v.map_off + (long long)min(max(j, 0), S - 1) * S + min(max(i, 0), S - 1);
        a0 = F1[q];
        a1 = F1[q + plane];
    } else {
        const CubeTap tp = taps[v.ring_off + cube_ring_entry(S, P, i, j)];
        const float *src = F1 + views[l - v.cube_face + tp.g].map_off;
        a0 = ((tp.w[0] * src[tp.o[0]] + tp.w[1] * src[tp.o[1]]) + tp.w[2] * src[tp.o[2]]) + tp.w[3] * src[tp.o[3]];
        a1 = ((tp.w[0] * src[plane + tp.o[0]] + tp.w[1] * src[plane + tp.o[1]]) + tp.w[2] * src[plane + tp.o[2]]) +
             tp.w[3] * src[plane + tp.o[3]];
    }
    F1[v.pad_off + t] = a0;
    F1[v.pad_off + pplane + t] = a1;
}

// First part of the transpose: every face texel takes the gradient of its own
// padded copy and, at a corner, of the corner block (plain stores).
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
    gF1[v.map_off + t] = a0;
    gF1[v.map_off + plane + t] = a1;
}

// Second part: the gradient of every edge-block texel goes to the four taps it
// was sampled from in the neighbouring face (atomic adds; runs after the
// first part).
__global__ void cube_ring_transpose_kernel(const ViewConst *__restrict__ views, const CubeTap *__restrict__ taps,
                                           float *__restrict__ gF1) {
    const int l = blockIdx.y;
    const ViewConst &v = views[l];
    if (v.fpad == 0) return;
    const int S = v.W, P = v.fpad, Sp = S + 2 * P;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= 4 * P * S) return;
    const int e = n / (P * S), k = (n / S) % P + 1, t = n % S;
    const int pi = e == 0 ? P - k : e == 1 ? P + S - 1 + k : t + P;
    const int pj = e == 2 ? P - k : e == 3 ? P + S - 1 + k : t + P;
    const long long plane = (long long)S * S, pplane = (long long)Sp * Sp;
    const float g0 = gF1[v.pad_off + (long long)pj * Sp + pi], g1 = gF1[v.pad_off + pplane + (long long)pj * Sp + pi];
    if (g0 == 0.f && g1 == 0.f) return;
    const CubeTap tp = taps[v.ring_off + n];
    float *dst = gF1 + views[l - v.cube_face + tp.g].map_off;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (tp.w[q] == 0.f) continue;
        atomic_add_f32(dst + tp.o[q], tp.w[q] * g0);
        atomic_add_f32(dst + plane + tp.o[q], tp.w[q] * g1);
    }
}

hipError_t launch_cube_pad(const ViewConst *views, int L, int max_padded, const CubeTap *taps, float *F1,
                           hipStream_t s) {
    if (L == 0 || max_padded == 0) return hipSuccess;
    hipLaunchKernelGGL(cube_pad_kernel, dim3((max_padded + 255) / 256, L), dim3(256), 0, s, views, taps, F1);
    return hipGetLastError();
}

hipError_t launch_cube_pad_transpose(const ViewConst *views, int L, int max_texels, int max_ring,
                                     const CubeTap *taps, float *gF1, hipStream_t s) {
    if (L == 0 || max_texels == 0) return hipSuccess;
    hipLaunchKernelGGL(cube_pad_transpose_kernel, dim3((max_texels + 255) / 256, L), dim3(256), 0, s, views, gF1);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess || max_ring == 0) return err;
    hipLaunchKernelGGL(cube_ring_transpose_kernel, dim3((max_ring + 255) / 256, L), dim3(256), 0, s, views, taps,
                       gF1);
    return hipGetLastError();
}

}  // namespace dsm
