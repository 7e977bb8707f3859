// Separable moment filter, forward (m = G f~, Eq. moment1 / moment2) and
// transpose (the gradient G^T of Sec. 4: the filter applied to the Jacobian).
//
// One workgroup filters a TX x TY tile of one 2-channel map in a single
// pass: the tile plus an r-texel halo is staged in LDS, the first 1D pass
// writes an LDS intermediate, the second writes the output.  Each input
// texel is read from HBM once per tile (halo re-reads are served by L2), each
// output texel written once: 16 bytes of algorithmic traffic per texel.
//
// Boundary: clamp-to-edge in the forward pass.  Its transpose is
// zero-padded correlation (the taps are symmetric) plus, on the first and
// last row/column, the weight of every tap that the forward pass clamped
// onto that texel.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

constexpr int kBlurTX = 64;
constexpr int kBlurThreads = 256;

__device__ __forceinline__ int find_job(const BlurJob *jobs, int njobs, int tile) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// jobs != nullptr: one flattened grid over the tiles of every job (maps of a
// batch may differ in size and filter).  jobs == nullptr: every map uses
// `single`; map blockIdx.y sits 2*S*S floats after the previous one.
template <bool ADJ>
__global__ __launch_bounds__(kBlurThreads) void blur_kernel(const BlurJob *__restrict__ jobs, int njobs,
                                                            BlurJob single, int TY, const float *__restrict__ in,
                                                            float *__restrict__ out) {
    extern __shared__ float smem[];
    __shared__ float w[kMaxTaps];
    __shared__ float cum[kMaxTaps];
    const int tile = blockIdx.x;
    const BlurJob &J = jobs ? jobs[find_job(jobs, njobs, tile)] : single;
    const int S = J.S, k = J.k, r = (k - 1) >> 1;
    const int t = tile - J.tile_off;
    const int x0 = (t % J.tiles_x) * kBlurTX;
    const int y0 = (t / J.tiles_x) * TY;
    const int tid = threadIdx.x;
    if (tid < k) w[tid] = J.w[tid];
    __syncthreads();
    if (tid == 0) {
        float c = 0.f;
        for (int i = 0; i < k; ++i) { c += w[i]; cum[i] = c; }
    }
    const int RW = kBlurTX + 2 * r;        // staged region width
    const int RH = TY + 2 * r;             // staged region height
    float *sin0 = smem;                    // [2][RH][RW]
    float *mid0 = smem + 2 * RH * RW;      // forward: [2][RH][TX]; adjoint: [2][TY][RW]
    const size_t plane = (size_t)S * S;
    const long long map_shift = jobs ? 0 : (long long)blockIdx.y * 2 * (long long)plane;
    const float *src = in + J.in_off + map_shift;
    float *dst = out + J.out_off + map_shift;

    // thread (cx, cy): cx = lane column 0..63, cy = row phase 0..3; no integer division
    const int cx = tid & 63, cy = tid >> 6;
    for (int ly = cy; ly < RH; ly += 4) {
        int gy = y0 - r + ly;
        bool rok = true;
        if (!ADJ) gy = min(max(gy, 0), S - 1);
        else rok = gy >= 0 && gy < S;
        const size_t rowo = (size_t)(rok ? gy : 0) * S;
        for (int lx = cx; lx < RW; lx += 64) {
            int gx = x0 - r + lx;
            bool ok = rok;
            if (!ADJ) gx = min(max(gx, 0), S - 1);
            else ok = ok && gx >= 0 && gx < S;
            const size_t o = rowo + (ok ? gx : 0);
            sin0[ly * RW + lx] = ok ? src[o] : 0.f;
            sin0[RH * RW + ly * RW + lx] = ok ? src[plane + o] : 0.f;
        }
    }
    __syncthreads();

    if (!ADJ) {
        // horizontal pass over all staged rows
        for (int ly = cy; ly < RH; ly += 4) {
            const float *ra = sin0 + ly * RW + cx;
            const float *rb = ra + RH * RW;
            float a = 0.f, bb = 0.f;
            for (int j = 0; j < k; ++j) { a += w[j] * ra[j]; bb += w[j] * rb[j]; }
            mid0[ly * kBlurTX + cx] = a;
            mid0[RH * kBlurTX + ly * kBlurTX + cx] = bb;
        }
        __syncthreads();
        // vertical pass
        const int gx = x0 + cx;
        for (int ly = cy; ly < TY; ly += 4) {
            const int gy = y0 + ly;
            if (gx >= S || gy >= S) continue;
            const float *ca = mid0 + ly * kBlurTX + cx;
            const float *cb = ca + RH * kBlurTX;
            float a = 0.f, bb = 0.f;
            for (int j = 0; j < k; ++j) { a += w[j] * ca[j * kBlurTX]; bb += w[j] * cb[j * kBlurTX]; }
            const size_t o = (size_t)gy * S + gx;
            dst[o] = a;
            dst[plane + o] = bb;
        }
    } else {
        // transpose of the vertical pass: rows [0, TY), all staged columns
        for (int ly = cy; ly < TY; ly += 4) {
            const int gy = y0 + ly;
            for (int lx = cx; lx < RW; lx += 64) {
                const float *ca = sin0 + ly * RW + lx;
                const float *cb = ca + RH * RW;
                float a = 0.f, bb = 0.f;
                for (int j = 0; j < k; ++j) { a += w[j] * ca[j * RW]; bb += w[j] * cb[j * RW]; }
                if (gy == 0) {             // taps clamped onto row 0: sum_{i<r} g[i] * cum(r-1-i)
                    for (int i = 0; i < r; ++i) {
                        const int l = (i - y0 + r) * RW + lx;
                        a += cum[r - 1 - i] * sin0[l];
                        bb += cum[r - 1 - i] * sin0[RH * RW + l];
                    }
                }
                if (gy == S - 1) {         // taps clamped onto the last row
                    for (int i = S - r; i < S; ++i) {
                        const int l = (i - y0 + r) * RW + lx;
                        a += cum[r - 1 - (S - 1 - i)] * sin0[l];
                        bb += cum[r - 1 - (S - 1 - i)] * sin0[RH * RW + l];
                    }
                }
                mid0[ly * RW + lx] = a;
                mid0[TY * RW + ly * RW + lx] = bb;
            }
        }
        __syncthreads();
        const int gx = x0 + cx;
        for (int ly = cy; ly < TY; ly += 4) {
            const int gy = y0 + ly;
            if (gx >= S || gy >= S) continue;
            const float *ra = mid0 + ly * RW + cx;
            const float *rb = ra + TY * RW;
            float a = 0.f, bb = 0.f;
            for (int j = 0; j < k; ++j) { a += w[j] * ra[j]; bb += w[j] * rb[j]; }
            // global column i sits at ra[i - gx + r]
            if (gx == 0) {
                for (int i = 0; i < r; ++i) {
                    a += cum[r - 1 - i] * ra[i + r];
                    bb += cum[r - 1 - i] * rb[i + r];
                }
            }
            if (gx == S - 1) {
                for (int i = S - r; i < S; ++i) {
                    a += cum[r - 1 - (S - 1 - i)] * ra[i - gx + r];
                    bb += cum[r - 1 - (S - 1 - i)] * rb[i - gx + r];
                }
            }
            const size_t o = (size_t)gy * S + gx;
            dst[o] = a;
            dst[plane + o] = bb;
        }
    }
}

static int blur_ty(int rmax) { return rmax > 8 ? 16 : 32; }

static size_t blur_smem(int rmax, int TY) {
    const size_t RW = kBlurTX + 2 * rmax, RH = TY + 2 * rmax;
    const size_t mid = 2 * RH * kBlurTX > 2 * TY * RW ? 2 * RH * kBlurTX : 2 * TY * RW;
    return sizeof(float) * (2 * RH * RW + mid);
}

hipError_t launch_blur(const BlurJob *jobs_dev, int njobs, int total_tiles, const float *in, float *out,
                       bool adjoint, int rmax, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    const int TY = blur_ty(rmax);
    const size_t sm = blur_smem(rmax, TY);
    BlurJob none{};
    if (adjoint)
        hipLaunchKernelGGL(blur_kernel<true>, dim3(total_tiles), dim3(kBlurThreads), sm, s, jobs_dev, njobs, none,
                           TY, in, out);
    else
        hipLaunchKernelGGL(blur_kernel<false>, dim3(total_tiles), dim3(kBlurThreads), sm, s, jobs_dev, njobs, none,
                           TY, in, out);
    return hipGetLastError();
}

hipError_t launch_blur_uniform(const BlurJob &job, int n_maps, const float *in, float *out, bool adjoint,
                               hipStream_t s) {
    const int r = (job.k - 1) / 2;
    const int TY = blur_ty(r);
    const int tiles_y = (job.S + TY - 1) / TY;
    BlurJob j = job;
    j.tile_off = 0;
    j.tiles_x = (job.S + kBlurTX - 1) / kBlurTX;
    const dim3 grid(j.tiles_x * tiles_y, n_maps);
    const size_t sm = blur_smem(r, TY);
    if (adjoint)
        hipLaunchKernelGGL(blur_kernel<true>, grid, dim3(kBlurThreads), sm, s, nullptr, 0, j, TY, in, out);
    else
        hipLaunchKernelGGL(blur_kernel<false>, grid, dim3(kBlurThreads), sm, s, nullptr, 0, j, TY, in, out);
    return hipGetLastError();
}

int blur_tiles(int S, int rmax) {
    const int TY = blur_ty(rmax);
    return ((S + kBlurTX - 1) / kBlurTX) * ((S + TY - 1) / TY);
}
int blur_tiles_x(int S) { return (S + kBlurTX - 1) / kBlurTX; }

int blur_tile_height(int rmax) { return blur_ty(rmax); }

void filter_taps_host(int filter, int k, float sigma, float *w) {
    const int r = (k - 1) / 2;
    if (filter == DSM_FILTER_BOX) {
        for (int i = 0; i < k; ++i) w[i] = (float)(1.0 / k);
        return;
    }
    double s = sigma > 0 ? (double)sigma : (k - 1) / 3.0;
    if (s <= 0) {
        w[0] = 1.f;
        return;
    }
    double acc = 0, tmp[kMaxTaps];
    for (int i = -r; i <= r; ++i) {
        tmp[i + r] = exp(-(double)(i * i) / (2.0 * s * s));
        acc += tmp[i + r];
    }
    for (int i = 0; i < k; ++i) w[i] = (float)(tmp[i] / acc);
}

}  // namespace dsm
