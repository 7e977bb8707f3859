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
// LDS row layout: [pad | halo r | 64 interior | halo r | pad], the interior
// starting at column H4 = 4 * ceil(r / 4) so that it is 16-byte aligned and
// read / written with 128-bit accesses; the row stride is 16 (mod 32) floats
// so that the two row phases of a half-wave fall into different LDS banks.
// Thread t handles column quad / columns of column phase t % 16 in rows
// t / 16 (+16, ...).
__host__ __device__ inline int blur_row_stride(int H4) {
    int s = kBlurTX + 2 * H4;
    while ((s & 31) != 16) s += 4;
    return s;
}

template <bool ADJ>
__global__ __launch_bounds__(kBlurThreads) void blur_kernel(const BlurJob *__restrict__ jobs, int njobs,
                                                            BlurJob single, int TY, const float *__restrict__ in,
                                                            float *__restrict__ out) {
    extern __shared__ float4 smem4[];
    float *smem = (float *)smem4;
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
    const int H4 = (r + 3) & ~3;
    const int RWP = blur_row_stride(H4);   // staged row stride (floats)
    const int RH = TY + 2 * r;             // staged rows
    float *sin0 = smem;                    // [2][RH][RWP]
    float *mid0 = smem + 2 * RH * RWP;     // forward: [2][RH][64]; adjoint: [2][TY][RWP]
    const size_t plane = (size_t)S * S;
    const long long map_shift = jobs ? 0 : (long long)blockIdx.y * 2 * (long long)plane;
    const float *src = in + J.in_off + map_shift;
    float *dst = out + J.out_off + map_shift;
    const bool vec = (S & 3) == 0 && x0 + kBlurTX <= S && ((J.in_off | J.out_off) & 3) == 0;
    const int cq = tid & 15, cr = tid >> 4;          // column quad, row phase (16 phases)

    // ---- stage rows [y0 - r, y0 + TY + r) x columns [x0 - r, x0 + 64 + r)
    for (int ly = cr; ly < RH; ly += 16) {
        int gy = y0 - r + ly;
        bool rok = true;
        if (!ADJ) gy = min(max(gy, 0), S - 1);
        else rok = gy >= 0 && gy < S;
        const size_t rowo = (size_t)(rok ? gy : 0) * S;
        float *la = sin0 + ly * RWP, *lb = la + RH * RWP;
        if (vec) {
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), bq = a;
            if (rok) {
                a = *(const float4 *)(src + rowo + x0 + 4 * cq);
                bq = *(const float4 *)(src + plane + rowo + x0 + 4 * cq);
            }
            *(float4 *)(la + H4 + 4 * cq) = a;
            *(float4 *)(lb + H4 + 4 * cq) = bq;
        } else {
            for (int e = 0; e < 4; ++e) {
                int gx = x0 + 4 * cq + e;
                bool ok = rok;
                if (!ADJ) gx = min(gx, S - 1);
                else ok = ok && gx < S;
                la[H4 + 4 * cq + e] = ok ? src[rowo + gx] : 0.f;
                lb[H4 + 4 * cq + e] = ok ? src[plane + rowo + gx] : 0.f;
            }
        }
        // halo columns: r on each side
        if (cq < 2) {
            for (int e = 0; e < r; ++e) {
                const int lx = cq == 0 ? H4 - r + e : H4 + kBlurTX + e;
                int gx = x0 - H4 + lx;
                bool ok = rok;
                if (!ADJ) gx = min(max(gx, 0), S - 1);
                else ok = ok && gx >= 0 && gx < S;
                la[lx] = ok ? src[rowo + gx] : 0.f;
                lb[lx] = ok ? src[plane + rowo + gx] : 0.f;
            }
        }
    }
    __syncthreads();

    if (!ADJ) {
        // horizontal pass: all staged rows, 64 output columns
        for (int ly = cr; ly < RH; ly += 16) {
            const float *ra = sin0 + ly * RWP + H4 - r + cq;
            const float *rb = ra + RH * RWP;
            float a[4] = {0.f, 0.f, 0.f, 0.f}, bq[4] = {0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < k; ++j) {
                const float wj = w[j];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    a[e] += wj * ra[j + 16 * e];
                    bq[e] += wj * rb[j + 16 * e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                mid0[ly * kBlurTX + cq + 16 * e] = a[e];
                mid0[RH * kBlurTX + ly * kBlurTX + cq + 16 * e] = bq[e];
            }
        }
        __syncthreads();
        // vertical pass: TY output rows
        for (int ly = cr; ly < TY; ly += 16) {
            const int gy = y0 + ly;
            if (gy >= S) continue;
            const float4 *ca = (const float4 *)(mid0 + ly * kBlurTX + 4 * cq);
            const float4 *cb = (const float4 *)(mid0 + RH * kBlurTX + ly * kBlurTX + 4 * cq);
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), bq = a;
            for (int j = 0; j < k; ++j) {
                const float wj = w[j];
                const float4 u = ca[j * (kBlurTX / 4)], v = cb[j * (kBlurTX / 4)];
                a.x += wj * u.x; a.y += wj * u.y; a.z += wj * u.z; a.w += wj * u.w;
                bq.x += wj * v.x; bq.y += wj * v.y; bq.z += wj * v.z; bq.w += wj * v.w;
            }
            const size_t o = (size_t)gy * S + x0 + 4 * cq;
            if (vec) {
                *(float4 *)(dst + o) = a;
                *(float4 *)(dst + plane + o) = bq;
            } else {
                const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {bq.x, bq.y, bq.z, bq.w};
                for (int e = 0; e < 4; ++e)
                    if (x0 + 4 * cq + e < S) {
                        dst[o + e] = av[e];
                        dst[plane + o + e] = bv[e];
                    }
            }
        }
    } else {
        // transpose of the vertical pass: TY rows, every staged column (quads of 4)
        const int nq = RWP / 4;
        for (int idx = tid; idx < TY * nq; idx += kBlurThreads) {
            const int ly = idx / nq, q4 = idx - ly * nq;
            const int gy = y0 + ly;
            float a[4] = {0.f, 0.f, 0.f, 0.f}, bq[4] = {0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < k; ++j) {
                const float wj = w[j];
                const float4 u = *(const float4 *)(sin0 + (ly + j) * RWP + 4 * q4);
                const float4 v = *(const float4 *)(sin0 + RH * RWP + (ly + j) * RWP + 4 * q4);
                a[0] += wj * u.x; a[1] += wj * u.y; a[2] += wj * u.z; a[3] += wj * u.w;
                bq[0] += wj * v.x; bq[1] += wj * v.y; bq[2] += wj * v.z; bq[3] += wj * v.w;
            }
            if (gy == 0 || gy == S - 1) {          // taps the forward pass clamped onto this row
                for (int e = 0; e < 4; ++e) {
                    const int lx = 4 * q4 + e;
                    if (gy == 0)
                        for (int i = 0; i < r; ++i) {
                            const int l = (i - y0 + r) * RWP + lx;
                            a[e] += cum[r - 1 - i] * sin0[l];
                            bq[e] += cum[r - 1 - i] * sin0[RH * RWP + l];
                        }
                    if (gy == S - 1)
                        for (int i = S - r; i < S; ++i) {
                            const int l = (i - y0 + r) * RWP + lx;
                            a[e] += cum[r - 1 - (S - 1 - i)] * sin0[l];
                            bq[e] += cum[r - 1 - (S - 1 - i)] * sin0[RH * RWP + l];
                        }
                }
            }
            *(float4 *)(mid0 + ly * RWP + 4 * q4) = make_float4(a[0], a[1], a[2], a[3]);
            *(float4 *)(mid0 + TY * RWP + ly * RWP + 4 * q4) = make_float4(bq[0], bq[1], bq[2], bq[3]);
        }
        __syncthreads();
        // transpose of the horizontal pass: TY rows, 64 output columns
        for (int ly = cr; ly < TY; ly += 16) {
            const int gy = y0 + ly;
            if (gy >= S) continue;
            const float *ra = mid0 + ly * RWP + H4 - r + cq;
            const float *rb = ra + TY * RWP;
            float a[4] = {0.f, 0.f, 0.f, 0.f}, bq[4] = {0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < k; ++j) {
                const float wj = w[j];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    a[e] += wj * ra[j + 16 * e];
                    bq[e] += wj * rb[j + 16 * e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gx = x0 + cq + 16 * e;
                // global column i sits at ra[16 e + i - gx + r]
                if (gx == 0)
                    for (int i = 0; i < r; ++i) {
                        a[e] += cum[r - 1 - i] * ra[16 * e + i + r];
                        bq[e] += cum[r - 1 - i] * rb[16 * e + i + r];
                    }
                if (gx == S - 1)
                    for (int i = S - r; i < S; ++i) {
                        a[e] += cum[r - 1 - (S - 1 - i)] * ra[16 * e + i - gx + r];
                        bq[e] += cum[r - 1 - (S - 1 - i)] * rb[16 * e + i - gx + r];
                    }
                if (gx < S) {
                    const size_t o = (size_t)gy * S + gx;
                    dst[o] = a[e];
                    dst[plane + o] = bq[e];
                }
            }
        }
    }
}

static int blur_ty(int rmax) { return rmax > 8 ? 16 : 32; }

static size_t blur_smem(int rmax, int TY) {
    // worst case over r <= rmax (the staged width grows with r)
    const size_t H4 = (size_t)((rmax + 3) & ~3);
    const size_t RWP = (size_t)blur_row_stride((int)H4), RH = TY + 2 * rmax;
    const size_t mid = 2 * RH * kBlurTX > 2 * TY * RWP ? 2 * RH * kBlurTX : 2 * TY * RWP;
    return sizeof(float) * (2 * RH * RWP + mid);
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
