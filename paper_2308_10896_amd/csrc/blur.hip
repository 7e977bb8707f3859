// Separable moment filter, forward (m = G f~, Eq. moment1 / moment2) and
// transpose (the gradient G^T of Sec. 4: the filter applied to the Jacobian).
//
// One workgroup (4 waves) filters a 64 x 64 tile of one 2-channel map.  The
// tile plus an r-texel halo is staged in LDS in one phase: every thread
// issues all of its loads before the first wait, so a workgroup keeps its
// whole footprint in flight.  Each lane then owns one column of 16 output
// rows: it forms the horizontal filter of that column for every staged row
// (the k taps are neighbouring LDS words) and pushes the results through a
// register ring of the last k rows, from which each output row is one
// k-tap dot product.  Each input texel is read from HBM once (halo re-reads
// of neighbouring tiles are served by L2) and each output texel written
// once: 16 bytes of algorithmic traffic per texel.
//
// Boundary: clamp-to-edge in the forward pass.  Its transpose is
// zero-padded correlation (the taps are symmetric) plus, on the first and
// last row / column, the weight of every tap that the forward pass clamped
// onto that texel.  Horizontal and vertical passes commute, so the transpose
// also runs horizontal-first.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

constexpr int kBlurTX = 64;                          // tile width: one column per lane
constexpr int kBlurThreads = 256;

// Tile height for radius R.  The staged tile carries 2R halo rows, so short
// tiles pay relatively more for wide filters, and tall tiles keep fewer
// workgroups resident.  Measured on this GPU (stand-alone filter and
// transpose, 64 x 512^2, 8 x 1024^2 and 3 x 2048^2 maps): 32 rows is
// fastest for R <= 4 (k <= 9), 64 rows from R = 5 (k >= 11) on; 16 rows is
// slower everywhere and 128 slower at R = 2.
__host__ __device__ constexpr int blur_ty(int R) { return R <= 4 ? 32 : 64; }

__device__ __forceinline__ int find_job(const BlurJob *jobs, int njobs, int tile) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Staged tile geometry for radius R.  LDS row layout: [pad | halo R | 64
// interior | halo R | pad] with the interior at column H4 = 4 ceil(R / 4), so
// that it is written with 128-bit stores.
template <int R>
struct BlurGeom {
    static constexpr int K = 2 * R + 1;
    static constexpr int H4 = (R + 3) & ~3;
    static constexpr int RWP = kBlurTX + 2 * H4;                    // LDS row stride (floats)
    static constexpr int TY = blur_ty(R);                           // tile height
    static constexpr int WR = TY / (kBlurThreads / kBlurTX);        // output rows per lane
    static constexpr int RH = TY + 2 * R;                           // staged rows
    static constexpr int NQ = RH * (kBlurTX / 4);                   // interior quads per channel
    static constexpr int QPT = (2 * NQ + kBlurThreads - 1) / kBlurThreads;
    static constexpr int NH = RH * 2 * R;                           // halo texels per channel
    static constexpr int HPT = R > 0 ? (2 * NH + kBlurThreads - 1) / kBlurThreads : 1;
};

// jobs != nullptr: one flattened grid over the tiles of every job of this
// radius.  jobs == nullptr: every map uses `single`, the grid holds per_map
// tiles of each map in turn, and map m sits 2*S*S*m floats after the first.
// IL: the filtered side (the output of the forward pass, the input of the
// transpose) holds (m1, m2) interleaved per texel, so that a bilinear tap of
// the lookup is one 8-byte load; the smoothed side stays channel-planar.
template <bool ADJ, int R, bool IL>
__global__ __launch_bounds__(kBlurThreads) void blur_kernel(const BlurJob *__restrict__ jobs, int njobs,
                                                            BlurJob single, int per_map,
                                                            const float *__restrict__ in, float *__restrict__ out) {
    using G = BlurGeom<R>;
    constexpr int K = G::K, H4 = G::H4, RWP = G::RWP, RH = G::RH;
    __shared__ __align__(16) float tile_s[2][RH][RWP];
    const int item = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const BlurJob &J = jobs ? jobs[find_job(jobs, njobs, item)] : single;
    const int S = J.S;
    const int map = jobs ? 0 : item / per_map;
    const int t = jobs ? item - J.tile_off : item - map * per_map;
    const int x0 = (t % J.tiles_x) * kBlurTX, y0 = (t / J.tiles_x) * G::TY;
    const int tid = (int)threadIdx.x;
    const size_t plane = (size_t)S * S;
    const long long map_shift = (long long)map * 2 * (long long)plane;
    const float *src = in + J.in_off + map_shift;
    float *dst = out + J.out_off + map_shift;

    // ---- stage rows [y0 - R, y0 + 64 + R) x columns [x0 - R, x0 + 64 + R)
    // staged row l holds map row y0 - R + l; staged column H4 - R + e holds
    // map column x0 - R + e.
    auto row_of = [&](int l, bool &ok) {
        int gy = y0 - R + l;
        ok = true;
        if (!ADJ) gy = min(max(gy, 0), S - 1);
        else ok = gy >= 0 && gy < S;
        return (size_t)(ok ? gy : 0) * S;
    };
    const bool vec = (S & 3) == 0 && x0 + kBlurTX <= S && ((J.in_off | J.out_off) & 3) == 0;
    // interleaved input texel (channel ch) of map row offset ro, column gx
    auto iload = [&](int ch, size_t ro, int gx) { return src[2 * (ro + gx) + ch]; };
    if (IL && ADJ) {
        // two 16-byte loads hold four texels of both channels; every load is
        // issued before the first LDS store, as in the planar path
        constexpr int NI = (G::NQ + kBlurThreads - 1) / kBlurThreads;
        float4 lo[NI], hi[NI];
        float h[G::HPT];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int r = tid + i * kBlurThreads;
            lo[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            hi[i] = lo[i];
            if (r < G::NQ) {
                const int l = r >> 4, cq = r & 15;
                bool rok;
                const size_t ro = row_of(l, rok);
                if (vec) {
                    if (rok) {
                        lo[i] = *(const float4 *)(src + 2 * (ro + x0 + 4 * cq));
                        hi[i] = *(const float4 *)(src + 2 * (ro + x0 + 4 * cq) + 4);
                    }
                } else {
                    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int gx = x0 + 4 * cq + e;
                        if (rok && gx < S) {
                            a[2 * e] = iload(0, ro, gx);
                            a[2 * e + 1] = iload(1, ro, gx);
                        }
                    }
                    lo[i] = make_float4(a[0], a[1], a[2], a[3]);
                    hi[i] = make_float4(a[4], a[5], a[6], a[7]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < G::HPT; ++i) {
            const int slot = tid + i * kBlurThreads;
            h[i] = 0.f;
            if (R > 0 && slot < 2 * G::NH) {
                const int ch = slot >= G::NH, r = slot - ch * G::NH;
                const int l = r / (2 * R), e = r - l * (2 * R);
                const int gx = e < R ? x0 - R + e : x0 + kBlurTX + (e - R);
                bool ok;
                const size_t ro = row_of(l, ok);
                if (ok && gx >= 0 && gx < S) h[i] = iload(ch, ro, gx);
            }
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int r = tid + i * kBlurThreads;
            if (r < G::NQ) {
                const int l = r >> 4, cq = r & 15;
                *(float4 *)&tile_s[0][l][H4 + 4 * cq] = make_float4(lo[i].x, lo[i].z, hi[i].x, hi[i].z);
                *(float4 *)&tile_s[1][l][H4 + 4 * cq] = make_float4(lo[i].y, lo[i].w, hi[i].y, hi[i].w);
            }
        }
#pragma unroll
        for (int i = 0; i < G::HPT; ++i) {
            const int slot = tid + i * kBlurThreads;
            if (R > 0 && slot < 2 * G::NH) {
                const int ch = slot >= G::NH, r = slot - ch * G::NH;
                const int l = r / (2 * R), e = r - l * (2 * R);
                tile_s[ch][l][e < R ? H4 - R + e : H4 + kBlurTX + (e - R)] = h[i];
            }
        }
    } else {
        float4 q[G::QPT];
        float h[G::HPT];
        if (vec) {
#pragma unroll
            for (int i = 0; i < G::QPT; ++i) {
                const int slot = tid + i * kBlurThreads;
                q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (slot < 2 * G::NQ) {
                    const int ch = slot >= G::NQ, r = slot - ch * G::NQ;
                    const int l = r >> 4, cq = r & 15;
                    bool rok;
                    const size_t ro = row_of(l, rok);
                    if (rok) q[i] = *(const float4 *)(src + ch * plane + ro + x0 + 4 * cq);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < G::QPT; ++i) {
                const int slot = tid + i * kBlurThreads;
                float v[4] = {0.f, 0.f, 0.f, 0.f};
                if (slot < 2 * G::NQ) {
                    const int ch = slot >= G::NQ, r = slot - ch * G::NQ;
                    const int l = r >> 4, cq = r & 15;
                    bool rok;
                    const size_t ro = row_of(l, rok);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        int gx = x0 + 4 * cq + e;
                        bool ok = rok;
                        if (!ADJ) gx = min(gx, S - 1);
                        else ok = ok && gx < S;
                        if (ok) v[e] = src[ch * plane + ro + gx];
                    }
                }
                q[i] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
#pragma unroll
        for (int i = 0; i < G::HPT; ++i) {
            const int slot = tid + i * kBlurThreads;
            h[i] = 0.f;
            if (R > 0 && slot < 2 * G::NH) {
                const int ch = slot >= G::NH, r = slot - ch * G::NH;
                const int l = r / (2 * R), e = r - l * (2 * R);
                int gx = e < R ? x0 - R + e : x0 + kBlurTX + (e - R);
                bool ok;
                const size_t ro = row_of(l, ok);
                if (!ADJ) gx = min(max(gx, 0), S - 1);
                else ok = ok && gx >= 0 && gx < S;
                if (ok) h[i] = src[ch * plane + ro + gx];
            }
        }
#pragma unroll
        for (int i = 0; i < G::QPT; ++i) {
            const int slot = tid + i * kBlurThreads;
            if (slot < 2 * G::NQ) {
                const int ch = slot >= G::NQ, r = slot - ch * G::NQ;
                *(float4 *)&tile_s[ch][r >> 4][H4 + 4 * (r & 15)] = q[i];
            }
        }
#pragma unroll
        for (int i = 0; i < G::HPT; ++i) {
            const int slot = tid + i * kBlurThreads;
            if (R > 0 && slot < 2 * G::NH) {
                const int ch = slot >= G::NH, r = slot - ch * G::NH;
                const int l = r / (2 * R), e = r - l * (2 * R);
                tile_s[ch][l][e < R ? H4 - R + e : H4 + kBlurTX + (e - R)] = h[i];
            }
        }
    }
    __syncthreads();

    float w[K], cum[R + 1];
    {
        float c = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            w[j] = J.w[j];
            if (j <= R) {
                c += w[j];
                cum[j] = c;
            }
        }
    }
    const int lane = tid & (kBlurTX - 1);
    const int x = x0 + lane;
    const int lr0 = (tid / kBlurTX) * G::WR;                  // first output row of this wave (tile-local)
    // horizontal filter of staged row l at this lane's column
    auto hfilter = [&](int l, float &ha, float &hb) {
        const float *pa = &tile_s[0][l][H4 - R + lane], *pb = &tile_s[1][l][H4 - R + lane];
        ha = 0.f;
        hb = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            ha += w[j] * pa[j];
            hb += w[j] * pb[j];
        }
        if (ADJ && R > 0) {
            if (x == 0)               // taps clamped onto column 0: column i at element H4 + i
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    ha += cum[R - 1 - i] * tile_s[0][l][H4 + i];
                    hb += cum[R - 1 - i] * tile_s[1][l][H4 + i];
                }
            if (x == S - 1)           // column S-1-i at element H4 + lane - i
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    ha += cum[R - 1 - i] * tile_s[0][l][H4 + lane - i];
                    hb += cum[R - 1 - i] * tile_s[1][l][H4 + lane - i];
                }
        }
    };
    float ra[K], rb[K];       // ring: ra[j] holds staged row (l - 2R + j)
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        hfilter(lr0 + j, ra[j], rb[j]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < G::WR; ++i) {
        hfilter(lr0 + 2 * R + i, ra[2 * R], rb[2 * R]);
        const int yy = y0 + lr0 + i;
        float va = 0.f, vb = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            va += w[j] * ra[j];
            vb += w[j] * rb[j];
        }
        if (ADJ && R > 0) {
            if (yy == 0) {             // taps clamped onto row 0: rows 0..R-1 sit at ring R..2R-1
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    va += cum[R - 1 - k] * ra[R + k];
                    vb += cum[R - 1 - k] * rb[R + k];
                }
            }
            if (yy == S - 1) {         // rows S-1-k sit at ring R-k
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    va += cum[R - 1 - k] * ra[R - k];
                    vb += cum[R - 1 - k] * rb[R - k];
                }
            }
        }
        if (yy < S && x < S) {
            const size_t o = (size_t)yy * S + x;
            if (IL && !ADJ) {
                *(float2 *)(dst + 2 * o) = make_float2(va, vb);
            } else {
                dst[o] = va;
                dst[plane + o] = vb;
            }
        }
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            ra[j] = ra[j + 1];
            rb[j] = rb[j + 1];
        }
        // keep each row's LDS reads next to their use: hoisting the reads of
        // many rows ahead of the arithmetic exhausts the register file
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <bool ADJ, bool IL>
static hipError_t launch_r(int R, dim3 grid, const BlurJob *jobs, int njobs, const BlurJob &single, int per_map,
                           const float *in, float *out, hipStream_t s) {
#define DSM_BR(RR)                                                                                                    \
    case RR:                                                                                                         \
        hipLaunchKernelGGL((blur_kernel<ADJ, RR, IL>), grid, dim3(kBlurThreads), 0, s, jobs, njobs, single, per_map, \
                           in, out);                                                                                  \
        break;
    switch (R) {
        DSM_BR(0) DSM_BR(1) DSM_BR(2) DSM_BR(3) DSM_BR(4) DSM_BR(5) DSM_BR(6) DSM_BR(7)
        DSM_BR(8) DSM_BR(9) DSM_BR(10) DSM_BR(11) DSM_BR(12) DSM_BR(13) DSM_BR(14) DSM_BR(15)
        default: return hipErrorInvalidValue;
    }
#undef DSM_BR
    return hipGetLastError();
}

int blur_tiles_x(int S) { return (S + kBlurTX - 1) / kBlurTX; }
int blur_tiles(int S, int R) { return blur_tiles_x(S) * ((S + blur_ty(R) - 1) / blur_ty(R)); }
int blur_tile_height(int R) { return blur_ty(R); }

// jobs_dev: njobs jobs of one radius R (job.k == 2R + 1), tile offsets from 0.
hipError_t launch_blur(const BlurJob *jobs_dev, int njobs, int total_tiles, const float *in, float *out,
                       bool adjoint, int R, hipStream_t s) {
    if (total_tiles == 0 || njobs == 0) return hipSuccess;
    BlurJob none{};
    if (adjoint) return launch_r<true, true>(R, dim3(total_tiles), jobs_dev, njobs, none, 1, in, out, s);
    return launch_r<false, true>(R, dim3(total_tiles), jobs_dev, njobs, none, 1, in, out, s);
}

hipError_t launch_blur_uniform(const BlurJob &job, int n_maps, const float *in, float *out, bool adjoint,
                               hipStream_t s) {
    const int R = (job.k - 1) / 2;
    BlurJob j = job;
    j.tile_off = 0;
    j.tiles_x = blur_tiles_x(job.S);
    const int per_map = blur_tiles(job.S, R);
    const long long total = (long long)per_map * n_maps;
    if (total >= (1LL << 31)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)total);
    if (adjoint) return launch_r<true, false>(R, grid, nullptr, 0, j, per_map, in, out, s);
    return launch_r<false, false>(R, grid, nullptr, 0, j, per_map, in, out, s);
}

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
