// unet.hip -- the learned warm start: a U-Net whose forward pass, backward
// pass and Adam updates run in the kernels below.  3x3 convolutions are
// implicit GEMMs on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16, float32
// accumulation); activations are NHWC bfloat16, gradients float32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/msr_unet.h"

namespace {

using bf16 = __bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr size_t kAlign = 256;
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Loads of 8 consecutive channels (16-byte aligned for bf16, 32 for float).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bf16x8 load8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x8 load8(const float* p) {
    const float4 u = reinterpret_cast<const float4*>(p)[0];
    const float4 v = reinterpret_cast<const float4*>(p)[1];
    bf16x8 r;
    r[0] = (bf16)u.x;
    r[1] = (bf16)u.y;
    r[2] = (bf16)u.z;
    r[3] = (bf16)u.w;
    r[4] = (bf16)v.x;
    r[5] = (bf16)v.y;
    r[6] = (bf16)v.z;
    r[7] = (bf16)v.w;
    return r;
}
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 r;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (bf16)0.0f;
    return r;
}

// The input of a 3x3 convolution: channels [0, c1) from x1, read at
// (y >> up1, x >> up1) of a (H >> up1) x (W >> up1) tensor (nearest
// upsampling when up1 = 1), channels [c1, c1 + c2) from x2 at (y, x).
template <typename T>
struct ConvIn {
    const T* x1;
    int c1, up1;
    const T* x2;
    int c2;
};

// Channels [k, k + 8) of the im2col row of output pixel (b, y, x): tap
// t = k / cin at offset (t / 3 - 1, t % 3 - 1); zero outside the image and
// for k >= 9 cin.
template <typename T>
__device__ __forceinline__ bf16x8 im2col8(const ConvIn<T>& in, int H, int W, int b, int y, int x, int k) {
    const int cin = in.c1 + in.c2;
    if (k >= 9 * cin) return zero8();
    const int t = k / cin;
    const int ci = k - t * cin;
    const int sy = y + t / 3 - 1, sx = x + t % 3 - 1;
    if (sy < 0 || sy >= H || sx < 0 || sx >= W) return zero8();
    if (ci < in.c1) {
        const int h = H >> in.up1, w = W >> in.up1;
        return load8(in.x1 + (((size_t)b * h + (sy >> in.up1)) * w + (sx >> in.up1)) * in.c1 + ci);
    }
    return load8(in.x2 + (((size_t)b * H + sy) * W + sx) * in.c2 + (ci - in.c1));
}

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM: D[p][co] = sum_k A[p][k] W[co][k],
// A = im2col of the input, k = tap * cin + ci.  A block computes an 8 x 16
// pixel tile of one image for 64 output channels; its 4 waves take two tile
// rows (32 pixels) x 64 channels each (two 32x32 MFMA tiles).  The input is
// staged 32 channels at a time as the 10 x 18 halo tile around the output
// tile (zero outside the image), once per chunk, so each of the nine taps of
// a chunk reads its A operand from LDS at a shifted pixel: no per-step
// index arithmetic or bounds checks.  The weights of one (chunk, tap) step
// (64 x 32) go through a second double buffer, loaded one step ahead.
// ---------------------------------------------------------------------------
constexpr int CBK = 32, CLD = CBK + 8;
#ifndef MSR_UNET_WAVE_ROWS
#define MSR_UNET_WAVE_ROWS 2
#endif
constexpr int WROWS = MSR_UNET_WAVE_ROWS;                  // tile rows of a wave: 32 pixels per two rows
constexpr int MT = WROWS / 2;                              // 32-pixel MFMA tiles per wave
constexpr int TR = 4 * WROWS, TC = 16, HR = TR + 2, HC = TC + 2;  // output tile, halo tile
constexpr int NHALO = HR * HC;                             // halo pixels
constexpr int HLD = CBK + 8;                               // bf16 per halo pixel in LDS (80 B: spreads the banks)
constexpr int HITEMS = NHALO * (CBK / 8);                  // 16-byte groups of one halo chunk
constexpr int HPT = (HITEMS + 255) / 256;                  // ... per thread

struct ConvOut {
    int B, H, W;
    int cout, kpad;
    const bf16* w;      // [cout][kpad]
    const float* bias;  // [cout] or null
    // forward: bf16 output with optional ReLU
    bf16* y;
    int relu;
    // backward (data): float outputs, channels [0, split) -> g1, [split, cout) -> g2;
    // each multiplied by (m > 0) when its mask is given; g2 accumulated when acc2
    float* g1;
    float* g2;
    const bf16* m1;
    const bf16* m2;
    int split, acc2;
};

// Output tiles of a layer (grid x of the convolution).
__host__ __device__ inline int conv_tiles(int B, int H, int W) { return B * ((H + TR - 1) / TR) * ((W + TC - 1) / TC); }

// Channels [ci, ci + 8) of input pixel (b, sy, sx); zero outside the image or
// beyond the input's channels (ci is a multiple of 8, and so is c1).
template <typename T>
__device__ __forceinline__ bf16x8 pixel8(const ConvIn<T>& in, int cin, int H, int W, int b, int sy, int sx, int ci) {
    if (ci >= cin || sy < 0 || sy >= H || sx < 0 || sx >= W) return zero8();
    if (ci < in.c1) {
        const int h = H >> in.up1, w = W >> in.up1;
        return load8(in.x1 + (((size_t)b * h + (sy >> in.up1)) * w + (sx >> in.up1)) * in.c1 + ci);
    }
    return load8(in.x2 + (((size_t)b * H + sy) * W + sx) * in.c2 + (ci - in.c1));
}

// NT 32-channel output tiles per wave (1 for layers of at most 32 output
// channels, else 2); the weights of a step are fetched WD steps ahead.
#ifndef MSR_UNET_WD
#define MSR_UNET_WD 3
#endif
#ifndef MSR_UNET_HALO_BUFS
#define MSR_UNET_HALO_BUFS 1
#endif
constexpr int WD = MSR_UNET_WD;
static_assert(9 % WD == 0, "the step loop advances WD steps at a time over 9 steps per chunk");
// halo buffers of a multi-chunk layer: 2 (the next chunk is written while the
// current one is read) or 1 (written after a barrier at the chunk's end: less
// LDS, one more barrier per chunk)
constexpr int HBUFS = MSR_UNET_HALO_BUFS;

// ONE: the input has at most 32 channels (one chunk, one halo buffer: half
// the LDS, so twice the resident blocks to cover the load latency).
template <typename T, bool BWD, int NT, bool ONE>
__global__ void __launch_bounds__(256) conv3x3_kernel(ConvIn<T> in, ConvOut o) {
    constexpr int BN = 32 * NT;  // output channels of a block
    __shared__ __attribute__((aligned(16))) bf16 Hs[ONE ? 1 : HBUFS][NHALO * HLD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BN * CLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (o.W + TC - 1) / TC, tiles_y = (o.H + TR - 1) / TR;
    const int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y, b = blockIdx.x / (tiles_x * tiles_y);
    const int y0 = ty * TR, x0 = tx * TC, n0 = blockIdx.y * BN;
    const int cin = in.c1 + in.c2;
    const int nsteps = 9 * ((cin + CBK - 1) / CBK);  // (chunk, tap) steps, a multiple of WD

    // halo items of this thread: pixel q / 4 of the halo tile, channels 8 (q % 4) of the chunk
    bf16x8 rh[HPT];
    auto fetch_halo = [&](int c0) {
#pragma unroll
        for (int u = 0; u < HPT; ++u) {
            const int q = tid + u * 256;
            const int hp = q >> 2;
            rh[u] = q < HITEMS ? pixel8(in, cin, o.H, o.W, b, y0 - 1 + hp / HC, x0 - 1 + hp % HC, c0 + (q & 3) * 8)
                               : zero8();
        }
    };
    auto stage_halo = [&](int buf) {
#pragma unroll
        for (int u = 0; u < HPT; ++u) {
            const int q = tid + u * 256;
            if (q < HITEMS) *reinterpret_cast<bf16x8*>(&Hs[buf][(q >> 2) * HLD + (q & 3) * 8]) = rh[u];
        }
    };
    // weights of step s = chunk * 9 + tap: row co, k = tap * cin + chunk * 32 + [0, 32);
    // WD steps in flight, in registers
    const int bco = n0 + tid / 4, bg = (tid % 4) * 8;
    const bool bthr = tid < 4 * BN;
    bf16x8 rb[WD];
    auto fetch_w = [&](int st, bf16x8& r) {
        const int c = st / 9, t = st - 9 * c;
        const int ci = c * CBK + bg;
        r = (bthr && st < nsteps && bco < o.cout && ci < cin) ? load8(o.w + (size_t)bco * o.kpad + t * cin + ci)
                                                               : zero8();
    };
    auto stage_w = [&](int buf, const bf16x8& r) {
        if (bthr) *reinterpret_cast<bf16x8*>(&Bs[buf][(tid / 4) * CLD + bg]) = r;
    };

    // A operand rows of this lane in MFMA tile m: tile pixel
    // (WROWS wave + 2 m + (l >> 4), l & 15), l = lane & 31
    const int pl = lane & 31;
    const int hbase = (WROWS * wave + (pl >> 4) + 1) * HC + (pl & 15) + 1;  // halo index of the pixel (m = 0)
    const int ko = (lane >> 5) * 8;

    f32x16 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x16{};
    fetch_halo(0);
    fetch_w(0, rb[0]);
    stage_halo(0);
    stage_w(0, rb[0]);
#pragma unroll
    for (int d = 1; d < WD; ++d) fetch_w(d, rb[d]);
    __syncthreads();
    int hcur = 0;
    // steps st = s0 + j, j < WD: register slot j holds step st + 1's weights
    // at the top of step st (for j = WD - 1, slot 0 receives step st + WD)
    for (int s0 = 0; s0 < nsteps; s0 += WD) {
#pragma unroll
        for (int j = 0; j < WD; ++j) {
            const int st = s0 + j;
            const int t = st % 9;
            const int cur = st & 1;
            const bool more = st + 1 < nsteps;
            if (!ONE && t == 0 && st + 9 < nsteps) fetch_halo((st / 9 + 1) * CBK);  // the next chunk, in registers
            const int hp = hbase + (t / 3 - 1) * HC + (t % 3 - 1);
#pragma unroll
            for (int kk = 0; kk < CBK; kk += 16) {
                bf16x8 av[MT], bv[NT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    av[m] = *reinterpret_cast<const bf16x8*>(&Hs[hcur][(hp + 2 * m * HC) * HLD + kk + ko]);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    bv[n] = *reinterpret_cast<const bf16x8*>(&Bs[cur][(32 * n + pl) * CLD + kk + ko]);
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bv[n], acc[m][n], 0, 0, 0);
            }
            // the other buffers were last read in the previous step (weights)
            // or chunk (halo), which every thread finished before the barrier
            // that ended it
            const int nxt = (j + 1) % WD;  // slot of step st + 1
            if (more) stage_w(cur ^ 1, rb[nxt]);
            fetch_w(st + WD, rb[j]);            // slot j is free again: step st + WD
            if constexpr (!ONE && HBUFS == 2) {
                if (t == 8 && more) stage_halo(hcur ^ 1);
            }
            __syncthreads();
            if constexpr (!ONE && HBUFS == 2) {
                if (t == 8) hcur ^= 1;
            }
            if constexpr (!ONE && HBUFS == 1) {
                // every wave has read this chunk's halo (the barrier above)
                if (t == 8 && more) {
                    stage_halo(0);
                    __syncthreads();
                }
            }
        }
    }

#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = n0 + nt * 32 + pl;
        if (co >= o.cout) continue;
        const float bias = o.bias ? o.bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int q = (WROWS * wave + 2 * m) * 16 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);  // tile pixel
            const int y = y0 + (q >> 4), x = x0 + (q & 15);
            if (y >= o.H || x >= o.W) continue;
            const size_t p = ((size_t)b * o.H + y) * o.W + x;
            const float v = acc[m][nt][r] + bias;
            if constexpr (!BWD) {
                o.y[p * o.cout + co] = (bf16)(o.relu ? fmaxf(v, 0.0f) : v);
            } else {
                if (co < o.split) {
                    const size_t i = p * o.split + co;
                    o.g1[i] = (o.m1 && !((float)o.m1[i] > 0.0f)) ? 0.0f : v;
                } else {
                    const int l2 = o.cout - o.split;
                    const size_t i = p * l2 + (co - o.split);
                    const float g = (o.m2 && !((float)o.m2[i] > 0.0f)) ? 0.0f : v;
                    o.g2[i] = o.acc2 ? o.g2[i] + g : g;
                }
            }
        }
    }
}

// Launches the convolution with the output-channel blocking of `cout`.
template <typename T, bool BWD>
void launch_conv(const ConvIn<T>& in, const ConvOut& o, hipStream_t s) {
    const unsigned tiles = (unsigned)conv_tiles(o.B, o.H, o.W);
    const bool one = in.c1 + in.c2 <= CBK;
    if (o.cout <= 32) {
        if (one) hipLaunchKernelGGL((conv3x3_kernel<T, BWD, 1, true>), dim3(tiles, 1), dim3(256), 0, s, in, o);
        else hipLaunchKernelGGL((conv3x3_kernel<T, BWD, 1, false>), dim3(tiles, 1), dim3(256), 0, s, in, o);
    } else {
        const dim3 g(tiles, (o.cout + 63) / 64);
        if (one) hipLaunchKernelGGL((conv3x3_kernel<T, BWD, 2, true>), g, dim3(256), 0, s, in, o);
        else hipLaunchKernelGGL((conv3x3_kernel<T, BWD, 2, false>), g, dim3(256), 0, s, in, o);
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[co][k] = sum_p G[p][co] A[p][k] over a chunk of pixels
// per block (grid z), partial tiles reduced afterwards.  Block: 64 output
// channels x 64 k, 4 waves of 32 x 32; 32 pixels staged per step, stored
// transposed in LDS so each MFMA operand is one 16-byte read.
// ---------------------------------------------------------------------------
struct WGradArgs {
    const float* g;  // [P][cout]
    int B, H, W, cout, kpad, chunk;
    float* part;     // [gridDim.z][cout][kpad]
};

template <typename T>
__global__ void __launch_bounds__(256) conv3x3_wgrad_kernel(ConvIn<T> in, WGradArgs a) {
    __shared__ __attribute__((aligned(16))) bf16 Gs[64 * CLD];
    __shared__ __attribute__((aligned(16))) bf16 Xs[64 * CLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int P = a.B * a.H * a.W, hw = a.H * a.W;
    const int c0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int pbeg = blockIdx.z * a.chunk, pend = min(P, pbeg + a.chunk);
    const int wc = (wave >> 1) * 32, wk = (wave & 1) * 32;
    const int lp = tid >> 3, lg = (tid & 7) * 8;  // staged pixel, 8-wide group

    f32x16 acc = {};
    for (int pp = pbeg; pp < pend; pp += 32) {
        const int p = pp + lp;
        const bool ok = p < pend;
        {
            const int co = c0 + lg;
            float gv[8];
            if (ok && co < a.cout) {
                const float4 u = *reinterpret_cast<const float4*>(a.g + (size_t)p * a.cout + co);
                const float4 v = *reinterpret_cast<const float4*>(a.g + (size_t)p * a.cout + co + 4);
                gv[0] = u.x, gv[1] = u.y, gv[2] = u.z, gv[3] = u.w, gv[4] = v.x, gv[5] = v.y, gv[6] = v.z, gv[7] = v.w;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) gv[j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Gs[(lg + j) * CLD + lp] = (bf16)gv[j];
        }
        {
            bf16x8 xv = zero8();
            if (ok && k0 + lg < a.kpad) {
                const int b = p / hw, r = p - b * hw, y = r / a.W, x = r - y * a.W;
                xv = im2col8(in, a.H, a.W, b, y, x, k0 + lg);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Xs[(lg + j) * CLD + lp] = xv[j];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 16) {
            const int po = kk + (lane >> 5) * 8;
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&Gs[(wc + (lane & 31)) * CLD + po]);
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Xs[(wk + (lane & 31)) * CLD + po]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int k = k0 + wk + (lane & 31);
    if (k >= a.kpad) return;
    float* part = a.part + (size_t)blockIdx.z * a.cout * a.kpad;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int co = c0 + wc + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (co < a.cout) part[(size_t)co * a.kpad + k] = acc[r];
    }
}

// out[i] = sum_z part[z][i]  (fixed order: deterministic)
__global__ void sum_parts_kernel(const float* __restrict__ part, int nz, size_t n, float* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int z = 0; z < nz; ++z) s += part[(size_t)z * n + i];
        out[i] = s;
    }
}

// Column sums of G [P][C] over pixel chunks: part[z][c] (bias gradients).
__global__ void colsum_kernel(const float* __restrict__ g, int P, int C, int chunk, float* __restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int pb = blockIdx.y * chunk, pe = min(P, pb + chunk);
    float s = 0.0f;
    for (int p = pb; p < pe; ++p) s += g[(size_t)p * C + c];
    part[(size_t)blockIdx.y * C + c] = s;
}

// ---------------------------------------------------------------------------
// Pooling, upsampling adjoints, head, loss, input/output, optimiser.
// ---------------------------------------------------------------------------
// 2x2 average pool, NHWC bf16: out (B, H/2, W/2, C).
__global__ void pool_kernel(const bf16* __restrict__ x, int B, int H, int W, int C, bf16* __restrict__ out) {
    const size_t n = (size_t)B * (H / 2) * (W / 2) * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int x2 = (int)(r % (W / 2));
        r /= (W / 2);
        const int y2 = (int)(r % (H / 2));
        const int b = (int)(r / (H / 2));
        const size_t base = (((size_t)b * H + 2 * y2) * W + 2 * x2) * C + c;
        const float s = (float)x[base] + (float)x[base + C] + (float)x[base + (size_t)W * C] +
                        (float)x[base + (size_t)W * C + C];
        out[i] = (bf16)(0.25f * s);
    }
}

// G[b,y,x,c] = (dpool[b,y/2,x/2,c] / 4 + dskip[b,y,x,c]) * (e > 0): the
// gradient of an encoder output feeding both the pool and the skip.
__global__ void pool_back_kernel(const float* __restrict__ dpool, const float* __restrict__ dskip,
                                 const bf16* __restrict__ e, int B, int H, int W, int C, float* __restrict__ g) {
    const size_t n = (size_t)B * H * W * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        float v = dskip ? dskip[i] : 0.0f;
        if (dpool) v += 0.25f * dpool[(((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
        g[i] = (float)e[i] > 0.0f ? v : 0.0f;
    }
}

// G[b,y,x,c] = (sum of dup over the 2x2 block) * (d > 0): the adjoint of the
// nearest upsampling of d (B, H, W, C); dup is (B, 2H, 2W, C).
__global__ void up_back_kernel(const float* __restrict__ dup, const bf16* __restrict__ d, int B, int H, int W, int C,
                               float* __restrict__ g) {
    const size_t n = (size_t)B * H * W * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        const size_t base = (((size_t)b * 2 * H + 2 * y) * 2 * W + 2 * x) * C + c;
        const size_t row = (size_t)2 * W * C;
        const float s = dup[base] + dup[base + C] + dup[base + row] + dup[base + row + C];
        g[i] = (float)d[i] > 0.0f ? s : 0.0f;
    }
}

// Input normalisation s = max |l| per image (1 when l = 0), in two passes:
// scale_partial_kernel's grid (nb, B) gives each image nb blocks that stride
// over its pixels and leave one maximum each in part[b][nb]; scale_kernel then
// takes the maximum of those nb values per image. A max is order-free, so the
// result does not depend on the split.
constexpr int kScaleBlocks = 256;

__device__ __forceinline__ float block_max256(float m, float* red) {
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    return red[0];
}

__global__ void scale_partial_kernel(const float* __restrict__ low, int HW, int nb, float* __restrict__ part) {
    __shared__ float red[256];
    const float* l = low + (size_t)blockIdx.y * HW;
    float m = 0.0f;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < HW; i += nb * 256) m = fmaxf(m, fabsf(l[i]));
    m = block_max256(m, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * nb + blockIdx.x] = m;
}

__global__ void scale_kernel(const float* __restrict__ part, int nb, float* __restrict__ scale) {
    __shared__ float red[256];
    const float* q = part + (size_t)blockIdx.x * nb;
    float m = 0.0f;
    for (int i = threadIdx.x; i < nb; i += 256) m = fmaxf(m, q[i]);
    m = block_max256(m, red);
    if (threadIdx.x == 0) scale[blockIdx.x] = m > 0.0f ? m : 1.0f;
}

// NHWC input with 8 channels: (i_H / s, l / s, 0, ...).
__global__ void pack_kernel(const float* __restrict__ dh, const float* __restrict__ low,
                            const float* __restrict__ scale, int B, int HW, bf16* __restrict__ x) {
    const size_t n = (size_t)B * HW;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float inv = 1.0f / scale[i / HW];
        bf16x8 v = zero8();
        v[0] = (bf16)(dh[i] * inv);
        v[1] = (bf16)(low[i] * inv);
        *reinterpret_cast<bf16x8*>(x + i * 8) = v;
    }
}

// Head: out[p] = b + sum_c w[c] x[p][c] (float32), x bf16 with C channels.
__global__ void head_kernel(const bf16* __restrict__ x, int P, int C, const float* __restrict__ wb,
                            float* __restrict__ out) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        float s = wb[C];
        for (int c = 0; c < C; c += 8) {
            const bf16x8 v = load8(x + (size_t)p * C + c);
#pragma unroll
            for (int j = 0; j < 8; ++j) s = fmaf(wb[c + j], (float)v[j], s);
        }
        out[p] = s;
    }
}

// Warm start x0 = s max(out, 0).
__global__ void unpack_kernel(const float* __restrict__ out, const float* __restrict__ scale, int B, int HW,
                              float* __restrict__ x0) {
    const size_t n = (size_t)B * HW;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x0[i] = scale[i / HW] * fmaxf(out[i], 0.0f);
}

// Loss partials sum (out - t/s)^2 per block and gout = 2 (out - t/s) / n.
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                                   const float* __restrict__ scale, int B, int HW,
                                                   float* __restrict__ gout, double* __restrict__ part) {
    __shared__ double red[256];
    const size_t n = (size_t)B * HW;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float d = out[i] - target[i] / scale[i / HW];
        s += (double)d * d;
        gout[i] = 2.0f * d / (float)n;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_double_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s;
    }
}

// Head backward: gx[p][c] = gout[p] w[c] (x > 0); per-block partials of
// dw[c] = sum_p gout[p] x[p][c] and db = sum_p gout[p] (blockDim = 256, C < 256).
__global__ void __launch_bounds__(256) head_back_kernel(const bf16* __restrict__ x, const float* __restrict__ gout,
                                                        int P, int C, const float* __restrict__ wb,
                                                        float* __restrict__ gx, float* __restrict__ part, int chunk) {
    const int pb = blockIdx.x * chunk, pe = min(P, pb + chunk);
    // one thread per channel (and one for the bias) accumulates over the chunk
    float s = 0.0f;
    if ((int)threadIdx.x <= C) {
        for (int p = pb; p < pe; ++p) {
            const float g = gout[p];
            s += (int)threadIdx.x < C ? g * (float)x[(size_t)p * C + threadIdx.x] : g;
        }
        part[(size_t)blockIdx.x * (C + 1) + threadIdx.x] = s;
    }
    for (int i = pb * C + threadIdx.x; i < pe * C; i += 256) {
        const int p = i / C, c = i - p * C;
        gx[i] = (float)x[i] > 0.0f ? gout[p] * wb[c] : 0.0f;
    }
}

// Adam on the float32 master vector; the bias corrections are folded into
// lr_t = lr sqrt(1 - b2^t) / (1 - b1^t) and eps_t = eps sqrt(1 - b2^t).
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, size_t n, float b1, float b2, float lr_t, float eps_t) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
    }
}

// bf16 weights of one convolution from the master copy: w16[co][k] (k < 9 cin,
// zero above) and the flipped, transposed copy for the data gradient:
// wt[ci][(8 - t) cout + co] = w[co][t cin + ci].
__global__ void weights_kernel(const float* __restrict__ w, int cout, int cin, int kpad, int kpadt,
                               bf16* __restrict__ w16, bf16* __restrict__ wt) {
    const int K = 9 * cin;
    const size_t n = (size_t)cout * kpad;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int co = (int)(i / kpad), k = (int)(i % kpad);
        const float v = k < K ? w[i] : 0.0f;
        w16[i] = (bf16)v;
        if (k < K) {
            const int t = k / cin, ci = k - t * cin;
            wt[(size_t)ci * kpadt + (8 - t) * cout + co] = (bf16)v;
        }
    }
    // zero the padding of wt (k >= 9 cout)
    const size_t nt = (size_t)cin * (kpadt - 9 * cout);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += (size_t)gridDim.x * blockDim.x) {
        const int span = kpadt - 9 * cout;
        const int ci = (int)(i / span), k = 9 * cout + (int)(i % span);
        wt[(size_t)ci * kpadt + k] = (bf16)0.0f;
    }
}

// Zero the parameter gradient entries a convolution never touches (k >= 9 cin).
__global__ void fill_kernel(float* __restrict__ p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

unsigned grid_for(size_t n, unsigned b = 256, unsigned cap = 4096) {
    return (unsigned)std::max<size_t>(1, std::min<size_t>(cap, (n + b - 1) / b));
}

// ---------------------------------------------------------------------------
// Network description
// ---------------------------------------------------------------------------
struct Layer {
    int cin, cout, kpad, kpadt;
    int c1, c2, up1;   // input split (decoder: upsampled c1 then skip c2)
    int level;         // resolution level
    size_t w_off, b_off;  // in the parameter vector (floats)
    size_t w16_off, wt_off;  // bf16 copies (elements)
};

struct Net {
    int in_ch = 2, cin0 = 8, width = 32, levels = 4;
    std::vector<Layer> L;  // enc (2 per level), dec (2 per level below the bottom)
    size_t head_off = 0, nparam = 0, nw16 = 0, nwt = 0;
};

bool make_net(const msr_unet_config* c, Net& n) {
    if (!c || c->in_channels < 1 || c->in_channels > 8 || c->base_width < 8 || c->base_width % 8 ||
        c->base_width > 128 || c->levels < 2 || c->levels > 6)
        return false;
    n.in_ch = c->in_channels;
    n.cin0 = 8;
    n.width = c->base_width;
    n.levels = c->levels;
    n.L.clear();
    size_t off = 0, o16 = 0, ot = 0;
    auto add = [&](int c1, int c2, int up1, int cout, int level) {
        Layer l{};
        l.c1 = c1;
        l.c2 = c2;
        l.up1 = up1;
        l.cin = c1 + c2;
        l.cout = cout;
        l.kpad = round_up(9 * l.cin, 32);
        l.kpadt = round_up(9 * cout, 32);
        l.level = level;
        l.w_off = off;
        off += (size_t)cout * l.kpad;
        l.b_off = off;
        off += cout;
        l.w16_off = o16;
        o16 += (size_t)cout * l.kpad;
        l.wt_off = ot;
        ot += (size_t)l.cin * l.kpadt;
        n.L.push_back(l);
    };
    int prev = n.cin0;
    for (int j = 0; j < n.levels; ++j) {
        const int w = n.width << j;
        add(prev, 0, 0, w, j);
        add(w, 0, 0, w, j);
        prev = w;
    }
    for (int j = n.levels - 2; j >= 0; --j) {
        const int w = n.width << j;
        add(prev, w, 1, w, j);
        add(w, 0, 0, w, j);
        prev = w;
    }
    n.head_off = off;
    off += n.width + 1;
    n.nparam = off;
    n.nw16 = o16;
    n.nwt = ot;
    return true;
}

int enc_idx(int j, int s) { return 2 * j + s; }                     // s = 0 first conv, 1 second
int dec_idx(const Net& n, int j, int s) { return 2 * n.levels + 2 * (n.levels - 2 - j) + s; }

// Workspace layout for (batch, H, W).
struct Plan {
    int B = 0, H = 0, W = 0;
    size_t params, m, v, grad, w16, wt;             // float / bf16 arrays
    size_t in0;                                     // bf16 (B, H, W, 8)
    std::vector<size_t> act;                        // per layer output, bf16
    std::vector<size_t> pin;                        // pooled input of level j >= 1, bf16
    std::vector<size_t> gact;                       // per layer output gradient, float
    std::vector<size_t> dpin;                       // gradient of pooled input, float
    std::vector<size_t> dskip;                      // gradient into the skip of level j, float
    size_t dup;                                     // full-resolution gradient of an upsampled input, float
    size_t out, gout, scale, part, dpart, lossv;
    size_t part_floats;
    size_t total;
};

int npix(const Plan& p, int level) { return p.B * (p.H >> level) * (p.W >> level); }

// Split-K chunk (pixels) of a weight-gradient launch: about 1024 blocks.
int wgrad_chunk(int P, int tiles) {
    int nz = std::max(1, std::min((P + 31) / 32, 1024 / std::max(tiles, 1)));
    int chunk = round_up((P + nz - 1) / nz, 32);
    return chunk;
}

bool make_plan(const Net& n, int B, int H, int W, Plan& p) {
    const int m = 1 << (n.levels - 1);
    if (B < 1 || H < m || W < m || H % m || W % m || (size_t)B * H * W > (size_t)1 << 31) return false;
    p.B = B;
    p.H = H;
    p.W = W;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    p.params = take(4 * n.nparam);
    p.m = take(4 * n.nparam);
    p.v = take(4 * n.nparam);
    p.grad = take(4 * n.nparam);
    p.w16 = take(2 * n.nw16);
    p.wt = take(2 * n.nwt);
    p.in0 = take(2 * (size_t)npix(p, 0) * n.cin0);
    p.act.resize(n.L.size());
    p.gact.resize(n.L.size());
    for (size_t i = 0; i < n.L.size(); ++i) {
        const size_t e = (size_t)npix(p, n.L[i].level) * n.L[i].cout;
        p.act[i] = take(2 * e);
        p.gact[i] = take(4 * e);
    }
    p.pin.assign(n.levels, 0);
    p.dpin.assign(n.levels, 0);
    p.dskip.assign(n.levels, 0);
    for (int j = 1; j < n.levels; ++j) {
        const size_t e = (size_t)npix(p, j) * (n.width << (j - 1));
        p.pin[j] = take(2 * e);
        p.dpin[j] = take(4 * e);
    }
    size_t dup = 0;
    for (int j = 0; j + 1 < n.levels; ++j) {
        p.dskip[j] = take(4 * (size_t)npix(p, j) * (n.width << j));
        dup = std::max(dup, (size_t)npix(p, j) * (n.width << (j + 1)));
    }
    p.dup = take(4 * dup);
    p.out = take(4 * (size_t)npix(p, 0));
    p.gout = take(4 * (size_t)npix(p, 0));
    p.scale = take(4 * (size_t)B);
    size_t pf = 0;
    for (const Layer& l : n.L) {
        const int P = npix(p, l.level);
        const int tiles = ((l.cout + 63) / 64) * ((l.kpad + 63) / 64);
        const int chunk = wgrad_chunk(P, tiles);
        const int nz = (P + chunk - 1) / chunk;
        pf = std::max(pf, (size_t)nz * l.cout * l.kpad);
        pf = std::max(pf, (size_t)((P + 1023) / 1024) * l.cout);  // bias partials
    }
    pf = std::max(pf, (size_t)((npix(p, 0) + 1023) / 1024) * (n.width + 1));  // head partials
    pf = std::max(pf, (size_t)B * kScaleBlocks);                              // input-scale partials
    p.part_floats = pf;
    p.part = take(4 * pf);
    p.dpart = take(8 * 1024);
    p.lossv = take(8);
    p.total = off;
    return true;
}

}  // namespace

struct msr_unet {
    msr_unet_config cfg{};
    Net net;
    Plan plan;
    char* ws = nullptr;
    long long step = 0;
    bool have_params = false;
    std::string err;
};

namespace {

msr_status ufail(msr_unet* u, msr_status s, const char* fmt, ...) {
    if (u) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        u->err = buf;
    }
    return s;
}

#define UHIP(u, expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ufail(u, MSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
#define ULAUNCH(u)                                                                                        \
    do {                                                                                                  \
        hipError_t e_ = hipGetLastError();                                                                \
        if (e_ != hipSuccess) return ufail(u, MSR_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)
#define UTRY(expr)                      \
    do {                                \
        msr_status st_ = (expr);        \
        if (st_ != MSR_OK) return st_;  \
    } while (0)

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct Run {
    msr_unet* u;
    const Net& n;
    const Plan& p;
    int B;  // images in this call (<= p.B)
    hipStream_t s;

    template <typename X>
    X* at(size_t off) const { return reinterpret_cast<X*>(u->ws + off); }
    int np(int level) const { return B * (p.H >> level) * (p.W >> level); }
    int hh(int level) const { return p.H >> level; }
    int ww(int level) const { return p.W >> level; }
    bf16* act(int i) const { return at<bf16>(p.act[i]); }
    float* gact(int i) const { return at<float>(p.gact[i]); }
    float* params() const { return at<float>(p.params); }
    float* grad() const { return at<float>(p.grad); }
    bf16* w16(const Layer& l) const { return at<bf16>(p.w16) + l.w16_off; }
    bf16* wt(const Layer& l) const { return at<bf16>(p.wt) + l.wt_off; }

    // input of layer i as the forward pass reads it
    ConvIn<bf16> input(int i) const {
        const Layer& l = n.L[i];
        ConvIn<bf16> in{};
        in.c1 = l.c1;
        in.up1 = l.up1;
        in.c2 = l.c2;
        const int nenc = 2 * n.levels;
        if (i == 0) {
            in.x1 = at<bf16>(p.in0);
        } else if (i < nenc) {
            in.x1 = (i % 2 == 1) ? act(i - 1) : at<bf16>(p.pin[l.level]);
        } else {
            const int j = l.level;
            const int s = (i - nenc) % 2;
            if (s == 0) {
                // upsampled output of the level below (bottleneck or decoder level j + 1), then the skip
                const int below = (j + 1 == n.levels - 1) ? enc_idx(j + 1, 1) : dec_idx(n, j + 1, 1);
                in.x1 = act(below);
                in.x2 = act(enc_idx(j, 1));
            } else {
                in.x1 = act(i - 1);
            }
        }
        return in;
    }

    msr_status conv_fwd(int i) {
        const Layer& l = n.L[i];
        ConvOut o{};
        o.B = B;
        o.H = hh(l.level);
        o.W = ww(l.level);
        o.cout = l.cout;
        o.kpad = l.kpad;
        o.w = w16(l);
        o.bias = params() + l.b_off;
        o.y = act(i);
        o.relu = 1;
        launch_conv<bf16, false>(input(i), o, s);
        ULAUNCH(u);
        return MSR_OK;
    }

    msr_status forward() {
        const int nenc = 2 * n.levels;
        for (int j = 0; j < n.levels; ++j) {
            if (j > 0) {
                const int C = n.width << (j - 1);
                const size_t e = (size_t)np(j) * C;
                hipLaunchKernelGGL(pool_kernel, dim3(grid_for(e)), dim3(256), 0, s, act(enc_idx(j - 1, 1)), B,
                                   hh(j - 1), ww(j - 1), C, at<bf16>(p.pin[j]));
                ULAUNCH(u);
            }
            UTRY(conv_fwd(enc_idx(j, 0)));
            UTRY(conv_fwd(enc_idx(j, 1)));
        }
        for (int i = nenc; i < (int)n.L.size(); ++i) UTRY(conv_fwd(i));
        const int top = (int)n.L.size() - 1;
        hipLaunchKernelGGL(head_kernel, dim3(grid_for(np(0))), dim3(256), 0, s, act(top), np(0), n.width,
                           params() + n.head_off, at<float>(p.out));
        ULAUNCH(u);
        return MSR_OK;
    }

    // dW, db of layer i from its output gradient and its input
    msr_status wgrad(int i) {
        const Layer& l = n.L[i];
        const int P = np(l.level);
        WGradArgs a{};
        a.g = gact(i);
        a.B = B;
        a.H = hh(l.level);
        a.W = ww(l.level);
        a.cout = l.cout;
        a.kpad = l.kpad;
        const int tiles = ((l.cout + 63) / 64) * ((l.kpad + 63) / 64);
        a.chunk = wgrad_chunk(P, tiles);
        const int nz = (P + a.chunk - 1) / a.chunk;
        if ((size_t)nz * l.cout * l.kpad > p.part_floats) return ufail(u, MSR_ERR_INVALID, "partials too small");
        a.part = at<float>(p.part);
        hipLaunchKernelGGL(conv3x3_wgrad_kernel<bf16>, dim3((l.cout + 63) / 64, (l.kpad + 63) / 64, nz), dim3(256), 0,
                           s, input(i), a);
        ULAUNCH(u);
        const size_t nw = (size_t)l.cout * l.kpad;
        hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(nw)), dim3(256), 0, s, at<float>(p.part), nz, nw,
                           grad() + l.w_off);
        ULAUNCH(u);
        const int chunk = 1024, nb = (P + chunk - 1) / chunk;
        hipLaunchKernelGGL(colsum_kernel, dim3((l.cout + 255) / 256, nb), dim3(256), 0, s, gact(i), P, l.cout, chunk,
                           at<float>(p.part));
        ULAUNCH(u);
        hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(l.cout)), dim3(256), 0, s, at<float>(p.part), nb,
                           (size_t)l.cout, grad() + l.b_off);
        ULAUNCH(u);
        return MSR_OK;
    }

    // data gradient of layer i: routed to g1 (first c1 input channels) and g2
    msr_status dgrad(int i, float* g1, const bf16* m1, float* g2, const bf16* m2, int acc2) {
        const Layer& l = n.L[i];
        ConvIn<float> in{};
        in.x1 = gact(i);
        in.c1 = l.cout;
        in.up1 = 0;
        in.x2 = nullptr;
        in.c2 = 0;
        ConvOut o{};
        o.B = B;
        o.H = hh(l.level);
        o.W = ww(l.level);
        o.cout = l.cin;
        o.kpad = l.kpadt;
        o.w = wt(l);
        o.bias = nullptr;
        o.g1 = g1;
        o.g2 = g2;
        o.m1 = m1;
        o.m2 = m2;
        o.split = l.c1;
        o.acc2 = acc2;
        launch_conv<float, true>(in, o, s);
        ULAUNCH(u);
        return MSR_OK;
    }

    msr_status loss(const float* target, double* loss_out) {
        const int P = np(0);
        const int nb = (int)std::min<size_t>(1024, (P + 255) / 256);
        hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, s, at<float>(p.out), target, at<float>(p.scale), B,
                           p.H * p.W, at<float>(p.gout), at<double>(p.dpart));
        ULAUNCH(u);
        hipLaunchKernelGGL(sum_double_kernel, dim3(1), dim3(64), 0, s, at<double>(p.dpart), nb, at<double>(p.lossv));
        ULAUNCH(u);
        double tot = 0.0;
        UHIP(u, hipMemcpyAsync(&tot, at<double>(p.lossv), sizeof(double), hipMemcpyDeviceToHost, s));
        UHIP(u, hipStreamSynchronize(s));
        if (loss_out) *loss_out = tot / (double)P;
        return MSR_OK;
    }

    msr_status backward() {
        const int top = (int)n.L.size() - 1;
        const int P0 = np(0);
        // parameters never touched by a gradient stay at zero
        hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n.nparam)), dim3(256), 0, s, grad(), n.nparam, 0.0f);
        ULAUNCH(u);
        // head
        {
            const int chunk = 1024, nb = (P0 + chunk - 1) / chunk;
            hipLaunchKernelGGL(head_back_kernel, dim3(nb), dim3(256), 0, s, act(top), at<float>(p.gout), P0, n.width,
                               params() + n.head_off, gact(top), at<float>(p.part), chunk);
            ULAUNCH(u);
            hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, at<float>(p.part), nb,
                               (size_t)(n.width + 1), grad() + n.head_off);
            ULAUNCH(u);
        }
        // decoder, top level first
        for (int j = 0; j + 1 < n.levels; ++j) {
            const int i2 = dec_idx(n, j, 1), i1 = dec_idx(n, j, 0);
            UTRY(wgrad(i2));
            UTRY(dgrad(i2, gact(i1), act(i1), nullptr, nullptr, 0));
            UTRY(wgrad(i1));
            UTRY(dgrad(i1, at<float>(p.dup), nullptr, at<float>(p.dskip[j]), nullptr, 0));
            const int below = (j + 1 == n.levels - 1) ? enc_idx(j + 1, 1) : dec_idx(n, j + 1, 1);
            const int C = n.L[below].cout;
            const size_t e = (size_t)np(j + 1) * C;
            hipLaunchKernelGGL(up_back_kernel, dim3(grid_for(e)), dim3(256), 0, s, at<float>(p.dup), act(below), B,
                               hh(j + 1), ww(j + 1), C, gact(below));
            ULAUNCH(u);
        }
        // encoder, bottom level first
        for (int j = n.levels - 1; j >= 0; --j) {
            const int i2 = enc_idx(j, 1), i1 = enc_idx(j, 0);
            if (j < n.levels - 1) {
                const int C = n.L[i2].cout;
                const size_t e = (size_t)np(j) * C;
                hipLaunchKernelGGL(pool_back_kernel, dim3(grid_for(e)), dim3(256), 0, s, at<float>(p.dpin[j + 1]),
                                   at<float>(p.dskip[j]), act(i2), B, hh(j), ww(j), C, gact(i2));
                ULAUNCH(u);
            }
            UTRY(wgrad(i2));
            UTRY(dgrad(i2, gact(i1), act(i1), nullptr, nullptr, 0));
            UTRY(wgrad(i1));
            if (j > 0) UTRY(dgrad(i1, at<float>(p.dpin[j]), nullptr, nullptr, nullptr, 0));
        }
        return MSR_OK;
    }

    msr_status refresh_weights() {
        for (const Layer& l : n.L) {
            const size_t e = (size_t)l.cout * l.kpad;
            hipLaunchKernelGGL(weights_kernel, dim3(grid_for(e)), dim3(256), 0, s, params() + l.w_off, l.cout, l.cin,
                               l.kpad, l.kpadt, w16(l), wt(l));
            ULAUNCH(u);
        }
        return MSR_OK;
    }

    msr_status prepare_input(const float* dh, const float* low) {
        const int HW = p.H * p.W;
        const int nb = std::min(kScaleBlocks, (HW + 255) / 256);
        hipLaunchKernelGGL(scale_partial_kernel, dim3(nb, B), dim3(256), 0, s, low, HW, nb, at<float>(p.part));
        ULAUNCH(u);
        hipLaunchKernelGGL(scale_kernel, dim3(B), dim3(256), 0, s, at<float>(p.part), nb, at<float>(p.scale));
        ULAUNCH(u);
        hipLaunchKernelGGL(pack_kernel, dim3(grid_for((size_t)B * HW)), dim3(256), 0, s, dh, low, at<float>(p.scale), B,
                           HW, at<bf16>(p.in0));
        ULAUNCH(u);
        return MSR_OK;
    }
};

msr_status ready(msr_unet* u, int batch) {
    if (!u) return MSR_ERR_INVALID;
    if (!u->ws) return ufail(u, MSR_ERR_OOM, "no workspace");
    if (!u->have_params) return ufail(u, MSR_ERR_STATE, "set_params first");
    if (batch < 1 || batch > u->plan.B) return ufail(u, MSR_ERR_INVALID, "batch must be in 1..%d", u->plan.B);
    UHIP(u, hipSetDevice(u->cfg.device));
    return MSR_OK;
}

}  // namespace

extern "C" {

size_t msr_unet_param_count(const msr_unet_config* cfg) {
    Net n;
    return make_net(cfg, n) ? n.nparam : 0;
}

size_t msr_unet_workspace_bytes(const msr_unet_config* cfg, int batch, int height, int width) {
    Net n;
    Plan p;
    if (!make_net(cfg, n) || !make_plan(n, batch, height, width, p)) return 0;
    return p.total;
}

msr_status msr_unet_init(const msr_unet_config* cfg, msr_unet** out) {
    if (!out) return MSR_ERR_INVALID;
    *out = nullptr;
    Net n;
    if (!make_net(cfg, n)) return MSR_ERR_INVALID;
    msr_unet* u = new (std::nothrow) msr_unet();
    if (!u) return MSR_ERR_OOM;
    u->cfg = *cfg;
    u->net = n;
    *out = u;
    return MSR_OK;
}

void msr_unet_destroy(msr_unet* u) { delete u; }

const char* msr_unet_last_error(const msr_unet* u) { return u ? u->err.c_str() : "null network"; }

msr_status msr_unet_set_workspace(msr_unet* u, void* dev, size_t bytes, int batch, int height, int width) {
    if (!u) return MSR_ERR_INVALID;
    Plan p;
    if (!make_plan(u->net, batch, height, width, p))
        return ufail(u, MSR_ERR_INVALID, "H and W must be multiples of %d", 1 << (u->net.levels - 1));
    if (!dev || bytes < p.total) return ufail(u, MSR_ERR_OOM, "workspace needs %zu bytes", p.total);
    if (reinterpret_cast<uintptr_t>(dev) % kAlign) return ufail(u, MSR_ERR_INVALID, "workspace must be 256-byte aligned");
    u->plan = p;
    u->ws = static_cast<char*>(dev);
    u->have_params = false;
    return MSR_OK;
}

msr_status msr_unet_set_params(msr_unet* u, const float* params, void* stream) {
    if (!u || !params) return MSR_ERR_INVALID;
    if (!u->ws) return ufail(u, MSR_ERR_OOM, "no workspace");
    UHIP(u, hipSetDevice(u->cfg.device));
    hipStream_t s = S(stream);
    Run r{u, u->net, u->plan, u->plan.B, s};
    const size_t nb = 4 * u->net.nparam;
    UHIP(u, hipMemcpyAsync(r.params(), params, nb, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(u->net.nparam)), dim3(256), 0, s, r.at<float>(u->plan.m),
                       u->net.nparam, 0.0f);
    ULAUNCH(u);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(u->net.nparam)), dim3(256), 0, s, r.at<float>(u->plan.v),
                       u->net.nparam, 0.0f);
    ULAUNCH(u);
    UTRY(r.refresh_weights());
    u->step = 0;
    u->have_params = true;
    return MSR_OK;
}

msr_status msr_unet_get_params(msr_unet* u, float* out, void* stream) {
    if (!u || !out) return MSR_ERR_INVALID;
    UTRY(ready(u, 1));
    Run r{u, u->net, u->plan, 1, S(stream)};
    UHIP(u, hipMemcpyAsync(out, r.params(), 4 * u->net.nparam, hipMemcpyDeviceToDevice, S(stream)));
    return MSR_OK;
}

// Checkpoint file: 8-byte magic, int32 in_channels, base_width, levels, 0,
// int64 parameter count, int64 Adam step, then the FP32 master parameters and
// Adam's first and second moments (host byte order).
static const char kUnetMagic[8] = {'M', 'S', 'R', 'U', 'N', 'E', 'T', '1'};

msr_status msr_unet_save(msr_unet* u, const char* path, void* stream) {
    if (!u || !path) return MSR_ERR_INVALID;
    UTRY(ready(u, 1));
    UHIP(u, hipSetDevice(u->cfg.device));
    const size_t n = u->net.nparam;
    Run r{u, u->net, u->plan, 1, S(stream)};
    std::vector<float> buf(3 * n);
    UHIP(u, hipMemcpyAsync(buf.data(), r.params(), 4 * n, hipMemcpyDeviceToHost, r.s));
    UHIP(u, hipMemcpyAsync(buf.data() + n, r.at<float>(u->plan.m), 4 * n, hipMemcpyDeviceToHost, r.s));
    UHIP(u, hipMemcpyAsync(buf.data() + 2 * n, r.at<float>(u->plan.v), 4 * n, hipMemcpyDeviceToHost, r.s));
    UHIP(u, hipStreamSynchronize(r.s));
    FILE* f = std::fopen(path, "wb");
    if (!f) return ufail(u, MSR_ERR_INVALID, "cannot open %s for writing", path);
    const int32_t hdr[4] = {u->cfg.in_channels, u->cfg.base_width, u->cfg.levels, 0};
    const int64_t cnt[2] = {(int64_t)n, (int64_t)u->step};
    bool ok = std::fwrite(kUnetMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(cnt, sizeof cnt, 1, f) == 1 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return ufail(u, MSR_ERR_INVALID, "writing %s failed", path);
    return MSR_OK;
}

msr_status msr_unet_load(msr_unet* u, const char* path, void* stream) {
    if (!u || !path) return MSR_ERR_INVALID;
    if (!u->ws) return ufail(u, MSR_ERR_OOM, "no workspace");
    UHIP(u, hipSetDevice(u->cfg.device));
    FILE* f = std::fopen(path, "rb");
    if (!f) return ufail(u, MSR_ERR_INVALID, "cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    int64_t cnt[2];
    const size_t n = u->net.nparam;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kUnetMagic, 8) == 0 &&
              std::fread(hdr, sizeof hdr, 1, f) == 1 && std::fread(cnt, sizeof cnt, 1, f) == 1;
    if (!ok) {
        std::fclose(f);
        return ufail(u, MSR_ERR_INVALID, "%s is not a network checkpoint", path);
    }
    if (hdr[0] != u->cfg.in_channels || hdr[1] != u->cfg.base_width || hdr[2] != u->cfg.levels ||
        cnt[0] != (int64_t)n || cnt[1] < 0) {
        std::fclose(f);
        return ufail(u, MSR_ERR_INVALID, "checkpoint of another configuration (%d, %d, %d)", hdr[0], hdr[1], hdr[2]);
    }
    std::vector<float> buf(3 * n);
    ok = std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return ufail(u, MSR_ERR_INVALID, "%s is truncated", path);
    hipStream_t s = S(stream);
    Run r{u, u->net, u->plan, u->plan.B, s};
    UHIP(u, hipMemcpyAsync(r.params(), buf.data(), 4 * n, hipMemcpyHostToDevice, s));
    UHIP(u, hipMemcpyAsync(r.at<float>(u->plan.m), buf.data() + n, 4 * n, hipMemcpyHostToDevice, s));
    UHIP(u, hipMemcpyAsync(r.at<float>(u->plan.v), buf.data() + 2 * n, 4 * n, hipMemcpyHostToDevice, s));
    UTRY(r.refresh_weights());
    UHIP(u, hipStreamSynchronize(s));  // the host buffer is released on return
    u->step = cnt[1];
    u->have_params = true;
    return MSR_OK;
}

msr_status msr_unet_forward(msr_unet* u, const float* dh, const float* low, float* x0, int batch, void* stream) {
    UTRY(ready(u, batch));
    if (!dh || !low || !x0) return ufail(u, MSR_ERR_INVALID, "null image");
    Run r{u, u->net, u->plan, batch, S(stream)};
    UTRY(r.prepare_input(dh, low));
    UTRY(r.forward());
    const int HW = u->plan.H * u->plan.W;
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for((size_t)batch * HW)), dim3(256), 0, r.s, r.at<float>(u->plan.out),
                       r.at<float>(u->plan.scale), batch, HW, x0);
    ULAUNCH(u);
    return MSR_OK;
}

msr_status msr_unet_loss_grad(msr_unet* u, const float* dh, const float* low, const float* target, int batch,
                              double* loss, float* grad_out, void* stream) {
    UTRY(ready(u, batch));
    if (!dh || !low || !target) return ufail(u, MSR_ERR_INVALID, "null image");
    Run r{u, u->net, u->plan, batch, S(stream)};
    UTRY(r.prepare_input(dh, low));
    UTRY(r.forward());
    UTRY(r.loss(target, loss));
    UTRY(r.backward());
    if (grad_out) UHIP(u, hipMemcpyAsync(grad_out, r.grad(), 4 * u->net.nparam, hipMemcpyDeviceToDevice, r.s));
    UHIP(u, hipStreamSynchronize(r.s));
    return MSR_OK;
}

msr_status msr_unet_train_step(msr_unet* u, const float* dh, const float* low, const float* target, int batch,
                               const msr_adam* opt, double* loss, void* stream) {
    UTRY(ready(u, batch));
    if (!dh || !low || !target || !opt) return ufail(u, MSR_ERR_INVALID, "null argument");
    if (!(opt->lr > 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) || !(opt->beta2 >= 0 && opt->beta2 < 1) ||
        !(opt->eps > 0))
        return ufail(u, MSR_ERR_INVALID, "bad Adam parameters");
    Run r{u, u->net, u->plan, batch, S(stream)};
    UTRY(r.prepare_input(dh, low));
    UTRY(r.forward());
    UTRY(r.loss(target, loss));
    UTRY(r.backward());
    const long long t = ++u->step;
    const double c1 = 1.0 - std::pow(opt->beta1, (double)t), c2 = 1.0 - std::pow(opt->beta2, (double)t);
    const float lr_t = (float)(opt->lr * std::sqrt(c2) / c1), eps_t = (float)(opt->eps * std::sqrt(c2));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(u->net.nparam)), dim3(256), 0, r.s, r.params(),
                       r.at<float>(u->plan.m), r.at<float>(u->plan.v), r.grad(), u->net.nparam, (float)opt->beta1,
                       (float)opt->beta2, lr_t, eps_t);
    ULAUNCH(u);
    UTRY(r.refresh_weights());
    UHIP(u, hipStreamSynchronize(r.s));
    return MSR_OK;
}

}  // extern "C"
