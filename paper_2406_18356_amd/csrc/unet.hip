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

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM: D[p][co] = sum_k A[p][k] W[co][k],
// A = im2col of the input, k = tap * cin + ci.  A block computes an 8 x 16
// pixel tile of one image for 64 output channels; its 4 waves take two tile
// rows (32 pixels) x 64 channels each (two 32x32 MFMA tiles).  The input is
// staged 32 channels at a time as the 10 x 18 halo tile around the output
// tile (zero outside the image), once per chunk, so each of the nine taps of
// a chunk reads its A operand from LDS at a shifted pixel: no per-step
// index arithmetic or bounds checks.  The weights go through LDS as well,
// one (chunk, tap) step (64 x 32) at a time in a double buffer loaded ahead,
// or a whole chunk at once (below: which layers take which).
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
// channels, else 2).  Two ways to stage the weights: a tap at a time (a
// barrier per tap; little LDS, so many resident blocks) or a chunk at a time
// (two barriers per chunk; nine taps of weights in LDS).  These layers wait on
// their loads more than on the matrix cores, so resident blocks count most:
// the chunk-wide staging is faster (24 % forward, 7 % backward at 4096^2)
// only for layers of at most 32 output channels and several input chunks,
// where its LDS is small and the per-tap path pays the most barriers; at 64
// output channels it halves the resident blocks and is 8-28 % slower.
#ifndef MSR_UNET_WD
#define MSR_UNET_WD 3
#endif
#ifndef MSR_UNET_HALO_BUFS
#define MSR_UNET_HALO_BUFS 1
#endif
constexpr int WD = MSR_UNET_WD;
static_assert(9 % WD == 0, "the step loop advances WD steps at a time over 9 steps per chunk");
// halo buffers of a multi-chunk layer (per-tap weights): 2 (the next chunk is
// written while the current one is read) or 1 (written after a barrier at the
// chunk's end: less LDS, one more barrier per chunk)
constexpr int HBUFS = MSR_UNET_HALO_BUFS;

// Output tile position of this block: image b, rows y0.., columns x0.., output channels n0..
struct ConvTile {
    int b, y0, x0, n0;
};
__device__ __forceinline__ ConvTile conv_tile(const ConvOut& o, int BN) {
    const int tiles_x = (o.W + TC - 1) / TC, tiles_y = (o.H + TR - 1) / TR;
    const int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y;
    return ConvTile{(int)blockIdx.x / (tiles_x * tiles_y), ty * TR, tx * TC, (int)blockIdx.y * BN};
}

// Halo items of thread tid: pixel q / 4 of the halo tile, channels 8 (q % 4) of chunk c0.
template <typename T>
__device__ __forceinline__ void conv_fetch_halo(const ConvIn<T>& in, const ConvOut& o, const ConvTile& tl, int cin,
                                                int c0, int tid, bf16x8 (&rh)[HPT]) {
#pragma unroll
    for (int u = 0; u < HPT; ++u) {
        const int q = tid + u * 256;
        const int hp = q >> 2;
        rh[u] = q < HITEMS ? pixel8(in, cin, o.H, o.W, tl.b, tl.y0 - 1 + hp / HC, tl.x0 - 1 + hp % HC, c0 + (q & 3) * 8)
                           : zero8();
    }
}
__device__ __forceinline__ void conv_stage_halo(bf16* hs, int tid, const bf16x8 (&rh)[HPT]) {
#pragma unroll
    for (int u = 0; u < HPT; ++u) {
        const int q = tid + u * 256;
        if (q < HITEMS) *reinterpret_cast<bf16x8*>(&hs[(q >> 2) * HLD + (q & 3) * 8]) = rh[u];
    }
}

// Bias, activation and stores of a wave's MT x NT accumulator tiles:
// acc[m][nt][r] is tile pixel (WROWS wave + 2 m) * 16 + (r / 4) * 8 +
// (lane / 32) * 4 + r % 4, output channel n0 + 32 nt + lane % 32.
template <bool BWD, int NT>
__device__ __forceinline__ void conv_epilogue(const ConvOut& o, const ConvTile& tl, const f32x16 (&acc)[MT][NT],
                                              int wave, int lane) {
    const int pl = lane & 31;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = tl.n0 + nt * 32 + pl;
        if (co >= o.cout) continue;
        const float bias = o.bias ? o.bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int q = (WROWS * wave + 2 * m) * 16 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);  // tile pixel
            const int y = tl.y0 + (q >> 4), x = tl.x0 + (q & 15);
            if (y >= o.H || x >= o.W) continue;
            const size_t p = ((size_t)tl.b * o.H + y) * o.W + x;
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

// Weights staged a chunk at a time.  LDS: the halo tile of the chunk and the
// chunk's weights, nine taps of BN rows x 32 channels (37 KB at NT = 1).  The next chunk's halo and weights are
// loaded into registers while the current chunk's 18 MFMA k-steps run from
// LDS, and written after the barrier that ends it.
template <typename T, bool BWD, int NT>
__device__ __forceinline__ void conv_body_chunk(const ConvIn<T>& in, const ConvOut& o) {
    constexpr int BN = 32 * NT;
    constexpr int WITEMS = 9 * BN * (CBK / 8);  // 16-byte groups of a chunk's weights
    constexpr int WPT = (WITEMS + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 Hs[NHALO * HLD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[9 * BN * CLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const ConvTile tl = conv_tile(o, BN);
    const int cin = in.c1 + in.c2;
    const int nchunks = (cin + CBK - 1) / CBK;

    bf16x8 rh[HPT];
    // weight item q: tap q / (4 BN), row (q / 4) % BN, channels 8 (q % 4) of the chunk
    bf16x8 rw[WPT];
    auto fetch_w = [&](int c) {
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int q = tid + u * 256;
            const int t = q / (4 * BN), r = q - t * (4 * BN);
            const int co = tl.n0 + (r >> 2), ci = c * CBK + (r & 3) * 8;
            rw[u] = (q < WITEMS && co < o.cout && ci < cin) ? load8(o.w + (size_t)co * o.kpad + t * cin + ci) : zero8();
        }
    };
    auto stage_w = [&]() {
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int q = tid + u * 256;
            if (q < WITEMS) {
                const int t = q / (4 * BN), r = q - t * (4 * BN);
                *reinterpret_cast<bf16x8*>(&Bs[(t * BN + (r >> 2)) * CLD + (r & 3) * 8]) = rw[u];
            }
        }
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
    conv_fetch_halo(in, o, tl, cin, 0, tid, rh);
    fetch_w(0);
    conv_stage_halo(Hs, tid, rh);
    stage_w();
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const bool more = c + 1 < nchunks;
        if (more) {  // the next chunk, in registers
            conv_fetch_halo(in, o, tl, cin, (c + 1) * CBK, tid, rh);
            fetch_w(c + 1);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int hp = hbase + (t / 3 - 1) * HC + (t % 3 - 1);
#pragma unroll
            for (int kk = 0; kk < CBK; kk += 16) {
                bf16x8 av[MT], bv[NT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    av[m] = *reinterpret_cast<const bf16x8*>(&Hs[(hp + 2 * m * HC) * HLD + kk + ko]);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    bv[n] = *reinterpret_cast<const bf16x8*>(&Bs[(t * BN + 32 * n + pl) * CLD + kk + ko]);
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bv[n], acc[m][n], 0, 0, 0);
            }
        }
        if (more) {
            __syncthreads();  // every wave has finished reading this chunk
            conv_stage_halo(Hs, tid, rh);
            stage_w();
            __syncthreads();
        }
    }
    conv_epilogue<BWD, NT>(o, tl, acc, wave, lane);
}

// Weights staged a tap at a time.  ONE: the input has at most 32 channels
// (one chunk, one halo buffer: half the LDS, so twice the resident blocks to
// cover the load latency).
template <typename T, bool BWD, int NT, bool ONE>
__device__ __forceinline__ void conv_body_tap(const ConvIn<T>& in, const ConvOut& o) {
    constexpr int BN = 32 * NT;  // output channels of a block
    __shared__ __attribute__((aligned(16))) bf16 Hs[ONE ? 1 : HBUFS][NHALO * HLD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BN * CLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const ConvTile tl = conv_tile(o, BN);
    const int cin = in.c1 + in.c2;
    const int nsteps = 9 * ((cin + CBK - 1) / CBK);  // (chunk, tap) steps, a multiple of WD

    bf16x8 rh[HPT];
    // weights of step s = chunk * 9 + tap: row co, k = tap * cin + chunk * 32 + [0, 32);
    // WD steps in flight, in registers
    const int bco = tl.n0 + tid / 4, bg = (tid % 4) * 8;
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

    const int pl = lane & 31;
    const int hbase = (WROWS * wave + (pl >> 4) + 1) * HC + (pl & 15) + 1;
    const int ko = (lane >> 5) * 8;

    f32x16 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x16{};
    conv_fetch_halo(in, o, tl, cin, 0, tid, rh);
    fetch_w(0, rb[0]);
    conv_stage_halo(Hs[0], tid, rh);
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
            if (!ONE && t == 0 && st + 9 < nsteps) conv_fetch_halo(in, o, tl, cin, (st / 9 + 1) * CBK, tid, rh);
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
            fetch_w(st + WD, rb[j]);  // slot j is free again: step st + WD
            if constexpr (!ONE && HBUFS == 2) {
                if (t == 8 && more) conv_stage_halo(Hs[hcur ^ 1], tid, rh);
            }
            __syncthreads();
            if constexpr (!ONE && HBUFS == 2) {
                if (t == 8) hcur ^= 1;
            }
            if constexpr (!ONE && HBUFS == 1) {
                // every wave has read this chunk's halo (the barrier above)
                if (t == 8 && more) {
                    conv_stage_halo(Hs[0], tid, rh);
                    __syncthreads();
                }
            }
        }
    }
    conv_epilogue<BWD, NT>(o, tl, acc, wave, lane);
}

template <typename T, bool BWD, int NT, bool ONE>
__global__ void __launch_bounds__(256) conv3x3_kernel(ConvIn<T> in, ConvOut o) {
    if constexpr (NT == 1 && !ONE) conv_body_chunk<T, BWD, NT>(in, o);
    else conv_body_tap<T, BWD, NT, ONE>(in, o);
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
// Weight gradient as an implicit GEMM over pixels:
//   dW[co][t cin + ci] = sum_p G[p][co] X[p + off_t][ci]
// (G the output gradient, X the layer's input, zero outside the image).  A
// block owns 32 NT output channels x one 32-channel input chunk x the nine
// taps (9 NT accumulator tiles of 32 x 32) and sums over every nz-th 8 x 16
// pixel tile (grid z; the partial results are added afterwards).  3 NT
// waves: wave w takes output subtile w / 3 and the tap row dy = w % 3, one
// accumulator per dx.  Per pixel tile, G is staged transposed (Gs[co][pixel])
// and the input chunk's 10 x 18 halo transposed in three copies shifted by
// dx (Xs[dx][ci][hrow][col] = X(hrow, col + dx)), so that both MFMA operands
// of a K step (one tile row, 16 pixels) are aligned 16-byte LDS reads at
// every tap.  The blocks of the first input chunk also sum G over their
// pixels in float32 (the bias gradient), one partial per pixel-tile group.
// ---------------------------------------------------------------------------
struct WGradArgs {
    const float* g;  // [P][cout]
    int B, H, W, cout, kpad;
    int nz;          // pixel-tile groups (grid z)
    float* part;     // [nz][cout][kpad]; entries k >= 9 cin are not written
    float* bpart;    // [nz][cout]: sums of G over each group's pixels
};

constexpr int GLD = TR * TC + 8;        // bf16 per Gs row (one output channel; 272 B)
constexpr int XCS = HR * TC + 8;        // bf16 per input channel of one Xs copy (336 B)
constexpr int WG_XITEMS = NHALO * (CBK / 8);  // 16-byte groups of one halo chunk

template <int NT>
__global__ void __launch_bounds__(192 * NT) conv3x3_wgrad_kernel(ConvIn<bf16> in, WGradArgs a) {
    constexpr int NTH = 192 * NT;            // threads
    constexpr int GITEMS = (TR * TC / 2) * 4 * NT;  // (pixel pair, 8-channel group) items of a G tile
    __shared__ __attribute__((aligned(16))) bf16 Gs[32 * NT * GLD];
    __shared__ __attribute__((aligned(16))) bf16 Xs[3 * CBK * XCS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n0 = blockIdx.x * 32 * NT, chunk = blockIdx.y;
    const int cin = in.c1 + in.c2;
    const int tiles_x = (a.W + TC - 1) / TC, tiles_y = (a.H + TR - 1) / TR;
    const int ntiles = a.B * tiles_x * tiles_y;
    const int sub = wave / 3, dy = wave % 3;
    const int pl = lane & 31, ko = (lane >> 5) * 8;

    f32x16 acc[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) acc[dx] = f32x16{};
    // this thread's G items are always channels 8 (tid % (4 NT)) ..: their sums
    float bsum[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bsum[j] = 0.0f;
    static_assert(NTH % (4 * NT) == 0, "a thread keeps one channel group");
    for (int tile = blockIdx.z; tile < ntiles; tile += a.nz) {
        const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, b = tile / (tiles_x * tiles_y);
        const int y0 = ty * TR, x0 = tx * TC;
        __syncthreads();  // the previous tile's operands have been read
        // G: item q = (pixel pair q / (4 NT), channels 8 (q % (4 NT))), written as bf16 pairs
        for (int q = tid; q < GITEMS; q += NTH) {
            const int pp = q / (4 * NT), grp = q - pp * (4 * NT);
            const int px = 2 * pp, co = n0 + grp * 8;
            const int y = y0 + px / TC, x = x0 + px % TC;  // both pixels of the pair are in one tile row
            float g0[8], g1[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) g0[j] = g1[j] = 0.0f;
            if (y < a.H && co < a.cout) {
                const size_t p = ((size_t)b * a.H + y) * a.W + x;
                if (x < a.W) {
                    const float4 u = *reinterpret_cast<const float4*>(a.g + p * a.cout + co);
                    const float4 v = *reinterpret_cast<const float4*>(a.g + p * a.cout + co + 4);
                    g0[0] = u.x, g0[1] = u.y, g0[2] = u.z, g0[3] = u.w, g0[4] = v.x, g0[5] = v.y, g0[6] = v.z, g0[7] = v.w;
                }
                if (x + 1 < a.W) {
                    const float4 u = *reinterpret_cast<const float4*>(a.g + (p + 1) * a.cout + co);
                    const float4 v = *reinterpret_cast<const float4*>(a.g + (p + 1) * a.cout + co + 4);
                    g1[0] = u.x, g1[1] = u.y, g1[2] = u.z, g1[3] = u.w, g1[4] = v.x, g1[5] = v.y, g1[6] = v.z, g1[7] = v.w;
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) bsum[j] += g0[j] + g1[j];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
                bf16x2 w2;
                w2[0] = (bf16)g0[j];
                w2[1] = (bf16)g1[j];
                *reinterpret_cast<bf16x2*>(&Gs[(grp * 8 + j) * GLD + px]) = w2;
            }
        }
        // X: item q = (halo pixel q / 4, channels 8 (q % 4) of the chunk) into each copy that holds it
        for (int q = tid; q < WG_XITEMS; q += NTH) {
            const int hp = q >> 2, ci = (q & 3) * 8;
            const int hr = hp / HC, hc = hp - hr * HC;
            const bf16x8 v = pixel8(in, cin, a.H, a.W, b, y0 - 1 + hr, x0 - 1 + hc, chunk * CBK + ci);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int col = hc - dx;
                if (col >= 0 && col < TC) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) Xs[(dx * CBK + ci + j) * XCS + hr * TC + col] = v[j];
                }
            }
        }
        __syncthreads();
        // K steps: tile rows r; A = G^T rows (this wave's 32 channels) over the
        // row's 16 pixels, B = the input at tap (dy, dx) over the same pixels
#pragma unroll
        for (int r = 0; r < TR; ++r) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&Gs[(sub * 32 + pl) * GLD + r * TC + ko]);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Xs[(dx * CBK + pl) * XCS + (r + dy) * TC + ko]);
                acc[dx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[dx], 0, 0, 0);
            }
        }
    }
    if (chunk == 0) {
        // bias partial of each of the block's channels: its threads' sums in thread order
        __syncthreads();  // Gs is free: every wave has done its last MFMA reads
        float* red = reinterpret_cast<float*>(Gs);
        static_assert(NTH * 8 * sizeof(float) <= sizeof(Gs), "reduction scratch fits Gs");
#pragma unroll
        for (int j = 0; j < 8; ++j) red[tid * 8 + j] = bsum[j];
        __syncthreads();
        if (tid < 32 * NT) {
            const int grp = tid >> 3, j = tid & 7;
            float tot = 0.0f;
            for (int t = grp; t < NTH; t += 4 * NT) tot += red[t * 8 + j];
            if (n0 + tid < a.cout) a.bpart[(size_t)blockIdx.z * a.cout + n0 + tid] = tot;
        }
    }
    // acc[dx][e]: output channel n0 + 32 sub + (e / 4) * 8 + (lane / 32) * 4 + e % 4, input channel
    // chunk * 32 + lane % 32, tap 3 dy + dx
    const int ci = chunk * CBK + pl;
    if (ci >= cin) return;
    float* part = a.part + (size_t)blockIdx.z * a.cout * a.kpad;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int k = (3 * dy + dx) * cin + ci;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int co = n0 + sub * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
            if (co < a.cout) part[(size_t)co * a.kpad + k] = acc[dx][e];
        }
    }
}

// dW[co][k] = sum_z part[z][co][k] for k < kvalid; entries k >= kvalid keep
// the zero the gradient was cleared to.  A block takes 32 consecutive
// entries; its 8 thread rows sum every 8th z, then the 8 row sums are added
// in order (deterministic).
__global__ void __launch_bounds__(256) sum_wparts_kernel(const float* __restrict__ part, int nz, int cout, int kpad,
                                                         int kvalid, float* __restrict__ out) {
    __shared__ float red[8][32];
    const size_t n = (size_t)cout * kpad;
    const int l = threadIdx.x & 31, sl = threadIdx.x >> 5;
    for (size_t i0 = (size_t)blockIdx.x * 32; i0 < n; i0 += (size_t)gridDim.x * 32) {
        const size_t i = i0 + l;
        const bool ok = i < n && (int)(i % (size_t)kpad) < kvalid;
        float sm = 0.0f;
        if (ok)
            for (int z = sl; z < nz; z += 8) sm += part[(size_t)z * n + i];
        red[sl][l] = sm;
        __syncthreads();
        if (sl == 0 && ok) {
            float t = 0.0f;
#pragma unroll
            for (int r = 0; r < 8; ++r) t += red[r][l];
            out[i] = t;
        }
        __syncthreads();
    }
}

// out[i] = sum_z part[z][i] for few outputs and many partials: one block
// per output, each thread summing every 256th partial in order, then a fixed
// tree across the block (deterministic).
__global__ void __launch_bounds__(256) sum_parts_wide_kernel(const float* __restrict__ part, int nz, int n,
                                                             float* __restrict__ out) {
    __shared__ float red[256];
    const int i = blockIdx.x, t = threadIdx.x;
    float s = 0.0f;
    for (int z = t; z < nz; z += 256) s += part[(size_t)z * n + i];
    red[t] = s;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[i] = red[0];
}

// Blocks of a head-gradient sum over P pixels, and the pixels of each.
inline int head_sum_blocks(int P) { return std::max(1, std::min(1024, (P + 4095) / 4096)); }
inline int head_sum_chunk(int P) { return (P + head_sum_blocks(P) - 1) / head_sum_blocks(P); }

// The head's weight and bias gradients over pixel chunks: part[z][c] = sum
// over the chunk's pixels of gout[p] x[p][c] for c < C, and of gout[p] for
// c = C.  With C + 1 <= 256 columns the block's threads form 256 / (C + 1)
// rows (thread t: column t % (C + 1), pixels t / (C + 1), + rows, ...), so each
// step of the block reads whole pixel rows; the rows' sums are added in order
// in LDS.  Wider heads take columns t, t + 256, ... over every pixel.
__global__ void __launch_bounds__(256) head_sums_kernel(const float* __restrict__ gout, const bf16* __restrict__ x,
                                                        int P, int C, int chunk, float* __restrict__ part) {
    __shared__ float red[256];
    const int NC = C + 1;  // columns summed
    const int t = threadIdx.x;
    const int pb = blockIdx.x * chunk, pe = min(P, pb + chunk);
    auto val = [&](int p, int c) -> float { return c < C ? gout[p] * (float)x[(size_t)p * C + c] : gout[p]; };
    if (NC > 256) {
        for (int c = t; c < NC; c += 256) {
            float s = 0.0f;
            for (int p = pb; p < pe; ++p) s += val(p, c);
            part[(size_t)blockIdx.x * NC + c] = s;
        }
        return;
    }
    const int rows = 256 / NC, c = t % NC, j = t / NC;
    float s = 0.0f;
    if (j < rows) {
        int p = pb + j;
        // four independent loads in flight, summed in a fixed order
        for (; p + 3 * rows < pe; p += 4 * rows) {
            const float a0 = val(p, c), a1 = val(p + rows, c), a2 = val(p + 2 * rows, c), a3 = val(p + 3 * rows, c);
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; p < pe; p += rows) s += val(p, c);
    }
    red[t] = s;
    __syncthreads();
    if (t < NC) {
        float tot = 0.0f;
        for (int r = 0; r < rows; ++r) tot += red[r * NC + t];
        part[(size_t)blockIdx.x * NC + t] = tot;
    }
}

// ---------------------------------------------------------------------------
// Pooling, upsampling adjoints, head, loss, input/output, optimiser.
// ---------------------------------------------------------------------------
// 2x2 average pool, NHWC bf16: out (B, H/2, W/2, C).
__global__ void pool_kernel(const bf16* __restrict__ x, int B, int H, int W, int C, bf16* __restrict__ out) {
    // item: output pixel q / (C / 8), channels 8 (q % (C / 8)); 16-byte loads
    // and stores, 32-bit index arithmetic (B H W < 2^31, C a multiple of 8)
    const unsigned G = (unsigned)C / 8, W2 = (unsigned)W / 2, H2 = (unsigned)H / 2;
    const unsigned n = (unsigned)B * H2 * W2 * G;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const unsigned p2 = q / G, g = q - p2 * G;
        const unsigned x2 = p2 % W2, r = p2 / W2, y2 = r % H2, b = r / H2;
        const size_t base = (((size_t)b * H + 2 * y2) * W + 2 * x2) * C + g * 8;
        const bf16x8 a = load8(x + base), c = load8(x + base + C);
        const bf16x8 d = load8(x + base + (size_t)W * C), e = load8(x + base + (size_t)W * C + C);
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float s = (float)a[j] + (float)c[j] + (float)d[j] + (float)e[j];
            o[j] = (bf16)(0.25f * s);
        }
        *reinterpret_cast<bf16x8*>(out + (size_t)p2 * C + g * 8) = o;
    }
}

// G[b,y,x,c] = (dpool[b,y/2,x/2,c] / 4 + dskip[b,y,x,c]) * (e > 0): the
// gradient of an encoder output feeding both the pool and the skip.
__global__ void pool_back_kernel(const float* __restrict__ dpool, const float* __restrict__ dskip,
                                 const bf16* __restrict__ e, int B, int H, int W, int C, float* __restrict__ g) {
    // 256 / C pixels of C channels per block step (C <= 256): one division per pixel
    const unsigned rows = C <= 256 ? 256 / C : 1, np = (unsigned)B * H * W;
    const unsigned j = threadIdx.x / C, c = threadIdx.x - j * C;
    if (j >= rows) return;
    for (unsigned p = blockIdx.x * rows + j; p < np; p += gridDim.x * rows) {
        const unsigned x = p % W, r = p / W, y = r % H, b = r / H;
        const size_t q = ((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2;
        for (unsigned cc = c; cc < (unsigned)C; cc += 256) {
            const size_t i = (size_t)p * C + cc;
            float v = dskip ? dskip[i] : 0.0f;
            if (dpool) v += 0.25f * dpool[q * C + cc];
            g[i] = (float)e[i] > 0.0f ? v : 0.0f;
        }
    }
}

// G[b,y,x,c] = (sum of dup over the 2x2 block) * (d > 0): the adjoint of the
// nearest upsampling of d (B, H, W, C); dup is (B, 2H, 2W, C).
__global__ void up_back_kernel(const float* __restrict__ dup, const bf16* __restrict__ d, int B, int H, int W, int C,
                               float* __restrict__ g) {
    const unsigned rows = C <= 256 ? 256 / C : 1, np = (unsigned)B * H * W;
    const unsigned j = threadIdx.x / C, c = threadIdx.x - j * C;
    if (j >= rows) return;
    const size_t row = (size_t)2 * W * C;
    for (unsigned p = blockIdx.x * rows + j; p < np; p += gridDim.x * rows) {
        const unsigned x = p % W, r = p / W, y = r % H, b = r / H;
        const size_t base = (((size_t)b * 2 * H + 2 * y) * 2 * W + 2 * x) * C;
        for (unsigned cc = c; cc < (unsigned)C; cc += 256) {
            const size_t i = (size_t)p * C + cc, q = base + cc;
            const float sm = dup[q] + dup[q + C] + dup[q + row] + dup[q + row + C];
            g[i] = (float)d[i] > 0.0f ? sm : 0.0f;
        }
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
        const float inv = 1.0f / scale[(unsigned)i / (unsigned)HW];  // B HW < 2^31
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
        x0[i] = scale[(unsigned)i / (unsigned)HW] * fmaxf(out[i], 0.0f);  // B HW < 2^31
}

// Loss partials sum (out - t/s)^2 per block and gout = 2 (out - t/s) / n.
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                                   const float* __restrict__ scale, int B, int HW,
                                                   float* __restrict__ gout, double* __restrict__ part) {
    __shared__ double red[256];
    const size_t n = (size_t)B * HW;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float d = out[i] - target[i] / scale[(unsigned)i / (unsigned)HW];  // B HW < 2^31
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

// Head backward, the input gradient: gx[p][c] = gout[p] w[c] where x > 0
// (the head's weight and bias gradients: head_sums_kernel).
__global__ void __launch_bounds__(256) head_back_kernel(const bf16* __restrict__ x, const float* __restrict__ gout,
                                                        int P, int C, const float* __restrict__ wb,
                                                        float* __restrict__ gx) {
    // 256 / C pixels of C channels per block step (C <= 256), no division per element
    const int rows = C <= 256 ? 256 / C : 1;
    const int j = threadIdx.x / C, c = threadIdx.x - j * C;
    if (j >= rows) return;
    for (size_t p = (size_t)blockIdx.x * rows + j; p < (size_t)P; p += (size_t)gridDim.x * rows) {
        const float g = gout[p];
        for (int cc = c; cc < C; cc += 256) {
            const size_t i = p * C + cc;
            gx[i] = (float)x[i] > 0.0f ? g * wb[cc] : 0.0f;
        }
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

// Weight-gradient launch of a layer: output-channel blocks (32 NT channels),
// input chunks and pixel-tile groups (grid z), about 2048 blocks in all.
struct WGradGrid {
    int nt, cob, chunks, nz;
};
WGradGrid wgrad_grid(int B, int H, int W, int cin, int cout) {
    WGradGrid g;
    g.nt = cout <= 32 ? 1 : 2;
    g.cob = (cout + 32 * g.nt - 1) / (32 * g.nt);
    g.chunks = (cin + CBK - 1) / CBK;
    const int ntiles = conv_tiles(B, H, W);
    g.nz = std::max(1, std::min(ntiles, (2048 + g.cob * g.chunks - 1) / (g.cob * g.chunks)));
    return g;
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
        const WGradGrid g = wgrad_grid(B, H >> l.level, W >> l.level, l.cin, l.cout);
        pf = std::max(pf, (size_t)g.nz * l.cout * (l.kpad + 1));  // weight and bias partials
    }
    pf = std::max(pf, (size_t)head_sum_blocks(npix(p, 0)) * (n.width + 1));  // head partials
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
        WGradArgs a{};
        a.g = gact(i);
        a.B = B;
        a.H = hh(l.level);
        a.W = ww(l.level);
        a.cout = l.cout;
        a.kpad = l.kpad;
        const ConvIn<bf16> in = input(i);
        const int cin = in.c1 + in.c2;
        const WGradGrid g = wgrad_grid(B, a.H, a.W, cin, l.cout);
        a.nz = g.nz;
        if ((size_t)g.nz * l.cout * (l.kpad + 1) > p.part_floats || 9 * cin > l.kpad)
            return ufail(u, MSR_ERR_INVALID, "weight-gradient partials too small");
        a.part = at<float>(p.part);
        a.bpart = a.part + (size_t)g.nz * l.cout * l.kpad;
        const dim3 grid(g.cob, g.chunks, g.nz);
        if (g.nt == 1) hipLaunchKernelGGL(conv3x3_wgrad_kernel<1>, grid, dim3(192), 0, s, in, a);
        else hipLaunchKernelGGL(conv3x3_wgrad_kernel<2>, grid, dim3(384), 0, s, in, a);
        ULAUNCH(u);
        const size_t nw = (size_t)l.cout * l.kpad;
        hipLaunchKernelGGL(sum_wparts_kernel, dim3(grid_for(nw, 32)), dim3(256), 0, s, at<float>(p.part), g.nz,
                           l.cout, l.kpad, 9 * cin, grad() + l.w_off);
        ULAUNCH(u);
        hipLaunchKernelGGL(sum_parts_wide_kernel, dim3(l.cout), dim3(256), 0, s, a.bpart, g.nz, l.cout,
                           grad() + l.b_off);
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
            hipLaunchKernelGGL(head_back_kernel, dim3(grid_for((size_t)P0 * n.width)), dim3(256), 0, s, act(top),
                               at<float>(p.gout), P0, n.width, params() + n.head_off, gact(top));
            ULAUNCH(u);
            const int nb = head_sum_blocks(P0);
            hipLaunchKernelGGL(head_sums_kernel, dim3(nb), dim3(256), 0, s, at<float>(p.gout), act(top), P0, n.width,
                               head_sum_chunk(P0), at<float>(p.part));
            ULAUNCH(u);
            hipLaunchKernelGGL(sum_parts_wide_kernel, dim3(n.width + 1), dim3(256), 0, s, at<float>(p.part), nb,
                               n.width + 1, grad() + n.head_off);
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
