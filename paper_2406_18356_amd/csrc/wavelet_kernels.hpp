// wavelet_kernels.hpp -- the wavelet dictionary W (concatenation of the
// orthonormal Daubechies bases db1 .. db8, 2-D, separable, periodic, nested
// coefficient layout) and the FISTA update on its coefficients.
//
// One level of one basis along an axis of length s (periodic), taps h[0..L),
// g[k] = (-1)^k h[L-1-k]:
//   analysis   lo[i] = sum_k h[k] x[(2i + k) mod s],  hi[i] = sum_k g[k] x[(2i + k) mod s]
//   synthesis  x[n]  = sum_{k = n mod 2, k < L} lo[m] h[k] + hi[m] g[k],  m = ((n - k) / 2) mod s/2
// (the synthesis is the transpose of the analysis, which is orthonormal).
// A 2-D level filters the rows, then the columns, of the top-left s x s
// block; its output quadrants are (rows: column filter, columns: row filter)
//   [0, s/2) x [0, s/2): lo-lo (the next level's input)   [0, s/2) x [s/2, s): lo rows of the row-hi half
//   [s/2, s) x [0, s/2): hi rows of the row-lo half        [s/2, s) x [s/2, s): hi-hi
//
// Offsets are 32-bit: 8 N^2 < 2^31 for N <= 8192.
//
// Each kernel does one whole 2-D level (both axes) for a tile, through LDS:
//   dwt_level   reads a (2T + 14)^2 input tile once and writes the four T x T
//               output quadrants of every basis the block handles;
//   idwt_level  reads four (R / 2 + 7) x (C / 2 + 7) quadrant tiles and writes
//               an R x C output tile, C = 4 R wide so that loads and stores
//               cover whole cache lines (level 0: the sum over all 8 bases,
//               so x is written once).
// Level 0 of the analysis shares its input (the image) between the bases, so
// one block loops over all 8 and reads the tile once; level 0 of the synthesis
// sums the bases in registers.  The other levels run one basis per block
// (grid z).  Coefficients that leave the transform (the detail quadrants, and
// the coarsest lo-lo quadrant) go through an epilogue: a plain store, or the
// FISTA step on the coefficients fused in (so W^T g is never stored).
#pragma once
#include <hip/hip_runtime.h>

namespace msr {

constexpr int kWaveletBases = 8;  // db1 .. db8
constexpr int kWaveletLevels = 4;
constexpr int kMaxTaps = 16;

template <typename R>
struct Taps {
    R h[kMaxTaps];
    R g[kMaxTaps];
    int L;
};

constexpr int kDwtT = 32;                        // analysis: output quadrant tile side
constexpr int kDwtIn = 2 * kDwtT + kMaxTaps - 2;  // input tile side (78)
constexpr int kDwtY = 2 * kDwtT + 4;             // row-pass row length: rows 8 apart fall 32 banks apart
constexpr int kIdwtTR = 32;                      // synthesis: output tile rows
constexpr int kIdwtTC = 128;                     // synthesis: output tile columns (wide: whole cache lines)
constexpr int kIdwtHalo = kMaxTaps / 2 - 1;      // 7 quadrant rows / columns before the tile
constexpr int kIdwtQR = kIdwtTR / 2 + kIdwtHalo;  // quadrant tile rows (23)
constexpr int kIdwtQC = kIdwtTC / 2 + kIdwtHalo;  // quadrant tile columns (71)
constexpr int kWavThreads = 256;
constexpr int kIdwtRowTasks = (kIdwtTR * kIdwtTC / 8) / kWavThreads;  // row-pass tasks (4 output pairs) a thread
// Waves per SIMD the LDS footprint allows (about 45 KB per block in FP32, 90 KB
// in FP64, of 160 KB): the register budget is capped to match.
template <typename R>
constexpr int kWavWaves = sizeof(R) == 4 ? 3 : 1;

// Where coefficients that leave the transform go.  Basis b's coefficients
// are at offset b * cstride, row stride ldc.
//   mode 0: out = scale * w
//   mode 1: one FISTA step with the gradient coefficient w = W^T of the
//           half-gradient image: alpha_{k-1} = b1 + t_prev (b1 - b2),
//           beta_k = soft(alpha_{k-1} - 2 mu w, mu lambda) -> b2,
//           alpha_k = beta_k + t_cur (beta_k - b1) -> a.
// threadIdx.x behind an empty asm: index arithmetic derived from it stays
// where it is written instead of being hoisted out of the basis loop and the
// tap-count switch, which would keep hundreds of addresses live (spills).
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// The tile of this block in a gx x gy tile grid launched as gridDim.x = gx gy.
// Consecutive blocks go to different XCDs (8 of them), so when g^2 is a
// multiple of 8 each XCD is given one contiguous row-major range of tiles:
// neighbouring tiles, whose input halos overlap, then share that XCD's L2.
__device__ __forceinline__ void xcd_tile(int gx, int gy, int& tx, int& ty) {
    const int n = gx * gy;
    int id = blockIdx.x;
    if ((n & 7) == 0) id = (id & 7) * (n >> 3) + (id >> 3);
    tx = id % gx;
    ty = id / gx;
}

template <typename R>
struct WavEpi {
    unsigned cstride;
    int ldc;
    int mode;
    R* out;
    R scale;
    const R* b1;
    R* b2;
    R* a;
    R two_mu, thr, t_prev, t_cur;
};

// The update's operands are loaded before the column sums (wav_fetch) so
// that their latency overlaps the arithmetic; wav_emit finishes.
template <typename R>
__device__ __forceinline__ void wav_fetch(const WavEpi<R>& e, int b, int row, int col, R& p1, R& p2) {
    const unsigned p = (unsigned)b * e.cstride + (unsigned)row * e.ldc + col;
    p1 = e.b1[p];
    p2 = e.b2[p];
}
template <typename R>
__device__ __forceinline__ void wav_emit(const WavEpi<R>& e, int b, int row, int col, R w, R p1, R p2) {
    const unsigned p = (unsigned)b * e.cstride + (unsigned)row * e.ldc + col;
    if (e.mode == 0) {
        e.out[p] = e.scale * w;
        return;
    }
    const R al = fma(e.t_prev, p1 - p2, p1);
    const R z = al - e.two_mu * w;
    const R zero = 0;
    const R beta = copysign(fmax(fabs(z) - e.thr, zero), z);
    e.b2[p] = beta;
    e.a[p] = fma(e.t_cur, beta - p1, beta);
}

template <typename R>
struct DwtArgs {
    const R* in;       // level input: top-left s x s block, row stride ld_in
    unsigned in_bs;    // basis stride of the input (0: one input shared by all bases)
    int ld_in;
    R* ll;             // lo-lo output (s/2 x s/2, row stride ld_ll, basis stride ll_bs); null: to the epilogue
    unsigned ll_bs;
    int ld_ll;
    int s;
    int bpb;           // bases per block (blockIdx.z * bpb is the first)
    const Taps<R>* taps;
    WavEpi<R> epi;
};

template <typename R, int L>
__device__ __forceinline__ void dwt_tile(const DwtArgs<R>& p, int b, R (*X)[kDwtIn + 1], R (*Y)[kDwtY],
                                         int i0, int c0) {
    const Taps<R>& t = p.taps[b];
    const int half = p.s >> 1;
    const int tid = opaque_tid();
    const int c = tid % kDwtT;
    const int q = tid / kDwtT;  // 0 .. 7
    const int col = c0 + c;
    // the update's operands of this thread's 16 outputs (band order ll, lh,
    // hl, hh), loaded first so that they arrive during both passes
    R o1[4][4], o2[4][4];
    const bool fetch = p.epi.mode == 1 && col < half;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = i0 + 4 * q + j;
        if (fetch && row < half) {
            if (!p.ll) wav_fetch(p.epi, b, row, col, o1[j][0], o2[j][0]);
            wav_fetch(p.epi, b, row, half + col, o1[j][1], o2[j][1]);
            wav_fetch(p.epi, b, half + row, col, o1[j][2], o2[j][2]);
            wav_fetch(p.epi, b, half + row, half + col, o1[j][3], o2[j][3]);
        }
    }
    // rows: Y[r][c] = lo, Y[r][T + c] = hi of input row r, output column c.
    // A task is 4 adjacent output columns c = 4 g + i, which read the window
    // X[r][8 g + k'], k' < L + 6 (column c takes k' = 2 i + k).
    constexpr int nrows = 2 * kDwtT + L - 2;
    for (int e = tid; e < nrows * (kDwtT / 4); e += kWavThreads) {
        const int r = e / (kDwtT / 4), g = e % (kDwtT / 4);
        R lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k2 = 0; k2 < L + 6; ++k2) {
            const R x = X[r][8 * g + k2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k2 - 2 * i;
                if (k >= 0 && k < L) {
                    lo[i] = fma(t.h[k], x, lo[i]);
                    hi[i] = fma(t.g[k], x, hi[i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Y[r][4 * g + i] = lo[i];
            Y[r][kDwtT + 4 * g + i] = hi[i];
        }
    }
    __syncthreads();
    // columns (below): each thread 4 consecutive output rows of one column
    R ll[4] = {0, 0, 0, 0}, lh[4] = {0, 0, 0, 0}, hl[4] = {0, 0, 0, 0}, hh[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < L + 6; ++u) {
        const R ylo = Y[8 * q + u][c], yhi = Y[8 * q + u][kDwtT + c];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = u - 2 * j;
            if (k >= 0 && k < L) {
                ll[j] = fma(t.h[k], ylo, ll[j]);
                lh[j] = fma(t.h[k], yhi, lh[j]);
                hl[j] = fma(t.g[k], ylo, hl[j]);
                hh[j] = fma(t.g[k], yhi, hh[j]);
            }
        }
    }
    if (col < half) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = i0 + 4 * q + j;
            if (row < half) {
                if (p.ll)
                    p.ll[(unsigned)b * p.ll_bs + (unsigned)row * p.ld_ll + col] = ll[j];
                else
                    wav_emit(p.epi, b, row, col, ll[j], o1[j][0], o2[j][0]);
                wav_emit(p.epi, b, row, half + col, lh[j], o1[j][1], o2[j][1]);
                wav_emit(p.epi, b, half + row, col, hl[j], o1[j][2], o2[j][2]);
                wav_emit(p.epi, b, half + row, half + col, hh[j], o1[j][3], o2[j][3]);
            }
        }
    }
}

// Grid: (g^2, 1, kWaveletBases / bpb) with g = ceil(s/2 / T), 256 threads.
template <typename R>
__global__ void __launch_bounds__(kWavThreads) __attribute__((amdgpu_waves_per_eu(kWavWaves<R>)))
dwt_level(DwtArgs<R> p) {
    __shared__ R X[kDwtIn][kDwtIn + 1];
    __shared__ R Y[kDwtIn][kDwtY];
    const int mask = p.s - 1;
    int tx, ty;
    const int gd = ((p.s >> 1) + kDwtT - 1) / kDwtT;
    xcd_tile(gd, gd, tx, ty);
    const int i0 = ty * kDwtT, c0 = tx * kDwtT;
    for (int bi = 0; bi < p.bpb; ++bi) {
        const int b = blockIdx.z * p.bpb + bi;
        if (bi > 0) __syncthreads();  // the previous basis is done with X and Y
        if (bi == 0 || p.in_bs != 0) {
            // all of a thread's loads are issued before the first LDS store
            constexpr int NL = (kDwtIn * kDwtIn + kWavThreads - 1) / kWavThreads;
            const int tid = opaque_tid();
            const R* src = p.in + (unsigned)b * p.in_bs;
            R v[NL];
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int e = tid + i * kWavThreads;
                const int r = e / kDwtIn, c = e % kDwtIn;
                if (e < kDwtIn * kDwtIn) v[i] = src[(unsigned)((2 * i0 + r) & mask) * p.ld_in + ((2 * c0 + c) & mask)];
            }
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int e = tid + i * kWavThreads;
                if (e < kDwtIn * kDwtIn) X[e / kDwtIn][e % kDwtIn] = v[i];
            }
            __syncthreads();
        }
        switch (p.taps[b].L) {
            case 2: dwt_tile<R, 2>(p, b, X, Y, i0, c0); break;
            case 4: dwt_tile<R, 4>(p, b, X, Y, i0, c0); break;
            case 6: dwt_tile<R, 6>(p, b, X, Y, i0, c0); break;
            case 8: dwt_tile<R, 8>(p, b, X, Y, i0, c0); break;
            case 10: dwt_tile<R, 10>(p, b, X, Y, i0, c0); break;
            case 12: dwt_tile<R, 12>(p, b, X, Y, i0, c0); break;
            case 14: dwt_tile<R, 14>(p, b, X, Y, i0, c0); break;
            default: dwt_tile<R, 16>(p, b, X, Y, i0, c0); break;
        }
    }
}

template <typename R>
struct IdwtArgs {
    const R* ll;       // lo-lo input (s/2 x s/2, row stride ld_ll, basis stride ll_bs); null: from the coefficients
    unsigned ll_bs;
    int ld_ll;
    const R* coef;     // coefficients: basis b at b * cstride, row stride ldc
    unsigned cstride;
    int ldc;
    R* out;            // s x s output, row stride ld_out, basis stride out_bs (bpb = 8: the sum, one image)
    unsigned out_bs;
    int ld_out;
    int s;
    int bpb;
    const Taps<R>* taps;
};

template <typename R, int L>
__device__ __forceinline__ void idwt_tile(const IdwtArgs<R>& p, int b, R (*Q)[kIdwtQR][kIdwtQC + 1],
                                          R (*U)[2 * kIdwtQC + 1], R (*acc)[2]) {
    const Taps<R>& t = p.taps[b];
    const int tid = opaque_tid();
    constexpr int H = L / 2;
    // columns: U[n][c] (c < Q: the row-lo half, c >= Q: the row-hi half).  The
    // output rows 2 np, 2 np + 1 both read quadrant rows np - kk + halo
    // (kk < L/2; the even row with taps 2 kk, the odd one with 2 kk + 1); a
    // task is 4 adjacent pairs np = 4 g + i of one column, which share a
    // window of L/2 + 3 quadrant rows.
    for (int e = tid; e < (kIdwtTR / 8) * (2 * kIdwtQC); e += kWavThreads) {
        const int g = e / (2 * kIdwtQC), cc = e % (2 * kIdwtQC);
        const int hiq = cc >= kIdwtQC;
        const int c = cc - hiq * kIdwtQC;
        const R (*qa)[kIdwtQC + 1] = Q[hiq];      // lo rows: ll or lh
        const R (*qb)[kIdwtQC + 1] = Q[2 + hiq];  // hi rows: hl or hh
        const int r0 = 4 * g + kIdwtHalo - (H - 1);
        R ev[4] = {0, 0, 0, 0}, od[4] = {0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < H + 3; ++u) {
            const R lo = qa[r0 + u][c], hi = qb[r0 + u][c];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kk = i + H - 1 - u;
                if (kk >= 0 && kk < H) {
                    ev[i] = fma(t.g[2 * kk], hi, fma(t.h[2 * kk], lo, ev[i]));
                    od[i] = fma(t.g[2 * kk + 1], hi, fma(t.h[2 * kk + 1], lo, od[i]));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            U[2 * (4 * g + i)][cc] = ev[i];
            U[2 * (4 * g + i) + 1][cc] = od[i];
        }
    }
    __syncthreads();
    // rows: output pairs (2 mp, 2 mp + 1) of row n read U[n][mp - kk + halo];
    // a task is 4 adjacent pairs mp = 4 g + i (acc[4 j + i]).
#pragma unroll
    for (int j = 0; j < kIdwtRowTasks; ++j) {
        const int e = tid + j * kWavThreads;
        const int n = e / (kIdwtTC / 8), g = e % (kIdwtTC / 8);
        const int m0 = 4 * g + kIdwtHalo - (H - 1);
        R ev[4] = {0, 0, 0, 0}, od[4] = {0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < H + 3; ++u) {
            const R lo = U[n][m0 + u], hi = U[n][kIdwtQC + m0 + u];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kk = i + H - 1 - u;
                if (kk >= 0 && kk < H) {
                    ev[i] = fma(t.g[2 * kk], hi, fma(t.h[2 * kk], lo, ev[i]));
                    od[i] = fma(t.g[2 * kk + 1], hi, fma(t.h[2 * kk + 1], lo, od[i]));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[4 * j + i][0] += ev[i];
            acc[4 * j + i][1] += od[i];
        }
    }
}

// Grid: (gx gy, 1, kWaveletBases / bpb) with gx = ceil(s / C), gy = ceil(s / R), 256 threads.
template <typename R>
__global__ void __launch_bounds__(kWavThreads) __attribute__((amdgpu_waves_per_eu(kWavWaves<R>)))
idwt_level(IdwtArgs<R> p) {
    __shared__ R Q[4][kIdwtQR][kIdwtQC + 1];  // lo-lo, lo rows of row-hi, hi rows of row-lo, hi-hi
    __shared__ R U[kIdwtTR][2 * kIdwtQC + 1];
    constexpr int J = (kIdwtTR * kIdwtTC / 2) / kWavThreads;
    const int half = p.s >> 1, hm = half - 1;
    int tx, ty;
    xcd_tile((p.s + kIdwtTC - 1) / kIdwtTC, (p.s + kIdwtTR - 1) / kIdwtTR, tx, ty);
    const int n0 = ty * kIdwtTR, m0 = tx * kIdwtTC;
    const int qr = n0 / 2 - kIdwtHalo, qc = m0 / 2 - kIdwtHalo;  // quadrant rows/cols of Q[.][0][0]
    R acc[J][2];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j][0] = acc[j][1] = 0;
    // The quadrant tiles of the next basis are loaded into registers while
    // the current one is computed; all of a thread's loads are issued before
    // any of them is waited for.
    constexpr int NL = (kIdwtQR * kIdwtQC + kWavThreads - 1) / kWavThreads;
    R v[4][NL];
    auto fetch = [&](int b) {
        const R* cf = p.coef + (unsigned)b * p.cstride;
        const R* llb = p.ll ? p.ll + (unsigned)b * p.ll_bs : nullptr;
        const int tid = opaque_tid();
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + i * kWavThreads;
            if (e < kIdwtQR * kIdwtQC) {
                const int row = (qr + e / kIdwtQC) & hm, col = (qc + e % kIdwtQC) & hm;
                v[0][i] = llb ? llb[(unsigned)row * p.ld_ll + col] : cf[(unsigned)row * p.ldc + col];
                v[1][i] = cf[(unsigned)row * p.ldc + half + col];
                v[2][i] = cf[(unsigned)(half + row) * p.ldc + col];
                v[3][i] = cf[(unsigned)(half + row) * p.ldc + half + col];
            }
        }
    };
    fetch(blockIdx.z * p.bpb);
    for (int bi = 0; bi < p.bpb; ++bi) {
        const int b = blockIdx.z * p.bpb + bi;
        {
            // Q is free: every thread has passed the barrier that ends the
            // previous basis's column pass
            const int tid = opaque_tid();
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int e = tid + i * kWavThreads;
                if (e < kIdwtQR * kIdwtQC) {
                    const int r = e / kIdwtQC, c = e % kIdwtQC;
#pragma unroll
                    for (int g = 0; g < 4; ++g) Q[g][r][c] = v[g][i];
                }
            }
        }
        __syncthreads();  // Q is written; the previous row pass is done with U
        if (bi + 1 < p.bpb) fetch(b + 1);
        switch (p.taps[b].L) {
            case 2: idwt_tile<R, 2>(p, b, Q, U, acc); break;
            case 4: idwt_tile<R, 4>(p, b, Q, U, acc); break;
            case 6: idwt_tile<R, 6>(p, b, Q, U, acc); break;
            case 8: idwt_tile<R, 8>(p, b, Q, U, acc); break;
            case 10: idwt_tile<R, 10>(p, b, Q, U, acc); break;
            case 12: idwt_tile<R, 12>(p, b, Q, U, acc); break;
            case 14: idwt_tile<R, 14>(p, b, Q, U, acc); break;
            default: idwt_tile<R, 16>(p, b, Q, U, acc); break;
        }
        if (p.bpb == 1 || bi == p.bpb - 1) {
            R* o = p.out + (unsigned)b * p.out_bs * (p.bpb == 1);
            const int tid = opaque_tid();
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int e = tid + (j / 4) * kWavThreads;  // acc[4 jt + i]: task jt, pair 4 g + i
                const int n = n0 + e / (kIdwtTC / 8), m = m0 + 2 * (4 * (e % (kIdwtTC / 8)) + j % 4);
                if (n < p.s && m < p.s) {
                    o[(unsigned)n * p.ld_out + m] = acc[j][0];
                    o[(unsigned)n * p.ld_out + m + 1] = acc[j][1];
                }
                acc[j][0] = acc[j][1] = 0;
            }
        }
    }
}

}  // namespace msr
