// fft_engine.hpp -- register/LDS radix-16 Stockham FFT building blocks for gfx950.
//
// A length-L complex FFT is computed cooperatively by TPF = L/E threads, each
// holding E = min(16, L) elements in registers.  Thread t holds element
// t + m*TPF in register m on entry and the output bin t + m*TPF on exit, so a
// forward transform followed by a pointwise multiply and an inverse transform
// needs no reordering: the inverse's first stage reads exactly the registers
// the forward's last stage wrote.  Stages are Stockham auto-sort passes of
// radix R = min(E, remaining length); between stages the data goes through
// LDS once (write, barrier, read, barrier).  Twiddles come from one table of
// exp(-2 pi i k / Pt), k < Pt, computed in double precision on the host and
// rounded to float (Pt = the logical transform length, L or 2L).
//
// Several independent arrays ("halves") can be transformed together so they
// share the barriers; each has its own LDS view.
#pragma once
#include <hip/hip_runtime.h>

namespace msr {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * w
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}
// a * conj(w)
__device__ __forceinline__ float2 cmulc(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, a.y * w.y), fmaf(a.y, w.x, -(a.x * w.y)));
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

template <int R>
__host__ __device__ constexpr int bit_reverse(int i) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// Multiply by w16^e (forward: exp(-2 pi i e/16); inverse: the conjugate), e in [0, 8).
template <bool INV>
__device__ __forceinline__ float2 rot16(float2 b, int e) {
    constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
    constexpr float S1 = 0.38268343236508978f;  // sin(pi/8)
    constexpr float H = 0.70710678118654752f;   // sqrt(1/2)
    if (e == 0) return b;
    if (e == 4) return INV ? make_float2(-b.y, b.x) : make_float2(b.y, -b.x);
    float c, s;
    switch (e) {
        case 1: c = C1; s = S1; break;
        case 2: c = H; s = H; break;
        case 3: c = S1; s = C1; break;
        case 5: c = -S1; s = C1; break;
        case 6: c = -H; s = H; break;
        default: c = -C1; s = S1; break;  // 7
    }
    // forward multiplies by (c, -s), inverse by (c, s)
    if (INV) return make_float2(fmaf(b.x, c, -(b.y * s)), fmaf(b.x, s, b.y * c));
    return make_float2(fmaf(b.x, c, b.y * s), fmaf(b.y, c, -(b.x * s)));
}

// In-register DFT of size R (2, 4, 8 or 16), natural order in and out.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
    float2 y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = x[bit_reverse<R>(i)];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const float2 a = y[i + k];
                const float2 b = rot16<INV>(y[i + k + len / 2], k * (16 / len));
                y[i + k] = cadd(a, b);
                y[i + k + len / 2] = csub(a, b);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = y[i];
}

// LDS view of one transform's data: element p lives at base[(p + p/16) * S + c]
// (one pad slot every 16 elements breaks the power-of-two strides of the
// Stockham writes; S interleaves several columns).
template <int S>
struct LdsView {
    float2* base;
    int c;
    __device__ __forceinline__ float2& operator[](int p) const { return base[(p + (p >> 4)) * S + c]; }
};

template <int L>
__host__ __device__ constexpr int padded_len() { return L + L / 16; }

template <int L>
__host__ __device__ constexpr int elems_per_thread() { return L >= 16 ? 16 : L; }

// One Stockham stage on NH arrays at once.  Butterfly b of thread t owns the
// register slots b + r*NB (r < R), so results go back into the same slots (last
// stage) or straight to LDS (other stages): no second register copy.
template <int L, int NS, bool INV, int TWS, int NH, int S>
__device__ __forceinline__ void fft_stage(float2 (&v)[NH][elems_per_thread<L>()], const LdsView<S> (&lds)[NH], int t,
                                          const float2* __restrict__ tw) {
    constexpr int E = elems_per_thread<L>();
    constexpr int TPF = L / E;
    constexpr int R = (L / NS) >= E ? E : (L / NS);
    constexpr int NB = E / R;
    constexpr bool LAST = (NS * R == L);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * TPF;
        const int jm = j & (NS - 1);
        float2 w[R];
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) w[r] = tw[(jm * r * (L / (NS * R))) * TWS];
        }
        const int idxD = (j - jm) * R + jm;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            float2 x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = v[h][b + r * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = INV ? cmulc(x[r], w[r]) : cmul(x[r], w[r]);
            }
            dft<R, INV>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[h][b + r * NB] = x[r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[h][idxD + r * NS] = x[r];
            }
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int m = 0; m < E; ++m) v[h][m] = lds[h][t + m * TPF];
        __syncthreads();
    }
}

template <int L, int NS, bool INV, int TWS, int NH, int S>
__device__ __forceinline__ void fft_from(float2 (&v)[NH][elems_per_thread<L>()], const LdsView<S> (&lds)[NH], int t,
                                         const float2* __restrict__ tw) {
    constexpr int E = elems_per_thread<L>();
    constexpr int R = (L / NS) >= E ? E : (L / NS);
    fft_stage<L, NS, INV, TWS, NH, S>(v, lds, t, tw);
    if constexpr (NS * R < L) fft_from<L, NS * R, INV, TWS, NH, S>(v, lds, t, tw);
}

// Full transform of NH arrays (unnormalised; INV uses conjugate twiddles).
// tw: the table of exp(-2 pi i k / (TWS * L)).  The caller must have a barrier
// between any earlier use of the LDS views and this call.
template <int L, bool INV, int TWS, int NH, int S>
__device__ __forceinline__ void fft(float2 (&v)[NH][elems_per_thread<L>()], const LdsView<S> (&lds)[NH], int t,
                                    const float2* __restrict__ tw) {
    fft_from<L, 1, INV, TWS, NH, S>(v, lds, t, tw);
}

// ---------------------------------------------------------------------------
// FP64 block reductions (deterministic: fixed shuffle tree, fixed wave order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums NQ doubles over a block of NT threads; thread 0 gets the totals in
// out[].  `scratch` must hold NQ * max(NT / 64, NT < 64 ? NT : 1) doubles.
template <int NQ, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double* scratch, double (&out)[NQ]) {
    if constexpr (NT >= 64) {
        constexpr int NW = NT / 64;
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double s = wave_sum(v[q]);
            if (lane == 0) scratch[q * NW + wave] = s;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double s = 0.0;
                for (int w = 0; w < NW; ++w) s += scratch[q * NW + w];
                out[q] = s;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) scratch[q * NT + threadIdx.x] = v[q];
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double s = 0.0;
                for (int w = 0; w < NT; ++w) s += scratch[q * NT + w];
                out[q] = s;
            }
        }
    }
    __syncthreads();
}

}  // namespace msr
