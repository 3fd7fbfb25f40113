// wavelet_kernels.hpp -- the wavelet dictionary W (concatenation of the
// orthonormal Daubechies bases db1 .. db8, 2-D, separable, periodic, nested
// coefficient layout) and the FISTA update on its coefficients.
//
// One level of one basis along an axis of length s (periodic), taps h[0..L),
// g[k] = (-1)^k h[L-1-k]:
//   analysis   lo[i] = sum_k h[k] x[(2i + k) mod s],  hi[i] = sum_k g[k] x[(2i + k) mod s]
//   synthesis  x[n]  = sum_{k = n mod 2, k < L} lo[m] h[k] + hi[m] g[k],  m = ((n - k) / 2) mod s/2
// (the synthesis is the transpose of the analysis, which is orthonormal).
// Arrays are row-major with row stride ld; a level works on the top-left
// s x s block.  Analysis: rows then columns; synthesis: columns then rows.
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

// Rows: out[r][i] = lo, out[r][s/2 + i] = hi, r < s, i < s/2.
template <typename R>
__global__ void dwt_rows(const R* __restrict__ in, int ld_in, R* __restrict__ out, int ld_out, int s,
                         const Taps<R>* __restrict__ taps) {
    const int r = blockIdx.y;
    const int half = s / 2;
    const Taps<R> t = *taps;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < half; i += gridDim.x * blockDim.x) {
        R lo = 0, hi = 0;
        for (int k = 0; k < t.L; ++k) {
            const R x = in[(size_t)r * ld_in + ((2 * i + k) & (s - 1))];
            lo += t.h[k] * x;
            hi += t.g[k] * x;
        }
        out[(size_t)r * ld_out + i] = lo;
        out[(size_t)r * ld_out + half + i] = hi;
    }
}

// Columns: out[i][c] = lo, out[s/2 + i][c] = hi, c < s, i < s/2.
template <typename R>
__global__ void dwt_cols(const R* __restrict__ in, int ld_in, R* __restrict__ out, int ld_out, int s,
                         const Taps<R>* __restrict__ taps) {
    const int i = blockIdx.y;
    const int half = s / 2;
    const Taps<R> t = *taps;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < s; c += gridDim.x * blockDim.x) {
        R lo = 0, hi = 0;
        for (int k = 0; k < t.L; ++k) {
            const R x = in[(size_t)((2 * i + k) & (s - 1)) * ld_in + c];
            lo += t.h[k] * x;
            hi += t.g[k] * x;
        }
        out[(size_t)i * ld_out + c] = lo;
        out[(size_t)(half + i) * ld_out + c] = hi;
    }
}

// Synthesis along columns of the s x s block: rows [0, s/2) are lo, [s/2, s)
// hi.  The top-left s/2 x s/2 quadrant comes from `ll` (row stride ld_ll)
// when given, everything else from `det` (row stride ld_det).
template <typename R>
__global__ void idwt_cols(const R* __restrict__ ll, int ld_ll, const R* __restrict__ det, int ld_det,
                          R* __restrict__ out, int ld_out, int s, const Taps<R>* __restrict__ taps) {
    const int n = blockIdx.y;
    const int half = s / 2;
    const Taps<R> t = *taps;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < s; c += gridDim.x * blockDim.x) {
        R acc = 0;
        for (int k = n & 1; k < t.L; k += 2) {
            const int m = ((n - k) / 2 + half) & (half - 1);  // (n - k) is even here
            const R lo = (ll && c < half) ? ll[(size_t)m * ld_ll + c] : det[(size_t)m * ld_det + c];
            const R hi = det[(size_t)(half + m) * ld_det + c];
            acc += t.h[k] * lo + t.g[k] * hi;
        }
        out[(size_t)n * ld_out + c] = acc;
    }
}

// Synthesis along rows: columns [0, s/2) lo, [s/2, s) hi; out += result when
// accumulate (the final level adds one basis's image into the sum).
template <typename R>
__global__ void idwt_rows(const R* __restrict__ in, int ld_in, R* __restrict__ out, int ld_out, int s,
                          const Taps<R>* __restrict__ taps, int accumulate) {
    const int r = blockIdx.y;
    const int half = s / 2;
    const Taps<R> t = *taps;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < s; n += gridDim.x * blockDim.x) {
        R acc = 0;
        for (int k = n & 1; k < t.L; k += 2) {
            const int m = ((n - k) / 2 + half) & (half - 1);
            acc += t.h[k] * in[(size_t)r * ld_in + m] + t.g[k] * in[(size_t)r * ld_in + half + m];
        }
        const size_t o = (size_t)r * ld_out + n;
        out[o] = accumulate ? out[o] + acc : acc;
    }
}

// FISTA update on coefficients (no positivity: the dictionary's prox is soft
// thresholding), with gc = W^T of the half-gradient image:
//   alpha_{k-1} = b1 + t_prev (b1 - b2);  beta_k = soft(alpha_{k-1} - 2 mu gc, mu lambda)
//   alpha_k = beta_k + t_cur (beta_k - b1);  beta_k -> b2, alpha_k -> a;  partial sums of |beta_k|.
template <typename R>
__global__ void __launch_bounds__(256) coeff_update(const R* __restrict__ b1, R* __restrict__ b2,
                                                    const R* __restrict__ gc, R* __restrict__ a, size_t n,
                                                    R two_mu, R thr, R t_prev, R t_cur,
                                                    double* __restrict__ partials) {
    __shared__ double red[4];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const R p1 = b1[i], p2 = b2[i];
        const R al = p1 + t_prev * (p1 - p2);
        const R z = al - two_mu * gc[i];
        const R zero = 0;
        const R beta = copysign(fmax(fabs(z) - thr, zero), z);
        b2[i] = beta;
        a[i] = beta + t_cur * (beta - p1);
        s += fabs((double)beta);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// dst[i] = a * src[i]
template <typename R>
__global__ void scale_copy(const R* __restrict__ src, R* __restrict__ dst, R a, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = a * src[i];
}

}  // namespace msr
