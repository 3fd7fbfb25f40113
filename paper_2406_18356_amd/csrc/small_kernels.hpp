// small_kernels.hpp -- reductions, PSF spectrum extraction and image helpers
// (included by the host API translation unit only).
#pragma once
#include "kernels.hpp"

namespace msr {

// Deterministic final reduction of per-block partials: out[q] = sum_b partials[b*NQ + q].
__global__ void __launch_bounds__(256) finalize_sums(const double* __restrict__ partials, int nblocks, int nq,
                                                     double* __restrict__ out) {
    __shared__ double red[4];
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)b * nq + q];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) out[q] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// One Lanczos step, in place: w <- w - alpha s_j u_j - cp u_p (q_j = s_j u_j,
// cp = beta_{j-1} s_{j-1}; u_p may be null for j = 1), with alpha read from
// device memory (the <q_j, A q_j> the preceding row pass reduced), and the
// per-block FP64 partial sums of ||w||^2.
template <typename R>
__global__ void __launch_bounds__(256) lanczos_step(R* __restrict__ w, const R* __restrict__ uj,
                                                    const R* __restrict__ up, const double* __restrict__ alpha,
                                                    R s_j, R cp, size_t n, double* __restrict__ partials) {
    __shared__ double red[4];
    const R a = (R)(alpha[0] * (double)s_j);
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        R r = w[i] - a * uj[i];
        if (up) r -= cp * up[i];
        w[i] = r;
        acc += (double)r * (double)r;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// PSF spectrum extraction: reads the complex forward spectrum (tiled with width
// TS, P rows), writes Re/P^2 tiled with width T (P rows), the per-column max
// |Re| and per-block partials (max |Re|, max |Im|).  One block per column.
template <typename R>
__global__ void __launch_bounds__(256) psf_extract(const cplx<R>* __restrict__ spec, int TS, int P, int T,
                                                   R* __restrict__ hh, double* __restrict__ colmax,
                                                   double* __restrict__ partials) {
    const int kx = blockIdx.x;
    __shared__ double mr[256], mi[256];
    double ar = 0.0, ai = 0.0;
    const R inv = (R)(1.0 / ((double)P * (double)P));
    for (int ky = threadIdx.x; ky < P; ky += 256) {
        const cplx<R> v = spec[((size_t)(kx / TS) * P + ky) * TS + kx % TS];
        ar = fmax(ar, fabs((double)v.x));
        ai = fmax(ai, fabs((double)v.y));
        hh[((size_t)(kx / T) * P + ky) * T + kx % T] = v.x * inv;
    }
    mr[threadIdx.x] = ar;
    mi[threadIdx.x] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            mr[threadIdx.x] = fmax(mr[threadIdx.x], mr[threadIdx.x + s]);
            mi[threadIdx.x] = fmax(mi[threadIdx.x], mi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        colmax[kx] = mr[0];
        partials[2 * kx] = mr[0];
        partials[2 * kx + 1] = mi[0];
    }
}

// Zero the columns [c0, c1) of a tiled P-row layout (tile tail of hh).
template <typename R>
__global__ void zero_hh_cols(R* __restrict__ hh, int P, int T, int c0, int c1) {
    const int ky = blockIdx.x * blockDim.x + threadIdx.x;
    if (ky >= P) return;
    for (int kx = c0; kx < c1; ++kx) hh[((size_t)(kx / T) * P + ky) * T + kx % T] = (R)0;
}

// Image reductions (FP64 partials, one per block):
//   mode 0: sum |x|          mode 1: sum x^2         mode 2: sum (x - y)^2
template <typename R>
__global__ void __launch_bounds__(256) image_sums(const R* __restrict__ x, const R* __restrict__ y, size_t n,
                                                  int mode, double* __restrict__ partials) {
    __shared__ double red[4];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double v = x[i];
        if (mode == 0) s += fabs(v);
        else if (mode == 1) s += v * v;
        else {
            const double d = v - (double)y[i];
            s += d * d;
        }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = a*x + b*y  (y may be null)
template <typename R>
__global__ void image_axpby(R* __restrict__ out, const R* __restrict__ x, const R* __restrict__ y, R a, R b,
                            size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R v = a * x[i];
    if (y) v = fmaR(b, y[i], v);
    out[i] = v;
}

// alpha_K = beta_K + t (beta_K - beta_{K-1}), with the update epilogue's
// operation order (a resumed solve continues from exactly this point).
template <typename R>
__global__ void momentum_point(R* __restrict__ out, const R* __restrict__ bk, const R* __restrict__ bp, R t,
                               size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const R b = bk[i];
    out[i] = fmaR(t, b - bp[i], b);
}

// The same from float64 iterates, rounded once to R.
template <typename R>
__global__ void momentum_point_it64(R* __restrict__ out, const double* __restrict__ bk,
                                    const double* __restrict__ bp, double t, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = bk[i];
    out[i] = (R)fma(t, b - bp[i], b);
}

// out[i] = (To) in[i]: float images to float64 iterates and back.
template <typename To, typename From>
__global__ void convert_image(To* __restrict__ out, const From* __restrict__ in, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (To)in[i];
}

// Power-iteration start vector: v[n] = splitmix64_mix(seed + n) * 2^-64 - 1/2,
// taking the top 53 bits for an exact double, then rounding to R.
__device__ __forceinline__ unsigned long long splitmix64_mix(unsigned long long c) {
    unsigned long long z = c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
template <typename R>
__global__ void start_vector(R* __restrict__ v, unsigned long long seed, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long z = splitmix64_mix(seed + (unsigned long long)i);
    v[i] = (R)((double)(z >> 11) * 0x1.0p-53 - 0.5);
}

// sigma2_hat: mean over all 5x5 windows inside the image of the population
// variance.  One thread per window top-left corner; FP64 accumulation.
template <typename R>
__global__ void __launch_bounds__(256) window_variance(const R* __restrict__ img, int n,
                                                       double* __restrict__ partials) {
    __shared__ double red[4];
    const int m = n - 4;  // windows per axis
    double s = 0.0;
    for (size_t w = (size_t)blockIdx.x * 256 + threadIdx.x; w < (size_t)m * m; w += (size_t)gridDim.x * 256) {
        const int i0 = (int)(w / m), j0 = (int)(w % m);
        double sum = 0.0, sq = 0.0;
#pragma unroll
        for (int di = 0; di < 5; ++di)
#pragma unroll
            for (int dj = 0; dj < 5; ++dj) {
                const double v = img[(size_t)(i0 + di) * n + j0 + dj];
                sum += v;
                sq += v * v;
            }
        const double mean = sum / 25.0;
        s += sq / 25.0 - mean * mean;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace msr
