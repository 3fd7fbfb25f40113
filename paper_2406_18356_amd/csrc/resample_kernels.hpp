// resample_kernels.hpp -- up-sampling of the down-sampled low-resolution
// image (Sect. 6.1): out = U l_s = K l_s K^T with the N x N_s periodic
// band-limited interpolation matrix K[n][j] = k((n - d j) mod N), a function
// of one index (the Dirichlet sum of the small grid's band, tabulated on the
// host).  Two matrix products per call, each a 64 x 64 output tile per block
// staged through LDS; the K operand is read from the table.  One call per
// step-2 solve, next to hundreds of iterations: plain FMA, FP32 or FP64.
#pragma once
#include <hip/hip_runtime.h>

namespace msr {

constexpr int kRsT = 64;        // output tile side
constexpr int kRsK = 16;        // depth of one LDS stage
constexpr int kRsThreads = 256; // 16 x 16 threads, 4 x 4 outputs each

template <typename R>
struct DenseOperand {  // M(i, k) = p[i * ld + k]
    const R* p;
    int ld;
    __device__ R operator()(int i, int k) const { return p[(unsigned)i * ld + k]; }
};

template <typename R>
struct KernelRows {  // K(n, j) = tab[(n - d j) mod N]
    const R* tab;
    int mask;  // N - 1
    int d;
    __device__ R operator()(int n, int j) const { return tab[(n - d * j) & mask]; }
};

template <typename R>
struct KernelCols {  // K^T(j, n) = tab[(n - d j) mod N]
    const R* tab;
    int mask;
    int d;
    __device__ R operator()(int j, int n) const { return tab[(n - d * j) & mask]; }
};

// C (M x Ncols, row stride ldc) = A (M x K) B (K x Ncols).
// Grid: (ceil(Ncols / 64), ceil(M / 64)), 256 threads.
template <typename R, typename OA, typename OB>
__global__ void __launch_bounds__(kRsThreads) resample_product(OA a, OB b, R* __restrict__ C, int ldc, int M,
                                                               int Ncols, int K) {
    __shared__ R As[kRsK][kRsT + 1];  // As[k][i]
    __shared__ R Bs[kRsK][kRsT + 1];  // Bs[k][j]
    const int i0 = blockIdx.y * kRsT, j0 = blockIdx.x * kRsT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    R acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0;
    for (int k0 = 0; k0 < K; k0 += kRsK) {
#pragma unroll
        for (int e = 0; e < (kRsT * kRsK) / kRsThreads; ++e) {
            const int idx = threadIdx.x + e * kRsThreads;
            const int ia = idx / kRsK, ka = idx % kRsK;  // A: 64 rows x 16
            As[ka][ia] = (i0 + ia < M && k0 + ka < K) ? a(i0 + ia, k0 + ka) : (R)0;
            const int kb = idx / kRsT, jb = idx % kRsT;  // B: 16 x 64 columns
            Bs[kb][jb] = (k0 + kb < K && j0 + jb < Ncols) ? b(k0 + kb, j0 + jb) : (R)0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRsK; ++k) {
            R ar[4], br[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ar[u] = As[k][ty * 4 + u];
                br[u] = Bs[k][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += ar[u] * br[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + ty * 4 + u;
        if (i >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j < Ncols) C[(unsigned)i * ldc + j] = acc[u][v];
        }
    }
}

}  // namespace msr
