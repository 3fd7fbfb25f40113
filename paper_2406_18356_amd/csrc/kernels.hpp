// kernels.hpp -- the passes of one FISTA iteration on gfx950.
//
// Data layout.  An image is N x N float32, row-major.  Its "row spectrum"
// (the DFT along x of each zero-embedded row, kept for the N image rows) is a
// complex64 array of N rows by K stored columns k_x (K <= P/2 + 1), laid out
// in column tiles of width T: element (row, k_x) lives at
//     spec[((k_x / T) * NR + row) * T + k_x % T].
// A column pass therefore reads one contiguous block per tile, and a row pass
// writes contiguous (rows x T) chunks.
//
// Zero padding.  With P = 2N the image occupies indices [0, N) of each
// length-P line (the placement inside the P grid does not change H, since the
// spectral multipliers are real and the shift commutes with them).  A
// length-P DFT of a half-zero line splits into two length-N DFTs: the
// even bins are DFT_N(y), the odd bins DFT_N(y . w_P^i).  The inverse,
// cropped to the first N outputs, is IDFT_N(even) + w_P^-i IDFT_N(odd).
// The same code with one half is the unpadded (circular, or PSF) transform.
//
// Two real rows are transformed together as one complex line z = a + i b and
// separated with X_a[k] = (Z[k] + conj Z[P-k]) / 2, X_b[k] = -i (Z[k] - conj Z[P-k]) / 2.
#pragma once
#include "fft_engine.hpp"

namespace msr {

template <int L, bool PADDED>
struct LineCfg {
    static constexpr int E = elems_per_thread<L>();
    static constexpr int TPF = L / E;               // threads per line (pair of rows) / per column
    static constexpr int NH = PADDED ? 2 : 1;       // half transforms per line
    static constexpr int PT = PADDED ? 2 * L : L;   // logical transform length P
    static constexpr int TWS = PADDED ? 2 : 1;      // stride of FFT_L twiddles in the P table
    static constexpr int HALF = PT / 2;             // last half-plane column index
};

__device__ __forceinline__ size_t spec_idx(int kx, int row, int NR, int T) {
    return ((size_t)(kx / T) * NR + row) * T + (kx % T);
}

// ===========================================================================
// Row pass
// ===========================================================================
struct RowArgs {
    const float2* __restrict__ spec_in;   // tiled row spectrum (INV_IN)
    const float2* __restrict__ spec_in2;  // optional second spectrum added for k_x < K_in2
    float2* __restrict__ spec_out;        // tiled row spectrum (FWD_OUT)
    const float2* __restrict__ tw;        // exp(-2 pi i k / P), k < P
    double* __restrict__ partials;        // NQ doubles per block
    int NR;                               // rows of the spectra (= image rows)
    int K_in;                             // stored columns of spec_in
    int K_in2;                            // columns of spec_in2 (0: none)
    int K_out;                            // columns to write (the tile tail is zero-filled)
};

template <int L, bool PADDED, int PAIRS, int T, bool INV_IN, bool FWD_OUT, class Epi>
__global__ void __launch_bounds__((PAIRS * LineCfg<L, PADDED>::TPF))
row_kernel(RowArgs a, Epi epi) {
    using C = LineCfg<L, PADDED>;
    constexpr int E = C::E, TPF = C::TPF, NH = C::NH, PT = C::PT, HALF = C::HALF;
    constexpr int ZLEN = padded_len<PT>();
    constexpr int NT = PAIRS * TPF;
    constexpr int NQ = Epi::NQ;
    __shared__ float2 lds[PAIRS * ZLEN];
    __shared__ double red[(NQ > 0 ? NQ : 1) * (NT >= 64 ? NT / 64 : NT)];

    const int tid = threadIdx.x;
    const int pair = tid / TPF;
    const int t = tid - pair * TPF;
    const int row0 = blockIdx.x * (2 * PAIRS);
    const int ra = row0 + 2 * pair;
    const LdsView<1> zv{lds + pair * ZLEN, 0};
    LdsView<1> hv[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hv[h] = LdsView<1>{lds + pair * ZLEN + h * padded_len<L>(), 0};

    float2 v[NH][E];
    float2 z[E];

    if constexpr (INV_IN) {
        // Half-plane columns of both rows -> full Hermitian-combined line Z in LDS.
        for (int q = tid; q < ((HALF + T) / T) * T * PAIRS; q += NT) {
            // q -> (kx, p) with kx % T fastest, then the pair, then the tile
            const int c = q % T;
            const int rest = q / T;
            const int p = rest % PAIRS;
            const int kx = (rest / PAIRS) * T + c;
            if (kx > HALF) continue;
            float2 xa = make_float2(0.f, 0.f), xb = xa;
            const int rr = row0 + 2 * p;
            if (kx < a.K_in) {
                xa = a.spec_in[spec_idx(kx, rr, a.NR, T)];
                xb = a.spec_in[spec_idx(kx, rr + 1, a.NR, T)];
            }
            if (kx < a.K_in2) {
                xa = cadd(xa, a.spec_in2[spec_idx(kx, rr, a.NR, T)]);
                xb = cadd(xb, a.spec_in2[spec_idx(kx, rr + 1, a.NR, T)]);
            }
            const LdsView<1> zp{lds + p * ZLEN, 0};
            zp[kx] = make_float2(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
            if (kx > 0 && kx < HALF) zp[PT - kx] = make_float2(xa.x + xb.y, xb.x - xa.y);  // conj Xa + i conj Xb
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int h = 0; h < NH; ++h) v[h][m] = zv[NH * (t + m * TPF) + h];
        __syncthreads();
        fft<L, true, C::TWS, NH, 1>(v, hv, t, a.tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            float2 s = v[0][m];
            if constexpr (PADDED) s = cadd(s, cmulc(v[1][m], a.tw[t + m * TPF]));
            z[m] = s;
        }
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = make_float2(0.f, 0.f);
    }

    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) acc[q] = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = epi.apply(ra, t + m * TPF, z[m], acc);

    if constexpr (FWD_OUT) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            v[0][m] = z[m];
            if constexpr (PADDED) v[1][m] = cmul(z[m], a.tw[t + m * TPF]);
        }
        __syncthreads();
        fft<L, false, C::TWS, NH, 1>(v, hv, t, a.tw);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int h = 0; h < NH; ++h) zv[NH * (t + m * TPF) + h] = v[h][m];
        __syncthreads();
        const int ntile = (a.K_out + T - 1) / T;
        for (int q = tid; q < ntile * T * PAIRS; q += NT) {
            const int c = q % T;
            const int rest = q / T;
            const int p = rest % PAIRS;
            const int kx = (rest / PAIRS) * T + c;
            const int rr = row0 + 2 * p;
            float2 xa = make_float2(0.f, 0.f), xb = xa;
            if (kx < a.K_out) {
                const LdsView<1> zp{lds + p * ZLEN, 0};
                const float2 zk = zp[kx];
                const float2 zm = zp[kx == 0 ? 0 : PT - kx];
                xa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
                xb = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            }
            a.spec_out[spec_idx(kx, rr, a.NR, T)] = xa;
            a.spec_out[spec_idx(kx, rr + 1, a.NR, T)] = xb;
        }
    }

    if constexpr (NQ > 0) {
        double tot[NQ];
        block_sum<NQ, NT>(acc, red, tot);
        if (tid == 0)
#pragma unroll
            for (int q = 0; q < NQ; ++q) a.partials[(size_t)blockIdx.x * NQ + q] = tot[q];
    }
}

// ---------------------------------------------------------------------------
// Row epilogues.  apply(row, i, z, acc) gets the cropped inverse result of
// rows (row, row+1) at column i packed as z = (x_row, x_row+1) and returns the
// pair to transform forward (or anything, when nothing follows).
// ---------------------------------------------------------------------------

// Load an image (times a scale): the forward pass of a plain row transform.
struct EpiLoad {
    static constexpr int NQ = 0;
    const float* __restrict__ img;
    int ld;
    float scale;
    __device__ __forceinline__ float2 apply(int r, int i, float2, double*) const {
        return make_float2(scale * img[(size_t)r * ld + i], scale * img[(size_t)(r + 1) * ld + i]);
    }
};

// Load a P x P PSF with ifftshift (row and column rolled by P/2).
struct EpiLoadShift {
    static constexpr int NQ = 0;
    const float* __restrict__ img;
    int P;
    __device__ __forceinline__ float2 apply(int r, int i, float2, double*) const {
        const int h = P / 2;
        const int c = (i + h) & (P - 1);
        return make_float2(img[(size_t)((r + h) & (P - 1)) * P + c], img[(size_t)((r + 1 + h) & (P - 1)) * P + c]);
    }
};

// Store the cropped inverse (times a scale) as an image.
struct EpiStore {
    static constexpr int NQ = 0;
    float* __restrict__ out;
    int ld;
    float scale;
    __device__ __forceinline__ float2 apply(int r, int i, float2 z, double*) const {
        out[(size_t)r * ld + i] = scale * z.x;
        out[(size_t)(r + 1) * ld + i] = scale * z.y;
        return z;
    }
};

// r = H x - y (y may be null): accumulates ||r||^2, optionally stores r, forwards r.
struct EpiResid {
    static constexpr int NQ = 1;
    const float* __restrict__ y;
    float* __restrict__ r_out;
    int ld;
    __device__ __forceinline__ float2 apply(int r, int i, float2 z, double* acc) const {
        if (y) {
            z.x -= y[(size_t)r * ld + i];
            z.y -= y[(size_t)(r + 1) * ld + i];
        }
        acc[0] += (double)z.x * z.x + (double)z.y * z.y;
        if (r_out) {
            r_out[(size_t)r * ld + i] = z.x;
            r_out[(size_t)(r + 1) * ld + i] = z.y;
        }
        return z;
    }
};

// The FISTA update (Algorithm 1) on gradient half-values s = grad/2:
//   alpha_{k-1} = b1 + t_prev (b1 - b2)        (b1 = beta_{k-1}, b2 = beta_{k-2})
//   beta_k      = prox(alpha_{k-1} - mu * 2 s)  (soft threshold at mu*lambda, or its positive part)
//   alpha_k     = beta_k + t_cur (beta_k - b1)
// beta_k overwrites b2 (same element, same thread); alpha_k is forwarded.
struct EpiUpdate {
    static constexpr int NQ = 1;
    const float* __restrict__ b1;
    float* __restrict__ b2;  // in: beta_{k-2}; out: beta_k
    int ld;
    float two_mu;     // 2 mu
    float thr;        // mu * lambda
    float t_prev, t_cur;
    int positivity;
    __device__ __forceinline__ float upd(float s, float p1, float& p2) const {
        const float alpha = fmaf(t_prev, p1 - p2, p1);
        const float zz = fmaf(-two_mu, s, alpha);
        float beta;
        if (positivity) beta = fmaxf(zz - thr, 0.f);
        else beta = copysignf(fmaxf(fabsf(zz) - thr, 0.f), zz);
        p2 = beta;
        return fmaf(t_cur, beta - p1, beta);
    }
    __device__ __forceinline__ float2 apply(int r, int i, float2 z, double* acc) const {
        const size_t ia = (size_t)r * ld + i, ib = ia + ld;
        float pa = b2[ia], pb = b2[ib];
        const float qa = upd(z.x, b1[ia], pa);
        const float qb = upd(z.y, b1[ib], pb);
        b2[ia] = pa;
        b2[ib] = pb;
        acc[0] += (double)fabsf(pa) + (double)fabsf(pb);
        return make_float2(qa, qb);
    }
};

// Power iteration: w = A v.  Accumulates <w, w> and <w, vprev>, stores w.
struct EpiPower {
    static constexpr int NQ = 2;
    const float* __restrict__ vprev;
    float* __restrict__ w_out;
    int ld;
    float vscale;  // v = vscale * vprev
    __device__ __forceinline__ float2 apply(int r, int i, float2 z, double* acc) const {
        const size_t ia = (size_t)r * ld + i, ib = ia + ld;
        acc[0] += (double)z.x * z.x + (double)z.y * z.y;
        acc[1] += (double)z.x * (vscale * vprev[ia]) + (double)z.y * (vscale * vprev[ib]);
        w_out[ia] = z.x;
        w_out[ib] = z.y;
        return z;
    }
};

// ===========================================================================
// Column pass: DFT along y of each stored column, pointwise multiply, inverse,
// crop.  One block handles T adjacent columns (one tile).
// ===========================================================================
struct ColArgs {
    const float2* __restrict__ spec_in;
    const float2* __restrict__ spec_in2;  // subtracted from spec_in before the transform (or null)
    float2* __restrict__ spec_out;
    const float2* __restrict__ tw;
    double* __restrict__ partials;
    int NR;   // rows of the spectra (L for the unpadded transforms, N when padded)
    int K;    // columns processed: tiles 0 .. ceil(K/T)-1; columns >= K read as zero
};

template <int L, bool PADDED, int T, class Mode>
__global__ void __launch_bounds__((T * LineCfg<L, PADDED>::TPF))
col_kernel(ColArgs a, Mode md) {
    using C = LineCfg<L, PADDED>;
    constexpr int E = C::E, TPF = C::TPF, NH = C::NH;
    constexpr int NT = T * TPF;
    constexpr int NQ = Mode::NQ;
    constexpr int HL = padded_len<L>();
    __shared__ float2 lds[NH * T * HL];
    __shared__ double red[(NQ > 0 ? NQ : 1) * (NT >= 64 ? NT / 64 : NT)];

    const int tid = threadIdx.x;
    const int c = tid % T;
    const int t = tid / T;
    const int tile = blockIdx.x;
    const int kx = tile * T + c;
    const bool live = kx < a.K;
    LdsView<T> hv[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hv[h] = LdsView<T>{lds + h * T * HL, c};

    float2 v[NH][E];
    const size_t base = (size_t)tile * a.NR * T + c;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = t + m * TPF;
        float2 y = make_float2(0.f, 0.f);
        if (live) {
            y = a.spec_in[base + (size_t)i * T];
            if (a.spec_in2) y = csub(y, a.spec_in2[base + (size_t)i * T]);
        }
        v[0][m] = y;
        if constexpr (PADDED) v[1][m] = cmul(y, a.tw[i]);
    }
    fft<L, false, C::TWS, NH, T>(v, hv, t, a.tw);

    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) acc[q] = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int ky = NH * (t + m * TPF) + h;
            const float2 r = md.apply(tile, c, kx, ky, live, v[h][m], acc);
            v[h][m] = live ? r : make_float2(0.f, 0.f);
        }

    if constexpr (Mode::INVERSE) {
        __syncthreads();
        fft<L, true, C::TWS, NH, T>(v, hv, t, a.tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = t + m * TPF;
            float2 s = v[0][m];
            if constexpr (PADDED) s = cadd(s, cmulc(v[1][m], a.tw[i]));
            a.spec_out[base + (size_t)i * T] = s;
        }
    } else if constexpr (Mode::STORE_SPECTRUM) {
        // unpadded forward transform only: bin ky = t + m*TPF
#pragma unroll
        for (int m = 0; m < E; ++m) a.spec_out[base + (size_t)(t + m * TPF) * T] = v[0][m];
    }

    if constexpr (NQ > 0) {
        double tot[NQ];
        block_sum<NQ, NT>(acc, red, tot);
        if (tid == 0)
#pragma unroll
            for (int q = 0; q < NQ; ++q) a.partials[(size_t)blockIdx.x * NQ + q] = tot[q];
    }
}

// Multiply by the cached PSF spectrum (already scaled by 1/P^2), tiled like
// the spectra with P rows: hh[((kx/T) * P + ky) * T + kx%T].
struct ModePsf {
    static constexpr int NQ = 0;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    const float* __restrict__ hh;
    int P;
    int T;
    __device__ __forceinline__ float2 apply(int tile, int c, int, int ky, bool, float2 y, double*) const {
        return cscale(y, hh[((size_t)tile * P + ky) * T + c]);
    }
};

// Filter responses of Eqs. 6-10 (squared), evaluated per DFT cell.
struct FilterCoef {
    float ell, delta, inv_sigma2, inv_eta2, sigma2, eta2, half_pi_over_delta;
    int P;
    __device__ __forceinline__ float radius(int kx, int ky) const {
        const int sy = ky < P / 2 ? ky : ky - P;
        const int sx = kx < P / 2 ? kx : kx - P;  // kx <= P/2 in the half plane
        return sqrtf((float)(sx * sx + sy * sy));
    }
    // returns (gL^2, gH^2)
    __device__ __forceinline__ float2 sq(int kx, int ky) const {
        const float r = radius(kx, ky);
        if (r > ell + delta) return make_float2(0.f, inv_sigma2);
        if (r < ell - delta) return make_float2(inv_eta2, 0.f);
        const float s = sinf(half_pi_over_delta * (r - ell));
        const float lo = (1.f - s) * (1.f - s), hi = (1.f + s) * (1.f + s);
        const float a2 = 1.f / (sigma2 * hi + eta2 * lo);
        return make_float2(a2 * lo, a2 * hi);
    }
};

__device__ __forceinline__ double col_weight(int kx, int P) { return (kx == 0 || kx == P / 2) ? 1.0 : 2.0; }

// Multiply by g_H^2 / P^2; accumulates (1/P^2) sum g_H^2 |Y|^2 over the full plane.
struct ModeFilterH {
    static constexpr int NQ = 1;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    FilterCoef f;
    float inv_p2;
    __device__ __forceinline__ float2 apply(int, int, int kx, int ky, bool live, float2 y, double* acc) const {
        const float g = f.sq(kx, ky).y;
        if (live) acc[0] += col_weight(kx, f.P) * (double)g * ((double)y.x * y.x + (double)y.y * y.y);
        return cscale(y, g * inv_p2);
    }
};

// Multiply by g_L^2 / P^2 (input: spectrum of alpha minus spectrum of l);
// accumulates (1/P^2) sum g_L^2 |Y|^2 = ||G_L (l - alpha)||^2 * P^2.
struct ModeFilterL {
    static constexpr int NQ = 1;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    FilterCoef f;
    float inv_p2;
    __device__ __forceinline__ float2 apply(int, int, int kx, int ky, bool live, float2 y, double* acc) const {
        const float g = f.sq(kx, ky).x;
        if (live) acc[0] += col_weight(kx, f.P) * (double)g * ((double)y.x * y.x + (double)y.y * y.y);
        return cscale(y, g * inv_p2);
    }
};

// Forward transform only (PSF spectrum), bins stored in place.
struct ModeForward {
    static constexpr int NQ = 0;
    static constexpr bool INVERSE = false;
    static constexpr bool STORE_SPECTRUM = true;
    __device__ __forceinline__ float2 apply(int, int, int, int, bool, float2 y, double*) const { return y; }
};

}  // namespace msr
