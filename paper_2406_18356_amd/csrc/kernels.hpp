// kernels.hpp -- the passes of one FISTA iteration on gfx950, in single or
// double precision (R = float or double, C = the complex type).
//
// Data layout.  An image is N x N, row-major.  Its "row spectrum" (the DFT
// along x of each zero-embedded row, kept for the N image rows) is a complex
// array of N rows by K stored columns k_x (K <= P/2 + 1), laid out in column
// tiles of width T: element (row, k_x) lives at
//     spec[((k_x / T) * NR + row) * T + k_x % T].
// A column pass therefore reads one contiguous block per tile, and a row pass
// writes contiguous (rows x T) chunks.
//
// Zero padding.  With P = 2N the image occupies indices [0, N) of each
// length-P line (the placement inside the P grid does not change H, since the
// spectral multipliers are real and the shift commutes with them).  A
// length-P DFT of a half-zero line splits into two length-N DFTs: the even
// bins are DFT_N(y), the odd bins DFT_N(y . w_P^i).  The inverse, cropped to
// the first N outputs, is IDFT_N(even) + w_P^-i IDFT_N(odd).  The same code
// with one half is the unpadded (circular, or PSF) transform.
//
// Two real rows are transformed together as one complex line z = a + i b and
// separated with X_a[k] = (Z[k] + conj Z[P-k]) / 2, X_b[k] = -i (Z[k] - conj Z[P-k]) / 2.
//
// Reductions (objective terms, power-iteration sums) are FP64 per-block
// partials, computed only when the launch asks for them (`reduce`).
#pragma once
#include <cstdint>

#include "fft_engine.hpp"

namespace msr {

template <int L, bool PADDED, typename R, int EMAX>
struct LineCfg {
    using C = cplx<R>;
    static constexpr int E = elems_per_thread(L, EMAX);
    static constexpr int TPF = L / E;               // threads per line (pair of rows) / per column
    static constexpr int NH = PADDED ? 2 : 1;       // half transforms per line
    static constexpr int PT = PADDED ? 2 * L : L;   // logical transform length P
    static constexpr int TWS = PADDED ? 2 : 1;      // stride of FFT_L twiddles in the P table
    static constexpr int HALF = PT / 2;             // last half-plane column index
};

// Workgroups are handed to the 8 XCDs of the chip round robin (block b runs on
// XCD b % 8), and each XCD has its own L2.  Remapping the block index so that
// consecutive logical blocks run on the same XCD lets neighbours share the L2
// lines of the tiled spectra (a 128-byte line holds several rows of a tile).
// XCD x runs blocks x, x + 8, ...: q + 1 of them for x < r and q for the
// others (nblocks = 8 q + r); they take the logical range starting at
// x q + min(x, r), so the map is a bijection for any grid size.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    constexpr int NX = 8;
    const int q = nblocks / NX, r = nblocks % NX, x = b % NX;
    return x * q + (x < r ? x : r) + b / NX;
}

__device__ __forceinline__ uint32_t spec_idx(int kx, int row, int NR, int T) {
    return ((uint32_t)kx / T * (uint32_t)NR + (uint32_t)row) * (uint32_t)T + (uint32_t)kx % T;
}

// ===========================================================================
// Batched launches.  The channels of one launch (blockIdx.y) have identical
// workspace layouts spaced `cstride` bytes apart, so every workspace pointer of
// channel c is the first channel's plus c * cstride; what differs in value per
// channel (step size, threshold, filters) comes from small per-channel arrays.
// ===========================================================================
template <typename R>
struct ChanScalars {
    R two_mu;      // 2 mu
    R thr;         // mu lambda
    R inv_sigma2;  // 1 / sigma^2 (step 2)
    R unused;
};
template <typename R>
struct FilterCoef;

template <typename T>
__device__ __forceinline__ T* shifted(T* p, long long off) {
    return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + off) : p;
}

// ===========================================================================
// Row pass
// ===========================================================================
template <typename R>
struct RowArgs {
    using C = cplx<R>;
    const C* __restrict__ spec_in;   // tiled row spectrum (INV_IN)
    const C* __restrict__ spec_in2;  // optional second spectrum added for k_x < K_in2
    C* __restrict__ spec_out;        // tiled row spectrum (FWD_OUT)
    const C* __restrict__ tw;        // exp(-2 pi i k / P), k < P
    const C* __restrict__ tws;       // FFT stage twiddle tables of length L
    double* __restrict__ partials;   // NQ doubles per block (when reduce)
    int NR;                          // rows of the spectra (= image rows)
    int K_in;                        // stored columns of spec_in
    int K_in2;                       // columns of spec_in2 (0: none)
    int K_out;                       // columns to write (the tile tail is zero-filled)
    int reduce;                      // accumulate the epilogue's FP64 sums
    int nch;                         // channels of a batched launch (grid y); 0 or 1: one
    long long cstride;               // batched: bytes between two channels' workspaces (0: not batched)
    const ChanScalars<R>* __restrict__ chan;  // batched: per-channel scalars (or null)
    __device__ __forceinline__ void to_channel(long long off) {
        spec_in = shifted(spec_in, off);
        spec_in2 = shifted(spec_in2, off);
        spec_out = shifted(spec_out, off);
        tw = shifted(tw, off);
        tws = shifted(tws, off);
        partials = shifted(partials, off);
    }
};

// Waves per SIMD the register allocation is made for: what the LDS footprint
// of the variant allows (2 with 16 complex per thread, 4 with 8 or fewer).
template <int EMAX, typename R>
constexpr int waves_per_eu() {
    return (EMAX * (int)sizeof(cplx<R>)) >= 128 ? 2 : 4;
}
#ifdef MSR_WAVES_PER_EU
#define MSR_WAVES_ATTR(EMAX, R) __attribute__((amdgpu_waves_per_eu(waves_per_eu<EMAX, R>())))
#else
#define MSR_WAVES_ATTR(EMAX, R)
#endif

// A row kernel whose epilogue holds prefetched values across the inverse
// transform (Epi::MIN_WAVES = 4) is compiled for four waves per SIMD when it
// keeps 8 or fewer complex values per thread, so that its register count stays
// within what two 512-thread blocks per CU allow.
template <class Epi, int EMAX, typename R>
constexpr int row_min_waves() {
    return (EMAX * (int)sizeof(cplx<R>)) < 128 ? Epi::MIN_WAVES : 1;
}
#ifdef MSR_WAVES_PER_EU
#define MSR_ROW_WAVES_ATTR(EMAX, R, Epi) MSR_WAVES_ATTR(EMAX, R)
#else
#define MSR_ROW_WAVES_ATTR(EMAX, R, Epi) __attribute__((amdgpu_waves_per_eu(row_min_waves<Epi, EMAX, R>())))
#endif

// Row kernels exchange FFT stages through two LDS arrays (one barrier per
// stage) when the doubled footprint still lets a CU hold blocks for 16 waves
// (4 per SIMD), or when the launch has no more blocks than the chip has CUs
// (256), so that no CU would hold a second one anyway.  Otherwise they use one
// array and two barriers per stage, and the extra resident blocks hide the
// global loads and stores of their neighbours (MSR_ROW_PINGPONG = 0 turns
// ping-pong off everywhere).
#ifndef MSR_ROW_PINGPONG
#define MSR_ROW_PINGPONG 1
#endif
#ifndef MSR_REFETCH
#define MSR_REFETCH 1
#endif
#ifndef MSR_TW_PRELOAD_INV
#define MSR_TW_PRELOAD_INV 0
#endif
#ifndef MSR_LATE_LDS
#define MSR_LATE_LDS 1
#endif

// LDS pointer type (ds_read / ds_write, not flat accesses).
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

// Copies the n reals at src (global, 16-byte aligned, n a multiple of
// 64 * 16 / sizeof(R) per wave) into LDS at dst without passing through
// registers: each of the nw waves of a line issues direct-to-LDS loads
// (global_load_lds_dwordx4) for its share; wave w of lane l moves 16 bytes at
// offset (w * share + c * 64 + l) * 16.  The data is in LDS once the issuing
// wave has waited for its vector memory counter; other waves see it after a
// barrier that follows that wait.
template <typename R, int N, int NW>
__device__ __forceinline__ void load_to_lds(const R* __restrict__ src, R* dst, int t) {
    constexpr int EL = 16 / (int)sizeof(R);
    constexpr int SHARE = N / NW;
    constexpr int NI = SHARE / (64 * EL);
    static_assert(N % NW == 0 && SHARE % (64 * EL) == 0, "share must be whole 1 KiB wave loads");
    const int w = t >> 6, lane = t & 63;
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        const int off = w * SHARE + c * 64 * EL;
        __builtin_amdgcn_global_load_lds((const void*)(src + off + lane * EL), (lds_ptr<void>)(dst + off), 16, 0, 0);
    }
}
constexpr size_t kLdsBytes = 160 * 1024;

// LDS slots of one row pair's line: the staged Hermitian line of length PT
// (one pad slot per 16) and the NH half transforms of length L placed over it.
__host__ __device__ constexpr int row_line_len(int L, bool padded, int E) {
    const int PT = padded ? 2 * L : L;
    const int NH = padded ? 2 : 1;
    const int a = padded_len(PT);
    const int b = NH * fft_lds_len(L, E < L ? E : L, 1);
    return a > b ? a : b;
}
constexpr bool row_pingpong(size_t line_bytes, int threads, int grid_blocks) {
    const int waves = threads >= 64 ? threads / 64 : 1;
    const int resident = (16 + waves - 1) / waves;
    return MSR_ROW_PINGPONG && 2 * line_bytes <= kLdsBytes - 4096 &&
           (grid_blocks <= 256 || (size_t)resident * 2 * line_bytes <= kLdsBytes);
}

// The column items of a row block: item u of thread `tid` is q = tid + u NT,
// i.e. column kx of row pair p (kx % T fastest, then the pair, then the tile).
// `ia` is the tiled spectrum index of row row0 + 2p at that column; the pair's
// second row is at ia + T.  When NT is a multiple of T * PAIRS, p does not
// depend on u and kx and ia advance by uniform steps.
template <int T, int PAIRS, int NT>
struct RowItems {
    static constexpr bool REG = NT % (T * PAIRS) == 0;
    int tid, row0, NR, p0, kx0;
    uint32_t i0, istep;
    __device__ __forceinline__ RowItems(int tid_, int row0_, int NR_) : tid(tid_), row0(row0_), NR(NR_) {
        p0 = (tid / T) % PAIRS;
        kx0 = (tid / T / PAIRS) * T + tid % T;
        i0 = spec_idx(kx0, row0 + 2 * p0, NR, T);
        istep = (uint32_t)(NT / PAIRS) * (uint32_t)NR;
    }
    __device__ __forceinline__ void get(int u, int& q, int& p, int& kx, uint32_t& ia) const {
        q = tid + u * NT;
        if constexpr (REG) {
            p = p0;
            kx = kx0 + u * (NT / PAIRS);
            ia = i0 + (uint32_t)u * istep;
        } else {
            const int rest = q / T;
            p = rest % PAIRS;
            kx = (rest / PAIRS) * T + q % T;
            ia = spec_idx(kx, row0 + 2 * p, NR, T);
        }
    }
};

// LDS of a row pass (complex slots and FP64 reduction scratch).
template <typename R, int L, bool PADDED, int EMAX, int PAIRS, class Epi, bool ALLOW_PP = true>
struct RowLds {
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    static constexpr int ZLEN = row_line_len(L, PADDED, Cf::E);
    static constexpr int NT = PAIRS * Cf::TPF;
    static constexpr bool PP = ALLOW_PP && row_pingpong(PAIRS * ZLEN * sizeof(cplx<R>), NT, L / (2 * PAIRS));
    static constexpr int SLOTS = (PP ? 2 : 1) * PAIRS * ZLEN;
    static constexpr int RED = (Epi::NQ > 0 ? Epi::NQ : 1) * (NT >= 64 ? NT / 64 : NT);
};

// One row-pass block: row pairs vb * PAIRS .. of the launch's spectra
// (channel already applied), LDS from the caller (RowLds slots and
// reduction scratch).  Partial sums go to partials[pblock * NQ ..].
// ALLOW_PP = false keeps one LDS line per pair (two barriers per stage).
template <typename R, int L, bool PADDED, int EMAX, int PAIRS, int T, bool INV_IN, bool FWD_OUT, class Epi,
          bool ALLOW_PP = true>
__device__ __forceinline__ void row_body(const RowArgs<R>& a, Epi& epi, int vb, int pblock, cplx<R>* lds,
                                         double* red, int tid_in) {
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    using C = cplx<R>;
    constexpr int E = Cf::E, TPF = Cf::TPF, NH = Cf::NH, PT = Cf::PT, HALF = Cf::HALF;
    // one pair's LDS: the staged Hermitian line (padded_len(PT) slots) and,
    // over the same memory, the NH half transforms (HLEN slots each)
    constexpr int HLEN = fft_lds_len(L, E, 1);
    constexpr int ZLEN = row_line_len(L, PADDED, E);
    constexpr int NT = PAIRS * TPF;
    constexpr int NQ = Epi::NQ;
    constexpr bool PP = RowLds<R, L, PADDED, EMAX, PAIRS, Epi, ALLOW_PP>::PP;

    const int tid = tid_in;
    const int pair = tid / TPF;
    const int t = tid - pair * TPF;
    const int row0 = vb * (2 * PAIRS);
    const int ra = row0 + 2 * pair;
    const LdsView<1, C> zv{lds + pair * ZLEN, 0};
    LdsView<1, C> hv[NH], hw[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        hv[h] = LdsView<1, C>{lds + pair * ZLEN + h * HLEN, 0};
        hw[h] = LdsView<1, C>{lds + (PP ? PAIRS * ZLEN : 0) + pair * ZLEN + h * HLEN, 0};
    }

    C v[NH][E];
    C z[E];
    const R zero = 0;
    // Image values the epilogue reads, loaded up front (after the spectrum
    // columns) so that their latency hides behind the inverse transform.
    constexpr int NPRE = Epi::NPRE > 0 ? Epi::NPRE : 1;
    typename Epi::Pre pre[E][NPRE];
    auto prefetch = [&]() {
        if constexpr (Epi::NPRE > 0) {
#pragma unroll
            for (int m = 0; m < E; ++m) epi.load(ra, t + m * TPF, pre[m]);
        }
    };

    // An epilogue that reads an image late (the update's beta_{k-2}) gets
    // the pair's two rows copied straight into the pair's LDS line while
    // the inverse transform's last stage computes (the LDS is idle then),
    // instead of a global load that stalls the epilogue.
    // The rows are of the epilogue's prefetch type (float64 iterates take
    // twice the bytes: they fit the line of a zero-padded pair, 2L complex).
    using P = typename Epi::Pre;
    constexpr bool LATE = INV_IN && MSR_LATE_LDS && Epi::LATE_ROWS && !PP && TPF % 64 == 0 &&
                          (2 * L) % ((TPF / 64) * 64 * (16 / (int)sizeof(P))) == 0 &&
                          2 * L * (int)sizeof(P) <= ZLEN * (int)sizeof(C);
    lds_ptr<const P> late = nullptr;

    if constexpr (INV_IN) {
        // Half-plane columns of both rows -> full Hermitian-combined line Z in
        // LDS.  Item q covers column kx of one pair (kx % T fastest, then the
        // pair, then the tile); all loads of a thread are issued before any
        // LDS write so their latencies overlap.
        constexpr int NITEMS = ((HALF + T) / T) * T * PAIRS;
        constexpr int IPT = (NITEMS + NT - 1) / NT;
        C xa[IPT], xb[IPT];
        const RowItems<T, PAIRS, NT> items(tid, row0, a.NR);
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            int q, p, kx;
            uint32_t ia;
            items.get(u, q, p, kx, ia);
            xa[u] = mk<C>(zero, zero);
            xb[u] = xa[u];
            if (q < NITEMS && kx < a.K_in) {
                xa[u] = el(a.spec_in, ia);
                xb[u] = el(a.spec_in, ia + T);
            }
        }
        if (a.K_in2 > 0) {
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                int q, p, kx;
                uint32_t ia;
                items.get(u, q, p, kx, ia);
                if (q < NITEMS && kx < a.K_in2) {
                    xa[u] = cadd(xa[u], el(a.spec_in2, ia));
                    xb[u] = cadd(xb[u], el(a.spec_in2, ia + T));
                }
            }
        }
        prefetch();
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            int q, p, kx;
            uint32_t ia;
            items.get(u, q, p, kx, ia);
            if (q < NITEMS && kx <= HALF) {
                const LdsView<1, C> zp{lds + p * ZLEN, 0};
                zp[kx] = mk<C>(xa[u].x - xb[u].y, xa[u].y + xb[u].x);  // Xa + i Xb
                if (kx > 0 && kx < HALF) zp[PT - kx] = mk<C>(xa[u].x + xb[u].y, xb[u].x - xa[u].y);  // conj Xa + i conj Xb
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int h = 0; h < NH; ++h) v[h][m] = zv[NH * (t + m * TPF) + h];
        __syncthreads();
        // The update epilogue keeps beta_{k-1} in registers across the inverse
        // transform within a four-wave budget: its inverse loads the twiddles
        // stage by stage.
        constexpr bool PRE_INV = MSR_TW_PRELOAD_INV || Epi::MIN_WAVES == 1;
        if constexpr (LATE) {
            P* line = reinterpret_cast<P*>(lds + pair * ZLEN);
            const P* src = epi.late_src(ra);
            auto hook = [&]() { load_to_lds<P, 2 * L, TPF / 64>(src, line, t); };
            fft<L, E, true, Cf::TWS, NH, 1, PRE_INV>(v, hv, t, a.tws, hook);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            late = (lds_ptr<const P>)line;
        } else if constexpr (PP) {
            fft_pp<L, E, true, Cf::TWS, NH, 1, PRE_INV>(v, hv, hw, t, a.tws);
        } else {
            fft<L, E, true, Cf::TWS, NH, 1, PRE_INV>(v, hv, t, a.tws);
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            C s = v[0][m];
            if constexpr (PADDED) s = cadd(s, cmulc(v[1][m], el(a.tw, t + m * TPF)));
            z[m] = s;
        }
    } else {
        prefetch();
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = mk<C>(zero, zero);
    }

    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) acc[q] = 0.0;
    if constexpr (LATE) {
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = epi.apply_late(ra, t + m * TPF, z[m], acc, pre[m], late);
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) z[m] = epi.apply(ra, t + m * TPF, z[m], acc, pre[m]);
    }

    if constexpr (FWD_OUT) {
        // The forward transform reads the same twiddles, and computes the same
        // LDS and global addresses, as the inverse one.  Through opaque copies
        // of the table pointers and thread indices it loads and computes them
        // again instead of keeping the inverse's values live in registers
        // across the epilogue (MSR_REFETCH = 0: keep them).
        const C* tw_f = a.tw;
        const C* tws_f = a.tws;
        int tf = t, tidf = tid;
#if MSR_REFETCH
        if constexpr (INV_IN) {
            asm volatile("" : "+s"(tw_f), "+s"(tws_f));
            asm volatile("" : "+v"(tf), "+v"(tidf));
        }
#endif
#pragma unroll
        for (int m = 0; m < E; ++m) {
            v[0][m] = z[m];
            if constexpr (PADDED) v[1][m] = cmul(z[m], el(tw_f, tf + m * TPF));
        }
        __syncthreads();
        if constexpr (PP) fft_pp<L, E, false, Cf::TWS, NH, 1>(v, hv, hw, tf, tws_f);
        else fft<L, E, false, Cf::TWS, NH, 1>(v, hv, tf, tws_f);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m)
#pragma unroll
            for (int h = 0; h < NH; ++h) zv[NH * (tf + m * TPF) + h] = v[h][m];
        __syncthreads();
        // Split the packed spectra and store columns [0, K_out) of both rows
        // (tile tail zero-filled); unrolled over a compile-time item bound.
        const int ntile = (a.K_out + T - 1) / T;
        const int nitems = ntile * T * PAIRS;
        constexpr int OMAX = ((HALF + T) / T) * T * PAIRS;
        constexpr int OPT = (OMAX + NT - 1) / NT;
        const R half = (R)0.5;
        const RowItems<T, PAIRS, NT> oitems(tidf, row0, a.NR);
#pragma unroll
        for (int u = 0; u < OPT; ++u) {
            int q, p, kx;
            uint32_t ia;
            oitems.get(u, q, p, kx, ia);
            if (q < nitems) {
                C xa = mk<C>(zero, zero), xb = xa;
                if (kx < a.K_out) {
                    const LdsView<1, C> zp{lds + p * ZLEN, 0};
                    const C zk = zp[kx];
                    const C zm = zp[kx == 0 ? 0 : PT - kx];
                    xa = mk<C>(half * (zk.x + zm.x), half * (zk.y - zm.y));
                    xb = mk<C>(half * (zk.y + zm.y), -half * (zk.x - zm.x));
                }
                el(a.spec_out, ia) = xa;
                el(a.spec_out, ia + T) = xb;
            }
        }
    }

    if constexpr (NQ > 0) {
        if (a.reduce) {
            double tot[NQ];
            block_sum<NQ, NT>(acc, red, tot);
            if (tid == 0)
#pragma unroll
                for (int q = 0; q < NQ; ++q) el(a.partials, pblock * NQ + q) = tot[q];
        }
    }
}

template <typename R, int L, bool PADDED, int EMAX, int PAIRS, int T, bool INV_IN, bool FWD_OUT, class Epi>
__global__ void __launch_bounds__((PAIRS * LineCfg<L, PADDED, R, EMAX>::TPF))
MSR_ROW_WAVES_ATTR(EMAX, R, Epi)
row_kernel(RowArgs<R> a0, Epi epi0) {
    using RL = RowLds<R, L, PADDED, EMAX, PAIRS, Epi>;
    __shared__ cplx<R> lds[RL::SLOTS];
    __shared__ double red[RL::RED];
    RowArgs<R> a = a0;
    Epi epi = epi0;
    if (a.cstride) {
        const long long off = (long long)blockIdx.y * a.cstride;
        a.to_channel(off);
        epi.to_channel(off);
    }
    if (a.chan) epi.use(a.chan[blockIdx.y]);
    row_body<R, L, PADDED, EMAX, PAIRS, T, INV_IN, FWD_OUT, Epi>(a, epi, xcd_block(blockIdx.x, gridDim.x), blockIdx.x,
                                                                 lds, red, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Row epilogues.  apply(row, i, z, acc, pre) gets the cropped inverse result
// of rows (row, row+1) at column i packed as z = (x_row, x_row+1) and returns
// the pair to transform forward (or anything, when nothing follows).  `pre`
// holds the NPRE values load(row, i, pre) fetched for that element at the
// start of the kernel.
// ---------------------------------------------------------------------------

// Load an image (times a scale): the forward pass of a plain row transform.
template <typename R>
struct EpiLoad {
    static constexpr int NQ = 0, NPRE = 0, MIN_WAVES = 1;
    static constexpr bool LATE_ROWS = false;
    using Pre = R;  // type of the prefetched image values
    const R* __restrict__ img;
    int ld;
    R scale;
    __device__ __forceinline__ void to_channel(long long off) { img = shifted(img, off); }
    __device__ __forceinline__ void use(const ChanScalars<R>&) {}
    __device__ __forceinline__ void load(int, int, R*) const {}
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R>, double*, const R*) const {
        const uint32_t ia = (uint32_t)r * ld + i;
        return mk<cplx<R>>(scale * el(img, ia), scale * el(img, ia + ld));
    }
};

// Load a P x P PSF with ifftshift (row and column rolled by P/2).
template <typename R>
struct EpiLoadShift {
    static constexpr int NQ = 0, NPRE = 0, MIN_WAVES = 1;
    static constexpr bool LATE_ROWS = false;
    using Pre = R;  // type of the prefetched image values
    const R* __restrict__ img;
    int P;
    __device__ __forceinline__ void to_channel(long long off) { img = shifted(img, off); }
    __device__ __forceinline__ void use(const ChanScalars<R>&) {}
    __device__ __forceinline__ void load(int, int, R*) const {}
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R>, double*, const R*) const {
        const int h = P / 2;
        const int c = (i + h) & (P - 1);
        return mk<cplx<R>>(el(img, (uint32_t)((r + h) & (P - 1)) * P + c),
                           el(img, (uint32_t)((r + 1 + h) & (P - 1)) * P + c));
    }
};

// Store the cropped inverse (times a scale) as an image.
template <typename R>
struct EpiStore {
    static constexpr int NQ = 0, NPRE = 0, MIN_WAVES = 1;
    static constexpr bool LATE_ROWS = false;
    using Pre = R;  // type of the prefetched image values
    R* __restrict__ out;
    int ld;
    R scale;
    __device__ __forceinline__ void to_channel(long long off) { out = shifted(out, off); }
    __device__ __forceinline__ void use(const ChanScalars<R>&) {}
    __device__ __forceinline__ void load(int, int, R*) const {}
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R> z, double*, const R*) const {
        const uint32_t ia = (uint32_t)r * ld + i;
        el(out, ia) = scale * z.x;
        el(out, ia + ld) = scale * z.y;
        return z;
    }
};

// r = H x - y (y may be null): accumulates ||r||^2, optionally stores r, forwards r.
template <typename R>
struct EpiResid {
    static constexpr int NQ = 1, NPRE = 2, MIN_WAVES = 1;
    static constexpr bool LATE_ROWS = false;
    using Pre = R;  // type of the prefetched image values
    const R* __restrict__ y;
    R* __restrict__ r_out;
    int ld;
    __device__ __forceinline__ void to_channel(long long off) {
        y = shifted(y, off);
        r_out = shifted(r_out, off);
    }
    __device__ __forceinline__ void use(const ChanScalars<R>&) {}
    __device__ __forceinline__ void load(int r, int i, R* p) const {
        if (y) {
            const uint32_t ia = (uint32_t)r * ld + i;
            p[0] = el(y, ia);
            p[1] = el(y, ia + ld);
        }
    }
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R> z, double* acc, const R* p) const {
        const uint32_t ia = (uint32_t)r * ld + i;
        if (y) {
            z.x -= p[0];
            z.y -= p[1];
        }
        acc[0] += (double)z.x * z.x + (double)z.y * z.y;
        if (r_out) {
            el(r_out, ia) = z.x;
            el(r_out, ia + ld) = z.y;
        }
        return z;
    }
};

// The FISTA update (Algorithm 1) on gradient half-values s = grad/2:
//   alpha_{k-1} = b1 + t_prev (b1 - b2)        (b1 = beta_{k-1}, b2 = beta_{k-2})
//   beta_k      = prox(alpha_{k-1} - mu * 2 s)  (soft threshold at mu*lambda, or its positive part)
//   alpha_k     = beta_k + t_cur (beta_k - b1)
// beta_k overwrites b2 (same element, same thread); alpha_k is forwarded.
// I is the type of the stored iterates and of this arithmetic: R, or double
// with R = float (FP32 transforms, FP64 iterates: the iterate is not rounded
// to float between iterations).
template <typename R, typename I = R>
struct EpiUpdate {
    // float64 iterates double the prefetched registers: a lower wave target
    static constexpr int NQ = 1, NPRE = 2, MIN_WAVES = std::is_same<R, I>::value ? 4 : 2;
    // beta_{k-2} of the pair's rows via LDS (row_kernel, where they fit)
    static constexpr bool LATE_ROWS = true;
    using Pre = I;
    const I* __restrict__ b1;
    I* __restrict__ b2;  // in: beta_{k-2}; out: beta_k
    int ld;
    // rows (r, r + 1) of beta_{k-2}, which the row kernel copies to LDS
    __device__ __forceinline__ const I* late_src(int r) const { return b2 + (size_t)r * ld; }
    I two_mu;     // 2 mu
    I thr;        // mu * lambda
    I t_prev, t_cur;
    int positivity;
    __device__ __forceinline__ void to_channel(long long off) {
        b1 = shifted(b1, off);
        b2 = shifted(b2, off);
    }
    __device__ __forceinline__ void use(const ChanScalars<R>& c) {
        two_mu = c.two_mu;
        thr = c.thr;
    }
    __device__ __forceinline__ I upd(R s, I p1, I& p2) const {
        const I alpha = fmaR(t_prev, p1 - p2, p1);
        const I zz = fmaR(-two_mu, (I)s, alpha);
        I beta;
        const I zero = 0;
        if (positivity) beta = fmax(zz - thr, zero);
        else beta = copysign(fmax(fabs(zz) - thr, zero), zz);
        p2 = beta;
        return fmaR(t_cur, beta - p1, beta);
    }
    // beta_{k-1} of both rows is prefetched; beta_{k-2} too would not fit the
    // register budget
    __device__ __forceinline__ void load(int r, int i, I* p) const {
        const uint32_t ia = (uint32_t)r * ld + i;
        p[0] = el(b1, ia);
        p[1] = el(b1, ia + ld);
    }
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R> z, double* acc, const I* p) const {
        const uint32_t ia = (uint32_t)r * ld + i;
        return update(ia, z, acc, p, el(b2, ia), el(b2, ia + ld));
    }
    // The same with beta_{k-2} of rows (r, r + 1) in LDS (late, ld apart).
    __device__ __forceinline__ cplx<R> apply_late(int r, int i, cplx<R> z, double* acc, const I* p,
                                                  lds_ptr<const I> late) const {
        return update((uint32_t)r * ld + i, z, acc, p, late[i], late[ld + i]);
    }
    __device__ __forceinline__ cplx<R> update(uint32_t ia, cplx<R> z, double* acc, const I* p, I pa, I pb) const {
        const uint32_t ib = ia + ld;
        const I qa = upd(z.x, p[0], pa);
        const I qb = upd(z.y, p[1], pb);
        el(b2, ia) = pa;
        el(b2, ib) = pb;
        acc[0] += (double)fabs(pa) + (double)fabs(pb);
        return mk<cplx<R>>((R)qa, (R)qb);
    }
};

// Power iteration: w = A v.  Accumulates <w, w> and <w, vprev>, stores w.
template <typename R>
struct EpiPower {
    static constexpr int NQ = 2, NPRE = 0, MIN_WAVES = 1;
    static constexpr bool LATE_ROWS = false;
    using Pre = R;  // type of the prefetched image values
    const R* __restrict__ vprev;
    R* __restrict__ w_out;
    int ld;
    R vscale;  // v = vscale * vprev
    __device__ __forceinline__ void to_channel(long long off) {
        vprev = shifted(vprev, off);
        w_out = shifted(w_out, off);
    }
    __device__ __forceinline__ void use(const ChanScalars<R>&) {}
    __device__ __forceinline__ void load(int, int, R*) const {}
    __device__ __forceinline__ cplx<R> apply(int r, int i, cplx<R> z, double* acc, const R*) const {
        const uint32_t ia = (uint32_t)r * ld + i, ib = ia + ld;
        acc[0] += (double)z.x * z.x + (double)z.y * z.y;
        acc[1] += (double)z.x * (double)(vscale * el(vprev, ia)) + (double)z.y * (double)(vscale * el(vprev, ib));
        el(w_out, ia) = z.x;
        el(w_out, ib) = z.y;
        return z;
    }
};

// ===========================================================================
// Column pass: DFT along y of each stored column, pointwise multiply, inverse,
// crop.  One block handles T adjacent columns (one tile).
// ===========================================================================
template <typename R>
struct ColArgs {
    using C = cplx<R>;
    const C* __restrict__ spec_in;
    const C* __restrict__ spec_in2;  // subtracted from spec_in before the transform (or null)
    C* __restrict__ spec_out;
    const C* __restrict__ tw;
    const C* __restrict__ tws;  // FFT stage twiddle tables of length L
    double* __restrict__ partials;
    int NR;      // rows of the spectra (L)
    int K;       // columns processed: tiles 0 .. ceil(K/T)-1; columns >= K read as zero
    int reduce;  // accumulate the mode's FP64 sums
    R in_scale;  // the transformed column is in_scale * spec_in - spec_in2
    int nch;                                    // channels of a batched launch (grid y); 0 or 1: one
    int chan_scale;                             // batched: in_scale = chan[c].inv_sigma2
    long long cstride;                          // batched: bytes between two channels' workspaces
    const ChanScalars<R>* __restrict__ chan;    // batched: per-channel scalars (or null)
    const FilterCoef<R>* __restrict__ chanf;    // batched: per-channel filters (or null)
    __device__ __forceinline__ void to_channel(long long off) {
        spec_in = shifted(spec_in, off);
        spec_in2 = shifted(spec_in2, off);
        spec_out = shifted(spec_out, off);
        tw = shifted(tw, off);
        tws = shifted(tws, off);
        partials = shifted(partials, off);
    }
};

// Moves a column launch's arguments to channel blockIdx.y of a batched launch.
template <typename R, class Mode>
__device__ __forceinline__ void col_channel(ColArgs<R>& a, Mode& md) {
    if (a.cstride) {
        const long long off = (long long)blockIdx.y * a.cstride;
        a.to_channel(off);
        md.to_channel(off);
    }
    if (a.chan && a.chan_scale) a.in_scale = a.chan[blockIdx.y].inv_sigma2;
    if (a.chanf) md.use(a.chanf[blockIdx.y]);
}

// A block transforms CB adjacent columns (CB divides the tile width T): logical
// block b covers columns b*CB .. b*CB + CB - 1 of tile (b*CB)/T.
template <typename R, int L, bool PADDED, int EMAX, int T, int CB, class Mode>
__device__ __forceinline__ void col_body(const ColArgs<R>& a, const Mode& md, int lblock, int pblock,
                                         cplx<R>* lds, double* red, int tid_in) {
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    using C = cplx<R>;
    constexpr int E = Cf::E, TPF = Cf::TPF, NH = Cf::NH;
    constexpr int NT = CB * TPF;
    constexpr int NQ = Mode::NQ;
    constexpr int HL = fft_lds_len(L, E, CB);
    static_assert(T % CB == 0, "CB must divide T");

    const int tid = tid_in;
    const int cl = tid % CB;
    const int t = tid / CB;
    const int kx = lblock * CB + cl;
    const int tile = kx / T;
    const int c = kx % T;
    const bool live = kx < a.K;
    const bool red_on = a.reduce != 0;
    const R zero = 0;
    LdsView<CB, C> hv[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hv[h] = LdsView<CB, C>{lds + h * CB * HL, cl};

    C v[NH][E];
    const uint32_t base = (uint32_t)tile * a.NR * T + c;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = t + m * TPF;
        C y = mk<C>(zero, zero);
        if (live) {
            y = cscale(el(a.spec_in, base + (uint32_t)i * T), a.in_scale);
            if (a.spec_in2) y = csub(y, el(a.spec_in2, base + (uint32_t)i * T));
        }
        v[0][m] = y;
        if constexpr (PADDED) v[1][m] = cmul(y, el(a.tw, i));
    }
    fft<L, E, false, Cf::TWS, NH, CB>(v, hv, t, a.tws);

    double acc[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) acc[q] = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int ky = NH * (t + m * TPF) + h;
            const C r = md.apply(tile, c, kx, ky, live && red_on, v[h][m], acc);
            v[h][m] = live ? r : mk<C>(zero, zero);
        }

    if constexpr (Mode::INVERSE) {
        // As in the row passes: opaque copies make the inverse transform load
        // its twiddles and compute its addresses again rather than keep the
        // forward transform's live across the pointwise step.
        const C* tw_i = a.tw;
        const C* tws_i = a.tws;
        int ti = t;
        uint32_t base_i = base;
#if MSR_REFETCH
        asm volatile("" : "+s"(tw_i), "+s"(tws_i));
        asm volatile("" : "+v"(ti), "+v"(base_i));
#endif
        __syncthreads();
        fft<L, E, true, Cf::TWS, NH, CB>(v, hv, ti, tws_i);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = ti + m * TPF;
            C s = v[0][m];
            if constexpr (PADDED) s = cadd(s, cmulc(v[1][m], el(tw_i, i)));
            el(a.spec_out, base_i + (uint32_t)i * T) = s;
        }
    } else if constexpr (Mode::STORE_SPECTRUM) {
        // unpadded forward transform only: bin ky = t + m*TPF
#pragma unroll
        for (int m = 0; m < E; ++m) el(a.spec_out, base + (uint32_t)(t + m * TPF) * T) = v[0][m];
    }

    if constexpr (NQ > 0) {
        if (red_on) {
            double tot[NQ];
            block_sum<NQ, NT>(acc, red, tot);
            if (tid == 0)
#pragma unroll
                for (int q = 0; q < NQ; ++q) el(a.partials, (uint32_t)pblock * NQ + q) = tot[q];
        }
    }
}

template <typename R, int L, bool PADDED, int EMAX, int T, int CB, class Mode>
__global__ void __launch_bounds__((CB * LineCfg<L, PADDED, R, EMAX>::TPF))
MSR_WAVES_ATTR(EMAX, R)
col_kernel(ColArgs<R> a0, Mode m0) {
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    constexpr int NT = CB * Cf::TPF;
    constexpr int NQ = Mode::NQ;
    __shared__ cplx<R> lds[Cf::NH * CB * fft_lds_len(L, Cf::E, CB)];
    __shared__ double red[(NQ > 0 ? NQ : 1) * (NT >= 64 ? NT / 64 : NT)];
    ColArgs<R> a = a0;
    Mode md = m0;
    col_channel(a, md);
    col_body<R, L, PADDED, EMAX, T, CB, Mode>(a, md, xcd_block(blockIdx.x, gridDim.x), blockIdx.x, lds, red,
                                              threadIdx.x);
}

// Two independent column passes in one launch: blocks [0, g1) run (a1, m1),
// the rest run (a2, m2).  Used for the two narrow low-band passes of step 2.
// Partial sums, if any, land at the launch-wide block index.
template <typename R, int L, bool PADDED, int EMAX, int T, int CB, class M1, class M2>
__global__ void __launch_bounds__((CB * LineCfg<L, PADDED, R, EMAX>::TPF))
MSR_WAVES_ATTR(EMAX, R)
col_dual_kernel(ColArgs<R> a1, M1 m1, int g1, ColArgs<R> a2, M2 m2) {
    col_channel(a1, m1);
    col_channel(a2, m2);
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    constexpr int NT = CB * Cf::TPF;
    constexpr int NQ = M1::NQ > M2::NQ ? M1::NQ : M2::NQ;
    __shared__ cplx<R> lds[Cf::NH * CB * fft_lds_len(L, Cf::E, CB)];
    __shared__ double red[(NQ > 0 ? NQ : 1) * (NT >= 64 ? NT / 64 : NT)];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b < g1) col_body<R, L, PADDED, EMAX, T, CB, M1>(a1, m1, b, b, lds, red, threadIdx.x);
    else col_body<R, L, PADDED, EMAX, T, CB, M2>(a2, m2, b - g1, b, lds, red, threadIdx.x);
}

// Multiply by the cached PSF spectrum (already scaled by 1/P^2), tiled like
// the spectra with P rows: hh[((kx/T) * P + ky) * T + kx%T].
template <typename R>
struct ModePsf {
    static constexpr int NQ = 0;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    const R* __restrict__ hh;
    int P;
    int T;
    __device__ __forceinline__ void to_channel(long long off) { hh = shifted(hh, off); }
    __device__ __forceinline__ void use(const FilterCoef<R>&) {}
    __device__ __forceinline__ cplx<R> apply(int tile, int c, int, int ky, bool, cplx<R> y, double*) const {
        return cscale(y, el(hh, ((uint32_t)tile * P + ky) * T + c));
    }
};

__device__ __forceinline__ float sqrtR(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrtR(double x) { return sqrt(x); }

// sin(x) for |x| <= pi/2.  Single precision: the Taylor series through x^11
// (truncation below 6e-8 on that interval, about one ulp); double precision:
// the library sine.
__device__ __forceinline__ float sin_half_pi(float x) {
    const float x2 = x * x;
    float p = -2.5052108385441720e-08f;          // -1/11!
    p = fmaf(p, x2, 2.7557319223985893e-06f);    //  1/9!
    p = fmaf(p, x2, -1.9841269841269841e-04f);   // -1/7!
    p = fmaf(p, x2, 8.3333333333333333e-03f);    //  1/5!
    p = fmaf(p, x2, -1.6666666666666667e-01f);   // -1/3!
    return fmaf(p * x2, x, x);
}
__device__ __forceinline__ double sin_half_pi(double x) { return sin(x); }

// Filter responses of Eqs. 6-10 (squared), evaluated per DFT cell.  The flat
// regions are decided on the integer squared radius r2 = kx^2 + ky^2:
// r > ell + delta  <=>  r2 > hi_r2 = floor((ell + delta)^2), and
// r < ell - delta  <=>  r2 < lo_r2 = ceil((ell - delta)^2) (0 when ell < delta).
template <typename R>
struct FilterCoef {
    R ell, delta, inv_sigma2, inv_eta2, sigma2, eta2, half_pi_over_delta;
    int hi_r2, lo_r2;  // clamped to [0, 2^31 - 1]; r2 <= P^2 / 2 < 2^31 for P <= 16384
    int P;
    // returns (gL^2, gH^2)
    __device__ __forceinline__ cplx<R> sq(int kx, int ky) const {
        const int sy = ky < P / 2 ? ky : ky - P;
        const int sx = kx < P / 2 ? kx : kx - P;  // kx <= P/2 in the half plane
        const int r2 = sx * sx + sy * sy;
        const R zero = 0, one = 1;
        if (r2 > hi_r2) return mk<cplx<R>>(zero, inv_sigma2);
        if (r2 < lo_r2) return mk<cplx<R>>(inv_eta2, zero);
        const R r = sqrtR((R)r2);
        const R s = sin_half_pi(half_pi_over_delta * (r - ell));
        const R lo = (one - s) * (one - s), hi = (one + s) * (one + s);
        const R a2 = one / (sigma2 * hi + eta2 * lo);
        return mk<cplx<R>>(a2 * lo, a2 * hi);
    }
};

__device__ __forceinline__ double col_weight(int kx, int P) { return (kx == 0 || kx == P / 2) ? 1.0 : 2.0; }

// Multiply by w / P^2 with w = 1/sigma^2 - g_H^2, which vanishes for
// r > ell + delta, so only the columns k_x <= ell + delta are processed.
// Accumulates sum w_kx w |Y|^2 over the half plane.  Because
// g_H^2 = 1/sigma^2 - w everywhere, E^T C_{g_H^2} E r = r / sigma^2 - E^T C_w E r
// and ||G_H r||^2 = ||r||^2 / sigma^2 - (1/P^2) sum w |Y|^2.
template <typename R>
struct ModeFilterW {
    static constexpr int NQ = 1;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    FilterCoef<R> f;
    R inv_p2;
    __device__ __forceinline__ void to_channel(long long) {}
    __device__ __forceinline__ void use(const FilterCoef<R>& c) { f = c; }
    __device__ __forceinline__ cplx<R> apply(int, int, int kx, int ky, bool acc_on, cplx<R> y, double* acc) const {
        const R g = f.inv_sigma2 - f.sq(kx, ky).y;
        if (acc_on) acc[0] += col_weight(kx, f.P) * (double)g * ((double)y.x * y.x + (double)y.y * y.y);
        return cscale(y, g * inv_p2);
    }
};

// Multiply by g_L^2 / P^2 (input: spectrum of alpha minus spectrum of l);
// accumulates sum w_kx g_L^2 |Y|^2 (= P^2 ||G_L (l - alpha)||^2).
template <typename R>
struct ModeFilterL {
    static constexpr int NQ = 1;
    static constexpr bool INVERSE = true;
    static constexpr bool STORE_SPECTRUM = false;
    FilterCoef<R> f;
    R inv_p2;
    __device__ __forceinline__ void to_channel(long long) {}
    __device__ __forceinline__ void use(const FilterCoef<R>& c) { f = c; }
    __device__ __forceinline__ cplx<R> apply(int, int, int kx, int ky, bool acc_on, cplx<R> y, double* acc) const {
        const R g = f.sq(kx, ky).x;
        if (acc_on) acc[0] += col_weight(kx, f.P) * (double)g * ((double)y.x * y.x + (double)y.y * y.y);
        return cscale(y, g * inv_p2);
    }
};

// Forward transform only (PSF spectrum), bins stored in place.
template <typename R>
struct ModeForward {
    static constexpr int NQ = 0;
    static constexpr bool INVERSE = false;
    static constexpr bool STORE_SPECTRUM = true;
    __device__ __forceinline__ void to_channel(long long) {}
    __device__ __forceinline__ void use(const FilterCoef<R>&) {}
    __device__ __forceinline__ cplx<R> apply(int, int, int, int, bool, cplx<R> y, double*) const { return y; }
};

}  // namespace msr
