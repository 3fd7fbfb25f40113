// fft_engine.hpp -- register/LDS radix-16 Stockham FFT building blocks for gfx950.
//
// A length-L complex FFT is computed cooperatively by TPF = L/E threads, each
// holding E elements in registers (E = 16 or 8, chosen per kernel variant).
// Thread t holds element t + m*TPF in register m on entry and the output bin
// t + m*TPF on exit, so a forward transform followed by a pointwise multiply
// and an inverse transform needs no reordering: the inverse's first stage
// reads exactly the registers the forward's last stage wrote.  Stages are
// Stockham auto-sort passes of radix R = min(E, remaining length); between
// stages the data goes through LDS once (write, barrier, read, barrier).
// Stage twiddles come from per-stage tables computed in double precision on
// the host and rounded to the working precision (see stage_offset).
//
// Several independent arrays ("halves") can be transformed together so they
// share the barriers; each has its own LDS view.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace msr {

// Element i of the global-memory array p, addressed as p plus a 32-bit byte
// offset.  The cast to the global address space lets the compiler emit
// global (not flat) loads and stores even where p was moved by integer
// arithmetic (a channel of a batched launch): flat accesses would also count
// against the LDS wait counter and need a full 64-bit address per lane.
// Every array the kernels index is smaller than 4 GiB, so an access costs one
// 32-bit add on top of a uniform base.
template <typename T>
__device__ __forceinline__ T& el(T* p, uint32_t i) {
    using B = std::conditional_t<std::is_const_v<T>, const char, char>;
    auto* g = (__attribute__((address_space(1))) B*)p;
    return *(T*)(g + (uint32_t)(i * (uint32_t)sizeof(T)));
}

template <typename R>
struct cplx_of;
template <>
struct cplx_of<float> {
    using type = float2;
};
template <>
struct cplx_of<double> {
    using type = double2;
};
template <typename R>
using cplx = typename cplx_of<R>::type;

template <typename C>
using real_of = std::conditional_t<std::is_same_v<C, float2>, float, double>;

__device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }

template <typename C>
__device__ __forceinline__ C mk(real_of<C> x, real_of<C> y) {
    C r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C cscale(C a, real_of<C> s) { return mk<C>(a.x * s, a.y * s); }
// a * w
template <typename C>
__device__ __forceinline__ C cmul(C a, C w) {
    return mk<C>(fmaR(a.x, w.x, -(a.y * w.y)), fmaR(a.x, w.y, a.y * w.x));
}
// a * conj(w)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C w) {
    return mk<C>(fmaR(a.x, w.x, a.y * w.y), fmaR(a.y, w.x, -(a.x * w.y)));
}

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
template <bool INV, typename C>
__device__ __forceinline__ C rot16(C b, int e) {
    using R = real_of<C>;
    constexpr R C1 = (R)0.92387953251128675613;  // cos(pi/8)
    constexpr R S1 = (R)0.38268343236508977173;  // sin(pi/8)
    constexpr R H = (R)0.70710678118654752440;   // sqrt(1/2)
    if (e == 0) return b;
    if (e == 4) return INV ? mk<C>(-b.y, b.x) : mk<C>(b.y, -b.x);
    R c, s;
    switch (e) {
        case 1: c = C1; s = S1; break;
        case 2: c = H; s = H; break;
        case 3: c = S1; s = C1; break;
        case 5: c = -S1; s = C1; break;
        case 6: c = -H; s = H; break;
        default: c = -C1; s = S1; break;  // 7
    }
    // forward multiplies by (c, -s), inverse by (c, s)
    if (INV) return mk<C>(fmaR(b.x, c, -(b.y * s)), fmaR(b.x, s, b.y * c));
    return mk<C>(fmaR(b.x, c, b.y * s), fmaR(b.y, c, -(b.x * s)));
}

// In-register DFT of size RD (2, 4, 8 or 16), natural order in and out.
template <int RD, bool INV, typename C>
__device__ __forceinline__ void dft(C (&x)[RD]) {
    C y[RD];
#pragma unroll
    for (int i = 0; i < RD; ++i) y[i] = x[bit_reverse<RD>(i)];
#pragma unroll
    for (int len = 2; len <= RD; len <<= 1) {
#pragma unroll
        for (int i = 0; i < RD; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const C a = y[i + k];
                const C b = rot16<INV>(y[i + k + len / 2], k * (16 / len));
                y[i + k] = cadd(a, b);
                y[i + k + len / 2] = csub(a, b);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RD; ++i) x[i] = y[i];
}

// LDS view of one transform's data, S columns interleaved: slot q of column c
// is base[q * S + c].  Element p of a line goes to slot p + p/16 when the
// line is staged (operator[]: one pad slot every 16 elements), and to slot
// p + A (p >> SH) in the exchange after FFT stage NS, with (A, SH) chosen per
// stage (stage_pad) so that the stage's strided writes and the contiguous
// reads that follow hit distinct LDS banks.
template <int S, typename C>
struct LdsView {
    C* base;
    int c;
    __device__ __forceinline__ C& operator[](int p) const { return base[(p + (p >> 4)) * S + c]; }
    __device__ __forceinline__ C& slot(int q) const { return base[q * S + c]; }
};

__host__ __device__ constexpr int padded_len(int L) { return L + L / 16; }

// Padding of the exchange after stage NS (radix RD) of a transform whose LDS
// view interleaves S columns: element p at slot p + A (p >> SH).  The LDS has
// 32 banks of 4 bytes, so a 64-lane access of 8-byte elements is served 16
// lanes at a time, and 16 lanes must hit 16 distinct 8-byte bank pairs.
// Reads (element t + m TPF, consecutive over lanes) do so under each padding
// below.  The writes of stage NS put lane j at
//   (j / NS) NS RD + j % NS + r NS:
// for NS >= 16 the lanes of a 16-group stay consecutive (no pad needed); for
// NS = 1 they are RD apart and a stride of one extra slot per 16 (or per 8
// when two or four columns interleave) separates them; for NS = 8 (RD = 8)
// the two 8-lane groups are 64 apart and need 2 extra slots per 16; for
// NS = 4 (RD = 4) four groups 16 apart need 4 per 16.  Every (L, E, S) the
// library builds was checked against this bank model.
struct LdsPad {
    int A, SH;
};
__host__ __device__ constexpr LdsPad stage_pad(int NS, int RD, int S) {
    if (NS >= 16) return LdsPad{0, 4};
    if (NS == 1) {
        if (RD >= 16 || S == 1) return LdsPad{1, 4};
        if (S >= 4 && RD <= 4) return LdsPad{1, 2};
        return LdsPad{1, 3};
    }
    if (NS == 8) return S == 1 ? LdsPad{2, 4} : LdsPad{0, 4};
    if (NS == 4) return S == 1 ? LdsPad{4, 4} : (S == 2 ? LdsPad{2, 3} : LdsPad{0, 4});
    return LdsPad{1, 4};
}
template <int A, int SH>
__host__ __device__ constexpr int pad_slot(int p) {
    return p + A * (p >> SH);
}
__host__ __device__ constexpr int pad_slot_rt(int p, LdsPad q) { return p + q.A * (p >> q.SH); }

// Slots one transform's LDS view needs: the largest padded index over the
// exchanges of a length-L, E-per-thread transform with S interleaved
// columns, plus one (at least L).
__host__ __device__ constexpr int fft_lds_len(int L, int E, int S) {
    int n = L;
    for (int NS = 1; NS < L;) {
        const int RD = (L / NS) >= E ? E : (L / NS);
        if (NS * RD < L) {
            const int m = pad_slot_rt(L - 1, stage_pad(NS, RD, S)) + 1;
            if (m > n) n = m;
        }
        NS *= RD;
    }
    return n;
}

// Elements per thread for a transform of length L when at most EMAX are wanted.
__host__ __device__ constexpr int elems_per_thread(int L, int EMAX) { return L >= EMAX ? EMAX : L; }

// The register array of NH transforms held by one thread (E elements each).
template <int NH, int E, typename C>
using RegArr = C[NH][E];

// Stage twiddle tables.  Stage NS (> 1) of a length-L transform with E
// elements per thread has radix RD = min(E, L / NS); butterfly class
// jm < NS needs w^r, r < RD, w = exp(-2 pi i jm / (NS RD)).  Its table row
// holds w^1, w^2, w^4, w^8 (4 complex, aligned): the other powers are products
// of two of these.  Rows of consecutive jm are adjacent, so a wave's loads
// are contiguous.  The tables of E = 2, 4, 8, 16 (those not above L) for one
// length are stored back to back.
__host__ __device__ constexpr int stage_radix(int L, int E, int NS) { return (L / NS) >= E ? E : (L / NS); }
__host__ __device__ constexpr int stage_offset(int L, int E, int NSq) {
    int off = 0;
    for (int NS = 1; NS < L && NS < NSq; NS *= stage_radix(L, E, NS))
        if (NS > 1) off += 4 * NS;
    return off;
}
__host__ __device__ constexpr int stage_table_len(int L, int E) { return stage_offset(L, E, L); }
__host__ __device__ constexpr int stage_tables_offset(int L, int E) {
    int off = 0;
    for (int e = 2; e < E && e <= L; e *= 2) off += stage_table_len(L, e);
    return off;
}
__host__ __device__ constexpr int stage_tables_len(int L) { return stage_tables_offset(L, 32); }

__host__ __device__ constexpr int ilog2(int x) {
    int r = 0;
    while ((2 << r) <= x) ++r;
    return r;
}

// Twiddle rows a thread needs, in registers.  Stage NS (> 1) reads, for each
// of its NB = E / RD butterflies, the log2(RD) table entries w^1, w^2, w^4
// (and w^8); the entries of all stages are loaded at the start of a
// transform so their global-memory latency overlaps the first stage instead
// of stalling every stage after its barrier.  pre[] index of stage NS:
// tw_pre_offset(L, E, NS) + b log2(RD) + lg.
__host__ __device__ constexpr int tw_pre_offset(int L, int E, int NSq) {
    int off = 0;
    for (int NS = 1; NS < L && NS < NSq; NS *= stage_radix(L, E, NS))
        if (NS > 1) off += (E / stage_radix(L, E, NS)) * ilog2(stage_radix(L, E, NS));
    return off;
}
__host__ __device__ constexpr int tw_pre_count(int L, int E) {
    const int n = tw_pre_offset(L, E, L);
    return n > 0 ? n : 1;
}

template <int L, int E, int NS, typename C>
__device__ __forceinline__ void tw_preload_from(C* pre, int t, const C* __restrict__ tws) {
    constexpr int TPF = L / E;
    constexpr int RD = stage_radix(L, E, NS);
    if constexpr (NS > 1) {
        constexpr int NB = E / RD, LG = ilog2(RD), OFF = tw_pre_offset(L, E, NS);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int jm = (t + b * TPF) & (NS - 1);
            const C* row = &el(tws, (uint32_t)(stage_offset(L, E, NS) + 4 * jm));
#pragma unroll
            for (int lg = 0; lg < LG; ++lg) pre[OFF + b * LG + lg] = row[lg];
        }
    }
    if constexpr (NS * RD < L) tw_preload_from<L, E, NS * RD, C>(pre, t, tws);
}

// Loads the twiddle rows of every stage of a length-L transform (tw: the
// stage tables of length L, all E).
template <int L, int E, typename C>
__device__ __forceinline__ void tw_preload(C (&pre)[tw_pre_count(L, E)], int t, const C* __restrict__ tw) {
    tw_preload_from<L, E, 1, C>(pre, t, tw + stage_tables_offset(L, E));
}

// A callable run by every thread at the start of a transform's last stage,
// when every exchange through LDS is done (all threads are past the last
// barrier): the LDS views are free from there until the caller's next write.
struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// One Stockham stage on NH arrays at once.  Butterfly b of thread t owns the
// register slots b + r*NB (r < RD), so results go back into the same slots
// (last stage) or straight to LDS (other stages): no second register copy.
// With ping-pong buffers (PP) consecutive stages exchange through different
// LDS arrays, so one barrier per stage suffices (a stage's writes cannot
// overtake the previous stage's reads of the other array); otherwise one array
// and two barriers.  Twiddles come from the preloaded rows `pre` of the stage
// tables of this (L, E): w^r for power-of-two r directly, the others as
// products of two.
template <int L, int E, int NS, bool INV, int TWS, int NH, int S, int BUF, bool PP, bool PRE, typename C,
          class Hook>
__device__ __forceinline__ void fft_stage(RegArr<NH, E, C>& v, const LdsView<S, C> (&lds0)[NH],
                                          const LdsView<S, C> (&lds1)[NH], int t, const C* pre,
                                          const C* __restrict__ tws, const Hook& hook) {
    constexpr int TPF = L / E;
    constexpr int RD = (L / NS) >= E ? E : (L / NS);
    constexpr int NB = E / RD;
    constexpr bool LAST = (NS * RD == L);
    constexpr LdsPad PD = stage_pad(NS, RD, S);
    const LdsView<S, C>(&lds)[NH] = (PP && BUF) ? lds1 : lds0;
    if constexpr (LAST) hook();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * TPF;
        const int jm = j & (NS - 1);
        C w[RD];
        if constexpr (NS > 1) {
            constexpr int LG = ilog2(RD), OFF = tw_pre_offset(L, E, NS);
            const C* row = &el(tws, (uint32_t)(stage_offset(L, E, NS) + 4 * jm));
#pragma unroll
            for (int r = 1; r < RD; ++r) {
                const int lg = 31 - __builtin_clz(r);
                const int hb = 1 << lg;  // highest power of two in r
                if (hb == r) w[r] = PRE ? pre[OFF + b * LG + lg] : row[lg];
                else w[r] = cmul(w[hb], w[r - hb]);
            }
        }
        const int idxD = (j - jm) * RD + jm;
        // idxD and r NS occupy disjoint bits (j/NS scaled by NS RD, j % NS,
        // r NS), so the padded slot splits into a per-thread part and a
        // compile-time part that folds into the LDS instruction's offset.
        const int q0 = pad_slot<PD.A, PD.SH>(idxD);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            C x[RD];
#pragma unroll
            for (int r = 0; r < RD; ++r) x[r] = v[h][b + r * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < RD; ++r) x[r] = INV ? cmulc(x[r], w[r]) : cmul(x[r], w[r]);
            }
            dft<RD, INV>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < RD; ++r) v[h][b + r * NB] = x[r];
            } else {
#pragma unroll
                for (int r = 0; r < RD; ++r) lds[h].slot(q0 + pad_slot<PD.A, PD.SH>(r * NS)) = x[r];
            }
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
        // t < TPF and m TPF occupy disjoint bits: the same split as above
        const int t0 = pad_slot<PD.A, PD.SH>(t);
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int m = 0; m < E; ++m) v[h][m] = lds[h].slot(t0 + pad_slot<PD.A, PD.SH>(m * TPF));
        if constexpr (!PP) __syncthreads();
    }
}

template <int L, int E, int NS, bool INV, int TWS, int NH, int S, int BUF, bool PP, bool PRE, typename C,
          class Hook>
__device__ __forceinline__ void fft_from(RegArr<NH, E, C>& v, const LdsView<S, C> (&lds0)[NH],
                                         const LdsView<S, C> (&lds1)[NH], int t, const C* pre,
                                         const C* __restrict__ tws, const Hook& hook) {
    constexpr int RD = (L / NS) >= E ? E : (L / NS);
    fft_stage<L, E, NS, INV, TWS, NH, S, BUF, PP, PRE, C, Hook>(v, lds0, lds1, t, pre, tws, hook);
    if constexpr (NS * RD < L)
        fft_from<L, E, NS * RD, INV, TWS, NH, S, 1 - BUF, PP, PRE, C, Hook>(v, lds0, lds1, t, pre, tws, hook);
}

// Full transform of NH arrays (unnormalised; INV uses conjugate twiddles).
// tw: the stage tables of length L (all E, see stage_tables_offset).  With
// PRE the twiddle rows of all stages are loaded into registers first (their
// latency overlaps the first stage); without, each stage loads its rows after
// the previous barrier (fewer live registers, for kernels that hold other
// values across the transform).  The caller must have a barrier between any
// earlier use of the LDS views and this call, and one between this call and
// any later LDS write.
template <int L, int E, bool INV, int TWS, int NH, int S, bool PRE = true, typename C, class Hook = NoHook>
__device__ __forceinline__ void fft(RegArr<NH, E, C>& v, const LdsView<S, C> (&lds)[NH], int t,
                                    const C* __restrict__ tw, const Hook& hook = Hook{}) {
    const C* tws = tw + stage_tables_offset(L, E);
    C pre[tw_pre_count(L, E)];
    if constexpr (PRE) tw_preload<L, E, C>(pre, t, tw);
    fft_from<L, E, 1, INV, TWS, NH, S, 0, false, PRE, C, Hook>(v, lds, lds, t, pre, tws, hook);
}

// The same with two LDS arrays used alternately (one barrier per stage).
template <int L, int E, bool INV, int TWS, int NH, int S, bool PRE = true, typename C, class Hook = NoHook>
__device__ __forceinline__ void fft_pp(RegArr<NH, E, C>& v, const LdsView<S, C> (&lds0)[NH],
                                       const LdsView<S, C> (&lds1)[NH], int t, const C* __restrict__ tw,
                                       const Hook& hook = Hook{}) {
    const C* tws = tw + stage_tables_offset(L, E);
    C pre[tw_pre_count(L, E)];
    if constexpr (PRE) tw_preload<L, E, C>(pre, t, tw);
    fft_from<L, E, 1, INV, TWS, NH, S, 0, true, PRE, C, Hook>(v, lds0, lds1, t, pre, tws, hook);
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
// out[].  `scratch` must hold NQ * (NT >= 64 ? NT / 64 : NT) doubles.
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
