// persist_kernels.hpp -- the persistent kernel: the work-item loop over the
// passes described in persist.hpp, with each image size's blocking.
#pragma once
#include "ops.hpp"  // kernels and the tile widths of the spectra
#include "persist.hpp"

namespace msr {

template <typename R, int L>
struct PersistShape {
    static constexpr int EMAX = persist_emax(L), PAIRS = persist_pairs(L), CB = persist_cb(L);
    static constexpr int T = tile_width(L, (int)sizeof(cplx<R>));
    using Cf = LineCfg<L, true, R, EMAX>;
    static_assert(PAIRS * Cf::TPF == 256 && CB * Cf::TPF == 256, "256 threads per pass");
    static_assert(T % CB == 0, "column blocks within a tile");
    static constexpr int ROW_SLOTS = RowLds<R, L, true, EMAX, PAIRS, EpiUpdate<R>, false>::SLOTS;
    static constexpr int COL_SLOTS = Cf::NH * CB * fft_lds_len(L, Cf::E, CB);
    static constexpr int SLOTS = ROW_SLOTS > COL_SLOTS ? ROW_SLOTS : COL_SLOTS;
};

__device__ __forceinline__ double momentum_w(int k) { return k >= 1 ? (k - 1.0) / (k + 2.0) : 0.0; }

// A block-uniform copy of *src (read by every lane, kept from lane 0), so
// that the pass arguments sit in scalar registers as kernel arguments do.
template <typename T>
__device__ __forceinline__ T uniform_copy(const T* src) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T out;
    const int* s = reinterpret_cast<const int*>(src);
    int* o = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return out;
}

// Runs block b of pass d (iteration k) with the blocking of size L.
template <typename R, int L>
__device__ __forceinline__ void persist_pass(const PassDesc<R>* d, int kind, int g1, int k, int b, cplx<R>* lds,
                                             double* red, int tid) {
    using S = PersistShape<R, L>;
    if (kind == kPassColPsf) {
        const ColArgs<R> a = uniform_copy(&d->ca);
        const ModePsf<R> m = uniform_copy(&d->mp);
        col_body<R, L, true, S::EMAX, S::T, S::CB, ModePsf<R>>(a, m, b, b, lds, red, tid);
    } else if (kind == kPassRowResid) {
        const RowArgs<R> a = uniform_copy(&d->ra);
        EpiResid<R> e = uniform_copy(&d->er);
        row_body<R, L, true, S::EMAX, S::PAIRS, S::T, true, true, EpiResid<R>, false>(a, e, b, b, lds, red, tid);
    } else if (kind == kPassColFilt) {
        if (b < g1) {
            const ColArgs<R> a = uniform_copy(&d->ca);
            const ModeFilterW<R> m = uniform_copy(&d->mw);
            col_body<R, L, true, S::EMAX, S::T, S::CB, ModeFilterW<R>>(a, m, b, b, lds, red, tid);
        } else {
            const ColArgs<R> a = uniform_copy(&d->ca2);
            const ModeFilterL<R> m = uniform_copy(&d->ml);
            col_body<R, L, true, S::EMAX, S::T, S::CB, ModeFilterL<R>>(a, m, b - g1, b, lds, red, tid);
        }
    } else {
        const RowArgs<R> a = uniform_copy(&d->ra);
        EpiUpdate<R> e = uniform_copy(&d->eu);
        e.t_prev = (R)momentum_w(k - 1);
        e.t_cur = (R)momentum_w(k);
        row_body<R, L, true, S::EMAX, S::PAIRS, S::T, true, true, EpiUpdate<R>, false>(a, e, b, b, lds, red, tid);
    }
}

// Index of the segment holding item r of an iteration: the last s with
// seg[s] <= r (segments may be empty).
__device__ __forceinline__ int persist_segment(const int* seg, int nseg, int r) {
    int lo = 0, hi = nseg;  // seg[lo] <= r < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool persist_stop(const PersistCtl* ctl) {
    return __hip_atomic_load(&ctl->give_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
           __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// The persistent kernel for sizes persist_size(0 .. NS - 1).
template <typename R, int NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) persist_kernel(PersistArgs<R> pa) {
    constexpr int S0 = PersistShape<R, 512>::SLOTS, S1 = PersistShape<R, 1024>::SLOTS;
    constexpr int S2 = PersistShape<R, 2048>::SLOTS, S3 = NS > 3 ? PersistShape<R, 4096>::SLOTS : 0;
    constexpr int SA = S0 > S1 ? S0 : S1, SB = S2 > S3 ? S2 : S3;
    __shared__ cplx<R> lds[SA > SB ? SA : SB];
    __shared__ double red[2 * 4];
    __shared__ int item[5];  // k, p, c, b, go
    const int tid = threadIdx.x;
    // this block's XCD and its queue: the XCD's channels and segments
    const int x = (int)blockIdx.x % kPersistXcds;
    const int nx = pa.xn[x];
    if (nx == 0) return;
    const int* seg = pa.seg + x * (pa.npass * pa.C + 1);
    const int* xch = pa.xch + x * pa.C;
    const int nseg = pa.npass * nx;
    const unsigned int per = (unsigned int)seg[nseg];
    const unsigned int total = per * (unsigned int)pa.iters;
    for (;;) {
        if (tid == 0) {
            int go = 0;
            if (!persist_stop(pa.ctl)) {
                const unsigned int t = __hip_atomic_fetch_add(&pa.ctl->ticket[x], 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                if (t < total) {
                    const int k = pa.k0 + (int)(t / per) + 1;
                    const int r = (int)(t % per);
                    const int sg = persist_segment(seg, nseg, r);
                    const int p = sg / nx, c = xch[sg % nx];
                    // the pass before this one in channel c's chain
                    const int pp = p > 0 ? p - 1 : pa.npass - 1;
                    const int kk = p > 0 ? k - pa.k0 : k - pa.k0 - 1;  // its completed iterations needed
                    const unsigned int need =
                        (unsigned int)kk * (unsigned int)pa.desc[(c * pa.npass + pp) * 2].nblocks;
                    go = 1;
                    unsigned int polls = 0;
                    while (__hip_atomic_load(&pa.done[c * pa.npass + pp], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (persist_stop(pa.ctl)) {
                            go = 0;
                            break;
                        }
                        if (++polls > pa.spin_limit) {
                            __hip_atomic_store(&pa.ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            go = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    if (go) {
                        // the dependency's results are in this XCD's L2: drop
                        // whatever this CU's L1 holds of them from earlier
                        // iterations (every wave of the block reads after the
                        // barrier below)
                        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
                    }
                    item[0] = k;
                    item[1] = p;
                    item[2] = c;
                    item[3] = r - seg[sg];
                }
            }
            item[4] = go;
        }
        __syncthreads();
        if (!item[4]) return;
        // block-uniform, so the pass's arguments load into scalar registers
        const int k = __builtin_amdgcn_readfirstlane(item[0]), p = __builtin_amdgcn_readfirstlane(item[1]);
        const int c = __builtin_amdgcn_readfirstlane(item[2]), b = __builtin_amdgcn_readfirstlane(item[3]);
        // an opaque copy of the thread index per item: nothing a pass derives
        // from it can be hoisted out of the loop (it would stay live across
        // every pass body and exhaust the registers)
        int tidx = tid;
        asm volatile("" : "+v"(tidx));
        const PassDesc<R>* d = pa.desc + (c * pa.npass + p) * 2 + (k & 1);
        const int kind = __builtin_amdgcn_readfirstlane(d->kind);
        const int g1 = __builtin_amdgcn_readfirstlane(d->g1);
        switch (__builtin_amdgcn_readfirstlane(d->size_idx)) {
            case 0: persist_pass<R, 512>(d, kind, g1, k, b, lds, red, tidx); break;
            case 1: persist_pass<R, 1024>(d, kind, g1, k, b, lds, red, tidx); break;
            case 2: persist_pass<R, 2048>(d, kind, g1, k, b, lds, red, tidx); break;
            default:
                if constexpr (NS > 3) persist_pass<R, 4096>(d, kind, g1, k, b, lds, red, tidx);
                break;
        }
        // every wave's stores of this item have reached the L2 (the vector L1
        // writes through) before the item is counted done
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0)
            __hip_atomic_fetch_add(&pa.done[c * pa.npass + p], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Zeroes the tickets, abort flag and done counters before a launch (a kernel,
// not a memset, so that the launch can be captured in a graph and replayed).
__global__ void persist_reset(PersistCtl* ctl, unsigned int* done, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kPersistXcds) ctl->ticket[i] = 0;
    if (i == 0) ctl->abort = 0;
    if (i < n) done[i] = 0;
}

}  // namespace msr
