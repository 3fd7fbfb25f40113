// persist.hpp -- one persistent launch for the FISTA iterations of
// many channels (frequency channels of one observation, each its own
// two-step problem, Sect. 3.1) of uneven image sizes.
//
// Work items.  One iteration of a channel is its chain of passes (4 in step
// 1, 6 in step 2; the same passes the per-launch path runs), each pass a
// number of blocks.  An item is (iteration k, pass p, channel c, block b);
// items are numbered pass-major within an iteration (every channel's pass 0,
// then every channel's pass 1, ...), iterations one after another, and
// blocks of the persistent grid take them in that order from one ticket
// counter.  Item (k, p, c, b) may start once every block of the pass before
// it in channel c's chain has finished: done[c][p-1] = k * blocks, or
// done[c][last] = (k - 1) * blocks for p = 0.  Every dependency of a ticket
// is a smaller ticket held by a running block, so the smallest unfinished
// ticket can always proceed.
//
// XCDs.  The device dispatches block b to XCD b % 8, and each XCD has its own
// L2.  Every channel is assigned to one XCD (host side, longest work first
// onto the least loaded XCD), and the blocks of XCD x take items only from
// XCD x's queue (its own ticket counter and segments over its channels), so
// an item and the items it depends on share one L2.  Memory ordering then
// needs no L2 write-back or invalidation: a block waits for its stores to
// complete (the vector L1 writes through to the L2) before it counts itself
// done, and a waiting block invalidates its CU's L1 once its dependency is
// met.  (Agent-scope fences instead write back and invalidate the whole L2
// of the XCD; executed by every wave after every item, they made one
// launch over four channels take minutes.)
//
// Bounded waits.  A wait polls its counter at most spin_limit times and also
// stops when the host raised ctl->give_up or another block set ctl->abort;
// a block that stops sets abort and returns, and every block checks abort
// before taking a ticket, so the launch always drains and returns.
#pragma once
#include "kernels.hpp"  // the pass arguments

namespace msr {

enum PassKind : int { kPassColPsf = 0, kPassRowResid = 1, kPassColFilt = 2, kPassRowUpdate = 3 };

// One pass of one channel's iteration, with the launch arguments the
// per-launch path would pass (recorded from it), for one parity of k (the
// two FISTA iterates swap roles every iteration).
template <typename R>
struct PassDesc {
    int kind;      // PassKind
    int size_idx;  // image size: persist_sizes[size_idx]
    int nblocks;   // blocks of this pass
    int g1;        // filter pass: blocks of its first (C_w) half
    RowArgs<R> ra;
    EpiResid<R> er;
    EpiUpdate<R> eu;
    ColArgs<R> ca, ca2;
    ModePsf<R> mp;
    ModeFilterW<R> mw;
    ModeFilterL<R> ml;
};

constexpr int kPersistXcds = 8;  // XCDs of the device; block b runs on XCD b % 8

struct PersistCtl {
    unsigned int ticket[kPersistXcds];  // the work queue of each XCD
    int abort;    // a block gave up: every block returns
    int give_up;  // raised by the host: every block returns
    int unused[2];
};

template <typename R>
struct PersistArgs {
    const PassDesc<R>* desc;  // [(c * npass + p) * 2 + (k & 1)]
    // XCD x: seg[x * (npass * C + 1) + s] = blocks before segment s = (p, j)
    // of an iteration, p-major over the XCD's channels j (seg[.. + npass n_x]
    // = all); xch[x * C + j] = its channel j; xn[x] = n_x
    const int* seg;
    const int* xch;
    const int* xn;
    unsigned int* done;       // [c * npass + p]: blocks of that pass finished, over all iterations
    PersistCtl* ctl;
    int C, npass, iters, k0;  // iterations k0 + 1 .. k0 + iters
    unsigned int spin_limit;  // polls before a wait gives up
};

// Image sizes the persistent kernel runs and their blocking: 256 threads per
// block for every pass (row passes PAIRS line pairs of L / E threads; column
// passes CB columns).
constexpr int kPersistSizes = 4;
__host__ __device__ constexpr int persist_size(int i) { return i == 0 ? 512 : i == 1 ? 1024 : i == 2 ? 2048 : 4096; }
__host__ __device__ constexpr int persist_emax(int L) { return L >= 4096 ? 16 : 8; }
__host__ __device__ constexpr int persist_pairs(int L) { return 256 / (L / persist_emax(L)); }
__host__ __device__ constexpr int persist_cb(int L) { return 256 / (L / persist_emax(L)); }
__host__ inline int persist_index(int L) {
    for (int i = 0; i < kPersistSizes; ++i)
        if (persist_size(i) == L) return i;
    return -1;
}

// Resets the counters and launches `grid` persistent blocks on stream s
// (single precision; with_4096: the kernel that also holds 4096-wide images).
hipError_t persist_launch_f32(const PersistArgs<float>& pa, bool with_4096, int grid, hipStream_t s);
// Blocks of the persistent kernel one CU holds at once.
int persist_occupancy_f32(bool with_4096);

}  // namespace msr
