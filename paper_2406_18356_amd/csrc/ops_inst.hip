// ops_inst.hip -- instantiates the passes for one line length MSR_L
// (compiled once per length by the build script).
#include "ops.hpp"

#ifndef MSR_L
#error "MSR_L must be defined"
#endif

namespace msr {
namespace {

template <int L, bool PADDED>
struct Inst {
    using C = LineCfg<L, PADDED>;
    static constexpr int T = tile_width(L);
    static constexpr int PAIRS = row_pairs(L, PADDED);
    static constexpr int RT = PAIRS * C::TPF;
    static constexpr int CT = T * C::TPF;

    template <bool INV_IN, bool FWD_OUT, class Epi>
    static void row(const RowArgs& a, const Epi& e, hipStream_t s) {
        const int grid = a.NR / (2 * PAIRS);
        hipLaunchKernelGGL((row_kernel<L, PADDED, PAIRS, T, INV_IN, FWD_OUT, Epi>), dim3(grid), dim3(RT), 0, s, a, e);
    }
    template <class Mode>
    static void col(const ColArgs& a, const Mode& m, hipStream_t s) {
        const int grid = (a.K + T - 1) / T;
        if (grid <= 0) return;
        hipLaunchKernelGGL((col_kernel<L, PADDED, T, Mode>), dim3(grid), dim3(CT), 0, s, a, m);
    }

    static Ops make(bool full) {
        Ops o;
        o.L = L;
        o.padded = PADDED;
        o.T = T;
        o.pairs = PAIRS;
        o.row_rows = 2 * PAIRS;
        o.row_threads = RT;
        o.col_threads = CT;
        if constexpr (!PADDED) {
            o.row_loadshift_fwd = &row<false, true, EpiLoadShift>;
            o.col_forward = &col<ModeForward>;
        }
        if (full) {
            o.row_load_fwd = &row<false, true, EpiLoad>;
            o.row_store = &row<true, false, EpiStore>;
            o.row_resid_fwd = &row<true, true, EpiResid>;
            o.row_resid = &row<true, false, EpiResid>;
            o.row_update_fwd = &row<true, true, EpiUpdate>;
            o.row_power = &row<true, false, EpiPower>;
            o.col_psf = &col<ModePsf>;
            o.col_filth = &col<ModeFilterH>;
            o.col_filtl = &col<ModeFilterL>;
        }
        return o;
    }
};

}  // namespace

#define MSR_CAT2(a, b) a##b
#define MSR_CAT(a, b) MSR_CAT2(a, b)

// Images are at most 8192 wide: the solver passes exist up to L = 8192, the
// unpadded forward transform (PSF spectra) up to L = 16384.
const Ops* MSR_CAT(ops_len_, MSR_L)(bool padded) {
    constexpr bool full = MSR_L <= 8192;
    if (padded) {
        if constexpr (full) {
            static const Ops o = Inst<MSR_L, true>::make(true);
            return &o;
        } else {
            return nullptr;
        }
    }
    static const Ops o = Inst<MSR_L, false>::make(full);
    return &o;
}

}  // namespace msr
