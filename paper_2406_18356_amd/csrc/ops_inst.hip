// ops_inst.hip -- instantiates the passes for one line length MSR_L
// (compiled once per length by the build script).
#include "ops.hpp"

#ifndef MSR_L
#error "MSR_L must be defined"
#endif

namespace msr {
namespace {

// Grid y of a launch: the channels of a batched launch, else one.
inline unsigned chans(int nch) { return nch > 1 ? (unsigned)nch : 1u; }

template <typename R, int L, bool PADDED, int EMAX, bool ONECOL>
struct Inst {
    static constexpr int ES = (int)sizeof(cplx<R>);
    using Cf = LineCfg<L, PADDED, R, EMAX>;
    static constexpr int T = tile_width(L, ES);
    static constexpr int CB = col_block(L, PADDED, ES, EMAX, ONECOL);
    static constexpr int PAIRS = row_pairs(L, PADDED, ES, EMAX);
    static constexpr int RT = PAIRS * Cf::TPF;
    static constexpr int CT = CB * Cf::TPF;

    template <bool INV_IN, bool FWD_OUT, class Epi>
    static void row(const RowArgs<R>& a, const Epi& e, hipStream_t s) {
        const int grid = a.NR / (2 * PAIRS);
        hipLaunchKernelGGL((row_kernel<R, L, PADDED, EMAX, PAIRS, T, INV_IN, FWD_OUT, Epi>), dim3(grid, chans(a.nch)),
                           dim3(RT), 0, s, a, e);
    }
    template <class Mode>
    static void col(const ColArgs<R>& a, const Mode& m, hipStream_t s) {
        const int grid = (a.K + CB - 1) / CB;
        if (grid <= 0) return;
        hipLaunchKernelGGL((col_kernel<R, L, PADDED, EMAX, T, CB, Mode>), dim3(grid, chans(a.nch)), dim3(CT), 0, s, a,
                           m);
    }

    template <class M1, class M2>
    static void col_dual(const ColArgs<R>& a1, const M1& m1, const ColArgs<R>& a2, const M2& m2, hipStream_t s) {
        const int g1 = (a1.K + CB - 1) / CB;
        const int g2 = (a2.K + CB - 1) / CB;
        if (g1 + g2 <= 0) return;
        hipLaunchKernelGGL((col_dual_kernel<R, L, PADDED, EMAX, T, CB, M1, M2>), dim3(g1 + g2, chans(a1.nch)), dim3(CT),
                           0, s, a1, m1, g1, a2, m2);
    }

    static Ops<R> make(bool full) {
        Ops<R> o;
        o.L = L;
        o.padded = PADDED;
        o.emax = EMAX;
        o.col_cb = CB;
        o.T = T;
        o.pairs = PAIRS;
        o.row_rows = 2 * PAIRS;
        o.row_threads = RT;
        o.col_threads = CT;
        if constexpr (!PADDED) {
            o.row_loadshift_fwd = &row<false, true, EpiLoadShift<R>>;
            o.col_forward = &col<ModeForward<R>>;
        }
        if (full) {
            o.row_load_fwd = &row<false, true, EpiLoad<R>>;
            o.row_store = &row<true, false, EpiStore<R>>;
            o.row_resid_fwd = &row<true, true, EpiResid<R>>;
            o.row_resid = &row<true, false, EpiResid<R>>;
            o.row_update_fwd = &row<true, true, EpiUpdate<R>>;
            if constexpr (std::is_same<R, float>::value) o.row_update_fwd_it64 = &row<true, true, EpiUpdate<R, double>>;
            o.row_power = &row<true, false, EpiPower<R>>;
            o.col_psf = &col<ModePsf<R>>;
            o.col_filtw = &col<ModeFilterW<R>>;
            o.col_filtl = &col<ModeFilterL<R>>;
            o.col_filt_wl = &col_dual<ModeFilterW<R>, ModeFilterL<R>>;
        }
        return o;
    }
};

// Solver passes exist for images up to 8192 wide; the unpadded forward
// transform (PSF spectra) up to L = 16384.  Combinations whose LDS footprint
// exceeds a CU's LDS are not built.
template <typename R, bool PADDED, int V>
const Ops<R>* table() {
    constexpr int ES = (int)sizeof(cplx<R>);
    constexpr int EMAX = variant_emax(ES, V);
    if constexpr (!fits_lds(MSR_L, PADDED, ES, EMAX, variant_single_column(V))) {
        return nullptr;
    } else {
        constexpr bool full = MSR_L <= 8192;
        if constexpr (PADDED && !full) {
            return nullptr;
        } else {
            static const Ops<R> o = Inst<R, MSR_L, PADDED, EMAX, variant_single_column(V)>::make(full);
            return &o;
        }
    }
}

template <typename R>
const Ops<R>* pick(bool padded, int variant) {
    switch (variant) {
        case 0: return padded ? table<R, true, 0>() : table<R, false, 0>();
        case 1: return padded ? table<R, true, 1>() : table<R, false, 1>();
        case 2: return padded ? table<R, true, 2>() : table<R, false, 2>();
        case 3: return padded ? table<R, true, 3>() : table<R, false, 3>();
        default: return nullptr;
    }
}

}  // namespace

#define MSR_CAT2(a, b) a##b
#define MSR_CAT(a, b) MSR_CAT2(a, b)

const Ops<float>* MSR_CAT(ops_len_f32_, MSR_L)(bool padded, int variant) { return pick<float>(padded, variant); }
const Ops<double>* MSR_CAT(ops_len_f64_, MSR_L)(bool padded, int variant) { return pick<double>(padded, variant); }

}  // namespace msr
