// ops.hpp -- launch table of the transform passes for one line length L.
//
// Each line length is compiled in its own translation unit (ops_inst.hip with
// MSR_L defined), which fills an Ops table for the zero-padded (P = 2L) and
// the unpadded (P = L) variants.  Host code only sees these tables.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace msr {

// Column-tile width of the row-spectrum layout for images of side L.
__host__ __device__ constexpr int tile_width(int L) { return L <= 1024 ? 4 : (L <= 4096 ? 2 : 1); }

// Pairs of rows handled by one row-pass block: about 256 threads, at most ~72 KB of LDS.
__host__ __device__ constexpr int row_pairs(int L, bool padded) {
    const int E = L >= 16 ? 16 : L;
    const int TPF = L / E;
    const int PT = padded ? 2 * L : L;
    const int lds_pair = (PT + PT / 16) * 8;
    int p = TPF >= 256 ? 1 : 256 / TPF;
    while (p > 1 && p * lds_pair > 72 * 1024) p /= 2;
    if (p > L / 2) p = L / 2;
    return p;
}

using RowLoadFn = void (*)(const RowArgs&, const EpiLoad&, hipStream_t);
using RowLoadShiftFn = void (*)(const RowArgs&, const EpiLoadShift&, hipStream_t);
using RowStoreFn = void (*)(const RowArgs&, const EpiStore&, hipStream_t);
using RowResidFn = void (*)(const RowArgs&, const EpiResid&, hipStream_t);
using RowUpdateFn = void (*)(const RowArgs&, const EpiUpdate&, hipStream_t);
using RowPowerFn = void (*)(const RowArgs&, const EpiPower&, hipStream_t);
using ColPsfFn = void (*)(const ColArgs&, const ModePsf&, hipStream_t);
using ColFiltHFn = void (*)(const ColArgs&, const ModeFilterH&, hipStream_t);
using ColFiltLFn = void (*)(const ColArgs&, const ModeFilterL&, hipStream_t);
using ColFwdFn = void (*)(const ColArgs&, const ModeForward&, hipStream_t);

struct Ops {
    int L = 0;
    bool padded = false;
    int T = 0;            // tile width of the spectra this table reads and writes
    int pairs = 0;        // row pairs per row-pass block
    int row_rows = 0;     // image rows per row-pass block (2 * pairs)
    int row_threads = 0;  // threads per row-pass block
    int col_threads = 0;  // threads per column-pass block
    RowLoadFn row_load_fwd = nullptr;           // image -> spectrum
    RowLoadShiftFn row_loadshift_fwd = nullptr; // ifftshift(PSF) -> spectrum (unpadded)
    RowStoreFn row_store = nullptr;             // spectrum -> image
    RowResidFn row_resid_fwd = nullptr;         // spectrum -> (x - y) -> spectrum
    RowResidFn row_resid = nullptr;             // spectrum -> (x - y), reduction only / stored
    RowUpdateFn row_update_fwd = nullptr;       // spectrum -> FISTA update -> spectrum of alpha
    RowPowerFn row_power = nullptr;             // spectrum -> w (power iteration sums)
    ColPsfFn col_psf = nullptr;
    ColFiltHFn col_filth = nullptr;
    ColFiltLFn col_filtl = nullptr;
    ColFwdFn col_forward = nullptr;             // unpadded forward transform only
};

// Tables per line length (L = 8 .. 16384); nullptr where not built.
const Ops* ops_for(int L, bool padded);

}  // namespace msr
