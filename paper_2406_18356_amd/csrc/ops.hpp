// ops.hpp -- launch tables of the transform passes for one line length L and
// one precision.
//
// Each line length is compiled in its own translation unit (ops_inst.hip with
// MSR_L defined), which fills Ops tables for the zero-padded (P = 2L) and the
// unpadded (P = L) variants in single and double precision.  Host code only
// sees these tables.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace msr {

// Column-tile width of the row-spectrum layout for lines of length L, for an
// element of `esize` bytes (8: complex64, 16: complex128).  The column pass
// keeps NH * T lines of L complex values in LDS.
__host__ __device__ constexpr int tile_width(int L, int esize) {
    if (esize == 8) return L <= 1024 ? 4 : (L <= 4096 ? 2 : 1);
    return L <= 1024 ? 4 : (L <= 2048 ? 2 : 1);
}

// Pairs of rows handled by one row-pass block: about 256 threads, at most
// ~72 KB of LDS (one pair may use more).
__host__ __device__ constexpr int row_pairs(int L, bool padded, int esize) {
    const int E = esize == 8 ? (L >= 16 ? 16 : L) : (L >= 8 ? 8 : L);
    const int TPF = L / E;
    const int PT = padded ? 2 * L : L;
    const int lds_pair = (PT + PT / 16) * esize;
    int p = TPF >= 256 ? 1 : 256 / TPF;
    while (p > 1 && p * lds_pair > 72 * 1024) p /= 2;
    if (p > L / 2) p = L / 2;
    return p;
}

// Whether the passes of a (length, padding, element size) combination fit the
// 160 KB of LDS of a gfx950 CU.
__host__ __device__ constexpr bool fits_lds(int L, bool padded, int esize) {
    const int NH = padded ? 2 : 1;
    const int col = NH * tile_width(L, esize) * (L + L / 16) * esize;
    const int PT = padded ? 2 * L : L;
    const int row = row_pairs(L, padded, esize) * (PT + PT / 16) * esize;
    return col <= 160 * 1024 - 4096 && row <= 160 * 1024 - 4096;
}

template <typename R>
struct Ops {
    int L = 0;
    bool padded = false;
    int T = 0;            // tile width of the spectra this table reads and writes
    int pairs = 0;        // row pairs per row-pass block
    int row_rows = 0;     // image rows per row-pass block (2 * pairs)
    int row_threads = 0;  // threads per row-pass block
    int col_threads = 0;  // threads per column-pass block
    void (*row_load_fwd)(const RowArgs<R>&, const EpiLoad<R>&, hipStream_t) = nullptr;            // image -> spectrum
    void (*row_loadshift_fwd)(const RowArgs<R>&, const EpiLoadShift<R>&, hipStream_t) = nullptr;  // PSF -> spectrum
    void (*row_store)(const RowArgs<R>&, const EpiStore<R>&, hipStream_t) = nullptr;              // spectrum -> image
    void (*row_resid_fwd)(const RowArgs<R>&, const EpiResid<R>&, hipStream_t) = nullptr;  // -> (x - y) -> spectrum
    void (*row_resid)(const RowArgs<R>&, const EpiResid<R>&, hipStream_t) = nullptr;      // -> (x - y), sums/stored
    void (*row_update_fwd)(const RowArgs<R>&, const EpiUpdate<R>&, hipStream_t) = nullptr;  // FISTA update
    void (*row_power)(const RowArgs<R>&, const EpiPower<R>&, hipStream_t) = nullptr;        // power iteration
    void (*col_psf)(const ColArgs<R>&, const ModePsf<R>&, hipStream_t) = nullptr;
    void (*col_filth)(const ColArgs<R>&, const ModeFilterH<R>&, hipStream_t) = nullptr;
    void (*col_filtl)(const ColArgs<R>&, const ModeFilterL<R>&, hipStream_t) = nullptr;
    void (*col_forward)(const ColArgs<R>&, const ModeForward<R>&, hipStream_t) = nullptr;  // unpadded forward only
};

// Tables per line length (L = 8 .. 16384); nullptr where not built.
const Ops<float>* ops_for_f32(int L, bool padded);
const Ops<double>* ops_for_f64(int L, bool padded);

template <typename R>
const Ops<R>* ops_for(int L, bool padded) {
    if constexpr (std::is_same_v<R, float>) return ops_for_f32(L, padded);
    else return ops_for_f64(L, padded);
}

}  // namespace msr
