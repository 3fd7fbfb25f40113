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
// element of `esize` bytes (8: complex64, 16: complex128).  A row pass reads
// and writes T adjacent columns of a row as one contiguous run.
__host__ __device__ constexpr int tile_width(int L, int esize) {
    if (esize == 8) return L <= 1024 ? 4 : (L <= 8192 ? 2 : 1);
    return L <= 1024 ? 4 : (L <= 2048 ? 2 : 1);
}

// Columns per column-pass block: the whole tile (T lines of NH halves in LDS)
// unless that does not fit a CU's LDS or the variant asks for single columns;
// then one column (the block reads every T-th value of each row run, and the
// tile's other columns are read by neighbouring blocks through the L2).
__host__ __device__ constexpr int col_block(int L, bool padded, int esize, int emax, bool onecol) {
    const int NH = padded ? 2 : 1;
    const int T = tile_width(L, esize);
    const int E = L >= emax ? emax : L;
    const int whole = NH * T * fft_lds_len(L, E, T) * esize;
    return (onecol || whole > 160 * 1024 - 4096) ? 1 : T;
}

// Largest number of complex elements a thread holds in a transform (the
// register / LDS trade-off): 16 in single precision, 8 in double.
__host__ __device__ constexpr int default_emax(int esize) { return esize == 8 ? 16 : 8; }

// Pairs of rows handled by one row-pass block: about 256 threads, at most
// ~72 KB of LDS (one pair may use more).
__host__ __device__ constexpr int row_pairs(int L, bool padded, int esize, int emax) {
    const int E = L >= emax ? emax : L;
    const int TPF = L / E;
    const int lds_pair = row_line_len(L, padded, E) * esize;
    int p = TPF >= 256 ? 1 : 256 / TPF;
    while (p > 1 && p * lds_pair > 72 * 1024) p /= 2;
    if (p > L / 2) p = L / 2;
    return p;
}

// Whether the passes of a (length, padding, element size, elements per
// thread, single-column) variant fit the 160 KB of LDS and the 1024-thread
// block limit.
__host__ __device__ constexpr bool fits_lds(int L, bool padded, int esize, int emax, bool onecol) {
    const int NH = padded ? 2 : 1;
    const int E = L >= emax ? emax : L;
    const int CB = col_block(L, padded, esize, emax, onecol);
    const int col = NH * CB * fft_lds_len(L, E, CB) * esize;
    const int pairs = row_pairs(L, padded, esize, emax);
    const int row = pairs * row_line_len(L, padded, E) * esize;
    return col <= 160 * 1024 - 4096 && row <= 160 * 1024 - 4096 && CB * (L / E) <= 1024 && pairs * (L / E) <= 1024;
}

// Kernel variants per precision: elements per thread (hence radix schedule
// and LDS per thread) and, for the column pass, whether a block takes a whole
// tile of T columns or a single column (more, shorter blocks for narrow
// spectra).  v0: large E, whole tile; v1: small E, whole tile; v2: small E,
// one column; v3: large E, one column.
constexpr int kVariants = 4;
__host__ __device__ constexpr int variant_emax(int esize, int v) {
    const bool big = (v == 0 || v == 3);
    return esize == 8 ? (big ? 16 : 8) : (big ? 8 : 4);
}
__host__ __device__ constexpr bool variant_single_column(int v) { return v >= 2; }

template <typename R>
struct Ops {
    int L = 0;
    bool padded = false;
    int emax = 0;         // elements per thread of this variant
    int col_cb = 0;       // columns per column-pass block
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
    // the same update with float64 iterates (R = float only)
    void (*row_update_fwd_it64)(const RowArgs<R>&, const EpiUpdate<R, double>&, hipStream_t) = nullptr;
    void (*row_power)(const RowArgs<R>&, const EpiPower<R>&, hipStream_t) = nullptr;        // power iteration
    void (*col_psf)(const ColArgs<R>&, const ModePsf<R>&, hipStream_t) = nullptr;
    void (*col_filtw)(const ColArgs<R>&, const ModeFilterW<R>&, hipStream_t) = nullptr;
    void (*col_filtl)(const ColArgs<R>&, const ModeFilterL<R>&, hipStream_t) = nullptr;
    void (*col_forward)(const ColArgs<R>&, const ModeForward<R>&, hipStream_t) = nullptr;  // unpadded forward only
    // the w and g_L^2 passes of a step-2 iteration in one launch
    void (*col_filt_wl)(const ColArgs<R>&, const ModeFilterW<R>&, const ColArgs<R>&, const ModeFilterL<R>&,
                        hipStream_t) = nullptr;
};

// Tables per line length (L = 8 .. 16384) and variant; nullptr where not built.
const Ops<float>* ops_for_f32(int L, bool padded, int variant);
const Ops<double>* ops_for_f64(int L, bool padded, int variant);

template <typename R>
const Ops<R>* ops_for(int L, bool padded, int variant = 0) {
    if constexpr (std::is_same_v<R, float>) return ops_for_f32(L, padded, variant);
    else return ops_for_f64(L, padded, variant);
}

}  // namespace msr
