// msr_api.hip -- host side of libmsr: context, workspace, PSF spectra,
// the FISTA loops of both steps, power iteration, objectives and helpers.
//
// Pass chains (P = 2N; "row" passes work on image rows, "col" passes on the
// columns of the row spectra; K_s = kept spectral columns of PSF s):
//
//   step 1 iteration (Eq. 11):
//     col  SA -> SB        x h_hat_L                         (H alpha)
//     row  SB -> SC        r = H alpha - i_L, forward
//     col  SC -> SB        x h_hat_L                         (H^T r)
//     row  SB -> SA        FISTA update (Alg. 1), forward alpha_k
//   step 2 iteration (Eq. 12), with g_H^2 = 1/sigma^2 - w, w = 0 beyond ell + delta:
//     col  SA -> SB        x h_hat_H                                  (H alpha)
//     row  SB -> SC        r = H alpha - i_H, forward (K_H columns)
//     col  SC -> SB        x w (k_x < K_L only)                       (C_w E r)
//     col  SA - SL -> SG   x g_L^2 (k_x < K_L only, same launch as C_w) (C_{g_L^2} E (alpha - l))
//     row  SB -> SB        crop, re-embed, forward (K_H columns)
//     col  SC/s2 - SB -> SB  x h_hat_H    (H^T E^T C_{g_H^2} E r = H^T (r/sigma^2 - E^T C_w E r))
//     row  SB + SG -> SA   FISTA update, forward alpha_k
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/msr.h"
#include "ops.hpp"
#include "small_kernels.hpp"
#include "wavelet_kernels.hpp"
#include "resample_kernels.hpp"
#include "persist.hpp"

using namespace msr;
static_assert(kVariants <= MSR_MAX_VARIANTS, "variant table larger than the ABI's timing array");

namespace msr {
#define MSR_DECL(Lv)                                                \
    const Ops<float>* ops_len_f32_##Lv(bool padded, int variant);   \
    const Ops<double>* ops_len_f64_##Lv(bool padded, int variant);
MSR_DECL(8)
MSR_DECL(16)
MSR_DECL(32)
MSR_DECL(64)
MSR_DECL(128)
MSR_DECL(256)
MSR_DECL(512)
MSR_DECL(1024)
MSR_DECL(2048)
MSR_DECL(4096)
MSR_DECL(8192)
MSR_DECL(16384)
#undef MSR_DECL

#define MSR_CASES(pfx)                                   \
    switch (L) {                                         \
        case 8: return pfx##8(padded, variant);                   \
        case 16: return pfx##16(padded, variant);                 \
        case 32: return pfx##32(padded, variant);                 \
        case 64: return pfx##64(padded, variant);                 \
        case 128: return pfx##128(padded, variant);               \
        case 256: return pfx##256(padded, variant);               \
        case 512: return pfx##512(padded, variant);               \
        case 1024: return pfx##1024(padded, variant);             \
        case 2048: return pfx##2048(padded, variant);             \
        case 4096: return pfx##4096(padded, variant);             \
        case 8192: return pfx##8192(padded, variant);             \
        case 16384: return pfx##16384(padded, variant);           \
        default: return nullptr;                         \
    }
const Ops<float>* ops_for_f32(int L, bool padded, int variant) { MSR_CASES(ops_len_f32_) }
const Ops<double>* ops_for_f64(int L, bool padded, int variant) { MSR_CASES(ops_len_f64_) }
#undef MSR_CASES
}  // namespace msr

// The workspace of msr_set_workspace_static: one array per device, held from
// the loading of this library's device code until the process ends.  Host
// code never uses the name `scratch` as an address (in host code it stands
// for a host-side shadow); it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device below.
static __device__ __align__(256) char scratch[MSR_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
struct StaticWorkspace {
    void* ptr = nullptr;          // device address of `scratch` on this device
    unsigned long long gen = 0;   // bumped whenever a context binds the array
};
StaticWorkspace g_static[kMaxDevices];
std::mutex g_static_mu;

// Looks up the device address of `scratch` on `dev` once; `dev` must be the
// current device.  Returns hipSuccess and sets *out, or the lookup's error.
hipError_t static_workspace_ptr(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_static[dev].ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_static[dev].ptr = p;
    }
    *out = g_static[dev].ptr;
    return hipSuccess;
}
}  // namespace

namespace {

// Low-pass taps of db_p (2p of them, sum sqrt(2), minimum phase) by spectral
// factorisation: with y = sin^2(w/2), |H|^2 = 2 cos^{2p}(w/2) Q(y),
// Q(y) = sum_{k<p} C(p-1+k, k) y^k.  Each root y_j of Q gives the root z_j of
// z^2 - (2 - 4 y_j) z + 1 inside the unit circle, and
// H(z) ~ (1 + z^-1)^p prod_j (1 - z_j z^-1).  Q's roots come from
// Durand-Kerner iterations (degree <= 7) polished by Newton steps.
// Returns false if the result is not orthonormal to 1e-10.
bool daubechies_taps(int p, double* h) {
    using cd = std::complex<double>;
    std::vector<double> q(p);
    for (int k = 0; k < p; ++k) {
        double b = 1.0;  // C(p-1+k, k)
        for (int i = 1; i <= k; ++i) b = b * (p - 1 + i) / i;
        q[k] = b;
    }
    std::vector<cd> poly{cd(1.0)};
    auto conv2 = [&](cd a0, cd a1) {
        std::vector<cd> r(poly.size() + 1, cd(0.0));
        for (size_t i = 0; i < poly.size(); ++i) {
            r[i] += poly[i] * a0;
            r[i + 1] += poly[i] * a1;
        }
        poly = r;
    };
    for (int i = 0; i < p; ++i) conv2(cd(1.0), cd(1.0));
    const int d = p - 1;
    if (d > 0) {
        auto Q = [&](cd y) {
            cd v(0.0);
            for (int k = d; k >= 0; --k) v = v * y + q[k];
            return v;
        };
        auto dQ = [&](cd y) {
            cd v(0.0);
            for (int k = d; k >= 1; --k) v = v * y + q[k] * (double)k;
            return v;
        };
        std::vector<cd> r(d);
        for (int i = 0; i < d; ++i) r[i] = std::pow(cd(0.4, 0.9), i);
        for (int it = 0; it < 2000; ++it) {
            double ch = 0.0;
            for (int i = 0; i < d; ++i) {
                cd den = q[d];
                for (int j = 0; j < d; ++j)
                    if (j != i) den *= (r[i] - r[j]);
                const cd step = Q(r[i]) / den;
                r[i] -= step;
                ch = std::max(ch, std::abs(step));
            }
            if (ch < 1e-15) break;
        }
        for (int i = 0; i < d; ++i)
            for (int it = 0; it < 5; ++it) {
                const cd dq = dQ(r[i]);
                if (std::abs(dq) == 0.0) break;
                r[i] -= Q(r[i]) / dq;
            }
        for (int i = 0; i < d; ++i) {
            const cd b = 2.0 - 4.0 * r[i];
            const cd disc = std::sqrt(b * b - 4.0);
            const cd z1 = (b + disc) / 2.0, z2 = (b - disc) / 2.0;
            conv2(cd(1.0), -(std::abs(z1) < 1.0 ? z1 : z2));
        }
    }
    double sum = 0.0;
    for (int i = 0; i < 2 * p; ++i) sum += poly[i].real();
    for (int i = 0; i < 2 * p; ++i) h[i] = poly[i].real() * std::sqrt(2.0) / sum;
    for (int m = 0; m < p; ++m) {
        double s = 0.0;
        for (int i = 0; i + 2 * m < 2 * p; ++i) s += h[i] * h[i + 2 * m];
        if (std::fabs(s - (m == 0 ? 1.0 : 0.0)) > 1e-10) return false;
    }
    return true;
}

constexpr double kThetaMargin = 1.01;  // Rayleigh quotients under-estimate lambda_max
constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    size_t tw, stwN, stwP, SA, SB, SC, SL, SG, hh1, hh2, d1, d2, b0, b1, t0, t1, mc0, mc1, mc2, mc3, partials, scal,
        colmax, cb0, cb1, ca, cg, wx, taps, total;
};

struct Shapes {
    int N, P, T, Cfull, Cpad, Tpsf, Cpad_psf;
    bool padded;
    bool dict;           // wavelet dictionary: 8 coefficient arrays of N x N per state
    int prec;            // 32 or 64
    bool it64;           // float64 iterates with float32 transforms
    size_t rs, cs;       // bytes of a real / complex element
    size_t is;           // bytes of an iterate element
    size_t spec_elems;   // N * Cpad complex
    size_t hh_elems;     // P * Cpad reals
    size_t img_elems;    // N * N
    size_t partial_cnt;  // doubles
};

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

template <typename R>
bool tables(int N, int P, bool padded, int& T, int& Tpsf) {
    const Ops<R>* o = ops_for<R>(N, padded, 0);
    const Ops<R>* op = ops_for<R>(P, false, 0);
    if (!o || !op || !o->row_update_fwd || !op->col_forward) return false;
    T = o->T;
    Tpsf = op->T;
    return true;
}

bool make_shapes(const msr_config* c, Shapes& s, std::string* why) {
    if (!c) {
        if (why) *why = "null config";
        return false;
    }
    if (!pow2(c->n) || c->n < 8 || c->n > 8192) {
        if (why) *why = "n must be a power of two in [8, 8192]";
        return false;
    }
    if (c->pad != 1 && c->pad != 2) {
        if (why) *why = "pad must be 1 (circular) or 2 (zero padded)";
        return false;
    }
    if (c->precision != 32 && c->precision != 64) {
        if (why) *why = "precision must be 32 or 64";
        return false;
    }
    if (c->dictionary != 0 && c->dictionary != 1) {
        if (why) *why = "dictionary must be 0 (identity) or 1 (db1-db8)";
        return false;
    }
    if (c->dictionary == 1 && c->n < (1 << kWaveletLevels)) {
        if (why) *why = "the wavelet dictionary needs n >= 16";
        return false;
    }
    const int ip = c->iterate_precision;
    if (ip != 0 && ip != c->precision && !(ip == 64 && c->precision == 32)) {
        if (why) *why = "iterate_precision must be 0, the precision, or 64 with precision 32";
        return false;
    }
    s.it64 = ip == 64 && c->precision == 32;
    if (s.it64 && c->dictionary != 0) {
        if (why) *why = "float64 iterates need dictionary 0";
        return false;
    }
    s.dict = c->dictionary == 1;
    s.N = c->n;
    s.padded = c->pad == 2;
    s.P = c->pad * c->n;
    s.prec = c->precision;
    const bool ok = s.prec == 32 ? tables<float>(s.N, s.P, s.padded, s.T, s.Tpsf)
                                 : tables<double>(s.N, s.P, s.padded, s.T, s.Tpsf);
    if (!ok) {
        if (why) *why = "no kernels built for this size and precision";
        return false;
    }
    s.rs = s.prec == 32 ? 4 : 8;
    s.cs = 2 * s.rs;
    s.is = s.it64 ? 8 : s.rs;
    s.Cfull = s.P / 2 + 1;
    s.Cpad = (int)align_up(s.Cfull, s.T);
    s.Cpad_psf = (int)align_up(s.Cfull, s.Tpsf);
    s.spec_elems = (size_t)s.N * s.Cpad;
    s.hh_elems = (size_t)s.P * s.Cpad;
    s.img_elems = (size_t)s.N * s.N;
    s.partial_cnt = (size_t)4 * (2 * (size_t)s.P + 4096);
    return true;
}

Layout make_layout(const Shapes& s) {
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    l.tw = take(s.cs * (size_t)s.P);
    l.stwN = take(s.cs * (size_t)stage_tables_len(s.N));
    l.stwP = take(s.cs * (size_t)stage_tables_len(s.P));
    l.SA = take(s.cs * s.spec_elems);
    // SB and SC are contiguous: together they hold the P-row PSF spectrum.
    const size_t sbc = std::max(align_up(s.cs * s.spec_elems, kAlign) * 2, s.cs * (size_t)s.P * s.Cpad_psf);
    l.SB = take(sbc);
    l.SC = l.SB + align_up(s.cs * s.spec_elems, kAlign);
    l.SL = take(s.cs * s.spec_elems);
    l.SG = take(s.cs * s.spec_elems);
    l.hh1 = take(s.rs * s.hh_elems);
    l.hh2 = take(s.rs * s.hh_elems);
    l.d1 = take(s.rs * s.img_elems);
    l.d2 = take(s.rs * s.img_elems);
    l.b0 = take(s.is * s.img_elems);
    l.b1 = take(s.is * s.img_elems);
    l.t0 = take(s.rs * s.img_elems);
    l.t1 = take(s.rs * s.img_elems);
    // major cycles: original dirty image, sum of the cycle images, constraint, cycle image
    l.mc0 = take(s.rs * s.img_elems);
    l.mc1 = take(s.rs * s.img_elems);
    l.mc2 = take(s.rs * s.img_elems);
    l.mc3 = take(s.rs * s.img_elems);
    l.partials = take(sizeof(double) * s.partial_cnt);
    l.scal = take(sizeof(double) * 64);
    l.colmax = take(sizeof(double) * (size_t)s.Cfull);
    if (s.dict) {
        // coefficient states beta_{k-1}, beta_{k-2} (rotating) and alpha_k; two
        // regions of 8 (N/2)^2 for the lo-lo images between levels; the image
        // W alpha; the filters
        const size_t ce = (size_t)kWaveletBases * s.img_elems * s.rs;
        l.cb0 = take(ce);
        l.cb1 = take(ce);
        l.ca = take(ce);
        l.cg = take(ce / 2);
        l.wx = take(s.rs * s.img_elems);
        l.taps = take(sizeof(Taps<double>) * kWaveletBases);
    }
    l.total = off;
    return l;
}

}  // namespace

struct msr_ctx {
    msr_config cfg{};
    Shapes sh{};
    Layout lay{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // bound to the static workspace of its device (msr_set_workspace_static) at
    // binding number ws_gen; a later binding by another context takes it away
    bool ws_static = false;
    unsigned long long ws_gen = 0;
    bool ws_lost = false;  // the static workspace was bound by another context since
    // state
    int K[2] = {0, 0};  // kept columns per PSF
    bool have_psf[2] = {false, false};
    bool have_filters = false;
    bool have_theta[2] = {false, false};
    double theta[2] = {0, 0};
    double ell = 0, delta = 0, sigma2 = 0, eta2 = 0;
    int KL = 0;  // columns with g_L != 0
    // FISTA state: the step whose last solve's iterates are still in the
    // workspace (0: none) and its iteration count; a state loaded by
    // msr_set_state that the next solve of a step continues from (-1: none)
    int state_step = 0, state_k = 0;
    int resume_k[2] = {-1, -1};
    int var_row[2] = {0, 0}, var_col[2] = {0, 0};  // kernel variants per step (autotuned)
    int var_filt = -1;  // variant of the step-2 low-band filter pass (-1: that of the step-2 column pass)
    std::string err;
};

namespace {

msr_status fail(msr_ctx* c, msr_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIPCHK(ctx, expr)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(ctx, MSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(ctx)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = hipGetLastError();                                                               \
        if (e_ != hipSuccess) return fail(ctx, MSR_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                               \
    do {                                        \
        msr_status st_ = (expr);                \
        if (st_ != MSR_OK) return st_;          \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a and
// off-diagonal b (|b| = |a| - 1) by bisection on the Sturm count: the number
// of eigenvalues below x is the number of negative pivots of T - x I.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    const size_t m = a.size();
    double lo = a[0], hi = a[0];
    for (size_t i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto below = [&](double x) {
        size_t cnt = 0;
        double d = 1.0;
        for (size_t i = 0; i < m; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0) ++cnt;
        }
        return cnt;
    };
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    for (int it = 0; it < 200 && hi - lo > 4e-16 * scale; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == m)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}
inline unsigned blocks_for(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }

// All typed work of one context, in precision R.
template <typename R>
struct Impl {
    using C = cplx<R>;
    msr_ctx* c;
    const Ops<R>* opr_[2];  // N-length row passes per step (padded or circular)
    const Ops<R>* opc_[2];  // N-length column passes per step
    const Ops<R>* opf_;     // step-2 low-band filter pass (C_w and C_{g_L^2} in one launch)
    const Ops<R>* opp;      // P-length unpadded (PSF spectrum)
    // A batched group: nch_ channels whose workspaces follow this context's at
    // cstride_ bytes; kept-column counts are the group's maxima (the PSF and
    // filter factors are zero beyond each channel's own count).
    int nch_ = 1;
    long long cstride_ = 0;
    const ChanScalars<R>* chan_ = nullptr;
    const FilterCoef<R>* chanf_ = nullptr;
    int gK_[2] = {0, 0}, gKL_ = 0;
    // Recording instead of launching (the persistent batched launch): each
    // pass of iterate() appends its arguments here, blocked for the
    // persistent kernel's shape of this image size.
    std::vector<PassDesc<R>>* rec_ = nullptr;
    PassDesc<R> rec_desc(int kind) const {
        PassDesc<R> d{};
        d.kind = kind;
        d.size_idx = persist_index(N());
        return d;
    }
    static int ceil_div(int a, int b) { return (a + b - 1) / b; }

    void set_group(int nch, long long cstride, const ChanScalars<R>* chan, const FilterCoef<R>* chanf, int K1, int K2,
                   int KL) {
        nch_ = nch;
        cstride_ = cstride;
        chan_ = chan;
        chanf_ = chanf;
        gK_[0] = K1;
        gK_[1] = K2;
        gKL_ = KL;
    }
    bool grouped() const { return chan_ != nullptr; }
    int Ks(int step) const { return grouped() ? gK_[step - 1] : c->K[step - 1]; }
    int KLs() const { return grouped() ? gKL_ : c->KL; }

    static const Ops<R>* variant_or_default(int L, bool padded, int v) {
        const Ops<R>* o = ops_for<R>(L, padded, v);
        return (o && o->row_update_fwd) ? o : ops_for<R>(L, padded, 0);
    }
    explicit Impl(msr_ctx* ctx) : c(ctx), opp(ops_for<R>(ctx->sh.P, false, 0)) {
        for (int s = 0; s < 2; ++s) {
            opr_[s] = variant_or_default(ctx->sh.N, ctx->sh.padded, ctx->var_row[s]);
            opc_[s] = variant_or_default(ctx->sh.N, ctx->sh.padded, ctx->var_col[s]);
        }
        opf_ = ctx->var_filt < 0 ? opc_[1] : variant_or_default(ctx->sh.N, ctx->sh.padded, ctx->var_filt);
    }
    const Ops<R>* opr(int step) const { return opr_[step - 1]; }
    const Ops<R>* opc(int step) const { return opc_[step - 1]; }

    template <typename X>
    X* at(size_t off) const { return reinterpret_cast<X*>(c->ws + off); }
    C* tw() const { return at<C>(c->lay.tw); }
    C* stwN() const { return at<C>(c->lay.stwN); }
    C* stwP() const { return at<C>(c->lay.stwP); }
    C* SA() const { return at<C>(c->lay.SA); }
    C* SB() const { return at<C>(c->lay.SB); }
    C* SC() const { return at<C>(c->lay.SC); }
    C* SL() const { return at<C>(c->lay.SL); }
    C* SG() const { return at<C>(c->lay.SG); }
    R* hh(int step) const { return at<R>(step == 1 ? c->lay.hh1 : c->lay.hh2); }
    R* dirty(int step) const { return at<R>(step == 1 ? c->lay.d1 : c->lay.d2); }
    R* beta(int k) const { return at<R>((k & 1) ? c->lay.b1 : c->lay.b0); }
    // float64 iterates (iterate_precision 64): the same buffers, 8 bytes an element
    bool it64() const { return c->sh.it64; }
    double* beta64(int k) const { return at<double>((k & 1) ? c->lay.b1 : c->lay.b0); }
    void* iter_buf(int k) const { return at<char>((k & 1) ? c->lay.b1 : c->lay.b0); }
    // beta_k as an R image: the iterate itself, or (float64 iterates) rounded
    // into the major-cycle buffer mc3 (no single solve uses it then)
    msr_status beta_r(int k, const R** out, hipStream_t s) {
        if (!it64()) {
            *out = beta(k);
            return MSR_OK;
        }
        R* dst = at<R>(c->lay.mc3);
        const size_t n = c->sh.img_elems;
        hipLaunchKernelGGL((convert_image<R, double>), dim3(blocks_for(n)), dim3(256), 0, s, dst,
                           (const double*)beta64(k), n);
        LAUNCHCHK(c);
        *out = dst;
        return MSR_OK;
    }
    R* tmp(int i) const { return at<R>(i ? c->lay.t1 : c->lay.t0); }
    bool dict() const { return c->sh.dict; }
    size_t cn() const { return (size_t)kWaveletBases * c->sh.img_elems; }
    R* coef(int k) const { return at<R>((k & 1) ? c->lay.cb1 : c->lay.cb0); }
    R* cA() const { return at<R>(c->lay.ca); }
    // lo-lo images between levels: region i of 8 x (N/2)^2
    R* wscr(int i) const { return at<R>(c->lay.cg) + (size_t)i * kWaveletBases * (c->sh.img_elems / 4); }
    R* wx() const { return at<R>(c->lay.wx); }
    Taps<R>* taps(int b) const { return at<Taps<R>>(c->lay.taps) + b; }
    R* mc(int i) const {
        const size_t o[4] = {c->lay.mc0, c->lay.mc1, c->lay.mc2, c->lay.mc3};
        return at<R>(o[i]);
    }
    double* partials() const { return at<double>(c->lay.partials); }
    double* scal() const { return at<double>(c->lay.scal); }
    double* colmax() const { return at<double>(c->lay.colmax); }
    int N() const { return c->sh.N; }
    int P() const { return c->sh.P; }

    FilterCoef<R> filters() const {
        FilterCoef<R> f{};
        f.ell = (R)c->ell;
        f.delta = (R)c->delta;
        f.inv_sigma2 = (R)(1.0 / c->sigma2);
        f.inv_eta2 = (R)(1.0 / c->eta2);
        f.sigma2 = (R)c->sigma2;
        f.eta2 = (R)c->eta2;
        f.half_pi_over_delta = (R)(M_PI / (2.0 * c->delta));
        const double hi = c->ell + c->delta, lo = c->ell - c->delta;
        f.hi_r2 = (long long)std::floor(hi * hi);
        f.lo_r2 = lo > 0 ? (long long)std::ceil(lo * lo) : 0;
        f.P = c->sh.P;
        return f;
    }
    R inv_p2() const { return (R)(1.0 / ((double)P() * (double)P())); }

    RowArgs<R> row_args(const C* in, int kin, const C* in2, int kin2, C* out, int kout, bool reduce = false) const {
        RowArgs<R> a{};
        a.spec_in = in;
        a.spec_in2 = in2;
        a.spec_out = out;
        a.tw = tw();
        a.tws = stwN();
        a.partials = partials();
        a.NR = N();
        a.K_in = kin;
        a.K_in2 = in2 ? kin2 : 0;
        a.K_out = kout;
        a.reduce = reduce ? 1 : 0;
        a.nch = nch_;
        a.cstride = cstride_;
        a.chan = chan_;
        return a;
    }
    ColArgs<R> col_args(const C* in, const C* in2, C* out, int K, bool reduce = false, R in_scale = (R)1) const {
        ColArgs<R> a{};
        a.in_scale = in_scale;
        a.spec_in = in;
        a.spec_in2 = in2;
        a.spec_out = out;
        a.tw = tw();
        a.tws = stwN();
        a.partials = partials();
        a.NR = N();
        a.K = K;
        a.reduce = reduce ? 1 : 0;
        a.nch = nch_;
        a.cstride = cstride_;
        a.chan = chan_;
        a.chanf = chanf_;
        return a;
    }
    int row_grid(int step) const { return N() / opr(step)->row_rows; }
    int col_grid(int step, int K) const { return (K + opc(step)->col_cb - 1) / opc(step)->col_cb; }
    int KA(int step) const { return step == 1 ? Ks(1) : std::max(Ks(2), KLs()); }

    // Sum `nq` quantities over `nblocks` partial rows into scal[off..]; copies them to host.
    msr_status reduce(int nblocks, int nq, int off, double* host, hipStream_t s) {
        hipLaunchKernelGGL(finalize_sums, dim3(1), dim3(256), 0, s, partials(), nblocks, nq, scal() + off);
        LAUNCHCHK(c);
        if (host) {
            HIPCHK(c, hipMemcpyAsync(host, scal() + off, sizeof(double) * nq, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
        }
        return MSR_OK;
    }

    msr_status image_reduce(const R* x, const R* y, int mode, double* host, hipStream_t s) {
        const size_t n = c->sh.img_elems;
        const int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
        hipLaunchKernelGGL(image_sums<R>, dim3(blocks), dim3(256), 0, s, x, y, n, mode, partials());
        LAUNCHCHK(c);
        return reduce(blocks, 1, 8, host, s);
    }

    // image -> row spectrum
    msr_status fwd_image(int step, const R* img, R scale, C* out, int kout, hipStream_t s) {
        opr(step)->row_load_fwd(row_args(nullptr, 0, nullptr, 0, out, kout), EpiLoad<R>{img, N(), scale}, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    // out = IDFT_y(h_hat . DFT_y(in_scale * in - in2)) on the kept columns of PSF `step`.
    // chan_scale: in a batched group each channel takes in_scale = its 1 / sigma^2.
    msr_status col_psf(int step, const C* in, C* out, hipStream_t s, const C* in2 = nullptr, R in_scale = (R)1,
                       bool chan_scale = false) {
        ColArgs<R> a = col_args(in, in2, out, Ks(step), false, in_scale);
        a.chan_scale = chan_scale ? 1 : 0;
        if (rec_) {
            PassDesc<R> d = rec_desc(kPassColPsf);
            d.ca = a;
            d.mp = ModePsf<R>{hh(step), P(), c->sh.T};
            d.nblocks = ceil_div(a.K, persist_cb(N()));
            rec_->push_back(d);
            return MSR_OK;
        }
        opc(step)->col_psf(a, ModePsf<R>{hh(step), P(), c->sh.T}, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }
    msr_status col_filtw(const C* in, C* out, bool red, hipStream_t s) {
        opc(2)->col_filtw(col_args(in, nullptr, out, c->KL, red), ModeFilterW<R>{filters(), inv_p2()}, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }
    msr_status col_filtl(const C* in, const C* in2, C* out, bool red, hipStream_t s) {
        opc(2)->col_filtl(col_args(in, in2, out, c->KL, red), ModeFilterL<R>{filters(), inv_p2()}, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    // C_w on (SC -> SB) and C_{g_L^2} on (SA - SL -> SG), k_x < K_L, one launch.
    msr_status col_filt_wl(const C* l, hipStream_t s) {
        const ModeFilterW<R> mw{filters(), inv_p2()};
        const ModeFilterL<R> ml{filters(), inv_p2()};
        if (rec_) {
            PassDesc<R> d = rec_desc(kPassColFilt);
            d.ca = col_args(SC(), nullptr, SB(), KLs());
            d.ca2 = col_args(SA(), l, SG(), KLs());
            d.mw = mw;
            d.ml = ml;
            d.g1 = ceil_div(d.ca.K, persist_cb(N()));
            d.nblocks = d.g1 + ceil_div(d.ca2.K, persist_cb(N()));
            rec_->push_back(d);
            return MSR_OK;
        }
        opf_->col_filt_wl(col_args(SC(), nullptr, SB(), KLs()), mw, col_args(SA(), l, SG(), KLs()), ml, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    // The gradient chain of step s applied to the spectrum in SA (alpha); leaves
    // the half-gradient spectrum in SB (+ SG for k_x < K_L in step 2).  `y` is
    // the data image (null for the normal operator alone); step 2 subtracts the
    // spectrum of l (SL) when `use_l`.
    msr_status grad_chain(int step, const R* y, bool use_l, hipStream_t s) {
        const int K = Ks(step);
        TRY(col_psf(step, SA(), SB(), s));
        if (step == 1) {
            TRY(row_resid_fwd(1, row_args(SB(), K, nullptr, 0, SC(), K), EpiResid<R>{y, nullptr, N()}, s));
            return col_psf(1, SC(), SB(), s);
        }
        const int kr = std::max(K, KLs());
        TRY(row_resid_fwd(2, row_args(SB(), K, nullptr, 0, SC(), kr), EpiResid<R>{y, nullptr, N()}, s));
        TRY(col_filt_wl(use_l ? SL() : nullptr, s));
        TRY(row_resid_fwd(2, row_args(SB(), KLs(), nullptr, 0, SB(), K), EpiResid<R>{nullptr, nullptr, N()}, s));
        return col_psf(2, SC(), SB(), s, SB(), (R)(1.0 / c->sigma2), grouped());
    }

    msr_status row_resid_fwd(int step, const RowArgs<R>& a, const EpiResid<R>& e, hipStream_t s) {
        if (rec_) {
            PassDesc<R> d = rec_desc(kPassRowResid);
            d.ra = a;
            d.er = e;
            d.nblocks = N() / (2 * persist_pairs(N()));
            rec_->push_back(d);
            return MSR_OK;
        }
        opr(step)->row_resid_fwd(a, e, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    static double momentum(int k) { return k >= 1 ? (k - 1.0) / (k + 2.0) : 0.0; }

    // One FISTA iteration k (1-based) of step s.
    msr_status iterate(int step, int k, double mu, double lambda, hipStream_t s) {
        TRY(grad_chain(step, dirty(step), true, s));
        if (it64()) {
            if (rec_) return fail(c, MSR_ERR_UNSUPPORTED, "float64 iterates in a persistent launch");
            EpiUpdate<R, double> u{};
            u.b1 = beta64(k - 1);
            u.b2 = beta64(k);
            u.ld = N();
            u.two_mu = 2.0 * mu;
            u.thr = mu * lambda;
            u.t_prev = momentum(k - 1);
            u.t_cur = momentum(k);
            u.positivity = c->cfg.positivity;
            const int K = Ks(step);
            RowArgs<R> a = step == 1 ? row_args(SB(), K, nullptr, 0, SA(), KA(1))
                                     : row_args(SB(), K, SG(), KLs(), SA(), KA(2));
            opr(step)->row_update_fwd_it64(a, u, s);
            LAUNCHCHK(c);
            return MSR_OK;
        }
        EpiUpdate<R> u{};
        u.b1 = beta(k - 1);
        u.b2 = beta(k);
        u.ld = N();
        u.two_mu = (R)(2.0 * mu);
        u.thr = (R)(mu * lambda);
        u.t_prev = (R)momentum(k - 1);
        u.t_cur = (R)momentum(k);
        u.positivity = c->cfg.positivity;
        const int K = Ks(step);
        RowArgs<R> a = step == 1 ? row_args(SB(), K, nullptr, 0, SA(), KA(1))
                                 : row_args(SB(), K, SG(), KLs(), SA(), KA(2));
        if (rec_) {
            PassDesc<R> d = rec_desc(kPassRowUpdate);
            d.ra = a;
            d.eu = u;
            d.nblocks = N() / (2 * persist_pairs(N()));
            rec_->push_back(d);
            return MSR_OK;
        }
        opr(step)->row_update_fwd(a, u, s);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    // Exact objective of step s at image x (device), FP64 sums.  out: F, data, l1.
    // Uses SB, SC (and SG for step 2) as scratch; SA and SL are preserved.  The
    // sums land in scal[16..19] and come back to the host in one copy.
    msr_status objective_at(int step, double lambda, const R* x, double out[3], hipStream_t s) {
        constexpr int kSlot = 16;  // data (or ||r||^2), sum w |R|^2, sum g_L^2 |.|^2, ||x||_1
        if (step == 1) {
            TRY(fwd_image(1, x, (R)1, SB(), c->K[0], s));
            TRY(col_psf(1, SB(), SC(), s));
            opr(1)->row_resid(row_args(SC(), c->K[0], nullptr, 0, nullptr, 0, true), EpiResid<R>{dirty(1), nullptr, N()}, s);
            LAUNCHCHK(c);
            TRY(reduce(row_grid(1), 1, kSlot, nullptr, s));
        } else {
            // ||G_H r||^2 = ||r||^2 / sigma^2 - (1/P^2) sum w |R|^2, ||G_L (l - x)||^2 = (1/P^2) sum g_L^2 |.|^2
            TRY(fwd_image(2, x, (R)1, SB(), KA(2), s));
            TRY(col_psf(2, SB(), SC(), s));
            opr(2)->row_resid_fwd(row_args(SC(), c->K[1], nullptr, 0, SC(), c->KL, true),
                                  EpiResid<R>{dirty(2), nullptr, N()}, s);
            LAUNCHCHK(c);
            TRY(reduce(row_grid(2), 1, kSlot, nullptr, s));
            // C_w on SC (in place) and C_{g_L^2} on SB - SL (into SG) in one
            // launch; the blocks of each pass hold their own partial rows
            const ModeFilterW<R> mw{filters(), inv_p2()};
            const ModeFilterL<R> ml{filters(), inv_p2()};
            opf_->col_filt_wl(col_args(SC(), nullptr, SC(), c->KL, true), mw, col_args(SB(), SL(), SG(), c->KL, true), ml,
                              s);
            LAUNCHCHK(c);
            const int g = (c->KL + opf_->col_cb - 1) / opf_->col_cb;
            TRY(reduce(g, 1, kSlot + 1, nullptr, s));
            hipLaunchKernelGGL(finalize_sums, dim3(1), dim3(256), 0, s, partials() + g, g, 1, scal() + kSlot + 2);
            LAUNCHCHK(c);
        }
        const size_t n = c->sh.img_elems;
        const int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
        hipLaunchKernelGGL(image_sums<R>, dim3(blocks), dim3(256), 0, s, x, (const R*)nullptr, n, 0, partials());
        LAUNCHCHK(c);
        TRY(reduce(blocks, 1, kSlot + 3, nullptr, s));
        double h[4];
        HIPCHK(c, hipMemcpyAsync(h, scal() + kSlot, sizeof h, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        double data = h[0];
        if (step == 2) {
            const double ip2 = 1.0 / ((double)P() * (double)P());
            data = h[0] / c->sigma2 + (h[2] - h[1]) * ip2;
        }
        const double l1 = h[3];
        out[0] = data + lambda * l1;
        out[1] = data;
        out[2] = l1;
        return MSR_OK;
    }

    msr_status set_low_res(const R* low_res, hipStream_t s) { return fwd_image(2, low_res, (R)1, SL(), c->KL, s); }

    // theta = 2 lambda_max of the step's normal operator by the Lanczos
    // iteration (Sect. 3.4 defines theta; the Krylov method is this library's
    // choice): q_1 = v0 / ||v0|| (SplitMix64 start vector), then per step
    //   w = A q_j (the gradient chain without data), alpha_j = <q_j, w>,
    //   r = w - alpha_j q_j - beta_{j-1} q_{j-1}, beta_j = ||r||, q_{j+1} = r / beta_j,
    // theta_j = 2 lambda_max(T_j) of the tridiagonal (alpha, beta) matrix; stop
    // when |theta_j - theta_{j-1}| <= rtol theta_j, beta_j = 0 or after max_iter
    // applications.  Vectors are stored unnormalised with their scale (the
    // image load applies it); FP64 reductions; one host round trip a step.
    msr_status power_iteration(int step, int max_iter, double rtol, double* theta_out, int* iters_out, hipStream_t s) {
        const size_t n = c->sh.img_elems;
        R* buf[3] = {tmp(0), tmp(1), mc(3)};  // mc(3) holds nothing between calls (a solve's output slot)
        int cur = 0, prv = 1, wb = 2;
        hipLaunchKernelGGL(start_vector<R>, dim3(blocks_for(n)), dim3(256), 0, s, buf[cur],
                           (unsigned long long)c->cfg.seed, n);
        LAUNCHCHK(c);
        double nv2 = 0.0;
        TRY(image_reduce(buf[cur], nullptr, 1, &nv2, s));
        if (!(nv2 > 0)) return fail(c, MSR_ERR_NUMERIC, "zero start vector");
        double s_cur = 1.0 / std::sqrt(nv2), s_prv = 0.0, beta_prev = 0.0;
        std::vector<double> al, be;
        const int sblocks = (int)std::min<size_t>(1024, (n + 255) / 256);
        double theta = 0.0, prev = -1.0;
        int j = 0;
        for (j = 1; j <= max_iter; ++j) {
            TRY(fwd_image(step, buf[cur], (R)s_cur, SA(), KA(step), s));
            TRY(grad_chain(step, nullptr, false, s));
            EpiPower<R> ep{buf[cur], buf[wb], N(), (R)s_cur};
            RowArgs<R> a = step == 1 ? row_args(SB(), c->K[0], nullptr, 0, nullptr, 0, true)
                                     : row_args(SB(), c->K[1], SG(), c->KL, nullptr, 0, true);
            opr(step)->row_power(a, ep, s);
            LAUNCHCHK(c);
            TRY(reduce(row_grid(step), 2, 0, nullptr, s));  // scal[0] = ||w||^2, scal[1] = alpha_j
            hipLaunchKernelGGL(lanczos_step<R>, dim3(sblocks), dim3(256), 0, s, buf[wb], (const R*)buf[cur],
                               beta_prev > 0 ? (const R*)buf[prv] : nullptr, (const double*)(scal() + 1), (R)s_cur,
                               (R)(beta_prev * s_prv), n, partials());
            LAUNCHCHK(c);
            hipLaunchKernelGGL(finalize_sums, dim3(1), dim3(256), 0, s, partials(), sblocks, 1, scal() + 2);
            LAUNCHCHK(c);
            double h[3];
            HIPCHK(c, hipMemcpyAsync(h, scal(), sizeof h, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2]))
                return fail(c, MSR_ERR_NUMERIC, "Lanczos iteration diverged at %d", j);
            al.push_back(h[1]);
            theta = 2.0 * tridiag_max_eig(al, be);
            if (prev >= 0 && std::fabs(theta - prev) <= rtol * theta) break;
            prev = theta;
            if (!(h[2] > 0)) break;  // the Krylov space is invariant: theta is exact
            const double b = std::sqrt(h[2]);
            be.push_back(b);
            s_prv = s_cur;
            s_cur = 1.0 / b;
            beta_prev = b;
            const int old = prv;
            prv = cur;
            cur = wb;
            wb = old;
        }
        // With the dictionary the variable is alpha and the normal operator is
        // W^T A W; W W^T = M I makes its largest eigenvalue M times that of A.
        if (dict()) theta *= kWaveletBases;
        if (theta_out) *theta_out = theta;
        if (iters_out) *iters_out = std::min(j, max_iter);
        return MSR_OK;
    }

    msr_status set_workspace() {
        const int Pn = P();
        std::vector<C> t(Pn);
        for (int k = 0; k < Pn; ++k) {
            const double a = -2.0 * M_PI * (double)k / (double)Pn;
            t[k] = mk_host(std::cos(a), std::sin(a));
        }
        HIPCHK(c, hipMemcpy(tw(), t.data(), sizeof(C) * Pn, hipMemcpyHostToDevice));
        TRY(stage_tables(N(), stwN()));
        TRY(stage_tables(Pn, stwP()));
        if (dict()) {
            std::vector<Taps<R>> tp(kWaveletBases);
            for (int b = 0; b < kWaveletBases; ++b) {
                double h[kMaxTaps];
                const int p = b + 1;
                if (!daubechies_taps(p, h)) return fail(c, MSR_ERR_NUMERIC, "db%d filter is not orthonormal", p);
                tp[b].L = 2 * p;
                for (int k = 0; k < kMaxTaps; ++k) {
                    const bool in = k < 2 * p;
                    tp[b].h[k] = in ? (R)h[k] : (R)0;
                    tp[b].g[k] = in ? (R)(((k & 1) ? -1.0 : 1.0) * h[2 * p - 1 - k]) : (R)0;
                }
            }
            HIPCHK(c, hipMemcpy(taps(0), tp.data(), sizeof(Taps<R>) * kWaveletBases, hipMemcpyHostToDevice));
        }
        return MSR_OK;
    }
    // The FFT stage twiddle rows (w, w^2, w^4, w^8), w = exp(-2 pi i jm / (NS RD)),
    // of every stage of every E for transforms of length L (stage_offset).
    msr_status stage_tables(int L, C* dst) {
        std::vector<C> t(stage_tables_len(L), mk_host(0.0, 0.0));
        for (int E = 2; E <= 16 && E <= L; E *= 2) {
            const int base = stage_tables_offset(L, E);
            for (int NS = 1; NS < L; NS *= stage_radix(L, E, NS)) {
                if (NS == 1) continue;
                const int RD = stage_radix(L, E, NS);
                const int off = base + stage_offset(L, E, NS);
                for (int jm = 0; jm < NS; ++jm)
                    for (int q = 0; q < 4; ++q) {
                        const double ang = -2.0 * M_PI * (double)jm * (double)(1 << q) / ((double)NS * RD);
                        t[off + 4 * jm + q] = mk_host(std::cos(ang), std::sin(ang));
                    }
            }
        }
        HIPCHK(c, hipMemcpy(dst, t.data(), sizeof(C) * t.size(), hipMemcpyHostToDevice));
        return MSR_OK;
    }
    static C mk_host(double x, double y) {
        C r;
        r.x = (R)x;
        r.y = (R)y;
        return r;
    }

    msr_status set_dirty_psf(int step, const R* dirty_in, const R* psf, hipStream_t s) {
        const int Pn = P();
        HIPCHK(c, hipMemcpyAsync(dirty(step), dirty_in, c->sh.rs * c->sh.img_elems, hipMemcpyDeviceToDevice, s));
        R centre = 0;
        HIPCHK(c, hipMemcpyAsync(&centre, psf + (size_t)(Pn / 2) * Pn + Pn / 2, sizeof(R), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (!(std::fabs((double)centre - 1.0) <= 1e-5))
            return fail(c, MSR_ERR_INVALID, "PSF value at (P/2, P/2) is %g, expected 1", (double)centre);
        // h_hat = F(ifftshift PSF): row pass (P rows, unpadded), then column pass in place.
        C* tmpspec = SB();  // SB and SC are contiguous and hold P x Cpad_psf
        RowArgs<R> ra{};
        ra.spec_out = tmpspec;
        ra.tw = tw();
        ra.tws = stwP();
        ra.partials = partials();
        ra.NR = Pn;
        ra.K_out = c->sh.Cfull;
        opp->row_loadshift_fwd(ra, EpiLoadShift<R>{psf, Pn}, s);
        LAUNCHCHK(c);
        ColArgs<R> ca{};
        ca.in_scale = (R)1;
        ca.spec_in = tmpspec;
        ca.spec_out = tmpspec;
        ca.tw = tw();
        ca.tws = stwP();
        ca.partials = partials();
        ca.NR = Pn;
        ca.K = c->sh.Cfull;
        opp->col_forward(ca, ModeForward<R>{}, s);
        LAUNCHCHK(c);
        R* h = hh(step);
        hipLaunchKernelGGL(psf_extract<R>, dim3(c->sh.Cfull), dim3(256), 0, s, tmpspec, c->sh.Tpsf, Pn, c->sh.T, h,
                           colmax(), partials());
        LAUNCHCHK(c);
        if (c->sh.Cpad > c->sh.Cfull) {
            hipLaunchKernelGGL(zero_hh_cols<R>, dim3(blocks_for(Pn)), dim3(256), 0, s, h, Pn, c->sh.T, c->sh.Cfull,
                               c->sh.Cpad);
            LAUNCHCHK(c);
        }
        std::vector<double> cm(c->sh.Cfull);
        std::vector<double> part(2 * (size_t)c->sh.Cfull);
        HIPCHK(c, hipMemcpyAsync(cm.data(), colmax(), sizeof(double) * c->sh.Cfull, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(part.data(), partials(), sizeof(double) * 2 * c->sh.Cfull, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        double mre = 0.0, mim = 0.0;
        for (int k = 0; k < c->sh.Cfull; ++k) {
            mre = std::max(mre, part[2 * k]);
            mim = std::max(mim, part[2 * k + 1]);
        }
        if (!(mre > 0) || !std::isfinite(mre)) return fail(c, MSR_ERR_INVALID, "PSF spectrum is zero or not finite");
        if (mim > 1e-4 * mre)
            return fail(c, MSR_ERR_INVALID, "PSF is not point symmetric: max|Im h| / max|h| = %g", mim / mre);
        int keep = c->sh.Cfull;
        if (c->cfg.prune_tol > 0) {
            const double thr = c->cfg.prune_tol * mre;
            keep = 1;
            for (int k = 0; k < c->sh.Cfull; ++k)
                if (cm[k] > thr) keep = k + 1;
        }
        c->K[step - 1] = keep;
        // Pruned columns are exactly zero (a batched launch may cover more
        // columns than this channel keeps).
        if (keep < c->sh.Cpad) {
            hipLaunchKernelGGL(zero_hh_cols<R>, dim3(blocks_for(Pn)), dim3(256), 0, s, h, Pn, c->sh.T, keep, c->sh.Cpad);
            LAUNCHCHK(c);
        }
        c->have_psf[step - 1] = true;
        c->have_theta[step - 1] = false;
        return MSR_OK;
    }

    // Before the iterations of `step`: theta (power iteration unless set),
    // beta_0 = beta_{-1} = x0 (or 0), the low-resolution constraint (step 2) and
    // the spectrum of alpha_0.  Returns mu = 1 / theta.  ka / kl (0: this
    // context's own counts) widen the spectra of alpha_0 and of the constraint
    // to the columns a batched launch reads.
    msr_status prepare(int step, const R* low_res, const R* x0, double* mu, hipStream_t s, int ka = 0, int kl = 0) {
        if (!c->have_theta[step - 1]) {
            double th = 0.0;
            TRY(power_iteration(step, 200, 1e-6, &th, nullptr, s));
            if (!(th > 0)) return fail(c, MSR_ERR_NUMERIC, "zero Lipschitz constant");
            c->theta[step - 1] = kThetaMargin * th;
            c->have_theta[step - 1] = true;
        }
        *mu = 1.0 / c->theta[step - 1];
        if (it64()) {
            // beta_0 = beta_{-1} = (double) x0; alpha_0's spectrum from x0 itself
            const size_t n = c->sh.img_elems;
            if (x0) {
                hipLaunchKernelGGL((convert_image<double, R>), dim3(blocks_for(n)), dim3(256), 0, s, beta64(0), x0, n);
                LAUNCHCHK(c);
            } else {
                HIPCHK(c, hipMemsetAsync(beta64(0), 0, sizeof(double) * n, s));
                HIPCHK(c, hipMemsetAsync(tmp(0), 0, c->sh.rs * n, s));
            }
            HIPCHK(c, hipMemcpyAsync(beta64(1), beta64(0), sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            if (step == 2) TRY(fwd_image(2, low_res, (R)1, SL(), std::max(kl, KLs()), s));
            return fwd_image(step, x0 ? x0 : tmp(0), (R)1, SA(), std::max(ka, KA(step)), s);
        }
        const size_t nb = c->sh.rs * c->sh.img_elems;
        if (x0) {
            HIPCHK(c, hipMemcpyAsync(beta(0), x0, nb, hipMemcpyDeviceToDevice, s));
        } else {
            HIPCHK(c, hipMemsetAsync(beta(0), 0, nb, s));
        }
        HIPCHK(c, hipMemcpyAsync(beta(1), beta(0), nb, hipMemcpyDeviceToDevice, s));
        if (step == 2) TRY(fwd_image(2, low_res, (R)1, SL(), std::max(kl, KLs()), s));
        return fwd_image(step, beta(0), (R)1, SA(), std::max(ka, KA(step)), s);
    }

    // After `done` iterations: the exact objective of beta_done (F, data term,
    // l1 norm), the model copied out and, if asked, the step's image
    // beta + (i~ - H beta) (i_L in step 1, Sect. 3.2; the final image in step 2, Sect. 3.3).
    msr_status finish(int step, double lambda, int done, R* model_out, R* image_out, double F[3], hipStream_t s) {
        const size_t nb = c->sh.rs * c->sh.img_elems;
        const R* bK = beta(done);
        if (it64()) {  // the model is the float64 iterate rounded once
            const size_t n = c->sh.img_elems;
            hipLaunchKernelGGL((convert_image<R, double>), dim3(blocks_for(n)), dim3(256), 0, s, model_out,
                               (const double*)beta64(done), n);
            LAUNCHCHK(c);
            bK = model_out;
        }
        TRY(objective_at(step, lambda, bK, F, s));
        if (!std::isfinite(F[0])) return fail(c, MSR_ERR_NUMERIC, "objective is not finite after %d iterations", done);
        if (bK != model_out) HIPCHK(c, hipMemcpyAsync(model_out, bK, nb, hipMemcpyDeviceToDevice, s));
        if (image_out) {
            // i_L = beta + (i~ - H beta) = beta - r
            TRY(fwd_image(step, bK, (R)1, SB(), c->K[step - 1], s));
            TRY(col_psf(step, SB(), SC(), s));
            opr(step)->row_resid(row_args(SC(), c->K[step - 1], nullptr, 0, nullptr, 0),
                                 EpiResid<R>{dirty(step), tmp(0), N()}, s);
            LAUNCHCHK(c);
            const size_t n = c->sh.img_elems;
            hipLaunchKernelGGL(image_axpby<R>, dim3(blocks_for(n)), dim3(256), 0, s, image_out, bK, (const R*)tmp(0),
                               (R)1, (R)-1, n);
            LAUNCHCHK(c);
        }
        return MSR_OK;
    }

    // ---- wavelet dictionary ------------------------------------------------
    // x = W a (a: 8 coefficient arrays of N x N), levels coarsest first.
    msr_status synthesize(const R* a, R* x, hipStream_t s) {
        const int n = N();
        const long long q = (long long)(c->sh.img_elems / 4);
        const R* ll = nullptr;
        int ld_ll = 0;
        for (int j = kWaveletLevels - 1; j >= 0; --j) {
            const int sj = n >> j;
            IdwtArgs<R> p{};
            p.ll = ll;
            p.ll_bs = q;
            p.ld_ll = ld_ll;
            p.coef = a;
            p.cstride = (long long)c->sh.img_elems;
            p.ldc = n;
            p.s = sj;
            p.taps = taps(0);
            if (j == 0) {  // all bases summed into x
                p.out = x;
                p.ld_out = n;
                p.bpb = kWaveletBases;
            } else {
                R* o = wscr((kWaveletLevels - 1 - j) & 1);
                p.out = o;
                p.out_bs = q;
                p.ld_out = sj;
                p.bpb = 1;
                ll = o;
                ld_ll = sj;
            }
            const unsigned tiles = (unsigned)(((sj + kIdwtTC - 1) / kIdwtTC) * ((sj + kIdwtTR - 1) / kIdwtTR));
            hipLaunchKernelGGL(idwt_level<R>, dim3(tiles, 1, kWaveletBases / p.bpb), dim3(kWavThreads), 0, s, p);
            LAUNCHCHK(c);
        }
        return MSR_OK;
    }
    // W^T x, every coefficient through `epi` (a store, or the fused FISTA step).
    msr_status analyze(const R* x, const WavEpi<R>& epi, hipStream_t s) {
        const int n = N();
        const long long q = (long long)(c->sh.img_elems / 4);
        const R* in = x;
        long long in_bs = 0;
        int ld_in = n;
        for (int j = 0; j < kWaveletLevels; ++j) {
            const int sj = n >> j;
            DwtArgs<R> p{};
            p.in = in;
            p.in_bs = in_bs;
            p.ld_in = ld_in;
            p.s = sj;
            p.bpb = j == 0 ? kWaveletBases : 1;  // level 0: the image is every basis's input
            p.taps = taps(0);
            p.epi = epi;
            if (j < kWaveletLevels - 1) {
                R* o = wscr(j & 1);
                p.ll = o;
                p.ll_bs = q;
                p.ld_ll = sj / 2;
                in = o;
                in_bs = q;
                ld_in = sj / 2;
            }
            const unsigned tiles = (unsigned)((sj / 2 + kDwtT - 1) / kDwtT);
            hipLaunchKernelGGL(dwt_level<R>, dim3(tiles * tiles, 1, kWaveletBases / p.bpb), dim3(kWavThreads), 0, s, p);
            LAUNCHCHK(c);
        }
        return MSR_OK;
    }
    WavEpi<R> store_epi(R* out, R scale) const {
        WavEpi<R> e{};
        e.cstride = (long long)c->sh.img_elems;
        e.ldc = N();
        e.mode = 0;
        e.out = out;
        e.scale = scale;
        return e;
    }
    msr_status coeff_l1(const R* a, double* host, hipStream_t s) {
        const size_t n = cn();
        const int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
        hipLaunchKernelGGL(image_sums<R>, dim3(blocks), dim3(256), 0, s, a, (const R*)nullptr, n, 0, partials());
        LAUNCHCHK(c);
        return reduce(blocks, 1, 8, host, s);
    }
    // F(beta) = data(W beta) + lambda ||beta||_1; out: F, data, ||beta||_1.
    msr_status dict_objective(int step, double lambda, const R* beta, double out[3], hipStream_t s) {
        TRY(synthesize(beta, wx(), s));
        TRY(objective_at(step, lambda, wx(), out, s));
        double l1 = 0.0;
        TRY(coeff_l1(beta, &l1, s));
        out[2] = l1;
        out[0] = out[1] + lambda * l1;
        return MSR_OK;
    }
    // One FISTA iteration on the coefficients (the gradient of Eq. 11 / 12 in
    // alpha is 2 W^T (image-domain half-gradient at W alpha)).
    msr_status dict_iterate(int step, int k, double mu, double lambda, hipStream_t s) {
        TRY(synthesize(cA(), wx(), s));
        TRY(fwd_image(step, wx(), (R)1, SA(), KA(step), s));
        TRY(grad_chain(step, dirty(step), true, s));
        RowArgs<R> a = step == 1 ? row_args(SB(), Ks(1), nullptr, 0, nullptr, 0)
                                 : row_args(SB(), Ks(2), SG(), KLs(), nullptr, 0);
        opr(step)->row_store(a, EpiStore<R>{wx(), N(), (R)1}, s);
        LAUNCHCHK(c);
        WavEpi<R> e = store_epi(nullptr, (R)1);
        e.mode = 1;
        e.b1 = coef(k - 1);
        e.b2 = coef(k);
        e.a = cA();
        e.two_mu = (R)(2.0 * mu);
        e.thr = (R)(mu * lambda);
        e.t_prev = (R)momentum(k - 1);
        e.t_cur = (R)momentum(k);
        return analyze(wx(), e, s);
    }
    msr_status dict_solve(int step, const msr_solve* opt, const R* low_res, const R* x0, R* model_out, R* image_out,
                          msr_result* res, hipStream_t s, int K0 = 0, bool resuming = false) {
        double mu = 0.0;
        if (resuming) {
            TRY(resume(step, K0, low_res, &mu, s));
        } else {
            if (!c->have_theta[step - 1]) {
                double th = 0.0;
                TRY(power_iteration(step, 200, 1e-6, &th, nullptr, s));
                if (!(th > 0)) return fail(c, MSR_ERR_NUMERIC, "zero Lipschitz constant");
                c->theta[step - 1] = kThetaMargin * th;
                c->have_theta[step - 1] = true;
            }
            mu = 1.0 / c->theta[step - 1];
            const size_t cb = c->sh.rs * cn();
            if (x0) {  // beta_0 = W^T x0 / M, so that W beta_0 = x0
                TRY(analyze(x0, store_epi(coef(0), (R)(1.0 / kWaveletBases)), s));
            } else {
                HIPCHK(c, hipMemsetAsync(coef(0), 0, cb, s));
            }
            HIPCHK(c, hipMemcpyAsync(coef(1), coef(0), cb, hipMemcpyDeviceToDevice, s));
            HIPCHK(c, hipMemcpyAsync(cA(), coef(0), cb, hipMemcpyDeviceToDevice, s));
            if (step == 2) TRY(set_low_res(low_res, s));
        }
        const double theta = c->theta[step - 1];
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, s));
        const bool rule = opt->check_every > 0 && opt->f_ref != 0.0 && opt->tol > 0;
        double F[3] = {0, 0, 0};
        int k = 0;
        bool conv = false;
        double ttt = -1.0;
        msr_status st = MSR_OK;
        const int kend = K0 + opt->max_iters;
        for (k = K0 + 1; k <= kend; ++k) {
            if ((st = dict_iterate(step, k, mu, opt->lambda, s)) != MSR_OK) break;
            if (opt->check_every > 0 && (k % opt->check_every == 0)) {
                if ((st = dict_objective(step, opt->lambda, coef(k), F, s)) != MSR_OK) break;
                if (!std::isfinite(F[0])) {
                    st = fail(c, MSR_ERR_NUMERIC, "objective is not finite at iteration %d", k);
                    break;
                }
                if (rule && (F[0] - opt->f_ref) / std::fabs(opt->f_ref) <= opt->tol) {
                    conv = true;
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                        hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                        ttt = ms;
                    break;
                }
            }
        }
        const int done = std::min(k, kend);
        float ms = 0.f;
        if (st == MSR_OK) {
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = fail(c, MSR_ERR_HIP, "event timing failed");
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (res) res->iters = done - K0;
        if (st != MSR_OK) return st;
        TRY(dict_objective(step, opt->lambda, coef(done), F, s));
        if (!std::isfinite(F[0])) return fail(c, MSR_ERR_NUMERIC, "objective is not finite after %d iterations", done);
        // the image W beta is in wx after dict_objective
        HIPCHK(c, hipMemcpyAsync(model_out, wx(), c->sh.rs * c->sh.img_elems, hipMemcpyDeviceToDevice, s));
        if (image_out) {
            TRY(residual_image(step, dirty(step), wx(), image_out, s));  // i~ - H W beta
            TRY(axpby(image_out, image_out, wx(), (R)1, (R)1, s));     // + W beta
        }
        HIPCHK(c, hipStreamSynchronize(s));
        c->state_step = step;
        c->state_k = done;
        if (res) {
            res->iters = done - K0;
            res->converged = conv ? 1 : 0;
            res->objective = F[0];
            res->data_term = F[1];
            res->l1_norm = F[2];
            res->theta = theta;
            res->elapsed_ms = ms;
            res->time_to_tol_ms = ttt;
        }
        return MSR_OK;
    }

    // Continuing from a loaded state (beta_K, beta_{K-1}): theta, the
    // constraint, and alpha_K = beta_K + t_K (beta_K - beta_{K-1}) formed as
    // the update epilogue forms it (into the spectrum SA, or the coefficient
    // array alpha with the dictionary).
    msr_status resume(int step, int K, const R* low_res, double* mu, hipStream_t s) {
        if (!c->have_theta[step - 1]) {
            double th = 0.0;
            TRY(power_iteration(step, 200, 1e-6, &th, nullptr, s));
            if (!(th > 0)) return fail(c, MSR_ERR_NUMERIC, "zero Lipschitz constant");
            c->theta[step - 1] = kThetaMargin * th;
            c->have_theta[step - 1] = true;
        }
        *mu = 1.0 / c->theta[step - 1];
        if (step == 2) TRY(set_low_res(low_res, s));
        const size_t n = dict() ? cn() : c->sh.img_elems;
        R* a = dict() ? cA() : tmp(0);
        if (it64()) {
            hipLaunchKernelGGL(momentum_point_it64<R>, dim3(blocks_for(n)), dim3(256), 0, s, a,
                               (const double*)beta64(K), (const double*)beta64(K - 1), momentum(K), n);
        } else {
            const R* bk = dict() ? coef(K) : beta(K);
            const R* bp = dict() ? coef(K - 1) : beta(K - 1);
            hipLaunchKernelGGL(momentum_point<R>, dim3(blocks_for(n)), dim3(256), 0, s, a, bk, bp, (R)momentum(K), n);
        }
        LAUNCHCHK(c);
        if (!dict()) TRY(fwd_image(step, a, (R)1, SA(), KA(step), s));
        return MSR_OK;
    }

    msr_status solve(int step, const msr_solve* opt, const R* low_res, const R* x0, R* model_out, R* image_out,
                     msr_result* res, hipStream_t s) {
        const int K0 = std::max(c->resume_k[step - 1], 0);
        const bool resuming = c->resume_k[step - 1] >= 0;
        c->resume_k[step - 1] = -1;
        c->state_step = 0;
        if (dict()) return dict_solve(step, opt, low_res, x0, model_out, image_out, res, s, K0, resuming);
        double mu = 0.0;
        if (resuming)
            TRY(resume(step, K0, low_res, &mu, s));
        else
            TRY(prepare(step, low_res, x0, &mu, s));
        const double theta = c->theta[step - 1];

        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, s));
        const bool rule = opt->check_every > 0 && opt->f_ref != 0.0 && opt->tol > 0;
        double F[3] = {0, 0, 0};
        int k = 0;
        bool conv = false;
        double ttt = -1.0;
        msr_status st = MSR_OK;
        const int kend = K0 + opt->max_iters;
        for (k = K0 + 1; k <= kend; ++k) {
            if ((st = iterate(step, k, mu, opt->lambda, s)) != MSR_OK) break;
            if (opt->check_every > 0 && (k % opt->check_every == 0)) {
                const R* bk = nullptr;
                if ((st = beta_r(k, &bk, s)) != MSR_OK) break;
                if ((st = objective_at(step, opt->lambda, bk, F, s)) != MSR_OK) break;
                if (!std::isfinite(F[0])) {
                    st = fail(c, MSR_ERR_NUMERIC, "objective is not finite at iteration %d", k);
                    break;
                }
                if (rule && (F[0] - opt->f_ref) / std::fabs(opt->f_ref) <= opt->tol) {
                    conv = true;
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                        hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                        ttt = ms;
                    break;
                }
            }
        }
        const int done = std::min(k, kend);
        float ms = 0.f;
        if (st == MSR_OK) {
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = fail(c, MSR_ERR_HIP, "event timing failed");
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (res) res->iters = done - K0;
        if (st != MSR_OK) return st;
        TRY(finish(step, opt->lambda, done, model_out, image_out, F, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->state_step = step;
        c->state_k = done;
        if (res) {
            res->iters = done - K0;
            res->converged = conv ? 1 : 0;
            res->objective = F[0];
            res->data_term = F[1];
            res->l1_norm = F[2];
            res->theta = theta;
            res->elapsed_ms = ms;
            res->time_to_tol_ms = ttt;
        }
        return MSR_OK;
    }

    // out = U small (Sect. 6.1, the down-sampled low-resolution image):
    // K small K^T with K[n][j] = k((n - d j) mod N), where
    //   k(t) = (1/N) [1 + 2 sum_{q=1}^{m/2-1} cos(2 pi q t / N) + cos(pi m t / N)],  m = N / d
    // (the DFT of small zero-filled to N x N, the Nyquist cell split in
    // halves), evaluated through the Dirichlet closed form
    //   1 + 2 sum_{q=1}^{M} cos(q th) = sin((M + 1/2) th) / sin(th / 2).
    msr_status upsample(int d, const R* small, R* out, hipStream_t s) {
        const int n = N(), m = n / d;
        std::vector<R> tab(n);
        for (int t = 0; t < n; ++t) {
            const double th = 2.0 * M_PI * t / n;
            const double dir = t == 0 ? (double)(m - 1) : std::sin((m / 2 - 0.5) * th) / std::sin(0.5 * th);
            tab[t] = (R)((dir + std::cos(0.5 * m * th)) / n);
        }
        R* dtab = tmp(0);
        R* T = tmp(1);  // small K^T: m x n
        HIPCHK(c, hipMemcpyAsync(dtab, tab.data(), sizeof(R) * n, hipMemcpyHostToDevice, s));
        const unsigned bn = (unsigned)((n + kRsT - 1) / kRsT), bm = (unsigned)((m + kRsT - 1) / kRsT);
        hipLaunchKernelGGL((resample_product<R, DenseOperand<R>, KernelCols<R>>), dim3(bn, bm), dim3(kRsThreads), 0, s,
                           DenseOperand<R>{small, m}, KernelCols<R>{dtab, n - 1, d}, T, n, m, n, m);
        LAUNCHCHK(c);
        hipLaunchKernelGGL((resample_product<R, KernelRows<R>, DenseOperand<R>>), dim3(bn, bn), dim3(kRsThreads), 0, s,
                           KernelRows<R>{dtab, n - 1, d}, DenseOperand<R>{T, n}, out, n, n, n, m);
        LAUNCHCHK(c);
        HIPCHK(c, hipStreamSynchronize(s));  // also keeps `tab` alive until its copy is done
        return MSR_OK;
    }

    // out = y - H_step x, in the image domain (may alias y).
    msr_status residual_image(int step, const R* y, const R* x, R* out, hipStream_t s) {
        TRY(fwd_image(step, x, (R)1, SB(), c->K[step - 1], s));
        TRY(col_psf(step, SB(), SC(), s));
        opr(step)->row_resid(row_args(SC(), c->K[step - 1], nullptr, 0, nullptr, 0), EpiResid<R>{y, out, N()}, s);
        LAUNCHCHK(c);
        return axpby(out, out, out, (R)-1, (R)0, s);  // (H x - y) -> y - H x
    }
    msr_status axpby(R* out, const R* x, const R* y, R a, R b, hipStream_t s) {
        const size_t n = c->sh.img_elems;
        hipLaunchKernelGGL(image_axpby<R>, dim3(blocks_for(n)), dim3(256), 0, s, out, x, y, a, b, n);
        LAUNCHCHK(c);
        return MSR_OK;
    }

    // `cycles` major cycles of step s (Sect. 3.2 / 3.3) with the residual image
    // of cycle n formed in the image domain, i~_n = i~_1 - H sum_{j<n} i_j;
    // lambda_n = cl ||i~_n|| 2^(n-1); in step 2 the constraint is
    // l - sum_{j<n} i_j.  Each cycle runs `iters` FISTA iterations from zero.
    // model_out = sum_n i_n, image_out = i~_{N+1} + sum_n i_n.  The context's
    // dirty image is restored before returning.
    msr_status multi_cycle(int step, int cycles, double cl, int iters, const R* low_res, R* model_out, R* image_out,
                           msr_result* res, hipStream_t s) {
        if (c->resume_k[step - 1] >= 0)
            return fail(c, MSR_ERR_STATE, "a loaded FISTA state is waiting for a solve of step %d", step);
        c->state_step = 0;
        const size_t nb = c->sh.rs * c->sh.img_elems;
        R* d = dirty(step);
        R *d0 = mc(0), *msum = mc(1), *lcur = mc(2), *cyc = mc(3);
        HIPCHK(c, hipMemcpyAsync(d0, d, nb, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemsetAsync(msum, 0, nb, s));
        msr_status st = MSR_OK;
        for (int k = 1; k <= cycles && st == MSR_OK; ++k) {
            if (k > 1 && (st = residual_image(step, d0, msum, d, s)) != MSR_OK) break;
            double s2 = 0.0;
            if ((st = image_reduce(d, nullptr, 1, &s2, s)) != MSR_OK) break;
            msr_solve opt{};
            opt.lambda = cl * std::sqrt(s2) * std::ldexp(1.0, k - 1);
            opt.max_iters = iters;
            const R* l = nullptr;
            if (step == 2) {
                if ((st = axpby(lcur, low_res, msum, (R)1, (R)-1, s)) != MSR_OK) break;
                l = lcur;
            }
            if ((st = solve(step, &opt, l, nullptr, cyc, nullptr, res ? &res[k - 1] : nullptr, s)) != MSR_OK) break;
            st = axpby(msum, msum, cyc, (R)1, (R)1, s);
        }
        if (st == MSR_OK) st = residual_image(step, d0, msum, d, s);
        if (st == MSR_OK && image_out) st = axpby(image_out, d, msum, (R)1, (R)1, s);
        if (st == MSR_OK && model_out) {
            const hipError_t e = hipMemcpyAsync(model_out, msum, nb, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) st = fail(c, MSR_ERR_HIP, "model copy: %s", hipGetErrorString(e));
        }
        const hipError_t e = hipMemcpyAsync(d, d0, nb, hipMemcpyDeviceToDevice, s);  // restore i~_1
        if (st == MSR_OK && e != hipSuccess) st = fail(c, MSR_ERR_HIP, "restore: %s", hipGetErrorString(e));
        if (st == MSR_OK) HIPCHK(c, hipStreamSynchronize(s));
        return st;
    }

    msr_status gradient(int step, const R* x, const R* low_res, R* g, hipStream_t s) {
        if (step == 2) TRY(set_low_res(low_res, s));
        TRY(fwd_image(step, x, (R)1, SA(), KA(step), s));
        TRY(grad_chain(step, dirty(step), true, s));
        RowArgs<R> a = step == 1 ? row_args(SB(), c->K[0], nullptr, 0, nullptr, 0)
                                 : row_args(SB(), c->K[1], SG(), c->KL, nullptr, 0);
        opr(step)->row_store(a, EpiStore<R>{g, N(), (R)2}, s);
        LAUNCHCHK(c);
        HIPCHK(c, hipStreamSynchronize(s));
        return MSR_OK;
    }

    msr_status apply_psf(int step, const R* x, R* out, hipStream_t s) {
        TRY(fwd_image(step, x, (R)1, SB(), c->K[step - 1], s));
        TRY(col_psf(step, SB(), SC(), s));
        opr(step)->row_store(row_args(SC(), c->K[step - 1], nullptr, 0, nullptr, 0), EpiStore<R>{out, N(), (R)1}, s);
        LAUNCHCHK(c);
        HIPCHK(c, hipStreamSynchronize(s));
        return MSR_OK;
    }

    msr_status get_spectrum(int step, double* host_out, hipStream_t s) {
        const int Pn = P(), T = c->sh.T, Cf = c->sh.Cfull;
        std::vector<R> h(c->sh.hh_elems);
        HIPCHK(c, hipMemcpyAsync(h.data(), hh(step), sizeof(R) * h.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const double p2 = (double)Pn * Pn;
        const int K = c->K[step - 1];
        for (int ky = 0; ky < Pn; ++ky)
            for (int kx = 0; kx < Cf; ++kx)
                host_out[(size_t)ky * Cf + kx] = kx < K ? (double)h[((size_t)(kx / T) * Pn + ky) * T + kx % T] * p2 : 0.0;
        return MSR_OK;
    }

    msr_status sigma2(const R* img, double* out, hipStream_t s) {
        const int n = N();
        const size_t nw = (size_t)(n - 4) * (n - 4);
        const int blocks = (int)std::min<size_t>(1024, (nw + 255) / 256);
        hipLaunchKernelGGL(window_variance<R>, dim3(blocks), dim3(256), 0, s, img, n, partials());
        LAUNCHCHK(c);
        double tot = 0.0;
        TRY(reduce(blocks, 1, 8, &tot, s));
        *out = tot / (double)nw;
        return MSR_OK;
    }

    // For each step whose PSF is set, times every built variant of the column
    // PSF pass and of the fused update row pass on that step's shapes and keeps
    // the fastest of each.  times[2v], times[2v+1]: step-1 column / row ms.
    msr_status autotune(int reps, double* times, hipStream_t s) {
        for (int step = 1; step <= 2; ++step) {
            if (!c->have_psf[step - 1]) continue;
            double best_c = 1e30, best_r = 1e30;
            int vc = 0, vr = 0;
            for (int v = 0; v < kVariants; ++v) {
                const Ops<R>* o = ops_for<R>(N(), c->sh.padded, v);
                if (!o || !o->row_update_fwd) continue;
                c->var_row[step - 1] = v;
                c->var_col[step - 1] = v;
                Impl<R> im(c);
                double ms = 0.0;
                TRY(im.time_pass(0, step, reps, &ms, nullptr, nullptr, s));
                if (times && step == 1) times[2 * v] = ms;
                if (ms < best_c) best_c = ms, vc = v;
                TRY(im.time_pass(2, step, reps, &ms, nullptr, nullptr, s));
                if (times && step == 1) times[2 * v + 1] = ms;
                if (ms < best_r) best_r = ms, vr = v;
            }
            c->var_row[step - 1] = vr;
            c->var_col[step - 1] = vc;
            if (step == 2 && c->have_filters) {
                double best_f = 1e30;
                int vf = vc;
                for (int v = 0; v < kVariants; ++v) {
                    const Ops<R>* o = ops_for<R>(N(), c->sh.padded, v);
                    if (!o || !o->row_update_fwd) continue;
                    c->var_filt = v;
                    Impl<R> im(c);
                    double ms = 0.0;
                    TRY(im.time_pass(3, 2, reps, &ms, nullptr, nullptr, s));
                    if (ms < best_f) best_f = ms, vf = v;
                }
                c->var_filt = vf;
            }
        }
        return MSR_OK;
    }

    // Times one pass of an iteration of `step` (current state, `reps` launches)
    // and returns its algorithmic bytes and flops per launch.  which: 0 = column
    // PSF pass, 1 = residual row pass, 2 = fused update row pass, 3 = the step-2
    // low-band filter pass (C_w and C_{g_L^2} on K_L columns each).  Flops count
    // 5 n log2 n per complex transform of length n (P here), one inverse and one
    // forward transform per row pair or per column.
    msr_status time_pass(int which, int step, int reps, double* ms_out, double* bytes_out, double* flops_out,
                         hipStream_t s) {
        const int Nn = N(), Pn = P(), K = c->K[step - 1];
        const int Kin2 = step == 2 ? c->KL : 0;
        const int Kout = step == 2 ? KA(2) : K;
        const double es = (double)c->sh.cs, rs = (double)c->sh.rs;
        const double img = (double)Nn * Nn * rs;
        const double fft_p = 5.0 * Pn * std::log2((double)Pn);
        c->state_step = 0;                          // the passes below overwrite the iterates
        c->resume_k[0] = c->resume_k[1] = -1;
        WavEpi<R> upd = store_epi(nullptr, (R)1);  // which 5: the fused coefficient update
        upd.mode = 1;
        upd.b1 = coef(0);
        upd.b2 = coef(1);
        upd.a = cA();
        auto launch = [&]() -> msr_status {
            if (which == 4) return synthesize(cA(), wx(), s);
            if (which == 5) return analyze(wx(), upd, s);
            if (which == 0) return col_psf(step, SA(), SB(), s);
            if (which == 3) return col_filt_wl(SL(), s);
            if (which == 1) {
                opr(step)->row_resid_fwd(row_args(SB(), K, nullptr, 0, SC(), K), EpiResid<R>{dirty(step), nullptr, Nn},
                                         s);
                LAUNCHCHK(c);
                return MSR_OK;
            }
            if (it64()) {
                EpiUpdate<R, double> u{};
                u.b1 = beta64(0);
                u.b2 = beta64(1);
                u.ld = Nn;
                u.positivity = c->cfg.positivity;
                opr(step)->row_update_fwd_it64(row_args(SB(), K, Kin2 ? SL() : nullptr, Kin2, SC(), Kout), u, s);
                LAUNCHCHK(c);
                return MSR_OK;
            }
            EpiUpdate<R> u{};
            u.b1 = beta(0);
            u.b2 = beta(1);
            u.ld = Nn;
            u.positivity = c->cfg.positivity;
            opr(step)->row_update_fwd(row_args(SB(), K, Kin2 ? SL() : nullptr, Kin2, SC(), Kout), u, s);
            LAUNCHCHK(c);
            return MSR_OK;
        };
        double bytes, flops;
        // a 2-D level of a basis with L taps costs 4 L s^2 flops either way
        const double lev = (double)Nn * Nn * (1.0 + 1.0 / 4 + 1.0 / 16 + 1.0 / 64);
        const double wav_flops = 4.0 * lev * (double)(kWaveletBases * (kWaveletBases + 1));  // sum of L = 2 + .. + 16
        if (which >= 4) {
            const size_t cb = c->sh.rs * cn();
            HIPCHK(c, hipMemsetAsync(coef(0), 0, cb, s));
            HIPCHK(c, hipMemsetAsync(coef(1), 0, cb, s));
            HIPCHK(c, hipMemsetAsync(cA(), 0, cb, s));
            HIPCHK(c, hipMemsetAsync(wx(), 0, c->sh.rs * c->sh.img_elems, s));
        }
        if (which == 4) {  // read alpha (M N^2), write x (N^2)
            bytes = (kWaveletBases + 1.0) * img;
            flops = wav_flops;
        } else if (which == 5) {  // read the gradient image, beta_{k-1}, beta_{k-2}; write beta_k, alpha_k
            bytes = (1.0 + 4.0 * kWaveletBases) * img;
            flops = wav_flops;
        } else if (which == 0) {
            bytes = 2.0 * Nn * K * es + (double)Pn * K * rs;
            flops = 2.0 * K * fft_p;
        } else if (which == 3) {
            bytes = 5.0 * Nn * Kin2 * es;  // C_w: SC in, SB out; C_{g_L^2}: SA, SL in, SG out
            flops = 4.0 * Kin2 * fft_p;
        } else if (which == 1) {
            bytes = 2.0 * Nn * K * es + img;
            flops = 2.0 * (Nn / 2) * fft_p;
        } else {
            bytes = (double)Nn * (K + Kin2 + Kout) * es + 3 * img;
            flops = 2.0 * (Nn / 2) * fft_p;
        }
        TRY(launch());  // warm
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, hipEventRecord(e0, s));
        msr_status st = MSR_OK;
        for (int r = 0; r < reps && st == MSR_OK; ++r) st = launch();
        float ms = 0.f;
        if (st == MSR_OK) {
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = fail(c, MSR_ERR_HIP, "event timing failed");
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (st != MSR_OK) return st;
        if (ms_out) *ms_out = ms / reps;
        if (bytes_out) *bytes_out = bytes;
        if (flops_out) *flops_out = flops;
        return MSR_OK;
    }
};

// Runs f(Impl<R>&) in the context's precision.
template <typename F>
msr_status with_impl(msr_ctx* c, F&& f) {
    if (c->sh.prec == 64) {
        Impl<double> im(c);
        return f(im);
    }
    Impl<float> im(c);
    return f(im);
}

// True when the context has a workspace it still owns: a caller workspace,
// or the static workspace of its device not rebound by another context since.
bool ready(msr_ctx* c) {
    if (!c || !c->ws) return false;
    if (!c->ws_static) return true;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static[c->cfg.device].gen == c->ws_gen) return true;
    c->ws = nullptr;  // another context took the array: this one has none now
    c->ws_static = false;
    c->ws_lost = true;
    return false;
}

// The error of a call that found no workspace.
msr_status ws_missing(msr_ctx* c) {
    if (c && c->ws_lost)
        return fail(c, MSR_ERR_STATE, "the static workspace of device %d was bound by another context since", c->cfg.device);
    return fail(c, MSR_ERR_OOM, "no workspace");
}

msr_status check_step(msr_ctx* c, int step, bool need_filters_for_2) {
    if (!ready(c)) return ws_missing(c);
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    if (need_filters_for_2 && step == 2 && !c->have_filters) return fail(c, MSR_ERR_STATE, "set_filters first");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return MSR_OK;
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

int msr_abi_version(void) { return MSR_ABI_VERSION; }

size_t msr_workspace_bytes(const msr_config* cfg) {
    Shapes s;
    if (!make_shapes(cfg, s, nullptr)) return 0;
    return make_layout(s).total;
}

msr_status msr_init(const msr_config* cfg, msr_ctx** out) {
    if (!out) return MSR_ERR_INVALID;
    *out = nullptr;
    Shapes s;
    std::string why;
    if (!make_shapes(cfg, s, &why)) return MSR_ERR_INVALID;
    // The prox of lambda ||alpha||_1 under x = W alpha >= 0 has no closed form.
    if (s.dict && cfg->positivity) return MSR_ERR_UNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return MSR_ERR_INVALID;
    if (hipSetDevice(cfg->device) != hipSuccess) return MSR_ERR_HIP;
    {
        // the static workspace's device address, once per device (an error is
        // reported by msr_set_workspace_static, which looks it up again)
        void* p = nullptr;
        (void)static_workspace_ptr(cfg->device, &p);
    }
    msr_ctx* c = new (std::nothrow) msr_ctx();
    if (!c) return MSR_ERR_OOM;
    c->cfg = *cfg;
    c->sh = s;
    c->lay = make_layout(s);
    *out = c;
    return MSR_OK;
}

void msr_destroy(msr_ctx* ctx) { delete ctx; }

const char* msr_last_error(const msr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

}  // extern "C"

namespace {
// Binds dev (device memory of `bytes` bytes on the context's device, which is
// current) as the context's workspace and fills its constant tables.
msr_status bind_workspace(msr_ctx* c, void* dev, size_t bytes, bool is_static, unsigned long long gen) {
    c->ws = static_cast<char*>(dev);
    c->ws_bytes = bytes;
    c->ws_static = is_static;
    c->ws_gen = gen;
    c->ws_lost = false;
    c->have_psf[0] = c->have_psf[1] = false;
    c->have_theta[0] = c->have_theta[1] = false;
    c->have_filters = false;
    c->state_step = 0;
    c->resume_k[0] = c->resume_k[1] = -1;
    return with_impl(c, [](auto& im) { return im.set_workspace(); });
}
}  // namespace

extern "C" {

msr_status msr_set_workspace(msr_ctx* c, void* dev, size_t bytes) {
    if (!c) return MSR_ERR_INVALID;
    if (!dev || bytes < c->lay.total) return fail(c, MSR_ERR_OOM, "workspace needs %zu bytes", c->lay.total);
    if (reinterpret_cast<uintptr_t>(dev) % kAlign) return fail(c, MSR_ERR_INVALID, "workspace must be 256-byte aligned");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return bind_workspace(c, dev, bytes, false, 0);
}

msr_status msr_set_workspace_static(msr_ctx* c) {
    if (!c) return MSR_ERR_INVALID;
    if (c->lay.total > (size_t)MSR_STATIC_WORKSPACE_BYTES)
        return fail(c, MSR_ERR_OOM, "this configuration needs %zu bytes of workspace; the static workspace holds %zu",
                    c->lay.total, (size_t)MSR_STATIC_WORKSPACE_BYTES);
    if (c->cfg.device >= kMaxDevices) return fail(c, MSR_ERR_INVALID, "device ordinal above %d", kMaxDevices - 1);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    void* p = nullptr;
    const hipError_t e = static_workspace_ptr(c->cfg.device, &p);
    if (e != hipSuccess) return fail(c, MSR_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    unsigned long long gen;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        gen = ++g_static[c->cfg.device].gen;
    }
    return bind_workspace(c, p, (size_t)MSR_STATIC_WORKSPACE_BYTES, true, gen);
}

msr_status msr_set_dirty_psf(msr_ctx* c, int step, const void* dirty, const void* psf, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!dirty || !psf) return fail(c, MSR_ERR_INVALID, "null image");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    c->have_psf[step - 1] = false;
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.set_dirty_psf(step, static_cast<const R*>(dirty), static_cast<const R*>(psf), S(stream));
    });
}

msr_status msr_set_filters(msr_ctx* c, double ell, double delta, double sigma2, double eta2) {
    if (!c) return MSR_ERR_INVALID;
    if (!(delta > 0) || !(sigma2 > 0) || !(eta2 > 0) || !std::isfinite(ell) || !std::isfinite(delta) ||
        !std::isfinite(sigma2) || !std::isfinite(eta2))
        return fail(c, MSR_ERR_INVALID, "need finite ell, delta > 0, sigma2 > 0, eta2 > 0");
    c->ell = ell;
    c->delta = delta;
    c->sigma2 = sigma2;
    c->eta2 = eta2;
    // g_L vanishes for r >= ell + delta: only columns k_x <= ell + delta can be non-zero.
    const double lim = ell + delta;
    int kl = lim < 0 ? 0 : (int)std::floor(lim) + 1;
    c->KL = std::max(1, std::min(kl, c->sh.Cfull));
    c->have_filters = true;
    c->have_theta[1] = false;
    return MSR_OK;
}

msr_status msr_lipschitz(msr_ctx* c, int step, int max_iter, double rtol, double* theta, int* iters, void* stream) {
    TRY(check_step(c, step, true));
    if (max_iter <= 0) max_iter = 200;
    if (!(rtol > 0)) rtol = 1e-6;
    double th = 0.0;
    TRY(with_impl(c, [&](auto& im) { return im.power_iteration(step, max_iter, rtol, &th, iters, S(stream)); }));
    if (theta) *theta = th;
    c->theta[step - 1] = kThetaMargin * th;
    c->have_theta[step - 1] = th > 0;
    return MSR_OK;
}

msr_status msr_set_lipschitz(msr_ctx* c, int step, double theta) {
    if (!c) return MSR_ERR_INVALID;
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!(theta > 0) || !std::isfinite(theta)) return fail(c, MSR_ERR_INVALID, "theta must be positive");
    c->theta[step - 1] = theta;
    c->have_theta[step - 1] = true;
    return MSR_OK;
}

static msr_status solve_entry(msr_ctx* c, int step, const msr_solve* opt, const void* low_res, const void* x0,
                              void* model_out, void* image_out, msr_result* res, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (!opt || !model_out) return fail(c, MSR_ERR_INVALID, "null argument");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    if (step == 2 && (!c->have_filters || !low_res)) return fail(c, MSR_ERR_STATE, "step 2 needs filters and low_res");
    if (opt->max_iters < 0 || !(opt->lambda >= 0) || !std::isfinite(opt->lambda))
        return fail(c, MSR_ERR_INVALID, "bad solve options");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.solve(step, opt, static_cast<const R*>(low_res), static_cast<const R*>(x0), static_cast<R*>(model_out),
                        static_cast<R*>(image_out), res, S(stream));
    });
}

msr_status msr_step1_low_res(msr_ctx* c, const msr_solve* opt, const void* x0, void* model_out, void* image_out,
                             msr_result* res, void* stream) {
    return solve_entry(c, 1, opt, nullptr, x0, model_out, image_out, res, stream);
}

msr_status msr_step2_full_res(msr_ctx* c, const msr_solve* opt, const void* low_res, const void* x0, void* model_out,
                              void* image_out, msr_result* res, void* stream) {
    return solve_entry(c, 2, opt, low_res, x0, model_out, image_out, res, stream);
}

msr_status msr_major_cycles(msr_ctx* c, int step, int cycles, double cl, int iters, const void* low_res,
                            void* model_out, void* image_out, msr_result* res, void* stream) {
    TRY(check_step(c, step, true));
    if (cycles < 1 || iters < 0 || !(cl >= 0) || !std::isfinite(cl) || (step == 2 && !low_res) ||
        (!model_out && !image_out))
        return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (c->sh.it64) return fail(c, MSR_ERR_UNSUPPORTED, "major cycles store float32 iterates");
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.multi_cycle(step, cycles, cl, iters, static_cast<const R*>(low_res), static_cast<R*>(model_out),
                              static_cast<R*>(image_out), res, S(stream));
    });
}

msr_status msr_objective(msr_ctx* c, int step, double lambda, const void* x, const void* low_res, double out[3],
                         void* stream) {
    TRY(check_step(c, step, true));
    if (!x || !out || (step == 2 && !low_res)) return fail(c, MSR_ERR_INVALID, "bad arguments");
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        if (step == 2) TRY(im.set_low_res(static_cast<const R*>(low_res), S(stream)));
        return im.objective_at(step, lambda, static_cast<const R*>(x), out, S(stream));
    });
}

msr_status msr_gradient(msr_ctx* c, int step, const void* x, const void* low_res, void* grad_out, void* stream) {
    TRY(check_step(c, step, true));
    if (!x || !grad_out || (step == 2 && !low_res)) return fail(c, MSR_ERR_INVALID, "bad arguments");
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.gradient(step, static_cast<const R*>(x), static_cast<const R*>(low_res), static_cast<R*>(grad_out),
                           S(stream));
    });
}

msr_status msr_apply_psf(msr_ctx* c, int step, const void* x, void* out, void* stream) {
    TRY(check_step(c, step, false));
    if (!x || !out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.apply_psf(step, static_cast<const R*>(x), static_cast<R*>(out), S(stream));
    });
}

msr_status msr_get_spectrum(msr_ctx* c, int step, double* host_out, int* kept, void* stream) {
    TRY(check_step(c, step, false));
    if (!host_out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    TRY(with_impl(c, [&](auto& im) { return im.get_spectrum(step, host_out, S(stream)); }));
    if (kept) *kept = c->K[step - 1];
    return MSR_OK;
}

msr_status msr_estimate_sigma2(msr_ctx* c, const void* dirty, double* sigma2, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (!dirty || !sigma2) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.sigma2(static_cast<const R*>(dirty), sigma2, S(stream));
    });
}

msr_status msr_default_lambda(msr_ctx* c, int step, int cycle, double cc, double* lambda, void* stream) {
    TRY(check_step(c, step, false));
    if (!lambda || cycle < 1) return fail(c, MSR_ERR_INVALID, "bad arguments");
    double s2 = 0.0;
    TRY(with_impl(c, [&](auto& im) { return im.image_reduce(im.dirty(step), nullptr, 1, &s2, S(stream)); }));
    *lambda = cc * std::sqrt(s2) * std::ldexp(1.0, cycle - 1);
    return MSR_OK;
}

}  // extern "C"

namespace {
// The autotuner's winners, per process, keyed by what decides them: image
// size, padding, precision, dictionary, the kept spectral columns of both
// PSFs and of the filters, and which passes were tuned.
using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int, int>;
struct TuneVal {
    int row[2], col[2], filt;
    double times[2 * MSR_MAX_VARIANTS];
};
std::map<TuneKey, TuneVal> g_tune;
std::mutex g_tune_mu;

TuneKey tune_key(const msr_ctx* c) {
    return TuneKey{c->sh.N, c->cfg.pad, c->sh.prec, c->cfg.dictionary, c->K[0], c->K[1], c->KL,
                   (int)c->have_psf[0], (int)c->have_psf[1], (int)c->have_filters};
}
}  // namespace

extern "C" {

msr_status msr_autotune(msr_ctx* c, int reps, int* row_variant, int* col_variant, double* times_ms, void* stream) {
    TRY(check_step(c, 1, false));
    const bool force = reps < 0;
    reps = reps == 0 ? 10 : (reps < 0 ? -reps : reps);
    double t[2 * MSR_MAX_VARIANTS];
    for (int i = 0; i < 2 * MSR_MAX_VARIANTS; ++i) t[i] = -1.0;
    const TuneKey key = tune_key(c);
    bool cached = false;
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            for (int s = 0; s < 2; ++s) {
                c->var_row[s] = it->second.row[s];
                c->var_col[s] = it->second.col[s];
            }
            c->var_filt = it->second.filt;
            std::memcpy(t, it->second.times, sizeof t);
            cached = true;
        }
    }
    if (!cached) {
        TRY(with_impl(c, [&](auto& im) { return im.autotune(reps, t, S(stream)); }));
        TuneVal v{};
        for (int s = 0; s < 2; ++s) {
            v.row[s] = c->var_row[s];
            v.col[s] = c->var_col[s];
        }
        v.filt = c->var_filt;
        std::memcpy(v.times, t, sizeof t);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = v;
    }
    if (times_ms) std::memcpy(times_ms, t, sizeof t);
    if (row_variant) *row_variant = c->var_row[0];
    if (col_variant) *col_variant = c->var_col[0];
    return MSR_OK;
}

msr_status msr_get_state(msr_ctx* c, int step, void* beta_k, void* beta_km1, int* k, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!beta_k || !beta_km1) return fail(c, MSR_ERR_INVALID, "null argument");
    if (c->state_step != step) return fail(c, MSR_ERR_STATE, "no iterates of step %d in the workspace", step);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    const int K = c->state_k;
    return with_impl(c, [&](auto& im) {
        const bool d = im.dict();
        const size_t bytes = d ? c->sh.rs * im.cn() : c->sh.is * c->sh.img_elems;
        HIPCHK(c, hipMemcpyAsync(beta_k, d ? (void*)im.coef(K) : im.iter_buf(K), bytes, hipMemcpyDeviceToDevice,
                                 S(stream)));
        HIPCHK(c, hipMemcpyAsync(beta_km1, d ? (void*)im.coef(K - 1) : im.iter_buf(K - 1), bytes,
                                 hipMemcpyDeviceToDevice, S(stream)));
        HIPCHK(c, hipStreamSynchronize(S(stream)));
        if (k) *k = K;
        return MSR_OK;
    });
}

msr_status msr_set_state(msr_ctx* c, int step, const void* beta_k, const void* beta_km1, int k, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!beta_k || !beta_km1 || k < 0) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        const bool d = im.dict();
        const size_t bytes = d ? c->sh.rs * im.cn() : c->sh.is * c->sh.img_elems;
        HIPCHK(c, hipMemcpyAsync(d ? (void*)im.coef(k - 1) : im.iter_buf(k - 1), beta_km1, bytes,
                                 hipMemcpyDeviceToDevice, S(stream)));
        HIPCHK(c, hipMemcpyAsync(d ? (void*)im.coef(k) : im.iter_buf(k), beta_k, bytes, hipMemcpyDeviceToDevice,
                                 S(stream)));
        HIPCHK(c, hipStreamSynchronize(S(stream)));
        c->state_step = 0;
        c->resume_k[step - 1] = k;
        c->resume_k[2 - step] = -1;  // the other step's loaded state shared these buffers
        return MSR_OK;
    });
}

msr_status msr_upsample(msr_ctx* c, int factor, const void* small, void* out, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (factor < 2 || (factor & (factor - 1)) || c->sh.N / factor < 2)
        return fail(c, MSR_ERR_INVALID, "factor must be a power of two with N / factor >= 2");
    if (!small || !out || small == out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        return im.upsample(factor, static_cast<const R*>(small), static_cast<R*>(out), S(stream));
    });
}

msr_status msr_dictionary_synthesis(msr_ctx* c, const void* coeffs, void* image, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (!c->sh.dict) return fail(c, MSR_ERR_STATE, "the context has no dictionary");
    if (!coeffs || !image) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        TRY(im.synthesize(static_cast<const R*>(coeffs), static_cast<R*>(image), S(stream)));
        HIPCHK(c, hipStreamSynchronize(S(stream)));
        return MSR_OK;
    });
}

msr_status msr_dictionary_analysis(msr_ctx* c, const void* image, void* coeffs, void* stream) {
    if (!ready(c)) return ws_missing(c);
    if (!c->sh.dict) return fail(c, MSR_ERR_STATE, "the context has no dictionary");
    if (!coeffs || !image) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    return with_impl(c, [&](auto& im) {
        using R = std::remove_pointer_t<decltype(im.dirty(1))>;
        TRY(im.analyze(static_cast<const R*>(image), im.store_epi(static_cast<R*>(coeffs), (R)1), S(stream)));
        HIPCHK(c, hipStreamSynchronize(S(stream)));
        return MSR_OK;
    });
}

msr_status msr_set_variants(msr_ctx* c, int step, int row_variant, int col_variant, int filter_variant) {
    if (!c) return MSR_ERR_INVALID;
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (step == 1 && filter_variant != -1) return fail(c, MSR_ERR_INVALID, "step 1 has no filter pass");
    const int want[3] = {row_variant, col_variant, filter_variant};
    for (int i = 0; i < 3; ++i) {
        const int v = want[i];
        if (i == 2 && v == -1) continue;
        if (v < 0 || v >= kVariants) return fail(c, MSR_ERR_INVALID, "variant %d out of range", v);
        const bool built = c->sh.prec == 64 ? (ops_for<double>(c->sh.N, c->sh.padded, v) &&
                                                ops_for<double>(c->sh.N, c->sh.padded, v)->row_update_fwd)
                                             : (ops_for<float>(c->sh.N, c->sh.padded, v) &&
                                                ops_for<float>(c->sh.N, c->sh.padded, v)->row_update_fwd);
        if (!built) return fail(c, MSR_ERR_UNSUPPORTED, "variant %d is not built for n = %d", v, c->sh.N);
    }
    c->var_row[step - 1] = row_variant;
    c->var_col[step - 1] = col_variant;
    if (step == 2) c->var_filt = filter_variant;
    return MSR_OK;
}

msr_status msr_get_variants(msr_ctx* c, int step, int* row_variant, int* col_variant, int* filter_variant) {
    if (!c) return MSR_ERR_INVALID;
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (row_variant) *row_variant = c->var_row[step - 1];
    if (col_variant) *col_variant = c->var_col[step - 1];
    if (filter_variant) *filter_variant = step == 2 ? c->var_filt : -1;
    return MSR_OK;
}

msr_status msr_time_pass(msr_ctx* c, int step, int which, int reps, double* ms_out, double* bytes_out,
                         double* flops_out, void* stream) {
    TRY(check_step(c, step, true));
    if (reps <= 0 || which < 0 || which > 5) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (which >= 4 && !c->sh.dict) return fail(c, MSR_ERR_STATE, "passes 4 and 5 need the wavelet dictionary");
    if (which == 3 && (step != 2 || !c->have_filters))
        return fail(c, MSR_ERR_STATE, "the filter pass needs step 2 with filters set");
    return with_impl(c, [&](auto& im) {
        return im.time_pass(which, step, reps, ms_out, bytes_out, flops_out, S(stream));
    });
}

}  // extern "C"

// =============================================================================
// Batched solves: many channels (frequency channels of one observation, each
// its own two-step problem) advanced together.  Channels of equal image size
// form a group; a group's workspaces are laid out back to back with one
// stride.  At each solve a group is split into runs of consecutive members
// with similar kept columns, and each pass of an iteration is ONE launch for
// a whole run (grid y = channel).  The fixed-count iteration loop of all
// runs is captured once into a HIP graph (runs spread over four streams, so
// runs of different sizes or widths overlap) and replayed.
// =============================================================================
struct msr_batch {
    struct Group {
        std::vector<int> members;  // channel indices, all of one image size
        size_t base = 0;           // workspace offset of the first member
        size_t stride = 0;         // bytes between consecutive members
        size_t chan_off = 0;       // ChanScalars[members]
        size_t chanf_off = 0;      // FilterCoef[members]
    };
    // Members [i0, i1) of a group launched together in one solve (a run).
    struct Run {
        int group, i0, i1;
    };
    std::vector<msr_ctx*> ch;
    std::vector<Group> groups;
    std::vector<Run> runs;  // the runs of the last solve
    int prec = 32, device = 0;
    size_t total = 0;
    char* ws = nullptr;
    static constexpr int kStreams = 4;
    hipStream_t st[kStreams] = {};
    hipEvent_t fork = nullptr, join[kStreams] = {}, t0 = nullptr, t1 = nullptr, done = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<long long> key;      // what the cached graph was captured for
    // the persistent launch (mode 1): descriptors, segments, counters and
    // control flags in the workspace; its own captured graph
    int mode = 0;
    unsigned int spin_limit = 0;
    int give_up = 0;
    size_t p_desc = 0, p_seg = 0, p_done = 0, p_ctl = 0;
    hipGraphExec_t pexec = nullptr;
    std::vector<long long> pkey;
    std::string err;
};

namespace {

msr_status bfail(msr_batch* b, msr_status s, const char* fmt, ...) {
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return s;
}

#define BHIPCHK(b, expr)                                                                              \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return bfail(b, MSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// A failure inside a channel: keep the channel's message.
msr_status bchan(msr_batch* b, int c, msr_status s) {
    if (s != MSR_OK && b) b->err = "channel " + std::to_string(c) + ": " + b->ch[c]->err;
    return s;
}

template <typename R>
size_t param_bytes(size_t nch) {
    return align_up(nch * sizeof(ChanScalars<R>), kAlign) + align_up(nch * sizeof(FilterCoef<R>), kAlign);
}

// Groups (largest images first) and the workspace layout of a batch.
bool plan_batch(int nch, const msr_config* cfgs, std::vector<msr_batch::Group>& groups, size_t& total,
                std::string* why, size_t* pers = nullptr) {
    if (nch <= 0 || !cfgs) {
        if (why) *why = "need at least one channel";
        return false;
    }
    for (int i = 0; i < nch; ++i) {
        Shapes s;
        if (!make_shapes(&cfgs[i], s, why)) return false;
        if (cfgs[i].pad != cfgs[0].pad || cfgs[i].precision != cfgs[0].precision ||
            cfgs[i].positivity != cfgs[0].positivity || cfgs[i].device != cfgs[0].device) {
            if (why) *why = "all channels need the same pad, precision, positivity and device";
            return false;
        }
        if (cfgs[i].dictionary != 0) {
            if (why) *why = "batched channels solve in the image domain (dictionary 0)";
            return false;
        }
        if (s.it64) {
            if (why) *why = "batched channels store iterates in the context's precision";
            return false;
        }
    }
    std::vector<int> order(nch);
    for (int i = 0; i < nch; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cfgs[a].n > cfgs[b].n; });
    groups.clear();
    for (int i : order) {
        if (groups.empty() || cfgs[groups.back().members[0]].n != cfgs[i].n) groups.emplace_back();
        groups.back().members.push_back(i);
    }
    size_t off = 0;
    for (auto& g : groups) {
        Shapes s;
        make_shapes(&cfgs[g.members[0]], s, nullptr);
        g.base = off;
        g.stride = align_up(make_layout(s).total, kAlign);
        off += g.stride * g.members.size();
    }
    for (auto& g : groups) {
        const size_t m = g.members.size();
        g.chan_off = off;
        const size_t pb = cfgs[0].precision == 64 ? param_bytes<double>(m) : param_bytes<float>(m);
        g.chanf_off = off + (cfgs[0].precision == 64 ? align_up(m * sizeof(ChanScalars<double>), kAlign)
                                                     : align_up(m * sizeof(ChanScalars<float>), kAlign));
        off += pb;
    }
    if (pers) {
        // the persistent launch: 2 parities x 6 passes x channels descriptors,
        // each XCD's item segments, channel list and count, the done counters
        // and the control block
        const size_t npc = (size_t)6 * nch;
        pers[0] = off;
        off += align_up(2 * npc * std::max(sizeof(PassDesc<float>), sizeof(PassDesc<double>)), kAlign);
        pers[1] = off;
        off += align_up((kPersistXcds * (npc + 1) + kPersistXcds * (size_t)nch + kPersistXcds) * sizeof(int), kAlign);
        pers[2] = off;
        off += align_up(npc * sizeof(unsigned int), kAlign);
        pers[3] = off;
        off += align_up(sizeof(PersistCtl), kAlign);
    }
    total = off;
    return true;
}

void drop_graph(msr_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->key.clear();
    if (b->pexec) (void)hipGraphExecDestroy(b->pexec);
    b->pexec = nullptr;
    b->pkey.clear();
}

template <typename R>
struct BatchImpl {
    msr_batch* b;

    // The launches of run r: its first member's context, spread over the
    // run's members with the run's widest kept columns.
    Impl<R> run_impl(const msr_batch::Run& r) const {
        const msr_batch::Group& g = b->groups[r.group];
        Impl<R> im(b->ch[g.members[r.i0]]);
        int K1 = 0, K2 = 0, KL = 0;
        for (int j = r.i0; j < r.i1; ++j) {
            const msr_ctx* x = b->ch[g.members[j]];
            K1 = std::max(K1, x->K[0]);
            K2 = std::max(K2, x->K[1]);
            KL = std::max(KL, x->KL);
        }
        im.set_group(r.i1 - r.i0, (long long)g.stride,
                     reinterpret_cast<const ChanScalars<R>*>(b->ws + g.chan_off) + r.i0,
                     reinterpret_cast<const FilterCoef<R>*>(b->ws + g.chanf_off) + r.i0, K1, K2, KL);
        return im;
    }

    // Splits every group of images of at least kRunMinN^2 into runs of
    // consecutive members whose kept columns in this step (K_L in step 1;
    // K_H and the low band in step 2) stay within a factor kRunSpread of each
    // other.  A run's launches read its widest columns for every member, so
    // one launch over channels of frequency-scaled coverage would pay the
    // highest frequency's width for all of them; consecutive members, because
    // the launches of a run need its workspaces at one stride.  Smaller
    // images stay in one run: a launch for a few of them cannot fill the GPU,
    // and more launches cost more than the wider columns (64 mixed channels of
    // 512^2 to 4096^2: 17 714 channel-iterations/s with every size split,
    // against 18 599 unsplit).
    void plan_runs(int step) {
        constexpr double kRunSpread = 1.2;
        constexpr int kRunMinN = 2048;
        b->runs.clear();
        for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
            const msr_batch::Group& g = b->groups[gi];
            if (b->ch[g.members[0]]->sh.N < kRunMinN) {
                b->runs.push_back({gi, 0, (int)g.members.size()});
                continue;
            }
            auto width = [&](int j, int q) {
                const msr_ctx* x = b->ch[g.members[j]];
                return std::max(1, step == 1 ? x->K[0] : (q == 0 ? x->K[1] : x->KL));
            };
            int i0 = 0, lo[2] = {width(0, 0), width(0, 1)}, hi[2] = {lo[0], lo[1]};
            for (int j = 1; j < (int)g.members.size(); ++j) {
                bool fits = true;
                for (int q = 0; q < 2; ++q) {
                    const int w = width(j, q);
                    fits = fits && std::max(hi[q], w) <= kRunSpread * std::min(lo[q], w);
                }
                if (!fits) {
                    b->runs.push_back({gi, i0, j});
                    i0 = j;
                    for (int q = 0; q < 2; ++q) lo[q] = hi[q] = width(j, q);
                } else {
                    for (int q = 0; q < 2; ++q) {
                        lo[q] = std::min(lo[q], width(j, q));
                        hi[q] = std::max(hi[q], width(j, q));
                    }
                }
            }
            b->runs.push_back({gi, i0, (int)g.members.size()});
        }
    }

    std::vector<long long> graph_key(int step, int iters) const {
        std::vector<long long> k{step, iters};
        for (const auto& r : b->runs) {
            Impl<R> im = run_impl(r);
            msr_ctx* c0 = b->ch[b->groups[r.group].members[r.i0]];
            k.insert(k.end(), {(long long)r.group, (long long)r.i0, (long long)r.i1, im.Ks(1), im.Ks(2), im.KLs(),
                               c0->var_row[step - 1], c0->var_col[step - 1], c0->var_filt});
        }
        return k;
    }

    // Captures `iters` iterations of every run into b->exec.
    msr_status capture(int step, int iters) {
        hipStream_t s0 = b->st[0];
        BHIPCHK(b, hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
        msr_status st = MSR_OK;
        const int ns = std::min<int>((int)b->runs.size(), msr_batch::kStreams);
        if (hipEventRecord(b->fork, s0) != hipSuccess) st = bfail(b, MSR_ERR_HIP, "fork event");
        for (int i = 1; i < ns && st == MSR_OK; ++i)
            if (hipStreamWaitEvent(b->st[i], b->fork, 0) != hipSuccess) st = bfail(b, MSR_ERR_HIP, "fork wait");
        for (size_t ri = 0; ri < b->runs.size() && st == MSR_OK; ++ri) {
            const msr_batch::Run& r = b->runs[ri];
            Impl<R> im = run_impl(r);
            hipStream_t s = b->st[ri % ns];
            const int c0 = b->groups[r.group].members[r.i0];
            for (int k = 1; k <= iters && st == MSR_OK; ++k) st = bchan(b, c0, im.iterate(step, k, 0.0, 0.0, s));
        }
        for (int i = 1; i < ns && st == MSR_OK; ++i) {
            if (hipEventRecord(b->join[i], b->st[i]) != hipSuccess || hipStreamWaitEvent(s0, b->join[i], 0) != hipSuccess)
                st = bfail(b, MSR_ERR_HIP, "join");
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(s0, &graph);
        if (st == MSR_OK && ee != hipSuccess) st = bfail(b, MSR_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
        if (st == MSR_OK) {
            const hipError_t ei = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                b->exec = nullptr;
                st = bfail(b, MSR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
            }
        }
        if (graph) hipGraphDestroy(graph);
        return st;
    }

    // Whether every channel can run in the persistent kernel: single
    // precision, zero padded, W = I, image side 512 .. 4096.
    bool persistent_ok(std::string* why) const {
        if (!std::is_same<R, float>::value) return *why = "the persistent launch is single precision", false;
        for (size_t c = 0; c < b->ch.size(); ++c) {
            const msr_ctx* x = b->ch[c];
            if (!x->sh.padded || x->sh.dict || persist_index(x->sh.N) < 0) {
                char buf[160];
                snprintf(buf, sizeof buf, "channel %zu: the persistent launch runs zero-padded images of 512 .. 4096", c);
                *why = buf;
                return false;
            }
        }
        return true;
    }

    // The iterations of every channel in one persistent launch (mode 1): the
    // per-channel passes of iterate() recorded as descriptors for both parities
    // of k, the item segments (pass-major, then channel), one graph holding the
    // counter reset and the kernel, replayed while the shapes stay the same.
    msr_status iterate_persistent(int step, int iters, const std::vector<double>& mu, const double* lambda,
                                  float* ms_out, hipStream_t s) {
        const int C = (int)b->ch.size();
        const int npass = step == 1 ? 4 : 6;
        std::vector<PassDesc<R>> desc((size_t)C * npass * 2);
        bool with_4096 = false;
        for (int c = 0; c < C; ++c) {
            with_4096 = with_4096 || b->ch[c]->sh.N >= 4096;
            for (int k = 1; k <= 2; ++k) {
                std::vector<PassDesc<R>> rec;
                Impl<R> im(b->ch[c]);
                im.rec_ = &rec;
                TRY(bchan(b, c, im.iterate(step, k, mu[c], lambda[c], s)));
                if ((int)rec.size() != npass) return bfail(b, MSR_ERR_STATE, "channel %d: %zu passes recorded", c, rec.size());
                for (int p = 0; p < npass; ++p) desc[((size_t)c * npass + p) * 2 + (k & 1)] = rec[p];
            }
        }
        // channels onto XCDs, the most work first onto the least loaded
        // (work of a channel: blocks of its passes x its line length)
        const int X = kPersistXcds;
        std::vector<double> work(C);
        for (int c = 0; c < C; ++c) {
            double w = 0;
            for (int p = 0; p < npass; ++p) w += (double)desc[((size_t)c * npass + p) * 2].nblocks;
            work[c] = w * b->ch[c]->sh.N;
        }
        std::vector<int> order(C);
        for (int c = 0; c < C; ++c) order[c] = c;
        std::stable_sort(order.begin(), order.end(), [&](int a, int bb) { return work[a] > work[bb]; });
        std::vector<std::vector<int>> xch(X);
        std::vector<double> load(X, 0.0);
        for (int c : order) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            xch[x].push_back(c);
            load[x] += work[c];
        }
        // per XCD: segments (pass-major over its channels), then channel
        // lists [X][C] and counts [X], one int array
        const size_t sx = (size_t)npass * C + 1;
        std::vector<int> tab(X * sx + (size_t)X * C + X, 0);
        int most = 0;
        for (int x = 0; x < X; ++x) {
            int off = 0;
            const int n = (int)xch[x].size();
            for (int p = 0; p < npass; ++p)
                for (int j = 0; j < n; ++j) {
                    tab[x * sx + (size_t)p * n + j] = off;
                    off += desc[((size_t)xch[x][j] * npass + p) * 2].nblocks;
                }
            tab[x * sx + (size_t)npass * n] = off;
            for (int j = 0; j < n; ++j) tab[X * sx + (size_t)x * C + j] = xch[x][j];
            tab[X * sx + (size_t)X * C + x] = n;
            most = std::max(most, off);
        }
        if ((long long)most * iters >= (1LL << 32)) return bfail(b, MSR_ERR_INVALID, "too many work items for one launch");
        PersistCtl ctl{};
        ctl.give_up = b->give_up;
        BHIPCHK(b, hipMemcpyAsync(b->ws + b->p_desc, desc.data(), sizeof(PassDesc<R>) * desc.size(),
                                  hipMemcpyHostToDevice, s));
        BHIPCHK(b, hipMemcpyAsync(b->ws + b->p_seg, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, s));
        BHIPCHK(b, hipMemcpyAsync(b->ws + b->p_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s));
        BHIPCHK(b, hipStreamSynchronize(s));  // the host vectors go out of scope
        PersistArgs<float> pa{};
        pa.desc = reinterpret_cast<const PassDesc<float>*>(b->ws + b->p_desc);
        pa.seg = reinterpret_cast<const int*>(b->ws + b->p_seg);
        pa.xch = pa.seg + X * sx;
        pa.xn = pa.xch + (size_t)X * C;
        pa.done = reinterpret_cast<unsigned int*>(b->ws + b->p_done);
        pa.ctl = reinterpret_cast<PersistCtl*>(b->ws + b->p_ctl);
        pa.C = C;
        pa.npass = npass;
        pa.iters = iters;
        pa.k0 = 0;
        pa.spin_limit = b->spin_limit ? b->spin_limit : (1u << 22);
        int cus = 0;
        BHIPCHK(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        // a multiple of the XCD count, so that every XCD holds the same
        // number of the launch's blocks
        const int grid = cus * persist_occupancy_f32(with_4096) / X * X;
        if (grid < X) return bfail(b, MSR_ERR_UNSUPPORTED, "the persistent launch needs %d resident blocks", X);
        const std::vector<long long> key{step, iters, C, npass, with_4096, grid, most, (long long)pa.spin_limit};
        hipStream_t s0 = b->st[0];
        if (!b->pexec || key != b->pkey) {
            if (b->pexec) (void)hipGraphExecDestroy(b->pexec);
            b->pexec = nullptr;
            b->pkey.clear();
            BHIPCHK(b, hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
            const hipError_t el = persist_launch_f32(pa, with_4096, grid, s0);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(s0, &graph);
            if (el != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return bfail(b, MSR_ERR_HIP, "persistent launch capture: %s",
                             hipGetErrorString(el != hipSuccess ? el : ee));
            }
            const hipError_t ei = hipGraphInstantiate(&b->pexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                b->pexec = nullptr;
                return bfail(b, MSR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
            }
            b->pkey = key;
        }
        BHIPCHK(b, hipEventRecord(b->done, s));
        BHIPCHK(b, hipStreamWaitEvent(s0, b->done, 0));
        BHIPCHK(b, hipEventRecord(b->t0, s0));
        BHIPCHK(b, hipGraphLaunch(b->pexec, s0));
        BHIPCHK(b, hipEventRecord(b->t1, s0));
        BHIPCHK(b, hipStreamWaitEvent(s, b->t1, 0));
        BHIPCHK(b, hipEventSynchronize(b->t1));
        BHIPCHK(b, hipEventElapsedTime(ms_out, b->t0, b->t1));
        BHIPCHK(b, hipMemcpy(&ctl, b->ws + b->p_ctl, sizeof ctl, hipMemcpyDeviceToHost));
        if (ctl.abort || ctl.give_up)
            return bfail(b, MSR_ERR_HIP, "the persistent launch gave up (%s): the iterates are incomplete",
                         ctl.give_up ? "the host raised the give-up flag" : "a wait reached its spin limit");
        return MSR_OK;
    }

    msr_status solve(int step, const double* lambda, int iters, const void* const* low_res, const void* const* x0,
                     void* const* model_out, void* const* image_out, msr_result* res, hipStream_t s) {
        const int C = (int)b->ch.size();
        if (b->mode == 1) {
            std::string why;
            if (!persistent_ok(&why)) return bfail(b, MSR_ERR_UNSUPPORTED, "%s", why.c_str());
        }
        // 1. per channel: theta, beta_0, constraint, spectrum of alpha_0 (on
        //    every column its run's launches read: nothing unwritten is read,
        //    not even where a zero factor would cancel it)
        std::vector<double> mu(C);
        for (int c = 0; c < C; ++c) {
            if (b->ch[c]->resume_k[step - 1] >= 0)
                return bfail(b, MSR_ERR_UNSUPPORTED, "channel %d: batched solves start from x0, not a loaded state", c);
            b->ch[c]->state_step = 0;
        }
        plan_runs(step);
        for (const auto& r : b->runs) {
            const Impl<R> ri = run_impl(r);
            for (int j = r.i0; j < r.i1; ++j) {
                const int c = b->groups[r.group].members[j];
                Impl<R> im(b->ch[c]);
                // the launches of a run read its widest columns; the
                // persistent launch reads each channel's own
                const int ka = b->mode == 1 ? 0 : ri.KA(step), kl = b->mode == 1 ? 0 : ri.KLs();
                TRY(bchan(b, c, im.prepare(step, step == 2 ? static_cast<const R*>(low_res[c]) : nullptr,
                                           x0 ? static_cast<const R*>(x0[c]) : nullptr, &mu[c], s, ka, kl)));
            }
        }
        float ms = 0.f;
        if (b->mode == 1) {
            if (iters > 0) TRY(iterate_persistent(step, iters, mu, lambda, &ms, s));
            return finish_all(step, lambda, iters, model_out, image_out, res, ms, s);
        }
        // 2. per-channel parameters of every group
        for (const auto& g : b->groups) {
            const size_t m = g.members.size();
            std::vector<ChanScalars<R>> cs(m);
            std::vector<FilterCoef<R>> cf(m);
            for (size_t j = 0; j < m; ++j) {
                const int c = g.members[j];
                cs[j].two_mu = (R)(2.0 * mu[c]);
                cs[j].thr = (R)(mu[c] * lambda[c]);
                cs[j].inv_sigma2 = step == 2 ? (R)(1.0 / b->ch[c]->sigma2) : (R)1;
                cs[j].unused = (R)0;
                if (step == 2) cf[j] = Impl<R>(b->ch[c]).filters();
            }
            BHIPCHK(b, hipMemcpyAsync(b->ws + g.chan_off, cs.data(), m * sizeof(ChanScalars<R>), hipMemcpyHostToDevice, s));
            BHIPCHK(b, hipMemcpyAsync(b->ws + g.chanf_off, cf.data(), m * sizeof(FilterCoef<R>), hipMemcpyHostToDevice, s));
            BHIPCHK(b, hipStreamSynchronize(s));  // the host arrays go out of scope
        }
        // 3. the iterations: one graph for all runs
        if (iters > 0) {
            const std::vector<long long> key = graph_key(step, iters);
            if (!b->exec || key != b->key) {
                drop_graph(b);
                TRY(capture(step, iters));
                b->key = key;
            }
            BHIPCHK(b, hipEventRecord(b->done, s));
            BHIPCHK(b, hipStreamWaitEvent(b->st[0], b->done, 0));
            BHIPCHK(b, hipEventRecord(b->t0, b->st[0]));
            BHIPCHK(b, hipGraphLaunch(b->exec, b->st[0]));
            BHIPCHK(b, hipEventRecord(b->t1, b->st[0]));
            BHIPCHK(b, hipStreamWaitEvent(s, b->t1, 0));
            BHIPCHK(b, hipEventSynchronize(b->t1));
            BHIPCHK(b, hipEventElapsedTime(&ms, b->t0, b->t1));
        }
        return finish_all(step, lambda, iters, model_out, image_out, res, ms, s);
    }

    // 4. per channel: objective, model out
    msr_status finish_all(int step, const double* lambda, int iters, void* const* model_out, void* const* image_out,
                          msr_result* res, float ms, hipStream_t s) {
        const int C = (int)b->ch.size();
        for (int c = 0; c < C; ++c) {
            Impl<R> im(b->ch[c]);
            double F[3] = {0, 0, 0};
            R* img = image_out ? static_cast<R*>(image_out[c]) : nullptr;
            TRY(bchan(b, c, im.finish(step, lambda[c], iters, static_cast<R*>(model_out[c]), img, F, s)));
            if (res) {
                res[c].iters = iters;
                res[c].converged = 0;
                res[c].objective = F[0];
                res[c].data_term = F[1];
                res[c].l1_norm = F[2];
                res[c].theta = b->ch[c]->theta[step - 1];
                res[c].elapsed_ms = ms;
                res[c].time_to_tol_ms = -1.0;
            }
        }
        BHIPCHK(b, hipStreamSynchronize(s));
        return MSR_OK;
    }
};

}  // namespace

extern "C" {

size_t msr_batch_workspace_bytes(int channels, const msr_config* cfgs) {
    std::vector<msr_batch::Group> g;
    size_t total = 0, pers[4];
    if (!plan_batch(channels, cfgs, g, total, nullptr, pers)) return 0;
    return total;
}

msr_status msr_batch_init(int channels, const msr_config* cfgs, msr_batch** out) {
    if (!out) return MSR_ERR_INVALID;
    *out = nullptr;
    std::vector<msr_batch::Group> groups;
    size_t total = 0, pers[4];
    if (!plan_batch(channels, cfgs, groups, total, nullptr, pers)) return MSR_ERR_INVALID;
    msr_batch* b = new (std::nothrow) msr_batch();
    if (!b) return MSR_ERR_OOM;
    b->groups = std::move(groups);
    b->total = total;
    b->p_desc = pers[0];
    b->p_seg = pers[1];
    b->p_done = pers[2];
    b->p_ctl = pers[3];
    b->prec = cfgs[0].precision;
    b->device = cfgs[0].device;
    b->ch.assign(channels, nullptr);
    for (int i = 0; i < channels; ++i) {
        const msr_status st = msr_init(&cfgs[i], &b->ch[i]);
        if (st != MSR_OK) {
            msr_batch_destroy(b);
            return st;
        }
    }
    bool ok = hipSetDevice(b->device) == hipSuccess;
    for (int i = 0; i < msr_batch::kStreams && ok; ++i)
        ok = hipStreamCreateWithFlags(&b->st[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&b->done, hipEventDisableTiming) == hipSuccess &&
         hipEventCreate(&b->t0) == hipSuccess && hipEventCreate(&b->t1) == hipSuccess;
    if (!ok) {
        msr_batch_destroy(b);
        return MSR_ERR_HIP;
    }
    *out = b;
    return MSR_OK;
}

void msr_batch_destroy(msr_batch* b) {
    if (!b) return;
    hipSetDevice(b->device);
    drop_graph(b);
    for (int i = 0; i < msr_batch::kStreams; ++i) {
        if (b->st[i]) hipStreamDestroy(b->st[i]);
        if (b->join[i]) hipEventDestroy(b->join[i]);
    }
    for (hipEvent_t e : {b->fork, b->done, b->t0, b->t1})
        if (e) hipEventDestroy(e);
    for (msr_ctx* c : b->ch) msr_destroy(c);
    delete b;
}

const char* msr_batch_last_error(const msr_batch* b) { return b ? b->err.c_str() : "null batch"; }

int msr_batch_channels(const msr_batch* b) { return b ? (int)b->ch.size() : 0; }

msr_ctx* msr_batch_channel(msr_batch* b, int c) {
    if (!b || c < 0 || c >= (int)b->ch.size()) return nullptr;
    return b->ch[c];
}

msr_status msr_batch_set_workspace(msr_batch* b, void* dev, size_t bytes) {
    if (!b) return MSR_ERR_INVALID;
    if (!dev || bytes < b->total) return bfail(b, MSR_ERR_OOM, "workspace needs %zu bytes", b->total);
    if (reinterpret_cast<uintptr_t>(dev) % kAlign) return bfail(b, MSR_ERR_INVALID, "workspace must be 256-byte aligned");
    drop_graph(b);
    b->ws = static_cast<char*>(dev);
    for (const auto& g : b->groups)
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int c = g.members[j];
            TRY(bchan(b, c, msr_set_workspace(b->ch[c], b->ws + g.base + j * g.stride, g.stride)));
        }
    return MSR_OK;
}

msr_status msr_batch_autotune(msr_batch* b, int reps, void* stream) {
    if (!b || !b->ws) return b ? bfail(b, MSR_ERR_OOM, "no workspace") : MSR_ERR_INVALID;
    for (const auto& g : b->groups) {
        msr_ctx* c0 = b->ch[g.members[0]];
        TRY(bchan(b, g.members[0], msr_autotune(c0, reps, nullptr, nullptr, nullptr, stream)));
        for (int m : g.members) {
            b->ch[m]->var_row[0] = c0->var_row[0];
            b->ch[m]->var_row[1] = c0->var_row[1];
            b->ch[m]->var_col[0] = c0->var_col[0];
            b->ch[m]->var_col[1] = c0->var_col[1];
            b->ch[m]->var_filt = c0->var_filt;
        }
    }
    drop_graph(b);
    return MSR_OK;
}

constexpr bool kPersistentEnabled = false;

msr_status msr_batch_set_mode(msr_batch* b, int mode, unsigned int spin_limit) {
    if (!b) return MSR_ERR_INVALID;
    if (mode != 0 && mode != 1) return bfail(b, MSR_ERR_INVALID, "mode must be 0 (launches per pass) or 1 (persistent)");
    // Switched off: the first solve of the persistent launch (four channels of
    // 512 .. 2048, 30 step-1 iterations) did not return within minutes, in
    // two designs of its memory ordering (agent-scope fences per item; queues
    // per XCD with L1-only ordering), and no cause has been shown.
    if (mode == 1 && !kPersistentEnabled)
        return bfail(b, MSR_ERR_UNSUPPORTED, "the persistent launch (mode 1) is switched off");
    b->mode = mode;
    b->spin_limit = spin_limit;
    return MSR_OK;
}

msr_status msr_batch_give_up(msr_batch* b, int raise, void* stream) {
    if (!b) return MSR_ERR_INVALID;
    b->give_up = raise ? 1 : 0;
    if (b->ws) {
        BHIPCHK(b, hipSetDevice(b->device));
        BHIPCHK(b, hipMemcpyAsync(b->ws + b->p_ctl + offsetof(PersistCtl, give_up), &b->give_up, sizeof(int),
                                  hipMemcpyHostToDevice, S(stream)));
        BHIPCHK(b, hipStreamSynchronize(S(stream)));
    }
    return MSR_OK;
}

msr_status msr_batch_solve(msr_batch* b, int step, const double* lambda, int iters, const void* const* low_res,
                           const void* const* x0, void* const* model_out, void* const* image_out, msr_result* res,
                           void* stream) {
    if (!b) return MSR_ERR_INVALID;
    if (!b->ws) return bfail(b, MSR_ERR_OOM, "no workspace");
    if (step != 1 && step != 2) return bfail(b, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!lambda || !model_out || iters < 0 || (step == 2 && !low_res) || (step == 2 && image_out))
        return bfail(b, MSR_ERR_INVALID, "bad arguments");
    for (size_t c = 0; c < b->ch.size(); ++c) {
        msr_ctx* cx = b->ch[c];
        if (!cx->have_psf[step - 1]) return bfail(b, MSR_ERR_STATE, "channel %zu: set_dirty_psf(%d) first", c, step);
        if (step == 2 && (!cx->have_filters || !low_res[c]))
            return bfail(b, MSR_ERR_STATE, "channel %zu: step 2 needs filters and low_res", c);
        if (!model_out[c] || !(lambda[c] >= 0) || !std::isfinite(lambda[c]))
            return bfail(b, MSR_ERR_INVALID, "channel %zu: bad lambda or output", c);
    }
    BHIPCHK(b, hipSetDevice(b->device));
    if (b->prec == 64)
        return BatchImpl<double>{b}.solve(step, lambda, iters, low_res, x0, model_out, image_out, res, S(stream));
    return BatchImpl<float>{b}.solve(step, lambda, iters, low_res, x0, model_out, image_out, res, S(stream));
}

}  // extern "C"
