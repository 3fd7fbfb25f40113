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
//   step 2 iteration (Eq. 12):
//     col  SA -> SB        x h_hat_H
//     row  SB -> SC        r = H alpha - i_H, forward (all columns)
//     col  SC -> SB        x g_H^2                           (C_{g_H^2} E r)
//     row  SB -> SC        crop, re-embed, forward (K_H columns)
//     col  SC -> SB        x h_hat_H                         (H^T ...)
//     col  SA - SL -> SC   x g_L^2 (k_x < K_L only)           (C_{g_L^2} E (alpha - l))
//     row  SB + SC -> SA   FISTA update, forward alpha_k
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/msr.h"
#include "ops.hpp"
#include "small_kernels.hpp"

using namespace msr;

namespace msr {
#define MSR_DECL(Lv) const Ops* ops_len_##Lv(bool padded);
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

const Ops* ops_for(int L, bool padded) {
    switch (L) {
        case 8: return ops_len_8(padded);
        case 16: return ops_len_16(padded);
        case 32: return ops_len_32(padded);
        case 64: return ops_len_64(padded);
        case 128: return ops_len_128(padded);
        case 256: return ops_len_256(padded);
        case 512: return ops_len_512(padded);
        case 1024: return ops_len_1024(padded);
        case 2048: return ops_len_2048(padded);
        case 4096: return ops_len_4096(padded);
        case 8192: return ops_len_8192(padded);
        case 16384: return ops_len_16384(padded);
        default: return nullptr;
    }
}
}  // namespace msr

namespace {

constexpr double kThetaMargin = 1.01;  // Rayleigh quotients under-estimate lambda_max
constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    size_t tw, SA, SB, SC, SL, hh1, hh2, d1, d2, b0, b1, t0, t1, partials, scal, colmax, total;
};

struct Shapes {
    int N, P, logN, T, Cfull, Cpad, Tpsf, Cpad_psf;
    bool padded;
    size_t spec_elems;   // N * Cpad complex
    size_t hh_elems;     // P * Cpad floats
    size_t img_elems;    // N * N
    size_t partial_cnt;  // doubles
};

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

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
    s.N = c->n;
    s.padded = c->pad == 2;
    s.P = c->pad * c->n;
    s.logN = 0;
    while ((1 << s.logN) < s.N) ++s.logN;
    const Ops* o = ops_for(s.N, s.padded);
    const Ops* op = ops_for(s.P, false);
    if (!o || !op || !o->row_update_fwd || !op->col_forward) {
        if (why) *why = "no kernels built for this size";
        return false;
    }
    s.T = o->T;
    s.Cfull = s.P / 2 + 1;
    s.Cpad = (int)align_up(s.Cfull, s.T);
    s.Tpsf = op->T;
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
    l.tw = take(sizeof(float2) * (size_t)s.P);
    l.SA = take(sizeof(float2) * s.spec_elems);
    // SB and SC are contiguous: together they hold the P-row PSF spectrum.
    const size_t sbc = std::max(2 * sizeof(float2) * s.spec_elems, sizeof(float2) * (size_t)s.P * s.Cpad_psf);
    l.SB = take(sbc);
    l.SC = l.SB + align_up(sizeof(float2) * s.spec_elems, kAlign);
    l.SL = take(sizeof(float2) * s.spec_elems);
    l.hh1 = take(sizeof(float) * s.hh_elems);
    l.hh2 = take(sizeof(float) * s.hh_elems);
    l.d1 = take(sizeof(float) * s.img_elems);
    l.d2 = take(sizeof(float) * s.img_elems);
    l.b0 = take(sizeof(float) * s.img_elems);
    l.b1 = take(sizeof(float) * s.img_elems);
    l.t0 = take(sizeof(float) * s.img_elems);
    l.t1 = take(sizeof(float) * s.img_elems);
    l.partials = take(sizeof(double) * s.partial_cnt);
    l.scal = take(sizeof(double) * 64);
    l.colmax = take(sizeof(float) * (size_t)s.Cfull);
    l.total = off;
    return l;
}

}  // namespace

struct msr_ctx {
    msr_config cfg{};
    Shapes sh{};
    Layout lay{};
    const Ops* op = nullptr;   // N-length passes (padded or circular)
    const Ops* opp = nullptr;  // P-length unpadded (PSF spectrum)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // device views
    float2 *tw = nullptr, *SA = nullptr, *SB = nullptr, *SC = nullptr, *SL = nullptr;
    float* hh[2] = {nullptr, nullptr};
    float* dirty[2] = {nullptr, nullptr};
    float* beta[2] = {nullptr, nullptr};
    float* tmp[2] = {nullptr, nullptr};
    double* partials = nullptr;
    double* scal = nullptr;
    float* colmax = nullptr;
    // state
    int K[2] = {0, 0};  // kept columns per PSF
    bool have_psf[2] = {false, false};
    bool have_filters = false;
    bool have_theta[2] = {false, false};
    double theta[2] = {0, 0};
    double ell = 0, delta = 0, sigma2 = 0, eta2 = 0;
    FilterCoef fc{};
    int KL = 0;  // columns with g_L != 0
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

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(ctx, MSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(ctx)                                                                              \
    do {                                                                                            \
        hipError_t e_ = hipGetLastError();                                                          \
        if (e_ != hipSuccess) return fail(ctx, MSR_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline RowArgs row_args(msr_ctx* c, const float2* in, int kin, const float2* in2, int kin2, float2* out, int kout) {
    RowArgs a{};
    a.spec_in = in;
    a.spec_in2 = in2;
    a.spec_out = out;
    a.tw = c->tw;
    a.partials = c->partials;
    a.NR = c->sh.N;
    a.K_in = kin;
    a.K_in2 = in2 ? kin2 : 0;
    a.K_out = kout;
    return a;
}

inline ColArgs col_args(msr_ctx* c, const float2* in, const float2* in2, float2* out, int K) {
    ColArgs a{};
    a.spec_in = in;
    a.spec_in2 = in2;
    a.spec_out = out;
    a.tw = c->tw;
    a.partials = c->partials;
    a.NR = c->sh.N;
    a.K = K;
    return a;
}

inline int row_grid(msr_ctx* c) { return c->sh.N / c->op->row_rows; }
inline int col_grid(msr_ctx* c, int K) { return (K + c->sh.T - 1) / c->sh.T; }

// Sum `nq` quantities over `nblocks` partial rows into scal[off..]; returns them to host if `host`.
msr_status reduce(msr_ctx* c, int nblocks, int nq, int off, double* host, hipStream_t s) {
    hipLaunchKernelGGL(finalize_sums, dim3(1), dim3(256), 0, s, c->partials, nblocks, nq, c->scal + off);
    LAUNCHCHK(c);
    if (host) {
        HIPCHK(c, hipMemcpyAsync(host, c->scal + off, sizeof(double) * nq, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return MSR_OK;
}

msr_status image_reduce(msr_ctx* c, const float* x, const float* y, int mode, double* host, hipStream_t s) {
    const size_t n = c->sh.img_elems;
    int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(image_sums, dim3(blocks), dim3(256), 0, s, x, y, n, mode, c->partials);
    LAUNCHCHK(c);
    return reduce(c, blocks, 1, 8, host, s);
}

bool ready(msr_ctx* c) { return c && c->ws; }

int KA(msr_ctx* c, int step) { return step == 1 ? c->K[0] : std::max(c->K[1], c->KL); }

// image -> SA-like spectrum
msr_status fwd_image(msr_ctx* c, const float* img, float scale, float2* out, int kout, hipStream_t s) {
    EpiLoad e{img, c->sh.N, scale};
    c->op->row_load_fwd(row_args(c, nullptr, 0, nullptr, 0, out, kout), e, s);
    LAUNCHCHK(c);
    return MSR_OK;
}

msr_status col_psf(msr_ctx* c, int step, const float2* in, float2* out, hipStream_t s) {
    ModePsf m{c->hh[step - 1], c->sh.P, c->sh.T};
    c->op->col_psf(col_args(c, in, nullptr, out, c->K[step - 1]), m, s);
    LAUNCHCHK(c);
    return MSR_OK;
}

msr_status col_filth(msr_ctx* c, const float2* in, float2* out, hipStream_t s) {
    ModeFilterH m{c->fc, (float)(1.0 / ((double)c->sh.P * c->sh.P))};
    c->op->col_filth(col_args(c, in, nullptr, out, c->sh.Cfull), m, s);
    LAUNCHCHK(c);
    return MSR_OK;
}

msr_status col_filtl(msr_ctx* c, const float2* in, const float2* in2, float2* out, hipStream_t s) {
    ModeFilterL m{c->fc, (float)(1.0 / ((double)c->sh.P * c->sh.P))};
    c->op->col_filtl(col_args(c, in, in2, out, c->KL), m, s);
    LAUNCHCHK(c);
    return MSR_OK;
}

// The gradient chain of step s applied to the spectrum in SA (alpha); leaves the
// half-gradient spectrum in SB (+ SC for k_x < K_L in step 2).  `y` is the data
// term's image (null for the normal operator alone); `l` spectrum SL is used in
// step 2 when `use_l`.
msr_status grad_chain(msr_ctx* c, int step, const float* y, bool use_l, hipStream_t s) {
    msr_status st;
    const int Ks = c->K[step - 1];
    if ((st = col_psf(c, step, c->SA, c->SB, s)) != MSR_OK) return st;
    EpiResid er{y, nullptr, c->sh.N};
    const int kr = step == 1 ? Ks : c->sh.Cfull;
    c->op->row_resid_fwd(row_args(c, c->SB, Ks, nullptr, 0, c->SC, kr), er, s);
    LAUNCHCHK(c);
    if (step == 1) return col_psf(c, 1, c->SC, c->SB, s);
    if ((st = col_filth(c, c->SC, c->SB, s)) != MSR_OK) return st;
    EpiResid rp{nullptr, nullptr, c->sh.N};
    c->op->row_resid_fwd(row_args(c, c->SB, c->sh.Cfull, nullptr, 0, c->SC, Ks), rp, s);
    LAUNCHCHK(c);
    if ((st = col_psf(c, 2, c->SC, c->SB, s)) != MSR_OK) return st;
    return col_filtl(c, c->SA, use_l ? c->SL : nullptr, c->SC, s);
}

double momentum(int k) { return k >= 1 ? (k - 1.0) / (k + 2.0) : 0.0; }

// One FISTA iteration k (1-based) of step s.
msr_status iterate(msr_ctx* c, int step, int k, double mu, double lambda, hipStream_t s) {
    msr_status st = grad_chain(c, step, c->dirty[step - 1], true, s);
    if (st != MSR_OK) return st;
    EpiUpdate u{};
    u.b1 = c->beta[(k - 1) & 1];
    u.b2 = c->beta[k & 1];
    u.ld = c->sh.N;
    u.two_mu = (float)(2.0 * mu);
    u.thr = (float)(mu * lambda);
    u.t_prev = (float)momentum(k - 1);
    u.t_cur = (float)momentum(k);
    u.positivity = c->cfg.positivity;
    const int Ks = c->K[step - 1];
    RowArgs a = step == 1 ? row_args(c, c->SB, Ks, nullptr, 0, c->SA, KA(c, 1))
                          : row_args(c, c->SB, Ks, c->SC, c->KL, c->SA, KA(c, 2));
    c->op->row_update_fwd(a, u, s);
    LAUNCHCHK(c);
    return MSR_OK;
}

// Exact objective of step s at image x (device), FP64 sums.  out: F, data, l1.
// Uses SB, SC (and SL for step 2) as scratch; SA is preserved.
msr_status objective_at(msr_ctx* c, int step, double lambda, const float* x, double out[3], hipStream_t s) {
    msr_status st;
    double data = 0.0;
    if (step == 1) {
        if ((st = fwd_image(c, x, 1.f, c->SB, c->K[0], s)) != MSR_OK) return st;
        if ((st = col_psf(c, 1, c->SB, c->SC, s)) != MSR_OK) return st;
        EpiResid er{c->dirty[0], nullptr, c->sh.N};
        c->op->row_resid(row_args(c, c->SC, c->K[0], nullptr, 0, nullptr, 0), er, s);
        LAUNCHCHK(c);
        if ((st = reduce(c, row_grid(c), 1, 0, &data, s)) != MSR_OK) return st;
    } else {
        const double ip2 = 1.0 / ((double)c->sh.P * c->sh.P);
        double dh = 0.0, dl = 0.0;
        if ((st = fwd_image(c, x, 1.f, c->SB, KA(c, 2), s)) != MSR_OK) return st;
        if ((st = col_psf(c, 2, c->SB, c->SC, s)) != MSR_OK) return st;
        EpiResid er{c->dirty[1], nullptr, c->sh.N};
        c->op->row_resid_fwd(row_args(c, c->SC, c->K[1], nullptr, 0, c->SC, c->sh.Cfull), er, s);
        LAUNCHCHK(c);
        if ((st = col_filth(c, c->SC, c->SC, s)) != MSR_OK) return st;
        if ((st = reduce(c, col_grid(c, c->sh.Cfull), 1, 0, &dh, s)) != MSR_OK) return st;
        if ((st = col_filtl(c, c->SB, c->SL, c->SC, s)) != MSR_OK) return st;
        if ((st = reduce(c, col_grid(c, c->KL), 1, 0, &dl, s)) != MSR_OK) return st;
        data = (dh + dl) * ip2;
    }
    double l1 = 0.0;
    if ((st = image_reduce(c, x, nullptr, 0, &l1, s)) != MSR_OK) return st;
    out[0] = data + lambda * l1;
    out[1] = data;
    out[2] = l1;
    return MSR_OK;
}

msr_status set_low_res(msr_ctx* c, const float* low_res, hipStream_t s) {
    return fwd_image(c, low_res, 1.f, c->SL, c->KL, s);
}

msr_status power_iteration(msr_ctx* c, int step, int max_iter, double rtol, double* theta_out, int* iters_out,
                           hipStream_t s) {
    msr_status st;
    const size_t n = c->sh.img_elems;
    float* v = c->tmp[0];
    float* w = c->tmp[1];
    hipLaunchKernelGGL(start_vector, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, (unsigned long long)c->cfg.seed, n);
    LAUNCHCHK(c);
    double nv2 = 0.0;
    if ((st = image_reduce(c, v, nullptr, 1, &nv2, s)) != MSR_OK) return st;
    if (!(nv2 > 0)) return fail(c, MSR_ERR_NUMERIC, "zero start vector");
    double scale = 1.0 / std::sqrt(nv2);
    double theta = 0.0, prev = -1.0;
    int j = 0;
    for (j = 1; j <= max_iter; ++j) {
        if ((st = fwd_image(c, v, (float)scale, c->SA, KA(c, step), s)) != MSR_OK) return st;
        if ((st = grad_chain(c, step, nullptr, false, s)) != MSR_OK) return st;
        EpiPower ep{v, w, c->sh.N, (float)scale};
        RowArgs a = step == 1 ? row_args(c, c->SB, c->K[0], nullptr, 0, nullptr, 0)
                              : row_args(c, c->SB, c->K[1], c->SC, c->KL, nullptr, 0);
        c->op->row_power(a, ep, s);
        LAUNCHCHK(c);
        double sums[2];
        if ((st = reduce(c, row_grid(c), 2, 0, sums, s)) != MSR_OK) return st;
        // v has unit norm: theta = 2 <v, A v>
        theta = 2.0 * sums[1];
        if (!std::isfinite(theta) || !(sums[0] > 0)) {
            if (sums[0] == 0.0) {
                theta = 0.0;
                break;
            }
            return fail(c, MSR_ERR_NUMERIC, "power iteration diverged at %d", j);
        }
        scale = 1.0 / std::sqrt(sums[0]);
        std::swap(v, w);
        if (prev >= 0 && std::fabs(theta - prev) <= rtol * theta) break;
        prev = theta;
    }
    if (theta_out) *theta_out = theta;
    if (iters_out) *iters_out = std::min(j, max_iter);
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
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return MSR_ERR_INVALID;
    if (hipSetDevice(cfg->device) != hipSuccess) return MSR_ERR_HIP;
    msr_ctx* c = new (std::nothrow) msr_ctx();
    if (!c) return MSR_ERR_OOM;
    c->cfg = *cfg;
    c->sh = s;
    c->lay = make_layout(s);
    c->op = ops_for(s.N, s.padded);
    c->opp = ops_for(s.P, false);
    *out = c;
    return MSR_OK;
}

void msr_destroy(msr_ctx* ctx) { delete ctx; }

const char* msr_last_error(const msr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

msr_status msr_set_workspace(msr_ctx* c, void* dev, size_t bytes) {
    if (!c) return MSR_ERR_INVALID;
    if (!dev || bytes < c->lay.total) return fail(c, MSR_ERR_OOM, "workspace needs %zu bytes", c->lay.total);
    if (reinterpret_cast<uintptr_t>(dev) % kAlign) return fail(c, MSR_ERR_INVALID, "workspace must be 256-byte aligned");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    c->ws = static_cast<char*>(dev);
    c->ws_bytes = bytes;
    const Layout& l = c->lay;
    c->tw = reinterpret_cast<float2*>(c->ws + l.tw);
    c->SA = reinterpret_cast<float2*>(c->ws + l.SA);
    c->SB = reinterpret_cast<float2*>(c->ws + l.SB);
    c->SC = reinterpret_cast<float2*>(c->ws + l.SC);
    c->SL = reinterpret_cast<float2*>(c->ws + l.SL);
    c->hh[0] = reinterpret_cast<float*>(c->ws + l.hh1);
    c->hh[1] = reinterpret_cast<float*>(c->ws + l.hh2);
    c->dirty[0] = reinterpret_cast<float*>(c->ws + l.d1);
    c->dirty[1] = reinterpret_cast<float*>(c->ws + l.d2);
    c->beta[0] = reinterpret_cast<float*>(c->ws + l.b0);
    c->beta[1] = reinterpret_cast<float*>(c->ws + l.b1);
    c->tmp[0] = reinterpret_cast<float*>(c->ws + l.t0);
    c->tmp[1] = reinterpret_cast<float*>(c->ws + l.t1);
    c->partials = reinterpret_cast<double*>(c->ws + l.partials);
    c->scal = reinterpret_cast<double*>(c->ws + l.scal);
    c->colmax = reinterpret_cast<float*>(c->ws + l.colmax);
    // twiddles exp(-2 pi i k / P), computed in double and rounded
    const int P = c->sh.P;
    std::vector<float2> tw(P);
    for (int k = 0; k < P; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)P;
        tw[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    HIPCHK(c, hipMemcpy(c->tw, tw.data(), sizeof(float2) * P, hipMemcpyHostToDevice));
    c->have_psf[0] = c->have_psf[1] = false;
    c->have_theta[0] = c->have_theta[1] = false;
    c->have_filters = false;
    return MSR_OK;
}

msr_status msr_set_dirty_psf(msr_ctx* c, int step, const float* dirty, const float* psf, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!dirty || !psf) return fail(c, MSR_ERR_INVALID, "null image");
    hipStream_t s = S(stream);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    const int N = c->sh.N, P = c->sh.P;
    HIPCHK(c, hipMemcpyAsync(c->dirty[step - 1], dirty, sizeof(float) * c->sh.img_elems, hipMemcpyDeviceToDevice, s));
    float centre = 0.f;
    HIPCHK(c, hipMemcpyAsync(&centre, psf + (size_t)(P / 2) * P + P / 2, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (!(std::fabs(centre - 1.f) <= 1e-5f))
        return fail(c, MSR_ERR_INVALID, "PSF value at (P/2, P/2) is %g, expected 1", (double)centre);
    // h_hat = F(ifftshift PSF): row pass (P rows, unpadded), then column pass in place.
    float2* tmp = c->SB;  // SB and SC are contiguous and hold P x Cpad_psf
    RowArgs ra{};
    ra.spec_out = tmp;
    ra.tw = c->tw;
    ra.partials = c->partials;
    ra.NR = P;
    ra.K_out = c->sh.Cfull;
    EpiLoadShift el{psf, P};
    c->opp->row_loadshift_fwd(ra, el, s);
    LAUNCHCHK(c);
    ColArgs ca{};
    ca.spec_in = tmp;
    ca.spec_out = tmp;
    ca.tw = c->tw;
    ca.partials = c->partials;
    ca.NR = P;
    ca.K = c->sh.Cfull;
    c->opp->col_forward(ca, ModeForward{}, s);
    LAUNCHCHK(c);
    float* hh = c->hh[step - 1];
    hipLaunchKernelGGL(psf_extract, dim3(c->sh.Cfull), dim3(256), 0, s, tmp, c->sh.Tpsf, P, c->sh.T, c->sh.Cfull, hh,
                       c->colmax, c->partials);
    LAUNCHCHK(c);
    if (c->sh.Cpad > c->sh.Cfull) {
        hipLaunchKernelGGL(zero_hh_cols, dim3((P + 255) / 256), dim3(256), 0, s, hh, P, c->sh.T, c->sh.Cfull, c->sh.Cpad);
        LAUNCHCHK(c);
    }
    std::vector<float> colmax(c->sh.Cfull);
    std::vector<double> part(2 * (size_t)c->sh.Cfull);
    HIPCHK(c, hipMemcpyAsync(colmax.data(), c->colmax, sizeof(float) * c->sh.Cfull, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials, sizeof(double) * 2 * c->sh.Cfull, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double mre = 0.0, mim = 0.0;
    for (int k = 0; k < c->sh.Cfull; ++k) {
        mre = std::max(mre, part[2 * k]);
        mim = std::max(mim, part[2 * k + 1]);
    }
    if (!(mre > 0) || !std::isfinite(mre)) return fail(c, MSR_ERR_INVALID, "PSF spectrum is zero or not finite");
    if (mim > 1e-4 * mre) return fail(c, MSR_ERR_INVALID, "PSF is not point symmetric: max|Im h| / max|h| = %g", mim / mre);
    int keep = c->sh.Cfull;
    if (c->cfg.prune_tol > 0) {
        const double thr = c->cfg.prune_tol * mre;
        keep = 1;
        for (int k = 0; k < c->sh.Cfull; ++k)
            if ((double)colmax[k] > thr) keep = k + 1;
    }
    c->K[step - 1] = keep;
    c->have_psf[step - 1] = true;
    c->have_theta[step - 1] = false;
    (void)N;
    return MSR_OK;
}

msr_status msr_set_filters(msr_ctx* c, double ell, double delta, double sigma2, double eta2) {
    if (!c) return MSR_ERR_INVALID;
    if (!(delta > 0) || !(sigma2 > 0) || !(eta2 > 0) || !std::isfinite(ell))
        return fail(c, MSR_ERR_INVALID, "need delta > 0, sigma2 > 0, eta2 > 0");
    c->ell = ell;
    c->delta = delta;
    c->sigma2 = sigma2;
    c->eta2 = eta2;
    FilterCoef f{};
    f.ell = (float)ell;
    f.delta = (float)delta;
    f.inv_sigma2 = (float)(1.0 / sigma2);
    f.inv_eta2 = (float)(1.0 / eta2);
    f.sigma2 = (float)sigma2;
    f.eta2 = (float)eta2;
    f.half_pi_over_delta = (float)(M_PI / (2.0 * delta));
    f.P = c->sh.P;
    c->fc = f;
    // g_L vanishes for r >= ell + delta: columns k_x <= ell + delta can be non-zero.
    const double lim = ell + delta;
    int kl = lim < 0 ? 0 : (int)std::floor(lim) + 1;
    c->KL = std::min(std::max(kl, 0), c->sh.Cfull);
    if (c->KL == 0) c->KL = 1;
    c->have_filters = true;
    c->have_theta[1] = false;
    return MSR_OK;
}

msr_status msr_lipschitz(msr_ctx* c, int step, int max_iter, double rtol, double* theta, int* iters, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if (step != 1 && step != 2) return fail(c, MSR_ERR_INVALID, "step must be 1 or 2");
    if (!c->have_psf[step - 1] || (step == 2 && !c->have_filters))
        return fail(c, MSR_ERR_STATE, "set the PSF (and filters for step 2) first");
    if (max_iter <= 0) max_iter = 200;
    if (!(rtol > 0)) rtol = 1e-6;
    HIPCHK(c, hipSetDevice(c->cfg.device));
    double th = 0.0;
    msr_status st = power_iteration(c, step, max_iter, rtol, &th, iters, S(stream));
    if (st != MSR_OK) return st;
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

static msr_status solve(msr_ctx* c, int step, const msr_solve* opt, const float* low_res, const float* x0,
                        float* model_out, float* image_out, msr_result* res, hipStream_t s) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if (!opt || !model_out) return fail(c, MSR_ERR_INVALID, "null argument");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    if (step == 2 && (!c->have_filters || !low_res)) return fail(c, MSR_ERR_STATE, "step 2 needs filters and low_res");
    if (opt->max_iters < 0 || !(opt->lambda >= 0)) return fail(c, MSR_ERR_INVALID, "bad solve options");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    msr_status st;
    if (!c->have_theta[step - 1]) {
        if ((st = msr_lipschitz(c, step, 200, 1e-6, nullptr, nullptr, s)) != MSR_OK) return st;
        if (!c->have_theta[step - 1]) return fail(c, MSR_ERR_NUMERIC, "zero Lipschitz constant");
    }
    const double theta = c->theta[step - 1];
    const double mu = 1.0 / theta;
    const size_t nb = sizeof(float) * c->sh.img_elems;
    if (x0) {
        HIPCHK(c, hipMemcpyAsync(c->beta[0], x0, nb, hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(c, hipMemsetAsync(c->beta[0], 0, nb, s));
    }
    HIPCHK(c, hipMemcpyAsync(c->beta[1], c->beta[0], nb, hipMemcpyDeviceToDevice, s));
    if (step == 2 && (st = set_low_res(c, low_res, s)) != MSR_OK) return st;
    if ((st = fwd_image(c, c->beta[0], 1.f, c->SA, KA(c, step), s)) != MSR_OK) return st;

    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, s));
    const bool rule = opt->check_every > 0 && opt->f_ref != 0.0 && opt->tol > 0;
    double F[3] = {0, 0, 0};
    int k = 0;
    bool conv = false;
    double ttt = -1.0;
    for (k = 1; k <= opt->max_iters; ++k) {
        if ((st = iterate(c, step, k, mu, opt->lambda, s)) != MSR_OK) break;
        if (opt->check_every > 0 && (k % opt->check_every == 0)) {
            if ((st = objective_at(c, step, opt->lambda, c->beta[k & 1], F, s)) != MSR_OK) break;
            if (!std::isfinite(F[0])) {
                st = fail(c, MSR_ERR_NUMERIC, "objective is not finite at iteration %d", k);
                break;
            }
            if (rule && (F[0] - opt->f_ref) / std::fabs(opt->f_ref) <= opt->tol) {
                conv = true;
                HIPCHK(c, hipEventRecord(e1, s));
                HIPCHK(c, hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                ttt = ms;
                break;
            }
        }
    }
    const int done = std::min(k, opt->max_iters);
    if (st != MSR_OK) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (res) res->iters = done;
        return st;
    }
    HIPCHK(c, hipEventRecord(e1, s));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    const float* bK = c->beta[done & 1];
    if ((st = objective_at(c, step, opt->lambda, bK, F, s)) != MSR_OK) return st;
    if (!std::isfinite(F[0])) {
        if (res) res->iters = done;
        return fail(c, MSR_ERR_NUMERIC, "objective is not finite at the end (%d iterations)", done);
    }
    HIPCHK(c, hipMemcpyAsync(model_out, bK, nb, hipMemcpyDeviceToDevice, s));
    if (image_out) {
        // i_L = beta + (i~ - H beta) = beta - r
        if ((st = fwd_image(c, bK, 1.f, c->SB, c->K[step - 1], s)) != MSR_OK) return st;
        if ((st = col_psf(c, step, c->SB, c->SC, s)) != MSR_OK) return st;
        EpiResid er{c->dirty[step - 1], c->tmp[0], c->sh.N};
        c->op->row_resid(row_args(c, c->SC, c->K[step - 1], nullptr, 0, nullptr, 0), er, s);
        LAUNCHCHK(c);
        const size_t n = c->sh.img_elems;
        hipLaunchKernelGGL(image_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, image_out, bK,
                           (const float*)c->tmp[0], 1.f, -1.f, n);
        LAUNCHCHK(c);
    }
    HIPCHK(c, hipStreamSynchronize(s));
    if (res) {
        res->iters = done;
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

msr_status msr_step1_low_res(msr_ctx* c, const msr_solve* opt, const float* x0, float* model_out, float* image_out,
                             msr_result* res, void* stream) {
    return solve(c, 1, opt, nullptr, x0, model_out, image_out, res, S(stream));
}

msr_status msr_step2_full_res(msr_ctx* c, const msr_solve* opt, const float* low_res, const float* x0,
                              float* model_out, msr_result* res, void* stream) {
    return solve(c, 2, opt, low_res, x0, model_out, nullptr, res, S(stream));
}

msr_status msr_objective(msr_ctx* c, int step, double lambda, const float* x, const float* low_res, double out[3],
                         void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if ((step != 1 && step != 2) || !x || !out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    if (step == 2 && (!c->have_filters || !low_res)) return fail(c, MSR_ERR_STATE, "step 2 needs filters and low_res");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    msr_status st;
    if (step == 2 && (st = set_low_res(c, low_res, s)) != MSR_OK) return st;
    return objective_at(c, step, lambda, x, out, s);
}

msr_status msr_gradient(msr_ctx* c, int step, const float* x, const float* low_res, float* grad_out, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if ((step != 1 && step != 2) || !x || !grad_out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    if (step == 2 && (!c->have_filters || !low_res)) return fail(c, MSR_ERR_STATE, "step 2 needs filters and low_res");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    msr_status st;
    if (step == 2 && (st = set_low_res(c, low_res, s)) != MSR_OK) return st;
    if ((st = fwd_image(c, x, 1.f, c->SA, KA(c, step), s)) != MSR_OK) return st;
    if ((st = grad_chain(c, step, c->dirty[step - 1], true, s)) != MSR_OK) return st;
    EpiStore es{grad_out, c->sh.N, 2.f};
    RowArgs a = step == 1 ? row_args(c, c->SB, c->K[0], nullptr, 0, nullptr, 0)
                          : row_args(c, c->SB, c->K[1], c->SC, c->KL, nullptr, 0);
    c->op->row_store(a, es, s);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(s));
    return MSR_OK;
}

msr_status msr_apply_psf(msr_ctx* c, int step, const float* x, float* out, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if ((step != 1 && step != 2) || !x || !out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    msr_status st;
    if ((st = fwd_image(c, x, 1.f, c->SB, c->K[step - 1], s)) != MSR_OK) return st;
    if ((st = col_psf(c, step, c->SB, c->SC, s)) != MSR_OK) return st;
    EpiStore es{out, c->sh.N, 1.f};
    c->op->row_store(row_args(c, c->SC, c->K[step - 1], nullptr, 0, nullptr, 0), es, s);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(s));
    return MSR_OK;
}

msr_status msr_get_spectrum(msr_ctx* c, int step, double* host_out, int* kept, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if ((step != 1 && step != 2) || !host_out) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    const int P = c->sh.P, T = c->sh.T, C = c->sh.Cfull;
    std::vector<float> hh(c->sh.hh_elems);
    HIPCHK(c, hipMemcpyAsync(hh.data(), c->hh[step - 1], sizeof(float) * hh.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const double p2 = (double)P * P;
    const int K = c->K[step - 1];
    for (int ky = 0; ky < P; ++ky)
        for (int kx = 0; kx < C; ++kx)
            host_out[(size_t)ky * C + kx] = kx < K ? (double)hh[((size_t)(kx / T) * P + ky) * T + kx % T] * p2 : 0.0;
    if (kept) *kept = K;
    return MSR_OK;
}

msr_status msr_estimate_sigma2(msr_ctx* c, const float* dirty, double* sigma2, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if (!dirty || !sigma2) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    const int n = c->sh.N;
    const size_t nw = (size_t)(n - 4) * (n - 4);
    const int blocks = (int)std::min<size_t>(1024, (nw + 255) / 256);
    hipLaunchKernelGGL(window_variance, dim3(blocks), dim3(256), 0, s, dirty, n, c->partials);
    LAUNCHCHK(c);
    double tot = 0.0;
    msr_status st = reduce(c, blocks, 1, 8, &tot, s);
    if (st != MSR_OK) return st;
    *sigma2 = tot / (double)nw;
    return MSR_OK;
}

msr_status msr_default_lambda(msr_ctx* c, int step, int cycle, double cc, double* lambda, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if ((step != 1 && step != 2) || !lambda || cycle < 1) return fail(c, MSR_ERR_INVALID, "bad arguments");
    if (!c->have_psf[step - 1]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(%d) first", step);
    HIPCHK(c, hipSetDevice(c->cfg.device));
    double s2 = 0.0;
    msr_status st = image_reduce(c, c->dirty[step - 1], nullptr, 1, &s2, S(stream));
    if (st != MSR_OK) return st;
    *lambda = cc * std::sqrt(s2) * std::ldexp(1.0, cycle - 1);
    return MSR_OK;
}

msr_status msr_time_pass(msr_ctx* c, int which, int reps, double* ms_out, double* bytes_out, void* stream) {
    if (!ready(c)) return fail(c, MSR_ERR_OOM, "no workspace");
    if (!c->have_psf[0]) return fail(c, MSR_ERR_STATE, "set_dirty_psf(1) first");
    if (reps <= 0 || which < 0 || which > 2) return fail(c, MSR_ERR_INVALID, "bad arguments");
    HIPCHK(c, hipSetDevice(c->cfg.device));
    hipStream_t s = S(stream);
    const int N = c->sh.N, P = c->sh.P, K = c->K[0];
    const double spec = (double)N * K * 8.0, img = (double)N * N * 4.0;
    double bytes = 0.0;
    auto launch = [&]() -> msr_status {
        if (which == 0) return col_psf(c, 1, c->SA, c->SB, s);
        if (which == 1) {
            EpiResid er{c->dirty[0], nullptr, N};
            c->op->row_resid_fwd(row_args(c, c->SB, K, nullptr, 0, c->SC, K), er, s);
            LAUNCHCHK(c);
            return MSR_OK;
        }
        EpiUpdate u{};
        u.b1 = c->beta[0];
        u.b2 = c->beta[1];
        u.ld = N;
        u.two_mu = 0.f;
        u.thr = 0.f;
        u.t_prev = 0.f;
        u.t_cur = 0.f;
        u.positivity = c->cfg.positivity;
        c->op->row_update_fwd(row_args(c, c->SB, K, nullptr, 0, c->SC, K), u, s);
        LAUNCHCHK(c);
        return MSR_OK;
    };
    if (which == 0) bytes = 2 * spec + (double)P * K * 4.0;
    else if (which == 1) bytes = 2 * spec + img;
    else bytes = 2 * spec + 3 * img;
    msr_status st = launch();  // warm
    if (st != MSR_OK) return st;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, s));
    for (int r = 0; r < reps && st == MSR_OK; ++r) st = launch();
    HIPCHK(c, hipEventRecord(e1, s));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != MSR_OK) return st;
    if (ms_out) *ms_out = ms / reps;
    if (bytes_out) *bytes_out = bytes;
    return MSR_OK;
}

}  // extern "C"
