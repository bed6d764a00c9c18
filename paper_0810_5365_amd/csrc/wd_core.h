// Host-side core of libwdirac: context, gauge objects, error reporting and
// the launch entry points of each kernel family.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>

#include "wd_device.h"
#include "wdirac.h"

namespace wd {

// thread-local error text behind wd_last_error()
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define WD_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            ::wd::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return e_ == hipErrorOutOfMemory ? WD_ENOMEM : WD_EHIP;                                \
        }                                                                                          \
    } while (0)

#define WD_TRY(expr)                      \
    do {                                  \
        wd_status s_ = (expr);            \
        if (s_ != WD_OK) return s_;       \
    } while (0)

#define WD_LAUNCHED()                                                                   \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) {                                                         \
            ::wd::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
            return WD_EHIP;                                                             \
        }                                                                               \
    } while (0)

// Launch shape of one kernel: workgroup size, XCD-aware block remap, and
// non-temporal (streaming) link loads.
struct TuneParam {
    int block = 64;
    int remap = 1;
    int nt = 1;   // non-temporal link loads
    int pf = 1;   // software-pipelined directions
    int rhs_inner = 1;   // several rhs: interleave them with the site tiles
    int zb = 0;          // z-blocked site traversal depth (0: natural order)
    int mf = 0;          // 16-bit, 12-real, 16k rhs: colour multiply on the matrix cores
};

inline bool valid_prec(int p) { return p >= WD_F64 && p <= WD_BF16; }
inline bool valid_subset(int s) { return s >= WD_FULL && s <= WD_ODD; }
inline bool valid_recon(int r) { return r == WD_RECON_12 || r == WD_RECON_18; }

// Bytes of one half field (Vh sites of one parity in planes ps apart, one rhs) at precision p.
inline size_t half_bytes(const Geom& g, int p) { return spinor_site_bytes(p) * (size_t)g.ps; }
// Reliable-update threshold: delta < 0 selects the default for the sloppy precision.
inline double default_delta(int prec)
{
    return prec == WD_F32 ? 1e-5 : (prec == WD_F16 ? 1e-2 : (prec == WD_BF16 ? 3e-2 : 0.1));
}
inline double resolve_delta(double delta, int prec) { return delta < 0.0 ? default_delta(prec) : delta; }
inline size_t halves_of(int subset, int nrhs) { return (size_t)nrhs * (subset == WD_FULL ? 2 : 1); }

wd_status make_geom(const wd_lattice* lat, Geom* g);

} // namespace wd

struct wd_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    // named grow-only workspace buffers
    std::map<std::string, std::pair<void*, size_t>> ws;
    // reduction scratch: per-block partial sums and final scalars
    double* partials = nullptr;
    size_t npartials = 0;
    double* dres = nullptr;    // device results
    double* hres = nullptr;    // pinned host copy (mapped: kernels write it directly)
    double* hres_dev = nullptr;   // device address of hres, or null if it is not mapped
    std::map<std::string, wd::TuneParam> tune;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // hopping-term applications queued on one parity (per rhs), plain and fused: the solvers
    // report their difference as the operator work of a solve
    long long hops = 0;
};

struct wd_gauge_s {
    wd_context ctx = nullptr;
    wd_lattice lat{};
    int recon = 12;
    wd::Geom geom{};
    double* canon = nullptr;       // float64 canonical links on the device
    void* packed[4] = {nullptr, nullptr, nullptr, nullptr};   // per wd_prec
    bool uploaded = false;
    bool gf = false;               // temporal gauge fixed by wd_gauge_fix_temporal
};

namespace wd {

wd_status ws_get(wd_context ctx, const std::string& name, size_t bytes, void** out);
wd_status ensure_reduction(wd_context ctx, size_t nblocks);
wd_status gauge_links(wd_gauge g, int prec, const void** out);
TuneParam tune_lookup(wd_context ctx, const std::string& key);

// ---- dslash.hip -------------------------------------------------------------
struct DslashCall {
    const void* gauge = nullptr;   // packed links at `prec`
    const void* in = nullptr;      // input half field, rhs 0 (parity 1 - par)
    void* out = nullptr;           // output half field, rhs 0 (parity par)
    const void* x = nullptr;       // xpay half field (parity par), or null
    long long in_stride = 0, out_stride = 0, x_stride = 0;   // bytes between rhs
    double a = 0.0, b = 1.0;       // out = a x + b D in  (or b D in without x)
    int par = 0;
    int nrhs = 1;
    int dagger = 0;
    int prec = WD_F32;
    int recon = 12;
    int gf = 0;                    // links in temporal gauge (unit t-links but the last slice)
};
wd_status launch_dslash(wd_context ctx, const Geom& g, const DslashCall& c);
wd_status launch_dslash_tuned(wd_context ctx, const Geom& g, const DslashCall& c, const TuneParam& tp);
// tuning-table key of a launch
std::string dslash_key(const Geom& g, const DslashCall& c);
// ---- dslash_red.hip: a fused-update launch (c.x set, one rhs) that also sums a reduction of
// its result per workgroup: RED_NORM |out|^2 (1 value); RED_XDOT <out, x> and |out|^2,
// RED_YDOT <y, out> and |out|^2 (3 values; y a half field at c.prec); these without the
// dagger; RED_NORM also with the dagger in float32 and float64.  In float64, with or without
// the dagger: RED_RESID stores out = y - (a x + b D in) and sums |out|^2; RED_YDIFF sums
// |y - out|^2.  RED_RESLO (float64, no dagger) is RED_RESID with out stored in float32 and the
// sum taken before that rounding.  RED_CGR (every precision, with the dagger; the CG residual
// update) does not store a x + b D in: it updates r -= alpha (a x + b D in) in place, r = c.out
// held at the accumulation precision (float64 for a float64 launch, else float32), alpha =
// coef[0] read from device memory, and sums |r|^2 of the stored r.  Value v of workgroup k
// lands in partials[v * nblocks + k]; the caller sizes partials for 3 values per workgroup of
// 64 sites.
enum { RED_NORM = 1, RED_XDOT = 2, RED_YDOT = 3, RED_RESID = 4, RED_YDIFF = 5, RED_RESLO = 6, RED_CGR = 7 };
constexpr int red_values(int red) { return red == RED_XDOT || red == RED_YDOT ? 3 : 1; }
wd_status launch_dslash_red(wd_context ctx, const Geom& g, const DslashCall& c, int red, const void* y,
                            double* partials, int* nblocks, const double* coef = nullptr);
// ---- dslash_mrhs.hip: 16 rhs per wave with the colour multiply on the matrix cores ----
bool mrhs_eligible(const DslashCall& c);
wd_status launch_dslash_mrhs(wd_context ctx, const Geom& g, const DslashCall& c);

// ---- pack.hip ----------------------------------------------------------------
wd_status launch_pack_gauge(wd_context ctx, const Geom& g, int prec, int recon, const double* canon, void* out);
wd_status launch_spinor_pack(wd_context ctx, const Geom& g, int subset, int prec, int nrhs, const double* canon,
                             void* packed, bool unpack);
wd_status launch_convert(wd_context ctx, const Geom& g, size_t nhalves, int sp, const void* src, int dp, void* dst);

// ---- blas.hip ----------------------------------------------------------------
// All operate on `nhalves` consecutive half fields.  Reductions leave their
// float64 results in ctx->dres and (when `fetch`) copy them to ctx->hres.
wd_status blas_dot(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* a, const void* b, bool fetch);
wd_status blas_norm2(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* a, bool fetch);
wd_status blas_caxpy(wd_context ctx, const Geom& g, size_t nhalves, int prec, double ar, double ai, const void* x, void* y);
wd_status blas_zero(wd_context ctx, const Geom& g, size_t nhalves, int prec, void* x);
// y = a*x + b*y with real a, b (y, x may differ in precision: x at px, y at py)
wd_status blas_axpby(wd_context ctx, const Geom& g, size_t nhalves, int px, const void* x, double a, int py, void* y, double b);
// CG with its scalars on the device, in dres[CG_SLOT + i] (and the sums in hres[CG_SLOT + i]):
// CG_RR the current sloppy ||r||^2, CG_ALPHA = rr / pap, CG_BETA, and the two the host reads,
// CG_PAP <p, A p> and CG_RRNEW (adjacent).
constexpr int CG_SLOT = 248, CG_RR = 0, CG_ALPHA = 1, CG_BETA = 2, CG_PAP = 3, CG_RRNEW = 4, CG_NSLOTS = 5;
// finish the one-value partials in ctx->partials[0 .. nblk): mode 0 sets pap and alpha, mode 1
// sets rr_new, beta = rr_new / rr and then rr = rr_new
wd_status blas_cg_coef(wd_context ctx, int nblk, int mode);
// rr and beta from the host (after a reliable update)
wd_status blas_cg_set(wd_context ctx, double rr, double beta);
// Before an iteration: mark hres[CG_SLOT + CG_PAP] and [CG_SLOT + CG_RRNEW] as pending.  After
// queueing it: wait until the coefficient kernels have written both (spinning on the mapped
// host buffer; with no mapped buffer, a stream synchronisation)
void blas_cg_arm(wd_context ctx);
wd_status blas_cg_wait(wd_context ctx);
// x += alpha p (xmode 0), x = alpha p (1) or x untouched (2); then q = r + beta p (q may be p).
// x, r at pacc; p, q at pop
wd_status blas_cg_xp(wd_context ctx, const Geom& g, size_t nhalves, int pacc, void* x, int xmode, const void* r,
                     int pop, const void* p, void* q);
wd_status fetch_results(wd_context ctx, int n);
// true when the float64 field (nhalves half fields) is all zeros (a norm sweep; false on error)
bool is_zero_f64(wd_context ctx, const Geom& g, size_t nhalves, const void* x);
// dres[slot + v] (and hres) = the sum of partials[v * nblk .. (v + 1) * nblk) for v < n, in a
// fixed order; not fetched
wd_status reduce_partials(wd_context ctx, int nblk, int n, int slot);
// out = sum_{i < n} (cre[i] + i cim[i]) x[i], n <= 3, out may alias an input; with r0 non-null also
// ||out||^2 and <r0, out> (dres/hres 0; 1, 2)
wd_status blas_lincomb(wd_context ctx, const Geom& g, size_t nhalves, int prec, int n, const void* const* x,
                       const double* cre, const double* cim, void* out, const void* r0, bool fetch);
// one EVEN half each: xs += alpha p + omega s; rs = s - omega t, with ||rs||^2, Re and Im <r0, rs>
// in slots 0, 1, 2
wd_status blas_bicg_xr(wd_context ctx, const Geom& g, int prec, void* xs, const void* p, const void* s, const void* t,
                       const void* r0, void* rs, double alpha_re, double alpha_im, double omega_re, double omega_im,
                       bool fetch);
// h_i = <V_i, w> for i < k, V_i = V + i * vstride bytes; complex results in dres[slot + 2i],
// dres[slot + 2i + 1] (and hres); with_norm adds ||w||^2 in dres[slot + 2k]
wd_status blas_mdot(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* V, size_t vstride, int k,
                    const void* w, bool with_norm, bool fetch, int slot = 0);
// out = scale (w + sum_i c_i V_i), complex c_i = (coef[2i], coef[2i + 1]), i < k <= WD_MAXPY; out may be w
constexpr int WD_MAXPY = 64;
wd_status blas_maxpy(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* V, size_t vstride, int k,
                     const double* coef, const void* w, double scale, void* out);
// w -= sum_i h1_i V_i (h1 = dres[slot1 ..], float-rounded as in blas_maxpy_dev), then
// <V_i, w> in dres/hres[2i], [2i + 1] for i < k <= MGS_KMAX and ||w||^2 in [2 MGS_KMAX]; fetched
constexpr int MGS_KMAX = 16;
wd_status blas_maxpy_mdot(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* V, size_t vstride, int k,
                          int slot1, void* w);
// the same with c_i = sign (dres[slot + 2i], dres[slot + 2i + 1]) read on the device (no host round trip)
wd_status blas_maxpy_dev(wd_context ctx, const Geom& g, size_t nhalves, int prec, const void* V, size_t vstride, int k,
                         int slot, float sign, const void* w, double scale, void* out);

// ---- ptconv.hip ----------------------------------------------------------------
// zero_par >= 0: input sites of that parity are zero (the matrix-core path skips the paths
// that read only them); even_out: only the even output sites are needed.
// spin_in / spin_out (matrix-core path, 4 spin channels, one sample): the input's even sites
// come from an EVEN float32 spinor half field (zero_par = 1), the even outputs go into one
// (even_out); ptconv_spin_io tells whether a layer shape can do that.  half_feat (matrix-core
// path, one sample, the layers of a 4 -> 8 -> ... -> 8 -> 4 network with spinor input first and
// spinor output last): the feature tensors in between hold bf16 pairs instead of float2.
wd_status ptconv_fwd(wd_gauge g, int cin, int cout, int wprec, const void* W, const void* in, void* out, int nsamples,
                     int zero_par = -1, bool even_out = false, const void* spin_in = nullptr, void* spin_out = nullptr,
                     bool half_feat = false);
bool ptconv_spin_io(int wprec, int cin, int cout);
// FULL float32 spinor <-> 4-channel features; even_only: the spinor is one EVEN half
// field (odd sites are zero on the way in and dropped on the way out).
wd_status launch_spinor_features(wd_context ctx, const Geom& g, int nsamples, void* spinor, void* feat,
                                 bool to_features, bool even_only = false);

} // namespace wd
