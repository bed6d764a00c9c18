// C ABI of libwdirac: argument checking, object lifetimes and operator
// composition on top of the kernels in dslash.hip, pack.hip and blas.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "wd_core.h"
#include "wd_ops.h"

namespace wd {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

wd_status make_geom(const wd_lattice* lat, Geom* g)
{
    if (!lat) {
        set_error("lattice is NULL");
        return WD_EINVAL;
    }
    long long V = 1;
    for (int d = 0; d < 4; ++d) {
        const int L = lat->dims[d];
        if (L < 2 || (L & 1)) {
            set_error("lattice dim %d = %d must be even and >= 2", d, L);
            return WD_ESHAPE;
        }
        if (lat->bc[d] != 1 && lat->bc[d] != -1) {
            set_error("boundary condition %d = %d must be +1 or -1", d, lat->bc[d]);
            return WD_EINVAL;
        }
        V *= L;
        if (plane_stride(V / 2) >= (1ll << 31)) {
            set_error("half volume exceeds 2^31 - 1");
            return WD_ESHAPE;
        }
    }
    memset(g, 0, sizeof *g);
    for (int d = 0; d < 4; ++d) {
        g->L[d] = lat->dims[d];
        g->bcf[d] = (float)lat->bc[d];
        g->bcd[d] = (double)lat->bc[d];
    }
    g->Xh = g->L[0] / 2;
    g->Vh = (int)(V / 2);
    g->ps = (int)plane_stride(V / 2);
    g->st[0] = 1;
    g->st[1] = g->Xh;
    g->st[2] = g->Xh * g->L[1];
    g->st[3] = g->Xh * g->L[1] * g->L[2];
    g->dxh = make_fastdiv((uint32_t)g->Xh);
    g->dy = make_fastdiv((uint32_t)g->L[1]);
    g->dz = make_fastdiv((uint32_t)g->L[2]);
    return WD_OK;
}

wd_status ws_get(wd_context ctx, const std::string& name, size_t bytes, void** out)
{
    auto& slot = ctx->ws[name];
    if (slot.second < bytes) {
        if (slot.first) {
            WD_HIP(hipStreamSynchronize(ctx->stream));
            WD_HIP(hipFree(slot.first));
            slot.first = nullptr;
            slot.second = 0;
        }
        void* p = nullptr;
        WD_HIP(hipMalloc(&p, bytes));
        slot.first = p;
        slot.second = bytes;
    }
    *out = slot.first;
    return WD_OK;
}

wd_status ensure_reduction(wd_context ctx, size_t n)
{
    if (ctx->npartials >= n) return WD_OK;
    if (ctx->partials) {
        WD_HIP(hipStreamSynchronize(ctx->stream));
        WD_HIP(hipFree(ctx->partials));
        ctx->partials = nullptr;
    }
    WD_HIP(hipMalloc(&ctx->partials, n * sizeof(double)));
    ctx->npartials = n;
    return WD_OK;
}

TuneParam tune_lookup(wd_context ctx, const std::string& key)
{
    // WD_DSLASH_MFMA forces the matrix-core multi-rhs path on (1) or off (0), tuned or not
    const char* mf = getenv("WD_DSLASH_MFMA");
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
        TuneParam tp = it->second;
        if (mf) tp.mf = atoi(mf);
        return tp;
    }
    TuneParam tp;
    if (mf) tp.mf = atoi(mf);
    if (const char* e = getenv("WD_DSLASH_BLOCK")) tp.block = atoi(e);
    if (const char* e = getenv("WD_DSLASH_REMAP")) tp.remap = atoi(e);
    if (const char* e = getenv("WD_DSLASH_NT")) tp.nt = atoi(e);
    if (const char* e = getenv("WD_DSLASH_PF")) tp.pf = atoi(e);
    if (const char* e = getenv("WD_DSLASH_RHS_INNER")) tp.rhs_inner = atoi(e);
    if (const char* e = getenv("WD_DSLASH_ZB")) tp.zb = atoi(e);
    return tp;
}

wd_status gauge_links(wd_gauge g, int prec, const void** out)
{
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    if (!g->packed[prec]) {
        void* p = nullptr;
        const size_t bytes = 8 * link_site_bytes(prec, g->recon) * (size_t)g->geom.ps;
        WD_HIP(hipSetDevice(g->ctx->device));
        WD_HIP(hipMalloc(&p, bytes));
        wd_status s = launch_pack_gauge(g->ctx, g->geom, prec, g->recon, g->canon, p);
        if (s != WD_OK) {
            hipFree(p);
            return s;
        }
        WD_HIP(hipStreamSynchronize(g->ctx->stream));
        g->packed[prec] = p;
    }
    *out = g->packed[prec];
    return WD_OK;
}

// ---- operator composition --------------------------------------------------------
// Half field (rhs r, parity par) of a field of `subset` at precision prec.
static inline long long rhs_stride(const Geom& g, int subset, int prec)
{
    return (long long)half_bytes(g, prec) * (subset == WD_FULL ? 2 : 1);
}

static DslashCall half_call(wd_gauge g, const void* links, int prec, int par, int dagger, int nrhs, const void* in,
                           long long in_stride, void* out, long long out_stride, const void* x, long long x_stride,
                           double a, double b)
{
    DslashCall c;
    c.gauge = links;
    c.in = in;
    c.out = out;
    c.x = x;
    c.in_stride = in_stride;
    c.out_stride = out_stride;
    c.x_stride = x_stride;
    c.a = a;
    c.b = b;
    c.par = par;
    c.nrhs = nrhs;
    c.dagger = dagger;
    c.prec = prec;
    c.recon = g->recon;
    c.gf = g->gf ? 1 : 0;
    return c;
}

wd_status hop_half(wd_gauge g, int prec, int par, int dagger, int nrhs, const void* in, long long in_stride, void* out,
                   long long out_stride, const void* x, long long x_stride, double a, double b)
{
    const void* links = nullptr;
    WD_TRY(gauge_links(g, prec, &links));
    return launch_dslash(g->ctx, g->geom,
                         half_call(g, links, prec, par, dagger, nrhs, in, in_stride, out, out_stride, x, x_stride, a, b));
}

// precision of the field a fused reduction stores
static int red_out_prec(int red, int prec)
{
    if (red == RED_RESLO) return WD_F32;
    if (red == RED_CGR) return prec == WD_F64 ? WD_F64 : WD_F32;
    return prec;
}

wd_status op_M_red_partials(wd_gauge g, double kappa, int subset, int dagger, int prec, const void* in, void* out,
                            int red, const void* y, const double* coef, int* nblk, void* hop_out)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    const long long hb = (long long)half_bytes(G, prec);
    const long long hbo = (long long)half_bytes(G, red_out_prec(red, prec));
    const void* links = nullptr;
    WD_TRY(gauge_links(g, prec, &links));
    WD_TRY(ensure_reduction(ctx, 3 * (((size_t)G.Vh + 63) / 64)));
    if (red_values(red) != 1) {
        set_error("fused reduction %d: more than one value per workgroup", red);
        return WD_EUNSUPPORTED;
    }
    if (subset == WD_FULL) {   // out_p = in_p - kappa D in_{1-p} for both parities, their sums side by side
        int n[2] = {0, 0};
        for (int par = 0; par < 2; ++par) {
            const char* yp = y ? (const char*)y + par * hb : nullptr;
            WD_TRY(launch_dslash_red(ctx, G, half_call(g, links, prec, par, dagger, 1, (const char*)in + (1 - par) * hb,
                                                       2 * hb, (char*)out + par * hbo, 2 * hbo,
                                                       (const char*)in + par * hb, 2 * hb, 1.0, -kappa),
                                     red, yp, ctx->partials + n[0], &n[par], coef));
        }
        *nblk = n[0] + n[1];
        return WD_OK;
    }
    void* tmp = hop_out;
    if (!tmp) WD_TRY(ws_get(ctx, "op_M.tmp", (size_t)hb, &tmp));
    const int par = subset == WD_EVEN ? 0 : 1;
    WD_TRY(hop_half(g, prec, 1 - par, dagger, 1, in, hb, tmp, hb, nullptr, 0, 0.0, 1.0));
    return launch_dslash_red(ctx, G, half_call(g, links, prec, par, dagger, 1, tmp, hb, out, hbo, in, hb, 1.0,
                                               -kappa * kappa), red, y, ctx->partials, nblk, coef);
}

wd_status op_M_red(wd_gauge g, double kappa, int subset, int dagger, int prec, const void* in, void* out, int red,
                   const void* y, int slot, void* hop_out)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    const long long hb = (long long)half_bytes(G, prec);
    const void* links = nullptr;
    WD_TRY(gauge_links(g, prec, &links));
    WD_TRY(ensure_reduction(ctx, 3 * (((size_t)G.Vh + 63) / 64)));
    if (subset == WD_FULL || red_values(red) == 1) {
        int n = 0;
        WD_TRY(op_M_red_partials(g, kappa, subset, dagger, prec, in, out, red, y, nullptr, &n, hop_out));
        return reduce_partials(ctx, n, 1, slot);
    }
    void* tmp = hop_out;
    if (!tmp) WD_TRY(ws_get(ctx, "op_M.tmp", (size_t)hb, &tmp));
    const int par = subset == WD_EVEN ? 0 : 1;
    int n = 0;
    WD_TRY(hop_half(g, prec, 1 - par, dagger, 1, in, hb, tmp, hb, nullptr, 0, 0.0, 1.0));
    WD_TRY(launch_dslash_red(ctx, G, half_call(g, links, prec, par, dagger, 1, tmp, hb, out, hb, in, hb, 1.0,
                                               -kappa * kappa), red, y, ctx->partials, &n));
    return reduce_partials(ctx, n, red_values(red), slot);
}

wd_status eo_finish(wd_gauge g, double kappa, const void* b, void* x, double* rr, const void* doe_xe, double schur_rr)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    const long long hb = (long long)half_bytes(G, WD_F64), h32 = (long long)half_bytes(G, WD_F32);
    const char* b_e = (const char*)b;
    char* x_e = (char*)x;
    const void* links = nullptr;
    WD_TRY(gauge_links(g, WD_F64, &links));
    WD_TRY(ensure_reduction(ctx, 3 * (((size_t)G.Vh + 63) / 64)));
    // x_o = b_o + kappa D_oe x_e
    if (doe_xe) {
        const void* in[2] = {b_e + hb, doe_xe};
        const double cr[2] = {1.0, kappa}, ci[2] = {0.0, 0.0};
        WD_TRY(blas_lincomb(ctx, G, 1, WD_F64, 2, in, cr, ci, x_e + hb, nullptr, false));
        *rr = schur_rr;   // the even rows are bhat - Mhat x_e, whose norm^2 the solver holds
        return WD_OK;
    } else {
        WD_TRY(hop_half(g, WD_F64, 1, 0, 1, x_e, hb, x_e + hb, hb, b_e + hb, hb, 1.0, kappa));
    }
    // the even rows of b - M x: b_e - (x_e - kappa D_eo x_o), summed in float64 (the residual
    // itself is kept only in float32)
    void* t = nullptr;
    WD_TRY(ws_get(ctx, "eo_finish.r", (size_t)h32, &t));
    int n = 0;
    WD_TRY(launch_dslash_red(ctx, G, half_call(g, links, WD_F64, 0, 0, 1, x_e + hb, hb, t, h32, x_e, hb, 1.0, -kappa),
                             RED_RESLO, b_e, ctx->partials, &n));
    WD_TRY(reduce_partials(ctx, n, 1, 0));
    WD_TRY(fetch_results(ctx, 1));
    *rr = ctx->hres[0];
    return WD_OK;
}

wd_status op_dslash(wd_gauge g, int subset, int dagger, int prec, int nrhs, const void* in, void* out, const void* x,
                    double a, double b)
{
    const Geom& G = g->geom;
    const long long hb = (long long)half_bytes(G, prec);
    if (subset == WD_FULL) {
        for (int par = 0; par < 2; ++par) {
            WD_TRY(hop_half(g, prec, par, dagger, nrhs, (const char*)in + (1 - par) * hb, 2 * hb, (char*)out + par * hb,
                            2 * hb, x ? (const char*)x + par * hb : nullptr, 2 * hb, a, b));
        }
        return WD_OK;
    }
    const int par = subset == WD_EVEN ? 0 : 1;
    return hop_half(g, prec, par, dagger, nrhs, in, hb, out, hb, x, hb, a, b);
}

wd_status op_M(wd_gauge g, double kappa, int subset, int dagger, int prec, int nrhs, const void* in, void* out)
{
    if (subset == WD_FULL) return op_dslash(g, WD_FULL, dagger, prec, nrhs, in, out, in, 1.0, -kappa);
    const Geom& G = g->geom;
    const long long hb = (long long)half_bytes(G, prec);
    void* tmp = nullptr;
    WD_TRY(ws_get(g->ctx, "op_M.tmp", (size_t)hb * nrhs, &tmp));
    const int par = subset == WD_EVEN ? 0 : 1;
    // tmp (other parity) = D in ; out = in - kappa^2 D tmp.  out may be in itself: the second
    // launch reads in only as its x, at the site it writes (callers inside the library use this)
    WD_TRY(hop_half(g, prec, 1 - par, dagger, nrhs, in, hb, tmp, hb, nullptr, 0, 0.0, 1.0));
    return hop_half(g, prec, par, dagger, nrhs, tmp, hb, out, hb, in, hb, 1.0, -kappa * kappa);
}

wd_status op_MdagM(wd_gauge g, double kappa, int subset, int prec, int nrhs, const void* in, void* out)
{
    const Geom& G = g->geom;
    if (subset != WD_FULL) {
        // out = Mhat in, then Mhat^dagger applied to out in place: tmp = D^dag out, and
        // out = out - k^2 D^dag tmp, whose fused update reads x at the very site it writes.
        // Three half fields (in, tmp, out) instead of four: the launches read spinors the
        // 256 MB last-level cache still holds (measured: a launch sequence touching three
        // fields runs 5-7% faster per launch than one touching four).
        const long long hb = (long long)half_bytes(G, prec);
        const int par = subset == WD_EVEN ? 0 : 1;
        void* tmp = nullptr;
        WD_TRY(ws_get(g->ctx, "op_M.tmp", (size_t)hb * nrhs, &tmp));
        WD_TRY(op_M(g, kappa, subset, 0, prec, nrhs, in, out));
        WD_TRY(hop_half(g, prec, 1 - par, 1, nrhs, out, hb, tmp, hb, nullptr, 0, 0.0, 1.0));
        return hop_half(g, prec, par, 1, nrhs, tmp, hb, out, hb, out, hb, 1.0, -kappa * kappa);
    }
    void* t = nullptr;
    WD_TRY(ws_get(g->ctx, "op_MdagM.t", (size_t)rhs_stride(G, subset, prec) * nrhs, &t));
    WD_TRY(op_M(g, kappa, subset, 0, prec, nrhs, in, t));
    return op_M(g, kappa, subset, 1, prec, nrhs, t, out);
}

} // namespace wd

using namespace wd;

// ============================================================================
// extern "C" entry points
// ============================================================================
extern "C" {

int wd_abi_version(void) { return WD_ABI_VERSION; }

const char* wd_status_string(int s)
{
    switch (s) {
    case WD_OK: return "WD_OK";
    case WD_EINVAL: return "WD_EINVAL: invalid argument";
    case WD_ESHAPE: return "WD_ESHAPE: lattice or field shape not supported";
    case WD_ENOMEM: return "WD_ENOMEM: device allocation failed";
    case WD_EHIP: return "WD_EHIP: HIP runtime error";
    case WD_ENOCONV: return "WD_ENOCONV: solver did not converge";
    case WD_ENAN: return "WD_ENAN: NaN or Inf in a reduction";
    case WD_EUNSUPPORTED: return "WD_EUNSUPPORTED: unsupported combination";
    }
    return "unknown wd_status";
}

const char* wd_last_error(void) { return g_last_error.c_str(); }

wd_status wd_context_create(int device, void* stream, wd_context* out)
{
    if (!out) {
        set_error("wd_context_create: out is NULL");
        return WD_EINVAL;
    }
    int n = 0;
    WD_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("wd_context_create: device %d out of range (%d devices)", device, n);
        return WD_EINVAL;
    }
    WD_HIP(hipSetDevice(device));
    wd_context c = new wd_context_s();
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipMalloc(&c->dres, 256 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(&c->hres, 256 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        set_error("wd_context_create: allocation failed");
        if (c->dres) hipFree(c->dres);
        delete c;
        return WD_ENOMEM;
    }
    // kernels write reduction results straight into the mapped host buffer; without a device
    // address for it (or with WD_RESULTS_UNMAPPED=1) they are copied behind the kernels and the
    // host synchronises the stream instead of spinning on the buffer
    if (hipHostGetDevicePointer((void**)&c->hres_dev, c->hres, 0) != hipSuccess) c->hres_dev = nullptr;
    if (const char* e = getenv("WD_RESULTS_UNMAPPED"))
        if (atoi(e) != 0) c->hres_dev = nullptr;
    wd_status s = ensure_reduction(c, 4 * 2048);
    if (s != WD_OK) {
        hipFree(c->dres);
        hipHostFree(c->hres);
        delete c;
        return s;
    }
    hipEventCreate(&c->ev0);
    hipEventCreate(&c->ev1);
    *out = c;
    return WD_OK;
}

wd_status wd_context_set_stream(wd_context ctx, void* stream)
{
    if (!ctx) {
        set_error("context is NULL");
        return WD_EINVAL;
    }
    ctx->stream = (hipStream_t)stream;
    return WD_OK;
}

wd_status wd_context_destroy(wd_context ctx)
{
    if (!ctx) {
        set_error("context is NULL");
        return WD_EINVAL;
    }
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->ws)
        if (kv.second.first) hipFree(kv.second.first);
    if (ctx->partials) hipFree(ctx->partials);
    if (ctx->dres) hipFree(ctx->dres);
    if (ctx->hres) hipHostFree(ctx->hres);
    if (ctx->ev0) hipEventDestroy(ctx->ev0);
    if (ctx->ev1) hipEventDestroy(ctx->ev1);
    delete ctx;
    return WD_OK;
}

wd_status wd_gauge_create(wd_context ctx, const wd_lattice* lat, wd_recon recon, wd_gauge* out)
{
    if (!ctx || !out) {
        set_error("wd_gauge_create: NULL argument");
        return WD_EINVAL;
    }
    if (!valid_recon(recon)) {
        set_error("wd_gauge_create: recon must be 12 or 18, got %d", (int)recon);
        return WD_EINVAL;
    }
    Geom g;
    WD_TRY(make_geom(lat, &g));
    wd_gauge G = new wd_gauge_s();
    G->ctx = ctx;
    G->lat = *lat;
    G->recon = recon;
    G->geom = g;
    *out = G;
    return WD_OK;
}

wd_status wd_gauge_upload(wd_gauge g, const double* links, int on_device)
{
    if (!g || !links) {
        set_error("wd_gauge_upload: NULL argument");
        return WD_EINVAL;
    }
    WD_HIP(hipSetDevice(g->ctx->device));
    const size_t bytes = (size_t)8 * g->geom.Vh * 18 * sizeof(double);
    if (!g->canon) WD_HIP(hipMalloc(&g->canon, bytes));
    WD_HIP(hipMemcpyAsync(g->canon, links, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          g->ctx->stream));
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    g->uploaded = true;
    g->gf = false;
    // repack every precision already in use
    for (int p = 0; p < 4; ++p)
        if (g->packed[p]) WD_TRY(launch_pack_gauge(g->ctx, g->geom, p, g->recon, g->canon, g->packed[p]));
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    return WD_OK;
}

wd_status wd_gauge_prepare(wd_gauge g, wd_prec prec)
{
    if (!g || !valid_prec(prec)) {
        set_error("wd_gauge_prepare: bad argument");
        return WD_EINVAL;
    }
    const void* p;
    return gauge_links(g, prec, &p);
}

size_t wd_gauge_bytes(wd_gauge g, wd_prec prec)
{
    if (!g || !valid_prec(prec)) return 0;
    return 8 * link_site_bytes(prec, g->recon) * (size_t)g->geom.ps;
}

wd_status wd_gauge_destroy(wd_gauge g)
{
    if (!g) {
        set_error("gauge is NULL");
        return WD_EINVAL;
    }
    hipSetDevice(g->ctx->device);
    hipStreamSynchronize(g->ctx->stream);
    if (g->canon) hipFree(g->canon);
    for (int p = 0; p < 4; ++p)
        if (g->packed[p]) hipFree(g->packed[p]);
    delete g;
    return WD_OK;
}

size_t wd_spinor_bytes(const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs)
{
    Geom g;
    if (!valid_prec(prec) || !valid_subset(subset) || nrhs < 1) return 0;
    if (make_geom(lat, &g) != WD_OK) return 0;
    return half_bytes(g, prec) * halves_of(subset, nrhs);
}

long long wd_plane_stride(const wd_lattice* lat)
{
    Geom g;
    if (make_geom(lat, &g) != WD_OK) return 0;
    return g.ps;
}

static wd_status field_args(const wd_lattice* lat, int subset, int prec, int nrhs, Geom* g)
{
    if (!valid_subset(subset)) {
        set_error("bad subset %d", subset);
        return WD_EINVAL;
    }
    if (!valid_prec(prec)) {
        set_error("bad precision %d", prec);
        return WD_EINVAL;
    }
    if (nrhs < 1 || nrhs > 65535) {
        set_error("nrhs = %d out of range [1, 65535]", nrhs);
        return WD_EINVAL;
    }
    return make_geom(lat, g);
}

wd_status wd_spinor_pack(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                         const double* canon, void* packed)
{
    Geom g;
    if (!ctx || !canon || !packed) {
        set_error("wd_spinor_pack: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, prec, nrhs, &g));
    return launch_spinor_pack(ctx, g, subset, prec, nrhs, canon, packed, false);
}

wd_status wd_spinor_unpack(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                           const void* packed, double* canon)
{
    Geom g;
    if (!ctx || !canon || !packed) {
        set_error("wd_spinor_unpack: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, prec, nrhs, &g));
    return launch_spinor_pack(ctx, g, subset, prec, nrhs, canon, (void*)packed, true);
}

wd_status wd_spinor_convert(wd_context ctx, const wd_lattice* lat, wd_subset subset, int nrhs, wd_prec sp,
                            const void* src, wd_prec dp, void* dst)
{
    Geom g;
    if (!ctx || !src || !dst) {
        set_error("wd_spinor_convert: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, sp, nrhs, &g));
    if (!valid_prec(dp)) {
        set_error("bad precision %d", (int)dp);
        return WD_EINVAL;
    }
    return launch_convert(ctx, g, halves_of(subset, nrhs), sp, src, dp, dst);
}

static wd_status op_args(wd_gauge g, int subset, int prec, int nrhs, const void* in, const void* out)
{
    if (!g || !in || !out) {
        set_error("NULL gauge or field pointer");
        return WD_EINVAL;
    }
    if (!valid_subset(subset) || !valid_prec(prec) || nrhs < 1 || nrhs > 65535) {
        set_error("bad subset (%d), precision (%d) or nrhs (%d)", subset, prec, nrhs);
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    return WD_OK;
}

wd_status wd_dslash(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, int nrhs, const void* in, void* out)
{
    WD_TRY(op_args(g, out_subset, prec, nrhs, in, out));
    return op_dslash(g, out_subset, dagger != 0, prec, nrhs, in, out, nullptr, 0.0, 1.0);
}

wd_status wd_dslash_xpay(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, int nrhs, const void* in,
                         const void* x, double a, double b, void* out)
{
    WD_TRY(op_args(g, out_subset, prec, nrhs, in, out));
    if (!x) {
        set_error("wd_dslash_xpay: x is NULL");
        return WD_EINVAL;
    }
    return op_dslash(g, out_subset, dagger != 0, prec, nrhs, in, out, x, a, b);
}

wd_status wd_apply_M(wd_gauge g, double kappa, wd_subset subset, int dagger, wd_prec prec, int nrhs, const void* in,
                     void* out)
{
    WD_TRY(op_args(g, subset, prec, nrhs, in, out));
    if (in == out) {
        set_error("wd_apply_M: in and out must not alias");
        return WD_EINVAL;
    }
    return op_M(g, kappa, subset, dagger != 0, prec, nrhs, in, out);
}

wd_status wd_apply_MdagM(wd_gauge g, double kappa, wd_subset subset, wd_prec prec, int nrhs, const void* in, void* out)
{
    WD_TRY(op_args(g, subset, prec, nrhs, in, out));
    if (in == out) {
        set_error("wd_apply_MdagM: in and out must not alias");
        return WD_EINVAL;
    }
    return op_MdagM(g, kappa, subset, prec, nrhs, in, out);
}

wd_status wd_dot(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs, const void* a,
                 const void* b, double* result)
{
    Geom g;
    if (!ctx || !a || !b || !result) {
        set_error("wd_dot: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, prec, nrhs, &g));
    WD_TRY(blas_dot(ctx, g, halves_of(subset, nrhs), prec, a, b, true));
    result[0] = ctx->hres[0];
    result[1] = ctx->hres[1];
    return WD_OK;
}

wd_status wd_norm2(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs, const void* a,
                   double* result)
{
    Geom g;
    if (!ctx || !a || !result) {
        set_error("wd_norm2: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, prec, nrhs, &g));
    WD_TRY(blas_norm2(ctx, g, halves_of(subset, nrhs), prec, a, true));
    result[0] = ctx->hres[0];
    return WD_OK;
}

wd_status wd_caxpy(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs, double ar,
                   double ai, const void* x, void* y)
{
    Geom g;
    if (!ctx || !x || !y) {
        set_error("wd_caxpy: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(field_args(lat, subset, prec, nrhs, &g));
    return blas_caxpy(ctx, g, halves_of(subset, nrhs), prec, ar, ai, x, y);
}

} // extern "C"
