// Conversion between the canonical float64 layouts and the packed
// structure-of-arrays device layouts (paper Section 5: fields split by parity,
// 16-byte vectors so that consecutive work-items read consecutive memory).
#include "wd_core.h"

namespace wd {

// ---- gauge ---------------------------------------------------------------
// One work-item per link (mu, lexicographic site).  Writes the packed group
// (mu, parity of the site) at the site's checkerboard index.
template <int P, int R>
__global__ void pack_gauge_kernel(const double* __restrict__ canon, char* __restrict__ out, Geom g, long long nlinks)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nlinks) return;
    const long long V = 2ll * g.Vh;
    const int mu = (int)(k / V);
    const long long lex = k - mu * V;
    long long r = lex;
    const int x = (int)(r % g.L[0]); r /= g.L[0];
    const int y = (int)(r % g.L[1]); r /= g.L[1];
    const int z = (int)(r % g.L[2]); r /= g.L[2];
    const int t = (int)r;
    const int par = (x + y + z + t) & 1;
    const uint32_t cb = (uint32_t)(lex >> 1);
    const double* u = canon + 18 * k;
    const int Vh = g.ps;   // plane stride
    char* grp = out + (size_t)(2 * mu + par) * link_site_bytes(P, R) * Vh;
    if constexpr (P == P_F32) {
        float4* p = (float4*)grp;
        float f[18];
        for (int i = 0; i < R; ++i) f[i] = (float)u[i];
        for (int q = 0; q < R / 4; ++q) p[(size_t)q * Vh + cb] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
        if (R == 18) ((float2*)(p + (size_t)4 * Vh))[cb] = make_float2(f[16], f[17]);
    } else if constexpr (P == P_F64) {
        double2* p = (double2*)grp;
        for (int q = 0; q < R / 2; ++q) p[(size_t)q * Vh + cb] = make_double2(u[2 * q], u[2 * q + 1]);
    } else {
        uint32_t h[9];
        for (int q = 0; q < R / 2; ++q) h[q] = pack2<P>((float)u[2 * q], (float)u[2 * q + 1]);
        uint4* p = (uint4*)grp;
        if (R == 12) {
            p[cb] = make_uint4(h[0], h[1], h[2], h[3]);
            ((uint2*)(p + (size_t)Vh))[cb] = make_uint2(h[4], h[5]);
        } else {
            p[cb] = make_uint4(h[0], h[1], h[2], h[3]);
            p[(size_t)Vh + cb] = make_uint4(h[4], h[5], h[6], h[7]);
            ((uint32_t*)(p + (size_t)2 * Vh))[cb] = h[8];
        }
    }
}

template <int P, int R>
static wd_status pack_gauge_t(wd_context ctx, const Geom& g, const double* canon, void* out)
{
    const long long n = 4ll * 2 * g.Vh;
    const int bs = 256;
    hipLaunchKernelGGL((pack_gauge_kernel<P, R>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, ctx->stream, canon,
                       (char*)out, g, n);
    WD_LAUNCHED();
    return WD_OK;
}

wd_status launch_pack_gauge(wd_context ctx, const Geom& g, int prec, int recon, const double* canon, void* out)
{
    const bool r12 = recon == 12;
    switch (prec) {
    case WD_F64: return r12 ? pack_gauge_t<P_F64, 12>(ctx, g, canon, out) : pack_gauge_t<P_F64, 18>(ctx, g, canon, out);
    case WD_F32: return r12 ? pack_gauge_t<P_F32, 12>(ctx, g, canon, out) : pack_gauge_t<P_F32, 18>(ctx, g, canon, out);
    case WD_F16: return r12 ? pack_gauge_t<P_F16, 12>(ctx, g, canon, out) : pack_gauge_t<P_F16, 18>(ctx, g, canon, out);
    case WD_BF16: return r12 ? pack_gauge_t<P_BF16, 12>(ctx, g, canon, out) : pack_gauge_t<P_BF16, 18>(ctx, g, canon, out);
    }
    set_error("pack_gauge: bad precision %d", prec);
    return WD_EINVAL;
}

// ---- spinors ---------------------------------------------------------------
// One work-item per (rhs, site).  FULL: canonical lexicographic site order;
// EVEN / ODD: canonical checkerboard order of that parity.
template <int P, bool UNPACK>
__global__ void spinor_pack_kernel(double* __restrict__ canon, char* __restrict__ packed, Geom g, int subset,
                                   long long nsites_per_rhs, long long ntotal)
{
    using T = typename RealOf<P>::T;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ntotal) return;
    const long long rhs = k / nsites_per_rhs;
    const long long s = k - rhs * nsites_per_rhs;
    const size_t hb = spinor_site_bytes(P) * (size_t)g.ps;
    int par;
    uint32_t cb;
    char* base;
    if (subset == WD_FULL) {
        long long r = s;
        const int x = (int)(r % g.L[0]); r /= g.L[0];
        const int y = (int)(r % g.L[1]); r /= g.L[1];
        const int z = (int)(r % g.L[2]); r /= g.L[2];
        const int t = (int)r;
        par = (x + y + z + t) & 1;
        cb = (uint32_t)(s >> 1);
        base = packed + (size_t)rhs * 2 * hb + (size_t)par * hb;
    } else {
        cb = (uint32_t)s;
        base = packed + (size_t)rhs * hb;
    }
    double* c = canon + 24 * k;
    T v[24];
    if constexpr (UNPACK) {
        SpinorIO<P>::load(base, g.ps, cb, v);
        for (int i = 0; i < 24; ++i) c[i] = (double)v[i];
    } else {
        for (int i = 0; i < 24; ++i) v[i] = (T)c[i];
        SpinorIO<P>::store(base, g.ps, cb, v);
    }
}

template <int P>
static wd_status spinor_pack_t(wd_context ctx, const Geom& g, int subset, int nrhs, const double* canon, void* packed,
                               bool unpack)
{
    const long long per = subset == WD_FULL ? 2ll * g.Vh : (long long)g.Vh;
    const long long n = per * nrhs;
    const int bs = 256;
    const dim3 grid((unsigned)((n + bs - 1) / bs));
    if (unpack)
        hipLaunchKernelGGL((spinor_pack_kernel<P, true>), grid, dim3(bs), 0, ctx->stream, (double*)canon,
                           (char*)packed, g, subset, per, n);
    else
        hipLaunchKernelGGL((spinor_pack_kernel<P, false>), grid, dim3(bs), 0, ctx->stream, (double*)canon,
                           (char*)packed, g, subset, per, n);
    WD_LAUNCHED();
    return WD_OK;
}

wd_status launch_spinor_pack(wd_context ctx, const Geom& g, int subset, int prec, int nrhs, const double* canon,
                             void* packed, bool unpack)
{
    switch (prec) {
    case WD_F64: return spinor_pack_t<P_F64>(ctx, g, subset, nrhs, canon, packed, unpack);
    case WD_F32: return spinor_pack_t<P_F32>(ctx, g, subset, nrhs, canon, packed, unpack);
    case WD_F16: return spinor_pack_t<P_F16>(ctx, g, subset, nrhs, canon, packed, unpack);
    case WD_BF16: return spinor_pack_t<P_BF16>(ctx, g, subset, nrhs, canon, packed, unpack);
    }
    set_error("spinor_pack: bad precision %d", prec);
    return WD_EINVAL;
}

// ---- precision conversion between packed fields --------------------------------
template <int SP, int DP>
__global__ void convert_kernel(const char* __restrict__ src, char* __restrict__ dst, int Vh, int ps, long long nsites)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsites) return;
    const long long h = k / Vh;
    const uint32_t cb = (uint32_t)(k - h * Vh);
    typename RealOf<SP>::T v[24];
    typename RealOf<DP>::T w[24];
    SpinorIO<SP>::load(src + (size_t)h * spinor_site_bytes(SP) * ps, ps, cb, v);
    for (int i = 0; i < 24; ++i) w[i] = (typename RealOf<DP>::T)v[i];
    SpinorIO<DP>::store(dst + (size_t)h * spinor_site_bytes(DP) * ps, ps, cb, w);
}

template <int SP, int DP>
static wd_status convert_t(wd_context ctx, const Geom& g, size_t nhalves, const void* src, void* dst)
{
    const long long n = (long long)nhalves * g.Vh;
    const int bs = 256;
    hipLaunchKernelGGL((convert_kernel<SP, DP>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, ctx->stream,
                       (const char*)src, (char*)dst, g.Vh, g.ps, n);
    WD_LAUNCHED();
    return WD_OK;
}

template <int SP>
static wd_status convert_s(wd_context ctx, const Geom& g, size_t nh, const void* src, int dp, void* dst)
{
    switch (dp) {
    case WD_F64: return convert_t<SP, P_F64>(ctx, g, nh, src, dst);
    case WD_F32: return convert_t<SP, P_F32>(ctx, g, nh, src, dst);
    case WD_F16: return convert_t<SP, P_F16>(ctx, g, nh, src, dst);
    case WD_BF16: return convert_t<SP, P_BF16>(ctx, g, nh, src, dst);
    }
    set_error("convert: bad precision %d", dp);
    return WD_EINVAL;
}

wd_status launch_convert(wd_context ctx, const Geom& g, size_t nhalves, int sp, const void* src, int dp, void* dst)
{
    switch (sp) {
    case WD_F64: return convert_s<P_F64>(ctx, g, nhalves, src, dp, dst);
    case WD_F32: return convert_s<P_F32>(ctx, g, nhalves, src, dp, dst);
    case WD_F16: return convert_s<P_F16>(ctx, g, nhalves, src, dp, dst);
    case WD_BF16: return convert_s<P_BF16>(ctx, g, nhalves, src, dp, dst);
    }
    set_error("convert: bad precision %d", sp);
    return WD_EINVAL;
}

} // namespace wd
