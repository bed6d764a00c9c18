// Launches of the even-odd hopping term: one work-item per output site on a
// 1-D grid of workgroups (optionally remapped so that each XCD walks one
// contiguous range), right-hand sides either on the grid's y axis or
// interleaved with the site tiles so that the workgroups sharing a tile's
// links run back to back on one XCD.
#include "dslash_body.h"

namespace wd {

template <int P, int R, bool DAG, bool XPAY, bool NT, bool PF>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs A)
{
    uint32_t bid = A.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    int rhs = blockIdx.y;
    if (A.rhs_inner > 1) {
        rhs = (int)(bid % (uint32_t)A.rhs_inner);
        bid /= (uint32_t)A.rhs_inner;
    }
    const uint32_t i = bid * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)A.g.Vh) return;
    if (A.zb > 0) {
        int c[4];
        const uint32_t cb = zblock_site(A, i, c);
        dslash_site<P, R, DAG, XPAY, NT, PF>(A, cb, c, rhs);
    } else {
        dslash_site<P, R, DAG, XPAY, NT, PF>(A, i, rhs);
    }
}

template <int P, int R, bool DAG, bool XPAY, bool NT, bool PF>
static wd_status run(wd_context ctx, const DslashArgs& A, int nrhs, const TuneParam& tp)
{
    dim3 block(tp.block);
    const unsigned nblk = (A.g.Vh + tp.block - 1) / tp.block;
    dim3 grid = A.rhs_inner > 1 ? dim3(nblk * (unsigned)nrhs, 1) : dim3(nblk, nrhs);
    hipLaunchKernelGGL((dslash_kernel<P, R, DAG, XPAY, NT, PF>), grid, block, 0, ctx->stream, A);
    WD_LAUNCHED();
    return WD_OK;
}

template <int P, int R>
static wd_status dispatch_pr(wd_context ctx, const DslashArgs& A, const DslashCall& c, const TuneParam& tp)
{
    const int sel = (c.dagger ? 1 : 0) | (c.x ? 2 : 0) | (tp.nt ? 4 : 0) | (tp.pf ? 8 : 0);
    switch (sel) {
#define WD_DS(K) case K: return run<P, R, (K & 1) != 0, (K & 2) != 0, (K & 4) != 0, (K & 8) != 0>(ctx, A, c.nrhs, tp);
    WD_DS(0) WD_DS(1) WD_DS(2) WD_DS(3) WD_DS(4) WD_DS(5) WD_DS(6) WD_DS(7)
    WD_DS(8) WD_DS(9) WD_DS(10) WD_DS(11) WD_DS(12) WD_DS(13) WD_DS(14) WD_DS(15)
#undef WD_DS
    }
    return WD_EINVAL;
}

wd_status dslash_setup(const Geom& g, const DslashCall& c, const TuneParam& tp, DslashArgs* out)
{
    if (tp.block <= 0 || tp.block > 256 || tp.block % 64) {
        set_error("dslash: workgroup size %d not in {64, 128, 192, 256}", tp.block);
        return WD_EINVAL;
    }
    DslashArgs A{};
    A.gauge = (const char*)c.gauge;
    A.in = (const char*)c.in;
    A.out = (char*)c.out;
    A.x = (const char*)c.x;
    A.in_stride = c.in_stride;
    A.out_stride = c.out_stride;
    A.x_stride = c.x_stride;
    A.a = c.a;
    A.b = c.b;
    A.g = g;
    A.par = c.par;
    A.remap = tp.remap;
    {   // the fused update's x is loaded non-temporally; WD_DSLASH_XNT=0 turns that off
        static const int xnt = getenv("WD_DSLASH_XNT") ? (atoi(getenv("WD_DSLASH_XNT")) != 0) : 1;
        A.xnt = xnt;
    }
    A.rhs_inner = (tp.rhs_inner && c.nrhs > 1) ? c.nrhs : 0;
    A.gf = c.gf;
    A.zb = 0;
    if (tp.zb > 0 && tp.zb < g.L[2] && g.L[2] % tp.zb == 0) {
        A.zb = tp.zb;
        A.dzb = make_fastdiv((uint32_t)tp.zb);
        A.dt = make_fastdiv((uint32_t)g.L[3]);
    }
    if ((long long)((g.Vh + tp.block - 1) / tp.block) * c.nrhs >= (1ll << 31)) A.rhs_inner = 0;
    *out = A;
    return WD_OK;
}

wd_status launch_dslash_tuned(wd_context ctx, const Geom& g, const DslashCall& c, const TuneParam& tp)
{
    if (tp.mf && mrhs_eligible(c)) return launch_dslash_mrhs(ctx, g, c);
    DslashArgs A;
    WD_TRY(dslash_setup(g, c, tp, &A));
    const bool r12 = c.recon == 12;
    switch (c.prec) {
    case WD_F64: return r12 ? dispatch_pr<P_F64, 12>(ctx, A, c, tp) : dispatch_pr<P_F64, 18>(ctx, A, c, tp);
    case WD_F32: return r12 ? dispatch_pr<P_F32, 12>(ctx, A, c, tp) : dispatch_pr<P_F32, 18>(ctx, A, c, tp);
    case WD_F16: return r12 ? dispatch_pr<P_F16, 12>(ctx, A, c, tp) : dispatch_pr<P_F16, 18>(ctx, A, c, tp);
    case WD_BF16: return r12 ? dispatch_pr<P_BF16, 12>(ctx, A, c, tp) : dispatch_pr<P_BF16, 18>(ctx, A, c, tp);
    default: set_error("dslash: bad precision %d", c.prec); return WD_EINVAL;
    }
}

std::string dslash_key(const Geom& g, const DslashCall& c)
{
    char key[160];
    snprintf(key, sizeof key, "dslash:%dx%dx%dx%d:p%d:r%d:n%d:d%d:x%d", g.L[0], g.L[1], g.L[2], g.L[3], c.prec,
             c.recon, c.nrhs, c.dagger, c.x != nullptr);
    return key;
}

wd_status launch_dslash(wd_context ctx, const Geom& g, const DslashCall& c)
{
    WD_TRY(launch_dslash_tuned(ctx, g, c, tune_lookup(ctx, dslash_key(g, c))));
    ctx->hops += c.nrhs;
    return WD_OK;
}

} // namespace wd
