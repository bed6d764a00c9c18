// The fused-update hopping term (out = a x + b D in) with a global sum of its
// result folded into the epilogue: the solvers' inner products of a freshly
// computed operator application (paper Section 4: global sums on the GPU in
// double precision) without a second pass over the fields.  Per workgroup the
// site values are summed (wave shuffles, then LDS); the fixed-order second
// pass of the other reductions finishes them.
#include "dslash_body.h"

namespace wd {

template <int P, int R, bool NT, bool PF, int RED>
__global__ void __launch_bounds__(256) dslash_red_kernel(DslashArgs A)
{
    constexpr int NV = RED == RED_NORM ? 1 : 3;
    const uint32_t bid = A.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t i = bid * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < (uint32_t)A.g.Vh) {   // work-items past the last site contribute zeros
        if (A.zb > 0) {
            int c[4];
            const uint32_t cb = zblock_site(A, i, c);
            dslash_site<P, R, false, true, NT, PF, RED>(A, cb, c, 0, v);
        } else {
            dslash_site<P, R, false, true, NT, PF, RED>(A, i, 0, v);
        }
    }
    __shared__ double lds[NV][4];
#pragma unroll
    for (int n = 0; n < NV; ++n) {
        double s = v[n];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == 0) lds[n][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NV; ++n) {
            double t = 0.0;
            for (uint32_t w = 0; w < blockDim.x / 64; ++w) t += lds[n][w];
            A.red[(size_t)n * gridDim.x + blockIdx.x] = t;
        }
    }
}

template <int P, int R>
static wd_status launch_pr(wd_context ctx, const DslashArgs& A, const TuneParam& tp, int red, unsigned nblk)
{
    const dim3 grid(nblk), block(tp.block);
    const int sel = (tp.nt ? 1 : 0) | (tp.pf ? 2 : 0) | ((red - 1) << 2);
    switch (sel) {
#define WD_RK(K) case K: hipLaunchKernelGGL((dslash_red_kernel<P, R, (K & 1) != 0, (K & 2) != 0, (K >> 2) + 1>), \
                                            grid, block, 0, ctx->stream, A); break;
    WD_RK(0) WD_RK(1) WD_RK(2) WD_RK(3) WD_RK(4) WD_RK(5) WD_RK(6) WD_RK(7) WD_RK(8) WD_RK(9) WD_RK(10) WD_RK(11)
#undef WD_RK
    default: set_error("dslash: bad fused reduction %d", red); return WD_EINVAL;
    }
    WD_LAUNCHED();
    return WD_OK;
}

wd_status launch_dslash_red(wd_context ctx, const Geom& g, const DslashCall& c, int red, const void* y,
                            double* partials, int* nblocks)
{
    if (!c.x || c.dagger || c.nrhs != 1 || red < RED_NORM || red > RED_YDOT || (red == RED_YDOT && !y) || !partials ||
        !nblocks) {
        set_error("dslash: a fused reduction needs a x + b D in, no dagger, one rhs (and y for <y, out>)");
        return WD_EINVAL;
    }
    // the launch shape tuned for the same launch without the reduction
    TuneParam tp = tune_lookup(ctx, dslash_key(g, c));
    tp.rhs_inner = 0;
    DslashArgs A;
    WD_TRY(dslash_setup(g, c, tp, &A));
    const unsigned nblk = (unsigned)((g.Vh + tp.block - 1) / tp.block);
    if ((size_t)nblk * (red == RED_NORM ? 1 : 3) > ctx->npartials) {
        set_error("dslash: %u workgroup sums do not fit the %zu reduction slots", nblk, ctx->npartials);
        return WD_EINVAL;
    }
    A.red = partials;
    A.y = (const char*)y;
    *nblocks = (int)nblk;
    const bool r12 = c.recon == 12;
    switch (c.prec) {
    case WD_F64: return r12 ? launch_pr<P_F64, 12>(ctx, A, tp, red, nblk) : launch_pr<P_F64, 18>(ctx, A, tp, red, nblk);
    case WD_F32: return r12 ? launch_pr<P_F32, 12>(ctx, A, tp, red, nblk) : launch_pr<P_F32, 18>(ctx, A, tp, red, nblk);
    case WD_F16: return r12 ? launch_pr<P_F16, 12>(ctx, A, tp, red, nblk) : launch_pr<P_F16, 18>(ctx, A, tp, red, nblk);
    case WD_BF16: return r12 ? launch_pr<P_BF16, 12>(ctx, A, tp, red, nblk) : launch_pr<P_BF16, 18>(ctx, A, tp, red, nblk);
    default: set_error("dslash: bad precision %d", c.prec); return WD_EINVAL;
    }
}

} // namespace wd
