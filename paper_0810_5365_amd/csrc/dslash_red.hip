// The fused-update hopping term (out = a x + b D in) with a global sum of its
// result folded into the epilogue: the solvers' inner products of a freshly
// computed operator application (paper Section 4: global sums on the GPU in
// double precision) without a second pass over the fields.  Per workgroup the
// site values are summed (wave shuffles, then LDS); the fixed-order second
// pass of the other reductions finishes them.
#include "dslash_body.h"

namespace wd {

template <int P, int R, bool DAG, bool NT, bool PF, int RED>
__global__ void __launch_bounds__(256) dslash_red_kernel(DslashArgs A)
{
    constexpr int NV = red_values(RED);
    const uint32_t bid = A.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t i = bid * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < (uint32_t)A.g.Vh) {   // work-items past the last site contribute zeros
        if (A.zb > 0) {
            int c[4];
            const uint32_t cb = zblock_site(A, i, c);
            dslash_site<P, R, DAG, true, NT, PF, RED>(A, cb, c, 0, v);
        } else {
            dslash_site<P, R, DAG, true, NT, PF, RED>(A, i, 0, v);
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

template <int P, int R, bool DAG, int RED>
static wd_status launch_k(wd_context ctx, const DslashArgs& A, const TuneParam& tp, unsigned nblk)
{
    const dim3 grid(nblk), block(tp.block);
    switch ((tp.nt ? 1 : 0) | (tp.pf ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((dslash_red_kernel<P, R, DAG, false, false, RED>), grid, block, 0, ctx->stream, A); break;
    case 1: hipLaunchKernelGGL((dslash_red_kernel<P, R, DAG, true, false, RED>), grid, block, 0, ctx->stream, A); break;
    case 2: hipLaunchKernelGGL((dslash_red_kernel<P, R, DAG, false, true, RED>), grid, block, 0, ctx->stream, A); break;
    default: hipLaunchKernelGGL((dslash_red_kernel<P, R, DAG, true, true, RED>), grid, block, 0, ctx->stream, A); break;
    }
    WD_LAUNCHED();
    return WD_OK;
}

// The solvers' inner products (RED_NORM, RED_XDOT, RED_YDOT) are built without the dagger for
// every precision, RED_NORM also with it in float32 and float64 (the accumulation precisions);
// the CG residual update RED_CGR with the dagger for every precision; the float64 residuals
// (RED_RESID, RED_YDIFF) with and without it and RED_RESLO without it, in F64.
template <int P, int R>
static wd_status launch_pr(wd_context ctx, const DslashArgs& A, const TuneParam& tp, int red, bool dag, unsigned nblk)
{
    if (red == RED_CGR) return dag ? launch_k<P, R, true, RED_CGR>(ctx, A, tp, nblk) : WD_EUNSUPPORTED;
    if (red == RED_NORM && dag) {
        if constexpr (P == P_F64 || P == P_F32) return launch_k<P, R, true, RED_NORM>(ctx, A, tp, nblk);
        return WD_EUNSUPPORTED;
    }
    if (red <= RED_YDOT) {
        if (dag) return WD_EUNSUPPORTED;
        switch (red) {
        case RED_NORM: return launch_k<P, R, false, RED_NORM>(ctx, A, tp, nblk);
        case RED_XDOT: return launch_k<P, R, false, RED_XDOT>(ctx, A, tp, nblk);
        default: return launch_k<P, R, false, RED_YDOT>(ctx, A, tp, nblk);
        }
    }
    if constexpr (P == P_F64) {
        if (red == RED_RESID)
            return dag ? launch_k<P, R, true, RED_RESID>(ctx, A, tp, nblk) : launch_k<P, R, false, RED_RESID>(ctx, A, tp, nblk);
        if (red == RED_RESLO) return dag ? WD_EUNSUPPORTED : launch_k<P, R, false, RED_RESLO>(ctx, A, tp, nblk);
        return dag ? launch_k<P, R, true, RED_YDIFF>(ctx, A, tp, nblk) : launch_k<P, R, false, RED_YDIFF>(ctx, A, tp, nblk);
    }
    return WD_EUNSUPPORTED;
}

wd_status launch_dslash_red(wd_context ctx, const Geom& g, const DslashCall& c, int red, const void* y,
                            double* partials, int* nblocks, const double* coef)
{
    const bool needs_y = red >= RED_YDOT && red <= RED_RESLO;
    if (!c.x || c.nrhs != 1 || red < RED_NORM || red > RED_CGR || (needs_y && !y) || (red == RED_CGR && !coef) ||
        !partials || !nblocks) {
        set_error("dslash: a fused reduction needs a x + b D in, one rhs (and y for RED_YDOT, RED_RESID, RED_YDIFF, "
                  "RED_RESLO; alpha in device memory for RED_CGR)");
        return WD_EINVAL;
    }
    // the launch shape tuned for the same launch without the reduction
    TuneParam tp = tune_lookup(ctx, dslash_key(g, c));
    tp.rhs_inner = 0;
    DslashArgs A;
    WD_TRY(dslash_setup(g, c, tp, &A));
    const unsigned nblk = (unsigned)((g.Vh + tp.block - 1) / tp.block);
    if ((size_t)nblk * red_values(red) > ctx->npartials) {
        set_error("dslash: %u workgroup sums do not fit the %zu reduction slots", nblk, ctx->npartials);
        return WD_EINVAL;
    }
    A.red = partials;
    A.y = (const char*)y;
    A.coef = coef;
    *nblocks = (int)nblk;
    const bool r12 = c.recon == 12, dag = c.dagger != 0;
    wd_status st = WD_EINVAL;
    switch (c.prec) {
    case WD_F64: st = r12 ? launch_pr<P_F64, 12>(ctx, A, tp, red, dag, nblk) : launch_pr<P_F64, 18>(ctx, A, tp, red, dag, nblk); break;
    case WD_F32: st = r12 ? launch_pr<P_F32, 12>(ctx, A, tp, red, dag, nblk) : launch_pr<P_F32, 18>(ctx, A, tp, red, dag, nblk); break;
    case WD_F16: st = r12 ? launch_pr<P_F16, 12>(ctx, A, tp, red, dag, nblk) : launch_pr<P_F16, 18>(ctx, A, tp, red, dag, nblk); break;
    case WD_BF16: st = r12 ? launch_pr<P_BF16, 12>(ctx, A, tp, red, dag, nblk) : launch_pr<P_BF16, 18>(ctx, A, tp, red, dag, nblk); break;
    default: set_error("dslash: bad precision %d", c.prec); return WD_EINVAL;
    }
    if (st == WD_EUNSUPPORTED)
        set_error("dslash: fused reduction %d is not built for precision %d %s the dagger", red, c.prec,
                  dag ? "with" : "without");
    if (st == WD_OK) ctx->hops += 1;
    return st;
}

} // namespace wd
