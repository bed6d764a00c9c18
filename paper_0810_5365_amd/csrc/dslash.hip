// Wilson hopping term restricted to one parity ("Dslash", paper Section 4),
// one work-item per output site (paper Section 4: one thread per site of the
// even or odd sub-lattice).
//
// Per output site x of parity par and each of the 8 directions:
//   1. fetch the neighbour spinor psi(x +- mu) (24 reals, structure-of-arrays),
//   2. project it to a half spinor with (1 -+ gamma_mu)  (12 reals, 12 flops),
//   3. fetch the link U_mu(x) or U_mu(x - mu) (12 reals + row-2 rebuild, or 18),
//   4. multiply both colour triplets by U or U^dagger  (132 flops),
//   5. expand to 4 spin rows and accumulate  (24 flops; 7 of 8 counted),
// then store, optionally fused with out = a x + b D in.  1320 flops per site.
#include "wd_core.h"

namespace wd {

// Keeps each direction's loads behind the previous direction's arithmetic.
// Without it the compiler hoists all 72 loads of the 8 directions to the top
// of the kernel, needs > 256 VGPRs and runs one wave per SIMD; with it the
// kernel fits in < 100 VGPRs and latency is hidden by occupancy instead.
template <typename T> __device__ __forceinline__ void order_fence(T* a)
{
#pragma unroll
    for (int k = 0; k < 24; k += 8)
        asm volatile("" : "+v"(a[k]), "+v"(a[k + 1]), "+v"(a[k + 2]), "+v"(a[k + 3]), "+v"(a[k + 4]), "+v"(a[k + 5]),
                     "+v"(a[k + 6]), "+v"(a[k + 7])::"memory");
}

struct DslashArgs {
    const char* gauge;
    const char* in;
    char* out;
    const char* x;
    long long in_stride, out_stride, x_stride;
    double a, b;
    Geom g;
    int par;
    int remap;
};

template <int D, int P, int R, bool DAG, bool NT, typename T>
__device__ __forceinline__ void hop(const DslashArgs& A, uint32_t cb, const int c[4], const char* in, size_t gbytes,
                                    T* acc)
{
    constexpr int MU = D >> 1;
    constexpr bool FWD = (D & 1) == 0;
    // D: (1 - gamma) on the forward hop, (1 + gamma) on the backward hop; D^dagger swaps them
    constexpr int S = (FWD != DAG) ? -1 : 1;
    const uint32_t nb = neighbour<MU, FWD>(A.g, cb, c);
    const int lpar = FWD ? A.par : 1 - A.par;
    const uint32_t lcb = FWD ? cb : nb;
    T u[18];
    LinkIO<P, R, NT>::load(A.gauge + (size_t)(2 * MU + lpar) * gbytes, A.g.Vh, lcb, u);
    T psi[24];
    SpinorIO<P>::load(in, A.g.Vh, nb, psi);
    T h[12];
    project<MU, S>(psi, h);
    T sg;
    if constexpr (sizeof(T) == 8) sg = on_boundary<MU, FWD>(A.g, c) ? A.g.bcd[MU] : 1.0;
    else sg = on_boundary<MU, FWD>(A.g, c) ? A.g.bcf[MU] : 1.0f;
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] *= sg;
    T w[12];
    su3_mul<!FWD>(u, h, w);
    accumulate<MU, S>(acc, w);
    order_fence(acc);
}

template <int P, int R, bool DAG, bool XPAY, bool NT>
__device__ __forceinline__ void dslash_site(const DslashArgs& A, uint32_t cb, int rhs)
{
    using T = typename RealOf<P>::T;
    int c[4];
    cb_coords(A.g, cb, A.par, c);
    const size_t gbytes = link_site_bytes(P, R) * (size_t)A.g.Vh;
    const char* in = A.in + rhs * A.in_stride;
    T acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    hop<0, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<1, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<2, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<3, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<4, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<5, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<6, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    hop<7, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    const T b = (T)A.b;
    if constexpr (XPAY) {
        T xv[24];
        SpinorIO<P>::load(A.x + rhs * A.x_stride, A.g.Vh, cb, xv);
        const T a = (T)A.a;
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = a * xv[k] + b * acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] *= b;
    }
    SpinorIO<P>::store(A.out + rhs * A.out_stride, A.g.Vh, cb, acc);
}

template <int P, int R, bool DAG, bool XPAY, bool NT>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs A)
{
    const uint32_t bid = A.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t cb = bid * blockDim.x + threadIdx.x;
    if (cb >= (uint32_t)A.g.Vh) return;
    dslash_site<P, R, DAG, XPAY, NT>(A, cb, blockIdx.y);
}

template <int P, int R, bool DAG, bool XPAY, bool NT>
static wd_status run(wd_context ctx, const DslashArgs& A, int nrhs, const TuneParam& tp)
{
    dim3 block(tp.block);
    dim3 grid((A.g.Vh + tp.block - 1) / tp.block, nrhs);
    hipLaunchKernelGGL((dslash_kernel<P, R, DAG, XPAY, NT>), grid, block, 0, ctx->stream, A);
    WD_LAUNCHED();
    return WD_OK;
}

template <int P, int R>
static wd_status dispatch_pr(wd_context ctx, const DslashArgs& A, const DslashCall& c, const TuneParam& tp)
{
    const bool xp = c.x != nullptr;
    const bool nt = tp.nt != 0;
#define WD_DS(DAG, XP, NT) return run<P, R, DAG, XP, NT>(ctx, A, c.nrhs, tp)
    if (!nt) {
        if (c.dagger) { if (xp) WD_DS(true, true, false); else WD_DS(true, false, false); }
        else { if (xp) WD_DS(false, true, false); else WD_DS(false, false, false); }
    } else {
        if (c.dagger) { if (xp) WD_DS(true, true, true); else WD_DS(true, false, true); }
        else { if (xp) WD_DS(false, true, true); else WD_DS(false, false, true); }
    }
#undef WD_DS
}

wd_status launch_dslash_tuned(wd_context ctx, const Geom& g, const DslashCall& c, const TuneParam& tp)
{
    if (tp.block <= 0 || tp.block > 256 || tp.block % 64) {
        set_error("dslash: workgroup size %d not in {64, 128, 192, 256}", tp.block);
        return WD_EINVAL;
    }
    DslashArgs A;
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
    const bool r12 = c.recon == 12;
    switch (c.prec) {
    case WD_F64: return r12 ? dispatch_pr<P_F64, 12>(ctx, A, c, tp) : dispatch_pr<P_F64, 18>(ctx, A, c, tp);
    case WD_F32: return r12 ? dispatch_pr<P_F32, 12>(ctx, A, c, tp) : dispatch_pr<P_F32, 18>(ctx, A, c, tp);
    case WD_F16: return r12 ? dispatch_pr<P_F16, 12>(ctx, A, c, tp) : dispatch_pr<P_F16, 18>(ctx, A, c, tp);
    case WD_BF16: return r12 ? dispatch_pr<P_BF16, 12>(ctx, A, c, tp) : dispatch_pr<P_BF16, 18>(ctx, A, c, tp);
    default: set_error("dslash: bad precision %d", c.prec); return WD_EINVAL;
    }
}

wd_status launch_dslash(wd_context ctx, const Geom& g, const DslashCall& c)
{
    char key[160];
    snprintf(key, sizeof key, "dslash:%dx%dx%dx%d:p%d:r%d:n%d:d%d:x%d", g.L[0], g.L[1], g.L[2], g.L[3], c.prec,
             c.recon, c.nrhs, c.dagger, c.x != nullptr);
    return launch_dslash_tuned(ctx, g, c, tune_lookup(ctx, key));
}

} // namespace wd
