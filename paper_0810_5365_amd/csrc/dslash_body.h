// The per-site body of the Wilson hopping term on one parity (paper
// Section 4: one work-item per site of the even or odd sub-lattice), shared
// by the plain launch (dslash.hip) and the persistent batch (batch.hip).
//
// Per output site x of parity par and each of the 8 directions:
//   1. fetch the neighbour spinor psi(x +- mu) (24 reals, structure-of-arrays),
//   2. project it to a half spinor with (1 -+ gamma_mu)  (12 reals, 12 flops),
//   3. fetch the link U_mu(x) or U_mu(x - mu) (12 reals + row-2 rebuild, or 18),
//   4. multiply both colour triplets by U or U^dagger  (132 flops),
//   5. expand to 4 spin rows and accumulate  (24 flops; 7 of 8 counted),
// then store, optionally fused with out = a x + b D in.  1320 flops per site.
#pragma once

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
    int rhs_inner;   // > 1: that many rhs interleaved with the site tiles on grid x
    int zb;          // > 0: z-blocked site traversal with this block depth (divides Z)
    int gf;          // links in temporal gauge: U_t = 1 except on the last time slice
    FastDiv dzb, dt; // division by zb and by T for the blocked traversal
    double* red;     // per-workgroup partial sums of a fused reduction (dslash_red.hip)
    const char* y;   // the other operand of the fused <y, out>
    const double* coef;   // RED_CGR: the step length alpha, in device memory
    int xnt;              // fused update: load x non-temporally
};

// Kernel arguments for a launch of the hopping term with launch shape tp (dslash.hip).
wd_status dslash_setup(const Geom& g, const DslashCall& c, const TuneParam& tp, DslashArgs* A);

// v <- the values that storing v at 16-bit precision and loading it back gives (the store's
// scale and rounding, repeated).
template <int P> __device__ __forceinline__ void quant_roundtrip(float* v)
{
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 24; ++k) s = fmaxf(s, fabsf(v[k]));
    const float inv = s > 0.0f ? 1.0f / s : 0.0f;
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = h2f<P>(f2h<P>(v[k] * inv)) * s;
}

// Reductions a fused-update launch (out = a x + b D in) can sum in its epilogue, per site in
// float64 from the stored values:
//   RED_NORM  |out|^2                        -> r[0]
//   RED_XDOT  <out, x>, |out|^2              -> r[0] + i r[1], r[2]
//   RED_YDOT  <y, out> (y = A.y), |out|^2    -> r[0] + i r[1], r[2]
//   RED_RESID out = y - (a x + b D in), |out|^2 -> r[0]   (a residual, stored instead)
//   RED_YDIFF |y - out|^2                    -> r[0]
//   RED_RESLO as RED_RESID, the residual stored in float32 -> r[0]
//   RED_CGR   r -= alpha out (r = A.out at the accumulation precision), |r|^2 -> r[0]
template <typename T>
__device__ __forceinline__ void site_dot_norm(const T* a, const T* b, const T* o, double* r)
{
    double re = 0.0, im = 0.0, nn = 0.0;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) nn += (double)o[k] * (double)o[k];
    r[0] = re;
    r[1] = im;
    r[2] = nn;
}

// Site order index i -> checkerboard index and coordinates of the z-blocked
// traversal: i = xh + Xh (y + Y (zi + zb (t + T b))), z = b zb + zi.  Sites of
// one z-block are walked through all t before the next block, so the slices
// t - 1, t, t + 1 of a block that the stencil reads stay close in time.
__device__ __forceinline__ uint32_t zblock_site(const DslashArgs& A, uint32_t i, int c[4])
{
    const Geom& g = A.g;
    const uint32_t q1 = fdiv(i, g.dxh);
    const uint32_t xh = i - q1 * (uint32_t)g.Xh;
    const uint32_t q2 = fdiv(q1, g.dy);
    const uint32_t y = q1 - q2 * (uint32_t)g.L[1];
    const uint32_t q3 = fdiv(q2, A.dzb);
    const uint32_t zi = q2 - q3 * (uint32_t)A.zb;
    const uint32_t b = fdiv(q3, A.dt);
    const uint32_t t = q3 - b * (uint32_t)g.L[3];
    const uint32_t z = b * (uint32_t)A.zb + zi;
    c[1] = (int)y;
    c[2] = (int)z;
    c[3] = (int)t;
    c[0] = (int)(2 * xh + ((A.par + y + z + t) & 1));
    return xh + (uint32_t)g.Xh * (y + (uint32_t)g.L[1] * (z + (uint32_t)g.L[2] * t));
}

// In temporal gauge the t-link of a hop is the identity unless the hop leaves
// the last time slice (forward from t = T - 1, backward into t = 0), so it is
// neither loaded nor multiplied (paper Sections 4 and 7: the gauge-fixing trick).
template <int MU, bool FWD>
__device__ __forceinline__ bool unit_link(const DslashArgs& A, const int c[4])
{
    if constexpr (MU != 3) return false;
    else return A.gf && (FWD ? c[3] != A.g.L[3] - 1 : c[3] != 0);
}

// Loads of direction D: the link (U_mu(x) forward, U_mu(x - mu) backward)
// and the neighbour spinor.
template <int D, int P, int R, bool NT, typename T>
__device__ __forceinline__ void hop_load(const DslashArgs& A, uint32_t cb, const int c[4], const char* in, size_t gbytes,
                                         T* u, T* psi)
{
    constexpr int MU = D >> 1;
    constexpr bool FWD = (D & 1) == 0;
    const uint32_t nb = neighbour<MU, FWD>(A.g, cb, c);
    const int lpar = FWD ? A.par : 1 - A.par;
    const uint32_t lcb = FWD ? cb : nb;
    if (!unit_link<MU, FWD>(A, c)) LinkIO<P, R, NT>::load(A.gauge + (size_t)(2 * MU + lpar) * gbytes, A.g.ps, lcb, u);
    SpinorIO<P>::load(in, A.g.ps, nb, psi);
}

// Arithmetic of direction D: project, boundary sign, colour multiply, accumulate.
template <int D, bool DAG, typename T>
__device__ __forceinline__ void hop_compute(const DslashArgs& A, const int c[4], const T* u, const T* psi, T* acc)
{
    constexpr int MU = D >> 1;
    constexpr bool FWD = (D & 1) == 0;
    // D: (1 - gamma) on the forward hop, (1 + gamma) on the backward hop; D^dagger swaps them
    constexpr int S = (FWD != DAG) ? -1 : 1;
    T h[12];
    project<MU, S>(psi, h);
    T sg;
    if constexpr (sizeof(T) == 8) sg = on_boundary<MU, FWD>(A.g, c) ? A.g.bcd[MU] : 1.0;
    else sg = on_boundary<MU, FWD>(A.g, c) ? A.g.bcf[MU] : 1.0f;
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] *= sg;
    T w[12];
    if (unit_link<MU, FWD>(A, c)) {
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = h[k];
    } else {
        su3_mul<!FWD>(u, h, w);
    }
    accumulate<MU, S>(acc, w);
}

// One direction at a time: its loads, then its arithmetic, then a fence.
template <int D, int P, int R, bool DAG, bool NT, typename T>
__device__ __forceinline__ void hop(const DslashArgs& A, uint32_t cb, const int c[4], const char* in, size_t gbytes,
                                    T* acc)
{
    T u[18], psi[24];
    hop_load<D, P, R, NT>(A, cb, c, in, gbytes, u, psi);
    hop_compute<D, DAG>(A, c, u, psi, acc);
    order_fence(acc);
}

// Software-pipelined: the loads of direction D + 1 are issued before the
// arithmetic of direction D, so each wave keeps two directions in flight.
template <int D, int P, int R, bool DAG, bool NT, typename T>
__device__ __forceinline__ void hop_pipelined(const DslashArgs& A, uint32_t cb, const int c[4], const char* in,
                                              size_t gbytes, T* acc, T* u_cur, T* p_cur, T* u_nxt, T* p_nxt)
{
    if constexpr (D + 1 < 8) hop_load<D + 1, P, R, NT>(A, cb, c, in, gbytes, u_nxt, p_nxt);
    asm volatile("" ::: "memory");
    hop_compute<D, DAG>(A, c, u_cur, p_cur, acc);
    order_fence(acc);
}

// RED > 0 (with XPAY): the site's values of that fused reduction go to red[0 .. 3).  The
// output is stored first, so the reduction adds no registers to the store.
template <int P, int R, bool DAG, bool XPAY, bool NT, bool PF, int RED = 0>
__device__ __forceinline__ void dslash_site(const DslashArgs& A, uint32_t cb, const int c[4], int rhs,
                                            double* red = nullptr)
{
    using T = typename RealOf<P>::T;
    const size_t gbytes = link_site_bytes(P, R) * (size_t)A.g.ps;
    const char* in = A.in + rhs * A.in_stride;
    T acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    if constexpr (PF) {
        T ua[18], pa[24], ub[18], pb[24];
        hop_load<0, P, R, NT>(A, cb, c, in, gbytes, ua, pa);
        hop_pipelined<0, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<1, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ub, pb, ua, pa);
        hop_pipelined<2, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<3, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ub, pb, ua, pa);
        hop_pipelined<4, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<5, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ub, pb, ua, pa);
        hop_pipelined<6, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<7, P, R, DAG, NT>(A, cb, c, in, gbytes, acc, ub, pb, ua, pa);
    } else {
        hop<0, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<1, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<2, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<3, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<4, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<5, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<6, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
        hop<7, P, R, DAG, NT>(A, cb, c, in, gbytes, acc);
    }
    const T b = (T)A.b;
    T xv[24];
    if constexpr (XPAY) {
        // x is read once, at the site written: a non-temporal load leaves the last-level cache
        // to the fields the next launch reads (measured: 0.75% on the Mhat^dag Mhat step)
        if (A.xnt) SpinorIO<P>::load_nt(A.x + rhs * A.x_stride, A.g.ps, cb, xv);
        else SpinorIO<P>::load(A.x + rhs * A.x_stride, A.g.ps, cb, xv);
        const T a = (T)A.a;
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = a * xv[k] + b * acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] *= b;
    }
    if constexpr (RED == RED_CGR) {
        // r -= alpha (a x + b D in) at the accumulation precision; the operator's own result
        // is never stored
        constexpr int PA = P == P_F64 ? P_F64 : P_F32;
        using TA = typename RealOf<PA>::T;
        char* rp = A.out + rhs * A.out_stride;
        TA rv[24];
        SpinorIO<PA>::load(rp, A.g.ps, cb, rv);
        const TA al = (TA)A.coef[0];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            rv[k] -= al * (TA)acc[k];
            s += (double)rv[k] * (double)rv[k];
        }
        SpinorIO<PA>::store(rp, A.g.ps, cb, rv);
        red[0] = s;
        return;
    }
    if constexpr (RED == RED_RESLO) {
        // the float64 residual y - (a x + b D in), its norm taken before it is stored in float32
        T yv[24];
        float lo[24];
        SpinorIO<P>::load(A.y + rhs * A.out_stride, A.g.ps, cb, yv);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            const double d = (double)yv[k] - (double)acc[k];
            s += d * d;
            lo[k] = (float)d;
        }
        SpinorIO<P_F32>::store(A.out + rhs * A.out_stride, A.g.ps, cb, lo);
        red[0] = s;
        return;
    }
    if constexpr (RED == 4) {   // the residual y - (a x + b D in) is what is stored
        T yv[24];
        SpinorIO<P>::load(A.y + rhs * A.out_stride, A.g.ps, cb, yv);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = yv[k] - acc[k];
    }
    SpinorIO<P>::store(A.out + rhs * A.out_stride, A.g.ps, cb, acc);
    if constexpr (RED > 0) {
        // the reduction sees the values a later load returns (16-bit: the codes times the scale)
        if constexpr (P == P_F16 || P == P_BF16) quant_roundtrip<P>(acc);
        if constexpr (RED == 1 || RED == 4) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 24; ++k) s += (double)acc[k] * (double)acc[k];
            red[0] = s;
        } else if constexpr (RED == 2) {
            site_dot_norm(acc, xv, acc, red);
        } else if constexpr (RED == 3) {
            T yv[24];
            SpinorIO<P>::load(A.y + rhs * A.out_stride, A.g.ps, cb, yv);
            site_dot_norm(yv, acc, acc, red);
        } else {
            T yv[24];
            SpinorIO<P>::load(A.y + rhs * A.out_stride, A.g.ps, cb, yv);
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 24; ++k) {
                const double d = (double)yv[k] - (double)acc[k];
                s += d * d;
            }
            red[0] = s;
        }
    }
}

template <int P, int R, bool DAG, bool XPAY, bool NT, bool PF, int RED = 0>
__device__ __forceinline__ void dslash_site(const DslashArgs& A, uint32_t cb, int rhs, double* red = nullptr)
{
    int c[4];
    cb_coords(A.g, cb, A.par, c);
    dslash_site<P, R, DAG, XPAY, NT, PF, RED>(A, cb, c, rhs, red);
}

} // namespace wd
