// Vector updates and float64 global sums on packed fields (paper Section 4:
// the dot product is a global sum done by the GPU in double precision by
// parallel reduction; the other solver steps are BLAS-like kernels).
//
// A field is a run of `nhalves` half fields, each holding Vh sites of 24
// reals; element-wise kernels walk sites, so every packed precision and
// subset shares one code path.  Reductions are deterministic: a fixed grid of
// workgroups each reduces a fixed strided set of sites (wave shuffles, then
// LDS), and one workgroup sums the partials in a fixed order.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "wd_core.h"

namespace wd {

constexpr int RED_BLOCK = 256;
constexpr int RED_MAXBLOCKS = 2048;

struct SiteRange {
    const char* base;
    int Vh;      // sites per half field
    int ps;      // plane stride of a half field
    size_t hb;   // bytes of one half field
    __device__ __forceinline__ const char* half(long long h) const { return base + (size_t)h * hb; }
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce N values over the workgroup; thread 0 writes partials[n * nblk + blockIdx.x].
template <int N> __device__ __forceinline__ void block_reduce(double* v, double* partials)
{
    __shared__ double lds[N][RED_BLOCK / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double s = wave_sum(v[n]);
        if (lane == 0) lds[n][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            double s = 0.0;
            for (int w = 0; w < RED_BLOCK / 64; ++w) s += lds[n][w];
            partials[(size_t)n * gridDim.x + blockIdx.x] = s;
        }
    }
}

// This thread's share of the sum of p[0 .. n) over a RED_BLOCK workgroup, in a fixed order:
// four accumulators, so that four loads are in flight per thread instead of one at a time.
__device__ __forceinline__ double thread_share(const double* __restrict__ p, int n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * RED_BLOCK < n; i += 4 * RED_BLOCK) {
        s0 += p[i];
        s1 += p[i + RED_BLOCK];
        s2 += p[i + 2 * RED_BLOCK];
        s3 += p[i + 3 * RED_BLOCK];
    }
    for (; i < n; i += RED_BLOCK) s0 += p[i];
    return (s0 + s1) + (s2 + s3);
}

// One workgroup per reduced value: partials of value k summed in a fixed order, the
// result written to device memory and to the mapped pinned host copy.
__global__ void __launch_bounds__(RED_BLOCK) finish_kernel(const double* __restrict__ partials, int nblk,
                                                           double* __restrict__ out, double* __restrict__ host_out)
{
    __shared__ double lds[RED_BLOCK / 64];
    const int k = blockIdx.x;
    double s = thread_share(partials + (size_t)k * nblk, nblk);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RED_BLOCK / 64; ++w) t += lds[w];
        out[k] = t;
        if (host_out) host_out[k] = t;
    }
}

static int red_blocks(long long nsites)
{
    long long b = (nsites + RED_BLOCK - 1) / RED_BLOCK;
    return (int)(b < RED_MAXBLOCKS ? (b < 1 ? 1 : b) : RED_MAXBLOCKS);
}

// With a mapped host buffer the host waits for results by spinning on the slots themselves:
// each is armed with a NaN payload before the kernel that writes it is queued (no arithmetic
// produces that payload).  A stream or event wait would also write the whole L2 back to memory
// and leave the GPU idle for tens of microseconds per wait.
constexpr uint64_t RES_PENDING = 0x7ff4c0ffee000001ull;

static void arm_slots(wd_context ctx, int slot, int n)
{
    if (!ctx->hres_dev) return;
    volatile uint64_t* h = (volatile uint64_t*)ctx->hres;
    for (int i = 0; i < n; ++i) h[slot + i] = RES_PENDING;
}

static wd_status wait_slots(wd_context ctx, int slot, int n)
{
    volatile uint64_t* h = (volatile uint64_t*)ctx->hres;
    auto ready = [&]() {
        for (int i = 0; i < n; ++i)
            if (h[slot + i] == RES_PENDING) return false;
        return true;
    };
    auto last = std::chrono::steady_clock::now();
    for (unsigned spins = 1; !ready(); ++spins) {
        // every 2 ms (a query takes the runtime's locks, so not more often): once the stream has
        // drained, the slots hold whatever was written, and a HIP error ends the wait
        if ((spins & 255u) == 0 && std::chrono::steady_clock::now() - last > std::chrono::milliseconds(2)) {
            last = std::chrono::steady_clock::now();
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) {
                set_error("HIP error while waiting for reduction results: %s", hipGetErrorString(e));
                return WD_EHIP;
            }
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return WD_OK;
}

// Values land in dres[slot ..] and its host copy hres[slot ..] (mapped: written by the
// kernel; else copied behind it on the stream).
static wd_status finish(wd_context ctx, int nblk, int n, bool fetch, int slot = 0)
{
    arm_slots(ctx, slot, n);
    hipLaunchKernelGGL(finish_kernel, dim3(n), dim3(RED_BLOCK), 0, ctx->stream, ctx->partials, nblk, ctx->dres + slot,
                       ctx->hres_dev ? ctx->hres_dev + slot : nullptr);
    WD_LAUNCHED();
    if (!ctx->hres_dev && slot != 0)
        WD_HIP(hipMemcpyAsync(ctx->hres + slot, ctx->dres + slot, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    if (!fetch) return WD_OK;
    if (ctx->hres_dev) return wait_slots(ctx, slot, n);
    return fetch_results(ctx, slot == 0 ? n : 0);
}

bool is_zero_f64(wd_context ctx, const Geom& g, size_t nhalves, const void* x)
{
    return blas_norm2(ctx, g, nhalves, WD_F64, x, true) == WD_OK && ctx->hres[0] == 0.0;
}

wd_status reduce_partials(wd_context ctx, int nblk, int n, int slot) { return finish(ctx, nblk, n, false, slot); }

wd_status fetch_results(wd_context ctx, int n)
{
    if (ctx->hres_dev) return wait_slots(ctx, 0, n);
    // no mapped host buffer: copy the results over
    WD_HIP(hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    WD_HIP(hipStreamSynchronize(ctx->stream));
    return WD_OK;
}

// ---- dot / norm ------------------------------------------------------------------
template <int P, bool DOT>
__global__ void __launch_bounds__(RED_BLOCK) dot_kernel(SiteRange A, SiteRange B, long long nsites, double* partials)
{
    double acc[2] = {0.0, 0.0};
    for (long long k = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; k < nsites; k += (long long)gridDim.x * RED_BLOCK) {
        const long long h = k / A.Vh;
        const uint32_t cb = (uint32_t)(k - h * A.Vh);
        typename RealOf<P>::T a[24];
        SpinorIO<P>::load(A.half(h), A.ps, cb, a);
        if constexpr (DOT) {
            typename RealOf<P>::T b[24];
            SpinorIO<P>::load(B.half(h), B.ps, cb, b);
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
                acc[0] += ar * br + ai * bi;   // Re conj(a) b
                acc[1] += ar * bi - ai * br;   // Im conj(a) b
            }
        } else {
#pragma unroll
            for (int i = 0; i < 24; ++i) acc[0] += (double)a[i] * (double)a[i];
        }
    }
    block_reduce<DOT ? 2 : 1>(acc, partials);
}

template <int P, bool DOT>
static wd_status dot_t(wd_context ctx, const Geom& g, size_t nh, const void* a, const void* b, bool fetch)
{
    const long long n = (long long)nh * g.Vh;
    const int nblk = red_blocks(n);
    WD_TRY(ensure_reduction(ctx, (size_t)nblk * 2));
    SiteRange A{(const char*)a, g.Vh, g.ps, half_bytes(g, P)}, B{(const char*)b, g.Vh, g.ps, half_bytes(g, P)};
    hipLaunchKernelGGL((dot_kernel<P, DOT>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, A, B, n, ctx->partials);
    WD_LAUNCHED();
    return finish(ctx, nblk, DOT ? 2 : 1, fetch);
}

wd_status blas_dot(wd_context ctx, const Geom& g, size_t nh, int prec, const void* a, const void* b, bool fetch)
{
    switch (prec) {
    case WD_F64: return dot_t<P_F64, true>(ctx, g, nh, a, b, fetch);
    case WD_F32: return dot_t<P_F32, true>(ctx, g, nh, a, b, fetch);
    case WD_F16: return dot_t<P_F16, true>(ctx, g, nh, a, b, fetch);
    case WD_BF16: return dot_t<P_BF16, true>(ctx, g, nh, a, b, fetch);
    }
    set_error("dot: bad precision %d", prec);
    return WD_EINVAL;
}

wd_status blas_norm2(wd_context ctx, const Geom& g, size_t nh, int prec, const void* a, bool fetch)
{
    switch (prec) {
    case WD_F64: return dot_t<P_F64, false>(ctx, g, nh, a, a, fetch);
    case WD_F32: return dot_t<P_F32, false>(ctx, g, nh, a, a, fetch);
    case WD_F16: return dot_t<P_F16, false>(ctx, g, nh, a, a, fetch);
    case WD_BF16: return dot_t<P_BF16, false>(ctx, g, nh, a, a, fetch);
    }
    set_error("norm2: bad precision %d", prec);
    return WD_EINVAL;
}

// ---- element-wise ----------------------------------------------------------------
#define WD_SITE_LOOP(nsites, Vh)                                                                         \
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;                                 \
    if (k >= (nsites)) return;                                                                            \
    const long long h = k / (Vh);                                                                         \
    const uint32_t cb = (uint32_t)(k - h * (Vh));

static dim3 site_grid(long long n) { return dim3((unsigned)((n + 255) / 256)); }

template <int P>
__global__ void caxpy_kernel(SiteRange X, SiteRange Y, long long n, double ar, double ai)
{
    WD_SITE_LOOP(n, X.Vh)
    using T = typename RealOf<P>::T;
    T x[24], y[24];
    SpinorIO<P>::load(X.half(h), X.ps, cb, x);
    SpinorIO<P>::load(Y.half(h), Y.ps, cb, y);
    const T a = (T)ar, b = (T)ai;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const T xr = x[2 * i], xi = x[2 * i + 1];
        y[2 * i] += a * xr - b * xi;
        y[2 * i + 1] += a * xi + b * xr;
    }
    SpinorIO<P>::store((char*)Y.half(h), Y.ps, cb, y);
}

wd_status blas_caxpy(wd_context ctx, const Geom& g, size_t nh, int prec, double ar, double ai, const void* x, void* y)
{
    const long long n = (long long)nh * g.Vh;
    SiteRange X{(const char*)x, g.Vh, g.ps, half_bytes(g, prec)}, Y{(const char*)y, g.Vh, g.ps, half_bytes(g, prec)};
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL(caxpy_kernel<P_F64>, site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, ar, ai); break;
    case WD_F32: hipLaunchKernelGGL(caxpy_kernel<P_F32>, site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, ar, ai); break;
    default: set_error("caxpy: precision %d not supported (F32, F64 only)", prec); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return WD_OK;
}

template <int P>
__global__ void zero_kernel(char* base, int Vh, int ps, size_t hb, long long n)
{
    WD_SITE_LOOP(n, Vh)
    typename RealOf<P>::T z[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) z[i] = 0;
    SpinorIO<P>::store(base + (size_t)h * hb, ps, cb, z);
}

wd_status blas_zero(wd_context ctx, const Geom& g, size_t nh, int prec, void* x)
{
    const long long n = (long long)nh * g.Vh;
    const size_t hb = half_bytes(g, prec);
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL(zero_kernel<P_F64>, site_grid(n), dim3(256), 0, ctx->stream, (char*)x, g.Vh, g.ps, hb, n); break;
    case WD_F32: hipLaunchKernelGGL(zero_kernel<P_F32>, site_grid(n), dim3(256), 0, ctx->stream, (char*)x, g.Vh, g.ps, hb, n); break;
    case WD_F16: hipLaunchKernelGGL(zero_kernel<P_F16>, site_grid(n), dim3(256), 0, ctx->stream, (char*)x, g.Vh, g.ps, hb, n); break;
    case WD_BF16: hipLaunchKernelGGL(zero_kernel<P_BF16>, site_grid(n), dim3(256), 0, ctx->stream, (char*)x, g.Vh, g.ps, hb, n); break;
    default: set_error("zero: bad precision %d", prec); return WD_EINVAL;
    }
    WD_LAUNCHED();
    return WD_OK;
}

// y = a x + b y, x at PX, y at PY; arithmetic in float64 if either is F64
template <int PX, int PY>
__global__ void axpby_kernel(SiteRange X, SiteRange Y, long long n, double a, double b)
{
    WD_SITE_LOOP(n, X.Vh)
    using T = typename std::conditional<(PX == P_F64 || PY == P_F64), double, float>::type;
    typename RealOf<PX>::T x[24];
    typename RealOf<PY>::T y[24];
    SpinorIO<PX>::load(X.half(h), X.ps, cb, x);
    SpinorIO<PY>::load(Y.half(h), Y.ps, cb, y);
#pragma unroll
    for (int i = 0; i < 24; ++i) y[i] = (typename RealOf<PY>::T)((T)a * (T)x[i] + (T)b * (T)y[i]);
    SpinorIO<PY>::store((char*)Y.half(h), Y.ps, cb, y);
}

template <int PX>
static wd_status axpby_x(wd_context ctx, long long n, SiteRange X, SiteRange Y, int py, double a, double b)
{
    switch (py) {
    case WD_F64: hipLaunchKernelGGL((axpby_kernel<PX, P_F64>), site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, a, b); break;
    case WD_F32: hipLaunchKernelGGL((axpby_kernel<PX, P_F32>), site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, a, b); break;
    case WD_F16: hipLaunchKernelGGL((axpby_kernel<PX, P_F16>), site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, a, b); break;
    case WD_BF16: hipLaunchKernelGGL((axpby_kernel<PX, P_BF16>), site_grid(n), dim3(256), 0, ctx->stream, X, Y, n, a, b); break;
    default: set_error("axpby: bad precision %d", py); return WD_EINVAL;
    }
    WD_LAUNCHED();
    return WD_OK;
}

wd_status blas_axpby(wd_context ctx, const Geom& g, size_t nh, int px, const void* x, double a, int py, void* y, double b)
{
    const long long n = (long long)nh * g.Vh;
    SiteRange X{(const char*)x, g.Vh, g.ps, half_bytes(g, px)}, Y{(const char*)y, g.Vh, g.ps, half_bytes(g, py)};
    switch (px) {
    case WD_F64: return axpby_x<P_F64>(ctx, n, X, Y, py, a, b);
    case WD_F32: return axpby_x<P_F32>(ctx, n, X, Y, py, a, b);
    case WD_F16: return axpby_x<P_F16>(ctx, n, X, Y, py, a, b);
    case WD_BF16: return axpby_x<P_BF16>(ctx, n, X, Y, py, a, b);
    }
    set_error("axpby: bad precision %d", px);
    return WD_EINVAL;
}

// ---- CG steps with their coefficients on the device ----------------------------------
// The CG scalars live in dres[CG_SLOT + ...] (CG_RR the current sloppy ||r||^2, CG_PAP, CG_ALPHA,
// CG_RRNEW, CG_BETA): the step length is formed on the device by the sum that produces <p, A p>
// and read there by the launch that updates r, so no host round trip sits between the two
// operator applications of an iteration.
static_assert(CG_SLOT + CG_NSLOTS <= 256, "CG scalars past the end of dres");

// mode 0: pap = the sum, alpha = rr / pap.  mode 1: rr_new = the sum, beta = rr_new / rr, and
// rr_new becomes rr.  The sum goes to the host copy as well.
__global__ void __launch_bounds__(RED_BLOCK) cg_coef_kernel(const double* __restrict__ partials, int nblk,
                                                            double* __restrict__ cg, double* __restrict__ host_cg,
                                                            int mode)
{
    __shared__ double lds[RED_BLOCK / 64];
    double s = thread_share(partials, nblk);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RED_BLOCK / 64; ++w) t += lds[w];
        if (mode == 0) {
            cg[CG_PAP] = t;
            cg[CG_ALPHA] = cg[CG_RR] / t;
            if (host_cg) host_cg[CG_PAP] = t;
        } else {
            cg[CG_RRNEW] = t;
            cg[CG_BETA] = t / cg[CG_RR];
            cg[CG_RR] = t;
            if (host_cg) host_cg[CG_RRNEW] = t;
        }
    }
}

__global__ void cg_set_kernel(double* cg, double rr, double beta)
{
    if (threadIdx.x == 0) {
        cg[CG_RR] = rr;
        cg[CG_BETA] = beta;
    }
}

wd_status blas_cg_coef(wd_context ctx, int nblk, int mode)
{
    double* host = ctx->hres_dev ? ctx->hres_dev + CG_SLOT : nullptr;
    hipLaunchKernelGGL(cg_coef_kernel, dim3(1), dim3(RED_BLOCK), 0, ctx->stream, ctx->partials, nblk,
                       ctx->dres + CG_SLOT, host, mode);
    WD_LAUNCHED();
    if (!ctx->hres_dev) {
        const int k = mode == 0 ? CG_PAP : CG_RRNEW;
        WD_HIP(hipMemcpyAsync(ctx->hres + CG_SLOT + k, ctx->dres + CG_SLOT + k, sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream));
    }
    return WD_OK;
}

void blas_cg_arm(wd_context ctx) { arm_slots(ctx, CG_SLOT + CG_PAP, 2); }

wd_status blas_cg_wait(wd_context ctx)
{
    if (!ctx->hres_dev) {   // the copies were queued behind the kernels
        WD_HIP(hipStreamSynchronize(ctx->stream));
        return WD_OK;
    }
    return wait_slots(ctx, CG_SLOT + CG_PAP, 2);
}

wd_status blas_cg_set(wd_context ctx, double rr, double beta)
{
    hipLaunchKernelGGL(cg_set_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->dres + CG_SLOT, rr, beta);
    WD_LAUNCHED();
    return WD_OK;
}

// x += alpha p (XM 0), x = alpha p (XM 1) or x untouched (XM 2); then q = r + beta p (q may be
// p).  x and r at the accumulation precision PA, p and q at the operator's PO; alpha and beta
// read on the device.
template <int PA, int PO, int XM>
__global__ void cg_xp_kernel(SiteRange X, SiteRange R, SiteRange Pp, char* q, long long n, const double* __restrict__ cg)
{
    WD_SITE_LOOP(n, R.Vh)
    using T = typename RealOf<PA>::T;
    T r[24];
    typename RealOf<PO>::T p[24];
    SpinorIO<PO>::load(Pp.half(h), Pp.ps, cb, p);
    SpinorIO<PA>::load(R.half(h), R.ps, cb, r);
    const T al = (T)cg[CG_ALPHA], be = (T)cg[CG_BETA];
    if constexpr (XM != 2) {
        T x[24];
        if constexpr (XM == 0) SpinorIO<PA>::load(X.half(h), X.ps, cb, x);
#pragma unroll
        for (int i = 0; i < 24; ++i) x[i] = XM == 0 ? x[i] + al * (T)p[i] : al * (T)p[i];
        SpinorIO<PA>::store((char*)X.half(h), X.ps, cb, x);
    }
#pragma unroll
    for (int i = 0; i < 24; ++i) p[i] = (typename RealOf<PO>::T)(r[i] + be * (T)p[i]);
    SpinorIO<PO>::store(q + (size_t)h * Pp.hb, Pp.ps, cb, p);
}

template <int PA, int PO>
static wd_status cg_xp_t(wd_context ctx, long long n, SiteRange X, SiteRange R, SiteRange Pp, char* q, int xmode)
{
    const double* cg = ctx->dres + CG_SLOT;
    switch (xmode) {
    case 0: hipLaunchKernelGGL((cg_xp_kernel<PA, PO, 0>), site_grid(n), dim3(256), 0, ctx->stream, X, R, Pp, q, n, cg); break;
    case 1: hipLaunchKernelGGL((cg_xp_kernel<PA, PO, 1>), site_grid(n), dim3(256), 0, ctx->stream, X, R, Pp, q, n, cg); break;
    default: hipLaunchKernelGGL((cg_xp_kernel<PA, PO, 2>), site_grid(n), dim3(256), 0, ctx->stream, X, R, Pp, q, n, cg); break;
    }
    WD_LAUNCHED();
    return WD_OK;
}

wd_status blas_cg_xp(wd_context ctx, const Geom& g, size_t nh, int pacc, void* x, int xmode, const void* r, int pop,
                     const void* p, void* q)
{
    const long long n = (long long)nh * g.Vh;
    SiteRange X{(const char*)x, g.Vh, g.ps, half_bytes(g, pacc)}, R{(const char*)r, g.Vh, g.ps, half_bytes(g, pacc)},
        Pp{(const char*)p, g.Vh, g.ps, half_bytes(g, pop)};
    if (xmode < 0 || xmode > 2) {
        set_error("cg_xp: bad mode %d", xmode);
        return WD_EINVAL;
    }
    char* qc = (char*)q;
    if (pacc == WD_F64 && pop == WD_F64) return cg_xp_t<P_F64, P_F64>(ctx, n, X, R, Pp, qc, xmode);
    if (pacc == WD_F32 && pop == WD_F32) return cg_xp_t<P_F32, P_F32>(ctx, n, X, R, Pp, qc, xmode);
    if (pacc == WD_F32 && pop == WD_F16) return cg_xp_t<P_F32, P_F16>(ctx, n, X, R, Pp, qc, xmode);
    if (pacc == WD_F32 && pop == WD_BF16) return cg_xp_t<P_F32, P_BF16>(ctx, n, X, R, Pp, qc, xmode);
    set_error("cg_xp: unsupported precision pair (%d, %d)", pacc, pop);
    return WD_EUNSUPPORTED;
}

// ---- fused linear combinations (BiCGstab) ------------------------------------------------
// out = sum_{i < n} c_i X_i (complex c_i, n <= 3; out may be one of the X_i).  RED adds the
// reductions ||out||^2 and <R0, out> (values 0, 1, 2 = ||out||^2, Re, Im), so one sweep both
// updates a vector and produces the next iteration's scalars.
struct Lincomb {
    SiteRange X[3];
    double cr[3], ci[3];
    int n;
};

template <int P, bool RED>
__global__ void __launch_bounds__(RED_BLOCK) lincomb_kernel(Lincomb L, SiteRange O, SiteRange R0, long long nsites,
                                                            double* partials)
{
    using T = typename RealOf<P>::T;
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long s = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; s < nsites; s += (long long)gridDim.x * RED_BLOCK) {
        const long long h = s / O.Vh;
        const uint32_t cb = (uint32_t)(s - h * O.Vh);
        T o[24];
#pragma unroll
        for (int q = 0; q < 24; ++q) o[q] = 0;
        for (int i = 0; i < L.n; ++i) {
            T x[24];
            SpinorIO<P>::load(L.X[i].half(h), O.ps, cb, x);
            const T ar = (T)L.cr[i], ai = (T)L.ci[i];
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                o[2 * q] += ar * x[2 * q] - ai * x[2 * q + 1];
                o[2 * q + 1] += ar * x[2 * q + 1] + ai * x[2 * q];
            }
        }
        SpinorIO<P>::store((char*)O.half(h), O.ps, cb, o);
        if constexpr (RED) {
            T r0[24];
            SpinorIO<P>::load(R0.half(h), O.ps, cb, r0);
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const double orr = o[2 * q], oi = o[2 * q + 1], ar = r0[2 * q], ai = r0[2 * q + 1];
                acc[0] += orr * orr + oi * oi;
                acc[1] += ar * orr + ai * oi;
                acc[2] += ar * oi - ai * orr;
            }
        }
    }
    if constexpr (RED) block_reduce<3>(acc, partials);
}

// BiCGstab's two closing updates in one sweep over s: xs += alpha p + omega s and
// r = s - omega t, with ||r||^2 and <r0, r> (values 0, 1, 2), each in the order and with the
// values lincomb_kernel uses for it alone.
struct BicgXR {
    SiteRange Xs, P, S, T, R0, Rs;
    double ar, ai, wr, wi;
};

template <int P>
__global__ void __launch_bounds__(RED_BLOCK) bicg_xr_kernel(BicgXR B, long long nsites, double* partials)
{
    using T = typename RealOf<P>::T;
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long st = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; st < nsites;
         st += (long long)gridDim.x * RED_BLOCK) {
        const long long h = st / B.Xs.Vh;
        const uint32_t cb = (uint32_t)(st - h * B.Xs.Vh);
        const int ps = B.Xs.ps;
        T sv[24], o[24], x[24];
        SpinorIO<P>::load(B.S.half(h), ps, cb, sv);
        // xs + alpha p + omega s
#pragma unroll
        for (int q = 0; q < 24; ++q) o[q] = 0;
        const T one = (T)1.0, zero = (T)0.0;
        SpinorIO<P>::load(B.Xs.half(h), ps, cb, x);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            o[2 * q] += one * x[2 * q] - zero * x[2 * q + 1];
            o[2 * q + 1] += one * x[2 * q + 1] + zero * x[2 * q];
        }
        SpinorIO<P>::load(B.P.half(h), ps, cb, x);
        const T ar = (T)B.ar, ai = (T)B.ai, wr = (T)B.wr, wi = (T)B.wi;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            o[2 * q] += ar * x[2 * q] - ai * x[2 * q + 1];
            o[2 * q + 1] += ar * x[2 * q + 1] + ai * x[2 * q];
        }
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            o[2 * q] += wr * sv[2 * q] - wi * sv[2 * q + 1];
            o[2 * q + 1] += wr * sv[2 * q + 1] + wi * sv[2 * q];
        }
        SpinorIO<P>::store((char*)B.Xs.half(h), ps, cb, o);
        // s - omega t
#pragma unroll
        for (int q = 0; q < 24; ++q) o[q] = 0;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            o[2 * q] += one * sv[2 * q] - zero * sv[2 * q + 1];
            o[2 * q + 1] += one * sv[2 * q + 1] + zero * sv[2 * q];
        }
        SpinorIO<P>::load(B.T.half(h), ps, cb, x);
        const T mwr = (T)(-B.wr), mwi = (T)(-B.wi);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            o[2 * q] += mwr * x[2 * q] - mwi * x[2 * q + 1];
            o[2 * q + 1] += mwr * x[2 * q + 1] + mwi * x[2 * q];
        }
        SpinorIO<P>::store((char*)B.Rs.half(h), ps, cb, o);
        SpinorIO<P>::load(B.R0.half(h), ps, cb, x);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const double orr = o[2 * q], oi = o[2 * q + 1], rr = x[2 * q], ri = x[2 * q + 1];
            acc[0] += orr * orr + oi * oi;
            acc[1] += rr * orr + ri * oi;
            acc[2] += rr * oi - ri * orr;
        }
    }
    block_reduce<3>(acc, partials);
}

wd_status blas_bicg_xr(wd_context ctx, const Geom& g, int prec, void* xs, const void* p, const void* s, const void* t,
                       const void* r0, void* rs, double alpha_re, double alpha_im, double omega_re, double omega_im,
                       bool fetch)
{
    const size_t hb = half_bytes(g, prec);
    auto R = [&](const void* q) { return SiteRange{(const char*)q, g.Vh, g.ps, hb}; };
    BicgXR B{R(xs), R(p), R(s), R(t), R(r0), R(rs), alpha_re, alpha_im, omega_re, omega_im};
    const long long ns = g.Vh;
    const int nblk = red_blocks(ns);
    WD_TRY(ensure_reduction(ctx, (size_t)nblk * 3));
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL((bicg_xr_kernel<P_F64>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, B, ns, ctx->partials); break;
    case WD_F32: hipLaunchKernelGGL((bicg_xr_kernel<P_F32>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, B, ns, ctx->partials); break;
    case WD_F16: hipLaunchKernelGGL((bicg_xr_kernel<P_F16>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, B, ns, ctx->partials); break;
    case WD_BF16: hipLaunchKernelGGL((bicg_xr_kernel<P_BF16>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, B, ns, ctx->partials); break;
    default: set_error("bicg_xr: bad precision %d", prec); return WD_EINVAL;
    }
    WD_LAUNCHED();
    return finish(ctx, nblk, 3, fetch);
}

wd_status blas_lincomb(wd_context ctx, const Geom& g, size_t nh, int prec, int n, const void* const* x,
                       const double* cre, const double* cim, void* out, const void* r0, bool fetch)
{
    if (n < 1 || n > 3) {
        set_error("lincomb: %d inputs (1..3)", n);
        return WD_EINVAL;
    }
    Lincomb L;
    L.n = n;
    const size_t hb = half_bytes(g, prec);
    for (int i = 0; i < 3; ++i) {
        L.X[i] = SiteRange{(const char*)(i < n ? x[i] : out), g.Vh, g.ps, hb};
        L.cr[i] = i < n ? cre[i] : 0.0;
        L.ci[i] = i < n ? cim[i] : 0.0;
    }
    SiteRange O{(const char*)out, g.Vh, g.ps, hb}, R{(const char*)(r0 ? r0 : out), g.Vh, g.ps, hb};
    const long long ns = (long long)nh * g.Vh;
    const int nblk = red_blocks(ns);
    if (r0) WD_TRY(ensure_reduction(ctx, (size_t)nblk * 3));
#define WD_LC(PP)                                                                                                   \
    if (r0) hipLaunchKernelGGL((lincomb_kernel<PP, true>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, L, O, R, ns,   \
                               ctx->partials);                                                                       \
    else hipLaunchKernelGGL((lincomb_kernel<PP, false>), dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, L, O, R, ns,     \
                            ctx->partials);
    switch (prec) {
    case WD_F64: WD_LC(P_F64) break;
    case WD_F32: WD_LC(P_F32) break;
    case WD_F16: WD_LC(P_F16) break;
    case WD_BF16: WD_LC(P_BF16) break;
    default: set_error("lincomb: bad precision %d", prec); return WD_EINVAL;
    }
#undef WD_LC
    WD_LAUNCHED();
    if (r0) return finish(ctx, nblk, 3, fetch);
    return WD_OK;
}

// ---- block Gram-Schmidt helpers (flexible GMRES) ---------------------------------------
// <V_i, w> for i < k, and (with_norm) ||w||^2 as value k.  Vectors go in groups of four:
// w is read once per group, so a pass reads k + ceil((k + 1) / 4) fields instead of 2 (k + 1).
constexpr int MDOT_GROUP = 4;

template <int P>
__global__ void __launch_bounds__(RED_BLOCK) mdot_kernel(SiteRange Vs, size_t vstride, int k, int with_norm, SiteRange W,
                                                         long long nsites, double* partials)
{
    const int n = k + (with_norm ? 1 : 0);
    for (int i0 = 0; i0 < n; i0 += MDOT_GROUP) {
        double acc[2 * MDOT_GROUP];
#pragma unroll
        for (int q = 0; q < 2 * MDOT_GROUP; ++q) acc[q] = 0.0;
        for (long long s = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; s < nsites; s += (long long)gridDim.x * RED_BLOCK) {
            const long long h = s / W.Vh;
            const uint32_t cb = (uint32_t)(s - h * W.Vh);
            typename RealOf<P>::T b[24];
            SpinorIO<P>::load(W.half(h), W.ps, cb, b);
#pragma unroll
            for (int u = 0; u < MDOT_GROUP; ++u) {
                const int i = i0 + u;
                if (i >= n) break;
                typename RealOf<P>::T a[24];
                if (i < k) SpinorIO<P>::load(Vs.half(h) + (size_t)i * vstride, W.ps, cb, a);
                else {
#pragma unroll
                    for (int q = 0; q < 24; ++q) a[q] = b[q];
                }
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const double ar = a[2 * q], ai = a[2 * q + 1], br = b[2 * q], bi = b[2 * q + 1];
                    acc[2 * u] += ar * br + ai * bi;
                    acc[2 * u + 1] += ar * bi - ai * br;
                }
            }
        }
        block_reduce<2 * MDOT_GROUP>(acc, partials + (size_t)2 * i0 * gridDim.x);
        __syncthreads();
    }
}

wd_status blas_mdot(wd_context ctx, const Geom& g, size_t nh, int prec, const void* V, size_t vstride, int k,
                    const void* w, bool with_norm, bool fetch, int slot)
{
    const int n = k + (with_norm ? 1 : 0);
    if (k < 0 || n < 1 || slot < 0 || slot + 2 * n > 256) {
        set_error("mdot: k = %d (slot %d) out of range", k, slot);
        return WD_EINVAL;
    }
    const long long ns = (long long)nh * g.Vh;
    const int nblk = red_blocks(ns);
    const int ngrp = (n + MDOT_GROUP - 1) / MDOT_GROUP;
    WD_TRY(ensure_reduction(ctx, (size_t)nblk * 2 * MDOT_GROUP * ngrp));
    SiteRange Vs{(const char*)V, g.Vh, g.ps, half_bytes(g, prec)}, W{(const char*)w, g.Vh, g.ps, half_bytes(g, prec)};
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL(mdot_kernel<P_F64>, dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, Vs, vstride, k, (int)with_norm, W, ns, ctx->partials); break;
    case WD_F32: hipLaunchKernelGGL(mdot_kernel<P_F32>, dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, Vs, vstride, k, (int)with_norm, W, ns, ctx->partials); break;
    default: set_error("mdot: precision %d not supported", prec); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return finish(ctx, nblk, 2 * n, fetch, slot);
}

struct MaxpyCoef {
    float c[2 * WD_MAXPY];
};

// out = scale * (w + sum_i c_i V_i); out may be w.  With dcoef non-null the coefficients are
// c_i = dsign * (dcoef[2i], dcoef[2i + 1]), read from device memory (a previous reduction).
template <int P>
__global__ void maxpy_kernel(SiteRange Vs, size_t vstride, int nvec, MaxpyCoef cf, const double* dcoef, float dsign,
                             float scale, SiteRange W, SiteRange O, long long n)
{
    WD_SITE_LOOP(n, W.Vh)
    using T = typename RealOf<P>::T;
    T w[24];
    SpinorIO<P>::load(W.half(h), W.ps, cb, w);
    for (int i = 0; i < nvec; ++i) {
        T v[24];
        SpinorIO<P>::load(Vs.half(h) + (size_t)i * vstride, W.ps, cb, v);
        const T cr = dcoef ? (T)(dsign * (float)dcoef[2 * i]) : (T)cf.c[2 * i];
        const T ci = dcoef ? (T)(dsign * (float)dcoef[2 * i + 1]) : (T)cf.c[2 * i + 1];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            w[2 * q] += cr * v[2 * q] - ci * v[2 * q + 1];
            w[2 * q + 1] += cr * v[2 * q + 1] + ci * v[2 * q];
        }
    }
#pragma unroll
    for (int q = 0; q < 24; ++q) w[q] *= (T)scale;
    SpinorIO<P>::store((char*)O.half(h), W.ps, cb, w);
}

static wd_status maxpy_any(wd_context ctx, const Geom& g, size_t nh, int prec, const void* V, size_t vstride, int k,
                           const double* coef, const double* dcoef, float dsign, const void* w, double scale, void* out)
{
    if (k < 0 || k > WD_MAXPY) {
        set_error("maxpy: k = %d out of range", k);
        return WD_EINVAL;
    }
    MaxpyCoef cf;
    for (int i = 0; i < 2 * k; ++i) cf.c[i] = coef ? (float)coef[i] : 0.f;
    const long long n = (long long)nh * g.Vh;
    SiteRange Vs{(const char*)V, g.Vh, g.ps, half_bytes(g, prec)}, W{(const char*)w, g.Vh, g.ps, half_bytes(g, prec)},
        O{(const char*)out, g.Vh, g.ps, half_bytes(g, prec)};
    switch (prec) {
    case WD_F32: hipLaunchKernelGGL(maxpy_kernel<P_F32>, site_grid(n), dim3(256), 0, ctx->stream, Vs, vstride, k, cf, dcoef, dsign, (float)scale, W, O, n); break;
    default: set_error("maxpy: precision %d not supported (F32 only)", prec); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return WD_OK;
}

wd_status blas_maxpy(wd_context ctx, const Geom& g, size_t nh, int prec, const void* V, size_t vstride, int k,
                     const double* coef, const void* w, double scale, void* out)
{
    return maxpy_any(ctx, g, nh, prec, V, vstride, k, coef, nullptr, 0.f, w, scale, out);
}

// Second Gram-Schmidt pass fused with the first pass's update: per site
//   w' = w - sum_i h1_i V_i   (h1 from dres[slot1 ..], written back to w)
//   partial <V_i, w'> for i < k and ||w'||^2, with V_i read once from HBM (the dots re-read
//   the site's V_i from cache right after the update).  Up to MGS_KMAX vectors; the norm
//   lands in value 2 MGS_KMAX.

template <int P>
__global__ void __launch_bounds__(RED_BLOCK) maxpy_mdot_kernel(SiteRange Vs, size_t vstride, int k, const double* h1,
                                                               SiteRange W, long long nsites, double* partials)
{
    using T = typename RealOf<P>::T;
    double acc[2 * MGS_KMAX + 1];
#pragma unroll
    for (int q = 0; q < 2 * MGS_KMAX + 1; ++q) acc[q] = 0.0;
    for (long long s = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; s < nsites; s += (long long)gridDim.x * RED_BLOCK) {
        const long long h = s / W.Vh;
        const uint32_t cb = (uint32_t)(s - h * W.Vh);
        T w[24];
        SpinorIO<P>::load(W.half(h), W.ps, cb, w);
        for (int i = 0; i < k; ++i) {
            T v[24];
            SpinorIO<P>::load(Vs.half(h) + (size_t)i * vstride, W.ps, cb, v);
            const T cr = (T)(-(float)h1[2 * i]), ci = (T)(-(float)h1[2 * i + 1]);
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                w[2 * q] += cr * v[2 * q] - ci * v[2 * q + 1];
                w[2 * q + 1] += cr * v[2 * q + 1] + ci * v[2 * q];
            }
        }
        SpinorIO<P>::store((char*)W.half(h), W.ps, cb, w);
#pragma unroll
        for (int i = 0; i < MGS_KMAX; ++i) {
            if (i < k) {
                T v[24];
                SpinorIO<P>::load(Vs.half(h) + (size_t)i * vstride, W.ps, cb, v);
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const double ar = v[2 * q], ai = v[2 * q + 1], br = w[2 * q], bi = w[2 * q + 1];
                    acc[2 * i] += ar * br + ai * bi;
                    acc[2 * i + 1] += ar * bi - ai * br;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 24; ++q) acc[2 * MGS_KMAX] += (double)w[q] * (double)w[q];
    }
    block_reduce<2 * MGS_KMAX + 1>(acc, partials);
}

wd_status blas_maxpy_mdot(wd_context ctx, const Geom& g, size_t nh, int prec, const void* V, size_t vstride, int k,
                          int slot1, void* w)
{
    if (k < 1 || k > MGS_KMAX || slot1 < 2 * MGS_KMAX + 1 || slot1 + 2 * k > 256) {
        set_error("maxpy_mdot: k = %d (slot %d) out of range", k, slot1);
        return WD_EINVAL;
    }
    const long long ns = (long long)nh * g.Vh;
    const int nblk = red_blocks(ns);
    WD_TRY(ensure_reduction(ctx, (size_t)nblk * (2 * MGS_KMAX + 1)));
    SiteRange Vs{(const char*)V, g.Vh, g.ps, half_bytes(g, prec)}, W{(const char*)w, g.Vh, g.ps, half_bytes(g, prec)};
    switch (prec) {
    case WD_F32: hipLaunchKernelGGL(maxpy_mdot_kernel<P_F32>, dim3(nblk), dim3(RED_BLOCK), 0, ctx->stream, Vs, vstride, k,
                                    (const double*)(ctx->dres + slot1), W, ns, ctx->partials); break;
    default: set_error("maxpy_mdot: precision %d not supported (F32 only)", prec); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return finish(ctx, nblk, 2 * MGS_KMAX + 1, true);
}

wd_status blas_maxpy_dev(wd_context ctx, const Geom& g, size_t nh, int prec, const void* V, size_t vstride, int k,
                         int slot, float sign, const void* w, double scale, void* out)
{
    if (slot < 0 || slot + 2 * k > 256) {
        set_error("maxpy: coefficient slot %d out of range", slot);
        return WD_EINVAL;
    }
    return maxpy_any(ctx, g, nh, prec, V, vstride, k, nullptr, ctx->dres + slot, sign, w, scale, out);
}

// ---- STREAM-style copy: the achievable HBM ceiling and the reference for
// the hardware byte counters ------------------------------------------------------
// Four 16-byte loads per work-item are issued before the four stores.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst, long long n)
{
    const long long stride = (long long)gridDim.x * 1024;
    for (long long base = (long long)blockIdx.x * 1024 + threadIdx.x; base < n; base += stride) {
        f32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (base + 256 * j < n) v[j] = __builtin_nontemporal_load(&src[base + 256 * j]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (base + 256 * j < n) __builtin_nontemporal_store(v[j], &dst[base + 256 * j]);
    }
}

wd_status launch_copy(wd_context ctx, const void* src, void* dst, size_t bytes)
{
    const long long n = (long long)(bytes / 16);
    long long blocks = (n + 1023) / 1024;
    if (blocks > 256 * 16) blocks = 256 * 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, (const f32x4*)src, (f32x4*)dst, n);
    WD_LAUNCHED();
    return WD_OK;
}

} // namespace wd

extern "C" wd_status wd_device_copy(wd_context ctx, const void* src, void* dst, size_t bytes)
{
    if (!ctx || !src || !dst || bytes % 16) {
        wd::set_error("wd_device_copy: NULL pointer or size not a multiple of 16");
        return WD_EINVAL;
    }
    return wd::launch_copy(ctx, src, dst, bytes);
}

// ---- the global sum <a, b> with no allocation anywhere ---------------------------------
// For callers that cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid it): the per-workgroup partial sums and the two final values
// live in a file-scope device array, one copy per GPU, held until the process ends.  Host
// code never passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in); it looks up each device's address once, with that device current, and passes
// that address.  Every call on one GPU shares its copy: calls that overlap in time on one GPU
// (two host threads, or two streams) race, and must be serialised by the caller.  Nothing
// needs clearing: every call writes all the partials it reads.
namespace wd {

constexpr int NOALLOC_SLOTS = 2 * RED_MAXBLOCKS + 2;   // two partial rows, then Re and Im
static __device__ __align__(256) double scratch[NOALLOC_SLOTS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mu;
static double* noalloc_ptr[NOALLOC_MAX_DEVICES];   // scratch's address on each device, once known

static wd_status noalloc_scratch(int device, double** out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        set_error("wd_dot_noalloc: device %d beyond the %d supported", device, NOALLOC_MAX_DEVICES);
        return WD_EINVAL;
    }
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[device]) {   // the current device is `device`
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("wd_dot_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                      hipGetErrorString(e));
            return WD_EHIP;
        }
        noalloc_ptr[device] = (double*)p;
    }
    *out = noalloc_ptr[device];
    return WD_OK;
}

template <int P>
static wd_status dot_noalloc_t(hipStream_t stream, const Geom& g, size_t nh, const void* a, const void* b,
                               double* dev_scratch)
{
    const long long n = (long long)nh * g.Vh;
    const int nblk = red_blocks(n);
    if (2 * nblk + 2 > NOALLOC_SLOTS) {   // red_blocks caps the grid, so this never fires
        set_error("wd_dot_noalloc: %d workgroups exceed the scratch array", nblk);
        return WD_EINVAL;
    }
    SiteRange A{(const char*)a, g.Vh, g.ps, half_bytes(g, P)}, B{(const char*)b, g.Vh, g.ps, half_bytes(g, P)};
    hipLaunchKernelGGL((dot_kernel<P, true>), dim3(nblk), dim3(RED_BLOCK), 0, stream, A, B, n, dev_scratch);
    WD_LAUNCHED();
    double* res = dev_scratch + 2 * RED_MAXBLOCKS;
    hipLaunchKernelGGL(finish_kernel, dim3(2), dim3(RED_BLOCK), 0, stream, dev_scratch, nblk, res, (double*)nullptr);
    WD_LAUNCHED();
    return WD_OK;
}

} // namespace wd

extern "C" wd_status wd_dot_noalloc(void* stream, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                                    const void* a, const void* b, double* result)
{
    using namespace wd;
    if (!a || !b || !result) {
        set_error("wd_dot_noalloc: NULL argument");
        return WD_EINVAL;
    }
    if (!valid_subset(subset) || !valid_prec(prec) || nrhs < 1 || nrhs > 65535) {
        set_error("wd_dot_noalloc: bad subset %d, precision %d or nrhs %d", (int)subset, (int)prec, nrhs);
        return WD_EINVAL;
    }
    Geom g;
    WD_TRY(make_geom(lat, &g));
    int device = 0;
    WD_HIP(hipGetDevice(&device));
    double* s = nullptr;
    WD_TRY(noalloc_scratch(device, &s));
    hipStream_t st = (hipStream_t)stream;
    const size_t nh = halves_of(subset, nrhs);
    switch (prec) {
    case WD_F64: WD_TRY(dot_noalloc_t<P_F64>(st, g, nh, a, b, s)); break;
    case WD_F32: WD_TRY(dot_noalloc_t<P_F32>(st, g, nh, a, b, s)); break;
    case WD_F16: WD_TRY(dot_noalloc_t<P_F16>(st, g, nh, a, b, s)); break;
    case WD_BF16: WD_TRY(dot_noalloc_t<P_BF16>(st, g, nh, a, b, s)); break;
    }
    WD_HIP(hipMemcpyAsync(result, s + 2 * RED_MAXBLOCKS, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    return WD_OK;
}
