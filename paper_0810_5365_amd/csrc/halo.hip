// One device's share of a lattice split into slabs along t (the multi-device
// layout of the hopping term; the exchange between devices is the caller's).
//
// A slab holds T_local time slices of the global lattice with its own links
// U_mu(x).  The hopping term needs, across each slab face, one spin-projected
// half spinor (12 reals) per face site instead of the full 24 (paper Section 4:
// the projection before the colour multiply):
//   - the forward t-hop of the last slice reads psi(x + t) from the next slab:
//     that slab sends (1 - s gamma_t) psi of its first slice (s = +1 for D,
//     -1 for D^dagger), and the receiver multiplies by its own U_t(x);
//   - the backward t-hop of the first slice needs U_t(x - t)^dagger, a link of
//     the previous slab: that slab sends U_t^dagger (1 + s gamma_t) psi of its
//     last slice, already multiplied, so no link crosses a face.
// The boundary condition enters as a sign on the received half spinors where
// the hop crosses the global t edge.  Spatial hops wrap inside the slab.
#include "dslash_body.h"

namespace wd {

// Face half spinors: 12 reals per site in 16-byte planes of `fs` sites
// (3 float4 planes in F32, 6 double2 planes in F64).
template <typename T> struct FaceIO;
template <> struct FaceIO<float> {
    __device__ __forceinline__ static void load(const char* base, int fs, uint32_t s, float* h)
    {
        const float4* p = (const float4*)base;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 q = p[(size_t)k * fs + s];
            h[4 * k] = q.x; h[4 * k + 1] = q.y; h[4 * k + 2] = q.z; h[4 * k + 3] = q.w;
        }
    }
    __device__ __forceinline__ static void store(char* base, int fs, uint32_t s, const float* h)
    {
        float4* p = (float4*)base;
#pragma unroll
        for (int k = 0; k < 3; ++k) p[(size_t)k * fs + s] = make_float4(h[4 * k], h[4 * k + 1], h[4 * k + 2], h[4 * k + 3]);
    }
};
template <> struct FaceIO<double> {
    __device__ __forceinline__ static void load(const char* base, int fs, uint32_t s, double* h)
    {
        const double2* p = (const double2*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 q = p[(size_t)k * fs + s];
            h[2 * k] = q.x; h[2 * k + 1] = q.y;
        }
    }
    __device__ __forceinline__ static void store(char* base, int fs, uint32_t s, const double* h)
    {
        double2* p = (double2*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[(size_t)k * fs + s] = make_double2(h[2 * k], h[2 * k + 1]);
    }
};

struct HaloArgs {
    DslashArgs d;          // gauge, in, out, geometry, parity (of the output, or of the packed input)
    const char* ghost_f;   // received for the forward t-hops of the last slice
    const char* ghost_b;   // received for the backward t-hops of the first slice
    char* face_f;          // packed: first slice, for the previous slab
    char* face_b;          // packed: last slice, for the next slab
    int fs;                // sites per parity in one time slice: X Y Z / 2
    double sign_f, sign_b;
};

// Pack both faces of the input half field (parity A.d.par): y = 0 the first slice,
// y = 1 the last.  The projection signs are those of the receiver's hops.
template <int P, int R, bool DAG>
__global__ void __launch_bounds__(256) halo_pack_kernel(HaloArgs H)
{
    using T = typename RealOf<P>::T;
    const DslashArgs& A = H.d;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (uint32_t)H.fs) return;
    const bool last = blockIdx.y == 1;
    const uint32_t cb = s + (last ? (uint32_t)(A.g.L[3] - 1) * (uint32_t)H.fs : 0u);
    T psi[24], h[12];
    SpinorIO<P>::load(A.in, A.g.ps, cb, psi);
    if (!last) {
        project<3, DAG ? 1 : -1>(psi, h);   // the receiver's forward hop
        FaceIO<T>::store(H.face_f, H.fs, s, h);
    } else {
        project<3, DAG ? -1 : 1>(psi, h);   // the receiver's backward hop
        T u[18], w[12];
        const size_t gbytes = link_site_bytes(P, R) * (size_t)A.g.ps;
        LinkIO<P, R, true>::load(A.gauge + (size_t)(2 * 3 + A.par) * gbytes, A.g.ps, cb, u);
        su3_mul<true>(u, h, w);
        FaceIO<T>::store(H.face_b, H.fs, s, w);
    }
}

// The hopping term on one parity of the slab, t-hops across the faces from the ghosts.
template <int P, int R, bool DAG>
__global__ void __launch_bounds__(256) dslash_halo_kernel(HaloArgs H)
{
    using T = typename RealOf<P>::T;
    const DslashArgs& A = H.d;
    const uint32_t bid = A.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t cb = bid * blockDim.x + threadIdx.x;
    if (cb >= (uint32_t)A.g.Vh) return;
    int c[4];
    cb_coords(A.g, cb, A.par, c);
    const size_t gbytes = link_site_bytes(P, R) * (size_t)A.g.ps;
    T acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    {   // the six spatial directions, each one's loads issued before the previous one's arithmetic
        T ua[18], pa[24], ub[18], pb[24];
        hop_load<0, P, R, true>(A, cb, c, A.in, gbytes, ua, pa);
        hop_pipelined<0, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<1, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc, ub, pb, ua, pa);
        hop_pipelined<2, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc, ua, pa, ub, pb);
        hop_pipelined<3, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc, ub, pb, ua, pa);
        hop_pipelined<4, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc, ua, pa, ub, pb);
        hop_compute<5, DAG>(A, c, ub, pb, acc);
        order_fence(acc);
    }
    const int T_l = A.g.L[3];
    if (c[3] == T_l - 1) {   // forward t-hop from the next slab: U_t(x) (s_f h)
        constexpr int S = DAG ? 1 : -1;
        T h[12], u[18], w[12];
        FaceIO<T>::load(H.ghost_f, H.fs, cb - (uint32_t)(T_l - 1) * (uint32_t)H.fs, h);
        const T sg = (T)H.sign_f;
#pragma unroll
        for (int k = 0; k < 12; ++k) h[k] *= sg;
        LinkIO<P, R, true>::load(A.gauge + (size_t)(2 * 3 + A.par) * gbytes, A.g.ps, cb, u);
        su3_mul<false>(u, h, w);
        accumulate<3, S>(acc, w);
        order_fence(acc);
    } else {
        hop<6, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc);
    }
    if (c[3] == 0) {   // backward t-hop from the previous slab: s_b U_t(x - t)^dagger h, multiplied there
        constexpr int S = DAG ? -1 : 1;
        T w[12];
        FaceIO<T>::load(H.ghost_b, H.fs, cb, w);
        const T sg = (T)H.sign_b;
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] *= sg;
        accumulate<3, S>(acc, w);
    } else {
        hop<7, P, R, DAG, true>(A, cb, c, A.in, gbytes, acc);
    }
    SpinorIO<P>::store(A.out, A.g.ps, cb, acc);
}

static wd_status halo_common(wd_gauge g, int subset, int prec, const void* in, const void* a, const void* b,
                             HaloArgs* H)
{
    if (!g || !in || !a || !b) {
        set_error("NULL gauge or field pointer");
        return WD_EINVAL;
    }
    if (subset != WD_EVEN && subset != WD_ODD) {
        set_error("slab faces: subset must be EVEN or ODD (got %d)", subset);
        return WD_EINVAL;
    }
    if (prec != WD_F32 && prec != WD_F64) {
        set_error("slab faces: precision %d not supported (F32 or F64)", prec);
        return WD_EUNSUPPORTED;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    if (g->gf) {
        set_error("slab faces: the links are in temporal gauge (a per-slab gauge fixing is not supported)");
        return WD_EUNSUPPORTED;
    }
    const void* links = nullptr;
    WD_TRY(gauge_links(g, prec, &links));
    *H = HaloArgs{};
    H->d.gauge = (const char*)links;
    H->d.in = (const char*)in;
    H->d.g = g->geom;
    H->d.par = subset == WD_EVEN ? 0 : 1;
    H->fs = g->geom.L[0] * g->geom.L[1] * g->geom.L[2] / 2;
    return WD_OK;
}

template <int P>
static wd_status launch_pack(wd_context ctx, const HaloArgs& H, int recon, int dagger)
{
    const dim3 grid((H.fs + 255) / 256, 2), block(256);
    const int sel = (recon == 12 ? 1 : 0) | (dagger ? 2 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((halo_pack_kernel<P, 18, false>), grid, block, 0, ctx->stream, H); break;
    case 1: hipLaunchKernelGGL((halo_pack_kernel<P, 12, false>), grid, block, 0, ctx->stream, H); break;
    case 2: hipLaunchKernelGGL((halo_pack_kernel<P, 18, true>), grid, block, 0, ctx->stream, H); break;
    default: hipLaunchKernelGGL((halo_pack_kernel<P, 12, true>), grid, block, 0, ctx->stream, H); break;
    }
    WD_LAUNCHED();
    return WD_OK;
}

// Workgroup size and block order: those tuned for the ordinary dslash on this slab
// (the same loads but for the faces), else the untuned default.
template <int P>
static wd_status launch_halo(wd_context ctx, const HaloArgs& H, int recon, int dagger, int block_size)
{
    const dim3 grid((H.d.g.Vh + block_size - 1) / block_size), block(block_size);
    const int sel = (recon == 12 ? 1 : 0) | (dagger ? 2 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((dslash_halo_kernel<P, 18, false>), grid, block, 0, ctx->stream, H); break;
    case 1: hipLaunchKernelGGL((dslash_halo_kernel<P, 12, false>), grid, block, 0, ctx->stream, H); break;
    case 2: hipLaunchKernelGGL((dslash_halo_kernel<P, 18, true>), grid, block, 0, ctx->stream, H); break;
    default: hipLaunchKernelGGL((dslash_halo_kernel<P, 12, true>), grid, block, 0, ctx->stream, H); break;
    }
    WD_LAUNCHED();
    return WD_OK;
}

} // namespace wd

using namespace wd;

extern "C" {

size_t wd_face_bytes(const wd_lattice* lat, wd_prec prec)
{
    Geom g;
    if (!lat || (prec != WD_F32 && prec != WD_F64) || make_geom(lat, &g) != WD_OK) return 0;
    return (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] / 2 * (prec == WD_F64 ? 96 : 48);
}

wd_status wd_halo_pack(wd_gauge g, wd_subset in_subset, int dagger, wd_prec prec, const void* in, void* face_fwd,
                       void* face_bwd)
{
    HaloArgs H;
    WD_TRY(halo_common(g, in_subset, prec, in, face_fwd, face_bwd, &H));
    H.face_f = (char*)face_fwd;
    H.face_b = (char*)face_bwd;
    return prec == WD_F64 ? launch_pack<P_F64>(g->ctx, H, g->recon, dagger) : launch_pack<P_F32>(g->ctx, H, g->recon, dagger);
}

wd_status wd_dslash_halo(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, const void* in,
                         const void* ghost_fwd, const void* ghost_bwd, double sign_fwd, double sign_bwd, void* out)
{
    HaloArgs H;
    WD_TRY(halo_common(g, out_subset, prec, in, ghost_fwd, ghost_bwd, &H));
    if (!out || out == in) {
        set_error("wd_dslash_halo: out is NULL or aliases in");
        return WD_EINVAL;
    }
    H.d.out = (char*)out;
    H.ghost_f = (const char*)ghost_fwd;
    H.ghost_b = (const char*)ghost_bwd;
    H.sign_f = sign_fwd;
    H.sign_b = sign_bwd;
    const Geom& G = g->geom;
    char key[160];
    snprintf(key, sizeof key, "dslash:%dx%dx%dx%d:p%d:r%d:n1:d%d:x0", G.L[0], G.L[1], G.L[2], G.L[3], (int)prec,
             g->recon, dagger != 0);
    const TuneParam tp = tune_lookup(g->ctx, key);
    H.d.remap = tp.remap;
    const int bs = (tp.block >= 64 && tp.block <= 256 && tp.block % 64 == 0) ? tp.block : 128;
    return prec == WD_F64 ? launch_halo<P_F64>(g->ctx, H, g->recon, dagger, bs)
                          : launch_halo<P_F32>(g->ctx, H, g->recon, dagger, bs);
}

} // extern "C"
