// Even-odd hopping term for 16 right-hand sides at once with the colour multiply on
// the matrix cores (16-bit storage, 12-real links).
//
// For one direction of one site the colour multiply is W = U H with H the projected
// half spinors of all right-hand sides: a 3 x 3 complex matrix times 3 x (2 spin x
// 16 rhs) complex values.  In real form (rows (colour, re/im)) that is 6 x 6 times
// 6 x 32.  Two sites share one v_mfma_f32_16x16x16_f16 per spin component: the A
// operand holds diag(U_s0, U_s1) (rows and K = (site, colour, re/im), 12 of 16), the
// B operand the two sites' half spinors (K rows) for the 16 rhs (columns).
//
// A wave covers 8 sites x 16 rhs.  Per direction:
//   1. each lane loads two (neighbour site, rhs) spinors (coalesced per rhs plane),
//      decodes them to code units (|q| <= 1, the per-site scale kept apart), projects
//      to half spinors and writes them as fp16 into its wave's B tiles in LDS;
//   2. lanes 0..7 load the 8 links, rebuild row 2, fold in the boundary sign (and
//      the dagger of a backward hop) and write them to LDS; every lane gathers its
//      A-fragment entries from there;
//   3. 8 matrix-core products (4 site pairs x 2 spin components); each lane scales
//      its rows by the input site's scale and expands them to four spin components
//      into float32 accumulators that stay in the matrix-core layout.
// At the end the accumulators go through LDS so that each lane again owns whole
// (site, rhs) spinors, which are scaled (and combined with x) and re-encoded.
// Inputs to the products are fp16 in code units, so no value can overflow; results
// are accumulated in float32.
#include "dslash_body.h"

namespace wd {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float mr_f32x4 __attribute__((ext_vector_type(4)));

constexpr int MR_SITES = 8;    // sites per wave
constexpr int MR_RHS = 16;     // rhs per wave (matrix-core columns)
constexpr int MR_LD = 20;      // fp16 per staged column: 16 K values + 4 of padding
// per-wave LDS: B tiles (4 pairs x 2 spin components x 16 columns x MR_LD fp16), links
// (8 x 18 float), input scales (8 x 16 float); at the end reused for the output spinors
// (8 x 16 x 24 float)
constexpr int MR_B_BYTES = 8 * MR_RHS * MR_LD * 2;
constexpr int MR_L_BYTES = MR_SITES * 18 * 4;
constexpr int MR_S_BYTES = MR_SITES * MR_RHS * 4;
constexpr int MR_O_BYTES = MR_SITES * MR_RHS * 24 * 4;
constexpr int MR_WAVE_BYTES = MR_O_BYTES > MR_B_BYTES + MR_L_BYTES + MR_S_BYTES ? MR_O_BYTES
                                                                               : MR_B_BYTES + MR_L_BYTES + MR_S_BYTES;

__device__ __forceinline__ void mr_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw loads of one direction: two neighbour spinors (codes and scales) and, in lanes
// 0..7, the link.  Issued one direction ahead of the arithmetic.
struct MrRaw {
    uint4 q[2][3];
    float s[2];
    uint4 l0;
    uint2 l1;
};

// Per-lane A-fragment pattern, the same for every direction and pair: entry t of the
// fragment is sign[t] * Ls[pair * 36 + off[t]] (sign 0: a zero of the block diagonal).
struct MrAPattern {
    int off[4];
    float sign[4];
};

__device__ __forceinline__ MrAPattern mr_a_pattern(int lane)
{
    MrAPattern a;
    const int m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int kk = 4 * g + t;
        const bool ok = m < 12 && kk < 12 && m / 6 == kk / 6;
        const int row_site = m / 6, ca = (m % 6) >> 1, c1 = m & 1, cb_ = (kk % 6) >> 1, c2 = kk & 1;
        // [[Er, -Ei], [Ei, Er]]: the real part where c1 == c2, else the imaginary part
        a.off[t] = ok ? row_site * 18 + 2 * (3 * ca + cb_) + (c1 == c2 ? 0 : 1) : 0;
        a.sign[t] = ok ? ((c1 == 0 && c2 == 1) ? -1.f : 1.f) : 0.f;
    }
    return a;
}

template <int D, int P>
__device__ __forceinline__ void mr_load(const DslashArgs& A, const char* in0, uint32_t cb, const int c[4], int lane,
                                        MrRaw& x)
{
    constexpr int MU = D >> 1;
    constexpr bool FWD = (D & 1) == 0;
    const uint32_t nb = neighbour<MU, FWD>(A.g, cb, c);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r = (lane >> 3) + 8 * j;
        const uint4* pl = (const uint4*)(in0 + (size_t)r * A.in_stride);
#pragma unroll
        for (int k = 0; k < 3; ++k) x.q[j][k] = pl[(size_t)k * A.g.ps + nb];
        x.s[j] = ((const float*)(pl + (size_t)3 * A.g.ps))[nb];
    }
    if (lane < MR_SITES) {
        const int lpar = FWD ? A.par : 1 - A.par;
        const uint4* grp = (const uint4*)(A.gauge + (size_t)(2 * MU + lpar) * link_site_bytes(P, 12) * A.g.ps);
        const uint32_t lcb = FWD ? cb : nb;
        x.l0 = grp[lcb];
        x.l1 = ((const uint2*)(grp + (size_t)A.g.ps))[lcb];
    }
}

template <int D, int P, bool DAG>
__device__ __forceinline__ void mr_compute(const DslashArgs& A, const int c[4], int lane, char* lds, const MrRaw& x,
                                           const MrAPattern& ap, float (&acc)[4][4][4])
{
    constexpr int MU = D >> 1;
    constexpr bool FWD = (D & 1) == 0;
    constexpr int S = (FWD != DAG) ? -1 : 1;
    using PJ = Proj<MU, S>;
    _Float16* Bt = (_Float16*)lds;
    float* Ls = (float*)(lds + MR_B_BYTES);
    float* Sc = (float*)(lds + MR_B_BYTES + MR_L_BYTES);
    const int sl = lane & 7;
    // 1. half spinors in code units -> fp16 B tiles; scales aside
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r = (lane >> 3) + 8 * j;
        float psi[24], h[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) unpack8<P>(x.q[j][k], 1.0f, psi + 8 * k);
        project<MU, S>(psi, h);
        const int p = sl >> 1, q = sl & 1;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            uint32_t* dst = (uint32_t*)(Bt + ((p * 2 + sp) * MR_RHS + r) * MR_LD + q * 6);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                typedef _Float16 h2 __attribute__((ext_vector_type(2)));
                const h2 v = {(_Float16)h[6 * sp + 2 * k], (_Float16)h[6 * sp + 2 * k + 1]};
                dst[k] = __builtin_bit_cast(uint32_t, v);
            }
        }
        Sc[sl * MR_RHS + r] = x.s[j];
    }
    // 2. links as E = U (forward) or U^dagger (backward), with the boundary sign
    if (lane < MR_SITES) {
        float u[18];
        unpack8<P>(x.l0, 1.0f, u);
        u[8] = h2f<P>(x.l1.x); u[9] = h2f<P>(x.l1.x >> 16);
        u[10] = h2f<P>(x.l1.y); u[11] = h2f<P>(x.l1.y >> 16);
        reconstruct_row2(u);
        const float sg = on_boundary<MU, FWD>(A.g, c) ? A.g.bcf[MU] : 1.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int e = FWD ? 3 * a + b : 3 * b + a;
                Ls[lane * 18 + 2 * (3 * a + b)] = sg * u[2 * e];
                Ls[lane * 18 + 2 * (3 * a + b) + 1] = FWD ? sg * u[2 * e + 1] : -sg * u[2 * e + 1];
            }
    }
    mr_wave_sync();
    // 3. products and spin expansion
    const int g = lane >> 4, n = lane & 15;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        half4_t af;
#pragma unroll
        for (int t = 0; t < 4; ++t) af[t] = (_Float16)(ap.sign[t] * Ls[p * 36 + ap.off[t]]);
        mr_f32x4 d[2];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const half4_t bf = *(const half4_t*)(Bt + ((p * 2 + sp) * MR_RHS + n) * MR_LD + 4 * g);
            d[sp] = __builtin_amdgcn_mfma_f32_16x16x16f16(af, bf, mr_f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
        if (g < 3)   // D rows 12..15 (g = 3) are the zero padding
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int row = 4 * g + 2 * z;
            const int rs = row < 6 ? 0 : 1;               // site of the row within the pair
            const float sc = Sc[(2 * p + rs) * MR_RHS + n];
            const float w0r = d[0][2 * z] * sc, w0i = d[0][2 * z + 1] * sc;
            const float w1r = d[1][2 * z] * sc, w1i = d[1][2 * z + 1] * sc;
            acc[p][0][2 * z] += w0r;
            acc[p][0][2 * z + 1] += w0i;
            acc[p][1][2 * z] += w1r;
            acc[p][1][2 * z + 1] += w1i;
            const float ar = PJ::J2 == 0 ? w0r : w1r, ai = PJ::J2 == 0 ? w0i : w1i;
            const float br = PJ::J3 == 0 ? w0r : w1r, bi = PJ::J3 == 0 ? w0i : w1i;
            acc[p][2][2 * z] += umul_re<PJ::C2>(ar, ai);
            acc[p][2][2 * z + 1] += umul_im<PJ::C2>(ar, ai);
            acc[p][3][2 * z] += umul_re<PJ::C3>(br, bi);
            acc[p][3][2 * z + 1] += umul_im<PJ::C3>(br, bi);
        }
    }
    mr_wave_sync();
}

// directions D..7, each one's loads issued before the previous one's arithmetic
template <int D, int P, bool DAG>
__device__ __forceinline__ void mr_pipe(const DslashArgs& A, const char* in0, uint32_t cb, const int c[4], int lane,
                                        char* lds, const MrAPattern& ap, float (&acc)[4][4][4], MrRaw& cur, MrRaw& nxt)
{
    // compiler barrier: the loads of direction D + 1 may not move above the arithmetic of D - 1
    asm volatile("" ::: "memory");
    if constexpr (D < 7) mr_load<D + 1, P>(A, in0, cb, c, lane, nxt);
    mr_compute<D, P, DAG>(A, c, lane, lds, cur, ap, acc);
    if constexpr (D < 7) mr_pipe<D + 1, P, DAG>(A, in0, cb, c, lane, lds, ap, acc, nxt, cur);
}

template <int P, bool DAG, bool XPAY>
__global__ void __launch_bounds__(256, 2) dslash_mrhs_kernel(DslashArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds_all[4][MR_WAVE_BYTES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    char* lds = lds_all[wave];
    const uint32_t Vh = (uint32_t)A.g.Vh;
    const uint32_t cb0 = (xcd_remap(blockIdx.x, gridDim.x) * 4 + wave) * MR_SITES;
    const int sl = lane & 7;
    const bool valid = cb0 + sl < Vh;
    const uint32_t cb = valid ? cb0 + sl : 0;   // sites past the end work on site 0, store nothing
    int c[4];
    cb_coords(A.g, cb, A.par, c);
    const int r0 = blockIdx.y * MR_RHS;
    const char* in0 = A.in + (size_t)r0 * A.in_stride;
    // zero K rows 12..15 of every B column once; the products never write them
    {
        _Float16* Bt = (_Float16*)lds;
        for (int i = lane; i < 8 * MR_RHS; i += 64) {
            uint32_t* col = (uint32_t*)(Bt + i * MR_LD + 12);
            col[0] = 0u;
            col[1] = 0u;
        }
    }
    float acc[4][4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[p][s][k] = 0.f;
    mr_wave_sync();
    const MrAPattern ap = mr_a_pattern(lane);
    MrRaw ra, rb;
    mr_load<0, P>(A, in0, cb, c, lane, ra);
    mr_pipe<0, P, DAG>(A, in0, cb, c, lane, lds, ap, acc, ra, rb);
    // accumulators -> [site][rhs][24] in LDS
    float* O = (float*)lds;
    const int g = lane >> 4, n = lane & 15;
    if (g < 3) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                const int row = 4 * g + 2 * z;                  // (site in pair, colour, re) row
                const int site = 2 * p + row / 6, a = (row % 6) >> 1;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    float* o = O + (site * MR_RHS + n) * 24 + (s * 3 + a) * 2;
                    o[0] = acc[p][s][2 * z];
                    o[1] = acc[p][s][2 * z + 1];
                }
            }
    }
    mr_wave_sync();
    if (!valid) return;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r = (lane >> 3) + 8 * j;
        const float* o = O + (sl * MR_RHS + r) * 24;
        float v[24];
        if constexpr (XPAY) {
            SpinorIO<P>::load(A.x + (size_t)(r0 + r) * A.x_stride, A.g.ps, cb, v);
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = (float)A.a * v[k] + (float)A.b * o[k];
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) v[k] = (float)A.b * o[k];
        }
        SpinorIO<P>::store(A.out + (size_t)(r0 + r) * A.out_stride, A.g.ps, cb, v);
    }
}

bool mrhs_eligible(const DslashCall& c)
{
    return (c.prec == WD_F16 || c.prec == WD_BF16) && c.recon == 12 && c.nrhs >= MR_RHS && c.nrhs % MR_RHS == 0;
}

wd_status launch_dslash_mrhs(wd_context ctx, const Geom& g, const DslashCall& c)
{
    if (!mrhs_eligible(c)) {
        set_error("dslash (matrix cores): needs 16-bit storage, 12-real links and a multiple of 16 rhs");
        return WD_EUNSUPPORTED;
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
    A.remap = 1;
    A.rhs_inner = 0;
    A.gf = 0;      // unit links are stored as exact identities: multiplying by them is exact
    A.zb = 0;
    const dim3 grid((unsigned)((g.Vh + 4 * MR_SITES - 1) / (4 * MR_SITES)), (unsigned)(c.nrhs / MR_RHS)), block(256);
    const int sel = (c.prec == WD_BF16 ? 4 : 0) | (c.dagger ? 1 : 0) | (c.x ? 2 : 0);
    switch (sel) {
#define WD_MR(K, PP)                                                                                                \
    case K: hipLaunchKernelGGL((dslash_mrhs_kernel<PP, (K & 1) != 0, (K & 2) != 0>), grid, block, 0, ctx->stream, A); \
        break;
        WD_MR(0, P_F16) WD_MR(1, P_F16) WD_MR(2, P_F16) WD_MR(3, P_F16)
        WD_MR(4, P_BF16) WD_MR(5, P_BF16) WD_MR(6, P_BF16) WD_MR(7, P_BF16)
#undef WD_MR
    }
    WD_LAUNCHED();
    return WD_OK;
}

} // namespace wd
