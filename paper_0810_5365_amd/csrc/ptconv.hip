// Parallel-transport convolution: the gauge-equivariant layer of the learned
// preconditioner.  A feature field holds C colour triplets per site; a layer
// maps C_in channels to C_out channels with nine paths p (stay, +mu, -mu):
//
//     psi^a(x) = sum_p sum_b W[p, a, b] (T_p phi^b)(x),
//     T_0 phi = phi,  T_{+mu} phi(x) = U_mu(x) s+ phi(x + mu),
//     T_{-mu} phi(x) = U_mu(x - mu)^dagger s- phi(x - mu),
//
// with the same links, boundary signs and even-odd site storage as the
// Wilson hopping term (one work-item per output site, links shared by all
// channels of a direction).  Gradients (PyTorch's convention for complex
// parameters, dL/dRe + i dL/dIm):
//     input:  gin^b = sum_p T_p^dagger sum_a conj(W[p, a, b]) gout^a
//             = the same layer with adjoint weights W'[p', b, a] = conj(W[p, a, b])
//               (p' swaps +mu and -mu), so it reuses the forward kernel;
//     weight: gW[p, a, b] = sum_x sum_c gout^a(x)_c conj((T_p phi^b)(x)_c), a lattice
//             reduction done per path with float64 partial sums.
//
// Packed feature layout (float32): sample n, channel c, parity par, colour k,
// site cb -> float2 at (((n C + c) 2 + par) 3 + k) Vh + cb (no plane padding: features are
// ordinary tensors that losses reduce over as a whole).
#include <stdlib.h>

#include "wd_core.h"

namespace wd {

struct PTArgs {
    const char* gauge;      // packed float32 links
    const float2* in;       // features (C_in channels)
    float2* out;            // features (C_out channels)
    const void* W;          // [9][C_out][C_in] complex at wprec
    Geom g;
    int cin;
    long long in_sample, out_sample;   // float2 elements between samples
    // Matrix-core path only (the vector path computes everything, which gives the same
    // result): input sites of parity zero_par (0 or 1; -1: none) are known to be zero, so
    // waves skip the paths that read only them; output sites [0, out_sites) are computed
    // (2 Vh: both parities; Vh: the even half).
    int zero_par = -1;
    int out_sites = 0;
    // Matrix-core path: zb > 0 walks the waves in z-blocks of that depth (all t for one block
    // of zb z-slices, then the next block), so the t - 1, t, t + 1 slices a wave reads are
    // close in time; needs X Y / 2 a multiple of 64 and zb dividing Z.
    int zb = 0;
    FastDiv dplane, dzb, dt;
    // Matrix-core path, 4 spin channels: spin_in reads the input's even sites straight from an
    // EVEN float32 spinor half field (its odd sites are zero: zero_par = 1), spin_out writes the
    // even output sites into one (even_out), in place of the feature tensors.
    const char* spin_in = nullptr;
    char* spin_out = nullptr;
};

// float2 index of (channel = spin b, colour k) of site cb in a float32 spinor half field:
// real (3 b + k) 2 of 24 sits in float4 plane (3 b + k) / 2, half (3 b + k) % 2.
__device__ __forceinline__ size_t spin_f2(int b, int k, int ps, uint32_t cb)
{
    const int r = 3 * b + k;
    return ((size_t)(r >> 1) * ps + cb) * 2 + (r & 1);
}

// First checkerboard site of the 64 consecutive sites i0 .. i0 + 63 of the z-blocked order
// i = r + (X/2) Y (zi + zb (t + T b)), z = b zb + zi (r < X Y / 2, a multiple of 64).
__device__ __forceinline__ uint32_t zb_first(const PTArgs& A, uint32_t i0)
{
    const uint32_t plane = (uint32_t)(A.g.Xh * A.g.L[1]);
    const uint32_t q = fdiv(i0, A.dplane), r = i0 - q * plane;
    const uint32_t q2 = fdiv(q, A.dzb), zi = q - q2 * (uint32_t)A.zb;
    const uint32_t b = fdiv(q2, A.dt), t = q2 - b * (uint32_t)A.g.L[3];
    return r + plane * (b * (uint32_t)A.zb + zi + (uint32_t)A.g.L[2] * t);
}

__device__ __forceinline__ size_t fidx(int c, int par, int k, int Vh, uint32_t cb)
{
    return ((size_t)(c * 2 + par) * 3 + k) * Vh + cb;
}

template <int WP> __device__ __forceinline__ float2 load_w(const void* W, int i)
{
    if constexpr (WP == P_F32) {
        return ((const float2*)W)[i];
    } else {
        const uint32_t q = ((const uint32_t*)W)[i];
        return make_float2(h2f<WP>(q), h2f<WP>(q >> 16));
    }
}

// w = U v or U^dagger v for a 3x3 complex U (row-major re, im pairs), as chains of
// fused multiply-adds.
template <typename T> __device__ __forceinline__ void mat_vec(const T* u, const T* v, T* w, bool dag)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = 0, im = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int e = dag ? (3 * b + a) : (3 * a + b);
            const T ur = u[2 * e], ui = dag ? -u[2 * e + 1] : u[2 * e + 1];
            re = fma(ur, v[2 * b], re);
            re = fma(-ui, v[2 * b + 1], re);
            im = fma(ur, v[2 * b + 1], im);
            im = fma(ui, v[2 * b], im);
        }
        w[2 * a] = re;
        w[2 * a + 1] = im;
    }
}

// Accumulate W[p] (T_p phi) over all input channels for one path.
template <int COUT, int WP>
__device__ __forceinline__ void mix_path(const PTArgs& A, int p, const float2* in, int par, uint32_t cb, const float* u,
                                         bool dag, float sign, bool transport, float* acc)
{
    const int Vh = A.g.Vh;
    for (int b = 0; b < A.cin; ++b) {
        float v[6], t[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 q = in[fidx(b, par, k, Vh, cb)];
            v[2 * k] = q.x;
            v[2 * k + 1] = q.y;
        }
        if (transport) {
            mat_vec(u, v, t, dag);
#pragma unroll
            for (int i = 0; i < 6; ++i) t[i] *= sign;
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) t[i] = v[i];
        }
#pragma unroll
        for (int a = 0; a < COUT; ++a) {
            const float2 w = load_w<WP>(A.W, (p * COUT + a) * A.cin + b);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc[6 * a + 2 * k] += w.x * t[2 * k] - w.y * t[2 * k + 1];
                acc[6 * a + 2 * k + 1] += w.x * t[2 * k + 1] + w.y * t[2 * k];
            }
        }
    }
}

template <int MU, bool FWD, int R, int COUT, int WP>
__device__ __forceinline__ void ptconv_dir(const PTArgs& A, const float2* in, int par, uint32_t cb, const int c[4],
                                           float* acc)
{
    const uint32_t nb = neighbour<MU, FWD>(A.g, cb, c);
    const int lpar = FWD ? par : 1 - par;
    const uint32_t lcb = FWD ? cb : nb;
    float u[18];
    LinkIO<P_F32, R, false>::load(A.gauge + (size_t)(2 * MU + lpar) * link_site_bytes(P_F32, R) * A.g.ps, A.g.ps, lcb, u);
    const float sign = on_boundary<MU, FWD>(A.g, c) ? A.g.bcf[MU] : 1.0f;
    mix_path<COUT, WP>(A, FWD ? 1 + MU : 5 + MU, in, 1 - par, nb, u, !FWD, sign, true, acc);
}

template <int R, int COUT, int WP>
__global__ void __launch_bounds__(256) ptconv_fwd_kernel(PTArgs A)
{
    // XCD-aware order: each XCD (own L2) walks one contiguous run of sites, so the neighbour
    // features and links a block reads were mostly fetched into the same L2 by its neighbours
    const uint32_t idx = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const uint32_t Vh = (uint32_t)A.g.Vh;
    if (idx >= 2 * Vh) return;
    const int par = idx >= Vh ? 1 : 0;
    const uint32_t cb = idx - (uint32_t)par * Vh;
    const float2* in = A.in + (size_t)blockIdx.y * A.in_sample;
    float2* out = A.out + (size_t)blockIdx.y * A.out_sample;
    int c[4];
    cb_coords(A.g, cb, par, c);
    float acc[6 * COUT];
#pragma unroll
    for (int i = 0; i < 6 * COUT; ++i) acc[i] = 0.f;
    mix_path<COUT, WP>(A, 0, in, par, cb, nullptr, false, 1.f, false, acc);
    ptconv_dir<0, true, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<1, true, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<2, true, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<3, true, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<0, false, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<1, false, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<2, false, R, COUT, WP>(A, in, par, cb, c, acc);
    ptconv_dir<3, false, R, COUT, WP>(A, in, par, cb, c, acc);
#pragma unroll
    for (int a = 0; a < COUT; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) out[fidx(a, par, k, A.g.Vh, cb)] = make_float2(acc[6 * a + 2 * k], acc[6 * a + 2 * k + 1]);
}

// W'[p'][b][a] = conj(W[p][a][b]) with p' = p for the stay path and +mu <-> -mu.
template <int WP>
__global__ void adjoint_weights_kernel(const void* W, void* Wt, int cin, int cout)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * cin * cout) return;
    const int p = i / (cin * cout);
    const int r = i - p * cin * cout;
    const int b = r / cout, a = r - b * cout;       // Wt index: [p'][b][a]
    const int pp = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
    const int src = (pp * cout + a) * cin + b;
    if constexpr (WP == P_F32) {
        const float2 w = ((const float2*)W)[src];
        ((float2*)Wt)[i] = make_float2(w.x, -w.y);
    } else {
        const uint32_t q = ((const uint32_t*)W)[src];
        ((uint32_t*)Wt)[i] = q ^ 0x80000000u;   // negate the imaginary half
    }
}

// gW partials: grid (nblk, 9 paths); each workgroup reduces its sites for every (b, a).
template <int R, int COUT>
__global__ void __launch_bounds__(256) ptconv_wgrad_kernel(PTArgs A, const float2* __restrict__ gout, int nsamples,
                                                           double* __restrict__ partials)
{
    const int p = blockIdx.y;
    const uint32_t Vh = (uint32_t)A.g.Vh;
    const long long nsites = 2ll * Vh * nsamples;
    __shared__ double lds[2 * COUT][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b = 0; b < A.cin; ++b) {
        double acc[2 * COUT];
#pragma unroll
        for (int i = 0; i < 2 * COUT; ++i) acc[i] = 0.0;
        for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < nsites; k += (long long)gridDim.x * 256) {
            const int n = (int)(k / (2 * Vh));
            const uint32_t idx = (uint32_t)(k - (long long)n * 2 * Vh);
            const int par = idx >= Vh ? 1 : 0;
            const uint32_t cb = idx - (uint32_t)par * Vh;
            const float2* in = A.in + (size_t)n * A.in_sample;
            const float2* go = gout + (size_t)n * A.out_sample;
            float t[6];
            if (p == 0) {
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    const float2 q = in[fidx(b, par, kk, Vh, cb)];
                    t[2 * kk] = q.x;
                    t[2 * kk + 1] = q.y;
                }
            } else {
                int c[4];
                cb_coords(A.g, cb, par, c);
                const int mu = (p - 1) & 3;
                const bool fwd = p <= 4;
                uint32_t nb;
                bool edge;
                switch (mu * 2 + (fwd ? 0 : 1)) {
                case 0: nb = neighbour<0, true>(A.g, cb, c); edge = on_boundary<0, true>(A.g, c); break;
                case 1: nb = neighbour<0, false>(A.g, cb, c); edge = on_boundary<0, false>(A.g, c); break;
                case 2: nb = neighbour<1, true>(A.g, cb, c); edge = on_boundary<1, true>(A.g, c); break;
                case 3: nb = neighbour<1, false>(A.g, cb, c); edge = on_boundary<1, false>(A.g, c); break;
                case 4: nb = neighbour<2, true>(A.g, cb, c); edge = on_boundary<2, true>(A.g, c); break;
                case 5: nb = neighbour<2, false>(A.g, cb, c); edge = on_boundary<2, false>(A.g, c); break;
                case 6: nb = neighbour<3, true>(A.g, cb, c); edge = on_boundary<3, true>(A.g, c); break;
                default: nb = neighbour<3, false>(A.g, cb, c); edge = on_boundary<3, false>(A.g, c); break;
                }
                const int lpar = fwd ? par : 1 - par;
                const uint32_t lcb = fwd ? cb : nb;
                float u[18], v[6];
                LinkIO<P_F32, R, false>::load(A.gauge + (size_t)(2 * mu + lpar) * link_site_bytes(P_F32, R) * A.g.ps, A.g.ps, lcb, u);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    const float2 q = in[fidx(b, 1 - par, kk, Vh, nb)];
                    v[2 * kk] = q.x;
                    v[2 * kk + 1] = q.y;
                }
                mat_vec(u, v, t, !fwd);
                const float s = edge ? A.g.bcf[mu] : 1.0f;
#pragma unroll
                for (int i = 0; i < 6; ++i) t[i] *= s;
            }
#pragma unroll
            for (int a = 0; a < COUT; ++a) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    const float2 gq = go[fidx(a, par, kk, Vh, cb)];
                    // g * conj(t)
                    re += gq.x * t[2 * kk] + gq.y * t[2 * kk + 1];
                    im += gq.y * t[2 * kk] - gq.x * t[2 * kk + 1];
                }
                acc[2 * a] += re;
                acc[2 * a + 1] += im;
            }
        }
        // workgroup reduction of the 2 COUT values
#pragma unroll
        for (int i = 0; i < 2 * COUT; ++i) {
            double s = acc[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            if (lane == 0) lds[i][wave] = s;
        }
        __syncthreads();
        if (threadIdx.x < 2 * COUT) {
            const double s = lds[threadIdx.x][0] + lds[threadIdx.x][1] + lds[threadIdx.x][2] + lds[threadIdx.x][3];
            // partials[((p * cin + b) * 2 COUT + i) * nblk + block]
            partials[((size_t)(p * A.cin + b) * 2 * COUT + threadIdx.x) * gridDim.x + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// gW[p][a][b] (float32 complex) from the partials, in a fixed order.
__global__ void wgrad_finish_kernel(const double* __restrict__ partials, int nblk, int cin, int cout, float2* __restrict__ gW)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // over (p, b, a)
    if (i >= 9 * cin * cout) return;
    const int p = i / (cin * cout);
    const int r = i - p * cin * cout;
    const int b = r / cout, a = r - b * cout;
    double re = 0.0, im = 0.0;
    const double* pr = partials + ((size_t)(p * cin + b) * 2 * cout + 2 * a) * nblk;
    const double* pi = pr + nblk;
    for (int k = 0; k < nblk; ++k) {
        re += pr[k];
        im += pi[k];
    }
    gW[(p * cout + a) * cin + b] = make_float2((float)re, (float)im);
}

// ---- spinor (float32 packed) <-> 4-channel features ----------------------------
// even_only: the spinor is one EVEN half field; odd sites read as zero and are not written.
__global__ void spinor_features_kernel(const char* spinor, float2* feat, int Vh, int ps, int nsamples, bool to_features,
                                       bool even_only)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2ll * Vh * nsamples) return;
    const int n = (int)(k / (2ll * Vh));
    const uint32_t idx = (uint32_t)(k - (long long)n * 2 * Vh);
    const int par = idx >= (uint32_t)Vh ? 1 : 0;
    const uint32_t cb = idx - (uint32_t)par * Vh;
    const size_t hb = spinor_site_bytes(P_F32) * (size_t)ps;
    char* sp = (char*)spinor + (even_only ? (size_t)n * hb : ((size_t)n * 2 + par) * hb);
    float2* f = feat + (size_t)n * 4 * 2 * 3 * Vh;
    float v[24];
    if (to_features) {
        if (even_only && par == 1) {
#pragma unroll
            for (int i = 0; i < 24; ++i) v[i] = 0.f;
        } else {
            SpinorIO<P_F32>::load(sp, ps, cb, v);
        }
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) f[fidx(s, par, c, Vh, cb)] = make_float2(v[(s * 3 + c) * 2], v[(s * 3 + c) * 2 + 1]);
    } else {
        if (even_only && par == 1) return;
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) {
                const float2 q = f[fidx(s, par, c, Vh, cb)];
                v[(s * 3 + c) * 2] = q.x;
                v[(s * 3 + c) * 2 + 1] = q.y;
            }
        SpinorIO<P_F32>::store(sp, ps, cb, v);
    }
}

// ---- canonical <-> packed features ----------------------------------------------------
// canonical: [n][C][T][Z][Y][X][3] complex128
__global__ void feature_pack_kernel(double* canon, float2* feat, Geom g, int C, long long total, bool unpack)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;   // k over (n, c, lex)
    const long long V = 2ll * g.Vh;
    const long long nc = k / V;
    const long long lex = k - nc * V;
    long long r = lex;
    const int x = (int)(r % g.L[0]); r /= g.L[0];
    const int y = (int)(r % g.L[1]); r /= g.L[1];
    const int z = (int)(r % g.L[2]); r /= g.L[2];
    const int t = (int)r;
    const int par = (x + y + z + t) & 1;
    const uint32_t cb = (uint32_t)(lex >> 1);
    const int c = (int)(nc % C);
    const long long n = nc / C;
    float2* f = feat + (size_t)n * C * 2 * 3 * g.Vh;
    double* cp = canon + 6 * k;
    for (int kk = 0; kk < 3; ++kk) {
        if (unpack) {
            const float2 q = f[fidx(c, par, kk, g.Vh, cb)];
            cp[2 * kk] = q.x;
            cp[2 * kk + 1] = q.y;
        } else {
            f[fidx(c, par, kk, g.Vh, cb)] = make_float2((float)cp[2 * kk], (float)cp[2 * kk + 1]);
        }
    }
}

// ---- channel mixing on matrix cores ------------------------------------------------
// For bf16 weights and C_in, C_out in {4, 8} the mixing sum_p sum_b W[p, a, b] (T_p phi^b)
// is a real GEMM per path: rows (a, re/im) (M = 2 C_out <= 16), K = (b, re/im)
// (2 C_in <= 16), columns (colour, site) (N = 3 x 64 per wave).  The transports run on
// the vector units, one site per lane, and are staged through LDS as bf16 in the
// B-operand layout; v_mfma_f32_16x16x16bf16 accumulates the nine paths in float32.
// Operand layout of the 16x16x16 instruction: lane l holds A[l % 16][4 (l / 16) + q],
// B[4 (l / 16) + q][l % 16] and D[4 (l / 16) + q][l % 16] for q = 0..3.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two floats -> packed bf16 pair, round to nearest even, in one conversion instruction.
__device__ __forceinline__ uint32_t cvt_bf16x2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}
constexpr int MF_LD = 20;   // bf16 per staged column: 16 K values + 4 of padding (40 B, conflict-free reads)

// Each wave stages its operands in its own LDS region, so the lanes of one wave only have
// to agree with each other: a wavefront-scope fence and wave barrier, no workgroup barrier.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One path in two halves so that the loads of path p + 1 are in flight while path p is
// transported, staged and multiplied (the layer is latency-bound on small lattices:
// one wave per 64 sites walks all nine paths).
// L16: the links are read as float16 codes (12 reals: 8 + 4 codes, 24 B instead of 48 B).
template <int R, int CIN, bool L16 = false> struct MfRaw {
    float4 l[L16 ? 1 : (R == 12 ? 3 : 4)];   // link planes as loaded (row 2 rebuilt later for 12 reals)
    float2 l18;                              // last two reals of an 18-real link
    uint4 h8;                                // L16: codes of reals 0..7
    uint2 h4;                                // L16: codes of reals 8..11
    float2 v[CIN][3];                        // neighbour features, channel b, colour k
    uint4 hv[6];                             // bf16 features as loaded (see hf_plane), decoded at use
};

// bf16 hidden features (8 channels): per parity six planes of 16 bytes per site, four complex
// numbers (bf16 pairs) each, in the order colour-major, channel-minor: complex (b, k) is word
// b % 4 of plane 2 k + b / 4.  A lane loads its site's 24 complexes in six 16-byte loads, and an
// accumulator tile's two channels of one colour are one 8-byte store.
__device__ __forceinline__ size_t hf_plane(int par, int pl, int Vh, uint32_t cb)
{
    return (size_t)(par * 6 + pl) * Vh + cb;
}

// bf16 feature pair (re in the low half, as cvt_bf16x2 packs it) -> float2
__device__ __forceinline__ float2 bf16x2_to_f2(uint32_t h)
{
    return make_float2(__uint_as_float(h << 16), __uint_as_float(h & 0xffff0000u));
}

// HF: the feature tensors (input and output, where not a spinor) hold bf16 pairs in the
// 16-byte planes of hf_plane
template <int PATH, int R, int CIN, bool SIN, bool HF, bool L16>
__device__ __forceinline__ void mf_load(const PTArgs& A, const float2* in, int par, uint32_t cb, const int c[4],
                                        MfRaw<R, CIN, L16>& x)
{
    const int Vh = A.g.Vh;
    uint32_t src = cb;
    int spar = par;
    if constexpr (PATH > 0) {
        constexpr int MU = (PATH - 1) & 3;
        constexpr bool FWD = PATH <= 4;
        const uint32_t nb = neighbour<MU, FWD>(A.g, cb, c);
        const int lpar = FWD ? par : 1 - par;
        const uint32_t ls = FWD ? cb : nb;
        if constexpr (L16) {   // the 16-bit 12-real layout: a plane of uint4, then a plane of uint2
            static_assert(R == 12, "16-bit links are read in the 12-real layout only");
            const uint4* grp = (const uint4*)(A.gauge + (size_t)(2 * MU + lpar) * link_site_bytes(P_F16, 12) * A.g.ps);
            x.h8 = grp[ls];
            x.h4 = ((const uint2*)(grp + (size_t)A.g.ps))[ls];
        } else {
            const float4* grp =
                (const float4*)(A.gauge + (size_t)(2 * MU + lpar) * link_site_bytes(P_F32, R) * A.g.ps) + ls;
#pragma unroll
            for (int k = 0; k < (R == 12 ? 3 : 4); ++k) x.l[k] = grp[(size_t)k * A.g.ps];
            if constexpr (R == 18) x.l18 = ((const float2*)(grp - ls + (size_t)4 * A.g.ps))[ls];
        }
        src = nb;
        spar = 1 - par;
    }
    if constexpr (SIN) {   // only even sources are ever loaded (the odd ones are skipped as zero)
        const float2* sp = (const float2*)A.spin_in;
#pragma unroll
        for (int b = 0; b < CIN; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) x.v[b][k] = sp[spin_f2(b, k, A.g.ps, src)];
    } else if constexpr (HF) {
        static_assert(CIN == 8, "bf16 hidden features have 8 channels");
        const uint4* hp = (const uint4*)in;
#pragma unroll
        for (int pl = 0; pl < 6; ++pl) x.hv[pl] = hp[hf_plane(spar, pl, Vh, src)];
    } else {
        // per-lane site offset once; the channel-plane offsets (b 6 + k) Vh are wave-uniform
        const float2* site = in + (size_t)spar * 3 * Vh + src;
#pragma unroll
        for (int b = 0; b < CIN; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) x.v[b][k] = site[(size_t)(b * 6 + k) * Vh];
    }
}

// HIN: the neighbour features arrived as bf16 planes (x.hv), else as float2 (x.v)
template <int PATH, int R, int CIN, bool L16, bool HIN>
__device__ __forceinline__ void mf_compute(const PTArgs& A, const int c[4], int lane, uint16_t* B,
                                           const MfRaw<R, CIN, L16>& x, const bf16x4& Af, f32x4* acc)
{
    float u[18];
    if constexpr (PATH > 0) {
        constexpr int MU = (PATH - 1) & 3;
        constexpr bool FWD = PATH <= 4;
        if constexpr (L16) {
            const uint32_t h[6] = {x.h8.x, x.h8.y, x.h8.z, x.h8.w, x.h4.x, x.h4.y};
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                u[2 * k] = h2f<P_F16>(h[k]);
                u[2 * k + 1] = h2f<P_F16>(h[k] >> 16);
            }
        } else {
#pragma unroll
            for (int k = 0; k < (R == 12 ? 3 : 4); ++k) {
                u[4 * k] = x.l[k].x; u[4 * k + 1] = x.l[k].y; u[4 * k + 2] = x.l[k].z; u[4 * k + 3] = x.l[k].w;
            }
        }
        if constexpr (R == 18) {
            u[16] = x.l18.x;
            u[17] = x.l18.y;
        } else {
            reconstruct_row2(u);
        }
        // boundary sign folded into the (reconstructed) link: 18 products instead of 6 C_in (a
        // branch that skips them where the sign is +1 measured 0.6% slower at 32^3 x 64)
        const float sign = on_boundary<MU, FWD>(A.g, c) ? A.g.bcf[MU] : 1.0f;
#pragma unroll
        for (int i = 0; i < 18; ++i) u[i] *= sign;
    }
    if constexpr (HIN) {
        // bf16 features in: the stay path stages them as they are; a hop transports them with
        // the link rounded to bf16 pairs, (Re, -Im) and (Im, Re) of each entry of U (U^dag for a
        // backward hop), so that each complex product-sum is two bf16 dot products accumulated
        // in float32 (v_dot2c_f32_bf16) instead of four FMAs on decoded values
        auto word = [&](int b, int k) -> uint32_t {
            const uint4 h = x.hv[2 * k + (b >> 2)];
            return (b & 3) == 0 ? h.x : (b & 3) == 1 ? h.y : (b & 3) == 2 ? h.z : h.w;
        };
        if constexpr (PATH == 0) {
#pragma unroll
            for (int b = 0; b < CIN; ++b)
#pragma unroll
                for (int k = 0; k < 3; ++k) *(uint32_t*)&B[(k * 64 + lane) * MF_LD + 2 * b] = word(b, k);
        } else {
            constexpr bool DAG = PATH > 4;
            bf16x2_t pre[9], pim[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) {
                    const int e = DAG ? 3 * c2 + a : 3 * a + c2;
                    const float ur = u[2 * e], ui = DAG ? -u[2 * e + 1] : u[2 * e + 1];
                    pre[3 * a + c2] = __builtin_bit_cast(bf16x2_t, cvt_bf16x2(ur, -ui));
                    pim[3 * a + c2] = __builtin_bit_cast(bf16x2_t, cvt_bf16x2(ui, ur));
                }
#pragma unroll
            for (int b = 0; b < CIN; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int c2 = 0; c2 < 3; ++c2) {
                        const bf16x2_t f = __builtin_bit_cast(bf16x2_t, word(b, c2));
                        re = __builtin_amdgcn_fdot2_f32_bf16(pre[3 * a + c2], f, re, false);
                        im = __builtin_amdgcn_fdot2_f32_bf16(pim[3 * a + c2], f, im, false);
                    }
                    *(uint32_t*)&B[(a * 64 + lane) * MF_LD + 2 * b] = cvt_bf16x2(re, im);
                }
        }
    } else {
#pragma unroll
        for (int b = 0; b < CIN; ++b) {
            float v[6], t[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                v[2 * k] = x.v[b][k].x;
                v[2 * k + 1] = x.v[b][k].y;
            }
            if constexpr (PATH > 0) {
                mat_vec(u, v, t, PATH > 4);
            } else {
#pragma unroll
                for (int i = 0; i < 6; ++i) t[i] = v[i];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
                *(uint32_t*)&B[(k * 64 + lane) * MF_LD + 2 * b] = cvt_bf16x2(t[2 * k], t[2 * k + 1]);
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 12; ++t) {
        const int n = t * 16 + (lane & 15);
        const bf16x4 bf = *(const bf16x4*)&B[n * MF_LD + 4 * (lane >> 4)];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Af, bf, acc[t], 0, 0, 0);
    }
    wave_lds_sync();
}

// paths P..LAST, each one's loads issued before the previous one's arithmetic
template <int P, int LAST, int R, int CIN, bool SIN, bool HF, bool L16>
__device__ __forceinline__ void mf_pipe(const PTArgs& A, const float2* in, int par, uint32_t cb, const int c[4],
                                        int lane, uint16_t* B, const bf16x4* Af, f32x4* acc, MfRaw<R, CIN, L16>& cur,
                                        MfRaw<R, CIN, L16>& nxt)
{
    if constexpr (P < LAST) mf_load<P + 1, R, CIN, SIN, HF, L16>(A, in, par, cb, c, nxt);
    mf_compute<P, R, CIN, L16, HF && !SIN>(A, c, lane, B, cur, Af[P], acc);
    if constexpr (P < LAST) mf_pipe<P + 1, LAST, R, CIN, SIN, HF, L16>(A, in, par, cb, c, lane, B, Af, acc, nxt, cur);
}

// SIN / SOUT: the input / output is an EVEN spinor half field (A.spin_in / A.spin_out);
// HF: the feature tensors hold bf16 pairs (one sample).
// SPLIT (no zero parity): two waves share each 64-site group, the first
// taking the stay path and the forward hops, the second the backward hops; the second's
// accumulators are added to the first's through LDS.  With few sites (one wave per SIMD
// otherwise) this halves each wave's chain of dependent path loads.
// L16: links read as float16 codes (A.gauge holds the 16-bit 12-real layout).
// The first layer of the bf16-feature network (4 input channels: latency-bound, a third of
// the VALU issue rate) runs three waves per SIMD (168 VGPRs, a few spilled): 3% less time per
// application at 32^3 x 64; the other layers keep two (with three the last one spills 24
// VGPRs and is slower).
template <int R, int CIN, int COUT, bool SIN, bool SOUT, bool HF, bool SPLIT, bool L16 = false>
__global__ void __launch_bounds__(256, CIN == 4 && HF ? 3 : 2) ptconv_mfma_kernel(PTArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t lds[4][192 * MF_LD];
    __shared__ f32x4 red[SPLIT ? 2 : 1][SPLIT ? 12 * 64 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint16_t* B = lds[wave];
    const uint32_t Vh = (uint32_t)A.g.Vh;
    // Every wave covers 64 consecutive checkerboard sites of one parity.  With both
    // parities computed, consecutive waves alternate parity over the same cb range, and
    // blocks run in XCD-contiguous order: the even and odd sites of one region (which read
    // each other's features and share their links) fill the same L2.  Under SPLIT the two
    // waves of a pair (0 and 1, 2 and 3 of a workgroup) cover one group.
    const bool both = A.out_sites > (int)Vh;
    const uint32_t gw = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const uint32_t gs = SPLIT ? gw >> 1 : gw;
    const int par = both ? (int)(gs & 1) : 0;
    const uint32_t i0 = (both ? gs >> 1 : gs) * 64;
    const uint32_t cb0 = A.zb > 0 ? zb_first(A, i0) : i0;
    // lanes past the end stage site 0 (in bounds); their columns are never stored
    const uint32_t cb = cb0 + lane < Vh ? cb0 + lane : 0;
    const float2* in = A.in + (size_t)blockIdx.y * A.in_sample;
    float2* out = A.out + (size_t)blockIdx.y * A.out_sample;
    int c[4];
    cb_coords(A.g, cb, par, c);
    // weights as A fragments, real form [[Wr, -Wi], [Wi, Wr]]
    bf16x4 Af[9];
    {
        const int m = lane & 15, g = lane >> 4;
        const int a = m >> 1, comp = m & 1;
#pragma unroll
        for (int p = 0; p < 9; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * g + q, b = k >> 1, kc = k & 1;
                float v = 0.f;
                if (a < COUT && b < CIN) {
                    const float2 wv = load_w<P_BF16>(A.W, (p * COUT + a) * CIN + b);
                    v = comp == 0 ? (kc == 0 ? wv.x : -wv.y) : (kc == 0 ? wv.y : wv.x);
                }
                Af[p][q] = (short)f2h<P_BF16>(v);
            }
    }
    if constexpr (CIN < 8) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int h = 2 * CIN; h < 16; h += 2) *(uint32_t*)&B[(k * 64 + lane) * MF_LD + h] = 0u;
    }
    f32x4 acc[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The stay path reads the wave's own parity, the hops the other one; a path whose
    // sources are all known zeros is skipped (par is wave-uniform).
    const bool skip_stay = A.zero_par >= 0 && par == A.zero_par;
    const bool skip_hops = A.zero_par >= 0 && 1 - par == A.zero_par;
    MfRaw<R, CIN, L16> ra, rb;
    if constexpr (SPLIT) {
        f32x4* rs = red[wave >> 1];
        if ((wave & 1) == 0) {
            mf_load<0, R, CIN, SIN, HF, L16>(A, in, par, cb, c, ra);
            mf_pipe<0, 4, R, CIN, SIN, HF, L16>(A, in, par, cb, c, lane, B, Af, acc, ra, rb);
        } else {
            mf_load<5, R, CIN, SIN, HF, L16>(A, in, par, cb, c, ra);
            mf_pipe<5, 8, R, CIN, SIN, HF, L16>(A, in, par, cb, c, lane, B, Af, acc, ra, rb);
#pragma unroll
            for (int t = 0; t < 12; ++t) rs[t * 64 + lane] = acc[t];
        }
        __syncthreads();
        if (wave & 1) return;
#pragma unroll
        for (int t = 0; t < 12; ++t) acc[t] += rs[t * 64 + lane];
    } else if (skip_hops) {
        mf_load<0, R, CIN, SIN, HF, L16>(A, in, par, cb, c, ra);
        mf_compute<0, R, CIN, L16, HF && !SIN>(A, c, lane, B, ra, Af[0], acc);
    } else if (skip_stay) {
        mf_load<1, R, CIN, SIN, HF, L16>(A, in, par, cb, c, ra);
        mf_pipe<1, 8, R, CIN, SIN, HF, L16>(A, in, par, cb, c, lane, B, Af, acc, ra, rb);
    } else {
        mf_load<0, R, CIN, SIN, HF, L16>(A, in, par, cb, c, ra);
        mf_pipe<0, 8, R, CIN, SIN, HF, L16>(A, in, par, cb, c, lane, B, Af, acc, ra, rb);
    }
    const int g = lane >> 4;
    float2* so = (float2*)A.spin_out;
#pragma unroll
    for (int t = 0; t < 12; ++t) {
        const int n = t * 16 + (lane & 15);
        const int k = n >> 6;
        const uint32_t scb = cb0 + (n & 63);
        if (scb >= Vh || i0 >= Vh) continue;   // (a wave past the last group stores nothing)
        if constexpr (SOUT) {   // even outputs straight into the spinor half field
            if (2 * g < COUT) so[spin_f2(2 * g, k, A.g.ps, scb)] = make_float2(acc[t][0], acc[t][1]);
            if (2 * g + 1 < COUT) so[spin_f2(2 * g + 1, k, A.g.ps, scb)] = make_float2(acc[t][2], acc[t][3]);
        } else if constexpr (HF) {   // channels 2 g, 2 g + 1 of colour k: words 2 (g % 2), + 1 of plane 2 k + g / 2
            static_assert(COUT == 8, "bf16 hidden features have 8 channels");
            uint2* ho = (uint2*)out;
            ho[hf_plane(par, 2 * k + (g >> 1), Vh, scb) * 2 + (g & 1)] =
                make_uint2(cvt_bf16x2(acc[t][0], acc[t][1]), cvt_bf16x2(acc[t][2], acc[t][3]));
        } else {
            if (2 * g < COUT) out[fidx(2 * g, par, k, Vh, scb)] = make_float2(acc[t][0], acc[t][1]);
            if (2 * g + 1 < COUT) out[fidx(2 * g + 1, par, k, Vh, scb)] = make_float2(acc[t][2], acc[t][3]);
        }
    }
}

// Split the nine paths of each 64-site group over two waves (the last layer of the learned
// preconditioner: even outputs only) when the unsplit launch would give the chip at most one
// round of two waves per SIMD (1024 SIMDs); WD_PTCONV_SPLIT = 0 / 1 forces it off / on.  The
// 8 -> 8 layers are bound by their vector arithmetic, where more waves do not help.
static bool ptconv_split(const PTArgs& A, bool hf, int cin, int cout, int nsamples)
{
    if (!(hf && cin == 8 && cout == 4 && A.spin_out && A.out_sites == A.g.Vh && A.zero_par < 0 && nsamples == 1))
        return false;
    if (const char* e = getenv("WD_PTCONV_SPLIT")) return atoi(e) != 0;
    return (A.g.Vh + 63) / 64 <= 2048;
}

// The bf16-feature layers (the learned preconditioner's network) with links as float16 codes.
static wd_status mfma_hf16(wd_context ctx, const PTArgs& A, int cin, int cout, bool split, dim3 grid, dim3 block)
{
    if (split) hipLaunchKernelGGL((ptconv_mfma_kernel<12, 8, 4, false, true, true, true, true>), grid, block, 0, ctx->stream, A);
    else if (cin == 4) hipLaunchKernelGGL((ptconv_mfma_kernel<12, 4, 8, true, false, true, false, true>), grid, block, 0, ctx->stream, A);
    else if (cout == 8) hipLaunchKernelGGL((ptconv_mfma_kernel<12, 8, 8, false, false, true, false, true>), grid, block, 0, ctx->stream, A);
    else hipLaunchKernelGGL((ptconv_mfma_kernel<12, 8, 4, false, true, true, false, true>), grid, block, 0, ctx->stream, A);
    WD_LAUNCHED();
    return WD_OK;
}

template <int R>
static wd_status mfma_r(wd_context ctx, const PTArgs& A, int cin, int cout, int nsamples, bool hf, bool l16)
{
    const bool split = ptconv_split(A, hf, cin, cout, nsamples);
    // one wave per 64-site group and parity computed, two when the group's paths are split
    const int waves = (A.out_sites > A.g.Vh ? 2 : 1) * (split ? 2 : 1) * ((A.g.Vh + 63) / 64);
    dim3 grid((waves + 3) / 4, nsamples), block(256);
    const bool si = A.spin_in != nullptr, so = A.spin_out != nullptr;
    if (l16) return mfma_hf16(ctx, A, cin, cout, split, grid, block);
    if (split) {
        hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 4, false, true, true, true>), grid, block, 0, ctx->stream, A);
    } else if (hf) {   // the 8-wide hidden layers of a 4 -> 8 -> ... -> 8 -> 4 network (checked by the caller)
        if (cin == 4) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 8, true, false, true, false>), grid, block, 0, ctx->stream, A);
        else if (cout == 8) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 8, false, false, true, false>), grid, block, 0, ctx->stream, A);
        else hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 4, false, true, true, false>), grid, block, 0, ctx->stream, A);
    } else if (cin == 4 && cout == 8) {
        if (si) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 8, true, false, false, false>), grid, block, 0, ctx->stream, A);
        else hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 8, false, false, false, false>), grid, block, 0, ctx->stream, A);
    } else if (cin == 8 && cout == 8) {
        hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 8, false, false, false, false>), grid, block, 0, ctx->stream, A);
    } else if (cin == 8 && cout == 4) {
        if (so) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 4, false, true, false, false>), grid, block, 0, ctx->stream, A);
        else hipLaunchKernelGGL((ptconv_mfma_kernel<R, 8, 4, false, false, false, false>), grid, block, 0, ctx->stream, A);
    } else {
        if (si && so) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 4, true, true, false, false>), grid, block, 0, ctx->stream, A);
        else if (si) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 4, true, false, false, false>), grid, block, 0, ctx->stream, A);
        else if (so) hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 4, false, true, false, false>), grid, block, 0, ctx->stream, A);
        else hipLaunchKernelGGL((ptconv_mfma_kernel<R, 4, 4, false, false, false, false>), grid, block, 0, ctx->stream, A);
    }
    WD_LAUNCHED();
    return WD_OK;
}

// z-block depth of the matrix-core layer's wave order: 4 from 2^18 sites per parity up (measured
// on 32^3 x 64: 10-14% less time per layer; on 16^3 x 32 within a few per cent either way, so
// the natural order stays there); WD_PTCONV_ZB overrides (0 = natural order).
static int ptconv_zblock(const Geom& G)
{
    int zb = G.Vh >= (1 << 18) ? 4 : 0;
    if (const char* e = getenv("WD_PTCONV_ZB")) zb = atoi(e);
    if (zb <= 0 || zb >= G.L[2] || G.L[2] % zb || (G.Xh * G.L[1]) % 64) return 0;
    return zb;
}

static bool use_mfma(int wprec, int cin, int cout)
{
    if (wprec != WD_BF16 || (cin != 4 && cin != 8) || (cout != 4 && cout != 8)) return false;
    const char* e = getenv("WD_PTCONV_MFMA");
    return !(e && atoi(e) == 0);
}

bool ptconv_spin_io(int wprec, int cin, int cout) { return use_mfma(wprec, cin, cout); }

// ---- launchers ---------------------------------------------------------------------------
template <int R, int WP>
static wd_status fwd_r_w(wd_context ctx, const PTArgs& A, int cout, int nsamples)
{
    dim3 grid((2 * A.g.Vh + 255) / 256, nsamples), block(256);
    switch (cout) {
#define WD_PT(C) case C: hipLaunchKernelGGL((ptconv_fwd_kernel<R, C, WP>), grid, block, 0, ctx->stream, A); break;
        WD_PT(1) WD_PT(2) WD_PT(3) WD_PT(4) WD_PT(8)
#undef WD_PT
    default: set_error("ptconv: C_out = %d not in {1, 2, 3, 4, 8}", cout); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return WD_OK;
}

wd_status ptconv_fwd(wd_gauge g, int cin, int cout, int wprec, const void* W, const void* in, void* out,
                            int nsamples, int zero_par, bool even_out, const void* spin_in, void* spin_out,
                            bool half_feat)
{
    if (half_feat && !(ptconv_spin_io(wprec, cin, cout) && nsamples == 1 &&
                       ((cin == 4 && cout == 8 && spin_in && !spin_out) || (cin == 8 && cout == 8 && !spin_in && !spin_out) ||
                        (cin == 8 && cout == 4 && !spin_in && spin_out)))) {
        set_error("ptconv: bf16 hidden features are built for the matrix-core layers of a 4 -> 8 -> ... -> 8 -> 4 "
                  "network (spinor in first, spinor out last), one sample");
        return WD_EINVAL;
    }
    if ((spin_in || spin_out) && !(ptconv_spin_io(wprec, cin, cout) && nsamples == 1 &&
                                   (!spin_in || (cin == 4 && zero_par == 1)) && (!spin_out || (cout == 4 && even_out)))) {
        set_error("ptconv: spinor input/output needs the matrix-core path, 4 spin channels, one sample, "
                  "a zero odd input half and even outputs only");
        return WD_EINVAL;
    }
    // The bf16-feature layers read the links as float16 codes (12 reals): the entries of an SU(3)
    // matrix are bounded by 1, so float16 keeps 2^-11 of them, below the bf16 rounding (2^-9) of
    // the transported features the layer applies anyway, in half the bytes of float32 links.
    // WD_PTCONV_LINKS32=1 keeps float32 links.
    const bool l16 = half_feat && g->recon == 12 && use_mfma(wprec, cin, cout) &&
                     !(getenv("WD_PTCONV_LINKS32") && atoi(getenv("WD_PTCONV_LINKS32")) != 0);
    const void* links;
    WD_TRY(gauge_links(g, l16 ? WD_F16 : WD_F32, &links));
    PTArgs A;
    A.gauge = (const char*)links;
    A.in = (const float2*)in;
    A.out = (float2*)out;
    A.W = W;
    A.g = g->geom;
    A.cin = cin;
    A.in_sample = (long long)cin * 6 * g->geom.Vh;
    A.out_sample = (long long)cout * 6 * g->geom.Vh;
    A.zero_par = zero_par;
    A.out_sites = even_out ? g->geom.Vh : 2 * g->geom.Vh;
    A.spin_in = (const char*)spin_in;
    A.spin_out = (char*)spin_out;
    {
        const Geom& G = g->geom;
        const int zb = ptconv_zblock(G);
        if (zb > 0) {
            A.zb = zb;
            A.dplane = make_fastdiv((uint32_t)(G.Xh * G.L[1]));
            A.dzb = make_fastdiv((uint32_t)zb);
            A.dt = make_fastdiv((uint32_t)G.L[3]);
        }
    }
    const bool r12 = g->recon == 12;
    if (use_mfma(wprec, cin, cout))
        return r12 ? mfma_r<12>(g->ctx, A, cin, cout, nsamples, half_feat, l16)
                   : mfma_r<18>(g->ctx, A, cin, cout, nsamples, half_feat, false);
    switch (wprec) {
    case WD_F32: return r12 ? fwd_r_w<12, P_F32>(g->ctx, A, cout, nsamples) : fwd_r_w<18, P_F32>(g->ctx, A, cout, nsamples);
    case WD_F16: return r12 ? fwd_r_w<12, P_F16>(g->ctx, A, cout, nsamples) : fwd_r_w<18, P_F16>(g->ctx, A, cout, nsamples);
    case WD_BF16: return r12 ? fwd_r_w<12, P_BF16>(g->ctx, A, cout, nsamples) : fwd_r_w<18, P_BF16>(g->ctx, A, cout, nsamples);
    }
    set_error("ptconv: weight precision %d not in {F32, F16, BF16}", wprec);
    return WD_EUNSUPPORTED;
}

wd_status launch_spinor_features(wd_context ctx, const Geom& g, int nsamples, void* spinor, void* feat,
                                 bool to_features, bool even_only)
{
    const long long n = 2ll * g.Vh * nsamples;
    hipLaunchKernelGGL(spinor_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                       (const char*)spinor, (float2*)feat, g.Vh, g.ps, nsamples, to_features, even_only);
    WD_LAUNCHED();
    return WD_OK;
}

static bool ok_channels(int c) { return c == 1 || c == 2 || c == 3 || c == 4 || c == 8; }

template <int R>
static wd_status wgrad_r(wd_context ctx, const PTArgs& A, int cout, const void* gout, int nsamples, int nblk, double* part)
{
    dim3 grid(nblk, 9), block(256);
    switch (cout) {
#define WD_PT(C) case C: hipLaunchKernelGGL((ptconv_wgrad_kernel<R, C>), grid, block, 0, ctx->stream, A, (const float2*)gout, nsamples, part); break;
        WD_PT(1) WD_PT(2) WD_PT(3) WD_PT(4) WD_PT(8)
#undef WD_PT
    default: set_error("ptconv: C_out = %d not supported", cout); return WD_EUNSUPPORTED;
    }
    WD_LAUNCHED();
    return WD_OK;
}

} // namespace wd

using namespace wd;

extern "C" {

size_t wd_feature_bytes(const wd_lattice* lat, int channels, int nsamples)
{
    Geom g;
    if (channels < 1 || nsamples < 1 || make_geom(lat, &g) != WD_OK) return 0;
    return (size_t)nsamples * channels * 2 * 3 * g.Vh * sizeof(float2);
}

static wd_status feature_io(wd_context ctx, const wd_lattice* lat, int channels, int nsamples, double* canon, void* packed,
                            bool unpack)
{
    Geom g;
    if (!ctx || !canon || !packed || channels < 1 || nsamples < 1) {
        set_error("feature pack/unpack: NULL pointer or bad channel/sample count");
        return WD_EINVAL;
    }
    WD_TRY(make_geom(lat, &g));
    const long long total = (long long)nsamples * channels * 2 * g.Vh;
    hipLaunchKernelGGL(feature_pack_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, ctx->stream, canon,
                       (float2*)packed, g, channels, total, unpack);
    WD_LAUNCHED();
    return WD_OK;
}

wd_status wd_feature_pack(wd_context ctx, const wd_lattice* lat, int channels, int nsamples, const double* canon,
                          void* packed)
{
    return feature_io(ctx, lat, channels, nsamples, (double*)canon, packed, false);
}

wd_status wd_feature_unpack(wd_context ctx, const wd_lattice* lat, int channels, int nsamples, const void* packed,
                            double* canon)
{
    return feature_io(ctx, lat, channels, nsamples, canon, (void*)packed, true);
}

wd_status wd_spinor_to_features(wd_context ctx, const wd_lattice* lat, int nsamples, const void* spinor, void* feat)
{
    Geom g;
    if (!ctx || !spinor || !feat || nsamples < 1) {
        set_error("wd_spinor_to_features: bad argument");
        return WD_EINVAL;
    }
    WD_TRY(make_geom(lat, &g));
    return launch_spinor_features(ctx, g, nsamples, (void*)spinor, feat, true);
}

wd_status wd_features_to_spinor(wd_context ctx, const wd_lattice* lat, int nsamples, const void* feat, void* spinor)
{
    Geom g;
    if (!ctx || !spinor || !feat || nsamples < 1) {
        set_error("wd_features_to_spinor: bad argument");
        return WD_EINVAL;
    }
    WD_TRY(make_geom(lat, &g));
    return launch_spinor_features(ctx, g, nsamples, spinor, (void*)feat, false);
}

wd_status wd_ptconv_forward(wd_gauge g, int cin, int cout, wd_prec wprec, int nsamples, const void* W, const void* in,
                            void* out)
{
    if (!g || !W || !in || !out || nsamples < 1 || nsamples > 65535) {
        set_error("wd_ptconv_forward: NULL pointer or bad sample count");
        return WD_EINVAL;
    }
    if (!ok_channels(cin) || !ok_channels(cout)) {
        set_error("wd_ptconv_forward: channels (%d, %d) not in {1, 2, 3, 4, 8}", cin, cout);
        return WD_EUNSUPPORTED;
    }
    if (in == out) {
        set_error("wd_ptconv_forward: in and out must not alias");
        return WD_EINVAL;
    }
    return ptconv_fwd(g, cin, cout, wprec, W, in, out, nsamples);
}

wd_status wd_ptconv_backward(wd_gauge g, int cin, int cout, wd_prec wprec, int nsamples, const void* W, const void* in,
                             const void* gout, void* gin, void* gW)
{
    if (!g || !W || !in || !gout || (!gin && !gW) || nsamples < 1 || nsamples > 65535) {
        set_error("wd_ptconv_backward: NULL pointer or bad sample count");
        return WD_EINVAL;
    }
    if (!ok_channels(cin) || !ok_channels(cout)) {
        set_error("wd_ptconv_backward: channels (%d, %d) not in {1, 2, 3, 4, 8}", cin, cout);
        return WD_EUNSUPPORTED;
    }
    if (wprec != WD_F32 && wprec != WD_F16 && wprec != WD_BF16) {
        set_error("wd_ptconv_backward: weight precision %d not supported", (int)wprec);
        return WD_EUNSUPPORTED;
    }
    wd_context ctx = g->ctx;
    if (gin) {
        void* Wt;
        const size_t wbytes = (size_t)9 * cin * cout * (wprec == WD_F32 ? 8 : 4);
        WD_TRY(ws_get(ctx, "ptconv.Wt", wbytes, &Wt));
        const int n = 9 * cin * cout;
        if (wprec == WD_F32)
            hipLaunchKernelGGL(adjoint_weights_kernel<P_F32>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, W, Wt, cin, cout);
        else
            hipLaunchKernelGGL(adjoint_weights_kernel<P_F16>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, W, Wt, cin, cout);
        WD_LAUNCHED();
        WD_TRY(ptconv_fwd(g, cout, cin, wprec, Wt, gout, gin, nsamples));
    }
    if (gW) {
        const void* links;
        WD_TRY(gauge_links(g, WD_F32, &links));
        PTArgs A;
        A.gauge = (const char*)links;
        A.in = (const float2*)in;
        A.out = nullptr;
        A.W = W;
        A.g = g->geom;
        A.cin = cin;
        A.in_sample = (long long)cin * 6 * g->geom.Vh;
        A.out_sample = (long long)cout * 6 * g->geom.Vh;
        const long long nsites = 2ll * g->geom.Vh * nsamples;
        long long nblk = (nsites + 255) / 256;
        if (nblk > 512) nblk = 512;
        void* part;
        WD_TRY(ws_get(ctx, "ptconv.partials", (size_t)9 * cin * 2 * cout * nblk * sizeof(double), &part));
        WD_TRY(g->recon == 12 ? wgrad_r<12>(ctx, A, cout, gout, nsamples, (int)nblk, (double*)part)
                              : wgrad_r<18>(ctx, A, cout, gout, nsamples, (int)nblk, (double*)part));
        const int n = 9 * cin * cout;
        hipLaunchKernelGGL(wgrad_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, (const double*)part,
                           (int)nblk, cin, cout, (float2*)gW);
        WD_LAUNCHED();
    }
    return WD_OK;
}

} // extern "C"
