// Device-side building blocks shared by the gfx950 kernels: lattice geometry,
// structure-of-arrays field access per storage precision, the 16-bit codec,
// and the spin projection tables of the Wilson hopping term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wd {

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

template <int P> struct RealOf { using T = float; };
template <> struct RealOf<P_F64> { using T = double; };

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
// Division by a runtime constant d for 0 <= n < 2^31 (Granlund & Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, Thm 4.2):
// with l = ceil(log2 d) and m = floor(2^(31+l) / d) + 1, n / d = (m n) >> (31 + l).
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.s = 31 + l;
    f.m = (uint32_t)(((1ull << (31 + l)) / d) + 1);
    return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    return (uint32_t)(((uint64_t)f.m * n) >> f.s);
}

struct Geom {
    int L[4];          // X, Y, Z, T
    int Xh;            // X / 2
    int Vh;            // sites per parity
    int ps;            // plane stride in sites (Vh, padded on large lattices)
    int st[4];         // checkerboard-index stride of a unit step in mu (st[0] unused)
    float bcf[4];      // boundary sign per direction
    double bcd[4];
    FastDiv dxh, dy, dz;
};

// Coordinates of checkerboard site cb of parity par.
__device__ __forceinline__ void cb_coords(const Geom& g, uint32_t cb, int par, int c[4])
{
    uint32_t q1 = fdiv(cb, g.dxh);
    uint32_t xh = cb - q1 * (uint32_t)g.Xh;
    uint32_t q2 = fdiv(q1, g.dy);
    uint32_t y = q1 - q2 * (uint32_t)g.L[1];
    uint32_t t = fdiv(q2, g.dz);
    uint32_t z = q2 - t * (uint32_t)g.L[2];
    c[1] = (int)y;
    c[2] = (int)z;
    c[3] = (int)t;
    c[0] = (int)(2 * xh + ((par + y + z + t) & 1));
}

// Checkerboard index of the neighbour x +- mu (always of the other parity).
template <int MU, bool FWD>
__device__ __forceinline__ uint32_t neighbour(const Geom& g, uint32_t cb, const int c[4])
{
    if constexpr (MU == 0) {
        int x = c[0];
        int xn = FWD ? (x + 1 == g.L[0] ? 0 : x + 1) : (x == 0 ? g.L[0] - 1 : x - 1);
        return cb - (uint32_t)(x >> 1) + (uint32_t)(xn >> 1);
    } else {
        const int L = g.L[MU];
        const uint32_t st = (uint32_t)g.st[MU];
        if (FWD) return c[MU] == L - 1 ? cb - (uint32_t)(L - 1) * st : cb + st;
        return c[MU] == 0 ? cb + (uint32_t)(L - 1) * st : cb - st;
    }
}

template <int MU, bool FWD>
__device__ __forceinline__ bool on_boundary(const Geom& g, const int c[4])
{
    return FWD ? (c[MU] == g.L[MU] - 1) : (c[MU] == 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); remap so XCD k walks one contiguous run of blocks, keeping spatially
// adjacent sites (and their shared neighbours) in one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblk)
{
    const uint32_t NX = 8;
    uint32_t xcd = bid % NX, local = bid / NX;
    uint32_t per = nblk / NX, rem = nblk % NX;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// ---------------------------------------------------------------------------
// 16-bit codec (round to nearest even)
// ---------------------------------------------------------------------------
template <int P> __device__ __forceinline__ float h2f(uint32_t b);
template <> __device__ __forceinline__ float h2f<P_F16>(uint32_t b)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}
template <> __device__ __forceinline__ float h2f<P_BF16>(uint32_t b)
{
    return __uint_as_float(b << 16);
}
template <int P> __device__ __forceinline__ uint32_t f2h(float f);
// The codec rounds a float32 value.  Left alone, the compiler folds a caller's product
// v * inv into the conversion (one mixed-precision FMA rounds the exact product straight
// to 16 bits), which differs from rounding the float32 product about once in 2^14 values;
// an empty register constraint makes the operand a float32 register value first.
template <> __device__ __forceinline__ uint32_t f2h<P_F16>(float f)
{
    asm("" : "+v"(f));
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
}
template <> __device__ __forceinline__ uint32_t f2h<P_BF16>(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <int P> __device__ __forceinline__ void unpack8(const uint4 q, float s, float* v)
{
    v[0] = h2f<P>(q.x) * s; v[1] = h2f<P>(q.x >> 16) * s;
    v[2] = h2f<P>(q.y) * s; v[3] = h2f<P>(q.y >> 16) * s;
    v[4] = h2f<P>(q.z) * s; v[5] = h2f<P>(q.z >> 16) * s;
    v[6] = h2f<P>(q.w) * s; v[7] = h2f<P>(q.w >> 16) * s;
}

template <int P> __device__ __forceinline__ uint32_t pack2(float a, float b)
{
    return f2h<P>(a) | (f2h<P>(b) << 16);
}
// bf16 and f16 pairs: gfx950 converts two floats with round-to-nearest-even in one instruction
typedef __bf16 wd_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 wd_f16x2 __attribute__((ext_vector_type(2)));
typedef float wd_f32x2 __attribute__((ext_vector_type(2)));
template <> __device__ __forceinline__ uint32_t pack2<P_F16>(float a, float b)
{
    asm("" : "+v"(a), "+v"(b));   // float32 operands, as in f2h<P_F16>
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(wd_f32x2{a, b}, wd_f16x2));
}
template <> __device__ __forceinline__ uint32_t pack2<P_BF16>(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(wd_f32x2{a, b}, wd_bf16x2));
}

// ---------------------------------------------------------------------------
// Plane stride.  On a lattice of 2^k sites every plane of a packed field
// would start a power of two bytes after the previous one, so the same site
// of all planes maps onto the same HBM channels and the streams of one
// kernel queue behind each other.  Large lattices therefore space planes
// ps = roundup(Vh, 64) + 256 sites apart (the tail of each plane is unused
// padding); below 4096 sites per parity ps = Vh.
__host__ __device__ constexpr long long plane_stride(long long Vh)
{
    return Vh < 4096 ? Vh : ((Vh + 63) / 64) * 64 + 256;
}

// ---------------------------------------------------------------------------
// Spinor half-field access.  A half field holds the Vh sites of one parity
// in planes ps sites apart (the stride argument of load and store):
//   F32 : 6 planes of float4            (96 B/site)
//   F64 : 12 planes of double2          (192 B/site)
//   F16/BF16: 3 planes of 8 x 16-bit + 1 plane of float32 scales (52 B/site)
// Real index inside a site: (spin * 3 + colour) * 2 + (re, im).
// ---------------------------------------------------------------------------
template <int P> struct SpinorIO;

template <> struct SpinorIO<P_F32> {
    static constexpr size_t site_bytes = 96;
    __device__ __forceinline__ static void load(const char* base, int Vh, uint32_t cb, float* v)
    {
        const float4* p = (const float4*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 q = p[(size_t)k * Vh + cb];
            v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
        }
    }
    __device__ __forceinline__ static void store(char* base, int Vh, uint32_t cb, const float* v)
    {
        float4* p = (float4*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[(size_t)k * Vh + cb] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    }
    // non-temporal: a field read once, that the caches need not keep
    __device__ __forceinline__ static void load_nt(const char* base, int Vh, uint32_t cb, float* v)
    {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4* p = (const f4*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const f4 q = __builtin_nontemporal_load(p + (size_t)k * Vh + cb);
            v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
        }
    }
};

template <> struct SpinorIO<P_F64> {
    static constexpr size_t site_bytes = 192;
    __device__ __forceinline__ static void load(const char* base, int Vh, uint32_t cb, double* v)
    {
        const double2* p = (const double2*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 q = p[(size_t)k * Vh + cb];
            v[2 * k] = q.x; v[2 * k + 1] = q.y;
        }
    }
    __device__ __forceinline__ static void store(char* base, int Vh, uint32_t cb, const double* v)
    {
        double2* p = (double2*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k) p[(size_t)k * Vh + cb] = make_double2(v[2 * k], v[2 * k + 1]);
    }
    __device__ __forceinline__ static void load_nt(const char* base, int Vh, uint32_t cb, double* v)
    {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2* p = (const d2*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const d2 q = __builtin_nontemporal_load(p + (size_t)k * Vh + cb);
            v[2 * k] = q.x; v[2 * k + 1] = q.y;
        }
    }
};

template <int P> struct SpinorIO16 {
    static constexpr size_t site_bytes = 52;
    __device__ __forceinline__ static void load(const char* base, int Vh, uint32_t cb, float* v)
    {
        const uint4* p = (const uint4*)base;
        const float s = ((const float*)(p + (size_t)3 * Vh))[cb];
#pragma unroll
        for (int k = 0; k < 3; ++k) unpack8<P>(p[(size_t)k * Vh + cb], s, v + 8 * k);
    }
    __device__ __forceinline__ static void load_nt(const char* base, int Vh, uint32_t cb, float* v)
    {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const u4* p = (const u4*)base;
        const float s = __builtin_nontemporal_load((const float*)(p + (size_t)3 * Vh) + cb);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const u4 q = __builtin_nontemporal_load(p + (size_t)k * Vh + cb);
            unpack8<P>(make_uint4(q.x, q.y, q.z, q.w), s, v + 8 * k);
        }
    }
    // s = max |v_i|, codes RNE16(v_i * RN(1/s)); an all-zero site stores s = 0.
    __device__ __forceinline__ static void store(char* base, int Vh, uint32_t cb, const float* v)
    {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < 24; ++k) s = fmaxf(s, fabsf(v[k]));
        const float inv = s > 0.0f ? 1.0f / s : 0.0f;
        uint4* p = (uint4*)base;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float* w = v + 8 * k;
            uint4 q;
            q.x = pack2<P>(w[0] * inv, w[1] * inv);
            q.y = pack2<P>(w[2] * inv, w[3] * inv);
            q.z = pack2<P>(w[4] * inv, w[5] * inv);
            q.w = pack2<P>(w[6] * inv, w[7] * inv);
            p[(size_t)k * Vh + cb] = q;
        }
        ((float*)(p + (size_t)3 * Vh))[cb] = s;
    }
};
template <> struct SpinorIO<P_F16> : SpinorIO16<P_F16> {};
template <> struct SpinorIO<P_BF16> : SpinorIO16<P_BF16> {};

__host__ __device__ constexpr size_t spinor_site_bytes(int P)
{
    return P == P_F64 ? 192 : (P == P_F32 ? 96 : 52);
}

// ---------------------------------------------------------------------------
// Link access.  Links are grouped by (mu, parity of the site they start at);
// each group holds Vh links as structure-of-arrays planes ps sites apart:
//   F32 r12: 3 x float4         r18: 4 x float4 + 1 x float2
//   F64 r12: 6 x double2        r18: 9 x double2
//   16-bit r12: uint4 + uint2   r18: 2 x uint4 + 1 x uint32
// Real index inside a link: (row * 3 + col) * 2 + (re, im); r12 keeps rows 0, 1.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr size_t link_site_bytes(int P, int R)
{
    return (P == P_F64 ? 8 : (P == P_F32 ? 4 : 2)) * (size_t)R;
}

// Plain or non-temporal (streaming, low cache retention) vector load.
template <typename V> struct ExtVec;
template <> struct ExtVec<float4> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct ExtVec<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct ExtVec<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct ExtVec<uint4> { typedef unsigned int T __attribute__((ext_vector_type(4))); };
template <> struct ExtVec<uint2> { typedef unsigned int T __attribute__((ext_vector_type(2))); };

template <bool NT, typename V> __device__ __forceinline__ V ldv(const V* p)
{
    if constexpr (NT) {
        typename ExtVec<V>::T r = __builtin_nontemporal_load((const typename ExtVec<V>::T*)p);
        V v;
        static_assert(sizeof(v) == sizeof(r), "vector size");
        __builtin_memcpy(&v, &r, sizeof(v));
        return v;
    } else {
        return *p;
    }
}
template <bool NT> __device__ __forceinline__ uint32_t ldv(const uint32_t* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T> __device__ __forceinline__ void reconstruct_row2(T* u)
{
    // row2 = conj(row0 x row1)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int p = (j + 1) % 3, q = (j + 2) % 3;
        const T ar = u[2 * p], ai = u[2 * p + 1], br = u[6 + 2 * q], bi = u[6 + 2 * q + 1];
        const T cr = u[2 * q], ci = u[2 * q + 1], dr = u[6 + 2 * p], di = u[6 + 2 * p + 1];
        // (a b - c d) as chains of fused multiply-adds
        const T re = fma(ar, br, fma(-ai, bi, fma(-cr, dr, ci * di)));
        const T im = fma(ar, bi, fma(ai, br, fma(-cr, di, -(ci * dr))));
        u[12 + 2 * j] = re;
        u[12 + 2 * j + 1] = -im;
    }
}

template <int P, int R, bool NT> struct LinkIO;

template <int R, bool NT> struct LinkIO<P_F32, R, NT> {
    __device__ __forceinline__ static void load(const char* grp, int Vh, uint32_t cb, float* u)
    {
        const float4* p = (const float4*)grp;
        constexpr int NV4 = (R == 12) ? 3 : 4;
#pragma unroll
        for (int k = 0; k < NV4; ++k) {
            float4 q = ldv<NT>(p + (size_t)k * Vh + cb);
            u[4 * k] = q.x; u[4 * k + 1] = q.y; u[4 * k + 2] = q.z; u[4 * k + 3] = q.w;
        }
        if constexpr (R == 18) {
            float2 q = ldv<NT>((const float2*)(p + (size_t)4 * Vh) + cb);
            u[16] = q.x; u[17] = q.y;
        } else {
            reconstruct_row2(u);
        }
    }
};

template <int R, bool NT> struct LinkIO<P_F64, R, NT> {
    __device__ __forceinline__ static void load(const char* grp, int Vh, uint32_t cb, double* u)
    {
        const double2* p = (const double2*)grp;
        constexpr int NC = R / 2;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            double2 q = ldv<NT>(p + (size_t)k * Vh + cb);
            u[2 * k] = q.x; u[2 * k + 1] = q.y;
        }
        if constexpr (R == 12) reconstruct_row2(u);
    }
};

template <int P, int R, bool NT> struct LinkIO16 {
    __device__ __forceinline__ static void load(const char* grp, int Vh, uint32_t cb, float* u)
    {
        const uint4* p = (const uint4*)grp;
        if constexpr (R == 12) {
            unpack8<P>(ldv<NT>(p + cb), 1.0f, u);
            uint2 q = ldv<NT>((const uint2*)(p + (size_t)Vh) + cb);
            u[8] = h2f<P>(q.x); u[9] = h2f<P>(q.x >> 16);
            u[10] = h2f<P>(q.y); u[11] = h2f<P>(q.y >> 16);
            reconstruct_row2(u);
        } else {
            unpack8<P>(ldv<NT>(p + cb), 1.0f, u);
            unpack8<P>(ldv<NT>(p + (size_t)Vh + cb), 1.0f, u + 8);
            uint32_t q = ldv<NT>((const uint32_t*)(p + (size_t)2 * Vh) + cb);
            u[16] = h2f<P>(q); u[17] = h2f<P>(q >> 16);
        }
    }
};
template <int R, bool NT> struct LinkIO<P_F16, R, NT> : LinkIO16<P_F16, R, NT> {};
template <int R, bool NT> struct LinkIO<P_BF16, R, NT> : LinkIO16<P_BF16, R, NT> {};

// ---------------------------------------------------------------------------
// Spin projection (1 + S gamma_mu) in the DeGrand-Rossi basis.
// The projector has rank 2: with h0 = psi_0 + CA psi_IA and h1 = psi_1 + CB psi_IB,
// the projected spinor is (h0, h1, C2 h_J2, C3 h_J3).  Unit codes:
// 0: +1, 1: -1, 2: +i, 3: -i; S = -1 flips every code's sign (code ^ 1).
// ---------------------------------------------------------------------------
template <int MU, int S> struct Proj {
    static constexpr int f = (S > 0) ? 0 : 1;
    static constexpr int IA = (MU <= 1) ? 3 : 2;
    static constexpr int IB = (MU <= 1) ? 2 : 3;
    static constexpr int CA = (MU == 0 ? 2 : MU == 1 ? 1 : MU == 2 ? 2 : 0) ^ f;
    static constexpr int CB = (MU == 0 ? 2 : MU == 1 ? 0 : MU == 2 ? 3 : 0) ^ f;
    static constexpr int C2 = (MU == 0 ? 3 : MU == 1 ? 0 : MU == 2 ? 3 : 0) ^ f;
    static constexpr int C3 = (MU == 0 ? 3 : MU == 1 ? 1 : MU == 2 ? 2 : 0) ^ f;
    static constexpr int J2 = (MU == 0 || MU == 1) ? 1 : 0;
    static constexpr int J3 = (MU == 0 || MU == 1) ? 0 : 1;
};

// z * unit(CODE), on (re, im) pairs
template <int CODE, typename T> __device__ __forceinline__ T umul_re(T re, T im)
{
    if constexpr (CODE == 0) return re;
    else if constexpr (CODE == 1) return -re;
    else if constexpr (CODE == 2) return -im;
    else return im;
}
template <int CODE, typename T> __device__ __forceinline__ T umul_im(T re, T im)
{
    if constexpr (CODE == 0) return im;
    else if constexpr (CODE == 1) return -im;
    else if constexpr (CODE == 2) return re;
    else return -re;
}

// psi: 24 reals; h: 12 reals (two colour triplets)
template <int MU, int S, typename T> __device__ __forceinline__ void project(const T* psi, T* h)
{
    using PJ = Proj<MU, S>;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T* a = psi + (PJ::IA * 3 + c) * 2;
        const T* b = psi + (PJ::IB * 3 + c) * 2;
        h[2 * c] = psi[(0 * 3 + c) * 2] + umul_re<PJ::CA>(a[0], a[1]);
        h[2 * c + 1] = psi[(0 * 3 + c) * 2 + 1] + umul_im<PJ::CA>(a[0], a[1]);
        h[6 + 2 * c] = psi[(1 * 3 + c) * 2] + umul_re<PJ::CB>(b[0], b[1]);
        h[6 + 2 * c + 1] = psi[(1 * 3 + c) * 2 + 1] + umul_im<PJ::CB>(b[0], b[1]);
    }
}

// acc (24 reals) += expansion of the colour-multiplied half spinor w (12 reals)
template <int MU, int S, typename T> __device__ __forceinline__ void accumulate(T* acc, const T* w)
{
    using PJ = Proj<MU, S>;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[(0 * 3 + c) * 2] += w[2 * c];
        acc[(0 * 3 + c) * 2 + 1] += w[2 * c + 1];
        acc[(1 * 3 + c) * 2] += w[6 + 2 * c];
        acc[(1 * 3 + c) * 2 + 1] += w[6 + 2 * c + 1];
        const T* a = w + 6 * PJ::J2 + 2 * c;
        const T* b = w + 6 * PJ::J3 + 2 * c;
        acc[(2 * 3 + c) * 2] += umul_re<PJ::C2>(a[0], a[1]);
        acc[(2 * 3 + c) * 2 + 1] += umul_im<PJ::C2>(a[0], a[1]);
        acc[(3 * 3 + c) * 2] += umul_re<PJ::C3>(b[0], b[1]);
        acc[(3 * 3 + c) * 2 + 1] += umul_im<PJ::C3>(b[0], b[1]);
    }
}

// w = U h (DAG = false) or U^dagger h (DAG = true), for both colour triplets of h.
template <bool DAG, typename T> __device__ __forceinline__ void su3_mul(const T* u, const T* h, T* w)
{
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int e = DAG ? (3 * b + a) : (3 * a + b);
                const T ur = u[2 * e], ui = DAG ? -u[2 * e + 1] : u[2 * e + 1];
                const T hr = h[6 * s + 2 * b], hi = h[6 * s + 2 * b + 1];
                re = fma(ur, hr, re);
                re = fma(-ui, hi, re);
                im = fma(ur, hi, im);
                im = fma(ui, hr, im);
            }
            w[6 * s + 2 * a] = re;
            w[6 * s + 2 * a + 1] = im;
        }
    }
}

} // namespace wd
