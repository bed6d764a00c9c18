/*
 * Seeded synthetic inputs for the Wilson-Dirac workloads: SU(3) gauge links
 * U = exp(i*eps*H) with H a traceless Hermitian matrix of Gaussian entries
 * (reunitarised), and complex Gaussian spinor entries.
 *
 * This file holds none of the operator's arithmetic.  It is the one input
 * source shared by the FP64 oracle and by the GPU library, so both sides
 * always see bit-identical inputs.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), a counter-based generator, so every
 * entry is a pure function of (seed, stream, index) and the fill is
 * embarrassingly parallel.  Each Philox call yields one pair of standard
 * normals via the Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Exposed for the known-answer test of the generator itself. */
void ls_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    philox4x32_10(ctr, key, out);
}

/* Two uniforms in the open interval (0,1) with 53 random bits each. */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

/* One pair of independent standard normals from counter (index, stream, sub). */
static void normal_pair(uint64_t seed, uint64_t index, uint32_t stream, uint32_t sub,
                        double* z0, double* z1)
{
    uint32_t ctr[4] = { (uint32_t)index, (uint32_t)(index >> 32), stream, sub };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    double u1 = u53(w[0], w[1]);
    double u2 = u53(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586476925286766559 * u2;
    *z0 = r * cos(th);
    *z1 = r * sin(th);
}

/*
 * n complex numbers out[2k], out[2k+1] with Re, Im ~ N(0, var/2) each, so that
 * E|z|^2 = var.  Entry k uses counter (k, stream, 0).
 */
void ls_gaussian(uint64_t n, uint64_t seed, uint32_t stream, double var, double* out)
{
    double s = sqrt(0.5 * var);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        double a, b;
        normal_pair(seed, (uint64_t)k, stream, 0u, &a, &b);
        out[2 * k] = s * a;
        out[2 * k + 1] = s * b;
    }
}

/* ---- 3x3 complex helpers on interleaved (re, im) doubles ---------------- */
typedef struct { double re, im; } cd;

static void mat_mul(const cd a[9], const cd b[9], cd c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; ++k) {
                re += a[3 * i + k].re * b[3 * k + j].re - a[3 * i + k].im * b[3 * k + j].im;
                im += a[3 * i + k].re * b[3 * k + j].im + a[3 * i + k].im * b[3 * k + j].re;
            }
            c[3 * i + j].re = re;
            c[3 * i + j].im = im;
        }
}

/* exp(X) for a 3x3 complex matrix by scaling and squaring of the Taylor series. */
static void mat_exp(const cd x[9], cd e[9])
{
    double fro = 0.0;
    for (int i = 0; i < 9; ++i) fro += x[i].re * x[i].re + x[i].im * x[i].im;
    fro = sqrt(fro);
    int s = 0;
    while (fro > 0.25) { fro *= 0.5; ++s; }
    double scale = ldexp(1.0, -s);
    cd y[9], term[9], tmp[9];
    for (int i = 0; i < 9; ++i) { y[i].re = x[i].re * scale; y[i].im = x[i].im * scale; }
    for (int i = 0; i < 9; ++i) { e[i].re = (i % 4 == 0) ? 1.0 : 0.0; e[i].im = 0.0; term[i] = e[i]; }
    for (int k = 1; k <= 16; ++k) {
        mat_mul(term, y, tmp);
        for (int i = 0; i < 9; ++i) {
            term[i].re = tmp[i].re / k;
            term[i].im = tmp[i].im / k;
            e[i].re += term[i].re;
            e[i].im += term[i].im;
        }
    }
    for (int q = 0; q < s; ++q) {
        mat_mul(e, e, tmp);
        for (int i = 0; i < 9; ++i) e[i] = tmp[i];
    }
}

/* Gram-Schmidt on rows 0 and 1, then row 2 = conj(row0 x row1): an exact SU(3) matrix. */
static void reunitarise(cd u[9])
{
    double n0 = 0.0;
    for (int j = 0; j < 3; ++j) n0 += u[j].re * u[j].re + u[j].im * u[j].im;
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; ++j) { u[j].re *= n0; u[j].im *= n0; }
    /* c = <row0, row1> = sum conj(r0_j) r1_j */
    double cre = 0.0, cim = 0.0;
    for (int j = 0; j < 3; ++j) {
        cre += u[j].re * u[3 + j].re + u[j].im * u[3 + j].im;
        cim += u[j].re * u[3 + j].im - u[j].im * u[3 + j].re;
    }
    for (int j = 0; j < 3; ++j) {
        u[3 + j].re -= cre * u[j].re - cim * u[j].im;
        u[3 + j].im -= cre * u[j].im + cim * u[j].re;
    }
    double n1 = 0.0;
    for (int j = 0; j < 3; ++j) n1 += u[3 + j].re * u[3 + j].re + u[3 + j].im * u[3 + j].im;
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; ++j) { u[3 + j].re *= n1; u[3 + j].im *= n1; }
    const cd* a = u;
    const cd* b = u + 3;
    for (int j = 0; j < 3; ++j) {
        int p = (j + 1) % 3, q = (j + 2) % 3;
        double re = a[p].re * b[q].re - a[p].im * b[q].im - (a[q].re * b[p].re - a[q].im * b[p].im);
        double im = a[p].re * b[q].im + a[p].im * b[q].re - (a[q].re * b[p].im + a[q].im * b[p].re);
        u[6 + j].re = re;
        u[6 + j].im = -im;
    }
}

/*
 * n SU(3) matrices, row-major, interleaved complex: out[18*k + 6*a + 2*b + {0,1}].
 * Matrix k: A_ab = N(0,1) + i N(0,1) from counter (k, stream, 3a+b);
 * H = (A + A^dagger)/2 - tr(.)/3; U = exp(i eps H), reunitarised.
 */
void ls_su3(uint64_t n, double eps, uint64_t seed, uint32_t stream, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        cd a[9], h[9], x[9], u[9];
        for (int j = 0; j < 9; ++j) normal_pair(seed, (uint64_t)k, stream, (uint32_t)j, &a[j].re, &a[j].im);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                h[3 * i + j].re = 0.5 * (a[3 * i + j].re + a[3 * j + i].re);
                h[3 * i + j].im = 0.5 * (a[3 * i + j].im - a[3 * j + i].im);
            }
        double tr = (h[0].re + h[4].re + h[8].re) / 3.0;
        h[0].re -= tr; h[4].re -= tr; h[8].re -= tr;
        for (int j = 0; j < 9; ++j) { x[j].re = -eps * h[j].im; x[j].im = eps * h[j].re; }
        mat_exp(x, u);
        reunitarise(u);
        double* o = out + 18 * k;
        for (int j = 0; j < 9; ++j) { o[2 * j] = u[j].re; o[2 * j + 1] = u[j].im; }
    }
}
