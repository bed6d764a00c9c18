/*
 * FP64 CPU oracle for the Wilson-Dirac hopping term -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the GPU library and is deliberately
 * plain: one loop over sites, full 4x4 gamma matrices, full 3x3 links, complex
 * doubles, no spin projection, no link compression, no even-odd reordering.
 *
 * Definition (Wilson-Dirac operator, M = 1 - kappa * D_hop; the paper's
 * Section 4 "Wilson inverter" applies its parity-restricted form):
 *
 *   D_hop psi(x) = sum_mu [ (1 - g_mu) U_mu(x)        s+_mu(x) psi(x + mu)
 *                         + (1 + g_mu) U_mu(x - mu)^+  s-_mu(x) psi(x - mu) ]
 *
 * with s+_mu(x) = bc_mu when x_mu = L_mu - 1 (else 1) and s-_mu(x) = bc_mu when
 * x_mu = 0 (else 1).  The dagger operator swaps the two projectors:
 * (1 + g_mu) on the forward hop, (1 - g_mu) on the backward hop.
 *
 * Gamma matrices: DeGrand-Rossi basis, mu = x, y, z, t <-> gamma_1..gamma_4.
 *
 * Layouts (interleaved re, im doubles; lattice dims X, Y, Z, T):
 *   U   [4][T][Z][Y][X][3][3][2]   U_mu(x)[row][col]
 *   psi [T][Z][Y][X][4][3][2]      [spin][colour]
 * A site's parity is (x + y + z + t) & 1.  With out_parity = 0 or 1 only the
 * output sites of that parity are computed (the rest are set to zero): that is
 * P_out D_hop, the operator restricted to one parity.  out_parity = -1 computes
 * every site.
 *
 * Built with -DWREF_FP32 the same source runs in single precision (float
 * storage and arithmetic, interleaved re, im floats): that build is only timed,
 * as the CPU counterpart of a single-precision operator, and never checked
 * against.
 */
#include <complex.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef WREF_FP32
typedef float real;
typedef float complex cplx;
#define conj_c conjf
#else
typedef double real;
typedef double complex cplx;
#define conj_c conj
#endif

/* gamma[mu][row][col] in the DeGrand-Rossi basis. */
static const cplx GAMMA[4][4][4] = {
    { { 0, 0, 0, I }, { 0, 0, I, 0 }, { 0, -I, 0, 0 }, { -I, 0, 0, 0 } },
    { { 0, 0, 0, -1 }, { 0, 0, 1, 0 }, { 0, 1, 0, 0 }, { -1, 0, 0, 0 } },
    { { 0, 0, I, 0 }, { 0, 0, 0, -I }, { -I, 0, 0, 0 }, { 0, I, 0, 0 } },
    { { 0, 0, 1, 0 }, { 0, 0, 0, 1 }, { 1, 0, 0, 0 }, { 0, 1, 0, 0 } },
};

void wref_gamma(int mu, double* out /* [4][4][2] */)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            out[(4 * r + c) * 2] = creal(GAMMA[mu][r][c]);
            out[(4 * r + c) * 2 + 1] = cimag(GAMMA[mu][r][c]);
        }
}

static size_t site_index(const int L[4], const int c[4])
{
    return (size_t)c[0] + (size_t)L[0] * ((size_t)c[1] + (size_t)L[1] * ((size_t)c[2] + (size_t)L[2] * (size_t)c[3]));
}

/*
 * Adds  sign * (1 + pm * gamma_mu) W chi  into acc, where chi is the full
 * neighbour spinor and W the 3x3 colour matrix (already daggered if needed).
 */
static void add_hop(cplx acc[4][3], int mu, real pm, real sign, const cplx W[3][3], const cplx chi[4][3])
{
    cplx wchi[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx v = 0;
            for (int b = 0; b < 3; ++b) v += W[a][b] * chi[s][b];
            wchi[s][a] = v;
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx g = 0;
            for (int r = 0; r < 4; ++r) g += GAMMA[mu][s][r] * wchi[r][a];
            acc[s][a] += sign * (wchi[s][a] + pm * g);
        }
}

void wref_dhop(const int dims[4], const int bc[4], const real* U_, const real* in_, real* out_,
               int dagger, int out_parity)
{
    const cplx* U = (const cplx*)U_;
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    /* forward hop projector (1 - g) for D, (1 + g) for D^dagger; backward the opposite */
    const real pm_fwd = dagger ? 1 : -1;
    const real pm_bwd = -pm_fwd;

#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < (int64_t)V; ++s) {
        int c[4];
        size_t rem = (size_t)s;
        for (int d = 0; d < 4; ++d) { c[d] = (int)(rem % (size_t)dims[d]); rem /= (size_t)dims[d]; }
        cplx* o = out + 12 * (size_t)s;
        int parity = (c[0] + c[1] + c[2] + c[3]) & 1;
        if (out_parity >= 0 && parity != out_parity) {
            for (int k = 0; k < 12; ++k) o[k] = 0;
            continue;
        }
        cplx acc[4][3] = { { 0 } };
        for (int mu = 0; mu < 4; ++mu) {
            int f[4] = { c[0], c[1], c[2], c[3] };
            int b[4] = { c[0], c[1], c[2], c[3] };
            real sf = 1, sb = 1;
            f[mu] = c[mu] + 1;
            if (f[mu] == dims[mu]) { f[mu] = 0; sf = (real)bc[mu]; }
            b[mu] = c[mu] - 1;
            if (b[mu] < 0) { b[mu] = dims[mu] - 1; sb = (real)bc[mu]; }
            size_t xf = site_index(dims, f), xb = site_index(dims, b);

            cplx W[3][3], chi[4][3];
            /* forward: U_mu(x) psi(x + mu) */
            const cplx* Uf = U + 9 * ((size_t)mu * V + (size_t)s);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) W[i][j] = Uf[3 * i + j];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) chi[sp][a] = in[12 * xf + 3 * sp + a];
            add_hop(acc, mu, pm_fwd, sf, W, chi);
            /* backward: U_mu(x - mu)^dagger psi(x - mu) */
            const cplx* Ub = U + 9 * ((size_t)mu * V + xb);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) W[i][j] = conj_c(Ub[3 * j + i]);
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) chi[sp][a] = in[12 * xb + 3 * sp + a];
            add_hop(acc, mu, pm_bwd, sb, W, chi);
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) o[3 * sp + a] = acc[sp][a];
    }
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int wref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
