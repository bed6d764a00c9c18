// Temporal gauge fixing (paper Sections 4 and 7): a gauge rotation Omega with
// Omega(x, 0) = 1 and Omega(x, t + 1) = Omega(x, t) U_t(x, t) makes every
// time-direction link the identity except those leaving the last time slice:
//     U'_mu(x) = Omega(x) U_mu(x) Omega(x + mu)^dagger,
//     U'_t(x, t) = 1 for t < T - 1,  U'_t(x, T - 1) = Omega(x, T - 1) U_t(x, T - 1).
// The Wilson operator is gauge covariant, M[U'] (Omega psi) = Omega M[U] psi, so
// solves in the fixed gauge return Omega x.  The dslash then skips the unit
// t-links (576 -> 480 algorithmic bytes per site in FP32 with 12-real links).
// The rotation is a sequential product along t, done once on the host.
#include <string.h>

#include <vector>

#include "wd_core.h"

namespace wd {

typedef double C2[2];

static inline void mmul(const double* a, const double* b, double* c)   // c = a b (3x3 complex)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
            for (int k = 0; k < 3; ++k) {
                const double* x = a + 2 * (3 * i + k);
                const double* y = b + 2 * (3 * k + j);
                re += x[0] * y[0] - x[1] * y[1];
                im += x[0] * y[1] + x[1] * y[0];
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

static inline void mmul_dag(const double* a, const double* b, double* c)   // c = a b^dagger
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
            for (int k = 0; k < 3; ++k) {
                const double* x = a + 2 * (3 * i + k);
                const double* y = b + 2 * (3 * j + k);
                re += x[0] * y[0] + x[1] * y[1];
                im += x[1] * y[0] - x[0] * y[1];
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

} // namespace wd

using namespace wd;

extern "C" wd_status wd_gauge_fix_temporal(wd_gauge g, double* omega_out)
{
    if (!g) {
        set_error("wd_gauge_fix_temporal: gauge is NULL");
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    const int X = g->geom.L[0], Y = g->geom.L[1], Z = g->geom.L[2], T = g->geom.L[3];
    const size_t V = (size_t)X * Y * Z * T;
    const size_t n = V * 4 * 18;
    std::vector<double> U(n), Om(V * 18);
    WD_HIP(hipSetDevice(g->ctx->device));
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    WD_HIP(hipMemcpy(U.data(), g->canon, n * sizeof(double), hipMemcpyDeviceToHost));
    const size_t S = (size_t)X * Y * Z;   // sites per time slice
    auto lex = [&](size_t s, int t) { return s + S * (size_t)t; };
    // Omega along t, for every spatial site
    for (size_t s = 0; s < S; ++s) {
        double* o0 = &Om[18 * lex(s, 0)];
        memset(o0, 0, 18 * sizeof(double));
        o0[0] = o0[8] = o0[16] = 1.0;
        for (int t = 0; t + 1 < T; ++t)
            mmul(&Om[18 * lex(s, t)], &U[18 * (3 * V + lex(s, t))], &Om[18 * lex(s, t + 1)]);
    }
    // U'_mu(x) = Omega(x) U_mu(x) Omega(x + mu)^dagger
    std::vector<double> tmp(18);
    for (size_t x = 0; x < V; ++x) {
        const int c0 = (int)(x % X), c1 = (int)(x / X % Y), c2 = (int)(x / ((size_t)X * Y) % Z),
                  c3 = (int)(x / S);
        for (int mu = 0; mu < 4; ++mu) {
            int c[4] = {c0, c1, c2, c3};
            c[mu] = (c[mu] + 1) % g->geom.L[mu];
            const size_t xf = (size_t)c[0] + X * ((size_t)c[1] + Y * ((size_t)c[2] + (size_t)Z * c[3]));
            double* u = &U[18 * ((size_t)mu * V + x)];
            if (mu == 3 && c3 + 1 < T) {
                memset(u, 0, 18 * sizeof(double));
                u[0] = u[8] = u[16] = 1.0;   // exactly the identity
                continue;
            }
            mmul(&Om[18 * x], u, tmp.data());
            mmul_dag(tmp.data(), &Om[18 * xf], u);
        }
    }
    WD_HIP(hipMemcpy(g->canon, U.data(), n * sizeof(double), hipMemcpyHostToDevice));
    for (int p = 0; p < 4; ++p)
        if (g->packed[p]) WD_TRY(launch_pack_gauge(g->ctx, g->geom, p, g->recon, g->canon, g->packed[p]));
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    g->gf = true;
    if (omega_out) memcpy(omega_out, Om.data(), Om.size() * sizeof(double));
    return WD_OK;
}
