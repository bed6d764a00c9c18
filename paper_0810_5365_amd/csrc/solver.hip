// Conjugate gradient on the normal equations (paper Section 4: even-odd
// preconditioned CG, every step a separate kernel, global sums in double
// precision, the fields never leaving the device) with mixed precision:
// the iterations run in a "sloppy" storage precision and the solution is
// accumulated in float64 through reliable updates, each of which recomputes
// the true residual b - A x in float64 (Sleijpen and van der Vorst's
// reliable-update scheme).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "wd_ops.h"

namespace wd {

// Number of eigenvalues below x of the symmetric tridiagonal matrix with diagonal
// d[0..n) and off-diagonal e[0..n-1), by the signs of the pivots of T - x
// (Sturm sequence count).
static int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x)
{
    int neg = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); i++) {
        q = d[i] - x - (i ? e[i - 1] * e[i - 1] / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) neg++;
    }
    return neg;
}

// Extreme eigenvalues of the Lanczos tridiagonal that CG builds implicitly from its
// step lengths alpha_j and ratios beta_j = |r_{j+1}|^2 / |r_j|^2: diagonal
// 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j.  Their
// eigenvalues (Ritz values) approach the ends of the spectrum of the solved operator
// as the iteration proceeds.  Bisection on the Sturm count to relative 1e-13.
static void cg_ritz_extremes(const std::vector<double>& alpha, const std::vector<double>& beta, double* lo,
                             double* hi)
{
    const size_t n = alpha.size();
    *lo = *hi = 0.0;
    if (n == 0) return;
    std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
    for (size_t j = 0; j < n; j++) {
        d[j] = 1.0 / alpha[j] + (j ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j + 1 < n) e[j] = std::sqrt(beta[j]) / alpha[j];
    }
    double a = d[0], b = d[0];   // Gershgorin interval
    for (size_t j = 0; j < n; j++) {
        const double r = (j ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < n ? std::fabs(e[j]) : 0.0);
        a = std::min(a, d[j] - r);
        b = std::max(b, d[j] + r);
    }
    auto kth = [&](int k) {   // the (k+1)-th smallest eigenvalue
        double l = a, u = b;
        for (int it = 0; it < 200 && u - l > 1e-13 * std::max(std::fabs(l), std::fabs(u)); it++) {
            const double m = 0.5 * (l + u);
            if (sturm_count(d, e, m) > k) u = m; else l = m;
        }
        return 0.5 * (l + u);
    };
    *lo = kth(0);
    *hi = kth((int)n - 1);
}

struct CGProblem {
    wd_gauge g;
    double kappa;
    int subset;
    const void* c;       // right-hand side of A x = c (float64)
    const void* bhat;    // non-null: also track ||bhat - Mhat x|| (Wilson-system residual)
    double wnorm2;       // reference norm^2 for the Wilson-system residual
};

// r = c - A x in float64; ww = ||bhat - Mhat x||^2 when tracked.
static wd_status true_residual(const CGProblem& P, const void* x, void* r, double* rr, double* ww)
{
    wd_context ctx = P.g->ctx;
    const Geom& G = P.g->geom;
    const size_t nh = halves_of(P.subset, 1);
    const size_t bytes = half_bytes(G, WD_F64) * nh;
    void* t1;
    WD_TRY(ws_get(ctx, "cg.t1", bytes, &t1));
    // t1 = M x (with ||bhat - t1||^2 when tracked), then r = c - M^dag t1 with ||r||^2, each
    // difference and norm taken by the launch that produces the operator's result
    if (P.bhat) WD_TRY(op_M_red(P.g, P.kappa, P.subset, 0, WD_F64, x, t1, RED_YDIFF, P.bhat, 1));
    else WD_TRY(op_M(P.g, P.kappa, P.subset, 0, WD_F64, 1, x, t1));
    WD_TRY(op_M_red(P.g, P.kappa, P.subset, 1, WD_F64, t1, r, RED_RESID, P.c, 0));
    WD_TRY(fetch_results(ctx, 2));
    *rr = ctx->hres[0];
    *ww = P.bhat ? ctx->hres[1] : -1.0;
    return WD_OK;
}

static wd_status cg_run(const CGProblem& P, const wd_solver_params& prm, void* x, wd_solver_info* info)
{
    wd_context ctx = P.g->ctx;
    const Geom& G = P.g->geom;
    const int pop = prm.sloppy;
    const int pacc = pop == WD_F64 ? WD_F64 : WD_F32;
    const size_t nh = halves_of(P.subset, 1);
    const bool pure = prm.pure_sloppy != 0;
    const double delta = resolve_delta(prm.delta, pop);
    const bool use_delta = pop != WD_F64 && delta > 0.0;

    void *r, *rs, *xs, *p, *ap, *mp;
    WD_TRY(ws_get(ctx, "cg.r", half_bytes(G, WD_F64) * nh, &r));
    WD_TRY(ws_get(ctx, "cg.rs", half_bytes(G, pacc) * nh, &rs));
    WD_TRY(ws_get(ctx, "cg.xs", half_bytes(G, pacc) * nh, &xs));
    WD_TRY(ws_get(ctx, "cg.p", half_bytes(G, pop) * nh, &p));
    // on one parity A p = Mhat^dag (Mhat p) is formed in place of Mhat p (the fused update of
    // Mhat^dag reads x at the site it writes), so the iteration touches one field fewer and
    // more of its fields stay in the last-level cache; on the full lattice it cannot be
    if (P.subset == WD_FULL) WD_TRY(ws_get(ctx, "cg.ap", half_bytes(G, pop) * nh, &ap));
    WD_TRY(ws_get(ctx, "cg.mp", half_bytes(G, pop) * nh, &mp));
    if (P.subset != WD_FULL) ap = mp;

    WD_TRY(blas_norm2(ctx, G, nh, WD_F64, P.c, true));
    const double cc = ctx->hres[0];
    const double tol2 = prm.tol * prm.tol;
    const double target_r = tol2 * cc;
    const double target_w = tol2 * P.wnorm2;
    *info = wd_solver_info{};
    std::vector<double> alphas, betas;   // for the Ritz-value estimates
    if (!std::isfinite(cc)) {   // NaN or Inf in the source: x is left as it was
        set_error("CG: the right-hand side holds NaN or Inf");
        info->true_resid = cc;
        info->true_resid_M = P.bhat ? cc : -1.0;
        info->status = WD_ENAN;
        return WD_ENAN;
    }
    if (!(cc > 0.0)) {
        WD_TRY(blas_zero(ctx, G, nh, WD_F64, x));
        info->true_resid = 0.0;
        info->true_resid_M = P.bhat ? 0.0 : -1.0;
        info->status = WD_OK;
        return WD_OK;
    }

    double rr, ww;
    if (is_zero_f64(ctx, G, nh, x)) {   // zero guess: r = c and bhat - Mhat x = bhat, without the operator
        WD_TRY(launch_convert(ctx, G, nh, WD_F64, P.c, WD_F64, r));
        rr = cc;
        ww = -1.0;
        if (P.bhat) {
            WD_TRY(blas_norm2(ctx, G, nh, WD_F64, P.bhat, true));
            ww = ctx->hres[0];
        }
    } else {
        WD_TRY(true_residual(P, x, r, &rr, &ww));
        info->operator_applies++;
    }
    auto converged = [&]() { return P.bhat ? ww <= target_w : rr <= target_r; };
    wd_status status = WD_ENOCONV;
    if (converged()) status = WD_OK;

    // sloppy residual level that triggers a float64 check of convergence
    double trigger = P.bhat ? (ww > 0 ? rr / ww : 1.0) * target_w : target_r;
    bool xs_dirty = false;
    if (status != WD_OK) {
        WD_TRY(launch_convert(ctx, G, nh, WD_F64, r, pacc, rs));
        WD_TRY(launch_convert(ctx, G, nh, WD_F64, r, pop, p));
        WD_TRY(blas_zero(ctx, G, nh, pacc, xs));
        double rr_s = rr, maxrr = rr;
        while (info->iters < prm.maxiter) {
            // A p = M^dag (M p), and <p, A p> = ||M p||^2 summed by the kernel that writes M p
            WD_TRY(op_M_red(P.g, P.kappa, P.subset, 0, pop, p, mp, RED_NORM, nullptr, 0));
            WD_TRY(op_M(P.g, P.kappa, P.subset, 1, pop, 1, mp, ap));
            WD_TRY(fetch_results(ctx, 1));
            info->operator_applies++;
            const double pap = ctx->hres[0];
            if (!std::isfinite(pap) || !(pap > 0.0)) {
                set_error("CG breakdown: <p, A p> = %g at iteration %d", pap, info->iters);
                status = WD_ENAN;
                break;
            }
            const double alpha = rr_s / pap;
            alphas.push_back(alpha);
            WD_TRY(blas_cg_xr(ctx, G, nh, pacc, xs, rs, pop, p, ap, alpha, true));
            xs_dirty = true;
            double rr_new = ctx->hres[0];
            info->iters++;
            if (!std::isfinite(rr_new)) {
                set_error("CG: non-finite residual at iteration %d", info->iters);
                status = WD_ENAN;
                break;
            }
            if (pure) {
                if (rr_new <= trigger) break;
            } else if ((use_delta && rr_new < delta * delta * maxrr) || rr_new <= trigger) {
                // reliable update: fold the sloppy solution into x and recompute r in float64
                WD_TRY(blas_axpby(ctx, G, nh, pacc, xs, 1.0, WD_F64, x, 1.0));
                WD_TRY(blas_zero(ctx, G, nh, pacc, xs));
                xs_dirty = false;
                WD_TRY(true_residual(P, x, r, &rr, &ww));
                info->operator_applies++;
                info->reliable_updates++;
                if (converged()) {
                    status = WD_OK;
                    break;
                }
                if (P.bhat && ww > 0) trigger = rr / ww * target_w;
                WD_TRY(launch_convert(ctx, G, nh, WD_F64, r, pacc, rs));
                rr_new = rr;
                maxrr = rr;
            }
            if (rr_new > maxrr) maxrr = rr_new;
            const double beta = rr_new / rr_s;
            betas.push_back(beta);
            WD_TRY(blas_cg_p(ctx, G, nh, pacc, rs, pop, p, beta));
            rr_s = rr_new;
        }
    }
    if (xs_dirty) {   // else rr, ww are those of the last reliable update, already of this x
        WD_TRY(blas_axpby(ctx, G, nh, pacc, xs, 1.0, WD_F64, x, 1.0));
        WD_TRY(true_residual(P, x, r, &rr, &ww));
        info->operator_applies++;
    }
    info->true_resid = std::sqrt(rr / cc);
    info->true_resid_M = P.bhat ? std::sqrt(ww / P.wnorm2) : -1.0;
    if (status != WD_ENAN) cg_ritz_extremes(alphas, betas, &info->lambda_min, &info->lambda_max);
    if (status != WD_ENAN) status = converged() ? WD_OK : WD_ENOCONV;
    if (status == WD_ENOCONV)
        set_error("CG did not reach tol %g in %d iterations (residual %g)", prm.tol, info->iters,
                  P.bhat ? info->true_resid_M : info->true_resid);
    info->status = status;
    return status;
}

static wd_status check_params(const wd_solver_params* prm)
{
    if (!prm) {
        set_error("solver params are NULL");
        return WD_EINVAL;
    }
    if (!(prm->tol > 0.0) || prm->maxiter < 0 || !valid_prec(prm->sloppy) || !(prm->delta < 1.0)) {
        set_error("bad solver params: tol %g, maxiter %d, sloppy %d, delta %g", prm->tol, prm->maxiter, prm->sloppy,
                  prm->delta);
        return WD_EINVAL;
    }
    return WD_OK;
}

} // namespace wd

using namespace wd;

extern "C" {

wd_status wd_cg_solve(wd_gauge g, double kappa, wd_subset subset, const wd_solver_params* params, const void* b,
                      void* x, wd_solver_info* info)
{
    if (!g || !b || !x || !info) {
        set_error("wd_cg_solve: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(check_params(params));
    if (!valid_subset(subset)) {
        set_error("wd_cg_solve: bad subset %d", (int)subset);
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    const auto t0 = std::chrono::steady_clock::now();
    CGProblem P{g, kappa, (int)subset, b, nullptr, 0.0};
    wd_status s = cg_run(P, *params, x, info);
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

wd_status wd_wilson_solve(wd_gauge g, double kappa, const wd_solver_params* params, const void* b, void* x,
                          wd_solver_info* info)
{
    if (!g || !b || !x || !info) {
        set_error("wd_wilson_solve: NULL argument");
        return WD_EINVAL;
    }
    WD_TRY(check_params(params));
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    WD_HIP(hipStreamSynchronize(ctx->stream));
    const auto t0 = std::chrono::steady_clock::now();
    const long long hb = (long long)half_bytes(G, WD_F64);
    const char* b_e = (const char*)b;
    const char* b_o = b_e + hb;
    char* x_e = (char*)x;
    char* x_o = x_e + hb;
    void *bhat, *c;
    WD_TRY(ws_get(ctx, "wilson.bhat", hb, &bhat));
    WD_TRY(ws_get(ctx, "wilson.c", hb, &c));
    // bhat = b_e + kappa D_eo b_o ; c = Mhat^dagger bhat
    WD_TRY(hop_half(g, WD_F64, 0, 0, 1, b_o, hb, bhat, hb, b_e, hb, 1.0, kappa));
    WD_TRY(op_M(g, kappa, WD_EVEN, 1, WD_F64, 1, bhat, c));
    WD_TRY(blas_norm2(ctx, G, 2, WD_F64, b, true));
    const double bb = ctx->hres[0];
    CGProblem P{g, kappa, WD_EVEN, c, bhat, bb};
    wd_status s = cg_run(P, *params, x_e, info);
    if (s != WD_OK && s != WD_ENOCONV) return s;
    // x_o = b_o + kappa D_oe x_e ; then the full-system residual in float64
    WD_TRY(hop_half(g, WD_F64, 1, 0, 1, x_e, hb, x_o, hb, b_o, hb, 1.0, kappa));
    void* r;
    WD_TRY(ws_get(ctx, "wilson.r", 2 * hb, &r));
    WD_TRY(op_M_red(g, kappa, WD_FULL, 0, WD_F64, x, r, RED_RESID, b, 0));   // r = b - M x, ||r||^2
    WD_TRY(fetch_results(ctx, 1));
    info->true_resid_M = bb > 0 ? std::sqrt(ctx->hres[0] / bb) : 0.0;
    info->operator_applies++;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

} // extern "C"
