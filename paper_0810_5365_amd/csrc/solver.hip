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
    const void* c;       // right-hand side of A x = c (float64); null for the Wilson system
    const void* bhat;    // the Wilson system on one parity: A x = Mhat^dag bhat, with the residual
                         // ||bhat - Mhat x|| tracked as well
    double wnorm2;       // reference norm^2 for the Wilson-system residual
};

// General system: r = c - A x in float64 with rr = ||r||^2 (four float64 launches), then rs = r
// at the accumulation precision.
static wd_status residual_general(const CGProblem& P, int pacc, const void* x, void* r, void* rs, double* rr)
{
    wd_context ctx = P.g->ctx;
    const Geom& G = P.g->geom;
    const size_t nh = halves_of(P.subset, 1);
    void* t1;
    WD_TRY(ws_get(ctx, "cg.t1", half_bytes(G, WD_F64) * nh, &t1));
    WD_TRY(op_M(P.g, P.kappa, P.subset, 0, WD_F64, 1, x, t1));
    WD_TRY(op_M_red(P.g, P.kappa, P.subset, 1, WD_F64, t1, r, RED_RESID, P.c, 0));
    WD_TRY(fetch_results(ctx, 1));
    *rr = ctx->hres[0];
    return launch_convert(ctx, G, nh, WD_F64, r, pacc, rs);
}

// Wilson system: t = bhat - Mhat x in float64, kept at the accumulation precision, with ww =
// ||t||^2 (two float64 launches; D_oe x stays in doe), then rs = Mhat^dag t with rr = ||rs||^2 at
// that precision.  Mhat^dag (bhat - Mhat x) is the normal-equation residual c - A x: the
// cancellation happens in the float64 difference, and the operator applied to that small vector
// only needs the precision rs is kept in.  With x_zero the first step is a conversion of bhat.
// need_rs: RS_ALWAYS queues both parts before waiting; RS_UNLESS_DONE reads ww first and skips
// rs when ww <= stop_w (the solve ends there); RS_NEVER computes ww only.  *rs_done tells whether
// rs and rr were formed.
enum { RS_ALWAYS, RS_UNLESS_DONE, RS_NEVER };
static wd_status residual_wilson(const CGProblem& P, int pacc, const void* x, bool x_zero, void* rs, void* doe,
                                 double* rr, double* ww, int need_rs, double stop_w, bool* rs_done)
{
    wd_context ctx = P.g->ctx;
    const Geom& G = P.g->geom;
    void* t;
    WD_TRY(ws_get(ctx, "cg.t", half_bytes(G, pacc), &t));
    *rs_done = false;
    if (x_zero) {
        WD_TRY(launch_convert(ctx, G, 1, WD_F64, P.bhat, pacc, t));
        WD_TRY(blas_norm2(ctx, G, 1, WD_F64, P.bhat, true));   // slot 0
    } else {
        WD_TRY(op_M_red(P.g, P.kappa, P.subset, 0, WD_F64, x, t, pacc == WD_F64 ? RED_RESID : RED_RESLO, P.bhat, 0,
                        doe));
        if (need_rs != RS_ALWAYS) {
            WD_TRY(fetch_results(ctx, 1));
            *ww = ctx->hres[0];
            if (need_rs == RS_NEVER || *ww <= stop_w) return WD_OK;
        }
    }
    WD_TRY(op_M_red(P.g, P.kappa, P.subset, 1, pacc, t, rs, RED_NORM, nullptr, 1));
    WD_TRY(fetch_results(ctx, 2));
    *ww = ctx->hres[0];
    *rr = ctx->hres[1];
    *rs_done = true;
    return WD_OK;
}

// One iteration keeps its scalars on the device (dres[CG_SLOT ..]):
//   mp = M p, pap = ||M p||^2 = <p, A p>, alpha = rr / pap     (two launches and a sum)
//   r -= alpha M^dag mp, rr_new = ||r||^2, beta = rr_new / rr  (two launches and a sum; A p is
//                                                              never stored)
//   xs += alpha p and p' = r + beta p                          (one sweep, into the other p buffer)
// The sweep is queued before the host looks at pap and rr_new (which the sums write straight
// into mapped host memory), so the host's wait overlaps it and the next iteration is queued
// behind it.  When rr_new calls for a reliable update, xs
// already holds alpha p: x += xs in float64, the residual is recomputed from x and p' is formed
// again from the old p (still in its buffer) with beta = rr / rr_s.
// doe_xe (Wilson system, may be null): set to a float64 half field holding D_oe x for the x
// returned, when one is at hand, else to null; *schur_rr then holds ||bhat - Mhat x||^2 of that
// same evaluation.
static wd_status cg_run(const CGProblem& P, const wd_solver_params& prm, void* x, wd_solver_info* info,
                        const void** doe_xe = nullptr, double* schur_rr = nullptr)
{
    wd_context ctx = P.g->ctx;
    const Geom& G = P.g->geom;
    const int pop = prm.sloppy;
    const int pacc = pop == WD_F64 ? WD_F64 : WD_F32;
    const size_t nh = halves_of(P.subset, 1);
    const bool pure = prm.pure_sloppy != 0;
    const bool wilson = P.bhat != nullptr;
    const double delta = resolve_delta(prm.delta, pop);
    const bool use_delta = pop != WD_F64 && delta > 0.0;

    void *r = nullptr, *rs, *xs, *pa, *pb, *mp;
    if (!wilson) WD_TRY(ws_get(ctx, "cg.r", half_bytes(G, WD_F64) * nh, &r));
    WD_TRY(ws_get(ctx, "cg.rs", half_bytes(G, pacc) * nh, &rs));
    WD_TRY(ws_get(ctx, "cg.xs", half_bytes(G, pacc) * nh, &xs));
    WD_TRY(ws_get(ctx, "cg.p", half_bytes(G, pop) * nh, &pa));
    WD_TRY(ws_get(ctx, "cg.p2", half_bytes(G, pop) * nh, &pb));
    WD_TRY(ws_get(ctx, "cg.mp", half_bytes(G, pop) * nh, &mp));
    void* doe = nullptr;
    if (wilson) WD_TRY(ws_get(ctx, "cg.doe", half_bytes(G, WD_F64), &doe));
    bool doe_at_x = false;   // doe holds D_oe x for the current x
    if (doe_xe) *doe_xe = nullptr;
    *info = wd_solver_info{};
    std::vector<double> alphas, betas;   // for the Ritz-value estimates

    // cc = ||c||^2; for the Wilson system c = Mhat^dag bhat is formed at the accumulation
    // precision (into rs: with a zero guess it is the first residual)
    const bool x_zero = is_zero_f64(ctx, G, nh, x);
    double cc, rr = 0.0, ww = -1.0;
    if (wilson) {
        bool rs_done;
        WD_TRY(residual_wilson(P, pacc, nullptr, true, rs, doe, &cc, &ww, RS_ALWAYS, 0.0, &rs_done));
        if (!std::isfinite(ww)) cc = ww;
    } else {
        WD_TRY(blas_norm2(ctx, G, nh, WD_F64, P.c, true));
        cc = ctx->hres[0];
    }
    const double tol2 = prm.tol * prm.tol;
    const double target_r = tol2 * cc;
    const double target_w = tol2 * P.wnorm2;
    if (!std::isfinite(cc)) {   // NaN or Inf in the source: x is left as it was
        set_error("CG: the right-hand side holds NaN or Inf");
        info->true_resid = cc;
        info->true_resid_M = wilson ? cc : -1.0;
        info->status = WD_ENAN;
        return WD_ENAN;
    }
    if (!(cc > 0.0)) {
        WD_TRY(blas_zero(ctx, G, nh, WD_F64, x));
        info->true_resid = 0.0;
        info->true_resid_M = wilson ? 0.0 : -1.0;
        info->status = WD_OK;
        return WD_OK;
    }

    // residual of the current x into rs (with rr, and ww for the Wilson system); for the Wilson
    // system need_rs says when rs may be left out (see residual_wilson)
    auto residual = [&](int need_rs) -> wd_status {
        if (!wilson) return residual_general(P, pacc, x, r, rs, &rr);
        bool rs_done;
        WD_TRY(residual_wilson(P, pacc, x, false, rs, doe, &rr, &ww, need_rs, target_w, &rs_done));
        doe_at_x = true;
        return WD_OK;
    };
    if (x_zero) {   // the residual is c itself, already at hand
        rr = cc;
        if (!wilson) WD_TRY(launch_convert(ctx, G, nh, WD_F64, P.c, pacc, rs));
    } else {
        WD_TRY(residual(RS_ALWAYS));
        info->operator_applies++;
    }
    auto converged = [&]() { return wilson ? ww <= target_w : rr <= target_r; };
    wd_status status = WD_ENOCONV;
    if (converged()) status = WD_OK;

    // sloppy residual level that triggers a float64 check of convergence
    double trigger = wilson ? (ww > 0 ? rr / ww : 1.0) * target_w : target_r;
    bool xs_live = false;   // xs holds a part of the solution not yet in x
    bool stale = false;     // x (with xs) has changed since rr, ww were computed
    if (status != WD_OK) {
        void* p = pa;    // the search direction of this iteration
        void* pn = pb;   // the next one
        WD_TRY(launch_convert(ctx, G, nh, pacc, rs, pop, p));
        WD_TRY(blas_cg_set(ctx, rr, 0.0));
        double rr_s = rr, maxrr = rr;
        const double* dalpha = ctx->dres + CG_SLOT + CG_ALPHA;   // read by the launch that updates r
        while (info->iters < prm.maxiter) {
            int n = 0;
            blas_cg_arm(ctx);
            WD_TRY(op_M_red_partials(P.g, P.kappa, P.subset, 0, pop, p, mp, RED_NORM, nullptr, nullptr, &n));
            WD_TRY(blas_cg_coef(ctx, n, 0));
            WD_TRY(op_M_red_partials(P.g, P.kappa, P.subset, 1, pop, mp, rs, RED_CGR, nullptr, dalpha, &n));
            WD_TRY(blas_cg_coef(ctx, n, 1));
            WD_TRY(blas_cg_xp(ctx, G, nh, pacc, xs, xs_live ? 0 : 1, rs, pop, p, pn));
            WD_TRY(blas_cg_wait(ctx));
            info->operator_applies++;
            const double pap = ctx->hres[CG_SLOT + CG_PAP];
            if (!std::isfinite(pap) || !(pap > 0.0)) {   // rs and xs are spoilt; x holds the last update
                set_error("CG breakdown: <p, A p> = %g at iteration %d", pap, info->iters);
                status = WD_ENAN;
                xs_live = false;
                break;
            }
            alphas.push_back(rr_s / pap);
            double rr_new = ctx->hres[CG_SLOT + CG_RRNEW];
            info->iters++;
            xs_live = true;
            stale = true;
            if (!std::isfinite(rr_new)) {
                set_error("CG: non-finite residual at iteration %d", info->iters);
                status = WD_ENAN;
                xs_live = false;
                break;
            }
            const bool done_sloppy = pure && rr_new <= trigger;
            const bool reliable = !pure && ((use_delta && rr_new < delta * delta * maxrr) || rr_new <= trigger);
            if (done_sloppy || reliable) {
                WD_TRY(blas_axpby(ctx, G, nh, pacc, xs, 1.0, WD_F64, x, 1.0));
                xs_live = false;
                doe_at_x = false;
                if (done_sloppy) break;
                // reliable update: the residual recomputed from x, the recurrence restarted from it;
                // when the sloppy residual says the target is reached, the float64 norm is read
                // before the rest is queued, which a converged solve no longer needs
                WD_TRY(residual(rr_new <= trigger ? RS_UNLESS_DONE : RS_ALWAYS));
                stale = false;
                info->operator_applies++;
                info->reliable_updates++;
                if (converged()) {
                    status = WD_OK;
                    break;
                }
                if (wilson && ww > 0) trigger = rr / ww * target_w;
                rr_new = rr;
                maxrr = rr;
                const double beta = rr_new / rr_s;
                betas.push_back(beta);
                WD_TRY(blas_cg_set(ctx, rr_new, beta));
                WD_TRY(blas_cg_xp(ctx, G, nh, pacc, xs, 2, rs, pop, p, pn));
            } else {
                if (rr_new > maxrr) maxrr = rr_new;
                betas.push_back(rr_new / rr_s);
            }
            std::swap(p, pn);
            rr_s = rr_new;
        }
    }
    if (xs_live) {
        WD_TRY(blas_axpby(ctx, G, nh, pacc, xs, 1.0, WD_F64, x, 1.0));
        doe_at_x = false;
    }
    if (stale) {   // else rr, ww are those of the last reliable update, already of this x
        WD_TRY(residual(RS_NEVER));
        info->operator_applies++;
    }
    // the Wilson system reports the float64 residual its convergence test uses,
    // ||bhat - Mhat x|| / ||b||; the general system ||c - A x|| / ||c||
    info->true_resid = wilson ? std::sqrt(ww / P.wnorm2) : std::sqrt(rr / cc);
    info->true_resid_M = wilson ? std::sqrt(ww / P.wnorm2) : -1.0;
    if (doe_xe && schur_rr && wilson && doe_at_x) {
        *doe_xe = doe;
        *schur_rr = ww;
    }
    if (status != WD_ENAN) cg_ritz_extremes(alphas, betas, &info->lambda_min, &info->lambda_max);
    if (status != WD_ENAN) status = converged() ? WD_OK : WD_ENOCONV;
    if (status == WD_ENOCONV)
        set_error("CG did not reach tol %g in %d iterations (residual %g)", prm.tol, info->iters,
                  wilson ? info->true_resid_M : info->true_resid);
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
    HopTally tally(g->ctx, info);
    const auto t0 = std::chrono::steady_clock::now();
    CGProblem P{g, kappa, (int)subset, b, nullptr, 0.0};
    wd_status s = cg_run(P, *params, x, info);
    hipStreamSynchronize(g->ctx->stream);   // synchronous: nothing of the solve left queued
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
    HopTally tally(ctx, info);
    const auto t0 = std::chrono::steady_clock::now();
    const long long hb = (long long)half_bytes(G, WD_F64);
    const char* b_e = (const char*)b;
    const char* b_o = b_e + hb;
    char* x_e = (char*)x;
    void* bhat;
    WD_TRY(ws_get(ctx, "wilson.bhat", hb, &bhat));
    // bhat = b_e + kappa D_eo b_o; CG solves Mhat^dagger Mhat x_e = Mhat^dagger bhat
    WD_TRY(hop_half(g, WD_F64, 0, 0, 1, b_o, hb, bhat, hb, b_e, hb, 1.0, kappa));
    WD_TRY(blas_norm2(ctx, G, 2, WD_F64, b, true));
    const double bb = ctx->hres[0];
    CGProblem P{g, kappa, WD_EVEN, nullptr, bhat, bb};
    const void* doe_xe = nullptr;   // D_oe x_e from the last float64 residual, if at hand
    double schur_rr = 0.0;          // and that residual's norm^2
    wd_status s = cg_run(P, *params, x_e, info, &doe_xe, &schur_rr);
    if (s != WD_OK && s != WD_ENOCONV) return s;
    // x_o, then the full-system residual in float64
    double rr;
    WD_TRY(eo_finish(g, kappa, b, x, &rr, doe_xe, schur_rr));
    info->true_resid_M = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (!doe_xe) info->operator_applies++;   // the closing float64 check applied the operator
    hipStreamSynchronize(g->ctx->stream);   // synchronous: nothing of the solve left queued
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

} // extern "C"
