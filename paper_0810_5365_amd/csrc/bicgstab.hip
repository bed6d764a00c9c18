// BiCGstab (van der Vorst 1992) on the even-odd Schur system Mhat x_e = bhat_e
// (the paper's second inverter, Section 7), with the same mixed-precision
// scheme as the CG: iterations in float32 or float64 storage and arithmetic,
// solution accumulated in float64 through reliable updates that recompute
// r = bhat - Mhat x in float64; the final residual is that of the full system.
#include <chrono>
#include <cmath>
#include <complex>

#include "wd_ops.h"

namespace wd {

typedef std::complex<double> cd;

// doe_xe: set to a float64 half field holding D_oe x for the x returned, when one is at hand,
// else to null; *schur_rr then holds ||bhat - Mhat x||^2 of that same evaluation.
static wd_status bicgstab_run(wd_gauge g, double kappa, const wd_solver_params& prm, const void* bhat, double bnorm2,
                              void* x, wd_solver_info* info, const void** doe_xe, double* schur_rr)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    const int ps = prm.sloppy;   // storage of the iteration's vectors; arithmetic in float32 (float64 for F64)
    const double delta = resolve_delta(prm.delta, ps);
    const size_t hs = half_bytes(G, ps), h64 = half_bytes(G, WD_F64);
    void *r, *rs, *r0, *p, *v, *s, *t, *xs;
    WD_TRY(ws_get(ctx, "bicg.r", h64, &r));
    WD_TRY(ws_get(ctx, "bicg.rs", hs, &rs));
    WD_TRY(ws_get(ctx, "bicg.r0", hs, &r0));
    WD_TRY(ws_get(ctx, "bicg.p", hs, &p));
    WD_TRY(ws_get(ctx, "bicg.v", hs, &v));
    WD_TRY(ws_get(ctx, "bicg.s", hs, &s));
    WD_TRY(ws_get(ctx, "bicg.t", hs, &t));
    WD_TRY(ws_get(ctx, "bicg.xs", hs, &xs));
    void* doe;
    WD_TRY(ws_get(ctx, "bicg.doe", h64, &doe));
    bool doe_at_x = false;   // doe holds D_oe x for the current x
    *doe_xe = nullptr;
    const double target = prm.tol * prm.tol * bnorm2;
    auto true_res = [&](double* rr) -> wd_status {
        // r = bhat - Mhat x, ||r||^2; D_oe x stays in doe
        WD_TRY(op_M_red(g, kappa, WD_EVEN, 0, WD_F64, x, r, RED_RESID, bhat, 0, doe));
        WD_TRY(fetch_results(ctx, 1));
        *rr = ctx->hres[0];
        info->operator_applies++;
        doe_at_x = true;
        return WD_OK;
    };
    auto dot = [&](const void* a, const void* b, cd* out) -> wd_status {
        WD_TRY(blas_dot(ctx, G, 1, ps, a, b, true));
        *out = cd(ctx->hres[0], ctx->hres[1]);
        return WD_OK;
    };
    double rr;
    if (is_zero_f64(ctx, G, 1, x)) {   // zero guess: r = bhat without the operator
        WD_TRY(launch_convert(ctx, G, 1, WD_F64, bhat, WD_F64, r));
        WD_TRY(blas_norm2(ctx, G, 1, WD_F64, bhat, true));
        rr = ctx->hres[0];
    } else {
        WD_TRY(true_res(&rr));
    }
    WD_TRY(launch_convert(ctx, G, 1, WD_F64, r, ps, rs));
    WD_TRY(launch_convert(ctx, G, 1, WD_F64, r, ps, r0));
    WD_TRY(blas_zero(ctx, G, 1, ps, p));
    WD_TRY(blas_zero(ctx, G, 1, ps, v));
    WD_TRY(blas_zero(ctx, G, 1, ps, xs));
    cd rho(1.0), alpha(1.0), omega(1.0);
    double maxrr = rr;
    bool dirty = false;
    wd_status status = WD_ENOCONV;
    if (rr <= target) status = WD_OK;
    // Each iteration: 2 operator applications, whose last launches also sum <r0, v> and
    // <t, s> with ||t||^2, and 4 fused vector sweeps, the last with ||r||^2 and <r0, r> (the
    // next rho); the host waits three times.
    cd rho_new;
    bool have_rho = false;
    while (status != WD_OK && info->iters < prm.maxiter) {
        if (!have_rho) WD_TRY(dot(r0, rs, &rho_new));
        if (!std::isfinite(rho_new.real()) || std::abs(rho_new) == 0.0) {
            set_error("BiCGstab breakdown: rho = 0 at iteration %d", info->iters);
            status = WD_ENAN;
            break;
        }
        const cd beta = (rho_new / rho) * (alpha / omega);
        {   // p = r + beta (p - omega v)
            const cd c2 = -beta * omega;
            const void* in[3] = {rs, p, v};
            const double cr[3] = {1.0, beta.real(), c2.real()}, ci[3] = {0.0, beta.imag(), c2.imag()};
            WD_TRY(blas_lincomb(ctx, G, 1, ps, 3, in, cr, ci, p, nullptr, false));
        }
        // v = Mhat p with <r0, v> summed by the launch that writes v
        WD_TRY(op_M_red(g, kappa, WD_EVEN, 0, ps, p, v, RED_YDOT, r0, 0));
        WD_TRY(fetch_results(ctx, 2));
        const cd r0v(ctx->hres[0], ctx->hres[1]);
        alpha = rho_new / r0v;
        {   // s = r - alpha v
            const void* in[2] = {rs, v};
            const double cr[2] = {1.0, -alpha.real()}, ci[2] = {0.0, -alpha.imag()};
            WD_TRY(blas_lincomb(ctx, G, 1, ps, 2, in, cr, ci, s, nullptr, false));
        }
        // t = Mhat s with <t, s> and ||t||^2 summed by the launch that writes t (s is its a x term)
        WD_TRY(op_M_red(g, kappa, WD_EVEN, 0, ps, s, t, RED_XDOT, nullptr, 0));
        WD_TRY(fetch_results(ctx, 3));
        info->operator_applies += 2;
        const cd ts(ctx->hres[0], ctx->hres[1]);
        const double tt = ctx->hres[2];
        omega = tt > 0.0 ? ts / tt : cd(0.0);
        // x_s += alpha p + omega s and r = s - omega t, with ||r||^2 and <r0, r> (the next rho),
        // in one sweep
        WD_TRY(blas_bicg_xr(ctx, G, ps, xs, p, s, t, r0, rs, alpha.real(), alpha.imag(), omega.real(), omega.imag(),
                            true));
        dirty = true;
        rho = rho_new;
        info->iters++;
        double rr_s = ctx->hres[0];
        rho_new = cd(ctx->hres[1], ctx->hres[2]);
        have_rho = true;
        if (!std::isfinite(rr_s)) {
            set_error("BiCGstab: non-finite residual at iteration %d", info->iters);
            status = WD_ENAN;
            break;
        }
        // omega = 0 with a converged s (t = Mhat s = 0) is no breakdown: r = s is the
        // residual, and the float64 check below decides
        if (std::abs(omega) == 0.0 && rr_s > target) {
            set_error("BiCGstab breakdown: omega = 0 at iteration %d", info->iters);
            status = WD_ENAN;
            break;
        }
        if (rr_s <= target || rr_s < delta * delta * maxrr) {
            WD_TRY(blas_axpby(ctx, G, 1, ps, xs, 1.0, WD_F64, x, 1.0));
            doe_at_x = false;
            WD_TRY(blas_zero(ctx, G, 1, ps, xs));
            dirty = false;
            WD_TRY(true_res(&rr));
            info->reliable_updates++;
            if (rr <= target) {
                status = WD_OK;
                break;
            }
            WD_TRY(launch_convert(ctx, G, 1, WD_F64, r, ps, rs));
            have_rho = false;   // r changed: rho = <r0, r> again
            maxrr = rr;
        } else if (rr_s > maxrr) {
            maxrr = rr_s;
        }
    }
    if (dirty) {   // else rr is that of the last reliable update, already of this x
        WD_TRY(blas_axpby(ctx, G, 1, ps, xs, 1.0, WD_F64, x, 1.0));
        doe_at_x = false;
        WD_TRY(true_res(&rr));
    }
    if (doe_at_x) {
        *doe_xe = doe;
        *schur_rr = rr;
    }
    info->true_resid = std::sqrt(rr / bnorm2);
    // the recomputed float64 residual decides: converged is WD_OK even after a breakdown
    // (the iterate it left may already meet tol), non-finite is WD_ENAN
    if (std::isfinite(rr) && rr <= target) status = WD_OK;
    else if (status == WD_ENAN || !std::isfinite(rr)) status = WD_ENAN;
    else status = WD_ENOCONV;
    return status;
}

} // namespace wd

using namespace wd;

extern "C" wd_status wd_bicgstab_solve(wd_gauge g, double kappa, const wd_solver_params* params, const void* b, void* x,
                                       wd_solver_info* info)
{
    if (!g || !params || !b || !x || !info) {
        set_error("wd_bicgstab_solve: NULL argument");
        return WD_EINVAL;
    }
    if (!(params->tol > 0.0) || params->maxiter < 0 || !valid_prec(params->sloppy) || !(params->delta < 1.0)) {
        set_error("wd_bicgstab_solve: bad solver params");
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    WD_HIP(hipStreamSynchronize(ctx->stream));
    HopTally tally(ctx, info);
    const auto t0 = std::chrono::steady_clock::now();
    *info = wd_solver_info{};
    const long long hb = (long long)half_bytes(G, WD_F64);
    const char* b_e = (const char*)b;
    const char* b_o = b_e + hb;
    char* x_e = (char*)x;
    void* bhat;
    WD_TRY(ws_get(ctx, "bicg.bhat", hb, &bhat));
    WD_TRY(hop_half(g, WD_F64, 0, 0, 1, b_o, hb, bhat, hb, b_e, hb, 1.0, kappa));
    WD_TRY(blas_norm2(ctx, G, 2, WD_F64, b, true));
    const double bb = ctx->hres[0];
    wd_status s = WD_OK;
    const void* doe_xe = nullptr;   // D_oe x_e from the last float64 residual, if at hand
    double schur_rr = 0.0;          // and that residual's norm^2
    if (!std::isfinite(bb)) {   // NaN or Inf in the source: nothing to iterate on
        set_error("wd_bicgstab_solve: the source holds NaN or Inf");
        info->true_resid = info->true_resid_M = bb;
        info->status = WD_ENAN;
        hipStreamSynchronize(g->ctx->stream);   // synchronous: nothing of the solve left queued
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return WD_ENAN;
    }
    if (bb > 0.0) {
        s = bicgstab_run(g, kappa, *params, bhat, bb, x_e, info, &doe_xe, &schur_rr);
        if (s != WD_OK && s != WD_ENOCONV) return s;
    } else {
        WD_TRY(blas_zero(ctx, G, 2, WD_F64, x));
    }
    double rr_full;
    WD_TRY(eo_finish(g, kappa, b, x, &rr_full, doe_xe, schur_rr));   // x_o, then ||b - M x||^2 in float64
    info->true_resid_M = bb > 0 ? std::sqrt(rr_full / bb) : 0.0;
    if (!doe_xe) info->operator_applies++;   // the closing float64 check applied the operator
    info->status = s;
    hipStreamSynchronize(g->ctx->stream);   // synchronous: nothing of the solve left queued
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}
