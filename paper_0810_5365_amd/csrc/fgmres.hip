// Flexible GMRES for the Wilson system M x = b with a right preconditioner
// that may change from one iteration to the next (Saad, "A flexible
// inner-outer preconditioned GMRES algorithm", SISC 1993).  The Krylov
// iteration runs on the even-odd Schur complement Mhat = 1 - kappa^2 D_eo D_oe
// (paper Section 4), whose inverse is exactly the even-even block of M^-1.
// So the learned parallel-transport network N ~ M^-1, applied to (v_e, 0),
// gives the preconditioner K v_e = [N (v_e, 0)]_e ~ Mhat^-1 v_e.
//
// Mixed precision by iterative refinement on the Schur system: with
// bhat = b_e + kappa D_eo b_o, rhat = bhat - Mhat x_e in float64; one float32
// cycle (operator, network, Krylov basis) solves Mhat e = rhat from zero for at
// most `restart` iterations or until its residual estimate falls by
// params->delta; x_e += e in float64 and rhat is recomputed, which decides
// convergence.  At the end x_o = b_o + kappa D_oe x_e, which zeroes the odd rows
// of b - M x and leaves rhat in the even rows; the even rows are recomputed in
// float64 from the x_o that was built, and reported.  Orthogonalisation is classical Gram-Schmidt applied
// twice: the first pass's coefficients never leave the device, the first pass's
// update and the second pass's dots share one sweep over the basis, and each
// iteration waits for the host once.  The plain solver is the fallback: a NaN,
// or a cycle that fails to reduce the residual tenfold, hands x to the even-odd
// CG (wd_wilson_solve), which then finishes the solve.
#include <stdlib.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <complex>
#include <vector>

#include "wd_ops.h"

namespace wd {

typedef std::complex<double> cd;

struct Net {
    int nlayers;
    std::vector<int> widths;
    std::vector<const void*> W;
    int wprec;
};

// z_e = [N (v_e, 0)]_e on float32 EVEN half fields (4 channels in and out)
static wd_status apply_net(wd_gauge g, const Net& net, const void* v, void* z, void* fa, void* fb)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    // WD_PTCONV_PARITY_SKIP=0 computes every path and site through the feature tensors (same
    // result, for checking)
    const char* env = getenv("WD_PTCONV_PARITY_SKIP");
    const bool skip = !(env && atoi(env) == 0);
    const int L = net.nlayers;
    // the first and last layers read and write the spinor half fields themselves when they can
    const bool sin = skip && ptconv_spin_io(net.wprec, net.widths[0], net.widths[1]);
    const bool sout = skip && ptconv_spin_io(net.wprec, net.widths[L - 1], net.widths[L]);
    // a 4 -> 8 -> ... -> 8 -> 4 network on the matrix cores keeps its hidden features in bf16
    // (the layers round their transported inputs to bf16 for the matrix cores anyway); the
    // feature tensors are the layers' only traffic besides the links
    bool hf = sin && sout && L >= 2;
    for (int l = 1; l < L; ++l) hf = hf && net.widths[l] == 8;
    if (const char* e = getenv("WD_PTNET_F32_FEATURES")) hf = hf && atoi(e) == 0;
    if (!sin) WD_TRY(launch_spinor_features(ctx, G, 1, (void*)v, fa, true, true));
    void* cur = fa;
    void* nxt = fb;
    for (int l = 0; l < L; ++l) {
        // the input's odd sites are zero, and only the even output sites are used
        WD_TRY(ptconv_fwd(g, net.widths[l], net.widths[l + 1], net.wprec, net.W[l], cur, nxt, 1,
                          skip && l == 0 ? 1 : -1, skip && l == L - 1, sin && l == 0 ? v : nullptr,
                          sout && l == L - 1 ? z : nullptr, hf));
        std::swap(cur, nxt);
    }
    return sout ? WD_OK : launch_spinor_features(ctx, G, 1, z, cur, false, true);
}

static wd_status fgmres_run(wd_gauge g, double kappa, const wd_solver_params& prm, int m, const Net* net, const void* b,
                            void* x, wd_solver_info* info, bool* fallback)
{
    wd_context ctx = g->ctx;
    const Geom& G = g->geom;
    const size_t nh = 1;   // Krylov vectors: EVEN half fields
    const size_t v32 = half_bytes(G, WD_F32);
    const size_t h64 = half_bytes(G, WD_F64);
    void *V, *Z, *wv, *e, *e64, *rhat, *fa = nullptr, *fb = nullptr;
    WD_TRY(ws_get(ctx, "fgmres.V", v32 * (m + 1), &V));
    WD_TRY(ws_get(ctx, "fgmres.Z", v32 * m, &Z));
    WD_TRY(ws_get(ctx, "fgmres.w", v32, &wv));
    WD_TRY(ws_get(ctx, "fgmres.e", v32, &e));
    WD_TRY(ws_get(ctx, "fgmres.e64", h64, &e64));
    WD_TRY(ws_get(ctx, "fgmres.rhat", h64, &rhat));
    if (net) {
        int cmax = 0;
        for (int c : net->widths) cmax = c > cmax ? c : cmax;
        const size_t fbytes = (size_t)cmax * 6 * G.Vh * 2 * sizeof(float);
        WD_TRY(ws_get(ctx, "fgmres.fa", fbytes, &fa));
        WD_TRY(ws_get(ctx, "fgmres.fb", fbytes, &fb));
    }
    auto Vi = [&](int i) { return (void*)((char*)V + (size_t)i * v32); };
    auto Zi = [&](int i) { return (void*)((char*)Z + (size_t)i * v32); };
    char* x_e = (char*)x;
    const char* b_e = (const char*)b;
    const char* b_o = b_e + h64;
    void* bhat;
    WD_TRY(ws_get(ctx, "fgmres.bhat", h64, &bhat));

    WD_TRY(blas_norm2(ctx, G, 2, WD_F64, b, true));
    const double bb = ctx->hres[0];
    const double tol2 = prm.tol * prm.tol * bb;
    info->iters = 0;
    info->reliable_updates = 0;
    info->operator_applies = 0;
    info->cycles = 0;
    info->fell_back = 0;
    *fallback = false;
    if (!std::isfinite(bb)) {   // NaN or Inf in the source: nothing to iterate on, no fallback
        set_error("wd_fgmres_solve: the source holds NaN or Inf");
        info->true_resid = info->true_resid_M = bb;
        return WD_ENAN;
    }
    if (!(bb > 0.0)) {
        WD_TRY(blas_zero(ctx, G, 2, WD_F64, x));
        info->true_resid = info->true_resid_M = 0.0;
        return WD_OK;
    }
    // The iterate is x_e; x_o = b_o + kappa D_oe x_e is formed at the end, which makes the odd
    // rows of b - M x vanish and the even rows equal bhat - Mhat x_e (bhat = b_e + kappa D_eo b_o):
    // so the float64 refinement only needs the Schur residual (two hops per cycle).
    WD_TRY(hop_half(g, WD_F64, 0, 0, 1, b_o, (long long)h64, bhat, (long long)h64, b_e, (long long)h64, 1.0, kappa));
    void* doe;   // D_oe x_e of the last Schur residual, reused for x_o at the end
    WD_TRY(ws_get(ctx, "fgm.doe", h64, &doe));
    bool doe_at_x = false;   // doe holds D_oe x_e for the current x_e
    auto schur_res = [&](double* rr) -> wd_status {
        // rhat = bhat - Mhat x_e
        WD_TRY(op_M_red(g, kappa, WD_EVEN, 0, WD_F64, x_e, rhat, RED_RESID, bhat, 0, doe));
        WD_TRY(fetch_results(ctx, 1));
        *rr = ctx->hres[0];
        info->operator_applies++;
        doe_at_x = true;
        return WD_OK;
    };
    auto finish_x = [&](double* rr) -> wd_status {   // x_o, then the full residual in float64
        // (*rr on entry: the last Schur residual's norm^2, of this x_e when doe_at_x)
        WD_TRY(eo_finish(g, kappa, b, x, rr, doe_at_x ? doe : nullptr, *rr));
        if (!doe_at_x) info->operator_applies++;   // the closing float64 check applied the operator
        return WD_OK;
    };
    double rr;
    if (is_zero_f64(ctx, G, 1, x_e)) {   // zero guess: rhat = bhat without the operator
        WD_TRY(launch_convert(ctx, G, 1, WD_F64, bhat, WD_F64, rhat));
        WD_TRY(blas_norm2(ctx, G, 1, WD_F64, bhat, true));
        rr = ctx->hres[0];
    } else {
        WD_TRY(schur_res(&rr));
    }
    // default cycle reduction 1e-5: on 16^3 x 32 (kappa 0.1248) the fastest of 1e-3 .. 1e-6 for
    // FGMRES with and without the network (one float64 refinement fewer than at 1e-4 with it)
    const double inner = prm.delta > 0.0 ? prm.delta : 1e-5;
    while (rr > tol2 && info->iters < prm.maxiter) {
        // ---- one float32 cycle on Mhat e_e = rhat_e --------------------------------
        // stop at delta, or earlier if that already meets the requested tolerance
        WD_TRY(launch_convert(ctx, G, nh, WD_F64, rhat, WD_F32, Vi(0)));
        WD_TRY(blas_norm2(ctx, G, nh, WD_F32, Vi(0), true));
        const double beta = std::sqrt(ctx->hres[0]);
        const double cycle_tol = std::max(inner, 0.5 * std::sqrt(tol2) / beta);
        if (!std::isfinite(beta) || beta == 0.0) {
            *fallback = !std::isfinite(beta);
            break;
        }
        WD_TRY(blas_axpby(ctx, G, nh, WD_F32, Vi(0), 0.0, WD_F32, Vi(0), 1.0 / beta));
        std::vector<std::vector<cd>> H(m + 1, std::vector<cd>(m, 0.0));
        std::vector<cd> gvec(m + 1, 0.0), cs(m), sn(m);
        gvec[0] = beta;
        int j = 0;
        bool bad = false;
        for (; j < m && info->iters < prm.maxiter; ++j) {
            if (net) WD_TRY(apply_net(g, *net, Vi(j), Zi(j), fa, fb));
            WD_TRY(op_M(g, kappa, WD_EVEN, 0, WD_F32, 1, net ? Zi(j) : Vi(j), wv));
            info->operator_applies++;
            info->iters++;
            // classical Gram-Schmidt applied twice ("twice is enough"): the first pass keeps its
            // coefficients on the device and feeds the first multi-axpy directly; only the second
            // pass (with ||w||^2 in the same reduction) waits for the host
            constexpr int SLOT_H1 = 128;
            WD_TRY(blas_mdot(ctx, G, nh, WD_F32, V, v32, j + 1, wv, false, false, SLOT_H1));
            int norm_at = 2 * (j + 1);
            if (j + 1 <= MGS_KMAX) {
                // the first pass's update and the second pass's dots in one sweep over V
                WD_TRY(blas_maxpy_mdot(ctx, G, nh, WD_F32, V, v32, j + 1, SLOT_H1, wv));
                norm_at = 2 * MGS_KMAX;
            } else {
                WD_TRY(blas_maxpy_dev(ctx, G, nh, WD_F32, V, v32, j + 1, SLOT_H1, -1.0f, wv, 1.0, wv));
                WD_TRY(blas_mdot(ctx, G, nh, WD_F32, V, v32, j + 1, wv, true, true));
            }
            const double w2 = ctx->hres[norm_at];
            double h2 = 0.0;
            std::vector<double> coef(2 * (j + 1));
            for (int i = 0; i <= j; ++i) {
                const cd h1((double)(float)ctx->hres[SLOT_H1 + 2 * i], (double)(float)ctx->hres[SLOT_H1 + 2 * i + 1]);
                const cd h(ctx->hres[2 * i], ctx->hres[2 * i + 1]);
                H[i][j] = h1 + h;
                h2 += std::norm(h);
                coef[2 * i] = -h.real();
                coef[2 * i + 1] = -h.imag();
            }
            const double hn2 = w2 - h2;
            const double hn = std::sqrt(hn2 > 0.0 ? hn2 : 0.0);
            if (!std::isfinite(hn) || !std::isfinite(w2)) {
                bad = true;
                break;
            }
            // V_{j+1} = (w - sum h_i V_i) / hn in one pass
            if (hn > 0.0) WD_TRY(blas_maxpy(ctx, G, nh, WD_F32, V, v32, j + 1, coef.data(), wv, 1.0 / hn, Vi(j + 1)));
            H[j + 1][j] = hn;
            // apply the previous rotations to column j, then make a new one
            for (int i = 0; i < j; ++i) {
                const cd a = H[i][j], c = H[i + 1][j];
                H[i][j] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
                H[i + 1][j] = -sn[i] * a + cs[i] * c;
            }
            const cd a = H[j][j], c = H[j + 1][j];
            const double den = std::sqrt(std::norm(a) + std::norm(c));
            if (den == 0.0) {
                bad = true;
                break;
            }
            cs[j] = a / den;
            sn[j] = c / den;
            H[j][j] = std::conj(cs[j]) * a + std::conj(sn[j]) * c;
            H[j + 1][j] = 0.0;
            gvec[j + 1] = -sn[j] * gvec[j];
            gvec[j] = std::conj(cs[j]) * gvec[j];
            if (std::abs(gvec[j + 1]) <= cycle_tol * beta || hn == 0.0) {
                ++j;
                break;
            }
        }
        if (bad) {
            *fallback = true;
            break;
        }
        // y = H^-1 g (upper triangular, j x j); e = sum y_i Z_i; x += e
        std::vector<cd> y(j);
        for (int i = j - 1; i >= 0; --i) {
            cd s = gvec[i];
            for (int k = i + 1; k < j; ++k) s -= H[i][k] * y[k];
            y[i] = s / H[i][i];
        }
        std::vector<double> coef(2 * j);
        bool finite = true;
        for (int i = 0; i < j; ++i) {
            coef[2 * i] = y[i].real();
            coef[2 * i + 1] = y[i].imag();
            finite = finite && std::isfinite(coef[2 * i]) && std::isfinite(coef[2 * i + 1]);
        }
        if (!finite) {
            *fallback = true;
            break;
        }
        WD_TRY(blas_zero(ctx, G, nh, WD_F32, e));
        for (int i0 = 0; i0 < j; i0 += WD_MAXPY) {
            const int k = j - i0 < WD_MAXPY ? j - i0 : WD_MAXPY;
            WD_TRY(blas_maxpy(ctx, G, nh, WD_F32, net ? Zi(i0) : Vi(i0), v32, k, coef.data() + 2 * i0, e, 1.0, e));
        }
        // x_e += e_e (float64), then the new Schur residual
        WD_TRY(launch_convert(ctx, G, nh, WD_F32, e, WD_F64, e64));
        WD_TRY(blas_axpby(ctx, G, nh, WD_F64, e64, 1.0, WD_F64, x_e, 1.0));
        doe_at_x = false;
        const double rr_prev = rr;
        WD_TRY(schur_res(&rr));
        info->reliable_updates++;
        info->cycles++;
        if (!std::isfinite(rr) || (rr > 0.01 * rr_prev && rr > tol2)) {   // NaN, or less than 10x per cycle
            *fallback = true;
            break;
        }
    }
    if (*fallback) return WD_OK;   // the plain solver rebuilds x_o and judges the residual
    WD_TRY(finish_x(&rr));
    info->true_resid = info->true_resid_M = std::sqrt(rr / bb);
    return rr <= tol2 ? WD_OK : WD_ENOCONV;
}

// the network arguments of the C entry points, checked
static wd_status make_net(const char* who, int nlayers, const int* widths, const void* const* weights, int wprec,
                          Net* net)
{
    if (widths[0] != 4 || widths[nlayers] != 4) {
        set_error("%s: the network must map 4 channels (spin) to 4 channels", who);
        return WD_EINVAL;
    }
    if (wprec != WD_F32 && wprec != WD_F16 && wprec != WD_BF16) {
        set_error("%s: weight precision %d not in {F32, F16, BF16}", who, wprec);
        return WD_EINVAL;
    }
    net->nlayers = nlayers;
    net->widths.assign(widths, widths + nlayers + 1);
    net->W.assign(weights, weights + nlayers);
    net->wprec = wprec;
    for (int l = 0; l < nlayers; ++l) {
        const int c = widths[l + 1];
        if (!(c == 1 || c == 2 || c == 3 || c == 4 || c == 8) || !weights[l]) {
            set_error("%s: layer %d: width %d unsupported or weights NULL", who, l, c);
            return WD_EUNSUPPORTED;
        }
    }
    return WD_OK;
}

} // namespace wd

using namespace wd;

extern "C" {

wd_status wd_ptnet_apply_even(wd_gauge g, int nlayers, const int* widths, const void* const* weights, wd_prec wprec,
                              const void* in, void* out)
{
    if (!g || nlayers < 1 || !widths || !weights || !in || !out || in == out) {
        set_error("wd_ptnet_apply_even: bad argument");
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    Net net;
    WD_TRY(make_net("wd_ptnet_apply_even", nlayers, widths, weights, wprec, &net));
    int cmax = 0;
    for (int c : net.widths) cmax = c > cmax ? c : cmax;
    const size_t fbytes = (size_t)cmax * 6 * g->geom.Vh * 2 * sizeof(float);
    void *fa, *fb;
    WD_TRY(ws_get(g->ctx, "fgmres.fa", fbytes, &fa));
    WD_TRY(ws_get(g->ctx, "fgmres.fb", fbytes, &fb));
    return apply_net(g, net, in, out, fa, fb);
}

wd_status wd_fgmres_solve(wd_gauge g, double kappa, const wd_solver_params* params, int restart, int nlayers,
                          const int* widths, const void* const* weights, wd_prec wprec, const void* b, void* x,
                          wd_solver_info* info)
{
    if (!g || !params || !b || !x || !info || restart < 1 || restart > WD_MAXPY - 1 || nlayers < 0 ||
        (nlayers > 0 && (!widths || !weights))) {
        set_error("wd_fgmres_solve: bad argument");
        return WD_EINVAL;
    }
    if (!(params->tol > 0.0) || params->maxiter < 0) {
        set_error("wd_fgmres_solve: bad tolerance or maxiter");
        return WD_EINVAL;
    }
    if (!g->uploaded) {
        set_error("gauge field has not been uploaded");
        return WD_EINVAL;
    }
    Net net;
    if (nlayers > 0) WD_TRY(make_net("wd_fgmres_solve", nlayers, widths, weights, wprec, &net));
    WD_HIP(hipStreamSynchronize(g->ctx->stream));
    HopTally tally(g->ctx, info);
    const auto t0 = std::chrono::steady_clock::now();
    bool fallback = false;
    wd_status s = fgmres_run(g, kappa, *params, restart, nlayers > 0 ? &net : nullptr, b, x, info, &fallback);
    if (s == WD_OK && fallback) {
        // hand the current iterate to the plain solver, which also judges the final residual
        wd_solver_info ci{};
        const int done = info->iters;
        wd_solver_params p2 = *params;
        p2.maxiter = params->maxiter - done > 0 ? params->maxiter - done : 1;
        if (p2.delta == 0.0 || !(p2.delta < 1.0)) p2.delta = -1.0;   // the plain solver's default
        if (p2.sloppy == WD_F64 || p2.sloppy > WD_BF16) p2.sloppy = WD_F32;
        s = wd_wilson_solve(g, kappa, &p2, b, x, &ci);
        info->iters += ci.iters;
        info->operator_applies += ci.operator_applies;
        info->true_resid = info->true_resid_M = ci.true_resid_M;
        info->reliable_updates += ci.reliable_updates;
        info->fell_back = 1;
    }
    info->status = s;
    hipStreamSynchronize(g->ctx->stream);   // synchronous: nothing of the solve left queued
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

} // extern "C"
