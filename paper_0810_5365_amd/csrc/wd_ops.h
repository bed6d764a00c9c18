// Operator composition shared by the C ABI and the solvers.
#pragma once

#include "wd_core.h"

namespace wd {

// out (parity par, nrhs half fields) = a x + b D in  (x may be null: out = b D in)
wd_status hop_half(wd_gauge g, int prec, int par, int dagger, int nrhs, const void* in, long long in_stride, void* out,
                   long long out_stride, const void* x, long long x_stride, double a, double b);
// D_hop on a FULL / EVEN / ODD field, optionally fused with a x + b D in
wd_status op_dslash(wd_gauge g, int subset, int dagger, int prec, int nrhs, const void* in, void* out, const void* x,
                    double a, double b);
// M (FULL) or Mhat (EVEN / ODD), or their daggers
wd_status op_M(wd_gauge g, double kappa, int subset, int dagger, int prec, int nrhs, const void* in, void* out);
// out = Mhat in (EVEN / ODD) or M in (FULL), or their daggers, one rhs, with the reduction
// `red` of the result summed by the last launch(es) into dres[slot ..] and hres[slot ..] (not
// fetched: synchronise before reading hres): RED_NORM ||out||^2; RED_XDOT <out, in>,
// ||out||^2 and RED_YDOT <y, out>, ||out||^2 (EVEN / ODD, no dagger); RED_RESID out = y - M in
// with ||out||^2, RED_YDIFF ||y - M in||^2 (F64).  y has the subset of out.  For EVEN / ODD the
// first hop D in goes to hop_out if given (a half field of precision prec that the caller keeps),
// else to a shared workspace.
wd_status op_M_red(wd_gauge g, double kappa, int subset, int dagger, int prec, const void* in, void* out, int red,
                   const void* y, int slot, void* hop_out = nullptr);
// The launches of op_M_red without the final sum: the per-workgroup values of the one-value
// reduction `red` are left in ctx->partials[0 .. *nblk) for the caller to finish.  With RED_RESLO
// out is float32; with RED_CGR out is r, updated in place (r -= coef[0] M in, coef in device
// memory) at the accumulation precision (float64 for F64, else float32).  hop_out as for op_M_red.
wd_status op_M_red_partials(wd_gauge g, double kappa, int subset, int dagger, int prec, const void* in, void* out,
                            int red, const void* y, const double* coef, int* nblk, void* hop_out = nullptr);
// The end of an even-odd solve, in float64 (b, x FULL fields, x_e solved): x_o = b_o + kappa
// D_oe x_e, then rr = ||b_e - (x_e - kappa D_eo x_o)||^2, the even rows of ||b - M x||^2.  The
// odd rows are b_o - x_o + kappa D_oe x_e, zero by the construction of x_o up to its rounding,
// and are not evaluated; the even rows test the x_o that was built.  doe_xe, if given, is
// D_oe x_e of the float64 Schur residual the solver last computed at this x_e, whose norm^2 it
// passes as schur_rr: x_o is then one linear combination instead of a hop, and the even rows,
// b_e - x_e + kappa D_eo (b_o + kappa D_oe x_e) = bhat - Mhat x_e, are that residual, so *rr =
// schur_rr without another launch.  Fetched.
wd_status eo_finish(wd_gauge g, double kappa, const void* b, void* x, double* rr, const void* doe_xe = nullptr,
                    double schur_rr = 0.0);
// Sets info->hops, when the enclosing solver call returns, to the hopping-term applications
// queued since its construction.
struct HopTally {
    wd_context ctx;
    wd_solver_info* info;
    long long h0;
    HopTally(wd_context c, wd_solver_info* i) : ctx(c), info(i), h0(c->hops) {}
    ~HopTally() { info->hops = ctx->hops - h0; }
    HopTally(const HopTally&) = delete;
    HopTally& operator=(const HopTally&) = delete;
};
// M^dagger M (FULL) or Mhat^dagger Mhat (EVEN / ODD)
wd_status op_MdagM(wd_gauge g, double kappa, int subset, int prec, int nrhs, const void* in, void* out);

} // namespace wd
