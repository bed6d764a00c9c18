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
// with ||out||^2, RED_YDIFF ||y - M in||^2 (F64).  y has the subset of out.
wd_status op_M_red(wd_gauge g, double kappa, int subset, int dagger, int prec, const void* in, void* out, int red,
                   const void* y, int slot);
// M^dagger M (FULL) or Mhat^dagger Mhat (EVEN / ODD)
wd_status op_MdagM(wd_gauge g, double kappa, int subset, int prec, int nrhs, const void* in, void* out);

} // namespace wd
