/*
 * wdirac.h -- C ABI of libwdirac, the MI355X (gfx950) Wilson-Dirac library.
 *
 * The library applies the Wilson-Dirac operator
 *
 *     M psi(x) = psi(x) - kappa * D_hop psi(x),
 *     D_hop psi(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                           + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ],
 *
 * with SU(3) links U and 4-spin x 3-colour fields on a 4-D lattice, its hopping
 * term restricted to even or odd sites ("Dslash", the paper's Section 4 "Wilson
 * inverter: main features"), the even-odd preconditioned operator
 * 1 - kappa^2 D_eo D_oe (caption of the paper's Fig. 2, Section 7), and a
 * conjugate-gradient solver with double-precision global sums (Section 4).
 * Gamma matrices are in the DeGrand-Rossi basis; mu = 0..3 is x, y, z, t.
 * Boundary conditions are a sign bc[mu] = +1 / -1 applied on the hop across
 * the lattice edge in direction mu.
 *
 * Conventions shared by every entry point
 * --------------------------------------
 * - Every function is extern "C", returns a wd_status (or a plain value where
 *   stated) and never throws or aborts.  On WD_EINVAL / WD_ESHAPE /
 *   WD_EUNSUPPORTED nothing is written.  wd_last_error() gives a thread-local
 *   description of the last failure.
 * - Field and weight buffers are DEVICE pointers owned by the caller (e.g. a
 *   torch tensor's data_ptr()), sized with wd_spinor_bytes / wd_feature_bytes.
 *   The library never frees them and keeps them past a call only where a
 *   function says so (wd_batch).  Only wd_gauge_upload accepts a host pointer.
 * - Work is enqueued on the context's HIP stream and is asynchronous, except
 *   where a function returns host scalars (reductions, solvers, autotune),
 *   which synchronise that stream.  An asynchronous device error is reported
 *   as WD_EHIP by the next synchronising call.
 * - Lattice dims X, Y, Z, T must be even and >= 2; the half volume V/2 must be
 *   below 2^31.  Sites are split by parity (x+y+z+t)&1; inside a parity a site
 *   has checkerboard index cb = lex >> 1, lex = x + X(y + Y(z + Z t)).
 *
 * Canonical (host-order) layouts, interleaved re, im doubles:
 *   links            [4][T][Z][Y][X][3][3][2]      U_mu(x)[row][col]
 *   spinor FULL      [nrhs][T][Z][Y][X][4][3][2]   [spin][colour]
 *   spinor EVEN/ODD  [nrhs][V/2][4][3][2]          sites of that parity in cb order
 * Packed (device) layouts are internal; wd_spinor_bytes gives their size.  A
 * packed FULL field is the EVEN half followed by the ODD half, per rhs.  Inside
 * a half field (and a packed gauge group) the structure-of-arrays planes lie
 * wd_plane_stride() sites apart: V/2 below 4096 sites per parity, otherwise
 * V/2 rounded up to 64 plus 256, so that planes never sit a power of two bytes
 * apart and the streams of one kernel spread over the HBM channels.  The tail
 * of each plane is padding that no function reads.
 */
#ifndef WDIRAC_H
#define WDIRAC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WD_ABI_VERSION 5

typedef enum {
    WD_OK = 0,
    WD_EINVAL = 1,        /* bad argument: null pointer, bad enum, bad size   */
    WD_ESHAPE = 2,        /* lattice dims or field shapes do not fit          */
    WD_ENOMEM = 3,        /* device allocation failed                          */
    WD_EHIP = 4,          /* a HIP runtime call or kernel failed               */
    WD_ENOCONV = 5,       /* solver reached maxiter; x holds the last iterate  */
    WD_ENAN = 6,          /* NaN or Inf met in a solver reduction              */
    WD_EUNSUPPORTED = 7   /* valid but unsupported combination                 */
} wd_status;

/* Storage precision of links and fields.  F16 / BF16 store 16-bit values with
 * a per-site float32 scale for spinors and compute in float32; F32 stores and
 * computes in float32; F64 in float64. */
typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2, WD_BF16 = 3 } wd_prec;

/* Link storage: 18 reals, or 12 reals (rows 0 and 1) with row 2 rebuilt on
 * the fly as conj(row0 x row1) (paper, Sections 4, 5 and 7). */
typedef enum { WD_RECON_12 = 12, WD_RECON_18 = 18 } wd_recon;

typedef enum { WD_FULL = 0, WD_EVEN = 1, WD_ODD = 2 } wd_subset;

typedef struct {
    int dims[4];   /* X, Y, Z, T: each even, >= 2                        */
    int bc[4];     /* +1 periodic, -1 antiperiodic, per direction         */
} wd_lattice;

typedef struct wd_context_s* wd_context;   /* device, stream, workspace, tuning table */
typedef struct wd_gauge_s* wd_gauge;       /* device link storage of one field        */
typedef struct wd_batch_s* wd_batch;       /* a captured batch of dslash applications  */

/* ---- version and errors ------------------------------------------------- */
int wd_abi_version(void);
const char* wd_status_string(int status);
/* Thread-local text for the most recent failing call on this thread. */
const char* wd_last_error(void);

/* ---- context -------------------------------------------------------------- */
/* Bind a context to HIP device `device` and stream `stream` (a hipStream_t, or
 * NULL for the null stream).  Owns the solver workspace (allocated on first
 * use, freed by wd_context_destroy) and the tuning table. */
wd_status wd_context_create(int device, void* stream, wd_context* out);
wd_status wd_context_set_stream(wd_context ctx, void* stream);
wd_status wd_context_destroy(wd_context ctx);

/* ---- gauge field (paper, Section 5: 18 floats per link, or 12 before
 *      reconstruction) ------------------------------------------------------- */
/* Create an empty gauge object for lattice `lat` with link storage `recon`.
 * The lattice (dims and bc) is copied. */
wd_status wd_gauge_create(wd_context ctx, const wd_lattice* lat, wd_recon recon, wd_gauge* out);
/* Upload canonical float64 links (layout above; host pointer if on_device == 0,
 * device pointer otherwise).  Synchronous.  Packed copies per precision are
 * built from this field on first use of that precision (wd_gauge_prepare
 * builds them ahead of time). */
wd_status wd_gauge_upload(wd_gauge g, const double* links, int on_device);
wd_status wd_gauge_prepare(wd_gauge g, wd_prec prec);
/* Bytes of packed device link storage at precision `prec` (0 on bad input). */
size_t wd_gauge_bytes(wd_gauge g, wd_prec prec);
wd_status wd_gauge_destroy(wd_gauge g);
/* Temporal gauge fixing (paper, Sections 4 and 7): rotate the uploaded links
 * by Omega(x, 0) = 1, Omega(x, t + 1) = Omega(x, t) U_t(x, t), so that every
 * t-link is exactly the identity except on the last time slice; from then on
 * the dslash skips those links.  Solutions in the fixed gauge are Omega x.
 * omega_out (host, may be NULL) receives Omega as [T][Z][Y][X][3][3][2].
 * A later wd_gauge_upload clears the fixed state.  Synchronous. */
wd_status wd_gauge_fix_temporal(wd_gauge g, double* omega_out);

/* ---- spinor fields (paper, Section 5: 24 floats per site, split by parity,
 *      stored as structure-of-arrays of 16-byte vectors) ---------------------- */
/* Bytes of a packed field; 0 on bad input. */
size_t wd_spinor_bytes(const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs);
/* Sites between consecutive planes of a packed half field (see the layout
 * notes above); 0 on bad input. */
long long wd_plane_stride(const wd_lattice* lat);
/* canonical float64 (device) -> packed (device), and back.  16-bit precisions
 * quantise each site with scale s = max |v_i| over its 24 float32 values and
 * codes RNE16(v_i * RN(1/s)). */
wd_status wd_spinor_pack(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                         const double* canon, void* packed);
wd_status wd_spinor_unpack(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                           const void* packed, double* canon);
/* dst = src converted between packed precisions (same subset, nrhs). */
wd_status wd_spinor_convert(wd_context ctx, const wd_lattice* lat, wd_subset subset, int nrhs,
                            wd_prec src_prec, const void* src, wd_prec dst_prec, void* dst);

/* ---- operators (paper, Sections 4 and 7) --------------------------------- */
/* out = D_hop in restricted to the sites of out_subset:
 *   WD_EVEN: out_e = D_eo in_o (in is an ODD field), WD_ODD: out_o = D_oe in_e,
 *   WD_FULL: out = D_hop in (both FULL fields).
 * dagger != 0 applies D_hop^dagger.  Links and fields share precision `prec`. */
wd_status wd_dslash(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, int nrhs,
                    const void* in, void* out);
/* out = a * x + b * D_hop in  (x has the subset and precision of out; x may alias out). */
wd_status wd_dslash_xpay(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, int nrhs,
                         const void* in, const void* x, double a, double b, void* out);
/* subset WD_FULL: out = M in = in - kappa D_hop in (M^dagger if dagger);
 * WD_EVEN: out = (1 - kappa^2 D_eo D_oe) in on even sites; WD_ODD: 1 - kappa^2 D_oe D_eo.
 * in and out must not alias. */
wd_status wd_apply_M(wd_gauge g, double kappa, wd_subset subset, int dagger, wd_prec prec, int nrhs,
                     const void* in, void* out);
/* out = M^dagger M in (FULL) or Mhat^dagger Mhat in (EVEN / ODD).  in and out must not alias. */
wd_status wd_apply_MdagM(wd_gauge g, double kappa, wd_subset subset, wd_prec prec, int nrhs,
                         const void* in, void* out);

/* ---- one device's slab of a lattice split along t (paper, Section 4: spin
 *      projection before the colour multiply halves what crosses a face) ------
 * The gauge object holds the slab's own sites, dims (X, Y, Z, T_local), with
 * its links U_mu(x); a slab's first global time slice must be even, so that
 * local and global parities agree.  Spatial hops wrap inside the slab; the
 * t-hops that leave it use half spinors exchanged with the neighbouring slabs
 * (by the caller: a device copy here, a transfer between devices in general).
 * Face buffer (device, caller-owned): 12 reals per face site, X Y Z / 2 sites,
 * as 3 planes of float4 (F32) or 6 planes of double2 (F64), plane k holding
 * reals 4k..4k+3 (2k, 2k+1) of every site in checkerboard order of the slice. */
/* Bytes of one face buffer (0 on bad input or a precision other than F32/F64). */
size_t wd_face_bytes(const wd_lattice* lat, wd_prec prec);
/* From the half field `in` of parity in_subset (EVEN or ODD) at prec (F32 or
 * F64), fill face_fwd with (1 - s gamma_t) in on the first time slice (for the
 * forward t-hops of the previous slab's last slice) and face_bwd with
 * U_t(x)^dagger (1 + s gamma_t) in(x) on the last slice (for the backward
 * t-hops of the next slab's first slice); s = +1 for D_hop, -1 for the dagger.
 * Errors: WD_EINVAL (NULL pointer, bad subset, links not uploaded),
 * WD_EUNSUPPORTED (16-bit precision, links in temporal gauge).  Asynchronous. */
wd_status wd_halo_pack(wd_gauge g, wd_subset in_subset, int dagger, wd_prec prec, const void* in,
                       void* face_fwd, void* face_bwd);
/* out (parity out_subset) = D_hop in (the dagger if dagger != 0) on the slab,
 * with the forward t-hops of the last slice taken from ghost_fwd (the next
 * slab's face_fwd of its input, times sign_fwd) and the backward t-hops of the
 * first slice from ghost_bwd (the previous slab's face_bwd, times sign_bwd).
 * The signs are the t boundary condition where the hop crosses the global t
 * edge, else +1.  in: half field of the other parity; out must not alias it.
 * Errors as wd_halo_pack.  Asynchronous. */
wd_status wd_dslash_halo(wd_gauge g, wd_subset out_subset, int dagger, wd_prec prec, const void* in,
                         const void* ghost_fwd, const void* ghost_bwd, double sign_fwd, double sign_bwd,
                         void* out);

/* ---- global sums in float64 (paper, Section 4) ---------------------------- */
/* result[0] + i result[1] = <a, b> = sum conj(a_i) b_i over the whole field
 * (all rhs).  Deterministic: fixed-order two-pass reduction.  Synchronous. */
wd_status wd_dot(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                 const void* a, const void* b, double* result);
wd_status wd_norm2(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                   const void* a, double* result);
/* <a, b> with no allocation of any kind, for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the result of wd_dot, bit for bit, on the CURRENT HIP device and on
 * `stream` (a hipStream_t, NULL for the null stream), with no context.
 * Scratch: the per-workgroup partial sums and the two final values live in a static
 * device array of 2 * 2048 + 2 doubles (32.8 KB) that every GPU the library runs on
 * holds until the process ends.  The reduction grid is capped at 2048 workgroups, so
 * fields of every size the library accepts fit it; there is no separate size limit.
 * All calls on one GPU share that array: calls that overlap in time on one GPU (from
 * several host threads or streams) race and must be serialised by the caller.
 * a, b: packed device fields (layout of wd_spinor_bytes); result: host, 2 doubles.
 * Synchronises `stream`.  WD_EINVAL: NULL pointer, bad subset, precision or nrhs, or a
 * current device index of 64 or more; WD_ESHAPE: bad lattice; WD_EHIP: a HIP failure. */
wd_status wd_dot_noalloc(void* stream, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                         const void* a, const void* b, double* result);
/* y = alpha * x + y with complex alpha = (alpha_re, alpha_im); F32 and F64 only. */
wd_status wd_caxpy(wd_context ctx, const wd_lattice* lat, wd_subset subset, wd_prec prec, int nrhs,
                   double alpha_re, double alpha_im, const void* x, void* y);

/* ---- solvers (paper, Section 4: even-odd preconditioned CG) --------------- */
typedef struct {
    double tol;        /* stop when ||r|| / ||b|| <= tol (true residual, float64) */
    int maxiter;       /* iteration cap; WD_ENOCONV when reached                   */
    int sloppy;        /* wd_prec of the inner iterations (F64, F32, F16, BF16)    */
    double delta;      /* reliable update when ||r|| < delta * max ||r|| since last;
                          < 0: the default for the sloppy precision (F32 1e-5,
                          F16 1e-2, BF16 3e-2; measured with CG and BiCGstab on
                          the 32^3 x 64 and 16^3 x 32 solves: 16-bit ~10x above
                          where the iteration count starts to grow, F32 ~170x
                          the float32 unit roundoff, with no growth down to it) */
    int pure_sloppy;   /* 1: never recompute the residual (reports the stall level) */
} wd_solver_params;

typedef struct {
    int iters;              /* CG iterations                                      */
    int reliable_updates;   /* float64 residual recomputations                    */
    int operator_applies;   /* applications of the solved operator, float64
                               residual checks included (one each)                 */
    int status;             /* wd_status of the solve                             */
    double true_resid;      /* ||b - A x|| / ||b|| in float64, A the solved operator;
                               the even-odd solvers of M x = b report the Schur
                               system's ||bhat - Mhat x_e|| / ||b|| (their
                               convergence test)                                  */
    double true_resid_M;    /* ||b - M x|| / ||b|| for wd_wilson_solve, else -1     */
    double seconds;         /* wall time from call to return                      */
    int cycles;             /* flexible GMRES: restart cycles (float64 residual updates) */
    int fell_back;          /* flexible GMRES: 1 if it handed over to the plain CG      */
    double lambda_min;      /* CG: smallest and largest Ritz value of the solved operator */
    double lambda_max;      /* (A = M^dag M or Mhat^dag Mhat) from the CG step lengths and
                               residual ratios (the Lanczos tridiagonal); estimates of the
                               ends of its spectrum, lambda_min from above, lambda_max
                               from below.  0 where not computed (other solvers, a
                               breakdown, or no iteration).                           */
    long long hops;         /* hopping-term applications D_eo / D_oe on one parity
                               (float64 ones included) over the whole call: the
                               operator work of the solve, 4 per Mhat^dag Mhat     */
} wd_solver_info;

/* Solve A x = b, A = M^dagger M (FULL) or Mhat^dagger Mhat (EVEN / ODD), by CG.
 * b and x are float64 packed fields; x holds the initial guess on entry.  The
 * iterations run in params->sloppy with float64 reliable updates.  Synchronous. */
wd_status wd_cg_solve(wd_gauge g, double kappa, wd_subset subset, const wd_solver_params* params,
                      const void* b, void* x, wd_solver_info* info);
/* Solve M x = b on the full lattice through the even-odd Schur complement:
 * b'_e = b_e + kappa D_eo b_o, CG on Mhat^dagger Mhat x_e = Mhat^dagger b'_e,
 * x_o = b_o + kappa D_oe x_e.  b, x: FULL float64 packed fields.  Reports
 * ||b - M x|| / ||b|| in true_resid_M, in float64: the odd rows are zero by the
 * construction of x_o, up to its float64 rounding, and the even rows
 * b_e - x_e + kappa D_eo x_o equal b'_e - Mhat x_e.  When x_o is built from the
 * D_oe x_e of the solver's last float64 Schur residual (taken at the returned
 * x_e: a converged or capped solve, or a non-zero guess) that residual is the
 * even rows; otherwise one more float64 launch evaluates them with the x_o
 * built.  true_resid is the float64 ||b'_e - Mhat x_e|| / ||b|| that decides
 * convergence.  Synchronous. */
wd_status wd_wilson_solve(wd_gauge g, double kappa, const wd_solver_params* params,
                          const void* b, void* x, wd_solver_info* info);

/* ---- parallel-transport convolution (the learned preconditioner's layer) ----
 * A feature field holds C colour triplets per site on the whole lattice, in
 * float32, for nsamples independent samples.  Canonical layout:
 * [nsamples][C][T][Z][Y][X][3][2] doubles.  One layer maps C_in -> C_out
 * channels along nine paths p = 0 (stay), 1..4 (+x, +y, +z, +t), 5..8 (-x..-t):
 *     out^a(x) = sum_p sum_b W[p][a][b] (T_p in^b)(x),
 *     T_{+mu} f(x) = U_mu(x) s+ f(x + mu),  T_{-mu} f(x) = U_mu(x - mu)^dagger s- f(x - mu),
 * with the links and boundary signs of the gauge object (float32 links).
 * W: [9][C_out][C_in] complex, (re, im) pairs at wprec (F32, F16 or BF16).
 * C_in and C_out must be 1, 2, 3, 4 or 8. */
size_t wd_feature_bytes(const wd_lattice* lat, int channels, int nsamples);
wd_status wd_feature_pack(wd_context ctx, const wd_lattice* lat, int channels, int nsamples,
                          const double* canon, void* packed);
wd_status wd_feature_unpack(wd_context ctx, const wd_lattice* lat, int channels, int nsamples,
                            const void* packed, double* canon);
/* FULL float32 packed spinor <-> 4-channel features (channel = spin). */
wd_status wd_spinor_to_features(wd_context ctx, const wd_lattice* lat, int nsamples, const void* spinor, void* feat);
wd_status wd_features_to_spinor(wd_context ctx, const wd_lattice* lat, int nsamples, const void* feat, void* spinor);
wd_status wd_ptconv_forward(wd_gauge g, int cin, int cout, wd_prec wprec, int nsamples, const void* W,
                            const void* in, void* out);
/* Gradients for a real loss L, PyTorch's complex convention (dL/dRe + i dL/dIm):
 *   gin^b = sum_p T_p^dagger sum_a conj(W[p][a][b]) gout^a            (if gin != NULL)
 *   gW[p][a][b] = sum_x sum_c gout^a(x)_c conj((T_p in^b)(x)_c)      (if gW != NULL;
 *                 float32 complex, summed over samples in float64 partials) */
wd_status wd_ptconv_backward(wd_gauge g, int cin, int cout, wd_prec wprec, int nsamples, const void* W,
                             const void* in, const void* gout, void* gin, void* gW);

/* ---- batches: many lattices and right-hand sides in one launch --------------- */
typedef struct {
    wd_gauge gauge;    /* links and lattice of this item (all items: one context, one wd_recon) */
    int out_subset;    /* WD_EVEN (out_e = D_eo in_o) or WD_ODD (out_o = D_oe in_e)             */
    int dagger;        /* nonzero: D_hop^dagger                                                 */
    int nrhs;          /* right-hand sides: nrhs packed half fields, back to back               */
    const void* in;    /* packed input half fields (device)                                    */
    void* out;         /* packed output half fields (device)                                   */
} wd_batch_item;
/* Capture the even-odd hopping term of every item (lattices of any volume,
 * each with its own nrhs) as ONE persistent kernel launch in a hipGraph.
 * All items use precision prec.  The batch RETAINS the gauge objects and the
 * in/out pointers: they must stay valid until wd_batch_destroy.  Links are
 * packed at prec during this call.  The launch shape (tile width = workgroup
 * size 64 / 128 / 256 sites, persistent waves per compute unit 8 / 16 / 24 / 32,
 * software-pipelined directions or not) is autotuned here: every candidate is
 * launched on the batch's own buffers and timed (so the outputs are written,
 * with the batch's result), and the fastest is captured; wd_batch_shape
 * reports it.  Synchronous. */
wd_status wd_batch_create(wd_context ctx, int n, const wd_batch_item* items, wd_prec prec, wd_batch* out);
/* Replay the graph on the context's stream (one kernel launch).  Asynchronous.
 * The captured launch knows whether each item's links were in temporal gauge at
 * creation; if a gauge has been uploaded again or fixed since, so that this no
 * longer holds, nothing is launched and WD_EINVAL is returned (create the batch
 * again).  Uploading new links of the same state between runs is allowed: the
 * links are repacked in place. */
wd_status wd_batch_run(wd_batch b);
/* Number of tiles (one workgroup's output sites of one rhs) and persistent workgroups. */
wd_status wd_batch_info(wd_batch b, long long* ntiles, int* grid);
/* The captured launch shape: tile width (sites = workgroup size), persistent waves
 * per compute unit, software-pipelined directions (1) or not (0). */
wd_status wd_batch_shape(wd_batch b, int* block, int* waves_per_cu, int* pf);
wd_status wd_batch_destroy(wd_batch b);

/* ---- bandwidth reference ----------------------------------------------------- */
/* dst = src for `bytes` bytes (a multiple of 16) with a streaming 16-byte-per-
 * lane copy kernel: the achievable-bandwidth ceiling the dslash is compared
 * with, and the reference for hardware byte counters.  Asynchronous. */
wd_status wd_device_copy(wd_context ctx, const void* src, void* dst, size_t bytes);

/* Solve M x = b on the full lattice through the even-odd Schur complement with
 * BiCGstab on Mhat x_e = b_e + kappa D_eo b_o (paper, Section 7: the second
 * inverter).  The iteration's vectors are stored at params->sloppy (F64, F32,
 * or 16-bit with the per-site scale; arithmetic in float32, float64 for F64);
 * reliable updates recompute bhat - Mhat x in float64 when the iterated
 * residual drops below delta times its running maximum.  true_resid is ||bhat - Mhat x_e|| / ||b||,
 * true_resid_M the full-system ||b - M x|| / ||b|| (float64, even rows taken as
 * for wd_wilson_solve).  Synchronous. */
wd_status wd_bicgstab_solve(wd_gauge g, double kappa, const wd_solver_params* params, const void* b, void* x,
                            wd_solver_info* info);

/* ---- learned-preconditioner solve ---------------------------------------------- */
/* Solve M x = b on the full lattice (b, x: FULL float64 packed fields; x is the
 * initial guess).  The Krylov iteration is flexible GMRES on the even-odd Schur
 * complement Mhat (paper Section 4), right-preconditioned by the even-even block
 * of a network N ~ M^-1: K v_e = [N (v_e, 0)]_e, exact if N = M^-1.  N is a
 * stack of nlayers parallel-transport convolutions with channel widths
 * widths[0..nlayers] (widths[0] = widths[nlayers] = 4: spin as channels) and
 * weights[l] the [9][widths[l+1]][widths[l]] complex weights at wprec (device
 * pointers); nlayers = 0 runs unpreconditioned GMRES on Mhat.  Only the even
 * half of the initial guess is used.  Cycles of at most `restart` iterations
 * run in float32 on rhat = bhat - Mhat x_e (bhat = b_e + kappa D_eo b_o, both in
 * float64) and stop when their residual estimate has fallen by params->delta
 * (> 0; else 1e-5); x_e and rhat are updated in float64 after each cycle until
 * ||rhat|| / ||b|| <= params->tol; then x_o = b_o + kappa D_oe x_e, and the full
 * residual ||b - M x|| / ||b|| is reported (it equals ||rhat|| / ||b|| up to
 * rounding; taken as for wd_wilson_solve).  A NaN or a cycle that reduces the residual
 * less than tenfold hands x to wd_wilson_solve (fell_back = 1), whose float64
 * residual is reported.
 * With BF16 weights of widths 4 -> 8 -> ... -> 8 -> 4 the network keeps its hidden
 * features in bf16 (see wd_ptnet_apply_even).  restart must be in [1, 63].
 * WD_EINVAL: a null pointer, restart out of range, tol <= 0, a network not mapping
 * 4 to 4 channels or a weight precision other than F32 / F16 / BF16;
 * WD_EUNSUPPORTED: a width outside {1, 2, 3, 4, 8}.  Synchronous. */
wd_status wd_fgmres_solve(wd_gauge g, double kappa, const wd_solver_params* params, int restart, int nlayers,
                          const int* widths, const void* const* weights, wd_prec wprec, const void* b, void* x,
                          wd_solver_info* info);
/* The preconditioner of wd_fgmres_solve on its own: out = [N (in, 0)]_e, the even
 * sites of the network applied to the EVEN float32 spinor half field `in` extended
 * by zero odd sites (channel = spin, as in wd_spinor_to_features).  nlayers >= 1,
 * widths and weights as for wd_fgmres_solve.  With BF16 weights the layers mix
 * channels on the matrix cores (transported inputs rounded to bf16, float32
 * accumulation); a 4 -> 8 -> ... -> 8 -> 4 network then also stores its hidden
 * features as bf16 pairs, so each layer moves half the feature bytes.  in, out:
 * distinct device pointers to EVEN F32 half fields (wd_spinor_bytes(lat, WD_EVEN,
 * WD_F32, 1) bytes); the hidden features live in the context's workspace.
 * Asynchronous on the context's stream.  WD_EINVAL: a null pointer, in == out, a
 * network not mapping 4 to 4 channels, a bad weight precision; WD_EUNSUPPORTED: a
 * width outside {1, 2, 3, 4, 8}. */
wd_status wd_ptnet_apply_even(wd_gauge g, int nlayers, const int* widths, const void* const* weights, wd_prec wprec,
                              const void* in, void* out);

/* ---- launch-shape tuning --------------------------------------------------- */
/* Time every launch shape of the dslash kernels used with gauge g at precision
 * prec and nrhs right-hand sides (workgroup size 64..256, XCD-aware block
 * remap, non-temporal link loads, software-pipelined directions, a z-blocked
 * site traversal of depth zb dividing Z and, for nrhs > 1, right-hand sides
 * interleaved with the site tiles; for 16-bit storage with 12-real links and a
 * multiple of 16 rhs also the kernel that runs the colour multiply of 16 rhs on
 * the matrix cores), for both
 * dagger settings with and without the fused a x + b D in, and keep the
 * fastest in the context's tuning table.  If cache_path is not NULL the file
 * is read first and the whole table written back after.  Synchronous; uses
 * three scratch half fields of the context workspace. */
wd_status wd_autotune_dslash(wd_gauge g, wd_prec prec, int nrhs, const char* cache_path);
/* Write / read the tuning table as JSON (a missing file reads as empty). */
wd_status wd_tune_save(wd_context ctx, const char* path);
wd_status wd_tune_load(wd_context ctx, const char* path);
/* Look up one tuning entry by key; fills out6 = {block, remap, nt, pf,
 * rhs_inner, zb} and returns 1, or returns 0 if the key is absent. */
int wd_tune_get(wd_context ctx, const char* key, int* out6);
/* The same with up to n values {block, remap, nt, pf, rhs_inner, zb, mf}, mf = 1
 * when the dslash runs its colour multiply on the matrix cores (16-bit storage,
 * 12-real links, a multiple of 16 rhs); returns 1, or 0 if the key is absent. */
int wd_tune_get_n(wd_context ctx, const char* key, int* out, int n);

/* ---- environment overrides (measurement and testing; results do not change, except as noted) ----
 * WD_DSLASH_BLOCK, _REMAP, _NT, _PF, _RHS_INNER, _ZB  launch shape of an untuned dslash
 * WD_DSLASH_MFMA = 0 / 1   16-bit multi-rhs dslash off / on the matrix cores, tuned or not
 * WD_BATCH_BLOCK, _WAVES, _PF  force the batch launch shape (tile width 64..256, waves per
 *                          compute unit, pipelined directions 0 / 1) instead of tuning it
 * WD_BATCH_TUNE = 0        no batch tuning: 256-site tiles, 24 waves per compute unit
 * WD_PTCONV_MFMA = 0       PT-conv channel mixing on the vector units even with bf16 weights
 * WD_PTCONV_ZB = depth     z-block depth of the matrix-core PT-conv wave order (0: natural)
 * WD_PTCONV_PARITY_SKIP = 0  the network inside FGMRES computes every path and site and
 *                          goes through float32 feature tensors (for checking: the result of
 *                          WD_PTNET_F32_FEATURES = 1)
 * WD_PTNET_F32_FEATURES = 1  the network inside FGMRES keeps float32 hidden features where it
 *                          would keep bf16 ones (changes the result within the bf16 rounding)
 * WD_PTCONV_SPLIT = 0 / 1  the network's last layer (bf16 hidden features) splits each site
 *                          group's paths over two waves never / always (default: on lattices of
 *                          at most 2048 groups of 64 even sites; float32 summation order changes) */

#ifdef __cplusplus
}
#endif

#endif /* WDIRAC_H */
