/*
 * lbe.h -- C ABI of the MI355X (gfx950) stabilized Lattice Boltzmann-Enskog
 * library: one time step of the double-distribution, trapezoidal-rule
 * (DD-TR) scheme of Melchionna and Marini Bettolo Marconi, arXiv:1202.3842.
 *
 * The problem follows the paper's statement of it:
 *   - M species of hard spheres with diameters sigma_a and unit mass
 *     (Sec. 2; Appendix, sigma_ab = (sigma_aa + sigma_bb)/2);
 *   - an external potential U with force F = -grad U per particle and an
 *     optional uniform body force (Sec. 4.1 eq. extpotential, Sec. 4.3);
 *   - solid nodes with mid-point bounce-back walls for f and g (Sec. 4.3);
 *   - BGK relaxation with inverse time omega = 1/tau (Sec. 2,
 *     eq. boltzoriginal) on the D3Q19 lattice with h = dx = 1, v_T^2 = kT;
 *   - observables n^a and u^a (Sec. 4.1 error measures, Sec. 4.2 moments).
 *
 * One step computes, on the GPU only:
 *   moments n~, Pi~, J~ (Sec. 4.2); weighted densities and contact values;
 *   the Enskog mean-field force C^mf and the collisional viscous force
 *   C^visc on the tilde moments (Appendix; Sec. 3 eq. relatemoments);
 *   the inversions to n, Pi, J; equilibria and sources (Sec. 4.2
 *   eqs. kernel-f-1 .. kernel-g-1); the trapezoidal BGK update (Sec. 4.1);
 *   Lagrangian streaming with mid-point bounce-back (Sec. 4.1, 4.3).
 *
 * Conventions shared by every call:
 *   - Every call returns lbe_status; no C++ exception crosses the ABI.
 *     lbe_last_error() returns a thread-local text for the last failure.
 *   - Memory: all device memory of a context lives in ONE caller-owned
 *     device workspace of lbe_workspace_bytes() bytes, 256-byte aligned,
 *     passed to lbe_create; the library never allocates device memory and
 *     never frees the workspace.  Host inputs are copied before the call
 *     returns.  Device inputs (where = LBE_DEVICE) must stay valid until the
 *     stream reaches the call.
 *   - Streams: work is enqueued on the HIP stream given to lbe_create (NULL
 *     = the null stream).  Setters and lbe_step are asynchronous; the getters,
 *     lbe_diagnostics and lbe_synchronize block until their results are
 *     ready.
 *   - Layout: node index idx = x + nx*(y + ny*z).  Scalar fields hold N =
 *     nx*ny*nz values, vector fields 3N (component-major: all x, then y,
 *     then z), populations 19N (direction-major, D3Q19 order below).
 *     D3Q19 order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),
 *     (-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
 *     (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *   - Populations returned and accepted are the post-streaming transformed
 *     populations f~, g~ of eq. (invertpops) at the current step.
 *   - After LBE_ERR_UNSTABLE (a packing fraction xi3 >= 1 or a non-finite
 *     density was met) the context refuses lbe_step until lbe_init_density
 *     or lbe_set_populations is called.
 */
#ifndef LBE_H
#define LBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbe_ctx lbe_ctx;

typedef enum {
  LBE_OK = 0,
  LBE_ERR_ARG = -1,          /* invalid argument or configuration          */
  LBE_ERR_STATE = -2,        /* call not valid in the context's state       */
  LBE_ERR_OOM = -3,          /* workspace too small                         */
  LBE_ERR_HIP = -4,          /* a HIP runtime call failed                   */
  LBE_ERR_UNSTABLE = -5,     /* xi3 >= 1 or a non-finite density            */
  LBE_ERR_UNSUPPORTED = -6   /* configuration outside what is built          */
} lbe_status;

typedef enum {
  LBE_FP64 = 0,      /* populations stored in FP64                          */
  LBE_FP32_POP = 1   /* populations stored in FP32, all arithmetic in FP64  */
} lbe_precision;

enum { LBE_HOST = 0, LBE_DEVICE = 1 };   /* the 'where' of user pointers    */

/* Scheme switches (readings of the paper where it is ambiguous).
 *  LBE_VISC         include C^visc (Appendix, eq. viscousforce) in S_f,
 *                   S_g and the J inversion (Sec. 4.2).
 *  LBE_PRINTED_INV  the inversions as printed in Sec. 4.2:
 *                   J = J~ + (C^mf + C^visc + nF)/2,
 *                   Pi = Pi~ - (beta/2) C^mf.u^a; default is the reading
 *                   derived from eq. (invertmoments): J = J~ + (C^visc+nF)/2,
 *                   Pi = Pi~ + (beta/2) C^mf.u^a.
 *  LBE_KAPPA4       the printed coefficient 4 on H2.u^a in the C^mf part of
 *                   S_g (Sec. 4.2); default is 2, the Hermite projection.
 *  LBE_IDEAL        C = 0: the ideal fluid of Sec. 4.1.
 * Scheme variants compared in Sec. 4 (default DD-TR: double distribution,
 * trapezoidal rule):
 *  LBE_EULER        Euler integration (EU): f* = f + omega (f_eq - f) + S_f
 *                   (and g), moments without half-step terms.
 *  LBE_SINGLE       single distribution (SD): only f evolves; its moments
 *                   give n and J (J = J~ + X/2 with the trapezoidal rule,
 *                   X the first moment of S_f); the g populations are not
 *                   read or written (their getters return unspecified
 *                   values).
 *  LBE_DRAG         add the interspecies drag (Appendix, eq. dragforce2),
 *                   C^drag_a = -n_a sum_b 2 sigma_ab^2 sqrt(kT/pi) (4pi/3)
 *                   G_ab n_b (u~_a - u~_b) with u~ = J~/n, to the
 *                   dissipative forces (with C^visc in X, Y and
 *                   lbe_get_force(which = 1)); zero for one species.
 * How the quasi-pressure Pi enters the step (Sec. 2).  The zeroth moment of
 * g is Pi by definition (eq. definition), and Pi is the potential function
 * of eq. quasipressure, which Sec. 2 computes by trapezoidal integration.
 * Default: each step, after the forces, Pi is evaluated at every node as
 * lbe_get_quasipressure does, with the route of lbe_set_quasipressure_route
 * (default: origin at the box centre, the mean over the six axis orders);
 * the zeroth moment of g~ is set to the Pi~ that the inversion below maps
 * to that Pi, and g_eq takes Pi.  (Not with LBE_SINGLE, which has no g.)
 *  LBE_PI_CARRIED   the other reading: Pi is carried by g from its initial
 *                   value and changed only by the zeroth source moment of
 *                   eq. kernel-g-1; no path integral is evaluated.          */
enum {
  LBE_VISC = 1u << 0,
  LBE_PRINTED_INV = 1u << 1,
  LBE_KAPPA4 = 1u << 2,
  LBE_IDEAL = 1u << 3,
  LBE_EULER = 1u << 4,
  LBE_SINGLE = 1u << 5,
  LBE_DRAG = 1u << 6,
  LBE_PI_CARRIED = 1u << 7
};

#define LBE_MAX_SPECIES 4

typedef struct {
  int nx, ny, nz;         /* lattice size                                    */
  unsigned periodic;      /* bit0 = x, bit1 = y, bit2 = z; non-periodic
                             directions have solid walls just outside       */
  int nspecies;           /* M = 1..4                                        */
  double sigma[4];        /* diameters sigma_a in lattice units (0 = point)  */
  double tau;             /* 1/omega of the BGK term                         */
  double kT;              /* must be 1/3 (v_T^2 of D3Q19, m = 1)             */
  lbe_precision prec;     /* population storage                              */
  unsigned flags;         /* LBE_* switches                                  */
  /* Attractive molecular field G^{ab} of the Appendix (the last term of
   * C^{a,mf}).  The paper leaves U^{ab} open; this library takes the
   * attractive r^-6 tail U^{ab}(r) = -att_eps[a][b] (sigma_ab/r)^6 on
   * sigma_ab <= r < att_rc (0 elsewhere) with g_ab = 1 there, so that
   * G^{ab}(r) = sum_e U'(|e|) e^ n_b(r + e) over the lattice points of that
   * range, and C^{a,mf} gains n_a sum_b G^{ab}.  att_eps in energy units
   * (kT = 1/3), symmetric, >= 0; all zero = no attraction.  A pair with
   * att_eps > 0 needs sigma_ab > 0 and sigma_ab < att_rc, and the points
   * must reach at most 8 nodes per axis (att_rc <= 9).  Not with LBE_IDEAL
   * (which drops every nonlocal force).  In a batch, a box with the field
   * needs a non-empty hard-sphere shell (sigma >= 1/2). */
  double att_eps[4][4];
  double att_rc;
} lbe_config;

typedef struct {
  double mass[4];         /* sum over fluid nodes of n^a                     */
  double gmom[3];         /* sum over species and nodes of J~^a              */
  double umax;            /* max |u| (barycentric, half-step corrected)      */
  double err_n;           /* max |n - n_eq| / n_0, n_eq = ideal-gas profile  */
  double err_u;           /* umax / v_T (Sec. 4.1 Err(u))                    */
  double err_J;           /* max |J| / (n_0 v_T) (Sec. 4.1 Err(J))           */
  int unstable;           /* 1 after a packing fraction >= 1 or a NaN        */
} lbe_diag;

/* Bytes of device workspace a context with this configuration needs, or 0
 * if the configuration is invalid (lbe_last_error says why). */
size_t lbe_workspace_bytes(const lbe_config *cfg);

/* Create a context for one lattice box on the current HIP device.
 * dev_workspace: caller-owned device memory of at least
 * lbe_workspace_bytes(cfg) bytes (256-byte aligned); hip_stream: a
 * hipStream_t or NULL.  On success *out holds the context; the populations
 * are zero until lbe_init_density or lbe_set_populations. */
lbe_status lbe_create(const lbe_config *cfg, void *dev_workspace,
                      size_t bytes, void *hip_stream, lbe_ctx **out);

/* Solid mask (Sec. 4.3 walls): N bytes, nonzero = solid.  Populations at
 * solid nodes are cleared. */
lbe_status lbe_set_solid(lbe_ctx *ctx, const uint8_t *mask, int where);

/* External potential U per particle (Sec. 4.1 eq. extpotential), N values,
 * shared by all species; F = -grad_h U with the isotropic D3Q19 gradient
 * (1/v_T^2) sum_p w_p c_p U(r + c_p), wrapped in periodic directions and
 * clamped in the others. */
lbe_status lbe_set_potential(lbe_ctx *ctx, const double *V, int where);

/* Uniform body force per particle on one species (Sec. 4.3 forcing). */
lbe_status lbe_set_body_force(lbe_ctx *ctx, int species, const double g[3]);

/* Rest-equilibrium initial state f~ = g~ = w_p n0 on fluid nodes (so u = 0
 * and Pi = n at t = 0), N values. */
lbe_status lbe_init_density(lbe_ctx *ctx, int species, const double *n0,
                            int where);

/* Advance nsteps DD-TR steps, asynchronously on the context's stream.
 * Returns LBE_ERR_UNSTABLE if the context is poisoned by an earlier
 * instability; an instability met during these steps is reported by the
 * next lbe_diagnostics or getter. */
lbe_status lbe_step(lbe_ctx *ctx, int nsteps);

/* One phase of lbe_step, for instrumentation (e.g. HIP events around one
 * kernel): phase 0 = moments, 1 = contact values, 2 = nonlocal forces,
 * 3 = the per-step quasi-pressure (nothing with LBE_PI_CARRIED or
 * LBE_SINGLE), 4 = collision + streaming store + buffer swap.  Calling
 * phases 0..4 in order is exactly one lbe_step; any other order is rejected
 * with LBE_ERR_STATE. */
lbe_status lbe_step_phase(lbe_ctx *ctx, int phase);

/* n^a = sum_p f~_p (Sec. 4.2), N values. */
lbe_status lbe_get_density(lbe_ctx *ctx, int species, double *out, int where);

/* u^a = J^a/n^a after the inversion (including the half-step force term),
 * or the barycentric u = sum_a J^a / sum_a n^a for species = -1; 3N values,
 * zero on solid nodes. */
lbe_status lbe_get_velocity(lbe_ctx *ctx, int species, double *out, int where);

/* J^a = J~^a + (half-step force term) after the inversion (Sec. 4.2
 * eq. mom-g, with the inversion selected by the flags), or the total
 * sum_a J^a for species = -1; 3N values (component-major), zero on solid
 * nodes. */
lbe_status lbe_get_momentum(lbe_ctx *ctx, int species, double *out, int where);

/* C^mf (which = 0) or C^visc (which = 1) of one species at the current
 * state, 3N values. */
lbe_status lbe_get_force(lbe_ctx *ctx, int species, int which, double *out,
                         int where);

/* Post-streaming populations f~ (dist = 0) or g~ (dist = 1) of one species,
 * 19N values in the context's storage precision (double or float). */
lbe_status lbe_get_populations(lbe_ctx *ctx, int species, int dist, void *out,
                               int where);
lbe_status lbe_set_populations(lbe_ctx *ctx, int species, int dist,
                               const void *in, int where);

/* Divergence of the barycentric velocity, D = div u / (v_T/dx) (Sec. 4.3,
 * the quantity of the channel validation), N values.  The derivative is the
 * isotropic D3Q19 one, (1/v_T^2) sum_p w_p c_p . u(r + c_p) (a central
 * difference along each axis); u = 0 on solid nodes and beyond non-periodic
 * faces; D = 0 on solid nodes.  Uses the second population buffer as
 * scratch (the state is not changed); blocks until out is written. */
lbe_status lbe_get_divergence(lbe_ctx *ctx, double *out, int where);

/* ---- quasi-pressure (Sec. 2, eq. quasipressure) ----------------------------
 * Pi^a(r) = n^a(r) - beta * Phi^a(r), Phi^a the line integral of v^a from an
 * origin r0 to r, evaluated with the trapezoidal rule on unit lattice steps
 * (as the paper does) along a path that runs along the axes in turn: in the
 * order x, y, z, from r0 to (x, y0, z0), then to (x, y, z0), then to r (mode
 * 0), or, with LBE_QP_SYMMETRIC, the mean of the integrals over the six axis
 * orders, which keeps the cubic symmetry of the lattice about r0 (the
 * default route of the per-step quasi-pressure).  No step crosses a
 * periodic face.  The paper fixes no path.  Its equation integrates
 * v^a = C^{a,mf} + n^a F^a;
 * the discrete g source of Sec. 4.2 keeps n^a F^a as a force, so the Pi
 * that the discrete scheme carries at rest is the integral of C^{a,mf}
 * alone.  That is the default (mode 0); mode LBE_QP_WITH_FEXT adds
 * n^a F^a (F^a = -grad_h U + body force) as printed.  v = 0 on solid nodes.
 * Both calls evaluate C^mf and n at the current state.  Errors:
 * LBE_ERR_ARG for a null pointer, an origin outside the box or on a solid
 * node, or unknown mode bits; LBE_ERR_UNSTABLE if the state has a packing
 * fraction >= 1 or a non-finite density. */
enum { LBE_QP_WITH_FEXT = 1u, LBE_QP_SYMMETRIC = 2u };

/* Pi of one species, N values (0 on solid nodes); origin = {x0, y0, z0}.
 * Blocks until the result is in out.  The state is not changed.  Refused
 * inside a phased step (LBE_ERR_STATE). */
lbe_status lbe_get_quasipressure(lbe_ctx *ctx, int species, const int origin[3],
                                 unsigned mode, double *out, int where);

/* Initialiser for a non-uniform start (for example a density profile set by
 * lbe_init_density): for every species, sets the zeroth moment of the
 * post-streaming g~ to Pi~, the tilde value of the quasi-pressure above,
 * by adding w_p (Pi~ - sum_q g~_q) to each g~_p on fluid nodes.  f~ and the
 * first moment of g~ are unchanged.  Pi~ follows from Pi by the inversion
 * of Sec. 4.2 at the current u^a: Pi~ = Pi - (beta/2) C^mf.u^a (derived
 * reading), Pi + (beta/2) C^mf.u^a (LBE_PRINTED_INV), Pi (LBE_EULER).  The
 * integration constant (the value at r0) does not enter the evolution.
 * Asynchronous after the moment evaluation.  Errors as above, plus
 * LBE_ERR_ARG with LBE_SINGLE (no g) and LBE_ERR_STATE inside a phased
 * step. */
lbe_status lbe_init_quasipressure(lbe_ctx *ctx, const int origin[3], unsigned mode);

/* Route of the per-step quasi-pressure (the default reading above): origin
 * {x0, y0, z0}, a fluid node, and mode bits as above (default: the box
 * centre and LBE_QP_SYMMETRIC).  The integration constant (the value at the
 * origin) does not enter n or u.  Errors as above (LBE_SINGLE accepts a
 * route and ignores it); lbe_step returns LBE_ERR_STATE while the origin is
 * a solid node (lbe_set_solid may make it one). */
lbe_status lbe_set_quasipressure_route(lbe_ctx *ctx, const int origin[3], unsigned mode);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): Pi of one
 * species as lbe_get_quasipressure computes it (same origin, mode and
 * errors), written to the caller's DEVICE buffer out (N doubles).  Its line
 * scans work in a scratch array that the library holds on every GPU it runs
 * on until the process ends (64 MiB: boxes of at most 2796202 nodes; larger
 * ones give LBE_ERR_ARG), not in the context's workspace; it calls no
 * allocation routine.  All calls on one GPU share that GPU's array, so calls
 * that overlap on one GPU race.  Synchronises for the read-out pass (as
 * lbe_get_quasipressure does), then the scans run asynchronously on the
 * context's stream. */
lbe_status lbe_get_quasipressure_noalloc(lbe_ctx *ctx, int species, const int origin[3],
                                         unsigned mode, double *out);

/* Mass, g-momentum, spurious-current and Sec. 4.1 error measures of the
 * current state; synchronises. */
lbe_status lbe_diagnostics(lbe_ctx *ctx, lbe_diag *out);

/* Block until all work queued by the context has finished. */
lbe_status lbe_synchronize(lbe_ctx *ctx);

/* z planes per workgroup of the force kernel (a tiling parameter: results
 * do not depend on it; the autotuner sets it).  1 <= zchunk <= nz. */
lbe_status lbe_set_force_zchunk(lbe_ctx *ctx, int zchunk);

/* zchunk as above; the order in which the force kernel's tiles are handed
 * out: 0 = hardware order, 1 = each of the 8 XCDs (one L2 each) gets a
 * contiguous range of tiles, x fastest (default: same speed, about half the
 * L2 -> fabric traffic), 2 = the same with z fastest;
 * shape of the output tile: 0 = 32 x 8, 256 threads (default), 1 = 32 x 16,
 * 256 threads with two rows each, 2 = 32 x 16, 512 threads.  Tiling
 * parameters only: results do not depend on them. */
lbe_status lbe_set_force_tiling(lbe_ctx *ctx, int zchunk, int order, int shape);

/* ---- batched boxes --------------------------------------------------------
 * Many independent boxes of different sizes and diameters stepped
 * together: every phase of a step is one launch covering all boxes (one
 * force launch per directed species pair and distinct shell range), and the
 * launches of two steps are captured once in a HIP graph and replayed.  The
 * results are bitwise those of stepping each box alone.  All boxes must
 * share nspecies, prec and flags; with several species every pair's shell
 * must be non-empty (sigma_ab >= 1/2). */
typedef struct lbe_batch lbe_batch;

/* Device workspace for a batch of nboxes configurations, or 0 if invalid. */
size_t lbe_batch_workspace_bytes(const lbe_config *cfgs, int nboxes);

/* Create the batch and its member contexts (see lbe_batch_box) in one
 * caller-owned workspace, all on one HIP stream. */
lbe_status lbe_batch_create(const lbe_config *cfgs, int nboxes, void *dev_workspace,
                            size_t bytes, void *hip_stream, lbe_batch **out);

/* The member context of box i (owned by the batch): use it with every
 * single-box setter, getter and lbe_diagnostics. */
lbe_ctx *lbe_batch_box(lbe_batch *batch, int box);

/* Step every box nsteps times.  mode 0 = box after box with per-box
 * launches (the reference serial schedule), 1 = batched launches,
 * 2 = batched launches replayed from a captured HIP graph (default). */
lbe_status lbe_batch_step(lbe_batch *batch, int nsteps, int mode);

void lbe_batch_destroy(lbe_batch *batch);

/* ---- adjoint with respect to the external potential ----------------------
 * Reverse mode of nsteps steps of one box: the gradient dL/dV(r) of an
 * objective L of the final state, where V is the potential of
 * lbe_set_potential (the step's dependence on V runs through F = -grad_h V,
 * Sec. 4.1).  The objective enters through its derivatives with respect to
 * the read-outs of the final state: n^a (lbe_get_density), J^a
 * (lbe_get_momentum) and the post-streaming populations
 * (lbe_get_populations).  Supported: every force
 * (C^mf, C^visc, the attractive field, the interspecies drag), either
 * inversion and either kappa, either reading of Pi (the per-step
 * quasi-pressure, every route mode, or LBE_PI_CARRIED), in every scheme
 * variant (LBE_EULER, LBE_SINGLE), and either storage.  With LBE_FP32_POP
 * the result is the
 * reverse of the FP64 step along the trajectory of the stored FP32
 * populations (the rounding to storage is taken as the identity), with
 * the adjoint state in FP64.  Under LBE_SINGLE the scheme has no g, so the
 * g part of dL_dpop is ignored and the g gradient is zero.
 * Memory: the forward keeps a copy of the state every `segment` steps, and
 * the backward recomputes one segment at a time from its copy into a tape
 * of segment + 1 slots (each slot holds one step's fields: n, G, forces,
 * tilde moments), so device memory grows as nsteps/segment states plus
 * segment slots.  With segment >= nsteps the forward itself fills the tape
 * (nsteps + 1 slots) and the backward recomputes nothing.  The context's
 * potential, body forces, solid mask and quasi-pressure route must not
 * change between lbe_adjoint_forward and lbe_adjoint_backward: the backward
 * then fails with LBE_ERR_STATE. */
typedef struct lbe_adjoint lbe_adjoint;

/* Device workspace of an adjoint over nsteps steps checkpointed every
 * `segment` steps, or 0 if unsupported or invalid (lbe_last_error says
 * why). */
size_t lbe_adjoint_workspace_bytes(const lbe_config *cfg, int nsteps, int segment);

/* Attach an adjoint to a context, in a caller-owned device workspace (256-
 * byte aligned) of lbe_adjoint_workspace_bytes bytes.  The context must
 * outlive the adjoint. */
lbe_status lbe_adjoint_create(lbe_ctx *ctx, int nsteps, int segment, void *dev_workspace,
                              size_t bytes, lbe_adjoint **out);

/* Advance the context nsteps steps from its current state (the t = 0 of the
 * objective), keeping the checkpoints (or, in one segment, the tape). */
lbe_status lbe_adjoint_forward(lbe_adjoint *adj);

/* dL/dV from the derivatives of L with respect to the final read-outs, any
 * of which may be NULL (= 0): dL_dn M*N values (species-major), dL_dJ 3M*N
 * ([species][component][node]), dL_dpop 2*M*19*N ([dist][species][p][node],
 * post-streaming populations).  where: LBE_HOST or LBE_DEVICE for the three
 * inputs; dL_dV: N values at where_out.  Synchronises. */
lbe_status lbe_adjoint_backward(lbe_adjoint *adj, const double *dL_dn, const double *dL_dJ,
                                const double *dL_dpop, int where, double *dL_dV, int where_out);

/* After lbe_adjoint_backward: dL/d(post-streaming populations at t = 0) of
 * one species and distribution, 19N values (zero on solid nodes). */
lbe_status lbe_adjoint_state_grad(lbe_adjoint *adj, int species, int dist, double *out,
                                  int where);

/* Test hook of the reverse sweep, for the dot-product tests of its
 * transposes: applies one linear stage K of the step, or (transpose = 1)
 * its transpose K^T as the reverse sweep computes it, at the fields of the
 * context's current state.  in and out are device pointers (FP64, no
 * overlap); the call runs on the context's stream and synchronises.
 *   LBE_PROBE_GRAD: K V = -grad_h V, the lattice gradient of the external
 *     potential (Sec. 4.1, F = -grad U; wrapped where periodic, clamped at
 *     walls); in N values, out 3N ([component][node]).
 *   LBE_PROBE_STREAM: pull streaming with mid-point bounce-back (Sec. 4.1,
 *     Sec. 4.3), both distributions; in and out in the population layout
 *     [dist][species][p][Ns] with Ns = N rounded up to a multiple of 64.
 *   LBE_PROBE_SHELL_N: the mean-field shell gather C^mf_a/n_a (Appendix) of
 *     every species, as a function of the densities n_b with the state's
 *     contact values; in M*N, out 3M*N ([species][component][node]).
 *   LBE_PROBE_SHELL_G: the same gather as a function of the contact values
 *     G_ab (pairs a <= b in the order (0,0), (0,1), ..., (1,1), ...) with the
 *     state's densities; in M(M+1)/2 * N, out 3M*N.
 *   LBE_PROBE_QP: the path integral Phi of eq. quasipressure along the
 *     context's route (no n F term) as a function of its integrand v; in
 *     3M*N, out M*N.  Needs the quasi-pressure evaluated every step.
 * The context's derived fields (densities, contact values, forces, Phi) are
 * overwritten; its populations are not, and the next step recomputes the
 * rest.  LBE_ERR_UNSUPPORTED for LBE_PROBE_STREAM with LBE_SINGLE, the
 * shell probes with LBE_IDEAL or an attractive field, and LBE_PROBE_QP with
 * LBE_PI_CARRIED or LBE_SINGLE. */
enum { LBE_PROBE_GRAD = 0, LBE_PROBE_STREAM = 1, LBE_PROBE_SHELL_N = 2, LBE_PROBE_SHELL_G = 3, LBE_PROBE_QP = 4 };
lbe_status lbe_adjoint_probe(lbe_adjoint *adj, int stage, int transpose, const double *in, double *out);

void lbe_adjoint_destroy(lbe_adjoint *adj);

/* Thread-local text of the last failure (never NULL). */
const char *lbe_last_error(void);

/* Release the context (never frees the caller's workspace). */
void lbe_destroy(lbe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
