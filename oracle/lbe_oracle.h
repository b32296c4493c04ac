/*
 * lbe_oracle.h -- plain FP64 CPU oracle of the stabilized Lattice
 * Boltzmann-Enskog step (double distribution, trapezoidal rule; Melchionna
 * and Marini Bettolo Marconi, arXiv:1202.3842).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no source, header, table or helper with the GPU library: the
 * configuration struct below is laid out like the GPU library's on purpose
 * so one Python harness can drive both, but it is declared independently.
 *
 * Everything is host memory, FP64, written for readability rather than
 * speed: explicit loops in the paper's notation, modular index arithmetic,
 * no blocking or fusion.  Loops over lattice nodes may run under OpenMP;
 * every reduction is evaluated in a fixed order so results do not depend on
 * the thread count.
 *
 * Node index: idx = x + nx*(y + ny*z).  Population arrays are
 * [19][N] per species and distribution (SoA), velocities are [3][N].
 * The stored state is the post-streaming transformed populations
 * f~ and g~ of Sec. 3 eq. (invertpops), i.e. the state at the start of a
 * step.
 */
#ifndef LBE_ORACLE_H
#define LBE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbeo_ctx lbeo_ctx;

enum {
  LBEO_OK = 0,
  LBEO_ERR_ARG = -1,
  LBEO_ERR_STATE = -2,
  LBEO_ERR_OOM = -3,
  LBEO_ERR_UNSTABLE = -5,
  LBEO_ERR_UNSUPPORTED = -6
};

/* Scheme switches (readings of the paper where it is ambiguous):
 *  VISC         include the collisional viscous force C^visc (Appendix,
 *               eq. viscousforce) in S_f, S_g and J (Sec. 4.2).
 *  PRINTED_INV  use the moment inversions as printed in Sec. 4.2
 *               (Pi = Pi~ - beta/2 C^mf.u^a, J = J~ + 1/2 (C^mf+C^visc+nF))
 *               instead of the ones derived from eq. (invertmoments).
 *  KAPPA4       use the printed coefficient 4 on H2.u^a in the C^mf part of
 *               S_g (Sec. 4.2, eq. kernel-g-1) instead of the projected 2.
 *  IDEAL        switch the collisional kernel off (C = 0, Sec. 4.1).
 * Scheme variants compared in Sec. 4 (default: DD-TR):
 *  EULER        Euler integration (EU, Sec. 4.1): f* = f + omega h (f_eq -
 *               f) + h S on the populations themselves, moments without
 *               half-step corrections.
 *  SINGLE       single distribution (SD): only f evolves (eqs.
 *               boltzoriginal and bolt2); its moments give n and J, and the
 *               trapezoidal inversion is J = J~ + h X/2 with X the first
 *               moment of S_f; g is not used (it is set to zero).
 *  DRAG         add the interspecies drag C^drag (Appendix, eq.
 *               dragforce2) to the dissipative forces: with u~_b = J~_b/n_b
 *               and the contact values G_ab(r),
 *               C^drag_a = -n_a sum_b 2 sigma_ab^2 sqrt(kT/pi) (4 pi/3)
 *                          G_ab n_b (u~_a - u~_b).
 *               It enters X and Y like C^visc (and is reported with it).
 * How the quasi-pressure Pi^a enters the step (Sec. 2).  The zeroth moment
 * of g is Pi^a by definition (eq. definition), and Pi^a is the potential
 * function of eq. quasipressure, which Sec. 2 evaluates numerically by the
 * trapezoidal rule.  Default: each step, after the forces, Pi^a is
 * evaluated at every node from the current C^{a,mf} (plus n^a F^a with
 * LBEO_QP_WITH_FEXT) as lbeo_quasipressure does, from the route origin and
 * with the route mode (default the box centre and the mean over the six
 * axis orders; lbeo_set_quasipressure_route), the zeroth
 * moment of g~ is set to the Pi~ that the inversion of Sec. 4.2 maps to
 * that Pi, and g_eq takes that Pi.  (Not with SINGLE, which has no g.)
 *  PI_CARRIED   the other reading: Pi is carried by g from its initial
 *               value, changed only by the zeroth source moment of
 *               eq. kernel-g-1, and no path integral is evaluated.
 *  BALL_FLUID   weighted densities average n_b over the fluid points of
 *               the ball only (normalised by their count); default: solid
 *               and out-of-domain points count as empty and the
 *               normalisation is the full ball size. */
enum {
  LBEO_VISC = 1u << 0,
  LBEO_PRINTED_INV = 1u << 1,
  LBEO_KAPPA4 = 1u << 2,
  LBEO_IDEAL = 1u << 3,
  LBEO_EULER = 1u << 4,
  LBEO_SINGLE = 1u << 5,
  LBEO_DRAG = 1u << 6,
  LBEO_PI_CARRIED = 1u << 7,
  LBEO_BALL_FLUID = 1u << 8
};

typedef struct {
  int nx, ny, nz;
  unsigned periodic;   /* bit0 = x, bit1 = y, bit2 = z                      */
  int nspecies;        /* M, 1..4                                            */
  double sigma[4];     /* hard-sphere diameters, lattice units               */
  double tau;          /* 1/omega of the BGK term, eq. (boltzoriginal)       */
  double kT;           /* k_B T with m = 1; D3Q19 needs kT = v_T^2 = 1/3     */
  int prec;            /* ignored: the oracle is FP64 throughout             */
  unsigned flags;      /* LBEO_* switches above                              */
  /* attractive molecular field G^{ab} (Appendix; our choice of U, which the */
  /* paper leaves open): U^{ab}(r) = -att_eps[a][b] (sigma_ab/r)^6 for        */
  /* sigma_ab <= r < att_rc, else 0; att_eps symmetric, >= 0 (0 = none)      */
  double att_eps[4][4];
  double att_rc;
} lbeo_config;

typedef struct {
  double mass[4];      /* sum over fluid nodes of n^a                        */
  double gmom[3];      /* sum over species and nodes of J~^a (from g~)       */
  double umax;         /* max |u| (barycentric, half-step corrected)         */
  double err_n;        /* max |n - n_eq| / n_0, n_eq the ideal-gas profile   */
  double err_u;        /* umax / v_T                                         */
  double err_J;        /* max |J| / (n_0 v_T)                                */
  int unstable;        /* 1 if a packing fraction >= 1 or a NaN was met      */
} lbeo_diag;

int  lbeo_create(const lbeo_config *cfg, lbeo_ctx **out);
void lbeo_destroy(lbeo_ctx *ctx);
const char *lbeo_last_error(void);
void lbeo_set_threads(int nthreads);

int lbeo_set_solid(lbeo_ctx *ctx, const uint8_t *mask);          /* N bytes */
int lbeo_set_potential(lbeo_ctx *ctx, const double *V);          /* N       */
int lbeo_set_body_force(lbeo_ctx *ctx, int species, const double g[3]);
int lbeo_init_density(lbeo_ctx *ctx, int species, const double *n0);
int lbeo_step(lbeo_ctx *ctx, int nsteps);
int lbeo_get_density(lbeo_ctx *ctx, int species, double *out);   /* N       */
int lbeo_get_velocity(lbeo_ctx *ctx, int species, double *out);  /* 3N, -1 = barycentric */
int lbeo_get_populations(lbeo_ctx *ctx, int species, int dist, double *out); /* 19N */
int lbeo_set_populations(lbeo_ctx *ctx, int species, int dist, const double *in);
int lbeo_diagnostics(lbeo_ctx *ctx, lbeo_diag *out);

/* ---- quasi-pressure (Sec. 2, eq. quasipressure) --------------------------- */
/* Pi^a(r) = n^a(r) - beta * (path integral from r0 to r of v^a . dr') with  */
/* v^a = C^{a,mf}, or C^{a,mf} + n^a F^a (the form printed in the equation)  */
/* with LBEO_QP_WITH_FEXT.  Trapezoidal rule on unit lattice steps along x,  */
/* then y, then z from the origin r0, which must be a fluid node; no step    */
/* crosses a periodic face.  Pi = 0 on solid nodes.                          */
#define LBEO_QP_WITH_FEXT 1u
/* mode bit: the mean of the integrals along the six axis orders (x,y,z),  */
/* (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x) instead of (x,y,z) alone;   */
/* it keeps the cubic symmetry of the lattice about the origin.            */
#define LBEO_QP_SYMMETRIC 2u
int lbeo_quasipressure(lbeo_ctx *ctx, int species, const int origin[3],
                       unsigned mode, double *out);                 /* N */
/* Sets the zeroth moment of every species' g~ to Pi~, the tilde value of    */
/* the quasi-pressure above at the current state, leaving f~ and the first   */
/* moment of g~ unchanged.  Not available with LBEO_SINGLE (no g).          */
int lbeo_init_quasipressure(lbeo_ctx *ctx, const int origin[3], unsigned mode);
/* Origin and mode (bits as above) of the per-step quasi-pressure (the      */
/* default reading, see PI_CARRIED); the origin must be a fluid node when a */
/* step runs.  Defaults: the box centre (nx/2, ny/2, nz/2) and              */
/* LBEO_QP_SYMMETRIC.                                                       */
int lbeo_set_quasipressure_route(lbeo_ctx *ctx, const int origin[3], unsigned mode);

/* ---- velocity divergence (Sec. 4.3, the D of the channel validation) ------ */
/* D = div_h u / (v_T / dx) of the barycentric velocity u, with the isotropic */
/* D3Q19 divergence (1/v_T^2) sum_p w_p c_p . u(r + c_p); u = 0 on solid     */
/* nodes and beyond non-periodic faces; D = 0 on solid nodes (N values).     */
int lbeo_get_divergence(lbeo_ctx *ctx, double *out);

/* ---- inspection entry points used by the pins ---------------------------- */
/* C^mf and C^visc of one species at the current state (3N each). */
int lbeo_get_forces(lbeo_ctx *ctx, int species, double *cmf, double *cvisc);
/* contact value G_ab at every node for the current state (N). */
int lbeo_get_contact(lbeo_ctx *ctx, int a, int b, double *G);
/* weighted (ball-averaged) density of one species (N). */
int lbeo_get_weighted_density(lbeo_ctx *ctx, int species, double *nbar);
/* external force per particle F^a = -grad_h V + body force (3N). */
int lbeo_get_external_force(lbeo_ctx *ctx, int species, double *F);
/* one streaming pass of one species' post-collision array (19N -> 19N). */
int lbeo_stream(lbeo_ctx *ctx, const double *post, double *out);

/* lattice shell of radius sigma: fills up to maxpts offsets (3 ints each,
 * the half shell S+ first, then the mirror images) and the uniform weight.
 * Returns the full point count, or a negative status. */
int lbeo_shell(double sigma, int maxpts, int *offs, double *weight);
/* ball of radius sigma/2: returns the point count, fills up to maxpts. */
int lbeo_ball(double sigma, int maxpts, int *offs);
/* BMCSL contact value of pair (a,b) from the weighted densities nbar[M]. */
double lbeo_bmcsl(int M, const double *sigma, const double *nbar, int a, int b);
/* the D3Q19 velocity set: c[19][3], w[19], opp[19]. */
void lbeo_d3q19(int *c, double *w, int *opp);

/* One-node collision of all M species, given the post-streaming populations
 * ft, gt ([M][19]), the nonlocal forces cmf, cvisc ([M][3]) and the external
 * force per particle F ([M][3]).  Writes the post-collision populations
 * fpost, gpost ([M][19]) and, if mom != NULL, per species
 * {n, Pi, J[3], u^a[3]} followed by the barycentric u[3] (8M+3 doubles). */
int lbeo_collide_node(int M, double tau, double kT, unsigned flags,
                      const double *ft, const double *gt,
                      const double *cmf, const double *cvisc, const double *F,
                      double *fpost, double *gpost, double *mom);

#ifdef __cplusplus
}
#endif
#endif
