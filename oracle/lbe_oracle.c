/*
 * lbe_oracle.c -- plain FP64 CPU oracle of one stabilized Lattice
 * Boltzmann-Enskog step, double distribution + trapezoidal rule (DD-TR),
 * after Melchionna and Marini Bettolo Marconi, arXiv:1202.3842.
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU library and is never part of
 * the product path.  It shares no code with the GPU library.
 *
 * The step follows the paper's order:
 *   1. moments n~, Pi~, J~ of the post-streaming populations
 *      (Sec. 4.2, eqs. mom-f-1-1 .. mom-g-1-1);
 *   2. weighted densities and contact values g_ab (Appendix; the averaging
 *      rule is our reading, see compute_contact());
 *   3. the Enskog mean-field force C^mf and, optionally, the collisional
 *      viscous force C^visc evaluated on the tilde moments (Sec. 3,
 *      eq. relatemoments; Appendix eqs. for C^mf and viscousforce);
 *   4. the inversion to the physical moments n, Pi, J (Sec. 4.2, eqs.
 *      mom-f .. mom-g, in the reading derived from eq. invertmoments);
 *   5. equilibria and sources f_eq, g_eq, S_f, S_g (Sec. 4.2,
 *      eqs. kernel-f-1 .. kernel-g-1);
 *   6. the trapezoidal BGK collision in closed form (Sec. 4.1, the update
 *      following eq. newevolution);
 *   7. streaming with mid-point bounce-back (Sec. 4.1 and Sec. 4.3).
 *
 * Units: h = dx = 1, m = 1, v_T^2 = kT, beta = 1/kT (Sec. 2, Sec. 4.1).
 */
#include "lbe_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define MAXM 4

/* ------------------------------------------------------------------------ */
/* D3Q19 velocity set and weights (a Gauss-Hermite quadrature, Sec. 3).     */
/* ------------------------------------------------------------------------ */
static const int CV[Q][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int OPPOSITE[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10,
                                9, 12, 11, 14, 13, 16, 15, 18, 17};
static double WEIGHT(int p) {
  if (p == 0) return 1.0 / 3.0;
  if (p <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

void lbeo_d3q19(int *c, double *w, int *opp) {
  for (int p = 0; p < Q; ++p) {
    for (int i = 0; i < 3; ++i) c[3 * p + i] = CV[p][i];
    w[p] = WEIGHT(p);
    opp[p] = OPPOSITE[p];
  }
}

/* ------------------------------------------------------------------------ */
/* error text                                                               */
/* ------------------------------------------------------------------------ */
static _Thread_local char g_err[512];
const char *lbeo_last_error(void) { return g_err; }
static int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

void lbeo_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* ------------------------------------------------------------------------ */
/* Shells and balls.                                                        */
/* The angular integral over the unit sphere in the Appendix (C^mf and      */
/* C^visc) is discretised on the lattice points whose distance lies in      */
/* [sigma - 1/2, sigma + 1/2), each with direction e/|e| and one uniform    */
/* weight 4 pi sigma / sum |e|; the paper does not give a discretisation,   */
/* this is our reading (it makes sum_e w e_i e_j/|e| = (4 pi/3) sigma       */
/* delta_ij, the continuum value).                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int npts;        /* full shell size                                    */
  int nplus;       /* half shell S+ (one of each +-e pair)               */
  int (*off)[3];   /* S+ first (nplus), then the mirror images           */
  double (*ehat)[3];
  double weight;   /* 4 pi sigma / sum |e|                                */
  double sigma;
} shell_t;

typedef struct {
  int npts;
  int (*off)[3];
} ball_t;

/* ------------------------------------------------------------------------ */
/* Attractive molecular field (Appendix: G^{ab} = -int dr' n_b(r')          */
/* g_ab(r,r') grad U^{ab}(r - r')).  The paper leaves U^{ab} open; our      */
/* choice is the attractive r^-6 tail U = -eps (sigma_ab/r)^6 for           */
/* sigma_ab <= r < rc (0 elsewhere) with g_ab = 1 there (mean field).  On   */
/* the lattice (dx^3 = 1) with r' = r + e:                                   */
/*   G^{ab}(r) = sum_e U'(|e|) e^ n_b(r + e),  U'(r) = 6 eps sigma^6 r^-7,   */
/* over the thick shell sigma_ab <= |e| < rc, summed as +-e pairs over the  */
/* half S+ so that a uniform state gives exactly zero.                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nplus;       /* points of S+                                        */
  int (*off)[3];
  double (*K)[3];  /* U'(|e|) e^                                           */
} att_t;

static int build_att(double sab, double eps, double rc, att_t *t) {
  memset(t, 0, sizeof *t);
  if (!(eps > 0.0) || !(sab > 0.0) || !(rc > sab)) return 0;
  int K = (int)ceil(rc);
  int cap = (2 * K + 1) * (2 * K + 1) * (2 * K + 1);
  t->off = malloc(sizeof(int[3]) * (size_t)cap);
  t->K = malloc(sizeof(double[3]) * (size_t)cap);
  if (!t->off || !t->K) return 1;
  double s6 = pow(sab, 6.0);
  for (int z = -K; z <= K; ++z)
    for (int y = -K; y <= K; ++y)
      for (int x = -K; x <= K; ++x) {
        int plus = z != 0 ? z > 0 : (y != 0 ? y > 0 : x > 0);
        if (!plus) continue;
        double r = sqrt((double)(x * x + y * y + z * z));
        if (r < sab || r >= rc) continue;
        double dU = 6.0 * eps * s6 / pow(r, 7.0);
        t->off[t->nplus][0] = x;
        t->off[t->nplus][1] = y;
        t->off[t->nplus][2] = z;
        t->K[t->nplus][0] = dU * x / r;
        t->K[t->nplus][1] = dU * y / r;
        t->K[t->nplus][2] = dU * z / r;
        t->nplus++;
      }
  return 0;
}

static void free_att(att_t *t) {
  free(t->off);
  free(t->K);
  memset(t, 0, sizeof *t);
}

static int in_shell(double sigma, int ex, int ey, int ez) {
  if (ex == 0 && ey == 0 && ez == 0) return 0;
  double r2 = (double)(ex * ex + ey * ey + ez * ez);
  double lo = sigma - 0.5, hi = sigma + 0.5;
  double lo2 = lo > 0 ? lo * lo : 0.0;
  return r2 >= lo2 && r2 < hi * hi;
}

/* canonical half: first nonzero component positive */
static int is_plus(int ex, int ey, int ez) {
  if (ex != 0) return ex > 0;
  if (ey != 0) return ey > 0;
  return ez > 0;
}

static int build_shell(double sigma, shell_t *s) {
  memset(s, 0, sizeof *s);
  s->sigma = sigma;
  if (sigma < 0.5) return 0; /* no lattice point can lie on the shell */
  int K = (int)ceil(sigma + 0.5);
  int count = 0;
  for (int ez = -K; ez <= K; ++ez)
    for (int ey = -K; ey <= K; ++ey)
      for (int ex = -K; ex <= K; ++ex)
        if (in_shell(sigma, ex, ey, ez)) ++count;
  s->npts = count;
  s->nplus = count / 2;
  if (count == 0) return 0;
  s->off = malloc(sizeof(int[3]) * (size_t)count);
  s->ehat = malloc(sizeof(double[3]) * (size_t)count);
  if (!s->off || !s->ehat) return -1;
  int k = 0;
  for (int ez = -K; ez <= K; ++ez)
    for (int ey = -K; ey <= K; ++ey)
      for (int ex = -K; ex <= K; ++ex)
        if (in_shell(sigma, ex, ey, ez) && is_plus(ex, ey, ez)) {
          s->off[k][0] = ex;
          s->off[k][1] = ey;
          s->off[k][2] = ez;
          ++k;
        }
  for (int j = 0; j < s->nplus; ++j) {
    s->off[s->nplus + j][0] = -s->off[j][0];
    s->off[s->nplus + j][1] = -s->off[j][1];
    s->off[s->nplus + j][2] = -s->off[j][2];
  }
  double sumlen = 0.0;
  for (int j = 0; j < count; ++j) {
    double len = sqrt((double)(s->off[j][0] * s->off[j][0] +
                               s->off[j][1] * s->off[j][1] +
                               s->off[j][2] * s->off[j][2]));
    for (int i = 0; i < 3; ++i) s->ehat[j][i] = s->off[j][i] / len;
    sumlen += len;
  }
  s->weight = 4.0 * M_PI * sigma / sumlen;
  return 0;
}

static void free_shell(shell_t *s) {
  free(s->off);
  free(s->ehat);
  memset(s, 0, sizeof *s);
}

/* Ball of radius sigma/2 used to average the density before the contact
 * value is evaluated (our reading; the paper defers the prescription of
 * g_ab to its reference JCP2011). */
static int build_ball(double sigma, ball_t *b) {
  double R = 0.5 * sigma;
  int K = (int)floor(R);
  int count = 0;
  for (int dz = -K; dz <= K; ++dz)
    for (int dy = -K; dy <= K; ++dy)
      for (int dx = -K; dx <= K; ++dx)
        if ((double)(dx * dx + dy * dy + dz * dz) <= R * R) ++count;
  b->npts = count;
  b->off = malloc(sizeof(int[3]) * (size_t)count);
  if (!b->off) return -1;
  int k = 0;
  for (int dz = -K; dz <= K; ++dz)
    for (int dy = -K; dy <= K; ++dy)
      for (int dx = -K; dx <= K; ++dx)
        if ((double)(dx * dx + dy * dy + dz * dz) <= R * R) {
          b->off[k][0] = dx;
          b->off[k][1] = dy;
          b->off[k][2] = dz;
          ++k;
        }
  return 0;
}

int lbeo_shell(double sigma, int maxpts, int *offs, double *weight) {
  shell_t s;
  if (build_shell(sigma, &s)) return fail(LBEO_ERR_OOM, "out of memory");
  for (int j = 0; j < s.npts && j < maxpts; ++j)
    for (int i = 0; i < 3; ++i) offs[3 * j + i] = s.off[j][i];
  if (weight) *weight = s.weight;
  int n = s.npts;
  free_shell(&s);
  return n;
}

int lbeo_ball(double sigma, int maxpts, int *offs) {
  ball_t b;
  if (build_ball(sigma, &b)) return fail(LBEO_ERR_OOM, "out of memory");
  for (int j = 0; j < b.npts && j < maxpts; ++j)
    for (int i = 0; i < 3; ++i) offs[3 * j + i] = b.off[j][i];
  int n = b.npts;
  free(b.off);
  return n;
}

/* ------------------------------------------------------------------------ */
/* Contact value of the pair distribution at contact, g_ab (Appendix).      */
/* The paper gives no closed form; we take the Boublik-Mansoori-Carnahan-   */
/* Starling-Leland expression in the weighted densities,                    */
/*   xi_k = (pi/6) sum_b sigma_b^k nbar_b,  d_ab = s_a s_b / (s_a + s_b),   */
/*   g_ab = 1/(1-xi3) + 3 d_ab xi2/(1-xi3)^2 + 2 d_ab^2 xi2^2/(1-xi3)^3,    */
/* which is Carnahan-Starling (1 - eta/2)/(1-eta)^3 for one species.        */
/* ------------------------------------------------------------------------ */
double lbeo_bmcsl(int M, const double *sigma, const double *nbar, int a,
                  int b) {
  double xi2 = 0.0, xi3 = 0.0;
  for (int k = 0; k < M; ++k) {
    xi2 += sigma[k] * sigma[k] * nbar[k];
    xi3 += sigma[k] * sigma[k] * sigma[k] * nbar[k];
  }
  xi2 *= M_PI / 6.0;
  xi3 *= M_PI / 6.0;
  double ssum = sigma[a] + sigma[b];
  double d = ssum > 0.0 ? sigma[a] * sigma[b] / ssum : 0.0;
  double one = 1.0 - xi3;
  return 1.0 / one + 3.0 * d * xi2 / (one * one) +
         2.0 * d * d * xi2 * xi2 / (one * one * one);
}

/* Hermite tensors of the velocity set (Sec. 4.1) */
typedef struct {
  double H1[Q][3], H2[Q][3][3];
} hermite_t;
static void hermite_tables(double vT2, hermite_t *t);

/* ------------------------------------------------------------------------ */
/* context                                                                  */
/* ------------------------------------------------------------------------ */
struct lbeo_ctx {
  lbeo_config cfg;
  int nx, ny, nz, M;
  long N;
  double vT2, beta, omega;
  uint8_t *solid;
  double *V;          /* external potential (per particle), N            */
  double *FV;         /* -grad_h V, 3N                                    */
  double body[MAXM][3];
  double *f, *g;      /* post-streaming populations [M][Q][N]             */
  double *fpost, *gpost;
  double *n, *Pit, *Jt, *ut;   /* [M][N], [M][N], [M][3][N], [M][3][N]    */
  double *nbar;                /* [M][N]                                  */
  double *G;                   /* [M][M][N], symmetric                    */
  double *cmf, *cvisc;         /* [M][3][N]                               */
  shell_t shell[MAXM][MAXM];   /* symmetric, [a][b] built for a <= b      */
  att_t att[MAXM][MAXM];       /* attractive tails, [a][b] for a <= b     */
  hermite_t herm;
  ball_t ball[MAXM];
  int unstable;
  /* per-step quasi-pressure (the default reading) */
  int qp_origin[3];
  unsigned qp_mode;
  double *pi;                  /* [M][N] Pi of eq. quasipressure          */
  double *qpx, *qpy;           /* running leg sums, max(n) and max(n)^2   */
  double *qpphi, *qpsum;       /* one axis order's Phi and the sum, N     */
};

static inline long IDX(const lbeo_ctx *c, int x, int y, int z) {
  return (long)x + (long)c->nx * ((long)y + (long)c->ny * (long)z);
}

/* Map a coordinate into the box; returns 0 if it falls outside a
 * non-periodic direction (out-of-domain nodes behave as solid). */
static inline int wrap1(int *x, int n, int periodic) {
  if (*x >= 0 && *x < n) return 1;
  if (!periodic) return 0;
  int r = *x % n;
  if (r < 0) r += n;
  *x = r;
  return 1;
}

/* index of r + d, or -1 if outside the domain */
static inline long neighbour(const lbeo_ctx *c, int x, int y, int z, int dx,
                             int dy, int dz) {
  int X = x + dx, Y = y + dy, Z = z + dz;
  if (!wrap1(&X, c->nx, c->cfg.periodic & 1u)) return -1;
  if (!wrap1(&Y, c->ny, c->cfg.periodic & 2u)) return -1;
  if (!wrap1(&Z, c->nz, c->cfg.periodic & 4u)) return -1;
  return IDX(c, X, Y, Z);
}

static inline int is_fluid(const lbeo_ctx *c, long i) {
  return i >= 0 && !c->solid[i];
}

static void free_ctx(lbeo_ctx *c) {
  if (!c) return;
  free(c->solid);
  free(c->V);
  free(c->FV);
  free(c->f);
  free(c->g);
  free(c->fpost);
  free(c->gpost);
  free(c->n);
  free(c->Pit);
  free(c->Jt);
  free(c->ut);
  free(c->nbar);
  free(c->G);
  free(c->cmf);
  free(c->cvisc);
  free(c->pi);
  free(c->qpx);
  free(c->qpy);
  free(c->qpphi);
  free(c->qpsum);
  for (int a = 0; a < MAXM; ++a) {
    for (int b = a; b < MAXM; ++b) {
      free_shell(&c->shell[a][b]);
      free_att(&c->att[a][b]);
    }
    free(c->ball[a].off);
  }
  free(c);
}

void lbeo_destroy(lbeo_ctx *ctx) { free_ctx(ctx); }

static void compute_external_force(lbeo_ctx *c);

int lbeo_create(const lbeo_config *cfg, lbeo_ctx **out) {
  if (!cfg || !out) return fail(LBEO_ERR_ARG, "null argument");
  *out = NULL;
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
    return fail(LBEO_ERR_ARG, "box dimensions must be positive");
  if (cfg->nspecies < 1 || cfg->nspecies > MAXM)
    return fail(LBEO_ERR_ARG, "nspecies must be 1..4");
  if (!(cfg->tau > 0.0)) return fail(LBEO_ERR_ARG, "tau must be positive");
  if (fabs(cfg->kT - 1.0 / 3.0) > 1e-12)
    return fail(LBEO_ERR_ARG, "D3Q19 requires kT = v_T^2 = 1/3 (m = 1)");
  for (int a = 0; a < cfg->nspecies; ++a)
    if (!(cfg->sigma[a] >= 0.0))
      return fail(LBEO_ERR_ARG, "sigma must be >= 0");
  for (int a = 0; a < cfg->nspecies; ++a)
    for (int b = 0; b < cfg->nspecies; ++b) {
      double e = cfg->att_eps[a][b];
      if (!(e >= 0.0) || e != cfg->att_eps[b][a])
        return fail(LBEO_ERR_ARG, "att_eps must be symmetric and >= 0");
      double sab = 0.5 * (cfg->sigma[a] + cfg->sigma[b]);
      if (e > 0.0 && !(sab > 0.0 && cfg->att_rc > sab))
        return fail(LBEO_ERR_ARG, "an attractive pair needs sigma_ab > 0 and att_rc > sigma_ab");
      if (e > 0.0 && (cfg->flags & LBEO_IDEAL))
        return fail(LBEO_ERR_ARG, "LBEO_IDEAL drops the attractive field");
    }
  lbeo_ctx *c = calloc(1, sizeof *c);
  if (!c) return fail(LBEO_ERR_OOM, "out of memory");
  c->cfg = *cfg;
  c->nx = cfg->nx;
  c->ny = cfg->ny;
  c->nz = cfg->nz;
  c->M = cfg->nspecies;
  c->N = (long)cfg->nx * cfg->ny * cfg->nz;
  c->vT2 = cfg->kT;
  c->beta = 1.0 / cfg->kT;
  c->omega = 1.0 / cfg->tau;
  long N = c->N;
  int M = c->M;
  c->solid = calloc((size_t)N, 1);
  c->V = calloc((size_t)N, sizeof(double));
  c->FV = calloc((size_t)3 * N, sizeof(double));
  c->f = calloc((size_t)M * Q * N, sizeof(double));
  c->g = calloc((size_t)M * Q * N, sizeof(double));
  c->fpost = calloc((size_t)M * Q * N, sizeof(double));
  c->gpost = calloc((size_t)M * Q * N, sizeof(double));
  c->n = calloc((size_t)M * N, sizeof(double));
  c->Pit = calloc((size_t)M * N, sizeof(double));
  c->Jt = calloc((size_t)M * 3 * N, sizeof(double));
  c->ut = calloc((size_t)M * 3 * N, sizeof(double));
  c->nbar = calloc((size_t)M * N, sizeof(double));
  c->G = calloc((size_t)M * M * N, sizeof(double));
  c->cmf = calloc((size_t)M * 3 * N, sizeof(double));
  c->cvisc = calloc((size_t)M * 3 * N, sizeof(double));
  c->pi = calloc((size_t)M * N, sizeof(double));
  int nmax = c->nx > c->ny ? c->nx : c->ny;
  if (c->nz > nmax) nmax = c->nz;
  c->qpx = calloc((size_t)nmax, sizeof(double));
  c->qpy = calloc((size_t)nmax * nmax, sizeof(double));
  c->qpphi = calloc((size_t)N, sizeof(double));
  c->qpsum = calloc((size_t)N, sizeof(double));
  c->qp_origin[0] = c->nx / 2;
  c->qp_origin[1] = c->ny / 2;
  c->qp_origin[2] = c->nz / 2;
  c->qp_mode = LBEO_QP_SYMMETRIC;
  if (!c->solid || !c->V || !c->FV || !c->f || !c->g || !c->fpost ||
      !c->gpost || !c->n || !c->Pit || !c->Jt || !c->ut || !c->nbar ||
      !c->G || !c->cmf || !c->cvisc || !c->pi || !c->qpx || !c->qpy || !c->qpphi || !c->qpsum) {
    free_ctx(c);
    return fail(LBEO_ERR_OOM, "out of memory");
  }
  for (int a = 0; a < M; ++a) {
    for (int b = a; b < M; ++b) {
      double sab = 0.5 * (cfg->sigma[a] + cfg->sigma[b]);
      if (build_shell(sab, &c->shell[a][b]) ||
          build_att(sab, cfg->att_eps[a][b], cfg->att_rc, &c->att[a][b])) {
        free_ctx(c);
        return fail(LBEO_ERR_OOM, "out of memory");
      }
    }
    if (build_ball(cfg->sigma[a], &c->ball[a])) {
      free_ctx(c);
      return fail(LBEO_ERR_OOM, "out of memory");
    }
  }
  hermite_tables(c->vT2, &c->herm);
  compute_external_force(c);
  *out = c;
  g_err[0] = 0;
  return LBEO_OK;
}

/* the default reading: Pi evaluated by the path integral every step */
static int qp_per_step(const lbeo_ctx *c) {
  return !(c->cfg.flags & (LBEO_PI_CARRIED | LBEO_SINGLE));
}

static const shell_t *pair_shell(const lbeo_ctx *c, int a, int b) {
  return a <= b ? &c->shell[a][b] : &c->shell[b][a];
}

/* ------------------------------------------------------------------------ */
/* External force per particle, F = -grad U (Sec. 4.1), on the lattice as   */
/* the isotropic D3Q19 gradient grad_h V = (1/v_T^2) sum_p w_p c_p V(r+c_p) */
/* (our reading: exact for per-node V).  Periodic directions wrap,          */
/* non-periodic ones clamp to the box.                                      */
/* ------------------------------------------------------------------------ */
static void compute_external_force(lbeo_ctx *c) {
  long N = c->N;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->nz; ++z)
    for (int y = 0; y < c->ny; ++y)
      for (int x = 0; x < c->nx; ++x) {
        long i = IDX(c, x, y, z);
        double grad[3] = {0, 0, 0};
        for (int p = 1; p < Q; ++p) {
          int X = x + CV[p][0], Y = y + CV[p][1], Z = z + CV[p][2];
          if (!wrap1(&X, c->nx, c->cfg.periodic & 1u)) X = X < 0 ? 0 : c->nx - 1;
          if (!wrap1(&Y, c->ny, c->cfg.periodic & 2u)) Y = Y < 0 ? 0 : c->ny - 1;
          if (!wrap1(&Z, c->nz, c->cfg.periodic & 4u)) Z = Z < 0 ? 0 : c->nz - 1;
          double v = c->V[IDX(c, X, Y, Z)];
          for (int k = 0; k < 3; ++k) grad[k] += WEIGHT(p) * CV[p][k] * v;
        }
        for (int k = 0; k < 3; ++k) c->FV[k * N + i] = -grad[k] / c->vT2;
      }
}

static inline double ext_force(const lbeo_ctx *c, int a, int k, long i) {
  return c->FV[(long)k * c->N + i] + c->body[a][k];
}

/* ------------------------------------------------------------------------ */
/* setters / getters                                                        */
/* ------------------------------------------------------------------------ */
static int check_species(const lbeo_ctx *c, int a) {
  return a >= 0 && a < c->M;
}

int lbeo_set_solid(lbeo_ctx *c, const uint8_t *mask) {
  if (!c || !mask) return fail(LBEO_ERR_ARG, "null argument");
  for (long i = 0; i < c->N; ++i) c->solid[i] = mask[i] ? 1 : 0;
  for (int a = 0; a < c->M; ++a)
    for (int p = 0; p < Q; ++p)
      for (long i = 0; i < c->N; ++i)
        if (c->solid[i]) {
          c->f[((long)a * Q + p) * c->N + i] = 0.0;
          c->g[((long)a * Q + p) * c->N + i] = 0.0;
        }
  return LBEO_OK;
}

int lbeo_set_potential(lbeo_ctx *c, const double *V) {
  if (!c || !V) return fail(LBEO_ERR_ARG, "null argument");
  memcpy(c->V, V, sizeof(double) * (size_t)c->N);
  compute_external_force(c);
  return LBEO_OK;
}

int lbeo_set_body_force(lbeo_ctx *c, int a, const double gb[3]) {
  if (!c || !gb) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  for (int k = 0; k < 3; ++k) c->body[a][k] = gb[k];
  return LBEO_OK;
}

/* Initial state (our reading; the paper is silent): rest equilibrium in the
 * transformed variables, f~ = g~ = w_p n0, i.e. u = 0 and Pi(0) = n(0). */
int lbeo_init_density(lbeo_ctx *c, int a, const double *n0) {
  if (!c || !n0) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  for (int p = 0; p < Q; ++p)
    for (long i = 0; i < c->N; ++i) {
      double v = c->solid[i] ? 0.0 : WEIGHT(p) * n0[i];
      c->f[((long)a * Q + p) * c->N + i] = v;
      c->g[((long)a * Q + p) * c->N + i] = v;
    }
  c->unstable = 0;
  return LBEO_OK;
}

int lbeo_get_populations(lbeo_ctx *c, int a, int dist, double *out) {
  if (!c || !out) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a) || dist < 0 || dist > 1)
    return fail(LBEO_ERR_ARG, "bad species or distribution");
  const double *src = (dist == 0 ? c->f : c->g) + (long)a * Q * c->N;
  memcpy(out, src, sizeof(double) * (size_t)Q * c->N);
  return LBEO_OK;
}

int lbeo_set_populations(lbeo_ctx *c, int a, int dist, const double *in) {
  if (!c || !in) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a) || dist < 0 || dist > 1)
    return fail(LBEO_ERR_ARG, "bad species or distribution");
  double *dst = (dist == 0 ? c->f : c->g) + (long)a * Q * c->N;
  for (int p = 0; p < Q; ++p)
    for (long i = 0; i < c->N; ++i)
      dst[(long)p * c->N + i] = c->solid[i] ? 0.0 : in[(long)p * c->N + i];
  c->unstable = 0;
  return LBEO_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 1: moments of the transformed populations (Sec. 4.2):               */
/*   n~ = sum_p f~_p,  Pi~ = sum_p g~_p,  J~ = sum_p c_p g~_p.              */
/* J~ is summed over +-c pairs so a mirror-symmetric state gives exactly 0. */
/* n = n~ because the BGK term and S_f conserve mass (Sec. 4.1).            */
/* ------------------------------------------------------------------------ */
static void node_moments(const double *fp, const double *gp, double *n,
                         double *Pi, double J[3]) {
  double sn = 0.0, sp = 0.0;
  for (int p = 0; p < Q; ++p) {
    sn += fp[p];
    sp += gp[p];
  }
  double j[3] = {0, 0, 0};
  for (int p = 1; p < Q; p += 2) {
    double d = gp[p] - gp[OPPOSITE[p]];
    for (int k = 0; k < 3; ++k) j[k] += CV[p][k] * d;
  }
  *n = sn;
  *Pi = sp;
  for (int k = 0; k < 3; ++k) J[k] = j[k];
}

static void compute_moments(lbeo_ctx *c) {
  long N = c->N;
  /* single distribution: the current is carried by f */
  int single = (c->cfg.flags & LBEO_SINGLE) != 0;
  for (int a = 0; a < c->M; ++a) {
    const double *fa = c->f + (long)a * Q * N;
    const double *ga = single ? fa : c->g + (long)a * Q * N;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
      double fp[Q], gp[Q], n = 0, Pi = 0, J[3] = {0, 0, 0};
      if (!c->solid[i]) {
        for (int p = 0; p < Q; ++p) {
          fp[p] = fa[(long)p * N + i];
          gp[p] = ga[(long)p * N + i];
        }
        node_moments(fp, gp, &n, &Pi, J);
      }
      c->n[(long)a * N + i] = n;
      c->Pit[(long)a * N + i] = Pi;
      for (int k = 0; k < 3; ++k) {
        c->Jt[((long)a * 3 + k) * N + i] = J[k];
        c->ut[((long)a * 3 + k) * N + i] = n != 0.0 ? J[k] / n : 0.0;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Step 2: weighted densities nbar_b (ball of radius sigma_b/2, solid and   */
/* out-of-domain nodes count as empty, normalised by the ball size; with    */
/* BALL_FLUID normalised by the number of fluid points instead) and the     */
/* contact values G_ab(r).  The pair value used by the forces is            */
/* g_ab(r, r') = (G_ab(r) + G_ab(r'))/2 (our reading of "g_ab at contact"). */
/* Returns 1 if some fluid node has a packing fraction xi3 >= 1 or a        */
/* non-finite value.                                                        */
/* ------------------------------------------------------------------------ */
static int compute_contact(lbeo_ctx *c) {
  long N = c->N;
  int M = c->M;
  for (int b = 0; b < M; ++b) {
    const ball_t *bl = &c->ball[b];
    const double *nb = c->n + (long)b * N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
      for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
          double s = 0.0;
          int nfl = 0;
          for (int k = 0; k < bl->npts; ++k) {
            long j = neighbour(c, x, y, z, bl->off[k][0], bl->off[k][1],
                               bl->off[k][2]);
            if (is_fluid(c, j)) {
              s += nb[j];
              ++nfl;
            }
          }
          /* BALL_FLUID: the average over the fluid points of the ball */
          int norm = (c->cfg.flags & LBEO_BALL_FLUID) ? nfl : bl->npts;
          c->nbar[(long)b * N + IDX(c, x, y, z)] = norm > 0 ? s / norm : 0.0;
        }
  }
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (long i = 0; i < N; ++i) {
    double nb[MAXM];
    double xi3 = 0.0;
    for (int b = 0; b < M; ++b) {
      nb[b] = c->nbar[(long)b * N + i];
      xi3 += c->cfg.sigma[b] * c->cfg.sigma[b] * c->cfg.sigma[b] * nb[b];
    }
    xi3 *= M_PI / 6.0;
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b) {
        double G = 0.0;
        if (!c->solid[i]) {
          G = lbeo_bmcsl(M, c->cfg.sigma, nb, a, b);
          if (!(xi3 < 1.0) || !isfinite(G)) bad = 1;
          for (int k = 0; k < M; ++k)
            if (!isfinite(c->n[(long)k * N + i])) bad = 1;
        }
        c->G[((long)a * M + b) * N + i] = G;
      }
  }
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Step 3: nonlocal forces on the tilde moments (Sec. 3, eq. relatemoments) */
/*                                                                          */
/* Mean-field force (Appendix, hard spheres, attractive field G^ab = 0):    */
/*   C^mf_a(r) = -kT n_a(r) sum_b sigma_ab^2 int dk k g_ab(r, r+s k)        */
/*                                                  n_b(r + s k)            */
/* Collisional viscous force (Appendix, eq. viscousforce, m = 1):           */
/*   C^visc_a(r) = n_a(r) sum_b 2 sigma_ab^2 sqrt(kT/pi) int dk k g_ab      */
/*                 n_b(r+s k) k.(u_b(r+s k) - u_b(r))                       */
/* with the unit-sphere integral replaced by the weighted lattice shell.    */
/* Each +-e pair is summed together so that a uniform state gives 0 exactly.*/
/* ------------------------------------------------------------------------ */
static void compute_forces(lbeo_ctx *c) {
  long N = c->N;
  int M = c->M;
  int visc = (c->cfg.flags & LBEO_VISC) != 0;
  int ideal = (c->cfg.flags & LBEO_IDEAL) != 0;
  int drag = (c->cfg.flags & LBEO_DRAG) != 0;
  double kT = c->cfg.kT;
  double cvpref = 2.0 * sqrt(kT / M_PI);
  for (int a = 0; a < M; ++a) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c->nz; ++z)
      for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
          long i = IDX(c, x, y, z);
          double mf[3] = {0, 0, 0}, vs[3] = {0, 0, 0};
          if (!c->solid[i] && !ideal) {
            for (int b = 0; b < M; ++b) {
              const shell_t *s = pair_shell(c, a, b);
              if (s->npts == 0) continue;
              const double *nb = c->n + (long)b * N;
              const double *Gab = c->G + ((long)a * M + b) * N;
              double G0 = Gab[i];
              double u0[3];
              for (int k = 0; k < 3; ++k) u0[k] = c->ut[((long)b * 3 + k) * N + i];
              double smf[3] = {0, 0, 0}, svs[3] = {0, 0, 0};
              for (int j = 0; j < s->nplus; ++j) {
                const int *e = s->off[j];
                const double *eh = s->ehat[j];
                long ip = neighbour(c, x, y, z, e[0], e[1], e[2]);
                long im = neighbour(c, x, y, z, -e[0], -e[1], -e[2]);
                double np = 0, gp = 0, nm = 0, gm = 0;
                if (is_fluid(c, ip)) {
                  np = nb[ip];
                  gp = 0.5 * (G0 + Gab[ip]);
                }
                if (is_fluid(c, im)) {
                  nm = nb[im];
                  gm = 0.5 * (G0 + Gab[im]);
                }
                double dmf = gp * np - gm * nm;
                for (int k = 0; k < 3; ++k) smf[k] += eh[k] * dmf;
                if (visc) {
                  /* +e and -e give k(k.du) with the same sign of k k */
                  double tp = 0, tm = 0;
                  if (is_fluid(c, ip)) {
                    double kdu = 0;
                    for (int k = 0; k < 3; ++k)
                      kdu += eh[k] * (c->ut[((long)b * 3 + k) * N + ip] - u0[k]);
                    tp = kdu * gp * np;
                  }
                  if (is_fluid(c, im)) {
                    double kdu = 0;
                    for (int k = 0; k < 3; ++k)
                      kdu += -eh[k] * (c->ut[((long)b * 3 + k) * N + im] - u0[k]);
                    tm = kdu * gm * nm;
                  }
                  /* k(k.du) at -e is (-k)(tm) */
                  for (int k = 0; k < 3; ++k) svs[k] += eh[k] * tp - eh[k] * tm;
                }
              }
              double sab = s->sigma;
              double na = c->n[(long)a * N + i];
              for (int k = 0; k < 3; ++k) {
                mf[k] += -kT * na * sab * sab * s->weight * smf[k];
                vs[k] += na * cvpref * sab * sab * s->weight * svs[k];
              }
            }
            /* attractive molecular field, part of C^mf (Appendix) */
            for (int b = 0; b < M; ++b) {
              const att_t *t = a <= b ? &c->att[a][b] : &c->att[b][a];
              if (t->nplus == 0) continue;
              const double *nb = c->n + (long)b * N;
              double Gv[3] = {0, 0, 0};
              for (int j = 0; j < t->nplus; ++j) {
                const int *e = t->off[j];
                long ip = neighbour(c, x, y, z, e[0], e[1], e[2]);
                long im = neighbour(c, x, y, z, -e[0], -e[1], -e[2]);
                double d = (is_fluid(c, ip) ? nb[ip] : 0.0) - (is_fluid(c, im) ? nb[im] : 0.0);
                for (int k = 0; k < 3; ++k) Gv[k] += t->K[j][k] * d;
              }
              double na = c->n[(long)a * N + i];
              for (int k = 0; k < 3; ++k) mf[k] += na * Gv[k];
            }
            /* interspecies drag (Appendix, eq. dragforce2), local */
            if (drag) {
              double na = c->n[(long)a * N + i];
              for (int b = 0; b < M; ++b) {
                double sab = 0.5 * (c->cfg.sigma[a] + c->cfg.sigma[b]);
                /* 2 sigma_ab^2 sqrt(kT/pi) (4 pi/3), cvpref = 2 sqrt(kT/pi) */
                double gam = sab * sab * cvpref * (4.0 * M_PI / 3.0);
                double coef = -na * gam * c->G[((long)a * M + b) * N + i] * c->n[(long)b * N + i];
                for (int k = 0; k < 3; ++k)
                  vs[k] += coef * (c->ut[((long)a * 3 + k) * N + i] - c->ut[((long)b * 3 + k) * N + i]);
              }
            }
          }
          for (int k = 0; k < 3; ++k) {
            c->cmf[((long)a * 3 + k) * N + i] = mf[k];
            c->cvisc[((long)a * 3 + k) * N + i] = vs[k];
          }
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Steps 4-6 at one node: inversions, equilibria, sources and the           */
/* trapezoidal BGK update, for all species.                                 */
/*                                                                          */
/* Hermite tensors (Sec. 4.1): H1_p = c_p / v_T^2,                          */
/*   H2_p = (c_p c_p - v_T^2 I) / (2 v_T^4).                                */
/* Inversions (Sec. 4.2, derived from eq. invertmoments applied to the g    */
/* kernel, whose zeroth source moment is beta C^mf.u^a and first is        */
/* Y = C^visc + n F):                                                       */
/*   J = J~ + Y/2,  u^a = J/n,  Pi = Pi~ + (beta/2) C^mf.u^a                */
/* or, with PRINTED_INV, the printed  J = J~ + (C^mf + C^visc + nF)/2 and   */
/* Pi = Pi~ - (beta/2) C^mf.u^a (beta inserted for dimensional consistency).*/
/* Equilibria and sources (eqs. kernel-f-1 .. kernel-g-1):                  */
/*   f_eq = w_p [n + J.H1 + n (2 u^a u - u u):H2]                           */
/*   g_eq = w_p [Pi + J.H1 + n (2 u^a u - u u):H2]                          */
/*   S_f  = w_p X.[H1 + 2 H2.u^a],  X = C^mf + C^visc + n F                 */
/*   S_g  = w_p {C^mf.[u^a/v_T^2 + kappa H2.u^a] + Y.[H1 + 2 H2.u^a]}       */
/* with kappa = 2 (projection of eq. palfa) or the printed 4 (KAPPA4).      */
/* Trapezoidal update (Sec. 4.1):                                           */
/*   f~* = f~ + (w h/(1 + w h/2)) (f_eq - f~) + (h/(1 + w h/2)) S_f         */
/* and the same for g~.                                                     */
/* Variants of Sec. 4: EULER updates f* = f + w h (f_eq - f) + h S_f (and g)*/
/* with J = sum c g, Pi = sum g and no half-step terms; SINGLE takes the    */
/* current from f (J = J~ + h X/2 for TR), Pi = n, and evolves no g.        */
/* ------------------------------------------------------------------------ */
static void hermite_tables(double vT2, hermite_t *t) {
  for (int p = 0; p < Q; ++p)
    for (int i = 0; i < 3; ++i) {
      t->H1[p][i] = CV[p][i] / vT2;
      for (int j = 0; j < 3; ++j)
        t->H2[p][i][j] = (CV[p][i] * CV[p][j] - (i == j ? vT2 : 0.0)) /
                         (2.0 * vT2 * vT2);
    }
}

static int collide_node_tab(const hermite_t *tab, int M, double tau,
                            double kT, unsigned flags, const double *ft,
                            const double *gt, const double *cmf,
                            const double *cvisc, const double *F,
                            const double *pipath, double *fpost,
                            double *gpost, double *mom);

int lbeo_collide_node(int M, double tau, double kT, unsigned flags,
                      const double *ft, const double *gt, const double *cmf,
                      const double *cvisc, const double *F, double *fpost,
                      double *gpost, double *mom) {
  if (M < 1 || M > MAXM) return fail(LBEO_ERR_ARG, "bad M");
  hermite_t tab;
  hermite_tables(kT, &tab);
  return collide_node_tab(&tab, M, tau, kT, flags, ft, gt, cmf, cvisc, F,
                          NULL, fpost, gpost, mom);
}

static int collide_node_tab(const hermite_t *tab, int M, double tau,
                            double kT, unsigned flags, const double *ft,
                            const double *gt, const double *cmf,
                            const double *cvisc, const double *F,
                            const double *pipath, double *fpost,
                            double *gpost, double *mom) {
  const double h = 1.0;
  double vT2 = kT, beta = 1.0 / kT, omega = 1.0 / tau;
  int euler = (flags & LBEO_EULER) != 0;
  int single = (flags & LBEO_SINGLE) != 0;
  /* trapezoidal update of the tilde populations (Sec. 4.1), or Euler */
  double acoef = euler ? omega * h : omega * h / (1.0 + 0.5 * omega * h);
  double bcoef = euler ? h : h / (1.0 + 0.5 * omega * h);
  double kappa = (flags & LBEO_KAPPA4) ? 4.0 : 2.0;
  int printed = (flags & LBEO_PRINTED_INV) != 0;
  const double(*H1)[3] = tab->H1;
  const double(*H2)[3][3] = tab->H2;

  double n[MAXM], Pit[MAXM], Jt[MAXM][3], J[MAXM][3], ua[MAXM][3], Pi[MAXM];
  double X[MAXM][3], Y[MAXM][3], dPit[MAXM];
  double ntot = 0.0, Jtot[3] = {0, 0, 0};
  for (int a = 0; a < M; ++a) {
    /* the current from g (DD) or from f itself (SD) */
    node_moments(ft + a * Q, single ? ft + a * Q : gt + a * Q, &n[a], &Pit[a], Jt[a]);
    for (int k = 0; k < 3; ++k) {
      double nF = n[a] * F[a * 3 + k];
      X[a][k] = cmf[a * 3 + k] + cvisc[a * 3 + k] + nF;
      Y[a][k] = cvisc[a * 3 + k] + nF;
      /* EU: no half-step terms; SD-TR: the f inversion J~ + h X/2 */
      double half = euler ? 0.0 : 0.5 * h * ((printed || single) ? X[a][k] : Y[a][k]);
      J[a][k] = Jt[a][k] + half;
      ua[a][k] = n[a] != 0.0 ? J[a][k] / n[a] : 0.0;
    }
    double cu = 0.0;
    for (int k = 0; k < 3; ++k) cu += cmf[a * 3 + k] * ua[a][k];
    if (euler || single)
      Pi[a] = Pit[a];
    else
      Pi[a] = printed ? Pit[a] - 0.5 * h * beta * cu : Pit[a] + 0.5 * h * beta * cu;
    dPit[a] = 0.0;
    if (pipath && !single) {
      /* default reading: Pi is the path integral; the zeroth moment of g~
         becomes the Pi~ that the same inversion maps to it */
      double target = pipath[a];
      if (!euler) target += (printed ? 0.5 : -0.5) * h * beta * cu;
      Pi[a] = pipath[a];
      dPit[a] = target - Pit[a];
    }
    ntot += n[a];
    for (int k = 0; k < 3; ++k) Jtot[k] += J[a][k];
  }
  double u[3];
  for (int k = 0; k < 3; ++k) u[k] = ntot != 0.0 ? Jtot[k] / ntot : 0.0;

  for (int a = 0; a < M; ++a) {
    double T[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[i][j] = 2.0 * ua[a][i] * u[j] - u[i] * u[j];
    for (int p = 0; p < Q; ++p) {
      double w = WEIGHT(p);
      double JH1 = 0.0, TH2 = 0.0, h2ua[3];
      for (int i = 0; i < 3; ++i) {
        JH1 += J[a][i] * H1[p][i];
        h2ua[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
          TH2 += T[i][j] * H2[p][i][j];
          h2ua[i] += H2[p][i][j] * ua[a][j];
        }
      }
      double feq = w * (n[a] + JH1 + n[a] * TH2);
      double geq = w * (Pi[a] + JH1 + n[a] * TH2);
      double sf = 0.0, sg = 0.0;
      for (int i = 0; i < 3; ++i) {
        sf += X[a][i] * (H1[p][i] + 2.0 * h2ua[i]);
        sg += cmf[a * 3 + i] * (ua[a][i] / vT2 + kappa * h2ua[i]) +
              Y[a][i] * (H1[p][i] + 2.0 * h2ua[i]);
      }
      sf *= w;
      sg *= w;
      double fo = ft[a * Q + p], go = gt[a * Q + p] + w * dPit[a];
      fpost[a * Q + p] = fo + acoef * (feq - fo) + bcoef * sf;
      gpost[a * Q + p] = single ? 0.0 : go + acoef * (geq - go) + bcoef * sg;
    }
  }
  if (mom) {
    for (int a = 0; a < M; ++a) {
      mom[8 * a + 0] = n[a];
      mom[8 * a + 1] = Pi[a];
      for (int k = 0; k < 3; ++k) {
        mom[8 * a + 2 + k] = J[a][k];
        mom[8 * a + 5 + k] = ua[a][k];
      }
    }
    for (int k = 0; k < 3; ++k) mom[8 * M + k] = u[k];
  }
  return LBEO_OK;
}

/* gather the per-node inputs of lbeo_collide_node from the context */
static void node_inputs(const lbeo_ctx *c, long i, double *ft, double *gt,
                        double *cm, double *cv, double *F) {
  long N = c->N;
  for (int a = 0; a < c->M; ++a) {
    for (int p = 0; p < Q; ++p) {
      ft[a * Q + p] = c->f[((long)a * Q + p) * N + i];
      gt[a * Q + p] = c->g[((long)a * Q + p) * N + i];
    }
    for (int k = 0; k < 3; ++k) {
      cm[a * 3 + k] = c->cmf[((long)a * 3 + k) * N + i];
      cv[a * 3 + k] = c->cvisc[((long)a * 3 + k) * N + i];
      F[a * 3 + k] = ext_force(c, a, k, i);
    }
  }
}

static void collide_all(lbeo_ctx *c) {
  long N = c->N;
  int M = c->M;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ft[MAXM * Q], gt[MAXM * Q], fo[MAXM * Q], go[MAXM * Q];
    double cm[MAXM * 3], cv[MAXM * 3], F[MAXM * 3];
    if (c->solid[i]) {
      for (int a = 0; a < M; ++a)
        for (int p = 0; p < Q; ++p) {
          c->fpost[((long)a * Q + p) * N + i] = 0.0;
          c->gpost[((long)a * Q + p) * N + i] = 0.0;
        }
      continue;
    }
    node_inputs(c, i, ft, gt, cm, cv, F);
    double pp[MAXM];
    if (qp_per_step(c))
      for (int a = 0; a < M; ++a) pp[a] = c->pi[(long)a * N + i];
    collide_node_tab(&c->herm, M, c->cfg.tau, c->cfg.kT, c->cfg.flags, ft, gt,
                     cm, cv, F, qp_per_step(c) ? pp : NULL, fo, go, NULL);
    for (int a = 0; a < M; ++a)
      for (int p = 0; p < Q; ++p) {
        c->fpost[((long)a * Q + p) * N + i] = fo[a * Q + p];
        c->gpost[((long)a * Q + p) * N + i] = go[a * Q + p];
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Step 7: streaming f~(r + c_p, t + h) = f~*(r, t) (Sec. 4.1) in pull form,*/
/* with mid-point bounce-back at solid and out-of-domain nodes (Sec. 4.3):  */
/* a population that would come from a solid node is the one that left r   */
/* in the opposite direction.                                               */
/* ------------------------------------------------------------------------ */
static void stream_one(const lbeo_ctx *c, const double *post, double *out) {
  long N = c->N;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->nz; ++z)
    for (int y = 0; y < c->ny; ++y)
      for (int x = 0; x < c->nx; ++x) {
        long i = IDX(c, x, y, z);
        for (int p = 0; p < Q; ++p) {
          double v = 0.0;
          if (!c->solid[i]) {
            long src = neighbour(c, x, y, z, -CV[p][0], -CV[p][1], -CV[p][2]);
            if (is_fluid(c, src))
              v = post[(long)p * N + src];
            else
              v = post[(long)OPPOSITE[p] * N + i];
          }
          out[(long)p * N + i] = v;
        }
      }
}

int lbeo_stream(lbeo_ctx *c, const double *post, double *out) {
  if (!c || !post || !out) return fail(LBEO_ERR_ARG, "null argument");
  stream_one(c, post, out);
  return LBEO_OK;
}

static void qp_field(const lbeo_ctx *c, int a, const int origin[3],
                     unsigned mode, double *out);

/* moments + contact values + forces of the current state */
static int prepare(lbeo_ctx *c) {
  compute_moments(c);
  int bad = compute_contact(c);
  if (bad) {
    c->unstable = 1;
    return fail(LBEO_ERR_UNSTABLE,
                "packing fraction >= 1 or non-finite density");
  }
  compute_forces(c);
  return LBEO_OK;
}

int lbeo_step(lbeo_ctx *c, int nsteps) {
  if (!c) return fail(LBEO_ERR_ARG, "null argument");
  if (nsteps < 0) return fail(LBEO_ERR_ARG, "nsteps < 0");
  if (c->unstable) return fail(LBEO_ERR_UNSTABLE, "context is unstable");
  for (int s = 0; s < nsteps; ++s) {
    int st = prepare(c);
    if (st != LBEO_OK) return st;
    if (qp_per_step(c)) {
      if (c->solid[IDX(c, c->qp_origin[0], c->qp_origin[1], c->qp_origin[2])])
        return fail(LBEO_ERR_STATE, "the quasi-pressure origin is a solid node");
      for (int a = 0; a < c->M; ++a)
        qp_field(c, a, c->qp_origin, c->qp_mode, c->pi + (long)a * c->N);
    }
    collide_all(c);
    for (int a = 0; a < c->M; ++a) {
      stream_one(c, c->fpost + (long)a * Q * c->N, c->f + (long)a * Q * c->N);
      stream_one(c, c->gpost + (long)a * Q * c->N, c->g + (long)a * Q * c->N);
    }
  }
  return LBEO_OK;
}

int lbeo_get_density(lbeo_ctx *c, int a, double *out) {
  if (!c || !out) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  compute_moments(c);
  memcpy(out, c->n + (long)a * c->N, sizeof(double) * (size_t)c->N);
  return LBEO_OK;
}

/* physical velocity u^a (or barycentric u for species -1) of the current
 * state, i.e. including the half-step correction of the inversion */
int lbeo_get_velocity(lbeo_ctx *c, int a, double *out) {
  if (!c || !out) return fail(LBEO_ERR_ARG, "null argument");
  if (a != -1 && !check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  int st = prepare(c);
  if (st != LBEO_OK) return st;
  long N = c->N;
  int M = c->M;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ft[MAXM * Q], gt[MAXM * Q], fo[MAXM * Q], go[MAXM * Q];
    double cm[MAXM * 3], cv[MAXM * 3], F[MAXM * 3], mom[8 * MAXM + 3];
    if (c->solid[i]) {
      for (int k = 0; k < 3; ++k) out[(long)k * N + i] = 0.0;
      continue;
    }
    node_inputs(c, i, ft, gt, cm, cv, F);
    collide_node_tab(&c->herm, M, c->cfg.tau, c->cfg.kT, c->cfg.flags, ft, gt,
                     cm, cv, F, NULL, fo, go, mom);
    for (int k = 0; k < 3; ++k)
      out[(long)k * N + i] = a < 0 ? mom[8 * M + k] : mom[8 * a + 5 + k];
  }
  return LBEO_OK;
}

int lbeo_get_forces(lbeo_ctx *c, int a, double *cmf, double *cvisc) {
  if (!c) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  int st = prepare(c);
  if (st != LBEO_OK) return st;
  long N = c->N;
  if (cmf) memcpy(cmf, c->cmf + (long)a * 3 * N, sizeof(double) * 3 * (size_t)N);
  if (cvisc)
    memcpy(cvisc, c->cvisc + (long)a * 3 * N, sizeof(double) * 3 * (size_t)N);
  return LBEO_OK;
}

int lbeo_get_contact(lbeo_ctx *c, int a, int b, double *G) {
  if (!c || !G) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a) || !check_species(c, b))
    return fail(LBEO_ERR_ARG, "bad species");
  compute_moments(c);
  int bad = compute_contact(c);
  memcpy(G, c->G + ((long)a * c->M + b) * c->N, sizeof(double) * (size_t)c->N);
  return bad ? fail(LBEO_ERR_UNSTABLE, "packing fraction >= 1") : LBEO_OK;
}

int lbeo_get_weighted_density(lbeo_ctx *c, int a, double *nbar) {
  if (!c || !nbar) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  compute_moments(c);
  (void)compute_contact(c);
  memcpy(nbar, c->nbar + (long)a * c->N, sizeof(double) * (size_t)c->N);
  return LBEO_OK;
}

int lbeo_get_external_force(lbeo_ctx *c, int a, double *F) {
  if (!c || !F) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  for (int k = 0; k < 3; ++k)
    for (long i = 0; i < c->N; ++i) F[(long)k * c->N + i] = ext_force(c, a, k, i);
  return LBEO_OK;
}

/* ------------------------------------------------------------------------ */
/* Quasi-pressure (Sec. 2, eq. quasipressure).  Pi^a is n^a minus beta     */
/* times the line integral of C^{a,mf} + n^a F^a/m from an origin, taken by */
/* the trapezoidal rule on the lattice (the paper says so).  The paper      */
/* fixes neither origin nor path; ours (a reading): from r0 along x to      */
/* (x, y0, z0), then along y to (x, y, z0), then along z, in unit steps     */
/* that never cross a periodic face.  The integrand is zero on solid nodes. */
/*                                                                          */
/* Integrand (a reading): the discrete g source of Sec. 4.2 keeps n F as a  */
/* force in its first moment and C^mf only in its zeroth, so the Pi that    */
/* the discrete scheme carries obeys grad Pi = grad n - beta C^mf; that is  */
/* the default.  LBEO_QP_WITH_FEXT adds n F as in the printed equation.     */
/* ------------------------------------------------------------------------ */
static double qp_integrand(const lbeo_ctx *c, int a, unsigned mode, int k,
                           const int r[3]) {
  long i = IDX(c, r[0], r[1], r[2]);
  if (c->solid[i]) return 0.0;
  double v = c->cmf[((long)a * 3 + k) * c->N + i];
  if (mode & LBEO_QP_WITH_FEXT) v += c->n[(long)a * c->N + i] * ext_force(c, a, k, i);
  return v;
}

static int qp_check(lbeo_ctx *c, const int origin[3], unsigned mode) {
  if (!c || !origin) return fail(LBEO_ERR_ARG, "null argument");
  if (mode & ~(LBEO_QP_WITH_FEXT | LBEO_QP_SYMMETRIC)) return fail(LBEO_ERR_ARG, "bad mode");
  if (origin[0] < 0 || origin[0] >= c->nx || origin[1] < 0 ||
      origin[1] >= c->ny || origin[2] < 0 || origin[2] >= c->nz)
    return fail(LBEO_ERR_ARG, "origin outside the box");
  if (c->solid[IDX(c, origin[0], origin[1], origin[2])])
    return fail(LBEO_ERR_ARG, "origin is a solid node");
  return LBEO_OK;
}

/* Pi of species a at every node, from the current forces and densities.   */
/* The path from the origin r0 to r runs along the three axes in a given    */
/* order (p0, p1, p2): along p0 to r's p0 coordinate (the other two at the  */
/* origin's), then along p1, then along p2.  Each leg is the trapezoidal    */
/* sum of unit steps walked away from the origin, accumulated one step at a */
/* time, a step from r to r' adding s (v_k(r) + v_k(r'))/2 with s = +1      */
/* walking up and -1 walking down:                                          */
/*   A0(c0)         along p0 (one line),                                    */
/*   A1(c0, c1)     along p1 (one line per c0),                             */
/*   A2(c0, c1, c2) along p2 (one line per (c0, c1)),                       */
/* and Phi_order = (A0 + A1) + A2.  Mode 0 takes the order (x, y, z);       */
/* LBEO_QP_SYMMETRIC takes the mean of the six orders, summed in the order  */
/* (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x) and divided by 6.   */
/* Pi = n - beta Phi on fluid nodes, 0 on solid ones.                       */
static double qp_step_term(const lbeo_ctx *c, int a, unsigned mode, int k,
                           const int from[3], int dir) {
  int to[3] = {from[0], from[1], from[2]};
  to[k] += dir;
  double va = qp_integrand(c, a, mode, k, from);
  double vb = qp_integrand(c, a, mode, k, to);
  return dir * 0.5 * (va + vb);
}

/* Phi along one axis order, written to phi (N values) */
static void qp_order(const lbeo_ctx *c, int a, const int origin[3],
                     unsigned mode, const int ord[3], double *phi) {
  const int ext[3] = {c->nx, c->ny, c->nz};
  const int p0 = ord[0], p1 = ord[1], p2 = ord[2];
  const int L0 = ext[p0], L1 = ext[p1], L2 = ext[p2];
  double *A0 = c->qpx, *A1 = c->qpy;
  /* leg along p0, through the origin */
  A0[origin[p0]] = 0.0;
  for (int k = origin[p0] + 1; k < L0; ++k) {
    int r[3] = {origin[0], origin[1], origin[2]};
    r[p0] = k - 1;
    A0[k] = A0[k - 1] + qp_step_term(c, a, mode, p0, r, +1);
  }
  for (int k = origin[p0] - 1; k >= 0; --k) {
    int r[3] = {origin[0], origin[1], origin[2]};
    r[p0] = k + 1;
    A0[k] = A0[k + 1] + qp_step_term(c, a, mode, p0, r, -1);
  }
  /* legs along p1, one per c0 */
#pragma omp parallel for schedule(static)
  for (int c0 = 0; c0 < L0; ++c0) {
    double *a1 = A1 + (long)c0 * L1;
    a1[origin[p1]] = 0.0;
    for (int k = origin[p1] + 1; k < L1; ++k) {
      int r[3] = {origin[0], origin[1], origin[2]};
      r[p0] = c0;
      r[p1] = k - 1;
      a1[k] = a1[k - 1] + qp_step_term(c, a, mode, p1, r, +1);
    }
    for (int k = origin[p1] - 1; k >= 0; --k) {
      int r[3] = {origin[0], origin[1], origin[2]};
      r[p0] = c0;
      r[p1] = k + 1;
      a1[k] = a1[k + 1] + qp_step_term(c, a, mode, p1, r, -1);
    }
  }
  /* legs along p2, one per (c0, c1) */
#pragma omp parallel for schedule(static)
  for (int c1 = 0; c1 < L1; ++c1)
    for (int c0 = 0; c0 < L0; ++c0) {
      double base = A0[c0] + A1[(long)c0 * L1 + c1];
      int r[3];
      r[p0] = c0;
      r[p1] = c1;
      double a2 = 0.0;
      for (int k = origin[p2]; k < L2; ++k) {
        if (k > origin[p2]) {
          r[p2] = k - 1;
          a2 += qp_step_term(c, a, mode, p2, r, +1);
        }
        r[p2] = k;
        phi[IDX(c, r[0], r[1], r[2])] = base + a2;
      }
      a2 = 0.0;
      for (int k = origin[p2] - 1; k >= 0; --k) {
        r[p2] = k + 1;
        a2 += qp_step_term(c, a, mode, p2, r, -1);
        r[p2] = k;
        phi[IDX(c, r[0], r[1], r[2])] = base + a2;
      }
    }
}

static void qp_field(const lbeo_ctx *c, int a, const int origin[3],
                     unsigned mode, double *out) {
  static const int orders[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                   {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double beta = 1.0 / c->cfg.kT;
  long N = c->N;
  double *phi = c->qpphi, *sum = c->qpsum;
  int nord = (mode & LBEO_QP_SYMMETRIC) ? 6 : 1;
  for (long i = 0; i < N; ++i) sum[i] = 0.0;
  for (int o = 0; o < nord; ++o) {
    qp_order(c, a, origin, mode, orders[o], phi);
    for (long i = 0; i < N; ++i) sum[i] += phi[i];
  }
  for (long i = 0; i < N; ++i) {
    double ph = nord == 6 ? sum[i] / 6.0 : sum[i];
    out[i] = c->solid[i] ? 0.0 : c->n[(long)a * N + i] - beta * ph;
  }
}

int lbeo_quasipressure(lbeo_ctx *c, int a, const int origin[3], unsigned mode,
                       double *out) {
  int st = qp_check(c, origin, mode);
  if (st != LBEO_OK) return st;
  if (!out) return fail(LBEO_ERR_ARG, "null argument");
  if (!check_species(c, a)) return fail(LBEO_ERR_ARG, "bad species");
  st = prepare(c);
  if (st != LBEO_OK) return st;
  qp_field(c, a, origin, mode, out);
  return LBEO_OK;
}

int lbeo_set_quasipressure_route(lbeo_ctx *c, const int origin[3], unsigned mode) {
  int st = qp_check(c, origin, mode);
  if (st != LBEO_OK) return st;
  for (int k = 0; k < 3; ++k) c->qp_origin[k] = origin[k];
  c->qp_mode = mode;
  return LBEO_OK;
}

/* The zeroth moment of g~ is Pi~, related to Pi by the inversion of        */
/* Sec. 4.2 at the node's current velocity u^a: Pi~ = Pi - (beta/2)         */
/* C^mf.u^a (derived reading), Pi + (beta/2) C^mf.u^a (printed inversion),  */
/* Pi~ = Pi for the Euler scheme.  Each g~_p gains w_p (Pi~ - sum_q g~_q),  */
/* which leaves sum_p c_p g~_p unchanged.                                   */
int lbeo_init_quasipressure(lbeo_ctx *c, const int origin[3], unsigned mode) {
  int st = qp_check(c, origin, mode);
  if (st != LBEO_OK) return st;
  if (c->cfg.flags & LBEO_SINGLE)
    return fail(LBEO_ERR_ARG, "the single-distribution scheme has no g");
  st = prepare(c);
  if (st != LBEO_OK) return st;
  long N = c->N;
  int M = c->M;
  double *pi = malloc(sizeof(double) * (size_t)M * (size_t)N);
  if (!pi) return fail(LBEO_ERR_OOM, "out of memory");
  for (int a = 0; a < M; ++a) qp_field(c, a, origin, mode, pi + (long)a * N);
  double beta = 1.0 / c->cfg.kT;
  int euler = (c->cfg.flags & LBEO_EULER) != 0;
  int printed = (c->cfg.flags & LBEO_PRINTED_INV) != 0;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ft[MAXM * Q], gt[MAXM * Q], fo[MAXM * Q], go[MAXM * Q];
    double cm[MAXM * 3], cv[MAXM * 3], F[MAXM * 3], mom[8 * MAXM + 3];
    if (c->solid[i]) continue;
    node_inputs(c, i, ft, gt, cm, cv, F);
    collide_node_tab(&c->herm, M, c->cfg.tau, c->cfg.kT, c->cfg.flags, ft, gt,
                     cm, cv, F, NULL, fo, go, mom);
    for (int a = 0; a < M; ++a) {
      double cu = 0.0;
      for (int k = 0; k < 3; ++k) cu += cm[a * 3 + k] * mom[8 * a + 5 + k];
      double target = pi[(long)a * N + i];
      if (!euler) target += (printed ? 0.5 : -0.5) * beta * cu;
      double sum = 0.0;
      for (int p = 0; p < Q; ++p) sum += gt[a * Q + p];
      for (int p = 0; p < Q; ++p)
        c->g[((long)a * Q + p) * N + i] = gt[a * Q + p] + WEIGHT(p) * (target - sum);
    }
  }
  free(pi);
  return LBEO_OK;
}

/* ------------------------------------------------------------------------ */
/* Divergence of the velocity field (Sec. 4.3, the quantity D of the        */
/* channel validation): D = div u / (v_T / dx), dx = 1.  The paper does not */
/* say how the derivative is taken; our reading uses the isotropic D3Q19    */
/* gradient of the external force, div_h u = (1/v_T^2) sum_p w_p c_p .      */
/* u(r + c_p), with u = 0 on solid nodes (no-slip) and beyond non-periodic  */
/* faces (the walls).                                                       */
/* ------------------------------------------------------------------------ */
int lbeo_get_divergence(lbeo_ctx *c, double *out) {
  if (!c || !out) return fail(LBEO_ERR_ARG, "null argument");
  long N = c->N;
  double *u = malloc(sizeof(double) * 3 * (size_t)N);
  if (!u) return fail(LBEO_ERR_OOM, "out of memory");
  int st = lbeo_get_velocity(c, -1, u);
  if (st != LBEO_OK) {
    free(u);
    return st;
  }
  double vT = sqrt(c->vT2);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < c->nz; ++z)
    for (int y = 0; y < c->ny; ++y)
      for (int x = 0; x < c->nx; ++x) {
        long i = IDX(c, x, y, z);
        if (c->solid[i]) {
          out[i] = 0.0;
          continue;
        }
        double div = 0.0;
        for (int p = 1; p < Q; ++p) {
          int X = x + CV[p][0], Y = y + CV[p][1], Z = z + CV[p][2];
          if (!wrap1(&X, c->nx, c->cfg.periodic & 1u) ||
              !wrap1(&Y, c->ny, c->cfg.periodic & 2u) ||
              !wrap1(&Z, c->nz, c->cfg.periodic & 4u))
            continue; /* beyond a wall: u = 0 */
          long j = IDX(c, X, Y, Z);
          double cu = 0.0;
          for (int k = 0; k < 3; ++k) cu += CV[p][k] * u[(long)k * N + j];
          div += WEIGHT(p) * cu;
        }
        out[i] = div / c->vT2 / vT;
      }
  free(u);
  return LBEO_OK;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.  Error measures of Sec. 4.1:                                */
/*   Err(n) = max |n - n_eq| / n_0,  Err(u) = max |u| / v_T,                */
/*   Err(J) = max |J| / (n_0 v_T),                                          */
/* with n_0 the mean density over fluid nodes and n_eq the ideal-gas        */
/* Boltzmann profile normalised to the same mass (meaningful for C = 0).    */
/* Sums run sequentially in node order.                                     */
/* ------------------------------------------------------------------------ */
int lbeo_diagnostics(lbeo_ctx *c, lbeo_diag *out) {
  if (!c || !out) return fail(LBEO_ERR_ARG, "null argument");
  memset(out, 0, sizeof *out);
  long N = c->N;
  int M = c->M;
  int st = prepare(c);
  if (st != LBEO_OK) {
    out->unstable = 1;
    return LBEO_OK;
  }
  long nfluid = 0;
  double mtot = 0.0, zsum = 0.0;
  for (long i = 0; i < N; ++i) {
    if (c->solid[i]) continue;
    ++nfluid;
    zsum += exp(-c->beta * c->V[i]);
  }
  for (int a = 0; a < M; ++a) {
    double m = 0.0;
    for (long i = 0; i < N; ++i)
      if (!c->solid[i]) m += c->n[(long)a * N + i];
    out->mass[a] = m;
    mtot += m;
  }
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int a = 0; a < M; ++a)
      for (long i = 0; i < N; ++i)
        if (!c->solid[i]) s += c->Jt[((long)a * 3 + k) * N + i];
    out->gmom[k] = s;
  }
  double n0 = nfluid ? mtot / (double)nfluid : 0.0;
  double vT = sqrt(c->vT2);
  double umax = 0.0, jmax = 0.0, emax = 0.0;
  for (long i = 0; i < N; ++i) {
    if (c->solid[i]) continue;
    double ft[MAXM * Q], gt[MAXM * Q], fo[MAXM * Q], go[MAXM * Q];
    double cm[MAXM * 3], cv[MAXM * 3], F[MAXM * 3], mom[8 * MAXM + 3];
    node_inputs(c, i, ft, gt, cm, cv, F);
    collide_node_tab(&c->herm, M, c->cfg.tau, c->cfg.kT, c->cfg.flags, ft, gt,
                     cm, cv, F, NULL, fo, go, mom);
    double uu = 0.0, jj = 0.0, nt = 0.0;
    for (int k = 0; k < 3; ++k) {
      double Jk = 0.0;
      for (int a = 0; a < M; ++a) Jk += mom[8 * a + 2 + k];
      uu += mom[8 * M + k] * mom[8 * M + k];
      jj += Jk * Jk;
    }
    for (int a = 0; a < M; ++a) nt += mom[8 * a];
    double neq = mtot * exp(-c->beta * c->V[i]) / zsum;
    if (sqrt(uu) > umax) umax = sqrt(uu);
    if (sqrt(jj) > jmax) jmax = sqrt(jj);
    if (fabs(nt - neq) > emax) emax = fabs(nt - neq);
  }
  out->umax = umax;
  out->err_u = umax / vT;
  out->err_J = n0 > 0 ? jmax / (n0 * vT) : 0.0;
  out->err_n = n0 > 0 ? emax / n0 : 0.0;
  out->unstable = c->unstable;
  return LBEO_OK;
}
