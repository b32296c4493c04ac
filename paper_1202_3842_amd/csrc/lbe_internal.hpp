// lbe_internal.hpp -- parameter blocks shared by the gfx950 kernels and the
// host runtime of the Lattice Boltzmann-Enskog library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbe.h"

namespace lbe {

constexpr int Q = 19;
constexpr int MAXM = LBE_MAX_SPECIES;
constexpr int MAXPAIRS = MAXM * (MAXM + 1) / 2;

// index of the unordered species pair (a, b) among the M(M+1)/2 pairs
__host__ __device__ constexpr int pair_index(int M, int a, int b) {
  return a <= b ? a * M - a * (a - 1) / 2 + (b - a)
                : b * M - b * (b - 1) / 2 + (a - b);
}

// Lattice geometry.  Populations and node-local arrays use the compact
// index i = x + nx*(y + ny*z).  The gathered scalar fields (densities,
// contact values, currents) live on a padded box with R ghost layers per
// side, filled with periodic images or zeros, so a shell or ball offset is
// one constant added to the padded index.
struct Geom {
  int nx, ny, nz;
  int N;            // nx*ny*nz
  int R;            // ghost layers
  int PX, PY, PZ;   // padded extents
  long long Np;     // padded node count
  unsigned periodic;
};

__host__ __device__ inline long long padded_index(const Geom &g, int x, int y, int z) {
  return (long long)(x + g.R) + (long long)g.PX * ((long long)(y + g.R) + (long long)g.PY * (z + g.R));
}

// Force-kernel tiling: a workgroup owns FORCE_TX x FORCE_TY output nodes and
// marches over FORCE_ZC planes; shells reach at most RING_MAX nodes out.
constexpr int FORCE_TX = 32, FORCE_TY = 8, FORCE_ZC = 8;
constexpr int RING_MAX = 8;

// Tables of the pair shells and of the averaging balls.  Each unordered pair
// k has a half shell S+ (e_z > 0, or e_z = 0 with e_y > 0, or e_z = e_y = 0
// with e_x > 0), stored ring by ring in e_z: entries ring_ofs[k][ez] ..
// ring_ofs[k][ez+1]-1 hold the LDS offset e_y*W_k + e_x of the point in a
// window of width W_k = FORCE_TX + 2 pair_R[k] and its unit vector.
struct Tables {
  const int *ring_ofs;        // (RING_MAX + 2) per pair
  const int *ring_off;        // one per S+ point, all pairs concatenated
  const double *ring_e;       // 3 doubles per S+ point
  int pair_R[MAXPAIRS];        // largest |component| of the pair's shell
  int pair_nent[MAXPAIRS];     // points in the pair's half shell S+
  double pair_cmf[MAXPAIRS];   // -kT sigma_ab^2 w_ab / 2
  double pair_cvisc[MAXPAIRS]; //  2 sigma_ab^2 sqrt(kT/pi) w_ab / 2
  double pair_d[MAXPAIRS];     // sigma_a sigma_b / (sigma_a + sigma_b)
  double pair_drag[MAXPAIRS];  // 2 sigma_ab^2 sqrt(kT/pi) 4 pi/3 (interspecies drag)
  const int *ball_off;        // all species' balls, concatenated (padded-field offsets)
  const int *ball_loff;       // the same points as offsets in a ball-kernel LDS block
  int ball_R;                 // largest reach of any species' ball
  int ball_total;             // points of all balls
  int ball_start[MAXM];
  int ball_n[MAXM];
  double sigma[MAXM];
  // attractive tails: per pair, the half thick shell sigma_ab <= |e| < rc in
  // the same ring layout (offsets for a window of FORCE_TX + 2 att_R[k]
  // columns) inside ring_off / ring_e, whose 3 doubles per point are here
  // U'(|e|) e^ instead of a unit vector
  const int *att_ring_ofs;     // (RING_MAX + 2) per pair
  int att_R[MAXPAIRS];         // 0 = no attraction for the pair
  int att_nent[MAXPAIRS];
};

struct alignas(8) StepArgs {
  Geom g;
  int M;
  unsigned flags;
  double acoef, bcoef;   // omega h/(1+omega h/2), h/(1+omega h/2)
  double beta;           // 1/kT
  double kappa;          // coefficient on H2.u^a in the C^mf part of S_g
  const uint32_t *bb;    // bit 0: node solid; bit p: r - c_p blocked
  const double *Fext;    // 3N: -grad_h V
  double body[MAXM][3];
  double *nfield;        // M * Np
  double *Gfield;        // npairs * Np
  double *Jfield;        // 3M * Np (only with LBE_VISC, or LBE_DRAG and M > 1)
  double *force;         // 6M * N: C^mf/n_a (3), C^visc/n_a (3) per species
  void *pop[2];          // the two ping-pong population buffers
  int zchunk;            // z planes per force-kernel workgroup
  int order;             // force-kernel tile order: 0 hardware order, 1 and 2
                         // XCD-grouped with x or z fastest
  int rows;              // force-kernel tile shape: 0 32x8, 1 32x16 (two rows
                         // per thread), 2 32x16 (512 threads)
  Tables t;
  unsigned *errflag;     // bit 0: packing fraction >= 1 or NaN
  // the quasi-pressure of eq. quasipressure evaluated every step (the
  // default reading; null with LBE_PI_CARRIED or LBE_SINGLE): the path
  // integral Phi of every species (M*N); the collision forms Pi = n - beta
  // Phi with its own n and gives Pi to g_eq and, through the inversion, to
  // the zeroth moment of g~
  const double *pifield;
};

// A batch launch: every block finds its box in blockbox and its first
// block in blockstart; cur selects the ping-pong buffer holding the state.
struct BatchArgs {
  const StepArgs *boxes;
  const int *blockbox;
  const int *blockstart;
  int cur;
};

// The quasi-pressure route of one batched box (read by the batched scans at
// run time, so a changed route needs no new graph): the origin, the mode
// bits as booleans, and the box's scan scratch (3*M*N doubles).  Phi goes
// to the box's StepArgs::pifield.
struct QpRoute {
  double *scan;
  int o[3];
  int sym, fext;
};

// Per-node outputs of the read-out pass (component-major, N each):
//   ua[M][3], u[3], cmf[M][3], cvisc[M][3], n[M], Jt_sum[3], J_sum[3], J[M][3]
struct Readout {
  double *ua, *u, *cmf, *cvisc, *n, *jt, *j, *ja;
};

// Buffers of the adjoint passes (FP64).  "bar" marks dL/d(quantity).  The
// adjoint state of a step is mu: one value per population in the
// post-streaming frame (the population layout of a state buffer), i.e. the
// adjoint of f~_p(r), g~_p(r); the adjoint of the stored pre-streaming value
// at (r, q) is mu at the node that pulls it.
struct AdjArgs {
  const double *PJ;        // 4M*N tilde moments of the state: Pi~ (M), J~ (3M)
  const double *mu_in;     // adjoint state after the step
  double *mu_out;          // adjoint state before the step
  double *node;            // 5M*N node adjoints of the collision: nbar (M), Pi~bar (M), J~bar (3M)
  double *nbar;            // M*N: the nonlocal part of the density adjoint
  double *phibar;          // 3M*Np padded: adjoint of the force per particle C^mf_a/n_a
  double *Gbar;            // npairs*N: adjoint of the contact values
  double *nbb;             // M*Np padded: adjoint of the ball-averaged densities
  double *Fbar;            // 3N: accumulated adjoint of the external force -grad_h V
  const double *dn;        // seeds of the read-out adjoint: dL/dn (M*N) or null
  const double *dJ;        // dL/dJ (3M*N) or null
  const double *dpop;      // dL/d(post-streaming populations) (2M*19*N) or null
  // with C^visc (null otherwise)
  double *psibar;          // 3M*Np padded: adjoint of the viscous force per particle C^visc_a/n_a
  double *ut;              // 3M*Np padded: u~ = J~/n of the step
  double *Jnl;             // 3M*N: the nonlocal part of the J~ adjoint
  // with the per-step quasi-pressure (null otherwise)
  double *qpbar;           // M*N: adjoint of the path integral Phi
  double *qpv;             // 3M*N: adjoint of its integrand v (C^mf, + n F with LBE_QP_WITH_FEXT)
  double *qpsum;           // nx*ny + nx*nz + ny*nz + nx + ny + nz per species: column and plane sums
};

// Launchers (lbe_kernels.hip)
void launch_bbmask(const Geom &g, const uint8_t *solid, uint32_t *bb, hipStream_t s);
void launch_extforce(const Geom &g, const double *V, double *F, hipStream_t s);
void launch_zero_solid(const Geom &g, int M, int prec, void *pop, const uint32_t *bb,
                       long long stride, hipStream_t s);
void launch_moments(const StepArgs &a, int prec, const void *pop, hipStream_t s);
void launch_contact(const StepArgs &a, hipStream_t s);
// LDS block of the ball kernels: (FORCE_TX + 2R) x (FORCE_TY + 2R) x (zc + 2R)
int ball_block_zc(const Geom &g);
void launch_forces(const StepArgs &a, hipStream_t s);
void launch_collide(const StepArgs &a, int prec, const void *pin, void *pout, hipStream_t s);
void launch_readout(const StepArgs &a, int prec, const void *pin, const Readout &r, hipStream_t s);
void launch_unstream(const Geom &g, int prec, const uint32_t *bb, const void *target_post,
                     void *pop_post_stream, hipStream_t s);
void launch_pull(const Geom &g, int prec, const uint32_t *bb, const void *pop_pre,
                 void *out_post, hipStream_t s);
void launch_rest_equilibrium(const Geom &g, int prec, const uint32_t *bb, const double *n0,
                             void *out, hipStream_t s);
void launch_diag_partials(const Geom &g, int M, const uint32_t *bb, const Readout &r,
                          const double *V, double beta, double *partials, int nblocks,
                          hipStream_t s);
void launch_diag_final(const double *partials, int nblocks, double *result, hipStream_t s);
// overwrites slot 11 of each block's partials with max |n - n_eq|
void launch_diag_errn(const Geom &g, int M, const uint32_t *bb, const Readout &r,
                      const double *V, double beta, const double *result, double *partials,
                      int nblocks, hipStream_t s);
int diag_nblocks(const Geom &g);
// blocks of the node-parallel kernels and of the force kernel for one box
int node_blocks(const Geom &g);
int force_blocks(const Geom &g, int zchunk, int ty = FORCE_TY);
// batched launches (M = 1 boxes sharing precision and flags)
void launch_batch_moments(const BatchArgs &b, int nblocks, int prec, bool visc, hipStream_t s);
// ball kernels of a batch: one launch per ball z depth zc
void launch_batch_ball(const BatchArgs &b, int nblocks, int zc, size_t lds_bytes, int M, hipStream_t s);
// the attractive field of the boxes of one tail reach R (after the force groups)
void launch_batch_att(const BatchArgs &b, int nblocks, int R, int alpha, int beta, hipStream_t s);
size_t ball_lds_bytes(int ball_R, int ball_total, int zc);
int ball_blocks(const Geom &g, int zc);
// the force groups of a batch: boxes of one shell reach R and one tile
// shape (StepArgs::rows); force_tile_rows gives the shape's tile height
void launch_batch_force(const BatchArgs &b, int nblocks, int R, int shape, bool visc, int entries, int alpha,
                        int beta, int acc, hipStream_t s);
int force_tile_rows(int shape);
void launch_batch_collide(const BatchArgs &b, int nblocks, int prec, int M, hipStream_t s);
void prepare_force_kernels(int maxR, bool visc, int max_entries);
// adjoint passes (FP64 populations, no C^visc)
void launch_tape_moments(const StepArgs &a, int prec, const void *pop, double *PJ, hipStream_t s);
void launch_adj_collide(const StepArgs &a, const AdjArgs &d, hipStream_t s);
void launch_adj_readout(const StepArgs &a, const AdjArgs &d, hipStream_t s);
// mu_out from the node adjoints, nbar and the incoming state (or the seed
// dpop at the final step)
void launch_adj_stream(const StepArgs &a, const AdjArgs &d, bool terminal, hipStream_t s);
void launch_adj_nonlocal(const StepArgs &a, const AdjArgs &d, hipStream_t s);
// the transpose of the per-step quasi-pressure's path integral: from
// d.qpbar (the adjoint of Phi) to the adjoint of the integrand, added to
// phibar, the density adjoint (d.node) and, with n F in the integrand, Fbar
void launch_adj_quasipressure(const StepArgs &a, const AdjArgs &d, const int origin[3], unsigned mode,
                              hipStream_t s);
size_t adj_qp_sum_doubles(const Geom &g);
void launch_adj_extforce(const Geom &g, const double *Fbar, double *Vbar, hipStream_t s);
// building blocks of lbe_adjoint_probe: compact <-> padded fields (nf
// fields; padding zero-fills first, solid nodes get 0), the pull of
// `blocks` FP64 population blocks, and the shell-gather transposes alone
// (phibar -> nbar, Gbar for every pair, without the ball part)
void launch_pad_fields(const Geom &g, const uint32_t *bb, int nf, const double *in, double *out, hipStream_t s);
void launch_unpad_fields(const Geom &g, int nf, const double *in, double *out, hipStream_t s);
void launch_pull_f64(const Geom &g, const uint32_t *bb, int blocks, const double *pre, double *out,
                     hipStream_t s);
void launch_adj_shell(const StepArgs &a, const AdjArgs &d, hipStream_t s);
void launch_adj_state_grad(const Geom &g, int M, const uint32_t *bb, const double *mu, int species,
                           int dist, double *out, hipStream_t s);
void launch_fill(double *p, long long n, double v, hipStream_t s);
void launch_divergence(const Geom &g, const uint32_t *bb, const double *u, double kT, double *out,
                       hipStream_t s);
// quasi-pressure: Pi (or, phi_only, the path integral Phi) of every species
// into pi (M*N) from the current densities and forces (after
// launch_forces), with 3*M*N doubles of scan scratch; mode bits
// LBE_QP_WITH_FEXT, LBE_QP_SYMMETRIC.  Then, per species,
// the zeroth-moment shift of a pulled g~ stage (the initialiser)
void launch_quasipressure(const StepArgs &a, const int origin[3], unsigned mode, bool phi_only,
                          double *scan, double *pi, hipStream_t s);
void launch_qp_apply(const StepArgs &a, const Readout &r, const double *pi, int species, int prec,
                     void *gstage, hipStream_t s);
// the path integral Phi of every box of a batch, into each box's pifield:
// the x, y and z scans take the tables of their own block counts
// (qp_blocks), the combine pass the node tables (node_blocks)
struct QpBatchTables {
  const int *box[3], *start[3];
  int nblocks[3];
};
int qp_blocks(const Geom &g, int axis);
void launch_batch_quasipressure(const BatchArgs &nodes, int node_nblocks, const QpRoute *routes,
                                const QpBatchTables &t, int M, hipStream_t s);
constexpr int DIAG_K = 12;  // reduced quantities per block

}  // namespace lbe
