// lbe_adjoint.hip -- reverse mode of the Lattice Boltzmann-Enskog step with
// respect to the external potential V(r), with step checkpointing.
//
// Forward: lbe_adjoint_forward runs nsteps steps of the box and copies the
// state (one population buffer) every `segment` steps and at the end.
// Backward: the adjoint of the read-out seeds the adjoint state at the final
// step; then, segment by segment from the last, the segment's states are
// recomputed from its checkpoint while a tape keeps, per step, the fields
// the adjoint needs (n, G, the forces per particle, the tilde moments Pi~,
// J~, and J~ as a padded field with C^visc or the interspecies drag), and the
// adjoint steps run in reverse over the tape.  The adjoint of the external
// force is accumulated over all steps and turned into dL/dV by the transpose
// of -grad_h at the end.  When the whole horizon is one segment (segment
// >= nsteps), the forward itself fills the tape as it steps, and the
// backward recomputes nothing.  The read-out adjoint has a tape slot of its
// own.  With the per-step quasi-pressure (the default reading), each reverse
// step also runs the transpose of the path integral after the collision's
// adjoint.  The backward refuses to run if the context's potential, body
// forces, solid mask or quasi-pressure route changed after the forward.
#include <string.h>

#include <algorithm>
#include <vector>

#include "lbe_host.hpp"

using namespace lbe;

namespace {

struct AdjPlan {
  Plan pl;
  int T = 0, S = 0, nseg = 0;
  size_t slot_bytes = 0, mu_bytes = 0, total = 0;
  size_t off_cp = 0, off_roll = 0, off_tape = 0, off_mu = 0, off_node = 0, off_nbar = 0,
         off_phibar = 0, off_Gbar = 0, off_nbb = 0, off_Fbar = 0, off_Vbar = 0, off_stage = 0;
  size_t off_psibar = 0, off_ut = 0, off_Jnl = 0;  // with C^visc
  size_t off_qpbar = 0, off_qpv = 0, off_qpsum = 0;  // with the per-step quasi-pressure
  // inside a tape slot
  size_t so_n = 0, so_G = 0, so_force = 0, so_PJ = 0, so_J = 0;
  bool drag = false, visc = false, qp = false;
};

lbe_status make_adj_plan(const lbe_config *cfg, int nsteps, int segment, AdjPlan &ap) {
  lbe_status st = make_plan(cfg, ap.pl);
  if (st != LBE_OK) return st;
  if (nsteps < 1 || segment < 1) return fail(LBE_ERR_ARG, "nsteps and segment must be >= 1");
  const Plan &P = ap.pl;
  const size_t N = P.g.N, Np = P.g.Np, M = P.M, npairs = P.npairs;
  ap.T = nsteps;
  ap.S = std::min(segment, nsteps);
  ap.nseg = (nsteps + ap.S - 1) / ap.S;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  ap.so_n = 0;
  ap.so_G = align256(sizeof(double) * M * Np);
  ap.so_force = ap.so_G + align256(sizeof(double) * npairs * Np);
  ap.so_PJ = ap.so_force + align256(sizeof(double) * 6 * M * N);
  ap.so_J = ap.so_PJ + align256(sizeof(double) * 4 * M * N);
  // C^visc and the drag of the recomputed steps read J~ as a padded field
  ap.drag = M > 1 && (cfg->flags & LBE_DRAG) && !(cfg->flags & LBE_IDEAL);
  ap.visc = (cfg->flags & LBE_VISC) && !(cfg->flags & LBE_IDEAL);
  ap.slot_bytes = ap.so_J + (ap.drag || ap.visc ? align256(sizeof(double) * 3 * M * Np) : 0);
  // the adjoint state: the layout of a state buffer, always FP64
  ap.mu_bytes = (size_t)2 * M * Q * P.Ns * sizeof(double);
  ap.off_cp = take(P.pop_bytes * (size_t)(ap.nseg + 1));
  ap.off_roll = take(P.pop_bytes * 2);
  ap.off_tape = take(ap.slot_bytes * (size_t)(ap.S + 1));  // S steps + the read-out
  ap.off_mu = take(ap.mu_bytes * 2);
  ap.off_node = take(sizeof(double) * 5 * M * N);
  ap.off_nbar = take(sizeof(double) * M * N);
  ap.off_phibar = take(sizeof(double) * 3 * M * Np);
  ap.off_Gbar = take(sizeof(double) * npairs * N);
  ap.off_nbb = take(sizeof(double) * M * Np);
  ap.off_Fbar = take(sizeof(double) * 3 * N);
  ap.off_Vbar = take(sizeof(double) * N);
  ap.off_stage = take(sizeof(double) * (2 * M * Q + 4 * M) * N);
  if (ap.visc) {
    ap.off_psibar = take(sizeof(double) * 3 * M * Np);
    ap.off_ut = take(sizeof(double) * 3 * M * Np);
    ap.off_Jnl = take(sizeof(double) * 3 * M * N);
  }
  ap.qp = qp_per_step(cfg->flags);
  if (ap.qp) {
    ap.off_qpbar = take(sizeof(double) * M * N);
    ap.off_qpv = take(sizeof(double) * 3 * M * N);
    ap.off_qpsum = take(sizeof(double) * M * adj_qp_sum_doubles(P.g));
  }
  ap.total = o;
  return LBE_OK;
}

}  // namespace

struct lbe_adjoint {
  lbe_ctx *c = nullptr;
  AdjPlan ap;
  char *ws = nullptr;
  int cur = 0;              // mu buffer holding the adjoint state
  bool forward_done = false, backward_done = false;
  bool taped = false;       // the forward filled the tape (one segment)
  unsigned long long fwd_epoch = 0;  // the context's parameter epoch at the forward

  char *cp(int k) const { return ws + ap.off_cp + (size_t)k * ap.pl.pop_bytes; }
  char *roll(int k) const { return ws + ap.off_roll + (size_t)k * ap.pl.pop_bytes; }
  char *slot(int j) const { return ws + ap.off_tape + (size_t)j * ap.slot_bytes; }
  double *mu(int k) const { return (double *)(ws + ap.off_mu + (size_t)k * ap.mu_bytes); }
  double *at(size_t off) const { return (double *)(ws + off); }

  // the box's parameter block with the fields of tape slot j
  StepArgs slot_args(int j) const {
    StepArgs a = c->args;
    a.nfield = (double *)(slot(j) + ap.so_n);
    a.Gfield = (double *)(slot(j) + ap.so_G);
    a.force = (double *)(slot(j) + ap.so_force);
    a.Jfield = ap.drag || ap.visc ? (double *)(slot(j) + ap.so_J) : nullptr;
    return a;
  }
  double *slot_PJ(int j) const { return (double *)(slot(j) + ap.so_PJ); }

  AdjArgs base_args() const {
    AdjArgs d;
    memset(&d, 0, sizeof d);
    d.node = at(ap.off_node);
    d.nbar = at(ap.off_nbar);
    d.phibar = at(ap.off_phibar);
    d.Gbar = at(ap.off_Gbar);
    d.nbb = at(ap.off_nbb);
    d.Fbar = at(ap.off_Fbar);
    if (ap.visc) {
      d.psibar = at(ap.off_psibar);
      d.ut = at(ap.off_ut);
      d.Jnl = at(ap.off_Jnl);
    }
    if (ap.qp) {
      d.qpbar = at(ap.off_qpbar);
      d.qpv = at(ap.off_qpv);
      d.qpsum = at(ap.off_qpsum);
    }
    return d;
  }

  // fields of state `pop` into slot j: n (padded) and Pi~, J~, then G and
  // C^mf/n, and the per-step quasi-pressure's path integral (into the
  // context's buffer, which the collision of this step reads)
  void fields(int j, const void *pop) const {
    StepArgs a = slot_args(j);
    launch_tape_moments(a, c->cfg.prec, pop, slot_PJ(j), c->stream);
    launch_contact(a, c->stream);
    launch_forces(a, c->stream);
    if (ap.qp)
      launch_quasipressure(a, c->qp_origin, c->qp_mode, true, c->at<double>(c->pl.off_qps),
                           c->at<double>(c->pl.off_pi), c->stream);
  }
};

extern "C" {

size_t lbe_adjoint_workspace_bytes(const lbe_config *cfg, int nsteps, int segment) {
  AdjPlan ap;
  if (make_adj_plan(cfg, nsteps, segment, ap) != LBE_OK) return 0;
  return ap.total;
}

lbe_status lbe_adjoint_create(lbe_ctx *c, int nsteps, int segment, void *ws, size_t bytes,
                              lbe_adjoint **out) {
  if (!out) return fail(LBE_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!c) return fail(LBE_ERR_ARG, "null context");
  AdjPlan ap;
  lbe_status st = make_adj_plan(&c->cfg, nsteps, segment, ap);
  if (st != LBE_OK) return st;
  if (!ws || ((uintptr_t)ws & 255u)) return fail(LBE_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < ap.total) return fail(LBE_ERR_OOM, "workspace of %zu bytes, %zu needed", bytes, ap.total);
  lbe_adjoint *A = new (std::nothrow) lbe_adjoint();
  if (!A) return fail(LBE_ERR_OOM, "host allocation failed");
  A->c = c;
  A->ap = std::move(ap);
  A->ws = (char *)ws;
  // zero ghost layers of the padded fields stay zero from here on
  if (hipMemsetAsync(A->ws, 0, A->ap.total, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    delete A;
    return fail(LBE_ERR_HIP, "adjoint workspace initialisation failed");
  }
  *out = A;
  return LBE_OK;
}

lbe_status lbe_adjoint_forward(lbe_adjoint *A) {
  if (!A) return fail(LBE_ERR_ARG, "null adjoint");
  lbe_ctx *c = A->c;
  if (c->poisoned) return fail(LBE_ERR_UNSTABLE, "context is unstable; reinitialise the state");
  if (c->next_phase != 0) return fail(LBE_ERR_STATE, "a phased step is incomplete");
  const AdjPlan &ap = A->ap;
  A->forward_done = A->backward_done = A->taped = false;
  if (ap.qp && c->qp_origin_solid) return fail(LBE_ERR_STATE, "the quasi-pressure origin is a solid node");
  A->fwd_epoch = c->epoch;
  if (ap.nseg == 1) {
    // one segment: each step's fields go to its tape slot, and the
    // collision reads them there (the kernels of lbe_step, on the tape)
    HIP_TRY(hipMemcpyAsync(A->cp(0), c->pop(c->cur), ap.pl.pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    for (int t = 0; t < ap.T; ++t) {
      A->fields(t, c->pop(c->cur));
      launch_collide(A->slot_args(t), c->cfg.prec, c->pop(c->cur), c->pop(c->cur ^ 1), c->stream);
      LAUNCH_CHECK();
      c->cur ^= 1;
    }
    A->taped = true;
  } else {
    for (int t = 0; t < ap.T; ++t) {
      if (t % ap.S == 0)
        HIP_TRY(hipMemcpyAsync(A->cp(t / ap.S), c->pop(c->cur), ap.pl.pop_bytes, hipMemcpyDeviceToDevice,
                               c->stream));
      lbe_status st = lbe_step(c, 1);
      if (st != LBE_OK) return st;
    }
  }
  HIP_TRY(hipMemcpyAsync(A->cp(ap.nseg), c->pop(c->cur), ap.pl.pop_bytes, hipMemcpyDeviceToDevice,
                         c->stream));
  A->forward_done = true;
  return LBE_OK;
}

lbe_status lbe_adjoint_backward(lbe_adjoint *A, const double *dL_dn, const double *dL_dJ,
                                const double *dL_dpop, int where, double *dL_dV, int where_out) {
  if (!A) return fail(LBE_ERR_ARG, "null adjoint");
  if (!A->forward_done) return fail(LBE_ERR_STATE, "lbe_adjoint_forward has not run");
  if (A->c->epoch != A->fwd_epoch)
    return fail(LBE_ERR_STATE,
                "the potential, a body force, the solid mask or the quasi-pressure route changed since "
                "lbe_adjoint_forward");
  if (where != LBE_HOST && where != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where'");
  if (where_out != LBE_HOST && where_out != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where_out'");
  if (!dL_dV) return fail(LBE_ERR_ARG, "null output");
  lbe_ctx *c = A->c;
  hipStream_t s = c->stream;
  const AdjPlan &ap = A->ap;
  const Geom &g = ap.pl.g;
  const size_t N = g.N, M = ap.pl.M;
  AdjArgs d = A->base_args();
  // seeds
  double *stage = A->at(ap.off_stage);
  auto seed = [&](const double *src, size_t count, double *dst) -> const double * {
    if (!src) return nullptr;
    if (where == LBE_DEVICE) return src;
    if (hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyHostToDevice, s) != hipSuccess)
      return nullptr;
    return dst;
  };
  d.dpop = seed(dL_dpop, 2 * M * Q * N, stage);
  d.dn = seed(dL_dn, M * N, stage + 2 * M * Q * N);
  d.dJ = seed(dL_dJ, 3 * M * N, stage + (2 * M * Q + M) * N);
  if ((dL_dpop && !d.dpop) || (dL_dn && !d.dn) || (dL_dJ && !d.dJ))
    return fail(LBE_ERR_HIP, "seed upload failed");
  launch_fill(d.Fbar, 3 * (long long)N, 0.0, s);
  // adjoint of the read-out of the final state, in the tape's last slot
  const int term = ap.S;
  A->fields(term, A->cp(ap.nseg));
  {
    StepArgs a = A->slot_args(term);
    AdjArgs e = d;
    e.qpbar = e.qpv = e.qpsum = nullptr;  // the read-out has no quasi-pressure
    e.PJ = A->slot_PJ(term);
    e.mu_out = A->mu(0);
    launch_adj_readout(a, e, s);
    launch_adj_nonlocal(a, e, s);
    launch_adj_stream(a, e, true, s);
  }
  if (where == LBE_HOST) HIP_TRY(hipStreamSynchronize(s));  // host seeds may go away
  int cur = 0;
  for (int k = ap.nseg - 1; k >= 0; --k) {
    const int t0 = k * ap.S, len = std::min(ap.S, ap.T - t0);
    if (!A->taped) {  // recompute the segment's tape from its checkpoint
      HIP_TRY(hipMemcpyAsync(A->roll(0), A->cp(k), ap.pl.pop_bytes, hipMemcpyDeviceToDevice, s));
      for (int j = 0; j < len; ++j) {
        A->fields(j, A->roll(j & 1));
        if (j + 1 < len)
          launch_collide(A->slot_args(j), c->cfg.prec, A->roll(j & 1), A->roll((j + 1) & 1), s);
      }
    }
    for (int j = len - 1; j >= 0; --j) {
      AdjArgs e = d;
      e.dpop = e.dn = e.dJ = nullptr;
      e.PJ = A->slot_PJ(j);
      e.mu_in = A->mu(cur);
      e.mu_out = A->mu(cur ^ 1);
      const StepArgs a = A->slot_args(j);
      launch_adj_collide(a, e, s);
      if (ap.qp) launch_adj_quasipressure(a, e, c->qp_origin, c->qp_mode, s);
      launch_adj_nonlocal(a, e, s);
      launch_adj_stream(a, e, false, s);
      cur ^= 1;
    }
  }
  double *Vbar = A->at(ap.off_Vbar);
  launch_adj_extforce(g, d.Fbar, Vbar, s);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(dL_dV, Vbar, sizeof(double) * N,
                         where_out == LBE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  A->cur = cur;
  A->backward_done = true;
  return LBE_OK;
}

lbe_status lbe_adjoint_state_grad(lbe_adjoint *A, int species, int dist, double *out, int where) {
  if (!A) return fail(LBE_ERR_ARG, "null adjoint");
  if (!A->backward_done) return fail(LBE_ERR_STATE, "lbe_adjoint_backward has not run");
  const AdjPlan &ap = A->ap;
  if (species < 0 || species >= ap.pl.M || dist < 0 || dist > 1)
    return fail(LBE_ERR_ARG, "bad species or distribution");
  if (!out) return fail(LBE_ERR_ARG, "null output");
  if (where != LBE_HOST && where != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where'");
  hipStream_t s = A->c->stream;
  double *stage = A->at(ap.off_stage);
  launch_adj_state_grad(ap.pl.g, ap.pl.M, A->c->args.bb, A->mu(A->cur), species, dist, stage, s);
  LAUNCH_CHECK();
  HIP_TRY(hipMemcpyAsync(out, stage, sizeof(double) * Q * ap.pl.g.N,
                         where == LBE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return LBE_OK;
}

lbe_status lbe_adjoint_probe(lbe_adjoint *A, int stage, int transpose, const double *in, double *out) {
  if (!A) return fail(LBE_ERR_ARG, "null adjoint");
  if (!in || !out) return fail(LBE_ERR_ARG, "null buffer");
  if (stage < LBE_PROBE_GRAD || stage > LBE_PROBE_QP || (transpose != 0 && transpose != 1))
    return fail(LBE_ERR_ARG, "bad stage %d or transpose %d", stage, transpose);
  lbe_ctx *c = A->c;
  const AdjPlan &ap = A->ap;
  const Geom &g = ap.pl.g;
  const unsigned flags = c->cfg.flags;
  const long long N = g.N;
  const int M = ap.pl.M, np = M * (M + 1) / 2;
  if (stage == LBE_PROBE_STREAM && (flags & LBE_SINGLE))
    return fail(LBE_ERR_UNSUPPORTED, "the streaming probe needs both distributions");
  if ((stage == LBE_PROBE_SHELL_N || stage == LBE_PROBE_SHELL_G) && (flags & LBE_IDEAL))
    return fail(LBE_ERR_UNSUPPORTED, "the ideal gas has no shell gather");
  if ((stage == LBE_PROBE_SHELL_N || stage == LBE_PROBE_SHELL_G)) {
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b)
        if (c->cfg.att_eps[a][b] > 0.0) return fail(LBE_ERR_UNSUPPORTED, "the shell probe takes no attraction");
  }
  if (stage == LBE_PROBE_QP && !ap.qp)
    return fail(LBE_ERR_UNSUPPORTED, "the quasi-pressure probe needs Pi evaluated every step");
  if (c->poisoned) return fail(LBE_ERR_UNSTABLE, "the context is unstable");
  hipStream_t s = c->stream;
  // the state's fields (n, G, forces) into tape slot 0
  A->fields(0, c->args.pop[c->cur]);
  StepArgs a = A->slot_args(0);
  AdjArgs d = A->base_args();
  // scratch: the context's own derived fields, recomputed by the next step
  double *cn = c->args.nfield, *cG = c->args.Gfield, *cf = c->args.force;
  auto cmf_out = [&](const double *force) {  // C^mf/n of every species -> out (3M*N)
    for (int sp = 0; sp < M; ++sp)
      (void)hipMemcpyAsync(out + 3LL * sp * N, force + 6LL * sp * N, sizeof(double) * 3 * N,
                           hipMemcpyDeviceToDevice, s);
  };
  switch (stage) {
    case LBE_PROBE_GRAD:
      if (transpose) launch_adj_extforce(g, in, out, s);
      else launch_extforce(g, in, out, s);
      break;
    case LBE_PROBE_STREAM:
      if (!transpose) {
        launch_pull_f64(g, a.bb, 2 * M, in, out, s);
      } else {  // k_adj_stream with no collision part: (1 - a) = 1, no node adjoints
        StepArgs t = a;
        t.acoef = 0.0;
        launch_fill(d.node, 5LL * M * N, 0.0, s);
        launch_fill(d.nbar, (long long)M * N, 0.0, s);
        d.Jnl = nullptr;
        d.mu_in = in;
        d.mu_out = out;
        launch_adj_stream(t, d, false, s);
      }
      break;
    case LBE_PROBE_SHELL_N:
    case LBE_PROBE_SHELL_G: {
      StepArgs t = a;
      t.flags &= ~(unsigned)(LBE_VISC | LBE_DRAG);
      const bool byn = stage == LBE_PROBE_SHELL_N;
      if (!transpose) {
        if (byn) {
          launch_pad_fields(g, a.bb, M, in, cn, s);
          t.nfield = cn;
        } else {
          launch_pad_fields(g, a.bb, np, in, cG, s);
          t.Gfield = cG;
        }
        t.force = cf;
        launch_forces(t, s);
        cmf_out(cf);
      } else {
        launch_pad_fields(g, a.bb, 3 * M, in, d.phibar, s);
        launch_adj_shell(t, d, s);
        (void)hipMemcpyAsync(out, byn ? d.nbar : d.Gbar, sizeof(double) * (byn ? M : np) * N,
                             hipMemcpyDeviceToDevice, s);
      }
      break;
    }
    case LBE_PROBE_QP: {
      // the integrand v = n (C^mf/n) with n = 1: v is the input itself
      StepArgs t = a;
      launch_fill(d.node, (long long)M * N, 1.0, s);
      launch_pad_fields(g, a.bb, M, d.node, cn, s);
      t.nfield = cn;
      const unsigned mode = c->qp_mode & LBE_QP_SYMMETRIC;
      if (!transpose) {
        for (int sp = 0; sp < M; ++sp)
          (void)hipMemcpyAsync(cf + 6LL * sp * N, in + 3LL * sp * N, sizeof(double) * 3 * N,
                               hipMemcpyDeviceToDevice, s);
        t.force = cf;
        launch_quasipressure(t, c->qp_origin, mode, true, c->at<double>(c->pl.off_qps), out, s);
      } else {
        launch_fill(d.node, (long long)M * N, 0.0, s);
        launch_fill(d.phibar, 3LL * M * g.Np, 0.0, s);
        d.qpbar = const_cast<double *>(in);
        launch_adj_quasipressure(t, d, c->qp_origin, mode, s);
        launch_unpad_fields(g, 3 * M, d.phibar, out, s);  // n vbar with n = 1
      }
      break;
    }
    default:
      break;
  }
  LAUNCH_CHECK();
  HIP_TRY(hipStreamSynchronize(s));
  return LBE_OK;
}

void lbe_adjoint_destroy(lbe_adjoint *A) {
  if (!A) return;
  (void)hipStreamSynchronize(A->c->stream);
  delete A;
}

}  // extern "C"
