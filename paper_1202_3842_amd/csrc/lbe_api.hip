// lbe_api.hip -- host runtime behind the C ABI of include/lbe.h: context,
// workspace carving, shell and ball tables, stepping and read-out.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lbe_host.hpp"

using namespace lbe;

namespace lbe {

namespace {
thread_local char g_err[512] = "";
}

lbe_status fail(lbe_status code, const char *fmt, ...) {
  char buf[sizeof g_err];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  memcpy(g_err, buf, sizeof buf);
  return code;
}

const char *error_text() { return g_err; }

void clear_error() { g_err[0] = 0; }

}  // namespace lbe

namespace {

HostShell make_shell(double s) {
  HostShell h;
  if (s < 0.5) return h;
  int K = (int)ceil(s + 0.5);
  double lo = s - 0.5, hi = s + 0.5;
  double lo2 = lo * lo, hi2 = hi * hi;
  double sumlen = 0.0;
  for (int z = -K; z <= K; ++z)
    for (int y = -K; y <= K; ++y)
      for (int x = -K; x <= K; ++x) {
        int r2 = x * x + y * y + z * z;
        if (r2 == 0 || (double)r2 < lo2 || (double)r2 >= hi2) continue;
        sumlen += sqrt((double)r2);
        h.maxc = std::max(h.maxc, std::max(abs(x), std::max(abs(y), abs(z))));
        bool plus = z != 0 ? z > 0 : (y != 0 ? y > 0 : x > 0);
        if (!plus) continue;
        h.e.push_back(x);
        h.e.push_back(y);
        h.e.push_back(z);
      }
  h.weight = sumlen > 0 ? 4.0 * M_PI * s / sumlen : 0.0;
  return h;
}

// averaging ball |d| <= sigma/2
std::vector<int> make_ball(double sigma, int *maxc) {
  std::vector<int> b;
  double R = 0.5 * sigma;
  int K = (int)floor(R);
  *maxc = K;
  for (int z = -K; z <= K; ++z)
    for (int y = -K; y <= K; ++y)
      for (int x = -K; x <= K; ++x)
        if ((double)(x * x + y * y + z * z) <= R * R) {
          b.push_back(x);
          b.push_back(y);
          b.push_back(z);
        }
  return b;
}

// attractive tail of one pair (see HostAtt): U'(r) = 6 eps sigma^6 r^-7
HostAtt make_att(double sab, double eps, double rc) {
  HostAtt h;
  if (!(eps > 0.0) || !(sab > 0.0) || !(rc > sab)) return h;
  int K = (int)ceil(rc);
  double s6 = pow(sab, 6.0);
  for (int z = -K; z <= K; ++z)
    for (int y = -K; y <= K; ++y)
      for (int x = -K; x <= K; ++x) {
        bool plus = z != 0 ? z > 0 : (y != 0 ? y > 0 : x > 0);
        if (!plus) continue;
        double r = sqrt((double)(x * x + y * y + z * z));
        if (r < sab || r >= rc) continue;
        double dU = 6.0 * eps * s6 / pow(r, 7.0);
        h.maxc = std::max(h.maxc, std::max(abs(x), std::max(abs(y), abs(z))));
        h.e.push_back(x);
        h.e.push_back(y);
        h.e.push_back(z);
        h.K.push_back(dU * x / r);
        h.K.push_back(dU * y / r);
        h.K.push_back(dU * z / r);
      }
  return h;
}

}  // namespace

namespace lbe {

// the default reading: Pi from the path integral every step (DD only)
bool qp_per_step(unsigned flags) { return !(flags & (LBE_PI_CARRIED | LBE_SINGLE)); }

lbe_status make_plan(const lbe_config *cfg, Plan &pl) {
  if (!cfg) return fail(LBE_ERR_ARG, "null config");
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
    return fail(LBE_ERR_ARG, "box dimensions must be positive");
  if ((long long)cfg->nx * cfg->ny * cfg->nz > 0x7fffffffLL)
    return fail(LBE_ERR_UNSUPPORTED, "more than 2^31-1 nodes in one box");
  if (cfg->nspecies < 1 || cfg->nspecies > MAXM) return fail(LBE_ERR_ARG, "nspecies must be 1..4");
  if (!(cfg->tau > 0.0)) return fail(LBE_ERR_ARG, "tau must be positive");
  if (fabs(cfg->kT - 1.0 / 3.0) > 1e-12)
    return fail(LBE_ERR_ARG, "D3Q19 requires kT = v_T^2 = 1/3 (m = 1)");
  if (cfg->prec != LBE_FP64 && cfg->prec != LBE_FP32_POP) return fail(LBE_ERR_ARG, "bad precision");
  for (int a = 0; a < cfg->nspecies; ++a) {
    if (!(cfg->sigma[a] >= 0.0)) return fail(LBE_ERR_ARG, "sigma must be >= 0");
    if (cfg->sigma[a] > (double)RING_MAX)
      return fail(LBE_ERR_UNSUPPORTED, "sigma above %d lattice units is not built", RING_MAX);
  }
  for (int a = 0; a < cfg->nspecies; ++a)
    for (int b = 0; b < cfg->nspecies; ++b) {
      const double e = cfg->att_eps[a][b];
      if (!(e >= 0.0) || e != cfg->att_eps[b][a] || !std::isfinite(e))
        return fail(LBE_ERR_ARG, "att_eps must be symmetric, finite and >= 0");
      const double sab = 0.5 * (cfg->sigma[a] + cfg->sigma[b]);
      if (e > 0.0 && !(sab > 0.0 && cfg->att_rc > sab))
        return fail(LBE_ERR_ARG, "an attractive pair needs sigma_ab > 0 and att_rc > sigma_ab");
      if (e > 0.0 && (cfg->flags & LBE_IDEAL))
        return fail(LBE_ERR_ARG, "LBE_IDEAL drops the attractive field");
    }
  pl.M = cfg->nspecies;
  pl.npairs = pl.M * (pl.M + 1) / 2;
  int R = 0;
  pl.shells.clear();
  pl.atts.clear();
  pl.balls.clear();
  pl.nshell = pl.nball = pl.natt = 0;
  for (int a = 0; a < pl.M; ++a)
    for (int b = a; b < pl.M; ++b) {
      const double sab = 0.5 * (cfg->sigma[a] + cfg->sigma[b]);
      HostShell h = make_shell(sab);
      R = std::max(R, h.maxc);
      pl.nshell += (int)h.e.size() / 3;
      pl.shells.push_back(std::move(h));
      HostAtt t = make_att(sab, cfg->att_eps[a][b], cfg->att_rc);
      if (t.maxc > RING_MAX)
        return fail(LBE_ERR_UNSUPPORTED, "att_rc reaches %d nodes per axis; at most %d are built", t.maxc,
                    RING_MAX);
      R = std::max(R, t.maxc);
      pl.natt += (int)t.e.size() / 3;
      pl.atts.push_back(std::move(t));
    }
  for (int a = 0; a < pl.M; ++a) {
    int mc = 0;
    pl.balls.push_back(make_ball(cfg->sigma[a], &mc));
    R = std::max(R, mc);
    pl.nball += (int)pl.balls.back().size() / 3;
  }
  Geom &g = pl.g;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->nz;
  g.N = cfg->nx * cfg->ny * cfg->nz;
  g.R = R;
  g.PX = g.nx + 2 * R;
  g.PY = g.ny + 2 * R;
  g.PZ = g.nz + 2 * R;
  g.Np = (long long)g.PX * g.PY * g.PZ;
  g.periodic = cfg->periodic & 7u;
  if (((g.periodic & 1u) && g.nx < R) || ((g.periodic & 2u) && g.ny < R) ||
      ((g.periodic & 4u) && g.nz < R))
    return fail(LBE_ERR_ARG, "a periodic box edge is shorter than the interaction range %d", R);
  pl.Ns = ((long long)g.N + 63) / 64 * 64;
  size_t P = cfg->prec == LBE_FP64 ? 8 : 4;
  pl.pop_bytes = (size_t)2 * pl.M * Q * pl.Ns * P;
  // the current fields J~: C^visc, or the drag of a mixture
  bool visc = ((cfg->flags & LBE_VISC) || ((cfg->flags & LBE_DRAG) && pl.M > 1)) &&
              !(cfg->flags & LBE_IDEAL);
  pl.nblocks = diag_nblocks(g);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  pl.off_flag = take(64);
  pl.off_result = take(sizeof(double) * 16);
  pl.off_ring_ofs = take(sizeof(int) * (RING_MAX + 2) * MAXPAIRS);
  pl.off_ring_off = take(sizeof(int) * std::max(pl.nshell + pl.natt, 1));
  pl.off_ring_e = take(sizeof(double) * 3 * std::max(pl.nshell + pl.natt, 1));
  pl.off_att_ofs = take(sizeof(int) * (RING_MAX + 2) * MAXPAIRS);
  pl.off_ball = take(sizeof(int) * 2 * std::max(pl.nball, 1));
  pl.off_bb = take(sizeof(uint32_t) * g.N);
  pl.off_V = take(sizeof(double) * g.N);
  pl.off_F = take(sizeof(double) * 3 * g.N);
  pl.off_solid = take(g.N);
  pl.off_pop0 = take(pl.pop_bytes);
  pl.off_pop1 = take(pl.pop_bytes);
  pl.off_n = take(sizeof(double) * pl.M * g.Np);
  pl.off_G = take(sizeof(double) * pl.npairs * g.Np);
  pl.off_J = take(visc ? sizeof(double) * 3 * pl.M * g.Np : 0);
  pl.off_force = take(sizeof(double) * 6 * pl.M * (size_t)g.N);
  pl.off_read = take(sizeof(double) * (13 * pl.M + 9) * (size_t)g.N);
  pl.off_part = take(sizeof(double) * DIAG_K * pl.nblocks);
  // quasi-pressure of every species and the three axis scans (the per-step
  // reading, lbe_get_quasipressure and lbe_init_quasipressure)
  pl.off_pi = take(sizeof(double) * pl.M * (size_t)g.N);
  pl.off_qps = take(sizeof(double) * 3 * pl.M * (size_t)g.N);
  pl.total = o;
  return LBE_OK;
}

}  // namespace lbe

extern "C" {

const char *lbe_last_error(void) { return lbe::error_text(); }

size_t lbe_workspace_bytes(const lbe_config *cfg) {
  Plan pl;
  if (make_plan(cfg, pl) != LBE_OK) return 0;
  return pl.total;
}

lbe_status lbe_create(const lbe_config *cfg, void *ws, size_t bytes, void *stream, lbe_ctx **out) {
  if (!out) return fail(LBE_ERR_ARG, "null output pointer");
  *out = nullptr;
  Plan pl;
  lbe_status st = make_plan(cfg, pl);
  if (st != LBE_OK) return st;
  if (!ws) return fail(LBE_ERR_ARG, "null workspace");
  if (((uintptr_t)ws & 255u) != 0) return fail(LBE_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < pl.total)
    return fail(LBE_ERR_OOM, "workspace of %zu bytes, %zu needed", bytes, pl.total);
  lbe_ctx *c = new (std::nothrow) lbe_ctx();
  if (!c) return fail(LBE_ERR_OOM, "host allocation failed");
  c->cfg = *cfg;
  c->pl = std::move(pl);
  c->ws = (char *)ws;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  const Plan &P = c->pl;
  const Geom &g = P.g;
  // tables
  std::vector<int> rofs((RING_MAX + 2) * MAXPAIRS, 0), roff;
  std::vector<double> reh;
  StepArgs &a = c->args;
  memset(&a, 0, sizeof a);
  a.g = g;
  a.M = P.M;
  a.flags = cfg->flags;
  double omega = 1.0 / cfg->tau;
  const bool euler = cfg->flags & LBE_EULER;
  a.acoef = euler ? omega : omega / (1.0 + 0.5 * omega);
  a.bcoef = euler ? 1.0 : 1.0 / (1.0 + 0.5 * omega);
  a.beta = 1.0 / cfg->kT;
  a.kappa = (cfg->flags & LBE_KAPPA4) ? 4.0 : 2.0;
  a.zchunk = FORCE_ZC < g.nz ? FORCE_ZC : g.nz;
  a.order = 1;
  a.rows = 0;
  a.pop[0] = c->pop(0);
  a.pop[1] = c->pop(1);
  int k = 0;
  for (int pa = 0; pa < P.M; ++pa)
    for (int pb = pa; pb < P.M; ++pb, ++k) {
      const HostShell &h = P.shells[k];
      int idx = pair_index(P.M, pa, pb);
      double sab = 0.5 * (cfg->sigma[pa] + cfg->sigma[pb]);
      int R = h.maxc;
      int W = FORCE_TX + 2 * R;
      a.t.pair_R[idx] = R;
      a.t.pair_cmf[idx] = -cfg->kT * sab * sab * h.weight * 0.5;
      a.t.pair_cvisc[idx] = 2.0 * sab * sab * sqrt(cfg->kT / M_PI) * h.weight * 0.5;
      a.t.pair_drag[idx] = 2.0 * sab * sab * sqrt(cfg->kT / M_PI) * (4.0 * M_PI / 3.0);
      double ssum = cfg->sigma[pa] + cfg->sigma[pb];
      a.t.pair_d[idx] = ssum > 0.0 ? cfg->sigma[pa] * cfg->sigma[pb] / ssum : 0.0;
      int *ofs = &rofs[idx * (RING_MAX + 2)];
      size_t j = 0, np = h.e.size() / 3;
      for (int ez = 0; ez <= R + 1 && ez <= RING_MAX + 1; ++ez) {
        ofs[ez] = (int)roff.size();
        while (j < np && h.e[3 * j + 2] == ez) {
          int ex = h.e[3 * j], ey = h.e[3 * j + 1];
          roff.push_back(ey * W + ex);
          double len = sqrt((double)(ex * ex + ey * ey + ez * ez));
          reh.push_back(ex / len);
          reh.push_back(ey / len);
          reh.push_back(ez / len);
          ++j;
        }
      }
      for (int ez = R + 2; ez <= RING_MAX + 1; ++ez) ofs[ez] = (int)roff.size();
      a.t.pair_nent[idx] = (int)np;
    }
  // the attractive tails, after all shells, in the same ring layout
  std::vector<int> arofs((RING_MAX + 2) * MAXPAIRS, 0);
  k = 0;
  for (int pa = 0; pa < P.M; ++pa)
    for (int pb = pa; pb < P.M; ++pb, ++k) {
      const HostAtt &h = P.atts[k];
      int idx = pair_index(P.M, pa, pb);
      int R = h.maxc;
      int W = FORCE_TX + 2 * R;
      size_t np = h.e.size() / 3;
      a.t.att_R[idx] = np ? R : 0;
      a.t.att_nent[idx] = (int)np;
      int *ofs = &arofs[idx * (RING_MAX + 2)];
      size_t j = 0;
      for (int ez = 0; ez <= RING_MAX + 1; ++ez) {
        ofs[ez] = (int)roff.size();
        while (j < np && h.e[3 * j + 2] == ez) {
          roff.push_back(h.e[3 * j + 1] * W + h.e[3 * j]);
          reh.push_back(h.K[3 * j]);
          reh.push_back(h.K[3 * j + 1]);
          reh.push_back(h.K[3 * j + 2]);
          ++j;
        }
      }
    }
  std::vector<int> boff, bloff;
  int bR = 0;
  for (int s = 0; s < P.M; ++s)
    for (size_t j = 0; j < P.balls[s].size(); ++j) bR = std::max(bR, abs(P.balls[s][j]));
  a.t.ball_R = bR;
  // LDS block of the ball kernels (see ball_block in lbe_kernels.hip)
  const int BW = FORCE_TX + 2 * bR, BH = FORCE_TY + 2 * bR;
  for (int s = 0; s < P.M; ++s) {
    a.t.ball_start[s] = (int)boff.size();
    const std::vector<int> &b = P.balls[s];
    a.t.ball_n[s] = (int)b.size() / 3;
    for (size_t j = 0; j < b.size(); j += 3) {
      boff.push_back(b[j] + g.PX * (b[j + 1] + g.PY * b[j + 2]));
      bloff.push_back(b[j] + BW * (b[j + 1] + BH * b[j + 2]));
    }
    a.t.sigma[s] = cfg->sigma[s];
  }
  a.t.ball_total = (int)boff.size();
  boff.insert(boff.end(), bloff.begin(), bloff.end());
  a.t.ring_ofs = c->at<int>(P.off_ring_ofs);
  a.t.ring_off = c->at<int>(P.off_ring_off);
  a.t.ring_e = c->at<double>(P.off_ring_e);
  a.t.att_ring_ofs = c->at<int>(P.off_att_ofs);
  a.force = c->at<double>(P.off_force);
  a.t.ball_off = c->at<int>(P.off_ball);
  a.t.ball_loff = a.t.ball_off + a.t.ball_total;
  a.bb = c->at<uint32_t>(P.off_bb);
  a.Fext = c->at<double>(P.off_F);
  a.nfield = c->at<double>(P.off_n);
  a.Gfield = c->at<double>(P.off_G);
  const bool currents = ((cfg->flags & LBE_VISC) || ((cfg->flags & LBE_DRAG) && P.M > 1)) &&
                        !(cfg->flags & LBE_IDEAL);
  a.Jfield = currents ? c->at<double>(P.off_J) : nullptr;
  a.errflag = c->at<unsigned>(P.off_flag);
  a.pifield = qp_per_step(cfg->flags) ? c->at<double>(P.off_pi) : nullptr;
  c->qp_origin[0] = g.nx / 2;
  c->qp_origin[1] = g.ny / 2;
  c->qp_origin[2] = g.nz / 2;
  c->qp_mode = LBE_QP_SYMMETRIC;
  c->qp_origin_solid = false;
  double *rb = c->at<double>(P.off_read);
  size_t N = g.N;
  int M = P.M;
  c->rd.ua = rb;
  c->rd.u = rb + 3 * M * N;
  c->rd.cmf = c->rd.u + 3 * N;
  c->rd.cvisc = c->rd.cmf + 3 * M * N;
  c->rd.n = c->rd.cvisc + 3 * M * N;
  c->rd.jt = c->rd.n + M * N;
  c->rd.j = c->rd.jt + 3 * N;
  c->rd.ja = c->rd.j + 3 * N;
  hipStream_t s = c->stream;
  lbe_status rs = LBE_OK;
  auto upload = [&](size_t off, const void *src, size_t n) -> bool {
    if (n == 0) return true;
    return hipMemcpyAsync(c->ws + off, src, n, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  if (hipMemsetAsync(c->ws, 0, P.total, s) != hipSuccess ||
      !upload(P.off_ring_ofs, rofs.data(), rofs.size() * sizeof(int)) ||
      !upload(P.off_ring_off, roff.data(), roff.size() * sizeof(int)) ||
      !upload(P.off_ring_e, reh.data(), reh.size() * sizeof(double)) ||
      !upload(P.off_att_ofs, arofs.data(), arofs.size() * sizeof(int)) ||
      !upload(P.off_ball, boff.data(), boff.size() * sizeof(int)))
    rs = fail(LBE_ERR_HIP, "workspace initialisation failed");
  if (rs == LBE_OK) {
    // no solids: bounce-back only at non-periodic box faces
    launch_bbmask(g, c->at<uint8_t>(P.off_solid), c->at<uint32_t>(P.off_bb), s);
    launch_extforce(g, c->at<double>(P.off_V), c->at<double>(P.off_F), s);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      rs = fail(LBE_ERR_HIP, "set-up kernels failed");
  }
  if (rs != LBE_OK) {
    delete c;
    return rs;
  }
  *out = c;
  clear_error();
  return LBE_OK;
}

void lbe_destroy(lbe_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

static lbe_status copy_in(lbe_ctx *c, void *dst, const void *src, size_t n, int where) {
  if (!src) return fail(LBE_ERR_ARG, "null input");
  if (where != LBE_HOST && where != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where'");
  HIP_TRY(hipMemcpyAsync(dst, src, n, where == LBE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                         c->stream));
  if (where == LBE_HOST) HIP_TRY(hipStreamSynchronize(c->stream));  // host buffer may go away
  return LBE_OK;
}

static lbe_status copy_out(lbe_ctx *c, void *dst, const void *src, size_t n, int where) {
  if (!dst) return fail(LBE_ERR_ARG, "null output");
  if (where != LBE_HOST && where != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where'");
  HIP_TRY(hipMemcpyAsync(dst, src, n, where == LBE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBE_OK;
}

// whether node origin is solid (reads one mask word; synchronises)
static lbe_status qp_check_origin(lbe_ctx *c, const int origin[3], bool *solid) {
  const Geom &g = c->pl.g;
  const long long io = origin[0] + (long long)g.nx * (origin[1] + (long long)g.ny * origin[2]);
  uint32_t m = 0;
  HIP_TRY(hipMemcpyAsync(&m, c->args.bb + io, sizeof m, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *solid = (m & 1u) != 0;
  return LBE_OK;
}

lbe_status lbe_set_solid(lbe_ctx *c, const uint8_t *mask, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  ++c->epoch;
  lbe_status st = copy_in(c, c->ws + c->pl.off_solid, mask, c->pl.g.N, where);
  if (st != LBE_OK) return st;
  launch_bbmask(c->pl.g, c->at<uint8_t>(c->pl.off_solid), c->at<uint32_t>(c->pl.off_bb), c->stream);
  launch_zero_solid(c->pl.g, c->pl.M, c->cfg.prec, c->pop(c->cur), c->args.bb, c->pl.Ns, c->stream);
  LAUNCH_CHECK();
  return qp_check_origin(c, c->qp_origin, &c->qp_origin_solid);
}

lbe_status lbe_set_potential(lbe_ctx *c, const double *V, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  ++c->epoch;
  lbe_status st = copy_in(c, c->ws + c->pl.off_V, V, sizeof(double) * c->pl.g.N, where);
  if (st != LBE_OK) return st;
  launch_extforce(c->pl.g, c->at<double>(c->pl.off_V), c->at<double>(c->pl.off_F), c->stream);
  LAUNCH_CHECK();
  return LBE_OK;
}

lbe_status lbe_set_body_force(lbe_ctx *c, int species, const double gb[3]) {
  if (!c || !gb) return fail(LBE_ERR_ARG, "null argument");
  if (species < 0 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  ++c->epoch;
  for (int k = 0; k < 3; ++k) c->args.body[species][k] = gb[k];
  return LBE_OK;
}

static lbe_status clear_instability(lbe_ctx *c) {
  HIP_TRY(hipMemsetAsync(c->args.errflag, 0, sizeof(unsigned), c->stream));
  c->poisoned = false;
  return LBE_OK;
}

lbe_status lbe_init_density(lbe_ctx *c, int species, const double *n0, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  double *stage = c->at<double>(c->pl.off_read);
  lbe_status st = copy_in(c, stage, n0, sizeof(double) * c->pl.g.N, where);
  if (st != LBE_OK) return st;
  for (int d = 0; d < 2; ++d)
    launch_rest_equilibrium(c->pl.g, c->cfg.prec, c->args.bb, stage, c->block(c->cur, d, species),
                            c->stream);
  LAUNCH_CHECK();
  return clear_instability(c);
}

// the per-step quasi-pressure (default reading), after the forces
static void launch_step_quasipressure(lbe_ctx *c) {
  if (!c->args.pifield) return;
  launch_quasipressure(c->args, c->qp_origin, c->qp_mode, true, c->at<double>(c->pl.off_qps),
                       c->at<double>(c->pl.off_pi), c->stream);
}

lbe_status lbe_step_phase(lbe_ctx *c, int phase) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (phase < 0 || phase > 4) return fail(LBE_ERR_ARG, "phase must be 0..4");
  if (c->poisoned) return fail(LBE_ERR_UNSTABLE, "context is unstable; reinitialise the state");
  if (phase != c->next_phase) return fail(LBE_ERR_STATE, "phase %d expected", c->next_phase);
  hipStream_t s = c->stream;
  if (phase == 0) launch_moments(c->args, c->cfg.prec, c->pop(c->cur), s);
  if (phase == 1) launch_contact(c->args, s);
  if (phase == 2) launch_forces(c->args, s);
  if (phase == 3) {
    if (c->args.pifield && c->qp_origin_solid)
      return fail(LBE_ERR_STATE, "the quasi-pressure origin is a solid node");
    launch_step_quasipressure(c);
  }
  if (phase == 4) {
    launch_collide(c->args, c->cfg.prec, c->pop(c->cur), c->pop(c->cur ^ 1), s);
    c->cur ^= 1;
  }
  LAUNCH_CHECK();
  c->next_phase = (phase + 1) % 5;
  return LBE_OK;
}

static lbe_status enqueue_step(lbe_ctx *c) {
  hipStream_t s = c->stream;
  launch_moments(c->args, c->cfg.prec, c->pop(c->cur), s);
  launch_contact(c->args, s);
  launch_forces(c->args, s);
  launch_step_quasipressure(c);
  launch_collide(c->args, c->cfg.prec, c->pop(c->cur), c->pop(c->cur ^ 1), s);
  LAUNCH_CHECK();
  c->cur ^= 1;
  return LBE_OK;
}

lbe_status lbe_step(lbe_ctx *c, int nsteps) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (nsteps < 0) return fail(LBE_ERR_ARG, "nsteps < 0");
  if (c->poisoned) return fail(LBE_ERR_UNSTABLE, "context is unstable; reinitialise the state");
  if (c->next_phase != 0) return fail(LBE_ERR_STATE, "a phased step is incomplete");
  if (c->args.pifield && c->qp_origin_solid && nsteps > 0)
    return fail(LBE_ERR_STATE, "the quasi-pressure origin is a solid node");
  for (int k = 0; k < nsteps; ++k) {
    lbe_status st = enqueue_step(c);
    if (st != LBE_OK) return st;
  }
  return LBE_OK;
}

// moments, contact values and the read-out pass of the current state;
// returns whether the instability flag is set
static lbe_status readout(lbe_ctx *c, bool *unstable) {
  hipStream_t s = c->stream;
  launch_moments(c->args, c->cfg.prec, c->pop(c->cur), s);
  launch_contact(c->args, s);
  launch_forces(c->args, s);
  launch_readout(c->args, c->cfg.prec, c->pop(c->cur), c->rd, s);
  LAUNCH_CHECK();
  unsigned flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, c->args.errflag, sizeof flag, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *unstable = flag != 0;
  if (*unstable) c->poisoned = true;
  return LBE_OK;
}

lbe_status lbe_get_density(lbe_ctx *c, int species, double *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  size_t N = c->pl.g.N;
  return copy_out(c, out, c->rd.n + species * N, sizeof(double) * N, where);
}

lbe_status lbe_get_velocity(lbe_ctx *c, int species, double *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < -1 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  size_t N = c->pl.g.N;
  const double *src = species < 0 ? c->rd.u : c->rd.ua + 3 * species * N;
  st = copy_out(c, out, src, sizeof(double) * 3 * N, where);
  if (st != LBE_OK) return st;
  return bad ? fail(LBE_ERR_UNSTABLE, "packing fraction >= 1 or non-finite density") : LBE_OK;
}

lbe_status lbe_get_momentum(lbe_ctx *c, int species, double *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < -1 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  size_t N = c->pl.g.N;
  const double *src = species < 0 ? c->rd.j : c->rd.ja + 3 * species * N;
  st = copy_out(c, out, src, sizeof(double) * 3 * N, where);
  if (st != LBE_OK) return st;
  return bad ? fail(LBE_ERR_UNSTABLE, "packing fraction >= 1 or non-finite density") : LBE_OK;
}

lbe_status lbe_get_force(lbe_ctx *c, int species, int which, double *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M || which < 0 || which > 1)
    return fail(LBE_ERR_ARG, "bad species or force index");
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  size_t N = c->pl.g.N;
  const double *src = (which == 0 ? c->rd.cmf : c->rd.cvisc) + 3 * species * N;
  st = copy_out(c, out, src, sizeof(double) * 3 * N, where);
  if (st != LBE_OK) return st;
  return bad ? fail(LBE_ERR_UNSTABLE, "packing fraction >= 1 or non-finite density") : LBE_OK;
}

lbe_status lbe_get_populations(lbe_ctx *c, int species, int dist, void *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M || dist < 0 || dist > 1)
    return fail(LBE_ERR_ARG, "bad species or distribution");
  char *stage = c->block(c->cur ^ 1, dist, species);
  launch_pull(c->pl.g, c->cfg.prec, c->args.bb, c->block(c->cur, dist, species), stage, c->stream);
  LAUNCH_CHECK();
  size_t N = c->pl.g.N, P = c->psize();
  if (!out) return fail(LBE_ERR_ARG, "null output");
  // rows are Ns apart in the stage; copy row by row to the packed 19N layout
  for (int p = 0; p < Q; ++p) {
    const char *src = stage + (size_t)p * c->pl.Ns * P;
    char *dst = (char *)out + (size_t)p * N * P;
    HIP_TRY(hipMemcpyAsync(dst, src, N * P,
                           where == LBE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBE_OK;
}

lbe_status lbe_set_populations(lbe_ctx *c, int species, int dist, const void *in, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M || dist < 0 || dist > 1)
    return fail(LBE_ERR_ARG, "bad species or distribution");
  if (!in) return fail(LBE_ERR_ARG, "null input");
  if (where != LBE_HOST && where != LBE_DEVICE) return fail(LBE_ERR_ARG, "bad 'where'");
  char *stage = c->block(c->cur ^ 1, dist, species);
  size_t N = c->pl.g.N, P = c->psize();
  for (int p = 0; p < Q; ++p)
    HIP_TRY(hipMemcpyAsync(stage + (size_t)p * c->pl.Ns * P, (const char *)in + (size_t)p * N * P, N * P,
                           where == LBE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c->stream));
  if (where == LBE_HOST) HIP_TRY(hipStreamSynchronize(c->stream));
  launch_unstream(c->pl.g, c->cfg.prec, c->args.bb, stage, c->block(c->cur, dist, species), c->stream);
  LAUNCH_CHECK();
  return clear_instability(c);
}

lbe_status lbe_get_divergence(lbe_ctx *c, double *out, int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (!out) return fail(LBE_ERR_ARG, "null output");
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  double *d = reinterpret_cast<double *>(c->pop(c->cur ^ 1));
  launch_divergence(c->pl.g, c->args.bb, c->rd.u, c->cfg.kT, d, c->stream);
  LAUNCH_CHECK();
  st = copy_out(c, out, d, sizeof(double) * c->pl.g.N, where);
  if (st != LBE_OK) return st;
  return bad ? fail(LBE_ERR_UNSTABLE, "packing fraction >= 1 or non-finite density") : LBE_OK;
}

// Origin and mode checks shared by the quasi-pressure calls.
static lbe_status qp_args(lbe_ctx *c, const int origin[3], unsigned mode) {
  if (!origin) return fail(LBE_ERR_ARG, "null origin");
  if (mode & ~(unsigned)(LBE_QP_WITH_FEXT | LBE_QP_SYMMETRIC))
    return fail(LBE_ERR_ARG, "unknown mode bits 0x%x", mode);
  const Geom &g = c->pl.g;
  if (origin[0] < 0 || origin[0] >= g.nx || origin[1] < 0 || origin[1] >= g.ny || origin[2] < 0 ||
      origin[2] >= g.nz)
    return fail(LBE_ERR_ARG, "origin (%d, %d, %d) outside the %dx%dx%d box", origin[0], origin[1],
                origin[2], g.nx, g.ny, g.nz);
  bool solid = false;
  lbe_status st = qp_check_origin(c, origin, &solid);
  if (st != LBE_OK) return st;
  if (solid) return fail(LBE_ERR_ARG, "origin is a solid node");
  return LBE_OK;
}

// Argument checks and the read-out pass (densities, contact values and
// forces of the current state) of the quasi-pressure calls; synchronises.
lbe_status lbe_qp_readout_for(lbe_ctx *c, const int origin[3], unsigned mode) {
  if (c->next_phase != 0) return fail(LBE_ERR_STATE, "a phased step is incomplete");
  lbe_status st = qp_args(c, origin, mode);
  if (st != LBE_OK) return st;
  bool bad = false;
  st = readout(c, &bad);
  if (st != LBE_OK) return st;
  if (bad) return fail(LBE_ERR_UNSTABLE, "packing fraction >= 1 or non-finite density");
  return LBE_OK;
}

// Quasi-pressure of every species at the current state into the context's
// Pi buffer (M*N doubles), after the read-out pass.
static lbe_status qp_prepare(lbe_ctx *c, const int origin[3], unsigned mode, double **phi) {
  lbe_status st = lbe_qp_readout_for(c, origin, mode);
  if (st != LBE_OK) return st;
  *phi = c->at<double>(c->pl.off_pi);
  launch_quasipressure(c->args, origin, mode, false, c->at<double>(c->pl.off_qps), *phi, c->stream);
  LAUNCH_CHECK();
  return LBE_OK;
}

lbe_status lbe_set_quasipressure_route(lbe_ctx *c, const int origin[3], unsigned mode) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (c->next_phase != 0) return fail(LBE_ERR_STATE, "a phased step is incomplete");
  lbe_status st = qp_args(c, origin, mode);
  if (st != LBE_OK) return st;
  for (int k = 0; k < 3; ++k) c->qp_origin[k] = origin[k];
  c->qp_mode = mode;
  c->qp_origin_solid = false;
  ++c->epoch;
  return LBE_OK;
}

lbe_status lbe_get_quasipressure(lbe_ctx *c, int species, const int origin[3], unsigned mode, double *out,
                                 int where) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  if (!out) return fail(LBE_ERR_ARG, "null output");
  double *phi = nullptr;
  lbe_status st = qp_prepare(c, origin, mode, &phi);
  if (st != LBE_OK) return st;
  size_t N = c->pl.g.N;
  return copy_out(c, out, phi + species * N, sizeof(double) * N, where);
}

lbe_status lbe_init_quasipressure(lbe_ctx *c, const int origin[3], unsigned mode) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (c->cfg.flags & LBE_SINGLE) return fail(LBE_ERR_ARG, "the single-distribution scheme has no g");
  if (c->next_phase != 0) return fail(LBE_ERR_STATE, "a phased step is incomplete");
  double *phi = nullptr;
  lbe_status st = qp_prepare(c, origin, mode, &phi);
  if (st != LBE_OK) return st;
  for (int s = 0; s < c->pl.M; ++s) {
    char *stage = c->block(c->cur ^ 1, 1, s);
    launch_pull(c->pl.g, c->cfg.prec, c->args.bb, c->block(c->cur, 1, s), stage, c->stream);
    launch_qp_apply(c->args, c->rd, phi, s, c->cfg.prec, stage, c->stream);
    launch_unstream(c->pl.g, c->cfg.prec, c->args.bb, stage, c->block(c->cur, 1, s), c->stream);
  }
  LAUNCH_CHECK();
  return LBE_OK;
}

lbe_status lbe_diagnostics(lbe_ctx *c, lbe_diag *out) {
  if (!c || !out) return fail(LBE_ERR_ARG, "null argument");
  memset(out, 0, sizeof *out);
  bool bad = false;
  lbe_status st = readout(c, &bad);
  if (st != LBE_OK) return st;
  const Plan &P = c->pl;
  hipStream_t s = c->stream;
  double *part = c->at<double>(P.off_part);
  double *res = c->at<double>(P.off_result);
  const double *V = c->at<double>(P.off_V);
  launch_diag_partials(P.g, P.M, c->args.bb, c->rd, V, c->args.beta, part, P.nblocks, s);
  launch_diag_final(part, P.nblocks, res, s);
  launch_diag_errn(P.g, P.M, c->args.bb, c->rd, V, c->args.beta, res, part, P.nblocks, s);
  launch_diag_final(part, P.nblocks, res, s);
  LAUNCH_CHECK();
  double h[DIAG_K];
  HIP_TRY(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double mtot = 0.0;
  for (int a = 0; a < P.M; ++a) {
    out->mass[a] = h[a];
    mtot += h[a];
  }
  for (int k = 0; k < 3; ++k) out->gmom[k] = h[4 + k];
  double nfl = h[10];
  double n0 = nfl > 0 ? mtot / nfl : 0.0;
  double vT = sqrt(c->cfg.kT);
  out->umax = h[8];
  out->err_u = h[8] / vT;
  out->err_J = n0 > 0 ? h[9] / (n0 * vT) : 0.0;
  out->err_n = n0 > 0 ? h[11] / n0 : 0.0;
  out->unstable = bad ? 1 : 0;
  return LBE_OK;
}

lbe_status lbe_set_force_zchunk(lbe_ctx *c, int zchunk) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  return lbe_set_force_tiling(c, zchunk, c->args.order, c->args.rows);
}

lbe_status lbe_set_force_tiling(lbe_ctx *c, int zchunk, int order, int shape) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (zchunk < 1 || zchunk > c->pl.g.nz) return fail(LBE_ERR_ARG, "zchunk must lie in [1, nz]");
  if (order < 0 || order > 2) return fail(LBE_ERR_ARG, "order must be 0, 1 or 2");
  if (shape < 0 || shape > 2) return fail(LBE_ERR_ARG, "shape must be 0, 1 or 2");
  c->args.zchunk = zchunk;
  c->args.order = order;
  c->args.rows = shape;
  return LBE_OK;
}

lbe_status lbe_synchronize(lbe_ctx *c) {
  if (!c) return fail(LBE_ERR_ARG, "null context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched boxes.  Workspace: the device array of per-box parameter blocks,
// the block -> box tables of the node-parallel kernels, of the ball kernel
// and of each force group (boxes sharing a shell range), then every member
// box's workspace.
// ---------------------------------------------------------------------------
namespace {

// z depth of the batched ball kernel's workgroups (every box): with depth 4
// three 43 KB workgroups fit a CU, against two of 60 KB at depth 8 (96-box
// set: 18.38 -> 18.22 ms per step; the same sums at any depth)
constexpr int BATCH_BALL_ZC = 4;

struct BatchPlan {
  std::vector<size_t> box_bytes, box_off;
  size_t off_args = 0, off_nodebox = 0, off_nodestart = 0, off_force = 0, off_ballbox = 0,
         off_ballstart = 0, total = 0;
  int node_blocks = 0, ball_blocks = 0;
  // the per-step quasi-pressure (default reading): the boxes' routes and
  // the block tables of the x, y and z scans
  bool qp = false;
  size_t off_qproutes = 0, off_qpbox[3] = {}, off_qpstart[3] = {};
  int qp_blocks[3] = {};
  size_t ball_lds = 0;     // LDS bytes of the batched ball kernel
  size_t force_bytes = 0;  // reserved for the force-group tables
};

// force-group tables (per directed pair: every box in one group of its
// reach and tile shape) are sized for the smallest zchunk (1) and the
// lowest tile (8 rows), so that any later tiling fits: the block entries
// once, plus per possible group (RING_MAX reaches x 3 shapes) its rounding
// and its start table
size_t force_table_bytes(const std::vector<Plan> &plans) {
  size_t blocks = 0;
  for (const Plan &p : plans) blocks += force_blocks(p.g, 1);
  const size_t groups = 3 * RING_MAX;
  return align256(sizeof(int) * blocks) + groups * (256 + align256(sizeof(int) * plans.size()));
}

lbe_status make_batch_plan(const lbe_config *cfgs, int nboxes, BatchPlan &bp) {
  if (!cfgs || nboxes < 1) return fail(LBE_ERR_ARG, "need at least one box");
  std::vector<Plan> plans(nboxes);
  for (int b = 0; b < nboxes; ++b) {
    lbe_status st = make_plan(&cfgs[b], plans[b]);
    if (st != LBE_OK) return fail(st, "box %d: %s", b, error_text());
    if (cfgs[b].nspecies != cfgs[0].nspecies)
      return fail(LBE_ERR_ARG, "batched boxes must have the same number of species");
    // with several species the pair gathers of one species add up, the first
    // writing: every pair's shell must be there to write in every box
    for (const HostShell &h : plans[b].shells)
      if (cfgs[b].nspecies > 1 && h.e.empty() && !(cfgs[b].flags & LBE_IDEAL))
        return fail(LBE_ERR_UNSUPPORTED, "box %d: a batched mixture needs every pair's shell (sigma_ab >= 1/2)",
                    b);
    // the attraction adds to the hard-sphere force, which must have written it
    if (cfgs[b].att_eps[0][0] > 0.0 && plans[b].shells[0].e.empty())
      return fail(LBE_ERR_UNSUPPORTED, "box %d: the attractive field in a batch needs a hard-sphere shell", b);
    if (cfgs[b].prec != cfgs[0].prec || cfgs[b].flags != cfgs[0].flags)
      return fail(LBE_ERR_ARG, "batched boxes must share precision and flags");
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  bp.node_blocks = 0;
  bp.ball_blocks = 0;
  bp.ball_lds = 0;
  for (const Plan &p : plans) {
    bp.node_blocks += node_blocks(p.g);
    bp.ball_blocks += ball_blocks(p.g, BATCH_BALL_ZC);
    int bR = 0;
    for (const auto &ball : p.balls)
      for (int v : ball) bR = std::max(bR, abs(v));
    bp.ball_lds = std::max(bp.ball_lds, ball_lds_bytes(bR, p.nball, BATCH_BALL_ZC));
  }
  bp.off_args = take(sizeof(StepArgs) * nboxes);
  bp.off_nodebox = take(sizeof(int) * bp.node_blocks);
  bp.off_nodestart = take(sizeof(int) * nboxes);
  bp.off_ballbox = take(sizeof(int) * bp.ball_blocks);
  bp.off_ballstart = take(sizeof(int) * nboxes);
  bp.qp = qp_per_step(cfgs[0].flags);
  if (bp.qp) {
    bp.off_qproutes = take(sizeof(QpRoute) * nboxes);
    for (int k = 0; k < 3; ++k) {
      bp.qp_blocks[k] = 0;
      for (const Plan &p : plans) bp.qp_blocks[k] += qp_blocks(p.g, k);
      bp.off_qpbox[k] = take(sizeof(int) * bp.qp_blocks[k]);
      bp.off_qpstart[k] = take(sizeof(int) * nboxes);
    }
  }
  // block tables of the force groups, then of the attraction groups, per
  // directed species pair
  const size_t M = (size_t)cfgs[0].nspecies;
  bp.force_bytes = 2 * M * M * force_table_bytes(plans);
  bp.off_force = take(bp.force_bytes);
  for (const Plan &p : plans) {
    bp.box_bytes.push_back(p.total);
    bp.box_off.push_back(take(p.total));
  }
  bp.total = o;
  return LBE_OK;
}

}  // namespace

struct lbe_batch {
  std::vector<lbe_ctx *> boxes;
  BatchPlan bp;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  int prec = 0;
  bool visc = false;
  int M = 1;
  bool currents = false;             // the moments keep J~ (C^visc or the drag)
  bool ideal = false;                // no nonlocal forces: no force groups
  struct Group {
    int R, shape, nblocks, entries, alpha, beta;
    int *blockbox, *blockstart;
  };
  std::vector<Group> groups, att_groups;
  std::vector<int> zchunks, shapes;  // each box's zchunk and tile shape the tables were built for
  std::vector<StepArgs> uploaded;    // the parameter blocks last copied to the device
  std::vector<QpRoute> routes;       // the quasi-pressure routes last copied to the device
  hipGraphExec_t graph[2] = {nullptr, nullptr};

  void drop_graphs() {
    for (auto &gx : graph)
      if (gx) {
        (void)hipGraphExecDestroy(gx);
        gx = nullptr;
      }
  }
};

namespace {

// (re)build the force-group block tables if any box's zchunk changed
lbe_status batch_tables(lbe_batch *B) {
  int n = (int)B->boxes.size();
  bool same = (int)B->zchunks.size() == n && (int)B->shapes.size() == n;
  for (int b = 0; same && b < n; ++b)
    same = B->zchunks[b] == B->boxes[b]->args.zchunk && B->shapes[b] == B->boxes[b]->args.rows;
  if (same) return LBE_OK;
  // steps already queued on the batch stream read the current tables and
  // graphs: let them finish before either is replaced (the table uploads
  // below are blocking copies, which do not wait for a non-blocking stream)
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->drop_graphs();
  B->groups.clear();
  B->att_groups.clear();
  B->zchunks.assign(n, 0);
  B->shapes.assign(n, 0);
  char *base = B->ws + B->bp.off_force;
  size_t used = 0;
  int maxR = 0, maxent = 0;
  // one group per directed species pair (alpha, beta), reach R and (for
  // the shell gathers) tile shape: the boxes whose pair reaches R nodes (its
  // shell, or with att its attractive tail) and that were tuned to that
  // shape, in the order alpha, beta, R, shape, so that for every box the
  // pairs of one species follow each other as in a single box (each box is
  // in exactly one group per pair)
  auto build = [&](bool att, std::vector<lbe_batch::Group> &out) -> lbe_status {
    for (int al = 0; al < B->M; ++al)
      for (int be = 0; be < B->M; ++be) {
        const int k = pair_index(B->M, al, be);
        for (int R = 1; R <= RING_MAX; ++R)
          for (int shape = 0; shape < (att ? 1 : 3); ++shape) {
            std::vector<int> box_of_block, start(n, 0);
            int ent = 0;
            for (int b = 0; b < n; ++b) {
              const StepArgs &a = B->boxes[b]->args;
              if ((att ? a.t.att_R[k] : a.t.pair_R[k]) != R) continue;
              if (!att && a.rows != shape) continue;
              start[b] = (int)box_of_block.size();
              box_of_block.insert(box_of_block.end(),
                                  force_blocks(a.g, a.zchunk, att ? FORCE_TY : force_tile_rows(shape)), b);
              if (!att) ent = std::max(ent, a.t.pair_nent[k]);
            }
            if (box_of_block.empty()) continue;
            lbe_batch::Group G;
            G.R = R;
            G.shape = shape;
            G.nblocks = (int)box_of_block.size();
            G.entries = ent;
            G.alpha = al;
            G.beta = be;
            G.blockbox = (int *)(base + used);
            used += align256(sizeof(int) * box_of_block.size());
            G.blockstart = (int *)(base + used);
            used += align256(sizeof(int) * n);
            if (used > B->bp.force_bytes) return fail(LBE_ERR_OOM, "force tables exceed their reservation");
            HIP_TRY(hipMemcpy(G.blockbox, box_of_block.data(), sizeof(int) * box_of_block.size(),
                              hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(G.blockstart, start.data(), sizeof(int) * n, hipMemcpyHostToDevice));
            out.push_back(G);
            if (!att) {
              maxR = std::max(maxR, R);
              maxent = std::max(maxent, ent);
            }
          }
      }
    return LBE_OK;
  };
  if (!B->ideal) {  // the ideal gas keeps its force buffers at zero
    lbe_status st = build(false, B->groups);
    if (st != LBE_OK) return st;
    st = build(true, B->att_groups);  // added after all hard-sphere gathers
    if (st != LBE_OK) return st;
  }
  prepare_force_kernels(maxR, B->visc, maxent);
  for (int b = 0; b < n; ++b) {
    B->zchunks[b] = B->boxes[b]->args.zchunk;
    B->shapes[b] = B->boxes[b]->args.rows;
  }
  return LBE_OK;
}

// copy the members' parameter blocks to the device when they changed
lbe_status batch_upload(lbe_batch *B) {
  int n = (int)B->boxes.size();
  std::vector<StepArgs> now(n);
  for (int b = 0; b < n; ++b) now[b] = B->boxes[b]->args;
  if (B->uploaded.size() == now.size() &&
      memcmp(B->uploaded.data(), now.data(), sizeof(StepArgs) * n) == 0)
    return LBE_OK;
  HIP_TRY(hipMemcpyAsync(B->ws + B->bp.off_args, now.data(), sizeof(StepArgs) * n,
                         hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->uploaded = now;
  return LBE_OK;
}

// copy the boxes' quasi-pressure routes to the device when they changed
// (the batched scans read them at run time: no new graph is needed)
lbe_status batch_upload_routes(lbe_batch *B) {
  if (!B->bp.qp) return LBE_OK;
  const int n = (int)B->boxes.size();
  std::vector<QpRoute> now(n);
  for (int b = 0; b < n; ++b) {
    lbe_ctx *c = B->boxes[b];
    QpRoute &r = now[b];
    r.scan = c->at<double>(c->pl.off_qps);
    for (int k = 0; k < 3; ++k) r.o[k] = c->qp_origin[k];
    r.sym = (c->qp_mode & LBE_QP_SYMMETRIC) ? 1 : 0;
    r.fext = (c->qp_mode & LBE_QP_WITH_FEXT) ? 1 : 0;
  }
  if (B->routes.size() == now.size() && memcmp(B->routes.data(), now.data(), sizeof(QpRoute) * n) == 0)
    return LBE_OK;
  HIP_TRY(hipMemcpyAsync(B->ws + B->bp.off_qproutes, now.data(), sizeof(QpRoute) * n, hipMemcpyHostToDevice,
                         B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->routes = now;
  return LBE_OK;
}

void batch_launch_step(lbe_batch *B, int cur) {
  BatchArgs ba;
  ba.boxes = (const StepArgs *)(B->ws + B->bp.off_args);
  ba.blockbox = (const int *)(B->ws + B->bp.off_nodebox);
  ba.blockstart = (const int *)(B->ws + B->bp.off_nodestart);
  ba.cur = cur;
  launch_batch_moments(ba, B->bp.node_blocks, B->prec, B->currents, B->stream);
  {
    BatchArgs bb = ba;
    bb.blockbox = (const int *)(B->ws + B->bp.off_ballbox);
    bb.blockstart = (const int *)(B->ws + B->bp.off_ballstart);
    launch_batch_ball(bb, B->bp.ball_blocks, BATCH_BALL_ZC, B->bp.ball_lds, B->M, B->stream);
  }
  for (const auto &G : B->groups) {
    BatchArgs bf = ba;
    bf.blockbox = G.blockbox;
    bf.blockstart = G.blockstart;
    // the first pair of a species writes its force, later pairs add
    launch_batch_force(bf, G.nblocks, G.R, G.shape, B->visc, G.entries, G.alpha, G.beta, G.beta > 0 ? 1 : 0,
                       B->stream);
  }
  for (const auto &G : B->att_groups) {
    BatchArgs bf = ba;
    bf.blockbox = G.blockbox;
    bf.blockstart = G.blockstart;
    launch_batch_att(bf, G.nblocks, G.R, G.alpha, G.beta, B->stream);
  }
  // the per-step quasi-pressure of every box (default reading)
  if (B->bp.qp) {
    QpBatchTables t;
    for (int k = 0; k < 3; ++k) {
      t.box[k] = (const int *)(B->ws + B->bp.off_qpbox[k]);
      t.start[k] = (const int *)(B->ws + B->bp.off_qpstart[k]);
      t.nblocks[k] = B->bp.qp_blocks[k];
    }
    launch_batch_quasipressure(ba, B->bp.node_blocks, (const QpRoute *)(B->ws + B->bp.off_qproutes), t, B->M,
                               B->stream);
  }
  launch_batch_collide(ba, B->bp.node_blocks, B->prec, B->M, B->stream);
}

}  // namespace

extern "C" {

size_t lbe_batch_workspace_bytes(const lbe_config *cfgs, int nboxes) {
  BatchPlan bp;
  if (make_batch_plan(cfgs, nboxes, bp) != LBE_OK) return 0;
  return bp.total;
}

lbe_status lbe_batch_create(const lbe_config *cfgs, int nboxes, void *ws, size_t bytes, void *stream,
                            lbe_batch **out) {
  if (!out) return fail(LBE_ERR_ARG, "null output pointer");
  *out = nullptr;
  BatchPlan bp;
  lbe_status st = make_batch_plan(cfgs, nboxes, bp);
  if (st != LBE_OK) return st;
  if (!ws || ((uintptr_t)ws & 255u)) return fail(LBE_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < bp.total) return fail(LBE_ERR_OOM, "workspace of %zu bytes, %zu needed", bytes, bp.total);
  lbe_batch *B = new (std::nothrow) lbe_batch();
  if (!B) return fail(LBE_ERR_OOM, "host allocation failed");
  B->bp = bp;
  B->ws = (char *)ws;
  B->stream = (hipStream_t)stream;
  B->prec = cfgs[0].prec;
  B->visc = (cfgs[0].flags & LBE_VISC) && !(cfgs[0].flags & LBE_IDEAL);
  B->M = cfgs[0].nspecies;
  B->ideal = (cfgs[0].flags & LBE_IDEAL) != 0;
  B->currents = ((cfgs[0].flags & LBE_VISC) || ((cfgs[0].flags & LBE_DRAG) && B->M > 1)) &&
                !(cfgs[0].flags & LBE_IDEAL);
  std::vector<int> nodebox, nodestart(nboxes), ballbox, ballstart(nboxes);
  for (int b = 0; b < nboxes; ++b) {
    lbe_ctx *c = nullptr;
    st = lbe_create(&cfgs[b], B->ws + bp.box_off[b], bp.box_bytes[b], stream, &c);
    if (st != LBE_OK) {
      lbe_batch_destroy(B);
      return st;
    }
    B->boxes.push_back(c);
    nodestart[b] = (int)nodebox.size();
    nodebox.insert(nodebox.end(), node_blocks(c->pl.g), b);
    ballstart[b] = (int)ballbox.size();
    ballbox.insert(ballbox.end(), ball_blocks(c->pl.g, BATCH_BALL_ZC), b);
  }
  bool up_ok = true;
  if (bp.qp)
    for (int k = 0; k < 3 && up_ok; ++k) {
      std::vector<int> qbox, qstart(nboxes);
      for (int b = 0; b < nboxes; ++b) {
        qstart[b] = (int)qbox.size();
        qbox.insert(qbox.end(), qp_blocks(B->boxes[b]->pl.g, k), b);
      }
      up_ok = hipMemcpy(B->ws + bp.off_qpbox[k], qbox.data(), sizeof(int) * qbox.size(),
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->ws + bp.off_qpstart[k], qstart.data(), sizeof(int) * nboxes,
                        hipMemcpyHostToDevice) == hipSuccess;
    }
  if (!up_ok ||
      hipMemcpy(B->ws + bp.off_nodebox, nodebox.data(), sizeof(int) * nodebox.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B->ws + bp.off_nodestart, nodestart.data(), sizeof(int) * nboxes,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B->ws + bp.off_ballbox, ballbox.data(), sizeof(int) * ballbox.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B->ws + bp.off_ballstart, ballstart.data(), sizeof(int) * nboxes,
                hipMemcpyHostToDevice) != hipSuccess) {
    lbe_batch_destroy(B);
    return fail(LBE_ERR_HIP, "batch table upload failed");
  }
  *out = B;
  return LBE_OK;
}

lbe_ctx *lbe_batch_box(lbe_batch *B, int box) {
  if (!B || box < 0 || box >= (int)B->boxes.size()) {
    fail(LBE_ERR_ARG, "bad box index");
    return nullptr;
  }
  return B->boxes[box];
}

lbe_status lbe_batch_step(lbe_batch *B, int nsteps, int mode) {
  if (!B) return fail(LBE_ERR_ARG, "null batch");
  if (nsteps < 0 || mode < 0 || mode > 2) return fail(LBE_ERR_ARG, "bad nsteps or mode");
  if (mode == 0) {
    for (lbe_ctx *c : B->boxes) {
      lbe_status st = lbe_step(c, nsteps);
      if (st != LBE_OK) return st;
    }
    return LBE_OK;
  }
  int cur = B->boxes[0]->cur;
  for (size_t b = 0; b < B->boxes.size(); ++b) {
    lbe_ctx *c = B->boxes[b];
    if (c->poisoned) return fail(LBE_ERR_UNSTABLE, "box %zu is unstable; reinitialise it", b);
    if (c->next_phase != 0) return fail(LBE_ERR_STATE, "box %zu has an incomplete phased step", b);
    if (c->cur != cur) return fail(LBE_ERR_STATE, "boxes are at different buffer parities");
  }
  for (size_t b = 0; b < B->boxes.size(); ++b) {
    const lbe_ctx *c = B->boxes[b];
    if (c->args.pifield && c->qp_origin_solid)
      return fail(LBE_ERR_STATE, "the quasi-pressure origin of box %zu is a solid node", b);
  }
  lbe_status st = batch_tables(B);
  if (st != LBE_OK) return st;
  st = batch_upload(B);
  if (st != LBE_OK) return st;
  st = batch_upload_routes(B);
  if (st != LBE_OK) return st;
  int left = nsteps;
  if (mode == 2) {
    if (left >= 2 && !B->graph[cur]) {
      hipGraph_t gr = nullptr;
      HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
      batch_launch_step(B, cur);
      batch_launch_step(B, cur ^ 1);
      HIP_TRY(hipStreamEndCapture(B->stream, &gr));
      hipError_t e = hipGraphInstantiate(&B->graph[cur], gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) return fail(LBE_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    for (; left >= 2; left -= 2) HIP_TRY(hipGraphLaunch(B->graph[cur], B->stream));
  }
  for (; left > 0; --left) {
    batch_launch_step(B, cur);
    cur ^= 1;
  }
  LAUNCH_CHECK();
  if (nsteps & 1)
    for (lbe_ctx *c : B->boxes) c->cur ^= 1;
  return LBE_OK;
}

void lbe_batch_destroy(lbe_batch *B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->stream);
  B->drop_graphs();
  for (lbe_ctx *c : B->boxes) lbe_destroy(c);
  delete B;
}

}  // extern "C"
