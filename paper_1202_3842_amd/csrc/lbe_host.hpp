// lbe_host.hpp -- host-side internals shared by the runtime sources of the
// Lattice Boltzmann-Enskog library (context, plan of the workspace, error
// reporting).  Not part of the ABI.
#pragma once

#include <stddef.h>

#include <vector>

#include "lbe_internal.hpp"

namespace lbe {

// record an error text for lbe_last_error() and return the code
lbe_status fail(lbe_status code, const char *fmt, ...);
// the last error text of this thread
const char *error_text();
void clear_error();

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::lbe::fail(LBE_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK()                                                             \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess)                                                          \
      return ::lbe::fail(LBE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Lattice shell of radius s: points e != 0 with s - 1/2 <= |e| < s + 1/2,
// kept as the half S+ (e_z > 0, or e_z = 0 and e_y > 0, or e_z = e_y = 0 and
// e_x > 0) grouped by e_z, with the uniform weight 4 pi s / sum_e |e| that
// makes the weighted first moment (4 pi/3) s delta_ij (Appendix integral
// over the unit sphere).
struct HostShell {
  std::vector<int> e;  // 3 per point of S+, ordered by e_z, then e_y, then e_x
  double weight = 0.0;
  int maxc = 0;
};

// Attractive tail of a pair: the half S+ of the thick shell sigma_ab <= |e|
// < rc, grouped by e_z, with K = U'(|e|) e^ per point for U = -eps
// (sigma_ab/r)^6.
struct HostAtt {
  std::vector<int> e;     // 3 per point of S+, ordered by e_z, then e_y, then e_x
  std::vector<double> K;  // 3 per point
  int maxc = 0;
};

struct Plan {
  Geom g;
  int M = 0, npairs = 0;
  long long Ns = 0;
  size_t pop_bytes = 0;  // one ping-pong buffer
  std::vector<HostShell> shells;
  std::vector<HostAtt> atts;  // one per unordered pair, empty without attraction
  std::vector<std::vector<int>> balls;
  int nshell = 0, nball = 0, natt = 0;
  size_t off_flag = 0, off_result = 0, off_ring_ofs = 0, off_ring_off = 0, off_ring_e = 0,
         off_ball = 0, off_bb = 0, off_V = 0, off_F = 0, off_solid = 0, off_pop0 = 0,
         off_pop1 = 0, off_n = 0, off_G = 0, off_J = 0, off_force = 0, off_read = 0,
         off_part = 0, off_att_ofs = 0, off_pi = 0, off_qps = 0, total = 0;
  int nblocks = 0;
};

// workspace plan of one box
lbe_status make_plan(const lbe_config *cfg, Plan &pl);
// whether the flags select the per-step quasi-pressure (the default reading)
bool qp_per_step(unsigned flags);

}  // namespace lbe

struct lbe_ctx {
  lbe_config cfg;
  lbe::Plan pl;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  int cur = 0;             // ping-pong buffer holding the current state
  int next_phase = 0;      // lbe_step_phase position inside a step
  bool poisoned = false;
  // route of the per-step quasi-pressure: origin, mode bits, and whether the
  // origin is a solid node (a step then fails)
  int qp_origin[3] = {0, 0, 0};
  unsigned qp_mode = LBE_QP_SYMMETRIC;
  bool qp_origin_solid = false;
  // bumped whenever a parameter the adjoint's backward re-reads changes
  // (potential, body forces, solid mask, quasi-pressure route)
  unsigned long long epoch = 0;
  lbe::StepArgs args;
  lbe::Readout rd;

  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  void *pop(int buf) const { return ws + (buf ? pl.off_pop1 : pl.off_pop0); }
  size_t psize() const { return cfg.prec == LBE_FP64 ? 8 : 4; }
  // one (dist, species) block of 19 populations in buffer buf
  char *block(int buf, int dist, int s) const {
    return (char *)pop(buf) + (size_t)(dist * pl.M + s) * lbe::Q * pl.Ns * psize();
  }
};

// Argument checks and the read-out pass of the quasi-pressure calls
// (lbe_api.hip), shared with lbe_get_quasipressure_noalloc; not exported.
extern "C" __attribute__((visibility("hidden"))) lbe_status lbe_qp_readout_for(lbe_ctx *c,
                                                                              const int origin[3],
                                                                              unsigned mode);
