// lbe_noalloc.hip -- the quasi-pressure read-out for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid allocation): lbe_get_quasipressure_noalloc.
//
// It runs the kernels of lbe_get_quasipressure for one species, but the
// three line scans of the path integral work in a file-scope device array
// instead of the context's workspace, and Pi goes straight to the caller's
// device buffer.  The array is QP_SCRATCH_BYTES on every GPU the library
// runs on and lives until the process ends; host code uses the per-device
// address from hipGetSymbolAddress, never the array's name.  Every call on
// a GPU shares that GPU's array: calls that overlap on one GPU race.
#include <mutex>

#include "lbe_host.hpp"

namespace {

constexpr size_t QP_SCRATCH_BYTES = (size_t)64 << 20;   // 3 scans of up to 2796202 nodes
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[QP_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this GPU's scratch array, looked up once per device
// with that device current.
lbe_status scratch_address(int device, void **out) {
  if (device < 0 || device >= MAX_DEVICES) return lbe::fail(LBE_ERR_UNSUPPORTED, "device %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return lbe::fail(LBE_ERR_HIP, "hipGetSymbolAddress of the scratch array failed: %s",
                       hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return LBE_OK;
}

}  // namespace

extern "C" lbe_status lbe_get_quasipressure_noalloc(lbe_ctx *c, int species, const int origin[3],
                                                   unsigned mode, double *out) {
  using namespace lbe;
  if (!c) return fail(LBE_ERR_ARG, "null context");
  if (species < 0 || species >= c->pl.M) return fail(LBE_ERR_ARG, "bad species %d", species);
  if (!out) return fail(LBE_ERR_ARG, "null output");
  const size_t need = sizeof(double) * 3 * (size_t)c->pl.g.N;
  if (need > QP_SCRATCH_BYTES)
    return fail(LBE_ERR_ARG, "the box has %d nodes; the allocation-free quasi-pressure takes at most %zu",
                c->pl.g.N, QP_SCRATCH_BYTES / (3 * sizeof(double)));
  void *scr = nullptr;
  lbe_status st = scratch_address(c->device, &scr);
  if (st != LBE_OK) return st;
  st = lbe_qp_readout_for(c, origin, mode);
  if (st != LBE_OK) return st;
  // the chosen species seen as species 0 of a one-species view
  StepArgs a = c->args;
  const Geom &g = c->pl.g;
  a.M = 1;
  a.nfield += (long long)species * g.Np;
  a.force += 6LL * species * g.N;
  for (int k = 0; k < 3; ++k) a.body[0][k] = c->args.body[species][k];
  launch_quasipressure(a, origin, mode, false, static_cast<double *>(scr), out, c->stream);
  LAUNCH_CHECK();
  return LBE_OK;
}
