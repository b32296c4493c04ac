// lbe_kernels.hip -- gfx950 kernels of one stabilized Lattice Boltzmann-Enskog
// step (double distribution, trapezoidal rule; arXiv:1202.3842).
//
// Data layout in HBM
//   populations  pop[dist][species][p][Ns]  (dist 0 = f~, 1 = g~), FP64 or
//                FP32, two ping-pong buffers.  A buffer holds the
//                post-collision, pre-streaming values; streaming happens in
//                the pull that the next pass performs.
//   fields       padded boxes (R ghost layers) of n^a, G_ab and J~^a, with
//                periodic images in the ghosts (zeros beyond walls), so that
//                shell and ball gathers are constant offsets.
//
// Kernels per step
//   k_moments  pull populations, n~ (and J~ with C^visc), write fields
//   k_ball     LDS-tiled ball-averaged densities -> BMCSL contact values G_ab
//   k_force    LDS-tiled shell gather of C^mf (and C^visc) per species pair
//   k_collide  pull, inversion, equilibria, sources, trapezoidal BGK
//              update, store
// and, for the adjoint with respect to V, their reverse passes (k_adj_*,
// k_ball modes 1 and 2, k_tape_moments).
#include <math.h>
#include <string.h>

#include <type_traits>

#include "lbe_internal.hpp"

namespace lbe {
namespace {

constexpr int BLOCK = 256;
// tiles of the LDS-tiled gathers: FTX x FTY nodes per workgroup of FNT threads
constexpr int FTX = FORCE_TX, FTY = FORCE_TY;
constexpr int FNT = FTX * FTY;
// force-kernel tile shapes (StepArgs::rows): output rows per thread,
// threads, and tile height
constexpr int shape_ny(int shape) { return shape == 1 ? 2 : 1; }
constexpr int shape_nt(int shape) { return shape == 2 ? 512 : 256; }
constexpr int shape_ty(int shape) { return shape_nt(shape) / FTX * shape_ny(shape); }

// D3Q19 velocities (order documented in lbe.h) and weights
__host__ __device__ constexpr int cvec(int p, int k) {
  constexpr int c[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return c[p][k];
}
__host__ __device__ constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }
__host__ __device__ constexpr double wgt(int p) {
  return p == 0 ? 1.0 / 3.0 : (p <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Read-only tables seen through the constant address space, so that loads
// with a workgroup-uniform index become scalar loads.
template <typename T>
__device__ inline const __attribute__((address_space(4))) T *cptr(const T *p) {
  return (const __attribute__((address_space(4))) T *)(p);
}

// The lattice geometry as a local value (member-wise, so it also works when
// the parameter block lives in the constant address space of a batch).
template <class A>
__device__ inline Geom geom_of(const A &a) {
  Geom g;
  g.nx = a.g.nx;
  g.ny = a.g.ny;
  g.nz = a.g.nz;
  g.N = a.g.N;
  g.R = a.g.R;
  g.PX = a.g.PX;
  g.PY = a.g.PY;
  g.PZ = a.g.PZ;
  g.Np = a.g.Np;
  g.periodic = a.g.periodic;
  return g;
}

// population loads and stores are streamed once per pass: non-temporal, so
// that they do not evict the gathered fields from the caches
template <typename T>
__device__ inline double ld(const T *__restrict__ a, long long i) {
  return (double)__builtin_nontemporal_load(a + i);
}

struct Coord {
  int x, y, z;
  int xm, xp, ym, yp, zm, zp;
};

__device__ inline Coord decode(const Geom &g, int i) {
  Coord c;
  c.x = i % g.nx;
  int t = i / g.nx;
  c.y = t % g.ny;
  c.z = t / g.ny;
  c.xm = c.x == 0 ? g.nx - 1 : c.x - 1;
  c.xp = c.x == g.nx - 1 ? 0 : c.x + 1;
  c.ym = c.y == 0 ? g.ny - 1 : c.y - 1;
  c.yp = c.y == g.ny - 1 ? 0 : c.y + 1;
  c.zm = c.z == 0 ? g.nz - 1 : c.z - 1;
  c.zp = c.z == g.nz - 1 ? 0 : c.z + 1;
  return c;
}

// node r - c_p (wrapped; blocked neighbours are excluded by the bb mask)
__device__ inline int upstream(const Geom &g, const Coord &c, int p) {
  int X = cvec(p, 0) > 0 ? c.xm : (cvec(p, 0) < 0 ? c.xp : c.x);
  int Y = cvec(p, 1) > 0 ? c.ym : (cvec(p, 1) < 0 ? c.yp : c.y);
  int Z = cvec(p, 2) > 0 ? c.zm : (cvec(p, 2) < 0 ? c.zp : c.z);
  return X + g.nx * (Y + g.ny * Z);
}
// node r + c_p
__device__ inline int downstream(const Geom &g, const Coord &c, int p) {
  int X = cvec(p, 0) > 0 ? c.xp : (cvec(p, 0) < 0 ? c.xm : c.x);
  int Y = cvec(p, 1) > 0 ? c.yp : (cvec(p, 1) < 0 ? c.ym : c.y);
  int Z = cvec(p, 2) > 0 ? c.zp : (cvec(p, 2) < 0 ? c.zm : c.z);
  return X + g.nx * (Y + g.ny * Z);
}

// Pull the 19 post-streaming populations of one (dist, species) block:
// f~_p(r) = f~*_p(r - c_p), or f~*_opp(p)(r) when r - c_p is blocked.
template <typename T>
__device__ inline void pull19(const Geom &g, const Coord &c, int i, uint32_t m,
                              const T *__restrict__ blk, long long Ns, double v[19]) {
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    if (p == 0) {
      v[0] = ld(blk, i);
    } else if ((m >> p) & 1u) {
      v[p] = ld(blk, (long long)opp(p) * Ns + i);
    } else {
      v[p] = ld(blk, (long long)p * Ns + upstream(g, c, p));
    }
  }
}

__device__ inline void moments0(const double v[19], double &s) {
  double a = 0.0;
#pragma unroll
  for (int p = 0; p < Q; ++p) a += v[p];
  s = a;
}

// J = sum_p c_p g_p, summed over +-c pairs so a mirror-symmetric node gives 0
__device__ inline void moments1(const double v[19], double J[3]) {
  double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int p = 1; p < Q; p += 2) {
    double d = v[p] - v[p + 1];
    if (cvec(p, 0) > 0) jx += d;
    if (cvec(p, 0) < 0) jx -= d;
    if (cvec(p, 1) > 0) jy += d;
    if (cvec(p, 1) < 0) jy -= d;
    if (cvec(p, 2) > 0) jz += d;
    if (cvec(p, 2) < 0) jz -= d;
  }
  J[0] = jx;
  J[1] = jy;
  J[2] = jz;
}

// periodic images of coordinate x in [-R, n+R)
__device__ inline int images(int x, int n, int R, bool per, int out[3]) {
  int k = 0;
  out[k++] = x;
  if (per) {
    if (x - n >= -R) out[k++] = x - n;
    if (x + n < n + R) out[k++] = x + n;
  }
  return k;
}

__device__ inline void store_images(const Geom &g, double *__restrict__ f, const Coord &c,
                                    double v) {
  int xs[3], ys[3], zs[3];
  int kx = images(c.x, g.nx, g.R, g.periodic & 1u, xs);
  int ky = images(c.y, g.ny, g.R, g.periodic & 2u, ys);
  int kz = images(c.z, g.nz, g.R, g.periodic & 4u, zs);
  for (int a = 0; a < kz; ++a)
    for (int b = 0; b < ky; ++b)
      for (int d = 0; d < kx; ++d) f[padded_index(g, xs[d], ys[b], zs[a])] = v;
}

__device__ inline long long pop_stride(const Geom &g) { return ((long long)g.N + 63) / 64 * 64; }

// ------------------------------------------------------------------------
// set-up kernels
// ------------------------------------------------------------------------
__global__ void k_bbmask(Geom g, const uint8_t *__restrict__ solid, uint32_t *__restrict__ bb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  Coord c = decode(g, i);
  uint32_t m = solid[i] ? 1u : 0u;
#pragma unroll
  for (int p = 1; p < Q; ++p) {
    int X = c.x - cvec(p, 0), Y = c.y - cvec(p, 1), Z = c.z - cvec(p, 2);
    bool out = false;
    if (X < 0 || X >= g.nx) out |= !(g.periodic & 1u);
    if (Y < 0 || Y >= g.ny) out |= !(g.periodic & 2u);
    if (Z < 0 || Z >= g.nz) out |= !(g.periodic & 4u);
    if (!out) out = solid[upstream(g, c, p)] != 0;
    if (out) m |= 1u << p;
  }
  bb[i] = m;
}

// F = -grad_h V = -(1/v_T^2) sum_p w_p c_p V(r + c_p); clamp at walls
__global__ void k_extforce(Geom g, const double *__restrict__ V, double *__restrict__ F) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  Coord c = decode(g, i);
  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int p = 1; p < Q; ++p) {
    int X = c.x + cvec(p, 0), Y = c.y + cvec(p, 1), Z = c.z + cvec(p, 2);
    X = X < 0 ? ((g.periodic & 1u) ? X + g.nx : 0) : (X >= g.nx ? ((g.periodic & 1u) ? X - g.nx : g.nx - 1) : X);
    Y = Y < 0 ? ((g.periodic & 2u) ? Y + g.ny : 0) : (Y >= g.ny ? ((g.periodic & 2u) ? Y - g.ny : g.ny - 1) : Y);
    Z = Z < 0 ? ((g.periodic & 4u) ? Z + g.nz : 0) : (Z >= g.nz ? ((g.periodic & 4u) ? Z - g.nz : g.nz - 1) : Z);
    double v = wgt(p) * V[X + g.nx * (Y + g.ny * Z)];
    if (cvec(p, 0)) gx += cvec(p, 0) * v;
    if (cvec(p, 1)) gy += cvec(p, 1) * v;
    if (cvec(p, 2)) gz += cvec(p, 2) * v;
  }
  // 1/v_T^2 = 3 for D3Q19
  F[i] = -3.0 * gx;
  F[(long long)g.N + i] = -3.0 * gy;
  F[2LL * g.N + i] = -3.0 * gz;
}

template <typename T>
__global__ void k_zero_solid(Geom g, int nblk, T *__restrict__ pop, const uint32_t *__restrict__ bb,
                             long long Ns) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N || !(bb[i] & 1u)) return;
  for (int k = 0; k < nblk * Q; ++k) pop[(long long)k * Ns + i] = T(0);
}

// Pre-streaming values whose pull gives the rest equilibrium w_p n0(r):
// slot (s, q) streams to s + c_q, or back to (s, opp q) at a wall.
template <typename T>
__global__ void k_rest_equilibrium(Geom g, const uint32_t *__restrict__ bb,
                                   const double *__restrict__ n0, T *__restrict__ out, long long Ns) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  uint32_t m = bb[i];
  Coord c = decode(g, i);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double v = 0.0;
    if (!(m & 1u)) {
      if (q == 0 || ((m >> opp(q)) & 1u))
        v = wgt(q) * n0[i];
      else
        v = wgt(q) * n0[downstream(g, c, q)];
    }
    out[(long long)q * Ns + i] = T(v);
  }
}

// inverse of the pull: pre-streaming values from post-streaming targets
template <typename T>
__global__ void k_unstream(Geom g, const uint32_t *__restrict__ bb, const T *__restrict__ target,
                           T *__restrict__ out, long long Ns) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  uint32_t m = bb[i];
  Coord c = decode(g, i);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    T v = T(0);
    if (!(m & 1u)) {
      if (q == 0)
        v = target[i];
      else if ((m >> opp(q)) & 1u)
        v = target[(long long)opp(q) * Ns + i];
      else
        v = target[(long long)q * Ns + downstream(g, c, q)];
    }
    out[(long long)q * Ns + i] = v;
  }
}

template <typename T>
__global__ void k_pull(Geom g, const uint32_t *__restrict__ bb, const T *__restrict__ pre,
                       T *__restrict__ out, long long Ns) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  uint32_t m = bb[i];
  Coord c = decode(g, i);
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    T v = T(0);
    if (!(m & 1u)) {
      if (p == 0)
        v = pre[i];
      else if ((m >> p) & 1u)
        v = pre[(long long)opp(p) * Ns + i];
      else
        v = pre[(long long)p * Ns + upstream(g, c, p)];
    }
    out[(long long)p * Ns + i] = v;
  }
}

// ------------------------------------------------------------------------
// step kernels
// ------------------------------------------------------------------------
template <typename T, bool VISC, class A>
__device__ inline void moments_body(const A &a, const T *__restrict__ pop, int i) {
  const Geom g = geom_of(a);
  if (i >= g.N) return;
  Coord c = decode(g, i);
  uint32_t m = a.bb[i];
  long long Ns = pop_stride(g);
  for (int s = 0; s < a.M; ++s) {
    double n = 0.0, J[3] = {0.0, 0.0, 0.0};
    if (!(m & 1u)) {
      double v[19];
      pull19(g, c, i, m, pop + (long long)s * Q * Ns, Ns, v);
      moments0(v, n);
      if (VISC) {
        // the current of C^visc: from g, or from f with a single distribution
        if (!(a.flags & LBE_SINGLE)) pull19(g, c, i, m, pop + (long long)(a.M + s) * Q * Ns, Ns, v);
        moments1(v, J);
      }
    }
    store_images(g, a.nfield + (long long)s * g.Np, c, n);
    if (VISC)
      for (int k = 0; k < 3; ++k) store_images(g, a.Jfield + (long long)(3 * s + k) * g.Np, c, J[k]);
  }
}

template <typename T, bool VISC>
__global__ __launch_bounds__(BLOCK) void k_moments(StepArgs a, const T *__restrict__ pop) {
  moments_body<T, VISC>(a, pop, blockIdx.x * BLOCK + threadIdx.x);
}

// ------------------------------------------------------------------------
// LDS-tiled ball gathers.  A workgroup owns FTX x FTY x ZC nodes; for each
// species it stages the (FTX + 2R) x (FTY + 2R) x (ZC + 2R) block of the
// padded field (R = the largest ball reach) in LDS and every thread sums
// the ball of each of its ZC nodes, one ball point for all ZC nodes at a
// time.  Each node's sum runs over the ball in table order (normalised by
// the full ball size), so the result does not depend on ZC.
//   MODE 0: ball averages of n -> BMCSL contact values G (forward)
//   MODE 1: ball averages of n and Gbar -> adjoint of the ball averages
//   MODE 2: ball averages of that adjoint, added into nbar (the transpose)
// ------------------------------------------------------------------------
template <int M, int MODE, int ZC, class A>
__device__ inline void ball_body(const A &a, const AdjArgs &d, int b, double *lds) {
  const Geom g = geom_of(a);
  const int Rb = a.t.ball_R;
  const int BW = FTX + 2 * Rb, BH = FTY + 2 * Rb, BZ = ZC + 2 * Rb, BP = BW * BH, BV = BP * BZ;
  int *loff = (int *)(lds + BV);
  const int nbx = (g.nx + FTX - 1) / FTX, nby = (g.ny + FTY - 1) / FTY;
  const int x0 = (b % nbx) * FTX, y0 = ((b / nbx) % nby) * FTY, z0 = (b / (nbx * nby)) * ZC;
  const int t = threadIdx.x, tx = t % FTX, ty = t / FTX;
  const int base = (ty + Rb) * BW + (tx + Rb) + Rb * BP;
  for (int j = t; j < a.t.ball_total; j += BLOCK) loff[j] = a.t.ball_loff[j];
  double nb[M][ZC];
  for (int sp = 0; sp < M; ++sp) {
    const double *src = (MODE == 2 ? d.nbb : a.nfield) + (long long)sp * g.Np;
    __syncthreads();  // the previous species' readers are done with the block
    for (int e = t; e < BV; e += BLOCK) {
      const int cx = e % BW, cy = (e / BW) % BH, cz = e / BP;
      const int X = x0 - Rb + cx + g.R, Y = y0 - Rb + cy + g.R, Z = z0 - Rb + cz + g.R;
      lds[e] = (X < g.PX && Y < g.PY && Z < g.PZ) ? src[X + (long long)g.PX * (Y + (long long)g.PY * Z)] : 0.0;
    }
    __syncthreads();
    double s[ZC];
#pragma unroll
    for (int zz = 0; zz < ZC; ++zz) s[zz] = 0.0;
    const int j0 = a.t.ball_start[sp], cnt = a.t.ball_n[sp];
    for (int j = 0; j < cnt; ++j) {
      const double *p = lds + base + loff[j0 + j];
#pragma unroll
      for (int zz = 0; zz < ZC; ++zz) s[zz] += p[zz * BP];
    }
#pragma unroll
    for (int zz = 0; zz < ZC; ++zz) nb[sp][zz] = s[zz] / (double)cnt;
  }
  const int x = x0 + tx, y = y0 + ty;
  if (x >= g.nx || y >= g.ny) return;
  bool bad = false;  // packing fraction >= 1 or a non-finite density here
#pragma unroll
  for (int zz = 0; zz < ZC; ++zz) {
    const int z = z0 + zz;
    if (z >= g.nz) break;
    const int i = x + g.nx * (y + g.ny * z);
    const bool solid = a.bb[i] & 1u;
    const Coord c = decode(g, i);
    if (MODE == 2) {
      for (int sp = 0; sp < M; ++sp) {
        double *o = d.nbar + (long long)sp * g.N + i;
        *o = solid ? 0.0 : *o + nb[sp][zz];
      }
      continue;
    }
    constexpr int NP = M * (M + 1) / 2;
    double xi2 = 0.0, xi3 = 0.0;
    bool finite = true;
    for (int sp = 0; sp < M; ++sp) {
      const double sg = a.t.sigma[sp];
      finite &= isfinite(nb[sp][zz]);
      xi2 += sg * sg * nb[sp][zz];
      xi3 += sg * sg * sg * nb[sp][zz];
    }
    xi2 *= M_PI / 6.0;
    xi3 *= M_PI / 6.0;
    if (MODE == 0) {
      double G[NP];
      if (solid) {
        for (int k = 0; k < NP; ++k) G[k] = 0.0;
      } else {
        bad |= !(xi3 < 1.0) || !finite;
        const double one = 1.0 - xi3;
        const double i1 = 1.0 / one;
        const double i2 = i1 * i1;
        const double i3 = i2 * i1;
        for (int pa = 0; pa < M; ++pa)
          for (int pb = pa; pb < M; ++pb) {
            const int k = pair_index(M, pa, pb);
            const double dd = a.t.pair_d[k];
            G[k] = i1 + 3.0 * dd * xi2 * i2 + 2.0 * dd * dd * xi2 * xi2 * i3;
          }
      }
      for (int k = 0; k < NP; ++k) store_images(g, a.Gfield + (long long)k * g.Np, c, G[k]);
    } else {
      double x2b = 0.0, x3b = 0.0;
      if (!solid) {
        const double i1 = 1.0 / (1.0 - xi3), i2 = i1 * i1, i3 = i2 * i1, i4 = i2 * i2;
        for (int pa = 0; pa < M; ++pa)
          for (int pb = pa; pb < M; ++pb) {
            const int k = pair_index(M, pa, pb);
            const double dd = a.t.pair_d[k];
            const double Gb = d.Gbar[(long long)k * g.N + i];
            x2b += Gb * (3.0 * dd * i2 + 4.0 * dd * dd * xi2 * i3);
            x3b += Gb * (i2 + 6.0 * dd * xi2 * i3 + 6.0 * dd * dd * xi2 * xi2 * i4);
          }
      }
      for (int sp = 0; sp < M; ++sp) {
        const double sg = a.t.sigma[sp];
        store_images(g, d.nbb + (long long)sp * g.Np, c,
                     solid ? 0.0 : (M_PI / 6.0) * (sg * sg * x2b + sg * sg * sg * x3b));
      }
    }
  }
  // one atomic per wave that saw a bad node (an unstable state would
  // otherwise issue one per node)
  if (MODE == 0) {
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && (int)(threadIdx.x & 63u) == __ffsll((long long)m) - 1) atomicOr(a.errflag, 1u);
  }
}

template <int M, int MODE, int ZC>
__global__ __launch_bounds__(BLOCK) void k_ball(StepArgs a, AdjArgs d) {
  extern __shared__ double lds[];
  ball_body<M, MODE, ZC>(a, d, blockIdx.x, lds);
}

// Nonlocal forces on the tilde moments, one directed species pair (a, b)
// per launch, per particle of species a (the factor n_a(r) is applied by the
// collision kernel):
//   C^mf_a / n_a  += -kT sigma_ab^2 w_ab sum_{e in S+} e^ [g(r,r+e) n_b(r+e)
//                                                    - g(r,r-e) n_b(r-e)]
//   C^visc_a / n_a += 2 sigma_ab^2 sqrt(kT/pi) w_ab sum_e e^ (e^.(u_b(r+e)
//                                      - u_b(r))) g(r,r+e) n_b(r+e)
// with g(r,q) = (G_ab(r) + G_ab(q))/2 and n_b u_b = J~_b.
//
// Tiling: a workgroup owns an FTX x FTY tile of output nodes and marches
// over zchunk planes in z.  For each output plane it stages, per e_z = 0..R,
// the two source planes z + e_z and z - e_z (with an R-wide halo in x and y)
// in LDS and walks the ring of shell points with that e_z; the +e and -e
// points of a pair sit in the two staged planes, so every pair is summed
// together and a uniform state gives exactly zero.  LDS holds 2 planes of
// n_b, G_ab (and J~_b with C^visc): 2 * NF * (FTX+2R)(FTY+2R) doubles.


typedef double dbl2 __attribute__((ext_vector_type(2)));

// where force_body reads its ring table from (see there): scalar loads for
// C^visc, the adjoint gather, the attraction and any tile with two rows per
// thread; LDS for C^mf alone with one row per thread
__host__ __device__ constexpr bool table_in_smem(int mode, int ny = 1) { return mode != 0 || ny > 1; }
// fields staged per plane by force_body
__host__ __device__ constexpr int force_fields(int mode) {
  return mode == 0 ? 2 : (mode == 3 ? 1 : (mode == 4 ? 3 : (mode == 5 ? 8 : 5)));
}
// dynamic LDS of force_body: two planes of NF fields, then the ring table
// when it is staged in LDS
__host__ __device__ constexpr size_t force_lds(int mode, int R, int ty, int entries, int ny = 1) {
  return sizeof(double) * ((size_t)2 * force_fields(mode) * (FTX + 2 * R) * (ty + 2 * R) +
                           (table_in_smem(mode, ny) ? 0 : 4 * (size_t)entries));
}

// MODE 0: C^mf; MODE 1: C^mf and C^visc; MODE 2: the transpose of the C^mf
// gather for the adjoint (fields n_b, G_ab and the adjoint force phi_a^bar,
// see k_adj_force); MODE 3: the attractive field G^{ab} = sum_e U'(|e|) e^
// n_b(r + e) over the pair's thick shell (field n_b; the table holds
// U'(|e|) e^), added to C^mf/n_a; MODE 4: the transpose of MODE 3 for the
// adjoint, n_b^bar(r) -= sum_e U'(|e|) e^.phibar_a(r + e) (field phibar_a, the
// same table); MODE 5: the transpose of the C^visc gather for the adjoint
// (see k_adj_visc), over the fields phibar'_a (the adjoint of C^visc/n_a),
// G_ab, u~_b and n_b.  NT threads in rows of FTX; NY = output rows per thread:
// the tile is FTX x (NT/FTX NY) and thread (tx, ty) owns rows ty,
// ty + NT/FTX, ...; one ring-table read and one address then serve NY nodes.
// Taller tiles shrink the staged window per node.
template <int R, int MODE, int NY, int NT, class A>
__device__ inline void force_body(const A &a, const AdjArgs *ad, int alpha, int beta, int accumulate,
                                  int bx, int by, int bz, double *lds) {
  constexpr bool VISC = MODE == 1;
  constexpr bool ADJ = MODE == 2;
  constexpr bool ATT = MODE == 3;
  constexpr bool AADJ = MODE == 4;
  constexpr bool VTF = MODE == 5;
  constexpr int NF = force_fields(MODE);
  constexpr int RY = NT / FTX;                  // thread rows of the workgroup
  constexpr int TY = RY * NY;
  constexpr int W = FTX + 2 * R, H = TY + 2 * R, WH = W * H;
  constexpr int SLOTS = (WH + NT - 1) / NT;     // window elements per thread and field
  constexpr int ROW = RY * W;                   // LDS distance between a thread's rows
  // NS accumulator sets per row, taking the pairs of a ring in turn (and
  // summed in order at the end): shorter dependency chains, and the same
  // summation order for every tile shape, so results do not depend on the
  // tiling (four sets for C^mf + C^visc: 0.789 -> 0.762 ms at 128^3, sigma = 6, where
  // three or six were no faster than two; four also for the attraction and
  // the C^mf and attraction transposes, a few per cent each; two for C^mf
  // alone, whose two-row tiles slowed from 0.245 to 0.269 ms with four, and
  // for the C^visc transpose, already at 256 VGPRs)
  constexpr int NS = (MODE == 0 || MODE == 5) ? 2 : 4;
  // LDS layout of a staged plane.  PAIRED: n and G interleaved, then the x and
  // y components of the vector field interleaved, then its z component, so a
  // point's n and G come in with one 16-byte read; otherwise one array per
  // field.  The separate arrays are faster with C^visc, the interleaved ones
  // for C^mf alone and for the adjoint gather (measured).
  constexpr bool PAIRED = MODE == 0 || MODE == 2;
  auto at = [&](int f, int e) {
    return PAIRED ? (f < 2 ? 2 * e + f : (f < 4 ? 2 * WH + 2 * e + (f - 2) : 4 * WH + e)) : f * WH + e;
  };
  const Geom g = geom_of(a);
  const int k = pair_index(a.M, alpha, beta);
  const int t = threadIdx.x, tx = t % FTX, ty = t / FTX;
  const int x0 = bx * FTX, y0 = by * TY;
  const int x = x0 + tx;
  const double *__restrict__ fld[8];
  fld[0] = a.nfield + (long long)beta * g.Np;
  fld[1] = a.Gfield + (long long)k * g.Np;
  if (VTF) {
    fld[0] = ad->psibar + (long long)(3 * alpha) * g.Np;
    fld[1] = fld[0] + g.Np;
    fld[2] = fld[1] + g.Np;
    fld[3] = a.Gfield + (long long)k * g.Np;
    fld[4] = ad->ut + (long long)(3 * beta) * g.Np;
    fld[5] = fld[4] + g.Np;
    fld[6] = fld[5] + g.Np;
    fld[7] = a.nfield + (long long)beta * g.Np;
  }
  if (VISC) {
    fld[2] = a.Jfield + (long long)(3 * beta) * g.Np;
    fld[3] = fld[2] + g.Np;
    fld[4] = fld[3] + g.Np;
  }
  if (ADJ) {
    fld[2] = ad->phibar + (long long)(3 * alpha) * g.Np;
    fld[3] = fld[2] + g.Np;
    fld[4] = fld[3] + g.Np;
  }
  if (AADJ) {
    fld[0] = ad->phibar + (long long)(3 * alpha) * g.Np;
    fld[1] = fld[0] + g.Np;
    fld[2] = fld[1] + g.Np;
  }
  const auto *ofs = cptr((ATT || AADJ ? a.t.att_ring_ofs : a.t.ring_ofs) + k * (RING_MAX + 2));
  const auto *roff = cptr(a.t.ring_off);
  const auto *re = cptr(a.t.ring_e);
  const double cmf = a.t.pair_cmf[k], cvs = a.t.pair_cvisc[k];
  const int base = (ty + R) * W + (tx + R);
  // this thread's window slots: in-plane padded offset, or -1 outside the box
  int soff[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int e = t + q * NT;
    const int c = e % W, r = e / W;
    const int X = x0 - R + c + g.R, Y = y0 - R + r + g.R;
    soff[q] = (e < WH && X < g.PX && Y < g.PY) ? X + g.PX * Y : -1;
  }
  // this pair's ring table ({e^, offset} per point; the ring offsets are
  // e_y*W_k + e_x for a window of FORCE_TX + 2R columns).  The point index is
  // the same in every lane.  With C^visc and in the adjoint (ten gathers per
  // pair), for the attraction and for any tile with two rows per thread, the
  // entries come in through scalar loads into SGPRs and cost no LDS bandwidth
  // (a broadcast LDS read of the 32-byte entry costs as much LDS return
  // bandwidth as four gathers of one field).  For C^mf alone with one row
  // (four gathers per pair) the wait on each scalar load is exposed, so the
  // table is staged once in LDS behind the plane buffers instead.  (C^mf
  // alone at 128^3, 32 x 16 tile with two rows: 0.297 ms with the LDS table,
  // 0.232 ms with scalar loads.)
  constexpr bool STAB = table_in_smem(MODE, NY);
  int rofs[R + 2];
#pragma unroll
  for (int ez = 0; ez <= R + 1; ++ez) rofs[ez] = ofs[ez];
  const int j0 = rofs[0];
  double *tab = lds + 2 * NF * WH;
  if (!STAB) {
    const int nent = rofs[R + 1] - rofs[0];
    for (int j = t; j < nent; j += NT) {
      tab[4 * j] = re[3 * (j0 + j)];
      tab[4 * j + 1] = re[3 * (j0 + j) + 1];
      tab[4 * j + 2] = re[3 * (j0 + j) + 2];
      tab[4 * j + 3] = __longlong_as_double((long long)roff[j0 + j]);
    }
  }
  const long long plane = (long long)g.PX * g.PY;
  const int zb = bz * a.zchunk;
  const int ze = zb + a.zchunk < g.nz ? zb + a.zchunk : g.nz;
  const int rounds = (ze - zb) * (R + 1);
  // planes of the next round, fetched while the current ring is computed:
  // [plane b][field f][slot q]
  double stage[2][NF][SLOTS];
  auto fetch = [&](int rho) {
    const int z = zb + rho / (R + 1), ez = rho % (R + 1);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long pz = (long long)((b ? z - ez : z + ez) + g.R) * plane;
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < SLOTS; ++q)
          stage[b][f][q] = (soff[q] >= 0 && (b == 0 || ez > 0)) ? fld[f][pz + soff[q]] : 0.0;
    }
  };
  fetch(0);
  // accumulators [row][set]: m (C^mf, or sum e^ n_b(r+e) for the adjoint)
  // and v (C^visc, or the two adjoint sums)
  double mx[NY][NS], my[NY][NS], mz[NY][NS], vx[NY][NS], vy[NY][NS], vz[NY][NS];
  double ox[NY][NS], oy[NY][NS], wx[NY][NS], wy[NY][NS], wz[NY][NS], we[NY][NS];  // MODE 5
  // centre values of each row: G_ab, and u_b (MODES 1, 6) or n_b and
  // phibar_a (MODE 2); phibar'_a and u~_b (MODE 5)
  double G0[NY], n0[NY], u0x[NY], u0y[NY], u0z[NY], p0x[NY], p0y[NY], p0z[NY];
  for (int rho = 0; rho < rounds; ++rho) {
    const int z = zb + rho / (R + 1), ez = rho % (R + 1);
    __syncthreads();  // previous round's readers are done with the buffers
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int e = t + q * NT;
        if (q < SLOTS - 1 || e < WH) {
          double *P = lds + b * NF * WH;
          if (PAIRED) {
            *reinterpret_cast<dbl2 *>(P + 2 * e) = dbl2{stage[b][0][q], stage[b][1][q]};
            if (NF == 5) {
              *reinterpret_cast<dbl2 *>(P + 2 * WH + 2 * e) = dbl2{stage[b][2 % NF][q], stage[b][3 % NF][q]};
              P[4 * WH + e] = stage[b][4 % NF][q];
            }
          } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) P[f * WH + e] = stage[b][f][q];
          }
        }
      }
    __syncthreads();
    if (rho + 1 < rounds) fetch(rho + 1);
    const double *Bp = lds;
    const double *Bm = ez ? lds + NF * WH : lds;
    if (ez == 0) {
#pragma unroll
      for (int jn = 0; jn < NY; ++jn) {
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          mx[jn][c] = my[jn][c] = mz[jn][c] = vx[jn][c] = vy[jn][c] = vz[jn][c] = 0.0;
          ox[jn][c] = oy[jn][c] = 0.0;
          wx[jn][c] = wy[jn][c] = wz[jn][c] = we[jn][c] = 0.0;
        }
        const int bj = base + jn * ROW;
        G0[jn] = ATT || AADJ ? 0.0 : (VTF ? Bp[3 * WH + bj] : Bp[at(1, bj)]);
        n0[jn] = AADJ ? 0.0 : (VTF ? Bp[7 * WH + bj] : Bp[at(0, bj)]);
        u0x[jn] = u0y[jn] = u0z[jn] = 0.0;
        p0x[jn] = p0y[jn] = p0z[jn] = 0.0;
        if (VTF) {  // phibar'_a and u~_b at the output node, staged
          p0x[jn] = Bp[bj];
          p0y[jn] = Bp[WH + bj];
          p0z[jn] = Bp[2 * WH + bj];
          u0x[jn] = Bp[4 * WH + bj];
          u0y[jn] = Bp[5 * WH + bj];
          u0z[jn] = Bp[6 * WH + bj];
        }
        if (VISC && n0[jn] != 0.0) {
          u0x[jn] = Bp[at(2, bj)] / n0[jn];
          u0y[jn] = Bp[at(3, bj)] / n0[jn];
          u0z[jn] = Bp[at(4, bj)] / n0[jn];
        }
        if (ADJ) {
          u0x[jn] = Bp[at(2, bj)];
          u0y[jn] = Bp[at(3, bj)];
          u0z[jn] = Bp[at(4, bj)];
        }
      }
    }
    const int jbeg = rofs[ez] - j0, jend = rofs[ez + 1] - j0;
    // C^mf + C^visc: the ten staged values of a pair for every row (n, G,
    // J~x, J~y, J~z at r + e and at r - e), and the pair's terms from them
    auto visc_load = [&](int o, double (&v)[NY][10]) {
#pragma unroll
      for (int jn = 0; jn < NY; ++jn) {
        const int qa = base + jn * ROW + o, qb = base + jn * ROW - o;
        v[jn][0] = Bp[qa];
        v[jn][1] = Bp[WH + qa];
        v[jn][2] = Bm[qb];
        v[jn][3] = Bm[WH + qb];
        v[jn][4] = Bp[2 * WH + qa];
        v[jn][5] = Bp[3 * WH + qa];
        v[jn][6] = Bm[2 * WH + qb];
        v[jn][7] = Bm[3 * WH + qb];
        v[jn][8] = Bp[4 * WH + qa];
        v[jn][9] = Bm[4 * WH + qb];
      }
    };
    auto visc_pair = [&](const double (&v)[NY][10], double e0, double e1, double e2, int c) {
#pragma unroll
      for (int jn = 0; jn < NY; ++jn) {
        const double npl = v[jn][0], nmi = v[jn][2];
        const double gp = G0[jn] + v[jn][1], gm = G0[jn] + v[jn][3];
        // two rounded products, then the difference (no fused multiply-add
        // across the pair), so that a uniform state gives exactly zero
        const double dp = gp * npl;
        const double dm = gm * nmi;
        const double d = dp - dm;
        mx[jn][c] += e0 * d;
        my[jn][c] += e1 * d;
        mz[jn][c] += e2 * d;
        // g(e.J~ - (e.u) n) at both points, with the products g n of the
        // C^mf term: (gp e.J~p + gm e.J~m) - (e.u)(dp + dm)
        const double eu = e0 * u0x[jn] + e1 * u0y[jn] + e2 * u0z[jn];
        const double ejp = e0 * v[jn][4] + e1 * v[jn][5] + e2 * v[jn][8];
        const double ejm = e0 * v[jn][6] + e1 * v[jn][7] + e2 * v[jn][9];
        const double tt = (gp * ejp + gm * ejm) - eu * (dp + dm);
        vx[jn][c] += e0 * tt;
        vy[jn][c] += e1 * tt;
        vz[jn][c] += e2 * tt;
      }
    };
    // one +-e pair for every row of the thread, into accumulator set c
    auto pair_at = [&](double e0, double e1, double e2, int o, int c) {
      if constexpr (VISC) {
        double v[NY][10];
        visc_load(o, v);
        visc_pair(v, e0, e1, e2, c);
      } else {
#pragma unroll
        for (int jn = 0; jn < NY; ++jn) {
          const int qa = base + jn * ROW + o, qb = base + jn * ROW - o;
          if constexpr (VTF) {
            // e^.phibar', e^.u~, G and n at r+e and r-e (the -e terms carry the
            // same signs: (-e^)(-e^.v) = e^(e^.v)); e^.J~ = n (e^.u~) there
            const double pp = e0 * Bp[qa] + e1 * Bp[WH + qa] + e2 * Bp[2 * WH + qa];
            const double pm = e0 * Bm[qb] + e1 * Bm[WH + qb] + e2 * Bm[2 * WH + qb];
            const double Gp = Bp[3 * WH + qa], Gm = Bm[3 * WH + qb];
            const double up = e0 * Bp[4 * WH + qa] + e1 * Bp[5 * WH + qa] + e2 * Bp[6 * WH + qa];
            const double um = e0 * Bm[4 * WH + qb] + e1 * Bm[5 * WH + qb] + e2 * Bm[6 * WH + qb];
            const double npl = Bp[7 * WH + qa], nmi = Bm[7 * WH + qb];
            const double s1 = pp + pm, s2 = pp * Gp + pm * Gm;
            mx[jn][c] += e0 * s1;
            my[jn][c] += e1 * s1;
            mz[jn][c] += e2 * s1;
            vx[jn][c] += e0 * s2;
            vy[jn][c] += e1 * s2;
            vz[jn][c] += e2 * s2;
            const double bp = pp * up, bm = pm * um;
            ox[jn][c] += bp + bm;
            oy[jn][c] += bp * Gp + bm * Gm;
            const double ep = e0 * p0x[jn] + e1 * p0y[jn] + e2 * p0z[jn];
            const double eu = e0 * u0x[jn] + e1 * u0y[jn] + e2 * u0z[jn];
            const double t1 = ep * (npl * (G0[jn] + Gp) + nmi * (G0[jn] + Gm));
            wx[jn][c] += e0 * t1;
            wy[jn][c] += e1 * t1;
            wz[jn][c] += e2 * t1;
            we[jn][c] += ep * (npl * (up - eu) + nmi * (um - eu));
            continue;
          }
          dbl2 ap, am, vp = {0.0, 0.0}, vm = {0.0, 0.0};
          double vpz = 0.0, vmz = 0.0;
          if (PAIRED) {
            ap = *reinterpret_cast<const dbl2 *>(Bp + 2 * qa);
            am = *reinterpret_cast<const dbl2 *>(Bm + 2 * qb);
            if (NF == 5) {
              vp = *reinterpret_cast<const dbl2 *>(Bp + 2 * WH + 2 * qa);
              vm = *reinterpret_cast<const dbl2 *>(Bm + 2 * WH + 2 * qb);
              vpz = Bp[4 * WH + qa];
              vmz = Bm[4 * WH + qb];
            }
          } else if (ATT) {
            ap = dbl2{Bp[qa], 0.0};
            am = dbl2{Bm[qb], 0.0};
          } else {  // AADJ
            ap = dbl2{Bp[qa], Bp[WH + qa]};
            am = dbl2{Bm[qb], Bm[WH + qb]};
            vpz = Bp[2 * WH + qa];
            vmz = Bm[2 * WH + qb];
          }
          const double npl = ap.x, nmi = am.x;
          if (AADJ) {
            // K(-e) = -K(e): the pair adds K.(phibar(r+e) - phibar(r-e))
            mx[jn][c] += e0 * (ap.x - am.x) + e1 * (ap.y - am.y) + e2 * (vpz - vmz);
          } else if (ATT) {
            // the table holds U'(|e|) e^; the pair adds K.(n_b(r+e) - n_b(r-e))
            const double dn = npl - nmi;
            mx[jn][c] += e0 * dn;
            my[jn][c] += e1 * dn;
            mz[jn][c] += e2 * dn;
          } else if (ADJ) {
            // m: sum_S e^ n_b(r+e); v: sum_S e^.phibar(r+e) and
            // sum_S (e^.phibar(r+e)) G(r+e), over both points of the pair
            const double tp = e0 * vp.x + e1 * vp.y + e2 * vpz;
            const double tm = e0 * vm.x + e1 * vm.y + e2 * vmz;
            const double dn = npl - nmi;
            mx[jn][c] += e0 * dn;
            my[jn][c] += e1 * dn;
            mz[jn][c] += e2 * dn;
            vx[jn][c] += tp - tm;
            vy[jn][c] += tp * ap.y - tm * am.y;
          } else {  // C^mf alone
            const double gp = G0[jn] + ap.y, gm = G0[jn] + am.y;
            // two rounded products, then the difference, as with C^visc
            const double dp = gp * npl;
            const double dm = gm * nmi;
            const double d = dp - dm;
            mx[jn][c] += e0 * d;
            my[jn][c] += e1 * d;
            mz[jn][c] += e2 * d;
          }
        }
      }
    };
    // table entry jj (scalar loads): unit vector and LDS offset of a pair
    auto entry = [&](int jj, double &e0, double &e1, double &e2, int &o) {
      e0 = re[3 * jj];
      e1 = re[3 * jj + 1];
      e2 = re[3 * jj + 2];
      o = roff[jj];
    };
    auto pair = [&](int j, int c) {
      double e0, e1, e2;
      int o;
      if (STAB) {
        entry(j0 + j, e0, e1, e2, o);
      } else {
        e0 = tab[4 * j];
        e1 = tab[4 * j + 1];
        e2 = tab[4 * j + 2];
        o = (int)__double_as_longlong(tab[4 * j + 3]);
      }
      pair_at(e0, e1, e2, o, c);
    };
    // a pair's terms are combined before they are accumulated, so a uniform
    // state still sums to exactly zero
    int j = jbeg;
    if constexpr (VISC) {
      // Pairs in groups of K, the K table entries first (scalar loads), then
      // the pairs, each one's LDS reads issued ahead of the previous pair's
      // arithmetic; pair c of a group goes to set c mod NS, as one at a time.
      // A scalar load shares its completion counter with the LDS reads and
      // may return out of order, so waiting for one waits for every read in
      // flight: with each entry loaded next to its pair, every pair waited
      // for all of its reads before any arithmetic.  Groups of eight and
      // four, pipelined: 128^3 step 1.328 -> 1.278 ms, the same sums bit
      // for bit.
      // (the 512-thread tile at reach 8 would spill; it loads each entry
      // next to its pair)
      constexpr bool PIPE = !(R >= 8 && NT >= 512);
      auto group = [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        if constexpr (PIPE) {
          double E0[K], E1[K], E2[K];
          int O[K];
#pragma unroll
          for (int c = 0; c < K; ++c) entry(j0 + j + c, E0[c], E1[c], E2[c], O[c]);
          double cur[NY][10], nxt[NY][10];
          visc_load(O[0], cur);
#pragma unroll
          for (int c = 0; c < K; ++c) {
            if (c + 1 < K) visc_load(O[c + 1], nxt);
            visc_pair(cur, E0[c], E1[c], E2[c], c % NS);
            if (c + 1 < K) {
#pragma unroll
              for (int jn = 0; jn < NY; ++jn)
#pragma unroll
                for (int q = 0; q < 10; ++q) cur[jn][q] = nxt[jn][q];
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < K; ++c) pair(j + c, c % NS);
        }
      };
      for (; j + 2 * NS - 1 < jend; j += 2 * NS) group(std::integral_constant<int, 2 * NS>{});
      for (; j + NS - 1 < jend; j += NS) group(std::integral_constant<int, NS>{});
    } else if constexpr (STAB && (ADJ || ATT || AADJ)) {
      // the same grouped table loads for the C^mf transpose and the
      // attraction gathers (channel adjoint backward 233 -> 227 ms; with the
      // attraction 577 -> 518 ms), and for the attraction also the reads
      // pipelined (128^3 step with the attraction 1.655 -> 1.611 ms).  The
      // C^visc transpose, already at 256 VGPRs, was slower with them (128^3
      // adjoint backward 125 -> 141 ms) and keeps the per-pair loads, as
      // does C^mf alone, not measured with them.
      auto group = [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        double E0[K], E1[K], E2[K];
        int O[K];
#pragma unroll
        for (int c = 0; c < K; ++c) entry(j0 + j + c, E0[c], E1[c], E2[c], O[c]);
        if constexpr (ATT) {
          // n_b at r + e and r - e for every row, the next pair's ahead of
          // this pair's arithmetic
          auto att_load = [&](int o, double (&v)[NY][2]) {
#pragma unroll
            for (int jn = 0; jn < NY; ++jn) {
              v[jn][0] = Bp[base + jn * ROW + o];
              v[jn][1] = Bm[base + jn * ROW - o];
            }
          };
          double cur[NY][2], nxt[NY][2];
          att_load(O[0], cur);
#pragma unroll
          for (int c = 0; c < K; ++c) {
            if (c + 1 < K) att_load(O[c + 1], nxt);
#pragma unroll
            for (int jn = 0; jn < NY; ++jn) {
              const double dn = cur[jn][0] - cur[jn][1];
              mx[jn][c % NS] += E0[c] * dn;
              my[jn][c % NS] += E1[c] * dn;
              mz[jn][c % NS] += E2[c] * dn;
            }
            if (c + 1 < K) {
#pragma unroll
              for (int jn = 0; jn < NY; ++jn) {
                cur[jn][0] = nxt[jn][0];
                cur[jn][1] = nxt[jn][1];
              }
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < K; ++c) pair_at(E0[c], E1[c], E2[c], O[c], c % NS);
        }
      };
      for (; j + 2 * NS - 1 < jend; j += 2 * NS) group(std::integral_constant<int, 2 * NS>{});
      for (; j + NS - 1 < jend; j += NS) group(std::integral_constant<int, NS>{});
    } else {
      for (; j + NS - 1 < jend; j += NS) {
#pragma unroll
        for (int c = 0; c < NS; ++c) pair(j + c, c);
      }
    }
    for (int c = 0; j < jend; ++j, ++c) pair(j, c);
    if (ez == R) {
      const long long N = g.N;
#pragma unroll
      for (int jn = 0; jn < NY; ++jn) {
        const int y = y0 + ty + jn * RY;
        if (!(x < g.nx && y < g.ny)) continue;
        // the sets summed in order
        auto sets = [&](const double (&v)[NY][NS]) {
          double r = v[jn][0];
#pragma unroll
          for (int c = 1; c < NS; ++c) r += v[jn][c];
          return r;
        };
        const double Mx = sets(mx), My = sets(my), Mz = sets(mz);
        const double Vx = sets(vx), Vy = sets(vy), Vz = sets(vz);
        const long long i = x + (long long)g.nx * (y + (long long)g.ny * z);
        if (ADJ) {
          // n_b^bar(r) += -c (sum (e^.phibar) G(r+e) + G(r) sum e^.phibar)
          // G_ab^bar(r) += c (phibar(r).sum e^ n_b(r+e) - n_b(r) sum e^.phibar)
          const double vn = -cmf * (Vy + G0[jn] * Vx);
          const double vg = cmf * (u0x[jn] * Mx + u0y[jn] * My + u0z[jn] * Mz - n0[jn] * Vx);
          double *pn = ad->nbar + beta * N + i, *pg = ad->Gbar + k * N + i;
          *pn = (accumulate & 1) ? *pn + vn : vn;
          *pg = (accumulate & 2) ? *pg + vg : vg;
        } else if (AADJ) {
          double *pn = ad->nbar + beta * N + i;
          *pn = (accumulate & 1) ? *pn - Mx : -Mx;
        } else if (VTF) {
          // with c = pair_cvisc (C^visc/n_a = c sum_S e^ [e^.J~(r+e) -
          // (e^.u~(r)) n_b(r+e)] (G(r) + G(r+e))) and pb = phibar'_a:
          //   J~_b^bar(r) += c (sum e^(e^.pb(r+e)) G(r+e) + G(r) sum e^(e^.pb(r+e)))
          //   n_b^bar(r)  -= c (sum (e^.pb)(e^.u~)(r+e) G(r+e) + G(r) sum (e^.pb)(e^.u~)(r+e))
          //   G^bar(r)    += c (J~_b(r).sum e^(e^.pb(r+e)) - n_b(r) sum (e^.pb)(e^.u~)(r+e))
          // from the neighbours' terms, and from the node's own u~_b(r) and G(r):
          //   u~^bar(r) = -c sum e^(e^.pb(r)) n_b(r+e)(G(r) + G(r+e)), into
          //     J~_b^bar += u~^bar/n_b, n_b^bar -= u~^bar.u~/n_b,
          //   G^bar(r) += c sum (e^.pb(r)) (e^.J~(r+e) - (e^.u~(r)) n_b(r+e))
          const double Ox = sets(ox), Oy = sets(oy);
          const double Wx = sets(wx), Wy = sets(wy), Wz = sets(wz);
          const double We = sets(we);
          const long long Pc = (x + g.R) + (long long)g.PX * ((y + g.R) + (long long)g.PY * (z + g.R));
          const double *Jc = a.Jfield + (long long)(3 * beta) * g.Np + Pc;
          const double inv = n0[jn] != 0.0 ? 1.0 / n0[jn] : 0.0;
          const double ub0 = -cvs * Wx, ub1 = -cvs * Wy, ub2 = -cvs * Wz;
          double jb[3];
          jb[0] = cvs * (Vx + G0[jn] * Mx) + ub0 * inv;
          jb[1] = cvs * (Vy + G0[jn] * My) + ub1 * inv;
          jb[2] = cvs * (Vz + G0[jn] * Mz) + ub2 * inv;
          const double vn = -cvs * (Oy + G0[jn] * Ox) - (ub0 * u0x[jn] + ub1 * u0y[jn] + ub2 * u0z[jn]) * inv;
          const double vg = cvs * (Jc[0] * Mx + Jc[g.Np] * My + Jc[2 * g.Np] * Mz - n0[jn] * Ox + We);
          double *pn = ad->nbar + beta * N + i, *pg = ad->Gbar + k * N + i, *pj = ad->Jnl + 3 * beta * N + i;
          *pn = (accumulate & 1) ? *pn + vn : vn;
          *pg = (accumulate & 2) ? *pg + vg : vg;
          for (int q = 0; q < 3; ++q) pj[q * N] = (accumulate & 4) ? pj[q * N] + jb[q] : jb[q];
        } else if (ATT) {
          // G^{ab} is a force per particle of species a: into C^mf/n_a
          double *F = a.force + 6LL * alpha * N + i;
          if (accumulate) {
            F[0] += Mx;
            F[N] += My;
            F[2 * N] += Mz;
          } else {
            F[0] = Mx;
            F[N] = My;
            F[2 * N] = Mz;
            F[3 * N] = 0.0;
            F[4 * N] = 0.0;
            F[5 * N] = 0.0;
          }
        } else {
          double *F = a.force + 6LL * alpha * N + i;
          if (accumulate) {
            F[0] += cmf * Mx;
            F[N] += cmf * My;
            F[2 * N] += cmf * Mz;
            F[3 * N] += cvs * Vx;
            F[4 * N] += cvs * Vy;
            F[5 * N] += cvs * Vz;
          } else {
            F[0] = cmf * Mx;
            F[N] = cmf * My;
            F[2 * N] = cmf * Mz;
            F[3 * N] = cvs * Vx;
            F[4 * N] = cvs * Vy;
            F[5 * N] = cvs * Vz;
          }
        }
      }
    }
  }
}

// The tile (bx, by, bz) of this workgroup.  Workgroups are handed to the 8
// XCDs round-robin (workgroup b to XCD b mod 8), each with its own L2; with
// order 1 or 2 the tiles are renumbered so that each XCD gets one
// contiguous range of tiles (x fastest, or z fastest), which keeps the
// halo planes that neighbouring tiles share in one L2.
constexpr int NXCD = 8;

struct Tile {
  int bx, by, bz;
};

__device__ inline Tile force_tile(const Geom &g, int zchunk, int order, int ty) {
  const int nbx = (g.nx + FTX - 1) / FTX, nby = (g.ny + ty - 1) / ty;
  const int nbz = (g.nz + zchunk - 1) / zchunk;
  const int b = blockIdx.x;
  const int nb = nbx * nby * nbz, q = nb / NXCD, r = nb % NXCD;
  const int k = b % NXCD, j = b / NXCD;
  const int t = order == 0 ? b : (k < r ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j);
  Tile T;
  if (order == 2) {
    T.bz = t % nbz;
    T.bx = (t / nbz) % nbx;
    T.by = t / (nbz * nbx);
  } else {
    T.bx = t % nbx;
    T.by = (t / nbx) % nby;
    T.bz = t / (nbx * nby);
  }
  return T;
}

template <int R, bool VISC, int NY, int NT>
__global__ __launch_bounds__(NT) void k_force(StepArgs a, int alpha, int beta, int accumulate) {
  extern __shared__ double lds[];
  const Tile T = force_tile(a.g, a.zchunk, a.order, NT / FTX * NY);
  force_body<R, VISC ? 1 : 0, NY, NT>(a, nullptr, alpha, beta, accumulate, T.bx, T.by, T.bz, lds);
}

// the attractive field of the directed pair (alpha, beta), added to C^mf/n_alpha.
// Two gathers per pair and row: the table entry comes through scalar loads
// (no LDS traffic), and two output rows per thread (a 32 x 16 tile) give each
// entry four gathers to hide its load behind.  At 128^3 with 604 pairs per
// node: 0.755 ms with an LDS table and one row, 0.59 ms with two rows, 0.35 ms
// with two rows and scalar loads.  A box that gives fewer than two such
// tiles per CU takes one row per thread (a 32 x 8 tile, twice the
// workgroups): on the 96 x 32 x 32 channel, 192 workgroups of 32 x 16 leave a
// quarter of the 256 CUs idle, and the 32 x 8 tile makes the four gathers
// 0.58 -> 0.53 ms; at 128^3 the 32 x 16 tile stays faster (1.15 against
// 1.32 ms).  Both give the same sums bit for bit.
template <int R, int NY>
__global__ __launch_bounds__(FNT) void k_force_att(StepArgs a, int alpha, int beta, int accumulate) {
  extern __shared__ double lds[];
  const Tile T = force_tile(a.g, a.zchunk, a.order, FNT / FTX * NY);
  force_body<R, 3, NY, FNT>(a, nullptr, alpha, beta, accumulate, T.bx, T.by, T.bz, lds);
}

// output rows per thread of the attraction gathers (forward and transpose)
constexpr int NCU = 256;
static int att_rows(const StepArgs &a) {
  return force_blocks(a.g, a.zchunk, FNT / FTX * 2) < 2 * NCU ? 1 : 2;
}

// per-particle forces of species s at node i, times n_s
template <int M, class A>
__device__ inline void load_forces(const A &a, int i, const Coord &c, const double n[M],
                                   double cmf[M][3], double cvisc[M][3]) {
  const long long N = a.g.N;
  for (int s = 0; s < M; ++s) {
    const double *F = a.force + 6LL * s * N + i;
    for (int k = 0; k < 3; ++k) {
      cmf[s][k] = n[s] * F[k * N];
      cvisc[s][k] = n[s] * F[(3 + k) * N];
    }
  }
  // interspecies drag (Appendix, eq. dragforce2), local, with the same
  // velocities u~ = J~/n as C^visc: C^drag_a = -n_a sum_b gamma_ab G_ab
  // n_b (u~_a - u~_b), added to the dissipative forces
  if (M > 1 && (a.flags & LBE_DRAG) && !(a.flags & LBE_IDEAL)) {
    const Geom g = geom_of(a);
    const long long P = padded_index(g, c.x, c.y, c.z);
    double u[M][3];
    for (int b = 0; b < M; ++b)
      for (int k = 0; k < 3; ++k)
        u[b][k] = n[b] != 0.0 ? a.Jfield[(long long)(3 * b + k) * g.Np + P] / n[b] : 0.0;
    for (int s = 0; s < M; ++s)
      for (int b = 0; b < M; ++b) {
        if (b == s) continue;
        const int k = pair_index(M, s, b);
        const double coef = -n[s] * a.t.pair_drag[k] * a.Gfield[(long long)k * g.Np + P] * n[b];
        for (int d = 0; d < 3; ++d) cvisc[s][d] += coef * (u[s][d] - u[b][d]);
      }
  }
}

// Inversions, equilibria, sources and the trapezoidal update of one node.
//  J = J~ + Y/2 (or + X/2 printed), u^a = J/n,
//  Pi = Pi~ + (beta/2) C^mf.u^a (or - printed), u = sum J / sum n,
//  (Euler: J = J~, Pi = Pi~; single distribution: J~ from f, J = J~ + X/2)
//  f_eq = w [n + 3 c.J + 4.5 n (2 (c.u^a)(c.u) - (c.u)^2) - 1.5 n (2 u^a.u - u.u)]
//  g_eq = f_eq + w (Pi - n)
//  S_f  = w [3 c.X + 9 (c.X)(c.u^a) - 3 X.u^a]
//  S_g  = w [4.5 kappa (c.C)(c.u^a) + (3 - 1.5 kappa) C.u^a
//            + 3 c.Y + 9 (c.Y)(c.u^a) - 3 Y.u^a]
//  out  = (1 - a) in + a eq + b S
template <int M>
struct NodeMoments {
  double n[M], Pi[M], J[M][3], ua[M][3], X[M][3], Y[M][3];
  double u[3];
  double dPit[M];   // shift of the zeroth moment of g~ (per-step quasi-pressure)
};

template <int M, class A>
__device__ inline void invert(const A &a, const double ft[M][19], const double gt[M][19],
                              const double cmf[M][3], const double cvisc[M][3], int i,
                              NodeMoments<M> &nm) {
  const bool printed = a.flags & LBE_PRINTED_INV;
  const bool euler = a.flags & LBE_EULER, single = a.flags & LBE_SINGLE;
  double ntot = 0.0, Jt0 = 0.0, Jt1 = 0.0, Jt2 = 0.0;
  for (int s = 0; s < M; ++s) {
    double n, Pit, Jt[3];
    moments0(ft[s], n);
    moments0(gt[s], Pit);
    moments1(gt[s], Jt);
    double cu = 0.0;
    for (int k = 0; k < 3; ++k) {
      double F = a.Fext[(long long)k * a.g.N + i] + a.body[s][k];
      double nF = n * F;
      nm.X[s][k] = cmf[s][k] + cvisc[s][k] + nF;
      nm.Y[s][k] = cvisc[s][k] + nF;
      // EU: no half-step term; SD: the f inversion with X
      nm.J[s][k] = euler ? Jt[k] : Jt[k] + 0.5 * ((printed || single) ? nm.X[s][k] : nm.Y[s][k]);
      nm.ua[s][k] = n != 0.0 ? nm.J[s][k] / n : 0.0;
      cu += cmf[s][k] * nm.ua[s][k];
    }
    nm.n[s] = n;
    nm.Pi[s] = (euler || single) ? Pit : (printed ? Pit - 0.5 * a.beta * cu : Pit + 0.5 * a.beta * cu);
    nm.dPit[s] = 0.0;
    if (a.pifield && !single) {
      // the per-step quasi-pressure Pi = n - beta Phi (this node's n): g_eq
      // takes Pi, and g~'s zeroth moment becomes the Pi~ that the inversion
      // maps to it
      const double pi = n - a.beta * a.pifield[(long long)s * a.g.N + i];
      const double target = euler ? pi : (printed ? pi + 0.5 * a.beta * cu : pi - 0.5 * a.beta * cu);
      nm.Pi[s] = pi;
      nm.dPit[s] = target - Pit;
    }
    ntot += n;
    Jt0 += nm.J[s][0];
    Jt1 += nm.J[s][1];
    Jt2 += nm.J[s][2];
  }
  nm.u[0] = ntot != 0.0 ? Jt0 / ntot : 0.0;
  nm.u[1] = ntot != 0.0 ? Jt1 / ntot : 0.0;
  nm.u[2] = ntot != 0.0 ? Jt2 / ntot : 0.0;
}

template <int p>
__device__ inline double cdot(const double v[3]) {
  double r = 0.0;
  if (cvec(p, 0) > 0) r += v[0];
  if (cvec(p, 0) < 0) r -= v[0];
  if (cvec(p, 1) > 0) r += v[1];
  if (cvec(p, 1) < 0) r -= v[1];
  if (cvec(p, 2) > 0) r += v[2];
  if (cvec(p, 2) < 0) r -= v[2];
  return r;
}

template <int p>
struct CollideP {
  template <typename T, int M, class A>
  __device__ static inline void run(const A &a, int s, const NodeMoments<M> &nm,
                                    const double cm[3], const double ft, const double gt_in,
                                    T *__restrict__ fo, T *__restrict__ go) {
    const double w = wgt(p);
    const double gt = gt_in + w * nm.dPit[s];
    const double n = nm.n[s];
    const double cJ = cdot<p>(nm.J[s]);
    const double cua = cdot<p>(nm.ua[s]);
    const double cu = cdot<p>(nm.u);
    const double uau = nm.ua[s][0] * nm.u[0] + nm.ua[s][1] * nm.u[1] + nm.ua[s][2] * nm.u[2];
    const double uu = nm.u[0] * nm.u[0] + nm.u[1] * nm.u[1] + nm.u[2] * nm.u[2];
    const double feq = w * (n + 3.0 * cJ + 4.5 * n * (2.0 * cua * cu - cu * cu) -
                            1.5 * n * (2.0 * uau - uu));
    const double geq = feq + w * (nm.Pi[s] - n);
    const double cX = cdot<p>(nm.X[s]);
    const double Xua = nm.X[s][0] * nm.ua[s][0] + nm.X[s][1] * nm.ua[s][1] + nm.X[s][2] * nm.ua[s][2];
    const double cY = cdot<p>(nm.Y[s]);
    const double Yua = nm.Y[s][0] * nm.ua[s][0] + nm.Y[s][1] * nm.ua[s][1] + nm.Y[s][2] * nm.ua[s][2];
    const double cC = cdot<p>(cm);
    const double Cua = cm[0] * nm.ua[s][0] + cm[1] * nm.ua[s][1] + cm[2] * nm.ua[s][2];
    const double Sf = w * (3.0 * cX + 9.0 * cX * cua - 3.0 * Xua);
    const double Sg = w * (4.5 * a.kappa * cC * cua + (3.0 - 1.5 * a.kappa) * Cua + 3.0 * cY +
                           9.0 * cY * cua - 3.0 * Yua);
    __builtin_nontemporal_store(T(ft + a.acoef * (feq - ft) + a.bcoef * Sf), fo);
    if (go) __builtin_nontemporal_store(T(gt + a.acoef * (geq - gt) + a.bcoef * Sg), go);
  }
};

template <typename T, int M, int p, class A>
__device__ inline void collide_all_p(const A &a, int s, const NodeMoments<M> &nm,
                                     const double cm[3], const double ft[19], const double gt[19],
                                     T *__restrict__ fblk, T *__restrict__ gblk, long long Ns, int i) {
  if constexpr (p < Q) {
    CollideP<p>::template run<T, M, A>(a, s, nm, cm, ft[p], gt[p], fblk + (long long)p * Ns + i,
                                    gblk ? gblk + (long long)p * Ns + i : nullptr);
    collide_all_p<T, M, p + 1, A>(a, s, nm, cm, ft, gt, fblk, gblk, Ns, i);
  }
}

template <typename T, int M, class A>
__device__ inline void collide_body(const A &a, const T *__restrict__ pin, T *__restrict__ pout,
                                    int i) {
  const Geom g = geom_of(a);
  if (i >= g.N) return;
  uint32_t m = a.bb[i];
  if (m & 1u) return;  // solid slots are never read
  Coord c = decode(g, i);
  long long Ns = pop_stride(g);
  const bool single = a.flags & LBE_SINGLE;
  double ft[M][19], gt[M][19], n[M];
  for (int s = 0; s < M; ++s) {
    pull19(g, c, i, m, pin + (long long)s * Q * Ns, Ns, ft[s]);
    if (!single) pull19(g, c, i, m, pin + (long long)(M + s) * Q * Ns, Ns, gt[s]);
    moments0(ft[s], n[s]);
  }
  double cmf[M][3], cvisc[M][3];
  load_forces<M>(a, i, c, n, cmf, cvisc);
  NodeMoments<M> nm;
  invert<M>(a, ft, single ? ft : gt, cmf, cvisc, i, nm);
  for (int s = 0; s < M; ++s)
    collide_all_p<T, M, 0>(a, s, nm, cmf[s], ft[s], single ? ft[s] : gt[s], pout + (long long)s * Q * Ns,
                           single ? nullptr : pout + (long long)(M + s) * Q * Ns, Ns, i);
}

template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void k_collide(StepArgs a, const T *__restrict__ pin,
                                                   T *__restrict__ pout) {
  collide_body<T, M>(a, pin, pout, blockIdx.x * BLOCK + threadIdx.x);
}

// ------------------------------------------------------------------------
// batched kernels: one launch covers every box of a batch.  Each block looks
// up its box in a block -> box table and reads that box's parameter block
// through scalar loads; the per-box bodies are the single-box ones.
// ------------------------------------------------------------------------
template <typename T, bool VISC>
__global__ __launch_bounds__(BLOCK) void kb_moments(BatchArgs ba) {
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const int i = (blockIdx.x - cptr(ba.blockstart)[b]) * BLOCK + threadIdx.x;
  moments_body<T, VISC>(a, (const T *)a.pop[ba.cur], i);
}

// boxes of M species and one ball z depth ZC; blockbox/blockstart index
// ball tiles here
template <int M, int ZC>
__global__ __launch_bounds__(BLOCK) void kb_ball(BatchArgs ba) {
  extern __shared__ double lds[];
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const AdjArgs none{};
  ball_body<M, 0, ZC>(a, none, blockIdx.x - cptr(ba.blockstart)[b], lds);
}

// the shell gather of the directed pair (alpha, beta) for every box of one
// shell reach R and tile shape SHAPE (each box's own tuned shape); acc: add
// to the force of species alpha (later pairs)
template <int R, bool VISC, int SHAPE>
__global__ __launch_bounds__(shape_nt(SHAPE)) void kb_force(BatchArgs ba, int alpha, int beta, int acc) {
  extern __shared__ double lds[];
  constexpr int TY = shape_ty(SHAPE);
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const int local = blockIdx.x - cptr(ba.blockstart)[b];
  const int nbx = (a.g.nx + FTX - 1) / FTX, nby = (a.g.ny + TY - 1) / TY;
  force_body<R, VISC ? 1 : 0, shape_ny(SHAPE), shape_nt(SHAPE)>(a, nullptr, alpha, beta, acc, local % nbx,
                                                                (local / nbx) % nby, local / (nbx * nby), lds);
}

// the attractive field of the directed pair (alpha, beta) for every box of
// one tail reach R, added to C^mf/n_alpha after the hard-sphere gathers;
// 32 x 8 tiles
template <int R>
__global__ __launch_bounds__(FNT) void kb_force_att(BatchArgs ba, int alpha, int beta) {
  extern __shared__ double lds[];
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const int local = blockIdx.x - cptr(ba.blockstart)[b];
  const int nbx = (a.g.nx + FTX - 1) / FTX, nby = (a.g.ny + FTY - 1) / FTY;
  force_body<R, 3, 1, FNT>(a, nullptr, alpha, beta, 1, local % nbx, (local / nbx) % nby,
                           local / (nbx * nby), lds);
}

template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void kb_collide(BatchArgs ba) {
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const int i = (blockIdx.x - cptr(ba.blockstart)[b]) * BLOCK + threadIdx.x;
  collide_body<T, M>(a, (const T *)a.pop[ba.cur], (T *)a.pop[ba.cur ^ 1], i);
}

template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void k_readout(StepArgs a, const T *__restrict__ pin, Readout r) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const Geom g = geom_of(a);
  if (i >= g.N) return;
  uint32_t m = a.bb[i];
  const int N = g.N;
  if (m & 1u) {
    for (int s = 0; s < M; ++s) {
      r.n[(long long)s * N + i] = 0.0;
      for (int k = 0; k < 3; ++k) {
        r.ua[(long long)(3 * s + k) * N + i] = 0.0;
        r.cmf[(long long)(3 * s + k) * N + i] = 0.0;
        r.cvisc[(long long)(3 * s + k) * N + i] = 0.0;
        r.ja[(long long)(3 * s + k) * N + i] = 0.0;
      }
    }
    for (int k = 0; k < 3; ++k) {
      r.u[(long long)k * N + i] = 0.0;
      r.jt[(long long)k * N + i] = 0.0;
      r.j[(long long)k * N + i] = 0.0;
    }
    return;
  }
  Coord c = decode(g, i);
  long long Ns = pop_stride(g);
  const bool single = a.flags & LBE_SINGLE;
  double ft[M][19], gt[M][19], n[M];
  for (int s = 0; s < M; ++s) {
    pull19(g, c, i, m, pin + (long long)s * Q * Ns, Ns, ft[s]);
    if (!single) pull19(g, c, i, m, pin + (long long)(M + s) * Q * Ns, Ns, gt[s]);
    moments0(ft[s], n[s]);
  }
  double cmf[M][3], cvisc[M][3];
  load_forces<M>(a, i, c, n, cmf, cvisc);
  NodeMoments<M> nm;
  invert<M>(a, ft, single ? ft : gt, cmf, cvisc, i, nm);
  double jt[3] = {0.0, 0.0, 0.0}, js[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < M; ++s) {
    double J1[3];
    moments1(single ? ft[s] : gt[s], J1);
    r.n[(long long)s * N + i] = nm.n[s];
    for (int k = 0; k < 3; ++k) {
      r.ua[(long long)(3 * s + k) * N + i] = nm.ua[s][k];
      r.cmf[(long long)(3 * s + k) * N + i] = cmf[s][k];
      r.cvisc[(long long)(3 * s + k) * N + i] = cvisc[s][k];
      r.ja[(long long)(3 * s + k) * N + i] = nm.J[s][k];
      jt[k] += J1[k];
      js[k] += nm.J[s][k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    r.u[(long long)k * N + i] = nm.u[k];
    r.jt[(long long)k * N + i] = jt[k];
    r.j[(long long)k * N + i] = js[k];
  }
}

// ------------------------------------------------------------------------
// diagnostics: per-block partial results, then one block combines them in
// block order (deterministic).  Quantities: mass[4], Jt[3], Z = sum e^{-beta V},
// umax, jmax, nfluid, spare.
// ------------------------------------------------------------------------
__device__ inline double block_sum(double v, double *sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double *sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = fmax(sh[t], sh[t + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(BLOCK) void k_diag_partials(Geom g, int M, const uint32_t *__restrict__ bb,
                                                        Readout r, const double *__restrict__ V,
                                                        double beta, double *__restrict__ partials) {
  __shared__ double sh[BLOCK];
  double acc[DIAG_K];
  for (int k = 0; k < DIAG_K; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < g.N; i += gridDim.x * BLOCK) {
    if (bb[i] & 1u) continue;
    for (int s = 0; s < M; ++s) acc[s] += r.n[(long long)s * g.N + i];
    double uu = 0.0, jj = 0.0;
    for (int k = 0; k < 3; ++k) {
      acc[4 + k] += r.jt[(long long)k * g.N + i];
      double u = r.u[(long long)k * g.N + i], j = r.j[(long long)k * g.N + i];
      uu += u * u;
      jj += j * j;
    }
    acc[7] += exp(-beta * V[i]);
    acc[8] = fmax(acc[8], sqrt(uu));
    acc[9] = fmax(acc[9], sqrt(jj));
    acc[10] += 1.0;
  }
  for (int k = 0; k < DIAG_K; ++k) {
    double v = (k == 8 || k == 9) ? block_max(acc[k], sh) : block_sum(acc[k], sh);
    if (threadIdx.x == 0) partials[(long long)blockIdx.x * DIAG_K + k] = v;
  }
}

// one wave: lane l combines the partials of blocks l, l + 64, ... in order,
// then a fixed shuffle tree combines the 64 lanes (the same order on every
// call, so the result is deterministic)
__global__ __launch_bounds__(64) void k_diag_final(const double *__restrict__ partials, int nblocks,
                                                   double *__restrict__ result) {
  const int l = threadIdx.x;
  for (int k = 0; k < DIAG_K; ++k) {
    const bool mx = k == 8 || k == 9 || k == 11;
    double a = 0.0;
    for (int b = l; b < nblocks; b += 64) {
      const double v = partials[(long long)b * DIAG_K + k];
      a = mx ? fmax(a, v) : a + v;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(a, off, 64);
      a = mx ? fmax(a, o) : a + o;
    }
    if (l == 0) result[k] = a;
  }
}

// second pass: max |n_tot - n_eq| with n_eq = mass e^{-beta V} / Z
__global__ __launch_bounds__(BLOCK) void k_diag_errn(Geom g, int M, const uint32_t *__restrict__ bb,
                                                    Readout r, const double *__restrict__ V,
                                                    double beta, const double *__restrict__ res,
                                                    double *__restrict__ partials) {
  __shared__ double sh[BLOCK];
  double mtot = 0.0;
  for (int s = 0; s < M; ++s) mtot += res[s];
  double Z = res[7];
  double e = 0.0;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < g.N; i += gridDim.x * BLOCK) {
    if (bb[i] & 1u) continue;
    double nt = 0.0;
    for (int s = 0; s < M; ++s) nt += r.n[(long long)s * g.N + i];
    double neq = mtot * exp(-beta * V[i]) / Z;
    e = fmax(e, fabs(nt - neq));
  }
  double v = block_max(e, sh);
  if (threadIdx.x == 0) partials[(long long)blockIdx.x * DIAG_K + 11] = v;
}

inline dim3 grid_for(int N) { return dim3((N + BLOCK - 1) / BLOCK); }

// ------------------------------------------------------------------------
// adjoint (reverse mode) of one step, for FP64 populations: C^mf, with or
// without C^visc, the interspecies drag and the attractive field;
// trapezoidal or Euler, two distributions or one.  "bar" marks the adjoint
// dL/d(quantity).  The adjoint state between steps is (mu, nbar) in the
// post-streaming frame (AdjArgs).
// ------------------------------------------------------------------------

// adjoint of the pre-streaming slot (r, q): the streaming map is a
// permutation, so it is the adjoint of the one population that reads the
// slot -- (r + c_q, q), or (r, opp q) when r + c_q is blocked
template <int q>
__device__ inline double adj_slot(const Geom &g, const Coord &c, int i, uint32_t m,
                                  const double *__restrict__ blk, long long Ns) {
  if (q == 0) return blk[i];
  if ((m >> opp(q)) & 1u) return blk[(long long)opp(q) * Ns + i];
  return blk[(long long)q * Ns + downstream(g, c, q)];
}

// sum_q w_q v_q, sum_q w_q c_q v_q, sum_q w_q c_q c_q v_q (xx yy zz xy xz yz)
struct WMoments {
  double m0, m1[3], m2[6];
};

template <int q>
__device__ inline void wacc(WMoments &b, double v) {
  constexpr int cx = cvec(q, 0), cy = cvec(q, 1), cz = cvec(q, 2);
  const double wv = wgt(q) * v;
  b.m0 += wv;
  if (cx) b.m1[0] += cx * wv;
  if (cy) b.m1[1] += cy * wv;
  if (cz) b.m1[2] += cz * wv;
  if (cx) b.m2[0] += wv;
  if (cy) b.m2[1] += wv;
  if (cz) b.m2[2] += wv;
  if (cx && cy) b.m2[3] += cx * cy * wv;
  if (cx && cz) b.m2[4] += cx * cz * wv;
  if (cy && cz) b.m2[5] += cy * cz * wv;
}

__device__ inline void wzero(WMoments &b) {
  b.m0 = 0.0;
  for (int k = 0; k < 3; ++k) b.m1[k] = 0.0;
  for (int k = 0; k < 6; ++k) b.m2[k] = 0.0;
}

// symmetric 3x3 (xx yy zz xy xz yz) times a vector
__device__ inline void symv(const double m[6], const double v[3], double o[3]) {
  o[0] = m[0] * v[0] + m[3] * v[1] + m[4] * v[2];
  o[1] = m[3] * v[0] + m[1] * v[1] + m[5] * v[2];
  o[2] = m[4] * v[0] + m[5] * v[1] + m[2] * v[2];
}

__device__ inline double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <int q, int M>
__device__ inline void adj_moments_all(const Geom &g, const Coord &c, int i, uint32_t m,
                                       const AdjArgs &d, long long Ns, WMoments bf[M], WMoments bg[M]) {
  if constexpr (q < Q) {
    for (int s = 0; s < M; ++s) {
      wacc<q>(bf[s], adj_slot<q>(g, c, i, m, d.mu_in + (long long)s * Q * Ns, Ns));
      wacc<q>(bg[s], adj_slot<q>(g, c, i, m, d.mu_in + (long long)(M + s) * Q * Ns, Ns));
    }
    adj_moments_all<q + 1, M>(g, c, i, m, d, Ns, bf, bg);
  }
}

// node adjoints of species s: nbar (local part), Pi~bar, J~bar
__device__ inline void store_node(const AdjArgs &d, int M, long long N, int i, int s, double nb,
                                  double Pib, const double Jb[3]) {
  d.node[(long long)s * N + i] = nb;
  d.node[(long long)(M + s) * N + i] = Pib;
  for (int k = 0; k < 3; ++k) d.node[(long long)(2 * M + 3 * s + k) * N + i] = Jb[k];
}

__device__ inline void store_phibar(const Geom &g, const AdjArgs &d, const Coord &c, int s,
                                    const double v[3]) {
  for (int k = 0; k < 3; ++k) store_images(g, d.phibar + (long long)(3 * s + k) * g.Np, c, v[k]);
}

// the interspecies drag is on (see load_forces)
template <class A>
__device__ inline bool drag_on(const A &a) {
  return a.M > 1 && (a.flags & LBE_DRAG) && !(a.flags & LBE_IDEAL);
}

// u~ = J~/n of every species at node i from the tape's tilde moments
template <int M>
__device__ inline void tape_ut(const AdjArgs &d, long long N, int i, const double n[M], double ut[M][3]) {
  for (int s = 0; s < M; ++s)
    for (int k = 0; k < 3; ++k) ut[s][k] = n[s] != 0.0 ? d.PJ[(long long)(M + 3 * s + k) * N + i] / n[s] : 0.0;
}

// the drag force of every species at node P / i, as load_forces adds it
template <int M, class A>
__device__ inline void drag_force(const A &a, long long P, const double n[M], const double ut[M][3],
                                  double D[M][3]) {
  const long long Np = a.g.Np;
  for (int s = 0; s < M; ++s) {
    for (int k = 0; k < 3; ++k) D[s][k] = 0.0;
    for (int b = 0; b < M; ++b) {
      if (b == s) continue;
      const int k = pair_index(M, s, b);
      const double coef = -n[s] * a.t.pair_drag[k] * a.Gfield[(long long)k * Np + P] * n[b];
      for (int x = 0; x < 3; ++x) D[s][x] += coef * (ut[s][x] - ut[b][x]);
    }
  }
}

// Reverse of the drag C^drag_s = -n_s sum_b gamma_sb G_sb n_b (u~_s - u~_b),
// u~ = J~/n, given Db = dL/dC^drag: adds to nbar and J~bar and writes Gbar
// of every pair at node i (the shell and ball transposes accumulate on it).
template <int M, class A>
__device__ inline void adj_drag(const A &a, const AdjArgs &d, long long P, int i, const double n[M],
                                const double ut[M][3], const double Db[M][3], double nbar[M],
                                double Jbar[M][3]) {
  const long long N = a.g.N, Np = a.g.Np;
  double utb[M][3], Gb[M * (M + 1) / 2];
  for (int k = 0; k < M * (M + 1) / 2; ++k) Gb[k] = 0.0;
  for (int s = 0; s < M; ++s)
    for (int k = 0; k < 3; ++k) utb[s][k] = 0.0;
  for (int s = 0; s < M; ++s)
    for (int b = 0; b < M; ++b) {
      if (b == s) continue;
      const int k = pair_index(M, s, b);
      const double gam = a.t.pair_drag[k], G = a.Gfield[(long long)k * Np + P];
      const double coef = -n[s] * gam * G * n[b];
      double cb = 0.0;
      for (int x = 0; x < 3; ++x) {
        cb += Db[s][x] * (ut[s][x] - ut[b][x]);
        utb[s][x] += coef * Db[s][x];
        utb[b][x] -= coef * Db[s][x];
      }
      nbar[s] -= gam * G * n[b] * cb;
      nbar[b] -= gam * G * n[s] * cb;
      Gb[k] -= gam * n[s] * n[b] * cb;
    }
  for (int s = 0; s < M; ++s)
    if (n[s] != 0.0) {
      for (int k = 0; k < 3; ++k) Jbar[s][k] += utb[s][k] / n[s];
      nbar[s] -= dot3(utb[s], ut[s]) / n[s];
    }
  for (int k = 0; k < M * (M + 1) / 2; ++k) d.Gbar[(long long)k * N + i] = Gb[k];
}

// the C^visc adjoint fields of species s at node c: phibar' = n Ybar and u~
__device__ inline void store_visc_fields(const Geom &g, const AdjArgs &d, const Coord &c, int s,
                                         const double pb[3], const double ut[3]) {
  for (int k = 0; k < 3; ++k) {
    store_images(g, d.psibar + (long long)(3 * s + k) * g.Np, c, pb[k]);
    store_images(g, d.ut + (long long)(3 * s + k) * g.Np, c, ut[k]);
  }
}

// Gbar of every pair at a solid node (with the drag)
template <int M>
__device__ inline void zero_Gbar(const AdjArgs &d, long long N, int i) {
  for (int k = 0; k < M * (M + 1) / 2; ++k) d.Gbar[(long long)k * N + i] = 0.0;
}

// Reverse of the collision of one node (inversion, equilibria, sources and
// trapezoidal update, as in collide_body).  Inputs: the tilde moments of
// the state (tape), n, the force per particle phi = C^mf/n and F; outputs
// the node adjoints of n, Pi~ and J~ (k_adj_stream turns them into the
// adjoint state), phibar (for the shell-gather transpose) and the
// external-force adjoint (accumulated).  Per species, with
//   A = a (m_f + m_g), B = b m_f, D = b m_g  (weighted moments of the
// incoming f- and g-adjoints),
//   nbar  = A0 + 4.5 (2 u^a.A2.u - u.A2.u) - 1.5 (2 u^a.u - u.u) A0 - a m_g0
//   Jbar  = 3 A1,  Pibar = a m_g0
//   uabar = 9n A2.u - 3n A0 u + 9 B2.X - 3 B0 X + 4.5 kappa D2.C
//           + (3 - 1.5 kappa) D0 C + 9 D2.Y - 3 D0 Y
//   ubar += 9n A2.(u^a - u) - 3n A0 (u^a - u)
//   Xbar  = 3 B1 + 9 B2.u^a - 3 B0 u^a
//   Cbar  = 4.5 kappa D2.u^a + (3 - 1.5 kappa) D0 u^a
//   Ybar  = 3 D1 + 9 D2.u^a - 3 D0 u^a
// then back through Pi, u, u^a = J/n, J = J~ + (X or Y)/2 (J~ for Euler),
// X = C + Y, Y = n F (+ n psi with C^visc, + C^drag) and C = n phi.  With
// C^visc it also writes psibar = n Ybar and u~ = J~/n (padded) for the
// C^visc transposes.
template <int M, class A>
__device__ inline void adj_collide_body(const A &a, const AdjArgs &d, int i) {
  const Geom g = geom_of(a);
  if (i >= g.N) return;
  const uint32_t m = a.bb[i];
  const Coord c = decode(g, i);
  const bool drag = drag_on(a);
  const bool visc = d.psibar != nullptr;  // C^visc (its force per particle in slots 3..5)
  const bool qp = d.qpbar != nullptr;  // the per-step quasi-pressure
  if (m & 1u) {
    const double z[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < M; ++s) {
      store_phibar(g, d, c, s, z);
      if (visc) store_visc_fields(g, d, c, s, z, z);
      if (qp) d.qpbar[(long long)s * g.N + i] = 0.0;
    }
    if (drag) zero_Gbar<M>(d, g.N, i);
    return;
  }
  const long long Ns = pop_stride(g), N = g.N;
  const long long P = padded_index(g, c.x, c.y, c.z);
  const bool printed = a.flags & LBE_PRINTED_INV;
  const bool euler = a.flags & LBE_EULER, single = a.flags & LBE_SINGLE;
  // the inversion J = J~ + h (X or Y): h = 0 for Euler; X for SD-TR
  const double half = euler ? 0.0 : 0.5;
  const bool withX = printed || single, shiftPi = !(euler || single);
  const double sgn = printed ? -1.0 : 1.0;
  double n[M], phi[M][3], F[M][3], C[M][3], Y[M][3], X[M][3], ua[M][3], u[3];
  double ut[M][3], Dr[M][3], psi[M][3];
  double ntot = 0.0, Jtot[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < M; ++s) n[s] = a.nfield[(long long)s * g.Np + P];
  if (drag || visc) tape_ut<M>(d, N, i, n, ut);
  if (drag) drag_force<M>(a, P, n, ut, Dr);
  for (int s = 0; s < M; ++s)
    for (int k = 0; k < 3; ++k) psi[s][k] = visc ? a.force[6LL * s * N + (3 + k) * N + i] : 0.0;
  for (int s = 0; s < M; ++s) {
    for (int k = 0; k < 3; ++k) {
      phi[s][k] = a.force[6LL * s * N + k * N + i];
      F[s][k] = a.Fext[(long long)k * N + i] + a.body[s][k];
      C[s][k] = n[s] * phi[s][k];
      // Y = C^visc (+ C^drag) + n F, in the order of the forward step
      const double cv = n[s] * psi[s][k] + (drag ? Dr[s][k] : 0.0);
      Y[s][k] = cv + n[s] * F[s][k];
      X[s][k] = C[s][k] + Y[s][k];
      const double J = d.PJ[(long long)(M + 3 * s + k) * N + i] + half * (withX ? X[s][k] : Y[s][k]);
      ua[s][k] = n[s] != 0.0 ? J / n[s] : 0.0;
      Jtot[k] += J;
    }
    ntot += n[s];
  }
  for (int k = 0; k < 3; ++k) u[k] = ntot != 0.0 ? Jtot[k] / ntot : 0.0;

  WMoments bf[M], bg[M];
  for (int s = 0; s < M; ++s) {
    wzero(bf[s]);
    wzero(bg[s]);
  }
  adj_moments_all<0, M>(g, c, i, m, d, Ns, bf, bg);

  const double ac = a.acoef, bc = a.bcoef, kap = a.kappa, hb = 0.5 * a.beta;
  double nbar[M], Pibar[M], Jbar[M][3], uabar[M][3], Cbar[M][3], Ybar[M][3], Xbar[M][3];
  double ubar[3] = {0.0, 0.0, 0.0};
  const double uu = dot3(u, u);
  for (int s = 0; s < M; ++s) {
    double A0 = ac * (bf[s].m0 + bg[s].m0), A1[3], A2[6], B2[6], D2[6];
    for (int k = 0; k < 3; ++k) A1[k] = ac * (bf[s].m1[k] + bg[s].m1[k]);
    for (int k = 0; k < 6; ++k) {
      A2[k] = ac * (bf[s].m2[k] + bg[s].m2[k]);
      B2[k] = bc * bf[s].m2[k];
      D2[k] = bc * bg[s].m2[k];
    }
    const double B0 = bc * bf[s].m0, D0 = bc * bg[s].m0;
    double A2u[3], A2ua[3], B2ua[3], D2ua[3], B2X[3], D2C[3], D2Y[3];
    symv(A2, u, A2u);
    symv(A2, ua[s], A2ua);
    symv(B2, ua[s], B2ua);
    symv(D2, ua[s], D2ua);
    symv(B2, X[s], B2X);
    symv(D2, C[s], D2C);
    symv(D2, Y[s], D2Y);
    const double uau = dot3(ua[s], u);
    nbar[s] = A0 + 4.5 * (2.0 * dot3(ua[s], A2u) - dot3(u, A2u)) - 1.5 * (2.0 * uau - uu) * A0 -
              ac * bg[s].m0;
    // Pi through g_eq; with the per-step quasi-pressure the zeroth moment
    // of g~ is replaced by the target T = Pi + s beta/2 C.u^a (s = -sgn; T =
    // Pi for Euler): T gets the (1 - a) part of the g adjoint's zeroth
    // moment, the old zeroth moment loses it (Pibar below, added to every
    // g~_q), and Pi = n - beta Phi passes the whole of it to n and Phi
    double pish = ac * bg[s].m0;       // what the Pi~ <-> Pi relation sees
    Pibar[s] = pish;
    if (qp) {
      const double Tb = (1.0 - ac) * bg[s].m0;
      const double pipath = ac * bg[s].m0 + Tb;
      Pibar[s] = -Tb;
      pish = -Tb;
      nbar[s] += pipath;
      d.qpbar[(long long)s * N + i] = -a.beta * pipath;
    }
    const double ns = n[s];
    for (int k = 0; k < 3; ++k) {
      Jbar[s][k] = 3.0 * A1[k];
      uabar[s][k] = 9.0 * ns * A2u[k] - 3.0 * ns * A0 * u[k] + 9.0 * B2X[k] - 3.0 * B0 * X[s][k] +
                    4.5 * kap * D2C[k] + (3.0 - 1.5 * kap) * D0 * C[s][k] + 9.0 * D2Y[k] -
                    3.0 * D0 * Y[s][k];
      ubar[k] += 9.0 * ns * (A2ua[k] - A2u[k]) - 3.0 * ns * A0 * (ua[s][k] - u[k]);
      Xbar[s][k] = 3.0 * bc * bf[s].m1[k] + 9.0 * B2ua[k] - 3.0 * B0 * ua[s][k];
      Cbar[s][k] = 4.5 * kap * D2ua[k] + (3.0 - 1.5 * kap) * D0 * ua[s][k];
      Ybar[s][k] = 3.0 * bc * bg[s].m1[k] + 9.0 * D2ua[k] - 3.0 * D0 * ua[s][k];
      // Pi = Pi~ +- (beta/2) C.u^a (Pi = Pi~ for Euler and SD), or the
      // shift target T = Pi -+ (beta/2) C.u^a
      if (shiftPi) {
        Cbar[s][k] += sgn * hb * pish * ua[s][k];
        uabar[s][k] += sgn * hb * pish * C[s][k];
      }
    }
  }
  if (ntot != 0.0) {
    const double ub = dot3(ubar, u) / ntot;
    for (int s = 0; s < M; ++s) {
      for (int k = 0; k < 3; ++k) Jbar[s][k] += ubar[k] / ntot;
      nbar[s] -= ub;
    }
  }
  double Fb[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < M; ++s) {
    if (n[s] != 0.0) {
      for (int k = 0; k < 3; ++k) Jbar[s][k] += uabar[s][k] / n[s];
      nbar[s] -= dot3(uabar[s], ua[s]) / n[s];
    }
    double pb[3];
    for (int k = 0; k < 3; ++k) {
      if (withX)
        Xbar[s][k] += half * Jbar[s][k];
      else
        Ybar[s][k] += half * Jbar[s][k];
      Cbar[s][k] += Xbar[s][k];
      Ybar[s][k] += Xbar[s][k];
      Fb[k] += n[s] * Ybar[s][k];
      pb[k] = n[s] * Cbar[s][k];
    }
    nbar[s] += dot3(Ybar[s], F[s]) + dot3(Cbar[s], phi[s]);
    store_phibar(g, d, c, s, pb);
    if (visc) {  // C^visc = n psi: phibar' = n Ybar
      double pv[3];
      for (int k = 0; k < 3; ++k) pv[k] = n[s] * Ybar[s][k];
      nbar[s] += dot3(Ybar[s], psi[s]);
      store_visc_fields(g, d, c, s, pv, ut[s]);
    }
  }
  // Y = n F + C^drag: Ybar is also the adjoint of the drag force
  if (drag) adj_drag<M>(a, d, P, i, n, ut, Ybar, nbar, Jbar);
  for (int s = 0; s < M; ++s) store_node(d, M, N, i, s, nbar[s], Pibar[s], Jbar[s]);
  for (int k = 0; k < 3; ++k) d.Fbar[(long long)k * N + i] += Fb[k];
}

template <int M>
__global__ __launch_bounds__(BLOCK) void k_adj_collide(StepArgs a, AdjArgs d) {
  adj_collide_body<M>(a, d, blockIdx.x * BLOCK + threadIdx.x);
}

// Reverse of the read-out of n^a and of the physical J^a = J~ + (X or Y)/2:
// node adjoints of the final state from the seeds dn, dJ (the seed dpop of
// the populations themselves enters in k_adj_stream).
template <int M>
__global__ __launch_bounds__(BLOCK) void k_adj_readout(StepArgs a, AdjArgs d) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const Geom g = a.g;
  if (i >= g.N) return;
  const uint32_t m = a.bb[i];
  const Coord c = decode(g, i);
  const bool drag = drag_on(a);
  const bool visc = d.psibar != nullptr;
  if (m & 1u) {
    const double z[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < M; ++s) {
      store_phibar(g, d, c, s, z);
      if (visc) store_visc_fields(g, d, c, s, z, z);
    }
    if (drag) zero_Gbar<M>(d, g.N, i);
    return;
  }
  const long long N = g.N;
  const long long P = padded_index(g, c.x, c.y, c.z);
  const bool printed = a.flags & LBE_PRINTED_INV;
  const double half = (a.flags & LBE_EULER) ? 0.0 : 0.5;
  const bool withX = printed || (a.flags & LBE_SINGLE);
  double Fb[3] = {0.0, 0.0, 0.0};
  double n[M], nb[M], Jb[M][3], Yb[M][3];
  for (int s = 0; s < M; ++s) {
    n[s] = a.nfield[(long long)s * g.Np + P];
    nb[s] = d.dn ? d.dn[(long long)s * N + i] : 0.0;
    double pb[3];
    for (int k = 0; k < 3; ++k) {
      Jb[s][k] = d.dJ ? d.dJ[(long long)(3 * s + k) * N + i] : 0.0;
      const double phi = a.force[6LL * s * N + k * N + i];
      const double F = a.Fext[(long long)k * N + i] + a.body[s][k];
      // J = J~ + (C + Y)/2 (printed, SD-TR) or J~ + Y/2, Y = nF (+ C^drag);
      // J = J~ for Euler
      Yb[s][k] = half * Jb[s][k];
      const double Cb = withX ? half * Jb[s][k] : 0.0;
      nb[s] += Yb[s][k] * F + Cb * phi;
      Fb[k] += n[s] * Yb[s][k];
      pb[k] = n[s] * Cb;
    }
    store_phibar(g, d, c, s, pb);
  }
  double ut[M][3];
  if (drag || visc) tape_ut<M>(d, N, i, n, ut);
  if (visc)  // Y holds C^visc = n psi too
    for (int s = 0; s < M; ++s) {
      double pv[3], psi[3];
      for (int k = 0; k < 3; ++k) {
        psi[k] = a.force[6LL * s * N + (3 + k) * N + i];
        pv[k] = n[s] * Yb[s][k];
      }
      nb[s] += dot3(Yb[s], psi);
      store_visc_fields(g, d, c, s, pv, ut[s]);
    }
  if (drag) adj_drag<M>(a, d, P, i, n, ut, Yb, nb, Jb);
  for (int s = 0; s < M; ++s) store_node(d, M, N, i, s, nb[s], 0.0, Jb[s]);
  for (int k = 0; k < 3; ++k) d.Fbar[(long long)k * N + i] += Fb[k];
}

// The adjoint state before the step, per node r and population q:
//   mu_f = (1 - a) lambda_f + nbar_loc + nbar,  mu_g = (1 - a) lambda_g + Pi~bar + c_q.J~bar
// (one distribution: mu_f = (1 - a) lambda_f + nbar_loc + nbar + c_q.J~bar, mu_g = 0)
// with lambda the adjoint of the pre-streaming slots (the streaming
// transpose of mu_in) -- or, at the final step, lambda the seed dpop and no
// (1 - a) (the read-out does not collide).
template <int q, int M, bool TERMINAL>
__device__ inline void adj_stream_q(const Geom &g, const Coord &c, int i, uint32_t m,
                                    const AdjArgs &d, long long Ns, long long N, double keep, bool single,
                                    const double nb[M], const double Pib[M], const double Jb[M][3]) {
  if constexpr (q < Q) {
    for (int s = 0; s < M; ++s) {
      double lf, lg;
      if (TERMINAL) {
        lf = d.dpop ? d.dpop[((long long)s * Q + q) * N + i] : 0.0;
        lg = d.dpop ? d.dpop[((long long)(M + s) * Q + q) * N + i] : 0.0;
      } else {
        lf = keep * adj_slot<q>(g, c, i, m, d.mu_in + (long long)s * Q * Ns, Ns);
        lg = keep * adj_slot<q>(g, c, i, m, d.mu_in + (long long)(M + s) * Q * Ns, Ns);
      }
      if (single) {  // f carries the current; no g
        d.mu_out[((long long)s * Q + q) * Ns + i] = lf + nb[s] + cdot<q>(Jb[s]);
        d.mu_out[((long long)(M + s) * Q + q) * Ns + i] = 0.0;
      } else {
        d.mu_out[((long long)s * Q + q) * Ns + i] = lf + nb[s];
        d.mu_out[((long long)(M + s) * Q + q) * Ns + i] = lg + Pib[s] + cdot<q>(Jb[s]);
      }
    }
    adj_stream_q<q + 1, M, TERMINAL>(g, c, i, m, d, Ns, N, keep, single, nb, Pib, Jb);
  }
}

template <int M, bool TERMINAL>
__global__ __launch_bounds__(BLOCK) void k_adj_stream(StepArgs a, AdjArgs d) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const Geom g = a.g;
  if (i >= g.N) return;
  const uint32_t m = a.bb[i];
  const long long Ns = pop_stride(g), N = g.N;
  if (m & 1u) {
    for (int k = 0; k < 2 * M * Q; ++k) d.mu_out[(long long)k * Ns + i] = 0.0;
    return;
  }
  const Coord c = decode(g, i);
  double nb[M], Pib[M], Jb[M][3];
  for (int s = 0; s < M; ++s) {
    nb[s] = d.node[(long long)s * N + i] + d.nbar[(long long)s * N + i];
    Pib[s] = d.node[(long long)(M + s) * N + i];
    for (int k = 0; k < 3; ++k)
      Jb[s][k] = d.node[(long long)(2 * M + 3 * s + k) * N + i] + (d.Jnl ? d.Jnl[(3LL * s + k) * N + i] : 0.0);
  }
  adj_stream_q<0, M, TERMINAL>(g, c, i, m, d, Ns, N, 1.0 - a.acoef, (a.flags & LBE_SINGLE) != 0, nb, Pib,
                               Jb);
}

// the tilde moments Pi~, J~ of a state (tape) and its densities n (padded
// field, as k_moments writes them), and J~ padded as well when the tape has
// a field for it
template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void k_tape_moments(StepArgs a, const T *__restrict__ pop,
                                                      double *__restrict__ PJ) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const Geom g = a.g;
  if (i >= g.N) return;
  const uint32_t m = a.bb[i];
  const Coord c = decode(g, i);
  const long long Ns = pop_stride(g), N = g.N;
  for (int s = 0; s < M; ++s) {
    double n = 0.0, Pi = 0.0, J[3] = {0.0, 0.0, 0.0};
    if (!(m & 1u)) {
      double v[19];
      pull19(g, c, i, m, pop + (long long)s * Q * Ns, Ns, v);
      moments0(v, n);
      // one distribution: f carries the current and there is no Pi~
      if (!(a.flags & LBE_SINGLE)) {
        pull19(g, c, i, m, pop + (long long)(M + s) * Q * Ns, Ns, v);
        moments0(v, Pi);
      }
      moments1(v, J);
    }
    store_images(g, a.nfield + (long long)s * g.Np, c, n);
    PJ[(long long)s * N + i] = Pi;
    for (int k = 0; k < 3; ++k) PJ[(long long)(M + 3 * s + k) * N + i] = J[k];
    if (a.Jfield)  // the drag of the recomputed step reads J~ there
      for (int k = 0; k < 3; ++k) store_images(g, a.Jfield + (long long)(3 * s + k) * g.Np, c, J[k]);
  }
}

// adjoint of the shell gather of one directed pair (alpha, beta), see
// force_body MODE 2: writes or (acc bit 0) accumulates into nbar, writes or
// (acc bit 1) accumulates into Gbar
template <int R, int NY, int NT>
__global__ __launch_bounds__(NT) void k_adj_force(StepArgs a, AdjArgs d, int alpha, int beta, int acc) {
  extern __shared__ double lds[];
  const Tile T = force_tile(a.g, a.zchunk, a.order, NT / FTX * NY);
  force_body<R, 2, NY, NT>(a, &d, alpha, beta, acc, T.bx, T.by, T.bz, lds);
}

// adjoint of the attractive field of the directed pair (alpha, beta), see
// force_body MODE 4: writes or (acc bit 0) accumulates into nbar; the tile
// shapes of the forward attraction gather
template <int R, int NY>
__global__ __launch_bounds__(FNT) void k_adj_att(StepArgs a, AdjArgs d, int alpha, int beta, int acc) {
  extern __shared__ double lds[];
  const Tile T = force_tile(a.g, a.zchunk, a.order, FNT / FTX * NY);
  force_body<R, 4, NY, FNT>(a, &d, alpha, beta, acc, T.bx, T.by, T.bz, lds);
}

// adjoint of the C^visc gather of the directed pair (alpha, beta), force_body
// MODE 5 (see there): writes or accumulates into nbar (acc bit 0),
// Gbar (bit 1) and Jnl (bit 2); 32 x (NT/32) tiles, the ring table through
// scalar loads
template <int R, int MODE, int NT>
__global__ __launch_bounds__(NT) void k_adj_visc(StepArgs a, AdjArgs d, int alpha, int beta, int acc) {
  extern __shared__ double lds[];
  const Tile T = force_tile(a.g, a.zchunk, a.order, NT / FTX);
  force_body<R, MODE, 1, NT>(a, &d, alpha, beta, acc, T.bx, T.by, T.bz, lds);
}

// Vbar = -(grad_h)^T Fbar: transpose of F(r) = -3 sum_p w_p c_p V(idx(r + c_p))
// (idx wraps periodic directions and clamps the others), as a gather over
// the nodes r with idx(r + c_p) = this node
__device__ inline int adj_sources(int x, int n, int c, bool per, int out[2]) {
  if (per) {
    int X = x - c;
    out[0] = X < 0 ? X + n : (X >= n ? X - n : X);
    return 1;
  }
  int k = 0;
  if (x - c >= 0 && x - c < n) out[k++] = x - c;
  if (c == -1 && x == 0 && !(k == 1 && out[0] == 0)) out[k++] = 0;
  if (c == 1 && x == n - 1 && !(k == 1 && out[0] == n - 1)) out[k++] = n - 1;
  return k;
}

__global__ __launch_bounds__(BLOCK) void k_adj_extforce(Geom g, const double *__restrict__ Fbar,
                                                       double *__restrict__ Vbar) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  const Coord c = decode(g, i);
  const long long N = g.N;
  double acc = 0.0;
  for (int p = 1; p < Q; ++p) {
    int xs[2], ys[2], zs[2];
    const int kx = adj_sources(c.x, g.nx, cvec(p, 0), g.periodic & 1u, xs);
    const int ky = adj_sources(c.y, g.ny, cvec(p, 1), g.periodic & 2u, ys);
    const int kz = adj_sources(c.z, g.nz, cvec(p, 2), g.periodic & 4u, zs);
    for (int a = 0; a < kz; ++a)
      for (int b = 0; b < ky; ++b)
        for (int e = 0; e < kx; ++e) {
          const long long r = xs[e] + (long long)g.nx * (ys[b] + (long long)g.ny * zs[a]);
          acc += wgt(p) * (cvec(p, 0) * Fbar[r] + cvec(p, 1) * Fbar[N + r] + cvec(p, 2) * Fbar[2 * N + r]);
        }
  }
  Vbar[i] = -3.0 * acc;
}

// compact fields (nf of them, N values each, zero on solid nodes) into
// padded ones with their periodic images; wall ghosts are left as they are
__global__ __launch_bounds__(BLOCK) void k_pad_fields(Geom g, const uint32_t *__restrict__ bb, int nf,
                                                     const double *__restrict__ in, double *__restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  const Coord c = decode(g, i);
  const bool solid = bb[i] & 1u;
  for (int f = 0; f < nf; ++f)
    store_images(g, out + (long long)f * g.Np, c, solid ? 0.0 : in[(long long)f * g.N + i]);
}

// padded fields back to compact ones (the node's own value)
__global__ __launch_bounds__(BLOCK) void k_unpad_fields(Geom g, int nf, const double *__restrict__ in,
                                                       double *__restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  const Coord c = decode(g, i);
  const long long P = padded_index(g, c.x, c.y, c.z);
  for (int f = 0; f < nf; ++f) out[(long long)f * g.N + i] = in[(long long)f * g.Np + P];
}

// the adjoint of the post-streaming populations of one (species, dist)
// block, compact 19N layout
__global__ __launch_bounds__(BLOCK) void k_adj_state_grad(Geom g, int M, const uint32_t *__restrict__ bb,
                                                         const double *__restrict__ mu, int s, int dist,
                                                         double *__restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  const long long Ns = pop_stride(g), N = g.N;
  const bool solid = bb[i] & 1u;
  for (int q = 0; q < Q; ++q)
    out[(long long)q * N + i] = solid ? 0.0 : mu[((long long)(dist * M + s) * Q + q) * Ns + i];
}

__global__ void k_fill(double *__restrict__ p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}


// ------------------------------------------------------------------------
// velocity divergence D = div_h u / (v_T/dx) of the barycentric velocity,
// with the isotropic D3Q19 divergence (1/v_T^2) sum_p w_p c_p . u(r + c_p);
// u = 0 on solid nodes and beyond non-periodic faces, D = 0 on solid nodes
__global__ __launch_bounds__(BLOCK) void k_divergence(Geom g, const uint32_t *__restrict__ bb,
                                                       const double *__restrict__ u, double scale,
                                                       double *__restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  if (bb[i] & 1u) {
    out[i] = 0.0;
    return;
  }
  const Coord c = decode(g, i);
  const bool px = g.periodic & 1u, py = g.periodic & 2u, pz = g.periodic & 4u;
  const long long N = g.N;
  double div = 0.0;
#pragma unroll
  for (int p = 1; p < Q; ++p) {
    const int cx = cvec(p, 0), cy = cvec(p, 1), cz = cvec(p, 2);
    if ((cx < 0 && c.x == 0 && !px) || (cx > 0 && c.x == g.nx - 1 && !px) ||
        (cy < 0 && c.y == 0 && !py) || (cy > 0 && c.y == g.ny - 1 && !py) ||
        (cz < 0 && c.z == 0 && !pz) || (cz > 0 && c.z == g.nz - 1 && !pz))
      continue;
    const long long j = downstream(g, c, p);
    double cu = 0.0;
    if (cx) cu += cx * u[j];
    if (cy) cu += cy * u[N + j];
    if (cz) cu += cz * u[2 * N + j];
    div += wgt(p) * cu;
  }
  out[i] = div * scale;
}

// ------------------------------------------------------------------------
// quasi-pressure (Sec. 2, eq. quasipressure): Pi^a = n^a - beta Phi^a, Phi
// the line integral of v^a = C^{a,mf} (+ n^a F^a) from the origin by the
// trapezoidal rule on unit lattice steps; v = 0 on solid nodes.  A path runs
// along the three axes in turn (p0, p1, p2): along p0 to r's coordinate with
// the other two at the origin's, then along p1 with p2 at the origin's, then
// along p2.  Every leg is a value of one of three volume scans
//   S_k(r) = signed trapezoidal sum along axis k from (r with k -> o_k) to r,
// so one launch per axis computes S_k on every line of that axis, and a
// combine pass adds, for each order, S_p0(r|p1,p2 -> o) + S_p1(r|p2 -> o) +
// S_p2(r): the order (x, y, z) alone, or the mean over the six orders.
//
// The scans.  Lines along x are contiguous: one wavefront takes a row and
// scans it 64 nodes at a time with a lane prefix sum (coalesced).  Lines
// along y and z: a workgroup holds QP_LANES lines at adjacent x (coalesced
// across lanes) and cuts each into QP_SEG segments; a thread keeps its
// segment's integrand in registers (at most QP_REG nodes, longer lines take
// a second read), and with P(e) = sum_{k<e} (v(k) + v(k+1))/2 along a line,
// S(e) = P(e) - P(o).  blockIdx.y is the species.
constexpr int QP_LANES = 64, QP_SEG = 16, QP_REG = 16;

struct QpScan {
  int axis;     // 1 y, 2 z (x has its own kernel)
  int L;        // nodes on a line
  int o;        // origin coordinate along the line
  int Lu;       // lines are (u, v) = (x, z) for y, (x, y) for z, u fastest
  int nlines;
  int fext;     // add n^a F^a to the integrand
};

// v_k at compact node i, padded node pi: n (C^mf/n + [F + body]), 0 on solid
// nodes
template <class A>
__device__ inline double qp_v(const A &a, int s, int k, bool fext, long long i, long long pi) {
  if (a.bb[i] & 1u) return 0.0;
  const double n = a.nfield[(long long)s * a.g.Np + pi];
  double v = a.force[(6LL * s + k) * a.g.N + i];
  if (fext) v += a.Fext[(long long)k * a.g.N + i] + a.body[s][k];
  return n * v;
}

// lane prefix sum over the 64 lanes of a wavefront (inclusive)
__device__ inline double wave_scan(double t, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double u = __shfl_up(t, d, 64);
    if (lane >= d) t += u;
  }
  return t;
}

// x lines: one wavefront per row (y, z), four rows per workgroup (block
// blk of the box), species s
template <class A>
__device__ inline void qp_scan_x_body(const A &a, int o, int fext, double *S, int blk, int s) {
  const int lane = threadIdx.x & 63;
  const int row = blk * 4 + (threadIdx.x >> 6);
  const Geom g = geom_of(a);
  if (row >= g.ny * g.nz) return;  // the whole wavefront leaves together
  const int y = row % g.ny, z = row / g.ny;
  const long long ib = (long long)g.nx * row;
  const long long pb = g.R + (long long)g.PX * ((y + g.R) + (long long)g.PY * (z + g.R));
  double *out = S + 3LL * s * g.N + ib;
  // S(e) = carry + exclusive prefix of t(e) = (v(e) + v(e+1))/2 (t = 0 at the
  // last node); a first sweep finds S(o), a second writes S(e) - S(o)
  double so = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    double carry = 0.0;
    for (int c0 = 0; c0 < g.nx; c0 += 64) {
      if (pass == 0 && c0 > o) break;
      const int e = c0 + lane;
      const double ve = e < g.nx ? qp_v(a, s, 0, fext, ib + e, pb + e) : 0.0;
      double vn = __shfl_down(ve, 1, 64);
      if (lane == 63) vn = e + 1 < g.nx ? qp_v(a, s, 0, fext, ib + e + 1, pb + e + 1) : 0.0;
      const double t = e + 1 < g.nx ? 0.5 * (ve + vn) : 0.0;
      const double incl = wave_scan(t, lane);
      const double Se = carry + (incl - t);
      if (pass == 0) {
        const double cand = __shfl(Se, o - c0 < 64 ? o - c0 : 0, 64);
        if (o - c0 < 64) so = cand;
      } else if (e < g.nx) {
        out[e] = Se - so;
      }
      carry += __shfl(incl, 63, 64);
    }
  }
}

__global__ __launch_bounds__(256) void k_qp_scan_x(StepArgs a, int o, int fext, double *S) {
  qp_scan_x_body(a, o, fext, S, blockIdx.x, blockIdx.y);
}

// the y (axis 1) or z (axis 2) lines of a box
__host__ __device__ inline QpScan qp_scan_of(const Geom &g, int axis, int o, int fext) {
  if (axis == 1) return {1, g.ny, o, g.nx, g.nx * g.nz, fext};
  return {2, g.nz, o, g.nx, g.nx * g.ny, fext};
}

// y and z lines: block blk of the box, species s
template <class A>
__device__ inline void qp_scan_body(const A &a, const QpScan &q, double *S, int blk, int s) {
  __shared__ double segsum[QP_SEG][QP_LANES];
  __shared__ double porigin[QP_LANES];
  const int lane = threadIdx.x % QP_LANES, sg = threadIdx.x / QP_LANES;
  const int l = blk * QP_LANES + lane;
  const bool live = l < q.nlines;
  const int Ls = (q.L + QP_SEG - 1) / QP_SEG;
  const int e0 = min(sg * Ls, q.L), e1 = min(e0 + Ls, q.L);
  const Geom g = geom_of(a);
  const int u = live ? l % q.Lu : 0, w = live ? l / q.Lu : 0;
  // element 0 of the line and the strides along it (compact and padded)
  long long ib, pb, es, ps;
  if (q.axis == 1) {  // (x, z) = (u, w)
    ib = u + (long long)g.nx * g.ny * w;
    pb = (u + g.R) + (long long)g.PX * (g.R + (long long)g.PY * (w + g.R));
    es = g.nx;
    ps = g.PX;
  } else {            // (x, y) = (u, w)
    ib = u + (long long)g.nx * w;
    pb = (u + g.R) + (long long)g.PX * ((w + g.R) + (long long)g.PY * g.R);
    es = (long long)g.nx * g.ny;
    ps = (long long)g.PX * g.PY;
  }
  // the segment's integrand, nodes e0 .. e1 (the last one belongs to the
  // next segment), in registers when the segment is short enough
  double vreg[QP_REG + 1];
  const bool inreg = e1 - e0 <= QP_REG;
  auto v = [&](int e) { return qp_v(a, s, q.axis, q.fext, ib + e * es, pb + e * ps); };
  double run = 0.0;
  if (live && e0 < e1) {
    if (inreg) {
#pragma unroll
      for (int k = 0; k <= QP_REG; ++k)
        vreg[k] = (e0 + k <= e1 && e0 + k < q.L) ? v(e0 + k) : 0.0;
#pragma unroll
      for (int k = 0; k < QP_REG; ++k) {
        const int e = e0 + k;
        if (e < e1) {
          if (e == q.o) porigin[lane] = run;
          if (e + 1 < q.L) run += 0.5 * (vreg[k] + vreg[k + 1]);
        }
      }
    } else {
      double vk = v(e0);
      for (int e = e0; e < e1; ++e) {
        if (e == q.o) porigin[lane] = run;
        if (e + 1 < q.L) {
          const double vn = v(e + 1);
          run += 0.5 * (vk + vn);
          vk = vn;
        }
      }
    }
  }
  segsum[sg][lane] = run;
  __syncthreads();
  if (!live || e0 >= e1) return;
  const int so = q.o / Ls;
  double off = 0.0, po = 0.0;
  for (int t = 0; t < QP_SEG; ++t) {
    if (t < sg) off += segsum[t][lane];
    if (t < so) po += segsum[t][lane];
  }
  po += porigin[lane];
  double *out = S + (3LL * s + q.axis) * g.N;
  double run2 = off;
  if (inreg) {
#pragma unroll
    for (int k = 0; k < QP_REG; ++k) {
      const int e = e0 + k;
      if (e < e1) {
        out[ib + e * es] = run2 - po;
        if (e + 1 < q.L) run2 += 0.5 * (vreg[k] + vreg[k + 1]);
      }
    }
    return;
  }
  double vk = v(e0);
  for (int e = e0; e < e1; ++e) {
    out[ib + e * es] = run2 - po;
    if (e + 1 < q.L) {
      const double vn = v(e + 1);
      run2 += 0.5 * (vk + vn);
      vk = vn;
    }
  }
}

__global__ __launch_bounds__(QP_LANES *QP_SEG) void k_qp_scan(StepArgs a, QpScan q, double *S) {
  qp_scan_body(a, q, S, blockIdx.x, blockIdx.y);
}

// Phi from the three scans, or (write_pi) Pi = n - beta Phi (0 on solid
// nodes); node i of the box, species s.  Orders are summed as (x,y,z),
// (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x), each as (leg 0 + leg 1) +
// leg 2.
template <class Args>
__device__ inline void qp_combine_body(const Args &a, const double *__restrict__ S, int ox, int oy, int oz,
                                       int sym, int write_pi, double *__restrict__ pi, int i, int s) {
  const Geom g = geom_of(a);
  if (i >= g.N) return;
  const long long N = g.N;
  double *out = pi + (long long)s * N;
  if (a.bb[i] & 1u) {
    out[i] = 0.0;
    return;
  }
  const int x = i % g.nx, t = i / g.nx, y = t % g.ny, z = t / g.ny;
  const double *Sx = S + 3LL * s * N, *Sy = Sx + N, *Sz = Sy + N;
  auto at = [&](const double *A, int X, int Y, int Z) { return A[X + (long long)g.nx * (Y + (long long)g.ny * Z)]; };
  double phi = (at(Sx, x, oy, oz) + at(Sy, x, y, oz)) + Sz[i];
  if (sym) {
    phi += (at(Sx, x, oy, oz) + at(Sz, x, oy, z)) + Sy[i];
    phi += (at(Sy, ox, y, oz) + at(Sx, x, y, oz)) + Sz[i];
    phi += (at(Sy, ox, y, oz) + at(Sz, ox, y, z)) + Sx[i];
    phi += (at(Sz, ox, oy, z) + at(Sx, x, oy, z)) + Sy[i];
    phi += (at(Sz, ox, oy, z) + at(Sy, ox, y, z)) + Sx[i];
    phi = phi / 6.0;
  }
  if (!write_pi) {
    out[i] = phi;
    return;
  }
  const double n = a.nfield[(long long)s * g.Np + padded_index(g, x, y, z)];
  out[i] = n - a.beta * phi;
}

__global__ __launch_bounds__(BLOCK) void k_qp_combine(StepArgs a, const double *__restrict__ S, int ox,
                                                      int oy, int oz, int sym, int write_pi,
                                                      double *__restrict__ pi) {
  qp_combine_body(a, S, ox, oy, oz, sym, write_pi, pi, blockIdx.x * BLOCK + threadIdx.x, blockIdx.y);
}

// The path integral of every box of a batch, one launch per phase: each
// block finds its box in the phase's block table, and the box's route in
// routes[box]; Phi goes to the box's pifield.
__global__ __launch_bounds__(256) void kb_qp_scan_x(BatchArgs ba, const QpRoute *routes) {
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const auto &r = *cptr(routes + b);
  qp_scan_x_body(a, r.o[0], r.fext, r.scan, blockIdx.x - cptr(ba.blockstart)[b], blockIdx.y);
}

__global__ __launch_bounds__(QP_LANES *QP_SEG) void kb_qp_scan(BatchArgs ba, const QpRoute *routes, int axis) {
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const auto &r = *cptr(routes + b);
  const QpScan q = qp_scan_of(geom_of(a), axis, r.o[axis], r.fext);
  qp_scan_body(a, q, r.scan, blockIdx.x - cptr(ba.blockstart)[b], blockIdx.y);
}

__global__ __launch_bounds__(BLOCK) void kb_qp_combine(BatchArgs ba, const QpRoute *routes) {
  const int b = cptr(ba.blockbox)[blockIdx.x];
  const auto &a = *cptr(ba.boxes + b);
  const auto &r = *cptr(routes + b);
  const int i = (blockIdx.x - cptr(ba.blockstart)[b]) * BLOCK + threadIdx.x;
  qp_combine_body(a, r.scan, r.o[0], r.o[1], r.o[2], r.sym, 0, const_cast<double *>(a.pifield), i, blockIdx.y);
}

// g~_p += w_p (Pi~ - sum_q g~_q) on the post-streaming g~ of species s, with
// Pi~ from Pi by the inversion of Sec. 4.2 at the node's current u^a
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_qp_apply(StepArgs a, Readout r, const double *__restrict__ pi,
                                                     int s, T *__restrict__ gst, long long Ns) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const long long N = a.g.N;
  if (i >= N || (a.bb[i] & 1u)) return;
  double target = pi[(long long)s * N + i];
  if (!(a.flags & LBE_EULER)) {
    double cu = 0.0;
    for (int k = 0; k < 3; ++k) cu += r.cmf[(3LL * s + k) * N + i] * r.ua[(3LL * s + k) * N + i];
    target += ((a.flags & LBE_PRINTED_INV) ? 0.5 : -0.5) * a.beta * cu;
  }
  double v[Q], sum = 0.0;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    v[p] = (double)gst[(long long)p * Ns + i];
    sum += v[p];
  }
  const double d = target - sum;
#pragma unroll
  for (int p = 0; p < Q; ++p) gst[(long long)p * Ns + i] = T(v[p] + wgt(p) * d);
}

// ------------------------------------------------------------------------
// Transpose of the per-step quasi-pressure's path integral.  Along one line
// with origin coordinate o, the trapezoidal leg S(e) = sum_j K(e, j) v(j)
// (K = 1/2 at the two ends and 1 between, negative when e < o) has the
// transpose
//   (K^T Y)(j) = theta(j) T - P(j) - Y(j)/2,
// with P(j) = sum_{e<j} Y(e), T the line total and theta = 1, 1/2, 0 for
// j >, =, < o.  The last leg of an axis order is transposed along every
// line of its axis; the middle leg, shared along the last axis, from column
// sums, onto the plane through the origin; the first leg from plane sums,
// onto the line through the origin.  Each term goes to an array of its own
// and the apply pass adds them per node (no two jobs write one element).
// One thread per line; blockIdx.y is the species, blockIdx.z the job.
struct QpLines {
  int nlines, L, o, Lu;
  long long is1, is2, ies;      // input: line l, element e at (l % Lu) is1 + (l / Lu) is2 + e ies
  long long os1, os2, oes;      // output, likewise
  long long isp, osp;           // species strides of input and output
};

constexpr int QP_MAXJOBS = 9;
struct QpJobs {
  int njobs;
  QpLines q[QP_MAXJOBS];
  const double *in[QP_MAXJOBS];
  double *out[QP_MAXJOBS];
  double coef[QP_MAXJOBS];
  int sum[QP_MAXJOBS];          // 1: line sums, 0: the transpose K^T
};

__global__ __launch_bounds__(BLOCK) void k_adj_qp_jobs(QpJobs J) {
  const int jb = blockIdx.z;
  const QpLines &q = J.q[jb];
  const int l = blockIdx.x * BLOCK + threadIdx.x;
  if (l >= q.nlines) return;
  const double *pin = J.in[jb] + blockIdx.y * q.isp + (l % q.Lu) * q.is1 + (l / q.Lu) * q.is2;
  double *pout = J.out[jb] + blockIdx.y * q.osp + (l % q.Lu) * q.os1 + (l / q.Lu) * q.os2;
  double T = 0.0;
  for (int e = 0; e < q.L; ++e) T += pin[e * q.ies];
  if (J.sum[jb]) {
    *pout = T;
    return;
  }
  const double c = J.coef[jb];
  double P = 0.0;
  for (int j = 0; j < q.L; ++j) {
    const double Y = pin[j * q.ies];
    const double th = j > q.o ? 1.0 : (j == q.o ? 0.5 : 0.0);
    pout[j * q.oes] = c * (th * T - P - 0.5 * Y);
    P += Y;
  }
}

// Small per-species arrays of the transpose (species stride: their total):
// column sums Cz(x,y), Cy(x,z), Cx(y,z); plane sums Sx(x), Sy(y), Sz(z);
// middle legs on the planes through the origin, Pyz(x,y) and Pxz(x,y) on
// z = oz, Pzy(x,z) and Pxy(x,z) on y = oy, Pzx(y,z) and Pyx(y,z) on x = ox
// (first letter: the axis of the leg); first legs Lx(x), Ly(y), Lz(z).
struct QpSmall {
  long long Cz, Cy, Cx, Sx, Sy, Sz, Pyz, Pxz, Pzy, Pxy, Pzx, Pyx, Lx, Ly, Lz, total;
};
__host__ __device__ inline QpSmall qp_small(int nx, int ny, int nz) {
  QpSmall o;
  const long long xy = (long long)nx * ny, xz = (long long)nx * nz, yz = (long long)ny * nz;
  o.Cz = 0; o.Cy = xy; o.Cx = o.Cy + xz;
  o.Sx = o.Cx + yz; o.Sy = o.Sx + nx; o.Sz = o.Sy + ny;
  o.Pyz = o.Sz + nz; o.Pxz = o.Pyz + xy; o.Pzy = o.Pxz + xy; o.Pxy = o.Pzy + xz;
  o.Pzx = o.Pxy + xz; o.Pyx = o.Pzx + yz;
  o.Lx = o.Pyx + yz; o.Ly = o.Lx + nx; o.Lz = o.Ly + ny;
  o.total = o.Lz + nz;
  return o;
}

// vbar = the integrand's adjoint (volume terms in qpv, plane and line terms
// from the small arrays), into the adjoints of the per-particle force
// (phibar = n vbar, padded with images), of n (phi.vbar, or (phi + F).vbar)
// and of the external force (n vbar, with n F in the integrand)
template <int M>
__global__ __launch_bounds__(BLOCK) void k_adj_qp_apply(StepArgs a, AdjArgs d, int ox, int oy, int oz, int sym,
                                                       int fext) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const Geom g = a.g;
  if (i >= g.N) return;
  if (a.bb[i] & 1u) return;
  const long long N = g.N;
  const Coord c = decode(g, i);
  const int x = c.x, y = c.y, z = c.z, nx = g.nx, ny = g.ny;
  const long long P = padded_index(g, x, y, z);
  const QpSmall o = qp_small(g.nx, g.ny, g.nz);
  double Fb[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < M; ++s) {
    const double *sm = d.qpsum + s * o.total;
    const double *vol = d.qpv + 3LL * s * N;
    double vb[3];
    vb[0] = sym ? vol[i] : 0.0;
    vb[1] = sym ? vol[N + i] : 0.0;
    vb[2] = vol[2 * N + i];
    if (z == oz) vb[1] += sm[o.Pyz + x + (long long)nx * y];
    if (y == oy && z == oz) vb[0] += sm[o.Lx + x];
    if (sym) {
      if (z == oz) vb[0] += sm[o.Pxz + x + (long long)nx * y];
      if (y == oy) {
        vb[2] += sm[o.Pzy + x + (long long)nx * z];
        vb[0] += sm[o.Pxy + x + (long long)nx * z];
      }
      if (x == ox) {
        vb[2] += sm[o.Pzx + y + (long long)ny * z];
        vb[1] += sm[o.Pyx + y + (long long)ny * z];
      }
      if (x == ox && z == oz) vb[1] += sm[o.Ly + y];
      if (x == ox && y == oy) vb[2] += sm[o.Lz + z];
    }
    const double n = a.nfield[(long long)s * g.Np + P];
    double pb[3], nb = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double phi = a.force[(6LL * s + k) * N + i];
      const double F = fext ? a.Fext[(long long)k * N + i] + a.body[s][k] : 0.0;
      nb += (phi + F) * vb[k];
      pb[k] = d.phibar[(long long)(3 * s + k) * g.Np + P] + n * vb[k];
      Fb[k] += n * vb[k];
    }
    store_phibar(g, d, c, s, pb);
    d.node[(long long)s * N + i] += nb;
  }
  if (fext)
    for (int k = 0; k < 3; ++k) d.Fbar[(long long)k * N + i] += Fb[k];
}

}  // namespace

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
void launch_bbmask(const Geom &g, const uint8_t *solid, uint32_t *bb, hipStream_t s) {
  hipLaunchKernelGGL(k_bbmask, grid_for(g.N), dim3(BLOCK), 0, s, g, solid, bb);
}

void launch_extforce(const Geom &g, const double *V, double *F, hipStream_t s) {
  hipLaunchKernelGGL(k_extforce, grid_for(g.N), dim3(BLOCK), 0, s, g, V, F);
}

void launch_zero_solid(const Geom &g, int M, int prec, void *pop, const uint32_t *bb,
                       long long stride, hipStream_t s) {
  if (prec == LBE_FP64)
    hipLaunchKernelGGL(k_zero_solid<double>, grid_for(g.N), dim3(BLOCK), 0, s, g, 2 * M,
                       (double *)pop, bb, stride);
  else
    hipLaunchKernelGGL(k_zero_solid<float>, grid_for(g.N), dim3(BLOCK), 0, s, g, 2 * M,
                       (float *)pop, bb, stride);
}

void launch_rest_equilibrium(const Geom &g, int prec, const uint32_t *bb, const double *n0,
                             void *out, hipStream_t s) {
  long long Ns = ((long long)g.N + 63) / 64 * 64;
  if (prec == LBE_FP64)
    hipLaunchKernelGGL(k_rest_equilibrium<double>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb, n0,
                       (double *)out, Ns);
  else
    hipLaunchKernelGGL(k_rest_equilibrium<float>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb, n0,
                       (float *)out, Ns);
}

void launch_unstream(const Geom &g, int prec, const uint32_t *bb, const void *target, void *out,
                     hipStream_t s) {
  long long Ns = ((long long)g.N + 63) / 64 * 64;
  if (prec == LBE_FP64)
    hipLaunchKernelGGL(k_unstream<double>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb,
                       (const double *)target, (double *)out, Ns);
  else
    hipLaunchKernelGGL(k_unstream<float>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb,
                       (const float *)target, (float *)out, Ns);
}

void launch_pull(const Geom &g, int prec, const uint32_t *bb, const void *pre, void *out,
                 hipStream_t s) {
  long long Ns = ((long long)g.N + 63) / 64 * 64;
  if (prec == LBE_FP64)
    hipLaunchKernelGGL(k_pull<double>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb,
                       (const double *)pre, (double *)out, Ns);
  else
    hipLaunchKernelGGL(k_pull<float>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb,
                       (const float *)pre, (float *)out, Ns);
}

void launch_moments(const StepArgs &a, int prec, const void *pop, hipStream_t s) {
  // the currents J~ are needed by C^visc and by the interspecies drag
  bool visc = a.Jfield != nullptr;
  dim3 gr = grid_for(a.g.N);
  if (prec == LBE_FP64) {
    if (visc)
      hipLaunchKernelGGL((k_moments<double, true>), gr, dim3(BLOCK), 0, s, a, (const double *)pop);
    else
      hipLaunchKernelGGL((k_moments<double, false>), gr, dim3(BLOCK), 0, s, a, (const double *)pop);
  } else {
    if (visc)
      hipLaunchKernelGGL((k_moments<float, true>), gr, dim3(BLOCK), 0, s, a, (const float *)pop);
    else
      hipLaunchKernelGGL((k_moments<float, false>), gr, dim3(BLOCK), 0, s, a, (const float *)pop);
  }
}

// z depth of a ball-kernel workgroup: the largest of 4 and 2 that still
// gives at least 1024 workgroups, else 1.  Depth 8 is not used: at 128^3
// its 60 KB workgroups fit two to a CU and ran in two rounds with the
// staging exposed, where depth 4 fits three (0.078 -> 0.068 ms).  A smaller
// depth costs more staging per node (2R planes of halo per ZC planes), so
// boxes that reach 1024 workgroups at depth 2 keep it.  The sums do not
// depend on the depth (each node adds its ball in table order).
int ball_block_zc(const Geom &g) {
  const long long tiles = (long long)((g.nx + FTX - 1) / FTX) * ((g.ny + FTY - 1) / FTY);
  for (int zc = 4; zc > 1; zc /= 2)
    if (tiles * ((g.nz + zc - 1) / zc) >= 1024) return zc;
  return 1;
}

template <int M, int MODE, int ZC>
static void ball_launch_zc(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  const Geom &g = a.g;
  const size_t bytes = ball_lds_bytes(a.t.ball_R, a.t.ball_total, ZC);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ball<M, MODE, ZC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  const int blocks = ((g.nx + FTX - 1) / FTX) * ((g.ny + FTY - 1) / FTY) * ((g.nz + ZC - 1) / ZC);
  hipLaunchKernelGGL((k_ball<M, MODE, ZC>), dim3(blocks), dim3(BLOCK), bytes, s, a, d);
}

template <int M, int MODE>
static void ball_launch_m(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  switch (ball_block_zc(a.g)) {
    case 8: ball_launch_zc<M, MODE, 8>(a, d, s); break;
    case 4: ball_launch_zc<M, MODE, 4>(a, d, s); break;
    case 2: ball_launch_zc<M, MODE, 2>(a, d, s); break;
    default: ball_launch_zc<M, MODE, 1>(a, d, s); break;
  }
}

template <int MODE>
static void ball_launch(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  switch (a.M) {
    case 1: ball_launch_m<1, MODE>(a, d, s); break;
    case 2: ball_launch_m<2, MODE>(a, d, s); break;
    case 3: ball_launch_m<3, MODE>(a, d, s); break;
    default: ball_launch_m<4, MODE>(a, d, s); break;
  }
}

void launch_contact(const StepArgs &a, hipStream_t s) {
  AdjArgs none;
  memset(&none, 0, sizeof none);
  ball_launch<0>(a, none, s);
}

// the force kernel's tile shapes (lbe_set_force_tiling): 0 = 256 threads,
// one row each (32 x 8); 1 = 256 threads, two rows each (32 x 16);
// 2 = 512 threads, one row each (32 x 16): shape_ny, shape_nt, shape_ty

template <int R, bool VISC, int SHAPE>
static void force_launch_shape(const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  constexpr int NY = shape_ny(SHAPE), NT = shape_nt(SHAPE), TY = shape_ty(SHAPE);
  const int k = pair_index(a.M, alpha, beta);
  const size_t bytes = force_lds(VISC ? 1 : 0, R, TY, a.t.pair_nent[k], NY);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_force<R, VISC, NY, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  const dim3 gr(force_blocks(a.g, a.zchunk, TY));
  hipLaunchKernelGGL((k_force<R, VISC, NY, NT>), gr, dim3(NT), bytes, s, a, alpha, beta, acc);
}

template <int R, bool VISC>
static void force_launch(const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  if (a.rows == 1)
    force_launch_shape<R, VISC, 1>(a, alpha, beta, acc, s);
  else if (a.rows == 2)
    force_launch_shape<R, VISC, 2>(a, alpha, beta, acc, s);
  else
    force_launch_shape<R, VISC, 0>(a, alpha, beta, acc, s);
}

template <bool VISC>
static void force_r(int R, const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  switch (R) {
    case 1: force_launch<1, VISC>(a, alpha, beta, acc, s); break;
    case 2: force_launch<2, VISC>(a, alpha, beta, acc, s); break;
    case 3: force_launch<3, VISC>(a, alpha, beta, acc, s); break;
    case 4: force_launch<4, VISC>(a, alpha, beta, acc, s); break;
    case 5: force_launch<5, VISC>(a, alpha, beta, acc, s); break;
    case 6: force_launch<6, VISC>(a, alpha, beta, acc, s); break;
    case 7: force_launch<7, VISC>(a, alpha, beta, acc, s); break;
    default: force_launch<8, VISC>(a, alpha, beta, acc, s); break;
  }
}

template <int R, int NY>
static void att_launch_rows(const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  constexpr int TY = FNT / FTX * NY;
  const int k = pair_index(a.M, alpha, beta);
  const size_t bytes = force_lds(3, R, TY, a.t.att_nent[k], NY);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_force_att<R, NY>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  hipLaunchKernelGGL((k_force_att<R, NY>), dim3(force_blocks(a.g, a.zchunk, TY)), dim3(FNT), bytes, s, a,
                     alpha, beta, acc);
}

template <int R>
static void att_launch(const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  if (att_rows(a) == 1)
    att_launch_rows<R, 1>(a, alpha, beta, acc, s);
  else
    att_launch_rows<R, 2>(a, alpha, beta, acc, s);
}

static void att_r(int R, const StepArgs &a, int alpha, int beta, int acc, hipStream_t s) {
  switch (R) {
    case 1: att_launch<1>(a, alpha, beta, acc, s); break;
    case 2: att_launch<2>(a, alpha, beta, acc, s); break;
    case 3: att_launch<3>(a, alpha, beta, acc, s); break;
    case 4: att_launch<4>(a, alpha, beta, acc, s); break;
    case 5: att_launch<5>(a, alpha, beta, acc, s); break;
    case 6: att_launch<6>(a, alpha, beta, acc, s); break;
    case 7: att_launch<7>(a, alpha, beta, acc, s); break;
    default: att_launch<8>(a, alpha, beta, acc, s); break;
  }
}

void launch_forces(const StepArgs &a, hipStream_t s) {
  if (a.flags & LBE_IDEAL) return;  // the force buffer stays zero
  bool visc = (a.flags & LBE_VISC) != 0;
  for (int al = 0; al < a.M; ++al) {
    int written = 0;
    for (int be = 0; be < a.M; ++be) {
      int R = a.t.pair_R[pair_index(a.M, al, be)];
      if (R == 0) continue;  // empty shell
      if (visc)
        force_r<true>(R, a, al, be, written, s);
      else
        force_r<false>(R, a, al, be, written, s);
      written = 1;
    }
    // the attractive field of every pair with one (Appendix, part of C^mf)
    for (int be = 0; be < a.M; ++be) {
      int R = a.t.att_R[pair_index(a.M, al, be)];
      if (R == 0) continue;
      att_r(R, a, al, be, written, s);
      written = 1;
    }
  }
}

template <typename T>
static void collide_m(const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  dim3 gr = grid_for(a.g.N);
  switch (a.M) {
    case 1: hipLaunchKernelGGL((k_collide<T, 1>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, (T *)pout); break;
    case 2: hipLaunchKernelGGL((k_collide<T, 2>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, (T *)pout); break;
    case 3: hipLaunchKernelGGL((k_collide<T, 3>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, (T *)pout); break;
    default: hipLaunchKernelGGL((k_collide<T, 4>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, (T *)pout); break;
  }
}

void launch_collide(const StepArgs &a, int prec, const void *pin, void *pout, hipStream_t s) {
  if (prec == LBE_FP64)
    collide_m<double>(a, pin, pout, s);
  else
    collide_m<float>(a, pin, pout, s);
}

template <typename T>
static void readout_m(const StepArgs &a, const void *pin, const Readout &r, hipStream_t s) {
  dim3 gr = grid_for(a.g.N);
  switch (a.M) {
    case 1: hipLaunchKernelGGL((k_readout<T, 1>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, r); break;
    case 2: hipLaunchKernelGGL((k_readout<T, 2>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, r); break;
    case 3: hipLaunchKernelGGL((k_readout<T, 3>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, r); break;
    default: hipLaunchKernelGGL((k_readout<T, 4>), gr, dim3(BLOCK), 0, s, a, (const T *)pin, r); break;
  }
}

void launch_readout(const StepArgs &a, int prec, const void *pin, const Readout &r, hipStream_t s) {
  if (prec == LBE_FP64)
    readout_m<double>(a, pin, r, s);
  else
    readout_m<float>(a, pin, r, s);
}

int node_blocks(const Geom &g) { return (g.N + BLOCK - 1) / BLOCK; }

int force_blocks(const Geom &g, int zchunk, int ty) {
  return ((g.nx + FTX - 1) / FTX) * ((g.ny + ty - 1) / ty) * ((g.nz + zchunk - 1) / zchunk);
}

int force_tile_rows(int shape) { return shape_ty(shape); }

template <int R, bool VISC, int SHAPE>
static size_t force_lds_bytes(int entries) {
  return force_lds(VISC ? 1 : 0, R, shape_ty(SHAPE), entries, shape_ny(SHAPE));
}

template <int R, bool VISC, int SHAPE>
static void prepare_shape(int entries) {
  const size_t bytes = force_lds_bytes<R, VISC, SHAPE>(entries);
  if (bytes <= 160 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_force<R, VISC, SHAPE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int R, bool VISC>
static void prepare_one(int entries) {
  prepare_shape<R, VISC, 0>(entries);
  prepare_shape<R, VISC, 1>(entries);
  prepare_shape<R, VISC, 2>(entries);
}

// raise the dynamic-LDS limit of every force kernel up to shell range maxR
// (done before a graph is captured)
void prepare_force_kernels(int maxR, bool visc, int max_entries) {
#define PREP(R)                                       \
  if (maxR >= R) {                                    \
    if (visc) prepare_one<R, true>(max_entries);      \
    else prepare_one<R, false>(max_entries);          \
  }
  PREP(1) PREP(2) PREP(3) PREP(4) PREP(5) PREP(6) PREP(7) PREP(8)
#undef PREP
}

// a runtime species count as the template argument MM of CALL
#define LBE_SWITCH_M(M_, CALL) \
  switch (M_) {                \
    case 1: { constexpr int MM = 1; CALL; } break; \
    case 2: { constexpr int MM = 2; CALL; } break; \
    case 3: { constexpr int MM = 3; CALL; } break; \
    default: { constexpr int MM = 4; CALL; } break; \
  }

void launch_batch_moments(const BatchArgs &b, int nblocks, int prec, bool visc, hipStream_t s) {
  if (prec == LBE_FP64) {
    if (visc) hipLaunchKernelGGL((kb_moments<double, true>), dim3(nblocks), dim3(BLOCK), 0, s, b);
    else hipLaunchKernelGGL((kb_moments<double, false>), dim3(nblocks), dim3(BLOCK), 0, s, b);
  } else {
    if (visc) hipLaunchKernelGGL((kb_moments<float, true>), dim3(nblocks), dim3(BLOCK), 0, s, b);
    else hipLaunchKernelGGL((kb_moments<float, false>), dim3(nblocks), dim3(BLOCK), 0, s, b);
  }
}

template <int M, int ZC>
static void batch_ball_zc(const BatchArgs &b, int nblocks, size_t bytes, hipStream_t s) {
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_ball<M, ZC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  hipLaunchKernelGGL((kb_ball<M, ZC>), dim3(nblocks), dim3(BLOCK), bytes, s, b);
}

void launch_batch_ball(const BatchArgs &b, int nblocks, int zc, size_t lds_bytes, int M, hipStream_t s) {
  switch (zc) {
    case 8: LBE_SWITCH_M(M, (batch_ball_zc<MM, 8>(b, nblocks, lds_bytes, s))) break;
    case 4: LBE_SWITCH_M(M, (batch_ball_zc<MM, 4>(b, nblocks, lds_bytes, s))) break;
    case 2: LBE_SWITCH_M(M, (batch_ball_zc<MM, 2>(b, nblocks, lds_bytes, s))) break;
    default: LBE_SWITCH_M(M, (batch_ball_zc<MM, 1>(b, nblocks, lds_bytes, s))) break;
  }
}

size_t ball_lds_bytes(int ball_R, int ball_total, int zc) {
  return sizeof(double) * (size_t)(FTX + 2 * ball_R) * (FTY + 2 * ball_R) * (zc + 2 * ball_R) +
         sizeof(int) * (size_t)ball_total;
}

int ball_blocks(const Geom &g, int zc) {
  return ((g.nx + FTX - 1) / FTX) * ((g.ny + FTY - 1) / FTY) * ((g.nz + zc - 1) / zc);
}

template <int R, bool VISC, int SHAPE>
static void batch_force_s(const BatchArgs &b, int nblocks, int entries, int alpha, int beta, int acc,
                          hipStream_t s) {
  const size_t bytes = force_lds_bytes<R, VISC, SHAPE>(entries);
  hipLaunchKernelGGL((kb_force<R, VISC, SHAPE>), dim3(nblocks), dim3(shape_nt(SHAPE)), bytes, s, b, alpha, beta,
                     acc);
}

template <int R, bool VISC>
static void batch_force_r(const BatchArgs &b, int nblocks, int shape, int entries, int alpha, int beta,
                          int acc, hipStream_t s) {
  if (shape == 1)
    batch_force_s<R, VISC, 1>(b, nblocks, entries, alpha, beta, acc, s);
  else if (shape == 2)
    batch_force_s<R, VISC, 2>(b, nblocks, entries, alpha, beta, acc, s);
  else
    batch_force_s<R, VISC, 0>(b, nblocks, entries, alpha, beta, acc, s);
}

void launch_batch_force(const BatchArgs &b, int nblocks, int R, int shape, bool visc, int entries, int alpha,
                        int beta, int acc, hipStream_t s) {
#define BF(RR)                                                                             \
  case RR:                                                                                 \
    if (visc) batch_force_r<RR, true>(b, nblocks, shape, entries, alpha, beta, acc, s);    \
    else batch_force_r<RR, false>(b, nblocks, shape, entries, alpha, beta, acc, s);        \
    break;
  switch (R) { BF(1) BF(2) BF(3) BF(4) BF(5) BF(6) BF(7) BF(8) default: break; }
#undef BF
}

template <int R>
static void batch_att_r(const BatchArgs &b, int nblocks, int alpha, int beta, hipStream_t s) {
  // one staged field and the table through scalar loads: at most 18 KB
  const size_t bytes = force_lds(3, R, FTY, 0, 1);
  hipLaunchKernelGGL((kb_force_att<R>), dim3(nblocks), dim3(FNT), bytes, s, b, alpha, beta);
}

void launch_batch_att(const BatchArgs &b, int nblocks, int R, int alpha, int beta, hipStream_t s) {
  switch (R) {
    case 1: batch_att_r<1>(b, nblocks, alpha, beta, s); break;
    case 2: batch_att_r<2>(b, nblocks, alpha, beta, s); break;
    case 3: batch_att_r<3>(b, nblocks, alpha, beta, s); break;
    case 4: batch_att_r<4>(b, nblocks, alpha, beta, s); break;
    case 5: batch_att_r<5>(b, nblocks, alpha, beta, s); break;
    case 6: batch_att_r<6>(b, nblocks, alpha, beta, s); break;
    case 7: batch_att_r<7>(b, nblocks, alpha, beta, s); break;
    default: batch_att_r<8>(b, nblocks, alpha, beta, s); break;
  }
}

void launch_batch_collide(const BatchArgs &b, int nblocks, int prec, int M, hipStream_t s) {
  if (prec == LBE_FP64)
    LBE_SWITCH_M(M, hipLaunchKernelGGL((kb_collide<double, MM>), dim3(nblocks), dim3(BLOCK), 0, s, b))
  else
    LBE_SWITCH_M(M, hipLaunchKernelGGL((kb_collide<float, MM>), dim3(nblocks), dim3(BLOCK), 0, s, b))
}

int diag_nblocks(const Geom &g) {
  int nb = (g.N + BLOCK - 1) / BLOCK;
  return nb < 1024 ? nb : 1024;
}

void launch_diag_partials(const Geom &g, int M, const uint32_t *bb, const Readout &r, const double *V,
                          double beta, double *partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_partials, dim3(nblocks), dim3(BLOCK), 0, s, g, M, bb, r, V, beta, partials);
}

void launch_diag_final(const double *partials, int nblocks, double *result, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, partials, nblocks, result);
}

void launch_diag_errn(const Geom &g, int M, const uint32_t *bb, const Readout &r, const double *V,
                      double beta, const double *result, double *partials, int nblocks,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_diag_errn, dim3(nblocks), dim3(BLOCK), 0, s, g, M, bb, r, V, beta, result,
                     partials);
}

// ------------------------------------------------------------------------
// adjoint launchers
// ------------------------------------------------------------------------

void launch_tape_moments(const StepArgs &a, int prec, const void *pop, double *PJ, hipStream_t s) {
  const dim3 gr = grid_for(a.g.N);
  if (prec == LBE_FP64)
    LBE_SWITCH_M(a.M, hipLaunchKernelGGL((k_tape_moments<double, MM>), gr, dim3(BLOCK), 0, s, a,
                                         (const double *)pop, PJ))
  else
    LBE_SWITCH_M(a.M, hipLaunchKernelGGL((k_tape_moments<float, MM>), gr, dim3(BLOCK), 0, s, a,
                                         (const float *)pop, PJ))
}

void launch_adj_collide(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  const dim3 gr = grid_for(a.g.N);
  LBE_SWITCH_M(a.M, hipLaunchKernelGGL(k_adj_collide<MM>, gr, dim3(BLOCK), 0, s, a, d))
}

void launch_adj_readout(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  const dim3 gr = grid_for(a.g.N);
  LBE_SWITCH_M(a.M, hipLaunchKernelGGL(k_adj_readout<MM>, gr, dim3(BLOCK), 0, s, a, d))
}

void launch_adj_stream(const StepArgs &a, const AdjArgs &d, bool terminal, hipStream_t s) {
  const dim3 gr = grid_for(a.g.N);
  if (terminal) {
    LBE_SWITCH_M(a.M, hipLaunchKernelGGL((k_adj_stream<MM, true>), gr, dim3(BLOCK), 0, s, a, d))
  } else {
    LBE_SWITCH_M(a.M, hipLaunchKernelGGL((k_adj_stream<MM, false>), gr, dim3(BLOCK), 0, s, a, d))
  }
}

// tiles of the adjoint gather of C^visc (MODE 5, eight staged fields):
// 512-thread 32 x 16 tiles where its two planes fit in LDS (reach up to 6;
// fewer window slots per thread and less halo per output) and the box still
// gives two such tiles per CU, else 32 x 8 (its planes fit for every reach).
// The sums do not depend on the tile.  An earlier split into two gathers
// (seven and five staged fields) took 1.03 + 0.86 ms at 128^3; the fused one
// saves 2% of the backward.
static bool wide_tiles(const StepArgs &a, int mode, int R) {
  return mode == 5 && force_lds(mode, R, 16, 0, 1) <= 160 * 1024 &&
         force_blocks(a.g, a.zchunk, 16) >= 2 * NCU;
}

template <int R, int SHAPE>
static void adj_force_launch_shape(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                                   hipStream_t s) {
  constexpr int NY = shape_ny(SHAPE), NT = shape_nt(SHAPE), TY = shape_ty(SHAPE);
  const int k = pair_index(a.M, alpha, beta);
  const size_t bytes = force_lds(2, R, TY, a.t.pair_nent[k], NY);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_adj_force<R, NY, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  const dim3 gr(force_blocks(a.g, a.zchunk, TY));
  hipLaunchKernelGGL((k_adj_force<R, NY, NT>), gr, dim3(NT), bytes, s, a, d, alpha, beta, acc);
}

// the adjoint gather stages five fields, like C^visc, for which the 32 x 8
// shape is the fast one (also at 128^3: 32 x 16 tiles of 512 threads gave
// the same time); zchunk and the tile order follow the box's tiling
template <int R>
static void adj_force_launch(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                             hipStream_t s) {
  adj_force_launch_shape<R, 0>(a, d, alpha, beta, acc, s);
}

template <int R, int NY>
static void adj_att_launch_rows(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                                hipStream_t s) {
  constexpr int TY = FNT / FTX * NY;
  const int k = pair_index(a.M, alpha, beta);
  const size_t bytes = force_lds(4, R, TY, a.t.att_nent[k], NY);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_adj_att<R, NY>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  hipLaunchKernelGGL((k_adj_att<R, NY>), dim3(force_blocks(a.g, a.zchunk, TY)), dim3(FNT), bytes, s, a, d,
                     alpha, beta, acc);
}

template <int R>
static void adj_att_launch(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                           hipStream_t s) {
  if (att_rows(a) == 1)
    adj_att_launch_rows<R, 1>(a, d, alpha, beta, acc, s);
  else
    adj_att_launch_rows<R, 2>(a, d, alpha, beta, acc, s);
}

static void adj_att_r(int R, const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                      hipStream_t s) {
  switch (R) {
    case 1: adj_att_launch<1>(a, d, alpha, beta, acc, s); break;
    case 2: adj_att_launch<2>(a, d, alpha, beta, acc, s); break;
    case 3: adj_att_launch<3>(a, d, alpha, beta, acc, s); break;
    case 4: adj_att_launch<4>(a, d, alpha, beta, acc, s); break;
    case 5: adj_att_launch<5>(a, d, alpha, beta, acc, s); break;
    case 6: adj_att_launch<6>(a, d, alpha, beta, acc, s); break;
    case 7: adj_att_launch<7>(a, d, alpha, beta, acc, s); break;
    default: adj_att_launch<8>(a, d, alpha, beta, acc, s); break;
  }
}

template <int R, int MODE, int NT>
static void adj_visc_launch_nt(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                               hipStream_t s) {
  constexpr int TY = NT / FTX;
  const int k = pair_index(a.M, alpha, beta);
  const size_t bytes = force_lds(MODE, R, TY, a.t.pair_nent[k], 1);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_adj_visc<R, MODE, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = bytes;
  }
  hipLaunchKernelGGL((k_adj_visc<R, MODE, NT>), dim3(force_blocks(a.g, a.zchunk, TY)), dim3(NT), bytes, s,
                     a, d, alpha, beta, acc);
}

template <int R, int MODE>
static void adj_visc_launch(const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                            hipStream_t s) {
  if (wide_tiles(a, MODE, R))
    adj_visc_launch_nt<R, MODE, 512>(a, d, alpha, beta, acc, s);
  else
    adj_visc_launch_nt<R, MODE, 256>(a, d, alpha, beta, acc, s);
}

template <int MODE>
static void adj_visc_r(int R, const StepArgs &a, const AdjArgs &d, int alpha, int beta, int acc,
                       hipStream_t s) {
  switch (R) {
    case 1: adj_visc_launch<1, MODE>(a, d, alpha, beta, acc, s); break;
    case 2: adj_visc_launch<2, MODE>(a, d, alpha, beta, acc, s); break;
    case 3: adj_visc_launch<3, MODE>(a, d, alpha, beta, acc, s); break;
    case 4: adj_visc_launch<4, MODE>(a, d, alpha, beta, acc, s); break;
    case 5: adj_visc_launch<5, MODE>(a, d, alpha, beta, acc, s); break;
    case 6: adj_visc_launch<6, MODE>(a, d, alpha, beta, acc, s); break;
    case 7: adj_visc_launch<7, MODE>(a, d, alpha, beta, acc, s); break;
    default: adj_visc_launch<8, MODE>(a, d, alpha, beta, acc, s); break;
  }
}

void launch_fill(double *p, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = (n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(BLOCK), 0, s, p, n, v);
}

// nbar of the step: the transposes of the shell gathers (every directed
// pair), of the attractive tails and of the contact values and ball averages.  The first launch that
// reaches an output writes it, later ones accumulate.
size_t adj_qp_sum_doubles(const Geom &g) { return (size_t)qp_small(g.nx, g.ny, g.nz).total; }

void launch_adj_quasipressure(const StepArgs &a, const AdjArgs &d, const int o[3], unsigned mode,
                              hipStream_t s) {
  const Geom &g = a.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz, M = a.M;
  const long long N = g.N, pl = (long long)nx * ny;
  const bool sym = mode & LBE_QP_SYMMETRIC;
  const double c6 = sym ? 1.0 / 6.0 : 1.0;
  const QpSmall q = qp_small(nx, ny, nz);
  const long long ns = q.total, vsp = 3 * N;
  double *sm = d.qpsum;
  double *vx = d.qpv, *vy = d.qpv + N, *vz = d.qpv + 2 * N;
  QpJobs J;
  int maxl = 0;
  auto reset = [&]() {
    memset(&J, 0, sizeof J);
    maxl = 0;
  };
  auto job = [&](const QpLines &ql, const double *in, double *out, double coef, int sum) {
    const int k = J.njobs++;
    J.q[k] = ql;
    J.in[k] = in;
    J.out[k] = out;
    J.coef[k] = coef;
    J.sum[k] = sum;
    maxl = std::max(maxl, ql.nlines);
  };
  auto run = [&]() {
    hipLaunchKernelGGL(k_adj_qp_jobs, dim3((maxl + BLOCK - 1) / BLOCK, M, J.njobs), dim3(BLOCK), 0, s, J);
  };
  // last legs along every line (2/6 of each axis, or z alone) and column sums
  reset();
  if (sym) {
    job({ny * nz, nx, o[0], ny * nz, nx, 0, 1, nx, 0, 1, N, vsp}, d.qpbar, vx, 2.0 * c6, 0);
    job({nx * nz, ny, o[1], nx, 1, pl, nx, 1, pl, nx, N, vsp}, d.qpbar, vy, 2.0 * c6, 0);
  }
  job({nx * ny, nz, o[2], (int)pl, 1, 0, pl, 1, 0, pl, N, vsp}, d.qpbar, vz, sym ? 2.0 * c6 : 1.0, 0);
  job({nx * ny, nz, 0, (int)pl, 1, 0, pl, 1, 0, 0, N, ns}, d.qpbar, sm + q.Cz, 0.0, 1);
  job({nx * nz, ny, 0, nx, 1, pl, nx, 1, nx, 0, N, ns}, d.qpbar, sm + q.Cy, 0.0, 1);
  job({ny * nz, nx, 0, ny * nz, nx, 0, 1, 1, 0, 0, N, ns}, d.qpbar, sm + q.Cx, 0.0, 1);
  run();
  // middle legs (from column sums) and plane sums
  reset();
  // (x,y,z): Cz(x, y) along y per x -> Pyz(x, y)
  job({nx, ny, o[1], nx, 1, 0, nx, 1, 0, nx, ns, ns}, sm + q.Cz, sm + q.Pyz, c6, 0);
  if (sym) {
    // (x,z,y): Cy(x, z) along z per x -> Pzy(x, z)
    job({nx, nz, o[2], nx, 1, 0, nx, 1, 0, nx, ns, ns}, sm + q.Cy, sm + q.Pzy, c6, 0);
    // (y,x,z): Cz(x, y) along x per y -> Pxz(x, y)
    job({ny, nx, o[0], ny, nx, 0, 1, nx, 0, 1, ns, ns}, sm + q.Cz, sm + q.Pxz, c6, 0);
    // (y,z,x): Cx(y, z) along z per y -> Pzx(y, z)
    job({ny, nz, o[2], ny, 1, 0, ny, 1, 0, ny, ns, ns}, sm + q.Cx, sm + q.Pzx, c6, 0);
    // (z,x,y): Cy(x, z) along x per z -> Pxy(x, z)
    job({nz, nx, o[0], nz, nx, 0, 1, nx, 0, 1, ns, ns}, sm + q.Cy, sm + q.Pxy, c6, 0);
    // (z,y,x): Cx(y, z) along y per z -> Pyx(y, z)
    job({nz, ny, o[1], nz, ny, 0, 1, ny, 0, 1, ns, ns}, sm + q.Cx, sm + q.Pyx, c6, 0);
  }
  // Sx(x) = sum_y Cz(x, y), Sy(y) = sum_x Cz(x, y), Sz(z) = sum_y Cx(y, z)
  job({nx, ny, 0, nx, 1, 0, nx, 1, 0, 0, ns, ns}, sm + q.Cz, sm + q.Sx, 0.0, 1);
  job({ny, nx, 0, ny, nx, 0, 1, 1, 0, 0, ns, ns}, sm + q.Cz, sm + q.Sy, 0.0, 1);
  job({nz, ny, 0, nz, ny, 0, 1, 1, 0, 0, ns, ns}, sm + q.Cx, sm + q.Sz, 0.0, 1);
  run();
  // first legs (from plane sums): 2/6 per axis, or x alone
  reset();
  job({1, nx, o[0], 1, 0, 0, 1, 0, 0, 1, ns, ns}, sm + q.Sx, sm + q.Lx, sym ? 2.0 * c6 : 1.0, 0);
  if (sym) {
    job({1, ny, o[1], 1, 0, 0, 1, 0, 0, 1, ns, ns}, sm + q.Sy, sm + q.Ly, 2.0 * c6, 0);
    job({1, nz, o[2], 1, 0, 0, 1, 0, 0, 1, ns, ns}, sm + q.Sz, sm + q.Lz, 2.0 * c6, 0);
  }
  run();
  LBE_SWITCH_M(M, hipLaunchKernelGGL(k_adj_qp_apply<MM>, grid_for(N), dim3(BLOCK), 0, s, a, d, o[0], o[1], o[2],
                                     sym ? 1 : 0, (mode & LBE_QP_WITH_FEXT) ? 1 : 0))
}

void launch_adj_nonlocal(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  const long long N = a.g.N;
  const int M = a.M, npairs = M * (M + 1) / 2;
  if (a.flags & LBE_IDEAL) {  // no force: densities enter only locally
    launch_fill(d.nbar, M * N, 0.0, s);
    return;
  }
  bool wn[MAXM] = {false, false, false, false}, wg[MAXPAIRS] = {};
  // with the drag, the collision (or read-out) adjoint has written Gbar
  if (M > 1 && (a.flags & LBE_DRAG))
    for (int k = 0; k < npairs; ++k) wg[k] = true;
  for (int al = 0; al < M; ++al)
    for (int be = 0; be < M; ++be) {
      const int k = pair_index(M, al, be);
      const int R = a.t.pair_R[k];
      if (R == 0) continue;  // empty shell
      const int acc = (wn[be] ? 1 : 0) | (wg[k] ? 2 : 0);
      wn[be] = wg[k] = true;
      switch (R) {
        case 1: adj_force_launch<1>(a, d, al, be, acc, s); break;
        case 2: adj_force_launch<2>(a, d, al, be, acc, s); break;
        case 3: adj_force_launch<3>(a, d, al, be, acc, s); break;
        case 4: adj_force_launch<4>(a, d, al, be, acc, s); break;
        case 5: adj_force_launch<5>(a, d, al, be, acc, s); break;
        case 6: adj_force_launch<6>(a, d, al, be, acc, s); break;
        case 7: adj_force_launch<7>(a, d, al, be, acc, s); break;
        default: adj_force_launch<8>(a, d, al, be, acc, s); break;
      }
    }
  // C^visc: its transpose per directed pair, into nbar, Gbar and Jnl
  if ((a.flags & LBE_VISC) && d.Jnl) {
    bool wj[MAXM] = {false, false, false, false};
    for (int al = 0; al < M; ++al)
      for (int be = 0; be < M; ++be) {
        const int k = pair_index(M, al, be);
        const int R = a.t.pair_R[k];
        if (R == 0) continue;
        adj_visc_r<5>(R, a, d, al, be, (wn[be] ? 1 : 0) | (wg[k] ? 2 : 0) | (wj[be] ? 4 : 0), s);
        wn[be] = wg[k] = wj[be] = true;
      }
    for (int b = 0; b < M; ++b)
      if (!wj[b]) launch_fill(d.Jnl + 3 * b * N, 3 * N, 0.0, s);
  }
  // the attractive tails: phibar_a gathered back onto n_b
  for (int al = 0; al < M; ++al)
    for (int be = 0; be < M; ++be) {
      const int R = a.t.att_R[pair_index(M, al, be)];
      if (R == 0) continue;
      adj_att_r(R, a, d, al, be, wn[be] ? 1 : 0, s);
      wn[be] = true;
    }
  for (int b = 0; b < M; ++b)
    if (!wn[b]) launch_fill(d.nbar + b * N, N, 0.0, s);
  for (int k = 0; k < npairs; ++k)
    if (!wg[k]) launch_fill(d.Gbar + k * N, N, 0.0, s);
  ball_launch<1>(a, d, s);
  ball_launch<2>(a, d, s);
}

void launch_pad_fields(const Geom &g, const uint32_t *bb, int nf, const double *in, double *out, hipStream_t s) {
  launch_fill(out, (long long)nf * g.Np, 0.0, s);
  hipLaunchKernelGGL(k_pad_fields, grid_for(g.N), dim3(BLOCK), 0, s, g, bb, nf, in, out);
}

void launch_unpad_fields(const Geom &g, int nf, const double *in, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_unpad_fields, grid_for(g.N), dim3(BLOCK), 0, s, g, nf, in, out);
}

void launch_pull_f64(const Geom &g, const uint32_t *bb, int blocks, const double *pre, double *out,
                     hipStream_t s) {
  const long long Ns = ((long long)g.N + 63) / 64 * 64;
  for (int b = 0; b < blocks; ++b)
    hipLaunchKernelGGL(k_pull<double>, grid_for(g.N), dim3(BLOCK), 0, s, g, bb, pre + (long long)b * Q * Ns,
                       out + (long long)b * Q * Ns, Ns);
}

void launch_adj_shell(const StepArgs &a, const AdjArgs &d, hipStream_t s) {
  bool wn[MAXM] = {false, false, false, false}, wg[MAXPAIRS] = {};
  for (int al = 0; al < a.M; ++al)
    for (int be = 0; be < a.M; ++be) {
      const int k = pair_index(a.M, al, be);
      const int R = a.t.pair_R[k];
      if (R == 0) continue;
      const int acc = (wn[be] ? 1 : 0) | (wg[k] ? 2 : 0);
      wn[be] = wg[k] = true;
      switch (R) {
        case 1: adj_force_launch<1>(a, d, al, be, acc, s); break;
        case 2: adj_force_launch<2>(a, d, al, be, acc, s); break;
        case 3: adj_force_launch<3>(a, d, al, be, acc, s); break;
        case 4: adj_force_launch<4>(a, d, al, be, acc, s); break;
        case 5: adj_force_launch<5>(a, d, al, be, acc, s); break;
        case 6: adj_force_launch<6>(a, d, al, be, acc, s); break;
        case 7: adj_force_launch<7>(a, d, al, be, acc, s); break;
        default: adj_force_launch<8>(a, d, al, be, acc, s); break;
      }
    }
  const long long N = a.g.N;
  for (int b = 0; b < a.M; ++b)
    if (!wn[b]) launch_fill(d.nbar + b * N, N, 0.0, s);
  for (int k = 0; k < a.M * (a.M + 1) / 2; ++k)
    if (!wg[k]) launch_fill(d.Gbar + k * N, N, 0.0, s);
}

void launch_adj_extforce(const Geom &g, const double *Fbar, double *Vbar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_extforce, grid_for(g.N), dim3(BLOCK), 0, s, g, Fbar, Vbar);
}

void launch_adj_state_grad(const Geom &g, int M, const uint32_t *bb, const double *mu, int species,
                           int dist, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_state_grad, grid_for(g.N), dim3(BLOCK), 0, s, g, M, bb, mu, species, dist,
                     out);
}


void launch_divergence(const Geom &g, const uint32_t *bb, const double *u, double kT, double *out,
                       hipStream_t s) {
  // 1/v_T^2 of the stencil times 1/v_T of the normalisation (dx = 1)
  const double scale = 1.0 / (kT * sqrt(kT));
  hipLaunchKernelGGL(k_divergence, grid_for(g.N), dim3(BLOCK), 0, s, g, bb, u, scale, out);
}

void launch_quasipressure(const StepArgs &a, const int o[3], unsigned mode, bool phi_only, double *scan,
                          double *pi, hipStream_t s) {
  const Geom &g = a.g;
  const int fext = (mode & LBE_QP_WITH_FEXT) ? 1 : 0;
  const int rows = g.ny * g.nz;
  hipLaunchKernelGGL(k_qp_scan_x, dim3((rows + 3) / 4, a.M), dim3(256), 0, s, a, o[0], fext, scan);
  const QpScan qy = qp_scan_of(g, 1, o[1], fext);
  const QpScan qz = qp_scan_of(g, 2, o[2], fext);
  for (const QpScan &q : {qy, qz})
    hipLaunchKernelGGL(k_qp_scan, dim3((q.nlines + QP_LANES - 1) / QP_LANES, a.M), dim3(QP_LANES * QP_SEG), 0,
                       s, a, q, scan);
  hipLaunchKernelGGL(k_qp_combine, dim3((g.N + BLOCK - 1) / BLOCK, a.M), dim3(BLOCK), 0, s, a, scan, o[0],
                     o[1], o[2], (mode & LBE_QP_SYMMETRIC) ? 1 : 0, phi_only ? 0 : 1, pi);
}

int qp_blocks(const Geom &g, int axis) {
  if (axis == 0) return (g.ny * g.nz + 3) / 4;
  return (qp_scan_of(g, axis, 0, 0).nlines + QP_LANES - 1) / QP_LANES;
}

void launch_batch_quasipressure(const BatchArgs &nodes, int node_nblocks, const QpRoute *routes,
                                const QpBatchTables &t, int M, hipStream_t s) {
  BatchArgs b = nodes;
  b.blockbox = t.box[0];
  b.blockstart = t.start[0];
  hipLaunchKernelGGL(kb_qp_scan_x, dim3(t.nblocks[0], M), dim3(256), 0, s, b, routes);
  for (int axis = 1; axis <= 2; ++axis) {
    b.blockbox = t.box[axis];
    b.blockstart = t.start[axis];
    hipLaunchKernelGGL(kb_qp_scan, dim3(t.nblocks[axis], M), dim3(QP_LANES * QP_SEG), 0, s, b, routes, axis);
  }
  hipLaunchKernelGGL(kb_qp_combine, dim3(node_nblocks, M), dim3(BLOCK), 0, s, nodes, routes);
}

void launch_qp_apply(const StepArgs &a, const Readout &r, const double *pi, int species, int prec,
                     void *gstage, hipStream_t s) {
  const long long Ns = ((long long)a.g.N + 63) / 64 * 64;
  if (prec == LBE_FP64)
    hipLaunchKernelGGL(k_qp_apply<double>, grid_for(a.g.N), dim3(BLOCK), 0, s, a, r, pi, species,
                       (double *)gstage, Ns);
  else
    hipLaunchKernelGGL(k_qp_apply<float>, grid_for(a.g.N), dim3(BLOCK), 0, s, a, r, pi, species,
                       (float *)gstage, Ns);
}

#undef LBE_SWITCH_M

}  // namespace lbe
