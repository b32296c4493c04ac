"""Seeded synthetic inputs for the Lattice Boltzmann-Enskog step.

This module generates problem set-ups only: initial densities, the cosine
potential well of Sec. 4.1 (eq. extpotential), solid masks of a channel with a
bottleneck (Sec. 4.3) and the smooth random potentials used by the gradient
check.  It contains none of the method's arithmetic, so both the GPU library's
tests and the CPU oracle's tests draw their inputs from here.

Arrays are numpy, shaped (nz, ny, nx) so that the flat index is
x + nx*(y + ny*z).  Random numbers come from numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

KT = 1.0 / 3.0          # k_B T = v_T^2 for D3Q19 with m = 1
PERIODIC_ALL = 7        # bit0 x, bit1 y, bit2 z
PERIODIC_XZ = 1 | 4


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    sigma: List[float]
    periodic: int = PERIODIC_ALL
    tau: float = 1.0
    kT: float = KT
    steps: int = 1
    density: List[np.ndarray] = field(default_factory=list)
    V: Optional[np.ndarray] = None
    solid: Optional[np.ndarray] = None
    body: List[List[float]] = field(default_factory=list)
    att_eps: Optional[list] = None      # attractive tail depths (M x M), None = none
    att_rc: float = 0.0                 # its cutoff
    # route of the per-step quasi-pressure: ((x0, y0, z0), mode bits), None =
    # the library default (box centre, mean over the six axis orders)
    qp_route: Optional[tuple] = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nspecies(self) -> int:
        return len(self.sigma)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def noisy_uniform(shape, n0: float, amp: float, seed: int) -> np.ndarray:
    """n0 * (1 + U[-amp, amp]) on every node (amp = 0 gives a uniform field)."""
    if amp == 0.0:
        return np.full(shape, n0, dtype=np.float64)
    return n0 * (1.0 + rng(seed).uniform(-amp, amp, size=shape))


def cosine_well(shape, xi: float, eps: float, center=None) -> np.ndarray:
    """U = -eps (1 + cos(pi r / xi)) for r < xi, else 0 (Sec. 4.1,
    eq. extpotential); r is the Euclidean distance to a lattice node at the
    box centre (no periodic image)."""
    nz, ny, nx = shape
    if center is None:
        center = (nx // 2, ny // 2, nz // 2)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    V = np.where(r < xi, -eps * (1.0 + np.cos(np.pi * r / xi)), 0.0)
    return V.astype(np.float64)


def bottleneck_mask(nx, ny, nz, x0, x1, gap_lo, gap_hi) -> np.ndarray:
    """Solid nodes of a channel constriction: x0 <= x < x1 and y outside
    [gap_lo, gap_hi).  The channel walls themselves lie just beyond y = 0 and
    y = ny - 1 (non-periodic y)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = (x >= x0) & (x < x1) & ((y < gap_lo) | (y >= gap_hi))
    return m.astype(np.uint8)


def smooth_field(shape, amp: float, nmodes: int, seed: int) -> np.ndarray:
    """Sum of nmodes random low-wavenumber Fourier modes, scaled to max |.| = amp."""
    nz, ny, nx = shape
    g = rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(nmodes):
        k = g.integers(0, 3, size=3)
        if not k.any():
            k[0] = 1
        phase = g.uniform(0, 2 * np.pi)
        a = g.uniform(0.5, 1.0)
        out += a * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + phase)
    m = np.abs(out).max()
    return amp * out / m if m > 0 else out


def packing_density(eta: float, sigma: float) -> float:
    """Number density of one species at packing fraction eta = (pi/6) n sigma^3."""
    return 6.0 * eta / (math.pi * sigma ** 3)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------
def well_box(L: int, sigma: float, nsig3: float, eps_kT: float, xi: float,
             noise: float, seed: int, steps: int, name: str = "well") -> Workload:
    """One-component hard spheres in a periodic cube with a cosine well at
    the centre: n = nsig3 / sigma^3 (1 + noise); eps_kT is the amplitude eps
    of eq. (extpotential) in kT units (the well is 2 eps deep)."""
    shape = (L, L, L)
    n0 = nsig3 / sigma ** 3
    return Workload(
        name=name, nx=L, ny=L, nz=L, sigma=[float(sigma)], steps=steps,
        density=[noisy_uniform(shape, n0, noise, seed)],
        V=cosine_well(shape, xi, eps_kT * KT), body=[[0.0, 0.0, 0.0]])


def eps_for_depth(depth_kT: float) -> float:
    """A well "depth D kT": eps = D in eq. (extpotential), which Sec. 4.1
    calls the potential depth (U(0) = -2 eps)."""
    return depth_kT


def c1_small_well() -> Workload:
    """32^3 periodic, sigma = 4, n sigma^3 = 0.3 with +-1e-3 noise (seed 1202),
    well radius 8 and depth 1 kT, 50 steps."""
    return well_box(32, 4.0, 0.3, eps_for_depth(1.0), 8.0, 1e-3, 1202, 50, "well32_s4")


def c2_large_well() -> Workload:
    """128^3 periodic, sigma = 6, n sigma^3 = 0.4, well radius 24 and depth
    2 kT, 2000 steps (no noise)."""
    return well_box(128, 6.0, 0.4, eps_for_depth(2.0), 24.0, 0.0, 0, 2000, "well128_s6")


def channel(nx=256, ny=64, nz=32, x0=112, x1=144, gap=24, sigma=(4.0, 6.0),
            eta=0.25, xA=0.5, force=1e-5, steps=5000, name=None) -> Workload:
    """Two-component channel with a bottleneck: walls beyond y in [0, ny-1],
    periodic x and z, a constriction of `gap` fluid sites over x0 <= x < x1,
    total packing fraction eta at mole fraction xA, body force along x."""
    sA, sB = sigma
    ntot = 6.0 * eta / (math.pi * (xA * sA ** 3 + (1 - xA) * sB ** 3))
    shape = (nz, ny, nx)
    lo = (ny - gap) // 2
    solid = bottleneck_mask(nx, ny, nz, x0, x1, lo, lo + gap)
    # quasi-pressure path: from the centre of the gap along x (the channel
    # axis, fluid all the way), then y, then z, so that no leg crosses the
    # obstacle; paths that start along y or z would
    return Workload(
        name=name or f"channel{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
        sigma=[sA, sB], periodic=PERIODIC_XZ, steps=steps,
        density=[np.full(shape, xA * ntot), np.full(shape, (1 - xA) * ntot)],
        V=np.zeros(shape), solid=solid,
        body=[[force, 0.0, 0.0], [force, 0.0, 0.0]],
        qp_route=((nx // 2, lo + gap // 2, nz // 2), 0))


def c3_channel() -> Workload:
    """256x64x32, sigma_A = 4, sigma_B = 6, x_A = 0.5, eta = 0.25, 24-site gap
    over 112 <= x < 144, body force 1e-5 along x, 5000 steps."""
    return channel()


def c5_channel() -> Workload:
    """96x32x32 channel, gap solid for 42 <= x < 54 and (y < 10 or y >= 22),
    400 steps; base potential a smooth 4-mode field of amplitude 0.1 kT."""
    w = channel(nx=96, ny=32, nz=32, x0=42, x1=54, gap=12, steps=400,
                name="channel96x32x32")
    w.V = smooth_field(w.shape, 0.1 * KT, 4, 1203)
    return w


def c4_boxes(count: int = 96, seed: int = 3842, steps: int = 500,
             Lmin: int = 24, Lmax: int = 96) -> List[Workload]:
    """Independent one-component boxes: edge L ~ U{Lmin..Lmax},
    sigma ~ {3, 4, 6}, n sigma^3 ~ U[0.1, 0.45], well depth ~ U[0.5, 3] kT,
    well radius L/4 at the centre, +-1e-3 density noise."""
    g = rng(seed)
    out = []
    for b in range(count):
        L = int(g.integers(Lmin, Lmax + 1))
        sigma = float(g.choice([3.0, 4.0, 6.0]))
        nsig3 = float(g.uniform(0.1, 0.45))
        depth = float(g.uniform(0.5, 3.0))
        out.append(well_box(L, sigma, nsig3, eps_for_depth(depth), L / 4.0, 1e-3, seed + 1 + b,
                            steps, name=f"box{b}"))
    return out


# --------------------------------------------------------------------------
# The gradient check on the channel: an objective of the final state whose
# gradient with respect to the potential V(r) the adjoint computes.
# --------------------------------------------------------------------------
FLUX_PLANE_X = 48


def c5_objective(w: Workload):
    """Inputs of the objective on the 96x32x32 channel after w.steps steps,
        L = sum_{fluid r} (n_A(r) - n_t(r))^2 + sum_{r in plane} sum_a J_x^a(r),
    with the target n_t = n_A0 (1 + 0.05 s(r)), s a 4-mode smooth field of
    unit amplitude (seed 1204), and the plane the fluid nodes of x = 48 (the
    middle of the constriction).  Returns (n_t, fluid_mask, plane_mask)."""
    s = smooth_field(w.shape, 1.0, 4, 1204)
    n_t = w.density[0] * (1.0 + 0.05 * s)
    fluid = (w.solid == 0) if w.solid is not None else np.ones(w.shape, dtype=bool)
    plane = np.zeros(w.shape, dtype=bool)
    plane[:, :, FLUX_PLANE_X] = True
    return n_t, fluid, plane & fluid


def sample_fluid_nodes(w: Workload, count: int = 32, seed: int = 1205) -> np.ndarray:
    """Flat indices of `count` distinct fluid nodes drawn with a fixed seed."""
    fluid = np.flatnonzero((w.solid.reshape(-1) == 0) if w.solid is not None
                           else np.ones(w.nodes, dtype=bool))
    return np.sort(rng(seed).choice(fluid, size=count, replace=False))
