"""Pins of the oracle's velocity divergence D = div u / (v_T/dx) (Sec. 4.3, the
channel validation) against closed forms.  The populations of an ideal gas
with no force are set to w_p n0 (1 + c_p.u/v_T^2), so that the inversion
returns exactly the prescribed u; the isotropic D3Q19 divergence is then a
central difference along each axis, with u = 0 beyond walls."""
import math

import numpy as np

KT = 1.0 / 3.0
VT = math.sqrt(KT)


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


def _with_velocity(o_lib, nx, ny, nz, u, periodic=7, n0=0.01, flags=None):
    o = o_lib.Oracle(nx, ny, nz, [1.0], periodic=periodic,
                     flags=o_lib.LBEO_IDEAL if flags is None else flags)
    c, w, _ = o_lib.d3q19()
    cu = np.tensordot(c.astype(float), u, axes=(1, 0))          # (19, nz, ny, nx)
    pops = n0 * w[:, None, None, None] * (1.0 + cu / KT)
    o.set_populations(0, 0, pops)
    o.set_populations(0, 1, pops)
    return o


def test_longitudinal_wave_gives_the_central_difference(oracle_lib):
    """u = (A sin k_x x, 0, B sin k_z z) in a periodic box: the prescribed
    velocity comes back (to rounding), and D = (A sin k_x cos k_x x +
    B sin k_z cos k_z z) / v_T, the central difference of each component."""
    nx, ny, nz = 16, 6, 12
    x, y, z = _grid(nx, ny, nz)
    kx, kz = 2 * math.pi / nx, 2 * math.pi / nz
    A, B = 1e-3, -2e-3
    u = np.stack([A * np.sin(kx * x), np.zeros_like(x, dtype=float), B * np.sin(kz * z)])
    o = _with_velocity(oracle_lib, nx, ny, nz, u)
    assert np.abs(o.velocity(-1) - u).max() < 1e-13 * abs(B)
    ref = (A * math.sin(kx) * np.cos(kx * x) + B * math.sin(kz) * np.cos(kz * z)) / VT
    assert np.abs(o.divergence() - ref).max() < 1e-15


def test_transverse_shear_has_no_divergence(oracle_lib):
    """u = (A sin ky, 0, 0): solenoidal, and the diagonal links of the D3Q19
    stencil cancel pairwise, so D = 0 to rounding."""
    nx, ny, nz = 8, 16, 6
    x, y, z = _grid(nx, ny, nz)
    u = np.stack([1e-3 * np.sin(2 * math.pi * y / ny), np.zeros(x.shape), np.zeros(x.shape)])
    o = _with_velocity(oracle_lib, nx, ny, nz, u)
    assert np.abs(o.divergence()).max() < 1e-19


def test_walls_contribute_zero_velocity(oracle_lib):
    """Walls beyond y = 0 and y = ny - 1 (periodic x, z).  With u_y =
    A sin(pi (y+1)/(ny+1)), which vanishes at y = -1 and y = ny, the central
    difference holds on every row, including the rows next to the walls:
    D = A sin(pi/(ny+1)) cos(pi (y+1)/(ny+1)) / v_T."""
    nx, ny, nz = 6, 14, 5
    x, y, z = _grid(nx, ny, nz)
    A = 2e-3
    q = math.pi / (ny + 1)
    u = np.stack([np.zeros(x.shape), A * np.sin(q * (y + 1)), np.zeros(x.shape)])
    o = _with_velocity(oracle_lib, nx, ny, nz, u, periodic=1 | 4)
    ref = A * math.sin(q) * np.cos(q * (y + 1)) / VT
    assert np.abs(o.divergence() - ref).max() < 1e-15


def test_solid_nodes(oracle_lib):
    """A solid slab: D = 0 on it, and its nodes count as u = 0 for their
    neighbours (a uniform flow into the slab has D = -A/(2 v_T) in front of
    it and +A/(2 v_T) behind it, zero elsewhere)."""
    nx, ny, nz = 12, 4, 4
    x, y, z = _grid(nx, ny, nz)
    A = 1e-3
    solid = (x == 6).astype(np.uint8)
    u = np.stack([np.where(solid == 1, 0.0, A), np.zeros(x.shape), np.zeros(x.shape)])
    o = _with_velocity(oracle_lib, nx, ny, nz, u)
    o.set_solid(solid)
    c, w, _ = oracle_lib.d3q19()
    cu = np.tensordot(c.astype(float), u, axes=(1, 0))
    pops = 0.01 * w[:, None, None, None] * (1.0 + cu / KT) * (1 - solid)
    o.set_populations(0, 0, pops)
    o.set_populations(0, 1, pops)
    D = o.divergence()
    ref = np.zeros(x.shape)
    ref[x == 5] = -A / (2 * VT)
    ref[x == 7] = A / (2 * VT)
    assert np.abs(D - ref).max() < 1e-15
