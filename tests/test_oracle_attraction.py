"""Pins of the oracle's attractive molecular field G^{ab} (Appendix, the last
term of C^{a,mf}), with the attractive r^-6 tail U = -eps (sigma_ab/r)^6 on
sigma_ab <= r < rc chosen for U (the paper leaves it open) and g = 1 there:
* the uniform state stays an exact fixed point;
* G equals an O(N^2) brute-force sum over all node pairs with minimum-image
  distances (a separate loop with its own distance test);
* long density waves: the lattice sum tends to the continuum integral of
  U' r^3, done in closed form;
* the mixture keeps total momentum (Newton's third law for U^{ab} = U^{ba})."""
import math

import numpy as np
import pytest

from paper_1202_3842_amd import workloads as W

KT = 1.0 / 3.0


def _oracle(o_lib, shape, sigma, eps, rc, flags=0, periodic=7):
    nz, ny, nx = shape
    return o_lib.Oracle(nx, ny, nz, sigma, periodic=periodic, flags=flags, att_eps=eps, att_rc=rc)


def test_uniform_state_is_a_fixed_point_with_attraction(oracle_lib):
    sh = (10, 11, 12)
    for sigma, eps in (([2.0], [[0.5 * KT]]), ([2.0, 3.0], [[0.3 * KT, 0.2 * KT], [0.2 * KT, 0.4 * KT]])):
        o = _oracle(oracle_lib, sh, sigma, eps, 4.5, flags=oracle_lib.LBEO_VISC)
        for a in range(len(sigma)):
            o.init_density(a, np.full(sh, 0.01 / (a + 1)))
        f0 = [o.populations(a, d) for a in range(len(sigma)) for d in (0, 1)]
        o.step(3)
        f1 = [o.populations(a, d) for a in range(len(sigma)) for d in (0, 1)]
        for x, y in zip(f0, f1):
            assert np.array_equal(x, y)


def _brute_force_G(n, sab, eps, rc):
    """G(r) = sum over all nodes r' with sigma_ab <= |d| < rc, d = r' - r the
    minimum-image displacement, of U'(|d|) d/|d| n(r')."""
    nz, ny, nx = n.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    dims = np.array([nx, ny, nz])
    nf = n.ravel()
    G = np.zeros((3, n.size))
    for i in range(n.size):
        d = pos - pos[i]
        d -= dims * np.round(d / dims).astype(int)
        r = np.sqrt((d ** 2).sum(axis=1))
        m = (r >= sab) & (r < rc)
        dU = 6.0 * eps * sab ** 6 / r[m] ** 7
        G[:, i] = ((dU / r[m] * nf[m])[:, None] * d[m]).sum(axis=0)
    return G.reshape((3,) + n.shape)


def test_attraction_equals_brute_force_pair_sum(oracle_lib):
    """One species sigma = 2, eps = kT/2, rc = 4.5 on a 12^3 periodic box
    (larger than 2 rc, so minimum images are unique) with a random density:
    the oracle's C^mf with attraction minus without, divided by n, is G."""
    sh = (12, 12, 12)
    eps, rc, sab = 0.5 * KT, 4.5, 2.0
    n = W.noisy_uniform(sh, 0.02, 0.3, 4242)
    with_att = _oracle(oracle_lib, sh, [sab], [[eps]], rc)
    without = _oracle(oracle_lib, sh, [sab], [[0.0]], rc)
    for o in (with_att, without):
        o.init_density(0, n)
    G = (with_att.forces(0)[0] - without.forces(0)[0]) / n
    ref = _brute_force_G(n, sab, eps, rc)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(G - ref).max() < 1e-12 * scale


def test_long_wavelength_limit_of_the_attraction(oracle_lib):
    """n = n0 (1 + A cos kx): for k rc << 1 the lattice sum becomes the
    continuum one, G_x -> (4 pi/3) (int_sigma^rc U'(r) r^3 dr) dn/dx, and for
    the r^-6 tail the integral is 2 eps sigma^3 (1 - (sigma/rc)^3) in closed
    form.  (The force comes from U' inside [sigma, rc) only: the jumps of the
    truncated U at the core and at rc add nothing.)  Compared at k rc = 0.2;
    the lattice thick shell over-weights its inner edge, where U' ~ r^-7 is
    largest, by about 6%."""
    sab, eps, rc = 4.0, 0.5 * KT, 8.0
    L = int(round(2 * math.pi * rc / 0.2))
    sh = (2, 2, L)                      # n varies along x only
    x = np.broadcast_to(np.arange(L), sh)
    k = 2 * math.pi / L
    n0, A = 0.01, 1e-3
    n = n0 * (1 + A * np.cos(k * x))
    with_att = _oracle(oracle_lib, sh, [sab], [[eps]], rc)
    without = _oracle(oracle_lib, sh, [sab], [[0.0]], rc)
    for o in (with_att, without):
        o.init_density(0, n)
    Gx = ((with_att.forces(0)[0] - without.forces(0)[0]) / n)[0, 0, 0]
    xs = np.arange(L)
    coef = (4 * math.pi / 3) * 2 * eps * sab ** 3 * (1 - (sab / rc) ** 3)
    ref = coef * (-n0 * A * k * np.sin(k * xs))
    amp = (Gx @ np.sin(k * xs)) / (ref @ np.sin(k * xs))
    assert 1.0 < amp < 1.1, amp


def test_mixture_with_attraction_conserves_momentum(oracle_lib):
    """Two species, unequal eps, random densities, periodic box, no external
    force: the total g-momentum stays zero over the steps (C^visc off, whose
    cross-species terms alone do not conserve it)."""
    sh = (12, 10, 11)
    eps = [[0.4 * KT, 0.25 * KT], [0.25 * KT, 0.3 * KT]]
    o = _oracle(oracle_lib, sh, [2.0, 3.0], eps, 5.0)
    o.init_density(0, W.noisy_uniform(sh, 0.02, 0.2, 5))
    o.init_density(1, W.noisy_uniform(sh, 0.01, 0.2, 6))
    scale = 0.03 * math.sqrt(KT)
    for _ in range(4):
        o.step(2)
        d = o.diagnostics()
        assert max(abs(v) for v in d["gmom"]) < 1e-13 * scale * np.prod(sh)
    assert o.diagnostics()["umax"] > 1e-8     # the attraction does move the fluid


def test_attraction_arguments(oracle_lib):
    with pytest.raises(oracle_lib.OracleError):
        _oracle(oracle_lib, (8, 8, 8), [2.0, 3.0], [[0.1, 0.2], [0.1, 0.1]], 5.0)  # not symmetric
    with pytest.raises(oracle_lib.OracleError):
        _oracle(oracle_lib, (8, 8, 8), [2.0], [[-0.1]], 5.0)                      # negative
    with pytest.raises(oracle_lib.OracleError):
        _oracle(oracle_lib, (8, 8, 8), [4.0], [[0.1]], 3.0)                       # rc <= sigma
    with pytest.raises(oracle_lib.OracleError):
        _oracle(oracle_lib, (8, 8, 8), [2.0], [[0.1]], 5.0, flags=oracle_lib.LBEO_IDEAL)
