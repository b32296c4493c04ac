"""Pins of the oracle's tables: D3Q19 quadrature, lattice shells, balls and
contact values, checked against what mathematics fixes (moment identities,
rotational symmetry, closed forms) rather than against retyped formulas."""
import itertools
import math

import numpy as np
import pytest


def test_d3q19_quadrature_moments(oracle_lib):
    """The velocity set is a Gauss-Hermite quadrature (Sec. 3): its weights
    reproduce the Maxwellian moments up to fourth order with v_T^2 = 1/3."""
    c, w, opp = oracle_lib.d3q19()
    c = c.astype(float)
    vt2 = 1.0 / 3.0
    I = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(np.einsum("p,pi->i", w, c)).max() < 1e-16
    assert np.abs(np.einsum("p,pi,pj->ij", w, c, c) - vt2 * I).max() < 1e-15
    assert np.abs(np.einsum("p,pi,pj,pk->ijk", w, c, c, c)).max() < 1e-16
    m4 = np.einsum("p,pi,pj,pk,pl->ijkl", w, c, c, c, c)
    iso = vt2 ** 2 * (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I)
                      + np.einsum("il,jk->ijkl", I, I))
    assert np.abs(m4 - iso).max() < 1e-15
    # opposite directions
    assert np.array_equal(c[opp], -c)
    assert len({tuple(v) for v in c}) == 19


def _cubic_group():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            m = np.zeros((3, 3), dtype=int)
            for i, j in enumerate(perm):
                m[i, j] = signs[i]
            mats.append(m)
    return mats


@pytest.mark.parametrize("sigma,count", [(3, 98), (4, 210), (5, 350), (6, 450), (8, 762)])
def test_shell_geometry(oracle_lib, sigma, count):
    """Shell of radius sigma (Appendix integral over the unit sphere): the set
    is closed under the 48 cubic symmetries, the second half mirrors the first,
    and the weighted first moment equals the continuum value
    int dk k_i (sigma k_j) = (4 pi / 3) sigma delta_ij exactly."""
    offs, w = oracle_lib.shell(sigma)
    assert len(offs) == count
    half = count // 2
    assert np.array_equal(offs[half:], -offs[:half])
    S = {tuple(v) for v in offs}
    assert len(S) == count
    for m in _cubic_group():
        assert {tuple(m @ np.array(v)) for v in S} == S
    r = np.linalg.norm(offs, axis=1)
    assert (r >= sigma - 0.5).all() and (r < sigma + 0.5).all()
    # brute-force count of all lattice points in the annulus
    K = int(math.ceil(sigma + 0.5))
    g = np.arange(-K, K + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    assert int(((R >= sigma - 0.5) & (R < sigma + 0.5)).sum()) == count
    ehat = offs / r[:, None]
    m1 = w * np.einsum("pi,pj->ij", offs.astype(float), ehat)
    assert np.abs(m1 - 4 * np.pi / 3 * sigma * np.eye(3)).max() < 1e-12
    # the fourth angular moment is close to the isotropic 1/5 (a few percent)
    m4 = (w / (4 * np.pi * sigma)) * (r * ehat[:, 0] ** 4).sum()
    assert abs(m4 / (1.0 / 5.0) - 1.0) < 0.05


@pytest.mark.parametrize("sigma,count", [(3, 19), (4, 33), (5, 81), (6, 123)])
def test_ball_counts(oracle_lib, sigma, count):
    """Averaging ball of radius sigma/2 used for the weighted density."""
    offs = oracle_lib.ball(sigma)
    assert len(offs) == count
    assert (np.linalg.norm(offs, axis=1) <= sigma / 2 + 1e-12).all()
    assert {tuple(v) for v in offs} == {tuple(-v) for v in offs}


def _cs(eta):
    """Carnahan-Starling contact value (textbook closed form)."""
    return (1 - eta / 2) / (1 - eta) ** 3


@pytest.mark.parametrize("eta", [0.0, 0.05, 0.1571, 0.2094, 0.25, 0.34, 0.45])
def test_bmcsl_reduces_to_carnahan_starling(oracle_lib, eta):
    """One species: the BMCSL contact value is the Carnahan-Starling one,
    and a binary mixture of equal diameters gives the same value for every
    pair at the same total packing fraction."""
    s = 4.0
    n = 6 * eta / (math.pi * s ** 3)
    assert abs(oracle_lib.bmcsl([s], [n], 0, 0) - _cs(eta)) < 1e-13 * _cs(eta)
    for xa in (0.3, 0.5):
        for a, b in ((0, 0), (0, 1), (1, 1)):
            g = oracle_lib.bmcsl([s, s], [xa * n, (1 - xa) * n], a, b)
            assert abs(g - _cs(eta)) < 1e-13 * _cs(eta)


def test_bmcsl_limits(oracle_lib):
    """BMCSL: symmetric in the pair, and a vanishing second diameter leaves
    the big spheres' contact value at CS of their own packing fraction
    (the point particles occupy no volume)."""
    sa, sb = 6.0, 4.0
    nb = [1e-3, 2e-3]
    assert oracle_lib.bmcsl([sa, sb], nb, 0, 1) == oracle_lib.bmcsl([sa, sb], nb, 1, 0)
    eta_a = math.pi / 6 * sa ** 3 * 1e-3
    g = oracle_lib.bmcsl([sa, 0.0], [1e-3, 5e-2], 0, 0)
    assert abs(g - _cs(eta_a)) < 1e-13
    # point-particle/big-sphere contact is the "ideal-wall" limit 1/(1-eta)
    g = oracle_lib.bmcsl([sa, 0.0], [1e-3, 5e-2], 0, 1)
    assert abs(g - 1 / (1 - eta_a)) < 1e-13


@pytest.mark.parametrize("seed", range(6))
def test_bmcsl_contact_values_give_the_bmcsl_pressure(oracle_lib, seed):
    """Thermodynamic consistency of the mixture contact values (Appendix):
    the virial pressure built from them,
        beta p = sum_a n_a + (2 pi / 3) sum_ab n_a n_b sigma_ab^3 g_ab(sigma_ab),
    is the Boublik-Mansoori-Carnahan-Starling-Leland equation of state,
        beta p = (6/pi) [xi0/(1-xi3) + 3 xi1 xi2/(1-xi3)^2 + (3-xi3) xi2^3/(1-xi3)^3],
    with xi_k = (pi/6) sum_a n_a sigma_a^k.  The identity holds for every
    composition, so a dropped term, a wrong pair diameter or a wrong
    coefficient in any g_ab breaks it for some of these 2- and 3-species
    mixtures with unequal diameters."""
    rng = np.random.default_rng(1100 + seed)
    M = 2 + seed % 2
    sig = list(rng.uniform(1.0, 7.0, M))
    eta = rng.uniform(0.05, 0.45)
    frac = rng.dirichlet(np.ones(M))
    # partial packing fractions frac_a * eta -> number densities
    n = [6 * frac[a] * eta / (math.pi * sig[a] ** 3) for a in range(M)]
    xi = [math.pi / 6 * sum(n[a] * sig[a] ** k for a in range(M)) for k in range(4)]
    x3 = xi[3]
    p_eos = 6 / math.pi * (xi[0] / (1 - x3) + 3 * xi[1] * xi[2] / (1 - x3) ** 2
                           + (3 - x3) * xi[2] ** 3 / (1 - x3) ** 3)
    p_vir = sum(n) + 2 * math.pi / 3 * sum(
        n[a] * n[b] * (0.5 * (sig[a] + sig[b])) ** 3 * oracle_lib.bmcsl(sig, n, a, b)
        for a in range(M) for b in range(M))
    assert abs(x3 - eta) < 1e-14
    assert abs(p_vir - p_eos) <= 1e-13 * p_eos
