"""GPU parity: the HIP library against the FP64 oracle, element by element, on
seeded inputs (FP64 bar: max-norm relative error 1e-11 on n and u)."""
import math

import numpy as np
import pytest

from paper_1202_3842_amd import workloads as W
from tests.parity_util import banner, compare_state, oracle_from_workload, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def L():
    import oracle
    if not oracle.LIB.exists():
        oracle.build()
    oracle.set_threads(8)
    from paper_1202_3842_amd import lbe
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lbe.lib()
    return lbe


def _pair(L, w, flags, prec=None):
    import oracle
    prec = L.LBE_FP64 if prec is None else prec
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, prec=prec, flags=flags)
    return o, b


def test_small_well_fp64(L):
    """32^3 periodic well, sigma = 4, n sigma^3 = 0.3 with noise, depth 1 kT,
    C^visc on, the default scheme: its stated 50 steps, compared on the way."""
    w = W.c1_small_well()
    banner(f"small well {w.name} fp64, {w.steps} steps")
    o, b = _pair(L, w, L.LBE_VISC)
    compare_state(o, b, 1, TOL, "t=0")
    t = 0
    for k in (10, 15, 25):
        o.step(k)
        b.step(k)
        t += k
        compare_state(o, b, 1, TOL, f"t={t}")
    assert t == w.steps
    # populations too
    for dist in (0, 1):
        assert rel_err(b.populations(0, dist), o.populations(0, dist)) <= TOL


SWITCHES = ["none", "printed", "kappa4", "ideal", "printed_kappa4_visc",
            "dd_eu_visc", "sd_tr_visc", "sd_eu_visc", "sd_tr_ideal", "dd_eu_printed",
            "carried_visc", "carried_printed", "carried_dd_eu"]


@pytest.mark.parametrize("flags_name", SWITCHES)
def test_scheme_switches(L, flags_name):
    import oracle
    flags = {"none": 0, "printed": L.LBE_PRINTED_INV | L.LBE_VISC, "kappa4": L.LBE_KAPPA4 | L.LBE_VISC,
             "ideal": L.LBE_IDEAL, "printed_kappa4_visc": L.LBE_VISC | L.LBE_PRINTED_INV | L.LBE_KAPPA4,
             "dd_eu_visc": L.LBE_EULER | L.LBE_VISC, "sd_tr_visc": L.LBE_SINGLE | L.LBE_VISC,
             "sd_eu_visc": L.LBE_SINGLE | L.LBE_EULER | L.LBE_VISC,
             "sd_tr_ideal": L.LBE_SINGLE | L.LBE_IDEAL,
             "dd_eu_printed": L.LBE_EULER | L.LBE_PRINTED_INV,
             "carried_visc": L.LBE_PI_CARRIED | L.LBE_VISC,
             "carried_printed": L.LBE_PI_CARRIED | L.LBE_VISC | L.LBE_PRINTED_INV,
             "carried_dd_eu": L.LBE_PI_CARRIED | L.LBE_EULER | L.LBE_VISC}[flags_name]
    w = W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 5, 6)
    w.body = [[1e-4, -2e-5, 0.0]]
    banner(f"switches {flags_name}")
    o, b = _pair(L, w, flags)
    o.step(6)
    b.step(6)
    compare_state(o, b, 1, TOL, flags_name)


@pytest.mark.parametrize("route", [((12, 7, 3), 0), ((3, 20, 9), 2), ((0, 0, 0), 3), ((23, 23, 23), 1)])
def test_quasipressure_routes(L, route):
    """The per-step quasi-pressure from an off-centre origin along the x, y, z
    path or as the six-order mean, with and without n F in the integrand:
    a non-uniform two-species well with body forces, 6 steps."""
    shape = (24, 24, 24)
    w = W.Workload("route24", 24, 24, 24, [3.0, 2.0], steps=6,
                   density=[W.noisy_uniform(shape, W.packing_density(0.12, 3.0), 2e-2, 70),
                            W.noisy_uniform(shape, W.packing_density(0.06, 2.0), 2e-2, 71)],
                   V=W.smooth_field(shape, 0.3 * W.KT, 3, 72), body=[[1e-4, 0, 0], [0, -5e-5, 2e-5]])
    w.qp_route = route
    banner(f"quasi-pressure route {route}")
    o, b = _pair(L, w, L.LBE_VISC | L.LBE_DRAG)
    o.step(6)
    b.step(6)
    compare_state(o, b, 2, TOL, f"route {route}")
    for a in range(2):
        assert rel_err(b.populations(a, 1), o.populations(a, 1)) <= TOL


@pytest.mark.parametrize("variant", ["sd_tr", "dd_eu", "sd_eu", "drag", "drag_visc", "drag_sd_tr"])
def test_scheme_variants_channel(L, variant):
    """Sec. 4 variants and the interspecies drag on the two-species channel
    with walls (C^visc on unless the name says otherwise)."""
    flags = {"sd_tr": L.LBE_SINGLE | L.LBE_VISC, "dd_eu": L.LBE_EULER | L.LBE_VISC,
             "sd_eu": L.LBE_SINGLE | L.LBE_EULER | L.LBE_VISC, "drag": L.LBE_DRAG,
             "drag_visc": L.LBE_DRAG | L.LBE_VISC,
             "drag_sd_tr": L.LBE_DRAG | L.LBE_SINGLE | L.LBE_VISC}[variant]
    w = W.channel(nx=48, ny=24, nz=16, x0=20, x1=28, gap=10, sigma=(4.0, 6.0), steps=5, name="channel48")
    banner(f"variant {variant} channel")
    o, b = _pair(L, w, flags)
    o.step(5)
    b.step(5)
    compare_state(o, b, 2, TOL, variant)
    for a in range(2):
        assert rel_err(b.populations(a, 0), o.populations(a, 0)) <= TOL
        if not (flags & L.LBE_SINGLE):
            assert rel_err(b.populations(a, 1), o.populations(a, 1)) <= TOL


def test_forces(L):
    w = W.well_box(24, 4.0, 0.3, 0.5, 6.0, 1e-2, 8, 3)
    banner("forces")
    o, b = _pair(L, w, L.LBE_VISC)
    o.step(3)
    b.step(3)
    cm, cv = o.forces(0)
    assert rel_err(b.force(0, 0), cm) <= TOL
    assert rel_err(b.force(0, 1), cv) <= TOL


def test_channel_two_species(L):
    """Reduced bottleneck channel: walls in y, solid constriction, M = 2,
    sigma 4 and 6, body force along x."""
    w = W.channel(nx=48, ny=24, nz=12, x0=20, x1=28, gap=10, force=1e-4, steps=8)
    for a in range(2):
        w.density[a] = w.density[a] * (1 + W.rng(60 + a).uniform(-1e-3, 1e-3, size=w.shape))
    banner("channel M=2 48x24x12")
    o, b = _pair(L, w, L.LBE_VISC)
    o.step(8)
    b.step(8)
    compare_state(o, b, 2, TOL, "channel t=8")


def test_three_species_ragged(L):
    """Three species on a ragged box (edges not multiples of the block)."""
    shape = (11, 13, 17)
    sig = [2.0, 3.0, 1.0]
    dens = [W.noisy_uniform(shape, 0.08 / s ** 3, 1e-2, 90 + i) for i, s in enumerate(sig)]
    w = W.Workload("ragged3", 17, 13, 11, sig, density=dens, V=W.smooth_field(shape, 0.05, 3, 7),
                   body=[[0, 0, 0]] * 3, periodic=7)
    banner("three species ragged 17x13x11")
    o, b = _pair(L, w, L.LBE_VISC)
    o.step(4)
    b.step(4)
    compare_state(o, b, 3, TOL, "ragged t=4")


@pytest.mark.parametrize("walls", [False, True])
def test_box_edge_at_the_interaction_range(L, walls):
    """The smallest periodic edge the library accepts: x = R = 6 for sigma = 6
    (y = 7, z = 9), where a shell point and its mirror r +- e can be the same
    node through the periodic wrap and every halo plane is an image of the
    box.  With walls beyond y, and a solid node, the shell also meets the
    walls from both sides.  C^visc on, the default scheme, 6 steps."""
    shape = (9, 7, 6)
    dens = [W.noisy_uniform(shape, W.packing_density(0.15, 6.0), 2e-2, 77 + walls)]
    solid = None
    if walls:
        solid = np.zeros(shape, dtype=bool)
        solid[4, 3, 2] = True
    w = W.Workload("edge_at_range", 6, 7, 9, [6.0], density=dens,
                   V=W.smooth_field(shape, 0.05, 2, 78), body=[[1e-4, 0, 0]],
                   periodic=W.PERIODIC_XZ if walls else 7, solid=solid)
    banner(f"box edge at the interaction range 6x7x9, walls={walls}")
    o, b = _pair(L, w, L.LBE_VISC)
    t = 0
    for k in (1, 2, 3):
        o.step(k)
        b.step(k)
        t += k
        compare_state(o, b, 1, TOL, f"edge at range, walls={walls}, t={t}")
    for dist in (0, 1):
        assert rel_err(b.populations(0, dist), o.populations(0, dist)) <= TOL


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_widest_shells_in_every_tile_shape(L, shape):
    """Diameters 8 and 6: shells of reach 8, 7 and 6, the widest the kernels
    take, with C^visc on, in each force tile shape (32 x 8 with 256 threads,
    32 x 16 with two rows per thread, 32 x 16 with 512 threads), where the
    gathers hold the most registers.  3 steps against the oracle."""
    dims = (17, 18, 20)
    sig = [8.0, 6.0]
    dens = [W.noisy_uniform(dims, W.packing_density(0.05, s), 1e-2, 120 + a) for a, s in enumerate(sig)]
    w = W.Workload("widest", 20, 18, 17, sig, density=dens, V=W.smooth_field(dims, 0.05, 3, 122),
                   body=[[1e-4, 0, 0], [0, 0, 0]], periodic=7)
    banner(f"widest shells 20x18x17, sigma 8 and 6, tile shape {shape}")
    o, b = _pair(L, w, L.LBE_VISC)
    b.set_force_tiling(1, 1, shape)
    o.step(3)
    b.step(3)
    compare_state(o, b, 2, TOL, f"widest shells, shape {shape}, t=3")


@pytest.mark.parametrize("drag", [False, True])
def test_a_species_with_no_particles(L, drag):
    """Empty input for one species: the second of two has zero density
    everywhere (walls beyond y, body forces on both, C^visc, with and
    without the drag).  Its density and velocity stay exactly zero (u = J/n
    is not formed where n = 0) and the first species evolves as in the
    oracle.  5 steps."""
    dims = (10, 12, 14)
    dens = [W.noisy_uniform(dims, W.packing_density(0.1, 3.0), 1e-2, 31), np.zeros(dims)]
    w = W.Workload("empty_species", 14, 12, 10, [3.0, 2.0], density=dens,
                   V=W.smooth_field(dims, 0.05, 2, 32), body=[[1e-4, 0, 0], [0, 1e-4, 0]],
                   periodic=W.PERIODIC_XZ)
    flags = L.LBE_VISC | (L.LBE_DRAG if drag else 0)
    banner(f"a species with no particles, drag={drag}")
    o, b = _pair(L, w, flags)
    o.step(5)
    b.step(5)
    compare_state(o, b, 2, TOL, f"empty species, drag={drag}, t=5")
    assert not np.any(b.density(1)) and not np.any(b.velocity(1))
    for dist in (0, 1):
        assert not np.any(b.populations(1, dist))


def test_an_empty_box(L):
    """No particles at all (one species, zero density, a potential and a
    body force): every population stays zero, and the diagnostics report
    zero mass and velocity without flagging the state."""
    dims = (8, 9, 10)
    w = W.Workload("empty_box", 10, 9, 8, [3.0], density=[np.zeros(dims)],
                   V=W.smooth_field(dims, 0.05, 2, 33), body=[[1e-4, 0, 0]], periodic=7)
    banner("an empty box")
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    b.step(3)
    for dist in (0, 1):
        assert not np.any(b.populations(0, dist))
    d = b.diagnostics()
    assert d["mass"][0] == 0.0 and d["umax"] == 0.0 and not d["unstable"]


def test_channel_one_node_wide(L):
    """A non-periodic edge of one node: walls on both sides of every node
    (12 x 1 x 10, x and z periodic, sigma = 3, C^visc on), so every shell
    point off the y = 0 plane lies beyond a wall and the y pulls all bounce
    back.  6 steps."""
    shape = (10, 1, 12)
    dens = [W.noisy_uniform(shape, W.packing_density(0.15, 3.0), 2e-2, 79)]
    w = W.Workload("one_node_channel", 12, 1, 10, [3.0], density=dens,
                   V=W.smooth_field(shape, 0.05, 2, 80), body=[[1e-4, 0, 0]],
                   periodic=W.PERIODIC_XZ)
    banner("channel one node wide 12x1x10")
    o, b = _pair(L, w, L.LBE_VISC)
    o.step(6)
    b.step(6)
    compare_state(o, b, 1, TOL, "one node wide, t=6")
    for dist in (0, 1):
        assert rel_err(b.populations(0, dist), o.populations(0, dist)) <= TOL


def test_populations_roundtrip(L):
    w = W.channel(nx=20, ny=12, nz=8, x0=8, x1=12, gap=4, sigma=(3.0, 2.0), steps=1)
    banner("populations roundtrip")
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    b.step(2)
    for dist in (0, 1):
        p = b.populations(1, dist)
        b.set_populations(1, dist, p)
        assert np.array_equal(b.populations(1, dist), p)


def test_uniform_fixed_point(L):
    L_ = 24
    shape = (L_, L_, L_)
    w = W.Workload("uni", L_, L_, L_, [4.0], density=[np.full(shape, 0.3 / 64)], V=np.zeros(shape),
                   body=[[0, 0, 0]])
    banner("uniform fixed point")
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    b.step(20)
    assert not np.any(b.velocity(-1))
    n = b.density(0)
    assert n.max() == n.min()
    assert abs(n.max() - 0.3 / 64) <= 1e-14 * 0.3 / 64


def test_mass_momentum_and_determinism(L):
    w = W.well_box(32, 4.0, 0.3, 0.0, 1.0, 1e-2, 21, 1)
    w.V = np.zeros(w.shape)
    banner("mass/momentum/determinism")
    b1 = L.box_from_workload(w, flags=L.LBE_VISC)
    b2 = L.box_from_workload(w, flags=L.LBE_VISC)
    d0 = b1.diagnostics()
    b1.step(15)
    b2.step(15)
    d1 = b1.diagnostics()
    m0, m1 = np.array(d0["mass"]), np.array(d1["mass"])
    assert np.abs(m1 - m0).max() <= 1e-13 * m0.max()
    scale = m0.sum() * math.sqrt(1 / 3)
    assert np.abs(np.array(d1["gmom"]) - np.array(d0["gmom"])).max() <= 1e-13 * scale
    for dist in (0, 1):
        assert np.array_equal(b1.populations(0, dist), b2.populations(0, dist))


def test_diagnostics_against_oracle(L):
    w = W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 33, 5)
    banner("diagnostics")
    o, b = _pair(L, w, L.LBE_VISC)
    o.step(5)
    b.step(5)
    do, dg = o.diagnostics(), b.diagnostics()
    for k in ("umax", "err_n", "err_u", "err_J"):
        assert abs(dg[k] - do[k]) <= 1e-11 * abs(do[k]), k
    assert abs(dg["mass"][0] - do["mass"][0]) <= 1e-13 * do["mass"][0]


def test_instability_is_reported(L):
    L_ = 16
    shape = (L_, L_, L_)
    w = W.Workload("dense", L_, L_, L_, [4.0], density=[np.full(shape, 1.1 * 6 / (math.pi * 64))],
                   V=np.zeros(shape), body=[[0, 0, 0]])
    banner("instability flag")
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    b.step(1)
    assert b.diagnostics()["unstable"]
    with pytest.raises(L.LBEError) as e:
        b.step(1)
    assert e.value.code == L.LBE_ERR_UNSTABLE
    b.init_density(0, np.full(shape, 0.3 / 64))
    b.step(1)
    assert not b.diagnostics()["unstable"]


def test_fp32_populations_report(L):
    """FP32 population storage (FP64 arithmetic): reported, with a loose bar."""
    w = W.c1_small_well()
    banner("fp32 populations")
    o, b = _pair(L, w, L.LBE_VISC, prec=L.LBE_FP32_POP)
    o.step(10)
    b.step(10)
    en = rel_err(b.density(0), o.density(0))
    eu = rel_err(b.velocity(-1), o.velocity(-1))
    print(f"[fp32] n rel err {en:.3e} u rel err {eu:.3e}", flush=True)
    assert en < 1e-5 and eu < 1e-3
