"""GPU parity of the quasi-pressure (Sec. 2, eq. quasipressure) and of its
initialiser: the HIP library against the FP64 oracle on seeded inputs, at
sizes that span several line groups and segments with ragged ends, with solid
nodes and two species, and at the full 128^3 benchmark size."""
import math
import os

import numpy as np
import pytest

from paper_1202_3842_amd import workloads as W
from tests.parity_util import banner, compare_state, oracle_from_workload, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11
KT = 1.0 / 3.0


@pytest.fixture(scope="module")
def L():
    import oracle
    if not oracle.LIB.exists():
        oracle.build()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    from paper_1202_3842_amd import lbe
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lbe.lib()
    return lbe


def _ragged_well():
    """70 x 9 x 6: the x line spans two lane groups and uneven segments, the
    z lines are shorter than the segment count."""
    sh = (6, 9, 70)
    return W.Workload(
        name="ragged70x9x6", nx=70, ny=9, nz=6, sigma=[2.0], steps=3,
        density=[W.noisy_uniform(sh, W.packing_density(0.15, 2.0), 0.05, 11)],
        V=W.smooth_field(sh, 0.3 * KT, 3, 12), body=[[1e-4, -5e-5, 2e-5]])


def _small_channel():
    w = W.channel(nx=48, ny=24, nz=16, x0=20, x1=28, gap=10, steps=3, name="channel48x24x16")
    w.V = W.smooth_field(w.shape, 0.2 * KT, 3, 13)
    return w


CASES = {
    "ragged_well": (_ragged_well, (65, 7, 1)),
    "channel_two_species": (_small_channel, (5, 12, 3)),
    "cube_well_corner": (lambda: W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 5, 3), (0, 0, 0)),
}


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("case", list(CASES))
def test_quasipressure_parity(L, case, mode):
    make, origin = CASES[case]
    w = make()
    flags = L.LBE_VISC
    banner(f"quasipressure {case} mode={mode} origin={origin}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(w.steps)
    b.step(w.steps)
    for a in range(w.nspecies):
        ref = o.quasipressure(a, origin, mode)
        got = b.quasipressure(a, origin, mode)
        err = rel_err(got, ref)
        print(f"[parity] Pi species {a}: {err:.2e}", flush=True)
        assert err <= TOL, (case, mode, a, err)
        if w.solid is not None:
            assert (got[w.solid.astype(bool)] == 0).all()
    b.close()


INIT_FLAGS = {
    "derived": lambda L: L.LBE_VISC,
    "printed": lambda L: L.LBE_VISC | L.LBE_PRINTED_INV,
    "euler": lambda L: L.LBE_VISC | L.LBE_EULER,
    "drag": lambda L: L.LBE_VISC | L.LBE_DRAG,
}


@pytest.mark.parametrize("variant", list(INIT_FLAGS))
def test_initialiser_parity_channel(L, variant):
    """Two-species channel, 3 steps, then the initialiser (default reading):
    g~ of both species against the oracle's, f~ untouched; then 3 more steps
    of both, compared node by node."""
    w = _small_channel()
    flags = INIT_FLAGS[variant](L)
    origin = (5, 12, 3)
    banner(f"quasipressure init channel {variant}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(3)
    b.step(3)
    f_before = [b.populations(a, 0) for a in range(2)]
    o.init_quasipressure(origin, 0)
    b.init_quasipressure(origin, 0)
    for a in range(2):
        assert np.array_equal(b.populations(a, 0), f_before[a])
        err = rel_err(b.populations(a, 1), o.populations(a, 1))
        print(f"[parity] g~ species {a} after init: {err:.2e}", flush=True)
        assert err <= TOL
    o.step(3)
    b.step(3)
    compare_state(o, b, 2, TOL, f"channel {variant} init + 3 steps")
    b.close()


def test_initialiser_printed_integrand_ragged(L):
    """The printed integrand (with n F) on the ragged box, origin near the far
    corner so that every leg runs both ways."""
    w = _ragged_well()
    flags = L.LBE_VISC
    origin = (65, 7, 1)
    banner("quasipressure init ragged printed integrand")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(3)
    b.step(3)
    o.init_quasipressure(origin, 1)
    b.init_quasipressure(origin, L.LBE_QP_WITH_FEXT)
    assert rel_err(b.populations(0, 1), o.populations(0, 1)) <= TOL
    b.close()


def test_initialiser_fp32_storage(L):
    """FP32 population storage: Pi and the shift are computed in FP64 and the
    shifted g~ is rounded to FP32 once."""
    w = W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 5, 3)
    flags = L.LBE_VISC
    banner("quasipressure init fp32")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, prec=L.LBE_FP32_POP, flags=flags)
    o.init_quasipressure((12, 12, 12), 0)
    b.init_quasipressure((12, 12, 12), 0)
    g = b.populations(0, 1)
    assert g.dtype == np.float32
    err = rel_err(g.astype(np.float64), o.populations(0, 1))
    print(f"[parity] fp32 g~ after init: {err:.2e}", flush=True)
    assert err <= 2e-6
    b.close()


def test_initialiser_restores_a_relaxed_slab(L):
    """The hard-sphere slab well relaxed by the library itself under the
    reading in which g carries Pi (no noise, 1000 steps): disturbing the zeroth moment of g~ and calling the
    initialiser gives back the relaxed g~ up to a uniform shift of Pi (the
    property the oracle is pinned to)."""
    nx, ny, nz = 32, 8, 8
    x = np.broadcast_to(np.arange(nx), (nz, ny, nx))
    V = -0.25 * KT * np.cos(2 * math.pi * x / nx)
    bz = np.exp(-3.0 * V) / np.exp(-3.0 * V).mean()
    banner("quasipressure relaxed slab")
    b = L.Box(nx, ny, nz, [3.0], flags=L.LBE_VISC | L.LBE_PI_CARRIED)
    b.set_potential(np.ascontiguousarray(V))
    b.init_density(0, W.packing_density(0.1, 3.0) * bz)
    b.step(1000)
    assert np.abs(b.velocity(0)).max() < 1e-11
    g = b.populations(0, 1)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    d = W.rng(77).uniform(-1e-3, 1e-3, size=g.shape[1:])
    b.set_populations(0, 1, g + w[:, None, None, None] * d)
    b.init_quasipressure((16, 4, 4), 0)
    g1 = b.populations(0, 1)
    shift = (g1 - g).sum(axis=0)[4, 4, 16]
    assert np.abs(g1 - g - w[:, None, None, None] * shift).max() < 1e-11 * np.abs(g).max()
    b.close()


def test_quasipressure_full_size_well128(L):
    """128^3 benchmark well (sigma = 6, n sigma^3 = 0.4, the default scheme),
    2 steps: Pi in every mode and g~ after the initialiser, every node."""
    w = W.c2_large_well()
    flags = L.LBE_VISC
    origin = (64, 64, 64)
    banner(f"quasipressure full size {w.name}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(2)
    b.step(2)
    for mode in (0, 1, 2, 3):
        err = rel_err(b.quasipressure(0, origin, mode), o.quasipressure(0, origin, mode))
        print(f"[parity] 128^3 Pi mode {mode}: {err:.2e}", flush=True)
        assert err <= TOL
    o.init_quasipressure(origin, 0)
    b.init_quasipressure(origin, 0)
    err = rel_err(b.populations(0, 1), o.populations(0, 1))
    print(f"[parity] 128^3 g~ after init: {err:.2e}", flush=True)
    assert err <= TOL
    b.close()
    o.close()


def test_argument_and_state_errors(L):
    w = _small_channel()
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    banner("quasipressure errors")
    for origin, mode in [((48, 1, 1), 0), ((5, -1, 1), 0), ((22, 0, 3), 0), ((5, 12, 3), 4)]:
        with pytest.raises(L.LBEError) as e:
            b.quasipressure(0, origin, mode)
        assert e.value.code == L.LBE_ERR_ARG
    b.step_phase(0)
    with pytest.raises(L.LBEError) as e:
        b.init_quasipressure((5, 12, 3), 0)
    assert e.value.code == L.LBE_ERR_STATE
    for ph in (1, 2, 3, 4):
        b.step_phase(ph)
    b.init_quasipressure((5, 12, 3), 0)
    b.close()
    s = L.box_from_workload(_ragged_well(), flags=L.LBE_SINGLE | L.LBE_VISC)
    with pytest.raises(L.LBEError) as e:
        s.init_quasipressure((1, 1, 1), 0)
    assert e.value.code == L.LBE_ERR_ARG
    s.quasipressure(0, (1, 1, 1), 0)      # Pi itself is defined for SD too
    s.close()


def test_initialiser_on_batch_members(L):
    """Members of a batched set share the batch's buffers: the initialiser on
    two of them, then batched steps (graph replay), equal bitwise a standalone
    box that does the same."""
    spec = [(24, 3.0, 0.3, 0.5), (30, 4.0, 0.25, 1.0), (17, 3.0, 0.2, 0.3)]
    ws = [W.well_box(n, s, ns3, eps, n / 4.0, 1e-3, 700 + i, 6, name=f"q{i}")
          for i, (n, s, ns3, eps) in enumerate(spec)]
    banner("quasipressure init on batch members")
    batch = L.batch_from_workloads(ws, flags=L.LBE_VISC)
    singles = [L.box_from_workload(w, flags=L.LBE_VISC) for w in ws]
    batch.step(3)
    for b in singles:
        b.step(3)
    for i in (0, 2):
        o = (ws[i].nx // 3, ws[i].ny // 2, 1)
        batch.boxes[i].init_quasipressure(o, 0)
        singles[i].init_quasipressure(o, 0)
        assert np.array_equal(batch.boxes[i].quasipressure(0, o), singles[i].quasipressure(0, o))
    batch.step(5)
    for b in singles:
        b.step(5)
    for bb, bs in zip(batch.boxes, singles):
        for dist in (0, 1):
            assert np.array_equal(bb.populations(0, dist), bs.populations(0, dist))
    for b in singles:
        b.close()
    batch.close()


def test_route_errors(L):
    """lbe_set_quasipressure_route refuses a solid origin, an origin outside
    the box and unknown mode bits; a step refuses to run once lbe_set_solid
    has made the origin solid, and runs again after a new route."""
    w = _small_channel()
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    banner("quasi-pressure route errors")
    for origin, mode in [((22, 0, 3), 0), ((48, 1, 1), 0), ((5, 12, 3), 4)]:
        with pytest.raises(L.LBEError) as e:
            b.set_quasipressure_route(origin, mode)
        assert e.value.code == L.LBE_ERR_ARG
    b.set_quasipressure_route((5, 12, 3), 0)
    mask = w.solid.copy()
    mask[3, 12, 5] = 1
    b.set_solid(mask)
    with pytest.raises(L.LBEError) as e:
        b.step(1)
    assert e.value.code == L.LBE_ERR_STATE
    b.set_quasipressure_route((6, 12, 3), 0)
    b.step(1)
    b.close()
