"""GPU parity of the attractive molecular field G^{ab} (Appendix, the last term
of C^{a,mf}; the r^-6 tail on [sigma_ab, rc) with g = 1, see lbe.h): the HIP
library against the FP64 oracle (bar 1e-11) on one and two species, with
walls and obstacles, C^visc, a scheme variant, and at the full 128^3 size."""
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


def _well(eps, rc):
    w = W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 5, 5)
    w.att_eps, w.att_rc = [[eps]], rc
    return w


def _channel(rc=7.0):
    w = W.channel(nx=48, ny=24, nz=16, x0=20, x1=28, gap=10, steps=4, name="channel48x24x16")
    w.V = W.smooth_field(w.shape, 0.2 * KT, 3, 13)
    w.att_eps = [[0.4 * KT, 0.3 * KT], [0.3 * KT, 0.2 * KT]]
    w.att_rc = rc
    return w


@pytest.mark.parametrize("eps,rc", [(0.5 * KT, 6.0), (1.0 * KT, 4.5), (0.3 * KT, 9.0)])
def test_attraction_well(L, eps, rc):
    """24^3 well, sigma = 3, C^visc on, 5 steps; rc from a thin range to the
    largest built (8 nodes per axis)."""
    w = _well(eps, rc)
    banner(f"attraction well eps={eps:.3f} rc={rc}")
    o = oracle_from_workload(w, L.LBE_VISC)
    b = L.box_from_workload(w, flags=L.LBE_VISC)
    assert rel_err(b.force(0, 0), o.forces(0)[0]) <= TOL
    o.step(5)
    b.step(5)
    compare_state(o, b, 1, TOL, f"attraction well rc={rc}")
    b.close()


@pytest.mark.parametrize("variant", ["dd_tr_visc", "sd_tr", "dd_tr_printed"])
def test_attraction_channel_two_species(L, variant):
    """Two-species channel with walls and the bottleneck, a body force and a
    smooth potential, unequal eps per pair, 4 steps."""
    flags = {"dd_tr_visc": L.LBE_VISC, "sd_tr": L.LBE_VISC | L.LBE_SINGLE,
             "dd_tr_printed": L.LBE_PRINTED_INV}[variant]
    w = _channel()
    banner(f"attraction channel {variant}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    for a in range(2):
        assert rel_err(b.force(a, 0), o.forces(a)[0]) <= TOL
    o.step(w.steps)
    b.step(w.steps)
    compare_state(o, b, 2, TOL, f"attraction channel {variant}")
    b.close()


def test_attraction_changes_the_force(L):
    """The field is really there: C^mf with and without it differ by n G, of
    the size the oracle gives."""
    w = _well(0.5 * KT, 6.0)
    b1 = L.box_from_workload(w, flags=L.LBE_VISC)
    w0 = _well(0.0, 6.0)
    w0.att_eps = None
    b0 = L.box_from_workload(w0, flags=L.LBE_VISC)
    d = b1.force(0, 0) - b0.force(0, 0)
    o1 = oracle_from_workload(w, L.LBE_VISC)
    o0 = oracle_from_workload(w0, L.LBE_VISC)
    ref = o1.forces(0)[0] - o0.forces(0)[0]
    assert np.abs(ref).max() > 0
    assert rel_err(d, ref) <= 1e-10
    b1.close()
    b0.close()


def test_attraction_full_size_well128(L):
    """128^3 benchmark well (sigma = 6, n sigma^3 = 0.4, printed inversions)
    with eps = kT/4 and rc = 8 (the thick shell 6 <= |e| < 8), 2 steps."""
    w = W.c2_large_well()
    w.att_eps, w.att_rc = [[0.25 * KT]], 8.0
    flags = L.LBE_VISC | L.LBE_PRINTED_INV
    banner("attraction full size well128")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(2)
    b.step(2)
    compare_state(o, b, 1, TOL, "attraction 128^3")
    b.close()
    o.close()


def test_attraction_fp32_storage(L):
    """FP32 population storage with the attractive field (FP64 arithmetic):
    the same loose bar as the plain FP32 check, after 10 steps."""
    w = _well(0.5 * KT, 6.0)
    banner("attraction fp32 populations")
    o = oracle_from_workload(w, L.LBE_VISC)
    b = L.box_from_workload(w, prec=L.LBE_FP32_POP, flags=L.LBE_VISC)
    o.step(10)
    b.step(10)
    en = rel_err(b.density(0), o.density(0))
    eu = rel_err(b.velocity(-1), o.velocity(-1))
    print(f"[fp32] attraction n rel err {en:.3e} u rel err {eu:.3e}", flush=True)
    assert en < 1e-5 and eu < 1e-3
    b.close()


def test_attraction_in_batched_boxes(L):
    """Uneven boxes, some with the attractive field (different depths and
    cutoffs: tail reaches of 5 and 7 nodes), stepped as a batch from graph replays and
    batched launches: bitwise equal to the same boxes stepped alone, and one
    of them equal to the oracle to 1e-11."""
    spec = [(20, 3.0, 0.3, 0.25 * KT, 5.5), (27, 4.0, 0.25, 0.0, 0.0), (17, 3.0, 0.2, 0.4 * KT, 7.5),
            (24, 6.0, 0.3, 0.2 * KT, 8.0)]
    ws = []
    for i, (n, sg, ns3, eps, rc) in enumerate(spec):
        w = W.well_box(n, sg, ns3, 0.5, n / 4.0, 1e-3, 800 + i, 6, name=f"att_batch{i}")
        if eps > 0:
            w.att_eps, w.att_rc = [[eps]], rc
        ws.append(w)
    flags = L.LBE_VISC
    banner("attraction in batched boxes")
    batch = L.batch_from_workloads(ws, flags=flags)
    singles = [L.box_from_workload(w, flags=flags) for w in ws]
    batch.step(5, mode=2)   # graph replays (odd: plus one batched step)
    batch.step(2, mode=1)   # batched launches
    for b in singles:
        b.step(7)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for dist in (0, 1):
            assert np.array_equal(bb.populations(0, dist), bs.populations(0, dist)), (i, dist)
    o = oracle_from_workload(ws[2], flags)
    o.step(7)
    compare_state(o, batch.boxes[2], 1, TOL, "batched box with attraction")
    for b in singles:
        b.close()
    batch.close()
