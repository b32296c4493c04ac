"""GPU: batched boxes (one launch per phase for all boxes, HIP-graph replay)
give bitwise the results of stepping every box alone."""
import numpy as np
import pytest

from paper_1202_3842_amd import workloads as W
from tests.parity_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1202_3842_amd import lbe
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lbe.lib()
    return lbe


def _boxes():
    spec = [(24, 3.0, 0.3, 0.5), (30, 4.0, 0.25, 1.0), (17, 3.0, 0.2, 0.3), (40, 6.0, 0.3, 0.5),
            (26, 4.0, 0.35, 0.75), (33, 6.0, 0.2, 0.25)]
    return [W.well_box(L, s, ns3, eps, L / 4.0, 1e-3, 500 + i, 10, name=f"b{i}")
            for i, (L, s, ns3, eps) in enumerate(spec)]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_equals_single_boxes(L, mode, prec):
    ws = _boxes()
    p = L.LBE_FP64 if prec == "fp64" else L.LBE_FP32_POP
    flags = L.LBE_VISC
    banner(f"batch mode {mode} {prec}")
    batch = L.batch_from_workloads(ws, prec=p, flags=flags)
    singles = [L.box_from_workload(w, prec=p, flags=flags) for w in ws]
    batch.step(7, mode=mode)  # odd: graph pairs plus one direct step
    batch.step(2, mode=mode)
    for b in singles:
        b.step(9)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for dist in (0, 1):
            assert np.array_equal(bb.populations(0, dist), bs.populations(0, dist)), (i, dist)
        assert np.array_equal(bb.velocity(0), bs.velocity(0))
    batch.close()


def test_batch_member_setters_and_diagnostics(L):
    ws = _boxes()[:3]
    banner("batch member setters")
    batch = L.batch_from_workloads(ws, flags=L.LBE_VISC)
    d0 = [b.diagnostics()["mass"][0] for b in batch.boxes]
    batch.boxes[1].set_body_force(0, [1e-4, 0, 0])
    batch.step(4)
    d1 = [b.diagnostics()["mass"][0] for b in batch.boxes]
    for a, b in zip(d0, d1):
        assert abs(a - b) <= 1e-13 * a
    single = L.box_from_workload(ws[1], flags=L.LBE_VISC)
    single.set_body_force(0, [1e-4, 0, 0])
    single.step(4)
    assert np.array_equal(batch.boxes[1].populations(0, 1), single.populations(0, 1))


def _mixtures(seed=900):
    """Uneven two-species boxes: cosine wells, diameters 2-6, a channel with
    walls and an obstacle among them."""
    out = []
    spec = [(18, (3.0, 2.0)), (25, (4.0, 6.0)), (21, (2.0, 2.0))]
    for i, (n, sg) in enumerate(spec):
        shape = (n, n, n)
        dens = [W.noisy_uniform(shape, W.packing_density(0.12, s), 1e-2, seed + 10 * i + a) for a, s in enumerate(sg)]
        out.append(W.Workload(name=f"mix{i}", nx=n, ny=n, nz=n, sigma=list(sg), steps=6, density=dens,
                              V=W.smooth_field(shape, 0.2 * W.KT, 3, seed + i),
                              body=[[1e-4, 0.0, 0.0], [0.0, -1e-4, 0.0]]))
    ch = W.channel(nx=40, ny=20, nz=12, x0=16, x1=22, gap=8, steps=6, name="mixchannel")
    ch.V = W.smooth_field(ch.shape, 0.1 * W.KT, 3, seed + 9)
    out.append(ch)
    return out


@pytest.mark.parametrize("flags", ["visc", "visc_drag_printed", "drag_single", "ideal"])
def test_batched_mixtures_equal_single_boxes(L, flags):
    """Two-species boxes in a batch: one force launch per directed pair and
    shell range (the first pair of a species writes, later ones add), the
    two-species ball and collision bodies; bitwise the boxes stepped alone,
    from graph replays, batched launches and the serial schedule."""
    f = {"visc": L.LBE_VISC, "visc_drag_printed": L.LBE_VISC | L.LBE_DRAG | L.LBE_PRINTED_INV,
         "drag_single": L.LBE_DRAG | L.LBE_SINGLE, "ideal": L.LBE_IDEAL}[flags]
    ws = _mixtures()
    banner(f"batched mixtures {flags}")
    batch = L.batch_from_workloads(ws, flags=f)
    singles = [L.box_from_workload(w, flags=f) for w in ws]
    batch.step(5, mode=2)
    batch.step(2, mode=1)
    batch.step(1, mode=0)
    for b in singles:
        b.step(8)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for a in range(2):
            for dist in ((0,) if f & L.LBE_SINGLE else (0, 1)):
                assert np.array_equal(bb.populations(a, dist), bs.populations(a, dist)), (i, a, dist)
    for b in singles:
        b.close()
    batch.close()


def test_batched_mixture_against_oracle(L):
    """One two-species box of the batch against the oracle, to 1e-11."""
    import oracle
    from tests.parity_util import compare_state, oracle_from_workload
    if not oracle.LIB.exists():
        oracle.build()
    ws = _mixtures()
    banner("batched mixture vs oracle")
    batch = L.batch_from_workloads(ws, flags=L.LBE_VISC)
    batch.step(6)
    o = oracle_from_workload(ws[1], L.LBE_VISC)
    o.step(6)
    compare_state(o, batch.boxes[1], 2, 1e-11, "batched mixture")
    batch.close()


def test_batch_of_boxes_at_the_smallest_edges(L):
    """Boxes whose periodic edges equal the interaction reach (6 at sigma = 6,
    4 at sigma = 4, 3 at sigma = 3) and a few just above it, batched: each
    force tile is mostly outside its box, every halo plane is an image, and
    the block -> box tables hold one or two blocks per box.  The batch equals
    the boxes stepped alone bit for bit, and the sigma = 6 box equals the
    oracle to 1e-11 (C^visc, the default scheme, 9 steps)."""
    import oracle
    from tests.parity_util import compare_state, oracle_from_workload
    if not oracle.LIB.exists():
        oracle.build()
    spec = [(6, 6.0, 0.2, 0.5), (4, 4.0, 0.25, 0.5), (3, 3.0, 0.2, 0.5), (7, 3.0, 0.3, 1.0),
            (5, 4.0, 0.2, 0.25)]
    ws = [W.well_box(L_, s, ns3, eps, L_ / 4.0, 1e-2, 900 + i, 9, name=f"t{i}")
          for i, (L_, s, ns3, eps) in enumerate(spec)]
    banner("batch of boxes at the smallest edges")
    batch = L.batch_from_workloads(ws, flags=L.LBE_VISC)
    singles = [L.box_from_workload(w, flags=L.LBE_VISC) for w in ws]
    batch.step(9)
    for b in singles:
        b.step(9)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for dist in (0, 1):
            assert np.array_equal(bb.populations(0, dist), bs.populations(0, dist)), (i, dist)
    o = oracle_from_workload(ws[0], L.LBE_VISC)
    o.step(9)
    compare_state(o, batch.boxes[0], 1, 1e-11, "batched 6^3 at sigma 6")
    for b in singles:
        b.close()
    batch.close()


def test_batched_three_species(L):
    """Three-species boxes of uneven sizes (C^visc and the drag): the batch
    equals the boxes stepped alone, bit for bit."""
    out = []
    for i, n in enumerate((16, 22)):
        sg = [2.0, 3.0, 2.5]
        shape = (n, n, n)
        dens = [W.noisy_uniform(shape, W.packing_density(0.08, s), 1e-2, 950 + 10 * i + a) for a, s in enumerate(sg)]
        out.append(W.Workload(name=f"three{i}", nx=n, ny=n, nz=n, sigma=sg, steps=6, density=dens,
                              V=W.smooth_field(shape, 0.2 * W.KT, 3, 960 + i),
                              body=[[1e-4, 0.0, 0.0], [0.0, -1e-4, 0.0], [0.0, 0.0, 5e-5]]))
    f = L.LBE_VISC | L.LBE_DRAG
    banner("batched three species")
    batch = L.batch_from_workloads(out, flags=f)
    singles = [L.box_from_workload(w, flags=f) for w in out]
    batch.step(5, mode=2)
    batch.step(1, mode=1)
    for b in singles:
        b.step(6)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for a in range(3):
            for dist in (0, 1):
                assert np.array_equal(bb.populations(a, dist), bs.populations(a, dist)), (i, a, dist)
    for b in singles:
        b.close()
    batch.close()


def test_batched_quasipressure_routes(L):
    """The batched path integral (one launch per scan for every box) reads
    each box's route at run time: boxes with their own origins and modes,
    and a route changed between graph replays, give bitwise the boxes
    stepped alone with the same routes."""
    ws = _boxes()[:4]
    obst = W.well_box(22, 3.0, 0.25, 0.5, 5.5, 1e-3, 777, 9, name="obstacle22")
    obst.solid = np.zeros(obst.shape, dtype=bool)
    obst.solid[5:10, 9:13, 8:12] = True               # (z, y, x): a block inside the box
    ws.append(obst)
    routes = [((2, 3, 5), 0), ((29, 0, 11), L.LBE_QP_SYMMETRIC), ((8, 8, 8), 1 | L.LBE_QP_SYMMETRIC),
              ((0, 39, 1), 1), ((20, 10, 6), L.LBE_QP_SYMMETRIC)]
    banner("batched quasi-pressure routes")
    batch = L.batch_from_workloads(ws, flags=L.LBE_VISC)
    singles = [L.box_from_workload(w, flags=L.LBE_VISC) for w in ws]
    for bx, (o, m) in zip(batch.boxes + singles, routes + routes):
        bx.set_quasipressure_route(o, m)
    batch.step(4, mode=2)
    for b in singles:
        b.step(4)
    batch.boxes[2].set_quasipressure_route((1, 2, 3), 0)
    singles[2].set_quasipressure_route((1, 2, 3), 0)
    batch.step(5, mode=2)
    for b in singles:
        b.step(5)
    for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
        for dist in (0, 1):
            assert np.array_equal(bb.populations(0, dist), bs.populations(0, dist)), (i, dist)
    for b in singles:
        b.close()
    batch.close()


@pytest.mark.parametrize("flags", ["visc", "mf"])
def test_batched_force_groups_by_tile_shape(L, flags):
    """Each batched box keeps its own force tiling: the force launches are
    grouped by shell reach and tile shape (32x8, 32x16 with two rows per
    thread, 32x16 with 512 threads), with each box's z depth.  The batch
    equals the boxes stepped alone, bit for bit, for one and two species."""
    f = L.LBE_VISC if flags == "visc" else 0
    tilings = [(2, 1, 0), (1, 0, 2), (4, 2, 1), (2, 0, 2), (1, 1, 1), (3, 1, 0)]
    for ws in (_boxes(), _mixtures()):
        banner(f"batched tile shapes {flags}, {len(ws[0].sigma)} species")
        batch = L.batch_from_workloads(ws, flags=f)
        singles = [L.box_from_workload(w, flags=f) for w in ws]
        for bb, t in zip(batch.boxes, tilings):
            bb.set_force_tiling(*t)
        batch.step(3, mode=2)
        batch.boxes[0].set_force_tiling(1, 0, 2)     # a retune between replays
        batch.step(3, mode=2)
        for b in singles:
            b.step(6)
        M = len(ws[0].sigma)
        for i, (bb, bs) in enumerate(zip(batch.boxes, singles)):
            for a in range(M):
                for dist in (0, 1):
                    assert np.array_equal(bb.populations(a, dist), bs.populations(a, dist)), (i, a, dist)
        for b in singles:
            b.close()
        batch.close()
