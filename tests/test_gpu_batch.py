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
