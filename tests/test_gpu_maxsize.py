"""GPU: one box near the size a single card holds comfortably, 512^3 nodes
(134M, a 118 GiB workspace in FP64), sigma = 6 with C^visc and the default
scheme.  Population offsets reach 2 x 19 x 134M > 2^32 and field offsets pass
2^31, so every 64-bit offset path runs.  The oracle cannot step this box, so
the checks are properties that hold at any size (Sec. 4.1 and the pair sums
of the Appendix):

* a uniform state is an exact fixed point: no velocity anywhere and the
  density after two steps equal, bit for bit, to the one read back after
  initialisation;
* from a seeded non-uniform state at rest, mass is conserved to rounding and
  the total current stays at zero to rounding (the pair forces cancel in
  sum), as the small-box conservation test requires."""
import math

import numpy as np
import pytest
import torch

from paper_1202_3842_amd import workloads as W
from tests.parity_util import banner

pytestmark = pytest.mark.gpu

L_EDGE = 512
SIGMA = 6.0


@pytest.fixture(scope="module")
def L():
    from paper_1202_3842_amd import lbe
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lbe.lib()
    return lbe


def test_largest_box_keeps_its_invariants(L):
    shape = (L_EDGE,) * 3
    n0 = W.packing_density(0.2, SIGMA)
    banner(f"box {L_EDGE}^3, sigma {SIGMA}, workspace "
           f"{L.workspace_bytes(L.make_config(L_EDGE, L_EDGE, L_EDGE, [SIGMA])) / 2 ** 30:.0f} GiB")
    box = L.Box(L_EDGE, L_EDGE, L_EDGE, [SIGMA], flags=L.LBE_VISC)
    try:
        # uniform state: an exact fixed point
        box.init_density(0, np.full(shape, n0))
        before = box.density(0)    # n0 up to the rounding of sum_p w_p n0
        assert before.max() == before.min() and abs(before.max() - n0) <= 1e-14 * n0
        box.step(2)
        d = box.diagnostics()
        assert d["umax"] == 0.0 and not d["unstable"]
        assert np.array_equal(box.density(0), before)
        del before
        banner("uniform state kept exactly")
        # a seeded non-uniform state at rest: mass and total current conserved
        box.init_density(0, W.noisy_uniform(shape, n0, 1e-2, 512))
        d0 = box.diagnostics()
        box.step(2)
        d1 = box.diagnostics()
        assert not d1["unstable"] and d1["umax"] > 0.0
        m0, m1 = d0["mass"][0], d1["mass"][0]
        assert abs(m1 - m0) <= 1e-13 * m0
        scale = m0 * math.sqrt(1 / 3)
        assert np.abs(np.array(d1["gmom"]) - np.array(d0["gmom"])).max() <= 1e-13 * scale
        banner(f"mass {m0:.6e} -> {m1:.6e}, umax {d1['umax']:.3e}")
    finally:
        box.close()
        del box
        torch.cuda.empty_cache()
