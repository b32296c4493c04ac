"""lbe_get_quasipressure_noalloc (the entry point for callers that cannot
allocate device memory) against lbe_get_quasipressure, through the C ABI:
two calls in a row on different boxes, the second smaller, and the size
limit of its static scratch."""
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


def _check(L, box, species, origin, mode):
    import torch
    ref = box.quasipressure(species, origin, mode)
    out = torch.full((box.N,), float("nan"), dtype=torch.float64, device="cuda")
    box.quasipressure_noalloc(out, species, origin, mode)
    box.synchronize()
    got = out.cpu().numpy().reshape(box.shape)
    print(f"[noalloc] species {species} mode {mode}: max |diff| {np.abs(got - ref).max():.3e}", flush=True)
    assert np.array_equal(got, ref)


def test_noalloc_equals_quasipressure_two_calls(L):
    """A two-species channel (48x24x16), then a smaller one-species well
    (24^3): every species and path mode, bitwise equal to the workspace
    version."""
    w = W.channel(nx=48, ny=24, nz=16, x0=20, x1=28, gap=10, steps=3, name="channel48x24x16")
    w.V = W.smooth_field(w.shape, 0.2 * W.KT, 3, 13)
    banner("noalloc quasi-pressure: channel 48x24x16, then well 24^3")
    b = L.box_from_workload(w, flags=L.LBE_VISC | L.LBE_DRAG)
    b.step(3)
    for species in (0, 1):
        for mode in (0, 1, 2, 3):
            _check(L, b, species, (5, 12, 3), mode)
    b.close()
    w2 = W.well_box(24, 3.0, 0.3, 0.5, 6.0, 1e-3, 5, 3)
    b2 = L.box_from_workload(w2, flags=L.LBE_VISC)
    b2.step(3)
    for mode in (0, 2):
        _check(L, b2, 0, (12, 12, 12), mode)
    b2.close()


def test_noalloc_rejects_boxes_beyond_its_scratch(L):
    import torch
    banner("noalloc quasi-pressure: size limit")
    b = L.Box(144, 144, 144, [2.0], flags=L.LBE_VISC)
    b.init_density(0, np.full(b.shape, 0.01))
    out = torch.empty(b.N, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LBEError) as e:
        b.quasipressure_noalloc(out, 0, (72, 72, 72), 0)
    assert e.value.code == L.LBE_ERR_ARG
    assert "at most" in str(e.value)
    b.close()
