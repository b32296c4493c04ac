"""GPU checks of the paper's quantitative comparison of its schemes (Sec. 4.2,
hard spheres in the cosine well): the spurious velocity of the trapezoidal
double-distribution scheme lies far below that of SD-EU.  The paper reports
a factor of about 10 for SD-TR and about 50 for DD-TR.

Which reading of Pi carries which claim: with Pi evaluated every step (the
default) DD-TR and SD-TR sit close together, about 18x below SD-EU on the
one-component well; with Pi carried by g (LBE_PI_CARRIED) DD-TR is about 90x
below SD-EU, the paper's order, but that reading cannot run the configured
128^3 well (it collapses), and its sound speed is the ideal-gas one."""
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


def _umax(L, w, steps):
    umax = {}
    for name, fl in (("DD-TR", L.LBE_VISC), ("DD-TR carried", L.LBE_VISC | L.LBE_PI_CARRIED),
                     ("SD-TR", L.LBE_VISC | L.LBE_SINGLE),
                     ("SD-EU", L.LBE_VISC | L.LBE_SINGLE | L.LBE_EULER)):
        b = L.box_from_workload(w, flags=fl)
        b.step(steps)
        d = b.diagnostics()
        assert not d["unstable"], name
        umax[name] = d["umax"]
        b.close()
    return umax


def test_trapezoidal_spurious_velocity_far_below_sd_eu(L):
    """32^3 periodic well, sigma = 4, n sigma^3 = 0.3 (eta 0.157), eps =
    0.5 kT (a well every variant runs), C^visc on, 3000 steps."""
    w = W.well_box(32, 4.0, 0.3, 0.5, 8.0, 1e-3, 1202, 3000, "well32_s4_eps05")
    banner("spurious velocity DD-TR / SD-TR / SD-EU, 32^3 well")
    umax = _umax(L, w, 3000)
    r = {k: umax["SD-EU"] / v for k, v in umax.items()}
    print(f"[claim] max |u|: {umax}, SD-EU / scheme: {r}", flush=True)
    assert r["DD-TR"] > 10.0 and r["SD-TR"] > 10.0
    assert r["DD-TR carried"] > 40.0
    assert umax["DD-TR carried"] < umax["DD-TR"]


def test_binary_mixture_scheme_order(L):
    """Binary hard spheres sigma 4 : 8 (x_A = 1/2, eta = 0.1) in the 32^3
    cosine well with eps = 0.5 kT, C^visc on, 3000 steps."""
    sh = (32, 32, 32)
    sA, sB, eta, xA = 4.0, 8.0, 0.1, 0.5
    ntot = 6 * eta / (np.pi * (xA * sA ** 3 + (1 - xA) * sB ** 3))
    w = W.Workload(name="binary32", nx=32, ny=32, nz=32, sigma=[sA, sB],
                   density=[W.noisy_uniform(sh, xA * ntot, 1e-3, 77),
                            W.noisy_uniform(sh, (1 - xA) * ntot, 1e-3, 78)],
                   V=W.cosine_well(sh, 8.0, 0.5 * W.KT), body=[[0, 0, 0], [0, 0, 0]])
    banner("spurious velocity, binary sigma 4:8, 32^3 well")
    umax = _umax(L, w, 3000)
    r = {k: umax["SD-EU"] / v for k, v in umax.items()}
    print(f"[claim] binary max |u|: {umax}, SD-EU / scheme: {r}", flush=True)
    assert r["DD-TR"] > 10.0 and r["SD-TR"] > 10.0
    assert r["DD-TR carried"] > 40.0
