"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (autotuned force tiling), and invariance of the
results under every force-kernel tiling (tile shape, tile order, z depth)."""
import os

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
    oracle.set_threads(min(16, os.cpu_count() or 1))
    from paper_1202_3842_amd import lbe
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    lbe.lib()
    return lbe


def test_well128_full_size_bench_configuration(L):
    """128^3, sigma = 6, n sigma^3 = 0.4, well depth 2 kT, C^visc on, printed
    inversions: the benchmark's workload, 3 steps, tuned tiling."""
    from paper_1202_3842_amd import autotune
    w = W.c2_large_well()
    flags = L.LBE_VISC | L.LBE_PRINTED_INV
    banner(f"full size {w.name}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    autotune.tune_zchunk(b)
    print("tiling", getattr(b, "tiling", None), flush=True)
    o.step(3)
    b.step(3)
    compare_state(o, b, 1, TOL, "well128 t=3")
    for dist in (0, 1):
        assert rel_err(b.populations(0, dist), o.populations(0, dist)) <= TOL
    b.close()
    o.close()


def test_channel256_full_size(L):
    """256x64x32 two-species channel with the bottleneck (sigma 4 and 6,
    eta = 0.25, walls, body force), C^visc on, 2 steps."""
    w = W.c3_channel()
    flags = L.LBE_VISC
    banner(f"full size {w.name}")
    o = oracle_from_workload(w, flags)
    b = L.box_from_workload(w, flags=flags)
    o.step(2)
    b.step(2)
    compare_state(o, b, 2, TOL, "channel256 t=2")
    b.close()
    o.close()


@pytest.mark.parametrize("flags_name", ["mf", "visc"])
def test_tiling_does_not_change_results(L, flags_name):
    """Every (zchunk, order, shape) gives bitwise the same state."""
    w = W.channel(nx=40, ny=20, nz=12, x0=15, x1=22, gap=8, sigma=(3.0, 4.0), steps=3, name="channel40")
    flags = L.LBE_VISC if flags_name == "visc" else 0
    ref = None
    for zc in (1, 3, 12):
        for order in (0, 1, 2):
            for shape in (0, 1, 2):
                banner(f"tiling {flags_name} zchunk {zc} order {order} shape {shape}")
                b = L.box_from_workload(w, flags=flags)
                b.set_force_tiling(zc, order, shape)
                b.step(3)
                st = [b.populations(a, d) for a in range(2) for d in range(2)]
                b.close()
                if ref is None:
                    ref = st
                    continue
                for x, y in zip(st, ref):
                    assert np.array_equal(x, y), (zc, order, shape)
