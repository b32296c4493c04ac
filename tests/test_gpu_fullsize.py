"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (autotuned force tiling), and invariance of the
results under every force-kernel tiling (tile shape, tile order, z depth)."""
import os
from pathlib import Path

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


GOLDEN = Path(__file__).resolve().parent / "golden"


def test_well128_full_size_bench_configuration(L):
    """128^3, sigma = 6, n sigma^3 = 0.4, well depth 2 kT, C^visc on, the
    default scheme: the benchmark's workload, 3 steps, tuned tiling, every
    node and population."""
    from paper_1202_3842_amd import autotune
    w = W.c2_large_well()
    flags = L.LBE_VISC
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


def _compare_golden(b, g, w, prefix, label):
    """n^a, u^a and the barycentric u of the box against a stored oracle
    state on its plane and sampled nodes (max-norm relative error)."""
    z = int(g["zplane"]) if "zplane" in g else w.nz // 2
    nodes = g[f"{prefix}nodes"]
    errs = {}
    for a in range(w.nspecies):
        n = b.density(a)
        u = b.velocity(a)
        errs[f"n{a}"] = max(rel_err(n[z], g[f"{prefix}n{a}_plane"]),
                            rel_err(n.reshape(-1)[nodes], g[f"{prefix}n{a}_nodes"]))
        errs[f"u{a}"] = max(rel_err(u[:, z], g[f"{prefix}u{a}_plane"]),
                            rel_err(u.reshape(3, -1)[:, nodes], g[f"{prefix}u{a}_nodes"]))
    ub = b.velocity(-1)
    errs["u"] = max(rel_err(ub[:, z], g[f"{prefix}u_plane"]),
                    rel_err(ub.reshape(3, -1)[:, nodes], g[f"{prefix}u_nodes"]))
    print(f"[parity] {label} {errs}", flush=True)
    for k, v in errs.items():
        assert v <= TOL, (label, k, v)


def test_well128_stated_2000_steps_against_oracle(L):
    """The 128^3 well over its stated 2000 steps in the benchmark's launch
    configuration, against the oracle's state (tests/golden/well128_2000.npz,
    written by make_fullsize_goldens.py): the full plane z = 64 and 32768
    seeded nodes."""
    from paper_1202_3842_amd import autotune
    path = GOLDEN / "well128_2000.npz"
    if not path.exists():
        pytest.skip("well128_2000.npz not generated")
    g = np.load(path)
    w = W.c2_large_well()
    assert int(g["steps"]) == w.steps == 2000
    banner(f"full size {w.name}, {w.steps} steps against the oracle")
    b = L.box_from_workload(w, flags=int(g["flags"]))
    autotune.tune_zchunk(b)
    b.step(w.steps)
    assert not b.diagnostics()["unstable"]
    _compare_golden(b, g, w, "", "well128 t=2000")
    b.close()


def test_well128_fp32_populations_2000_steps(L):
    """The FP32-population variant of the 128^3 well over its stated 2000
    steps against the same FP64 oracle golden: the storage rounds every
    population to 24 bits each step, so the state drifts from the FP64 one
    by far more than 1e-11; the measured errors are printed and held to
    1e-5 (n) and 1e-2 (u, whose max is 4e-4), with the spurious max|u|."""
    from paper_1202_3842_amd import autotune
    path = GOLDEN / "well128_2000.npz"
    if not path.exists():
        pytest.skip("well128_2000.npz not generated")
    g = np.load(path)
    w = W.c2_large_well()
    banner(f"full size {w.name}, FP32 populations, {w.steps} steps against the FP64 oracle")
    b = L.box_from_workload(w, prec=L.LBE_FP32_POP, flags=int(g["flags"]))
    autotune.tune_zchunk(b)
    b.step(w.steps)
    d = b.diagnostics()
    assert not d["unstable"]
    z = int(g["zplane"])
    en = max(rel_err(b.density(0)[z], g["n0_plane"]),
             rel_err(b.density(0).reshape(-1)[g["nodes"]], g["n0_nodes"]))
    eu = max(rel_err(b.velocity(-1)[:, z], g["u_plane"]),
             rel_err(b.velocity(-1).reshape(3, -1)[:, g["nodes"]], g["u_nodes"]))
    print(f"[fp32] well128 t=2000: n rel err {en:.2e}, u rel err {eu:.2e}, max|u| {d['umax']:.3e}", flush=True)
    assert en <= 1e-5 and eu <= 1e-2, (en, eu)
    b.close()


def test_channel256_stated_5000_steps_against_oracle(L):
    """The 256x64x32 two-species channel over its stated 5000 steps (C^visc
    off: with it on the channel collapses within a few hundred steps under
    every reading tried), against the oracle's state
    (tests/golden/channel256_5000.npz)."""
    path = GOLDEN / "channel256_5000.npz"
    if not path.exists():
        pytest.skip("channel256_5000.npz not generated")
    g = np.load(path)
    w = W.c3_channel()
    assert int(g["steps"]) == w.steps == 5000
    banner(f"full size {w.name}, {w.steps} steps against the oracle")
    b = L.box_from_workload(w, flags=int(g["flags"]))
    b.step(w.steps)
    assert not b.diagnostics()["unstable"]
    _compare_golden(b, g, w, "", "channel256 t=5000")
    b.close()


def test_batched_boxes_500_steps_against_oracle(L):
    """A seeded sample of the 96-box set (boxes_500.npz: four boxes with
    edges up to 64 that stay stable), stepped 500 times inside the whole
    batched set (graph replay), against the oracle's states."""
    path = GOLDEN / "boxes_500.npz"
    if not path.exists():
        pytest.skip("boxes_500.npz not generated")
    g = np.load(path)
    ws = W.c4_boxes()
    steps = int(g["steps"])
    banner(f"batched 96 boxes, {steps} steps, boxes {list(g['boxes'])} against the oracle")
    batch = L.batch_from_workloads(ws, flags=int(g["flags"]))
    batch.step(steps)
    for k in g["boxes"]:
        b = batch.boxes[int(k)]
        assert not b.diagnostics()["unstable"], int(k)
        _compare_golden(b, g, ws[int(k)], f"box{int(k)}_", f"box {int(k)} t={steps}")
    batch.close()


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
