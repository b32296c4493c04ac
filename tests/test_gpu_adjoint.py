"""GPU adjoint (lbe_adjoint_*) against the reference gradient of
oracle/autograd_ref.py (autograd of the step re-expressed in torch, CPU
FP64), and on the 96x32x32 channel against central finite differences of
the C oracle (tests/golden/channel96_fd_grad.json)."""
import json
from pathlib import Path

import numpy as np
import pytest
import torch

from adjoint_util import small_channel, objective_terms, pop_weights
from paper_1202_3842_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden" / "channel96_fd_grad.json"
GOLDEN_VISC = Path(__file__).resolve().parent / "golden" / "channel96_visc_fd_grad.json"
GOLDEN_ALL = Path(__file__).resolve().parent / "golden" / "channel96_all_fd_grad.json"
GOLDEN_QP = Path(__file__).resolve().parent / "golden" / "channel96_qp_fd_grad.json"
# the reading in which g carries Pi (LBE_PI_CARRIED); without it the
# quasi-pressure is evaluated every step (the default)
CARRIED = 1 << 7


def reference(w, flags, T, pw):
    from oracle import autograd_ref as AR
    n_t, fluid, plane = objective_terms(w)
    geo = AR.Geometry(w.nx, w.ny, w.nz, w.periodic,
                      (w.solid if w.solid is not None else np.zeros(w.shape)).astype(bool))
    route = w.qp_route if w.qp_route is not None else (None, 2)
    st = AR.Stepper(geo, w.sigma, w.tau, w.kT, flags, w.body, att_eps=w.att_eps, att_rc=w.att_rc,
                    qp_origin=route[0], qp_symmetric=bool(route[1] & 2))
    V = torch.tensor(w.V.reshape(-1), requires_grad=True)
    f0, g0 = st.rest_state(np.stack(w.density))
    f0.requires_grad_(True)
    g0.requires_grad_(True)
    f, g = st.run(f0, g0, V, T)
    n, J = st.readout(f, g, V)
    L = ((n[0] - torch.tensor(n_t.reshape(-1))) ** 2 * torch.tensor(fluid.reshape(-1), dtype=torch.float64)).sum()
    L = L + (J[:, 0, :] * torch.tensor(plane.reshape(-1), dtype=torch.float64)).sum()
    if pw is not None:
        pwt = torch.tensor(pw.reshape(2, w.nspecies, 19, -1))
        L = L + (pwt[0] * f).sum() + (pwt[1] * g).sum()
    L.backward()
    # with one distribution g0 takes no part in L
    rg = g0.grad.numpy() if g0.grad is not None else np.zeros(tuple(g0.shape))
    return V.grad.numpy().reshape(w.shape), f0.grad.numpy(), rg


def gpu_gradient(w, flags, T, segment, pw, prec=0):
    from paper_1202_3842_amd import lbe
    box = lbe.box_from_workload(w, prec=prec, flags=flags)
    adj = lbe.Adjoint(box, T, segment)
    adj.forward()
    n_t, fluid, plane = objective_terms(w)
    M = w.nspecies
    dn = np.zeros((M,) + w.shape)
    dn[0] = 2.0 * (box.density(0) - n_t) * fluid
    dJ = np.zeros((M, 3) + w.shape)
    for a in range(M):
        dJ[a, 0] = plane
    gV = adj.backward(dn, dJ, pw)
    gf = np.stack([adj.state_grad(a, 0).reshape(19, -1) for a in range(M)])
    gg = np.stack([adj.state_grad(a, 1).reshape(19, -1) for a in range(M)])
    adj.close()
    box.close()
    return gV, gf, gg


def assert_close(got, ref, rtol, what):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    print(f"{what}: max|ref| {scale:.3e} max err {err:.3e}", flush=True)
    assert err <= rtol * scale, (what, err, scale)


@pytest.mark.parametrize("flags,T,segment", [
    (0, 6, 6), (0, 6, 4), (0, 7, 1), (2, 6, 3), (4, 5, 2), (2 | 4, 5, 5),
    (CARRIED, 6, 4), (CARRIED | 2, 6, 3), (CARRIED | 2 | 4, 5, 5)])
def test_adjoint_matches_reference(flags, T, segment):
    w = small_channel()
    pw = pop_weights(w) * 1e-3
    print(f"small channel flags {flags} T {T} segment {segment}", flush=True)
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, segment, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("flags,T,segment", [(0, 6, 6), (0, 7, 3), (2 | 4, 5, 2)])
def test_adjoint_with_attraction_matches_reference(flags, T, segment):
    """The two-species channel with the attractive tails on (depths 0.2 to
    0.3 kT, cutoff 5): the transpose of the attraction gather joins the
    adjoint of the density."""
    w = small_channel()
    w.att_eps = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]]
    w.att_rc = 5.0
    pw = pop_weights(w) * 1e-3
    print(f"small channel with attraction flags {flags} T {T} segment {segment}", flush=True)
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, segment, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("flags,att,T,segment", [(64, False, 6, 3), (64 | 2, False, 5, 5),
                                                 (64 | 4, True, 6, 2)])
def test_adjoint_with_drag_matches_reference(flags, att, T, segment):
    """The two-species channel with the interspecies drag (flag 64): its
    reverse joins the collision and read-out adjoints (n, J~ and the contact
    values), with either inversion, and with the attractive tails on too."""
    w = small_channel()
    if att:
        w.att_eps, w.att_rc = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]], 5.0
    pw = pop_weights(w) * 1e-3
    print(f"small channel with drag flags {flags} att {att} T {T} segment {segment}", flush=True)
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, segment, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("flags,T,segment", [(16, 6, 3), (16 | 2 | 64, 5, 5), (32, 6, 2),
                                               (32 | 16, 5, 3), (32 | 64, 6, 6), (CARRIED | 16, 6, 3)])
def test_adjoint_scheme_variants_match_reference(flags, T, segment):
    """The scheme variants of Sec. 4 on the two-species channel: DD-EU
    (flag 16; with the printed inversion and the drag too), SD-TR (32),
    SD-EU and SD-TR with the drag.  With one distribution there is no g: the
    g part of the seed is zero and the g gradient is zero."""
    w = small_channel()
    pw = pop_weights(w) * 1e-3
    single = bool(flags & 32)
    if single:
        pw[1] = 0.0
    print(f"small channel scheme variant flags {flags} T {T} segment {segment}", flush=True)
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, segment, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    if single:
        assert not gg.any() and not rg.any()
    else:
        assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("flags,att,T,segment", [(1, False, 6, 3), (1 | 2, False, 5, 5), (1 | 4, False, 6, 1),
                                                 (1 | 64, False, 6, 2), (1 | 32, False, 5, 5),
                                                 (1 | 2 | 64, True, 5, 2)])
def test_adjoint_with_visc_matches_reference(flags, att, T, segment):
    """C^visc (flag 1) on the two-species channel: its two transposes per
    directed pair (MODE 5 over phibar', G and u~; MODE 6 over n, G and J~
    with the centre phibar') with either inversion, kappa = 4, the drag,
    one distribution, and the drag and attractive tails together."""
    w = small_channel()
    if att:
        w.att_eps, w.att_rc = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]], 5.0
    pw = pop_weights(w) * 1e-3
    single = bool(flags & 32)
    if single:
        pw[1] = 0.0
    print(f"small channel with C^visc flags {flags} att {att} T {T} segment {segment}", flush=True)
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, segment, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    if not single:
        assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("flags", [1, 1 | 2], ids=["default", "printed"])
def test_adjoint_visc_one_species_periodic_well(flags):
    """One species, sigma = 3, periodic, C^visc on: the default scheme (the
    128^3 benchmark box's: derived inversion, quasi-pressure every step as
    the six-order mean from the centre) and the printed inversions."""
    w = W.well_box(16, 3.0, 0.3, W.eps_for_depth(1.0), 5.0, 1e-2, 33, 5, "well16_s3_visc")
    w.V = w.V + W.smooth_field(w.shape, 0.02, 3, 34)
    w.solid = np.zeros(w.shape, dtype=np.uint8)
    pw = pop_weights(w, 8) * 1e-3
    print(f"well16 sigma 3 one species with C^visc, flags {flags}", flush=True)
    rV, rf, rg = reference(w, flags, 5, pw)
    gV, gf, gg = gpu_gradient(w, flags, 5, 2, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


def test_adjoint_attraction_one_species_periodic():
    """One species, periodic box, a cutoff of 7.5 (the widest transpose
    window, 7 nodes per axis) and a potential well."""
    w = W.well_box(18, 3.0, 0.25, W.eps_for_depth(1.0), 5.0, 1e-2, 41, 5, "well18_s3_att")
    w.V = w.V + W.smooth_field(w.shape, 0.02, 3, 42)
    w.solid = np.zeros(w.shape, dtype=np.uint8)
    w.att_eps, w.att_rc = [[0.3 * W.KT]], 7.5
    pw = pop_weights(w, 7) * 1e-3
    print("well18 sigma 3 one species with attraction", flush=True)
    rV, rf, rg = reference(w, 0, 4, pw)
    gV, gf, gg = gpu_gradient(w, 0, 4, 2, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")


def test_adjoint_one_species_periodic_well():
    w = W.well_box(16, 3.0, 0.3, W.eps_for_depth(1.0), 5.0, 1e-2, 31, 5, "well16_s3")
    w.V = w.V + W.smooth_field(w.shape, 0.02, 3, 32)
    w.solid = np.zeros(w.shape, dtype=np.uint8)
    pw = pop_weights(w, 6) * 1e-3
    print("well16 sigma 3 one species", flush=True)
    rV, rf, rg = reference(w, 0, 5, pw)
    gV, gf, gg = gpu_gradient(w, 0, 5, 2, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")


def test_autograd_function_matches_adjoint():
    from paper_1202_3842_amd import lbe
    w = small_channel()
    n_t, fluid, plane = objective_terms(w)
    box = lbe.box_from_workload(w, flags=0)
    adj = lbe.Adjoint(box, 5, 2)
    n0 = [torch.tensor(d, device="cuda") for d in w.density]

    def reset(b):
        for a, d in enumerate(n0):
            b.init_density(a, d.reshape(-1))

    V = torch.tensor(w.V, device="cuda", requires_grad=True)
    n, J = lbe.potential_to_state(V, adj, reset)
    nt = torch.tensor(n_t, device="cuda")
    fl = torch.tensor(fluid, device="cuda", dtype=torch.float64)
    pl = torch.tensor(plane, device="cuda", dtype=torch.float64)
    L = (((n[0] - nt) ** 2) * fl).sum() + (J[:, 0] * pl).sum()
    L.backward()
    rV, _, _ = reference(w, 0, 5, None)
    assert_close(V.grad.cpu().numpy(), rV, 1e-10, "autograd dL/dV")


@pytest.mark.parametrize("golden,steps,segment", [(GOLDEN_QP, 400, 20), (GOLDEN, 400, 20), (GOLDEN_VISC, 40, 10),
                                                    (GOLDEN_ALL, 40, 40)],
                         ids=["cmf_400_default", "cmf_400_carried", "visc_printed_40", "all_forces_40"])
def test_channel96_gradient_against_oracle_fd(golden, steps, segment):
    """dL/dV on the 96x32x32 channel against central differences of the
    oracle: C^mf with the derived inversions over 400 steps, with the
    quasi-pressure evaluated every step (the default) and with Pi carried by
    g; C^visc with
    the printed inversions over 40 steps; and every force (C^visc, the drag
    and the attractive tails, printed inversions) over 40 steps in one
    segment."""
    from paper_1202_3842_amd import lbe
    if not golden.exists():
        pytest.skip(f"finite-difference golden file {golden.name} not generated")
    gold = json.loads(golden.read_text())
    w = W.c5_channel()
    w.steps = steps
    if gold.get("att_eps_kT", 0.0) > 0:
        w.att_eps = [[gold["att_eps_kT"] * w.kT] * w.nspecies] * w.nspecies
        w.att_rc = gold["att_rc"]
    assert gold["workload"] == w.name and gold["steps"] == w.steps
    n_t, fluid, plane = W.c5_objective(w)
    box = lbe.box_from_workload(w, flags=gold["flags"])
    adj = lbe.Adjoint(box, w.steps, segment)
    adj.forward()
    nA = box.density(0)
    d = box.diagnostics()
    assert not d["unstable"]
    M = w.nspecies
    dn = np.zeros((M,) + w.shape)
    dn[0] = 2.0 * (nA - n_t) * fluid
    dJ = np.zeros((M, 3) + w.shape)
    for a in range(M):
        dJ[a, 0] = plane
    L = float(np.sum(((nA - n_t) ** 2)[fluid])) + sum(
        float(np.sum(box.momentum(a)[0][plane])) for a in range(M))
    assert abs(L - gold["L0"]) <= 1e-9 * abs(gold["L0"])
    gV = adj.backward(dn, dJ).reshape(-1)
    rows = gold["rows"]
    scale = max(abs(r["grad"]) for r in rows)
    # central differences carry ~eps |L| / h of rounding noise
    noise = 2.2e-16 * abs(gold["L0"]) / gold["h"]
    worst = 0.0
    rel = []
    for r in rows:
        err = abs(gV[r["node"]] - r["grad"])
        worst = max(worst, err)
        assert err <= 1e-6 * scale + 10 * noise, (r["node"], gV[r["node"]], r["grad"])
        # per node, relative to its own gradient where that stands clear of
        # the finite-difference noise; the two runs of a central difference
        # round differently over hundreds of steps (two FP64 forwards agree
        # to ~1e-13 relative after 400 steps, ~500 eps), so the noise floor
        # here is 100 x eps |L| / h
        if abs(r["grad"]) > 1e4 * noise:
            rel.append(err / abs(r["grad"]))
            assert err <= 1e-6 * abs(r["grad"]) + 100 * noise, (r["node"], gV[r["node"]], r["grad"])
    rel = np.array(rel if rel else [0.0])
    print(f"channel96: {len(rows)} nodes, max|grad| {scale:.3e}, worst err {worst:.3e}, "
          f"fd noise {noise:.1e}; per node ({len(rel)} above 1e4 x noise): relative error "
          f"median {np.median(rel):.1e}, max {rel.max():.1e}", flush=True)


@pytest.mark.parametrize("att,flags", [(False, 0), (True, 0), (False, 1)])
def test_adjoint_tiling_does_not_change_gradient(att, flags):
    """The adjoint shell-gather transposes (and those of the attraction and
    of C^visc) under every force tiling."""
    from paper_1202_3842_amd import lbe
    w = small_channel()
    if att:
        w.att_eps, w.att_rc = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]], 5.0
    n_t, fluid, plane = objective_terms(w)
    ref = None
    for zc, order, shape in ((1, 0, 0), (3, 1, 1), (8, 2, 2), (2, 0, 1)):
        print(f"adjoint tiling att {att} flags {flags} zchunk {zc} order {order} shape {shape}", flush=True)
        box = lbe.box_from_workload(w, flags=flags)
        box.set_force_tiling(zc, order, shape)
        adj = lbe.Adjoint(box, 4, 2)
        adj.forward()
        dn = np.zeros((2,) + w.shape)
        dn[0] = 2.0 * (box.density(0) - n_t) * fluid
        g = adj.backward(dn, None, None)
        adj.close()
        box.close()
        if ref is None:
            ref = g
        else:
            assert np.array_equal(g, ref), (zc, order, shape)


def test_adjoint_attraction_tile_rows_agree():
    """The attraction gathers take one or two output rows per thread by the
    number of tiles: on a 128 x 64 x 64 box, z-chunks of 1 give 1024 tiles of
    32 x 16 (two rows per thread), z-chunks of 4 give 256 (one row, 32 x 8
    tiles).  The gradient is bitwise the same on both paths (the small-box
    checks above compare the one-row path with the reference)."""
    from paper_1202_3842_amd import lbe
    nx, ny, nz = 128, 64, 64
    sh = (nz, ny, nx)
    w = W.Workload(name="box128x64x64_att", nx=nx, ny=ny, nz=nz, sigma=[3.0], steps=3,
                   density=[W.noisy_uniform(sh, W.packing_density(0.2, 3.0), 1e-2, 51)],
                   V=W.smooth_field(sh, 0.1 * W.KT, 3, 52), body=[[1e-4, 0.0, 0.0]])
    w.att_eps, w.att_rc = [[0.25 * W.KT]], 6.0
    grads, dens = [], []
    for zc in (1, 4):
        print(f"adjoint attraction tile rows: zchunk {zc}", flush=True)
        box = lbe.box_from_workload(w, flags=0)
        box.set_force_tiling(zc, 1, 0)
        adj = lbe.Adjoint(box, 3, 3)
        adj.forward()
        n = box.density(0)
        dn = (n - n.mean())[None]
        grads.append(adj.backward(dn, None, None))
        dens.append(n)
        adj.close()
        box.close()
    assert np.array_equal(dens[0], dens[1])
    assert np.abs(grads[0]).max() > 0
    assert np.array_equal(grads[0], grads[1])


@pytest.mark.parametrize("att", [False, True], ids=["visc", "visc_attraction"])
def test_adjoint_full_size_directional_derivative(att):
    """The 128^3 benchmark box (sigma = 6, C^visc, the default scheme) in the
    launch configuration bench.py times, 3 steps: the adjoint's dL/dV along
    a smooth direction dV equals the central difference of L along dV (the
    library's own forward at V +- h dV), for L = sum_r c(r) n(r, T) with
    seeded weights c.  Also with the attractive tail (eps = kT/4, rc = 8),
    whose transpose takes its two-row tiles at this size.  A property that
    holds at any size; the reference gradient covers the small boxes."""
    from paper_1202_3842_amd import lbe, autotune
    w = W.c2_large_well()
    if att:
        w.att_eps, w.att_rc = [[0.25 * W.KT]], 8.0
    flags = lbe.LBE_VISC
    T = 3
    c = W.rng(61).uniform(-1.0, 1.0, size=w.shape)
    dV = W.smooth_field(w.shape, 0.1 * W.KT, 4, 62)
    box = lbe.box_from_workload(w, flags=flags)
    autotune.tune_zchunk(box)
    print(f"full size adjoint, tiling {getattr(box, 'tiling', None)}", flush=True)
    adj = lbe.Adjoint(box, T, T)
    lbe.load_workload(box, w)
    adj.forward()
    gV = adj.backward(c[None], None, None)
    adj.close()
    ana = float(np.sum(gV * dV))

    def loss(V):
        lbe.load_workload(box, w)
        box.set_potential(np.ascontiguousarray(V))
        box.step(T)
        return float(np.sum(c * box.density(0)))

    h = 1e-4
    L0 = loss(w.V)
    fd = (loss(w.V + h * dV) - loss(w.V - h * dV)) / (2 * h)
    box.close()
    noise = 2.2e-16 * np.abs(c).sum() * float(w.density[0].max()) / h
    print(f"full size: adjoint {ana:.9e}, central difference {fd:.9e}, L {L0:.6e}, noise {noise:.1e}",
          flush=True)
    assert abs(ana) > 100 * noise
    assert abs(ana - fd) <= 1e-6 * abs(ana) + 10 * noise


@pytest.mark.parametrize("seed", range(12))
def test_adjoint_random_configurations(seed):
    """Seeded random channels (sizes, diameters, C^visc, printed inversion,
    kappa = 4, Euler, one distribution, drag and the attractive tails each
    switched on at random; random horizon and segment) against the reference
    gradient."""
    import math
    g = W.rng(7000 + seed)
    sig = [(2.0, 3.0), (3.0, 2.0), (2.0, 2.0), (1.0, 3.0)][int(g.integers(0, 4))]
    w = small_channel(nx=int(g.integers(10, 16)), ny=10, nz=int(g.integers(7, 12)), sigma=sig, seed=100 + seed)
    flags = 0
    for bit in (1, 2, 4, 16, 32, 64):
        if g.uniform() < 0.4:
            flags |= bit
    att = g.uniform() < 0.4
    if att:
        w.att_eps, w.att_rc = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]], float(g.uniform(4.0, 6.0))
        for k, d in enumerate((w.nx, w.ny, w.nz)):
            if (w.periodic >> k) & 1 and d < math.ceil(w.att_rc):
                w.periodic &= ~(1 << k)
    T = int(g.integers(3, 7))
    seg = int(g.integers(1, T + 1))
    if g.uniform() < 0.3:                 # the carried reading of Pi (drawn last)
        flags |= CARRIED
    print(f"random adjoint {seed}: {w.nx}x{w.ny}x{w.nz} sigma {sig} flags {flags} att {att} T {T} "
          f"segment {seg}", flush=True)
    pw = pop_weights(w) * 1e-3
    if flags & 32:
        pw[1] = 0.0
    rV, rf, rg = reference(w, flags, T, pw)
    gV, gf, gg = gpu_gradient(w, flags, T, seg, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")


@pytest.mark.parametrize("flags", [1 | 2, 0, 1 | 64])
def test_adjoint_fp32_storage(flags):
    """FP32 population storage: the reverse of the FP64 step along the FP32
    trajectory.  It differs from the FP64 gradient by the storage rounding
    only (bar 1e-5 of the max-norm; the forward's FP32 error is ~5e-8)."""
    from paper_1202_3842_amd import lbe
    w = small_channel()
    pw = pop_weights(w) * 1e-3
    print(f"small channel FP32 storage flags {flags}", flush=True)
    rV, rf, rg = reference(w, flags, 5, pw)
    gV, gf, gg = gpu_gradient(w, flags, 5, 2, pw, prec=lbe.LBE_FP32_POP)
    assert_close(gV, rV, 1e-5, "dL/dV (fp32 storage)")
    assert_close(gf, rf, 1e-5, "dL/df0 (fp32 storage)")
    assert_close(gg, rg, 1e-5, "dL/dg0 (fp32 storage)")


@pytest.mark.parametrize("flags", [0, 1 | 2 | 64, CARRIED])
def test_taped_forward_equals_checkpointed(flags):
    """With one segment the forward records the tape and the backward does
    no recompute: the final state equals plain stepping and the gradient
    equals the checkpointed one, bit for bit."""
    from paper_1202_3842_amd import lbe
    w = small_channel()
    n_t, fluid, plane = objective_terms(w)
    T = 6
    plain = lbe.box_from_workload(w, flags=flags)
    plain.step(T)
    grads = []
    for seg in (T, 2):
        box = lbe.box_from_workload(w, flags=flags)
        adj = lbe.Adjoint(box, T, seg)
        adj.forward()
        for dist in (0, 1):
            assert np.array_equal(box.populations(0, dist), plain.populations(0, dist)), (seg, dist)
        dn = np.zeros((2,) + w.shape)
        dn[0] = 2.0 * (box.density(0) - n_t) * fluid
        grads.append(adj.backward(dn, None, None))
        adj.close()
        box.close()
    plain.close()
    assert np.abs(grads[0]).max() > 0
    assert np.array_equal(grads[0], grads[1])


@pytest.mark.parametrize("flags,att", [(1 | 64, True), (2 | 4, False)])
def test_adjoint_three_species(flags, att):
    """Three species (sigma 2, 3 and 2.5) on the small channel: every
    directed pair's transposes, the drag between three species and the
    attractive tails of six pairs, against the reference gradient."""
    w = small_channel()
    w.sigma = [2.0, 3.0, 2.5]
    w.density = w.density + [W.noisy_uniform(w.shape, float(w.density[0].mean()) * 0.5, 1e-2, 431)]
    w.body = w.body + [[-5e-5, 1e-5, 0.0]]
    if att:
        e = np.array([[0.3, 0.2, 0.25], [0.2, 0.25, 0.15], [0.25, 0.15, 0.2]]) * W.KT
        w.att_eps, w.att_rc = e.tolist(), 5.0
    pw = pop_weights(w) * 1e-3
    print(f"small channel three species flags {flags} att {att}", flush=True)
    rV, rf, rg = reference(w, flags, 5, pw)
    gV, gf, gg = gpu_gradient(w, flags, 5, 2, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


@pytest.mark.parametrize("route", [((3, 5, 2), 0), ((9, 4, 6), 2), ((6, 4, 3), 3)])
def test_adjoint_quasipressure_routes(route):
    """The per-step quasi-pressure from off-centre origins, along the x, y, z
    path and as the six-order mean (with n F in the integrand too: mode 3),
    on the two-species channel with C^visc and the drag."""
    from oracle import autograd_ref as AR
    w = small_channel()
    w.qp_route = route
    pw = pop_weights(w) * 1e-3
    flags = 1 | 64
    print(f"small channel quasi-pressure route {route}", flush=True)
    if route[1] & 1:
        # the reference integrates C^mf alone: check the library against
        # itself along a direction instead (central difference of L)
        from paper_1202_3842_amd import lbe
        n_t, fluid, plane = objective_terms(w)
        dV = W.smooth_field(w.shape, 0.05 * W.KT, 3, 91)
        box = lbe.box_from_workload(w, flags=flags)
        adj = lbe.Adjoint(box, 5, 2)
        adj.forward()
        dn = np.zeros((2,) + w.shape)
        dn[0] = 2.0 * (box.density(0) - n_t) * fluid
        dJ = np.zeros((2, 3) + w.shape)
        dJ[:, 0] = plane
        gV = adj.backward(dn, dJ, None)
        adj.close()

        def L(V):
            lbe.load_workload(box, w)
            box.set_potential(np.ascontiguousarray(V))
            box.step(5)
            return float(np.sum(((box.density(0) - n_t) ** 2)[fluid])) + sum(
                float(np.sum(box.momentum(a)[0][plane])) for a in range(2))

        h = 1e-5
        fd = (L(w.V + h * dV) - L(w.V - h * dV)) / (2 * h)
        ana = float(np.sum(gV * dV))
        box.close()
        print(f"route {route}: adjoint {ana:.10e} central difference {fd:.10e}", flush=True)
        assert abs(ana - fd) <= 1e-7 * abs(ana)
        return
    rV, rf, rg = reference(w, flags, 5, pw)
    gV, gf, gg = gpu_gradient(w, flags, 5, 2, pw)
    assert_close(gV, rV, 1e-10, "dL/dV")
    assert_close(gf, rf, 1e-10, "dL/df0")
    assert_close(gg, rg, 1e-10, "dL/dg0")


def test_backward_refuses_changed_parameters():
    """lbe_adjoint_backward after the potential, a body force or the
    quasi-pressure route changed since the forward: LBE_ERR_STATE; and the
    autograd Function refuses a backward whose forward was overwritten by a
    later one on the same Adjoint."""
    import torch
    from paper_1202_3842_amd import lbe
    w = small_channel()
    n_t, fluid, plane = objective_terms(w)
    dn = np.zeros((2,) + w.shape)
    for change in ("potential", "body", "route"):
        box = lbe.box_from_workload(w, flags=0)
        adj = lbe.Adjoint(box, 3, 3)
        adj.forward()
        if change == "potential":
            box.set_potential(np.ascontiguousarray(w.V * 1.01))
        elif change == "body":
            box.set_body_force(0, np.array([2e-4, 0.0, 0.0]))
        else:
            box.set_quasipressure_route((4, 5, 3), 0)
        with pytest.raises(lbe.LBEError) as e:
            adj.backward(dn, None, None)
        assert e.value.code == lbe.LBE_ERR_STATE
        adj.close()
        box.close()
    box = lbe.box_from_workload(w, flags=0)
    adj = lbe.Adjoint(box, 3, 3)
    n0 = [torch.tensor(d, device="cuda") for d in w.density]

    def reset(b):
        for a, d in enumerate(n0):
            b.init_density(a, d.reshape(-1))

    V = torch.tensor(w.V, device="cuda", requires_grad=True)
    n1, J1 = lbe.potential_to_state(V, adj, reset)
    n2, J2 = lbe.potential_to_state(V * 1.0, adj, reset)
    with pytest.raises(RuntimeError):
        n1.sum().backward()
    adj.close()
    box.close()
