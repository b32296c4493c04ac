#!/usr/bin/env python
"""Throughput of the stabilized Lattice Boltzmann-Enskog step (DD-TR) on one
MI355X: MLUPS per species and the HBM-roofline fraction of the dominant
kernel, with the CPU oracle timed beside it.

Workload (default): one-component hard spheres, D3Q19, 128^3 periodic box,
sigma = 6, n sigma^3 = 0.4, cosine well of radius 24 and depth 2 kT at the
centre, collisional viscous force on, FP64.  A "step" is one full DD-TR step
(moments, contact values, force gather, collision, streaming) of the whole
box.  Inputs are resident in HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes_collide(M, P, qp=True):
    """Algorithmic bytes per node of the collision kernel: pull of 2 x 19
    populations per species, store of the same, the per-particle forces
    (6 doubles per species), the path integral of the per-step
    quasi-pressure (one double per species), the external force (3 doubles)
    and the bounce-back mask (4 bytes)."""
    return M * (2 * 19 * P * 2 + 48 + (8 if qp else 0)) + 24 + 4


def alg_flops_force(pairs, visc):
    """FP64 flops per node of the shell gather (FMA = 2): per +-e pair the
    mean-field term costs 11 and the viscous term 27."""
    return pairs * (11 + (27 if visc else 0))


def alg_bytes_step(M, npairs, P, visc, qp=True):
    """Per node and step: populations read once and written once (the
    minimum the method must move) plus one pass over the node fields: n and
    G written and read, V, J~ with C^visc, and the per-step quasi-pressure's
    path integral written once and read once by the collision."""
    fields = 8 * M + 8 * M + 8 * npairs + 8 * npairs + 8  # n write+read, G write+read, V
    if visc:
        fields += 48 * M
    if qp:
        fields += 16 * M
    return M * 2 * 38 * P + fields


def shell_pairs(sigma):
    """Number of +-e pairs in the lattice shell of radius sigma."""
    K = int(sigma + 1.5)
    n = 0
    for z in range(-K, K + 1):
        for y in range(-K, K + 1):
            for x in range(-K, K + 1):
                r2 = x * x + y * y + z * z
                if r2 and (sigma - 0.5) ** 2 <= r2 < (sigma + 0.5) ** 2:
                    n += 1
    return n // 2


FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_well128_s6.json")
# the kernel sources the committed counter summary was taken on; a summary of
# other sources is not used
TRAFFIC_REV = "pi-per-step-4"
TRAFFIC_SOURCE = ("profiles/hbm_traffic_well128_s6.json: rocprofv3 FETCH_SIZE and WRITE_SIZE "
                  "of this launch, committed, scaled by a plain copy (not measured in this run)")


def measured_traffic(kernel, grid, order=None):
    """HBM bytes per launch of `kernel` launched with `grid` threads (and, for
    the force kernel, tile order `order`), from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary scaled by a plain copy, or None when that
    launch was not measured on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
        if data.get("rev") != TRAFFIC_REV:
            return None
        table = data["kernels"]
    except (OSError, ValueError, KeyError):
        return None
    key = f"{kernel}|{grid}" + ("" if order is None else f"|order{order}")
    v = table.get(key)
    return None if v is None else int(round(v))


def force_launch(box, sigma, visc):
    """(kernel name, grid threads) of the force kernel for the box's tiling."""
    z, order, shape = getattr(box, "tiling", (2, 1, 0))
    nt = 512 if shape == 2 else 256
    ny = 2 if shape == 1 else 1
    ty = nt // 32 * ny
    R = int(sigma + 0.5)
    c = box.cfg
    blocks = -(-c.nx // 32) * -(-c.ny // ty) * -(-c.nz // z)
    return f"k_force<{R}, {'true' if visc else 'false'}, {ny}, {nt}>", blocks * nt


LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12   # 256 CUs x 128 B/clk x 2.4 GHz = 78.6 TB/s


def lds_bytes_force(pairs, visc):
    """LDS bytes read per node by the force gather: per +-e pair, n and G at
    both points (and J~ with C^visc), 8 bytes each."""
    return pairs * 8 * (2 * (5 if visc else 2))


def kernel_views(r, N, M, P, pairs, prec_name):
    """Per-kernel roofline views: the collision kernel against HBM, the force
    gather against FP64 vector throughput (and, beside it, LDS bandwidth)."""
    bcoll = alg_bytes_collide(M, P)
    coll_gbs = bcoll * N / (r["collide_ms"] / 1e3) / 1e9
    fl = alg_flops_force(pairs, True) * M * M
    force_tf = fl * N / (r["force_ms"] / 1e3) / 1e12
    lds = lds_bytes_force(pairs, True) * M * M
    lds_tbs = lds * N / (r["force_ms"] / 1e3) / 1e12
    fname, fgrid = r["force_launch"]
    return {
        "k_collide": {"bound": "hbm", "achieved": round(coll_gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(coll_gbs / HBM_PEAK_GBS, 4),
                      "alg_bytes_per_node": bcoll, "avg_launch_ms": round(r["collide_ms"], 4),
                      "traffic": measured_traffic(f"k_collide<{prec_name}, {M}>", N),
                      "traffic_source": TRAFFIC_SOURCE},
        "k_force": {"bound": "alu", "achieved": round(force_tf, 2), "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(force_tf / FP64_PEAK_TFLOPS, 4),
                    "alg_flops_per_node": fl, "avg_launch_ms": round(r["force_ms"], 4),
                    "traffic": measured_traffic(fname, fgrid, r["tiling"][1] if r["tiling"] else None),
                    "traffic_source": TRAFFIC_SOURCE,
                    "launch": fname, "grid": fgrid,
                    "tiling": r["tiling"],
                    "lds_view": {"achieved": round(lds_tbs, 2), "peak": round(LDS_PEAK_TBS, 1),
                                 "unit": "TB/s", "frac": round(lds_tbs / LDS_PEAK_TBS, 4),
                                 "lds_bytes_per_node": lds}},
    }


def dominant(kv):
    name = max(kv, key=lambda k: kv[k]["avg_launch_ms"])
    d = dict(kv[name])
    d["kernel"] = name
    return d


def run_gpu(w, prec, flags, steps, warmup, lbe, torch, runs=5):
    """Warm up, then time exactly `steps` steps as `runs` consecutive runs
    (HIP events on the box's stream around every phase of every step);
    ms_per_step is the median over the runs."""
    from paper_1202_3842_amd import autotune
    box = lbe.box_from_workload(w, prec=prec, flags=flags)
    z = autotune.tune_zchunk(box)
    log(f"force-kernel tiling (zchunk, order, shape) {getattr(box, 'tiling', (z, None, None))}")
    box.step(warmup)
    box.synchronize()
    log(f"warmup {warmup} steps done ({'fp64' if prec == lbe.LBE_FP64 else 'fp32-pop'})")
    stream = box.stream
    mk = lambda: torch.cuda.Event(enable_timing=True)
    runs = max(1, min(runs, steps))
    sizes = [steps // runs + (1 if r < steps % runs else 0) for r in range(runs)]
    ev = [[mk() for _ in range(5)] for _ in range(steps)]
    rev = [(mk(), mk()) for _ in range(runs)]
    torch.cuda.synchronize()
    k = 0
    for r, size in enumerate(sizes):
        rev[r][0].record(stream)
        for _ in range(size):
            box.step_phase(0)
            box.step_phase(1)
            ev[k][0].record(stream)
            box.step_phase(2)
            ev[k][1].record(stream)
            box.step_phase(3)
            ev[k][2].record(stream)
            box.step_phase(4)
            ev[k][3].record(stream)
            k += 1
        rev[r][1].record(stream)
    rev[-1][1].synchronize()
    torch.cuda.synchronize()
    run_ms = [a.elapsed_time(b) / size for (a, b), size in zip(rev, sizes)]
    total_ms = sum(a.elapsed_time(b) for a, b in rev)
    force = [e[0].elapsed_time(e[1]) for e in ev]
    qp = [e[1].elapsed_time(e[2]) for e in ev]
    coll = [e[2].elapsed_time(e[3]) for e in ev]
    med = sorted(run_ms)[len(run_ms) // 2]
    diag = box.diagnostics()
    res = {"total_ms": total_ms, "ms_per_step": med, "run_ms_per_step": run_ms,
           "force_ms": sum(force) / steps, "qp_ms": sum(qp) / steps, "collide_ms": sum(coll) / steps,
           "diag": diag, "force_launch": force_launch(box, w.sigma[0], bool(flags & lbe.LBE_VISC)),
           "tiling": list(getattr(box, "tiling", ()))}
    log(f"timed {steps} steps in {runs} runs: median {med:.4f} ms/step (runs {[round(x, 4) for x in run_ms]}), "
        f"force {res['force_ms']:.3f} ms, quasi-pressure {res['qp_ms']:.3f} ms, collide {res['collide_ms']:.3f} ms")
    box.close()
    return res


def batch_leg(lbe, torch, W, flags, prec, steps, serial_steps, tune=True, Lmin=24, Lmax=96):
    """96 independent boxes of uneven sizes and diameters: batched launches
    replayed from a HIP graph against the same boxes stepped one after
    another with per-box launches.  The specified set has edges 24..96; with
    smaller edges the per-box launch cost dominates the serial schedule."""
    from paper_1202_3842_amd import autotune
    ws = W.c4_boxes(Lmin=Lmin, Lmax=Lmax)
    nodes = sum(w.nodes for w in ws)
    batch = lbe.batch_from_workloads(ws, prec=prec, flags=flags)
    if tune:
        for b in batch.boxes:
            autotune.tune_zchunk(b)
    st = batch.stream
    batch.step(2, mode=2)
    torch.cuda.synchronize()
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    e0.record(st)
    batch.step(steps, mode=2)
    e1.record(st)
    e1.synchronize()
    t_batch = e0.elapsed_time(e1) / steps
    log(f"batched {len(ws)} boxes: {t_batch:.3f} ms/step")
    e2.record(st)
    batch.step(serial_steps, mode=0)
    e3.record(st)
    e3.synchronize()
    t_serial = e2.elapsed_time(e3) / serial_steps
    log(f"serial {len(ws)} boxes: {t_serial:.3f} ms/step")
    unstable = sum(1 for b in batch.boxes if b.diagnostics()["unstable"])
    batch.close()
    return {
        "workload": f"{len(ws)} one-component boxes, edge {Lmin}..{Lmax}, sigma in {{3,4,6}}, "
                    "n sigma^3 in [0.1,0.45], well depth 0.5..3 kT",
        "nodes": nodes, "steps": steps, "serial_steps": serial_steps,
        "ms_per_step": round(t_batch, 4), "serial_ms_per_step": round(t_serial, 4),
        "value": round(nodes / (t_batch / 1e3) / 1e6, 2), "unit": "MLUPS",
        "serial_value": round(nodes / (t_serial / 1e3) / 1e6, 2),
        "batched_vs_serial": round(t_serial / t_batch, 3),
        "boxes_flagged_unstable": unstable,
    }


def variants_leg(lbe, torch, w, base_flags, steps, warmup):
    """The other schemes of Sec. 4 on the same workload and precision (FP64):
    DD-EU, SD-TR and SD-EU (SD streams and collides f only)."""
    out = {}
    N, M = w.nodes, w.nspecies
    for name, fl in (("DD-EU", lbe.LBE_EULER), ("SD-TR", lbe.LBE_SINGLE),
                     ("SD-EU", lbe.LBE_SINGLE | lbe.LBE_EULER)):
        r = run_gpu(w, lbe.LBE_FP64, base_flags | fl, steps, warmup, lbe, torch)
        out[name] = {
            "value": round(N * M / (r["ms_per_step"] / 1e3) / 1e6, 2), "unit": "MLUPS",
            "steps": steps, "ms_per_step": round(r["ms_per_step"], 4),
            "force_ms": round(r["force_ms"], 4), "collide_ms": round(r["collide_ms"], 4),
            "umax": r["diag"]["umax"], "unstable": r["diag"]["unstable"],
        }
    return out


def adjoint_leg(lbe, torch, W, segment=20, att=False):
    """dL/dV on the 96x32x32 two-species channel (C^mf scheme, the default
    per-step quasi-pressure; 400 steps):
    the forward with a checkpoint every `segment` steps and the backward
    (segment recompute + adjoint steps) against 400 plain forward steps.
    With att, the attractive tails are on (eps = kT/4 for every pair,
    rc = 8)."""
    from paper_1202_3842_amd import autotune
    import numpy as np
    w = W.c5_channel()
    if att:
        w.att_eps, w.att_rc = [[0.25 * W.KT] * w.nspecies] * w.nspecies, 8.0
    T = w.steps
    n_t, fluid, plane = W.c5_objective(w)
    box = lbe.box_from_workload(w, flags=0)
    autotune.tune_zchunk(box)
    st = box.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    box.step(10)
    lbe.load_workload(box, w)
    torch.cuda.synchronize()
    ev[0].record(st)
    box.step(T)
    ev[1].record(st)
    ev[1].synchronize()
    t_plain = ev[0].elapsed_time(ev[1])
    adj = lbe.Adjoint(box, T, segment)
    lbe.load_workload(box, w)
    torch.cuda.synchronize()
    ev[2].record(st)
    adj.forward()
    ev[3].record(st)
    ev[3].synchronize()
    t_fwd = ev[2].elapsed_time(ev[3])
    M = w.nspecies
    nA = box.density(0)
    dn = np.zeros((M,) + w.shape)
    dn[0] = 2.0 * (nA - n_t) * fluid
    dJ = np.zeros((M, 3) + w.shape)
    for a in range(M):
        dJ[a, 0] = plane
    dn_d = torch.tensor(dn, device="cuda")
    dJ_d = torch.tensor(dJ, device="cuda")
    out = torch.empty(w.nodes, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ev[4].record(st)
    adj.backward(dn_d, dJ_d, None, out=out)
    ev[5].record(st)
    ev[5].synchronize()
    t_bwd = ev[4].elapsed_time(ev[5])
    gnorm = float(out.abs().max())
    adj.close()
    # the same with one segment: the forward records the whole tape
    # (T + 1 slots) and the backward recomputes nothing
    one = None
    if not att:
        adj = lbe.Adjoint(box, T, T)
        lbe.load_workload(box, w)
        torch.cuda.synchronize()
        ev[2].record(st)
        adj.forward()
        ev[3].record(st)
        ev[3].synchronize()
        t_fwd1 = ev[2].elapsed_time(ev[3])
        torch.cuda.synchronize()
        ev[4].record(st)
        adj.backward(dn_d, dJ_d, None, out=out)
        ev[5].record(st)
        ev[5].synchronize()
        t_bwd1 = ev[4].elapsed_time(ev[5])
        adj.close()
        one = {"forward_taped_ms": round(t_fwd1, 3), "backward_ms": round(t_bwd1, 3),
               "adjoint_vs_forward": round(t_bwd1 / t_plain, 3)}
        log(f"adjoint, one segment: taped forward {t_fwd1:.1f} ms, backward {t_bwd1:.1f} ms")
    box.close()
    log(f"adjoint{' with attraction' if att else ''}: plain forward {t_plain:.1f} ms, "
        f"checkpointed forward {t_fwd:.1f} ms, backward {t_bwd:.1f} ms ({T} steps)")
    return {
        "workload": w.name, "steps": T, "segment": segment, "species": M, "sigma": w.sigma,
        "scheme": "C^mf, derived inversion, per-step quasi-pressure" + (", attraction eps = kT/4, rc = 8" if att else ""),
        "forward_ms": round(t_plain, 3), "forward_checkpointed_ms": round(t_fwd, 3),
        "backward_ms": round(t_bwd, 3),
        "adjoint_vs_forward": round(t_bwd / t_plain, 3),
        "max_abs_dL_dV": gnorm,
        "one_segment": one,
    }


def adjoint_box_leg(lbe, torch, W, flags, T=40, segment=40):
    """dL/dV on the 128^3 benchmark box with its own scheme (C^visc on, the
    default per-step quasi-pressure), T steps in one segment (the forward records the
    tape, 41 slots of about 0.27 GB, and the backward recomputes nothing):
    forward, taped forward and backward times, L = sum of n^2 at the end."""
    from paper_1202_3842_amd import autotune
    w = W.c2_large_well()
    box = lbe.box_from_workload(w, flags=flags)
    autotune.tune_zchunk(box)
    st = box.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    box.step(5)
    lbe.load_workload(box, w)
    torch.cuda.synchronize()
    ev[0].record(st)
    box.step(T)
    ev[1].record(st)
    ev[1].synchronize()
    t_plain = ev[0].elapsed_time(ev[1])
    adj = lbe.Adjoint(box, T, segment)
    lbe.load_workload(box, w)
    torch.cuda.synchronize()
    ev[2].record(st)
    adj.forward()
    ev[3].record(st)
    ev[3].synchronize()
    t_fwd = ev[2].elapsed_time(ev[3])
    dn = torch.tensor(2.0 * box.density(0)[None], device="cuda")
    out = torch.empty(w.nodes, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ev[4].record(st)
    adj.backward(dn, None, None, out=out)
    ev[5].record(st)
    ev[5].synchronize()
    t_bwd = ev[4].elapsed_time(ev[5])
    adj.close()
    box.close()
    log(f"adjoint on {w.name}: plain forward {t_plain:.1f} ms, checkpointed forward {t_fwd:.1f} ms, "
        f"backward {t_bwd:.1f} ms ({T} steps)")
    return {"workload": w.name, "steps": T, "segment": segment,
            "scheme": "C^mf + C^visc, derived inversion, per-step quasi-pressure",
            "forward_ms": round(t_plain, 3), "forward_checkpointed_ms": round(t_fwd, 3),
            "backward_ms": round(t_bwd, 3), "adjoint_vs_forward": round(t_bwd / t_plain, 3),
            "max_abs_dL_dV": float(out.abs().max())}


def quasipressure_leg(lbe, torch, w, flags, reps=20):
    """The quasi-pressure initialiser of Sec. 2 (eq. quasipressure) and the
    divergence diagnostic of Sec. 4.3 on the benchmark box after 10 steps:
    wall time per call of a plain read-out (moments, contact values, forces,
    read-out pass), of Pi into device memory, of the g~ initialiser and of D;
    each call synchronises.  The path integral
    itself adds three line-scan launches to the read-out, the initialiser a
    pull, a zeroth-moment shift and an unstream per species."""
    box = lbe.box_from_workload(w, flags=flags)
    box.step(10)
    origin = (w.nx // 2, w.ny // 2, w.nz // 2)
    out = torch.empty(w.nodes, dtype=torch.float64, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    t_read = timed(lambda: box.density(0, out=out))
    t_pi = timed(lambda: box.quasipressure(0, origin, 0, out=out))
    t_init = timed(lambda: box.init_quasipressure(origin, 0))
    t_div = timed(lambda: box.divergence(out=out))
    box.close()
    log(f"quasipressure: read-out {t_read:.3f} ms, Pi {t_pi:.3f} ms, initialiser {t_init:.3f} ms, "
        f"divergence {t_div:.3f} ms")
    return {
        "workload": w.name, "origin": list(origin), "calls": reps,
        "readout_ms": round(t_read, 4), "quasipressure_ms": round(t_pi, 4),
        "init_ms": round(t_init, 4),
        "path_integral_extra_ms": round(t_pi - t_read, 4),
        "divergence_ms": round(t_div, 4),
    }


def attraction_leg(lbe, torch, w, flags, steps, warmup, base_force_ms):
    """The benchmark box with the attractive molecular field of the Appendix
    switched on (the r^-6 tail, eps = kT/4, rc = 8: the thick shell
    6 <= |e| < 8): step time, and the cost of the extra gather against its
    LDS and FP64 work (two 8-byte LDS reads and 7 flops per +-e pair and node)."""
    import copy
    import numpy as np
    wa = copy.copy(w)
    wa.att_eps, wa.att_rc = [[0.25 * w.kT]], 8.0
    r = run_gpu(wa, lbe.LBE_FP64, flags, steps, warmup, lbe, torch)
    K = 8
    g = np.arange(-K, K + 1)
    d = np.sqrt(g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2)
    pairs = int(((d >= w.sigma[0]) & (d < wa.att_rc)).sum()) // 2
    extra = r["force_ms"] - base_force_ms
    N = w.nodes
    out = {"eps_kT": 0.25, "rc": wa.att_rc, "pairs_per_node": pairs, "steps": steps,
           "ms_per_step": round(r["ms_per_step"], 4),
           "value": round(N * w.nspecies / (r["ms_per_step"] / 1e3) / 1e6, 2), "unit": "MLUPS",
           "force_phase_ms": round(r["force_ms"], 4), "attraction_ms": round(extra, 4),
           "umax": r["diag"]["umax"], "unstable": r["diag"]["unstable"]}
    if extra > 0:
        out["attraction_lds_TBps"] = round(N * pairs * 16 / (extra * 1e-3) / 1e12, 2)
        out["attraction_TFLOPs"] = round(N * pairs * 7 / (extra * 1e-3) / 1e12, 2)
    log(f"attraction: {out['ms_per_step']:.3f} ms/step, gather {extra:.3f} ms ({pairs} pairs/node)")
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_for(oracle, w, flags):
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.sigma, periodic=w.periodic, tau=w.tau, kT=w.kT, flags=flags)
    if w.solid is not None:
        o.set_solid(w.solid)
    if w.V is not None:
        o.set_potential(w.V)
    for a, g in enumerate(w.body):
        o.set_body_force(a, g)
    for a, n in enumerate(w.density):
        o.init_density(a, n)
    if w.qp_route is not None:
        o.set_quasipressure_route(*w.qp_route)
    return o


def cpu_baseline(w, flags, budget_s, compare=None, budget_1t=12.0):
    """The oracle as it stands, on the host cores, over a bounded number of
    steps of the same workload from its initial state, with all the cores
    the box grants (at most 16) and then with one thread.  After the
    timing, compare(oracle, steps) may check GPU runs of the same steps
    against the oracle's state; its result is returned alongside."""
    import oracle
    if not oracle.LIB.exists():
        oracle.build()
    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16")), 16)

    def timed(nthreads, budget, max_steps):
        oracle.set_threads(nthreads)
        o = _oracle_for(oracle, w, flags)
        steps = 0
        t = time.perf_counter()
        while True:
            try:
                o.step(1)
            except oracle.OracleError as e:
                log(f"cpu oracle stopped: {e}")
                break
            steps += 1
            el = time.perf_counter() - t
            log(f"cpu oracle ({nthreads} threads) step {steps}: {el:.1f} s")
            if el > budget or steps >= max_steps:
                break
        el = time.perf_counter() - t
        return o, steps, el

    o, steps, el = timed(threads, budget_s, 50)
    mlups = w.nodes * w.nspecies * steps / el / 1e6
    checked = compare(o, steps) if compare is not None and steps > 0 else None
    o.close()
    o1, steps1, el1 = timed(1, budget_1t, 50)
    o1.close()
    oracle.set_threads(threads)
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the same {w.nx}x{w.ny}x{w.nz} workload from its initial "
                      f"state ({el:.1f} s wall)",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": {"value": round(w.nodes * w.nspecies * steps1 / el1 / 1e6, 4), "unit": "MLUPS",
                           "cores": 1, "sample": f"{steps1} steps ({el1:.1f} s wall)"}}, checked


def oracle_comparison(lbe, w, flags):
    """GPU runs in FP64 and with FP32 populations, from the same initial
    state and for as many steps as the oracle took, against the oracle:
    max-norm relative error of n and of the barycentric u, and max |u|."""
    import numpy as np
    from paper_1202_3842_amd import autotune

    def compare(o, steps):
        n_ref, u_ref = o.density(0), o.velocity(-1)
        out = {"steps": steps}
        for name, prec in (("fp64", lbe.LBE_FP64), ("fp32_pop", lbe.LBE_FP32_POP)):
            box = lbe.box_from_workload(w, prec=prec, flags=flags)
            autotune.tune_zchunk(box)
            box.step(steps)
            n, u = box.density(0), box.velocity(-1)
            box.close()
            out[name] = {"n_rel_err": float(np.abs(n - n_ref).max() / np.abs(n_ref).max()),
                         "u_rel_err": float(np.abs(u - u_ref).max() / np.abs(u_ref).max()),
                         "umax": float(np.sqrt((u ** 2).sum(axis=0)).max())}
        out["oracle_umax"] = float(np.sqrt((u_ref ** 2).sum(axis=0)).max())
        log(f"against the oracle after {steps} steps: fp64 n {out['fp64']['n_rel_err']:.2e} "
            f"u {out['fp64']['u_rel_err']:.2e}; fp32 n {out['fp32_pop']['n_rel_err']:.2e} "
            f"u {out['fp32_pop']['u_rel_err']:.2e}")
        return out
    return compare


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fp32-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-quasipressure", action="store_true")
    ap.add_argument("--no-attraction", action="store_true")
    ap.add_argument("--quasipressure-only", action="store_true",
                    help="run only the quasi-pressure leg and print its JSON (for profiling)")
    ap.add_argument("--variant-steps", type=int, default=300)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (a plain copy kernel of "
                         "known traffic, to scale HBM counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition of the lattice is designed but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1202_3842_amd import lbe
    from paper_1202_3842_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)
        return
    if args.adjoint_only:
        adj = adjoint_leg(lbe, torch, W)
        adj["with_attraction"] = adjoint_leg(lbe, torch, W, att=True)
        adj["benchmark_box"] = adjoint_box_leg(lbe, torch, W, lbe.LBE_VISC)
        print(json.dumps({"adjoint": adj}), flush=True)
        return
    w = W.c2_large_well()
    # the library's default scheme: derived inversions, the quasi-pressure
    # evaluated every step (six-order mean from the box centre), C^visc on
    flags = lbe.LBE_VISC
    if args.quasipressure_only:
        print(json.dumps({"quasipressure": quasipressure_leg(lbe, torch, w, flags)}), flush=True)
        return
    M = w.nspecies
    npairs = M * (M + 1) // 2

    r64 = run_gpu(w, lbe.LBE_FP64, flags, args.steps, args.warmup, lbe, torch)
    N = w.nodes
    ms_step = r64["ms_per_step"]
    mlups = N * M / (ms_step / 1e3) / 1e6
    balg = alg_bytes_step(M, npairs, 8, True)
    pairs = shell_pairs(w.sigma[0])
    kern64 = kernel_views(r64, N, M, 8, pairs, "double")
    falg = alg_flops_force(pairs, True) * M * M
    floor_ms = max(N * balg / (HBM_PEAK_GBS * 1e9), N * falg / (FP64_PEAK_TFLOPS * 1e12)) * 1e3

    fp32_steps = args.fp32_steps if args.fp32_steps is not None else max(args.steps // 4, 10)
    r32 = run_gpu(w, lbe.LBE_FP32_POP, flags, fp32_steps, args.warmup, lbe, torch)
    mlups32 = N * M / (r32["ms_per_step"] / 1e3) / 1e6
    kern32 = kernel_views(r32, N, M, 4, pairs, "float")

    batched = None
    if not args.no_batch:
        batched = {
            "fp64": batch_leg(lbe, torch, W, flags, lbe.LBE_FP64, args.batch_steps, args.batch_steps),
            "fp32_pop": batch_leg(lbe, torch, W, flags, lbe.LBE_FP32_POP, max(args.batch_steps // 5, 10),
                                  max(args.batch_steps // 5, 10)),
            "fp64_small_boxes": batch_leg(lbe, torch, W, flags, lbe.LBE_FP64, args.batch_steps,
                                          args.batch_steps, Lmin=8, Lmax=24),
        }

    variants = None if args.no_variants else variants_leg(lbe, torch, w, flags, args.variant_steps,
                                                             args.warmup)

    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_leg(lbe, torch, W)
        adjoint["with_attraction"] = adjoint_leg(lbe, torch, W, att=True)
        adjoint["benchmark_box"] = adjoint_box_leg(lbe, torch, W, flags)

    qp = None if args.no_quasipressure else quasipressure_leg(lbe, torch, w, flags)

    att = None if args.no_attraction else attraction_leg(lbe, torch, w, flags, args.variant_steps,
                                                          args.warmup, r64["force_ms"])

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        cpu, parity = cpu_baseline(w, flags, args.cpu_budget, oracle_comparison(lbe, w, flags))

    out = {
        "metric": "MLUPS per species + % HBM roofline (FP64 & FP32); batched vs serial; adjoint/fwd",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name, "lattice": "D3Q19", "box": [w.nx, w.ny, w.nz], "periodic": "xyz",
            "species": M, "sigma": w.sigma, "n_sigma3": 0.4, "well_radius": 24, "well_depth_kT": 2.0,
            "well_eps_kT": 2.0, "tau": w.tau, "kT": w.kT, "collisional_viscous_force": True,
            "inversion": "derived (eq. invertmoments)", "kappa": 2,
            "quasi_pressure": "evaluated every step, mean of the six axis-order paths from the centre",
        },
        "timing": {"runs": len(r64["run_ms_per_step"]), "statistic": "median",
                   "run_ms_per_step": [round(x, 4) for x in r64["run_ms_per_step"]],
                   "phase_ms": {"force": round(r64["force_ms"], 4), "quasi_pressure": round(r64["qp_ms"], 4),
                                "collide": round(r64["collide_ms"], 4)}},
        "roofline": dict(dominant(kern64), step={
            "alg_bytes_per_node": balg, "alg_flops_per_node": falg,
            "hbm_frac": round(mlups * 1e6 * balg / (HBM_PEAK_GBS * 1e9), 4),
            "floor_ms": round(floor_ms, 4),
            "floor": "max(B_alg / 8 TB/s, F_alg / 78.6 TFLOP/s)",
            "frac": round(floor_ms / ms_step, 4)}),
        "kernels": kern64,
        "step_alg_frac": round(mlups * 1e6 * balg / (HBM_PEAK_GBS * 1e9), 4),
        "step_alg_bytes_per_node": balg,
        "fp32_pop": {
            "value": round(mlups32, 2), "unit": "MLUPS", "steps": fp32_steps,
            "ms_per_step": round(r32["ms_per_step"], 4),
            "roofline": dominant(kern32), "kernels": kern32,
            "umax": r32["diag"]["umax"], "unstable": r32["diag"]["unstable"],
            "vs_oracle": parity and {"steps": parity["steps"], **parity["fp32_pop"]},
        },
        "vs_oracle": parity and {"steps": parity["steps"], "oracle_umax": parity["oracle_umax"],
                                 **parity["fp64"]},
        "state_after": {"umax": r64["diag"]["umax"], "unstable": r64["diag"]["unstable"]},
        "batched": batched,
        "variants": variants,
        "adjoint": adjoint,
        "quasipressure": qp,
        "attraction": att,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
