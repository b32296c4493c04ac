"""Oracle states of the configured workloads after their stated step counts.

Writes, for each case, an ``.npz`` file (numpy, no pickled objects) with the
oracle's n and u on one full z plane and at a seeded sample of nodes:

* ``well128_2000.npz``: the 128^3 well (sigma = 6, n sigma^3 = 0.4, radius 24,
  depth 2 kT), C^visc on, the default scheme, 2000 steps; the plane z = 64
  and 32768 seeded nodes (seed 4001).
* ``channel256_5000.npz``: the 256x64x32 two-species channel with the
  bottleneck, 5000 steps, C^visc off (with C^visc on the channel collapses
  within a few hundred steps under every reading tried); the plane z = 16
  and 32768 seeded nodes (seed 4002); both species.
* ``boxes_500.npz``: boxes of the 96-box batched set, 500 steps each, C^visc
  on: boxes are drawn in a seeded order (seed 4003) among those with an edge
  of at most 64 nodes (oracle time), and the first four that stay stable
  are kept; for each, the plane z = L/2 and 4096 seeded nodes.

Only the oracle computes anything here (``oracle/`` and the set-up
generators of ``paper_1202_3842_amd.workloads``, which hold none of the
method's arithmetic).  tests/test_gpu_fullsize.py compares the GPU library
with these values.

    python tests/golden/make_fullsize_goldens.py --case c2 [--threads 8]   (about 70 min on 8 cores)
    python tests/golden/make_fullsize_goldens.py --case c3                 (about 45 min)
    python tests/golden/make_fullsize_goldens.py --case c4                 (about 15 min)
"""
from __future__ import annotations

import argparse
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_1202_3842_amd import workloads as W  # noqa: E402

HERE = Path(__file__).resolve().parent
VISC = oracle.LBEO_VISC


def build(w, flags):
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.sigma, w.periodic, w.tau, w.kT, flags=flags,
                      att_eps=w.att_eps, att_rc=w.att_rc)
    if w.solid is not None:
        o.set_solid(w.solid)
    if w.V is not None:
        o.set_potential(w.V)
    for a in range(w.nspecies):
        o.set_body_force(a, np.asarray(w.body[a], dtype=float))
        o.init_density(a, w.density[a])
    if w.qp_route is not None:
        o.set_quasipressure_route(*w.qp_route)
    return o


def sample(w, count, seed):
    return np.sort(W.rng(seed).choice(w.nodes, size=min(count, w.nodes), replace=False))


def state(o, w, zplane, nodes, prefix, out):
    """n^a and u^a of every species, and the barycentric u, on the plane and
    at the sampled nodes."""
    for a in range(w.nspecies):
        n = o.density(a)
        u = o.velocity(a)
        out[f"{prefix}n{a}_plane"] = n[zplane]
        out[f"{prefix}u{a}_plane"] = u[:, zplane]
        out[f"{prefix}n{a}_nodes"] = n.reshape(-1)[nodes]
        out[f"{prefix}u{a}_nodes"] = u.reshape(3, -1)[:, nodes]
    ub = o.velocity(-1)
    out[f"{prefix}u_plane"] = ub[:, zplane]
    out[f"{prefix}u_nodes"] = ub.reshape(3, -1)[:, nodes]


def run(w, flags, steps, label, every=100):
    o = build(w, flags)
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        try:
            o.step(k)
        except oracle.OracleError as e:  # the oracle refuses to step a collapsed state
            print(f"{label}: {e} within steps {done + 1}..{done + k}", flush=True)
            return o, done + k, True
        done += k
        d = o.diagnostics()
        print(f"{label}: step {done}/{steps} umax {d['umax']:.4e} unstable {d['unstable']} "
              f"{time.time() - t0:.0f}s", flush=True)
        if d["unstable"]:
            return o, done, True
    return o, done, False


def case_c2():
    w = W.c2_large_well()
    o, done, bad = run(w, VISC, w.steps, "well128")
    assert not bad, "the 128^3 well went unstable"
    out = {"steps": np.array(w.steps), "flags": np.array(VISC), "zplane": np.array(w.nz // 2)}
    nodes = sample(w, 32768, 4001)
    out["nodes"] = nodes
    state(o, w, w.nz // 2, nodes, "", out)
    out["mass"] = np.array(o.diagnostics()["mass"])
    np.savez(HERE / "well128_2000.npz", **out)


def case_c3():
    w = W.c3_channel()
    o, done, bad = run(w, 0, w.steps, "channel256", every=250)
    assert not bad, "the channel went unstable"
    out = {"steps": np.array(w.steps), "flags": np.array(0), "zplane": np.array(w.nz // 2)}
    nodes = sample(w, 32768, 4002)
    out["nodes"] = nodes
    state(o, w, w.nz // 2, nodes, "", out)
    out["mass"] = np.array(o.diagnostics()["mass"])
    np.savez(HERE / "channel256_5000.npz", **out)


def case_c4():
    boxes = W.c4_boxes()
    order = W.rng(4003).permutation(len(boxes))
    out = {"flags": np.array(VISC)}
    kept = []
    for b in order:
        w = boxes[b]
        if w.nx > 64:
            continue
        o, done, bad = run(w, VISC, w.steps, f"box{b} L={w.nx} sigma={w.sigma[0]}", every=100)
        if bad:
            print(f"box{b}: unstable at step {done}; next", flush=True)
            continue
        nodes = sample(w, 4096, 4004 + int(b))
        out[f"box{b}_nodes"] = nodes
        state(o, w, w.nz // 2, nodes, f"box{b}_", out)
        kept.append(int(b))
        if len(kept) == 4:
            break
    out["boxes"] = np.array(kept)
    out["steps"] = np.array(boxes[0].steps)
    np.savez(HERE / "boxes_500.npz", **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=["c2", "c3", "c4"], required=True)
    ap.add_argument("--threads", type=int, default=8)
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    {"c2": case_c2, "c3": case_c3, "c4": case_c4}[args.case]()
    print("done", flush=True)


if __name__ == "__main__":
    main()
