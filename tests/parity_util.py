"""Helpers shared by the GPU parity tests: run the same seeded workload through
the oracle and through the HIP library and compare fields."""
from __future__ import annotations

import sys

import numpy as np

from paper_1202_3842_amd import workloads as W


def banner(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_from_workload(w: W.Workload, flags: int):
    import oracle
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.sigma, periodic=w.periodic, tau=w.tau, kT=w.kT, flags=flags,
                      att_eps=w.att_eps, att_rc=w.att_rc)
    if w.solid is not None:
        o.set_solid(w.solid)
    if w.V is not None:
        o.set_potential(w.V)
    for a, g in enumerate(w.body):
        o.set_body_force(a, g)
    for a, n in enumerate(w.density):
        o.init_density(a, n)
    if getattr(w, "qp_route", None) is not None:
        o.set_quasipressure_route(*w.qp_route)
    return o


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (max-norm relative error)."""
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    if den == 0.0:
        return float(num)
    return float(num / den)


def compare_state(o, box, M: int, tol: float, label: str = "") -> dict:
    errs = {}
    for a in range(M):
        errs[f"n{a}"] = rel_err(box.density(a), o.density(a))
        errs[f"u{a}"] = rel_err(box.velocity(a), o.velocity(a))
    errs["u"] = rel_err(box.velocity(-1), o.velocity(-1))
    print(f"[parity] {label} {errs}", flush=True)
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    return errs
