"""Shared set-up of the adjoint tests: a small two-species channel and the
objective L = sum_fluid (n_A - n_t)^2 + sum_plane sum_a J_x^a (+ an optional
linear functional of the final populations)."""
from __future__ import annotations

import numpy as np

from paper_1202_3842_amd import workloads as W


def small_channel(nx=12, ny=10, nz=8, sigma=(2.0, 3.0), seed=77):
    """Periodic x, z; walls beyond y in [0, ny-1]; an obstacle over x in
    [5, 7) leaving a 4-site gap; smooth V of 0.1 kT; body force along x;
    densities at packing 0.25 with 1e-2 noise."""
    w = W.channel(nx=nx, ny=ny, nz=nz, x0=5, x1=7, gap=4, sigma=sigma, steps=6,
                  name=f"channel{nx}x{ny}x{nz}")
    w.V = W.smooth_field(w.shape, 0.1 * W.KT, 4, seed)
    w.density = [W.noisy_uniform(w.shape, float(d.mean()), 1e-2, seed + 1 + a)
                 for a, d in enumerate(w.density)]
    w.body = [[1e-4, 0.0, 0.0], [1e-4, 2e-5, 0.0]]
    return w


def objective_terms(w, plane_x=None):
    """(n_t, fluid mask, plane mask) of the objective on workload w."""
    s = W.smooth_field(w.shape, 1.0, 4, 1204)
    n_t = w.density[0] * (1.0 + 0.05 * s)
    fluid = w.solid == 0
    plane = np.zeros(w.shape, dtype=bool)
    plane[:, :, w.nx // 2 if plane_x is None else plane_x] = True
    return n_t, fluid, plane & fluid


def pop_weights(w, seed=5):
    """A fixed random linear functional of the final post-streaming
    populations, shaped (2, M, 19, nz, ny, nx), zero on solid nodes."""
    r = W.rng(seed).uniform(-1.0, 1.0, size=(2, w.nspecies, 19) + w.shape)
    return r * (w.solid == 0)[None, None, None]


def loss_numpy(nA, J_list, n_t, fluid, plane, pops=None, pw=None):
    L = float(np.sum(((nA - n_t) ** 2)[fluid]))
    for J in J_list:
        L += float(np.sum(J[0][plane]))
    if pops is not None:
        L += float(np.sum(pw * pops))
    return L
