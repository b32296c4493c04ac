"""Pins of the reference gradient (oracle/autograd_ref.py): its forward
equals the C oracle's step, and its autograd gradients equal central finite
differences of the C oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import autograd_ref as AR
from adjoint_util import small_channel, objective_terms, loss_numpy, pop_weights
from paper_1202_3842_amd import workloads as W

T = 4


# attractive tails for the two-species channel (sigma 2 and 3)
ATT_EPS = [[0.3 * W.KT, 0.2 * W.KT], [0.2 * W.KT, 0.25 * W.KT]]
ATT_RC = 5.0


def c_oracle(w, flags, V=None, att=False):
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.sigma, w.periodic, w.tau, w.kT, flags=flags,
                      att_eps=ATT_EPS if att else None, att_rc=ATT_RC if att else 0.0)
    o.set_solid(w.solid)
    o.set_potential(w.V if V is None else V)
    for a in range(w.nspecies):
        o.init_density(a, w.density[a])
        o.set_body_force(a, w.body[a])
    return o


def stepper(w, flags, att=False):
    geo = AR.Geometry(w.nx, w.ny, w.nz, w.periodic, w.solid.astype(bool))
    return AR.Stepper(geo, w.sigma, w.tau, w.kT, flags, w.body,
                      att_eps=ATT_EPS if att else None, att_rc=ATT_RC if att else 0.0)


def torch_loss(st, w, f, g, V, n_t, fluid, plane, pw=None):
    n, J = st.readout(f, g, V)
    L = ((n[0] - torch.tensor(n_t.reshape(-1))) ** 2 * torch.tensor(fluid.reshape(-1), dtype=torch.float64)).sum()
    L = L + (J[:, 0, :] * torch.tensor(plane.reshape(-1), dtype=torch.float64)).sum()
    if pw is not None:
        pwt = torch.tensor(pw.reshape(2, w.nspecies, 19, -1))
        L = L + (pwt[0] * f).sum() + (pwt[1] * g).sum()
    return L


@pytest.mark.parametrize("flags,att", [(0, False), (AR.PRINTED_INV, False), (AR.KAPPA4, False),
                                       (0, True), (AR.PRINTED_INV | AR.KAPPA4, True),
                                       (AR.DRAG, False), (AR.DRAG | AR.PRINTED_INV, True),
                                       (AR.EULER, False), (AR.SINGLE, True),
                                       (AR.SINGLE | AR.EULER | AR.DRAG, False),
                                       (AR.VISC, False), (AR.VISC | AR.PRINTED_INV | AR.DRAG, True),
                                       (AR.VISC | AR.SINGLE, False)])
def test_forward_equals_c_oracle(flags, att):
    w = small_channel()
    o = c_oracle(w, flags, att=att)
    o.step(5)
    st = stepper(w, flags, att)
    f, g = st.rest_state(np.stack(w.density))
    f, g = st.run(f, g, torch.tensor(w.V), 5)
    for a in range(w.nspecies):
        for dist, t in ((0, f), (1, g)):
            ref = o.populations(a, dist).reshape(19, -1)
            assert np.abs(t[a].numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    n, J = st.readout(f, g, torch.tensor(w.V))
    for a in range(w.nspecies):
        assert np.abs(n[a].numpy() - o.density(a).reshape(-1)).max() <= 1e-15
        Jo = (o.density(a) * o.velocity(a)).reshape(3, -1)
        assert np.abs(J[a].numpy() - Jo).max() <= 1e-13 * np.abs(Jo).max()


@pytest.mark.parametrize("flags,att", [(0, False), (AR.PRINTED_INV, False), (0, True),
                                       (AR.DRAG, False), (AR.DRAG | AR.PRINTED_INV, False),
                                       (AR.EULER, False), (AR.SINGLE, False),
                                       (AR.SINGLE | AR.EULER, False),
                                       (AR.VISC, False), (AR.VISC | AR.PRINTED_INV | AR.DRAG, False)])
def test_gradient_equals_oracle_fd(flags, att):
    w = small_channel()
    n_t, fluid, plane = objective_terms(w)
    pw = pop_weights(w) * 1e-3
    st = stepper(w, flags, att)
    V = torch.tensor(w.V.reshape(-1), requires_grad=True)
    f0, g0 = st.rest_state(np.stack(w.density))
    f0.requires_grad_(True)
    g0.requires_grad_(True)
    f, g = st.run(f0, g0, V, T)
    L = torch_loss(st, w, f, g, V, n_t, fluid, plane, pw)
    L.backward()
    gV = V.grad.numpy()
    gf = f0.grad.numpy()

    def oracle_loss(Vx=None, pop=None):
        o = c_oracle(w, flags, Vx, att)
        if pop is not None:
            a, p, i, h = pop
            f_in = o.populations(a, 0).reshape(19, -1).copy()
            f_in[p, i] += h
            o.set_populations(a, 0, f_in)
        o.step(T)
        J = [o.density(a) * o.velocity(a) for a in range(w.nspecies)]
        pops = np.stack([np.stack([o.populations(a, d) for a in range(w.nspecies)]) for d in range(2)])
        return loss_numpy(o.density(0), J, n_t, fluid, plane, pops, pw)

    oracle.set_threads(2)
    assert abs(L.item() - oracle_loss()) <= 1e-13 * abs(L.item())
    h = 1e-6
    scale = np.abs(gV).max()
    for i in W.sample_fluid_nodes(w, 4, 9):
        Vp = w.V.copy().reshape(-1)
        Vm = Vp.copy()
        Vp[i] += h
        Vm[i] -= h
        fd = (oracle_loss(Vp.reshape(w.shape)) - oracle_loss(Vm.reshape(w.shape))) / (2 * h)
        assert abs(gV[i] - fd) <= 1e-7 * scale, (i, gV[i], fd)
    # gradient with respect to an initial population
    scale = np.abs(gf).max()
    for (a, p, i) in ((0, 3, 140), (1, 11, 611)):
        fd = (oracle_loss(pop=(a, p, i, h)) - oracle_loss(pop=(a, p, i, -h))) / (2 * h)
        assert abs(gf[a, p, i] - fd) <= 1e-6 * scale, (a, p, i, gf[a, p, i], fd)
