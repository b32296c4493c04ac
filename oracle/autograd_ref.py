"""Reference gradient: the DD-TR step re-expressed in PyTorch (CPU, FP64),
differentiated by autograd.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the GPU adjoint is
checked against the gradients computed here.  This is a second, vectorised
expression of the same step as ``lbe_oracle.c`` -- written again from the
paper, not translated from the C code -- whose forward is pinned to the C
oracle and whose gradient is pinned to central finite differences of the C
oracle (tests/test_oracle_adjoint_ref.py).

The step (arXiv:1202.3842, Secs. 2-4 and the Appendix), per species a, on
post-streaming populations f~, g~:
  * moments n = sum f~, Pi~ = sum g~, J~ = sum c g~ (Sec. 4.2);
  * ball averages of n of radius sigma_b/2 -> xi_2, xi_3 -> BMCSL contact
    values G_ab (zero on solid nodes);
  * C^mf_a = -kT n_a sum_b sigma_ab^2 w_ab sum_{e in shell}
    e^ (G_ab(r) + G_ab(r+e))/2 n_b(r+e)  (Appendix, lattice shell);
  * F = -grad_h V + body force, grad_h V = (1/v_T^2) sum_p w_p c_p V(r+c_p)
    with wrapped or clamped neighbours;
  * inversion J = J~ + Y/2 (or X/2 printed), u^a = J/n, u = sum J / sum n;
  * Pi, by default the quasi-pressure of eq. quasipressure, n - beta times
    the trapezoidal path integral of C^mf from the origin, the mean over the
    six axis orders of the paths that run along x, y and z in turn (or the
    order x, y, z alone); the zeroth moment of g~ is
    set to Pi - (beta/2) C.u^a (plus, printed; Pi itself, Euler) before the
    update.  With PI_CARRIED, Pi = Pi~ + (beta/2) C.u^a (minus, printed)
    from the carried g~;
  * Hermite equilibria and sources of eqs. kernel-f-1 .. kernel-g-1 with
    the kappa of the C^mf part of S_g;
  * trapezoidal update f~* = f~ + a (f_eq - f~) + b S_f (Sec. 4.1) and the
    pull streaming with mid-point bounce-back (Sec. 4.3).
The C^mf scheme is expressed, optionally with the collisional viscous
force of the Appendix (C^visc_a = n_a sum_b 2 sigma_ab^2 sqrt(kT/pi) w_ab
sum_{e in shell} e^ [e^.(u~_b(r+e) - u~_b(r))] g(r, r+e) n_b(r+e), u~ =
J~/n), the interspecies drag of the Appendix (eq. dragforce2: the local force
-n_a sum_b gamma_ab G_ab n_b (u~_a - u~_b), u~ = J~/n, gamma_ab =
sigma_ab^2 2 sqrt(kT/pi) 4 pi/3, which joins C^visc in the sources) and the
attractive molecular field of the Appendix (the r^-6 tail U = -eps (sigma/r)^6
for sigma_ab <= r < rc, g = 1 there), which adds
n_a sum_b sum_e U'(|e|) e^ n_b(r+e) to C^mf_a.  Neighbour access uses index
tables built once per geometry; an index of N points at a zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

Q = 19
# D3Q19: rest, 6 axis neighbours, 12 face diagonals (the population order
# of the library's ABI)
C_VEL = np.array([
    [0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
    [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W_VEL = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = np.array([int(np.flatnonzero((C_VEL == -c).all(1))[0]) for c in C_VEL])

VISC = 1 << 0
PRINTED_INV = 1 << 1
KAPPA4 = 1 << 2
EULER = 1 << 4
SINGLE = 1 << 5
DRAG = 1 << 6
PI_CARRIED = 1 << 7


def lattice_shell(s: float):
    """Offsets e with s - 1/2 <= |e| < s + 1/2 and the weight 4 pi s / sum |e|."""
    K = int(math.ceil(s + 0.5))
    pts = []
    for z in range(-K, K + 1):
        for y in range(-K, K + 1):
            for x in range(-K, K + 1):
                r = math.sqrt(x * x + y * y + z * z)
                if r > 0 and (s - 0.5) ** 2 <= x * x + y * y + z * z < (s + 0.5) ** 2:
                    pts.append((x, y, z, r))
    if not pts:
        return np.zeros((0, 3), dtype=np.int64), np.zeros((0, 3)), 0.0
    e = np.array([p[:3] for p in pts], dtype=np.int64)
    r = np.array([p[3] for p in pts])
    return e, e / r[:, None], 4 * math.pi * s / r.sum()


def attraction_offsets(sab: float, eps: float, rc: float):
    """Offsets e with sigma_ab <= |e| < rc and U'(|e|) e^ for
    U = -eps (sigma_ab/r)^6, so U' = 6 eps sigma_ab^6 / r^7."""
    K = int(math.ceil(rc))
    e = np.array([(x, y, z) for z in range(-K, K + 1) for y in range(-K, K + 1) for x in range(-K, K + 1)],
                 dtype=np.int64)
    r = np.sqrt((e ** 2).sum(1).astype(float))
    keep = (r >= sab) & (r < rc)
    e, r = e[keep], r[keep]
    return e, (6.0 * eps * sab ** 6 / r ** 7 / r)[:, None] * e


def lattice_ball(sigma: float):
    R = 0.5 * sigma
    K = int(math.floor(R))
    return np.array([(x, y, z) for z in range(-K, K + 1) for y in range(-K, K + 1)
                     for x in range(-K, K + 1) if x * x + y * y + z * z <= R * R],
                    dtype=np.int64).reshape(-1, 3)


@dataclass
class Geometry:
    nx: int
    ny: int
    nz: int
    periodic: int
    solid: np.ndarray  # (nz, ny, nx) bool

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def coords(self):
        z, y, x = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        return x.reshape(-1), y.reshape(-1), z.reshape(-1)

    def shifted(self, d, clamp=False):
        """Flat index of r + d for every node r; N where r + d leaves the box
        through a wall (or the clamped index if clamp)."""
        x, y, z = self.coords()
        out_ok = np.ones(self.N, dtype=bool)
        res = []
        for k, (v, n) in enumerate(((x, self.nx), (y, self.ny), (z, self.nz))):
            w = v + int(d[k])
            if self.periodic >> k & 1:
                w = np.mod(w, n)
            elif clamp:
                w = np.clip(w, 0, n - 1)
            else:
                out_ok &= (w >= 0) & (w < n)
                w = np.clip(w, 0, n - 1)
            res.append(w)
        idx = res[0] + self.nx * (res[1] + self.ny * res[2])
        return np.where(out_ok, idx, self.N)


class Stepper:
    """One configuration: geometry, species diameters, tau, flags, body forces."""

    def __init__(self, geom: Geometry, sigma, tau=1.0, kT=1.0 / 3.0, flags=0, body=None,
                 att_eps=None, att_rc=0.0, qp_origin=None, qp_symmetric=True):
        self.g = geom
        self.M = len(sigma)
        self.sigma = [float(s) for s in sigma]
        self.kT = kT
        self.vT2 = kT
        self.beta = 1.0 / kT
        omega = 1.0 / tau
        # the scheme variants of Sec. 4: Euler (f* = f + omega (f_eq - f) + S)
        # or the trapezoidal rule; one distribution (f carries the current,
        # no g) or two
        self.euler = bool(flags & EULER)
        self.single = bool(flags & SINGLE)
        self.a = omega if self.euler else omega / (1 + 0.5 * omega)
        self.b = 1.0 if self.euler else 1.0 / (1 + 0.5 * omega)
        self.printed = bool(flags & PRINTED_INV)
        self.kappa = 4.0 if flags & KAPPA4 else 2.0
        self.drag = bool(flags & DRAG) and self.M > 1
        self.visc = bool(flags & VISC)
        # Pi from the path integral every step (default) or carried by g
        self.qp = not (flags & PI_CARRIED) and not self.single
        self.qp_origin = tuple(qp_origin) if qp_origin is not None else (
            geom.nx // 2, geom.ny // 2, geom.nz // 2)
        self.qp_symmetric = qp_symmetric
        # drag coefficients: the collision integral of C^visc over the unit
        # sphere, 2 sigma_ab^2 sqrt(kT/pi) (4 pi/3)
        self.gamma = [[(0.5 * (sa + sb)) ** 2 * 2.0 * math.sqrt(kT / math.pi) * (4.0 * math.pi / 3.0)
                       for sb in self.sigma] for sa in self.sigma]
        self.body = torch.tensor(np.zeros((self.M, 3)) if body is None else np.asarray(body, float),
                                 dtype=torch.float64)
        N = geom.N
        solid = geom.solid.reshape(-1).astype(bool)
        self.fluid = torch.tensor(~solid, dtype=torch.float64)
        fluid_ext = np.concatenate([~solid, [False]])
        # streaming: population p at r comes from r - c_p, or bounces back
        src = np.zeros((Q, N), dtype=np.int64)
        blocked = np.zeros((Q, N), dtype=bool)
        for p in range(Q):
            j = geom.shifted(-C_VEL[p])
            blocked[p] = ~fluid_ext[j]
            src[p] = np.where(blocked[p], np.arange(N), j)
        self.src = torch.tensor(src)
        self.blocked = torch.tensor(blocked)
        # external-force neighbours (wrapped or clamped)
        self.vnb = torch.tensor(np.stack([geom.shifted(C_VEL[p], clamp=True) for p in range(Q)]))
        # shells of every ordered pair and balls of every species
        self.shell = {}
        for a in range(self.M):
            for b in range(self.M):
                s = 0.5 * (self.sigma[a] + self.sigma[b])
                e, eh, w = lattice_shell(s) if s >= 0.5 else (np.zeros((0, 3), np.int64), np.zeros((0, 3)), 0.0)
                idx = np.stack([geom.shifted(v) for v in e]) if len(e) else np.zeros((0, N), np.int64)
                self.shell[a, b] = (torch.tensor(idx), torch.tensor(eh), s, w)
        # attractive tails of every ordered pair with a positive depth
        self.att = {}
        for a in range(self.M):
            for b in range(self.M):
                eps = 0.0 if att_eps is None else float(att_eps[a][b])
                if eps > 0.0:
                    s = 0.5 * (self.sigma[a] + self.sigma[b])
                    e, K = attraction_offsets(s, eps, att_rc)
                    self.att[a, b] = (torch.tensor(np.stack([geom.shifted(v) for v in e])), torch.tensor(K))
        self.ball = []
        for b in range(self.M):
            d = lattice_ball(self.sigma[b])
            self.ball.append((torch.tensor(np.stack([geom.shifted(v) for v in d])), len(d)))
        c = torch.tensor(C_VEL, dtype=torch.float64)
        self.c = c
        self.w = torch.tensor(W_VEL)
        self.H1 = c / self.vT2
        eye = torch.eye(3, dtype=torch.float64)
        self.H2 = (c[:, :, None] * c[:, None, :] - self.vT2 * eye) / (2 * self.vT2 ** 2)

    # -- pieces ---------------------------------------------------------------
    @staticmethod
    def _ext(v):
        return torch.cat([v, v.new_zeros(1)])

    def external_force(self, V):
        Vn = V.reshape(-1)[self.vnb]                      # (Q, N)
        grad = (self.w[:, None, None] * self.c[:, :, None] * Vn[:, None, :]).sum(0) / self.vT2
        return -grad                                       # (3, N)

    def contact(self, n):
        xi2 = 0.0
        xi3 = 0.0
        for b in range(self.M):
            idx, cnt = self.ball[b]
            nbar = self._ext(n[b])[idx].sum(0) / cnt
            xi2 = xi2 + self.sigma[b] ** 2 * nbar
            xi3 = xi3 + self.sigma[b] ** 3 * nbar
        xi2 = xi2 * math.pi / 6
        xi3 = xi3 * math.pi / 6
        G = {}
        for a in range(self.M):
            for b in range(self.M):
                sa, sb = self.sigma[a], self.sigma[b]
                d = sa * sb / (sa + sb) if sa + sb > 0 else 0.0
                one = 1.0 - xi3
                G[a, b] = (1 / one + 3 * d * xi2 / one ** 2 + 2 * d * d * xi2 ** 2 / one ** 3) * self.fluid
        return G

    def mean_field(self, n, G):
        """C^mf of every species, (M, 3, N)."""
        out = []
        for a in range(self.M):
            acc = n.new_zeros(3, n.shape[1])
            for b in range(self.M):
                idx, eh, s, w = self.shell[a, b]
                if idx.shape[0] == 0:
                    continue
                Gab = G[a, b]
                pair = 0.5 * (Gab[None, :] + self._ext(Gab)[idx]) * self._ext(n[b])[idx]   # (E, N)
                acc = acc + s * s * w * (eh.T @ pair)
            Ca = -self.kT * n[a][None, :] * acc
            for b in range(self.M):
                if (a, b) in self.att:
                    idx, K = self.att[a, b]
                    Ca = Ca + n[a][None, :] * (K.T @ self._ext(n[b])[idx])
            out.append(Ca)
        return torch.stack(out)

    def visc_force(self, n, G, Jt):
        """C^visc of every species, (M, 3, N), over the same shells as C^mf."""
        pos = n > 0
        ut = Jt / torch.where(pos, n, torch.ones_like(n))[:, None, :] * pos[:, None, :]
        pref = 2.0 * math.sqrt(self.kT / math.pi)
        out = []
        for a in range(self.M):
            acc = n.new_zeros(3, n.shape[1])
            for b in range(self.M):
                idx, eh, s, w = self.shell[a, b]
                if idx.shape[0] == 0:
                    continue
                ub = ut[b]
                ue = torch.stack([self._ext(ub[k])[idx] for k in range(3)])        # (3, E, N)
                kdu = (eh.T[:, :, None] * (ue - ub[:, None, :])).sum(0)            # (E, N)
                g = 0.5 * (G[a, b][None, :] + self._ext(G[a, b])[idx])
                acc = acc + s * s * w * (eh.T @ (kdu * g * self._ext(n[b])[idx]))
            out.append(pref * n[a][None, :] * acc)
        return torch.stack(out)

    def drag_force(self, n, G, Jt):
        """C^drag of every species, (M, 3, N), from u~ = J~/n."""
        pos = n > 0
        ut = Jt / torch.where(pos, n, torch.ones_like(n))[:, None, :] * pos[:, None, :]
        out = []
        for a in range(self.M):
            acc = n.new_zeros(3, n.shape[1])
            for b in range(self.M):
                if b != a:
                    acc = acc + (self.gamma[a][b] * G[a, b] * n[b])[None, :] * (ut[a] - ut[b])
            out.append(-n[a][None, :] * acc)
        return torch.stack(out)

    def invert(self, f, g, n, Cmf, F, G):
        """Physical moments: J, u^a, Pi, u (Sec. 4.2 with the chosen inversion)."""
        Pit = g.sum(1)                                               # (M, N)
        Jt = torch.einsum("pk,mpn->mkn", self.c, f if self.single else g)   # (M, 3, N)
        nF = n[:, None, :] * F
        Y = nF + self.drag_force(n, G, Jt) if self.drag else nF
        if self.visc:
            Y = Y + self.visc_force(n, G, Jt)
        X = Cmf + Y
        if self.euler:                      # no half-step terms
            J = Jt
        else:                               # SD-TR takes the f inversion, with X
            J = Jt + 0.5 * (X if (self.printed or self.single) else Y)
        pos = n > 0
        nsafe = torch.where(pos, n, torch.ones_like(n))
        ua = J / nsafe[:, None, :] * pos[:, None, :]
        Cu = (Cmf * ua).sum(1)
        if self.qp:
            Pi = self.quasipressure(n, Cmf)
        elif self.euler or self.single:
            Pi = Pit
        else:
            Pi = Pit - 0.5 * self.beta * Cu if self.printed else Pit + 0.5 * self.beta * Cu
        ntot = n.sum(0)
        tpos = ntot > 0
        u = J.sum(0) / torch.where(tpos, ntot, torch.ones_like(ntot)) * tpos
        return J, ua, Pi, u, X, Y

    def quasipressure(self, n, Cmf):
        """Pi = n - beta Phi (Sec. 2, eq. quasipressure), Phi the trapezoidal
        line integral of C^mf from the origin along the axes in the order
        (x, y, z), or (symmetric mode) the mean over the six axis orders; the
        integrand and Pi vanish on solid nodes.  Returns (M, N)."""
        g = self.g
        o = self.qp_origin
        v = (Cmf * self.fluid).reshape(self.M, 3, g.nz, g.ny, g.nx)

        def dim(k):                 # tensor dimension of axis k in (M, z, y, x)
            return 3 - k

        def leg(vk, k):
            # S(e) = sum_{j<e} (v(j) + v(j+1))/2 along axis k, minus S(origin)
            d = dim(k)
            t = 0.5 * (vk.narrow(d, 0, vk.shape[d] - 1) + vk.narrow(d, 1, vk.shape[d] - 1))
            S = torch.cat([torch.zeros_like(vk.narrow(d, 0, 1)), torch.cumsum(t, d)], d)
            return S - S.narrow(d, o[k], 1)

        def at(t, k):               # fix axis k at the origin's coordinate
            return t.narrow(dim(k), o[k], 1)

        def order_phi(p0, p1, p2):
            A0 = leg(at(at(v[:, p0], p1), p2), p0)
            A1 = leg(at(v[:, p1], p2), p1)
            A2 = leg(v[:, p2], p2)
            return (A0 + A1) + A2

        orders = ([(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
                  if self.qp_symmetric else [(0, 1, 2)])
        phi = sum(order_phi(*od) for od in orders) / len(orders)
        return (n - self.beta * phi.reshape(self.M, -1)) * self.fluid

    def fields(self, f, V):
        n = f.sum(1) * self.fluid
        G = self.contact(n)
        Cmf = self.mean_field(n, G)
        F = self.external_force(V)[None, :, :] + self.body[:, :, None]
        return n, G, Cmf, F

    def step(self, f, g, V):
        """One step on post-streaming populations (M, Q, N) -> next ones."""
        n, G, Cmf, F = self.fields(f, V)
        J, ua, Pi, u, X, Y = self.invert(f, g, n, Cmf, F, G)
        w = self.w[None, :, None]
        # Hermite contractions, (M, Q, N)
        JH1 = torch.einsum("mkn,pk->mpn", J, self.H1)
        T = 2 * ua[:, :, None, :] * u[None, None, :, :] - u[None, :, None, :] * u[None, None, :, :]
        TH2 = torch.einsum("mijn,pij->mpn", T, self.H2)
        h2ua = torch.einsum("pij,mjn->mpin", self.H2, ua)                   # (M, Q, 3, N)
        feq = w * (n[:, None, :] + JH1 + n[:, None, :] * TH2)
        geq = w * (Pi[:, None, :] + JH1 + n[:, None, :] * TH2)
        H1b = self.H1[None, :, :, None]
        sf = w * (X[:, None, :, :] * (H1b + 2 * h2ua)).sum(2)
        sg = w * ((Cmf[:, None, :, :] * (ua[:, None, :, :] / self.vT2 + self.kappa * h2ua)).sum(2)
                  + (Y[:, None, :, :] * (H1b + 2 * h2ua)).sum(2))
        fs = (f + self.a * (feq - f) + self.b * sf) * self.fluid
        if self.single:                     # no g is evolved
            return self.stream(fs), torch.zeros_like(g)
        if self.qp:
            # the zeroth moment of g~ becomes the Pi~ that the inversion
            # maps to the quasi-pressure Pi
            Cu = (Cmf * ua).sum(1)
            target = Pi if self.euler else (Pi + 0.5 * self.beta * Cu if self.printed
                                            else Pi - 0.5 * self.beta * Cu)
            g = g + w * (target - g.sum(1))[:, None, :]
        gs = (g + self.a * (geq - g) + self.b * sg) * self.fluid
        return self.stream(fs), self.stream(gs)

    def stream(self, post):
        """Pull streaming with mid-point bounce-back, (M, Q, N)."""
        pulled = torch.stack([post[:, p, :][:, self.src[p]] for p in range(Q)], 1)
        bounced = post[:, OPP, :]
        return torch.where(self.blocked[None], bounced, pulled) * self.fluid

    def readout(self, f, g, V):
        n, G, Cmf, F = self.fields(f, V)
        J, ua, Pi, u, X, Y = self.invert(f, g, n, Cmf, F, G)
        return n, J * self.fluid

    def rest_state(self, n0):
        """f~ = g~ = w_p n0 on fluid nodes, (M, Q, N) each."""
        n0 = torch.as_tensor(np.asarray(n0, float).reshape(self.M, -1))
        f = self.w[None, :, None] * n0[:, None, :] * self.fluid
        return f.clone(), f.clone()

    def run(self, f, g, V, nsteps):
        for _ in range(nsteps):
            f, g = self.step(f, g, V)
        return f, g
