"""Plain FP64 CPU oracle of the stabilized Lattice Boltzmann-Enskog step.

TEST INFRASTRUCTURE ONLY.  The oracle (``lbe_oracle.c``) checks the GPU
library against the paper (arXiv:1202.3842, Secs. 2-4 and the Appendix).  Only
the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product path never does.  It shares
no code with ``paper_1202_3842_amd``.

``build()`` compiles the C source with gcc (``-O2``, no fast-math, OpenMP);
``Oracle`` wraps one context through ctypes with numpy arrays in host memory.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "lbe_oracle.c"
# LBEO_LIB points the loader at another build of the same source (the
# sanitizer test builds one with AddressSanitizer and UBSan)
LIB = Path(os.environ.get("LBEO_LIB", HERE / "liblbe_oracle.so"))

LBEO_VISC = 1 << 0
LBEO_PRINTED_INV = 1 << 1
LBEO_KAPPA4 = 1 << 2
LBEO_IDEAL = 1 << 3
LBEO_EULER = 1 << 4
LBEO_SINGLE = 1 << 5
LBEO_DRAG = 1 << 6
LBEO_PI_CARRIED = 1 << 7
LBEO_BALL_FLUID = 1 << 8
LBEO_QP_WITH_FEXT = 1
LBEO_QP_SYMMETRIC = 2

Q = 19


def build(verbose: bool = False) -> Path:
    """Compile the oracle into ``oracle/liblbe_oracle.so`` (always rebuilds)."""
    cmd = [
        "gcc", "-std=gnu11", "-O2", "-fno-fast-math", "-ffp-contract=off",
        "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
        "-Wno-unused-parameter", "-o", str(LIB) + ".tmp", str(SRC), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(str(LIB) + ".tmp", LIB)
    return LIB


class lbeo_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("periodic", C.c_uint), ("nspecies", C.c_int),
        ("sigma", C.c_double * 4), ("tau", C.c_double), ("kT", C.c_double),
        ("prec", C.c_int), ("flags", C.c_uint),
        ("att_eps", (C.c_double * 4) * 4), ("att_rc", C.c_double),
    ]


class lbeo_diag(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 4), ("gmom", C.c_double * 3),
        ("umax", C.c_double), ("err_n", C.c_double), ("err_u", C.c_double),
        ("err_J", C.c_double), ("unstable", C.c_int),
    ]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.lbeo_create.argtypes = [C.POINTER(lbeo_config), C.POINTER(P)]
        L.lbeo_destroy.argtypes = [P]
        L.lbeo_destroy.restype = None
        L.lbeo_last_error.restype = C.c_char_p
        L.lbeo_set_threads.argtypes = [C.c_int]
        L.lbeo_set_threads.restype = None
        L.lbeo_set_solid.argtypes = [P, C.POINTER(C.c_uint8)]
        L.lbeo_set_potential.argtypes = [P, dp]
        L.lbeo_set_body_force.argtypes = [P, C.c_int, dp]
        L.lbeo_init_density.argtypes = [P, C.c_int, dp]
        L.lbeo_step.argtypes = [P, C.c_int]
        L.lbeo_get_density.argtypes = [P, C.c_int, dp]
        L.lbeo_get_velocity.argtypes = [P, C.c_int, dp]
        L.lbeo_get_populations.argtypes = [P, C.c_int, C.c_int, dp]
        L.lbeo_set_populations.argtypes = [P, C.c_int, C.c_int, dp]
        L.lbeo_diagnostics.argtypes = [P, C.POINTER(lbeo_diag)]
        L.lbeo_get_forces.argtypes = [P, C.c_int, dp, dp]
        L.lbeo_get_contact.argtypes = [P, C.c_int, C.c_int, dp]
        L.lbeo_get_weighted_density.argtypes = [P, C.c_int, dp]
        L.lbeo_get_external_force.argtypes = [P, C.c_int, dp]
        L.lbeo_stream.argtypes = [P, dp, dp]
        L.lbeo_quasipressure.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.c_uint, dp]
        L.lbeo_init_quasipressure.argtypes = [P, C.POINTER(C.c_int), C.c_uint]
        L.lbeo_set_quasipressure_route.argtypes = [P, C.POINTER(C.c_int), C.c_uint]
        L.lbeo_get_divergence.argtypes = [P, dp]
        L.lbeo_shell.argtypes = [C.c_double, C.c_int, C.POINTER(C.c_int), dp]
        L.lbeo_ball.argtypes = [C.c_double, C.c_int, C.POINTER(C.c_int)]
        L.lbeo_bmcsl.argtypes = [C.c_int, dp, dp, C.c_int, C.c_int]
        L.lbeo_bmcsl.restype = C.c_double
        L.lbeo_d3q19.argtypes = [C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
        L.lbeo_d3q19.restype = None
        L.lbeo_collide_node.argtypes = [C.c_int, C.c_double, C.c_double, C.c_uint,
                                        dp, dp, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def _check(st: int):
    if st != 0:
        raise OracleError(st, lib().lbeo_last_error().decode())


def set_threads(n: int) -> None:
    lib().lbeo_set_threads(int(n))


def d3q19():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().lbeo_d3q19(c.ctypes.data_as(C.POINTER(C.c_int)), _dp(w),
                     opp.ctypes.data_as(C.POINTER(C.c_int)))
    return c, w, opp


def shell(sigma: float):
    """Full lattice shell of radius sigma: (offsets[npts,3], weight); the
    first half is S+ and the second half its mirror images."""
    n = lib().lbeo_shell(float(sigma), 0, None, None)
    _check(0 if n >= 0 else n)
    offs = np.zeros((max(n, 1), 3), dtype=np.int32)
    w = C.c_double(0.0)
    lib().lbeo_shell(float(sigma), n, offs.ctypes.data_as(C.POINTER(C.c_int)),
                     C.byref(w))
    return offs[:n], w.value


def ball(sigma: float):
    n = lib().lbeo_ball(float(sigma), 0, None)
    offs = np.zeros((max(n, 1), 3), dtype=np.int32)
    lib().lbeo_ball(float(sigma), n, offs.ctypes.data_as(C.POINTER(C.c_int)))
    return offs[:n]


def bmcsl(sigma, nbar, a: int, b: int) -> float:
    s = np.zeros(4)
    s[:len(sigma)] = sigma
    nb = np.zeros(4)
    nb[:len(nbar)] = nbar
    return lib().lbeo_bmcsl(len(sigma), _dp(s), _dp(nb), a, b)


def collide_node(M, tau, kT, flags, ft, gt, cmf, cvisc, F):
    ft = np.ascontiguousarray(ft, dtype=np.float64).reshape(M * Q)
    gt = np.ascontiguousarray(gt, dtype=np.float64).reshape(M * Q)
    cmf = np.ascontiguousarray(cmf, dtype=np.float64).reshape(M * 3)
    cvisc = np.ascontiguousarray(cvisc, dtype=np.float64).reshape(M * 3)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(M * 3)
    fo = np.zeros(M * Q)
    go = np.zeros(M * Q)
    mom = np.zeros(8 * M + 3)
    _check(lib().lbeo_collide_node(M, tau, kT, flags, _dp(ft), _dp(gt), _dp(cmf),
                                   _dp(cvisc), _dp(F), _dp(fo), _dp(go), _dp(mom)))
    return fo.reshape(M, Q), go.reshape(M, Q), mom


class Oracle:
    """One oracle context (host memory, FP64).  Arrays use the node index
    x + nx*(y + ny*z); numpy arrays shaped (nz, ny, nx) are accepted."""

    def __init__(self, nx, ny, nz, sigma, periodic=7, tau=1.0, kT=1.0 / 3.0,
                 flags=LBEO_VISC, att_eps=None, att_rc=0.0):
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.M = len(sigma)
        cfg = lbeo_config()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.periodic = periodic
        cfg.nspecies = self.M
        for i, s in enumerate(sigma):
            cfg.sigma[i] = s
        cfg.tau = tau
        cfg.kT = kT
        cfg.prec = 0
        cfg.flags = flags
        if att_eps is not None:
            e = np.asarray(att_eps, dtype=float)
            for a in range(self.M):
                for b in range(self.M):
                    cfg.att_eps[a][b] = float(e[a, b]) if e.ndim == 2 else float(e)
        cfg.att_rc = float(att_rc)
        self.cfg = cfg
        h = C.c_void_p()
        _check(lib().lbeo_create(C.byref(cfg), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().lbeo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _flat(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        assert a.size == self.N
        return a

    def set_solid(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        assert m.size == self.N
        _check(lib().lbeo_set_solid(self.h, m.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_potential(self, V):
        _check(lib().lbeo_set_potential(self.h, _dp(self._flat(V))))

    def set_body_force(self, species, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        _check(lib().lbeo_set_body_force(self.h, species, _dp(g)))

    def init_density(self, species, n0):
        _check(lib().lbeo_init_density(self.h, species, _dp(self._flat(n0))))

    def step(self, n=1):
        _check(lib().lbeo_step(self.h, int(n)))

    def density(self, species=0):
        out = np.zeros(self.N)
        _check(lib().lbeo_get_density(self.h, species, _dp(out)))
        return out.reshape(self.shape)

    def velocity(self, species=-1):
        out = np.zeros(3 * self.N)
        _check(lib().lbeo_get_velocity(self.h, species, _dp(out)))
        return out.reshape((3,) + self.shape)

    def populations(self, species=0, dist=0):
        out = np.zeros(19 * self.N)
        _check(lib().lbeo_get_populations(self.h, species, dist, _dp(out)))
        return out.reshape((19,) + self.shape)

    def set_populations(self, species, dist, pops):
        p = np.ascontiguousarray(pops, dtype=np.float64).reshape(-1)
        assert p.size == 19 * self.N
        _check(lib().lbeo_set_populations(self.h, species, dist, _dp(p)))

    def diagnostics(self):
        d = lbeo_diag()
        _check(lib().lbeo_diagnostics(self.h, C.byref(d)))
        return {
            "mass": list(d.mass)[: self.M], "gmom": list(d.gmom), "umax": d.umax,
            "err_n": d.err_n, "err_u": d.err_u, "err_J": d.err_J,
            "unstable": bool(d.unstable),
        }

    def forces(self, species=0):
        cm = np.zeros(3 * self.N)
        cv = np.zeros(3 * self.N)
        _check(lib().lbeo_get_forces(self.h, species, _dp(cm), _dp(cv)))
        return cm.reshape((3,) + self.shape), cv.reshape((3,) + self.shape)

    def contact(self, a=0, b=0):
        out = np.zeros(self.N)
        _check(lib().lbeo_get_contact(self.h, a, b, _dp(out)))
        return out.reshape(self.shape)

    def weighted_density(self, species=0):
        out = np.zeros(self.N)
        _check(lib().lbeo_get_weighted_density(self.h, species, _dp(out)))
        return out.reshape(self.shape)

    def external_force(self, species=0):
        out = np.zeros(3 * self.N)
        _check(lib().lbeo_get_external_force(self.h, species, _dp(out)))
        return out.reshape((3,) + self.shape)

    def stream(self, post):
        p = np.ascontiguousarray(post, dtype=np.float64).reshape(-1)
        assert p.size == 19 * self.N
        out = np.zeros_like(p)
        _check(lib().lbeo_stream(self.h, _dp(p), _dp(out)))
        return out.reshape((19,) + self.shape)

    def quasipressure(self, species=0, origin=(0, 0, 0), mode=0):
        """Pi of eq. quasipressure by the trapezoidal path integral; origin
        is (x, y, z)."""
        o = (C.c_int * 3)(*[int(v) for v in origin])
        out = np.zeros(self.N)
        _check(lib().lbeo_quasipressure(self.h, species, o, mode, _dp(out)))
        return out.reshape(self.shape)

    def init_quasipressure(self, origin=(0, 0, 0), mode=0):
        o = (C.c_int * 3)(*[int(v) for v in origin])
        _check(lib().lbeo_init_quasipressure(self.h, o, mode))

    def set_quasipressure_route(self, origin=(0, 0, 0), mode=LBEO_QP_SYMMETRIC):
        """Origin (x, y, z) and integrand of the per-step quasi-pressure
        (the default reading; see LBEO_PI_CARRIED)."""
        o = (C.c_int * 3)(*[int(v) for v in origin])
        _check(lib().lbeo_set_quasipressure_route(self.h, o, mode))

    def divergence(self):
        """D = div_h u / (v_T / dx) of the barycentric velocity."""
        out = np.zeros(self.N)
        _check(lib().lbeo_get_divergence(self.h, _dp(out)))
        return out.reshape(self.shape)
