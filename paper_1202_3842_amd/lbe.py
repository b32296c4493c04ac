"""Python binding of the C ABI in ``include/lbe.h`` (liblbe.so, built in-tree).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  PyTorch supplies the device workspace (one uint8 tensor) and
the HIP stream.  There is no CPU fallback: if ``liblbe.so`` is missing the
import-time loader raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from pathlib import Path
from typing import Optional, Sequence

import numpy as np

PKG = Path(__file__).resolve().parent
# LBE_LIB points the loader at another build of the same sources (the
# sanitizer test loads a host-only build with AddressSanitizer and UBSan)
LIB_PATH = Path(os.environ.get("LBE_LIB", PKG / "liblbe.so"))
HEADER = PKG.parent / "include" / "lbe.h"

LBE_OK = 0
LBE_ERR_ARG = -1
LBE_ERR_STATE = -2
LBE_ERR_OOM = -3
LBE_ERR_HIP = -4
LBE_ERR_UNSTABLE = -5
LBE_ERR_UNSUPPORTED = -6

LBE_FP64 = 0
LBE_FP32_POP = 1
LBE_HOST = 0
LBE_DEVICE = 1

LBE_VISC = 1 << 0
LBE_PRINTED_INV = 1 << 1
LBE_KAPPA4 = 1 << 2
LBE_IDEAL = 1 << 3
LBE_EULER = 1 << 4
LBE_SINGLE = 1 << 5
LBE_DRAG = 1 << 6
LBE_PI_CARRIED = 1 << 7
LBE_QP_WITH_FEXT = 1
LBE_QP_SYMMETRIC = 2
LBE_PROBE_GRAD, LBE_PROBE_STREAM, LBE_PROBE_SHELL_N, LBE_PROBE_SHELL_G, LBE_PROBE_QP = range(5)


class lbe_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("periodic", C.c_uint), ("nspecies", C.c_int),
        ("sigma", C.c_double * 4), ("tau", C.c_double), ("kT", C.c_double),
        ("prec", C.c_int), ("flags", C.c_uint),
        ("att_eps", (C.c_double * 4) * 4), ("att_rc", C.c_double),
    ]


class lbe_diag(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 4), ("gmom", C.c_double * 3),
        ("umax", C.c_double), ("err_n", C.c_double), ("err_u", C.c_double),
        ("err_J", C.c_double), ("unstable", C.c_int),
    ]


class LBEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbe status {code}: {msg}")
        self.code = code


_lib: Optional[C.CDLL] = None


def declared_symbols() -> list:
    """Names of the functions declared in include/lbe.h."""
    text = HEADER.read_text()
    return sorted(set(re.findall(r"\b(lbe_[a-z_0-9]+)\s*\(", text)))


def lib() -> C.CDLL:
    """Load liblbe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1202_3842_amd.build.build() first")
    L = C.CDLL(str(LIB_PATH))
    P = C.c_void_p
    L.lbe_last_error.restype = C.c_char_p
    L.lbe_workspace_bytes.restype = C.c_size_t
    L.lbe_workspace_bytes.argtypes = [C.POINTER(lbe_config)]
    L.lbe_create.argtypes = [C.POINTER(lbe_config), P, C.c_size_t, P, C.POINTER(P)]
    L.lbe_destroy.argtypes = [P]
    L.lbe_destroy.restype = None
    L.lbe_set_solid.argtypes = [P, P, C.c_int]
    L.lbe_set_potential.argtypes = [P, P, C.c_int]
    L.lbe_set_body_force.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
    L.lbe_init_density.argtypes = [P, C.c_int, P, C.c_int]
    L.lbe_step.argtypes = [P, C.c_int]
    L.lbe_step_phase.argtypes = [P, C.c_int]
    L.lbe_get_density.argtypes = [P, C.c_int, P, C.c_int]
    L.lbe_get_velocity.argtypes = [P, C.c_int, P, C.c_int]
    L.lbe_get_force.argtypes = [P, C.c_int, C.c_int, P, C.c_int]
    L.lbe_get_momentum.argtypes = [P, C.c_int, P, C.c_int]
    L.lbe_get_populations.argtypes = [P, C.c_int, C.c_int, P, C.c_int]
    L.lbe_set_populations.argtypes = [P, C.c_int, C.c_int, P, C.c_int]
    L.lbe_get_divergence.argtypes = [P, P, C.c_int]
    L.lbe_get_quasipressure.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.c_uint, P, C.c_int]
    L.lbe_init_quasipressure.argtypes = [P, C.POINTER(C.c_int), C.c_uint]
    L.lbe_set_quasipressure_route.argtypes = [P, C.POINTER(C.c_int), C.c_uint]
    L.lbe_get_quasipressure_noalloc.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.c_uint, P]
    L.lbe_diagnostics.argtypes = [P, C.POINTER(lbe_diag)]
    L.lbe_synchronize.argtypes = [P]
    L.lbe_set_force_zchunk.argtypes = [P, C.c_int]
    L.lbe_set_force_tiling.argtypes = [P, C.c_int, C.c_int, C.c_int]
    L.lbe_batch_workspace_bytes.restype = C.c_size_t
    L.lbe_batch_workspace_bytes.argtypes = [C.POINTER(lbe_config), C.c_int]
    L.lbe_batch_create.argtypes = [C.POINTER(lbe_config), C.c_int, P, C.c_size_t, P, C.POINTER(P)]
    L.lbe_batch_box.restype = P
    L.lbe_batch_box.argtypes = [P, C.c_int]
    L.lbe_batch_step.argtypes = [P, C.c_int, C.c_int]
    L.lbe_batch_destroy.argtypes = [P]
    L.lbe_batch_destroy.restype = None
    L.lbe_adjoint_workspace_bytes.restype = C.c_size_t
    L.lbe_adjoint_workspace_bytes.argtypes = [C.POINTER(lbe_config), C.c_int, C.c_int]
    L.lbe_adjoint_create.argtypes = [P, C.c_int, C.c_int, P, C.c_size_t, C.POINTER(P)]
    L.lbe_adjoint_forward.argtypes = [P]
    L.lbe_adjoint_backward.argtypes = [P, P, P, P, C.c_int, P, C.c_int]
    L.lbe_adjoint_state_grad.argtypes = [P, C.c_int, C.c_int, P, C.c_int]
    L.lbe_adjoint_probe.argtypes = [P, C.c_int, C.c_int, P, P]
    L.lbe_adjoint_destroy.argtypes = [P]
    L.lbe_adjoint_destroy.restype = None
    _lib = L
    return L


def _check(st: int):
    if st != LBE_OK:
        raise LBEError(st, lib().lbe_last_error().decode())


def make_config(nx, ny, nz, sigma: Sequence[float], periodic=7, tau=1.0, kT=1.0 / 3.0,
                prec=LBE_FP64, flags=LBE_VISC, att_eps=None, att_rc=0.0) -> lbe_config:
    """att_eps: M x M symmetric depths of the attractive tail (a scalar is
    taken for every pair), att_rc: its cutoff; see lbe_config in lbe.h."""
    cfg = lbe_config()
    cfg.nx, cfg.ny, cfg.nz = int(nx), int(ny), int(nz)
    cfg.periodic = int(periodic)
    cfg.nspecies = len(sigma)
    for i, s in enumerate(sigma):
        cfg.sigma[i] = float(s)
    cfg.tau = float(tau)
    cfg.kT = float(kT)
    cfg.prec = int(prec)
    cfg.flags = int(flags)
    if att_eps is not None:
        e = np.asarray(att_eps, dtype=float)
        for a in range(len(sigma)):
            for b in range(len(sigma)):
                cfg.att_eps[a][b] = float(e[a, b]) if e.ndim == 2 else float(e)
    cfg.att_rc = float(att_rc)
    return cfg


def workspace_bytes(cfg: lbe_config) -> int:
    n = lib().lbe_workspace_bytes(C.byref(cfg))
    if n == 0:
        raise LBEError(LBE_ERR_ARG, lib().lbe_last_error().decode())
    return int(n)


class Box:
    """One lattice box on the current HIP device.

    Host inputs are numpy arrays shaped (nz, ny, nx) (or flat); device inputs
    are torch CUDA tensors.  Outputs are numpy arrays unless ``out`` (a torch
    CUDA tensor) is given.
    """

    def __init__(self, nx, ny, nz, sigma, periodic=7, tau=1.0, kT=1.0 / 3.0,
                 prec=LBE_FP64, flags=LBE_VISC, stream=None, _member=None, att_eps=None, att_rc=0.0):
        import torch
        self.torch = torch
        self.cfg = make_config(nx, ny, nz, sigma, periodic, tau, kT, prec, flags, att_eps, att_rc)
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.M = len(sigma)
        self.prec = prec
        self.flags = flags
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if _member is not None:  # a member context owned by a Batch
            self.h = _member
            self.owned = False
            return
        nbytes = workspace_bytes(self.cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _check(lib().lbe_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()),
                                nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.owned = True

    # ---- lifetime -------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and getattr(self, "owned", False):
            lib().lbe_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- marshalling ----------------------------------------------------
    def _src(self, a, dtype, count):
        """(pointer, where, keepalive) for an input array."""
        t = self.torch
        if isinstance(a, t.Tensor) and a.is_cuda:
            a = a.contiguous()
            assert a.numel() == count and a.element_size() == np.dtype(dtype).itemsize
            return C.c_void_p(a.data_ptr()), LBE_DEVICE, a
        arr = np.ascontiguousarray(np.asarray(a), dtype=dtype).reshape(-1)
        assert arr.size == count, (arr.size, count)
        return C.c_void_p(arr.ctypes.data), LBE_HOST, arr

    def _dst(self, out, dtype, count):
        t = self.torch
        if out is not None:
            assert out.is_cuda and out.is_contiguous() and out.numel() == count
            return C.c_void_p(out.data_ptr()), LBE_DEVICE, out
        arr = np.empty(count, dtype=dtype)
        return C.c_void_p(arr.ctypes.data), LBE_HOST, arr

    # ---- ABI calls ------------------------------------------------------
    def set_solid(self, mask):
        p, w, keep = self._src(mask, np.uint8, self.N)
        _check(lib().lbe_set_solid(self.h, p, w))

    def set_potential(self, V):
        p, w, keep = self._src(V, np.float64, self.N)
        _check(lib().lbe_set_potential(self.h, p, w))

    def set_body_force(self, species, g):
        arr = (C.c_double * 3)(*[float(v) for v in g])
        _check(lib().lbe_set_body_force(self.h, int(species), arr))

    def init_density(self, species, n0):
        p, w, keep = self._src(n0, np.float64, self.N)
        _check(lib().lbe_init_density(self.h, int(species), p, w))

    def step(self, n=1):
        _check(lib().lbe_step(self.h, int(n)))

    def step_phase(self, phase):
        _check(lib().lbe_step_phase(self.h, int(phase)))

    def synchronize(self):
        _check(lib().lbe_synchronize(self.h))

    def set_force_zchunk(self, zchunk):
        _check(lib().lbe_set_force_zchunk(self.h, int(zchunk)))

    def set_force_tiling(self, zchunk, order=0, shape=0):
        _check(lib().lbe_set_force_tiling(self.h, int(zchunk), int(order), int(shape)))

    def density(self, species=0, out=None):
        p, w, arr = self._dst(out, np.float64, self.N)
        _check(lib().lbe_get_density(self.h, int(species), p, w))
        return arr.reshape(self.shape) if out is None else arr

    def velocity(self, species=-1, out=None):
        p, w, arr = self._dst(out, np.float64, 3 * self.N)
        _check(lib().lbe_get_velocity(self.h, int(species), p, w))
        return arr.reshape((3,) + self.shape) if out is None else arr

    def momentum(self, species=-1, out=None):
        p, w, arr = self._dst(out, np.float64, 3 * self.N)
        _check(lib().lbe_get_momentum(self.h, int(species), p, w))
        return arr.reshape((3,) + self.shape) if out is None else arr

    def force(self, species=0, which=0, out=None):
        p, w, arr = self._dst(out, np.float64, 3 * self.N)
        _check(lib().lbe_get_force(self.h, int(species), int(which), p, w))
        return arr.reshape((3,) + self.shape) if out is None else arr

    @property
    def pop_dtype(self):
        return np.float64 if self.prec == LBE_FP64 else np.float32

    def populations(self, species=0, dist=0, out=None):
        p, w, arr = self._dst(out, self.pop_dtype, 19 * self.N)
        _check(lib().lbe_get_populations(self.h, int(species), int(dist), p, w))
        return arr.reshape((19,) + self.shape) if out is None else arr

    def set_populations(self, species, dist, pops):
        p, w, keep = self._src(pops, self.pop_dtype, 19 * self.N)
        _check(lib().lbe_set_populations(self.h, int(species), int(dist), p, w))

    def divergence(self, out=None):
        """D = div_h u / (v_T/dx) of the barycentric velocity."""
        p, w, arr = self._dst(out, np.float64, self.N)
        _check(lib().lbe_get_divergence(self.h, p, w))
        return arr.reshape(self.shape) if out is None else arr

    def _origin(self, origin):
        if origin is None:
            nz, ny, nx = self.shape
            origin = (nx // 2, ny // 2, nz // 2)
        return (C.c_int * 3)(*[int(v) for v in origin])

    def quasipressure(self, species=0, origin=None, mode=0, out=None):
        """Pi of eq. quasipressure (trapezoidal path integral from origin =
        (x, y, z), the box centre by default); mode LBE_QP_WITH_FEXT adds
        n F to the integrand as printed, LBE_QP_SYMMETRIC averages the six
        axis orders of the path."""
        p, w, arr = self._dst(out, np.float64, self.N)
        _check(lib().lbe_get_quasipressure(self.h, int(species), self._origin(origin), int(mode), p, w))
        return arr.reshape(self.shape) if out is None else arr

    def init_quasipressure(self, origin=None, mode=0):
        """Set the zeroth moment of every species' g~ to the quasi-pressure
        of the current state (for a start from a non-uniform profile)."""
        _check(lib().lbe_init_quasipressure(self.h, self._origin(origin), int(mode)))

    def quasipressure_noalloc(self, out, species=0, origin=None, mode=0):
        """lbe_get_quasipressure_noalloc: Pi into `out`, a float64 CUDA tensor
        of N values (the scans use the library's static scratch)."""
        t = self.torch
        assert isinstance(out, t.Tensor) and out.is_cuda and out.dtype == t.float64
        assert out.numel() == self.N and out.is_contiguous()
        _check(lib().lbe_get_quasipressure_noalloc(self.h, int(species), self._origin(origin), int(mode),
                                                   C.c_void_p(out.data_ptr())))
        return out

    def set_quasipressure_route(self, origin=None, mode=LBE_QP_SYMMETRIC):
        """Origin (x, y, z) and mode of the per-step quasi-pressure (the
        default reading; see LBE_PI_CARRIED)."""
        _check(lib().lbe_set_quasipressure_route(self.h, self._origin(origin), int(mode)))

    def diagnostics(self):
        d = lbe_diag()
        _check(lib().lbe_diagnostics(self.h, C.byref(d)))
        return {
            "mass": list(d.mass)[: self.M], "gmom": list(d.gmom), "umax": d.umax,
            "err_n": d.err_n, "err_u": d.err_u, "err_J": d.err_J,
            "unstable": bool(d.unstable),
        }


def box_from_workload(w, prec=LBE_FP64, flags=LBE_VISC) -> Box:
    """Create a Box and load a paper_1202_3842_amd.workloads.Workload into it."""
    b = Box(w.nx, w.ny, w.nz, w.sigma, periodic=w.periodic, tau=w.tau, kT=w.kT,
            prec=prec, flags=flags, att_eps=getattr(w, "att_eps", None), att_rc=getattr(w, "att_rc", 0.0))
    if w.solid is not None:
        b.set_solid(w.solid)
    if w.V is not None:
        b.set_potential(w.V)
    for a, g in enumerate(w.body):
        b.set_body_force(a, g)
    for a, n in enumerate(w.density):
        b.init_density(a, n)
    _set_route(b, w, flags)
    return b


def _set_route(b: "Box", w, flags) -> None:
    route = getattr(w, "qp_route", None)
    if route is not None and not (flags & LBE_SINGLE):
        b.set_quasipressure_route(*route)


def load_workload(b: "Box", w) -> None:
    """Load a paper_1202_3842_amd.workloads.Workload into an existing Box."""
    if w.solid is not None:
        b.set_solid(w.solid)
    if w.V is not None:
        b.set_potential(w.V)
    for a, g in enumerate(w.body):
        b.set_body_force(a, g)
    for a, n in enumerate(w.density):
        b.init_density(a, n)
    _set_route(b, w, b.flags)


class Batch:
    """Independent boxes (same species count) stepped together (lbe_batch_*).  Member
    boxes are Box objects sharing the batch's workspace and stream."""

    SERIAL, BATCHED, GRAPH = 0, 1, 2

    def __init__(self, configs, stream=None):
        import torch
        self.torch = torch
        n = len(configs)
        arr = (lbe_config * n)(*configs)
        self._cfgs = arr
        nbytes = lib().lbe_batch_workspace_bytes(arr, n)
        if nbytes == 0:
            raise LBEError(LBE_ERR_ARG, lib().lbe_last_error().decode())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        # graph capture needs a stream other than the null stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().lbe_batch_create(arr, n, C.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.boxes = []
        for i, c in enumerate(configs):
            m = lib().lbe_batch_box(self.h, i)
            sig = [c.sigma[k] for k in range(c.nspecies)]
            self.boxes.append(Box(c.nx, c.ny, c.nz, sig, c.periodic, c.tau, c.kT, c.prec, c.flags,
                                  stream=self.stream, _member=C.c_void_p(m)))

    def step(self, n=1, mode=2):
        _check(lib().lbe_batch_step(self.h, int(n), int(mode)))

    def synchronize(self):
        self.boxes[0].synchronize()

    def close(self):
        if getattr(self, "h", None):
            for b in self.boxes:
                b.h = None
            lib().lbe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_from_workloads(ws, prec=LBE_FP64, flags=LBE_VISC) -> Batch:
    cfgs = [make_config(w.nx, w.ny, w.nz, w.sigma, w.periodic, w.tau, w.kT, prec, flags,
                        att_eps=getattr(w, "att_eps", None), att_rc=getattr(w, "att_rc", 0.0)) for w in ws]
    b = Batch(cfgs)
    for box, w in zip(b.boxes, ws):
        load_workload(box, w)
    return b


class Adjoint:
    """Reverse mode of `nsteps` steps of a Box with respect to its potential
    V (lbe_adjoint_*), checkpointed every `segment` steps.

    forward() advances the box from its current state; backward(dn, dJ, dpop)
    takes dL/d(final n^a), dL/d(final J^a) and dL/d(final populations) (any
    may be None; numpy arrays or torch CUDA tensors shaped (M, nz, ny, nx),
    (M, 3, nz, ny, nx) and (2, M, 19, nz, ny, nx)) and returns dL/dV.
    """

    def __init__(self, box: Box, nsteps: int, segment: int = 20):
        torch = box.torch
        self.box = box
        self.nsteps = int(nsteps)
        self.segment = int(segment)
        n = lib().lbe_adjoint_workspace_bytes(C.byref(box.cfg), self.nsteps, self.segment)
        if n == 0:
            raise LBEError(LBE_ERR_UNSUPPORTED, lib().lbe_last_error().decode())
        self.workspace = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _check(lib().lbe_adjoint_create(box.h, self.nsteps, self.segment,
                                        C.c_void_p(self.workspace.data_ptr()), int(n), C.byref(h)))
        self.h = h

    def forward(self):
        _check(lib().lbe_adjoint_forward(self.h))
        # a token of this forward: a backward through an older one is refused
        self.forwards = getattr(self, "forwards", 0) + 1

    def backward(self, dn=None, dJ=None, dpop=None, out=None):
        b = self.box
        M, N = b.M, b.N
        t = b.torch
        dev = any(isinstance(a, t.Tensor) and a.is_cuda for a in (dn, dJ, dpop) if a is not None)
        ptrs, keep = [], []
        for a, count in ((dn, M * N), (dJ, 3 * M * N), (dpop, 2 * M * 19 * N)):
            if a is None:
                ptrs.append(None)
                continue
            if dev:
                a = t.as_tensor(a, dtype=t.float64, device="cuda").contiguous().reshape(-1)
                ptrs.append(C.c_void_p(a.data_ptr()))
            else:
                a = np.ascontiguousarray(np.asarray(a), dtype=np.float64).reshape(-1)
                ptrs.append(C.c_void_p(a.ctypes.data))
            assert a.numel() == count if dev else a.size == count
            keep.append(a)
        where = LBE_DEVICE if dev else LBE_HOST
        p, w, arr = b._dst(out, np.float64, N)
        _check(lib().lbe_adjoint_backward(self.h, ptrs[0], ptrs[1], ptrs[2], where, p, w))
        return arr.reshape(b.shape) if out is None else arr

    def probe(self, stage, transpose, x):
        """lbe_adjoint_probe: one linear stage K of the step (LBE_PROBE_*) or,
        with transpose, K^T as the reverse sweep computes it, applied to the
        torch CUDA tensor x (FP64) at the box's current state.  Returns a new
        flat tensor of the output's length."""
        b = self.box
        t = b.torch
        M, N = b.M, b.N
        Ns = (N + 63) // 64 * 64
        npairs = M * (M + 1) // 2
        sizes = {LBE_PROBE_GRAD: (N, 3 * N), LBE_PROBE_STREAM: (2 * M * 19 * Ns, 2 * M * 19 * Ns),
                 LBE_PROBE_SHELL_N: (M * N, 3 * M * N), LBE_PROBE_SHELL_G: (npairs * N, 3 * M * N),
                 LBE_PROBE_QP: (3 * M * N, M * N)}
        n_in, n_out = sizes[stage]
        if transpose:
            n_in, n_out = n_out, n_in
        x = t.as_tensor(x, dtype=t.float64, device="cuda").contiguous().reshape(-1)
        assert x.numel() == n_in, (x.numel(), n_in)
        out = t.zeros(n_out, dtype=t.float64, device="cuda")
        t.cuda.synchronize()
        _check(lib().lbe_adjoint_probe(self.h, int(stage), int(transpose), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(out.data_ptr())))
        return out

    def state_grad(self, species=0, dist=0, out=None):
        b = self.box
        p, w, arr = b._dst(out, np.float64, 19 * b.N)
        _check(lib().lbe_adjoint_state_grad(self.h, int(species), int(dist), p, w))
        return arr.reshape((19,) + b.shape) if out is None else arr

    def close(self):
        if getattr(self, "h", None):
            lib().lbe_adjoint_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def potential_to_state(V, adjoint: Adjoint, reset):
    """Differentiable map V -> (n, J) of the final state, for torch autograd.

    V: float64 torch tensor (nz, ny, nx) on the GPU; reset(box) puts the box
    into the initial state (called before each forward).  Returns n shaped
    (M, nz, ny, nx) and J shaped (M, 3, nz, ny, nx), CUDA float64; their
    gradients flow back to V through lbe_adjoint_backward.
    """
    return _PotentialToState.apply(V, adjoint, reset)


def _autograd_function():
    import torch

    class PotentialToState(torch.autograd.Function):
        @staticmethod
        def forward(ctx, V, adjoint, reset):
            b = adjoint.box
            Vd = V.detach().to(device="cuda", dtype=torch.float64).contiguous()
            b.set_potential(Vd)
            reset(b)
            adjoint.forward()
            n = torch.empty((b.M,) + b.shape, dtype=torch.float64, device="cuda")
            J = torch.empty((b.M, 3) + b.shape, dtype=torch.float64, device="cuda")
            for a in range(b.M):
                b.density(a, out=n[a].view(-1))
                b.momentum(a, out=J[a].view(-1))
            ctx.adjoint = adjoint
            ctx.token = adjoint.forwards
            ctx.V_device = V.device
            return n, J

        @staticmethod
        def backward(ctx, gn, gJ):
            adj = ctx.adjoint
            if adj.forwards != ctx.token:
                raise RuntimeError("the Adjoint ran another forward after this one; its tape "
                                   "belongs to the later forward")
            b = adj.box
            out = torch.empty(b.shape, dtype=torch.float64, device="cuda")
            gn = None if gn is None else gn.to(device="cuda", dtype=torch.float64).contiguous()
            gJ = None if gJ is None else gJ.to(device="cuda", dtype=torch.float64).contiguous()
            if gn is None and gJ is None:
                return torch.zeros(b.shape, dtype=torch.float64, device=ctx.V_device), None, None
            adj.backward(gn, gJ, None, out=out.view(-1))
            return out.to(ctx.V_device), None, None

    return PotentialToState


class _Lazy:
    fn = None

    def apply(self, *args):
        if _Lazy.fn is None:
            _Lazy.fn = _autograd_function()
        return _Lazy.fn.apply(*args)


_PotentialToState = _Lazy()
