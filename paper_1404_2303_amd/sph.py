"""Python binding of the C ABI in include/sph.h (ctypes; argument marshalling only).

Torch tensors provide device memory and the stream; every computation runs in
the HIP kernels of libsph_mi355x.so.  The low-level functions carry the C
names (``sph_create``, ``sph_build_cells``, ``sph_sort``, ``sph_density``,
``sph_force``, ``sph_step``, ``sph_step_adaptive``, ``sph_integrate``,
``sph_backward``); :class:`Context` wraps them
for tensors and :class:`SPHPass` exposes the pass to torch.autograd.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph_mi355x.so")

SPH_OK, SPH_E_INVALID_ARG, SPH_E_NONFINITE, SPH_E_H_TOO_LARGE, SPH_E_NOT_CONVERGED = 0, 1, 2, 3, 4
SPH_E_CAPACITY, SPH_E_OOM, SPH_E_HIP, SPH_E_STATE = 5, 6, 7, 8
SPH_FP64, SPH_FP32_ACC64 = 0, 1
SPH_BALSARA_CURL, SPH_BALSARA_DIV = 0, 1
SPH_REUSE_OFF, SPH_REUSE_ORDERINGS, SPH_REUSE_CELLS = 0, 1, 2
SPH_STAGING_COMPACT, SPH_STAGING_WIDE = 0, 1
SPH_SWEEP_AUTO, SPH_SWEEP_SHARED, SPH_SWEEP_SPLIT = 0, 1, 2

EXPORTED = ["sph_default_params", "sph_create", "sph_destroy", "sph_build_cells", "sph_sort",
            "sph_density", "sph_force", "sph_step", "sph_get_stats", "sph_status_string",
            "sph_enable_timing", "sph_get_kernel_times", "sph_density_async", "sph_check",
            "sph_graph_capture", "sph_graph_launch", "sph_backward", "sph_estimate_h", "sph_step_adaptive",
            "sph_integrate", "sph_refresh", "sph_mts_init", "sph_mts_step"]

P = ctypes.c_void_p


class sph_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("n_ngb", ctypes.c_double), ("ngb_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("balsara_eps", ctypes.c_double), ("precision", ctypes.c_int),
                ("cell_target", ctypes.c_int), ("h_margin", ctypes.c_double),
                ("max_rebuilds", ctypes.c_int), ("max_depth", ctypes.c_int), ("split_count", ctypes.c_int),
                ("split_frac", ctypes.c_double), ("cfl", ctypes.c_double), ("balsara_form", ctypes.c_int),
                ("reuse", ctypes.c_int), ("staging", ctypes.c_int), ("shared_min", ctypes.c_int),
                ("fixed_h", ctypes.c_int), ("keep_adjoint", ctypes.c_int), ("sweep", ctypes.c_int)]


class sph_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, P) for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m", "h")]


class sph_batch(ctypes.Structure):
    _fields_ = [("nbox", ctypes.c_int), ("box_offsets", P), ("box_len", P)]


DENSITY_FIELDS = ("rho", "omega", "n_ngb", "div_v", "curl_v", "balsara", "pressure", "sound", "n_iter",
                  "n_dens")


class sph_density_out(ctypes.Structure):
    _fields_ = [(k, P) for k in DENSITY_FIELDS]


class sph_kernel_times(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_float), ("sort_ms", ctypes.c_float), ("density_ms", ctypes.c_float),
                ("force_ms", ctypes.c_float), ("backward_ms", ctypes.c_float)]


FORCE_FIELDS = ("ax", "ay", "az", "dudt", "n_pairs", "dt")


class sph_force_out(ctypes.Structure):
    _fields_ = [(k, P) for k in FORCE_FIELDS]


class sph_grad_in(ctypes.Structure):
    _fields_ = [(k, P) for k in ("rho", "ax", "ay", "az", "dudt")]


class sph_grad_out(ctypes.Structure):
    _fields_ = [(k, P) for k in ("x", "y", "z", "h")]


class sph_stats(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_units", ctypes.c_int64), ("grid", ctypes.c_int32 * 3),
                ("rebuilds", ctypes.c_int32), ("max_iter_used", ctypes.c_int32),
                ("unconverged", ctypes.c_int32), ("depth", ctypes.c_int32), ("refreshes", ctypes.c_int32),
                ("drift", ctypes.c_double), ("generation", ctypes.c_uint64)]


_lib = None


def load_library():
    """Load libsph_mi355x.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        lib.sph_default_params.restype = None
        lib.sph_default_params.argtypes = [ctypes.POINTER(sph_params)]
        lib.sph_create.restype = st
        lib.sph_create.argtypes = [ctypes.POINTER(sph_params), ctypes.POINTER(P)]
        lib.sph_destroy.restype = st
        lib.sph_destroy.argtypes = [P]
        lib.sph_build_cells.restype = st
        lib.sph_build_cells.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch), P]
        lib.sph_sort.restype = st
        lib.sph_sort.argtypes = [P, P]
        lib.sph_density.restype = st
        lib.sph_density.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_density_out), P]
        lib.sph_force.restype = st
        lib.sph_force.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_force_out), P]
        lib.sph_step.restype = st
        lib.sph_step.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch),
                                 ctypes.POINTER(sph_force_out), ctypes.c_double, P]
        lib.sph_step_adaptive.restype = st
        lib.sph_step_adaptive.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch),
                                          ctypes.POINTER(sph_force_out), ctypes.c_double, ctypes.c_double, P, P, P]
        lib.sph_integrate.restype = st
        lib.sph_integrate.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch),
                                      ctypes.POINTER(sph_force_out), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P]
        lib.sph_mts_init.restype = st
        lib.sph_mts_init.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_force_out), P,
                                     ctypes.c_double, ctypes.c_int, P]
        lib.sph_mts_step.restype = st
        lib.sph_mts_step.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_force_out), P,
                                     ctypes.POINTER(ctypes.c_int64), P]
        lib.sph_refresh.restype = st
        lib.sph_refresh.argtypes = [P, ctypes.POINTER(sph_particles), P]
        lib.sph_get_stats.restype = st
        lib.sph_get_stats.argtypes = [P, ctypes.POINTER(sph_stats)]
        lib.sph_enable_timing.restype = st
        lib.sph_enable_timing.argtypes = [P, ctypes.c_int]
        lib.sph_get_kernel_times.restype = st
        lib.sph_get_kernel_times.argtypes = [P, ctypes.POINTER(sph_kernel_times)]
        lib.sph_density_async.restype = st
        lib.sph_density_async.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_density_out), P]
        lib.sph_check.restype = st
        lib.sph_check.argtypes = [P, P]
        lib.sph_graph_capture.restype = st
        lib.sph_graph_capture.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch), P,
                                          ctypes.POINTER(sph_density_out), ctypes.POINTER(sph_force_out), P]
        lib.sph_graph_launch.restype = st
        lib.sph_graph_launch.argtypes = [P, P]
        lib.sph_backward.restype = st
        lib.sph_backward.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_grad_in),
                                     ctypes.POINTER(sph_grad_out), ctypes.c_int, ctypes.c_uint64, P]
        lib.sph_pass_noalloc.restype = st
        lib.sph_pass_noalloc.argtypes = [ctypes.POINTER(sph_params), ctypes.POINTER(sph_particles),
                                         ctypes.POINTER(sph_density_out), ctypes.POINTER(sph_force_out), P]
        lib.sph_estimate_h.restype = st
        lib.sph_estimate_h.argtypes = [P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_batch), P]
        lib.sph_status_string.restype = ctypes.c_char_p
        lib.sph_status_string.argtypes = [st]
        _lib = lib
    return _lib


class SPHError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load_library().sph_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def _check(status: int, where: str, allow=()):
    if status != SPH_OK and status not in allow:
        raise SPHError(status, where)
    return status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- C names
def sph_default_params() -> sph_params:
    p = sph_params()
    load_library().sph_default_params(ctypes.byref(p))
    return p


def sph_create(params: sph_params):
    ctx = P()
    _check(load_library().sph_create(ctypes.byref(params), ctypes.byref(ctx)), "sph_create")
    return ctx


def sph_destroy(ctx):
    return load_library().sph_destroy(ctx)


def sph_build_cells(ctx, parts: sph_particles, batch: Optional[sph_batch], stream):
    return load_library().sph_build_cells(ctx, ctypes.byref(parts),
                                          ctypes.byref(batch) if batch is not None else None, stream)


def sph_estimate_h(ctx, parts: sph_particles, batch: Optional[sph_batch], stream):
    return load_library().sph_estimate_h(ctx, ctypes.byref(parts), ctypes.byref(batch) if batch is not None else None,
                                         stream)


def sph_sort(ctx, stream):
    return load_library().sph_sort(ctx, stream)


def sph_density(ctx, parts: sph_particles, out: Optional[sph_density_out], stream):
    return load_library().sph_density(ctx, ctypes.byref(parts), ctypes.byref(out) if out is not None else None,
                                      stream)


def sph_force(ctx, parts: sph_particles, out: sph_force_out, stream):
    return load_library().sph_force(ctx, ctypes.byref(parts), ctypes.byref(out), stream)


def sph_step(ctx, parts: sph_particles, batch: Optional[sph_batch], acc: sph_force_out, dt: float, stream):
    return load_library().sph_step(ctx, ctypes.byref(parts), ctypes.byref(batch) if batch is not None else None,
                                   ctypes.byref(acc), float(dt), stream)


def sph_step_adaptive(ctx, parts: sph_particles, batch: Optional[sph_batch], acc: sph_force_out, dt_max: float,
                      t_end: float, t_box, dt_box, stream):
    return load_library().sph_step_adaptive(ctx, ctypes.byref(parts),
                                            ctypes.byref(batch) if batch is not None else None, ctypes.byref(acc),
                                            float(dt_max), float(t_end), t_box, dt_box, stream)


def sph_integrate(ctx, parts: sph_particles, batch: Optional[sph_batch], acc: sph_force_out, t_end: float,
                  dt_max: float, max_steps: int, steps, stream):
    return load_library().sph_integrate(ctx, ctypes.byref(parts), ctypes.byref(batch) if batch is not None else None,
                                        ctypes.byref(acc), float(t_end), float(dt_max), int(max_steps), steps,
                                        stream)


def sph_density_async(ctx, parts: sph_particles, out: Optional[sph_density_out], stream):
    return load_library().sph_density_async(ctx, ctypes.byref(parts),
                                            ctypes.byref(out) if out is not None else None, stream)


def sph_check(ctx, stream):
    return load_library().sph_check(ctx, stream)


def sph_graph_capture(ctx, parts: sph_particles, batch: Optional[sph_batch], h_init, dout, fout, stream):
    return load_library().sph_graph_capture(ctx, ctypes.byref(parts),
                                            ctypes.byref(batch) if batch is not None else None, h_init,
                                            ctypes.byref(dout) if dout is not None else None,
                                            ctypes.byref(fout), stream)


def sph_graph_launch(ctx, stream):
    return load_library().sph_graph_launch(ctx, stream)


def sph_backward(ctx, parts: sph_particles, gin: sph_grad_in, gout: sph_grad_out, implicit_h: int, generation: int,
                 stream):
    return load_library().sph_backward(ctx, ctypes.byref(parts), ctypes.byref(gin), ctypes.byref(gout),
                                       int(implicit_h), int(generation), stream)


SPH_NOALLOC_MAX_PARTICLES = 32768


def sph_pass_noalloc(params: sph_params, parts: sph_particles, dout: Optional[sph_density_out],
                     fout: sph_force_out, stream):
    return load_library().sph_pass_noalloc(ctypes.byref(params), ctypes.byref(parts),
                                           ctypes.byref(dout) if dout is not None else None, ctypes.byref(fout),
                                           stream)


# ---------------------------------------------------------------- tensor layer
@dataclass
class Particles:
    """FP64 device tensors, one entry per particle (positions/velocities as (N,3) are split)."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    vz: torch.Tensor
    u: torch.Tensor
    m: torch.Tensor
    h: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x.numel())

    @staticmethod
    def from_numpy(ps, device="cuda"):
        """From a workloads.ParticleSet (numpy) to contiguous FP64 device tensors."""
        def t(a):
            return torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)
        return Particles(x=t(ps.pos[:, 0]), y=t(ps.pos[:, 1]), z=t(ps.pos[:, 2]),
                         vx=t(ps.vel[:, 0]), vy=t(ps.vel[:, 1]), vz=t(ps.vel[:, 2]),
                         u=t(ps.u), m=t(ps.m), h=t(ps.h0))

    def c_struct(self) -> sph_particles:
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m", "h"):
            t = getattr(self, k)
            if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != self.n or not t.is_cuda:
                raise ValueError(f"particle field {k} must be a contiguous float64 CUDA tensor of length n")
        return sph_particles(self.n, *[_ptr(getattr(self, k)) for k in
                                       ("x", "y", "z", "vx", "vy", "vz", "u", "m", "h")])


def _as_f64(t):
    return None if t is None else t.to(torch.float64).contiguous()


class Batch:
    """Host-side batch descriptor (box offsets and lengths), kept alive with its ctypes view."""

    def __init__(self, offsets, lengths):
        import numpy as np
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.lengths = np.ascontiguousarray(lengths, dtype=np.float64).reshape(-1)
        self.nbox = len(self.offsets) - 1
        self.c = sph_batch(self.nbox, self.offsets.ctypes.data_as(P), self.lengths.ctypes.data_as(P))


class Context:
    """One library context (device workspace) with tensor-level calls."""

    def __init__(self, box=(1.0, 1.0, 1.0), precision: str = "fp32", **kw):
        p = sph_default_params()
        for d in range(3):
            p.box[d] = float(box[d])
        p.precision = SPH_FP64 if precision in ("fp64", SPH_FP64) else SPH_FP32_ACC64
        for k, v in kw.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        self.params = p
        self.ctx = sph_create(p)

    def close(self):
        if self.ctx:
            sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_cells(self, parts: Particles, batch: Optional[Batch] = None):
        _check(sph_build_cells(self.ctx, parts.c_struct(), batch.c if batch else None, _stream()),
               "sph_build_cells")

    def mts_init(self, parts: Particles, dt_base: float, max_bin: int, acc: Optional[dict] = None):
        """Multiple time-stepping: full pass and time bins; returns (acc, bins)."""
        if acc is None:
            acc = self.force_buffers(parts.n, parts.x.device)
        bins = torch.zeros(parts.n, dtype=torch.int32, device=parts.x.device)
        c = sph_force_out(*[_ptr(acc.get(k)) for k in FORCE_FIELDS])
        _check(load_library().sph_mts_init(self.ctx, ctypes.byref(parts.c_struct()), ctypes.byref(c), _ptr(bins),
                                           float(dt_base), int(max_bin), _stream()), "sph_mts_init",
               (SPH_E_NOT_CONVERGED,))
        return acc, bins

    def mts_step(self, parts: Particles, acc: dict, bins: torch.Tensor, count: bool = False):
        """One base step of multiple time-stepping; returns the number of active particles
        (with count=True, which synchronises) or None."""
        if bins.dtype != torch.int32 or bins.numel() != parts.n or not bins.is_cuda:
            raise ValueError("bins must be an int32 CUDA tensor with one value per particle")
        c = sph_force_out(*[_ptr(acc.get(k)) for k in FORCE_FIELDS])
        na = ctypes.c_int64(0)
        _check(load_library().sph_mts_step(self.ctx, ctypes.byref(parts.c_struct()), ctypes.byref(c), _ptr(bins),
                                           ctypes.byref(na) if count else None, _stream()), "sph_mts_step",
               (SPH_E_NOT_CONVERGED,))
        return int(na.value) if count else None

    def refresh(self, parts: Particles):
        """Refresh the cell-ordered particle data in the cells and orderings of the last build."""
        _check(load_library().sph_refresh(self.ctx, ctypes.byref(parts.c_struct()), _stream()), "sph_refresh")

    def sort(self):
        _check(sph_sort(self.ctx, _stream()), "sph_sort")

    def estimate_h(self, parts: Particles, batch: Optional[Batch] = None):
        """Overwrite parts.h with the local-density estimate (needs max_depth >= 1)."""
        _check(sph_estimate_h(self.ctx, parts.c_struct(), batch.c if batch else None, _stream()), "sph_estimate_h")

    def density(self, parts: Particles, want=DENSITY_FIELDS, allow_unconverged=False):
        n = parts.n
        dev = parts.x.device
        out = {}
        for k in want:
            if k in ("n_iter", "n_dens"):
                out[k] = torch.empty(n, dtype=torch.int32, device=dev)
            elif k == "curl_v":
                out[k] = torch.empty((n, 3), dtype=torch.float64, device=dev)
            else:
                out[k] = torch.empty(n, dtype=torch.float64, device=dev)
        c = sph_density_out(*[_ptr(out.get(k)) for k in DENSITY_FIELDS])
        allow = (SPH_E_NOT_CONVERGED,) if allow_unconverged else ()
        self.last_density_status = _check(sph_density(self.ctx, parts.c_struct(), c, _stream()), "sph_density",
                                          allow)
        return out

    @staticmethod
    def force_buffers(n, dev):
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("ax", "ay", "az", "dudt", "dt")}
        out["n_pairs"] = torch.empty(n, dtype=torch.int32, device=dev)
        return out

    def force(self, parts: Particles, out=None):
        if out is None:
            out = self.force_buffers(parts.n, parts.x.device)
        c = sph_force_out(*[_ptr(out.get(k)) for k in FORCE_FIELDS])
        _check(sph_force(self.ctx, parts.c_struct(), c, _stream()), "sph_force")
        return out

    def step(self, parts: Particles, acc: dict, dt: float, batch: Optional[Batch] = None):
        """One kick-drift-kick step of fixed length dt; acc (a, du/dt, optionally dt) is updated."""
        c = sph_force_out(*[_ptr(acc.get(k)) for k in FORCE_FIELDS])
        return _check(sph_step(self.ctx, parts.c_struct(), batch.c if batch else None, c, dt, _stream()),
                      "sph_step", (SPH_E_NOT_CONVERGED,))

    def step_adaptive(self, parts: Particles, acc: dict, t_box: torch.Tensor, t_end: float, dt_max: float,
                      batch: Optional[Batch] = None, dt_box: Optional[torch.Tensor] = None):
        """One step whose length per box is the smallest time step of Eq. (6) in acc["dt"]
        (capped by dt_max, clipped at t_end); t_box (FP64, one per box) is advanced."""
        nbox = batch.nbox if batch else 1
        for t in (t_box, dt_box):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or t.numel() < nbox
                                  or not t.is_contiguous()):
                raise ValueError("t_box and dt_box must be contiguous float64 CUDA tensors of one value per box")
        if acc.get("dt") is None:
            raise ValueError("acc needs the time steps of the last force evaluation (key 'dt')")
        c = sph_force_out(*[_ptr(acc.get(k)) for k in FORCE_FIELDS])
        return _check(sph_step_adaptive(self.ctx, parts.c_struct(), batch.c if batch else None, c, dt_max, t_end,
                                        _ptr(t_box), _ptr(dt_box), _stream()),
                      "sph_step_adaptive", (SPH_E_NOT_CONVERGED,))

    def integrate(self, parts: Particles, t_end: float, dt_max: float, max_steps: int = 1 << 30,
                  batch: Optional[Batch] = None, acc: Optional[dict] = None):
        """Integrate from t = 0 to t_end with steps limited by Eq. (6); returns (acc, steps)."""
        if acc is None:
            acc = self.force_buffers(parts.n, parts.x.device)
        c = sph_force_out(*[_ptr(acc.get(k)) for k in FORCE_FIELDS])
        steps = ctypes.c_int64(0)
        _check(sph_integrate(self.ctx, parts.c_struct(), batch.c if batch else None, c, t_end, dt_max, max_steps,
                             ctypes.byref(steps), _stream()), "sph_integrate", (SPH_E_NOT_CONVERGED,))
        return acc, int(steps.value)

    def backward(self, parts: Particles, g_rho=None, g_a=None, g_dudt=None, implicit_h=True, want_h=False,
                 generation: int = 0):
        """Gradients of L at the state of the last density(): dL/dx as (N,3) and, if want_h
        (fixed h only), dL/dh.  g_a is (N,3) or None; missing upstream gradients count as 0.
        generation (from stats()) names the density evaluation meant; 0 takes the last one.
        Needs a context created with keep_adjoint=1."""
        n = parts.n
        dev = parts.x.device

        def col(t, k):
            return None if t is None else t[:, k].contiguous()

        keep = [_as_f64(g_rho), col(g_a, 0), col(g_a, 1), col(g_a, 2), _as_f64(g_dudt)]
        gin = sph_grad_in(*[_ptr(t) for t in keep])
        gx, gy, gz = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        gh = torch.empty(n, dtype=torch.float64, device=dev) if want_h else None
        gout = sph_grad_out(_ptr(gx), _ptr(gy), _ptr(gz), _ptr(gh))
        _check(sph_backward(self.ctx, parts.c_struct(), gin, gout, int(bool(implicit_h)), generation, _stream()),
               "sph_backward")
        gpos = torch.stack([gx, gy, gz], dim=1)
        return (gpos, gh) if want_h else gpos

    def enable_timing(self, on=True):
        _check(load_library().sph_enable_timing(self.ctx, int(on)), "sph_enable_timing")

    def kernel_times(self) -> dict:
        t = sph_kernel_times()
        _check(load_library().sph_get_kernel_times(self.ctx, ctypes.byref(t)), "sph_get_kernel_times")
        return {"build_ms": t.build_ms, "sort_ms": t.sort_ms, "density_ms": t.density_ms, "force_ms": t.force_ms,
                "backward_ms": t.backward_ms}

    def check(self, allow_unconverged=False):
        allow = (SPH_E_NOT_CONVERGED,) if allow_unconverged else ()
        return _check(sph_check(self.ctx, _stream()), "sph_check", allow)

    def graph_capture(self, parts: Particles, batch: Optional[Batch] = None, h_init: Optional[torch.Tensor] = None,
                      dout: Optional[dict] = None, fout: Optional[dict] = None):
        """Capture build -> sort -> density -> force (optionally preceded by h <- h_init) as one graph.

        The tensors passed here (particles, h_init, outputs) are kept by the graph: keep them alive.
        """
        n = parts.n
        dev = parts.x.device
        if fout is None:
            fout = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("ax", "ay", "az", "dudt")}
            fout["n_pairs"] = torch.empty(n, dtype=torch.int32, device=dev)
        dc = None
        if dout is not None:
            dc = sph_density_out(*[_ptr(dout.get(k)) for k in DENSITY_FIELDS])
        fc = sph_force_out(*[_ptr(fout.get(k)) for k in FORCE_FIELDS])
        self._graph_keep = (parts, batch, h_init, dout, fout, dc, fc)
        pc = parts.c_struct()
        self._graph_pc = pc
        _check(sph_graph_capture(self.ctx, pc, batch.c if batch else None, _ptr(h_init), dc, fc, _stream()),
               "sph_graph_capture", (SPH_E_NOT_CONVERGED,))
        return dout, fout

    def graph_launch(self):
        _check(sph_graph_launch(self.ctx, _stream()), "sph_graph_launch")

    def stats(self) -> dict:
        s = sph_stats()
        _check(load_library().sph_get_stats(self.ctx, ctypes.byref(s)), "sph_get_stats")
        return {"n_cells": s.n_cells, "n_units": s.n_units, "grid": tuple(s.grid), "rebuilds": s.rebuilds,
                "depth": s.depth, "refreshes": s.refreshes, "drift": s.drift, "generation": int(s.generation)}

    def run(self, parts: Particles, batch: Optional[Batch] = None, allow_unconverged=False):
        """build -> sort -> density (h solved in place) -> force."""
        self.build_cells(parts, batch)
        self.sort()
        d = self.density(parts, allow_unconverged=allow_unconverged)
        f = self.force(parts)
        return d, f


def pass_noalloc(parts: Particles, box=(1.0, 1.0, 1.0), precision: str = "fp32", dout: Optional[dict] = None,
                 fout: Optional[dict] = None, allow_unconverged=False, **kw):
    """build -> sort -> density (h solved in place) -> force through sph_pass_noalloc,
    which allocates no device memory: the library works in its fixed per-GPU array.
    The output tensors (dout, fout: dicts of DENSITY_FIELDS / FORCE_FIELDS keys)
    are the caller's; missing ones are made here, before the call."""
    p = sph_default_params()
    for d in range(3):
        p.box[d] = float(box[d])
    p.precision = SPH_FP64 if precision in ("fp64", SPH_FP64) else SPH_FP32_ACC64
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    n, dev = parts.n, parts.x.device
    if fout is None:
        fout = Context.force_buffers(n, dev)
    dc = None
    if dout is not None:
        dc = sph_density_out(*[_ptr(dout.get(k)) for k in DENSITY_FIELDS])
    fc = sph_force_out(*[_ptr(fout.get(k)) for k in FORCE_FIELDS])
    allow = (SPH_E_NOT_CONVERGED,) if allow_unconverged else ()
    _check(sph_pass_noalloc(p, parts.c_struct(), dc, fc, _stream()), "sph_pass_noalloc", allow)
    return dout, fout


def _parts_from(pos, vel, m, u, h):
    pos = pos.detach().to(torch.float64)
    vel = vel.detach().to(torch.float64)
    return Particles(x=pos[:, 0].contiguous(), y=pos[:, 1].contiguous(), z=pos[:, 2].contiguous(),
                     vx=vel[:, 0].contiguous(), vy=vel[:, 1].contiguous(), vz=vel[:, 2].contiguous(),
                     u=_as_f64(u.detach()), m=_as_f64(m.detach()), h=h.detach().to(torch.float64).clone())


def _forward_on(context: "Context", parts: Particles, fctx, fixed: bool):
    p = context.params
    if not p.keep_adjoint:
        raise ValueError("the context must be created with keep_adjoint=1 to be differentiated")
    if bool(p.fixed_h) != fixed:
        raise ValueError("SPHPassFixedH needs a context with fixed_h=1, SPHPass one with fixed_h=0")
    d, f = context.run(parts)
    fctx.context = context
    fctx.parts = parts
    fctx.generation = context.stats()["generation"]
    return d, f


class SPHPass(torch.autograd.Function):
    """rho, a (N,3) and du/dt of one pass as a differentiable function of the
    positions pos (N,3), with h the solved root of Eq. (3) (its dependence on
    the positions enters through the implicit derivative).

    SPHPass.apply(pos, vel, m, u, h0, context) runs build, sort, density (h
    solved from the guess h0) and force through ``context`` (created with
    keep_adjoint=1, fixed_h=0); backward calls sph_backward on the density
    evaluation of this forward, and fails (SPH_E_STATE) if another forward
    pass has run on the context since.  The solved h is left in
    context.last_h.  Velocities, masses and u are treated as constants.
    """

    @staticmethod
    def forward(fctx, pos, vel, m, u, h0, context: "Context"):
        parts = _parts_from(pos, vel, m, u, h0)
        d, f = _forward_on(context, parts, fctx, fixed=False)
        context.last_h = parts.h
        a = torch.stack([f["ax"], f["ay"], f["az"]], dim=1)
        return d["rho"], a, f["dudt"]

    @staticmethod
    def backward(fctx, g_rho, g_a, g_dudt):
        gpos = fctx.context.backward(fctx.parts, g_rho, g_a, g_dudt, implicit_h=True, generation=fctx.generation)
        return gpos, None, None, None, None, None


class SPHPassFixedH(torch.autograd.Function):
    """rho, a (N,3) and du/dt of one pass as a differentiable function of the
    positions pos (N,3) and of the smoothing lengths h (N,), both independent
    inputs: the sums of Eqs. (2)-(5) at the given h, without the iteration of
    Eq. (3) (so N_i need not equal n_ngb).

    SPHPassFixedH.apply(pos, h, vel, m, u, context) runs build, sort, density
    and force through ``context`` (created with fixed_h=1, keep_adjoint=1);
    backward returns dL/dpos and dL/dh from sph_backward with implicit_h = 0
    on the density evaluation of this forward.  Velocities, masses and u are
    treated as constants.
    """

    @staticmethod
    def forward(fctx, pos, h, vel, m, u, context: "Context"):
        parts = _parts_from(pos, vel, m, u, h)
        d, f = _forward_on(context, parts, fctx, fixed=True)
        a = torch.stack([f["ax"], f["ay"], f["az"]], dim=1)
        return d["rho"], a, f["dudt"]

    @staticmethod
    def backward(fctx, g_rho, g_a, g_dudt):
        gpos, gh = fctx.context.backward(fctx.parts, g_rho, g_a, g_dudt, implicit_h=False, want_h=True,
                                         generation=fctx.generation)
        return gpos, gh, None, None, None, None
