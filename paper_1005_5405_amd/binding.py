"""ctypes binding of libboltz (include/boltz.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libboltz.so; this module
checks tensor shapes, dtypes and devices, passes raw device pointers and the
current HIP stream, and turns negative status codes into exceptions.  PyTorch
is used for device memory and streams only.  There is no fallback: if the
library is missing or was not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libboltz.so")

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BC_CAVITY, BC_PERIODIC = 0, 1
ALLOW_UNSTABLE, WITH_ADJOINT = 1, 2
CONTINUOUS_PAIRS = 4  # pair velocities from the continuous Maxwellian (Box-Muller), binned to cells
SEQUENTIAL_UPDATE = 8  # collision in place, sample after sample (Alg. 3); shared samples only
NO_CORRECTION = 1
STATUS_NOT_SPD, STATUS_NONFINITE = 1, 2


class BoltzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nv", ctypes.c_int32 * 3),
                ("vmax", ctypes.c_double * 3), ("delta", ctypes.c_double), ("eps", ctypes.c_double),
                ("cfl", ctypes.c_double), ("dt", ctypes.c_double), ("order", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("sample_group", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("cavity_id", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("mix16", ctypes.c_uint32), ("rv", ctypes.c_double), ("rx", ctypes.c_double),
                ("ry", ctypes.c_double)]


class _Walls(ctypes.Structure):
    _fields_ = [("lid_u", ctypes.c_double), ("tau_left", ctypes.c_double), ("tau_right", ctypes.c_double),
                ("tau_bottom", ctypes.c_double), ("tau_top", ctypes.c_double), ("tau_bottom_x", ctypes.c_void_p)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("collide_block", ctypes.c_int32), ("nodes", ctypes.c_int64),
                ("pair_cells", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("classes", ctypes.c_int32),
                ("stream_tile", ctypes.c_int32 * 2), ("reserved", ctypes.c_int32)]


class _BatchClass(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32 * 3), ("problems", ctypes.c_int32), ("cells", ctypes.c_int64),
                ("pair_cells", ctypes.c_int64), ("collide_block", ctypes.c_int32),
                ("pairs_per_lane", ctypes.c_int32), ("spread", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("cells_per_group", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("ncells", ctypes.c_int64), ("nv", ctypes.c_int64), ("dt", ctypes.c_double),
                ("K", ctypes.c_double), ("W", ctypes.c_double), ("qfac", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("collide_layout", ctypes.c_int32),
                ("collide_block", ctypes.c_int32), ("collide_lds_nodes", ctypes.c_int32),
                ("collide_per_cu", ctypes.c_int32)]


# LDS layouts of the collision kernel (boltz_info.collide_layout)
LAYOUTS = {0: "cas", 1: "fixed", 2: "split", 3: "hybrid", 4: "part", 5: "sequential"}


EXPORTS = ("boltz_create", "boltz_destroy", "boltz_query", "boltz_last_error", "boltz_stream",
           "boltz_collide", "boltz_moments", "boltz_step", "boltz_stream_adjoint", "boltz_collide_adjoint",
           "boltz_step_adjoint", "boltz_lid_shear_adjoint", "boltz_debug_pairs", "boltz_axis_thresholds",
           "boltz_read_status", "boltz_batch_create", "boltz_batch_destroy", "boltz_batch_query",
           "boltz_batch_last_error", "boltz_batch_offsets", "boltz_batch_problem", "boltz_batch_set_step",
           "boltz_batch_step", "boltz_batch_tune", "boltz_batch_set_block", "boltz_collide_noalloc",
           "boltz_batch_class_info", "boltz_batch_set_class", "boltz_batch_set_stream_tile")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libboltz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime (same soname as the system one); load it
    # first so that libboltz binds to the runtime that owns torch's device
    # memory and streams instead of mapping a second runtime.
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError("libboltz.so not found at %s: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950)" % path)
    L = ctypes.CDLL(path)
    P, V, I64, U32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32
    W = ctypes.POINTER(_Walls)
    L.boltz_create.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(P)]
    L.boltz_destroy.argtypes = [P]
    L.boltz_query.argtypes = [P, ctypes.POINTER(_Info)]
    L.boltz_last_error.argtypes = [P]
    L.boltz_last_error.restype = ctypes.c_char_p
    L.boltz_stream.argtypes = [P, V, V, W, V]
    L.boltz_collide.argtypes = [P, V, V, I64, U32, V, V]
    L.boltz_collide_noalloc.argtypes = [P, V, V, I64, U32, V, V]
    L.boltz_moments.argtypes = [P, V, W, V, V, V]
    L.boltz_step.argtypes = [P, V, V, W, I64, V]
    L.boltz_stream_adjoint.argtypes = [P, V, V, V, V, W, V]
    L.boltz_collide_adjoint.argtypes = [P, V, V, V, I64, U32, V]
    L.boltz_step_adjoint.argtypes = [P, V, V, V, V, W, I64, V]
    L.boltz_lid_shear_adjoint.argtypes = [P, V, W, ctypes.c_double, V, V, V]
    L.boltz_debug_pairs.argtypes = [P, I64, I64, I64, I64, V, V, V]
    L.boltz_axis_thresholds.argtypes = [P, ctypes.c_int, V]
    L.boltz_read_status.argtypes = [P, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, V]
    L.boltz_batch_create.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(P)]
    L.boltz_batch_destroy.argtypes = [P]
    L.boltz_batch_query.argtypes = [P, ctypes.POINTER(_BatchInfo)]
    L.boltz_batch_last_error.argtypes = [P]
    L.boltz_batch_last_error.restype = ctypes.c_char_p
    L.boltz_batch_offsets.argtypes = [P, V]
    L.boltz_batch_problem.argtypes = [P, ctypes.c_int]
    L.boltz_batch_set_step.argtypes = [P, I64, V]
    L.boltz_batch_step.argtypes = [P, V, V, W, V]
    L.boltz_batch_tune.argtypes = [P, V, V, W, ctypes.c_int, V, V]
    L.boltz_batch_set_block.argtypes = [P, ctypes.c_int]
    L.boltz_batch_class_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(_BatchClass)]
    L.boltz_batch_set_class.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.boltz_batch_set_stream_tile.argtypes = [P, ctypes.c_int, ctypes.c_int]
    for name in EXPORTS:
        if name not in ("boltz_last_error", "boltz_destroy", "boltz_batch_last_error", "boltz_batch_destroy",
                        "boltz_batch_problem"):
            getattr(L, name).restype = ctypes.c_int
    L.boltz_destroy.restype = None
    L.boltz_batch_destroy.restype = None
    L.boltz_batch_problem.restype = ctypes.c_void_p
    _lib = L
    return L


@dataclass
class Walls:
    """Wall state of one call: lid x velocity and wall temperatures T_w/T0;
    tau_bottom_x (None or nx values) gives every bottom face its own."""
    lid_u: float = 0.0
    tau_left: float = 1.0
    tau_right: float = 1.0
    tau_bottom: float = 1.0
    tau_top: float = 1.0
    tau_bottom_x: object = None

    def _c(self) -> _Walls:
        ptr = None
        if self.tau_bottom_x is not None:
            self._tbx = np.ascontiguousarray(self.tau_bottom_x, dtype=np.float64)
            ptr = self._tbx.ctypes.data
        return _Walls(self.lid_u, self.tau_left, self.tau_right, self.tau_bottom, self.tau_top, ptr)


# wall-parameter gradient entries (then one per bottom face)
GRAD_NAMES = ("lid_u", "tau_left", "tau_right", "tau_top")


def _ptr(t, numel, dtype, what, allow_none=False):
    import torch

    if t is None:
        if allow_none:
            return None
        raise ValueError("%s: tensor required" % what)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s: expected a CUDA (HIP) tensor" % what)
    if t.dtype != dtype:
        raise ValueError("%s: expected dtype %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s: expected a contiguous tensor of %d elements" % (what, numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _problem(nx, ny, nv, vmax, delta, eps, n_pairs, cfl=0.5, dt=0.0, order=2, bc=BC_CAVITY, sample_group=1,
             seed=1, cavity_id=0, flags=0, mix16=4, rv=0.0, rx=0.0, ry=0.0) -> _Problem:
    nv = tuple(int(x) for x in (nv if np.ndim(nv) else (nv, nv, nv)))
    vmax = tuple(float(x) for x in (vmax if np.ndim(vmax) else (vmax, vmax, vmax)))
    return _Problem(int(nx), int(ny), (ctypes.c_int32 * 3)(*nv), (ctypes.c_double * 3)(*vmax), float(delta),
                    float(eps), float(cfl), float(dt), int(order), int(bc), int(n_pairs), int(sample_group),
                    int(seed), int(cavity_id), int(flags), int(mix16), float(rv), float(rx), float(ry))


class Boltz:
    """One problem on the current HIP device (a boltz_ctx)."""

    def __init__(self, nx, ny, nv, vmax, delta, eps, n_pairs, cfl=0.5, dt=0.0, order=2, bc=BC_CAVITY,
                 sample_group=1, seed=1, cavity_id=0, flags=0, mix16=4, rv=0.0, rx=0.0, ry=0.0, _borrowed=None):
        L = load_library()
        if _borrowed is None:
            p = _problem(nx, ny, nv, vmax, delta, eps, n_pairs, cfl, dt, order, bc, sample_group, seed, cavity_id,
                         flags, mix16, rv, rx, ry)
            ctx = ctypes.c_void_p()
            rc = L.boltz_create(ctypes.byref(p), ctypes.byref(ctx))
            if rc != OK:
                raise BoltzError(rc, "boltz_create: " + L.boltz_last_error(None).decode())
            self._owned = True
        else:
            ctx = ctypes.c_void_p(_borrowed)
            self._owned = False
        self._ctx = ctx
        info = _Info()
        L.boltz_query(ctx, ctypes.byref(info))
        nv = tuple(int(x) for x in (nv if np.ndim(nv) else (nv, nv, nv)))
        self.nx, self.ny, self.nv3 = int(nx), int(ny), nv
        self.ncells, self.nv = int(info.ncells), int(info.nv)
        self.numel = self.ncells * self.nv
        self.shape = (self.ny, self.nx, self.nv)
        self.dt, self.K, self.W, self.qfac = info.dt, info.K, info.W, info.qfac
        self.device_bytes = int(info.device_bytes)
        self.collide_layout = LAYOUTS.get(int(info.collide_layout), str(info.collide_layout))
        self.collide_block = int(info.collide_block)
        self.collide_lds_nodes = int(info.collide_lds_nodes)
        self.collide_per_cu = int(info.collide_per_cu)
        self.n_pairs, self.order, self.bc, self.eps = int(n_pairs), int(order), int(bc), float(eps)
        self.mix16 = int(mix16)

    def close(self):
        if getattr(self, "_ctx", None) is not None and _lib is not None and getattr(self, "_owned", True):
            _lib.boltz_destroy(self._ctx)
        self._ctx = None

    def __del__(self):
        self.close()

    def _check(self, rc, what):
        if rc != OK:
            raise BoltzError(rc, "%s: %s" % (what, _lib.boltz_last_error(self._ctx).decode()))

    def _walls(self, walls):
        if walls is None:
            return None
        return ctypes.byref(walls._c())

    def empty(self, fill=None):
        import torch

        t = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        if fill is not None:
            t.fill_(fill)
        return t

    # ---- hot path
    def stream(self, h_in, h_out, walls=None, stream=None):
        import torch

        self._check(_lib.boltz_stream(self._ctx, _ptr(h_in, self.numel, torch.float32, "h_in"),
                                      _ptr(h_out, self.numel, torch.float32, "h_out"), self._walls(walls),
                                      _stream(stream)), "boltz_stream")

    def collide(self, h_s, h_out, step, correction=True, defect=None, stream=None):
        import torch

        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_collide(self._ctx, _ptr(h_s, self.numel, torch.float32, "h_s"),
                                       _ptr(h_out, self.numel, torch.float32, "h_out"), int(step), flags,
                                       _ptr(defect, self.ncells * 5, torch.float64, "defect", True),
                                       _stream(stream)), "boltz_collide")

    def collide_noalloc(self, h_s, h_out, step, correction=True, defect=None, stream=None):
        """boltz_collide with the shared-sample records in the library's
        static device scratch (no allocation; calls on one GPU must not
        overlap)."""
        import torch

        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_collide_noalloc(self._ctx, _ptr(h_s, self.numel, torch.float32, "h_s"),
                                               _ptr(h_out, self.numel, torch.float32, "h_out"), int(step), flags,
                                               _ptr(defect, self.ncells * 5, torch.float64, "defect", True),
                                               _stream(stream)), "boltz_collide_noalloc")

    def moments(self, h, mom, walls=None, lid_shear=None, stream=None):
        import torch

        self._check(_lib.boltz_moments(self._ctx, _ptr(h, self.numel, torch.float32, "h"), self._walls(walls),
                                       _ptr(mom, self.ncells * 11, torch.float64, "mom"),
                                       _ptr(lid_shear, 1, torch.float64, "lid_shear", True), _stream(stream)),
                    "boltz_moments")

    def step(self, h_in, h_out, walls, step, stream=None):
        import torch

        self._check(_lib.boltz_step(self._ctx, _ptr(h_in, self.numel, torch.float32, "h_in"),
                                    _ptr(h_out, self.numel, torch.float32, "h_out"), self._walls(walls), int(step),
                                    _stream(stream)), "boltz_step")

    # ---- reverse mode (adjoints FP64; grad_walls: None or 4 + nx FP64 values
    # that the calls add to, see GRAD_NAMES)
    def grad_size(self):
        return 4 + self.nx

    def empty_adjoint(self, fill=None):
        import torch

        t = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        if fill is not None:
            t.fill_(fill)
        return t

    def _grad(self, g):
        import torch

        return _ptr(g, self.grad_size(), torch.float64, "grad_walls", True)

    def stream_adjoint(self, h_in, lam_out, lam_in, grad_walls=None, walls=None, stream=None):
        import torch

        self._check(_lib.boltz_stream_adjoint(self._ctx, _ptr(h_in, self.numel, torch.float32, "h_in"),
                                              _ptr(lam_out, self.numel, torch.float64, "lam_out"),
                                              _ptr(lam_in, self.numel, torch.float64, "lam_in"),
                                              self._grad(grad_walls), self._walls(walls), _stream(stream)),
                    "boltz_stream_adjoint")

    def collide_adjoint(self, h_s, lam_out, lam_s, step, correction=True, stream=None):
        import torch

        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_collide_adjoint(self._ctx, _ptr(h_s, self.numel, torch.float32, "h_s"),
                                               _ptr(lam_out, self.numel, torch.float64, "lam_out"),
                                               _ptr(lam_s, self.numel, torch.float64, "lam_s"), int(step), flags,
                                               _stream(stream)), "boltz_collide_adjoint")

    def step_adjoint(self, h_in, lam_out, lam_in, grad_walls, walls, step, stream=None):
        import torch

        self._check(_lib.boltz_step_adjoint(self._ctx, _ptr(h_in, self.numel, torch.float32, "h_in"),
                                            _ptr(lam_out, self.numel, torch.float64, "lam_out"),
                                            _ptr(lam_in, self.numel, torch.float64, "lam_in"),
                                            self._grad(grad_walls), self._walls(walls), int(step), _stream(stream)),
                    "boltz_step_adjoint")

    def lid_shear_adjoint(self, h, walls, weight, lam, grad_walls=None, stream=None):
        import torch

        self._check(_lib.boltz_lid_shear_adjoint(self._ctx, _ptr(h, self.numel, torch.float32, "h"),
                                                 self._walls(walls), float(weight),
                                                 _ptr(lam, self.numel, torch.float64, "lam"),
                                                 self._grad(grad_walls), _stream(stream)),
                    "boltz_lid_shear_adjoint")

    # ---- test hooks
    def debug_pairs(self, cell, step, m0, count, words=False):
        idx = np.zeros((count, 4), dtype=np.int32)
        q = np.zeros(count)
        wd = np.zeros((count, 4), dtype=np.uint32) if words else None
        self._check(_lib.boltz_debug_pairs(self._ctx, int(cell), int(step), int(m0), int(count), idx.ctypes.data,
                                           q.ctypes.data, wd.ctypes.data if words else None), "boltz_debug_pairs")
        return (idx, q, wd) if words else (idx, q)

    def axis_thresholds(self, axis):
        out = np.zeros(max(self.nv3[axis] - 1, 1), dtype=np.uint64)
        self._check(_lib.boltz_axis_thresholds(self._ctx, int(axis), out.ctypes.data), "boltz_axis_thresholds")
        return out[: self.nv3[axis] - 1]

    def read_status(self, clear=True, stream=None):
        v = ctypes.c_uint32(0)
        self._check(_lib.boltz_read_status(self._ctx, ctypes.byref(v), 1 if clear else 0, _stream(stream)),
                    "boltz_read_status")
        return int(v.value)


class Batch:
    """Many problems advanced together (a boltz_batch): one launch per phase
    for the whole batch.  problems: list of keyword dicts as for Boltz.  The
    state of the batch is one FP32 tensor of ``nodes`` values; problem i
    occupies ``view(h, i)``."""

    def __init__(self, problems):
        L = load_library()
        n = len(problems)
        arr = (_Problem * n)(*[_problem(**p) for p in problems])
        b = ctypes.c_void_p()
        rc = L.boltz_batch_create(arr, n, ctypes.byref(b))
        if rc != OK:
            raise BoltzError(rc, "boltz_batch_create: " + L.boltz_batch_last_error(None).decode())
        self._b = b
        self.count = n
        self.offsets = np.zeros(n, dtype=np.int64)
        L.boltz_batch_offsets(b, self.offsets.ctypes.data)
        self.problems = [Boltz(**p, _borrowed=L.boltz_batch_problem(b, i)) for i, p in enumerate(problems)]
        self._refresh()

    def _refresh(self):
        info = _BatchInfo()
        _lib.boltz_batch_query(self._b, ctypes.byref(info))
        self.nodes, self.pair_cells = int(info.nodes), int(info.pair_cells)
        self.collide_block, self.device_bytes = int(info.collide_block), int(info.device_bytes)
        self.nclasses, self.stream_tile = int(info.classes), (int(info.stream_tile[0]), int(info.stream_tile[1]))

    def close(self):
        if getattr(self, "_b", None) is not None and _lib is not None:
            for p in self.problems:
                p._ctx = None
            _lib.boltz_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        self.close()

    def _check(self, rc, what):
        if rc != OK:
            raise BoltzError(rc, "%s: %s" % (what, _lib.boltz_batch_last_error(self._b).decode()))

    def empty(self, fill=None):
        import torch

        t = torch.empty(self.nodes, dtype=torch.float32, device="cuda")
        if fill is not None:
            t.fill_(fill)
        return t

    def view(self, h, i):
        p = self.problems[i]
        o = int(self.offsets[i])
        return h[o:o + p.numel].view(p.shape)

    def _walls(self, walls):
        if walls is None:
            return None
        if len(walls) != self.count:
            raise ValueError("Batch: one wall state per problem")
        arr = (_Walls * self.count)(*[(w if w is not None else Walls())._c() for w in walls])
        self._walls_keep = (walls, arr)
        return arr

    def set_step(self, step, stream=None):
        self._check(_lib.boltz_batch_set_step(self._b, int(step), _stream(stream)), "boltz_batch_set_step")

    def step(self, h_in, h_out, walls=None, stream=None):
        import torch

        self._check(_lib.boltz_batch_step(self._b, _ptr(h_in, self.nodes, torch.float32, "h_in"),
                                          _ptr(h_out, self.nodes, torch.float32, "h_out"), self._walls(walls),
                                          _stream(stream)), "boltz_batch_step")

    def tune(self, h_a, h_b, walls=None, steps=2, stream=None):
        """Tune the stream tile shape, then each class's collision settings
        (block size, records per lane, workgroup spread); returns
        {"before": ms, "after": ms} per whole step.  Overwrites h_a, h_b and
        advances the step counter."""
        import torch

        ms = np.zeros(2)
        self._check(_lib.boltz_batch_tune(self._b, _ptr(h_a, self.nodes, torch.float32, "h_a"),
                                          _ptr(h_b, self.nodes, torch.float32, "h_b"), self._walls(walls),
                                          int(steps), _stream(stream), ms.ctypes.data), "boltz_batch_tune")
        self._refresh()
        return {"before": float(ms[0]), "after": float(ms[1])}

    def set_block(self, block):
        self._check(_lib.boltz_batch_set_block(self._b, int(block)), "boltz_batch_set_block")
        self._refresh()

    def classes(self):
        """Settings of every class (problems with one velocity grid)."""
        out = []
        for k in range(self.nclasses):
            c = _BatchClass()
            self._check(_lib.boltz_batch_class_info(self._b, k, ctypes.byref(c)), "boltz_batch_class_info")
            out.append({"nv": tuple(int(x) for x in c.nv), "problems": int(c.problems), "cells": int(c.cells),
                        "pair_cells": int(c.pair_cells), "collide_block": int(c.collide_block),
                        "pairs_per_lane": int(c.pairs_per_lane), "spread": int(c.spread), "grid": int(c.grid),
                        "cells_per_group": int(c.cells_per_group), "ms": float(c.ms)})
        return out

    def set_class(self, index, block, pairs_per_lane=4, spread=0):
        self._check(_lib.boltz_batch_set_class(self._b, int(index), int(block), int(pairs_per_lane), int(spread)),
                    "boltz_batch_set_class")
        self._refresh()

    def set_stream_tile(self, tx, ty):
        self._check(_lib.boltz_batch_set_stream_tile(self._b, int(tx), int(ty)), "boltz_batch_set_stream_tile")
        self._refresh()
        self._refresh()
