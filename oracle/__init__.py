"""Plain FP64 CPU oracle of the semi-regular Boltzmann step.

TEST INFRASTRUCTURE ONLY: this package checks the HIP library and is never
part of the product path.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It imports nothing from
the product package, and the product package imports nothing from it.

The C source (``boltz_ref.c``) follows the paper's statement of the method;
this module only builds it with gcc and marshals numpy arrays through ctypes.
Arrays are float64 of shape (ny, nx, nv), cell-major with the velocity index
j = (jx*ny_v + jy)*nz_v + jz fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "boltz_ref.c")
_SO = os.path.join(_HERE, "liboracle.so")

BC_CAVITY = 0
BC_PERIODIC = 1
ALLOW_UNSTABLE = 1
CONTINUOUS = 4  # pair velocities from the continuous Maxwellian (Box-Muller), binned to cells
SEQUENTIAL = 8  # collision updates h in place, sample after sample (Alg. 3)
NO_CORRECTION = 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP contraction off, OpenMP on)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nv", ctypes.c_int32 * 3),
                ("vmax", ctypes.c_double * 3), ("delta", ctypes.c_double), ("eps", ctypes.c_double),
                ("cfl", ctypes.c_double), ("dt", ctypes.c_double), ("order", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("sample_group", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("cavity_id", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("mix16", ctypes.c_uint32), ("rv", ctypes.c_double), ("rx", ctypes.c_double),
                ("ry", ctypes.c_double)]


class _Walls(ctypes.Structure):
    _fields_ = [("lid_u", ctypes.c_double), ("tau_left", ctypes.c_double),
                ("tau_right", ctypes.c_double), ("tau_bottom", ctypes.c_double),
                ("tau_top", ctypes.c_double), ("tau_bottom_x", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P, V, D, I64, U32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_uint32
        L.boltz_ref_create.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(P)]
        L.boltz_ref_destroy.argtypes = [P]
        L.boltz_ref_last_error.argtypes = [P]
        L.boltz_ref_last_error.restype = ctypes.c_char_p
        L.boltz_ref_info.argtypes = [P, V]
        L.boltz_ref_set_threads.argtypes = [ctypes.c_int]
        L.boltz_ref_get_threads.restype = ctypes.c_int
        L.boltz_ref_axis.argtypes = [P, ctypes.c_int, V, V, V]
        L.boltz_ref_axis_edges.argtypes = [P, ctypes.c_int, V]
        L.boltz_ref_cell_widths.argtypes = [P, ctypes.c_int, V]
        L.boltz_ref_axis_draw.argtypes = [P, ctypes.c_int, U32]
        L.boltz_ref_philox4x32_10.argtypes = [V, V, V]
        L.boltz_ref_cos_sin_2pi.argtypes = [D, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.boltz_ref_neg_ln.argtypes = [D]
        L.boltz_ref_neg_ln.restype = D
        L.boltz_ref_debug_pairs.argtypes = [P, I64, I64, I64, I64, V, V, V, V]
        L.boltz_ref_wall_density.argtypes = [P, V, ctypes.POINTER(_Walls), V]
        L.boltz_ref_stream.argtypes = [P, V, V, ctypes.POINTER(_Walls)]
        L.boltz_ref_collide.argtypes = [P, V, V, I64, U32, V, V]
        L.boltz_ref_collide_cells.argtypes = [P, V, V, I64, U32, V, I64]
        L.boltz_ref_moments.argtypes = [P, V, ctypes.POINTER(_Walls), V, V]
        L.boltz_ref_step.argtypes = [P, V, V, ctypes.POINTER(_Walls), I64]
        L.boltz_ref_stream_adjoint.argtypes = [P, V, V, V, V, ctypes.POINTER(_Walls)]
        L.boltz_ref_collide_adjoint.argtypes = [P, V, V, V, I64, U32]
        L.boltz_ref_step_adjoint.argtypes = [P, V, V, V, V, ctypes.POINTER(_Walls), I64]
        L.boltz_ref_lid_shear_adjoint.argtypes = [P, V, ctypes.POINTER(_Walls), D, V, V]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    _load().boltz_ref_set_threads(int(n))


def get_threads() -> int:
    return int(_load().boltz_ref_get_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().boltz_ref_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def neg_ln(u: float) -> float:
    """-ln u of the continuous sampler (u in (0, 1])."""
    return float(_load().boltz_ref_neg_ln(float(u)))


def cos_sin_2pi(u: float):
    c, s = ctypes.c_double(), ctypes.c_double()
    _load().boltz_ref_cos_sin_2pi(float(u), ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


@dataclass
class Walls:
    lid_u: float = 0.0
    tau_left: float = 1.0
    tau_right: float = 1.0
    tau_bottom: float = 1.0
    tau_top: float = 1.0
    tau_bottom_x: object = None   # None, or nx per-face temperatures of the bottom wall

    def _c(self) -> _Walls:
        ptr = None
        if self.tau_bottom_x is not None:
            self._tbx = np.ascontiguousarray(self.tau_bottom_x, dtype=np.float64)
            ptr = self._tbx.ctypes.data
        return _Walls(self.lid_u, self.tau_left, self.tau_right, self.tau_bottom, self.tau_top, ptr)


# entries of the wall-parameter gradient (then one per bottom face)
GRAD_NAMES = ("lid_u", "tau_left", "tau_right", "tau_top")


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != int(np.prod(shape)):
        raise ValueError("array of %d elements, expected shape %s" % (a.size, shape))
    return a


class Oracle:
    """One problem set-up of the oracle (FP64, host memory)."""

    def __init__(self, nx, ny, nv, vmax, delta, eps, n_pairs, cfl=0.5, dt=0.0, order=2,
                 bc=BC_CAVITY, sample_group=1, seed=1, cavity_id=0, flags=0, mix16=4, rv=0.0, rx=0.0, ry=0.0):
        L = _load()
        nv = tuple(int(x) for x in (nv if np.ndim(nv) else (nv, nv, nv)))
        vmax = tuple(float(x) for x in (vmax if np.ndim(vmax) else (vmax, vmax, vmax)))
        p = _Problem(int(nx), int(ny), (ctypes.c_int32 * 3)(*nv), (ctypes.c_double * 3)(*vmax),
                     float(delta), float(eps), float(cfl), float(dt), int(order), int(bc),
                     int(n_pairs), int(sample_group), int(seed), int(cavity_id), int(flags), int(mix16),
                     float(rv), float(rx), float(ry))
        ctx = ctypes.c_void_p()
        rc = L.boltz_ref_create(ctypes.byref(p), ctypes.byref(ctx))
        if rc != 0:
            raise ValueError("boltz_ref_create: %s (rc=%d)" % (L.boltz_ref_last_error(None).decode(), rc))
        self._ctx = ctx
        self.nx, self.ny, self.nv3 = int(nx), int(ny), nv
        self.nv = nv[0] * nv[1] * nv[2]
        self.shape = (self.ny, self.nx, self.nv)
        self.order, self.bc, self.eps = int(order), int(bc), float(eps)
        info = np.zeros(8)
        L.boltz_ref_info(ctx, info.ctypes.data)
        self.dt, self.K, self.W, self.qfac, self.dx, self.dy = (float(x) for x in info[:6])
        # spatial cell widths along x and y (Sec. 5.1 stretching, else 1/n)
        self.wx, self.wy = np.zeros(self.nx), np.zeros(self.ny)
        L.boltz_ref_cell_widths(ctx, 0, self.wx.ctypes.data)
        L.boltz_ref_cell_widths(ctx, 1, self.wy.ctypes.data)
        self.v = []
        self.omega = []
        self.thresholds = []
        self.edges = []
        for k in range(3):
            e = np.zeros(nv[k] + 1)
            L.boltz_ref_axis_edges(ctx, k, e.ctypes.data)
            self.edges.append(e)
            v = np.zeros(nv[k])
            om = np.zeros(nv[k])
            thr = np.zeros(max(nv[k] - 1, 1), dtype=np.uint64)
            L.boltz_ref_axis(ctx, k, v.ctypes.data, om.ctypes.data, thr.ctypes.data)
            self.v.append(v)
            self.omega.append(om)
            self.thresholds.append(thr[: nv[k] - 1])

    def __del__(self):
        if getattr(self, "_ctx", None) is not None and _lib is not None:
            _lib.boltz_ref_destroy(self._ctx)
            self._ctx = None

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError("%s failed: %s (rc=%d)" % (what, _lib.boltz_ref_last_error(self._ctx).decode(), rc))

    # --- velocity-grid helpers (views of the oracle's own tables) ---
    def node_velocities(self) -> np.ndarray:
        vx, vy, vz = np.meshgrid(*self.v, indexing="ij")
        return np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1)

    def node_weights(self) -> np.ndarray:
        ox, oy, oz = np.meshgrid(*self.omega, indexing="ij")
        return ((ox * oy) * oz).ravel()

    def axis_draw(self, axis: int, r: int) -> int:
        return int(_lib.boltz_ref_axis_draw(self._ctx, int(axis), int(r)))

    # --- method ---
    def wall_density(self, h, walls: Walls) -> np.ndarray:
        h = _f64(h, self.shape)
        nw = np.zeros(2 * (self.nx + self.ny))
        self._check(_lib.boltz_ref_wall_density(self._ctx, h.ctypes.data, ctypes.byref(walls._c()),
                                                nw.ctypes.data), "wall_density")
        return nw

    def stream(self, h, walls: Walls | None = None) -> np.ndarray:
        h = _f64(h, self.shape)
        out = np.empty(self.shape)
        w = ctypes.byref(walls._c()) if walls is not None else None
        self._check(_lib.boltz_ref_stream(self._ctx, h.ctypes.data, out.ctypes.data, w), "stream")
        return out

    def collide(self, h, step, correction=True, want_dN=False, want_defect=False):
        h = _f64(h, self.shape)
        out = np.empty(self.shape)
        dN = np.empty(self.shape) if want_dN else None
        defect = np.empty((self.ny, self.nx, 5)) if want_defect else None
        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_ref_collide(self._ctx, h.ctypes.data, out.ctypes.data, int(step), flags,
                                           dN.ctypes.data if want_dN else None,
                                           defect.ctypes.data if want_defect else None), "collide")
        if want_dN or want_defect:
            return out, dN, defect
        return out

    def collide_cells(self, h_cells, step, cells, correction=True):
        """Collision of the listed cells only: h_cells (count, nv) holds their
        post-stream values; returns their outputs (count, nv)."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        h = _f64(h_cells, (len(cells), self.nv))
        out = np.zeros((len(cells), self.nv))
        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_ref_collide_cells(self._ctx, h.ctypes.data, out.ctypes.data, int(step), flags,
                                                 cells.ctypes.data, len(cells)), "collide_cells")
        return out

    def moments(self, h, walls: Walls | None = None, lid_shear=False):
        h = _f64(h, self.shape)
        mom = np.empty((self.ny, self.nx, 11))
        D = np.zeros(1)
        w = ctypes.byref(walls._c()) if walls is not None else None
        self._check(_lib.boltz_ref_moments(self._ctx, h.ctypes.data, w, mom.ctypes.data,
                                           D.ctypes.data if lid_shear else None), "moments")
        return (mom, float(D[0])) if lid_shear else mom

    def step(self, h, walls: Walls | None, step: int) -> np.ndarray:
        h = _f64(h, self.shape)
        out = np.empty(self.shape)
        w = ctypes.byref(walls._c()) if walls is not None else None
        self._check(_lib.boltz_ref_step(self._ctx, h.ctypes.data, out.ctypes.data, w, int(step)), "step")
        return out

    # --- adjoint (reverse-mode derivatives of the functions above) ---
    def grad_size(self) -> int:
        return 4 + self.nx

    def stream_adjoint(self, h, lam_out, walls: Walls | None = None):
        """(lam_in, grad): the adjoint of stream at h applied to lam_out."""
        h = _f64(h, self.shape)
        lo = _f64(lam_out, self.shape)
        lam = np.empty(self.shape)
        grad = np.zeros(self.grad_size())
        w = ctypes.byref(walls._c()) if walls is not None else None
        self._check(_lib.boltz_ref_stream_adjoint(self._ctx, h.ctypes.data, lo.ctypes.data, lam.ctypes.data,
                                                  grad.ctypes.data, w), "stream_adjoint")
        return lam, grad

    def collide_adjoint(self, h_s, lam_out, step, correction=True):
        h = _f64(h_s, self.shape)
        lo = _f64(lam_out, self.shape)
        lam = np.empty(self.shape)
        flags = 0 if correction else NO_CORRECTION
        self._check(_lib.boltz_ref_collide_adjoint(self._ctx, h.ctypes.data, lo.ctypes.data, lam.ctypes.data,
                                                   int(step), flags), "collide_adjoint")
        return lam

    def step_adjoint(self, h, lam_out, walls: Walls | None, step: int):
        """(lam_in, grad) of one full step at h (forward recomputed)."""
        h = _f64(h, self.shape)
        lo = _f64(lam_out, self.shape)
        lam = np.empty(self.shape)
        grad = np.zeros(self.grad_size())
        w = ctypes.byref(walls._c()) if walls is not None else None
        self._check(_lib.boltz_ref_step_adjoint(self._ctx, h.ctypes.data, lo.ctypes.data, lam.ctypes.data,
                                                grad.ctypes.data, w, int(step)), "step_adjoint")
        return lam, grad

    def lid_shear_adjoint(self, h, walls: Walls, weight=1.0):
        """(dD/dh * weight, dD/dtheta * weight) of the lid shear D."""
        h = _f64(h, self.shape)
        lam = np.zeros(self.shape)
        grad = np.zeros(self.grad_size())
        self._check(_lib.boltz_ref_lid_shear_adjoint(self._ctx, h.ctypes.data, ctypes.byref(walls._c()),
                                                     float(weight), lam.ctypes.data, grad.ctypes.data),
                    "lid_shear_adjoint")
        return lam, grad

    def debug_pairs(self, cell, step, m0, count, words=False, velocities=False):
        """Pairs m0..m0+count-1 of (cell, step): idx (count, 4) = a, b, a*, b*
        (-1 for a discarded pair), q (count,), optionally the Philox words
        (count, 4) and the continuous velocities (count, 4, 3)."""
        idx = np.zeros((count, 4), dtype=np.int32)
        q = np.zeros(count)
        wd = np.zeros((count, 4), dtype=np.uint32) if words else None
        vel = np.zeros((count, 4, 3)) if velocities else None
        self._check(_lib.boltz_ref_debug_pairs(self._ctx, int(cell), int(step), int(m0), int(count),
                                               idx.ctypes.data, q.ctypes.data,
                                               wd.ctypes.data if words else None,
                                               vel.ctypes.data if velocities else None), "debug_pairs")
        out = [idx, q]
        if words:
            out.append(wd)
        if velocities:
            out.append(vel)
        return tuple(out)
