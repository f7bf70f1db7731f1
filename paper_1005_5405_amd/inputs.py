"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Only random fields live here; nothing of the method is computed.

Fields are float64 numpy arrays of shape (ny, nx, nv) in the cell-major layout
of the library; callers cast them to float32 for the device.
"""
from __future__ import annotations

import numpy as np


def random_field(shape, seed: int, scale: float = 0.5, smooth: float = 0.5) -> np.ndarray:
    """A deviation field mixing a smooth spatial pattern with white noise."""
    rng = np.random.default_rng(seed)
    ny, nx, nv = shape
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    X, Y = np.meshgrid(x, y)
    amp = rng.standard_normal(nv)
    phase = rng.uniform(0, 2 * np.pi, size=nv)
    base = np.sin(2 * np.pi * X[..., None] + phase) * np.cos(2 * np.pi * Y[..., None]) * amp
    noise = rng.standard_normal(shape)
    return scale * (smooth * base + (1.0 - smooth) * noise)


def velocity_polynomial(v: np.ndarray, seed: int, scale: float = 0.3) -> np.ndarray:
    """Random low-order polynomial in the node velocities v (nv, 3): a smooth
    deviation in velocity space, the kind the collision step acts on."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(10) * scale
    vx, vy, vz = v[:, 0], v[:, 1], v[:, 2]
    return (c[0] + c[1] * vx + c[2] * vy + c[3] * vz + c[4] * vx * vy + c[5] * vx * vz + c[6] * vy * vz
            + c[7] * vx * vx + c[8] * vy * vy + c[9] * vz * vz)
