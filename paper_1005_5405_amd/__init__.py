"""MI355X (gfx950) implementation of one time-split step of the semi-regular
Boltzmann solver of Frezzotti, Ghiroldi and Gibelli (arXiv:1005.5405).

The compute path is libboltz.so (hand-written HIP kernels behind the C ABI of
include/boltz.h); :mod:`.binding` marshals torch device tensors into it.
"""
from .binding import (BC_CAVITY, BC_PERIODIC, CONTINUOUS_PAIRS, GRAD_NAMES, SEQUENTIAL_UPDATE, WITH_ADJOINT, Batch, Boltz, BoltzError,  # noqa: F401
                      Walls, load_library)
from .config import CAVITY_16, CAVITY_64, CAVITY_200, CAVITY_PAPER, CAVITY_PAPER_LITERAL, PRESETS, Preset  # noqa: F401
