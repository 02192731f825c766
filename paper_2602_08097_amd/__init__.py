"""MI355X-native RP-Tuning: RobustPrune sweeps over an existing graph and
GreedySearch, as hand-written HIP kernels for gfx950 behind the C-ABI in
include/rp.h.  This package holds the HIP sources (csrc/), their build step
(build.py) and the ctypes binding (rp.py)."""
from .rp import (Graph, Server, RPError, build_slow, knn_u8, knn_u8_sets, load_library,  # noqa: F401
                 LIB_PATH, EXPORTS)
