"""Plain single-threaded CPU oracle for RP-Tuning and GreedySearch.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library: the C source (``rpo.c``) is compiled by gcc into
``librpo.so`` and called through ctypes; ``reach.py`` holds the
alpha-reachability meter (Definition 2.1) and the closed forms of Table 1.

Paper: "Prune, Don't Rebuild: Efficiently Tuning alpha-Reachable Graphs for
Nearest Neighbor Search" (arXiv 2602.08097).
"""
from .binding import (  # noqa: F401
    U8,
    F32,
    build,
    lib_path,
    sqdist,
    robust_prune,
    robust_prune_smat,
    prune_graph,
    search,
    groundtruth,
    recall_at_k,
)
