"""MI355X-native zero-copy graph traversal (EMOGI, arxiv 2006.06890).

BFS, SSSP, connected components and PageRank over a CSR graph whose edge list can stay
in pinned host memory and is read in place by the GPU, through the C ABI of
``libemogi.so`` (``include/emogi.h``).  See ``emogi.py`` for the binding.
"""
from .emogi import (  # noqa: F401
    EmogiError, Graph, PinnedArray, Stats, VARIANTS, INF, N_SCHED_PARAMS, lib, to_u32, to_u64,
    calibrate_link,
)
