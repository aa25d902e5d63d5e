"""Seeded synthetic graph pairs for FRAM (inputs only).

This module draws the random graph pairs that both the FP64 oracle and the
GPU path are fed.  It holds none of FRAM's arithmetic: it only samples
adjacency matrices, hidden permutations and noise, so that the oracle and
the HIP path can share inputs without sharing any step of the method.
"""
from .graphs import (  # noqa: F401
    GraphPair,
    AttributedPair,
    make_attributed_pair,
    er_adjacency,
    permuted_noisy_copy,
    make_pair,
    config_pairs,
    config_sizes,
    batched_pairs,
    serve_requests,
    CONFIGS,
)
