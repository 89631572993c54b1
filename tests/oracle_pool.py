"""Run the CPU oracle over many inputs in a pool of spawned processes
(test infrastructure: the workers import only the oracle and the input
generators, never the GPU library)."""
from __future__ import annotations

import multiprocessing as mp
import os

import oracle


def variant_probabilities(v):
    return oracle.variant_probabilities(v)


def workers() -> int:
    """The host share of one GPU machine (at most 16 processes)."""
    return max(1, min(16, os.cpu_count() or 1))


def pool_map(fn, items, chunksize: int = 1):
    """fn over items in spawned worker processes, one BLAS thread each (the
    workers inherit the environment at spawn), results in item order."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers()) as pool:
        return pool.map(fn, items, chunksize=chunksize)
