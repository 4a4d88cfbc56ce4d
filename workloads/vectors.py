"""Seeded random vectors.

Lanczos initial vectors are "uniform random from seed": entries
U[0, 1) - 1/2 from numpy's PCG64 ``default_rng`` seeded with
(seed, stream), generated once on the host and handed to whichever side
consumes them.
"""
from __future__ import annotations

import numpy as np


def seeded_vector(n, seed, stream=0):
    """Length-n float64 vector with entries uniform in [-1/2, 1/2)."""
    return np.random.default_rng([int(seed), int(stream)]).random(int(n)) - 0.5


def init_vector(n, step, seed=0):
    """The Lanczos initial vector of DMRG step ``step`` (stream 1000 + step)."""
    return seeded_vector(n, seed, 1000 + int(step))
