"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module only draws random inputs (address permutations and the serving request
table).  It holds none of the synchronization arithmetic and none of the workload
hashing; both sides consume its arrays as given.

Generators use numpy's PCG64 bit generator so that a seed names the same input on
every machine that runs the same numpy.
"""

from __future__ import annotations

import numpy as np

SEEDS = (42, 0xC0FFEE, 7)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed & 0xFFFFFFFF, stream]))


def permutation(T: int, seed: int) -> np.ndarray:
    """Seeded permutation of [0, T) used to scatter microbenchmark targets."""
    return _rng(seed, 1).permutation(T).astype(np.uint32)


def request_table(n: int, rate_per_s: float, seed: int, mu: float = 5.0, sigma: float = 1.5,
                  lmax: int = 65536, bytes_per_step: int = 4096) -> dict:
    """Serving workload: n requests arriving as a Poisson stream of the given rate.

    L[r]       hash-chain length, round(exp(mu + sigma * Z)) clipped to [1, lmax]
               (a lognormal with median exp(mu));
    t_arr[r]   arrival time in seconds from the start (exponential inter-arrivals);
    nbytes[r]  workspace the request holds while it runs, L[r] * bytes_per_step.
    """
    g = _rng(seed, 2)
    z = g.standard_normal(n)
    L = np.clip(np.rint(np.exp(mu + sigma * z)), 1, lmax).astype(np.uint32)
    gaps = g.exponential(1.0 / rate_per_s, n)
    t_arr = np.cumsum(gaps)
    nbytes = L.astype(np.uint64) * np.uint64(bytes_per_step)
    return {"L": L, "t_arr": t_arr, "nbytes": nbytes}
