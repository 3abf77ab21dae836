"""splitmix64 stream and the seeded draws of the synthetic workloads.

splitmix64 is written from its published definition (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014; constants of
Vigna's public-domain reference version): the state advances by the golden
gamma 0x9E3779B97F4A7C15 and each output is the state passed through the
two xor-shift-multiply mixing rounds.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    """Sequential splitmix64 generator (64-bit unsigned outputs)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1): the top 53 bits scaled by 2**-53."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_pm1(self) -> float:
        """Uniform double in [-1, 1)."""
        return 2.0 * self.uniform() - 1.0


def fourier_coefficients(dim: int, seed: int, kmax: int = 4) -> np.ndarray:
    """Coefficients a[c, k, l(, m)] uniform in [-1, 1) for the velocity perturbation.

    Drawn in the loop order (c, k, l, m) with k, l, m = 1..kmax, from one
    splitmix64 stream seeded with ``seed``.  Shape (dim, kmax, kmax[, kmax]).
    """
    g = SplitMix64(seed)
    shape = (dim,) + (kmax,) * dim
    a = np.empty(int(np.prod(shape)), dtype=np.float64)
    for i in range(a.size):
        a[i] = g.uniform_pm1()
    return a.reshape(shape)


@dataclass(frozen=True)
class Request:
    """One independent system of the serving stream."""

    index: int
    nx: int
    ny: int
    levels: int
    mu_s: float
    u_peak: float
    seed: int
    arrival_s: float
    transient: bool = False


def serving_stream(n: int = 256, seed_base: int = 1000, arrival_seed: int = 4242,
                   rate_per_s: float = 100.0,
                   meshes=((32, 8, 2), (64, 16, 3), (128, 32, 4))) -> list:
    """The Poisson stream of independent 2D systems: sweep points (steady
    systems) and time steps (one Crank-Nicolson step).

    System i draws, from splitmix64(seed_base + i): the mesh uniformly from
    ``meshes`` (nx, ny, levels; coarsest 16x4), the solid shear modulus
    10**(4 + 2U) (log-uniform in [1e4, 1e6]), the inflow peak 0.05 + 0.25U
    and then the kind (a time step when U < 0.5); its state seed is
    seed_base + i.  Inter-arrival gaps are exponential with the given rate,
    from splitmix64(arrival_seed).
    """
    arr = SplitMix64(arrival_seed)
    t = 0.0
    out = []
    for i in range(n):
        g = SplitMix64(seed_base + i)
        mi = min(int(g.uniform() * len(meshes)), len(meshes) - 1)
        nx, ny, lv = meshes[mi]
        mu_s = 10.0 ** (4.0 + 2.0 * g.uniform())
        u_peak = 0.05 + 0.25 * g.uniform()
        transient = g.uniform() < 0.5
        gap = -math.log(1.0 - arr.uniform()) / rate_per_s
        t += gap
        out.append(Request(i, nx, ny, lv, mu_s, u_peak, seed_base + i, t, transient))
    return out
