"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and describes workload shapes.  It holds
none of the method's arithmetic (no phase, no kernel entries, no transforms), so
both the GPU path and the CPU oracle can consume what it produces without either
depending on the other.

Workload shapes follow the paper's numerical section: 1D problems with
N = n points (Example 1, section 6) and 2D problems with N = n^2 points
(Example 3, section 6).  Right-hand sides are complex with independent
standard-normal real and imaginary parts.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def gaussian_complex(shape, seed: int) -> np.ndarray:
    """Complex128 array with i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex128)


def uniform_indices(count: int, high: int, seed: int) -> np.ndarray:
    """Sorted distinct integers in [0, high), for sampled output checks."""
    rng = np.random.default_rng(seed)
    count = min(count, high)
    return np.sort(rng.choice(high, size=count, replace=False)).astype(np.int64)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic solve workload: problem shape, tolerance and batch."""
    name: str
    d: int            # dimension (1 or 2)
    n: int            # points per dimension; N = n**d
    phase: str        # "linear", "1d_ex1" or "2d_radon"
    c_div: float      # divisor of c(x) for the 1D phase
    eps: float        # requested tolerance
    nrhs: int         # right-hand sides per batch
    seed: int

    @property
    def N(self) -> int:
        return self.n ** self.d


# The paper's examples with the sizes used for parity and measurement.
WORKLOADS = {
    "1d_n256": Workload("1d_n256", 1, 256, "1d_ex1", 16.0, 1e-6, 1, 1000),
    "1d_n4096": Workload("1d_n4096", 1, 4096, "1d_ex1", 16.0, 1e-6, 64, 1001),
    "1d_n65536": Workload("1d_n65536", 1, 65536, "1d_ex1", 16.0, 1e-6, 64, 1001),
    "2d_n64": Workload("2d_n64", 2, 64, "2d_radon", 16.0, 1e-4, 16, 1002),
    "2d_n128": Workload("2d_n128", 2, 128, "2d_radon", 16.0, 1e-4, 256, 1003),
    "2d_n256": Workload("2d_n256", 2, 256, "2d_radon", 16.0, 1e-4, 256, 1003),
}


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


@dataclasses.dataclass(frozen=True)
class Request:
    """A solve request of the serving mix."""
    rid: int
    arrival: float
    d: int
    n: int
    phase: str
    eps: float
    nrhs: int
    seed: int


def serving_mix(count: int, rate: float, seed: int = 2000,
                sizes_1d=(1024, 2048, 4096, 8192, 16384, 32768, 65536),
                sizes_2d=(32, 64, 128, 256), max_rhs: int = 32,
                eps_choices=(1e-4, 1e-6)) -> list:
    """Seeded mix of 1D and 2D solve requests with Poisson arrivals."""
    rng = np.random.default_rng(seed)
    times = poisson_arrivals(rate, count, seed + 1)
    out = []
    for j in range(count):
        if rng.random() < 0.5:
            d, n, phase = 1, int(rng.choice(sizes_1d)), "1d_ex1"
        else:
            d, n, phase = 2, int(rng.choice(sizes_2d)), "2d_radon"
        eps = float(rng.choice(eps_choices))
        nrhs = int(rng.integers(1, max_rhs + 1))
        out.append(Request(j, float(times[j]), d, n, phase, eps, nrhs, 3000 + j))
    return out
