"""Seeded synthetic inputs for the heat solver's workloads.

This module holds no part of the solver's arithmetic: it only produces the
initial fields and request streams that both the GPU library and the CPU
oracle are fed.  Grid convention: n interior points per axis, x = (i+1)/(n+1),
arrays in [z][y][x] order (x fastest).

Workloads (section 1 of the paper sets the problem; the sizes below follow
the benchmark configurations):
  * ``sine_product``   -- u0 = sin(pi x) sin(pi y) sin(pi z), the initial value
    of the manufactured solution u = s(x) cos t at t = 0 (eq. (4)).
  * ``random_modes`` / ``modes_field`` -- smooth random data: a sum of 8 sine
    modes, wave numbers uniform in {1..8}^3, amplitudes N(0,1).
  * ``random_field``   -- N(0,1) white noise for kernel-level checks.
  * ``uneven_sizes``   -- grid sizes drawn uniformly from {31, 63, 127}.
  * ``serving_requests`` -- Poisson arrivals of heat solves with n from
    {31, 63, 127, 255, 511} weighted 8:4:2:1:1, nu ~ U[0.05, 0.2],
    dt ~ U[0.005, 0.05], 1..20 steps, per-request seeds for the data.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def coords(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def sine_mode(n: int, k=(1, 1, 1)) -> np.ndarray:
    x = coords(n)
    sx = np.sin(k[0] * np.pi * x)
    sy = np.sin(k[1] * np.pi * x)
    sz = np.sin(k[2] * np.pi * x)
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def sine_product(n: int) -> np.ndarray:
    return sine_mode(n, (1, 1, 1))


def random_modes(seed: int, nmodes: int = 8, kmax: int = 8):
    """List of (kx, ky, kz, amplitude); duplicates allowed (they add up)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, kmax + 1, size=(nmodes, 3))
    amps = rng.standard_normal(nmodes)
    return [(int(k[0]), int(k[1]), int(k[2]), float(a)) for k, a in zip(ks, amps)]


def modes_field(n: int, modes) -> np.ndarray:
    u = np.zeros((n, n, n))
    for kx, ky, kz, a in modes:
        u += a * sine_mode(n, (kx, ky, kz))
    return u


def random_smooth(n: int, seed: int) -> np.ndarray:
    return modes_field(n, random_modes(seed))


def random_field(n: int, seed: int, count: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if count is None else (count, n, n, n)
    return rng.standard_normal(shape)


def uneven_sizes(seed: int, count: int = 64, choices=(31, 63, 127)) -> list[int]:
    rng = np.random.default_rng(seed)
    return [int(choices[i]) for i in rng.integers(0, len(choices), size=count)]


@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the stream starts
    n: int
    nu: float
    dt: float
    nsteps: int
    seed: int           # seed of the initial data (random_smooth)


def serving_requests(seed: int, count: int, rate: float,
                     sizes=(31, 63, 127, 255, 511), weights=(8, 4, 2, 1, 1)) -> list[Request]:
    """Poisson stream: exponential inter-arrival times with mean 1/rate."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    w /= w.sum()
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=count, p=w)
    nus = rng.uniform(0.05, 0.2, size=count)
    dts = rng.uniform(0.005, 0.05, size=count)
    steps = rng.integers(1, 21, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [Request(i, float(t[i]), int(ns[i]), float(nus[i]), float(dts[i]), int(steps[i]),
                    int(seeds[i])) for i in range(count)]
