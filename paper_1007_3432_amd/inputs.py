"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU
reference.  This module draws random numbers only; it holds none of the
method's arithmetic.

Recipe (one numpy PCG64 stream per lattice, site-major order, spatial
coordinate 0 fastest, time slowest):
  1. sigma = rng.uniform(-pi, pi, V)   auxiliary field, i.i.d. uniform
  2. eta   = rng.standard_normal(V)    Gaussian source, phi = M^T eta
The HMC chains of the serving workload draw sigma from seed 1000 + chain and
eta of request k from seed (1000 + chain) * 2**32 + k.
"""
from __future__ import annotations

import math

import numpy as np

# Workload shapes: (d, nx, nt).
SHAPES = {
    "c0_d1_32x64": (1, 32, 64),
    "c1_d1_2048x512": (1, 2048, 512),
    "c2_d3_16x160": (3, 16, 160),
    "c3_d3_32x256": (3, 32, 256),
}
SERVE_SHAPES = [(1, 256, 128), (1, 1024, 256), (3, 8, 80), (3, 16, 160)]


def volume(d: int, nx: int, nt: int) -> int:
    return nx ** d * nt


def sigma_eta(d: int, nx: int, nt: int, seed: int = 0):
    """sigma then eta from one stream, both float64 of length nx^d * nt."""
    V = volume(d, nx, nt)
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(-math.pi, math.pi, V)
    eta = rng.standard_normal(V)
    return sigma, eta


def random_vector(V: int, seed: int) -> np.ndarray:
    """A standard-normal test vector (apply-kernel parity inputs)."""
    return np.random.default_rng(seed).standard_normal(V)


def chain_shape(chain: int):
    """Lattice shape of serving chain `chain`, uniform over SERVE_SHAPES."""
    rng = np.random.default_rng(1000 + chain)
    return SERVE_SHAPES[int(rng.integers(0, len(SERVE_SHAPES)))]


def chain_sigma(chain: int) -> np.ndarray:
    d, nx, nt = chain_shape(chain)
    rng = np.random.default_rng([1000 + chain, 1])
    return rng.uniform(-math.pi, math.pi, volume(d, nx, nt))


def chain_eta(chain: int, request: int) -> np.ndarray:
    d, nx, nt = chain_shape(chain)
    rng = np.random.default_rng((1000 + chain) * 2 ** 32 + request)
    return rng.standard_normal(volume(d, nx, nt))
