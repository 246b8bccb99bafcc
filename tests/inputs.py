"""Seeded synthetic inputs shared by the oracle pins and the GPU parity tests.

Only random numbers and array shapes live here: no part of the lattice method
(actions, updates, measurements) is computed in this module.
"""
import numpy as np


def random_links(L: int, T: int, seed: int) -> np.ndarray:
    """Uniform link angles in [-pi, pi), shape (T, L, L, L, 4) = theta[t][z][y][x][mu]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(T, L, L, L, 4))


def random_gauge(L: int, T: int, seed: int) -> np.ndarray:
    """Site angles phi[t][z][y][x] in [-pi, pi) for a random gauge transformation."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(T, L, L, L))


def random_sites(V: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, V, size=k)


def random_angles(k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=k)
