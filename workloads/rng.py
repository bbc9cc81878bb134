"""Seeded random draws (NumPy PCG64) used as inputs by the oracle, tests and benchmark."""
from __future__ import annotations

import numpy as np


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def unit_directions(count: int, seed: int) -> np.ndarray:
    """``count`` directions uniform on the unit sphere: normalised N(0, I3) draws."""
    g = generator(seed)
    d = g.standard_normal((count, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_complex(shape, seed: int) -> np.ndarray:
    """complex128 array with independent standard normal real and imaginary parts."""
    g = generator(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)
