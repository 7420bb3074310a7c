"""Seeded random vectors."""
import numpy as np


def complex_normal(shape, seed=0):
    """i.i.d. standard complex normal entries (E|z|^2 = 1), complex128."""
    rng = np.random.default_rng(seed)
    if isinstance(shape, int):
        shape = (shape,)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)
