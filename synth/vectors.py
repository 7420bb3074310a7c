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


def mlp_weights(s_max, hidden, seed=0, zero_last=True, bias_std=0.0):
    """Initial parameters of the per-leaf network with layer shapes
    [hidden][4 s_max], [hidden], [hidden][hidden], [hidden], [2 s_max][hidden],
    [2 s_max] (row-major, concatenated): weight matrices normal with standard
    deviation sqrt(2 / fan_in) (He et al. 2015), biases normal with bias_std,
    the last weight matrix and bias zero when zero_last.  Values are rounded to
    the nearest FP16 number and returned as float32."""
    rng = np.random.default_rng(seed)
    shapes = [(hidden, 4 * s_max), (hidden,), (hidden, hidden), (hidden,),
              (2 * s_max, hidden), (2 * s_max,)]
    parts = []
    for i, s in enumerate(shapes):
        if len(s) == 2:
            p = rng.standard_normal(s) * np.sqrt(2.0 / s[1])
        else:
            p = rng.standard_normal(s) * bias_std
        if zero_last and i >= 4:
            p = np.zeros(s)
        parts.append(p.ravel())
    return np.concatenate(parts).astype(np.float16).astype(np.float32)
