"""The C loop form of the oracle's product (oracle/nesa_c.c) against the NumPy
oracle: near-field blocks entry by entry (Sec. 2, Eq. 3) and the whole NESA
product (Sec. 3, Eq. 9-14) on trees of one, two and three levels."""
import numpy as np
import pytest

import synth
from oracle import nesa, nesa_c


@pytest.fixture(scope="module")
def sphere_two_levels(sphere1):
    return nesa.NesaOracle(*sphere1, leaf=0.125, d0=3, tau=1e-8)


def test_near_blocks_match_numpy_oracle(sphere_two_levels):
    ref = sphere_two_levels
    c = nesa_c.NesaC(ref, threads=4)
    t = ref.t
    sizes = np.array([len(r) for r in t.leaf_rwgs])
    widths = [sizes[np.asarray(x)].sum() for x in t.near]
    zoff = np.concatenate([[0], np.cumsum(sizes * widths)])
    for a in (0, 17, 100, len(sizes) - 1):
        rows, cols, Z = ref.near_block(a)
        Zc = c.Z[zoff[a]:zoff[a + 1]].reshape(len(cols), len(rows)).T
        assert np.abs(Zc - Z).max() <= 1e-12 * np.abs(Z).max()


@pytest.mark.parametrize("leaf", [0.25, 0.125])
def test_product_matches_numpy_oracle(sphere1, sphere_two_levels, leaf):
    ref = sphere_two_levels if leaf == 0.125 else nesa.NesaOracle(*sphere1, leaf=leaf, d0=3, tau=1e-8)
    c = nesa_c.NesaC(ref, threads=4)
    x = synth.complex_normal(ref.m.n, 3)
    y = ref.matvec(x)
    yc = c.matvec(x)
    assert np.linalg.norm(yc - y) <= 1e-12 * np.linalg.norm(y)
    # thread count does not change the result (owner-computes sums)
    nesa_c.set_threads(1)
    y1 = c.matvec(x)
    nesa_c.set_threads(4)
    assert np.array_equal(y1, yc)


def test_three_levels_rows():
    v, t = synth.icosphere(20, 1.0)
    ref = nesa.NesaOracle(v, t, leaf=0.125, d0=3, tau=1e-8)
    assert len(ref.levels) == 3
    c = nesa_c.NesaC(ref, threads=8)
    x = synth.complex_normal(ref.m.n, 4)
    rows = np.sort(np.random.default_rng(2).choice(ref.m.n, 40, replace=False))
    yr = ref.matvec_rows(x, rows)
    assert np.linalg.norm(c.matvec(x)[rows] - yr) <= 1e-12 * np.linalg.norm(yr)
