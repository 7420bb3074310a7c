"""Pins of the oracle's nested passes against the dense Galerkin matrix.

On a tree of one level no transfer runs, so these cases use trees of two and
three levels (leaf 0.125 wavelength on the 3000-unknown sphere, leaf 0.125 on
the 12 000-unknown sphere).  They pin the source transfer C of Sec. 3, Eq. (11),
and the potential transfer B = C^T of Eq. (13) against quantities fixed without
the oracle's own product:

* the whole product against the dense matrix (Sec. 2, Eq. 3), with the error
  falling as the number of equivalent sources grows (Sec. 5.1: accuracy is set
  by the number of equivalent sources per group);
* a far block of two leaves whose parents interact, U_a B D C V_b, against the
  dense block (Sec. 2, Eq. 4-7: the nested form of a far block);
* complex symmetry y^T (A x) = x^T (A y) of the two-level operator (the Galerkin
  EFIE matrix is symmetric; with U = V^T and B = C^T the NESA operator is too);
* the parent's equivalent sources C s reproduce, at points two and a half
  parent sides away, the field of the child's equivalent sources s (the
  equivalence condition the transfer matrices are built from, Sec. 2).

A wrong octant, an untransposed B or a dropped level each give errors of order
one in these checks (the wrong-octant case is exercised below).
"""
import numpy as np
import pytest

import synth
from oracle import efie, nesa

# frozen NESA truncation errors ||(Z_NESA - Z) x|| / ||Z x|| (x i.i.d. complex
# normal, seed 0), measured once with this oracle and rounded up:
# 3000-unknown sphere at leaf 0.125 (levels 2..3): 5.33e-3 (d0 = 3), 2.52e-3 (d0 = 5)
NESA_ERR_SPHERE1_LEAF125 = {3: 6e-3, 5: 3e-3}
# 12 000-unknown sphere, 48 seeded dense rows: leaf 0.125 (levels 2..4) 5.58e-3
# at d0 = 3; leaf 0.25 (levels 2..3) 4.64e-4 at d0 = 3
NESA_ERR_SPHERE12K_ROWS = {0.125: 7e-3, 0.25: 6e-4}


@pytest.fixture(scope="module")
def nested1(sphere1):
    return {d0: nesa.NesaOracle(*sphere1, leaf=0.125, d0=d0, tau=1e-8) for d0 in (1, 3, 5)}


def test_two_levels(nested1):
    for op in nested1.values():
        assert (op.t.l0, op.t.L) == (2, 3)
        assert sum(len(x) for x in op.t.il[2]) > 0 and sum(len(x) for x in op.t.il[3]) > 0


def test_two_level_error_vs_dense_falls_with_q(nested1, dense1):
    x = synth.complex_normal(dense1.shape[0], 0)
    yd = dense1 @ x
    err = {d0: np.linalg.norm(op.matvec(x) - yd) / np.linalg.norm(yd) for d0, op in nested1.items()}
    assert err[3] <= NESA_ERR_SPHERE1_LEAF125[3]
    assert err[5] <= NESA_ERR_SPHERE1_LEAF125[5]
    assert err[1] > err[3] > err[5]


def test_two_level_complex_symmetric(nested1):
    op = nested1[3]
    x = synth.complex_normal(op.m.n, 1)
    y = synth.complex_normal(op.m.n, 2)
    a, b = y @ op.matvec(x), x @ op.matvec(y)
    assert abs(a - b) <= 1e-12 * abs(a)


def _nested_far_blocks(op, leaves, wrong_octant=False):
    """Relative errors of U_a B D C V_b against the dense block, for every leaf b
    under a box of the interaction list of a's parent (level l0)."""
    t = op.t
    L, l0 = t.L, t.l0
    errs = []
    for a in leaves:
        P = t.parent[L][a]
        kP = t.boxes[l0][P]
        oa = op.octant(L, a)
        Ba = op.C(L, (7 - oa) if wrong_octant else oa).T          # potential transfer, Eq. (13)
        Va = op.V(a)
        for Bx in t.il[l0][P]:
            kB = t.boxes[l0][Bx]
            D = op.D(l0, (kP[0] - kB[0], kP[1] - kB[1], kP[2] - kB[2]))
            for b in np.nonzero(np.array([t.parent[L][i] for i in range(len(t.boxes[L]))]) == Bx)[0]:
                Cb = op.C(L, op.octant(L, b))                    # source transfer, Eq. (11)
                Vb = op.V(b)
                Zf = sum(op.w[c] * (Va[c].T @ Ba @ D @ Cb @ Vb[c]) for c in range(4))
                Zd = efie.z_block(op.m, t.leaf_rwgs[a], t.leaf_rwgs[b])
                errs.append(np.linalg.norm(Zf - Zd) / np.linalg.norm(Zd))
    return np.array(errs)


def test_nested_far_blocks_vs_dense(nested1):
    """Far blocks that go up one level (C), across (D) and down (B = C^T):
    medians 0.10 (d0 = 3) and 0.043 (d0 = 5) on these small leaves (the RWGs
    reach half a leaf beyond their box); a wrong child octant gives about 0.8."""
    leaves = (0, 40, 150)
    e3 = _nested_far_blocks(nested1[3], leaves)
    e5 = _nested_far_blocks(nested1[5], leaves)
    assert len(e5) > 100
    assert np.median(e5) < 0.06 and e5.max() < 0.2
    assert np.median(e5) < 0.6 * np.median(e3)
    bad = _nested_far_blocks(nested1[5], leaves[:1], wrong_octant=True)
    assert np.median(bad) > 0.4


def test_source_transfer_reproduces_child_field(nested1):
    """C = R_parent G(X_parent, E_child + delta): the parent's sources C s give
    the field of the child's sources s at points 2.5 parent sides from the
    parent centre (measured 0.7-2.1e-2 at d0 = 5), for every octant; the matrix
    of the opposite octant misses by about 0.7."""
    op = nested1[5]
    t = op.t
    L, l0 = t.L, t.l0
    rng = np.random.default_rng(0)
    pts = 2.5 * t.side(l0) * nesa.fibonacci_sphere(50)
    for oc in range(8):
        s = rng.standard_normal(op.Q[L]) + 1j * rng.standard_normal(op.Q[L])
        delta = np.array([(oc & 1) - 0.5, ((oc >> 1) & 1) - 0.5, ((oc >> 2) & 1) - 0.5]) * t.side(L)
        true = nesa.gmat(pts, op.E[L] + delta) @ s
        fit = nesa.gmat(pts, op.E[l0]) @ (op.C(L, oc) @ s)
        wrong = nesa.gmat(pts, op.E[l0]) @ (op.C(L, 7 - oc) @ s)
        assert np.linalg.norm(fit - true) <= 3e-2 * np.linalg.norm(true)
        assert np.linalg.norm(wrong - true) >= 0.4 * np.linalg.norm(true)


@pytest.mark.parametrize("leaf", [0.125, 0.25])
def test_sampled_rows_vs_dense_12k(leaf):
    """12 000-unknown sphere (radius 1): three levels at leaf 0.125, two at
    0.25; 48 seeded rows of the product against the same rows of the dense
    matrix times x."""
    v, t = synth.icosphere(20, 1.0)
    op = nesa.NesaOracle(v, t, leaf=leaf, d0=3, tau=1e-8)
    assert len(op.levels) == (3 if leaf == 0.125 else 2)
    rows = np.sort(np.random.default_rng(7).choice(op.m.n, 48, replace=False))
    x = synth.complex_normal(op.m.n, 0)
    yd = efie.z_block(op.m, rows, np.arange(op.m.n)) @ x
    err = np.linalg.norm(op.matvec_rows(x, rows) - yd) / np.linalg.norm(yd)
    assert err <= NESA_ERR_SPHERE12K_ROWS[leaf]
