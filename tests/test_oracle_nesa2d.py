"""Pins of the 2D model-problem oracle (oracle/nesa2d.py) against what the
definition and the mathematics fix: closed-form kernel values, the dense
product, convergence in Q, symmetry of the NESA operator, the tree's partition
of all point pairs into near and far interactions, and the total charge of the
fitted equivalent charges."""
import numpy as np
import pytest

import synth
from oracle import nesa2d as o2


def test_kernel_closed_form():
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, np.e]])
    K = o2.dense_matrix(x)
    assert K[0, 1] == 0.0 and K[1, 0] == 0.0          # -log 1
    assert abs(K[0, 2] + 1.0) < 1e-15                  # -log e
    assert abs(K[1, 2] + 0.5 * np.log(1.0 + np.e ** 2)) < 1e-15
    assert np.all(np.diag(K) == 0.0)


@pytest.fixture(scope="module")
def curve():
    x = synth.smooth_curve(1500, 1)
    q = synth.real_normal(1500, 2)
    return x, q, o2.dense_matrix(x) @ q


def test_error_falls_with_q(curve):
    x, q, yd = curve
    errs = []
    for Q in (8, 16, 32, 64):
        y = o2.Nesa2D(x, 50, Q).matvec(q)
        errs.append(np.linalg.norm(y - yd) / np.linalg.norm(yd))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[1] < 1e-4 and errs[3] < 1e-10


def test_nesa_operator_is_symmetric():
    x = synth.smooth_curve(400, 3)
    op = o2.Nesa2D(x, 8, 12)
    assert op.t.L > op.t.l0 + 1                        # transfers are exercised
    A = np.stack([op.matvec(e) for e in np.eye(len(x))], axis=1)
    assert np.linalg.norm(A - A.T) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(A - o2.dense_matrix(x)) <= 1e-3 * np.linalg.norm(A)


def test_tree_partitions_all_pairs():
    """Every pair of finest-level groups is covered exactly once: near at the
    finest level, or far between their ancestors at exactly one level."""
    x = synth.smooth_curve(2000, 5)
    t = o2.Tree2D(x, 20)
    L, l0 = t.L, t.l0
    assert L >= l0 + 3
    nl = len(t.boxes[L])
    cover = np.zeros((nl, nl), dtype=int)
    for a in range(nl):
        for b in t.near[a]:
            cover[a, b] += 1
    anc = {L: list(range(nl))}
    for l in range(L - 1, l0 - 1, -1):
        anc[l] = [t.index[l][(t.boxes[L][a][0] >> (L - l), t.boxes[L][a][1] >> (L - l))] for a in range(nl)]
    for l in t.levels:
        far = [set(v) for v in t.il[l]]
        for a in range(nl):
            fa = far[anc[l][a]]
            for b in range(nl):
                if anc[l][b] in fa:
                    cover[a, b] += 1
    assert np.all(cover == 1)
    # near lists: at most 9 groups including self; far lists: at most 27 per group
    assert max(len(v) for v in t.near) <= 9
    assert max(len(v) for l in t.levels for v in t.il[l]) <= 27


def test_leaf_rule_and_coarsest_level():
    x = synth.smooth_curve(5000, 7)
    for P in (30, 100, 400):
        t = o2.Tree2D(x, P)
        occ = lambda l: len(x) / len(np.unique(t.cells(l), axis=0))
        assert occ(t.L) >= P > occ(t.L + 1)
        # four groups along the longest side at l0
        assert max(c[0] for c in t.boxes[t.l0]) == 3 and t.l0 == 2


def test_equivalent_charges_keep_total_charge():
    """Far from a group, its potential is -log r times its total charge; the
    fitted equivalent charges must reproduce it (one check circle of radius near
    1 could not)."""
    rng = np.random.default_rng(11)
    x = synth.smooth_curve(4000, 9)
    op = o2.Nesa2D(x, 50, 16)
    t, L = op.t, op.t.L
    for b in rng.choice(len(t.boxes[L]), 5, replace=False):
        pts = t.leaf_points[b]
        qq = rng.standard_normal(len(pts)) + 0.5
        s = op.V[b] @ qq
        assert abs(s.sum() - qq.sum()) <= 1e-6 * np.abs(qq).sum()
        c = t.center(L, t.boxes[L][b])
        far = c + o2.circle(40, 50.0 * t.side(L), 0.3)
        exact = o2.gmat(far, x[pts]) @ qq
        fit = o2.gmat(far, op.E[L] + c) @ s
        assert np.linalg.norm(fit - exact) <= 1e-6 * np.linalg.norm(exact)


def test_single_level_tree():
    """P above the points per coarsest group: the tree stops at l0, the far field
    is the translations of level l0 alone (no transfers), and the product still
    matches the dense one to the accuracy of Q."""
    x = synth.smooth_curve(400, 13)
    op = o2.Nesa2D(x, 1000, 32)
    assert op.t.L == op.t.l0 and sum(len(v) for v in op.t.il[op.t.l0]) > 0
    q = synth.real_normal(400, 14)
    yd = o2.dense_matrix(x) @ q
    assert np.linalg.norm(op.matvec(q) - yd) <= 1e-8 * np.linalg.norm(yd)
