"""GPU parity of the 2D model problem (include/nesa2d.h) against the FP64
oracle (oracle/nesa2d.py): the same seeded points, the tree and group order,
the NESA product element by element at sizes the oracle runs in seconds, the
paper's full size (N = 100 000) at its (P, Q) settings, and the edge cases."""
import numpy as np
import pytest

import synth
from oracle import nesa2d as o2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def nesa():
    from paper_1801_03589_amd import nesa as n
    n.lib()
    return n


def _run(torch, op, q):
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    yd = torch.empty_like(qd)
    op.matvec(qd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("n,P,Q", [(3000, 50, 10), (3000, 50, 32), (2000, 12, 16), (1500, 400, 24)])
def test_tree_and_product_match_oracle(torch_dev, nesa, n, P, Q):
    x = synth.smooth_curve(n, 21)
    q = synth.real_normal(n, 22)
    ref = o2.Nesa2D(x, P, Q)
    t = ref.t
    op = nesa.Model2D(x, P, Q)
    info = op.info()
    assert (info["l0"], info["L"]) == (t.l0, t.L)
    assert info["n_box"] == [len(t.boxes[l]) for l in t.levels]
    assert info["n_far"] == [sum(len(v) for v in t.il[l]) for l in t.levels]
    assert np.array_equal(op.perm(), np.concatenate(t.leaf_points))
    y = _run(torch_dev, op, q)
    yr = ref.matvec(q)
    err = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print("n %d P %d Q %d levels %d..%d: rel err vs oracle %.2e" % (n, P, Q, t.l0, t.L, err))
    assert err <= 1e-10
    assert np.abs(y - yr).max() <= 1e-9 * np.abs(yr).max()
    # bitwise repeatable (no atomics)
    assert np.array_equal(y, _run(torch_dev, op, q))


def test_full_size_p50_q10_against_oracle(torch_dev, nesa):
    """N = 100 000 at (P, Q) = (50, 10): the whole vector against the oracle."""
    x = synth.smooth_curve(100000, 23)
    q = synth.real_normal(100000, 24)
    ref = o2.Nesa2D(x, 50, 10)
    op = nesa.Model2D(x, 50, 10)
    assert op.info()["L"] == ref.t.L
    y = _run(torch_dev, op, q)
    yr = ref.matvec(q)
    err = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print("N 100000 P 50 Q 10: %d levels, rel err vs oracle %.2e" % (ref.t.L - ref.t.l0 + 1, err))
    assert err <= 1e-10


@pytest.mark.parametrize("P", [300, 400])
def test_full_size_q100_sampled_rows_against_definition(torch_dev, nesa, P):
    """N = 100 000 at (P, Q) = (P, 100): sampled rows against the dense
    definition (the NESA error at Q = 100 is far below the tolerance)."""
    n = 100000
    x = synth.smooth_curve(n, 23)
    q = synth.real_normal(n, 24)
    op = nesa.Model2D(x, P, 100)
    y = _run(torch_dev, op, q)
    rows = np.random.default_rng(25).choice(n, 64, replace=False)
    d = np.hypot(x[rows, None, 0] - x[None, :, 0], x[rows, None, 1] - x[None, :, 1])
    d[np.arange(64), rows] = 1.0
    yr = (-np.log(d)) @ q
    err = np.linalg.norm(y[rows] - yr) / np.linalg.norm(yr)
    print("N 100000 P %d Q 100: levels %s, sampled rel err vs definition %.2e" % (P, op.info()["n_box"], err))
    assert err <= 1e-6


def test_edge_cases(torch_dev, nesa):
    # two points: one far pair at the coarsest level, no transfers
    x = np.array([[0.0, 0.0], [1.0, 0.5]])
    op = nesa.Model2D(x, 1, 32)
    y = _run(torch_dev, op, np.array([2.0, -3.0]))
    assert np.allclose(y, o2.Nesa2D(x, 1, 32).matvec(np.array([2.0, -3.0])), rtol=1e-10, atol=0)
    k = -np.log(np.hypot(1.0, 0.5))
    assert np.allclose(y, [k * -3.0, k * 2.0], rtol=1e-6, atol=0)
    # P = 1 runs to the deepest level (20) and still matches the oracle
    x = synth.smooth_curve(300, 26)
    q = synth.real_normal(300, 27)
    ref = o2.Nesa2D(x, 1, 12)
    op = nesa.Model2D(x, 1, 12)
    assert op.info()["L"] == ref.t.L
    yr = ref.matvec(q)
    assert np.linalg.norm(_run(torch_dev, op, q) - yr) <= 1e-10 * np.linalg.norm(yr)
    # zero charges give exactly zero
    assert not np.any(_run(torch_dev, op, np.zeros(300)))
    # invalid parameters are rejected
    for P, Q, tau in [(0, 10, 1e-12), (10, 1, 1e-12), (10, 129, 1e-12), (10, 10, 0.0)]:
        with pytest.raises(nesa.NesaError):
            nesa.Model2D(x, P, Q, tau)
    with pytest.raises(nesa.NesaError):
        nesa.Model2D(x[:1], 10, 10)
