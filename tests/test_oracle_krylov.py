"""Pins of the GMRES / FGMRES oracle against LAPACK and Krylov identities."""
import numpy as np

import synth
from oracle import krylov


def _system(n, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = synth.complex_normal(n, seed + 1)
    return A, b


def test_gmres_full_space_equals_lapack():
    A, b = _system(40, 0)
    x, info = krylov.gmres(lambda v: A @ v, b, m=40, tol=1e-14, max_iters=40)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_gmres_residual_monotone_and_restarts_converge():
    A, b = _system(200, 1)
    x, info = krylov.gmres(lambda v: A @ v, b, m=10, tol=1e-10, max_iters=500)
    h = np.array(info["history"])
    assert info["converged"] and info["true_rel_residual"] <= 1e-10
    # within a cycle the least-squares residual never increases
    assert (np.diff(h[1:11]) <= 1e-15).all()


def test_fgmres_identity_equals_gmres():
    A, b = _system(120, 2)
    x1, i1 = krylov.gmres(lambda v: A @ v, b, m=15, tol=1e-9)
    x2, i2 = krylov.gmres(lambda v: A @ v, b, m=15, tol=1e-9, M=lambda v: v.copy())
    assert i1["iters"] == i2["iters"]
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)


def test_block_diagonal_preconditioner_is_blockwise_inverse():
    rng = np.random.default_rng(3)
    sizes = [5, 9, 3]
    blocks, off = [], 0
    for s in sizes:
        B = np.eye(s) + 0.3 * (rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s)))
        blocks.append((np.arange(off, off + s), B))
        off += s
    M = krylov.block_diagonal(blocks)
    r = synth.complex_normal(off, 4)
    z = M(r)
    for rows, B in blocks:
        assert np.linalg.norm(B @ z[rows] - r[rows]) <= 1e-12 * np.linalg.norm(r[rows])
    # block-diagonal preconditioning makes a block-diagonal system converge in one step
    from scipy.linalg import block_diag
    A = block_diag(*[B for _, B in blocks])
    x, info = krylov.gmres(lambda v: A @ v, r, m=5, tol=1e-12, M=M)
    assert info["iters"] == 1
