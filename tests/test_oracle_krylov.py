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


def test_near_schwarz_exact_when_blocks_decouple():
    """With a block-diagonal system whose near lists hold only the leaf itself,
    the Schwarz preconditioner is the exact inverse."""
    rng = np.random.default_rng(5)
    sizes = [4, 6, 5]
    leaf_rwgs, off = [], 0
    for s_ in sizes:
        leaf_rwgs.append(np.arange(off, off + s_))
        off += s_
    Z = np.zeros((off, off), dtype=complex)
    for rw in leaf_rwgs:
        Z[np.ix_(rw, rw)] = np.eye(len(rw)) * 2 + 0.3 * rng.standard_normal((len(rw), len(rw)))
    near = [[0], [1], [2]]
    M = krylov.near_schwarz(leaf_rwgs, near, lambda a: (leaf_rwgs[a], leaf_rwgs[a], Z[np.ix_(leaf_rwgs[a], leaf_rwgs[a])]),
                            lambda b, c: b == c)
    r = synth.complex_normal(off, 6)
    assert np.linalg.norm(Z @ M(r) - r) <= 1e-12 * np.linalg.norm(r)


def test_near_schwarz_chain_matches_restricted_inverse():
    """Three leaves in a chain, near lists = neighbours: z_a equals the rows of
    the inverse of the restricted near-field matrix, built here by hand."""
    rng = np.random.default_rng(7)
    leaf_rwgs = [np.arange(0, 3), np.arange(3, 7), np.arange(7, 9)]
    n = 9
    Z = np.eye(n) * 3 + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    near = [[0, 1], [0, 1, 2], [1, 2]]
    is_near = lambda b, c: abs(b - c) <= 1
    nb_fn = lambda a: (leaf_rwgs[a], np.concatenate([leaf_rwgs[b] for b in near[a]]),
                       Z[np.ix_(leaf_rwgs[a], np.concatenate([leaf_rwgs[b] for b in near[a]]))])
    M = krylov.near_schwarz(leaf_rwgs, near, nb_fn, is_near)
    r = synth.complex_normal(n, 8)
    z = M(r)
    # leaf 1: all three leaves, but leaves 0 and 2 are not near each other
    cols = np.arange(9)
    ZN = Z.copy()
    ZN[np.ix_(leaf_rwgs[0], leaf_rwgs[2])] = 0
    ZN[np.ix_(leaf_rwgs[2], leaf_rwgs[0])] = 0
    assert np.allclose(z[leaf_rwgs[1]], (np.linalg.inv(ZN) @ r)[leaf_rwgs[1]], atol=1e-12)
    cols0 = np.arange(7)
    assert np.allclose(z[leaf_rwgs[0]], (np.linalg.inv(Z[np.ix_(cols0, cols0)]) @ r[cols0])[leaf_rwgs[0]],
                       atol=1e-12)


def test_arnoldi_relation_of_the_gmres_basis():
    """A V_m = V_{m+1} H_m to round-off for the oracle's Arnoldi process (the
    Hessenberg matrix rebuilt from the same modified Gram-Schmidt steps)."""
    rng = np.random.default_rng(12)
    n, m = 40, 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V = [b / np.linalg.norm(b)]
    H = np.zeros((m + 1, m), dtype=complex)
    for j in range(m):
        w = A @ V[j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
    Vm, Vm1 = np.array(V[:m]).T, np.array(V).T
    assert np.linalg.norm(A @ Vm - Vm1 @ H) <= 1e-12 * np.linalg.norm(A) * np.sqrt(m)
    assert np.linalg.norm(Vm1.conj().T @ Vm1 - np.eye(m + 1)) <= 1e-12
    # the oracle's GMRES after m steps reaches the least-squares minimum over the
    # same Krylov space
    x, info = krylov.gmres(lambda v: A @ v, b, m=m, tol=1e-30, max_iters=m)
    e1 = np.zeros(m + 1, dtype=complex)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(H, e1, rcond=None)[0]
    assert np.linalg.norm(x - Vm @ y) <= 1e-10 * np.linalg.norm(x)
