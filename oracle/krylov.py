"""Restarted GMRES and flexible GMRES (plain FP64 reference).

The paper names GMRES as the iterative solver around the matrix-vector
product (Sec. 2) without details; this is the textbook method (Saad & Schultz
1986; flexible variant Saad 1993): Arnoldi with modified Gram-Schmidt, complex
Givens rotations on the Hessenberg matrix, restart after m steps, x0 = 0 by
default, stop when the relative residual ||b - A x|| / ||b|| <= tol, which is
confirmed on the true residual at every restart.
"""
import numpy as np


def _givens(a, b):
    """c (real), s (complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    rho = np.hypot(abs(a), abs(b))
    c = abs(a) / rho
    s = a * np.conj(b) / (abs(a) * rho)
    return c, s, a * rho / abs(a)


def gmres(A, b, m=30, tol=1e-6, max_iters=1000, x0=None, M=None):
    """Solve A x = b.  A and the optional right preconditioner M are callables.
    With M given this is flexible GMRES (the preconditioned vectors are kept).
    Returns (x, info) with info = {iters, history (estimated relative residuals),
    true_rel_residual, converged}."""
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    iters = 0
    if nb == 0:
        return x, {"iters": 0, "history": [0.0], "true_rel_residual": 0.0, "converged": True}
    r = b - A(x) if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    hist.append(beta / nb)
    while beta / nb > tol and iters < max_iters:
        V = [r / beta]
        Zs = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            z = M(V[j]) if M is not None else V[j]
            Zs.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t0 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t0
            c, s, rr = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            iters += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= tol or iters >= max_iters:
                break
            hn = np.linalg.norm(w)
            if hn == 0:
                break
            V.append(w / hn)
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * Zs[i]
        r = b - A(x)
        beta = np.linalg.norm(r)
    true_rel = float(np.linalg.norm(b - A(x)) / nb)
    return x, {"iters": iters, "history": hist, "true_rel_residual": true_rel,
               "converged": true_rel <= tol}


def block_diagonal(blocks):
    """Near-field block-diagonal preconditioner: z_a = Z_aa^{-1} r_a for every leaf.
    blocks: list of (rows, Z_aa).  Returns a callable."""
    inv = [(rows, np.linalg.inv(Zaa)) for rows, Zaa in blocks]

    def apply(r):
        z = np.zeros_like(r)
        for rows, Ai in inv:
            z[rows] = Ai @ r[rows]
        return z
    return apply


def near_schwarz_rows(a, leaf_rwgs, near, near_block, is_near):
    """Leaf a's part of the restricted additive Schwarz preconditioner (see
    near_schwarz): (RWGs of a, RWGs of N(a) in near-list order, the rows of
    Z_N^-1 that belong to a)."""
    nb = near[a]
    cols = np.concatenate([leaf_rwgs[b] for b in nb])
    off = np.cumsum([0] + [len(leaf_rwgs[b]) for b in nb])
    ZN = np.zeros((len(cols), len(cols)), dtype=np.complex128)
    for i, b in enumerate(nb):
        rows_b, cols_b, Zb = near_block(b)
        pos = {c: j for j, c in enumerate(cols_b)}
        for j, c in enumerate(nb):
            if is_near(b, c):
                idx = [pos[x] for x in leaf_rwgs[c]]
                ZN[off[i]:off[i + 1], off[j]:off[j + 1]] = Zb[:, idx]
    Mi = np.linalg.inv(ZN)
    ia = nb.index(a)
    return leaf_rwgs[a], cols, Mi[off[ia]:off[ia + 1]]


def near_schwarz(leaf_rwgs, near, near_block, is_near):
    """Restricted additive Schwarz over the near lists: for leaf a, with N(a) its
    near leaves and Z_N the near-field matrix restricted to the RWGs of N(a)
    (blocks of leaf pairs that are not near each other are zero, as they are
    not part of the near-field matrix), z_a = [Z_N^-1 r_N]_a.
    leaf_rwgs[a]: RWGs of leaf a; near[a]: its near leaves; near_block(a) ->
    (rows, cols, Z rows of leaf a against the RWGs of near[a]); is_near(b, c)."""
    blocks = [near_schwarz_rows(a, leaf_rwgs, near, near_block, is_near) for a in range(len(leaf_rwgs))]

    def apply(r):
        z = np.zeros_like(r)
        for rw, cols, Ma in blocks:
            z[rw] = Ma @ r[cols]
        return z
    return apply
