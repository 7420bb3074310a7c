"""Learned per-leaf preconditioner correction (plain FP64 reference).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module.

The paper has nothing on preconditioning; this is the network the library
trains and applies inside flexible GMRES (Saad 1993), written out plainly:

* features of leaf a for a vector r (leaf a's RWGs in leaf order, S_a of them,
  padded to S = s_max) and the base preconditioner's output b = M_base r:
  u_a = [Re r_a, Im r_a] / ||r_a||  and  [Re b_a, Im b_a] / ||b_a||, each block
  of length S (zero padded; a block whose norm is zero is all zeros), so
  u_a has 4 S entries;
* network (weights shared by all leaves): h1 = relu(W1 u + c1),
  h2 = relu(W2 h1 + c2), y = W3 h2 + c3, W1 [H][4S], W2 [H][H], W3 [2S][H];
* correction of leaf a: ||b_a|| (y[0:S_a] + i y[S:S+S_a]); the preconditioned
  vector is z = M_base r + correction.  With W3 = 0 and c3 = 0 the network is
  the base preconditioner;
* training pairs (r, e) with A e = r (residuals and errors of the method's own
  solves); target of leaf a: t_a = [Re, Im of (e_a - b_a)] / ||b_a|| on the
  S_a valid entries; loss = mean over leaves with ||b_a|| > 0 of
  sum_valid (y - t)^2;
* Adam (Kingma & Ba 2015) with bias correction.

Parameter vector order (FP32 on the library side): W1, c1, W2, c2, W3, c3,
each row-major.
"""
import numpy as np


def shapes(S, H):
    return [(H, 4 * S), (H,), (H, H), (H,), (2 * S, H), (2 * S,)]


def n_params(S, H):
    return sum(int(np.prod(s)) for s in shapes(S, H))


def unpack(theta, S, H):
    out, o = [], 0
    for s in shapes(S, H):
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def features(r, b, leaf_ptr, S):
    """u [nleaf][4S] and the output scale ||b_a|| [nleaf] of one vector r
    (leaf order) with base output b."""
    nleaf = len(leaf_ptr) - 1
    u = np.zeros((nleaf, 4 * S))
    scale = np.zeros(nleaf)
    for a in range(nleaf):
        p0, p1 = leaf_ptr[a], leaf_ptr[a + 1]
        Sa = p1 - p0
        if Sa > S:
            raise ValueError("leaf larger than s_max")
        ra, ba = r[p0:p1], b[p0:p1]
        nr, nb = np.linalg.norm(ra), np.linalg.norm(ba)
        if nr > 0:
            u[a, 0:Sa] = ra.real / nr
            u[a, S:S + Sa] = ra.imag / nr
        if nb > 0:
            u[a, 2 * S:2 * S + Sa] = ba.real / nb
            u[a, 3 * S:3 * S + Sa] = ba.imag / nb
        scale[a] = nb
    return u, scale


def targets(e, b, leaf_ptr, S):
    """t [nleaf][2S], mask [nleaf][2S] (valid entries of leaves with ||b_a|| > 0)."""
    nleaf = len(leaf_ptr) - 1
    t = np.zeros((nleaf, 2 * S))
    mask = np.zeros((nleaf, 2 * S))
    for a in range(nleaf):
        p0, p1 = leaf_ptr[a], leaf_ptr[a + 1]
        Sa = p1 - p0
        nb = np.linalg.norm(b[p0:p1])
        if nb == 0:
            continue
        d = (e[p0:p1] - b[p0:p1]) / nb
        t[a, 0:Sa], t[a, S:S + Sa] = d.real, d.imag
        mask[a, 0:Sa] = mask[a, S:S + Sa] = 1.0
    return t, mask


def forward(theta, u, S, H):
    """(y, cache) for rows u [B][4S]."""
    W1, c1, W2, c2, W3, c3 = unpack(theta, S, H)
    p1 = u @ W1.T + c1
    h1 = np.maximum(p1, 0.0)
    p2 = h1 @ W2.T + c2
    h2 = np.maximum(p2, 0.0)
    y = h2 @ W3.T + c3
    return y, (u, p1, h1, p2, h2)


def loss_and_grad(theta, u, t, mask, S, H):
    """Loss (mean over rows with any valid entry of the masked squared error)
    and its gradient with respect to theta (backpropagation)."""
    W1, c1, W2, c2, W3, c3 = unpack(theta, S, H)
    y, (u, p1, h1, p2, h2) = forward(theta, u, S, H)
    nrow = max(1, int((mask.sum(axis=1) > 0).sum()))
    diff = (y - t) * mask
    loss = float((diff ** 2).sum() / nrow)
    dy = 2.0 * diff / nrow
    gW3 = dy.T @ h2
    gc3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dp2 = dh2 * (p2 > 0)
    gW2 = dp2.T @ h1
    gc2 = dp2.sum(axis=0)
    dh1 = dp2 @ W2
    dp1 = dh1 * (p1 > 0)
    gW1 = dp1.T @ u
    gc1 = dp1.sum(axis=0)
    return loss, pack([gW1, gc1, gW2, gc2, gW3, gc3])


def correction(theta, r, b, leaf_ptr, S, H):
    """Network correction of one vector (leaf order)."""
    u, scale = features(r, b, leaf_ptr, S)
    y, _ = forward(theta, u, S, H)
    c = np.zeros_like(r, dtype=np.complex128)
    for a in range(len(leaf_ptr) - 1):
        p0, p1 = leaf_ptr[a], leaf_ptr[a + 1]
        Sa = p1 - p0
        c[p0:p1] = scale[a] * (y[a, 0:Sa] + 1j * y[a, S:S + Sa])
    return c


def apply(theta, r, base, leaf_ptr, S, H):
    """z = M_base r + correction (leaf order); base is a callable."""
    b = base(r)
    return b + correction(theta, r, b, leaf_ptr, S, H)


class Adam:
    """Adam with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)
