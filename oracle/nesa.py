"""Plain NESA matrix-vector product (FP64 reference).

The operator follows Sec. 2, Eq. (4)-(7): a far block is approximated by a
receiving matrix U, translation D, radiation V and nested transfer matrices
B, C; near blocks are stored exactly.  The product applies the near-field
update and the five far-field stages of Sec. 3 in the paper's order:
near field Eq. (9), radiation Eq. (10), source transfer Eq. (11), translation
Eq. (12), potential transfer Eq. (13), reception Eq. (14).

The paper defers the construction of U, D, V, B, C to Li et al. (2014) and only
states that they come from equivalence conditions on fictitious surfaces around
the groups, with auxiliary sources on spheres in 3D.  Reading taken here:

* channels: the mixed-potential EFIE kernel splits into four scalar channels
  sharing g, densities f = (phi_x, phi_y, phi_z, div phi) with weights
  w = (-i eta k, -i eta k, -i eta k, +i eta / k);
* per level l: Q_l equivalent points on a sphere of complex radius
  r_e (1 + i eps) (complex source points; eps = 0.1) and 4 Q_l check points on
  the real radius r_c (Fibonacci spirals), the same for every box of the level
  (translated to the box centre).  The Green's function of a complex point
  uses the principal square root of sum_d (x_d - e_d)^2.  Monopoles on a real
  sphere cannot radiate the spherical modes n with j_n(k r_e) = 0, which spoils
  the fit of every box whose k r_e sits near such a zero; the complex radius
  keeps every mode strength j_n(k r_e (1 + i eps)) away from zero;
* Q_l = (ceil(kr + 1.8 d0^(2/3) (kr)^(1/3)) + 1)^2, r = (sqrt 3 / 2) a_l
  (excess-bandwidth count);
* r_e at the leaf level = 1.02 x the largest distance from a leaf centre to a
  quadrature point of its RWGs (a batch of bodies takes the largest over its
  bodies, re_leaf); r_e one level up = 1.02 x (child-centre offset
  + child r_e); r_c = a_l (midway between r_e and 2 a_l - r_e), raised to
  1.05 r_e where the mesh is too coarse for r_e < a_l / 1.05;
* fitting operator R_l = Tikhonov pseudo-inverse of G(X, E) with
  lambda = tau * sigma_max:  R = V diag(s/(s^2 + lambda^2)) U^H from the SVD;
* V^c_b = R_L G^c_src (field of each RWG channel density at the check points),
  C_{P,b} = R_{l-1} G(X_{l-1}, E_l + delta_octant),  D_ab = G(E_a, E_b);
* U^c_a = (V^c_a)^T and B_{a,P} = C_{P,a}^T (reciprocity of the symmetric
  kernel under Galerkin testing).
"""
import math

import numpy as np

from . import efie
from .tree import Octree



def weights(k=efie.K0, eta=efie.ETA0):
    """Channel weights of the mixed-potential split of Sec. 2, Eq. (1)/(3)."""
    return np.array([-1j * eta * k, -1j * eta * k, -1j * eta * k, 1j * eta / k])


def q_rule(a, d0, k=efie.K0):
    r = math.sqrt(3.0) / 2.0 * a
    kr = k * r
    p = math.ceil(kr + 1.8 * d0 ** (2.0 / 3.0) * kr ** (1.0 / 3.0)) + 1
    return p * p


def fibonacci_sphere(n):
    """n deterministic, nearly uniform unit vectors (golden-angle spiral)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rad = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rad * np.cos(phi), rad * np.sin(phi), z], axis=1)


def tikhonov_pinv(G, tau):
    U, s, Vh = np.linalg.svd(G, full_matrices=False)
    lam = tau * s[0]
    f = s / (s * s + lam * lam)
    return (Vh.conj().T * f[None, :]) @ U.conj().T


def gmat(A, B, k=efie.K0):
    """G[i, j] = g(R_ij), R_ij = sqrt(sum_d (A_id - B_jd)^2); the points may be
    complex (complex source points), then R is the principal square root."""
    d = A[:, None, :] - B[None, :, :]
    if np.iscomplexobj(d):
        R = np.sqrt((d * d).sum(axis=-1))
    else:
        R = np.linalg.norm(d, axis=-1)
    return efie.green(R, k)


def leaf_radius_of(m, t):
    """Leaf equivalent radius: 1.02 x the largest distance from a leaf centre to
    a quadrature point of the leaf's RWGs."""
    rmax = 0.0
    for b, rw in enumerate(t.leaf_rwgs):
        c = t.center(t.L, b)
        pts = m.qp[m.tri[rw].ravel()].reshape(-1, 3)
        rmax = max(rmax, float(np.linalg.norm(pts - c, axis=1).max()))
    return 1.02 * rmax


def leaf_radius(verts, tris, leaf=0.25):
    """Leaf equivalent radius a body needs (the largest over a batch is shared)."""
    m = efie.RWG(verts, tris)
    return leaf_radius_of(m, Octree(verts, m.midpoints(), leaf=leaf))


class NesaOracle:
    """NESA operator of a closed mesh, built from the mesh alone."""

    def __init__(self, verts, tris, leaf=0.25, d0=3, tau=1e-9, buffer=1,
                 k=efie.K0, eta=efie.ETA0, l0_max=2, eps=0.1, re_leaf=None):
        self.m = efie.RWG(verts, tris)
        self.k, self.eta, self.tau, self.d0 = k, eta, tau, d0
        self.w = weights(k, eta)
        self.t = Octree(verts, self.m.midpoints(), leaf=leaf, l0_max=l0_max, buffer=buffer)
        t = self.t
        self.levels = list(range(t.l0, t.L + 1))
        self.Q = {l: q_rule(t.side(l), d0, k) for l in self.levels}
        # radii
        self.re = {t.L: leaf_radius_of(self.m, t)}
        if re_leaf is not None:
            # a batch of bodies shares the spheres of a level: the leaf radius
            # is the largest any body of the batch needs
            if re_leaf < self.re[t.L]:
                raise ValueError("leaf equivalent radius smaller than this body needs")
            self.re[t.L] = float(re_leaf)
        for l in range(t.L - 1, t.l0 - 1, -1):
            self.re[l] = 1.02 * (math.sqrt(3.0) / 2.0 * t.side(l + 1) + self.re[l + 1])
        self.rc = {l: max(t.side(l), 1.05 * self.re[l]) for l in self.levels}
        for l in self.levels:
            if self.re[l] >= 1.5 * t.side(l):
                raise ValueError("equivalent sphere radius exceeds 1.5 box sides at level %d "
                                 "(mesh too coarse for this leaf size)" % l)
        self.eps = eps
        self.E = {l: self.re[l] * (1.0 + 1j * eps) * fibonacci_sphere(self.Q[l]) for l in self.levels}
        self.X = {l: self.rc[l] * fibonacci_sphere(4 * self.Q[l]) for l in self.levels}
        self.R = {l: tikhonov_pinv(gmat(self.X[l], self.E[l], k), tau) for l in self.levels}
        self._V = {}
        self._C = {}
        self._D = {}
        self._near = {}

    # ---------------------------------------------------------------- operators
    def V(self, b):
        """Radiation matrices of leaf b: [4, Q_L, S_b] (channels x, y, z, div)."""
        if b not in self._V:
            t, m = self.t, self.m
            c = t.center(t.L, b)
            Xp = c + self.X[t.L]
            rw = t.leaf_rwgs[b]
            Gs = np.zeros((4, len(Xp), len(rw)), dtype=np.complex128)
            for j, n in enumerate(rw):
                pts, w, ph, dv = m.values_at_quad(n)
                g = gmat(Xp, pts, self.k) * w[None, :]            # [M, 6]
                Gs[0:3, :, j] = (g @ ph).T
                Gs[3, :, j] = g @ dv
            self._V[b] = np.einsum("qm,cmn->cqn", self.R[t.L], Gs)
        return self._V[b]

    def C(self, l, octant):
        """Source transfer from a child at level l (octant) to its parent: Q_{l-1} x Q_l."""
        key = (l, octant)
        if key not in self._C:
            a = self.t.side(l)
            delta = np.array([(octant & 1) - 0.5, ((octant >> 1) & 1) - 0.5,
                              ((octant >> 2) & 1) - 0.5]) * a
            self._C[key] = self.R[l - 1] @ gmat(self.X[l - 1], self.E[l] + delta, self.k)
        return self._C[key]

    def D(self, l, offset):
        """Translation between boxes whose integer indices differ by offset (a - b)."""
        key = (l, tuple(offset))
        if key not in self._D:
            d = np.asarray(offset, dtype=np.float64) * self.t.side(l)
            self._D[key] = gmat(self.E[l] + d, self.E[l], self.k)
        return self._D[key]

    def near_block(self, a):
        """Exact Z rows of leaf a against the RWGs of its near list: (rows, cols, Z)."""
        if a not in self._near:
            t = self.t
            rows = t.leaf_rwgs[a]
            cols = np.concatenate([t.leaf_rwgs[b] for b in t.near[a]])
            self._near[a] = (rows, cols, efie.z_block(self.m, rows, cols, self.k, self.eta))
        return self._near[a]

    def octant(self, l, i):
        k = self.t.boxes[l][i]
        return (k[0] & 1) | ((k[1] & 1) << 1) | ((k[2] & 1) << 2)

    # ---------------------------------------------------------------- product
    def upward(self, x):
        """Radiation (Eq. 10) and source transfer (Eq. 11): s[l][box] of shape [4, Q_l]."""
        t = self.t
        s = {l: [np.zeros((4, self.Q[l]), dtype=np.complex128) for _ in t.boxes[l]]
             for l in self.levels}
        # a leaf (box) whose sources are all zero contributes exact zeros: it is
        # skipped, so a vector supported on a few leaves needs only their V
        live = set()
        for b, rw in enumerate(t.leaf_rwgs):
            if np.any(x[rw] != 0):
                s[t.L][b] = self.V(b) @ x[rw]
                live.add(b)
        for l in range(t.L, t.l0, -1):
            up = set()
            for b in sorted(live):
                p = t.parent[l][b]
                s[l - 1][p] = s[l - 1][p] + (self.C(l, self.octant(l, b)) @ s[l][b].T).T
                up.add(p)
            live = up
        return s

    def translate(self, s, l, a):
        """Translation (Eq. 12) into box a at level l."""
        t = self.t
        ka = t.boxes[l][a]
        o = np.zeros((4, self.Q[l]), dtype=np.complex128)
        for b in t.il[l][a]:
            if not np.any(s[l][b]):
                continue                 # zero sources contribute exact zeros
            kb = t.boxes[l][b]
            off = (ka[0] - kb[0], ka[1] - kb[1], ka[2] - kb[2])
            o += (self.D(l, off) @ s[l][b].T).T
        return o

    def matvec(self, x):
        """y = Z_NESA x for the full vector (canonical RWG order)."""
        t = self.t
        x = np.asarray(x, dtype=np.complex128)
        y = np.zeros(self.m.n, dtype=np.complex128)
        # near field (Eq. 9)
        for a in range(len(t.boxes[t.L])):
            rows, cols, Z = self.near_block(a)
            y[rows] += Z @ x[cols]
        s = self.upward(x)
        # translation (Eq. 12) at every level
        o = {l: [self.translate(s, l, a) for a in range(len(t.boxes[l]))] for l in self.levels}
        # potential transfer (Eq. 13), parents before children
        for l in range(t.l0 + 1, t.L + 1):
            for a in range(len(t.boxes[l])):
                p = t.parent[l][a]
                B = self.C(l, self.octant(l, a)).T
                o[l][a] = o[l][a] + (B @ o[l - 1][p].T).T
        # reception (Eq. 14) with the channel weights
        for a, rw in enumerate(t.leaf_rwgs):
            V = self.V(a)
            y[rw] += np.einsum("c,cqn,cq->n", self.w, V, o[t.L][a])
        return y

    def matvec_rows(self, x, rows):
        """y[rows] of Z_NESA x: full upward pass, translation and downward pass only
        along the ancestors of the leaves holding the requested rows."""
        t = self.t
        x = np.asarray(x, dtype=np.complex128)
        rows = np.asarray(rows)
        s = self.upward(x)
        out = np.zeros(len(rows), dtype=np.complex128)
        for a in sorted(set(t.rwg_leaf[rows].tolist())):
            # near rows of leaf a that were requested
            rw = t.leaf_rwgs[a]
            want = [i for i, r in enumerate(rows) if t.rwg_leaf[r] == a]
            rloc = np.array([int(np.nonzero(rw == rows[i])[0][0]) for i in want])
            cols = np.concatenate([t.leaf_rwgs[b] for b in t.near[a]])
            Zr = efie.z_block(self.m, rw[rloc], cols, self.k, self.eta)
            yv = Zr @ x[cols]
            # far field along the ancestor chain
            chain = [a]
            for l in range(t.L, t.l0, -1):
                chain.append(t.parent[l][chain[-1]])
            chain = chain[::-1]                      # level l0 .. L
            ov = self.translate(s, t.l0, chain[0])
            for i, l in enumerate(range(t.l0 + 1, t.L + 1)):
                B = self.C(l, self.octant(l, chain[i + 1])).T
                ov = self.translate(s, l, chain[i + 1]) + (B @ ov.T).T
            V = self.V(a)
            yf = np.einsum("c,cqn,cq->n", self.w, V[:, :, rloc], ov)
            for j, i in enumerate(want):
                out[i] = yv[j] + yf[j]
        return out
