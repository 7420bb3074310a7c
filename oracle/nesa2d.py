"""Plain 2D potential problem and its NESA product (FP64 reference, test
infrastructure).

The model problem (Sec. "The model problem", Eq. (pot)): N charges q_j at points
x_j on a curve in the plane; the potential at the same points is phi = K q with
k_ij = -log |x_i - x_j| for i != j and k_ii = 0.  `dense_matrix` writes that
definition out.

`Nesa2D` applies the NESA form of K in the paper's order: the near-field block
product (Eq. (algnf)) between neighbouring finest-level groups, then radiation
(Eq. (algrad)), source transfer (Eq. (algsou)), translation (Eq. (algtrans)),
potential transfer (Eq. (algpot)) and reception (Eq. (algrec)).

The tree follows the same section: the coarsest level l0 has 4 groups along the
longest side of the domain; groups are subdivided as long as the mean number of
points per finest-level group does not fall below P (read as: L is the deepest
level whose mean occupancy over non-empty groups is still >= P); near groups are
the group itself and its 8 neighbours; the far groups of a group at level l are
the groups that are not neighbours but whose parents are (at l0: every
non-neighbour).

The paper leaves the construction of the matrices to Li et al. (2014), naming
only equivalent charges on a circle per group and potentials matched on a test
circle.  Reading taken here (box side a_l at level l):
* Q equivalent points on a circle of radius 0.75 a_l around the box centre, at
  angles 2 pi (k + 1/2) / Q;
* 2Q check points on each of two circles, radius 1.05 a_l and 1.6 a_l, at angles
  2 pi k / (2Q).  One circle cannot fix the total charge of the fit when its
  radius is near 1 (the mean of -log over a circle of radius r is -log r for any
  source inside); two radii always do.  With only Q check points per circle the
  alternating pattern of equivalent charges would radiate a mode that vanishes
  at every check point (a null space of the fit);
* R_l = Tikhonov pseudo-inverse of G(X_l, E_l), lambda = tau * sigma_max, from
  the SVD (G = -log distance);
* V_b = R_L G(X_L + c_b, x_b), C_{P,b} = R_{l-1} G(X_{l-1}, E_l + delta_quadrant),
  D_ab = G(E_l + c_a, E_l + c_b);
* U_a = V_a^T and B_{a,P} = C_{P,a}^T (the kernel is symmetric).
"""
import numpy as np

R_EQ = 0.75      # equivalent circle radius / box side
R_CHK = (1.05, 1.6)   # check circle radii / box side


def dense_matrix(x):
    """K of Eq. (pot): k_ij = -log |x_i - x_j|, k_ii = 0."""
    d = np.hypot(x[:, None, 0] - x[None, :, 0], x[:, None, 1] - x[None, :, 1])
    np.fill_diagonal(d, 1.0)
    K = -np.log(d)
    np.fill_diagonal(K, 0.0)
    return K


def gmat(t, s):
    """-log |t_i - s_j| between two point sets (no coincident points)."""
    return -np.log(np.hypot(t[:, None, 0] - s[None, :, 0], t[:, None, 1] - s[None, :, 1]))


def tikhonov_pinv(G, tau):
    U, sv, Vh = np.linalg.svd(G, full_matrices=False)
    lam = tau * sv[0]
    return (Vh.T * (sv / (sv * sv + lam * lam))) @ U.T


class Tree2D:
    """Quadtree over the points (Sec. "The model problem")."""

    def __init__(self, x, P, l0=2, max_level=20):
        self.x = x
        lo = x.min(axis=0)
        ext = x.max(axis=0) - lo
        self.origin = lo
        self.root = float(max(ext[0], ext[1])) * (1.0 + 2.0 ** -20)
        self.l0 = l0
        # deepest level whose mean occupancy of non-empty boxes is >= P
        L = l0
        for l in range(l0 + 1, max_level + 1):
            n_nonempty = len(np.unique(self.cells(l), axis=0))
            if len(x) / n_nonempty >= P:
                L = l
            else:
                break
        self.L = L
        self.levels = list(range(l0, L + 1))
        # boxes: non-empty cells per level, sorted by (i, j)
        self.boxes = {}
        self.index = {}
        for l in self.levels:
            cells = np.unique(self.cells(l), axis=0)
            self.boxes[l] = [tuple(int(v) for v in c) for c in cells]
            self.index[l] = {c: k for k, c in enumerate(self.boxes[l])}
        leaf_of = self.cells(L)
        li = self.index[L]
        self.leaf_points = [[] for _ in self.boxes[L]]
        for p, c in enumerate(leaf_of):
            self.leaf_points[li[(int(c[0]), int(c[1]))]].append(p)
        self.leaf_points = [np.array(v, dtype=np.int64) for v in self.leaf_points]
        # near lists (leaf level) and interaction lists (every level)
        self.near = [self._neighbours(L, c) for c in self.boxes[L]]
        self.il = {}
        for l in self.levels:
            lst = []
            for c in self.boxes[l]:
                if l == l0:
                    cand = self.boxes[l]
                else:
                    cand = []
                    pc = (c[0] // 2, c[1] // 2)
                    for pb in self._neighbours(l - 1, pc):
                        pcell = self.boxes[l - 1][pb]
                        for di in (0, 1):
                            for dj in (0, 1):
                                cc = (2 * pcell[0] + di, 2 * pcell[1] + dj)
                                if cc in self.index[l]:
                                    cand.append(cc)
                lst.append([self.index[l][b] for b in cand
                            if max(abs(b[0] - c[0]), abs(b[1] - c[1])) >= 2])
            self.il[l] = lst

    def side(self, l):
        return self.root / 2 ** l

    def cells(self, l):
        a = self.side(l)
        c = np.floor((self.x - self.origin) / a).astype(np.int64)
        return np.clip(c, 0, 2 ** l - 1)

    def center(self, l, c):
        a = self.side(l)
        return self.origin + (np.array(c, dtype=np.float64) + 0.5) * a

    def _neighbours(self, l, c):
        out = []
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                b = (c[0] + di, c[1] + dj)
                if b in self.index[l]:
                    out.append(self.index[l][b])
        return sorted(out)


def circle(n, radius, phase):
    t = 2.0 * np.pi * (np.arange(n) + phase) / n
    return radius * np.stack([np.cos(t), np.sin(t)], axis=1)


class Nesa2D:
    """NESA product of the 2D potential operator (FP64)."""

    def __init__(self, x, P, Q, tau=1e-12):
        self.t = Tree2D(x, P)
        self.Q = Q
        t = self.t
        self.E = {l: circle(Q, R_EQ * t.side(l), 0.5) for l in t.levels}
        self.X = {l: np.concatenate([circle(2 * Q, r * t.side(l), 0.0) for r in R_CHK]) for l in t.levels}
        self.R = {l: tikhonov_pinv(gmat(self.X[l], self.E[l]), tau) for l in t.levels}
        L = t.L
        # radiation matrices of the leaves, Eq. (algrad)
        self.V = []
        for b, c in enumerate(t.boxes[L]):
            xc = t.center(L, c)
            self.V.append(self.R[L] @ gmat(self.X[L] + xc, x[t.leaf_points[b]]))
        # source transfer per child quadrant, Eq. (algsou)
        self.C = {}
        for l in t.levels[1:]:
            a = t.side(l)
            for qi in (0, 1):
                for qj in (0, 1):
                    delta = np.array([(qi - 0.5) * a, (qj - 0.5) * a])
                    self.C[(l, qi, qj)] = self.R[l - 1] @ gmat(self.X[l - 1], self.E[l] + delta)
        self._D = {}

    def D(self, l, off):
        """Translation matrix of level l for the centre offset off = c_a - c_b (cells)."""
        key = (l, off)
        if key not in self._D:
            a = self.t.side(l)
            self._D[key] = gmat(self.E[l] + np.array(off, dtype=np.float64) * a, self.E[l])
        return self._D[key]

    def matvec(self, q):
        t, L, l0 = self.t, self.t.L, self.t.l0
        x = t.x
        phi = np.zeros(len(x))
        # near field, Eq. (algnf)
        for a, pa in enumerate(t.leaf_points):
            for b in t.near[a]:
                pb = t.leaf_points[b]
                K = gmat(x[pa], x[pb]) if a != b else _self_block(x[pa])
                phi[pa] += K @ q[pb]
        # radiation, Eq. (algrad)
        s = {l: np.zeros((len(t.boxes[l]), self.Q)) for l in t.levels}
        for b, pb in enumerate(t.leaf_points):
            s[L][b] = self.V[b] @ q[pb]
        # source transfer, Eq. (algsou)
        for l in range(L, l0, -1):
            for b, c in enumerate(t.boxes[l]):
                p = t.index[l - 1][(c[0] // 2, c[1] // 2)]
                s[l - 1][p] += self.C[(l, c[0] % 2, c[1] % 2)] @ s[l][b]
        # translation, Eq. (algtrans)
        o = {l: np.zeros((len(t.boxes[l]), self.Q)) for l in t.levels}
        for l in t.levels:
            for a, c in enumerate(t.boxes[l]):
                for b in t.il[l][a]:
                    cb = t.boxes[l][b]
                    o[l][a] += self.D(l, (c[0] - cb[0], c[1] - cb[1])) @ s[l][b]
        # potential transfer, Eq. (algpot)
        for l in range(l0 + 1, L + 1):
            for a, c in enumerate(t.boxes[l]):
                p = t.index[l - 1][(c[0] // 2, c[1] // 2)]
                o[l][a] += self.C[(l, c[0] % 2, c[1] % 2)].T @ o[l - 1][p]
        # reception, Eq. (algrec)
        for a, pa in enumerate(t.leaf_points):
            phi[pa] += self.V[a].T @ o[L][a]
        return phi


def _self_block(xa):
    K = gmat_safe(xa)
    return K


def gmat_safe(xa):
    d = np.hypot(xa[:, None, 0] - xa[None, :, 0], xa[:, None, 1] - xa[None, :, 1])
    np.fill_diagonal(d, 1.0)
    K = -np.log(d)
    np.fill_diagonal(K, 0.0)
    return K
