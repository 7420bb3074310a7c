"""Octree, near lists and interaction lists (plain reference).

Follows Sec. 2 (hierarchical partition with near blocks stored directly and
far blocks compressed; coarsest far level chosen so that the ancestors do not
touch) and Sec. 3 (coarsest level with 4 groups along the longest side; near
neighbours are the adjacent groups including diagonal ones and the group
itself; a pair interacts in the far field at the level where the two groups
are not neighbours but their parents were).

Readings taken where the paper is silent:

* the leaf side is fixed (default 0.25 wavelength) instead of an occupancy
  target; L = ceil(log2(longest bounding-box side / leaf side)) (0 if the body
  fits in one leaf), root cube of side leaf * 2^L anchored 1e-9 below the
  bounding-box minimum of the vertices;
* an RWG belongs to the leaf containing its edge midpoint
  (index floor((p - lo)/a), clamped to the grid);
* coarsest level l0 = min(2, L); at l0 every non-neighbour pair interacts;
* empty boxes do not exist (sparse tree).
"""
import math

import numpy as np


def cheb(a, b):
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]), abs(a[2] - b[2]))


class Octree:
    def __init__(self, verts, midpoints, leaf=0.25, l0_max=2, buffer=1):
        v = np.asarray(verts, dtype=np.float64)
        self.lo = v.min(axis=0) - 1e-9
        ext = float((v.max(axis=0) - v.min(axis=0)).max())
        self.leaf = float(leaf)
        self.L = int(math.ceil(math.log2(ext / self.leaf))) if ext > self.leaf else 0
        self.l0 = min(l0_max, self.L)
        self.buffer = buffer
        nside = 1 << self.L
        idx = np.floor((np.asarray(midpoints) - self.lo) / self.leaf).astype(np.int64)
        idx = np.clip(idx, 0, nside - 1)
        self.rwg_leaf_idx = idx
        # boxes per level: sorted integer triples
        self.boxes = {}
        self.box_id = {}
        for l in range(self.l0, self.L + 1):
            sh = self.L - l
            keys = sorted(set(map(tuple, (idx >> sh).tolist())))
            self.boxes[l] = keys
            self.box_id[l] = {k: i for i, k in enumerate(keys)}
        # RWGs of every leaf
        leaf_of = [self.box_id[self.L][tuple(p)] for p in idx.tolist()]
        self.rwg_leaf = np.array(leaf_of, dtype=np.int64)
        self.leaf_rwgs = [[] for _ in self.boxes[self.L]]
        for n, b in enumerate(leaf_of):
            self.leaf_rwgs[b].append(n)
        self.leaf_rwgs = [np.array(x, dtype=np.int64) for x in self.leaf_rwgs]
        # parents
        self.parent = {}
        for l in range(self.l0 + 1, self.L + 1):
            self.parent[l] = np.array([self.box_id[l - 1][(k[0] >> 1, k[1] >> 1, k[2] >> 1)]
                                       for k in self.boxes[l]], dtype=np.int64)
        # near list at the leaf level (Chebyshev distance <= buffer, self included)
        rng = range(-buffer, buffer + 1)
        offs = [(a, b, c) for a in rng for b in rng for c in rng]
        idsL = self.box_id[self.L]
        self.near = []
        for ka in self.boxes[self.L]:
            nb = [idsL.get((ka[0] + o[0], ka[1] + o[1], ka[2] + o[2])) for o in offs]
            self.near.append(sorted(j for j in nb if j is not None))
        # interaction lists
        self.il = {}
        for l in range(self.l0, self.L + 1):
            keys = self.boxes[l]
            ids = self.box_id[l]
            lst = []
            for ka in keys:
                if l == self.l0:
                    cand = range(len(keys))
                else:
                    # children of the parent's neighbours
                    pa = (ka[0] >> 1, ka[1] >> 1, ka[2] >> 1)
                    cand = []
                    for o in offs:
                        q = (pa[0] + o[0], pa[1] + o[1], pa[2] + o[2])
                        for c in range(8):
                            j = ids.get((2 * q[0] + (c & 1), 2 * q[1] + ((c >> 1) & 1),
                                         2 * q[2] + ((c >> 2) & 1)))
                            if j is not None:
                                cand.append(j)
                lst.append(sorted(j for j in cand if cheb(ka, keys[j]) > buffer))
            self.il[l] = lst

    def side(self, l):
        return self.leaf * (1 << (self.L - l))

    def center(self, l, i):
        return self.lo + (np.array(self.boxes[l][i], dtype=np.float64) + 0.5) * self.side(l)
