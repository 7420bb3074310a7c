"""The NumPy oracle's NESA operator applied by the plain C loops of nesa_c.c.

TEST INFRASTRUCTURE ONLY (see the package docstring).  NesaC takes a built
NesaOracle (tree, point sets, fitting operators, transfer and translation
matrices, all from oracle/nesa.py) and computes in C, FP64, with OpenMP over
leaves and boxes: the near-field Galerkin blocks (Sec. 2, Eq. 1-3), the
radiation matrices (Sec. 3, Eq. 10) and the whole product (Eq. 9-14) in the
paper's stage order.  It exists so that the product of the large workloads can
be run whole on the host's cores; on small meshes it is pinned against
NesaOracle.matvec (tests/test_oracle_c.py).

build() compiles liboracle_nesa.so with gcc (-O2 -fopenmp).
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nesa_c.c")
LIB = os.path.join(HERE, "liboracle_nesa.so")

_lib = None


def build():
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _lib.oc_set_threads.argtypes = [C.c_int]
        _lib.oc_max_threads.restype = C.c_int
    return _lib


class _Mesh(C.Structure):
    _fields_ = [("v", C.c_void_p), ("t", C.c_void_p), ("area", C.c_void_p), ("normal", C.c_void_p),
                ("qp", C.c_void_p), ("tri", C.c_void_p), ("freev", C.c_void_p), ("len", C.c_void_p),
                ("k", C.c_double), ("eta", C.c_double)]


class _Nesa(C.Structure):
    _fields_ = [("nlev", C.c_int), ("Q", C.c_void_p), ("nbox", C.c_void_p), ("s_off", C.c_void_p),
                ("parent", C.c_void_p), ("par_off", C.c_void_p), ("octant", C.c_void_p),
                ("ch_ptr", C.c_void_p), ("ch_off", C.c_void_p), ("ch_idx", C.c_void_p),
                ("il_ptr", C.c_void_p), ("il_off", C.c_void_p), ("il_src", C.c_void_p), ("il_d", C.c_void_p),
                ("Dall", C.c_void_p), ("Call", C.c_void_p), ("c_off", C.c_void_p),
                ("V", C.c_void_p), ("voff", C.c_void_p), ("Z", C.c_void_p), ("zoff", C.c_void_p),
                ("nleaf", C.c_int64), ("rw_ptr", C.c_void_p), ("rw_idx", C.c_void_p),
                ("near_ptr", C.c_void_p), ("near_idx", C.c_void_p), ("w", C.c_double * 8)]


def _p(a):
    return C.c_void_p(a.ctypes.data)


def _i64(x):
    return np.ascontiguousarray(x, dtype=np.int64)


class NesaC:
    """Operators of `ref` (a NesaOracle) in the C layout; matvec(x) = Z_NESA x."""

    def __init__(self, ref, threads=None):
        L_ = lib()
        if threads is not None:
            L_.oc_set_threads(int(threads))
        self.ref = ref
        m, t = ref.m, ref.t
        keep = []                                    # arrays the C structs point into

        def k(a):
            keep.append(a)
            return a

        self.mesh = _Mesh(_p(k(np.ascontiguousarray(m.verts, dtype=np.float64))),
                          _p(k(_i64(m.tris))), _p(k(np.ascontiguousarray(m.area))),
                          _p(k(np.ascontiguousarray(m.normal))), _p(k(np.ascontiguousarray(m.qp))),
                          _p(k(_i64(m.tri))), _p(k(_i64(m.free))), _p(k(np.ascontiguousarray(m.length))),
                          ref.k, ref.eta)
        # leaves: RWGs in the oracle's order, near lists
        nleaf = len(t.leaf_rwgs)
        sizes = np.array([len(r) for r in t.leaf_rwgs], dtype=np.int64)
        rw_ptr = k(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))
        rw_idx = k(_i64(np.concatenate(t.leaf_rwgs)))
        near_ptr = k(np.concatenate([[0], np.cumsum([len(x) for x in t.near])]).astype(np.int64))
        near_idx = k(_i64(np.concatenate([np.asarray(x, dtype=np.int64) for x in t.near])))
        widths = np.array([sizes[np.asarray(x)].sum() for x in t.near], dtype=np.int64)
        zoff = k(np.concatenate([[0], np.cumsum(sizes * widths)]).astype(np.int64))
        self.Z = k(np.zeros(int(zoff[-1]), dtype=np.complex128))
        L_.oc_near_blocks(C.byref(self.mesh), C.c_int64(nleaf), _p(rw_ptr), _p(rw_idx), _p(near_ptr),
                          _p(near_idx), _p(zoff), _p(self.Z))
        # radiation matrices of every leaf
        QL = ref.Q[t.L]
        voff = k(np.concatenate([[0], np.cumsum(4 * QL * sizes)]).astype(np.int64))
        self.V = k(np.zeros(int(voff[-1]), dtype=np.complex128))
        cen = k(np.ascontiguousarray([t.center(t.L, b) for b in range(nleaf)], dtype=np.float64))
        R = k(np.ascontiguousarray(ref.R[t.L], dtype=np.complex128))
        X = k(np.ascontiguousarray(ref.X[t.L], dtype=np.float64))
        L_.oc_radiation(C.byref(self.mesh), C.c_int64(nleaf), _p(rw_ptr), _p(rw_idx), _p(cen), C.c_int(QL),
                        C.c_int(len(X)), _p(R), _p(X), _p(voff), _p(self.V))
        # levels: Q, boxes, parents, octants, children, interaction lists with
        # the offset of each pair's translation matrix, transfer matrices
        lv = ref.levels
        Q = k(np.array([ref.Q[l] for l in lv], dtype=np.int32))
        nbox = k(np.array([len(t.boxes[l]) for l in lv], dtype=np.int64))
        s_off = k(np.concatenate([[0], np.cumsum(4 * nbox * Q.astype(np.int64))]).astype(np.int64))
        par, octs, par_off = [], [], [0]
        ch_ptr, ch_idx, ch_off = [], [], []
        for i, l in enumerate(lv):
            if i > 0:
                par.append(np.asarray(t.parent[l], dtype=np.int64))
                octs.append(np.array([ref.octant(l, b) for b in range(len(t.boxes[l]))], dtype=np.int32))
            else:
                par.append(np.zeros(len(t.boxes[l]), dtype=np.int64))
                octs.append(np.zeros(len(t.boxes[l]), dtype=np.int32))
            par_off.append(par_off[-1] + len(par[-1]))
        for i, l in enumerate(lv):
            ch_off.append(sum(len(x) for x in ch_ptr))
            if i + 1 < len(lv):
                pc = par[i + 1]
                order = np.argsort(pc, kind="stable")
                cnt = np.bincount(pc, minlength=len(t.boxes[l]))
                ch_ptr.append(np.concatenate([[0], np.cumsum(cnt)]) + sum(len(x) for x in ch_idx))
                ch_idx.append(order.astype(np.int64))
            else:
                ch_ptr.append(np.zeros(len(t.boxes[l]) + 1, dtype=np.int64))
        dmats, dpos, il_ptr, il_off, il_src, il_d = [], {}, [], [], [], []
        dsize = 0
        for i, l in enumerate(lv):
            il_off.append(sum(len(x) for x in il_ptr))
            ptr = [sum(len(x) for x in il_src)]
            keys = t.boxes[l]
            for a, lst in enumerate(t.il[l]):
                ka = keys[a]
                for b in lst:
                    kb = keys[b]
                    off = (l, ka[0] - kb[0], ka[1] - kb[1], ka[2] - kb[2])
                    if off not in dpos:
                        D = np.ascontiguousarray(ref.D(l, off[1:]), dtype=np.complex128)
                        dpos[off] = dsize
                        dsize += D.size
                        dmats.append(D.ravel())
                    il_d.append(dpos[off])
                il_src.append(np.asarray(lst, dtype=np.int64))
                ptr.append(ptr[-1] + len(lst))
            il_ptr.append(np.array(ptr, dtype=np.int64))
        cmats, c_off = [], [0] * len(lv)
        csize = 0
        for i, l in enumerate(lv):
            if i == 0:
                continue
            c_off[i] = csize
            for o in range(8):
                Cm = np.ascontiguousarray(ref.C(l, o), dtype=np.complex128)
                cmats.append(Cm.ravel())
                csize += Cm.size
        cat = lambda xs, dt: k(np.ascontiguousarray(np.concatenate(xs) if xs else np.zeros(1), dtype=dt))
        self.op = _Nesa()
        o = self.op
        o.nlev = len(lv)
        o.Q, o.nbox, o.s_off = _p(Q), _p(nbox), _p(s_off)
        o.parent, o.par_off, o.octant = _p(cat(par, np.int64)), _p(k(_i64(par_off))), _p(cat(octs, np.int32))
        o.ch_ptr, o.ch_off, o.ch_idx = _p(cat(ch_ptr, np.int64)), _p(k(_i64(ch_off))), _p(cat(ch_idx, np.int64))
        o.il_ptr, o.il_off = _p(cat(il_ptr, np.int64)), _p(k(_i64(il_off)))
        o.il_src, o.il_d = _p(cat(il_src, np.int64)), _p(k(_i64(il_d if il_d else [0])))
        o.Dall, o.Call, o.c_off = _p(cat(dmats, np.complex128)), _p(cat(cmats, np.complex128)), _p(k(_i64(c_off)))
        o.V, o.voff, o.Z, o.zoff = _p(self.V), _p(voff), _p(self.Z), _p(zoff)
        o.nleaf = nleaf
        o.rw_ptr, o.rw_idx, o.near_ptr, o.near_idx = _p(rw_ptr), _p(rw_idx), _p(near_ptr), _p(near_idx)
        for c in range(4):
            o.w[2 * c] = ref.w[c].real
            o.w[2 * c + 1] = ref.w[c].imag
        self._keep = keep
        self.n = m.n
        self._s = np.zeros(int(s_off[-1]), dtype=np.complex128)
        self._o = np.zeros(int(s_off[-1]), dtype=np.complex128)

    def matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros(self.n, dtype=np.complex128)
        lib().oc_matvec(C.byref(self.op), _p(x), _p(y), _p(self._s), _p(self._o))
        return y


def set_threads(n):
    lib().oc_set_threads(int(n))


def max_threads():
    return lib().oc_max_threads()
