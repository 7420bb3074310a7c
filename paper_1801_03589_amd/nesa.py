"""ctypes binding of the C ABI in include/nesa.h (argument marshalling only).

Device vectors are torch tensors (complex64 / complex128, contiguous, on the
current HIP device); streams are torch streams.  Every call raises NesaError
when the library returns a non-zero status.  The library must have been built
(paper_1801_03589_amd/build.py): there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnesa.so")

C128, C64, C64_SPLIT, C64_SPLIT_FP16 = 0, 1, 2, 3
PRECOND_NONE, PRECOND_BLOCKDIAG, PRECOND_LEARNED, PRECOND_SCHWARZ = 0, 1, 2, 3
ETA0 = 376.730313668
K0 = 2.0 * np.pi


class NesaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nesa error %d: %s" % (code, msg))
        self.code = code


class TreeParams(C.Structure):
    _fields_ = [("leaf_size", C.c_double), ("l0_max", C.c_int), ("buffer", C.c_int)]


class EmParams(C.Structure):
    _fields_ = [("k", C.c_double), ("eta", C.c_double)]


class FarParams(C.Structure):
    _fields_ = [("d0", C.c_int), ("q_min", C.c_int), ("tau", C.c_double), ("eps", C.c_double)]


class TreeInfo(C.Structure):
    _fields_ = [("n_rwg", C.c_int64), ("n_tri", C.c_int64), ("L", C.c_int), ("l0", C.c_int),
                ("n_box", C.c_int64 * 32), ("near_entries", C.c_int64),
                ("n_pairs", C.c_int64 * 32), ("Q", C.c_int * 32), ("max_leaf", C.c_int64),
                ("near_entries_half", C.c_int64), ("near_transposed", C.c_int64)]


class GmresParams(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("tol", C.c_double),
                ("precond", C.c_int), ("fallback_ratio", C.c_double)]


class GmresReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("true_rel_residual", C.c_double),
                ("seconds", C.c_double), ("fell_back", C.c_int)]


class MlpParams(C.Structure):
    _fields_ = [("s_max", C.c_int), ("hidden", C.c_int), ("base", C.c_int)]


class AdamParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


class Model2DParams(C.Structure):
    _fields_ = [("P", C.c_int), ("Q", C.c_int), ("tau", C.c_double)]


MODEL2D_MAX_LEVELS = 24


class Model2DInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("l0", C.c_int), ("L", C.c_int), ("Q", C.c_int),
                ("n_box", C.c_int64 * MODEL2D_MAX_LEVELS), ("n_far", C.c_int64 * MODEL2D_MAX_LEVELS),
                ("near_pairs", C.c_int64), ("max_leaf", C.c_int64)]


_P = C.c_void_p
_SIGS = {
    "nesa_build_tree": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.POINTER(TreeParams), C.POINTER(_P)]),
    "nesa_tree_get_info": (C.c_int, [_P, C.POINTER(TreeInfo)]),
    "nesa_build_forest": (C.c_int, [C.c_int, _P, _P, _P, _P, C.POINTER(TreeParams), C.POINTER(_P)]),
    "nesa_tree_bodies": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_int)]),
    "nesa_tree_perm": (C.c_int, [_P, _P]),
    "nesa_tree_leaf_sizes": (C.c_int, [_P, _P, _P]),
    "nesa_tree_free": (None, [_P]),
    "nesa_assemble_near": (C.c_int, [_P, C.POINTER(EmParams), C.POINTER(_P)]),
    "nesa_assemble_near_device": (C.c_int, [_P, C.POINTER(EmParams), C.POINTER(_P)]),
    "nesa_near_entries": (C.c_int, [_P, _P, _P, C.c_int64, _P, C.c_int64, _P]),
    "nesa_near_free": (None, [_P]),
    "nesa_assemble_translations": (C.c_int, [_P, C.POINTER(EmParams), C.POINTER(FarParams), C.POINTER(_P)]),
    "nesa_far_get_q": (C.c_int, [_P, _P, C.c_int]),
    "nesa_far_free": (None, [_P]),
    "nesa_op_create": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.POINTER(_P)]),
    "nesa_op_free": (None, [_P]),
    "nesa_matvec": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "nesa_matvec_leaf": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "nesa_matvec_batched": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "nesa_matvec_phase_times": (C.c_int, [_P, _P, _P, _P, _P]),
    "nesa_matvec_launch_times": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_int32, _P]),
    "nesa_matvec_launch_times_nrhs": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P, _P, C.c_int32, _P]),
    "nesa_rhs_plane_wave_host": (C.c_int, [_P, C.c_double, _P, _P, C.c_int64, _P]),
    "nesa_rhs_plane_wave": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P]),
    "nesa_gmres_solve": (C.c_int, [_P, _P, _P, C.c_int64, C.POINTER(GmresParams),
                                   C.POINTER(GmresReport), _P, C.c_int64, _P]),
    "nesa_gmres_solve_noalloc": (C.c_int, [_P, _P, _P, C.c_int64, C.POINTER(GmresParams),
                                           C.POINTER(GmresReport), _P, C.c_int64, _P]),
    "nesa_precond_setup": (C.c_int, [_P, C.c_int]),
    "nesa_precond_apply": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "nesa_mlp_num_params": (C.c_int, [C.POINTER(MlpParams), C.POINTER(C.c_int64)]),
    "nesa_mlp_create": (C.c_int, [_P, C.POINTER(MlpParams), _P, C.POINTER(_P)]),
    "nesa_mlp_save": (C.c_int, [_P, C.c_char_p]),
    "nesa_mlp_load": (C.c_int, [_P, C.c_char_p, C.POINTER(_P)]),
    "nesa_mlp_free": (None, [_P]),
    "nesa_mlp_set_params": (C.c_int, [_P, _P]),
    "nesa_mlp_get_params": (C.c_int, [_P, _P]),
    "nesa_mlp_set_data": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "nesa_mlp_train": (C.c_int, [_P, C.POINTER(AdamParams), C.c_int, _P, _P]),
    "nesa_mlp_gradient": (C.c_int, [_P, _P, _P]),
    "nesa_mlp_outputs": (C.c_int, [_P, _P]),
    "nesa_mlp_apply": (C.c_int, [_P, _P, _P, _P]),
    "nesa_op_set_mlp": (C.c_int, [_P, _P]),
    "nesa_residual_error": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "nesa_last_error": (C.c_char_p, []),
    "nesa2d_create": (C.c_int, [_P, C.c_int64, C.POINTER(Model2DParams), C.POINTER(_P)]),
    "nesa2d_info_get": (C.c_int, [_P, C.POINTER(Model2DInfo)]),
    "nesa2d_perm": (C.c_int, [_P, _P]),
    "nesa2d_matvec": (C.c_int, [_P, _P, _P, _P]),
    "nesa2d_free": (C.c_int, [_P]),
}

_lib = None


def lib():
    """Load libnesa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same SONAME; loading torch
        # first makes this library bind to that single runtime instance
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise NesaError(-7, "libnesa.so not built (run paper_1801_03589_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise NesaError(rc, lib().nesa_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class _Handle:
    _free = None

    def __init__(self, h):
        self.h = h

    def __del__(self):
        if self.h and _lib is not None:
            getattr(_lib, self._free)(self.h)
            self.h = None


class Tree(_Handle):
    _free = "nesa_tree_free"

    def info(self):
        i = TreeInfo()
        _check(lib().nesa_tree_get_info(self.h, C.byref(i)))
        nl = i.L - i.l0 + 1
        return {"n_rwg": i.n_rwg, "n_tri": i.n_tri, "L": i.L, "l0": i.l0,
                "n_box": list(i.n_box[:nl]), "n_pairs": list(i.n_pairs[:nl]),
                "near_entries": i.near_entries, "max_leaf": i.max_leaf,
                "near_entries_half": i.near_entries_half, "near_transposed": i.near_transposed}

    def bodies(self):
        """Canonical RWG range of every body: array [nbodies + 1]."""
        nb = C.c_int()
        _check(lib().nesa_tree_bodies(self.h, None, 0, C.byref(nb)))
        out = np.zeros(nb.value + 1, dtype=np.int64)
        _check(lib().nesa_tree_bodies(self.h, _ptr(out), nb.value + 1, C.byref(nb)))
        return out

    def perm(self):
        p = np.zeros(self.info()["n_rwg"], dtype=np.int64)
        _check(lib().nesa_tree_perm(self.h, _ptr(p)))
        return p

    def leaf_sizes(self):
        """(S, W) per leaf: RWGs of the leaf and of its near leaves."""
        nleaf = self.info()["n_box"][-1]
        S = np.zeros(nleaf, dtype=np.int64)
        W = np.zeros(nleaf, dtype=np.int64)
        _check(lib().nesa_tree_leaf_sizes(self.h, _ptr(S), _ptr(W)))
        return S, W


class Near(_Handle):
    _free = "nesa_near_free"


class Far(_Handle):
    _free = "nesa_far_free"

    def q(self, nlevels):
        out = np.zeros(nlevels, dtype=np.int32)
        _check(lib().nesa_far_get_q(self.h, _ptr(out), nlevels))
        return out


class Op(_Handle):
    _free = "nesa_op_free"


def build_forest(bodies, leaf_size=0.25, l0_max=2, buffer=1):
    """bodies: list of (verts, tris)."""
    vs = [np.ascontiguousarray(v, dtype=np.float64) for v, _ in bodies]
    ts = [np.ascontiguousarray(t, dtype=np.int32) for _, t in bodies]
    nb = len(bodies)
    vp = (C.c_void_p * nb)(*[v.ctypes.data for v in vs])
    tp = (C.c_void_p * nb)(*[t.ctypes.data for t in ts])
    nv = np.array([len(v) for v in vs], dtype=np.int64)
    nt = np.array([len(t) for t in ts], dtype=np.int64)
    h = C.c_void_p()
    prm = TreeParams(leaf_size, l0_max, buffer)
    _check(lib().nesa_build_forest(nb, C.cast(vp, C.c_void_p), _ptr(nv), C.cast(tp, C.c_void_p), _ptr(nt),
                                   C.byref(prm), C.byref(h)))
    tr = Tree(h)
    tr._keep = (vs, ts)
    return tr


def build_tree(verts, tris, leaf_size=0.25, l0_max=2, buffer=1):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    h = C.c_void_p()
    prm = TreeParams(leaf_size, l0_max, buffer)
    _check(lib().nesa_build_tree(_ptr(v), len(v), _ptr(t), len(t), C.byref(prm), C.byref(h)))
    return Tree(h)


def assemble_near(tree, k=K0, eta=ETA0):
    h = C.c_void_p()
    _check(lib().nesa_assemble_near(tree.h, C.byref(EmParams(k, eta)), C.byref(h)))
    return Near(h)


def assemble_near_device(tree, k=K0, eta=ETA0):
    """Near-field blocks computed on the current GPU, returned as a host handle."""
    h = C.c_void_p()
    _check(lib().nesa_assemble_near_device(tree.h, C.byref(EmParams(k, eta)), C.byref(h)))
    return Near(h)


def near_entries(tree, near, rows, cols):
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros((len(r), len(c)), dtype=np.complex128)
    _check(lib().nesa_near_entries(tree.h, near.h, _ptr(r), len(r), _ptr(c), len(c), _ptr(out)))
    return out


def assemble_translations(tree, k=K0, eta=ETA0, d0=3, q_min=0, tau=1e-8, eps=0.1):
    h = C.c_void_p()
    _check(lib().nesa_assemble_translations(tree.h, C.byref(EmParams(k, eta)),
                                            C.byref(FarParams(d0, q_min, tau, eps)), C.byref(h)))
    return Far(h)


def op_create(tree, near, far, precision=C64, max_nrhs=1):
    h = C.c_void_p()
    _check(lib().nesa_op_create(tree.h, near.h, far.h, precision, max_nrhs, C.byref(h)))
    op = Op(h)
    op.keep = (tree, near, far)
    op.precision = precision
    return op


def matvec(op, x, y, nrhs=1, stream=None):
    _check(lib().nesa_matvec(op.h, _dptr(x), _dptr(y), nrhs, _stream(stream)))


def matvec_batched(ops, xs, ys, nrhs=None, stream=None):
    """y_i = Z_i x_i for several operators in one call (nesa_matvec_batched)."""
    n = len(ops)
    nr = np.ascontiguousarray(nrhs if nrhs is not None else [1] * n, dtype=np.int64)
    oh = (C.c_void_p * n)(*[o.h for o in ops])
    xp = (C.c_void_p * n)(*[_dptr(x).value for x in xs])
    yp = (C.c_void_p * n)(*[_dptr(y).value for y in ys])
    _check(lib().nesa_matvec_batched(oh, n, xp, yp, _ptr(nr), _stream(stream)))


def matvec_leaf(op, x, y, nrhs=1, stream=None):
    _check(lib().nesa_matvec_leaf(op.h, _dptr(x), _dptr(y), nrhs, _stream(stream)))


def matvec_phase_times(op, x, y, stream=None):
    ms = np.zeros(5, dtype=np.float32)
    _check(lib().nesa_matvec_phase_times(op.h, _dptr(x), _dptr(y), _stream(stream), _ptr(ms)))
    return ms


KIND_NAMES = {1: "radiate", 2: "upward_gemm", 3: "upward_sum", 4: "upward_fp64", 5: "translate_gemm",
              6: "translate_sum", 7: "translate_fp64", 8: "downward_gemm", 9: "downward_fp64",
              10: "near_recv", 11: "receive"}


def matvec_launch_times(op, x, y, stream=None, max_launches=128, nrhs=1):
    """[(kind name, level, ms)] for every kernel launch of one product (leaf order)."""
    ms = np.zeros(max_launches, dtype=np.float32)
    kind = np.zeros(max_launches, dtype=np.int32)
    lev = np.zeros(max_launches, dtype=np.int32)
    cnt = C.c_int32()
    _check(lib().nesa_matvec_launch_times_nrhs(op.h, _dptr(x), _dptr(y), nrhs, _stream(stream), _ptr(ms),
                                               _ptr(kind), _ptr(lev), max_launches, C.byref(cnt)))
    return [(KIND_NAMES[int(kind[i])], int(lev[i]), float(ms[i])) for i in range(cnt.value)]


def rhs_plane_wave_host(tree, khat, pol, k=K0):
    kh = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
    po = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
    n = tree.info()["n_rwg"]
    b = np.zeros((len(kh), n), dtype=np.complex128)
    _check(lib().nesa_rhs_plane_wave_host(tree.h, k, _ptr(kh), _ptr(po), len(kh), _ptr(b)))
    return b


def rhs_plane_wave(op, khat, pol, b, stream=None):
    kh = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
    po = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
    _check(lib().nesa_rhs_plane_wave(op.h, _ptr(kh), _ptr(po), len(kh), _dptr(b), _stream(stream)))


def precond_setup(op, precond):
    _check(lib().nesa_precond_setup(op.h, precond))


def precond_apply(op, precond, r, z, stream=None):
    """z = M r (leaf order, one vector)."""
    _check(lib().nesa_precond_apply(op.h, precond, _dptr(r), _dptr(z), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 256 << 20


def gmres_solve(op, b, x, nrhs=1, restart=30, max_iters=1000, tol=1e-6, precond=PRECOND_NONE,
                history_len=0, stream=None, check=True, fallback_ratio=0.5, noalloc=False):
    """noalloc: nesa_gmres_solve_noalloc (work buffers from the library's fixed
    device array; right-hand sides one at a time)."""
    prm = GmresParams(restart, max_iters, tol, precond, fallback_ratio)
    rep = (GmresReport * nrhs)()
    hist = np.zeros(max(1, history_len), dtype=np.float64)
    fn = lib().nesa_gmres_solve_noalloc if noalloc else lib().nesa_gmres_solve
    rc = fn(op.h, _dptr(b), _dptr(x), nrhs, C.byref(prm), rep, _ptr(hist), history_len, _stream(stream))
    if check and rc not in (0, -5):
        _check(rc)
    reports = [{"iters": r.iters, "restarts": r.restarts, "true_rel_residual": r.true_rel_residual,
                "seconds": r.seconds, "fell_back": r.fell_back} for r in rep]
    return rc, reports, hist[:history_len]


def mlp_num_params(s_max, hidden, base=PRECOND_SCHWARZ):
    c = C.c_int64()
    _check(lib().nesa_mlp_num_params(C.byref(MlpParams(s_max, hidden, base)), C.byref(c)))
    return c.value


class Mlp(_Handle):
    """Learned per-leaf preconditioner network of one operator."""
    _free = "nesa_mlp_free"

    def __init__(self, op, s_max, hidden, base, theta0):
        theta0 = np.ascontiguousarray(theta0, dtype=np.float32)
        n = mlp_num_params(s_max, hidden, base)
        if theta0.size != n:
            raise ValueError("expected %d parameters" % n)
        h = C.c_void_p()
        _check(lib().nesa_mlp_create(op.h, C.byref(MlpParams(s_max, hidden, base)), _ptr(theta0),
                                     C.byref(h)))
        super().__init__(h)
        self.op, self.s_max, self.hidden, self.base, self.n_params = op, s_max, hidden, base, n

    @classmethod
    def load(cls, op, path):
        """Network for `op` from a file written by save()."""
        h = C.c_void_p()
        _check(lib().nesa_mlp_load(op.h, os.fsencode(path), C.byref(h)))
        self = cls.__new__(cls)
        _Handle.__init__(self, h)
        with open(path, "rb") as f:             # s_max, hidden, base after the 8-byte tag
            hdr = np.frombuffer(f.read(20)[8:], dtype=np.int32)
        self.op, self.s_max, self.hidden, self.base = op, int(hdr[0]), int(hdr[1]), int(hdr[2])
        self.n_params = mlp_num_params(self.s_max, self.hidden, self.base)
        return self

    def save(self, path):
        _check(lib().nesa_mlp_save(self.h, os.fsencode(path)))

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.size != self.n_params:
            raise ValueError("expected %d parameters" % self.n_params)
        _check(lib().nesa_mlp_set_params(self.h, _ptr(theta)))

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().nesa_mlp_get_params(self.h, _ptr(out)))
        return out

    def set_data(self, r, e, stream=None):
        """r, e: device tensors [nsamples][n_rwg] (canonical order)."""
        if r.shape != e.shape or r.dim() != 2:
            raise ValueError("r and e must be [nsamples][n_rwg]")
        _check(lib().nesa_mlp_set_data(self.h, _dptr(r), _dptr(e), r.shape[0], _stream(stream)))
        self.nsamples = r.shape[0]

    def train(self, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        hist = np.zeros(max(1, steps), dtype=np.float64)
        _check(lib().nesa_mlp_train(self.h, C.byref(AdamParams(lr, beta1, beta2, eps)), steps, _ptr(hist),
                                    _stream(stream)))
        return hist[:steps]

    def gradient(self):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_double()
        _check(lib().nesa_mlp_gradient(self.h, _ptr(g), C.byref(loss)))
        return loss.value, g

    def outputs(self, nleaf):
        y = np.zeros((self.nsamples * nleaf, 2 * self.s_max), dtype=np.float32)
        _check(lib().nesa_mlp_outputs(self.h, _ptr(y)))
        return y

    def apply(self, r, z, stream=None):
        """z = M_base r + correction (one vector, leaf order)."""
        _check(lib().nesa_mlp_apply(self.h, _dptr(r), _dptr(z), _stream(stream)))


def op_set_mlp(op, net):
    _check(lib().nesa_op_set_mlp(op.h, net.h if net is not None else None))
    op._mlp = net


def residual_error(op, b, xs, x, r, e, stream=None):
    """r = b - Z x, e = xs - x (one vector each, canonical order)."""
    _check(lib().nesa_residual_error(op.h, _dptr(b), _dptr(xs), _dptr(x), _dptr(r), _dptr(e), _stream(stream)))


def solve_pairs(op, b, xs, iters, restart, precond):
    """Training pairs from the method's own solves: for each k in `iters` the
    iterate x_k of FGMRES(restart) with `precond` after k iterations from zero,
    and (r_k, e_k) = (b - Z x_k, xs - x_k).  Returns r, e as [len(iters)][n]."""
    import torch
    n = b.shape[-1]
    R = torch.empty((len(iters), n), dtype=b.dtype, device=b.device)
    E = torch.empty_like(R)
    for i, k in enumerate(iters):
        x = torch.zeros_like(b)
        if k > 0:
            gmres_solve(op, b, x, restart=restart, max_iters=k, tol=1e-12, precond=precond, check=False)
        residual_error(op, b, xs, x, R[i], E[i])
    return R, E


class Model2D:
    """NESA operator of the 2D potential problem phi = K q, k_ij = -log|x_i - x_j|
    (real FP64; tree, matrices and conventions in include/nesa2d.h)."""

    def __init__(self, xy, P, Q, tau=1e-12):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        if xy.ndim != 2 or xy.shape[1] != 2:
            raise NesaError(-1, "xy must be an (n, 2) array")
        h = _P()
        prm = Model2DParams(int(P), int(Q), float(tau))
        _check(lib().nesa2d_create(_ptr(xy), len(xy), C.byref(prm), C.byref(h)))
        self.h = h

    def info(self):
        inf = Model2DInfo()
        _check(lib().nesa2d_info_get(self.h, C.byref(inf)))
        nl = inf.L - inf.l0 + 1
        return {"n": inf.n, "l0": inf.l0, "L": inf.L, "Q": inf.Q, "n_box": list(inf.n_box[:nl]),
                "n_far": list(inf.n_far[:nl]), "near_pairs": inf.near_pairs, "max_leaf": inf.max_leaf}

    def perm(self):
        out = np.zeros(self.info()["n"], dtype=np.int32)
        _check(lib().nesa2d_perm(self.h, _ptr(out)))
        return out

    def matvec(self, q, phi, stream=None):
        """phi = K_NESA q for float64 device tensors of n entries."""
        _check(lib().nesa2d_matvec(self.h, _dptr(q), _dptr(phi), _stream(stream)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.nesa2d_free(h)
            self.h = None
