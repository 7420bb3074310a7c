"""CPU tests of the library's host side through the C ABI: exported symbols,
tree, near-field entries and right-hand sides against the oracle, error paths.
No GPU compute calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import efie
from oracle.tree import Octree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nesa():
    from paper_1801_03589_amd import nesa as n
    n.lib()
    return n


def test_every_declared_symbol_is_exported(nesa):
    import glob
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        names |= set(re.findall(r"\b(nesa2?d?_[a-z0-9_]+)\s*\(", open(h).read()))
    assert len(names) > 15
    assert {"nesa2d_create", "nesa2d_matvec", "nesa2d_free"} <= names
    so = ctypes.CDLL(nesa.LIB_PATH)
    for name in sorted(names):
        assert hasattr(so, name), name


@pytest.mark.parametrize("leaf", [0.25, 0.125])
def test_tree_matches_oracle(nesa, sphere1, leaf):
    v, t = sphere1
    tr = nesa.build_tree(v, t, leaf)
    info = tr.info()
    m = efie.RWG(v, t)
    ot = Octree(v, m.midpoints(), leaf=leaf)
    assert (info["L"], info["l0"], info["n_rwg"]) == (ot.L, ot.l0, m.n)
    assert info["n_box"] == [len(ot.boxes[l]) for l in range(ot.l0, ot.L + 1)]
    assert info["n_pairs"] == [sum(len(x) for x in ot.il[l]) for l in range(ot.l0, ot.L + 1)]
    # leaf order groups exactly the oracle's leaves
    perm = tr.perm()
    assert np.array_equal(np.sort(perm), np.arange(m.n))
    leaf_seq = ot.rwg_leaf[perm]
    changes = np.count_nonzero(np.diff(leaf_seq)) + 1
    assert changes == len(ot.boxes[ot.L])


def test_leaf_order_is_morton_then_canonical(nesa, sphere1):
    """Leaf order: leaves by the Morton code of their integer key (x in the
    lowest bit of each triple), RWGs of a leaf by canonical index."""
    v, t = sphere1
    m = efie.RWG(v, t)
    for leaf in (0.25, 0.125):
        ot = Octree(v, m.midpoints(), leaf=leaf)

        def morton(k):
            return sum(((int(k[d]) >> b) & 1) << (3 * b + d) for b in range(21) for d in range(3))
        leaves = sorted(range(len(ot.boxes[ot.L])), key=lambda a: morton(ot.boxes[ot.L][a]))
        perm = np.concatenate([np.sort(np.asarray(ot.leaf_rwgs[a], dtype=np.int64)) for a in leaves])
        assert np.array_equal(perm, nesa.build_tree(v, t, leaf).perm())


def test_near_entries_match_oracle(nesa, sphere1, dense1):
    v, t = sphere1
    tr = nesa.build_tree(v, t, 0.25)
    nr = nesa.assemble_near(tr)
    m = efie.RWG(v, t)
    ot = Octree(v, m.midpoints(), leaf=0.25)
    for r in (0, 5, 100, 1500, 2999):
        a = ot.rwg_leaf[r]
        cols = np.concatenate([ot.leaf_rwgs[b] for b in ot.near[a]])
        z = nesa.near_entries(tr, nr, [r], cols)[0]
        assert np.abs(z - dense1[r, cols]).max() <= 1e-13 * np.abs(dense1[r, cols]).max()


@pytest.mark.parametrize("leaf", [0.25, 0.125])
def test_half_storage_counts_match_oracle(nesa, sphere1, leaf):
    """Reciprocity half storage keeps, per leaf a, the blocks Z_ab of its near
    leaves b >= a in leaf order (Morton order of the leaf keys): sum_a S_a^2
    plus S_a S_b once per neighbouring pair, and Z_ab^T x_a yields S_b outputs
    per pair a < b.  Counted here on the oracle's own tree."""
    v, t = sphere1
    info = nesa.build_tree(v, t, leaf).info()
    m = efie.RWG(v, t)
    ot = Octree(v, m.midpoints(), leaf=leaf)

    def morton(k):
        return sum(((int(k[d]) >> b) & 1) << (3 * b + d) for b in range(21) for d in range(3))
    nleaf = len(ot.boxes[ot.L])
    rank = {a: r for r, a in enumerate(sorted(range(nleaf), key=lambda a: morton(ot.boxes[ot.L][a])))}
    S = [len(ot.leaf_rwgs[a]) for a in range(nleaf)]
    full = sum(S[a] * sum(S[b] for b in ot.near[a]) for a in range(nleaf))
    half = sum(S[a] * sum(S[b] for b in ot.near[a] if rank[b] >= rank[a]) for a in range(nleaf))
    trans = sum(S[b] for a in range(nleaf) for b in ot.near[a] if rank[b] > rank[a])
    diag = sum(s * s for s in S)
    assert 2 * half - diag == full          # every off-diagonal block once
    assert (info["near_entries"], info["near_entries_half"], info["near_transposed"]) == (full, half, trans)
    assert half < 0.6 * full
    # per-leaf sizes in leaf order: S_a and the RWGs W_a of a's near leaves
    Sl, Wl = nesa.build_tree(v, t, leaf).leaf_sizes()
    order = sorted(range(nleaf), key=lambda a: rank[a])
    assert Sl.tolist() == [S[a] for a in order]
    assert Wl.tolist() == [sum(S[b] for b in ot.near[a]) for a in order]


def test_rhs_matches_oracle(nesa, sphere1, rwg1):
    tr = nesa.build_tree(*sphere1, 0.25)
    kh = np.array([[0, 0, 1.0], [0.6, 0, 0.8]])
    po = np.array([[1.0, 0, 0], [0, 1.0, 0]])
    b = nesa.rhs_plane_wave_host(tr, kh, po)
    for i in range(2):
        bo = efie.plane_wave_rhs(rwg1, kh[i], po[i])
        assert np.abs(b[i] - bo).max() <= 1e-13 * np.abs(bo).max()


def test_q_rule_matches_oracle(nesa, sphere1):
    from oracle import nesa as onesa
    tr = nesa.build_tree(*sphere1, 0.125)
    for d0 in (1, 3, 5):
        far = nesa.assemble_translations(tr, d0=d0)
        assert list(far.q(2)) == [onesa.q_rule(0.25, d0), onesa.q_rule(0.125, d0)]


def test_error_paths(nesa):
    v, t = synth.icosphere(2, 1.0)
    with pytest.raises(nesa.NesaError) as e:
        nesa.build_tree(v, t[:-1], 0.25)           # open surface
    assert e.value.code == -4
    bad = t.copy()
    bad[0, 0] = len(v) + 5
    with pytest.raises(nesa.NesaError) as e:
        nesa.build_tree(v, bad, 0.25)
    assert e.value.code == -1
    with pytest.raises(nesa.NesaError):
        nesa.build_tree(v, t, -1.0)
    lib = nesa.lib()
    assert lib.nesa_build_tree(None, 0, None, 0, None, None) == -1
    assert lib.nesa_matvec(None, None, None, 1, None) == -1
    tr = nesa.build_tree(v, t, 0.25)
    with pytest.raises(nesa.NesaError):
        nesa.assemble_translations(tr, d0=0)
    # the device near-field assembly checks its arguments before touching a GPU
    assert lib.nesa_assemble_near_device(None, None, None) == -1
    with pytest.raises(nesa.NesaError) as e:
        nesa.assemble_near_device(tr, k=-1.0)
    assert e.value.code == -1
    with pytest.raises(nesa.NesaError) as e:
        nesa.assemble_near_device(tr, eta=0.0)
    assert e.value.code == -1
    # a mesh far too coarse for the leaf: equivalent sphere outside the check sphere
    with pytest.raises(nesa.NesaError) as e:
        nesa.assemble_translations(nesa.build_tree(*synth.icosphere(2, 1.0), 0.05))
    assert e.value.code == -4


def _bodies():
    return [synth.icosphere(6, 0.3), synth.box_mesh((0.5, 0.3, 0.4), 0.06),
            synth.spheroid((0.6, 0.3, 0.3), 0.07), synth.capped_cylinder(0.2, 0.8, 0.07)]


def test_forest_matches_per_body_trees(nesa):
    """Forest of several meshes: body i keeps its own tree, shifted so that all
    leaf levels align; RWGs and leaves numbered body by body."""
    bodies = _bodies()
    fr = nesa.build_forest(bodies, 0.25)
    fi = fr.info()
    trees = [nesa.build_tree(v, t, 0.25) for v, t in bodies]
    infos = [tr.info() for tr in trees]
    ptr = fr.bodies()
    assert list(np.diff(ptr)) == [i["n_rwg"] for i in infos]
    assert fi["L"] == max(i["L"] for i in infos)
    assert fi["l0"] == min(i["l0"] + fi["L"] - i["L"] for i in infos)
    for l in range(fi["l0"], fi["L"] + 1):
        nb = 0
        npairs = 0
        for i in infos:
            li = l - (fi["L"] - i["L"])
            if li >= i["l0"]:
                nb += i["n_box"][li - i["l0"]]
                npairs += i["n_pairs"][li - i["l0"]]
        assert fi["n_box"][l - fi["l0"]] == nb
        assert fi["n_pairs"][l - fi["l0"]] == npairs
    assert fi["near_entries"] == sum(i["near_entries"] for i in infos)
    perm = np.concatenate([tr.perm() + ptr[i] for i, tr in enumerate(trees)])
    assert np.array_equal(fr.perm(), perm)


def test_forest_near_entries_match_oracle(nesa):
    """Near-field entries of every body of a forest against the dense oracle
    matrix of that body (bodies never couple)."""
    bodies = _bodies()[:2]
    fr = nesa.build_forest(bodies, 0.25)
    nr = nesa.assemble_near(fr)
    ptr = fr.bodies()
    for i, (v, t) in enumerate(bodies):
        m = efie.RWG(v, t)
        ot = Octree(v, m.midpoints(), leaf=0.25)
        Zd = efie.z_block(m, np.arange(m.n), np.arange(m.n))
        for r in (0, m.n // 2, m.n - 1):
            a = ot.rwg_leaf[r]
            cols = np.concatenate([ot.leaf_rwgs[b] for b in ot.near[a]])
            z = nesa.near_entries(fr, nr, [r + ptr[i]], cols + ptr[i])[0]
            assert np.abs(z - Zd[r, cols]).max() <= 1e-13 * np.abs(Zd[r, cols]).max()
        # no entry couples two bodies
        other = ptr[1 - i] + np.arange(5)
        assert np.all(nesa.near_entries(fr, nr, [ptr[i]], other)[0] == 0)
