"""Stated NESA truncation error of the benchmark operators: the library's
product against seeded rows of the dense Galerkin EFIE matrix (Sec. 2, Eq. 1-3)
times a seeded vector, stored in ``tests/golden/dense_rows_*.json`` by
``tests/golden/make_dense_rows.py`` (oracle only).

This is the second tier of parity: the GPU product matches the oracle's NESA
product to round-off (the other GPU tests), and NESA itself stays within its
truncation error of the dense matrix (these).  The bounds are the measured
errors rounded up; they are properties of the operator (equivalent sources per
box, one-box buffer), not of the GPU arithmetic."""
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_dense_rows as golden  # noqa: E402

# ||(Z_NESA x)[rows] - (Z x)[rows]|| / ||(Z x)[rows]||, d0 = 3, leaf 0.25,
# complex64 on the GPU
ERR_SPHERE201720 = 3e-3        # measured 2.05e-3 (levels 2..5, Q = 441/196/81/49)
# bodies 0-3 of the uneven family in one forest (shared leaf radius 0.263):
# the oracle's errors on these rows are 4.18e-3, 2.63e-3, 3.65e-3, 1.17e-3
ERR_BODY4 = [5e-3, 3e-3, 4e-3, 1.5e-3]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def nesa():
    from paper_1801_03589_amd import nesa as n
    n.lib()
    return n


def _err(y, yd):
    return np.linalg.norm(y - yd) / np.linalg.norm(yd)


def test_bench_sphere_vs_dense_rows(torch_dev, nesa):
    """The benchmark operator exactly as bench.py builds it (near field
    assembled on the device, d0 = 3, complex64)."""
    torch = torch_dev
    mesh, n, rows, yd = golden.load("sphere201720")
    v, t = eval(mesh, {"synth": synth})
    tr = nesa.build_tree(v, t, 0.25)
    op = nesa.op_create(tr, nesa.assemble_near_device(tr), nesa.assemble_translations(tr, d0=3, tau=1e-8),
                        nesa.C64)
    assert tr.info()["n_rwg"] == n
    xd = torch.from_numpy(synth.complex_normal(n, 0)).to(torch.complex64).cuda()
    yg = torch.empty_like(xd)
    nesa.matvec(op, xd, yg)
    torch.cuda.synchronize()
    e = _err(yg.cpu().numpy().astype(np.complex128)[rows], yd)
    print("sphere N=%d: %d dense rows, NESA truncation error %.3e" % (n, len(rows), e))
    assert e <= ERR_SPHERE201720


def test_uneven_bodies_vs_dense_rows(torch_dev, nesa):
    """Bodies 0-3 of the uneven family as one forest (the batched form): each
    body's rows against its own dense matrix."""
    torch = torch_dev
    cases = ["body4_%d" % i for i in range(4)]
    meshes, xs, fx = [], [], []
    for c in cases:
        mesh, n, rows, yd = golden.load(c)
        v, t = eval(mesh, {"synth": synth})
        meshes.append((v, t))
        xs.append(synth.complex_normal(n, int(golden.CASES[c][3])))
        fx.append((rows, yd))
    fr = nesa.build_forest(meshes, 0.25)
    op = nesa.op_create(fr, nesa.assemble_near_device(fr), nesa.assemble_translations(fr, d0=3, tau=1e-8),
                        nesa.C64)
    ptr = fr.bodies()
    xd = torch.from_numpy(np.concatenate(xs)).to(torch.complex64).cuda()
    yg = torch.empty_like(xd)
    nesa.matvec(op, xd, yg)
    torch.cuda.synchronize()
    y = yg.cpu().numpy().astype(np.complex128)
    for i, (rows, yd) in enumerate(fx):
        e = _err(y[ptr[i]:ptr[i + 1]][rows], yd)
        print("body %d (N=%d): %d dense rows, NESA truncation error %.3e" % (i, ptr[i + 1] - ptr[i], len(rows), e))
        assert e <= ERR_BODY4[i]
