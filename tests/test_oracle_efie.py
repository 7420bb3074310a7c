"""Pins of the dense EFIE oracle (Sec. 2, Eq. 1-3) against mathematics and the
exact Mie solution, not against itself."""
import math

import numpy as np
import pytest

import synth
from oracle import efie, mie


def test_three_point_rule_exact_for_quadratics():
    # int over the unit right triangle of x^a y^b = a! b! / (a+b+2)!
    tv = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    m = efie.RWG(*synth.icosphere(1, 1.0))      # any mesh, only to reach the rule
    qp = efie._BARY @ tv
    w = np.full(3, 0.5 / 3)
    for a in range(3):
        for b in range(3 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs((w * qp[:, 0] ** a * qp[:, 1] ** b).sum() - exact) < 1e-15
    assert m.n == 30


def test_rwg_charge_neutral_and_continuous(rwg1):
    m = rwg1
    # total charge of every RWG vanishes: sum over its two triangles of div * area
    q = np.asarray((m.inc_div.multiply(np.repeat(m.area, 3)[:, None])).sum(axis=0)).ravel()
    assert np.abs(q).max() < 1e-12 * np.abs(m.length).max()
    # normal component of phi_n continuous across its edge: at the edge midpoint
    # both halves give l/(2A) * distance-to-edge-line * ... = 1 (unit normal flux)
    v = m.verts
    for n in range(0, m.n, 97):
        mid = 0.5 * (v[m.edge[n, 0]] + v[m.edge[n, 1]])
        fl = []
        for side in range(2):
            tpos = m.tri[n, side]
            p = v[m.free[n, side]]
            s = 1.0 if side == 0 else -1.0
            phi = s * m.length[n] / (2 * m.area[tpos]) * (mid - p)
            e = v[m.edge[n, 1]] - v[m.edge[n, 0]]
            nrm = np.cross(m.normal[tpos], e)
            nrm /= np.linalg.norm(nrm)
            if nrm @ (mid - p) < 0:
                nrm = -nrm
            fl.append(phi @ nrm * (1 if side == 0 else -1))
        assert abs(fl[0] - 1.0) < 1e-12 and abs(fl[1] - 1.0) < 1e-12


def _brute_static(r, tv, lev=7):
    n = 2 ** lev
    A = 0.5 * np.linalg.norm(np.cross(tv[1] - tv[0], tv[2] - tv[0]))
    nh = np.cross(tv[1] - tv[0], tv[2] - tv[0]) / (2 * A)
    rho = r - ((r - tv[0]) @ nh) * nh
    pts = []
    for i in range(n):
        for j in range(n - i):
            P = lambda u, v: tv[0] + (tv[1] - tv[0]) * u / n + (tv[2] - tv[0]) * v / n
            sub = [(P(i, j), P(i + 1, j), P(i, j + 1))]
            if i + j + 2 <= n:
                sub.append((P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)))
            for s_ in sub:
                pts.append(efie._BARY @ np.array(s_))
    pts = np.concatenate(pts)
    w = A / n / n / 3
    R = np.linalg.norm(pts - r, axis=1)
    return (w / R).sum(), ((w / R)[:, None] * (pts - rho)).sum(0)


@pytest.mark.parametrize("r", [(0.3, 0.3, 0.5), (2.0, 1.0, 0.3), (-0.5, 0.2, 0.0),
                               (1.5, -0.3, 0.01), (0.2, 0.2, -0.7)])
def test_static_integrals_closed_form_vs_quadrature(r):
    tv = np.array([[0.0, 0, 0], [1.0, 0.1, 0], [0.3, 0.9, 0.05]])
    r = np.array(r)
    I1, Ir = efie.potential_integrals(r[None], tv)
    b1, br = _brute_static(r, tv)
    assert abs(I1[0] - b1) < 1e-8 * abs(b1)
    assert np.abs(Ir[0] - br).max() < 1e-8 * np.abs(br).max()


def test_z_reciprocal(dense1):
    Z = dense1
    assert np.abs(Z - Z.T).max() <= 1e-13 * np.abs(Z).max()


def test_z_regular_entries_by_direct_loops():
    """Entries of well-separated RWG pairs re-evaluated by plain loops over the
    six quadrature points of each function."""
    v, t = synth.icosphere(2, 1.0)
    m = efie.RWG(v, t)
    Z = efie.dense_z(m)
    k, eta = efie.K0, efie.ETA0
    shared = lambda a, b: bool(set(m.tris[m.tri[a]].ravel()) & set(m.tris[m.tri[b]].ravel()))
    checked = 0
    for a in range(0, m.n, 7):
        for b in range(0, m.n, 5):
            if shared(a, b):
                continue
            pa, wa, fa, da = m.values_at_quad(a)
            pb, wb, fb, db = m.values_at_quad(b)
            acc = 0j
            for i in range(6):
                for j in range(6):
                    R = np.linalg.norm(pa[i] - pb[j])
                    g = np.exp(-1j * k * R) / (4 * math.pi * R)
                    acc += wa[i] * wb[j] * (fa[i] @ fb[j] - da[i] * db[j] / k ** 2) * g
            assert abs(-1j * eta * k * acc - Z[a, b]) <= 1e-12 * np.abs(Z).max()
            checked += 1
    assert checked > 50


def test_null_field_inside_sphere(rwg1, dense1):
    """PEC: the total field vanishes inside the closed surface (pins the RHS sign)."""
    b = efie.plane_wave_rhs(rwg1, [0, 0, 1], [1, 0, 0])
    j = np.linalg.solve(dense1, b)
    pts = np.array([[0, 0, 0], [0.1, 0.1, 0], [0, -0.2, 0.1], [0.25, 0, 0], [0, 0, -0.3]])
    es = efie.scattered_field(rwg1, j, pts)
    ei = np.array([1.0, 0, 0])[None, :] * np.exp(-1j * efie.K0 * pts[:, 2])[:, None]
    rel = np.linalg.norm(es + ei, axis=1) / np.linalg.norm(ei, axis=1)
    assert rel.max() < 1e-3


def test_far_field_matches_mie(rwg1, dense1):
    """Complex far field of the dense solution vs the Mie series (E- and H-plane)."""
    b = efie.plane_wave_rhs(rwg1, [0, 0, 1], [1, 0, 0])
    j = np.linalg.solve(dense1, b)
    th = np.linspace(0.01, math.pi - 0.01, 37)
    for phi in (0.0, math.pi / 2):
        rh = np.stack([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)], 1)
        F = efie.far_field(rwg1, j, rh)
        Fm = mie.far_field(th, phi, 0.5)
        assert np.linalg.norm(F - Fm) / np.linalg.norm(Fm) < 0.02


def test_mie_small_sphere_rayleigh_limit():
    """ka -> 0: PEC backscatter RCS -> 9 pi a^2 (ka)^4 (Rayleigh)."""
    a = 0.01
    F = mie.far_field(np.array([math.pi]), 0.0, a)
    sigma = 4 * math.pi * np.linalg.norm(F[0]) ** 2
    ka = efie.K0 * a
    assert abs(sigma / (9 * math.pi * a * a * ka ** 4) - 1) < 1e-2
