"""Seeded closed triangle meshes (lengths in wavelengths).

Every generator returns ``(verts, tris)``: ``verts`` float64 [nv, 3] and
``tris`` int32 [nt, 3], each triangle ordered counter-clockwise when seen
from outside, every edge shared by exactly two triangles (closed 2-manifold
surfaces, possibly of several components).

Two constructions are used:

* a geodesic icosphere of frequency ``nu`` (each icosahedron face split into
  ``nu**2`` triangles, vertices projected to the sphere): 20 nu^2 triangles,
  30 nu^2 edges;
* a structured cube surface whose lattice is mapped onto a box, a spheroid or a
  capped cylinder, used for the uneven body families and the aircraft-like body.

Vertices shared between faces are generated once from an exact integer key,
so no floating-point de-duplication is involved.
"""
import math

import numpy as np


# --------------------------------------------------------------------------- icosphere
def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def icosphere(nu, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Geodesic icosphere of frequency ``nu`` (20 nu^2 triangles, 30 nu^2 edges)."""
    if nu < 1:
        raise ValueError("nu must be >= 1")
    base, faces = _icosahedron()
    keys = {}
    pos = []

    def vid(key, p):
        i = keys.get(key)
        if i is None:
            i = len(pos)
            keys[key] = i
            pos.append(p)
        return i

    def point(face, a, b):
        # integer barycentric weights (nu-a-b, a, b) on the face corners
        c0, c1, c2 = (int(x) for x in face)
        w = {c0: nu - a - b, c1: a, c2: b}
        nz = sorted(k for k, x in w.items() if x > 0)
        if len(nz) == 1:
            key = ("v", nz[0])
        elif len(nz) == 2:
            key = ("e", nz[0], nz[1], w[nz[0]])
        else:
            key = ("f", c0, c1, c2, a, b)
        p = sum(w[k] * base[k] for k in nz) / nu
        return vid(key, p)

    tris = []
    for face in faces:
        idx = {}
        for a in range(nu + 1):
            for b in range(nu + 1 - a):
                idx[a, b] = point(face, a, b)
        for a in range(nu):
            for b in range(nu - a):
                tris.append((idx[a, b], idx[a + 1, b], idx[a, b + 1]))
                if a + b + 2 <= nu:
                    tris.append((idx[a + 1, b], idx[a + 1, b + 1], idx[a, b + 1]))
    v = np.array(pos)
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * radius + np.asarray(center)
    return v, np.array(tris, dtype=np.int32)


# --------------------------------------------------------------------------- cube lattice
def _cube_lattice(n):
    """Surface of the integer lattice box [0,nx]x[0,ny]x[0,nz]: (int coords, outward tris)."""
    n = [int(x) for x in n]
    keys = {}
    pts = []

    def vid(p):
        i = keys.get(p)
        if i is None:
            i = len(pts)
            keys[p] = i
            pts.append(p)
        return i

    tris = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (0, 1):
            for i in range(n[b]):
                for j in range(n[c]):
                    quad = []
                    for (di, dj) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0, 0, 0]
                        p[a] = side * n[a]
                        p[b] = i + di
                        p[c] = j + dj
                        quad.append(vid(tuple(p)))
                    q0, q1, q2, q3 = quad
                    # alternate the diagonal so the lattice has no preferred direction
                    if (i + j) % 2 == 0:
                        t1, t2 = (q0, q1, q2), (q0, q2, q3)
                    else:
                        t1, t2 = (q0, q1, q3), (q1, q2, q3)
                    if side == 0:  # inward-facing lattice normal -> flip
                        t1, t2 = t1[::-1], t2[::-1]
                    tris.extend([t1, t2])
    u = np.array(pts, dtype=np.float64) / np.array(n, dtype=np.float64) * 2.0 - 1.0
    return u, np.array(tris, dtype=np.int32)


def _equal_angle(u):
    return np.tan(u * (math.pi / 4.0))


def box_mesh(size, h, center=(0.0, 0.0, 0.0)):
    """Closed box of side lengths ``size`` with edge length about ``h``."""
    size = np.asarray(size, dtype=np.float64)
    n = np.maximum(1, np.ceil(size / h)).astype(int)
    u, t = _cube_lattice(n)
    return u * (size / 2.0) + np.asarray(center), t


def spheroid(semi_axes, h, center=(0.0, 0.0, 0.0)):
    """Closed ellipsoid with the given semi-axes, edge length about ``h``."""
    s = np.asarray(semi_axes, dtype=np.float64)
    # a quarter of a great-circle per cube face side
    n = np.maximum(2, np.ceil(np.pi * s / 2.0 / h)).astype(int)
    u, t = _cube_lattice(n)
    w = _equal_angle(u)
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    return w * s + np.asarray(center), t


def capped_cylinder(radius, length, h, center=(0.0, 0.0, 0.0)):
    """Closed cylinder along x (radius, length) with flat caps, edge length about ``h``."""
    nx = max(1, int(math.ceil(length / h)))
    nr = max(2, int(math.ceil(math.pi * radius / 2.0 / h)))
    u, t = _cube_lattice((nx, nr, nr))
    yz = _equal_angle(u[:, 1:])
    m = np.max(np.abs(u[:, 1:]), axis=1)
    r = np.linalg.norm(yz, axis=1)
    scale = np.where(r > 0, m / np.where(r > 0, r, 1.0), 0.0)
    out = np.empty_like(u)
    out[:, 0] = u[:, 0] * (length / 2.0)
    out[:, 1:] = yz * scale[:, None] * radius
    return out + np.asarray(center), t


def _vertex_normals(v, t):
    n = np.zeros_like(v)
    fn = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    for k in range(3):
        np.add.at(n, t[:, k], fn)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _merge(parts):
    vs, ts, off = [], [], 0
    for v, t in parts:
        vs.append(v)
        ts.append(t + off)
        off += len(v)
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32)


def _wing(root_x, root_y, span, chord_root, chord_tip, sweep_deg, thickness, h, side):
    """Thin tapered swept slab attached (with a gap) at y = root_y, extending along +-y."""
    n = (max(1, int(math.ceil(chord_root / h))), max(1, int(math.ceil(span / h))),
         max(1, int(math.ceil(thickness / h))))
    u, t = _cube_lattice(n)
    s = (u[:, 1] + 1.0) / 2.0                      # 0 at root, 1 at tip
    chord = chord_root + (chord_tip - chord_root) * s
    x = root_x + s * span * math.tan(math.radians(sweep_deg)) + (u[:, 0] + 1.0) / 2.0 * chord
    y = root_y + s * span
    z = u[:, 2] * thickness / 2.0
    v = np.stack([x, side * y, z], axis=1)
    if side < 0:  # mirroring flips the orientation
        t = t[:, ::-1]
    return v, np.ascontiguousarray(t)


def aircraft_like(seed=3, h=1.0 / 17.0, fuselage_radius=2.0, fuselage_length=50.0,
                  span=15.0, chord_root=7.0, chord_tip=3.0, sweep_deg=30.0,
                  thickness=0.3, wing_x=20.0, gap=0.05, noise=0.02):
    """Elongated aircraft-like body: capped-cylinder fuselage along x plus two swept
    tapered wing slabs separated from it by a small gap (every component closed).
    Vertex noise of standard deviation ``noise`` is applied along vertex normals."""
    rng = np.random.default_rng(seed)
    parts = [capped_cylinder(fuselage_radius, fuselage_length, h,
                             center=(fuselage_length / 2.0, 0.0, 0.0))]
    for side in (1, -1):
        parts.append(_wing(wing_x, fuselage_radius + gap, span, chord_root, chord_tip,
                           sweep_deg, thickness, h, side))
    out = []
    for v, t in parts:
        nrm = _vertex_normals(v, t)
        amp = rng.normal(0.0, noise, size=len(v))
        out.append((v + nrm * amp[:, None], t))
    return _merge(out)


def body_family(n_bodies, seed=4, n_min=2000, n_max=50000, density=1000.0):
    """Uneven bodies: type in {spheroid, cube, cylinder}, unknown count log-uniform in
    [n_min, n_max], aspect ratio in [1, 3].  Body i uses seed ``seed*1000 + i``.
    Returns a list of (verts, tris, kind)."""
    bodies = []
    for i in range(n_bodies):
        rng = np.random.default_rng(seed * 1000 + i)
        kind = ("spheroid", "cube", "cylinder")[int(rng.integers(0, 3))]
        n_target = float(np.exp(rng.uniform(math.log(n_min), math.log(n_max))))
        aspect = float(rng.uniform(1.0, 3.0))
        area = n_target / density          # wavelengths^2
        # RWG count ~ 1.5 * triangles, triangle area ~ sqrt(3)/4 h^2
        h = math.sqrt(area / (n_target / 1.5) * 4.0 / math.sqrt(3.0))
        if kind == "spheroid":
            # area of a prolate spheroid approximated by 4 pi a^p... use ellipsoid estimate
            b = math.sqrt(area / (4.0 * math.pi * ((aspect ** 1.6 + 2 * aspect ** 0.8) / 3.0) ** (1 / 1.6)))
            v, t = spheroid((aspect * b, b, b), h)
        elif kind == "cube":
            b = math.sqrt(area / (2.0 + 4.0 * aspect))
            v, t = box_mesh((aspect * b, b, b), h)
        else:
            r = math.sqrt(area / (2.0 * math.pi * (1.0 + 2.0 * aspect)))
            v, t = capped_cylinder(r, 2.0 * aspect * r, h)
        bodies.append((v, t, kind))
    return bodies
