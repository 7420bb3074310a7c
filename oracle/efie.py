"""Dense Galerkin EFIE with RWG basis functions (plain FP64 reference).

Follows Sec. 2 of the paper: the field radiated by a surface current (Eq. 1,
Green's function exp(-ikR)/(4 pi R), so the time convention is exp(+i w t)),
expansion of the current in basis functions, and Galerkin testing (Eq. 2),
which gives Z j = b with Z_mn the tested field of basis n (Eq. 3).

Readings taken where the paper is silent:

* basis: Rao-Wilton-Glisson functions on the interior edges of a closed
  triangle mesh.  Edges are numbered in increasing (min vertex, max vertex)
  order; the plus triangle is the lower-index one of the two sharing the edge.
* right-hand side sign: the tested null-field condition of Eq. (2) is taken as
  written, so b_m = -<e_inc, phi_m> and Z j = b (the sign of Eq. (3)'s vector is
  inconsistent with Eq. (2); the null-field test pins this choice).
* quadrature: the 3-point interior rule (barycentric 2/3, 1/6, 1/6, weights
  area/3) on every triangle.
* the gradient in Eq. (1) is moved onto the test function by the surface
  divergence theorem (closed surface), giving the mixed-potential kernel
  phi_m . phi_n - k^-2 div(phi_m) div(phi_n).
* singular triangle pairs (sharing at least one vertex): the inner integral is
  split into the smooth part (exp(-ikR)-1)/(4 pi R) on the 3-point rule and the
  static part 1/(4 pi R) integrated in closed form (Wilton et al. 1984;
  Graglia 1993); the pair integral is the mean of both integration orders, so
  Z = Z^T holds to rounding.
"""
import math

import numpy as np
import scipy.sparse as sp

ETA0 = 376.730313668          # free-space impedance mu0*c (ohm)
K0 = 2.0 * math.pi            # wavenumber for lengths measured in wavelengths

# barycentric weights of the 3-point interior rule
_BARY = np.array([[2.0 / 3, 1.0 / 6, 1.0 / 6],
                  [1.0 / 6, 2.0 / 3, 1.0 / 6],
                  [1.0 / 6, 1.0 / 6, 2.0 / 3]])


class RWG:
    """RWG functions of a closed mesh.

    Attributes (N = number of interior edges):
      edge[N,2]      vertex ids (min, max)
      tri[N,2]       (T+, T-) triangle ids, T+ < T-
      free[N,2]      free vertex of T+ and of T-
      length[N]      edge length
      area[nt]       triangle areas
      tri_rwg[nt,3]  RWG attached to the edge opposite local vertex a of each triangle
      tri_sign[nt,3] +1 if the triangle is that RWG's T+, -1 if T-
    On T+: phi = l/(2A+) (r - p+), div = +l/A+;  on T-: phi = l/(2A-) (p- - r), div = -l/A-.
    """

    def __init__(self, verts, tris):
        v = np.asarray(verts, dtype=np.float64)
        t = np.asarray(tris, dtype=np.int64)
        self.verts, self.tris = v, t
        nt = len(t)
        edges = {}
        for ti in range(nt):
            for a in range(3):
                e = (int(t[ti, (a + 1) % 3]), int(t[ti, (a + 2) % 3]))
                key = (min(e), max(e))
                edges.setdefault(key, []).append((ti, a))
        bad = [k for k, x in edges.items() if len(x) != 2]
        if bad:
            raise ValueError("mesh is not a closed 2-manifold (%d bad edges)" % len(bad))
        keys = sorted(edges)
        n = len(keys)
        self.edge = np.array(keys, dtype=np.int64)
        self.tri = np.zeros((n, 2), dtype=np.int64)
        self.free = np.zeros((n, 2), dtype=np.int64)
        self.tri_rwg = np.full((nt, 3), -1, dtype=np.int64)
        self.tri_sign = np.zeros((nt, 3))
        for i, key in enumerate(keys):
            (t0, a0), (t1, a1) = sorted(edges[key])
            self.tri[i] = (t0, t1)
            self.free[i] = (t[t0, a0], t[t1, a1])
            self.tri_rwg[t0, a0], self.tri_sign[t0, a0] = i, 1.0
            self.tri_rwg[t1, a1], self.tri_sign[t1, a1] = i, -1.0
        self.length = np.linalg.norm(v[self.edge[:, 0]] - v[self.edge[:, 1]], axis=1)
        cr = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / (2.0 * self.area[:, None])
        self.n = n
        # quadrature points [nt,3,3] and weights [nt,3]
        self.qp = np.einsum("qa,tad->tqd", _BARY, v[t])
        self.qw = np.repeat(self.area[:, None] / 3.0, 3, axis=1)
        # incidence (3*nt x N): local function (t, a) -> RWG, with the vector and
        # divergence coefficients  s l/(2A)  and  s l/A
        rows = (3 * np.arange(nt)[:, None] + np.arange(3)[None, :]).ravel()
        cols = self.tri_rwg.ravel()
        lv = self.length[cols] * self.tri_sign.ravel()
        a_ = np.repeat(self.area, 3)
        self.inc_vec = sp.csr_matrix((lv / (2 * a_), (rows, cols)), shape=(3 * nt, n))
        self.inc_div = sp.csr_matrix((lv / a_, (rows, cols)), shape=(3 * nt, n))

    def midpoints(self):
        return 0.5 * (self.verts[self.edge[:, 0]] + self.verts[self.edge[:, 1]])

    def values_at_quad(self, n):
        """phi_n and div phi_n at the 6 quadrature points of RWG n.
        Returns points [6,3], weights [6], phi [6,3], div [6]."""
        pts, w, ph, dv = [], [], [], []
        for side in range(2):
            ti = self.tri[n, side]
            s = 1.0 if side == 0 else -1.0
            p = self.verts[self.free[n, side]]
            A = self.area[ti]
            for q in range(3):
                r = self.qp[ti, q]
                pts.append(r)
                w.append(self.qw[ti, q])
                ph.append(s * self.length[n] / (2 * A) * (r - p))
                dv.append(s * self.length[n] / A)
        return np.array(pts), np.array(w), np.array(ph), np.array(dv)


def green(R, k=K0):
    """Free-space Green's function exp(-ikR)/(4 pi R) (Sec. 2, after Eq. 1)."""
    return np.exp(-1j * k * R) / (4.0 * math.pi * R)


def green_smooth(R, k=K0):
    """(exp(-ikR) - 1)/(4 pi R), with its limit -ik/(4 pi) at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape, dtype=np.complex128)
    small = R < 1e-12
    Rs = np.where(small, 1.0, R)
    out[...] = np.expm1(-1j * k * Rs) / (4.0 * math.pi * Rs)
    out[small] = -1j * k / (4.0 * math.pi)
    return out


def potential_integrals(r, tv):
    """Closed-form static integrals over flat triangles.

    r: observation points [n,3]; tv: triangle vertices [3,3] (one triangle for
    all points) or [n,3,3] (one triangle per point).
    Returns (I1 [n], Irho [n,3]) with
      I1   = int_T 1/|r - r'| dS'
      Irho = int_T (rho' - rho)/|r - r'| dS',   rho = projection of r on the plane.
    Wilton et al. (1984) / Graglia (1993) line-integral forms.
    """
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    tv = np.asarray(tv, dtype=np.float64)
    if tv.ndim == 2:
        tv = np.broadcast_to(tv, (len(r), 3, 3))
    n_hat = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    n_hat /= np.linalg.norm(n_hat, axis=1, keepdims=True)
    h = np.einsum("nd,nd->n", r - tv[:, 0], n_hat)
    rho = r - h[:, None] * n_hat
    ah = np.abs(h)
    I1 = np.zeros(len(r))
    Irho = np.zeros((len(r), 3))
    for i in range(3):
        pm, pp = tv[:, i], tv[:, (i + 1) % 3]
        lhat = (pp - pm) / np.linalg.norm(pp - pm, axis=1, keepdims=True)
        uhat = np.cross(lhat, n_hat)
        lp = np.einsum("nd,nd->n", pp - rho, lhat)
        lm = np.einsum("nd,nd->n", pm - rho, lhat)
        P0 = np.einsum("nd,nd->n", pp - rho, uhat)
        R0sq = P0 * P0 + h * h
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)

        def log_arg(R, l):
            # R + l, computed without cancellation when l < 0
            return np.where(l >= 0, R + l, R0sq / np.where(R - l > 0, R - l, 1.0))

        with np.errstate(divide="ignore", invalid="ignore"):
            Lg = np.log(log_arg(Rp, lp)) - np.log(log_arg(Rm, lm))
        Lg = np.where(R0sq > 1e-30, Lg, 0.0)
        at = np.arctan2(P0 * lp, R0sq + ah * Rp) - np.arctan2(P0 * lm, R0sq + ah * Rm)
        I1 += P0 * Lg - ah * at
        Irho += 0.5 * (R0sq * Lg + lp * Rp - lm * Rm)[:, None] * uhat
    return I1, Irho


def _share_vertex(t, ta, tb):
    A = t[ta]
    B = t[tb]
    return (A[:, :, None] == B[:, None, :]).any(axis=(1, 2))


def _pair_integrals(m, ta, tb, k):
    """Local integrals for triangle pairs (ta[i], tb[i]).

    Returns Avec [n,3,3] = int_Ta int_Tb (r - va).(r' - vb) g  and
            B    [n]     = int_Ta int_Tb g,
    where va, vb run over the local vertices of each triangle.
    """
    v, t = m.verts, m.tris
    ra, wa = m.qp[ta], m.qw[ta]          # [n,3,3], [n,3]
    rb, wb = m.qp[tb], m.qw[tb]
    va, vb = v[t[ta]], v[t[tb]]          # [n,3(vertex),3]
    d = ra[:, :, None, :] - rb[:, None, :, :]
    R = np.linalg.norm(d, axis=-1)       # [n,i,j]
    sing = _share_vertex(t, ta, tb)
    G = np.zeros_like(R, dtype=np.complex128)
    reg = ~sing
    G[reg] = green(R[reg], k)
    W = wa[:, :, None] * wb[:, None, :] * G                        # [n,i,j]
    B = W.sum(axis=(1, 2))
    # (r_i - va).(r'_j - vb) = r_i.r'_j - r_i.vb - va.r'_j + va.vb
    rr = np.matmul(ra, rb.transpose(0, 2, 1))                      # [n,i,j]
    rvb = np.matmul(ra, vb.transpose(0, 2, 1))                     # [n,i,b]
    var = np.matmul(va, rb.transpose(0, 2, 1))                     # [n,a,j]
    vv = np.matmul(va, vb.transpose(0, 2, 1))                      # [n,a,b]
    wi = W.sum(axis=2)                                             # [n,i]
    wj = W.sum(axis=1)                                             # [n,j]
    Avec = ((W * rr).sum(axis=(1, 2))[:, None, None]
            - np.matmul(wi[:, None, :], rvb)
            - np.matmul(var, wj[:, :, None])
            + B[:, None, None] * vv)
    si = np.nonzero(sing)[0]
    if len(si):
        a1, b1 = _singular_pairs(m, ta[si], tb[si], k)
        a2, b2 = _singular_pairs(m, tb[si], ta[si], k)
        Avec[si] = 0.5 * (a1 + a2.transpose(0, 2, 1))
        B[si] = 0.5 * (b1 + b2)
    return Avec, B


def _singular_pairs(m, ta, tb, k):
    """Outer 3-point rule on ta[n], inner integral over tb[n] with the static
    part in closed form.  Returns (Avec [n,3,3], B [n])."""
    v, t = m.verts, m.tris
    ra, wa = m.qp[ta], m.qw[ta]                    # [n,i,3], [n,i]
    rb, wb = m.qp[tb], m.qw[tb]
    va, vb = v[t[ta]], v[t[tb]]                    # [n,a,3]
    n = len(ta)
    R = np.linalg.norm(ra[:, :, None, :] - rb[:, None, :, :], axis=-1)   # [n,i,j]
    Gs = green_smooth(R, k)
    tvb = np.repeat(vb, 3, axis=0)                 # triangle per outer point
    I1, Irho = potential_integrals(ra.reshape(-1, 3), tvb)
    I1 = I1.reshape(n, 3)
    Irho = Irho.reshape(n, 3, 3)
    nb = m.normal[tb]
    h = np.einsum("nid,nd->ni", ra - vb[:, :1, :], nb)
    rho = ra - h[:, :, None] * nb[:, None, :]
    inv4pi = 1.0 / (4.0 * math.pi)
    Gw = Gs * wb[:, None, :]                                           # [n,i,j]
    Jg = Gw.sum(axis=2) + inv4pi * I1                                 # [n,i]
    # Jv[n,i,b,:] = int (r' - vb_b) g(r_i, r') dr'
    Jv = (np.einsum("nij,njd->nid", Gw, rb)[:, :, None, :]
          - Gw.sum(axis=2)[:, :, None, None] * vb[:, None, :, :]
          + inv4pi * (Irho[:, :, None, :]
                      + (rho[:, :, None, :] - vb[:, None, :, :]) * I1[:, :, None, None]))
    Avec = np.einsum("ni,niad,nibd->nab", wa, ra[:, :, None, :] - va[:, None, :, :], Jv)
    Bv = (wa * Jg).sum(axis=1)
    return Avec, Bv


def triangle_block(m, ta, tb, k=K0, eta=ETA0):
    """Local-function interaction matrix between triangle sets ta and tb:
    returns a dense (3|ta| x 3|tb|) complex array M with
      M[(a,i),(b,j)] = -i eta k [ cv_a cv_b Avec - k^-2 cd_a cd_b B ]
    still without the RWG coefficients (applied by the incidence matrices)."""
    ta = np.asarray(ta)
    tb = np.asarray(tb)
    TA, TB = np.meshgrid(ta, tb, indexing="ij")
    Avec, B = _pair_integrals(m, TA.ravel(), TB.ravel(), k)
    na, nb = len(ta), len(tb)
    Avec = Avec.reshape(na, nb, 3, 3).transpose(0, 2, 1, 3).reshape(3 * na, 3 * nb)
    Bm = np.repeat(np.repeat(B.reshape(na, nb), 3, axis=0), 3, axis=1)
    return Avec, Bm


def z_block(m, rows, cols, k=K0, eta=ETA0, chunk=400):
    """Z[rows][:, cols] (Sec. 2, Eq. 3) by the triangle-pair rule."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    tr = np.unique(m.tri[rows].ravel())
    tc = np.unique(m.tri[cols].ravel())
    loc_r = (3 * tr[:, None] + np.arange(3)[None, :]).ravel()
    loc_c = (3 * tc[:, None] + np.arange(3)[None, :]).ravel()
    Ev_r = m.inc_vec[loc_r][:, rows].tocsc()
    Ed_r = m.inc_div[loc_r][:, rows].tocsc()
    Ev_c = m.inc_vec[loc_c][:, cols].tocsr()
    Ed_c = m.inc_div[loc_c][:, cols].tocsr()
    Z = np.zeros((len(rows), len(cols)), dtype=np.complex128)
    for i0 in range(0, len(tr), chunk):
        sl = slice(i0, i0 + chunk)
        Av, Bm = triangle_block(m, tr[sl], tc, k)
        rs = slice(3 * i0, 3 * i0 + 3 * len(tr[sl]))
        er, dr = Ev_r[rs].T.tocsr(), Ed_r[rs].T.tocsr()
        Z += (er @ (Ev_c.T @ Av.T).T) - (1.0 / k ** 2) * (dr @ (Ed_c.T @ Bm.T).T)
    return -1j * eta * k * Z


def dense_z(m, k=K0, eta=ETA0):
    """Full dense Z (N x N)."""
    idx = np.arange(m.n)
    return z_block(m, idx, idx, k, eta)


def plane_wave_rhs(m, khat, pol, k=K0):
    """b_m = -int e_inc . phi_m,  e_inc = pol exp(-ik khat.r)  (Sec. 2, Eq. 2)."""
    khat = np.asarray(khat, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    t = m.tris
    ph = np.exp(-1j * k * (m.qp @ khat))                 # [nt,3]
    # per local function (t,a): int (r - v_a).pol e dS
    va = m.verts[t]                                      # [nt,3,3]
    rp = m.qp @ pol                                      # [nt,q]
    vp = va @ pol                                        # [nt,a]
    loc = (m.qw * ph * rp).sum(axis=1)[:, None] - (m.qw * ph).sum(axis=1)[:, None] * vp
    return -(m.inc_vec.T @ loc.ravel())


def current_at_quad(m, j):
    """Surface current J = sum_n j_n phi_n at all quadrature points: [nt,3,3]."""
    t = m.tris
    va = m.verts[t]                                      # [nt,a,3]
    coef = (m.inc_vec @ j).reshape(-1, 3)                # [nt,a]
    # J(r) = sum_a coef_a (r - v_a)
    return coef.sum(axis=1)[:, None, None] * m.qp - np.einsum("ta,tad->td", coef, va)[:, None, :]


def charge_at_quad(m, j):
    """Surface divergence of the current, constant per triangle: [nt]."""
    return (m.inc_div @ j).reshape(-1, 3).sum(axis=1)


def scattered_field(m, j, pts, k=K0, eta=ETA0):
    """e_s(j)(r) of Sec. 2, Eq. (1) at points off the surface, 3-point rule."""
    J = current_at_quad(m, j).reshape(-1, 3)
    rho = np.repeat(charge_at_quad(m, j), 3)
    w = m.qw.ravel()
    rq = m.qp.reshape(-1, 3)
    out = np.zeros((len(pts), 3), dtype=np.complex128)
    for i, r in enumerate(np.asarray(pts)):
        d = r[None, :] - rq
        R = np.linalg.norm(d, axis=1)
        g = green(R, k)
        grad = (-(1.0 + 1j * k * R) / R ** 2 * g)[:, None] * d   # grad_r g
        out[i] = -1j * eta * k * ((w * g) @ J + (1.0 / k ** 2) * ((w * rho) @ grad))
    return out


def far_field(m, j, rhat, k=K0, eta=ETA0):
    """Far-field pattern F(rhat) with e_s ~ F exp(-ikr)/r:
    F = -i eta k/(4 pi) int [J - rhat (rhat.J)] exp(ik rhat.r') dS'."""
    J = current_at_quad(m, j).reshape(-1, 3)
    w = m.qw.ravel()
    rq = m.qp.reshape(-1, 3)
    out = np.zeros((len(rhat), 3), dtype=np.complex128)
    for i, u in enumerate(np.asarray(rhat)):
        ph = np.exp(1j * k * (rq @ u)) * w
        v = ph @ J
        out[i] = -1j * eta * k / (4 * math.pi) * (v - u * (u @ v))
    return out
