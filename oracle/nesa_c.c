/* Plain FP64 NESA product on the CPU, in C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the CPU baseline of the
 * benchmark and the tests call it; the product library never does.  It is a
 * second, loop-level form of the NumPy oracle (oracle/nesa.py, oracle/efie.py),
 * pinned against it on small meshes (tests/test_oracle_c.py), fast enough to
 * run the whole product of the large workloads on the host's cores.
 *
 * What it computes, with the paper's notation:
 *   near blocks Z_ab (Sec. 2, Eq. 1-3): the Galerkin EFIE entries of RWG pairs,
 *     Z_mn = -i eta k sum over (T_m, T_n) of
 *              [ c_m c_n int int (r - p_m).(r' - p_n) g  -  k^-2 d_m d_n int int g ],
 *     c = s l / (2A), d = s l / A (s = +1 on T+, -1 on T-, p the free vertex),
 *     3-point rule on both triangles; a pair sharing a vertex integrates the
 *     inner triangle with the static part 1/(4 pi R) in closed form (Wilton et
 *     al. 1984, Graglia 1993) and the smooth rest on the rule, and takes the
 *     mean of both integration orders;
 *   radiation V^c_b = R_L G^c_src (Sec. 3, Eq. 10), transfer C = R_{l-1}
 *     G(X_{l-1}, E_l + delta) (Eq. 11, B = C^T in Eq. 13), translation
 *     D = G(E_a, E_b) (Eq. 12), reception U^c = (V^c)^T (Eq. 14);
 *   the product y = Z_near x + sum_c w_c U^c B..B D C..C V^c x in the order of
 *     Sec. 3: near field, radiation, source transfer (children before
 *     parents), translation, potential transfer (parents before children),
 *     reception.
 * The fitting operators R_l (a Tikhonov pseudo-inverse by SVD), the point
 * sets and the tree come from the NumPy oracle; every loop here is one of the
 * sums above, written out, each output owned by one loop iteration. */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- geometry */
typedef struct {
  const double* v;        /* [nv][3] vertices */
  const int64_t* t;       /* [nt][3] triangles */
  const double* area;     /* [nt] */
  const double* normal;   /* [nt][3] unit normals */
  const double* qp;       /* [nt][3][3] quadrature points (3-point rule) */
  const int64_t* tri;     /* [n][2] T+, T- of each RWG */
  const int64_t* freev;   /* [n][2] free vertex on T+, T- */
  const double* len;      /* [n] edge length */
  double k, eta;
} Mesh;

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double dist3(const double* a, const double* b) {
  double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}
static cplx green(double R, double k) { return cexp(-I * k * R) / (4.0 * PI * R); }
/* (exp(-ikR) - 1) / (4 pi R), limit -ik / (4 pi) at R = 0; the numerator as
 * -2 sin^2(kR/2) - i sin(kR) (no cancellation for small kR) */
static cplx green_smooth(double R, double k) {
  if (R < 1e-12) return -I * k / (4.0 * PI);
  const double h = sin(0.5 * k * R);
  return (-2.0 * h * h - I * sin(k * R)) / (4.0 * PI * R);
}

/* Closed-form static integrals over triangle tv (3 vertices) seen from r:
 * I1 = int 1/|r - r'|, Irho = int (rho' - rho)/|r - r'|, rho the projection of
 * r on the plane (line-integral forms of Wilton et al. / Graglia). */
static void potential_integrals(const double* r, const double tv[3][3], double* I1, double Irho[3]) {
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = tv[1][d] - tv[0][d];
    e2[d] = tv[2][d] - tv[0][d];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  double nn = sqrt(dot3(n, n));
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double rv[3] = {r[0] - tv[0][0], r[1] - tv[0][1], r[2] - tv[0][2]};
  double h = dot3(rv, n), ah = fabs(h);
  double rho[3] = {r[0] - h * n[0], r[1] - h * n[1], r[2] - h * n[2]};
  *I1 = 0.0;
  Irho[0] = Irho[1] = Irho[2] = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double* pm = tv[i];
    const double* pp = tv[(i + 1) % 3];
    double l[3] = {pp[0] - pm[0], pp[1] - pm[1], pp[2] - pm[2]};
    double ll = sqrt(dot3(l, l));
    for (int d = 0; d < 3; ++d) l[d] /= ll;
    double u[3] = {l[1] * n[2] - l[2] * n[1], l[2] * n[0] - l[0] * n[2], l[0] * n[1] - l[1] * n[0]};
    double a[3] = {pp[0] - rho[0], pp[1] - rho[1], pp[2] - rho[2]};
    double b[3] = {pm[0] - rho[0], pm[1] - rho[1], pm[2] - rho[2]};
    double lp = dot3(a, l), lm = dot3(b, l), P0 = dot3(a, u);
    double R0s = P0 * P0 + h * h;
    double Rp = sqrt(lp * lp + R0s), Rm = sqrt(lm * lm + R0s);
    double Lg = 0.0;
    if (R0s > 1e-30) {
      /* R + l without cancellation when l < 0: (R^2 - l^2) / (R - l) */
      double ap = lp >= 0 ? Rp + lp : R0s / (Rp - lp);
      double am = lm >= 0 ? Rm + lm : R0s / (Rm - lm);
      Lg = log(ap) - log(am);
    }
    double at = atan2(P0 * lp, R0s + ah * Rp) - atan2(P0 * lm, R0s + ah * Rm);
    *I1 += P0 * Lg - ah * at;
    double f = 0.5 * (R0s * Lg + lp * Rp - lm * Rm);
    for (int d = 0; d < 3; ++d) Irho[d] += f * u[d];
  }
}

static int share_vertex(const Mesh* m, int64_t ta, int64_t tb) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (m->t[3 * ta + i] == m->t[3 * tb + j]) return 1;
  return 0;
}

/* Singular pair, one order: outer 3-point rule on ta, inner integral over tb
 * with the static part in closed form.  A = int int (r - pa).(r' - pb) g,
 * B = int int g. */
static void singular_order(const Mesh* m, int64_t ta, const double* pa, int64_t tb, const double* pb, cplx* A,
                           cplx* B) {
  double tv[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) tv[i][d] = m->v[3 * m->t[3 * tb + i] + d];
  const double* nb = &m->normal[3 * tb];
  const double wa = m->area[ta] / 3.0, wb = m->area[tb] / 3.0;
  const double inv4pi = 1.0 / (4.0 * PI);
  *A = 0;
  *B = 0;
  for (int i = 0; i < 3; ++i) {
    const double* r = &m->qp[9 * ta + 3 * i];
    double I1, Irho[3];
    potential_integrals(r, tv, &I1, Irho);
    double rv[3] = {r[0] - tv[0][0], r[1] - tv[0][1], r[2] - tv[0][2]};
    double h = dot3(rv, nb);
    double rho[3] = {r[0] - h * nb[0], r[1] - h * nb[1], r[2] - h * nb[2]};
    /* Jg = int g(r, r');  Jv = int (r' - pb) g(r, r') */
    cplx Jg = inv4pi * I1, Jv[3];
    for (int d = 0; d < 3; ++d) Jv[d] = inv4pi * (Irho[d] + (rho[d] - pb[d]) * I1);
    for (int j = 0; j < 3; ++j) {
      const double* rp = &m->qp[9 * tb + 3 * j];
      cplx gs = green_smooth(dist3(r, rp), m->k) * wb;
      Jg += gs;
      for (int d = 0; d < 3; ++d) Jv[d] += gs * (rp[d] - pb[d]);
    }
    cplx acc = 0;
    for (int d = 0; d < 3; ++d) acc += (r[d] - pa[d]) * Jv[d];
    *A += wa * acc;
    *B += wa * Jg;
  }
}

/* Triangle pair integrals A = int_Ta int_Tb (r - pa).(r' - pb) g, B = int int g */
static void pair_integrals(const Mesh* m, int64_t ta, const double* pa, int64_t tb, const double* pb, cplx* A,
                           cplx* B) {
  if (share_vertex(m, ta, tb)) {
    cplx A1, B1, A2, B2;
    singular_order(m, ta, pa, tb, pb, &A1, &B1);
    singular_order(m, tb, pb, ta, pa, &A2, &B2);
    *A = 0.5 * (A1 + A2);
    *B = 0.5 * (B1 + B2);
    return;
  }
  const double wa = m->area[ta] / 3.0, wb = m->area[tb] / 3.0;
  *A = 0;
  *B = 0;
  for (int i = 0; i < 3; ++i) {
    const double* r = &m->qp[9 * ta + 3 * i];
    for (int j = 0; j < 3; ++j) {
      const double* rp = &m->qp[9 * tb + 3 * j];
      cplx g = green(dist3(r, rp), m->k) * (wa * wb);
      double rr = 0;
      for (int d = 0; d < 3; ++d) rr += (r[d] - pa[d]) * (rp[d] - pb[d]);
      *A += rr * g;
      *B += g;
    }
  }
}

/* Z_mn (Sec. 2, Eq. 3) */
static cplx z_entry(const Mesh* m, int64_t mi, int64_t ni) {
  cplx z = 0;
  for (int sa = 0; sa < 2; ++sa) {
    const int64_t ta = m->tri[2 * mi + sa];
    const double* pa = &m->v[3 * m->freev[2 * mi + sa]];
    const double sgn_a = sa == 0 ? 1.0 : -1.0;
    const double ca = sgn_a * m->len[mi] / (2.0 * m->area[ta]), da = sgn_a * m->len[mi] / m->area[ta];
    for (int sb = 0; sb < 2; ++sb) {
      const int64_t tb = m->tri[2 * ni + sb];
      const double* pb = &m->v[3 * m->freev[2 * ni + sb]];
      const double sgn_b = sb == 0 ? 1.0 : -1.0;
      const double cb = sgn_b * m->len[ni] / (2.0 * m->area[tb]), db = sgn_b * m->len[ni] / m->area[tb];
      cplx A, B;
      pair_integrals(m, ta, pa, tb, pb, &A, &B);
      z += ca * cb * A - da * db * B / (m->k * m->k);
    }
  }
  return -I * m->eta * m->k * z;
}

/* ---------------------------------------------------------------- operators */
/* Near blocks of every leaf: rows = RWGs of leaf a, columns = RWGs of its
 * near leaves in list order, column-major [col][row] at zoff[a]. */
void oc_near_blocks(const Mesh* m, int64_t nleaf, const int64_t* rw_ptr, const int64_t* rw_idx,
                    const int64_t* near_ptr, const int64_t* near_idx, const int64_t* zoff, cplx* Z) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < nleaf; ++a) {
    const int64_t S = rw_ptr[a + 1] - rw_ptr[a];
    int64_t col = 0;
    for (int64_t e = near_ptr[a]; e < near_ptr[a + 1]; ++e) {
      const int64_t b = near_idx[e];
      for (int64_t jb = rw_ptr[b]; jb < rw_ptr[b + 1]; ++jb, ++col)
        for (int64_t ia = 0; ia < S; ++ia)
          Z[zoff[a] + col * S + ia] = z_entry(m, rw_idx[rw_ptr[a] + ia], rw_idx[jb]);
    }
  }
}

/* Radiation matrices V^c_b [c][q][j] (Sec. 3, Eq. 10) at voff[b]:
 * V = R_L Gs, Gs^c[mm][j] = sum over the 6 quadrature points p of RWG j of
 * w_p g(|centre_b + X_mm - r_p|) f^c_j(r_p), f = (phi_x, phi_y, phi_z, div phi).
 * R [Q][M] complex, X [M][3] real (check points around the origin). */
void oc_radiation(const Mesh* m, int64_t nleaf, const int64_t* rw_ptr, const int64_t* rw_idx,
                  const double* centre, int Q, int M, const cplx* R, const double* X, const int64_t* voff,
                  cplx* V) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nleaf; ++b) {
    const int64_t S = rw_ptr[b + 1] - rw_ptr[b];
    cplx* Gs = (cplx*)malloc(sizeof(cplx) * 4 * (size_t)M * (size_t)S);
    for (int64_t j = 0; j < S; ++j) {
      const int64_t n = rw_idx[rw_ptr[b] + j];
      for (int mm = 0; mm < M; ++mm) {
        double xp[3] = {centre[3 * b] + X[3 * mm], centre[3 * b + 1] + X[3 * mm + 1],
                        centre[3 * b + 2] + X[3 * mm + 2]};
        cplx acc[4] = {0, 0, 0, 0};
        for (int side = 0; side < 2; ++side) {
          const int64_t tt = m->tri[2 * n + side];
          const double s = side == 0 ? 1.0 : -1.0;
          const double* p = &m->v[3 * m->freev[2 * n + side]];
          const double A = m->area[tt];
          for (int q = 0; q < 3; ++q) {
            const double* r = &m->qp[9 * tt + 3 * q];
            cplx g = green(dist3(xp, r), m->k) * (A / 3.0);
            for (int d = 0; d < 3; ++d) acc[d] += g * (s * m->len[n] / (2.0 * A) * (r[d] - p[d]));
            acc[3] += g * (s * m->len[n] / A);
          }
        }
        for (int c = 0; c < 4; ++c) Gs[((size_t)c * M + mm) * S + j] = acc[c];
      }
    }
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < Q; ++q)
        for (int64_t j = 0; j < S; ++j) {
          cplx acc = 0;
          for (int mm = 0; mm < M; ++mm) acc += R[(size_t)q * M + mm] * Gs[((size_t)c * M + mm) * S + j];
          V[voff[b] + ((size_t)c * Q + q) * S + j] = acc;
        }
    free(Gs);
  }
}

/* ---------------------------------------------------------------- product */
typedef struct {
  int nlev;                  /* levels l0 .. L as 0 .. nlev-1 */
  const int* Q;              /* [nlev] */
  const int64_t* nbox;       /* [nlev] */
  const int64_t* s_off;      /* [nlev] offset of box 0 in s / o (complex elements, 4 Q per box) */
  const int64_t* parent;     /* per level (level i > 0): [nbox_i] parent index at level i-1 */
  const int64_t* par_off;    /* [nlev] offsets into parent / octant */
  const int32_t* octant;
  const int64_t* ch_ptr;     /* per level i < L: children at level i+1 of box P, in increasing */
  const int64_t* ch_off;     /*   index order: ch_idx[ch_ptr[ch_off[i] + P] .. ch_ptr[ch_off[i] + P + 1]) */
  const int64_t* ch_idx;
  const int64_t* il_ptr;     /* per level CSR at il_off[i] (nbox_i + 1 entries) */
  const int64_t* il_off;
  const int64_t* il_src;     /* sources, at il_ptr values (global across levels) */
  const int64_t* il_d;       /* offset of the pair's D matrix in Dall */
  const cplx* Dall;          /* translation matrices [Q][Q] row-major */
  const cplx* Call;          /* transfer matrices: level i > 0, octant o at c_off[i] + o Q_{i-1} Q_i, [Q_{i-1}][Q_i] */
  const int64_t* c_off;
  const cplx* V;             /* radiation matrices at voff[b], [4][Q_L][S_b] */
  const int64_t* voff;
  const cplx* Z;             /* near blocks at zoff[a], [W_a][S_a] */
  const int64_t* zoff;
  int64_t nleaf;
  const int64_t* rw_ptr;     /* RWGs of leaf a: rw_idx[rw_ptr[a] .. rw_ptr[a+1]) (canonical ids) */
  const int64_t* rw_idx;
  const int64_t* near_ptr;
  const int64_t* near_idx;
  cplx w[4];                 /* channel weights */
} Nesa;

/* y = Z_NESA x (canonical order).  s, o: work arrays of s_off[nlev] complex
 * values (4 Q_l per box of level l). */
void oc_matvec(const Nesa* op, const cplx* x, cplx* y, cplx* s, cplx* o) {
  const int nl = op->nlev, L = nl - 1;
  const int QL = op->Q[L];
  memset(y, 0, sizeof(cplx) * (size_t)op->rw_ptr[op->nleaf]);
  /* near field (Eq. 9): y_a += sum over near b of Z_ab x_b */
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < op->nleaf; ++a) {
    const int64_t S = op->rw_ptr[a + 1] - op->rw_ptr[a];
    int64_t col = 0;
    for (int64_t e = op->near_ptr[a]; e < op->near_ptr[a + 1]; ++e) {
      const int64_t b = op->near_idx[e];
      for (int64_t jb = op->rw_ptr[b]; jb < op->rw_ptr[b + 1]; ++jb, ++col) {
        const cplx xv = x[op->rw_idx[jb]];
        const cplx* zc = &op->Z[op->zoff[a] + col * S];
        for (int64_t i = 0; i < S; ++i) y[op->rw_idx[op->rw_ptr[a] + i]] += zc[i] * xv;
      }
    }
  }
  /* radiation (Eq. 10): s_L[b][c] = V^c_b x_b */
  cplx* sL = s + op->s_off[L];
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t b = 0; b < op->nleaf; ++b) {
    const int64_t S = op->rw_ptr[b + 1] - op->rw_ptr[b];
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < QL; ++q) {
        cplx acc = 0;
        const cplx* Vr = &op->V[op->voff[b] + ((size_t)c * QL + q) * S];
        for (int64_t j = 0; j < S; ++j) acc += Vr[j] * x[op->rw_idx[op->rw_ptr[b] + j]];
        sL[(b * 4 + c) * QL + q] = acc;
      }
  }
  /* source transfer (Eq. 11), children before parents: s_P = sum C_oct s_child */
  for (int i = L; i > 0; --i) {
    const int Qc = op->Q[i], Qp = op->Q[i - 1];
    const int64_t nc = op->nbox[i], np = op->nbox[i - 1];
    cplx* sp = s + op->s_off[i - 1];
    const cplx* sc = s + op->s_off[i];
    memset(sp, 0, sizeof(cplx) * (size_t)np * 4 * Qp);
    (void)nc;
    /* parent-owned sums: each parent gathers its children in index order */
    const int64_t* cp = op->ch_ptr + op->ch_off[i - 1];
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t P = 0; P < np; ++P)
      for (int64_t e = cp[P]; e < cp[P + 1]; ++e) {
        const int64_t b = op->ch_idx[e];
        const cplx* C = &op->Call[op->c_off[i] + (size_t)op->octant[op->par_off[i] + b] * Qp * Qc];
        for (int c = 0; c < 4; ++c)
          for (int p = 0; p < Qp; ++p) {
            cplx acc = 0;
            for (int q = 0; q < Qc; ++q) acc += C[(size_t)p * Qc + q] * sc[(b * 4 + c) * Qc + q];
            sp[(P * 4 + c) * Qp + p] += acc;
          }
      }
  }
  /* translation (Eq. 12) at every level: o_a = sum over IL(a) of D_ab s_b */
  for (int i = 0; i < nl; ++i) {
    const int Qi = op->Q[i];
    const cplx* si = s + op->s_off[i];
    cplx* oi = o + op->s_off[i];
    const int64_t* ip = op->il_ptr + op->il_off[i];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < op->nbox[i]; ++a) {
      cplx* oa = &oi[a * 4 * Qi];
      memset(oa, 0, sizeof(cplx) * 4 * Qi);
      for (int64_t e = ip[a]; e < ip[a + 1]; ++e) {
        const int64_t b = op->il_src[e];
        const cplx* D = &op->Dall[op->il_d[e]];
        for (int c = 0; c < 4; ++c)
          for (int p = 0; p < Qi; ++p) {
            cplx acc = 0;
            for (int q = 0; q < Qi; ++q) acc += D[(size_t)p * Qi + q] * si[(b * 4 + c) * Qi + q];
            oa[c * Qi + p] += acc;
          }
      }
    }
  }
  /* potential transfer (Eq. 13), parents before children: o_a += C_oct^T o_P */
  for (int i = 1; i < nl; ++i) {
    const int Qc = op->Q[i], Qp = op->Q[i - 1];
    const cplx* op_ = o + op->s_off[i - 1];
    cplx* oc = o + op->s_off[i];
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t a = 0; a < op->nbox[i]; ++a) {
      const int64_t P = op->parent[op->par_off[i] + a];
      const cplx* C = &op->Call[op->c_off[i] + (size_t)op->octant[op->par_off[i] + a] * Qp * Qc];
      for (int c = 0; c < 4; ++c)
        for (int q = 0; q < Qc; ++q) {
          cplx acc = 0;
          for (int p = 0; p < Qp; ++p) acc += C[(size_t)p * Qc + q] * op_[(P * 4 + c) * Qp + p];
          oc[(a * 4 + c) * Qc + q] += acc;
        }
    }
  }
  /* reception (Eq. 14): y_a += sum_c w_c (V^c_a)^T o_a */
  const cplx* oL = o + op->s_off[L];
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t a = 0; a < op->nleaf; ++a) {
    const int64_t S = op->rw_ptr[a + 1] - op->rw_ptr[a];
    for (int64_t j = 0; j < S; ++j) {
      cplx acc = 0;
      for (int c = 0; c < 4; ++c) {
        cplx part = 0;
        for (int q = 0; q < QL; ++q) part += op->V[op->voff[a] + ((size_t)c * QL + q) * S + j] * oL[(a * 4 + c) * QL + q];
        acc += op->w[c] * part;
      }
      y[op->rw_idx[op->rw_ptr[a] + j]] += acc;
    }
  }
}

void oc_set_threads(int n) { omp_set_num_threads(n); }
int oc_max_threads(void) { return omp_get_max_threads(); }
