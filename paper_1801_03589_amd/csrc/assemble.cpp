// Host assembly (FP64): near-field Galerkin EFIE blocks, NESA far-field
// operators and plane-wave right-hand sides.
//
// EFIE (Sec. 2, Eq. 1-3): Z_mn = -i eta k sum_{T,T'} int_T int_T'
//   [phi_m . phi_n - k^-2 div phi_m div' phi_n] g,  g = exp(-ikR)/(4 pi R),
// the gradient of Eq. (1) moved onto the test function.  Quadrature: 3-point
// interior rule.  Triangle pairs sharing a vertex: the inner integral splits
// into (exp(-ikR)-1)/(4 pi R) on the 3-point rule plus 1/(4 pi R) in closed
// form (line-integral formulas of Wilton et al. 1984 / Graglia 1993); the pair
// value is the mean of both integration orders.
//
// NESA operators (Sec. 2, Eq. 4-7: equivalence on fictitious surfaces around
// the boxes; U = V^T, B = C^T by reciprocity): four scalar channels
// (phi_x, phi_y, phi_z, div phi) share g; per level Q equivalent points on a
// sphere of radius r_e and 4Q check points on radius r_c = max(box side, 1.05 r_e)
// (golden-angle spirals); the fitting operator R = argmin ||G(X,E) R - I||^2 +
// lambda^2 ||R||^2 (lambda = tau * sigma_max, sigma_max by Lanczos) is computed by Householder QR of
// [G; lambda I]; C = R_parent G(X_parent, E_child + delta).  V = R_L G_src and
// D_ab = G(E_a, E_b) are assembled on the device (kernels k_fill_radiation,
// k_fill_translation).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <memory>

#include "nesa_host.h"

namespace nesa {

static const double PI = 3.14159265358979323846;

struct P3 {
  double x, y, z;
};
static inline P3 sub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static inline P3 add(P3 a, P3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
static inline P3 mul(P3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
static inline double dot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline P3 cross(P3 a, P3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
static inline double norm(P3 a) { return std::sqrt(dot(a, a)); }

static inline cd green(double R, double k) {
  return std::exp(cd(0.0, -k * R)) / (4.0 * PI * R);
}
// (exp(-ikR) - 1)/(4 pi R), limit -ik/(4 pi)
static inline cd green_smooth(double R, double k) {
  double x = k * R;
  if (x < 1e-3)  // series of exp(-ix) - 1 divided by R
    return (k / (4.0 * PI)) * cd(-0.5 * x + x * x * x / 24.0, -1.0 + x * x / 6.0);
  return (std::exp(cd(0.0, -x)) - 1.0) / (4.0 * PI * R);
}

struct TriGeo {
  P3 v[3];
  P3 q[3];      // quadrature points
  double w;     // weight (area / 3)
  P3 n;         // unit normal
};

static TriGeo tri_geo(const Rwg& r, int64_t t) {
  TriGeo g;
  for (int a = 0; a < 3; ++a) {
    const double* p = &r.v[3 * r.t[3 * t + a]];
    g.v[a] = {p[0], p[1], p[2]};
    g.q[a] = {r.qp[9 * t + 3 * a], r.qp[9 * t + 3 * a + 1], r.qp[9 * t + 3 * a + 2]};
  }
  g.w = r.area[t] / 3.0;
  g.n = {r.normal[3 * t], r.normal[3 * t + 1], r.normal[3 * t + 2]};
  return g;
}

// Static integrals over triangle T at observation point r:
//   I1 = int 1/|r-r'| dS',  Ir = int (rho' - rho)/|r-r'| dS'
static void static_integrals(const TriGeo& T, P3 r, double& I1, P3& Ir) {
  double h = dot(sub(r, T.v[0]), T.n);
  P3 rho = sub(r, mul(T.n, h));
  double ah = std::fabs(h);
  I1 = 0;
  Ir = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    P3 pm = T.v[i], pp = T.v[(i + 1) % 3];
    P3 e = sub(pp, pm);
    P3 lh = mul(e, 1.0 / norm(e));
    P3 uh = cross(lh, T.n);
    double lp = dot(sub(pp, rho), lh), lm = dot(sub(pm, rho), lh);
    double P0 = dot(sub(pp, rho), uh);
    double R0s = P0 * P0 + h * h;
    double Rp = std::sqrt(lp * lp + R0s), Rm = std::sqrt(lm * lm + R0s);
    double lg = 0;
    if (R0s > 1e-30) {
      double ap = lp >= 0 ? Rp + lp : R0s / (Rp - lp);
      double am = lm >= 0 ? Rm + lm : R0s / (Rm - lm);
      lg = std::log(ap) - std::log(am);
    }
    double at = std::atan2(P0 * lp, R0s + ah * Rp) - std::atan2(P0 * lm, R0s + ah * Rm);
    I1 += P0 * lg - ah * at;
    Ir = add(Ir, mul(uh, 0.5 * (R0s * lg + lp * Rp - lm * Rm)));
  }
}

// Pair integrals for triangles A (test) and B (source):
//   Av[a][b] = int_A int_B (r - vA_a).(r' - vB_b) g,   Bs = int_A int_B g
struct PairInt {
  cd Av[3][3];
  cd Bs;
};

static void regular_pair(const TriGeo& A, const TriGeo& B, double k, PairInt& out) {
  cd G[3][3];
  cd Bs = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      G[i][j] = green(norm(sub(A.q[i], B.q[j])), k) * (A.w * B.w);
      Bs += G[i][j];
    }
  out.Bs = Bs;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cd acc = 0;
      for (int i = 0; i < 3; ++i) {
        P3 ra = sub(A.q[i], A.v[a]);
        for (int j = 0; j < 3; ++j) acc += G[i][j] * dot(ra, sub(B.q[j], B.v[b]));
      }
      out.Av[a][b] = acc;
    }
}

// outer 3-point rule on A, inner integral over B with the static part exact
static void singular_order(const TriGeo& A, const TriGeo& B, double k, PairInt& out) {
  const double inv4pi = 1.0 / (4.0 * PI);
  out.Bs = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out.Av[a][b] = 0;
  for (int i = 0; i < 3; ++i) {
    P3 r = A.q[i];
    double I1;
    P3 Ir;
    static_integrals(B, r, I1, Ir);
    double h = dot(sub(r, B.v[0]), B.n);
    P3 rho = sub(r, mul(B.n, h));
    cd gs[3];
    cd sg = 0;
    for (int j = 0; j < 3; ++j) {
      gs[j] = green_smooth(norm(sub(r, B.q[j])), k) * B.w;
      sg += gs[j];
    }
    cd Jg = sg + inv4pi * I1;
    out.Bs += A.w * Jg;
    // Jv_b = int (r' - vB_b) g dr'
    for (int b = 0; b < 3; ++b) {
      cd jx = 0, jy = 0, jz = 0;
      for (int j = 0; j < 3; ++j) {
        P3 d = sub(B.q[j], B.v[b]);
        jx += gs[j] * d.x;
        jy += gs[j] * d.y;
        jz += gs[j] * d.z;
      }
      P3 st = add(Ir, mul(sub(rho, B.v[b]), I1));
      jx += inv4pi * st.x;
      jy += inv4pi * st.y;
      jz += inv4pi * st.z;
      for (int a = 0; a < 3; ++a) {
        P3 ra = sub(r, A.v[a]);
        out.Av[a][b] += A.w * (ra.x * jx + ra.y * jy + ra.z * jz);
      }
    }
  }
}

static bool share_vertex(const Rwg& r, int64_t ta, int64_t tb) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (r.t[3 * ta + a] == r.t[3 * tb + b]) return true;
  return false;
}

static void pair_integrals(const Rwg& r, int64_t ta, int64_t tb, double k, PairInt& out) {
  TriGeo A = tri_geo(r, ta), B = tri_geo(r, tb);
  if (!share_vertex(r, ta, tb)) {
    regular_pair(A, B, k, out);
    return;
  }
  PairInt p1, p2;
  singular_order(A, B, k, p1);
  singular_order(B, A, k, p2);
  out.Bs = 0.5 * (p1.Bs + p2.Bs);
  // p2 has the roles swapped: its [b][a] entry pairs vertex a of A with b of B
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out.Av[a][b] = 0.5 * (p1.Av[a][b] + p2.Av[b][a]);
}

// local vertex of triangle t that is the free vertex of RWG n
static int local_free(const Rwg& r, int64_t t, int64_t n) {
  for (int a = 0; a < 3; ++a)
    if (r.tri_rwg[3 * t + a] == n) return a;
  return -1;
}

Near* assemble_near(const Tree& t, double k, double eta) {
  std::unique_ptr<Near> N(new Near());
  N->k = k;
  N->eta = eta;
  const Rwg& r = t.rwg;
  const int64_t nleaf = t.level(t.L).nbox;
  N->off.resize(nleaf + 1);
  N->off[0] = 0;
  for (int64_t a = 0; a < nleaf; ++a) {
    int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a], W = 0;
    for (int64_t j = t.near_ptr[a]; j < t.near_ptr[a + 1]; ++j) {
      int64_t b = t.near_idx[j];
      W += t.leaf_ptr[b + 1] - t.leaf_ptr[b];
    }
    N->off[a + 1] = N->off[a] + S * W;
  }
  N->z.assign(N->off[nleaf], cd(0, 0));
  const cd pref(0.0, -eta * k);
  const double ik2 = 1.0 / (k * k);
  parallel_for(nleaf, [&](int64_t a) {
    // columns: RWGs of the near leaves in list order
    std::vector<int64_t> cols;
    for (int64_t j = t.near_ptr[a]; j < t.near_ptr[a + 1]; ++j) {
      int64_t b = t.near_idx[j];
      for (int64_t p = t.leaf_ptr[b]; p < t.leaf_ptr[b + 1]; ++p) cols.push_back(t.perm[p]);
    }
    const int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
    const int64_t W = (int64_t)cols.size();
    // triangle-pair cache for this leaf: rows' triangles x columns' triangles
    std::vector<int64_t> rt, ct;
    for (int64_t p = t.leaf_ptr[a]; p < t.leaf_ptr[a + 1]; ++p)
      for (int s = 0; s < 2; ++s) rt.push_back(r.tri[2 * t.perm[p] + s]);
    for (int64_t c : cols)
      for (int s = 0; s < 2; ++s) ct.push_back(r.tri[2 * c + s]);
    std::sort(rt.begin(), rt.end());
    rt.erase(std::unique(rt.begin(), rt.end()), rt.end());
    std::sort(ct.begin(), ct.end());
    ct.erase(std::unique(ct.begin(), ct.end()), ct.end());
    std::vector<PairInt> cache(rt.size() * ct.size());
    for (size_t i = 0; i < rt.size(); ++i)
      for (size_t j = 0; j < ct.size(); ++j) pair_integrals(r, rt[i], ct[j], k, cache[i * ct.size() + j]);
    auto ridx = [&](int64_t tt) { return std::lower_bound(rt.begin(), rt.end(), tt) - rt.begin(); };
    auto cidx = [&](int64_t tt) { return std::lower_bound(ct.begin(), ct.end(), tt) - ct.begin(); };
    cd* Z = &N->z[N->off[a]];
    for (int64_t i = 0; i < S; ++i) {
      const int64_t m = t.perm[t.leaf_ptr[a] + i];
      for (int64_t jc = 0; jc < W; ++jc) {
        const int64_t n = cols[jc];
        cd acc = 0;
        for (int sm = 0; sm < 2; ++sm) {
          int64_t T = r.tri[2 * m + sm];
          double cm = (sm == 0 ? 1.0 : -1.0) * r.len[m] / r.area[T];
          int am = local_free(r, T, m);
          for (int sn = 0; sn < 2; ++sn) {
            int64_t Tp = r.tri[2 * n + sn];
            double cn = (sn == 0 ? 1.0 : -1.0) * r.len[n] / r.area[Tp];
            int bn = local_free(r, Tp, n);
            const PairInt& P = cache[ridx(T) * ct.size() + cidx(Tp)];
            acc += (0.25 * cm * cn) * P.Av[am][bn] - (ik2 * cm * cn) * P.Bs;
          }
        }
        Z[jc * S + i] = pref * acc;
      }
    }
  });
  return N.release();
}

// ------------------------------------------------------------------ far field
static int q_rule(double side, int d0, int q_min, double k) {
  double kr = k * std::sqrt(3.0) / 2.0 * side;
  int p = (int)std::ceil(kr + 1.8 * std::pow((double)d0, 2.0 / 3.0) * std::cbrt(kr)) + 1;
  return std::max(p * p, q_min);
}

static void fibonacci(int n, cd radius, std::vector<cd>& out) {
  out.resize(3 * n);
  const double ga = PI * (3.0 - std::sqrt(5.0));
  for (int i = 0; i < n; ++i) {
    double z = 1.0 - (2.0 * i + 1.0) / n;
    double rad = std::sqrt(std::max(0.0, 1.0 - z * z));
    double ph = i * ga;
    out[3 * i] = radius * rad * std::cos(ph);
    out[3 * i + 1] = radius * rad * std::sin(ph);
    out[3 * i + 2] = radius * z;
  }
}

// column-major complex matrix helper
struct CMat {
  int64_t m = 0, n = 0;
  std::vector<cd> a;
  CMat() {}
  CMat(int64_t m_, int64_t n_) : m(m_), n(n_), a(m_ * n_) {}
  cd& operator()(int64_t i, int64_t j) { return a[j * m + i]; }
  const cd& operator()(int64_t i, int64_t j) const { return a[j * m + i]; }
};

// G[i][j] = g(R_ij) with R_ij the principal square root of
// sum_d (A_id + shift_d - B_jd)^2; the points may be complex (complex source
// points), real points are complex with zero imaginary part.
static CMat gmat(const std::vector<cd>& A, P3 shift, const std::vector<cd>& B, double k) {
  int64_t na = A.size() / 3, nb = B.size() / 3;
  CMat G(na, nb);
  const double sh[3] = {shift.x, shift.y, shift.z};
  // (threads only where the matrix is large enough to pay for them)
  auto col = [&](int64_t j) {
    for (int64_t i = 0; i < na; ++i) {
      cd r2 = 0;
      for (int d = 0; d < 3; ++d) {
        cd e = A[3 * i + d] + sh[d] - B[3 * j + d];
        r2 += e * e;
      }
      cd R = std::sqrt(r2);
      G(i, j) = std::exp(cd(0.0, -k) * R) / (4.0 * PI * R);
    }
  };
  if (na * nb >= ((int64_t)1 << 16))
    parallel_for(nb, col);
  else
    for (int64_t j = 0; j < nb; ++j) col(j);
  return G;
}

// largest eigenvalue of the symmetric tridiagonal matrix (a, b) by bisection
// on the Sturm count (number of eigenvalues below x)
static double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const size_t k = a.size();
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto below = [&](double x) {
    size_t c = 0;
    double d = 1.0;
    for (size_t i = 0; i < k; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-16 * std::max(std::fabs(hi), std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) == k)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// largest singular value of G: Lanczos on G^H G with full reorthogonalisation
// (the largest Ritz value approaches the largest eigenvalue from below, much
// faster than power iteration when the top singular values are clustered)
static double sigma_max(const CMat& G) {
  const int64_t M = G.m, Q = G.n;
  const int kmax = (int)std::min<int64_t>(Q, 300);
  std::vector<std::vector<cd>> qs;
  std::vector<double> al, be;
  std::vector<cd> q(Q, cd(1.0 / std::sqrt((double)Q), 0.0)), u(M), w(Q);
  double est = 0;
  for (int j = 0; j < kmax; ++j) {
    qs.push_back(q);
    // u = G q by blocks of rows, w = G^H u by columns (every sum in the same
    // order as one loop over the whole matrix)
    constexpr int64_t RB = 256;
    auto rows = [&](int64_t rb) {
      const int64_t i0 = rb * RB, i1 = std::min(M, i0 + RB);
      for (int64_t i = i0; i < i1; ++i) u[i] = 0;
      for (int64_t c = 0; c < Q; ++c)
        for (int64_t i = i0; i < i1; ++i) u[i] += G(i, c) * q[c];
    };
    auto cols = [&](int64_t c) {
      cd s = 0;
      for (int64_t i = 0; i < M; ++i) s += std::conj(G(i, c)) * u[i];
      w[c] = s;
    };
    if (M * Q >= ((int64_t)1 << 18)) {
      parallel_for((M + RB - 1) / RB, rows);
      parallel_for(Q, cols);
    } else {
      for (int64_t rb = 0; rb < (M + RB - 1) / RB; ++rb) rows(rb);
      for (int64_t c = 0; c < Q; ++c) cols(c);
    }
    cd aj = 0;
    for (int64_t c = 0; c < Q; ++c) aj += std::conj(q[c]) * w[c];
    al.push_back(aj.real());
    // w -= sum_i q_i (q_i^H w), twice
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& qi : qs) {
        cd h = 0;
        for (int64_t c = 0; c < Q; ++c) h += std::conj(qi[c]) * w[c];
        for (int64_t c = 0; c < Q; ++c) w[c] -= h * qi[c];
      }
    double nb = 0;
    for (const auto& x : w) nb += std::norm(x);
    nb = std::sqrt(nb);
    const bool last = j + 1 == kmax || nb <= 1e-14 * std::sqrt(std::fabs(al[0]) + 1e-300);
    if (last || (j + 1) % 10 == 0) {
      const double e = tridiag_max_eig(al, be);
      if (last || (est > 0 && std::fabs(e - est) <= 1e-14 * e)) return std::sqrt(std::max(e, 0.0));
      est = e;
    }
    be.push_back(nb);
    for (int64_t c = 0; c < Q; ++c) q[c] = w[c] / nb;
  }
  return std::sqrt(std::max(est, 0.0));
}

// R = argmin ||G R - I_M||_F^2 + lambda^2 ||R||_F^2  (Q x M), via Householder QR
// of the stacked matrix [G; lambda I] (M+Q) x Q.
static CMat tikhonov_fit(const CMat& G, double tau) {
  const int64_t M = G.m, Q = G.n, m = M + Q;
  const double lam = tau * sigma_max(G);
  // the same steps on the device when there is one (NESA_FIT_HOST=1: here)
  const char* on_host = std::getenv("NESA_FIT_HOST");
  if (!(on_host && std::atoi(on_host) == 1)) {
    CMat X(Q, M);
    if (tikhonov_fit_device(G.a, M, Q, lam, X.a)) return X;
  }
  CMat A(m, Q);
  for (int64_t j = 0; j < Q; ++j) {
    for (int64_t i = 0; i < M; ++i) A(i, j) = G(i, j);
    A(M + j, j) = lam;
  }
  std::vector<std::vector<cd>> vs(Q);
  for (int64_t j = 0; j < Q; ++j) {
    double nx = 0;
    for (int64_t i = j; i < m; ++i) nx += std::norm(A(i, j));
    nx = std::sqrt(nx);
    cd x0 = A(j, j);
    cd alpha = (std::abs(x0) > 0 ? -x0 / std::abs(x0) : cd(-1.0, 0.0)) * nx;
    std::vector<cd> v(m - j);
    for (int64_t i = j; i < m; ++i) v[i - j] = A(i, j);
    v[0] -= alpha;
    double nv = 0;
    for (auto& x : v) nv += std::norm(x);
    nv = std::sqrt(nv);
    if (nv > 0)
      for (auto& x : v) x /= nv;
    // A[j:, j:] -= 2 v (v^H A[j:, j:])
    parallel_for(Q - j, [&](int64_t cc) {
      int64_t c = j + cc;
      cd s = 0;
      for (int64_t i = j; i < m; ++i) s += std::conj(v[i - j]) * A(i, c);
      s *= 2.0;
      for (int64_t i = j; i < m; ++i) A(i, c) -= v[i - j] * s;
    });
    vs[j] = std::move(v);
  }
  // Y = Q^H [I_M; 0]: column col of Y is the conjugate of row col of the thin
  // factor Q[:, 0:Q] = H_1 ... H_Q [I_Q; 0] (accumulated backwards, m Q^2
  // operations instead of M m Q for the reflectors applied to every e_col);
  // then solve R_qr X = Y
  CMat Qt(m, Q);
  for (int64_t j = 0; j < Q; ++j) Qt(j, j) = 1.0;
  for (int64_t j = Q - 1; j >= 0; --j) {
    const auto& v = vs[j];
    parallel_for(Q - j, [&](int64_t cc) {
      const int64_t c = j + cc;      // columns left of j are still zero in rows >= j
      cd s = 0;
      for (int64_t i = j; i < m; ++i) s += std::conj(v[i - j]) * Qt(i, c);
      s *= 2.0;
      for (int64_t i = j; i < m; ++i) Qt(i, c) -= v[i - j] * s;
    });
  }
  CMat X(Q, M);
  parallel_for(M, [&](int64_t col) {
    for (int64_t i = Q - 1; i >= 0; --i) {
      cd s = std::conj(Qt(col, i));
      for (int64_t c = i + 1; c < Q; ++c) s -= A(i, c) * X(c, col);
      X(i, col) = s / A(i, i);
    }
  });
  return X;
}

Far* assemble_far(const Tree& t, double k, double eta, int d0, int q_min, double tau, double eps) {
  if (d0 < 1 || q_min < 0 || !(tau > 0) || !(tau < 1) || !(eps >= 0) || !(eps < 1))
    throw Error(-1, "bad far-field parameters");
  std::unique_ptr<Far> F(new Far());
  F->k = k;
  F->eta = eta;
  F->d0 = d0;
  F->tau = tau;
  F->eps = eps;
  const Rwg& r = t.rwg;
  const int nl = t.L - t.l0 + 1;
  F->lev.resize(nl);
  // radii
  double rmax = 0;
  const Level& LL = t.level(t.L);
  for (int64_t b = 0; b < LL.nbox; ++b) {
    auto c = t.center(t.L, b);
    for (int64_t p = t.leaf_ptr[b]; p < t.leaf_ptr[b + 1]; ++p) {
      int64_t n = t.perm[p];
      for (int s = 0; s < 2; ++s) {
        int64_t T = r.tri[2 * n + s];
        for (int q = 0; q < 3; ++q) {
          P3 d = {r.qp[9 * T + 3 * q] - c[0], r.qp[9 * T + 3 * q + 1] - c[1], r.qp[9 * T + 3 * q + 2] - c[2]};
          rmax = std::max(rmax, norm(d));
        }
      }
    }
  }
  F->lev[nl - 1].re = 1.02 * rmax;
  for (int l = t.L - 1; l >= t.l0; --l)
    F->lev[l - t.l0].re = 1.02 * (std::sqrt(3.0) / 2.0 * t.level(l + 1).side + F->lev[l + 1 - t.l0].re);
  std::vector<CMat> R(nl);
  for (int l = t.l0; l <= t.L; ++l) {
    FarLevel& fl = F->lev[l - t.l0];
    const double side = t.level(l).side;
    // check sphere midway between r_e and 2a - r_e (= a), kept 5% outside r_e
    fl.rc = std::max(side, 1.05 * fl.re);
    if (fl.re >= 1.5 * side)
      throw Error(-4, "equivalent sphere radius exceeds 1.5 box sides at level " + std::to_string(l) +
                          " (mesh too coarse for the leaf size)");
    fl.Q = q_rule(side, d0, q_min, k);
    fl.M = 4 * fl.Q;
    fibonacci(fl.Q, cd(fl.re, eps * fl.re), fl.E);
    fibonacci(fl.M, cd(fl.rc, 0.0), fl.X);
    R[l - t.l0] = tikhonov_fit(gmat(fl.X, {0, 0, 0}, fl.E, k), tau);
  }
  // radiation matrices V = R_L G_src are assembled on the device (kernel
  // k_fill_radiation) from the finest level's fitting operator and check points
  F->RLt = R[nl - 1].a;
  // transfer matrices C (child level l, octant o): Q_{l-1} x Q_l row-major
  for (int l = t.l0 + 1; l <= t.L; ++l) {
    FarLevel& fc = F->lev[l - t.l0];
    const FarLevel& fp = F->lev[l - 1 - t.l0];
    const CMat& Rp = R[l - 1 - t.l0];
    const double a = t.level(l).side;
    // on the device when there is one (NESA_C_HOST=1: on the host)
    const char* on_host = std::getenv("NESA_C_HOST");
    if (!(on_host && std::atoi(on_host) == 1) &&
        transfer_matrices_device(Rp.a, fp.Q, fp.M, fp.X, fc.E, fc.Q, a, k, fc.Cup))
      continue;
    fc.Cup.assign((size_t)8 * fp.Q * fc.Q, cd(0, 0));
    // G(X_p, E_c + delta) = g(|X_p - delta - E_c|) per octant (column-major, so
    // that column q is contiguous over the check points j)
    std::vector<CMat> G(8);
    parallel_for(8, [&](int64_t o) {
      P3 delta = {((o & 1) - 0.5) * a, (((o >> 1) & 1) - 0.5) * a, (((o >> 2) & 1) - 0.5) * a};
      G[o] = gmat(fp.X, mul(delta, -1.0), fc.E, k);
    });
    // rows of R_parent contiguous over j
    std::vector<cd> Rrow((size_t)fp.Q * fp.M);
    for (int j = 0; j < fp.M; ++j)
      for (int p = 0; p < fp.Q; ++p) Rrow[(size_t)p * fp.M + j] = Rp(p, j);
    parallel_for((int64_t)8 * fp.Q, [&](int64_t op) {
      const int o = (int)(op / fp.Q), p = (int)(op % fp.Q);
      const cd* rp = &Rrow[(size_t)p * fp.M];
      for (int q = 0; q < fc.Q; ++q) {
        const cd* gq = &G[o].a[(size_t)q * fp.M];
        cd s = 0;
        for (int j = 0; j < fp.M; ++j) s += rp[j] * gq[j];
        fc.Cup[((size_t)o * fp.Q + p) * fc.Q + q] = s;
      }
    });
  }
  // translation matrices D: only the offset slots that occur are recorded here;
  // their entries D_d[p][q] = g(E_p + d - E_q) are computed on the device when
  // an operator is created
  for (int l = t.l0; l <= t.L; ++l) {
    FarLevel& fl = F->lev[l - t.l0];
    fl.slot_used.assign(t.nslot(), 0);
    for (int32_t s : t.level(l).il_slot) fl.slot_used[s] = 1;
  }
  return F.release();
}

void plane_wave_rhs(const Tree& t, double k, const double* khat, const double* pol, cd* b) {
  const Rwg& r = t.rwg;
  P3 kh = {khat[0], khat[1], khat[2]}, po = {pol[0], pol[1], pol[2]};
  parallel_for(r.n, [&](int64_t n) {
    cd acc = 0;
    for (int s = 0; s < 2; ++s) {
      const int64_t T = r.tri[2 * n + s];
      const double sg = (s == 0 ? 1.0 : -1.0);
      const int64_t fv = r.freev[2 * n + s];
      P3 pv = {r.v[3 * fv], r.v[3 * fv + 1], r.v[3 * fv + 2]};
      const double cv = sg * r.len[n] / (2.0 * r.area[T]);
      const double w = r.area[T] / 3.0;
      for (int q = 0; q < 3; ++q) {
        P3 rq = {r.qp[9 * T + 3 * q], r.qp[9 * T + 3 * q + 1], r.qp[9 * T + 3 * q + 2]};
        acc += w * cv * dot(sub(rq, pv), po) * std::exp(cd(0.0, -k * dot(kh, rq)));
      }
    }
    b[n] = -acc;
  });
}

}  // namespace nesa
