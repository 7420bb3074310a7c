// Device assembly of the near-field Galerkin blocks (FP64), the same integrals
// as the host assembly: EFIE (Sec. 2, Eq. 1-3)
//   Z_mn = -i eta k sum_{T,T'} int_T int_T' [phi_m . phi_n - k^-2 div phi_m div' phi_n] g,
// g = exp(-ikR)/(4 pi R), 3-point rule on both triangles; a triangle pair that
// shares a vertex takes the inner integral as (exp(-ikR)-1)/(4 pi R) on the
// 3-point rule plus 1/(4 pi R) in closed form, and the mean of both integration
// orders (so Z = Z^T).  One thread per block entry; the entry needs, per pair of
// its triangles, only the vertex-weighted integral of its two free vertices and
// the plain integral.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "nesa_host.h"

namespace nesa {
namespace {

constexpr int NTA = 256;
constexpr int MAX_NEAR_A = 128;
constexpr double PI_D = 3.14159265358979323846;

struct P {
  double x, y, z;
};
__device__ inline P psub(P a, P b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline P padd(P a, P b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline P pmul(P a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double pdot(P a, P b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline P pcross(P a, P b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double pnorm(P a) { return sqrt(pdot(a, a)); }

struct C {
  double re, im;
};
__device__ inline C cadd(C a, C b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline C cscale(C a, double s) { return {a.re * s, a.im * s}; }

// exp(-ikR) / (4 pi R)
__device__ inline C green(double R, double k) {
  double s, c;
  sincos(k * R, &s, &c);
  const double f = 1.0 / (4.0 * PI_D * R);
  return {c * f, -s * f};
}
// (exp(-ikR) - 1) / (4 pi R), limit -ik / (4 pi)
__device__ inline C green_smooth(double R, double k) {
  const double x = k * R;
  if (x < 1e-3) {
    const double f = k / (4.0 * PI_D);
    return {f * (-0.5 * x + x * x * x / 24.0), f * (-1.0 + x * x / 6.0)};
  }
  double s, c;
  sincos(x, &s, &c);
  const double f = 1.0 / (4.0 * PI_D * R);
  return {(c - 1.0) * f, -s * f};
}

struct Tri {
  P v[3];
  P q[3];
  double w;
  P n;
};

struct Geo {
  const int32_t* perm;
  const int32_t* leaf_ptr;
  const int32_t* near_ptr;
  const int32_t* near_idx;
  const int64_t* off;
  const int32_t* rtri;      // [n][2] triangles T+, T- of each RWG
  const int32_t* tv;        // [nt][3] vertex ids
  const int32_t* tri_rwg;   // [nt][3] RWG on the edge opposite local vertex a
  const double* v;          // [nv][3]
  const double* qp;         // [nt][3][3]
  const double* area;       // [nt]
  const double* normal;     // [nt][3]
  const double* len;        // [n]
  double k, eta;
};

// v[a] for a runtime a without indexing a private array
__device__ inline P pick(const P* v, int a) { return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]); }

__device__ inline Tri load_tri(const Geo& g, int t) {
  Tri r;
  for (int a = 0; a < 3; ++a) {
    const double* p = g.v + 3 * g.tv[3 * t + a];
    r.v[a] = {p[0], p[1], p[2]};
    r.q[a] = {g.qp[9 * t + 3 * a], g.qp[9 * t + 3 * a + 1], g.qp[9 * t + 3 * a + 2]};
  }
  r.w = g.area[t] / 3.0;
  r.n = {g.normal[3 * t], g.normal[3 * t + 1], g.normal[3 * t + 2]};
  return r;
}

// I1 = int_T 1/|r - r'| dS', Ir = int_T (rho' - rho)/|r - r'| dS' (closed form,
// edge by edge: Wilton et al. 1984, Graglia 1993)
__device__ __noinline__ void static_integrals(const Tri& T, P r, double& I1, P& Ir) {
  const double h = pdot(psub(r, T.v[0]), T.n);
  const P rho = psub(r, pmul(T.n, h));
  const double ah = fabs(h);
  I1 = 0;
  Ir = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const P pm = T.v[i], pp = T.v[(i + 1) % 3];
    const P e = psub(pp, pm);
    const P lh = pmul(e, 1.0 / pnorm(e));
    const P uh = pcross(lh, T.n);
    const double lp = pdot(psub(pp, rho), lh), lm = pdot(psub(pm, rho), lh);
    const double P0 = pdot(psub(pp, rho), uh);
    const double R0s = P0 * P0 + h * h;
    const double Rp = sqrt(lp * lp + R0s), Rm = sqrt(lm * lm + R0s);
    double lg = 0;
    if (R0s > 1e-30) {
      const double ap = lp >= 0 ? Rp + lp : R0s / (Rp - lp);
      const double am = lm >= 0 ? Rm + lm : R0s / (Rm - lm);
      lg = log(ap) - log(am);
    }
    const double at = atan2(P0 * lp, R0s + ah * Rp) - atan2(P0 * lm, R0s + ah * Rm);
    I1 += P0 * lg - ah * at;
    Ir = padd(Ir, pmul(uh, 0.5 * (R0s * lg + lp * Rp - lm * Rm)));
  }
}

// outer 3-point rule on A, inner integral over B with the static part exact:
// Av = int_A int_B (r - vA_a).(r' - vB_b) g, Bs = int_A int_B g
__device__ __noinline__ void singular_order(const Tri& A, int a, const Tri& B, int b, double k, C& Av, C& Bs) {
  const double inv4pi = 1.0 / (4.0 * PI_D);
  const P va = pick(A.v, a), vb = pick(B.v, b);
  Av = {0, 0};
  Bs = {0, 0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const P r = A.q[i];
    double I1;
    P Ir;
    static_integrals(B, r, I1, Ir);
    const double h = pdot(psub(r, B.v[0]), B.n);
    const P rho = psub(r, pmul(B.n, h));
    C gs[3];
    C sg = {0, 0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gs[j] = cscale(green_smooth(pnorm(psub(r, B.q[j])), k), B.w);
      sg = cadd(sg, gs[j]);
    }
    const C Jg = {sg.re + inv4pi * I1, sg.im};
    Bs = cadd(Bs, cscale(Jg, A.w));
    // J_b = int_B (r' - vB_b) g dr'
    C jx = {0, 0}, jy = {0, 0}, jz = {0, 0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const P d = psub(B.q[j], vb);
      jx = cadd(jx, cscale(gs[j], d.x));
      jy = cadd(jy, cscale(gs[j], d.y));
      jz = cadd(jz, cscale(gs[j], d.z));
    }
    const P st = padd(Ir, pmul(psub(rho, vb), I1));
    jx.re += inv4pi * st.x;
    jy.re += inv4pi * st.y;
    jz.re += inv4pi * st.z;
    const P ra = psub(r, va);
    Av = cadd(Av, cscale({ra.x * jx.re + ra.y * jy.re + ra.z * jz.re, ra.x * jx.im + ra.y * jy.im + ra.z * jz.im},
                         A.w));
  }
}

__device__ void pair_integrals(const Geo& g, int ta, int a, int tb, int b, C& Av, C& Bs) {
  const Tri A = load_tri(g, ta), B = load_tri(g, tb);
  bool share = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) share = share || g.tv[3 * ta + i] == g.tv[3 * tb + j];
  if (!share) {
    const P va = pick(A.v, a), vb = pick(B.v, b);
    Av = {0, 0};
    Bs = {0, 0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const P ra = psub(A.q[i], va);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const C G = cscale(green(pnorm(psub(A.q[i], B.q[j])), g.k), A.w * B.w);
        Bs = cadd(Bs, G);
        Av = cadd(Av, cscale(G, pdot(ra, psub(B.q[j], vb))));
      }
    }
    return;
  }
  C A1, B1, A2, B2;
  singular_order(A, a, B, b, g.k, A1, B1);
  singular_order(B, b, A, a, g.k, A2, B2);   // roles swapped: vertex b of B against a of A
  Av = cscale(cadd(A1, A2), 0.5);
  Bs = cscale(cadd(B1, B2), 0.5);
}

__device__ inline int local_free(const Geo& g, int t, int n) {
  for (int a = 0; a < 3; ++a)
    if (g.tri_rwg[3 * t + a] == n) return a;
  return 0;
}

// one workgroup per leaf a: entries of its S x W block, column-major
__global__ __launch_bounds__(NTA) void k_assemble_near(Geo g, double2* __restrict__ Z) {
  __shared__ int seg_col[MAX_NEAR_A + 1];
  __shared__ int seg_x[MAX_NEAR_A];
  const int a = blockIdx.x;
  const int p0 = g.leaf_ptr[a], S = g.leaf_ptr[a + 1] - p0;
  const int n0 = g.near_ptr[a], nn = g.near_ptr[a + 1] - n0;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int kk = 0; kk < nn; ++kk) {
      const int b = g.near_idx[n0 + kk];
      seg_col[kk] = c;
      seg_x[kk] = g.leaf_ptr[b];
      c += g.leaf_ptr[b + 1] - g.leaf_ptr[b];
    }
    seg_col[nn] = c;
  }
  __syncthreads();
  const int64_t cnt = (int64_t)S * seg_col[nn];
  const double ik2 = 1.0 / (g.k * g.k);
  for (int64_t e = threadIdx.x; e < cnt; e += NTA) {
    const int i = (int)(e % S), jc = (int)(e / S);
    int kk = 0;
    while (seg_col[kk + 1] <= jc) ++kk;
    const int m = g.perm[p0 + i], n = g.perm[seg_x[kk] + (jc - seg_col[kk])];
    C acc = {0, 0};
    for (int sm = 0; sm < 2; ++sm) {
      const int T = g.rtri[2 * m + sm];
      const double cm = (sm == 0 ? 1.0 : -1.0) * g.len[m] / g.area[T];
      const int am = local_free(g, T, m);
      for (int sn = 0; sn < 2; ++sn) {
        const int Tp = g.rtri[2 * n + sn];
        const double cn = (sn == 0 ? 1.0 : -1.0) * g.len[n] / g.area[Tp];
        const int bn = local_free(g, Tp, n);
        C Av, Bs;
        pair_integrals(g, T, am, Tp, bn, Av, Bs);
        acc = cadd(acc, cadd(cscale(Av, 0.25 * cm * cn), cscale(Bs, -ik2 * cm * cn)));
      }
    }
    // times -i eta k
    const double pk = g.eta * g.k;
    Z[g.off[a] + e] = make_double2(pk * acc.im, -pk * acc.re);
  }
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(-3, std::string(what) + ": " + hipGetErrorString(e));
}

// device copies that are freed when the scope ends
struct DevBuffers {
  std::vector<void*> p;
  ~DevBuffers() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename X>
  const X* put(const std::vector<X>& h) {
    void* d = nullptr;
    check(hipMalloc(&d, std::max<size_t>(h.size() * sizeof(X), 16)), "hipMalloc");
    p.push_back(d);
    if (!h.empty()) check(hipMemcpy(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice), "hipMemcpy");
    return static_cast<const X*>(d);
  }
};

template <typename X>
std::vector<int32_t> i32(const std::vector<X>& v) {
  return std::vector<int32_t>(v.begin(), v.end());
}

// ------------------------------------------------------------------ transfer matrices
// G_o[q][j] = g(X_j - delta_o - E_q), g = exp(-ikR) / (4 pi R) with R the
// principal square root of the summed squared (complex) coordinate
// differences; one thread per (o, q, j), j fastest.
__global__ void k_fill_transfer_g(const double2* __restrict__ X, const double2* __restrict__ E, int Mp, int Qc,
                                  double a, double k, double2* __restrict__ G) {
  const int64_t i = (int64_t)blockIdx.x * NTA + threadIdx.x;
  const int64_t total = (int64_t)8 * Qc * Mp;
  if (i >= total) return;
  const int j = (int)(i % Mp);
  const int64_t rest = i / Mp;
  const int q = (int)(rest % Qc), o = (int)(rest / Qc);
  const double d[3] = {((o & 1) - 0.5) * a, (((o >> 1) & 1) - 0.5) * a, (((o >> 2) & 1) - 0.5) * a};
  double zr = 0, zi = 0;
  for (int c = 0; c < 3; ++c) {
    const double er = X[3 * j + c].x - d[c] - E[3 * q + c].x;
    const double ei = X[3 * j + c].y - E[3 * q + c].y;
    zr += er * er - ei * ei;
    zi += 2.0 * er * ei;
  }
  // principal square root of zr + i zi: the branch without cancellation first
  const double m = hypot(zr, zi);
  double sr, si;
  if (zr >= 0) {
    sr = sqrt(0.5 * (m + zr));
    si = sr > 0 ? zi / (2.0 * sr) : 0.0;
  } else {
    si = sqrt(0.5 * (m - zr));
    if (zi < 0) si = -si;
    sr = zi / (2.0 * si);
  }
  // exp(-ik R) / (4 pi R) with R = sr + i si
  const double ex = exp(k * si) / (4.0 * PI_D);
  const double cr = ex * cos(k * sr), ci = -ex * sin(k * sr);      // exp(-ikR) / (4 pi)
  const double den = sr * sr + si * si;
  G[i] = make_double2((cr * sr + ci * si) / den, (ci * sr - cr * si) / den);
}

// cup[o][p][q] = sum_j R[j][p] G_o[q][j] (R column-major Qp x Mp): 32 x 32
// output tiles, j in chunks of 16 staged in LDS, four outputs per thread,
// FP64 complex sums in increasing j.
constexpr int TG_T = 32, TG_K = 16;
__global__ __launch_bounds__(NTA) void k_transfer_gemm_f64(const double2* __restrict__ R, const double2* __restrict__ G,
                                                           int Qp, int Mp, int Qc, double2* __restrict__ cup) {
  __shared__ double2 Rs[TG_K][TG_T];          // [j][p]
  __shared__ double2 Gs[TG_T][TG_K + 1];      // [q][j]
  const int o = blockIdx.z, p0 = blockIdx.y * TG_T, q0 = blockIdx.x * TG_T;
  const int t = threadIdx.x, tp = t % TG_T, tq = (t / TG_T) * 4;   // 4 consecutive q per thread
  const double2* Go = G + (size_t)o * Qc * Mp;
  double2 acc[4];
  for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < Mp; j0 += TG_K) {
    __syncthreads();
    for (int e = t; e < TG_K * TG_T; e += NTA) {
      const int jj = e / TG_T, pp = e % TG_T;
      Rs[jj][pp] = (j0 + jj < Mp && p0 + pp < Qp) ? R[(size_t)(j0 + jj) * Qp + p0 + pp] : make_double2(0.0, 0.0);
      const int qq = e / TG_K, jk = e % TG_K;
      Gs[qq][jk] = (j0 + jk < Mp && q0 + qq < Qc) ? Go[(size_t)(q0 + qq) * Mp + j0 + jk] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int jj = 0; jj < TG_K; ++jj) {
      const double2 r = Rs[jj][tp];
      for (int u = 0; u < 4; ++u) {
        const double2 g = Gs[tq + u][jj];
        acc[u].x += r.x * g.x - r.y * g.y;
        acc[u].y += r.x * g.y + r.y * g.x;
      }
    }
  }
  for (int u = 0; u < 4; ++u)
    if (p0 + tp < Qp && q0 + tq + u < Qc) cup[((size_t)o * Qp + p0 + tp) * Qc + q0 + tq + u] = acc[u];
}

// ------------------------------------------------------------------ Tikhonov fits
// Householder QR of the stacked matrix A = [G; lambda I] (m = M + Q rows, Q
// columns, column-major), one reflector per column in order, the thin
// orthogonal factor accumulated backwards from [I_Q; 0], then the fitting
// operator X = R^-1 Q^H [I_M; 0] by back substitution.  FP64 complex; the sums
// over rows are workgroup reductions.
constexpr int NTF = 256;

// complex sum over the workgroup, returned to every thread (red: NTF / 64 slots)
__device__ double2 fit_wg_sum(double2 v, double2* red) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();                    // earlier reads of red are done
  if (lane == 0) red[w] = v;
  __syncthreads();
  double2 s = red[0];
  for (int i = 1; i < NTF / 64; ++i) {
    s.x += red[i].x;
    s.y += red[i].y;
  }
  return s;
}

// reflector of column j (one workgroup): with x = A[j:, j] and
// alpha = -(x_0 / |x_0|) |x| (-|x| for x_0 = 0), v = (x - alpha e_1) / |x - alpha e_1|
// into rows j .. m-1 of column j of V
__global__ __launch_bounds__(NTF) void k_fit_reflector(const double2* __restrict__ A, int64_t m, int j,
                                                       double2* __restrict__ V) {
  __shared__ double2 red[NTF / 64];
  const double2* a = A + (int64_t)j * m;
  double2* v = V + (int64_t)j * m;
  double2 p = make_double2(0.0, 0.0);
  for (int64_t i = j + threadIdx.x; i < m; i += NTF) {
    const double2 x = a[i];
    p.x += x.x * x.x + x.y * x.y;
  }
  const double nx = sqrt(fit_wg_sum(p, red).x);
  const double2 x0 = a[j];
  const double ax0 = hypot(x0.x, x0.y);
  const double2 alpha = ax0 > 0 ? make_double2(-x0.x / ax0 * nx, -x0.y / ax0 * nx) : make_double2(-nx, 0.0);
  double2 q = make_double2(0.0, 0.0);
  for (int64_t i = j + threadIdx.x; i < m; i += NTF) {
    double2 x = a[i];
    if (i == j) x = make_double2(x.x - alpha.x, x.y - alpha.y);
    q.x += x.x * x.x + x.y * x.y;
  }
  const double nv = sqrt(fit_wg_sum(q, red).x);
  for (int64_t i = j + threadIdx.x; i < m; i += NTF) {
    double2 x = a[i];
    if (i == j) x = make_double2(x.x - alpha.x, x.y - alpha.y);
    if (nv > 0) x = make_double2(x.x / nv, x.y / nv);
    v[i] = x;
  }
}

// B[j:, c] -= 2 v (v^H B[j:, c]) for column c = c0 + blockIdx.x of B (m rows),
// v = rows j .. m-1 of column j of V
__global__ __launch_bounds__(NTF) void k_fit_reflect(double2* __restrict__ B, int64_t m, int j, int c0,
                                                     const double2* __restrict__ V) {
  __shared__ double2 red[NTF / 64];
  const double2* v = V + (int64_t)j * m;
  double2* b = B + (int64_t)(c0 + (int)blockIdx.x) * m;
  double2 p = make_double2(0.0, 0.0);
  for (int64_t i = j + threadIdx.x; i < m; i += NTF) {
    const double2 vi = v[i], bi = b[i];
    p.x += vi.x * bi.x + vi.y * bi.y;
    p.y += vi.x * bi.y - vi.y * bi.x;
  }
  double2 s = fit_wg_sum(p, red);
  s = make_double2(2.0 * s.x, 2.0 * s.y);
  for (int64_t i = j + threadIdx.x; i < m; i += NTF) {
    const double2 vi = v[i];
    double2 bi = b[i];
    bi.x -= vi.x * s.x - vi.y * s.y;
    bi.y -= vi.x * s.y + vi.y * s.x;
    b[i] = bi;
  }
}

// X = R^-1 Y, R the upper triangle of A (Q x Q), Y(i, col) = conj(Qt(col, i))
// for the M columns: one wave per column, y in LDS, rows from the last up;
// each step divides by the diagonal and takes the row's multiple of column i
// of R (contiguous above the diagonal) from the rows above it, the lanes
// sharing those rows.  Xt row-major (Q x M).  Dynamic LDS: Q complex values.
constexpr int NTS = 64;
__global__ __launch_bounds__(NTS) void k_fit_solve(const double2* __restrict__ A, const double2* __restrict__ Qt,
                                                   int64_t m, int Q, int M, double2* __restrict__ Xt) {
  extern __shared__ double2 fit_y[];
  const int col = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < Q; i += NTS) {
    const double2 q = Qt[(int64_t)i * m + col];
    fit_y[i] = make_double2(q.x, -q.y);
  }
  __syncthreads();
  for (int i = Q - 1; i >= 0; --i) {
    const double2 d = A[(int64_t)i * m + i];
    const double2 s = fit_y[i];
    const double den = d.x * d.x + d.y * d.y;
    const double2 x = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
    if (lane == 0) Xt[(int64_t)i * M + col] = x;
    const double2* r = A + (int64_t)i * m;
    for (int j = lane; j < i; j += NTS) {
      const double2 a = r[j];
      double2 v = fit_y[j];
      v.x -= a.x * x.x - a.y * x.y;
      v.y -= a.x * x.y + a.y * x.x;
      fit_y[j] = v;
    }
    __syncthreads();
  }
}

}  // namespace

bool transfer_matrices_device(const std::vector<cd>& Rcm, int Qp, int Mp, const std::vector<cd>& X,
                              const std::vector<cd>& E, int Qc, double a, double k, std::vector<cd>& cup) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();           // (no device: the caller computes on the host)
    return false;
  }
  if ((int64_t)Rcm.size() != (int64_t)Qp * Mp || (int64_t)X.size() != 3 * (int64_t)Mp ||
      (int64_t)E.size() != 3 * (int64_t)Qc)
    throw Error(-1, "transfer matrix operand sizes");
  DevBuffers buf;
  const double2* Rd = reinterpret_cast<const double2*>(buf.put(Rcm));
  const double2* Xd = reinterpret_cast<const double2*>(buf.put(X));
  const double2* Ed = reinterpret_cast<const double2*>(buf.put(E));
  void* Gd = nullptr;
  void* Cd = nullptr;
  const int64_t ng = (int64_t)8 * Qc * Mp, nc = (int64_t)8 * Qp * Qc;
  check(hipMalloc(&Gd, std::max<size_t>(ng * sizeof(cd), 16)), "hipMalloc");
  buf.p.push_back(Gd);
  check(hipMalloc(&Cd, std::max<size_t>(nc * sizeof(cd), 16)), "hipMalloc");
  buf.p.push_back(Cd);
  cup.assign(nc, cd(0, 0));
  if (ng > 0) {
    k_fill_transfer_g<<<(unsigned)((ng + NTA - 1) / NTA), NTA>>>(Xd, Ed, Mp, Qc, a, k, static_cast<double2*>(Gd));
    check(hipGetLastError(), "kernel launch");
  }
  if (nc > 0) {
    const dim3 grid((unsigned)((Qc + TG_T - 1) / TG_T), (unsigned)((Qp + TG_T - 1) / TG_T), 8);
    k_transfer_gemm_f64<<<grid, NTA>>>(Rd, static_cast<const double2*>(Gd), Qp, Mp, Qc, static_cast<double2*>(Cd));
    check(hipGetLastError(), "kernel launch");
    check(hipMemcpy(cup.data(), Cd, nc * sizeof(cd), hipMemcpyDeviceToHost), "hipMemcpy");
  }
  return true;
}

bool tikhonov_fit_device(const std::vector<cd>& G, int64_t M, int64_t Q, double lam, std::vector<cd>& X) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();           // (no device: the caller computes on the host)
    return false;
  }
  if ((int64_t)G.size() != M * Q || M < 1 || Q < 1 || (M + Q) * Q > (int64_t)1 << 31)
    throw Error(-1, "fit operand sizes");
  if (Q > 4096) return false;          // (the solve keeps a column of Q values in LDS: larger fits on the host)
  const int64_t m = M + Q;
  // A = [G; lambda I] and the start [I_Q; 0] of the orthogonal factor
  std::vector<cd> A((size_t)(m * Q), cd(0, 0)), Qt((size_t)(m * Q), cd(0, 0));
  for (int64_t j = 0; j < Q; ++j) {
    std::copy(G.begin() + j * M, G.begin() + (j + 1) * M, A.begin() + j * m);
    A[(size_t)(j * m + M + j)] = lam;
    Qt[(size_t)(j * m + j)] = 1.0;
  }
  DevBuffers buf;
  double2* Ad = reinterpret_cast<double2*>(const_cast<cd*>(buf.put(A)));
  double2* Qd = reinterpret_cast<double2*>(const_cast<cd*>(buf.put(Qt)));
  void* Vd = nullptr;
  void* Xd = nullptr;
  check(hipMalloc(&Vd, (size_t)(m * Q) * sizeof(cd)), "hipMalloc");
  buf.p.push_back(Vd);
  check(hipMalloc(&Xd, (size_t)(Q * M) * sizeof(cd)), "hipMalloc");
  buf.p.push_back(Xd);
  double2* V = static_cast<double2*>(Vd);
  for (int j = 0; j < (int)Q; ++j) {
    k_fit_reflector<<<1, NTF>>>(Ad, m, j, V);
    k_fit_reflect<<<(unsigned)(Q - j), NTF>>>(Ad, m, j, j, V);
  }
  // columns left of j are still unit vectors with zero rows from j on
  for (int j = (int)Q - 1; j >= 0; --j) k_fit_reflect<<<(unsigned)(Q - j), NTF>>>(Qd, m, j, j, V);
  double2* Xt = static_cast<double2*>(Xd);
  k_fit_solve<<<(unsigned)M, NTS, (size_t)Q * sizeof(double2)>>>(Ad, Qd, m, (int)Q, (int)M, Xt);
  check(hipGetLastError(), "kernel launch");
  std::vector<cd> xt((size_t)(Q * M));
  check(hipMemcpy(xt.data(), Xt, xt.size() * sizeof(cd), hipMemcpyDeviceToHost), "hipMemcpy");
  X.assign((size_t)(Q * M), cd(0, 0));
  for (int64_t i = 0; i < Q; ++i)
    for (int64_t col = 0; col < M; ++col) X[(size_t)(col * Q + i)] = xt[(size_t)(i * M + col)];
  return true;
}

Near* assemble_near_device(const Tree& t, double k, double eta) {
  std::unique_ptr<Near> N(new Near());
  N->k = k;
  N->eta = eta;
  const Rwg& r = t.rwg;
  const int64_t nleaf = t.level(t.L).nbox;
  N->off.resize(nleaf + 1);
  N->off[0] = 0;
  for (int64_t a = 0; a < nleaf; ++a) {
    if (t.near_ptr[a + 1] - t.near_ptr[a] > MAX_NEAR_A) throw Error(-1, "near list longer than 128");
    int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a], W = 0;
    for (int64_t j = t.near_ptr[a]; j < t.near_ptr[a + 1]; ++j) {
      int64_t b = t.near_idx[j];
      W += t.leaf_ptr[b + 1] - t.leaf_ptr[b];
    }
    N->off[a + 1] = N->off[a] + S * W;
  }
  N->z.assign(N->off[nleaf], cd(0, 0));
  if (nleaf == 0 || N->off[nleaf] == 0) return N.release();
  DevBuffers buf;
  Geo g;
  g.perm = buf.put(i32(t.perm));
  g.leaf_ptr = buf.put(i32(t.leaf_ptr));
  g.near_ptr = buf.put(i32(t.near_ptr));
  g.near_idx = buf.put(i32(t.near_idx));
  g.off = buf.put(N->off);
  g.rtri = buf.put(i32(r.tri));
  g.tv = buf.put(r.t);
  g.tri_rwg = buf.put(i32(r.tri_rwg));
  g.v = buf.put(r.v);
  g.qp = buf.put(r.qp);
  g.area = buf.put(r.area);
  g.normal = buf.put(r.normal);
  g.len = buf.put(r.len);
  g.k = k;
  g.eta = eta;
  void* Zd = nullptr;
  const size_t bytes = (size_t)N->off[nleaf] * sizeof(cd);
  check(hipMalloc(&Zd, bytes), "hipMalloc");
  buf.p.push_back(Zd);
  k_assemble_near<<<(unsigned)nleaf, NTA>>>(g, static_cast<double2*>(Zd));
  check(hipGetLastError(), "kernel launch");
  check(hipMemcpy(N->z.data(), Zd, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
  return N.release();
}

}  // namespace nesa
