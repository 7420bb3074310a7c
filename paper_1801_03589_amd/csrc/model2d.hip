// 2D model problem (Sec. "The model problem"): the NESA form of the potential
// operator phi = K q, k_ij = -log |x_i - x_j|, over a quadtree, in real FP64.
// Host side: tree, lists and matrices (built once); device side: one kernel
// per stage and level, owner computes (every output element is written by one
// thread), no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/nesa2d.h"

namespace nesa {
int report_failure(int code, const std::string& msg);   // sets nesa_last_error()
}

namespace {

constexpr int NT2 = 256;
constexpr int QMAX = 128;
constexpr int MAX_LEVEL = 20;                       // finest level at most 20 (box side root / 2^20)
constexpr double R_EQ = 0.75;                       // equivalent circle / box side
constexpr double R_CHK[2] = {1.05, 1.6};            // check circles / box side

struct Fail : std::runtime_error {
  int code;
  Fail(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_ok2(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Fail(NESA_ENOMEM, std::string(what) + ": out of device memory");
    throw Fail(NESA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

// ------------------------------------------------------------------ host tree
struct Level2 {
  double a = 0;                                  // box side
  std::vector<std::pair<int64_t, int64_t>> cell; // non-empty cells, (i, j) order
  std::map<std::pair<int64_t, int64_t>, int64_t> index;
  std::vector<int32_t> il_ptr, il_src, il_off;   // far list (CSR), offset slot per pair
  std::vector<int32_t> child;                    // [nbox][4] child index per quadrant (2 qi + qj), -1 if empty
  std::vector<int32_t> parent, quad;             // [nbox] (l > l0)
};

struct Tree2 {
  int l0 = 2, L = 2;
  double ox = 0, oy = 0, root = 0;
  std::vector<Level2> lev;                       // index l - l0
  std::vector<int32_t> perm;                     // group order -> point index
  std::vector<int32_t> leaf_ptr;                 // [nleaf + 1]
  std::vector<int32_t> near_ptr, near_idx;       // leaf near lists
  double side(int l) const { return root / (double)(int64_t(1) << l); }
};

std::pair<int64_t, int64_t> cell_of(const Tree2& t, double x, double y, int l) {
  const double a = t.side(l);
  const int64_t hi = (int64_t(1) << l) - 1;
  int64_t i = (int64_t)std::floor((x - t.ox) / a), j = (int64_t)std::floor((y - t.oy) / a);
  return {std::min(std::max(i, int64_t(0)), hi), std::min(std::max(j, int64_t(0)), hi)};
}

// translation offsets (di, dj) with max(|di|, |dj|) in [2, 3]: slot index
int off_slot(int64_t di, int64_t dj) { return (int)((di + 3) * 7 + (dj + 3)); }

Tree2 build_tree(const double* xy, int64_t n, int P) {
  Tree2 t;
  double xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
  for (int64_t p = 0; p < n; ++p) {
    xmin = std::min(xmin, xy[2 * p]);
    xmax = std::max(xmax, xy[2 * p]);
    ymin = std::min(ymin, xy[2 * p + 1]);
    ymax = std::max(ymax, xy[2 * p + 1]);
  }
  t.ox = xmin;
  t.oy = ymin;
  t.root = std::max(xmax - xmin, ymax - ymin) * (1.0 + std::ldexp(1.0, -20));
  if (!(t.root > 0)) throw Fail(NESA_EINVAL, "points must not all coincide");
  // deepest level whose mean occupancy of non-empty boxes is >= P
  t.L = t.l0;
  for (int l = t.l0 + 1; l <= MAX_LEVEL; ++l) {
    std::set<std::pair<int64_t, int64_t>> cells;
    for (int64_t p = 0; p < n; ++p) cells.insert(cell_of(t, xy[2 * p], xy[2 * p + 1], l));
    if ((double)n / (double)cells.size() >= (double)P)
      t.L = l;
    else
      break;
  }
  if (t.L - t.l0 + 1 > NESA2D_MAX_LEVELS) throw Fail(NESA_EINVAL, "too many levels");
  t.lev.resize(t.L - t.l0 + 1);
  for (int l = t.l0; l <= t.L; ++l) {
    Level2& lv = t.lev[l - t.l0];
    lv.a = t.side(l);
    std::set<std::pair<int64_t, int64_t>> cells;
    for (int64_t p = 0; p < n; ++p) cells.insert(cell_of(t, xy[2 * p], xy[2 * p + 1], l));
    lv.cell.assign(cells.begin(), cells.end());
    for (size_t k = 0; k < lv.cell.size(); ++k) lv.index[lv.cell[k]] = (int64_t)k;
  }
  // points by finest-level box, by index inside a box
  const Level2& LL = t.lev.back();
  std::vector<std::vector<int32_t>> pts(LL.cell.size());
  for (int64_t p = 0; p < n; ++p) pts[LL.index.at(cell_of(t, xy[2 * p], xy[2 * p + 1], t.L))].push_back((int32_t)p);
  t.leaf_ptr.assign(1, 0);
  for (auto& v : pts) {
    t.perm.insert(t.perm.end(), v.begin(), v.end());
    t.leaf_ptr.push_back((int32_t)t.perm.size());
  }
  auto neighbours = [&](const Level2& lv, std::pair<int64_t, int64_t> c) {
    std::vector<int32_t> out;
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        auto it = lv.index.find({c.first + di, c.second + dj});
        if (it != lv.index.end()) out.push_back((int32_t)it->second);
      }
    std::sort(out.begin(), out.end());
    return out;
  };
  t.near_ptr.assign(1, 0);
  for (auto& c : LL.cell) {
    auto nb = neighbours(LL, c);
    t.near_idx.insert(t.near_idx.end(), nb.begin(), nb.end());
    t.near_ptr.push_back((int32_t)t.near_idx.size());
  }
  for (int l = t.l0; l <= t.L; ++l) {
    Level2& lv = t.lev[l - t.l0];
    lv.il_ptr.assign(1, 0);
    for (auto& c : lv.cell) {
      std::vector<std::pair<int64_t, int64_t>> cand;
      if (l == t.l0) {
        cand = lv.cell;
      } else {
        const Level2& pl = t.lev[l - 1 - t.l0];
        for (int32_t pb : neighbours(pl, {c.first / 2, c.second / 2}))
          for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj) {
              std::pair<int64_t, int64_t> cc{2 * pl.cell[pb].first + di, 2 * pl.cell[pb].second + dj};
              if (lv.index.count(cc)) cand.push_back(cc);
            }
      }
      for (auto& b : cand) {
        const int64_t di = c.first - b.first, dj = c.second - b.second;
        if (std::max(std::llabs(di), std::llabs(dj)) >= 2) {
          if (std::max(std::llabs(di), std::llabs(dj)) > 3) throw Fail(NESA_EINVAL, "interaction offset beyond 3 boxes");
          lv.il_src.push_back((int32_t)lv.index.at(b));
          lv.il_off.push_back(off_slot(di, dj));
        }
      }
      lv.il_ptr.push_back((int32_t)lv.il_src.size());
    }
    if (l > t.l0) {
      const Level2& pl = t.lev[l - 1 - t.l0];
      lv.parent.resize(lv.cell.size());
      lv.quad.resize(lv.cell.size());
      for (size_t k = 0; k < lv.cell.size(); ++k) {
        lv.parent[k] = (int32_t)pl.index.at({lv.cell[k].first / 2, lv.cell[k].second / 2});
        lv.quad[k] = (int32_t)(2 * (lv.cell[k].first % 2) + lv.cell[k].second % 2);
      }
    }
  }
  for (int l = t.l0; l < t.L; ++l) {
    Level2& pl = t.lev[l - t.l0];
    const Level2& cl = t.lev[l + 1 - t.l0];
    pl.child.assign(4 * pl.cell.size(), -1);
    for (size_t k = 0; k < cl.cell.size(); ++k) pl.child[4 * cl.parent[k] + cl.quad[k]] = (int32_t)k;
  }
  return t;
}

// ------------------------------------------------------------------ host matrices
// row-major dense matrices
using Mat = std::vector<double>;

double glog(double tx, double ty, double sx, double sy) { return -std::log(std::hypot(tx - sx, ty - sy)); }

std::vector<double> circle_pts(int n, double radius, double phase) {
  std::vector<double> p(2 * n);
  for (int k = 0; k < n; ++k) {
    const double a = 2.0 * M_PI * (k + phase) / n;
    p[2 * k] = radius * std::cos(a);
    p[2 * k + 1] = radius * std::sin(a);
  }
  return p;
}

// Tikhonov pseudo-inverse (Q x M) of G (M x Q, row-major), lambda = tau sigma_max:
// (G^T G + lambda^2 I)^-1 G^T from the Householder QR of [G; lambda I].
Mat tikhonov(const Mat& G, int M, int Q, double tau) {
  // sigma_max by power iteration on G^T G
  std::vector<double> v(Q, 1.0), w(M), u(Q);
  double smax = 0;
  for (int it = 0; it < 200; ++it) {
    for (int i = 0; i < M; ++i) {
      double s = 0;
      for (int j = 0; j < Q; ++j) s += G[(size_t)i * Q + j] * v[j];
      w[i] = s;
    }
    for (int j = 0; j < Q; ++j) {
      double s = 0;
      for (int i = 0; i < M; ++i) s += G[(size_t)i * Q + j] * w[i];
      u[j] = s;
    }
    double nu = 0;
    for (double x : u) nu += x * x;
    nu = std::sqrt(nu);
    const double s_new = std::sqrt(nu);
    for (int j = 0; j < Q; ++j) v[j] = u[j] / nu;
    if (std::fabs(s_new - smax) <= 1e-15 * s_new) {
      smax = s_new;
      break;
    }
    smax = s_new;
  }
  const double lam = tau * smax;
  const int R = M + Q;
  Mat A((size_t)R * Q, 0.0), B((size_t)R * M, 0.0);   // [G; lam I], [I_M; 0]
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < Q; ++j) A[(size_t)i * Q + j] = G[(size_t)i * Q + j];
  for (int j = 0; j < Q; ++j) A[(size_t)(M + j) * Q + j] = lam;
  for (int i = 0; i < M; ++i) B[(size_t)i * M + i] = 1.0;
  std::vector<double> h(R);
  for (int k = 0; k < Q; ++k) {
    double nrm = 0;
    for (int i = k; i < R; ++i) nrm += A[(size_t)i * Q + k] * A[(size_t)i * Q + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0) throw Fail(NESA_EINVAL, "singular fitting matrix");
    const double alpha = A[(size_t)k * Q + k] > 0 ? -nrm : nrm;
    for (int i = 0; i < R; ++i) h[i] = i < k ? 0.0 : A[(size_t)i * Q + k];
    h[k] -= alpha;
    double hh = 0;
    for (int i = k; i < R; ++i) hh += h[i] * h[i];
    if (hh == 0) continue;
    for (int j = k; j < Q; ++j) {
      double s = 0;
      for (int i = k; i < R; ++i) s += h[i] * A[(size_t)i * Q + j];
      s = 2.0 * s / hh;
      for (int i = k; i < R; ++i) A[(size_t)i * Q + j] -= s * h[i];
    }
    for (int j = 0; j < M; ++j) {
      double s = 0;
      for (int i = k; i < R; ++i) s += h[i] * B[(size_t)i * M + j];
      s = 2.0 * s / hh;
      for (int i = k; i < R; ++i) B[(size_t)i * M + j] -= s * h[i];
    }
  }
  // back substitution R X = (Q^T B)[0:Q]
  Mat X((size_t)Q * M);
  for (int j = 0; j < M; ++j)
    for (int k = Q - 1; k >= 0; --k) {
      double s = B[(size_t)k * M + j];
      for (int i = k + 1; i < Q; ++i) s -= A[(size_t)k * Q + i] * X[(size_t)i * M + j];
      X[(size_t)k * M + j] = s / A[(size_t)k * Q + k];
    }
  return X;
}

// ------------------------------------------------------------------ device kernels
// near blocks (Eq. algnf), assembled once on the device: leaf a holds one
// column-major block of n_a rows and W_a = sum of its near groups' sizes
// columns (near groups in list order); k_ii = 0 by point identity
__global__ __launch_bounds__(NT2) void k2_near_fill(const double2* __restrict__ xy,
                                                    const int32_t* __restrict__ leaf_ptr,
                                                    const int32_t* __restrict__ near_ptr,
                                                    const int32_t* __restrict__ near_idx,
                                                    const int64_t* __restrict__ zoff, double* __restrict__ Z) {
  __shared__ int seg_col[10], seg_pt[10];
  const int a = blockIdx.x, t = threadIdx.x;
  const int p0 = leaf_ptr[a], na = leaf_ptr[a + 1] - p0;
  const int k0 = near_ptr[a], nn = near_ptr[a + 1] - k0;      // nn <= 9
  if (t == 0) {
    int c = 0;
    for (int k = 0; k < nn; ++k) {
      const int b = near_idx[k0 + k];
      seg_col[k] = c;
      seg_pt[k] = leaf_ptr[b];
      c += leaf_ptr[b + 1] - leaf_ptr[b];
    }
    seg_col[nn] = c;
  }
  __syncthreads();
  const int W = seg_col[nn];
  double* Za = Z + zoff[a];
  for (int64_t e = t; e < (int64_t)na * W; e += NT2) {
    const int col = (int)(e / na), i = (int)(e % na);
    int k = 0;
    while (seg_col[k + 1] <= col) ++k;
    const int j = seg_pt[k] + (col - seg_col[k]);             // source point (group order)
    const double2 xi = xy[p0 + i], xj = xy[j];
    const double dx = xi.x - xj.x, dy = xi.y - xj.y;
    Za[e] = (p0 + i == j) ? 0.0 : -0.5 * log(dx * dx + dy * dy);
  }
}

// near-field product (Eq. algnf): phi_a = Z_a [q of the near groups].  A
// workgroup takes up to 64 rows of one group (grid y = row chunks); thread
// (row i, column group g) sums the columns g, g + G, ...; the G partial sums
// are added in a fixed order
constexpr int NEAR_CW = 1024;      // columns of q staged in LDS at a time
constexpr int NEAR_RW = 64;        // rows per workgroup
__global__ __launch_bounds__(NT2) void k2_near(const double* __restrict__ Z, const int64_t* __restrict__ zoff,
                                               const int32_t* __restrict__ leaf_ptr,
                                               const int32_t* __restrict__ near_ptr,
                                               const int32_t* __restrict__ near_idx, const double* __restrict__ q,
                                               double* __restrict__ phi) {
  __shared__ double qs[NEAR_CW];
  __shared__ double red[NT2];
  __shared__ int seg_col[10], seg_pt[10];
  const int a = blockIdx.x, t = threadIdx.x;
  const int p0 = leaf_ptr[a], na = leaf_ptr[a + 1] - p0;
  const int r0 = blockIdx.y * NEAR_RW;
  if (r0 >= na) return;                                        // whole workgroup
  const int nr = min(NEAR_RW, na - r0);
  const int G = NT2 / nr;                                      // column groups
  const int k0 = near_ptr[a], nn = near_ptr[a + 1] - k0;
  if (t == 0) {
    int c = 0;
    for (int k = 0; k < nn; ++k) {
      const int b = near_idx[k0 + k];
      seg_col[k] = c;
      seg_pt[k] = leaf_ptr[b];
      c += leaf_ptr[b + 1] - leaf_ptr[b];
    }
    seg_col[nn] = c;
  }
  __syncthreads();
  const int W = seg_col[nn];
  const int i = r0 + t % nr, g = t / nr;
  const double* Za = Z + zoff[a];
  double acc = 0.0;
  for (int c0 = 0; c0 < W; c0 += NEAR_CW) {
    const int cw = min(NEAR_CW, W - c0);
    __syncthreads();
    for (int c = t; c < cw; c += NT2) {
      const int col = c0 + c;
      int k = 0;
      while (seg_col[k + 1] <= col) ++k;
      qs[c] = q[seg_pt[k] + (col - seg_col[k])];
    }
    __syncthreads();
    if (g < G) {
      const double* Zc = Za + (size_t)c0 * na + i;
#pragma unroll 8
      for (int c = g; c < cw; c += G) acc += Zc[(size_t)c * na] * qs[c];
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < nr) {
    double y = red[t];
    for (int gg = 1; gg < G; ++gg) y += red[gg * nr + t];
    phi[p0 + r0 + t] = y;
  }
}

// The far-field kernels below take one box per workgroup of NT2 threads:
// thread t owns output row t % Q and reduction slice g = t / Q of G = NT2 / Q
// slices (every G-th term of the sum); the G partial sums of a row are added in
// slice order, so results do not depend on timing.
template <int NT = NT2>
__device__ __forceinline__ void slice_sum_store(double acc, double* red, double* out, int Q, bool add) {
  const int t = threadIdx.x, G = NT / Q;
  red[t] = acc;
  __syncthreads();
  if (t < Q) {
    double y = red[t];
    for (int g = 1; g < G; ++g) y += red[g * Q + t];
    out[t] = add ? out[t] + y : y;
  }
}

// radiation (Eq. algrad): s_b[k] = sum_j V_b[j][k] q_j (V stored point-major)
__global__ __launch_bounds__(NT2) void k2_radiate(const double* __restrict__ V, const int64_t* __restrict__ voff,
                                                  const int32_t* __restrict__ leaf_ptr,
                                                  const double* __restrict__ q, double* __restrict__ s, int Q) {
  __shared__ double red[NT2];
  const int b = blockIdx.x, t = threadIdx.x, G = NT2 / Q, k = t % Q, g = t / Q;
  const int p0 = leaf_ptr[b], nb = leaf_ptr[b + 1] - p0;
  const double* Vb = V + voff[b];
  double acc = 0.0;
  if (g < G) {
#pragma unroll 4
    for (int j = g; j < nb; j += G) acc += Vb[(size_t)j * Q + k] * q[p0 + j];
  }
  slice_sum_store(acc, red, s + (size_t)b * Q, Q, false);
}

// source transfer (Eq. algsou), one parent per workgroup, terms (child quadrant,
// r): s_P[p] = sum_c sum_r C_quad[p][r] s_c[r] (C stored column-major)
__global__ __launch_bounds__(NT2) void k2_upward(const double* __restrict__ Ccm, const int32_t* __restrict__ child,
                                                 const double* __restrict__ s_child, double* __restrict__ s_par,
                                                 int Q) {
  __shared__ double red[NT2];
  const int P = blockIdx.x, t = threadIdx.x, G = NT2 / Q, p = t % Q, g = t / Q;
  double acc = 0.0;
  if (g < G) {
    for (int c = 0; c < 4; ++c) {
      const int ch = child[4 * P + c];
      if (ch < 0) continue;
      const double* C = Ccm + (size_t)c * Q * Q;
      const double* sc = s_child + (size_t)ch * Q;
#pragma unroll 4
      for (int r = g; r < Q; r += G) acc += C[(size_t)r * Q + p] * sc[r];
    }
  }
  slice_sum_store(acc, red, s_par + (size_t)P * Q, Q, false);
}

// translation (Eq. algtrans): o_a[p] = sum_{b in far(a)} sum_r D_off[p][r] s_b[r]
// (D stored column-major per offset slot); one launch for every level (the
// levels are independent): workgroup = box of the concatenated level ranges;
// 1024 threads per box, so that every thread's chain of terms stays short
constexpr int NT_TR = 1024;
struct TransLevels {
  int n;                                         // levels
  int64_t box0[NESA2D_MAX_LEVELS + 1];           // first box of each level in the grid
  const double* Dcm[NESA2D_MAX_LEVELS];
  const int32_t* il_ptr[NESA2D_MAX_LEVELS];
  const int32_t* il_src[NESA2D_MAX_LEVELS];
  const int32_t* il_off[NESA2D_MAX_LEVELS];
  const double* s[NESA2D_MAX_LEVELS];
  double* o[NESA2D_MAX_LEVELS];
};
__global__ __launch_bounds__(NT_TR) void k2_translate(TransLevels tl, int Q) {
  __shared__ double red[NT_TR];
  int lv = 0;
  while (lv + 1 < tl.n && (int64_t)blockIdx.x >= tl.box0[lv + 1]) ++lv;
  const int a = (int)((int64_t)blockIdx.x - tl.box0[lv]);
  const int t = threadIdx.x, G = NT_TR / Q, p = t % Q, g = t / Q;
  const double* Dcm = tl.Dcm[lv];
  const double* s = tl.s[lv];
  const int32_t* il_src = tl.il_src[lv];
  const int32_t* il_off = tl.il_off[lv];
  double acc = 0.0;
  if (g < G) {
    for (int k = tl.il_ptr[lv][a]; k < tl.il_ptr[lv][a + 1]; ++k) {
      const double* D = Dcm + (size_t)il_off[k] * Q * Q;
      const double* sb = s + (size_t)il_src[k] * Q;
#pragma unroll 4
      for (int r = g; r < Q; r += G) acc += D[(size_t)r * Q + p] * sb[r];
    }
  }
  slice_sum_store<NT_TR>(acc, red, tl.o[lv] + (size_t)a * Q, Q, false);
}

// potential transfer (Eq. algpot): o_c[p] += sum_r B_quad[p][r] o_P[r], B = C^T
// (stored column-major, i.e. C row-major)
__global__ __launch_bounds__(NT2) void k2_downward(const double* __restrict__ Bcm, const int32_t* __restrict__ parent,
                                                   const int32_t* __restrict__ quad,
                                                   const double* __restrict__ o_par, double* __restrict__ o_child,
                                                   int Q) {
  __shared__ double red[NT2];
  const int c = blockIdx.x, t = threadIdx.x, G = NT2 / Q, p = t % Q, g = t / Q;
  double acc = 0.0;
  if (g < G) {
    const double* B = Bcm + (size_t)quad[c] * Q * Q;
    const double* op = o_par + (size_t)parent[c] * Q;
#pragma unroll 4
    for (int r = g; r < Q; r += G) acc += B[(size_t)r * Q + p] * op[r];
  }
  slice_sum_store(acc, red, o_child + (size_t)c * Q, Q, true);
}

// reception (Eq. algrec): phi_j += sum_k V_b[j][k] o_b[k], U = V^T; 16 lanes
// per point, 16 points per workgroup (grid y = chunks of points)
__global__ __launch_bounds__(NT2) void k2_receive(const double* __restrict__ V, const int64_t* __restrict__ voff,
                                                  const int32_t* __restrict__ leaf_ptr,
                                                  const double* __restrict__ o, double* __restrict__ phi, int Q) {
  __shared__ double ob[QMAX];
  constexpr int LP = 16;
  const int b = blockIdx.x, t = threadIdx.x;
  const int p0 = leaf_ptr[b], nb = leaf_ptr[b + 1] - p0;
  const int j = blockIdx.y * (NT2 / LP) + t / LP, c = t % LP;
  if ((int)blockIdx.y * (NT2 / LP) >= nb) return;              // whole workgroup
  if (t < Q) ob[t] = o[(size_t)b * Q + t];
  __syncthreads();
  const double* Vb = V + voff[b];
  double acc = 0.0;
  if (j < nb) {
#pragma unroll 4
    for (int k = c; k < Q; k += LP) acc += Vb[(size_t)j * Q + k] * ob[k];
  }
  for (int off = LP / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (c == 0 && j < nb) phi[p0 + j] += acc;
}

__global__ void k2_gather(const double* __restrict__ x, double* __restrict__ xl, const int32_t* __restrict__ perm,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) xl[i] = x[perm[i]];
}
__global__ void k2_scatter(const double* __restrict__ yl, double* __restrict__ y, const int32_t* __restrict__ perm,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[perm[i]] = yl[i];
}

}  // namespace

// ------------------------------------------------------------------ operator
struct DevLevel2 {
  int64_t nbox = 0;
  double* s = nullptr;
  double* o = nullptr;
  int32_t *il_ptr = nullptr, *il_src = nullptr, *il_off = nullptr;
  double* Dcm = nullptr;          // [49 slots][Q][Q] column-major
  double *Ccm = nullptr, *Bcm = nullptr;   // [4][Q][Q] (this level's children -> parents), l > l0
  int32_t *child = nullptr, *parent = nullptr, *quad = nullptr;
};

struct nesa2d {
  nesa2d_info info{};
  Tree2 tree;
  std::vector<void*> allocs;
  std::vector<DevLevel2> lev;
  double2* xy = nullptr;          // points in group order
  double *ql = nullptr, *phil = nullptr;
  double* V = nullptr;
  int64_t* voff = nullptr;
  int32_t *perm = nullptr, *leaf_ptr = nullptr, *near_ptr = nullptr, *near_idx = nullptr;
  double* Z = nullptr;            // near blocks
  int64_t* zoff = nullptr;        // [nleaf] block offsets
  ~nesa2d() {
    (void)hipDeviceSynchronize();
    for (void* p : allocs) (void)hipFree(p);
  }
  template <typename X>
  X* upload(const std::vector<X>& h) {
    void* p = nullptr;
    hip_ok2(hipMalloc(&p, std::max<size_t>(sizeof(X), h.size() * sizeof(X))), "hipMalloc");
    allocs.push_back(p);
    if (!h.empty()) hip_ok2(hipMemcpy(p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice), "hipMemcpy");
    return static_cast<X*>(p);
  }
  template <typename X>
  X* alloc(size_t count) {
    void* p = nullptr;
    hip_ok2(hipMalloc(&p, std::max<size_t>(sizeof(X), count * sizeof(X))), "hipMalloc");
    allocs.push_back(p);
    return static_cast<X*>(p);
  }
};

template <class F>
static int guarded2(F&& fn) {
  try {
    return fn();
  } catch (const Fail& e) {
    return nesa::report_failure(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return nesa::report_failure(NESA_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return nesa::report_failure(NESA_EINVAL, e.what());
  }
}

extern "C" nesa_status nesa2d_create(const double* xy, int64_t n, const nesa2d_params* prm, nesa2d** out) {
  return (nesa_status)guarded2([&]() -> int {
    if (!xy || !prm || !out) throw Fail(NESA_EINVAL, "null pointer");
    *out = nullptr;
    if (n < 2 || n > (int64_t)1 << 30) throw Fail(NESA_EINVAL, "n must be in [2, 2^30]");
    if (prm->P < 1) throw Fail(NESA_EINVAL, "P must be >= 1");
    if (prm->Q < 2 || prm->Q > QMAX) throw Fail(NESA_EINVAL, "Q must be in [2, 128]");
    if (!(prm->tau > 0)) throw Fail(NESA_EINVAL, "tau must be > 0");
    const int Q = prm->Q;
    auto h = std::make_unique<nesa2d>();
    h->tree = build_tree(xy, n, prm->P);
    Tree2& t = h->tree;
    const int nl = t.L - t.l0 + 1;
    const int64_t nleaf = (int64_t)t.leaf_ptr.size() - 1;
    // fitting operators per level
    std::vector<Mat> R(nl);
    std::vector<std::vector<double>> E(nl), X(nl);
    for (int i = 0; i < nl; ++i) {
      const double a = t.lev[i].a;
      E[i] = circle_pts(Q, R_EQ * a, 0.5);
      X[i].clear();
      for (double rc : R_CHK) {
        auto c = circle_pts(2 * Q, rc * a, 0.0);
        X[i].insert(X[i].end(), c.begin(), c.end());
      }
      const int M = 4 * Q;
      Mat G((size_t)M * Q);
      for (int r = 0; r < M; ++r)
        for (int k = 0; k < Q; ++k) G[(size_t)r * Q + k] = glog(X[i][2 * r], X[i][2 * r + 1], E[i][2 * k], E[i][2 * k + 1]);
      R[i] = tikhonov(G, M, Q, prm->tau);
    }
    // radiation matrices V_b = R_L G(X_L + c_b, x_b), stored [point][k]
    const int M = 4 * Q;
    const Level2& LL = t.lev.back();
    std::vector<double> Vh((size_t)n * Q);
    std::vector<int64_t> voff(nleaf);
    {
      std::vector<double> Gb;
      for (int64_t b = 0; b < nleaf; ++b) {
        const double cx = t.ox + (LL.cell[b].first + 0.5) * LL.a, cy = t.oy + (LL.cell[b].second + 0.5) * LL.a;
        const int p0 = t.leaf_ptr[b], nb = t.leaf_ptr[b + 1] - p0;
        voff[b] = (int64_t)p0 * Q;
        Gb.assign((size_t)M * nb, 0.0);
        for (int r = 0; r < M; ++r)
          for (int j = 0; j < nb; ++j) {
            const int p = t.perm[p0 + j];
            Gb[(size_t)r * nb + j] = glog(X[nl - 1][2 * r] + cx, X[nl - 1][2 * r + 1] + cy, xy[2 * p], xy[2 * p + 1]);
          }
        const Mat& Rl = R[nl - 1];
        for (int j = 0; j < nb; ++j)
          for (int k = 0; k < Q; ++k) {
            double s = 0;
            for (int r = 0; r < M; ++r) s += Rl[(size_t)k * M + r] * Gb[(size_t)r * nb + j];
            Vh[(size_t)(p0 + j) * Q + k] = s;
          }
      }
    }
    // device data
    std::vector<double2> xyl(n);
    for (int64_t k = 0; k < n; ++k) xyl[k] = make_double2(xy[2 * t.perm[k]], xy[2 * t.perm[k] + 1]);
    h->xy = h->upload(xyl);
    h->V = h->upload(Vh);
    h->voff = h->upload(voff);
    h->perm = h->upload(t.perm);
    h->leaf_ptr = h->upload(t.leaf_ptr);
    h->near_ptr = h->upload(t.near_ptr);
    h->near_idx = h->upload(t.near_idx);
    h->ql = h->alloc<double>(n);
    h->phil = h->alloc<double>(n);
    {
      std::vector<int64_t> zoff(nleaf);
      int64_t tot = 0;
      for (int64_t a = 0; a < nleaf; ++a) {
        zoff[a] = tot;
        int64_t W = 0;
        for (int k = t.near_ptr[a]; k < t.near_ptr[a + 1]; ++k)
          W += t.leaf_ptr[t.near_idx[k] + 1] - t.leaf_ptr[t.near_idx[k]];
        tot += (int64_t)(t.leaf_ptr[a + 1] - t.leaf_ptr[a]) * W;
      }
      h->zoff = h->upload(zoff);
      h->Z = h->alloc<double>((size_t)tot);
      k2_near_fill<<<(unsigned)nleaf, NT2>>>(h->xy, h->leaf_ptr, h->near_ptr, h->near_idx, h->zoff, h->Z);
      hip_ok2(hipGetLastError(), "near block assembly");
      hip_ok2(hipDeviceSynchronize(), "near block assembly");
    }
    h->lev.resize(nl);
    for (int i = 0; i < nl; ++i) {
      const Level2& lv = t.lev[i];
      DevLevel2& dl = h->lev[i];
      dl.nbox = (int64_t)lv.cell.size();
      dl.s = h->alloc<double>((size_t)dl.nbox * Q);
      dl.o = h->alloc<double>((size_t)dl.nbox * Q);
      dl.il_ptr = h->upload(lv.il_ptr);
      dl.il_src = h->upload(lv.il_src);
      dl.il_off = h->upload(lv.il_off);
      // translation matrices D_slot = G(E + off a, E), column-major
      std::vector<double> D((size_t)49 * Q * Q, 0.0);
      for (int di = -3; di <= 3; ++di)
        for (int dj = -3; dj <= 3; ++dj) {
          if (std::max(std::abs(di), std::abs(dj)) < 2) continue;
          double* Ds = D.data() + (size_t)off_slot(di, dj) * Q * Q;
          for (int p = 0; p < Q; ++p)
            for (int r = 0; r < Q; ++r)
              Ds[(size_t)r * Q + p] = glog(E[i][2 * p] + di * lv.a, E[i][2 * p + 1] + dj * lv.a, E[i][2 * r], E[i][2 * r + 1]);
        }
      dl.Dcm = h->upload(D);
      if (i > 0) {
        // C_quad = R_{l-1} G(X_{l-1}, E_l + delta): column-major (upward) and row-major (downward, B = C^T)
        std::vector<double> Cc((size_t)4 * Q * Q), Cr((size_t)4 * Q * Q);
        for (int qi = 0; qi < 2; ++qi)
          for (int qj = 0; qj < 2; ++qj) {
            const int qd = 2 * qi + qj;
            const double dx = (qi - 0.5) * lv.a, dy = (qj - 0.5) * lv.a;
            Mat G((size_t)M * Q);
            for (int r = 0; r < M; ++r)
              for (int k = 0; k < Q; ++k)
                G[(size_t)r * Q + k] = glog(X[i - 1][2 * r], X[i - 1][2 * r + 1], E[i][2 * k] + dx, E[i][2 * k + 1] + dy);
            const Mat& Rp = R[i - 1];
            for (int p = 0; p < Q; ++p)
              for (int k = 0; k < Q; ++k) {
                double s = 0;
                for (int r = 0; r < M; ++r) s += Rp[(size_t)p * M + r] * G[(size_t)r * Q + k];
                Cc[(size_t)qd * Q * Q + (size_t)k * Q + p] = s;    // C[p][k] at (k, p)
                Cr[(size_t)qd * Q * Q + (size_t)p * Q + k] = s;    // B[k][p] = C[p][k], column-major B
              }
          }
        dl.Ccm = h->upload(Cc);
        dl.Bcm = h->upload(Cr);
        dl.parent = h->upload(lv.parent);
        dl.quad = h->upload(lv.quad);
      }
      if (i + 1 < nl) dl.child = h->upload(lv.child);
    }
    // info
    nesa2d_info& inf = h->info;
    inf.n = n;
    inf.l0 = t.l0;
    inf.L = t.L;
    inf.Q = Q;
    for (int i = 0; i < nl; ++i) {
      inf.n_box[i] = (int64_t)t.lev[i].cell.size();
      inf.n_far[i] = (int64_t)t.lev[i].il_src.size();
    }
    inf.near_pairs = 0;
    inf.max_leaf = 0;
    for (int64_t a = 0; a < nleaf; ++a) {
      const int64_t na = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      inf.max_leaf = std::max(inf.max_leaf, na);
      for (int k = t.near_ptr[a]; k < t.near_ptr[a + 1]; ++k)
        inf.near_pairs += na * (int64_t)(t.leaf_ptr[t.near_idx[k] + 1] - t.leaf_ptr[t.near_idx[k]]);
    }
    *out = h.release();
    return NESA_OK;
  });
}

extern "C" nesa_status nesa2d_info_get(const nesa2d* h, nesa2d_info* out) {
  return (nesa_status)guarded2([&]() -> int {
    if (!h || !out) throw Fail(NESA_EINVAL, "null pointer");
    *out = h->info;
    return NESA_OK;
  });
}

extern "C" nesa_status nesa2d_perm(const nesa2d* h, int32_t* perm) {
  return (nesa_status)guarded2([&]() -> int {
    if (!h || !perm) throw Fail(NESA_EINVAL, "null pointer");
    std::memcpy(perm, h->tree.perm.data(), h->tree.perm.size() * sizeof(int32_t));
    return NESA_OK;
  });
}

extern "C" nesa_status nesa2d_matvec(nesa2d* h, const double* q, double* phi, void* stream) {
  return (nesa_status)guarded2([&]() -> int {
    if (!h || !q || !phi) throw Fail(NESA_EINVAL, "null pointer");
    if (q == phi) throw Fail(NESA_EINVAL, "q and phi must be distinct buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Tree2& t = h->tree;
    const int64_t n = h->info.n;
    const int Q = h->info.Q;
    const int nl = t.L - t.l0 + 1;
    const unsigned nleaf = (unsigned)(t.leaf_ptr.size() - 1);
    const unsigned gb = (unsigned)((n + 255) / 256);
    k2_gather<<<gb, 256, 0, st>>>(q, h->ql, h->perm, n);
    const unsigned rchunks = (unsigned)((h->info.max_leaf + NEAR_RW - 1) / NEAR_RW);
    k2_near<<<dim3(nleaf, rchunks), NT2, 0, st>>>(h->Z, h->zoff, h->leaf_ptr, h->near_ptr, h->near_idx, h->ql,
                                                  h->phil);
    k2_radiate<<<nleaf, NT2, 0, st>>>(h->V, h->voff, h->leaf_ptr, h->ql, h->lev[nl - 1].s, Q);
    for (int i = nl - 1; i > 0; --i)
      k2_upward<<<(unsigned)h->lev[i - 1].nbox, NT2, 0, st>>>(h->lev[i].Ccm, h->lev[i - 1].child, h->lev[i].s,
                                                               h->lev[i - 1].s, Q);
    {
      TransLevels tl{};
      tl.n = nl;
      tl.box0[0] = 0;
      for (int i = 0; i < nl; ++i) {
        tl.box0[i + 1] = tl.box0[i] + h->lev[i].nbox;
        tl.Dcm[i] = h->lev[i].Dcm;
        tl.il_ptr[i] = h->lev[i].il_ptr;
        tl.il_src[i] = h->lev[i].il_src;
        tl.il_off[i] = h->lev[i].il_off;
        tl.s[i] = h->lev[i].s;
        tl.o[i] = h->lev[i].o;
      }
      k2_translate<<<(unsigned)tl.box0[nl], NT_TR, 0, st>>>(tl, Q);
    }
    for (int i = 1; i < nl; ++i)
      k2_downward<<<(unsigned)h->lev[i].nbox, NT2, 0, st>>>(h->lev[i].Bcm, h->lev[i].parent, h->lev[i].quad,
                                                             h->lev[i - 1].o, h->lev[i].o, Q);
    k2_receive<<<dim3(nleaf, (unsigned)((h->info.max_leaf + 15) / 16)), NT2, 0, st>>>(h->V, h->voff, h->leaf_ptr,
                                                                                     h->lev[nl - 1].o, h->phil, Q);
    k2_scatter<<<gb, 256, 0, st>>>(h->phil, phi, h->perm, n);
    hip_ok2(hipGetLastError(), "kernel launch");
    return NESA_OK;
  });
}

extern "C" nesa_status nesa2d_free(nesa2d* h) {
  delete h;
  return NESA_OK;
}
