// Near-field preconditioners (host setup, FP64 / FP32 complex).
//
// Restricted additive Schwarz over the near lists: for leaf a with near leaves
// N(a), Z_N is the near-field matrix restricted to the RWGs of N(a) (blocks of
// two leaves of N(a) that are not near each other are not part of the near-
// field matrix and are zero); the preconditioner returns z_a = [Z_N^-1 r_N]_a.
// The rows of Z_N^-1 that belong to leaf a are stored exactly like leaf a's
// near block (S_a x W_a column-major, columns in near-list order), so the GPU
// applies it with the near-field kernel.
#include <algorithm>
#include <cmath>
#include <memory>

#include "nesa_host.h"

namespace nesa {

namespace {

template <typename R>
struct Cx {
  R re, im;
};
template <typename R>
inline Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
inline Cx<R> cdiv(Cx<R> a, Cx<R> b) {
  const R d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// In-place LU with partial pivoting of an n x n column-major complex matrix
// held as separate real and imaginary parts (so that the column updates
// vectorise); piv[k] is the row swapped with row k at step k.
template <typename R>
void lu(R* Ar, R* Ai, int n, std::vector<int>& piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    R best = -1;
    for (int i = k; i < n; ++i) {
      const R m = std::fabs(Ar[(size_t)k * n + i]) + std::fabs(Ai[(size_t)k * n + i]);
      if (m > best) {
        best = m;
        p = i;
      }
    }
    piv[k] = p;
    if (!(best > 0)) throw Error(-1, "singular near-field matrix in the Schwarz preconditioner");
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(Ar[(size_t)j * n + k], Ar[(size_t)j * n + p]);
        std::swap(Ai[(size_t)j * n + k], Ai[(size_t)j * n + p]);
      }
    const Cx<R> d = {Ar[(size_t)k * n + k], Ai[(size_t)k * n + k]};
    R* __restrict__ kr = Ar + (size_t)k * n;
    R* __restrict__ ki = Ai + (size_t)k * n;
    for (int i = k + 1; i < n; ++i) {
      const Cx<R> q = cdiv(Cx<R>{kr[i], ki[i]}, d);
      kr[i] = q.re;
      ki[i] = q.im;
    }
    for (int j = k + 1; j < n; ++j) {
      R* __restrict__ jr = Ar + (size_t)j * n;
      R* __restrict__ ji = Ai + (size_t)j * n;
      const R fr = jr[k], fi = ji[k];
      if (fr == 0 && fi == 0) continue;
      for (int i = k + 1; i < n; ++i) {
        jr[i] -= kr[i] * fr - ki[i] * fi;
        ji[i] -= kr[i] * fi + ki[i] * fr;
      }
    }
  }
}

// Solve (LU) x = b in place for one right-hand side.
template <typename R>
void lu_solve(const R* Ar, const R* Ai, int n, const std::vector<int>& piv, Cx<R>* b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) std::swap(b[k], b[piv[k]]);
  for (int j = 0; j < n; ++j) {
    const Cx<R> bj = b[j];
    for (int i = j + 1; i < n; ++i) {
      const Cx<R> l = {Ar[(size_t)j * n + i], Ai[(size_t)j * n + i]};
      b[i].re -= l.re * bj.re - l.im * bj.im;
      b[i].im -= l.re * bj.im + l.im * bj.re;
    }
  }
  for (int j = n - 1; j >= 0; --j) {
    b[j] = cdiv(b[j], Cx<R>{Ar[(size_t)j * n + j], Ai[(size_t)j * n + j]});
    const Cx<R> bj = b[j];
    for (int i = 0; i < j; ++i) {
      const Cx<R> u = {Ar[(size_t)j * n + i], Ai[(size_t)j * n + i]};
      b[i].re -= u.re * bj.re - u.im * bj.im;
      b[i].im -= u.re * bj.im + u.im * bj.re;
    }
  }
}

template <typename R>
void schwarz_leaf(const Tree& t, const Near& nr, int64_t a, std::vector<cd>& out) {
  const int64_t na = t.near_ptr[a + 1] - t.near_ptr[a];
  std::vector<int64_t> nb(na), off(na + 1, 0);
  for (int64_t i = 0; i < na; ++i) {
    nb[i] = t.near_idx[t.near_ptr[a] + i];
    off[i + 1] = off[i] + (t.leaf_ptr[nb[i] + 1] - t.leaf_ptr[nb[i]]);
  }
  const int W = (int)off[na];
  // T = Z_N^T, column-major: T[i][j] = Z_N[j][i] (real and imaginary parts apart)
  std::vector<R> Tr((size_t)W * W, R(0)), Ti((size_t)W * W, R(0));
  for (int64_t i = 0; i < na; ++i) {
    const int64_t b = nb[i];
    const int64_t Sb = t.leaf_ptr[b + 1] - t.leaf_ptr[b];
    const cd* Zb = &nr.z[nr.off[b]];
    // columns of b's near block: leaves of N(b) in list order
    int64_t cb = 0;
    for (int64_t q = t.near_ptr[b]; q < t.near_ptr[b + 1]; ++q) {
      const int64_t c = t.near_idx[q];
      const int64_t Sc = t.leaf_ptr[c + 1] - t.leaf_ptr[c];
      const auto it = std::find(nb.begin(), nb.end(), c);
      if (it != nb.end()) {
        const int64_t j = it - nb.begin();
        for (int64_t cc = 0; cc < Sc; ++cc)
          for (int64_t rr = 0; rr < Sb; ++rr) {
            const cd v = Zb[(cb + cc) * Sb + rr];          // Z_N[off_i + rr][off_j + cc]
            Tr[(size_t)(off[i] + rr) * W + off[j] + cc] = (R)v.real();
            Ti[(size_t)(off[i] + rr) * W + off[j] + cc] = (R)v.imag();
          }
      }
      cb += Sc;
    }
  }
  std::vector<int> piv;
  lu(Tr.data(), Ti.data(), W, piv);
  // rows of Z_N^-1 for leaf a: solve Z_N^T y = e_r for every RWG r of a
  const int64_t ia = std::find(nb.begin(), nb.end(), a) - nb.begin();
  const int64_t Sa = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
  out.assign((size_t)Sa * W, cd(0, 0));
  std::vector<Cx<R>> y(W);
  for (int64_t r = 0; r < Sa; ++r) {
    std::fill(y.begin(), y.end(), Cx<R>{0, 0});
    y[off[ia] + r] = {1, 0};
    lu_solve(Tr.data(), Ti.data(), W, piv, y.data());
    for (int j = 0; j < W; ++j) out[(size_t)j * Sa + r] = cd(y[j].re, y[j].im);   // column-major S_a x W
  }
}

}  // namespace

Near* near_schwarz(const Tree& t, const Near& nr, bool single) {
  std::unique_ptr<Near> P(new Near());
  P->k = nr.k;
  P->eta = nr.eta;
  P->off = nr.off;
  P->z.assign(nr.z.size(), cd(0, 0));
  const int64_t nleaf = t.level(t.L).nbox;
  parallel_for(nleaf, [&](int64_t a) {
    std::vector<cd> blk;
    if (single)
      schwarz_leaf<float>(t, nr, a, blk);
    else
      schwarz_leaf<double>(t, nr, a, blk);
    std::copy(blk.begin(), blk.end(), P->z.begin() + nr.off[a]);
  });
  return P.release();
}

}  // namespace nesa
