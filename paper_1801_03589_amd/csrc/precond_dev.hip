// Restricted additive Schwarz preconditioner assembled on the device
// (complex64 operators).  For leaf a with near leaves N(a), Z_N is the
// near-field matrix restricted to the RWGs of N(a) (blocks of two leaves of
// N(a) that are not near each other are zero); the preconditioner keeps the
// rows of Z_N^-1 that belong to leaf a, in the layout of leaf a's near block
// (S_a x W_a column-major, columns in near-list order).  Those rows are the
// solutions y_r of T y_r = e_r with T = Z_N^T, one per RWG r of leaf a.
//
// Persistent workgroups (as many as fit the device at once) take the leaves,
// largest first, from a counter.  For each the workgroup builds T (W x W
// column-major, FP32 complex) from the near blocks in its own workspace,
// factors T = P^T L U (right-looking LU with partial pivoting: pivot = the
// largest |re| + |im| on or below the diagonal, the first such row; panels of
// 32 columns factored in sub-panels of 8; complex updates on the FP32 matrix
// cores) and solves T y_r = e_r for the S_a RWGs r of leaf a, in place in the
// preconditioner's arena (element (r, j) of leaf a's block is y_r[j]).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "precond_dev.h"

namespace nesa {

namespace {

constexpr int SW_NT = 256;
constexpr int SW_NB = 32;      // panel width of the factorisation, block size of the solves
constexpr int SW_NS = 8;       // sub-panel width
constexpr int SW_TM = 64;      // GEMM tile (rows and columns)
constexpr int SW_MAXN = SCHWARZ_MAXN;

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_div(float2 a, float2 b) {
  const float d = b.x * b.x + b.y * b.y;
  return make_float2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

struct SwLds {
  union {
    struct {
      float2 As[SW_NB * SW_TM];          // GEMM: A tile, As[q][i]
      float2 Bs[SW_NB * (SW_TM + 1)];    // GEMM: B tile, Bs[q][j] (rows padded)
    };
    struct {                             // gather
      short seg[SCHWARZ_WMAX];           // near leaf (entry of N(a)) of every RWG of N(a)
      int cps[SW_MAXN * SW_MAXN];
      int nbs[SW_MAXN], offs[SW_MAXN + 1];
      int64_t zho[SW_MAXN];
    };
  };
  float2 Ls[SW_NB * SW_NB];          // triangular block, Ls[q][i] = T(k0 + i, k0 + q)
  float rv[SW_NT / 64];
  int ri[SW_NT / 64];
  int mv_dst[2 * SW_NB], mv_src[2 * SW_NB];
  int nmv;
  int item;      // entry of the leaf order taken by the workgroup
  int first;     // first step of the forward solve that touches a nonzero row
};

// T[j W + i] = Z_N[j][i]: row j of Z_N is RWG jr of leaf lb = nb[jb], column
// i is RWG ic of leaf lc = nb[ib].  The near field is read from its
// reciprocity half storage (leaf x keeps Z_xy for its near leaves y >= x,
// S_x rows, columns in near-list order from its own on): for lc >= lb the
// entry is element (jr, colpos + ic) of lb's half block, for lc < lb it is
// element (ic, colpos + jr) of lc's (Z_{lb lc} = Z_{lc lb}^T); colpos < 0 when
// the two leaves are not near each other (zero block).  Column j of T at a
// time, threads along i.
__device__ void sw_gather(SwLds& s, const SchwarzWork& b, int a, float2* T, const float2* __restrict__ Zh,
                          const int64_t* __restrict__ zh_off) {
  const int t = threadIdx.x;
  const int na = b.na[a], W = b.W[a];
  __syncthreads();
  for (int e = t; e < na * na; e += SW_NT)
    s.cps[e] = b.colpos[(int64_t)a * SW_MAXN * SW_MAXN + (e / na) * SW_MAXN + e % na];
  if (t < na) {
    const int l = b.nb[(int64_t)a * SW_MAXN + t];
    s.nbs[t] = l;
    s.zho[t] = zh_off[l];
  }
  if (t <= na) s.offs[t] = b.off[(int64_t)a * (SW_MAXN + 1) + t];
  __syncthreads();
  for (int i = t; i < W; i += SW_NT) {
    int k = 0;
    while (k + 1 < na && s.offs[k + 1] <= i) ++k;
    s.seg[i] = (short)k;
  }
  __syncthreads();
  for (int j = 0; j < W; ++j) {
    const int jb = s.seg[j], jr = j - s.offs[jb], Sj = s.offs[jb + 1] - s.offs[jb], lb = s.nbs[jb];
    float2* col = T + (int64_t)j * W;
    for (int i = t; i < W; i += SW_NT) {
      const int ib = s.seg[i], cp = s.cps[jb * na + ib];
      float2 v = make_float2(0.f, 0.f);
      if (cp >= 0) {
        const int ic = i - s.offs[ib];
        if (s.nbs[ib] >= lb)
          v = Zh[s.zho[jb] + (int64_t)(cp + ic) * Sj + jr];
        else
          v = Zh[s.zho[ib] + (int64_t)(cp + jr) * (s.offs[ib + 1] - s.offs[ib]) + ic];
      }
      col[i] = v;
    }
  }
  __syncthreads();
}

// Columns [c0, c1) of a panel whose columns are [p0, p1): for every column the
// pivot (largest |re| + |im| on or below the diagonal, the first such row), the
// row swap across the panel's columns, the multipliers and the rank-1 update of
// the columns up to c1 (row-owned; the updated next column's pivot search is
// taken on the way).
__device__ void sw_factor_cols(SwLds& s, float2* T, int W, int c0, int c1, int p0, int p1, int32_t* piv,
                               int32_t* status) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  float best = -1.f;
  int bi = W;
  for (int i = c0 + t; i < W; i += SW_NT) {
    const float2 v = T[(int64_t)c0 * W + i];
    const float m = fabsf(v.x) + fabsf(v.y);
    if (m > best) {
      best = m;
      bi = i;
    }
  }
  for (int c = c0; c < c1; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float v2 = __shfl_xor(best, o);
      const int i2 = __shfl_xor(bi, o);
      if (v2 > best || (v2 == best && i2 < bi)) {
        best = v2;
        bi = i2;
      }
    }
    if (lane == 0) {
      s.rv[wv] = best;
      s.ri[wv] = bi;
    }
    __syncthreads();
    float bv = s.rv[0];
    int bix = s.ri[0];
#pragma unroll
    for (int w = 1; w < SW_NT / 64; ++w)
      if (s.rv[w] > bv || (s.rv[w] == bv && s.ri[w] < bix)) {
        bv = s.rv[w];
        bix = s.ri[w];
      }
    const int p = bix < W ? bix : c;
    if (t == 0) {
      piv[c] = p;
      if (!(bv > 0.f)) status[0] = 1;
    }
    if (p != c && t < p1 - p0) {
      float2* col = T + (int64_t)(p0 + t) * W;
      const float2 x = col[c];
      col[c] = col[p];
      col[p] = x;
    }
    __syncthreads();
    const float2 d = T[(int64_t)c * W + c];
    float2 u[SW_NS - 1];
#pragma unroll
    for (int jj = 0; jj < SW_NS - 1; ++jj)
      u[jj] = (c + 1 + jj < c1) ? T[(int64_t)(c + 1 + jj) * W + c] : make_float2(0.f, 0.f);
    best = -1.f;
    bi = W;
    float2* cc = T + (int64_t)c * W;
    for (int i = c + 1 + t; i < W; i += SW_NT) {
      const float2 l = c_div(cc[i], d);
      cc[i] = l;
#pragma unroll
      for (int jj = 0; jj < SW_NS - 1; ++jj) {
        if (c + 1 + jj < c1) {
          float2* cj = T + (int64_t)(c + 1 + jj) * W;
          float2 v = cj[i];
          v.x -= l.x * u[jj].x - l.y * u[jj].y;
          v.y -= l.x * u[jj].y + l.y * u[jj].x;
          cj[i] = v;
          if (jj == 0) {
            const float m = fabsf(v.x) + fabsf(v.y);
            if (m > best) {
              best = m;
              bi = i;
            }
          }
        }
      }
    }
  }
  __syncthreads();
}

// Diagonal block T[k0 .. k0 + nb)^2 into s.Ls, the NBT x NBT frame padded with
// the identity (so that the padded unknowns stay zero in either solve).
template <int NBT>
__device__ void sw_stage_tri(SwLds& s, const float2* T, int W, int k0, int nb) {
  __syncthreads();
  for (int e = threadIdx.x; e < NBT * NBT; e += SW_NT) {
    const int q = e / NBT, i = e % NBT;
    float2 v = make_float2(i == q ? 1.f : 0.f, 0.f);
    if (q < nb && i < nb) v = T[(int64_t)(k0 + q) * W + k0 + i];
    s.Ls[q * SW_NB + i] = v;
  }
  __syncthreads();
}

// X = L^-1 X (L unit lower, from s.Ls) or X = U^-1 X (U upper, non-unit) for
// ncols columns of nb <= NBT rows: element (q, j) of X at X[q rs + j cs]; one
// column per thread, in blocks of 8 rows: a block is solved in registers,
// then every later (lower) or earlier (upper) block of the column is loaded
// whole, updated and stored.
template <int NBT, bool UPPER>
__device__ void sw_trsm(SwLds& s, int nb, float2* X, int64_t rs, int64_t cs, int ncols) {
  constexpr int R = 8, NR = NBT / R;
  static_assert(NBT % R == 0, "blocks of 8 rows");
  for (int j = threadIdx.x; j < ncols; j += SW_NT) {
    float2* x = X + j * cs;
#pragma unroll 1
    for (int bb = 0; bb < NR; ++bb) {
      const int rb = UPPER ? (NR - 1 - bb) * R : bb * R;
      if (rb >= nb) continue;
      float2 y[R];
#pragma unroll
      for (int q = 0; q < R; ++q) y[q] = rb + q < nb ? x[(rb + q) * rs] : make_float2(0.f, 0.f);
      if (!UPPER) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int i = q + 1; i < R; ++i) {
            const float2 l = s.Ls[(rb + q) * SW_NB + rb + i];
            y[i].x -= l.x * y[q].x - l.y * y[q].y;
            y[i].y -= l.x * y[q].y + l.y * y[q].x;
          }
      } else {
#pragma unroll
        for (int q = R - 1; q >= 0; --q) {
          y[q] = c_div(y[q], s.Ls[(rb + q) * SW_NB + rb + q]);
#pragma unroll
          for (int i = 0; i < q; ++i) {
            const float2 uv = s.Ls[(rb + q) * SW_NB + rb + i];
            y[i].x -= uv.x * y[q].x - uv.y * y[q].y;
            y[i].y -= uv.x * y[q].y + uv.y * y[q].x;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (rb + q < nb) x[(rb + q) * rs] = y[q];
      const int ib0 = UPPER ? 0 : rb + R, ib1 = UPPER ? rb : nb;
#pragma unroll 1
      for (int ib = ib0; ib < ib1; ib += R) {
        float2 z[R];
#pragma unroll
        for (int i = 0; i < R; ++i) z[i] = ib + i < ib1 ? x[(ib + i) * rs] : make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const float2 l = s.Ls[(rb + q) * SW_NB + ib + i];
            z[i].x -= l.x * y[q].x - l.y * y[q].y;
            z[i].y -= l.x * y[q].y + l.y * y[q].x;
          }
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (ib + i < ib1) x[(ib + i) * rs] = z[i];
      }
    }
  }
}

// C -= A B for m x n, inner size kb <= SW_NB (32-bit element offsets: every
// operand lies inside one leaf's matrix or arena): A(i, q) = A[q lda + i], B(q, j)
// at B[q + j ldb] (BQ) or B[q ldb + j], C(i, j) at C[i + j ldc] (CI) or
// C[i ldc + j].  64 x 64 tiles with A and B staged through LDS; each wave
// takes a 32 x 32 quarter as 2 x 2 FP32 matrix-core tiles of 16 x 16
// (v_mfma_f32_16x16x4f32, four real products per complex product).  With a
// column-major C the transposed product C^T -= B^T A^T is formed, so that the
// 16 consecutive output columns of an instruction are consecutive rows of C.
template <bool BQ, bool CI>
__device__ void sw_gemm(SwLds& s, const float2* A, int lda, const float2* B, int ldb, float2* C, int ldc, int m,
                        int n, int kb) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32, l16 = lane & 15, lq = lane >> 4;
  for (int tm = 0; tm < m; tm += SW_TM) {
    __syncthreads();
    for (int e = t; e < SW_TM * SW_NB; e += SW_NT) {
      const int i = e % SW_TM, q = e / SW_TM;
      s.As[q * SW_TM + i] = (q < kb && tm + i < m) ? A[q * lda + tm + i] : make_float2(0.f, 0.f);
    }
    // B tiles go through registers: the next tile's loads, and this tile's C
    // values, are in flight during the matrix-core products
    constexpr int NBE = SW_TM * SW_NB / SW_NT;
    float2 rb[NBE];
    auto load_b = [&](int tn) {
#pragma unroll
      for (int k = 0; k < NBE; ++k) {
        const int e = t + k * SW_NT;
        const int q = BQ ? e % SW_NB : e / SW_TM, j = BQ ? e / SW_NB : e % SW_TM;
        rb[k] = make_float2(0.f, 0.f);
        if (q < kb && tn + j < n) rb[k] = BQ ? B[q + (tn + j) * ldb] : B[q * ldb + tn + j];
      }
    };
    load_b(0);
    for (int tn = 0; tn < n; tn += SW_TM) {
      if (tn > 0) __syncthreads();
#pragma unroll
      for (int k = 0; k < NBE; ++k) {
        const int e = t + k * SW_NT;
        const int q = BQ ? e % SW_NB : e / SW_TM, j = BQ ? e / SW_NB : e % SW_TM;
        s.Bs[q * (SW_TM + 1) + j] = rb[k];
      }
      __syncthreads();
      if (tn + SW_TM < n) load_b(tn + SW_TM);
      // accumulator element e of tile (u, v): matrix-core row 16 u + 4 lq + e,
      // column 16 v + l16
      float2 cv[2][2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = CI ? tm + wr + 16 * v + l16 : tm + wr + 16 * u + 4 * lq + e;
            const int j = CI ? tn + wc + 16 * u + 4 * lq + e : tn + wc + 16 * v + l16;
            cv[u][v][e] = make_float2(0.f, 0.f);
            if (i < m && j < n) cv[u][v][e] = CI ? C[i + j * ldc] : C[i * ldc + j];
          }
      floatx4 re[2][2], im[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          re[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
          im[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll 2
      for (int kk = 0; kk < kb; kk += 4) {
        const int q = kk + lq;
        float2 x[2], y[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const float2 av = s.As[q * SW_TM + wr + 16 * u + l16];
          const float2 bv = s.Bs[q * (SW_TM + 1) + wc + 16 * u + l16];
          x[u] = CI ? bv : av;
          y[u] = CI ? av : bv;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            re[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].x, y[v].x, re[u][v], 0, 0, 0);
            re[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x[u].y, y[v].y, re[u][v], 0, 0, 0);
            im[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].x, y[v].y, im[u][v], 0, 0, 0);
            im[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].y, y[v].x, im[u][v], 0, 0, 0);
          }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = CI ? tm + wr + 16 * v + l16 : tm + wr + 16 * u + 4 * lq + e;
            const int j = CI ? tn + wc + 16 * u + 4 * lq + e : tn + wc + 16 * v + l16;
            if (i < m && j < n) {
              float2& c = CI ? C[i + j * ldc] : C[i * ldc + j];
              c = make_float2(cv[u][v][e].x - re[u][v][e], cv[u][v][e].y - im[u][v][e]);
            }
          }
    }
  }
  __syncthreads();
}

// The net row moves of the swaps of rows k0 .. k0 + kb (in order; row k0 + c
// with piv[k0 + c] >= k0 + c): rows involved in lanes of the first wave,
// their final contents by simulation, the moves (dst <- src) into s.mv_*.
__device__ void sw_build_moves(SwLds& s, const int32_t* piv, int k0, int kb) {
  const int t = threadIdx.x, lane = t & 63;
  if (t < 64) {
    int pos = lane < kb ? k0 + lane : -1;
    int np = kb;
    for (int c = 0; c < kb; ++c) {
      const int p = piv[k0 + c];
      if (p >= k0 + kb && __ballot(pos == p) == 0) {
        if (lane == np) pos = p;
        ++np;
      }
    }
    int content = lane;
    for (int c = 0; c < kb; ++c) {
      const int p = piv[k0 + c];
      const int b = __ffsll((unsigned long long)__ballot(pos == p)) - 1;
      const int ca = __shfl(content, c), cb = __shfl(content, b);
      if (lane == c) content = cb;
      if (lane == b) content = ca;
    }
    const int src = __shfl(pos, content);
    const bool mv = lane < np && content != lane;
    const unsigned long long mm = __ballot(mv);
    if (mv) {
      const int idx = __popcll(mm & ((1ull << lane) - 1ull));
      s.mv_dst[idx] = pos;
      s.mv_src[idx] = src;
    }
    if (lane == 0) s.nmv = __popcll(mm);
  }
  __syncthreads();
}

// The moves applied to ncols columns: element (row, col) at X[row rs + col cs];
// four threads per column take 16 moves each, all loads before any store.
__device__ void sw_apply_moves(SwLds& s, float2* X, int64_t rs, int64_t cs, int ncols) {
  const int nmv = s.nmv;
  if (nmv == 0) return;
  const int t = threadIdx.x, chunk = t & 3;
  for (int cb = 0; cb < ncols; cb += SW_NT / 4) {
    const int col = cb + (t >> 2);
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int m = chunk + 4 * k;
      if (m < nmv && col < ncols) v[k] = X[s.mv_src[m] * rs + col * cs];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int m = chunk + 4 * k;
      if (m < nmv && col < ncols) X[s.mv_dst[m] * rs + col * cs] = v[k];
    }
  }
  __syncthreads();
}

// Leaf a by one workgroup: T = P^T L U (right-looking, panels of SW_NB columns
// factored in sub-panels of SW_NS; a panel's swaps are applied to its own
// columns at once and to the columns right of it before their update, never
// to the columns left of it), then Y = U^-1 L^-1 P E for the unit vectors of
// leaf a's RWGs, the swaps replayed panel by panel in the forward solve.
__device__ void sw_leaf(SwLds& s, const SchwarzWork& b, int a, float2* T, int32_t* piv, float2* __restrict__ out,
                        const int64_t* __restrict__ zoff, const int32_t* __restrict__ leaf_ptr) {
  const int W = b.W[a], r0 = b.rowa[a];
  const int S = leaf_ptr[a + 1] - leaf_ptr[a];
  for (int k0 = 0; k0 < W; k0 += SW_NB) {
    const int kb = min(SW_NB, W - k0), k1 = k0 + kb;
    for (int s0 = k0; s0 < k1; s0 += SW_NS) {
      const int s1 = min(s0 + SW_NS, k1);
      sw_factor_cols(s, T, W, s0, s1, k0, k1, piv, b.status);
      if (s1 < k1) {
        sw_stage_tri<SW_NS>(s, T, W, s0, s1 - s0);
        sw_trsm<SW_NS, false>(s, s1 - s0, T + (int64_t)s1 * W + s0, 1, W, k1 - s1);
        sw_gemm<true, true>(s, T + (int64_t)s0 * W + s1, W, T + (int64_t)s1 * W + s0, W, T + (int64_t)s1 * W + s1, W,
                            W - s1, k1 - s1, s1 - s0);
      }
    }
    if (k1 < W) {
      sw_build_moves(s, piv, k0, kb);
      sw_apply_moves(s, T + (int64_t)k1 * W, 1, W, W - k1);
      sw_stage_tri<SW_NB>(s, T, W, k0, kb);
      sw_trsm<SW_NB, false>(s, kb, T + (int64_t)k1 * W + k0, 1, W, W - k1);
      sw_gemm<true, true>(s, T + (int64_t)k0 * W + k1, W, T + (int64_t)k1 * W + k0, W, T + (int64_t)k1 * W + k1, W,
                          W - k1, W - k1, kb);
    }
  }
  // Y[j S + r] = y_r[j]: the arena of leaf a (S x W column-major)
  float2* Y = out + zoff[a];
  for (int e = threadIdx.x; e < S * W; e += SW_NT) {
    const int r = e % S, j = e / S;
    Y[e] = make_float2(j == r0 + r ? 1.f : 0.f, 0.f);
  }
  // rows above r0 of P E are zero and stay so through every step c < r0 whose
  // pivot row is above r0 too: the forward solve starts at the block of the
  // first other step
  if (threadIdx.x == 0) s.first = r0;
  __syncthreads();
  for (int c = threadIdx.x; c < r0; c += SW_NT)
    if (piv[c] >= r0) atomicMin(&s.first, c);
  __syncthreads();
  const int kfirst = s.first / SW_NB * SW_NB;
  for (int k0 = kfirst; k0 < W; k0 += SW_NB) {
    const int kb = min(SW_NB, W - k0), k1 = k0 + kb;
    sw_build_moves(s, piv, k0, kb);
    sw_apply_moves(s, Y, S, 1, S);
    sw_stage_tri<SW_NB>(s, T, W, k0, kb);
    sw_trsm<SW_NB, false>(s, kb, Y + (int64_t)k0 * S, S, 1, S);
    if (k1 < W)
      sw_gemm<false, false>(s, T + (int64_t)k0 * W + k1, W, Y + (int64_t)k0 * S, S, Y + (int64_t)k1 * S, S, W - k1, S, kb);
  }
  for (int k0 = (W - 1) / SW_NB * SW_NB; k0 >= 0; k0 -= SW_NB) {
    const int kb = min(SW_NB, W - k0);
    sw_stage_tri<SW_NB>(s, T, W, k0, kb);
    sw_trsm<SW_NB, true>(s, kb, Y + (int64_t)k0 * S, S, 1, S);
    if (k0 > 0) sw_gemm<false, false>(s, T + (int64_t)k0 * W, W, Y + (int64_t)k0 * S, S, Y, S, k0, S, kb);
  }
}

// Persistent workgroups, each with its own W x W matrix and pivots, take the
// leaves in order from the counter until none is left.
__global__ __launch_bounds__(SW_NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_schwarz(
    SchwarzWork b, const float2* __restrict__ Zh, const int64_t* __restrict__ zh_off, float2* __restrict__ out,
    const int64_t* __restrict__ zoff, const int32_t* __restrict__ leaf_ptr) {
  __shared__ SwLds s;
  float2* T = b.ws + (int64_t)blockIdx.x * b.ws_stride;
  int32_t* piv = b.piv + (int64_t)blockIdx.x * b.piv_stride;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s.item = atomicAdd(b.counter, 1);
    __syncthreads();
    const int it = s.item;
    if (it >= b.nleaf) break;
    const int a = b.order[it];
    sw_gather(s, b, a, T, Zh, zh_off);
    sw_leaf(s, b, a, T, piv, out, zoff, leaf_ptr);
  }
}

}  // namespace

int schwarz_slots() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_schwarz, SW_NT, 0) != hipSuccess) return 0;
  return cus * per;
}

void launch_schwarz(const float2* Zh, const int64_t* zh_off, const int64_t* zoff, const int32_t* leaf_ptr,
                    const SchwarzWork& w, int slots, float2* out, hipStream_t st) {
  if (w.nleaf <= 0 || slots <= 0) return;
  (void)hipMemsetAsync(w.counter, 0, sizeof(int32_t), st);
  k_schwarz<<<(unsigned)slots, SW_NT, 0, st>>>(w, Zh, zh_off, out, zoff, leaf_ptr);
}

}  // namespace nesa
