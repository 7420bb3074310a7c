// Leaf-level stages of products with many right-hand sides on the FP32
// matrix cores (complex64): near field (Eq. 9), radiation (Eq. 10) and
// reception (Eq. 14).  With R right-hand sides each is a small complex GEMM per
// leaf whose third dimension is R:
//   near field  y_a[m][r]  = sum_k Z_a[m][k] x_r[pos(k)]   (K = W_a, columns m < S_a)
//   radiation   s_b[j][r]  = sum_i V[p0 + i][j] x_r[p0 + i] (K = S_b, columns j < 4 Q)
//   reception   y_a[m][r] += sum_j V[p0 + m][j] w_j o_a[j][r] (K = 4 Q, columns m < S_a)
// One workgroup per (leaf, block of 64 right-hand sides) forms the transposed
// product out^T (64 x ncol) = A (64 x K) B (K x ncol) with A the right-hand-side
// operand: each wave owns 16 right-hand sides, the columns go in groups of 64
// (four 16 x 16 tiles), K in chunks of 32 staged through LDS (four workgroups
// per CU), complex products
// as four real v_mfma_f32_16x16x4f32.  Output columns run along the
// contiguous dimension of every destination.  Each output element is written
// by one lane, sums in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace nesa {

namespace {

constexpr int LG_NT = 256;
constexpr int LG_KC = 32;        // K per staged chunk
constexpr int LG_CG = 64;        // output columns per group (four tiles of 16)
constexpr int LG_PAD = 65;       // LDS row stride (float2)
constexpr int LG_MAXN = 128;     // near-list entries per leaf

typedef float lg_f4 __attribute__((ext_vector_type(4)));

struct LgLds {
  float2 As[LG_KC * LG_PAD];       // As[k][r]
  float2 Bs[LG_KC * LG_PAD];       // Bs[k][c]
  int posk[LG_KC];
  int seg_col[LG_MAXN + 1];
  int seg_x[LG_MAXN];
};

// out^T(r, c) for r < 64, c < ncol, K terms: la(r, k0, kl) and lb(k0, kl, c)
// give the operands of term k0 + kl (zero past the data), prep(k0, kc) runs
// before each chunk is staged (all threads), st(r, c, v) takes the result.
// AKF / BKF: the operand is contiguous along k (staging threads run along k),
// else along r / c.
template <bool AKF, bool BKF, class PR, class LA, class LB, class ST>
__device__ void lg_gemm(LgLds& s, int K, int ncol, PR prep, LA la, LB lb, ST st) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, l16 = lane & 15, lq = lane >> 4;
  for (int cg = 0; cg < ncol; cg += LG_CG) {
    lg_f4 re[4], im[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      re[ct] = lg_f4{0.f, 0.f, 0.f, 0.f};
      im[ct] = lg_f4{0.f, 0.f, 0.f, 0.f};
    }
    for (int k0 = 0; k0 < K; k0 += LG_KC) {
      const int kc = min(LG_KC, K - k0);
      __syncthreads();
      prep(k0, kc);
      __syncthreads();
#pragma unroll 4
      for (int u = 0; u < LG_KC * 64 / LG_NT; ++u) {
        const int e = t + u * LG_NT;
        const int k = AKF ? e % LG_KC : e / 64, r = AKF ? e / LG_KC : e % 64;
        s.As[k * LG_PAD + r] = k < kc ? la(r, k0, k) : make_float2(0.f, 0.f);
      }
#pragma unroll 4
      for (int u = 0; u < LG_KC * LG_CG / LG_NT; ++u) {
        const int e = t + u * LG_NT;
        const int k = BKF ? e % LG_KC : e / LG_CG, c = BKF ? e / LG_KC : e % LG_CG;
        s.Bs[k * LG_PAD + c] = (k < kc && cg + c < ncol) ? lb(k0, k, cg + c) : make_float2(0.f, 0.f);
      }
      __syncthreads();
      const int ksteps = (kc + 3) / 4;
      for (int ks = 0; ks < ksteps; ++ks) {
        const int k = 4 * ks + lq;
        const float2 a = s.As[k * LG_PAD + w * 16 + l16];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const float2 b = s.Bs[k * LG_PAD + ct * 16 + l16];
          re[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, re[ct], 0, 0, 0);
          re[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, re[ct], 0, 0, 0);
          im[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, im[ct], 0, 0, 0);
          im[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, im[ct], 0, 0, 0);
        }
      }
    }
    // element i of tile ct: row 4 lq + i of the wave's 16, column 16 ct + l16
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int c = cg + ct * 16 + l16;
      if (c < ncol)
#pragma unroll
        for (int i = 0; i < 4; ++i) st(w * 16 + 4 * lq + i, c, make_float2(re[ct][i], im[ct][i]));
    }
  }
}

__global__ __launch_bounds__(LG_NT) void k_near_mfma(const float2* __restrict__ Z, const int64_t* __restrict__ zoff,
                                                     const int32_t* __restrict__ leaf_ptr,
                                                     const int32_t* __restrict__ near_ptr,
                                                     const int32_t* __restrict__ near_idx,
                                                     const float2* __restrict__ x, float2* __restrict__ y, int R,
                                                     int64_t n) {
  __shared__ LgLds s;
  const int a = blockIdx.x, r0 = blockIdx.y * 64;
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int n0 = near_ptr[a], nn = near_ptr[a + 1] - n0;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int k = 0; k < nn; ++k) {
      const int b = near_idx[n0 + k];
      s.seg_col[k] = c;
      s.seg_x[k] = leaf_ptr[b];
      c += leaf_ptr[b + 1] - leaf_ptr[b];
    }
    s.seg_col[nn] = c;
  }
  __syncthreads();
  const int W = s.seg_col[nn];
  const float2* Za = Z + zoff[a];
  auto prep = [&](int k0, int kc) {
    const int t = threadIdx.x;
    if (t < kc) {
      const int col = k0 + t;
      int k = 0;
      while (s.seg_col[k + 1] <= col) ++k;
      s.posk[t] = s.seg_x[k] + (col - s.seg_col[k]);
    }
  };
  auto la = [&](int r, int, int kl) {
    return r0 + r < R ? x[(int64_t)(r0 + r) * n + s.posk[kl]] : make_float2(0.f, 0.f);
  };
  auto lb = [&](int k0, int kl, int c) { return Za[(int64_t)(k0 + kl) * S + c]; };
  auto st = [&](int r, int c, float2 v) {
    if (r0 + r < R) y[(int64_t)(r0 + r) * n + p0 + c] = v;
  };
  lg_gemm<true, false>(s, W, S, prep, la, lb, st);
}

__global__ __launch_bounds__(LG_NT) void k_radiate_mfma(const float2* __restrict__ V, const float2* __restrict__ x,
                                                        const int32_t* __restrict__ leaf_ptr,
                                                        float2* __restrict__ sv, int Q, int R, int64_t n) {
  __shared__ LgLds s;
  const int b = blockIdx.x, r0 = blockIdx.y * 64;
  const int p0 = leaf_ptr[b], S = leaf_ptr[b + 1] - p0;
  const int J = 4 * Q;
  auto prep = [](int, int) {};
  auto la = [&](int r, int k0, int kl) {
    return r0 + r < R ? x[(int64_t)(r0 + r) * n + p0 + k0 + kl] : make_float2(0.f, 0.f);
  };
  auto lb = [&](int k0, int kl, int c) { return V[(int64_t)(p0 + k0 + kl) * J + c]; };
  auto st = [&](int r, int c, float2 v) {
    if (r0 + r < R) {
      const int ch = c / Q, q = c - ch * Q;
      sv[(((int64_t)b * 4 + ch) * R + r0 + r) * Q + q] = v;
    }
  };
  lg_gemm<true, false>(s, S, J, prep, la, lb, st);
}

__global__ __launch_bounds__(LG_NT) void k_recv_mfma(const float2* __restrict__ V, const float2* __restrict__ o,
                                                     const int32_t* __restrict__ leaf_ptr, float2* __restrict__ y,
                                                     int Q, int R, int64_t n, float wr_xyz, float wi_xyz, float wr_d,
                                                     float wi_d) {
  __shared__ LgLds s;
  const int a = blockIdx.x, r0 = blockIdx.y * 64;
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int J = 4 * Q;
  auto prep = [](int, int) {};
  auto la = [&](int r, int k0, int kl) {
    float2 v = make_float2(0.f, 0.f);
    if (r0 + r < R) {
      const int j = k0 + kl, ch = j / Q, q = j - ch * Q;
      const float2 ov = o[(((int64_t)a * 4 + ch) * R + r0 + r) * Q + q];
      const float wr = ch < 3 ? wr_xyz : wr_d, wi = ch < 3 ? wi_xyz : wi_d;
      v = make_float2(ov.x * wr - ov.y * wi, ov.x * wi + ov.y * wr);
    }
    return v;
  };
  auto lb = [&](int k0, int kl, int c) { return V[(int64_t)(p0 + c) * J + k0 + kl]; };
  auto st = [&](int r, int c, float2 v) {
    if (r0 + r < R) {
      float2* yp = y + (int64_t)(r0 + r) * n + p0 + c;
      float2 out = *yp;
      out.x += v.x;
      out.y += v.y;
      *yp = out;
    }
  };
  lg_gemm<true, true>(s, J, S, prep, la, lb, st);
}

}  // namespace

void launch_near_mfma(const float2* Z, const int64_t* zoff, const int32_t* leaf_ptr, const int32_t* near_ptr,
                      const int32_t* near_idx, const float2* x, float2* y, int64_t nleaf, int R, int64_t n,
                      hipStream_t st) {
  if (nleaf == 0 || R <= 0) return;
  k_near_mfma<<<dim3((unsigned)nleaf, (unsigned)((R + 63) / 64)), LG_NT, 0, st>>>(Z, zoff, leaf_ptr, near_ptr,
                                                                                  near_idx, x, y, R, n);
}

void launch_radiate_mfma(const float2* V, const float2* x, const int32_t* leaf_ptr, float2* s, int64_t nleaf, int Q,
                         int R, int64_t n, hipStream_t st) {
  if (nleaf == 0 || R <= 0) return;
  k_radiate_mfma<<<dim3((unsigned)nleaf, (unsigned)((R + 63) / 64)), LG_NT, 0, st>>>(V, x, leaf_ptr, s, Q, R, n);
}

void launch_recv_mfma(const float2* V, const float2* o, const int32_t* leaf_ptr, float2* y, int64_t nleaf, int Q,
                      int R, int64_t n, const double* w, hipStream_t st) {
  if (nleaf == 0 || R <= 0) return;
  k_recv_mfma<<<dim3((unsigned)nleaf, (unsigned)((R + 63) / 64)), LG_NT, 0, st>>>(
      V, o, leaf_ptr, y, Q, R, n, (float)w[0], (float)w[1], (float)w[2], (float)w[3]);
}

}  // namespace nesa
