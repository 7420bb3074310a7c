// Restricted additive Schwarz preconditioner assembled on the device
// (complex64 operators).  For leaf a with near leaves N(a), Z_N is the
// near-field matrix restricted to the RWGs of N(a) (blocks of two leaves of
// N(a) that are not near each other are zero); the preconditioner keeps the
// rows of Z_N^-1 that belong to leaf a, in the layout of leaf a's near block
// (S_a x W_a column-major, columns in near-list order).  Those rows are the
// solutions y_r of T y_r = e_r with T = Z_N^T, one per RWG r of leaf a.
//
// Per batch of leaves: k_schwarz_gather builds every T (W x W column-major,
// FP32 complex) from the near blocks, one workgroup per (leaf, pair of near
// leaves), through an LDS transpose; k_schwarz_lu factors each T = P^T L U by
// right-looking LU with partial pivoting (pivot = largest |re| + |im|, the
// first such row; rows swapped across the whole matrix), one workgroup per
// leaf, panels of SW_NB columns and rank-SW_NB trailing updates in 4 x 4
// register tiles, then solves the S_a unit right-hand sides, one thread each,
// in place in the preconditioner's arena (element (r, j) of leaf a's block is
// y_r[j]; a step of all threads touches consecutive addresses).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "precond_dev.h"

namespace nesa {

namespace {

constexpr int SW_NT = 256;
constexpr int SW_NB = 16;
constexpr int SW_MAXN = SCHWARZ_MAXN;
constexpr int SW_TILE = 32;

__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_div(float2 a, float2 b) {
  const float d = b.x * b.x + b.y * b.y;
  return make_float2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// T[j W + i] = Z_N[j][i]: row j of Z_N is RWG jr of leaf nb[jb], column i is
// RWG ic of leaf nb[ib]; when nb[ib] is near nb[jb] the entry is element
// (jr, colpos[jb][ib] + ic) of leaf nb[jb]'s near block (column-major, S_jb
// rows), else zero.  Workgroup (pair p = jb * 27 + ib, leaf) moves that
// S_jb x S_ib block in 32 x 32 tiles: read along jr, written along ic.
__global__ __launch_bounds__(SW_NT) void k_schwarz_gather(const float2* __restrict__ Z, const int64_t* __restrict__ zoff,
                                                          const int32_t* __restrict__ leaf_ptr, SchwarzBatch b) {
  __shared__ float2 tile[SW_TILE][SW_TILE + 1];
  const int a = b.first + blockIdx.y;
  const int na = b.na[a];
  const int jb = blockIdx.x / SW_MAXN, ib = blockIdx.x % SW_MAXN;
  if (jb >= na || ib >= na) return;
  const int W = b.W[a];
  const int32_t* off = b.off + (int64_t)a * (SW_MAXN + 1);
  const int cp = b.colpos[(int64_t)a * SW_MAXN * SW_MAXN + jb * SW_MAXN + ib];
  const int j0 = off[jb], Sj = off[jb + 1] - j0;
  const int i0 = off[ib], Si = off[ib + 1] - i0;
  float2* T = b.ws + b.ws_off[a];
  const int tx = threadIdx.x % SW_TILE, ty = threadIdx.x / SW_TILE;   // 32 x 8
  if (cp < 0) {
    for (int jr = ty; jr < Sj; jr += SW_NT / SW_TILE)
      for (int ic = tx; ic < Si; ic += SW_TILE) T[(int64_t)(j0 + jr) * W + i0 + ic] = make_float2(0.f, 0.f);
    return;
  }
  const int lb = b.nb[(int64_t)a * SW_MAXN + jb];
  const float2* Zb = Z + zoff[lb];
  const int Sb = leaf_ptr[lb + 1] - leaf_ptr[lb];   // = Sj
  for (int r0 = 0; r0 < Sj; r0 += SW_TILE)
    for (int c0 = 0; c0 < Si; c0 += SW_TILE) {
      // load: tx along jr (contiguous in Z), ty along ic
      for (int y = ty; y < SW_TILE; y += SW_NT / SW_TILE) {
        const int jr = r0 + tx, ic = c0 + y;
        tile[y][tx] = (jr < Sj && ic < Si) ? Zb[(int64_t)(cp + ic) * Sb + jr] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      // store: tx along ic (contiguous in T), ty along jr
      for (int y = ty; y < SW_TILE; y += SW_NT / SW_TILE) {
        const int jr = r0 + y, ic = c0 + tx;
        if (jr < Sj && ic < Si) T[(int64_t)(j0 + jr) * W + i0 + ic] = tile[tx][y];
      }
      __syncthreads();
    }
}

__global__ __launch_bounds__(SW_NT) void k_schwarz_lu(SchwarzBatch b, float2* __restrict__ out,
                                                      const int64_t* __restrict__ zoff,
                                                      const int32_t* __restrict__ leaf_ptr) {
  __shared__ float red_v[SW_NT];
  __shared__ int red_i[SW_NT];
  const int a = b.first + blockIdx.x;
  const int W = b.W[a], r0 = b.rowa[a];
  const int S = leaf_ptr[a + 1] - leaf_ptr[a];
  float2* T = b.ws + b.ws_off[a];
  int32_t* piv = b.piv + b.piv_off[a];
  const int t = threadIdx.x;
  for (int k0 = 0; k0 < W; k0 += SW_NB) {
    const int kb = min(SW_NB, W - k0);
    // ---- panel: columns k0 .. k0 + kb - 1, unblocked with partial pivoting
    for (int jj = 0; jj < kb; ++jj) {
      const int c = k0 + jj;
      float2* cw = T + (int64_t)c * W;
      float best = -1.f;
      int bi = W;
      for (int i = c + t; i < W; i += SW_NT) {
        const float m = fabsf(cw[i].x) + fabsf(cw[i].y);
        if (m > best) {
          best = m;
          bi = i;
        }
      }
      red_v[t] = best;
      red_i[t] = bi;
      __syncthreads();
      for (int s = SW_NT / 2; s > 0; s >>= 1) {
        if (t < s) {
          const float v2 = red_v[t + s];
          const int i2 = red_i[t + s];
          if (v2 > red_v[t] || (v2 == red_v[t] && i2 < red_i[t])) {
            red_v[t] = v2;
            red_i[t] = i2;
          }
        }
        __syncthreads();
      }
      const int p = red_i[0] < W ? red_i[0] : c;
      if (t == 0) {
        piv[c] = p;
        if (!(red_v[0] > 0.f)) b.status[0] = 1;
      }
      if (p != c)
        for (int jc = t; jc < W; jc += SW_NT) {
          float2* cc = T + (int64_t)jc * W;
          const float2 x = cc[c];
          cc[c] = cc[p];
          cc[p] = x;
        }
      __syncthreads();
      const float2 d = cw[c];
      for (int i = c + 1 + t; i < W; i += SW_NT) cw[i] = c_div(cw[i], d);
      __syncthreads();
      // rank-1 update of the panel's remaining columns
      const int nr = W - c - 1, ncw = k0 + kb - c - 1;
      for (int e = t; e < nr * ncw; e += SW_NT) {
        const int i = c + 1 + e % nr, jc = c + 1 + e / nr;
        float2* cj = T + (int64_t)jc * W;
        const float2 lf = c_mul(cw[i], cj[c]);
        cj[i].x -= lf.x;
        cj[i].y -= lf.y;
      }
      __syncthreads();
    }
    const int k1 = k0 + kb, n2 = W - k1;
    if (n2 <= 0) break;
    // ---- U12 = L11^-1 A12 (unit lower triangular), one column per thread
    for (int jc = k1 + t; jc < W; jc += SW_NT) {
      float2* cj = T + (int64_t)jc * W;
      for (int r = 1; r < kb; ++r) {
        float2 acc = cj[k0 + r];
        for (int q = 0; q < r; ++q) {
          const float2 lv = c_mul(T[(int64_t)(k0 + q) * W + k0 + r], cj[k0 + q]);
          acc.x -= lv.x;
          acc.y -= lv.y;
        }
        cj[k0 + r] = acc;
      }
    }
    __syncthreads();
    // ---- A22 -= L21 U12 in 4 x 4 tiles
    const int nt4 = (n2 + 3) / 4;
    for (int e = t; e < nt4 * nt4; e += SW_NT) {
      const int i0 = k1 + 4 * (e % nt4), j0 = k1 + 4 * (e / nt4);
      float2 acc[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = make_float2(0.f, 0.f);
      for (int q = 0; q < kb; ++q) {
        float2 l[4], u[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) l[x] = (i0 + x < W) ? T[(int64_t)(k0 + q) * W + i0 + x] : make_float2(0.f, 0.f);
#pragma unroll
        for (int y = 0; y < 4; ++y) u[y] = (j0 + y < W) ? T[(int64_t)(j0 + y) * W + k0 + q] : make_float2(0.f, 0.f);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            acc[x][y].x += l[x].x * u[y].x - l[x].y * u[y].y;
            acc[x][y].y += l[x].x * u[y].y + l[x].y * u[y].x;
          }
      }
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x)
          if (i0 + x < W && j0 + y < W) {
            float2& v = T[(int64_t)(j0 + y) * W + i0 + x];
            v.x -= acc[x][y].x;
            v.y -= acc[x][y].y;
          }
    }
    __syncthreads();
  }
  // ---- solves in place: Y[j S + r] = y_r[j], right-hand side e_{r0 + r}
  float2* Y = out + zoff[a];
  for (int e = t; e < S * W; e += SW_NT) {
    const int r = e % S, j = e / S;
    Y[e] = make_float2(j == r0 + r ? 1.f : 0.f, 0.f);
  }
  __syncthreads();
  for (int r = t; r < S; r += SW_NT) {
    for (int k = 0; k < W; ++k) {                 // the row swaps in factorisation order
      const int p = piv[k];
      if (p != k) {
        const float2 x = Y[(int64_t)k * S + r];
        Y[(int64_t)k * S + r] = Y[(int64_t)p * S + r];
        Y[(int64_t)p * S + r] = x;
      }
    }
    for (int j = 0; j < W; ++j) {                 // unit lower L, column by column
      const float2 yj = Y[(int64_t)j * S + r];
      if (yj.x == 0.f && yj.y == 0.f) continue;
      const float2* cl = T + (int64_t)j * W;
      for (int i = j + 1; i < W; ++i) {
        const float2 lv = c_mul(cl[i], yj);
        Y[(int64_t)i * S + r].x -= lv.x;
        Y[(int64_t)i * S + r].y -= lv.y;
      }
    }
    for (int j = W - 1; j >= 0; --j) {            // upper U, from the last column
      const float2* cu = T + (int64_t)j * W;
      const float2 yj = c_div(Y[(int64_t)j * S + r], cu[j]);
      Y[(int64_t)j * S + r] = yj;
      for (int i = 0; i < j; ++i) {
        const float2 uv = c_mul(cu[i], yj);
        Y[(int64_t)i * S + r].x -= uv.x;
        Y[(int64_t)i * S + r].y -= uv.y;
      }
    }
  }
}

}  // namespace

void launch_schwarz_batch(const float2* Z, const int64_t* zoff, const int32_t* leaf_ptr, const SchwarzBatch& b,
                          float2* out, hipStream_t st) {
  if (b.count <= 0) return;
  k_schwarz_gather<<<dim3(SW_MAXN * SW_MAXN, (unsigned)b.count), SW_NT, 0, st>>>(Z, zoff, leaf_ptr, b);
  k_schwarz_lu<<<(unsigned)b.count, SW_NT, 0, st>>>(b, out, zoff, leaf_ptr);
}

}  // namespace nesa
