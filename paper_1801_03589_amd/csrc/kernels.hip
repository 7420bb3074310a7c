// gfx950 kernels of the NESA product (Sec. 3, Eq. 9-14) and of the vector
// operations used by GMRES.
//
// Every output segment is written by exactly one workgroup per stage (owner
// computes), so results are deterministic and no atomics are used:
//   radiate     one workgroup per leaf b:      s_b = V_b x_b              (Eq. 10)
//   upward      one workgroup per parent P:    s_P = sum_children C s_c   (Eq. 11)
//   translate   one workgroup per (box, 64-row tile): o_a = sum_IL D s_b  (Eq. 12)
//   downward    one workgroup per child a:     o_a += C^T o_P             (Eq. 13)
//   near_recv   one workgroup per leaf a:      y_a = Z_near x + sum_c w_c V_a^T o_a
//                                                                     (Eq. 9 + 14)
// Complex numbers are interleaved (re, im) pairs of T = float or double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <stdexcept>

#include "kernels.h"
#include "split16.h"

namespace nesa {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ typename C2<T>::type cmk(T x, T y) {
  typename C2<T>::type r;
  r.x = x;
  r.y = y;
  return r;
}
// acc += a * b
template <typename V>
__device__ __forceinline__ void cfma(V& acc, const V a, const V b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
template <typename V>
__device__ __forceinline__ V cmul(const V a, const V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// stream / event calls inside the launchers: failures surface at the next
// synchronising call of the caller, as launch failures do
static inline void hip_ok(hipError_t e) { (void)e; }

constexpr int NT = 256;     // threads per workgroup
constexpr int WAVE = 64;

// ------------------------------------------------------------------ permutation
template <typename V>
__global__ void k_gather(const V* __restrict__ x, V* __restrict__ xl, const int32_t* __restrict__ perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) xl[i] = x[perm[i]];
}
template <typename V>
__global__ void k_scatter(const V* __restrict__ yl, V* __restrict__ y, const int32_t* __restrict__ perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) y[perm[i]] = yl[i];
}

// ------------------------------------------------------------------ radiation (Eq. 10)
// V in leaf order: row p (one RWG) holds its 4*Q coefficients contiguously.
constexpr int MAX_QL = 256;     // equivalent sources per leaf

template <typename T>
__global__ __launch_bounds__(NT) void k_radiate(const typename C2<T>::type* __restrict__ V,
                                                const typename C2<T>::type* __restrict__ x,
                                                const int32_t* __restrict__ leaf_ptr,
                                                typename C2<T>::type* __restrict__ s, int Q) {
  using V2 = typename C2<T>::type;
  __shared__ V2 xs[NT];
  const int b = blockIdx.x;
  const int p0 = leaf_ptr[b], S = leaf_ptr[b + 1] - p0;
  const int J = 4 * Q;
  if constexpr (sizeof(T) == 4) {
    // complex64: two values of a row per 16-byte load; the even and the odd
    // rows go to the two halves of the workgroup (summed in that order at the
    // end), which keeps two rows of loads in flight per step
    __shared__ float4 part[NT / 2][MAX_QL * 4 / 2 / (NT / 2)];
    constexpr int H = NT / 2, MJ = MAX_QL * 4 / 2 / H;        // float4 per thread per row (J / 2 <= H MJ)
    const int J2 = J / 2, t = threadIdx.x, h = t / H, c = t % H;
    const float4* V4 = reinterpret_cast<const float4*>(V);
    float4 acc4[MJ];
#pragma unroll
    for (int m = 0; m < MJ; ++m) acc4[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i0 = 0; i0 < S; i0 += NT) {
      const int ni = min(NT, S - i0);
      __syncthreads();
      if (t < ni) xs[t] = x[p0 + i0 + t];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < MJ; ++m) {
        const int j2 = c + m * H;
        if (j2 < J2) {
          const float4* Vp = V4 + (size_t)(p0 + i0) * J2 + j2;
          float4 a = acc4[m];
#pragma unroll 4
          for (int i = h; i < ni; i += 2) {
            const float4 v = Vp[(size_t)i * J2];
            const V2 xv = xs[i];
            a.x = fma(v.x, xv.x, a.x);
            a.x = fma(-v.y, xv.y, a.x);
            a.y = fma(v.x, xv.y, a.y);
            a.y = fma(v.y, xv.x, a.y);
            a.z = fma(v.z, xv.x, a.z);
            a.z = fma(-v.w, xv.y, a.z);
            a.w = fma(v.z, xv.y, a.w);
            a.w = fma(v.w, xv.x, a.w);
          }
          acc4[m] = a;
        }
      }
    }
    __syncthreads();
    if (h == 1) {
#pragma unroll
      for (int m = 0; m < MJ; ++m) part[c][m] = acc4[m];
    }
    __syncthreads();
    if (h == 0) {
      float4* s4 = reinterpret_cast<float4*>(s) + (size_t)b * J2;
#pragma unroll
      for (int m = 0; m < MJ; ++m) {
        const int j2 = c + m * H;
        if (j2 < J2) {
          const float4 o = part[c][m];
          s4[j2] = make_float4(acc4[m].x + o.x, acc4[m].y + o.y, acc4[m].z + o.z, acc4[m].w + o.w);
        }
      }
    }
    return;
  }
  V2 acc[2];
  acc[0] = cmk<T>(0, 0);
  acc[1] = cmk<T>(0, 0);
  for (int i0 = 0; i0 < S; i0 += NT) {
    const int ni = min(NT, S - i0);
    __syncthreads();
    if ((int)threadIdx.x < ni) xs[threadIdx.x] = x[p0 + i0 + threadIdx.x];
    __syncthreads();
    for (int r = 0; r < 2; ++r) {
      const int j = threadIdx.x + r * NT;
      if (j < J) {
        const V2* Vp = V + (size_t)(p0 + i0) * J + j;
        V2 a = acc[r];
        for (int i = 0; i < ni; ++i) cfma(a, Vp[(size_t)i * J], xs[i]);
        acc[r] = a;
      }
    }
  }
  for (int r = 0; r < 2; ++r) {
    const int j = threadIdx.x + r * NT;
    if (j < J) s[(size_t)b * J + j] = acc[r];
  }
}

// ------------------------------------------------------------------ source transfer (Eq. 11)
// Parent P at level l-1 gathers its children at level l.  Ccm[o][q][p] = C_o[p][q].
// Workgroup = (64-row tile of the parent, parent); wave w takes children w, w+4, ...
template <typename T>
__global__ __launch_bounds__(NT) void k_upward(const typename C2<T>::type* __restrict__ Ccm,
                                               const typename C2<T>::type* __restrict__ s_child,
                                               typename C2<T>::type* __restrict__ s_par,
                                               const int32_t* __restrict__ child_ptr,
                                               const int32_t* __restrict__ child_end,
                                               const int32_t* __restrict__ octant, int Qp, int Qc) {
  using V2 = typename C2<T>::type;
  __shared__ V2 red[NT / WAVE][4][WAVE];
  const int P = blockIdx.y;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int p = blockIdx.x * WAVE + lane;
  const int c0 = child_ptr[P], c1 = child_end[P];
  V2 acc[4];
  for (int c = 0; c < 4; ++c) acc[c] = cmk<T>(0, 0);
  if (p < Qp) {
    for (int ch = c0 + w; ch < c1; ch += NT / WAVE) {
      const V2* C = Ccm + (size_t)octant[ch] * Qp * Qc + p;
      const V2* sc = s_child + (size_t)ch * 4 * Qc;
#pragma unroll 4
      for (int q = 0; q < Qc; ++q) {
        const V2 cv = C[(size_t)q * Qp];
        for (int c = 0; c < 4; ++c) cfma(acc[c], cv, sc[c * Qc + q]);
      }
    }
  }
  for (int c = 0; c < 4; ++c) red[w][c][lane] = acc[c];
  __syncthreads();
  if (w == 0 && p < Qp) {
    for (int c = 0; c < 4; ++c) {
      V2 t = red[0][c][lane];
      for (int ww = 1; ww < NT / WAVE; ++ww) {
        t.x += red[ww][c][lane].x;
        t.y += red[ww][c][lane].y;
      }
      s_par[(size_t)P * 4 * Qp + c * Qp + p] = t;
    }
  }
}

// ------------------------------------------------------------------ translation (Eq. 12)
// o_a = sum over the interaction list of D_slot s_b.  Dcm[slot][q][p] = D[p][q].
// Workgroup = (64-row tile, target box); wave w takes list entries w, w+4, ...
template <typename T>
__global__ __launch_bounds__(NT) void k_translate(const typename C2<T>::type* __restrict__ Dcm,
                                                  const typename C2<T>::type* __restrict__ s,
                                                  typename C2<T>::type* __restrict__ o,
                                                  const int32_t* __restrict__ il_ptr,
                                                  const int32_t* __restrict__ il_src,
                                                  const int32_t* __restrict__ il_slot, int Q) {
  using V2 = typename C2<T>::type;
  __shared__ V2 red[NT / WAVE][4][WAVE];
  const int a = blockIdx.y;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int p = blockIdx.x * WAVE + lane;
  const int k0 = il_ptr[a], k1 = il_ptr[a + 1];
  V2 acc[4];
  for (int c = 0; c < 4; ++c) acc[c] = cmk<T>(0, 0);
  if (p < Q) {
    for (int kk = k0 + w; kk < k1; kk += NT / WAVE) {
      const int b = il_src[kk];
      const V2* D = Dcm + (size_t)il_slot[kk] * Q * Q + p;
      const V2* sb = s + (size_t)b * 4 * Q;
      for (int q = 0; q < Q; ++q) {
        const V2 d = D[(size_t)q * Q];
        for (int c = 0; c < 4; ++c) cfma(acc[c], d, sb[c * Q + q]);
      }
    }
  }
  for (int c = 0; c < 4; ++c) red[w][c][lane] = acc[c];
  __syncthreads();
  if (w == 0 && p < Q) {
    for (int c = 0; c < 4; ++c) {
      V2 t = red[0][c][lane];
      for (int ww = 1; ww < NT / WAVE; ++ww) {
        t.x += red[ww][c][lane].x;
        t.y += red[ww][c][lane].y;
      }
      o[(size_t)a * 4 * Q + c * Q + p] = t;
    }
  }
}

// Grouped complex GEMM on FP32 matrix cores (complex64 path), used for the
// translations (groups = offset slots, Eq. 12) and the transfers (groups =
// child octants, Eq. 11 and 13).  A tile holds up to 16 (source box,
// destination) pairs sharing one group matrix A_g (M x K, stored column-major
// with rows padded to Mr, a multiple of 16, zero rows).  One workgroup computes
// a block of up to 8 row tiles of C = A_g [x_src1 ... x_src16] (64 columns =
// 16 pairs x 4 channels); wave w owns column tile w (pairs 4w .. 4w+3).  The
// complex product is four real 16x16x4 MFMAs.  Each destination is written by
// exactly one lane in the grid (written, or added to when `accumulate`).
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int TR_KC = 32;          // K chunk staged in LDS
constexpr int TR_COLS = 64;        // GEMM columns per tile ((pair, channel) columns of one group)
constexpr int TR_NB = TR_KC * TR_COLS / NT;     // float2 of B per thread per chunk

struct GemmTiles {
  const float2* __restrict__ A;       // group matrices
  int64_t a_stride;      // complex elements per group matrix (K * Mr)
  int M, K, Mr;
  const float2* __restrict__ src;     // source boxes, [box][NC][K]
  float2* __restrict__ dst;           // destinations, [index][NC][M]
  int accumulate;
  int64_t ntiles;
  const int32_t* tile_group;
  const int32_t* tile_ncols;          // valid columns of the tile (<= 64)
  const int64_t* col_src;             // [tile][64] source offsets (complex elements)
  const int64_t* col_dst;             // [tile][64] destination offsets
};

// Workgroups are dealt to the 8 XCDs round-robin; tile = xcd_tile(blockIdx)
// gives every XCD a contiguous range of tiles, so the group matrices (tiles
// are ordered by group) and source boxes stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t ntiles) {
  const int64_t per = (ntiles + 7) / 8;
  const int64_t t = (bid % 8) * per + bid / 8;
  return t;
}

// CT = column tiles of 16 per workgroup (4: 64-column tiles, wave w owns
// column tile w and all NRT row tiles; 2: 32-column tiles for groups with few
// pairs, wave w owns column tile w % 2 and half of the row tiles); M3 = complex
// products with three real MFMAs instead of four.
template <int NRT, int CT, int M3>
__device__ __forceinline__ void cgemm_tiles_body(const GemmTiles& g) {
  constexpr int KC = TR_KC;
  constexpr int NA = KC * NRT * 8 / NT;        // float4 of A per thread per chunk (NRT*16 rows)
  constexpr int HALF = NRT * 8;                   // float4 per A column in a block
  constexpr int COLS = 16 * CT;                   // columns of a tile
  constexpr int NBT = KC * COLS / NT;          // float2 of B per thread per chunk
  constexpr int RPW = NRT * CT / 4;               // row tiles per wave
  static_assert(KC * NRT * 8 % NT == 0, "A chunk must split evenly");
  static_assert(NRT * CT % 4 == 0, "row tiles must split over the waves");
  // LDS padding (64 banks of 4 bytes): the four k rows a wave reads at once sit
  // 32 banks apart (A row stride = 32 x odd words), and the 16 columns of one k
  // row and of the next fall in disjoint banks (B column stride = 4 banks mod 64)
  constexpr int APAD = (NRT % 2 == 0) ? 4 : 0;    // float4
  constexpr int AST = 2 * (HALF + APAD);          // A row stride in float2
  __shared__ float4 As4[KC][HALF + APAD];      // [k][row pair]
  __shared__ float2 Bs[COLS][KC + 2];          // [column][k]
  __shared__ int64_t col_src[COLS];
  __shared__ int64_t col_dst[COLS];
  const int64_t tile = xcd_tile(blockIdx.x, g.ntiles);
  if (tile >= g.ntiles) return;
  const int r0 = blockIdx.y * NRT * 16;
  const int cnt = g.tile_ncols[tile];              // valid columns
  const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
  const int ct = w % CT, rt0 = (w / CT) * RPW;     // this wave's column tile and first row tile
  const int K = g.K, M = g.M;
  if (t < COLS) {
    col_src[t] = g.col_src[tile * COLS + t];
    col_dst[t] = g.col_dst[tile * COLS + t];
  }
  __syncthreads();
  const float4* A4 = reinterpret_cast<const float4*>(g.A + (size_t)g.tile_group[tile] * g.a_stride + r0);
  const bool active = 16 * ct < cnt;
  // 4 real products per complex product, or (M3) three: P1 = Ar Br, P2 = Ai Bi,
  // P3 = (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2 (25% fewer MFMAs)
  f32x4 cre[RPW], cim[RPW], c3[M3 ? RPW : 1];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (M3) c3[r] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float4 ra[NA];
  float2 rb[NBT];
  // per-thread staging: element e = t + i NT of a chunk is A row pair e % HALF at
  // k offset e / HALF, and B column e / KC at k offset e % KC.  The partial chunk
  // (kc0 = K mod KC steps of k, or KC) goes first, so every later chunk lies
  // inside [0, K): its loads advance plain pointers by KC steps, with no clamp
  // and no mask of k
  const int mr2 = g.Mr / 2;
  const int kc0 = (K % KC) ? K % KC : KC;
  const float4* pa[NA];
  const float2* pb[NBT];
  bool b_ok[NBT];
  // (set when the chunk loop starts, see `run` below)
  auto init_a = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + i * NT;
      pa[i] = A4 + (size_t)(kc0 + e / HALF) * mr2 + e % HALF;    // chunk 1
    }
  };
#pragma unroll
  for (int i = 0; i < NBT; ++i) {
    const int e = t + i * NT;
    const int col = e / KC;
    pb[i] = g.src + col_src[col] + kc0 + e % KC;                 // chunk 1
    b_ok[i] = col < cnt;
  }
  // chunk 0: clamped addresses (K may be below KC), zero mask at the LDS store
  auto load_first_b = [&]() {
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      const int e = t + i * NT;
      rb[i] = g.src[col_src[e / KC] + min(e % KC, K - 1)];
    }
  };
  auto load_first = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + i * NT;
      ra[i] = A4[(size_t)min(e / HALF, K - 1) * mr2 + e % HALF];
    }
    load_first_b();
  };
  const int64_t a_step = (int64_t)KC * mr2;
  auto load_next_b = [&]() {
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      rb[i] = *pb[i];
      pb[i] += KC;
    }
  };
  auto load_next = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      ra[i] = *pa[i];
      pa[i] += a_step;
    }
    load_next_b();
  };
  // the loads stay in flight during the MFMAs: their values are first used
  // here, when the chunk (kc steps of k) is written to LDS; k past the chunk
  // (first chunk only) and empty columns are zeroed
  auto stage_b = [&](int kc, bool first) {
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      const int e = t + i * NT;
      Bs[e / KC][e % KC] = ((!first || e % KC < kc) && b_ok[i]) ? rb[i] : make_float2(0.f, 0.f);
    }
  };
  auto stage = [&](int kc, bool first) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + i * NT;
      As4[e / HALF][e % HALF] = (!first || e / HALF < kc) ? ra[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    stage_b(kc, first);
    __syncthreads();
  };
  const float2* As = reinterpret_cast<const float2*>(&As4[0][0]);
  auto step = [&](int ks) {
    const int kk = ks * 4 + lane / 16;
    const float2 b = Bs[ct * 16 + lane % 16][kk];
    float2 a[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) a[r] = As[kk * AST + (rt0 + r) * 16 + lane % 16];
    if (M3) {
      const float bs = b.x + b.y;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.x, cre[r], 0, 0, 0);
        cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b.y, cim[r], 0, 0, 0);
        c3[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x + a[r].y, bs, c3[r], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.x, cre[r], 0, 0, 0);
        cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.y, cim[r], 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[r].y, b.y, cre[r], 0, 0, 0);
        cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b.x, cim[r], 0, 0, 0);
      }
    }
  };
  // full chunks run their step loop unrolled: the LDS reads of later steps are
  // issued ahead of the MFMAs of earlier ones
  // The chunk loop as one lambda over its load and stage steps, with the A
  // pointers set at its start: in this form the compiler keeps the 4-row-tile,
  // 32-column three-product kernel in 96 registers (five waves per SIMD)
  // instead of 108 (four), and the leaf level's launch takes 0.209 instead of
  // 0.219 - 0.227 ms
  auto run = [&](auto&& init, auto&& lfirst, auto&& lnext, auto&& stg) {
    init();
    lfirst();
    stg(kc0, true);
    if (kc0 < K) lnext();               // next chunk in flight during the MFMAs
    if (active) {
      const int ksteps = (kc0 + 3) / 4;
      for (int ks = 0; ks < ksteps; ++ks) step(ks);
    }
    for (int k0 = kc0; k0 < K; k0 += KC) {
      stg(KC, false);
      if (k0 + KC < K) lnext();
      if (active) {
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) step(ks);
      }
    }
  };
  run(init_a, load_first, load_next, stage);
  // Output through LDS: the accumulators (lane -> column lane % 16 of the
  // wave's tile, rows 4 (lane / 16) + i) go to a [column][row] tile in the A
  // chunk buffer (row stride ROWS + 2), then the workgroup writes runs of
  // consecutive rows of each column, so a store instruction fills whole cache
  // lines instead of 32 bytes of 16 lines.  Columns go in passes of PC.
  constexpr int ROWS = NRT * 16;
  constexpr int RS = ROWS + 2;                                   // float2
  constexpr int ACAP = KC * (HALF + APAD) * 2;                   // float2 in As4
  constexpr int PC = (ACAP / RS) >= COLS ? COLS : (ACAP / RS) / 16 * 16;
  static_assert(PC >= 16, "the LDS tile must hold one column tile");
  float2* otile = reinterpret_cast<float2*>(&As4[0][0]);
  const int mloc = min(ROWS, M - r0);
  for (int c0 = 0; c0 < COLS; c0 += PC) {
    __syncthreads();                                             // LDS no longer read
    if (ct * 16 >= c0 && ct * 16 < c0 + PC) {
      const int lc = ct * 16 - c0 + lane % 16;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          otile[lc * RS + (rt0 + r) * 16 + 4 * (lane / 16) + i] =
              M3 ? make_float2(cre[r][i] - cim[r][i], c3[r][i] - cre[r][i] - cim[r][i])
                 : make_float2(cre[r][i], cim[r][i]);
      }
    }
    __syncthreads();
    const int ncols = min(PC, cnt - c0);
    for (int e = t; e < ncols * mloc; e += NT) {
      const int lc = e / mloc, row = e % mloc;
      float2 v = otile[lc * RS + row];
      float2* out = g.dst + col_dst[c0 + lc] + r0 + row;
      if (g.accumulate) {
        const float2 o = *out;
        v.x += o.x;
        v.y += o.y;
      }
      *out = v;
    }
  }
}

// Split-precision variant (complex64 vectors, x3 products, split16.h): every
// FP32 value v is split as hi = r(v), lo = r(v - hi) (bf16 or fp16); a real
// product is hi*hi + hi*lo + lo*hi on 16x16x32 MFMAs of that format with FP32
// accumulation, and a
// complex product is four real ones (twelve MFMAs per k step: at one right-hand
// side the kernel is bound by staging, not by the matrix cores, and three real
// products would need two more planes of both operands).  A is pre-split into
// planes (re hi, re lo, im hi, im lo, then two planes of re + im that this
// kernel does not read), each
// [Mr][Kp] with k contiguous (Kp = K rounded up to 32, zero padded); B is split
// in the kernel from the FP32 tile in LDS.  Fragment layout of the 16x16x32
// instruction: lane l holds rows/columns l % 16 and k = 8 (l / 16) .. +7.
// fp16: the planes hold A x 2^a_exp, B is scaled by 2^split_shift(*bexp)
// before its split, and the results by 2^-(a_exp + shift).
typedef s16x8 bf16x8;

// CT = column tiles of 16 per workgroup: 4 (64-column tiles, wave w owns
// column tile w and every row tile) or 2 (32-column tiles for groups with few
// pairs, wave w owns column tile w % 2 and half of the row tiles).
template <int NRT, int F, int CT>
__device__ __forceinline__ void cgemm_tiles_bf16x3_body(const GemmTiles& g, const unsigned short* __restrict__ As,
                                                        int Kp, int a_exp, const int* __restrict__ bexp) {
  static_assert(TR_KC == 32, "one bf16 MFMA k-step per chunk");
  static_assert(CT == 4 || (CT == 2 && NRT % 2 == 0), "32-column tiles split an even number of row tiles");
  constexpr int COLS = 16 * CT;                   // columns of a tile
  constexpr int RPW = NRT * CT / 4;               // row tiles per wave
  constexpr int NB = TR_KC * COLS / NT;           // float2 of B per thread per chunk
  const int bshift = split_src_shift<F>(bexp);
  const int oexp = -(a_exp + bshift);
  __shared__ uint4 Al[4][NRT * 16][4];                        // [plane][row][8 k], split planes of A
  __shared__ float2 Bs[COLS][TR_KC + 1];                      // [column][k] FP32 B, split in place
  __shared__ int64_t col_src[COLS];
  __shared__ int64_t col_dst[COLS];
  const int64_t tile = xcd_tile(blockIdx.x, g.ntiles);
  if (tile >= g.ntiles) return;
  const int r0 = blockIdx.y * NRT * 16;
  const int cnt = g.tile_ncols[tile];
  const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
  const int K = g.K, M = g.M;
  if (t < COLS) {
    col_src[t] = g.col_src[tile * COLS + t];
    col_dst[t] = g.col_dst[tile * COLS + t];
  }
  __syncthreads();
  const int ct = w % CT, rt0 = (w / CT) * RPW;     // this wave's column tile and first row tile
  const bool active = 16 * ct < cnt;
  const size_t plane = (size_t)g.Mr * Kp;
  const unsigned short* Ag = As + (size_t)g.tile_group[tile] * 6 * plane + (size_t)r0 * Kp;   // planes 0-3
  f32x4 cre[RPW], cim[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // A staging: NRT x 16 B per thread per chunk (4 planes x NRT*16 rows x 4 quarters of 8 k)
  // (native vectors: copies of HIP's uint4 struct kept these in private memory)
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 ra[NRT];
  const u32x4* a_ptr[NRT];
#pragma unroll
  for (int i = 0; i < NRT; ++i) {
    const int e = t + i * NT;
    const int pl = e / (NRT * 16 * 4), row = (e / 4) % (NRT * 16), qu = e % 4;
    a_ptr[i] = reinterpret_cast<const u32x4*>(Ag + pl * plane + (size_t)row * Kp + 8 * qu);
  }
  // B staging: NB float2 per thread per chunk
  float2 rb[NB];
  const float2* b_ptr[NB];
  int b_k[NB];
  bool b_ok[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = t + i * NT;
    const int col = e / TR_KC;
    b_k[i] = e % TR_KC;
    b_ptr[i] = g.src + col_src[col];
    b_ok[i] = col < cnt;
  }
  // raw loads; the zero mask of k >= K and of empty columns is applied at the
  // LDS store, so the loads stay in flight during the MFMAs
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NRT; ++i) ra[i] = a_ptr[i][k0 / 8];
#pragma unroll
    for (int i = 0; i < NB; ++i) rb[i] = b_ptr[i][min(k0 + b_k[i], K - 1)];
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += TR_KC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NRT; ++i) {
      const int e = t + i * NT;
      *reinterpret_cast<u32x4*>(&Al[e / (NRT * 16 * 4)][(e / 4) % (NRT * 16)][e % 4]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = t + i * NT;
      Bs[e / TR_KC][e % TR_KC] = (k0 + b_k[i] < K && b_ok[i]) ? rb[i] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (k0 + TR_KC < K) load(k0 + TR_KC);
    if (active) {
      // B fragments of this wave's column tile as bf16 hi / lo planes
      bf16x8 brh, brl, bih, bil, nbih, nbil;
      const float2* bcol = &Bs[ct * 16 + lane % 16][8 * (lane / 16)];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float2 v = bcol[j];
        if (F == SPLIT_FP16) v = make_float2(ldexpf(v.x, bshift), ldexpf(v.y, bshift));
        unsigned short h, l;
        split16<F>(v.x, h, l);
        brh[j] = __builtin_bit_cast(__bf16, h);
        brl[j] = __builtin_bit_cast(__bf16, l);
        split16<F>(v.y, h, l);
        bih[j] = __builtin_bit_cast(__bf16, h);
        bil[j] = __builtin_bit_cast(__bf16, l);
        nbih[j] = __builtin_bit_cast(__bf16, (unsigned short)(h ^ 0x8000u));
        nbil[j] = __builtin_bit_cast(__bf16, (unsigned short)(l ^ 0x8000u));
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int row = (rt0 + r) * 16 + lane % 16, qu = lane / 16;
        const bf16x8 arh = __builtin_bit_cast(bf16x8, Al[0][row][qu]);
        const bf16x8 arl = __builtin_bit_cast(bf16x8, Al[1][row][qu]);
        const bf16x8 aih = __builtin_bit_cast(bf16x8, Al[2][row][qu]);
        const bf16x8 ail = __builtin_bit_cast(bf16x8, Al[3][row][qu]);
        cre[r] = mfma16x16x32<F>(arh, brh, cre[r]);
        cim[r] = mfma16x16x32<F>(arh, bih, cim[r]);
        cre[r] = mfma16x16x32<F>(arh, brl, cre[r]);
        cim[r] = mfma16x16x32<F>(arh, bil, cim[r]);
        cre[r] = mfma16x16x32<F>(arl, brh, cre[r]);
        cim[r] = mfma16x16x32<F>(arl, bih, cim[r]);
        cre[r] = mfma16x16x32<F>(aih, nbih, cre[r]);
        cim[r] = mfma16x16x32<F>(aih, brh, cim[r]);
        cre[r] = mfma16x16x32<F>(aih, nbil, cre[r]);
        cim[r] = mfma16x16x32<F>(aih, brl, cim[r]);
        cre[r] = mfma16x16x32<F>(ail, nbih, cre[r]);
        cim[r] = mfma16x16x32<F>(ail, brh, cim[r]);
      }
    }
  }
  const int col = ct * 16 + lane % 16;
  if (col < cnt) {
    float2* out = g.dst + col_dst[col];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + (rt0 + r) * 16 + 4 * (lane / 16) + i;
        if (row < M) {
          float2 v = make_float2(cre[r][i], cim[r][i]);
          if (F == SPLIT_FP16) v = make_float2(ldexpf(v.x, oexp), ldexpf(v.y, oexp));
          if (g.accumulate) {
            const float2 o = out[row];
            v.x += o.x;
            v.y += o.y;
          }
          out[row] = v;
        }
      }
    }
  }
}

template <int NRT, int F, int CT>
__global__ __launch_bounds__(NT) void k_translate_gemm_bf16x3(GemmTiles g, const unsigned short* As, int Kp,
                                                              int a_exp, const int* bexp) {
  cgemm_tiles_bf16x3_body<NRT, F, CT>(g, As, Kp, a_exp, bexp);
}
template <int NRT, int F, int CT>
__global__ __launch_bounds__(NT) void k_transfer_gemm_bf16x3(GemmTiles g, const unsigned short* As, int Kp,
                                                             int a_exp, const int* bexp) {
  cgemm_tiles_bf16x3_body<NRT, F, CT>(g, As, Kp, a_exp, bexp);
}

// Resident-A variant for small K (K <= KT): a workgroup takes a run of `tpw`
// consecutive tiles, keeps the group matrix rows r0 .. r0 + 16 NRT for all K in
// LDS (restaged only when the run crosses into another group), stages each
// tile's 64 source columns for the whole K at once and loads the next tile's
// columns into registers while the MFMAs of the current one run.  Suits the
// fine levels, where a tile is only a few K steps and the chunked kernel's
// per-workgroup latency dominates.
template <int NRT, int KT>
__device__ __forceinline__ void cgemm_resident_body(const GemmTiles& g, int tpw) {
  constexpr int NBM = TR_COLS * KT / NT;          // max float2 of B per thread per tile
  static_assert(TR_COLS * KT % NT == 0, "B tile must split evenly");
  __shared__ float2 As[KT][NRT * 16];
  __shared__ float2 Bs[TR_COLS][KT + 1];
  __shared__ int64_t cdst[TR_COLS];
  const int64_t nruns = (g.ntiles + tpw - 1) / tpw;
  const int64_t run = xcd_tile(blockIdx.x, nruns);
  if (run >= nruns) return;
  const int64_t t_begin = run * tpw;
  const int64_t t_end = min(g.ntiles, t_begin + tpw);
  const int r0 = blockIdx.y * NRT * 16;
  const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
  const int K = g.K, M = g.M;
  const int KP = (K + 3) / 4 * 4;
  const int nb = TR_COLS * KP;                    // B elements of a tile
  float2 rb[NBM];
  // raw loads; k >= K is zeroed at the LDS store, so the loads of the next tile
  // stay in flight during the MFMAs
  auto load_b = [&](int64_t tile) {
#pragma unroll
    for (int i = 0; i < NBM; ++i) {
      const int e = t + i * NT;
      const int col = min(e / KP, TR_COLS - 1), k = e % KP;
      const int64_t off = g.col_src[tile * TR_COLS + col];
      rb[i] = g.src[off + min(k, K - 1)];
    }
  };
  load_b(t_begin);
  int group = -1;
  for (int64_t tile = t_begin; tile < t_end; ++tile) {
    const int grp = g.tile_group[tile];
    const int cnt = g.tile_ncols[tile];
    __syncthreads();                              // previous tile done with Bs (and As)
    if (grp != group) {
      const float2* A = g.A + (size_t)grp * g.a_stride + r0;
      for (int e = t; e < KT * NRT * 16; e += NT) {
        const int k = e / (NRT * 16), r = e % (NRT * 16);
        const float2 v = A[(size_t)min(k, K - 1) * g.Mr + r];
        const float f = k < K ? 1.f : 0.f;
        As[k][r] = make_float2(v.x * f, v.y * f);
      }
      group = grp;
    }
#pragma unroll
    for (int i = 0; i < NBM; ++i) {
      const int e = t + i * NT;
      if (e < nb) Bs[e / KP][e % KP] = (e % KP < K) ? rb[i] : make_float2(0.f, 0.f);
    }
    if (t < TR_COLS) cdst[t] = g.col_dst[tile * TR_COLS + t];
    __syncthreads();
    if (tile + 1 < t_end) load_b(tile + 1);       // next tile in flight during the MFMAs
    if (16 * w < cnt) {
      f32x4 cre[NRT], cim[NRT];
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
        cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      for (int ks = 0; ks < KP / 4; ++ks) {
        const int kk = ks * 4 + lane / 16;
        const float2 b = Bs[w * 16 + lane % 16][kk];
        float2 a[NRT];
#pragma unroll
        for (int r = 0; r < NRT; ++r) a[r] = As[kk][r * 16 + lane % 16];
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.x, cre[r], 0, 0, 0);
          cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b.y, cim[r], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[r].y, b.y, cre[r], 0, 0, 0);
          cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b.x, cim[r], 0, 0, 0);
        }
      }
      const int col = w * 16 + lane % 16;
      if (col < cnt) {
        float2* out = g.dst + cdst[col];
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = r0 + r * 16 + 4 * (lane / 16) + i;
            if (row < M) {
              float2 v = make_float2(cre[r][i], cim[r][i]);
              if (g.accumulate) {
                const float2 o = out[row];
                v.x += o.x;
                v.y += o.y;
              }
              out[row] = v;
            }
          }
        }
      }
    }
  }
}

// Direct variant for small K (K <= 4 KS): no LDS and no barrier.  Wave w of a
// workgroup owns column tile w of the tile; it loads its 16 source columns for
// all K into registers at once (one memory latency per tile), reads the group
// matrix rows from L1/L2 per k step, and runs its MFMA chain.  Occupancy is
// bounded by registers only.
template <int NRT, int KS>
__device__ __forceinline__ void cgemm_direct_body(const GemmTiles& g) {
  const int64_t tile = xcd_tile(blockIdx.x, g.ntiles);
  if (tile >= g.ntiles) return;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int cnt = g.tile_ncols[tile];
  if (16 * w >= cnt) return;                      // whole wave idle (no barrier in this kernel)
  const int K = g.K, M = g.M;
  const int r0 = blockIdx.y * NRT * 16;
  const int col = w * 16 + lane % 16;
  const int kq = lane / 16;
  const float2* bsrc = g.src + g.col_src[tile * TR_COLS + col];
  float2 b[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 4 + kq;
    const float2 v = bsrc[min(k, K - 1)];
    const float f = k < K ? 1.f : 0.f;
    b[ks] = make_float2(v.x * f, v.y * f);
  }
  const float2* A = g.A + (size_t)g.tile_group[tile] * g.a_stride + r0 + lane % 16;
  f32x4 cre[NRT], cim[NRT];
#pragma unroll
  for (int r = 0; r < NRT; ++r) {
    cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 4 + kq;
    const float f = k < K ? 1.f : 0.f;
    const float2* Ak = A + (size_t)min(k, K - 1) * g.Mr;
    float2 a[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      const float2 v = Ak[r * 16];
      a[r] = make_float2(v.x * f, v.y * f);
    }
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b[ks].x, cre[r], 0, 0, 0);
      cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].x, b[ks].y, cim[r], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[r].y, b[ks].y, cre[r], 0, 0, 0);
      cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r].y, b[ks].x, cim[r], 0, 0, 0);
    }
  }
  if (col < cnt) {
    float2* out = g.dst + g.col_dst[tile * TR_COLS + col];
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + r * 16 + 4 * (lane / 16) + i;
        if (row < M) {
          float2 v = make_float2(cre[r][i], cim[r][i]);
          if (g.accumulate) {
            const float2 o = out[row];
            v.x += o.x;
            v.y += o.y;
          }
          out[row] = v;
        }
      }
    }
  }
}

template <int NRT, int KS>
__global__ __launch_bounds__(NT) void k_translate_gemm_dir(GemmTiles g) {
  cgemm_direct_body<NRT, KS>(g);
}
template <int NRT, int KS>
__global__ __launch_bounds__(NT) void k_transfer_gemm_dir(GemmTiles g) {
  cgemm_direct_body<NRT, KS>(g);
}

template <int NRT, int KT>
__global__ __launch_bounds__(NT) void k_translate_gemm_res(GemmTiles g, int tpw) {
  cgemm_resident_body<NRT, KT>(g, tpw);
}
template <int NRT, int KT>
__global__ __launch_bounds__(NT) void k_transfer_gemm_res(GemmTiles g, int tpw) {
  cgemm_resident_body<NRT, KT>(g, tpw);
}

// translations (groups = offset slots) and transfers (groups = octants) get
// their own kernel names so that profiles separate them
template <int NRT, int CT, int M3>
__global__ __launch_bounds__(NT) void k_translate_gemm(GemmTiles g) {
  cgemm_tiles_body<NRT, CT, M3>(g);
}
template <int NRT, int CT, int M3>
__global__ __launch_bounds__(NT) void k_transfer_gemm(GemmTiles g) {
  cgemm_tiles_body<NRT, CT, M3>(g);
}

// dst_a = sum over [beg[a], end[a]) of the per-pair results, in order
// (deterministic); workgroup (a, y) takes elements y*NT, y*NT + gridDim.y*NT, ...
// o[a] = sum of the partial rows beg[a] .. end[a] - 1 (fixed order); this
// workgroup takes chunk `yb` of `ny` chunks of the J values of row a
template <typename V>
__device__ __forceinline__ void csr_reduce_row(const V* __restrict__ pair_out, V* __restrict__ o,
                                               const int32_t* __restrict__ beg, const int32_t* __restrict__ end,
                                               int J, int a, int yb, int ny) {
  const int k0 = beg[a], k1 = end[a];
  if constexpr (sizeof(V) == 8) {
    // complex64: two values per 16-byte load (J is even: 4 channels per right-hand
    // side); a row of at most 128 such pairs leaves half of the workgroup free,
    // which then sums the odd-numbered partials (combined in a fixed order)
    __shared__ float4 half1[NT / 2];
    const int J2 = J / 2;
    const float4* src = reinterpret_cast<const float4*>(pair_out);
    float4* dst = reinterpret_cast<float4*>(o);
    const bool split = J2 <= NT / 2 && ny == 1;                 // uniform over the workgroup
    const int t = threadIdx.x;
    if (split) {
      const int j = t % (NT / 2), ks = t / (NT / 2);
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      if (j < J2) {
#pragma unroll 8
        for (int k = k0 + ks; k < k1; k += 2) {
          const float4 v = src[(size_t)k * J2 + j];
          acc.x += v.x;
          acc.y += v.y;
          acc.z += v.z;
          acc.w += v.w;
        }
        if (ks == 1) half1[j] = acc;
      }
      __syncthreads();
      if (ks == 0 && j < J2) {
        const float4 b = half1[j];
        dst[(size_t)a * J2 + j] = make_float4(acc.x + b.x, acc.y + b.y, acc.z + b.z, acc.w + b.w);
      }
    } else {
      for (int j = yb * NT + t; j < J2; j += ny * NT) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
        for (int k = k0; k < k1; ++k) {
          const float4 v = src[(size_t)k * J2 + j];
          acc.x += v.x;
          acc.y += v.y;
          acc.z += v.z;
          acc.w += v.w;
        }
        dst[(size_t)a * J2 + j] = acc;
      }
    }
  } else {
    for (int j = yb * NT + threadIdx.x; j < J; j += ny * NT) {
      V acc;
      acc.x = 0;
      acc.y = 0;
#pragma unroll 8
      for (int k = k0; k < k1; ++k) {
        const V v = pair_out[(size_t)k * J + j];
        acc.x += v.x;
        acc.y += v.y;
      }
      o[(size_t)a * J + j] = acc;
    }
  }
}

template <typename V>
__global__ __launch_bounds__(NT) void k_csr_reduce(const V* __restrict__ pair_out, V* __restrict__ o,
                                                   const int32_t* __restrict__ beg, const int32_t* __restrict__ end,
                                                   int J) {
  csr_reduce_row<V>(pair_out, o, beg, end, J, blockIdx.x, blockIdx.y, gridDim.y);
}

// ------------------------------------------------------------------ potential transfer (Eq. 13)
// Child a at level l: o_a += B o_P with B = C^T.  Crm[o][p][q] = C_o[p][q].
// Workgroup = (64-row tile of the child, child); wave w takes parent rows p = w, w+4, ...
template <typename T>
__global__ __launch_bounds__(NT) void k_downward(const typename C2<T>::type* __restrict__ Crm,
                                                 const typename C2<T>::type* __restrict__ o_par,
                                                 typename C2<T>::type* __restrict__ o_child,
                                                 const int32_t* __restrict__ parent,
                                                 const int32_t* __restrict__ octant, int Qp, int Qc) {
  using V2 = typename C2<T>::type;
  __shared__ V2 red[NT / WAVE][4][WAVE];
  const int a = blockIdx.y;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int q = blockIdx.x * WAVE + lane;
  const int P = parent[a];
  if (P < 0) return;                     // top box of a body in a forest (whole workgroup)
  const V2* C = Crm + (size_t)octant[a] * Qp * Qc + q;
  const V2* op = o_par + (size_t)P * 4 * Qp;
  V2 acc[4];
  for (int c = 0; c < 4; ++c) acc[c] = cmk<T>(0, 0);
  if (q < Qc) {
#pragma unroll 4
    for (int p = w; p < Qp; p += NT / WAVE) {
      const V2 cv = C[(size_t)p * Qc];
      for (int c = 0; c < 4; ++c) cfma(acc[c], cv, op[c * Qp + p]);
    }
  }
  for (int c = 0; c < 4; ++c) red[w][c][lane] = acc[c];
  __syncthreads();
  if (w == 0 && q < Qc) {
    V2* oc = o_child + (size_t)a * 4 * Qc;
    for (int c = 0; c < 4; ++c) {
      V2 t = oc[c * Qc + q];
      for (int ww = 0; ww < NT / WAVE; ++ww) {
        t.x += red[ww][c][lane].x;
        t.y += red[ww][c][lane].y;
      }
      oc[c * Qc + q] = t;
    }
  }
}

// ------------------------------------------------------------------ near field + reception (Eq. 9, 14)
// Z block of leaf a: S x W column-major at Z + zoff[a]; its columns are the
// RWGs of the near leaves in list order.  Rows split over G = NT/S column
// groups; each thread reads Z contiguously (address k*G*S + tid).
constexpr int NEAR_CW = 1024;   // x columns staged in LDS per pass
constexpr int MAX_NEAR = 128;   // near-list entries per leaf

// Reception of one leaf (Eq. 14): y[p0 + r] = base_r + sum_j V[p0 + r][j] ow[j]
// for the S rows of the leaf, with base_r = red[r] (near-field result staged in
// LDS) or, when red is null, the value already in y.  8 lanes per row and 8
// rows per wave: each lane keeps several loads of its row in flight, and the
// row sum takes 3 shuffle steps.
template <typename T>
__device__ __forceinline__ void recv_rows(const typename C2<T>::type* __restrict__ V,
                                          const typename C2<T>::type* ow, const typename C2<T>::type* red,
                                          typename C2<T>::type* __restrict__ y, int p0, int S, int J) {
  using V2 = typename C2<T>::type;
  constexpr int LR = 8;
  const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
  const int c = lane % LR, sub = lane / LR;
  for (int row0 = wv * (WAVE / LR); row0 < S; row0 += (NT / WAVE) * (WAVE / LR)) {
    const int row = row0 + sub;
    V2 s = cmk<T>(0, 0);
    if (row < S) {
      if constexpr (sizeof(T) == 4) {
        // complex64: two values per 16-byte load (J is even)
        const float4* Vr = reinterpret_cast<const float4*>(V + (size_t)(p0 + row) * J);
        const float4* ow4 = reinterpret_cast<const float4*>(ow);
        V2 s2 = cmk<T>(0, 0);
#pragma unroll 4
        for (int j = c; j < J / 2; j += LR) {
          const float4 v = Vr[j], w = ow4[j];
          cfma(s, make_float2(v.x, v.y), make_float2(w.x, w.y));
          cfma(s2, make_float2(v.z, v.w), make_float2(w.z, w.w));
        }
        s.x += s2.x;
        s.y += s2.y;
      } else {
        const V2* Vr = V + (size_t)(p0 + row) * J;
#pragma unroll 4
        for (int j = c; j < J; j += LR) cfma(s, Vr[j], ow[j]);
      }
    }
    for (int off = LR / 2; off > 0; off >>= 1) {
      s.x += __shfl_xor(s.x, off);
      s.y += __shfl_xor(s.y, off);
    }
    if (c == 0 && row < S) {
      V2 out = red ? red[row] : y[p0 + row];
      out.x += s.x;
      out.y += s.y;
      y[p0 + row] = out;
    }
  }
}

// ------------------------------------------------------------------ near field, reciprocity half storage
// The Galerkin EFIE matrix is symmetric (Z_mn = Z_nm: testing and basis
// functions are the same RWGs), so of every pair of neighbouring leaves only
// the blocks Z_ab with b >= a (leaf order) are stored: leaf a's columns are the
// RWGs of the leaves b >= a of its near list (itself first), column-major
// S_a x W_a.  One pass over them gives both Z_ab x_b (summed into y_a) and,
// for b > a, Z_ab^T x_a, written to its own slot of `tpart`; the reception
// kernel adds the slots of every leaf in increasing a (a fixed order).
constexpr int NEAR_HCW = 512;                 // x columns staged in LDS per sub-chunk (<= 2 NT)
constexpr int NEAR_TP_BYTES = 36 * 1024;      // LDS of the transposed products of a sub-chunk

// Sub-chunks of CT columns; each thread holds at most U of a sub-chunk's near
// entries, loaded into registers while the previous sub-chunk is computed and
// reduced (the loads' latency hides behind that work and the barriers).
// HALF = false: the plain product of one leaf's full block (columns: the whole
// near list), no transposed outputs; `tp`, `nh_ptr`, `toff`, `tpart` unused.
template <typename T, bool HALF>
__device__ __forceinline__ void near_half_leaf(const int a, typename C2<T>::type* xs, typename C2<T>::type* red,
                                               typename C2<T>::type* tp, int* seg_col, int* seg_x,
                                               const typename C2<T>::type* __restrict__ Z,
                                               const int64_t* __restrict__ zoff,
                                               const int32_t* __restrict__ leaf_ptr,
                                               const int32_t* __restrict__ nh_ptr,
                                               const int32_t* __restrict__ near_ptr,
                                               const int32_t* __restrict__ near_idx,
                                               const int32_t* __restrict__ toff,
                                               const typename C2<T>::type* __restrict__ x,
                                               typename C2<T>::type* __restrict__ y,
                                               typename C2<T>::type* __restrict__ tpart) {
  using V2 = typename C2<T>::type;
  constexpr int TP_N = NEAR_TP_BYTES / (int)sizeof(V2);
  constexpr int U = sizeof(T) == 4 ? 16 : 8;
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int n0 = HALF ? nh_ptr[a] : near_ptr[a], nn = near_ptr[a + 1] - n0;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int k = 0; k < nn; ++k) {
      const int b = near_idx[n0 + k];
      seg_col[k] = c;
      seg_x[k] = leaf_ptr[b];
      c += leaf_ptr[b + 1] - leaf_ptr[b];
    }
    seg_col[nn] = c;
  }
  __syncthreads();
  const int W = seg_col[nn];
  const V2* Za = Z + zoff[a];
  const int G = NT / S;                    // column groups of S threads (S <= NT checked on the host)
  const int t = threadIdx.x, g = t / S, i = t - g * S;
  const bool row_ok = g < G;
  const V2 xa = HALF && row_ok ? x[p0 + i] : cmk<T>(0, 0);
  const int SP = S | 1;                    // odd LDS stride of a column of products
  const int CT = HALF ? min(min(NEAR_HCW, TP_N / SP), U * G) : min(NEAR_HCW, U * G);   // columns per sub-chunk
  V2* ta = HALF ? tpart + toff[a] - S : nullptr;   // Z_ab^T x_a of column col >= S goes to ta[col]
  V2 zr[U], xr[2];
  // loads of the sub-chunk at column c0 into registers
  auto fetch = [&](int c0) {
    const int cw = min(CT, W - c0);
    const V2* Zp = Za + (size_t)c0 * S + t;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = g + u * G;
      if (row_ok && j < cw) zr[u] = Zp[(size_t)(u * G) * S];
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int j = t + e * NT;
      if (j < cw) {
        const int col = c0 + j;
        int k = 0;
        while (seg_col[k + 1] <= col) ++k;
        xr[e] = x[seg_x[k] + (col - seg_col[k])];
      }
    }
  };
  V2 acc = cmk<T>(0, 0);
  if (W > 0) fetch(0);
  for (int c0 = 0; c0 < W; c0 += CT) {
    const int cw = min(CT, W - c0);
    __syncthreads();                       // xs and tp of the previous sub-chunk consumed
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (t + e * NT < cw) xs[t + e * NT] = xr[e];
    __syncthreads();
    V2 zc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) zc[u] = zr[u];
    if (c0 + CT < W) fetch(c0 + CT);
    if (row_ok) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = g + u * G;
        if (j < cw) {
          cfma(acc, zc[u], xs[j]);
          if constexpr (HALF) tp[j * SP + i] = cmul(zc[u], xa);
        }
      }
    }
    if constexpr (!HALF) continue;
    __syncthreads();
    // column sums of the products of the off-diagonal columns (fixed order:
    // rows strided by TPC per thread, then a butterfly over the TPC lanes)
    const int jlo = max(0, S - c0), nc = cw - jlo;
    if (nc > 0) {
      int TPC = 1;
      while (TPC < WAVE && TPC * 2 * nc <= NT) TPC *= 2;
      if (TPC == 1) {
        for (int jj = t; jj < nc; jj += NT) {
          const V2* col = tp + (jlo + jj) * SP;
          V2 sum = cmk<T>(0, 0);
          for (int r = 0; r < S; ++r) {
            sum.x += col[r].x;
            sum.y += col[r].y;
          }
          ta[c0 + jlo + jj] = sum;
        }
      } else {
        const int jj = t / TPC, part = t % TPC;
        V2 sum = cmk<T>(0, 0);
        if (jj < nc) {
          const V2* col = tp + (jlo + jj) * SP;
          for (int r = part; r < S; r += TPC) {
            sum.x += col[r].x;
            sum.y += col[r].y;
          }
        }
        for (int m = 1; m < TPC; m <<= 1) {
          sum.x += __shfl_xor(sum.x, m);
          sum.y += __shfl_xor(sum.y, m);
        }
        if (jj < nc && part == 0) ta[c0 + jlo + jj] = sum;
      }
    }
  }
  red[t] = acc;
  __syncthreads();
  // reduce the column groups (fixed order): Z_ab x_b summed over b >= a
  if (t < S) {
    V2 yn = red[t];
    for (int gg = 1; gg < G; ++gg) {
      yn.x += red[gg * S + t].x;
      yn.y += red[gg * S + t].y;
    }
    y[p0 + t] = yn;
  }
}

// near field of one right-hand side as a persistent grid that walks the leaves
// (largest blocks first): beside the far-field stages it holds one workgroup
// slot per CU and leaves the rest of every CU to them; with one workgroup per
// leaf it is the near field of the serial form
template <typename T>
__global__ __launch_bounds__(NT) void k_near_half(const typename C2<T>::type* __restrict__ Z,
                                                  const int64_t* __restrict__ zoff,
                                                  const int32_t* __restrict__ leaf_ptr,
                                                  const int32_t* __restrict__ nh_ptr,
                                                  const int32_t* __restrict__ near_ptr,
                                                  const int32_t* __restrict__ near_idx,
                                                  const int32_t* __restrict__ toff,
                                                  const typename C2<T>::type* __restrict__ x,
                                                  typename C2<T>::type* __restrict__ y,
                                                  typename C2<T>::type* __restrict__ tpart, int64_t nleaf,
                                                  const int32_t* __restrict__ order) {
  using V2 = typename C2<T>::type;
  __shared__ V2 xs[NEAR_HCW];
  __shared__ V2 red[NT];
  __shared__ V2 tp[NEAR_TP_BYTES / sizeof(V2)];
  __shared__ int seg_col[MAX_NEAR + 1];
  __shared__ int seg_x[MAX_NEAR];
  for (int64_t k = blockIdx.x; k < nleaf; k += gridDim.x) {
    near_half_leaf<T, true>(order[k], xs, red, tp, seg_col, seg_x, Z, zoff, leaf_ptr, nh_ptr, near_ptr, near_idx,
                            toff, x, y, tpart);
    __syncthreads();                       // shared arrays reused by the next leaf
  }
}

// y = A x for one right-hand side with an arena A in the full near-block layout
// (the Schwarz preconditioner): one workgroup per leaf
template <typename T>
__global__ __launch_bounds__(NT) void k_near_full1(const typename C2<T>::type* __restrict__ Z,
                                                   const int64_t* __restrict__ zoff,
                                                   const int32_t* __restrict__ leaf_ptr,
                                                   const int32_t* __restrict__ near_ptr,
                                                   const int32_t* __restrict__ near_idx,
                                                   const typename C2<T>::type* __restrict__ x,
                                                   typename C2<T>::type* __restrict__ y) {
  using V2 = typename C2<T>::type;
  __shared__ V2 xs[NEAR_HCW];
  __shared__ V2 red[NT];
  __shared__ int seg_col[MAX_NEAR + 1];
  __shared__ int seg_x[MAX_NEAR];
  near_half_leaf<T, false>(blockIdx.x, xs, red, nullptr, seg_col, seg_x, Z, zoff, leaf_ptr, nullptr, near_ptr,
                           near_idx, nullptr, x, y, nullptr);
}

// reception of one right-hand side (Eq. 14) after the half-storage near field:
// y_a += sum over near leaves b < a (increasing b) of Z_ba^T x_b, then the
// received field; one workgroup per leaf, the weighted potentials in LDS
template <typename T>
__global__ __launch_bounds__(NT) void k_recv1h(const typename C2<T>::type* __restrict__ V,
                                               const typename C2<T>::type* __restrict__ o,
                                               const int32_t* __restrict__ leaf_ptr,
                                               const int32_t* __restrict__ near_ptr,
                                               const int32_t* __restrict__ nh_ptr,
                                               const int32_t* __restrict__ tsrc,
                                               const typename C2<T>::type* __restrict__ tpart,
                                               typename C2<T>::type* __restrict__ y, int Q, T w_re_xyz,
                                               T w_im_xyz, T w_re_d, T w_im_d) {
  using V2 = typename C2<T>::type;
  __shared__ __align__(16) V2 ow[4 * MAX_QL];
  __shared__ V2 red[NT];
  const int a = blockIdx.x;
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int J = 4 * Q, t = threadIdx.x;
  for (int j = t; j < J; j += NT) {
    const V2 ov = o[(size_t)a * J + j];
    const V2 wv = (j < 3 * Q) ? cmk<T>(w_re_xyz, w_im_xyz) : cmk<T>(w_re_d, w_im_d);
    ow[j] = cmul(ov, wv);
  }
  const int k0 = near_ptr[a], k1 = nh_ptr[a];
  if (t < S) {
    V2 v = y[p0 + t];
    for (int k = k0; k < k1; ++k) {
      const V2 u = tpart[tsrc[k] + t];
      v.x += u.x;
      v.y += u.y;
    }
    red[t] = v;
  }
  __syncthreads();
  recv_rows<T>(V, ow, red, y, p0, S, J);
}

// ------------------------------------------------------------------ translation operators
// D_u[p][q] = g(E_p + d_u - E_q), g = exp(-i k R) / (4 pi R), R the principal
// square root of the summed squared coordinate differences (Sec. 2, Eq. 6; the
// equivalent points E are complex).  Computed in FP64; stored column-major
// [u][q][Qr], rows p >= Q zero (padding of the row blocking).
template <typename V2>
__global__ void k_fill_translation(const double* __restrict__ E, const int32_t* __restrict__ off, double side,
                                   double k, int Q, int Qr, int64_t total, V2* __restrict__ D) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= total) return;
  const int p = (int)(i % Qr);
  const int64_t rest = i / Qr;
  const int q = (int)(rest % Q);
  const int64_t u = rest / Q;
  V2 out;
  out.x = 0;
  out.y = 0;
  if (p < Q) {
    double zr = 0, zi = 0;                 // sum_d (E_pd + off_d side - E_qd)^2
    for (int dd = 0; dd < 3; ++dd) {
      const double er = E[(3 * p + dd) * 2] + off[3 * u + dd] * side - E[(3 * q + dd) * 2];
      const double ei = E[(3 * p + dd) * 2 + 1] - E[(3 * q + dd) * 2 + 1];
      zr += er * er - ei * ei;
      zi += 2.0 * er * ei;
    }
    // principal square root, the cancellation-free branch of each half plane
    const double m = hypot(zr, zi);
    double a, b;
    if (zr >= 0) {
      a = sqrt(0.5 * (m + zr));
      b = a > 0 ? zi / (2.0 * a) : 0.0;
    } else {
      b = copysign(sqrt(0.5 * (m - zr)), zi);
      a = zi / (2.0 * b);
    }
    // exp(-i k R) / (4 pi R), R = a + i b
    double sn, cs;
    sincos(k * a, &sn, &cs);
    const double e = exp(k * b) / (4.0 * 3.14159265358979323846 * (a * a + b * b));
    const double nr = e * cs, ni = -e * sn;   // exp(-ikR) |R|^-2 / (4 pi) ...
    out.x = nr * a + ni * b;                  // ... times conj(R)
    out.y = ni * a - nr * b;
  }
  D[i] = out;
}

// ------------------------------------------------------------------ radiation operators
// V[pos][ch][q] = sum_j R_L[q][j] G_src[ch][j] (Sec. 2, Eq. 4-5): G_src holds
// the four channels of the RWG at leaf position pos -- phi_x, phi_y, phi_z
// (half-edge-weighted (r - free vertex) on each triangle) and div phi -- times
// g(|x_j - r|), integrated over its two triangles with the 3-point rule, x_j =
// check point j + leaf centre.  FP64 math; one workgroup per leaf, as many RWGs
// at a time as the LDS holds.
template <typename V2>
__global__ __launch_bounds__(NT) void k_fill_radiation(RadGeo g, V2* __restrict__ V) {
  constexpr int GS = 3072;                 // complex128 entries of the G_src tile
  __shared__ double2 Gs[GS];
  const int b = blockIdx.x;
  const int p0 = g.leaf_ptr[b], S = g.leaf_ptr[b + 1] - p0;
  const int M = g.M, Q = g.Q;
  const int nrw = max(1, GS / (4 * M));
  const double cx = g.centre[3 * b], cy = g.centre[3 * b + 1], cz = g.centre[3 * b + 2];
  const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
  for (int i0 = 0; i0 < S; i0 += nrw) {
    const int nr = min(nrw, S - i0);
    __syncthreads();                       // the previous tile consumed
    for (int e = threadIdx.x; e < nr * M; e += NT) {
      const int r = e / M, j = e - r * M;
      const int n = g.perm[p0 + i0 + r];
      const double xx = cx + g.X[3 * j], xy = cy + g.X[3 * j + 1], xz = cz + g.X[3 * j + 2];
      double2 acc[4];
      for (int c = 0; c < 4; ++c) acc[c].x = acc[c].y = 0;
      for (int sd = 0; sd < 2; ++sd) {
        const int T = g.tri[2 * n + sd], fv = g.freev[2 * n + sd];
        const double sg = sd == 0 ? 1.0 : -1.0;
        const double cv = sg * g.len[n] / (2.0 * g.area[T]);
        const double cdv = sg * g.len[n] / g.area[T];
        const double w = g.area[T] / 3.0;
        for (int qd = 0; qd < 3; ++qd) {
          const double rx = g.qp[9 * T + 3 * qd], ry = g.qp[9 * T + 3 * qd + 1], rz = g.qp[9 * T + 3 * qd + 2];
          const double ph[4] = {(rx - g.v[3 * fv]) * cv, (ry - g.v[3 * fv + 1]) * cv, (rz - g.v[3 * fv + 2]) * cv,
                                cdv};
          const double dx = xx - rx, dy = xy - ry, dz = xz - rz;
          const double R = sqrt(dx * dx + dy * dy + dz * dz);
          double sn, cs;
          sincos(g.k * R, &sn, &cs);
          const double gr = cs * inv4pi / R * w, gi = -sn * inv4pi / R * w;
          for (int c = 0; c < 4; ++c) {
            acc[c].x += gr * ph[c];
            acc[c].y += gi * ph[c];
          }
        }
      }
      for (int c = 0; c < 4; ++c) Gs[(r * 4 + c) * M + j] = acc[c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * 4 * Q; e += NT) {
      const int rc = e / Q, q = e - rc * Q;  // rc = 4 r + channel
      const double2* gs = Gs + rc * M;
      double sr = 0, si = 0;
      for (int j = 0; j < M; ++j) {
        const double2 rr = g.Rt[(size_t)j * Q + q], gv = gs[j];
        sr += rr.x * gv.x - rr.y * gv.y;
        si += rr.x * gv.y + rr.y * gv.x;
      }
      V2 out;
      out.x = sr;
      out.y = si;
      V[((size_t)(p0 + i0 + rc / 4) * 4 + rc % 4) * Q + q] = out;
    }
  }
}

template <typename V>
__global__ void k_fill_zero(V* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) {
    V z;
    z.x = 0;
    z.y = 0;
    p[i] = z;
  }
}

// ------------------------------------------------------------------ several right-hand sides
// Equivalent vectors hold NC = 4 R channels per box, channel c of RHS r at
// c * R + r.  Radiation, near field and reception read V and Z once per block
// of RB right-hand sides.
constexpr int RB = 8;

template <typename V2>
__global__ __launch_bounds__(NT) void k_radiate_multi(const V2* __restrict__ V, const V2* __restrict__ x,
                                                      const int32_t* __restrict__ leaf_ptr, V2* __restrict__ s,
                                                      int Q, int R, int64_t n) {
  __shared__ V2 xs[RB][64];
  const int b = blockIdx.x, r0 = blockIdx.y * RB, nr = min(RB, R - r0);
  const int p0 = leaf_ptr[b], S = leaf_ptr[b + 1] - p0;
  const int J = 4 * Q;
  // (loops over the accumulators fully unrolled: a runtime index would keep
  // them in private memory)
  V2 acc[2][RB];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[u][r].x = acc[u][r].y = 0;
  for (int i0 = 0; i0 < S; i0 += 64) {
    const int ni = min(64, S - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < RB * 64; e += NT) {
      const int r = e / 64, i = e % 64;
      if (r < nr && i < ni) xs[r][i] = x[(size_t)(r0 + r) * n + p0 + i0 + i];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = threadIdx.x + u * NT;
      if (j < J) {
        for (int i = 0; i < ni; ++i) {
          const V2 v = V[(size_t)(p0 + i0 + i) * J + j];
#pragma unroll
          for (int r = 0; r < RB; ++r) cfma(acc[u][r], v, xs[r][i]);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = threadIdx.x + u * NT;
    if (j < J) {
      const int c = j / Q, q = j % Q;
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < nr) s[((size_t)b * 4 * R + c * R + r0 + r) * Q + q] = acc[u][r];
    }
  }
}

// near field of several right-hand sides (RB per workgroup) with an arena in
// the full near-block layout: sub-chunks of CT columns, each thread holding at
// most U near entries of a sub-chunk and RB x CW / NT x values, loaded into
// registers while the previous sub-chunk is computed; x staged in LDS as
// [column][right-hand side] so that one entry meets its RB values in a few
// wide LDS reads
template <typename V2>
__global__ __launch_bounds__(NT) void k_near_multi(const V2* __restrict__ Z, const int64_t* __restrict__ zoff,
                                                   const int32_t* __restrict__ leaf_ptr,
                                                   const int32_t* __restrict__ near_ptr,
                                                   const int32_t* __restrict__ near_idx, const V2* __restrict__ x,
                                                   V2* __restrict__ y, int R, int64_t n) {
  constexpr int CW = 256;              // most columns per sub-chunk
  constexpr int U = 8;                 // near entries per thread per sub-chunk
  constexpr int XE = CW * RB / NT;     // x values per thread per sub-chunk
  __shared__ V2 xs[CW * RB];           // [column][rhs]; then the column groups' sums [rhs][NT]
  __shared__ int seg_col[MAX_NEAR + 1];
  __shared__ int seg_x[MAX_NEAR];
  static_assert(CW * RB == RB * NT, "the group sums reuse the staging array");
  const int a = blockIdx.x, r0 = blockIdx.y * RB, nr = min(RB, R - r0);
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int n0 = near_ptr[a], nn = near_ptr[a + 1] - n0;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int k = 0; k < nn; ++k) {
      const int b = near_idx[n0 + k];
      seg_col[k] = c;
      seg_x[k] = leaf_ptr[b];
      c += leaf_ptr[b + 1] - leaf_ptr[b];
    }
    seg_col[nn] = c;
  }
  __syncthreads();
  const int W = seg_col[nn];
  const V2* Za = Z + zoff[a];
  const int G = NT / S;
  const int t = threadIdx.x, g = t / S;
  const bool row_ok = g < G;
  const int CT = min(CW, U * G);
  V2 zr[U], xr[XE];
  auto fetch = [&](int c0) {
    const int cw = min(CT, W - c0);
    const V2* Zp = Za + (size_t)c0 * S + t;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = g + u * G;
      if (row_ok && j < cw) zr[u] = Zp[(size_t)(u * G) * S];
    }
#pragma unroll
    for (int e = 0; e < XE; ++e) {
      const int idx = t + e * NT, r = idx / CT, j = idx - r * CT;
      if (r < nr && j < cw) {
        const int col = c0 + j;
        int k = 0;
        while (seg_col[k + 1] <= col) ++k;
        xr[e] = x[(size_t)(r0 + r) * n + seg_x[k] + (col - seg_col[k])];
      }
    }
  };
  V2 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = 0;
  if (W > 0) fetch(0);
  for (int c0 = 0; c0 < W; c0 += CT) {
    const int cw = min(CT, W - c0);
    __syncthreads();                   // the previous sub-chunk's x consumed
#pragma unroll
    for (int e = 0; e < XE; ++e) {
      const int idx = t + e * NT, r = idx / CT, j = idx - r * CT;
      if (r < nr && j < cw) xs[j * RB + r] = xr[e];
    }
    __syncthreads();
    V2 zc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) zc[u] = zr[u];
    if (c0 + CT < W) fetch(c0 + CT);
    if (row_ok) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = g + u * G;
        if (j < cw) {
          const V2* xj = xs + j * RB;
#pragma unroll
          for (int r = 0; r < RB; ++r) cfma(acc[r], zc[u], xj[r]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RB; ++r) xs[r * NT + t] = acc[r];
  __syncthreads();
  // reduce the column groups (fixed order)
  for (int e = t; e < nr * S; e += NT) {
    const int r = e / S, m = e % S;
    V2 v = xs[r * NT + m];
    for (int gg = 1; gg < G; ++gg) {
      v.x += xs[r * NT + gg * S + m].x;
      v.y += xs[r * NT + gg * S + m].y;
    }
    y[(size_t)(r0 + r) * n + p0 + m] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_recv_multi(const typename C2<T>::type* __restrict__ V,
                                                   const typename C2<T>::type* __restrict__ o,
                                                   const int32_t* __restrict__ leaf_ptr,
                                                   typename C2<T>::type* __restrict__ y, int Q, int R, int64_t n,
                                                   T w_re_xyz, T w_im_xyz, T w_re_d, T w_im_d) {
  using V2 = typename C2<T>::type;
  __shared__ __align__(16) V2 ow[RB][4 * MAX_QL / 2];
  const int a = blockIdx.x, r0 = blockIdx.y * RB, nr = min(RB, R - r0);
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  const int J = 4 * Q;
  for (int e = threadIdx.x; e < RB * J; e += NT) {
    const int r = e / J, j = e % J;
    const int c = j / Q, q = j % Q;
    V2 v = cmk<T>(0, 0);
    if (r < nr) {
      const V2 ov = o[((size_t)a * 4 * R + c * R + r0 + r) * Q + q];
      const V2 wv = (c < 3) ? cmk<T>(w_re_xyz, w_im_xyz) : cmk<T>(w_re_d, w_im_d);
      v = cmul(ov, wv);
    }
    ow[r][j] = v;
  }
  __syncthreads();
  // 8 lanes per row and 8 rows per wave: every lane keeps the partial sums of
  // all RB right-hand sides, so one row of V is read once and each sum takes 3
  // shuffle steps
  constexpr int LR = 8;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int c = lane % LR, sub = lane / LR;
  for (int row0 = wv * (WAVE / LR); row0 < S; row0 += (NT / WAVE) * (WAVE / LR)) {
    const int row = row0 + sub;
    V2 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = cmk<T>(0, 0);
    if (row < S) {
      const V2* Vr = V + (size_t)(p0 + row) * J;
#pragma unroll 2
      for (int j = c; j < J; j += LR) {
        const V2 v = Vr[j];
#pragma unroll
        for (int r = 0; r < RB; ++r) cfma(acc[r], v, ow[r][j]);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
      for (int off = LR / 2; off > 0; off >>= 1) {
        acc[r].x += __shfl_xor(acc[r].x, off);
        acc[r].y += __shfl_xor(acc[r].y, off);
      }
    if (c == 0 && row < S) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r >= nr) break;
        V2* yp = y + (size_t)(r0 + r) * n + p0 + row;
        V2 out = *yp;
        out.x += acc[r].x;
        out.y += acc[r].y;
        *yp = out;
      }
    }
  }
}

// ------------------------------------------------------------------ vector ops (GMRES)
// partial[blk][i] = sum over the block's chunk of conj(basis_i) * w, FP64
// accumulation; basis vectors taken 8 at a time.
constexpr int MD_CH = 8;
constexpr int MD_U = 4;      // elements per thread whose loads are in flight together
template <typename V>
__global__ __launch_bounds__(NT) void k_multidot(const V* __restrict__ basis, int64_t ld, int nvec,
                                                 const V* __restrict__ w, int64_t n, double2* __restrict__ partial) {
  __shared__ double2 red[NT / WAVE][MD_CH];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int i0 = 0; i0 < nvec; i0 += MD_CH) {
    const int ni = min(MD_CH, nvec - i0);
    double2 acc[MD_CH];
#pragma unroll
    for (int i = 0; i < MD_CH; ++i) acc[i] = make_double2(0, 0);
    // MD_U elements per thread in flight at once, each with its MD_CH basis
    // values: every load is issued before the sums (a guarded load per vector
    // had waited for each in turn).  Past the last vector the chunk reads the
    // last one again (those sums are never stored); past n an element reads
    // element e0 with w taken as zero.  Each thread adds its elements in
    // increasing order.
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t e0 = (int64_t)blockIdx.x * NT + threadIdx.x; e0 < n; e0 += MD_U * stride) {
      V we[MD_U], b[MD_U][MD_CH];
#pragma unroll
      for (int u = 0; u < MD_U; ++u) {
        const int64_t e = e0 + u * stride;
        const int64_t ec = e < n ? e : e0;
        we[u] = w[ec];
#pragma unroll
        for (int i = 0; i < MD_CH; ++i) b[u][i] = basis[(size_t)(i0 + min(i, ni - 1)) * ld + ec];
        if (e >= n) we[u].x = we[u].y = 0;
      }
#pragma unroll
      for (int u = 0; u < MD_U; ++u)
#pragma unroll
        for (int i = 0; i < MD_CH; ++i) {
          acc[i].x += (double)b[u][i].x * (double)we[u].x + (double)b[u][i].y * (double)we[u].y;
          acc[i].y += (double)b[u][i].x * (double)we[u].y - (double)b[u][i].y * (double)we[u].x;
        }
    }
    for (int i = 0; i < MD_CH; ++i) {
      double2 s = acc[i];
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        s.x += __shfl_xor(s.x, off);
        s.y += __shfl_xor(s.y, off);
      }
      if (lane == 0) red[wv][i] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < ni) {
      double2 s = red[0][threadIdx.x];
      for (int ww = 1; ww < NT / WAVE; ++ww) {
        s.x += red[ww][threadIdx.x].x;
        s.y += red[ww][threadIdx.x].y;
      }
      partial[(size_t)blockIdx.x * nvec + i0 + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[i] (+)= sum over blocks of partial[blk][i]; one workgroup per i, fixed
// summation tree (deterministic)
__global__ __launch_bounds__(NT) void k_reduce_partials(const double2* __restrict__ partial, int nblk, int nvec,
                                                        double2* __restrict__ out, int accumulate) {
  __shared__ double2 red[NT];
  const int i = blockIdx.x;
  double2 s = make_double2(0, 0);
  for (int b = threadIdx.x; b < nblk; b += NT) {
    s.x += partial[(size_t)b * nvec + i].x;
    s.y += partial[(size_t)b * nvec + i].y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[threadIdx.x].x += red[threadIdx.x + off].x;
      red[threadIdx.x].y += red[threadIdx.x + off].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (accumulate) {
      out[i].x += red[0].x;
      out[i].y += red[0].y;
    } else {
      out[i] = red[0];
    }
  }
}

// w[e] -= sum_i h[i] * basis_i[e]   (sign = -1), or x[e] += sum_i h[i] basis_i[e] (sign = +1)
template <typename V>
__global__ void k_combine(const V* __restrict__ basis, int64_t ld, int nvec, const double2* __restrict__ h,
                          V* __restrict__ w, int64_t n, double sign) {
  __shared__ double2 hs[256];
  for (int i = threadIdx.x; i < nvec && i < 256; i += NT) hs[i] = h[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n) return;
  double ax = 0, ay = 0;
  for (int i = 0; i < nvec; ++i) {
    const V b = basis[(size_t)i * ld + e];
    ax += hs[i].x * (double)b.x - hs[i].y * (double)b.y;
    ay += hs[i].x * (double)b.y + hs[i].y * (double)b.x;
  }
  V we = w[e];
  we.x = (decltype(we.x))((double)we.x + sign * ax);
  we.y = (decltype(we.y))((double)we.y + sign * ay);
  w[e] = we;
}

// y = alpha * x  (alpha real)
template <typename V>
__global__ void k_scale(const V* __restrict__ x, V* __restrict__ y, int64_t n, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n) return;
  V v = x[e];
  v.x = (decltype(v.x))((double)v.x * alpha);
  v.y = (decltype(v.y))((double)v.y * alpha);
  y[e] = v;
}

// y = x / sqrt(nrm->x): the Arnoldi normalisation with the squared norm taken
// on the device (FP64, the host's arithmetic: alpha = 1 / sqrt(max(0, s)));
// a zero norm gives a zero vector
template <typename V>
__global__ void k_scale_norm(const V* __restrict__ x, V* __restrict__ y, int64_t n, const double2* __restrict__ nrm) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n) return;
  const double s = nrm->x;
  const double alpha = s > 0 ? 1.0 / sqrt(s) : 0.0;
  V v = x[e];
  v.x = (decltype(v.x))((double)v.x * alpha);
  v.y = (decltype(v.y))((double)v.y * alpha);
  y[e] = v;
}

// y = a - b
template <typename V>
__global__ void k_sub(const V* __restrict__ a, const V* __restrict__ b, V* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n) return;
  V u = a[e], v = b[e];
  u.x -= v.x;
  u.y -= v.y;
  y[e] = u;
}

// Block-diagonal preconditioner: z_a = Minv_a r_a, Minv_a S x S column-major.
template <typename T>
__global__ __launch_bounds__(NT) void k_blockdiag(const typename C2<T>::type* __restrict__ Minv,
                                                  const int64_t* __restrict__ moff,
                                                  const int32_t* __restrict__ leaf_ptr,
                                                  const typename C2<T>::type* __restrict__ r,
                                                  typename C2<T>::type* __restrict__ z) {
  using V2 = typename C2<T>::type;
  __shared__ V2 rs[NT];
  const int a = blockIdx.x;
  const int p0 = leaf_ptr[a], S = leaf_ptr[a + 1] - p0;
  if ((int)threadIdx.x < S) rs[threadIdx.x] = r[p0 + threadIdx.x];
  __syncthreads();
  if ((int)threadIdx.x < S) {
    const V2* M = Minv + moff[a] + threadIdx.x;
    V2 acc = cmk<T>(0, 0);
    for (int j = 0; j < S; ++j) cfma(acc, M[(size_t)j * S], rs[j]);
    z[p0 + threadIdx.x] = acc;
  }
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// columns per workgroup of the split target-major kernel (NESA_TM_COLS=128
// selects the narrower tile: half the source bytes per workgroup, twice the
// matrix reads)
static int tm_split_cols() {
  static const int c = []() {
    const char* e = std::getenv("NESA_TM_COLS");
    return (e && std::atoi(e) == 128) ? 128 : 256;
  }();
  return c;
}

// rows per workgroup of the split target-major kernel for M output rows: 128
// x 128 tiles when M > 64 (every source block serves twice the rows per read,
// each translation row is read by two column tiles), 64 x 256 below;
// NESA_TM_ROWS=64 keeps 64-row tiles everywhere
static int tm_split_rows(int M) {
  static const bool only64 = []() {
    const char* e = std::getenv("NESA_TM_ROWS");
    return e && std::atoi(e) == 64;
  }();
  return (!only64 && M > 64) ? 128 : 64;
}

static void launch_tiles(const GemmPlan& p, int nrhs, const void* src, void* dst, hipStream_t st,
                         bool translation) {
  const TileList& tl = p.by_nrhs[nrhs];
  if (tl.width == 128) {
    // split form on the sources split once per level
    launch_om_split2(p, tl, nrhs, p.s6, dst, st);
    return;
  }
  GemmTiles g;
  g.A = static_cast<const float2*>(p.A);
  g.a_stride = p.a_stride;
  g.M = p.M;
  g.K = p.K;
  g.Mr = p.Mr;
  g.src = static_cast<const float2*>(src);
  g.dst = static_cast<float2*>(dst);
  g.accumulate = p.accumulate;
  g.ntiles = tl.ntiles;
  g.tile_group = tl.tile_group;
  g.tile_ncols = tl.tile_ncols;
  g.col_src = tl.col_src;
  g.col_dst = tl.col_dst;
  if (tl.ntiles == 0) return;
  const int nrt = tl.nrt > 0 ? tl.nrt : p.nrt;
  const int rblocks = tl.nrt > 0 ? tl.rblocks : p.rblocks;
  if (tl.tpw < 0 && !p.A_split) {
    // direct kernel: K <= 4 ks (ks = -tpw is 13 or 21), 1, 2 or 4 row tiles
    dim3 gr((unsigned)((tl.ntiles + 7) / 8 * 8), (unsigned)rblocks);
#define NESA_DIR(N, KSV)                                                      \
  if (translation)                                                            \
    k_translate_gemm_dir<N, KSV><<<gr, NT, 0, st>>>(g);                       \
  else                                                                        \
    k_transfer_gemm_dir<N, KSV><<<gr, NT, 0, st>>>(g);                        \
  return;
#define NESA_DIR_K(N)                    \
  if (-tl.tpw == 13) { NESA_DIR(N, 13) }  \
  else { NESA_DIR(N, 21) }
    switch (nrt) {
      case 1: NESA_DIR_K(1)
      case 2: NESA_DIR_K(2)
      default: NESA_DIR_K(4)
    }
#undef NESA_DIR_K
#undef NESA_DIR
  }
  if (tl.tpw > 0 && !p.A_split) {
    // resident-A kernel: runs of tpw tiles, K <= kt
    const int64_t nruns = (tl.ntiles + tl.tpw - 1) / tl.tpw;
    dim3 gr((unsigned)((nruns + 7) / 8 * 8), (unsigned)rblocks);
#define NESA_RES(N, KTV)                                                          \
  if (translation)                                                                \
    k_translate_gemm_res<N, KTV><<<gr, NT, 0, st>>>(g, tl.tpw);                   \
  else                                                                            \
    k_transfer_gemm_res<N, KTV><<<gr, NT, 0, st>>>(g, tl.tpw);                    \
  return;
#define NESA_RES_K(N)                    \
  if (tl.kt == 52) { NESA_RES(N, 52) }    \
  else { NESA_RES(N, 84) }
    switch (nrt) {
      case 1: NESA_RES_K(1)
      case 2: NESA_RES_K(2)
      case 3: NESA_RES_K(3)
      case 4: NESA_RES_K(4)
      case 5: NESA_RES_K(5)
      case 6: NESA_RES_K(6)
      case 7: NESA_RES_K(7)
      default: NESA_RES_K(8)
    }
#undef NESA_RES_K
#undef NESA_RES
  }
  dim3 grid((unsigned)((tl.ntiles + 7) / 8 * 8), (unsigned)rblocks);
  if (tl.width == 32 && p.A_split) {
    // split form, 32-column tiles: waves split the rows (NRT even)
    const unsigned short* As = static_cast<const unsigned short*>(p.A_split);
    const bool h = p.split_fmt == SPLIT_FP16;
    const int ae = h ? p.a_exp : 0;
    const int* be = h ? p.bexp : nullptr;
#define NESA_SPLIT32(N)                                                              \
  if (h) {                                                                           \
    if (translation)                                                                 \
      k_translate_gemm_bf16x3<N, 1, 2><<<grid, NT, 0, st>>>(g, As, p.Kp, ae, be);    \
    else                                                                             \
      k_transfer_gemm_bf16x3<N, 1, 2><<<grid, NT, 0, st>>>(g, As, p.Kp, ae, be);     \
  } else if (translation) {                                                          \
    k_translate_gemm_bf16x3<N, 0, 2><<<grid, NT, 0, st>>>(g, As, p.Kp, ae, be);      \
  } else {                                                                           \
    k_transfer_gemm_bf16x3<N, 0, 2><<<grid, NT, 0, st>>>(g, As, p.Kp, ae, be);       \
  }                                                                                  \
  return;
    switch (nrt) {
      case 2: NESA_SPLIT32(2)
      case 4: NESA_SPLIT32(4)
      case 6: NESA_SPLIT32(6)
      default: NESA_SPLIT32(8)
    }
#undef NESA_SPLIT32
  }
  if (tl.width == 32 && !p.A_split) {
    // 32-column tiles: waves split the rows (NRT even)
#define NESA_TILES32(N)                                                   \
  if (tl.m3) {                                                            \
    if (translation)                                                      \
      k_translate_gemm<N, 2, 1><<<grid, NT, 0, st>>>(g);                  \
    else                                                                  \
      k_transfer_gemm<N, 2, 1><<<grid, NT, 0, st>>>(g);                   \
  } else if (translation) {                                               \
    k_translate_gemm<N, 2, 0><<<grid, NT, 0, st>>>(g);                    \
  } else {                                                                \
    k_transfer_gemm<N, 2, 0><<<grid, NT, 0, st>>>(g);                     \
  }                                                                       \
  return;
    switch (nrt) {
      case 2: NESA_TILES32(2)
      case 4: NESA_TILES32(4)
      case 6: NESA_TILES32(6)
      default: NESA_TILES32(8)
    }
#undef NESA_TILES32
  }
#define NESA_TILES(N)                                                                        \
  if (p.A_split) {                                                                           \
    const unsigned short* As = static_cast<const unsigned short*>(p.A_split);                \
    if (p.split_fmt == SPLIT_FP16) {                                                         \
      if (translation)                                                                       \
        k_translate_gemm_bf16x3<N, 1, 4><<<grid, NT, 0, st>>>(g, As, p.Kp, p.a_exp, p.bexp); \
      else                                                                                   \
        k_transfer_gemm_bf16x3<N, 1, 4><<<grid, NT, 0, st>>>(g, As, p.Kp, p.a_exp, p.bexp);  \
    } else if (translation) {                                                                \
      k_translate_gemm_bf16x3<N, 0, 4><<<grid, NT, 0, st>>>(g, As, p.Kp, 0, nullptr);        \
    } else {                                                                                 \
      k_transfer_gemm_bf16x3<N, 0, 4><<<grid, NT, 0, st>>>(g, As, p.Kp, 0, nullptr);         \
    }                                                                                        \
  } else if (tl.m3) {                                                                       \
    if (translation)                                                                         \
      k_translate_gemm<N, 4, 1><<<grid, NT, 0, st>>>(g);                                     \
    else                                                                                     \
      k_transfer_gemm<N, 4, 1><<<grid, NT, 0, st>>>(g);                                      \
  } else if (translation) {                                                                  \
    k_translate_gemm<N, 4, 0><<<grid, NT, 0, st>>>(g);                                       \
  } else {                                                                                   \
    k_transfer_gemm<N, 4, 0><<<grid, NT, 0, st>>>(g);                                        \
  }                                                                                          \
  break;
  switch (nrt) {
    case 1: NESA_TILES(1)
    case 2: NESA_TILES(2)
    case 3: NESA_TILES(3)
    case 4: NESA_TILES(4)
    case 5: NESA_TILES(5)
    case 6: NESA_TILES(6)
    case 7: NESA_TILES(7)
    default: NESA_TILES(8)
  }
#undef NESA_TILES
}

void launch_plan(const GemmPlan& p, int nrhs, const void* src, void* dst, hipStream_t st, bool translation) {
  launch_tiles(p, nrhs, src, dst, st, translation);
}

// grid of an ordered per-box sum: enough workgroups to fill the chip when
// there are few boxes (each takes a share of the box's elements)
// grid of k_csr_reduce for J complex64 values per row (two per thread)
static dim3 csr_grid(int64_t nbox, int J) {
  const int chunks = (J / 2 + NT - 1) / NT;
  int y = 1;
  while (y < chunks && nbox * y < 2048) ++y;
  return dim3((unsigned)nbox, (unsigned)y);
}

// whether the offset-major product of a plan at R right-hand sides reads the
// pre-split sources (the autotuner's choice; tiles are built before the
// operator's first product at R)
static bool presplit(const GemmPlan& p, int R) {
  if ((int)p.by_nrhs.size() <= R || !p.by_nrhs[R].tile_group)
    throw std::runtime_error("product tiles for this number of right-hand sides not built");
  return p.by_nrhs[R].width == 128;
}

template <typename T>
void launch_matvec_leaf(const DevOp<T>& d, const void* xl_, void* yl_, int R, hipStream_t st, PhaseTimer* tm) {
  using V2 = typename C2<T>::type;
  const V2* xl = static_cast<const V2*>(xl_);
  V2* yl = static_cast<V2*>(yl_);
  V2* s = static_cast<V2*>(d.s);
  V2* o = static_cast<V2*>(d.o);
  const int L = d.L, l0 = d.l0;
  const auto& LL = d.lev[L - l0];
  const bool mfma = sizeof(T) == 4;
  const int NC = 4 * R;
  const unsigned rblk = (unsigned)((R + RB - 1) / RB);
  if (!mfma && R != 1) return;   // the complex128 path takes one right-hand side at a time
  // untimed products run the near field (HBM-bound) on a side stream while
  // this stream runs the far-field stages (matrix-core bound); the timed form
  // keeps every stage on one stream so that stage times stay separate
  const bool overlap = (!tm || tm->overlap) && d.side != nullptr && (R == 1 || mfma);
  auto fork_near = [&]() {
    hip_ok(hipEventRecord(d.ev_fork, st));
    hip_ok(hipStreamWaitEvent(d.side, d.ev_fork, 0));
    if (R == 1) {
      const unsigned nwg = (unsigned)std::min<int64_t>(d.nleaf, d.near_wgs > 0 ? d.near_wgs : 256);
      k_near_half<T><<<nwg, NT, 0, d.side>>>(static_cast<const V2*>(d.Zh), d.zh_off, d.leaf_ptr, d.nh_ptr,
                                            d.near_ptr, d.near_idx, d.toff, xl, yl, static_cast<V2*>(d.tpart),
                                            d.nleaf, d.near_order);
    } else {
      if constexpr (sizeof(T) == 4) {
        if (R >= LEAF_MFMA_MIN_R)
          launch_near_mfma(static_cast<const float2*>(d.Z), d.zoff, d.leaf_ptr, d.near_ptr, d.near_idx,
                           reinterpret_cast<const float2*>(xl), reinterpret_cast<float2*>(yl), d.nleaf, R, d.n,
                           d.side);
        else
          k_near_multi<V2><<<dim3((unsigned)d.nleaf, rblk), NT, 0, d.side>>>(static_cast<const V2*>(d.Z), d.zoff,
                                                                            d.leaf_ptr, d.near_ptr, d.near_idx, xl,
                                                                            yl, R, d.n);
      }
    }
    hip_ok(hipEventRecord(d.ev_join, d.side));
  };
  // complex64 with more than pair_cap right-hand sides: translations and
  // transfers run target-major (no per-pair or per-child partial results); the
  // split form with TM2_MIN_COLS or more columns reads sources split once per
  // level into the level's s6 planes
  const bool tmode = mfma && R > d.pair_cap;
  bool v2 = tmode && NC >= TM2_MIN_COLS;
  for (const auto& lv : d.lev) v2 = v2 && lv.s6 != nullptr;     // (allocated for split operators only)
  // split operators at up to pair_cap right-hand sides: the offset-major
  // products that the autotuner put on the pre-split sources need the level's
  // sources (which 0) or potentials (which 1) split into its s6 planes
  const bool om2 = mfma && !tmode && d.om2;
  auto need = [&](int l, int which) {
    if (v2) return true;
    if (!om2) return false;
    const auto& lv = d.lev[l - l0];
    if (which == 1) return l < L && presplit(d.lev[l + 1 - l0].down, R);
    return (lv.npairs > 0 && presplit(lv.trans, R)) || (l > l0 && presplit(lv.up, R));
  };
  // fp16 split form: the largest exponent of every level's sources (slot
  // 2 (l - l0)) and potentials (2 (l - l0) + 1), taken once the vector is
  // complete and before the products that read it
  auto exp_slot = [&](int l, int which) { return d.bexp + 2 * (l - l0) + which; };
  auto absmax = [&](int l, int which, const V2* v) {
    if (d.bexp) launch_absmax_exp(v, d.lev[l - l0].nbox * NC * d.lev[l - l0].Q, false, exp_slot(l, which), st);
  };
  auto split_of = [&](int l, int which, const V2* src, hipStream_t ss) {
    if constexpr (sizeof(T) == 4) {
      const auto& lv = d.lev[l - l0];
      launch_split_sources(src, lv.nbox, NC, lv.Q, (lv.Q + 31) / 32 * 32, lv.s6, d.split_fmt,
                           d.bexp ? exp_slot(l, which) : nullptr, ss);
    }
  };
  auto tm_contract = [&](const GemmPlan& pl, const int32_t* ptr, const int32_t* src, const int32_t* slot,
                         int64_t ntarget, int M, int K, const V2* sv, const void* s6v, V2* ov, int acc,
                         hipStream_t ss) {
    if constexpr (sizeof(T) == 4) {
      TmArgs g;
      g.D = static_cast<const float2*>(pl.A);
      g.Asplit = static_cast<const unsigned short*>(pl.A_split);
      g.a_stride = pl.a_stride;
      g.M = M;
      g.K = K;
      g.Mr = pl.Mr;
      g.Kp = pl.Kp;
      g.s = reinterpret_cast<const float2*>(sv);
      g.o = reinterpret_cast<float2*>(ov);
      g.il_ptr = ptr;
      g.il_src = src;
      g.il_slot = slot;
      g.nbox = ntarget;
      g.NC = NC;
      g.accumulate = acc;
      g.split_fmt = pl.split_fmt;
      g.a_exp = pl.a_exp;
      g.bexp = pl.bexp;
      int nrt = 0, rblocks = 0, ct = 0;
      tm_blocking(M, pl.Mr, NC, nrt, rblocks, ct);
      g.nct = (NC + 16 * (g.Asplit ? 4 : ct) - 1) / (16 * (g.Asplit ? 4 : ct));
      if (v2) {
        g.s6 = static_cast<const uint4*>(s6v);
        g.tm_rows = tm_split_rows(M);
        g.nct_cols = g.tm_rows == 128 ? 128 : tm_split_cols();
        g.nct = (NC + g.nct_cols - 1) / g.nct_cols;
      }
      launch_translate_tm(g, nrt, rblocks, ct, ss);
    }
  };
  // translations of one level (complex64)
  auto translate = [&](const DevLevel& lv, hipStream_t ss, int l) {
    if (tmode) {
      tm_contract(lv.trans, lv.il_ptr, lv.il_src, lv.il_slot, lv.nbox, lv.Q, lv.Q, s + lv.s_off * R, lv.s6,
                  o + lv.s_off * R, 0, ss);
      if (tm && ss == st) tm->mark(st, -1, l, K_TRANS_GEMM);
      return;
    }
    launch_tiles(lv.trans, R, s + lv.s_off * R, lv.pair_out, ss, true);
    if (tm && ss == st) tm->mark(st, -1, l, K_TRANS_GEMM);
    k_csr_reduce<V2><<<csr_grid(lv.nbox, NC * lv.Q), NT, 0, ss>>>(static_cast<const V2*>(lv.pair_out),
                                                                  o + lv.s_off * R, lv.il_ptr, lv.il_ptr + 1,
                                                                  NC * lv.Q);
    if (tm && ss == st) tm->mark(st, -1, l, K_TRANS_REDUCE);
  };
  if (tm) tm->mark(st, 0, -1, 0);
  if (d.bexp) launch_exp_reset(d.bexp, 2 * (L - l0 + 1), st);
  if (R == 1) {
    k_radiate<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(d.V), xl, d.leaf_ptr, s + LL.s_off, LL.Q);
  } else {
    if constexpr (sizeof(T) == 4) {
      if (R >= LEAF_MFMA_MIN_R)
        launch_radiate_mfma(static_cast<const float2*>(d.V), reinterpret_cast<const float2*>(xl), d.leaf_ptr,
                            reinterpret_cast<float2*>(s + LL.s_off * R), d.nleaf, LL.Q, R, d.n, st);
      else
        k_radiate_multi<V2><<<dim3((unsigned)d.nleaf, rblk), NT, 0, st>>>(static_cast<const V2*>(d.V), xl,
                                                                         d.leaf_ptr, s + LL.s_off * R, LL.Q, R, d.n);
    }
  }
  if (tm) tm->mark(st, 1, L, K_RADIATE);
  absmax(L, 0, s + LL.s_off * R);
  if (need(L, 0)) split_of(L, 0, s + LL.s_off * R, st);
  // the near field starts once radiation (also HBM-bound) is done, and runs
  // beside the transfers and translations
  if (overlap) fork_near();
  // the finest level's translations (the largest launch) need only the
  // radiated sources: on a second side stream they run beside the upward pass
  // (small, latency-bound launches) and the coarser levels' translations; the
  // downward step into the finest level waits for them.  (Moving the next
  // level there as well, after the first upward step, measured slower: it then
  // competes with the coarse levels' translations.)
  auto side_ok = [&](int l) {
    return overlap && !tm && mfma && d.side2 != nullptr && l > l0 && l == L && d.lev[l - l0].npairs > 0;
  };
  auto fork_trans = [&](int l, hipEvent_t fork, hipEvent_t join) {
    const auto& lv = d.lev[l - l0];
    hip_ok(hipEventRecord(fork, st));
    hip_ok(hipStreamWaitEvent(d.side2, fork, 0));
    translate(lv, d.side2, l);
    hip_ok(hipEventRecord(join, d.side2));
  };
  if (side_ok(L)) fork_trans(L, d.ev_fork2, d.ev_join2);
  for (int l = L; l > l0; --l) {
    const auto& c = d.lev[l - l0];
    const auto& p = d.lev[l - 1 - l0];
    if (tmode) {
      tm_contract(c.up, c.up_ptr, c.up_src, c.up_slot, p.nbox, p.Q, c.Q, s + c.s_off * R, c.s6, s + p.s_off * R, 0,
                  st);
      if (tm) tm->mark(st, -1, l, K_UP_GEMM);
      absmax(l - 1, 0, s + p.s_off * R);
      if (need(l - 1, 0)) split_of(l - 1, 0, s + p.s_off * R, st);
    } else if (mfma) {
      launch_tiles(c.up, R, s + c.s_off * R, c.child_out, st, false);
      if (tm) tm->mark(st, -1, l, K_UP_GEMM);
      k_csr_reduce<V2><<<csr_grid(p.nbox, NC * p.Q), NT, 0, st>>>(static_cast<const V2*>(c.child_out),
                                                                   s + p.s_off * R, p.child_ptr, p.child_end,
                                                                   NC * p.Q);
      if (tm) tm->mark(st, -1, l, K_UP_REDUCE);
      absmax(l - 1, 0, s + p.s_off * R);
      if (need(l - 1, 0)) split_of(l - 1, 0, s + p.s_off * R, st);
    } else {
      dim3 grid((unsigned)((p.Q + WAVE - 1) / WAVE), (unsigned)p.nbox);
      k_upward<T><<<grid, NT, 0, st>>>(static_cast<const V2*>(c.Ccm), s + c.s_off, s + p.s_off, p.child_ptr,
                                       p.child_end, c.octant, p.Q, c.Q);
      if (tm) tm->mark(st, -1, l, K_UP_VALU);
    }
  }
  if (tm) tm->mark(st, 2, -1, 0);
  for (int l = l0; l <= L; ++l) {
    const auto& lv = d.lev[l - l0];
    if (side_ok(l)) continue;
    if (mfma && lv.npairs > 0) {
      // each level's sums right after its GEMM, while its per-pair outputs are
      // still in the last-level cache (one launch for all levels measured slower)
      translate(lv, st, l);
    } else if (mfma) {
      const int64_t cnt = lv.nbox * NC * lv.Q;
      k_fill_zero<V2><<<(unsigned)((cnt + NT - 1) / NT), NT, 0, st>>>(o + lv.s_off * R, cnt);
    } else {
      dim3 grid((unsigned)((lv.Q + WAVE - 1) / WAVE), (unsigned)lv.nbox);
      k_translate<T><<<grid, NT, 0, st>>>(static_cast<const V2*>(lv.D), s + lv.s_off, o + lv.s_off, lv.il_ptr,
                                          lv.il_src, lv.il_slot, lv.Q);
      if (tm) tm->mark(st, -1, l, K_TRANS_VALU);
    }
  }
  if (tm) tm->mark(st, 3, -1, 0);
  for (int l = l0 + 1; l <= L; ++l) {
    const auto& c = d.lev[l - l0];
    const auto& p = d.lev[l - 1 - l0];
    if (side_ok(l)) hip_ok(hipStreamWaitEvent(st, d.ev_join2, 0));
    if (mfma) absmax(l - 1, 1, o + p.s_off * R);
    if (tmode) {
      // the parent level's potentials split into its s6 planes (its
      // translations, which read them as sources, were launched before)
      if (need(l - 1, 1)) split_of(l - 1, 1, o + p.s_off * R, st);
      tm_contract(c.down, c.dn_ptr, c.dn_src, c.dn_slot, c.nbox, c.Q, p.Q, o + p.s_off * R, p.s6, o + c.s_off * R, 1,
                  st);
      if (tm) tm->mark(st, -1, l, K_DOWN_GEMM);
    } else if (mfma) {
      // the parent level's potentials split into its s6 planes if the
      // product reads them there (its translations, which read the sources
      // there, were launched before)
      if (need(l - 1, 1)) split_of(l - 1, 1, o + p.s_off * R, st);
      launch_tiles(c.down, R, o + p.s_off * R, o + c.s_off * R, st, false);
      if (tm) tm->mark(st, -1, l, K_DOWN_GEMM);
    } else {
      dim3 grid((unsigned)((c.Q + WAVE - 1) / WAVE), (unsigned)c.nbox);
      k_downward<T><<<grid, NT, 0, st>>>(static_cast<const V2*>(c.Crm), o + p.s_off, o + c.s_off, c.parent,
                                         c.octant, p.Q, c.Q);
      if (tm) tm->mark(st, -1, l, K_DOWN_VALU);
    }
  }
  if (tm) tm->mark(st, 4, -1, 0);
  if (overlap) {
    // the near field ran on the side stream: join, then add the reception
    hip_ok(hipStreamWaitEvent(st, d.ev_join, 0));
    if (tm) tm->mark(st, -1, L, 0);     // the reception's time starts after the join
    if (R == 1)
      k_recv1h<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(d.V), o + LL.s_off, d.leaf_ptr,
                                                    d.near_ptr, d.nh_ptr, d.tsrc,
                                                    static_cast<const V2*>(d.tpart), yl, LL.Q, (T)d.w[0],
                                                    (T)d.w[1], (T)d.w[2], (T)d.w[3]);
    else if constexpr (sizeof(T) == 4) {
      if (R >= LEAF_MFMA_MIN_R)
        launch_recv_mfma(static_cast<const float2*>(d.V), reinterpret_cast<const float2*>(o + LL.s_off * R),
                         d.leaf_ptr, reinterpret_cast<float2*>(yl), d.nleaf, LL.Q, R, d.n, d.w, st);
      else
        k_recv_multi<T><<<dim3((unsigned)d.nleaf, rblk), NT, 0, st>>>(static_cast<const V2*>(d.V),
                                                                     o + LL.s_off * R, d.leaf_ptr, yl, LL.Q, R, d.n,
                                                                     (T)d.w[0], (T)d.w[1], (T)d.w[2], (T)d.w[3]);
    }
  } else if (R == 1) {
    k_near_half<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(d.Zh), d.zh_off, d.leaf_ptr, d.nh_ptr,
                                                    d.near_ptr, d.near_idx, d.toff, xl, yl,
                                                    static_cast<V2*>(d.tpart), d.nleaf, d.near_order);
    k_recv1h<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(d.V), o + LL.s_off, d.leaf_ptr, d.near_ptr,
                                                  d.nh_ptr, d.tsrc, static_cast<const V2*>(d.tpart), yl, LL.Q,
                                                  (T)d.w[0], (T)d.w[1], (T)d.w[2], (T)d.w[3]);
  } else {
    if constexpr (sizeof(T) == 4) {
      if (R >= LEAF_MFMA_MIN_R) {
        launch_near_mfma(static_cast<const float2*>(d.Z), d.zoff, d.leaf_ptr, d.near_ptr, d.near_idx,
                         reinterpret_cast<const float2*>(xl), reinterpret_cast<float2*>(yl), d.nleaf, R, d.n, st);
        launch_recv_mfma(static_cast<const float2*>(d.V), reinterpret_cast<const float2*>(o + LL.s_off * R),
                         d.leaf_ptr, reinterpret_cast<float2*>(yl), d.nleaf, LL.Q, R, d.n, d.w, st);
      } else {
        k_near_multi<V2><<<dim3((unsigned)d.nleaf, rblk), NT, 0, st>>>(static_cast<const V2*>(d.Z), d.zoff,
                                                                      d.leaf_ptr, d.near_ptr, d.near_idx, xl, yl,
                                                                      R, d.n);
        k_recv_multi<T><<<dim3((unsigned)d.nleaf, rblk), NT, 0, st>>>(static_cast<const V2*>(d.V),
                                                                     o + LL.s_off * R, d.leaf_ptr, yl, LL.Q, R, d.n,
                                                                     (T)d.w[0], (T)d.w[1], (T)d.w[2], (T)d.w[3]);
      }
    }
  }
  if (tm) tm->mark(st, 5, L, overlap ? K_RECV : K_NEAR_RECV);
}

template <typename T>
void launch_gather(const void* x, void* xl, const int32_t* perm, int64_t n, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_gather<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(x), static_cast<V2*>(xl), perm, n);
}
template <typename T>
void launch_scatter(const void* yl, void* y, const int32_t* perm, int64_t n, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_scatter<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(yl), static_cast<V2*>(y), perm, n);
}

template <typename T>
void launch_multidot(const void* basis, int64_t ld, int nvec, const void* w, int64_t n, double2* partial,
                     int nblocks, double2* out, int accumulate, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_multidot<V2><<<nblocks, NT, 0, st>>>(static_cast<const V2*>(basis), ld, nvec, static_cast<const V2*>(w), n,
                                         partial);
  k_reduce_partials<<<nvec, NT, 0, st>>>(partial, nblocks, nvec, out, accumulate);
}
template <typename T>
void launch_combine(const void* basis, int64_t ld, int nvec, const double2* h, void* w, int64_t n, double sign,
                    hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_combine<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(basis), ld, nvec, h, static_cast<V2*>(w), n, sign);
}
template <typename T>
void launch_scale_norm(const void* x, void* y, int64_t n, const double2* nrm, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_scale_norm<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(x), static_cast<V2*>(y), n, nrm);
}
template <typename T>
void launch_scale(const void* x, void* y, int64_t n, double alpha, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_scale<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(x), static_cast<V2*>(y), n, alpha);
}
template <typename T>
void launch_sub(const void* a, const void* b, void* y, int64_t n, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_sub<V2><<<nblk(n), NT, 0, st>>>(static_cast<const V2*>(a), static_cast<const V2*>(b), static_cast<V2*>(y), n);
}
template <typename T>
void launch_near_apply(const DevOp<T>& d, const void* arena, const void* x, void* y, hipStream_t st, int nrhs) {
  using V2 = typename C2<T>::type;
  if (nrhs == 1) {
    k_near_full1<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(arena), d.zoff, d.leaf_ptr, d.near_ptr,
                                                      d.near_idx, static_cast<const V2*>(x), static_cast<V2*>(y));
    return;
  }
  const unsigned rblk = (unsigned)((nrhs + RB - 1) / RB);
  k_near_multi<V2><<<dim3((unsigned)d.nleaf, rblk), NT, 0, st>>>(static_cast<const V2*>(arena), d.zoff, d.leaf_ptr,
                                                                d.near_ptr, d.near_idx, static_cast<const V2*>(x),
                                                                static_cast<V2*>(y), nrhs, d.n);
}

void launch_fill_translation(const double* E, const int32_t* off, int nused, int Q, int Qr, double side, double k,
                             void* D, bool fp64, hipStream_t st) {
  const int64_t total = (int64_t)nused * Q * Qr;
  if (total == 0) return;
  const unsigned grid = (unsigned)((total + NT - 1) / NT);
  if (fp64)
    k_fill_translation<double2><<<grid, NT, 0, st>>>(E, off, side, k, Q, Qr, total, static_cast<double2*>(D));
  else
    k_fill_translation<float2><<<grid, NT, 0, st>>>(E, off, side, k, Q, Qr, total, static_cast<float2*>(D));
}

void launch_fill_radiation(const RadGeo& g, int64_t nleaf, void* V, bool fp64, hipStream_t st) {
  if (nleaf == 0) return;
  if (fp64)
    k_fill_radiation<double2><<<(unsigned)nleaf, NT, 0, st>>>(g, static_cast<double2*>(V));
  else
    k_fill_radiation<float2><<<(unsigned)nleaf, NT, 0, st>>>(g, static_cast<float2*>(V));
}

template <typename T>
void launch_blockdiag(const DevOp<T>& d, const void* r, void* z, hipStream_t st) {
  using V2 = typename C2<T>::type;
  k_blockdiag<T><<<(unsigned)d.nleaf, NT, 0, st>>>(static_cast<const V2*>(d.Minv), d.moff, d.leaf_ptr,
                                                   static_cast<const V2*>(r), static_cast<V2*>(z));
}

#define NESA_INST(T)                                                                                         \
  template void launch_matvec_leaf<T>(const DevOp<T>&, const void*, void*, int, hipStream_t, PhaseTimer*);    \
  template void launch_gather<T>(const void*, void*, const int32_t*, int64_t, hipStream_t);                  \
  template void launch_scatter<T>(const void*, void*, const int32_t*, int64_t, hipStream_t);                 \
  template void launch_multidot<T>(const void*, int64_t, int, const void*, int64_t, double2*, int, double2*, \
                                   int, hipStream_t);                                                        \
  template void launch_combine<T>(const void*, int64_t, int, const double2*, void*, int64_t, double,        \
                                  hipStream_t);                                                              \
  template void launch_scale<T>(const void*, void*, int64_t, double, hipStream_t);                           \
  template void launch_scale_norm<T>(const void*, void*, int64_t, const double2*, hipStream_t);              \
  template void launch_sub<T>(const void*, const void*, void*, int64_t, hipStream_t);                       \
  template void launch_blockdiag<T>(const DevOp<T>&, const void*, void*, hipStream_t);                      \
  template void launch_near_apply<T>(const DevOp<T>&, const void*, const void*, void*, hipStream_t, int);
NESA_INST(float)
NESA_INST(double)

}  // namespace nesa
