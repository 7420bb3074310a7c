// Target-major contractions for several right-hand sides: the translations
// (Sec. 3, Eq. 12), and with the same kernels the transfers (Eq. 11: targets =
// parents, pairs = children, matrix = C of the child's octant; Eq. 13: targets
// = children, one pair = the parent, matrix = C^T, added to the translated
// potentials).  For the translations:
// o_a = sum over b in IL(a) of D_{a-b} s_b, one workgroup per (target box a,
// tile of GEMM columns, block of rows).  With 4 nrhs channel columns per box
// (nrhs >= 8 gives 32 or more), the columns of one target already fill the
// matrix-core tiles, so the sum over the interaction list runs inside the
// accumulators: the pairs are consecutive K segments of one GEMM,
//   o_a[rows, cols] = [D_{a-b1} D_{a-b2} ...] [s_b1; s_b2; ...][K, cols],
// and every output is written once, in the list order, with no per-pair
// partial results.  (One right-hand side has only 4 columns per box; there the
// offset-major grouped GEMM of kernels.hip shares each D across many pairs.)
//
// FP32 form: complex products as three real 16x16x4 MFMAs (Ar Br, Ai Bi,
// (Ar + Ai)(Br + Bi)).  Split form: each FP32 value v = hi + lo with
// hi = bf16(v), lo = bf16(v - hi); a real product is hi hi + hi lo + lo hi on
// 16x16x32 bf16 MFMAs with FP32 accumulation, and the complex product takes
// the same three real products, i.e. nine bf16 MFMAs per complex k step.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "split16.h"

namespace nesa {

namespace {

constexpr int TM_NT = 256;
constexpr int TM_WAVE = 64;
constexpr int TM_KC = 32;     // K chunk staged in LDS
typedef float tm_f32x4 __attribute__((ext_vector_type(4)));

// Work item of a workgroup: items dealt to the 8 XCDs so that each XCD takes a
// contiguous range (neighbouring targets share sources and offsets in its L2).
__device__ __forceinline__ int64_t tm_item(int64_t bid, int64_t nitems) {
  const int64_t per = (nitems + 7) / 8;
  return (bid % 8) * per + bid / 8;
}

// NRT row tiles of 16 per workgroup, CT column tiles of 16 (CT = 4: wave w
// owns column tile w and all row tiles; CT = 2: wave w owns column tile w % 2
// and half of the row tiles).
template <int NRT, int CT>
__device__ __forceinline__ void translate_tm_body(const TmArgs& g) {
  constexpr int KC = TM_KC;
  constexpr int HALF = NRT * 8;                 // float4 per A column of the row block
  constexpr int NA = KC * HALF / TM_NT;         // float4 of A per thread per chunk
  constexpr int COLS = 16 * CT;
  constexpr int NBT = KC * COLS / TM_NT;        // float2 of B per thread per chunk
  constexpr int RPW = NRT * CT / 4;             // row tiles per wave
  static_assert(KC * HALF % TM_NT == 0 && KC * COLS % TM_NT == 0, "chunks must split evenly");
  static_assert(NRT * CT % 4 == 0, "row tiles must split over the waves");
  // LDS padding as in the offset-major kernel: the four k rows a wave reads at
  // once sit 32 banks apart, and neighbouring B columns fall in other banks
  constexpr int APAD = (NRT % 2 == 0) ? 4 : 0;
  constexpr int AST = 2 * (HALF + APAD);
  __shared__ float4 As4[KC][HALF + APAD];
  __shared__ float2 Bs[COLS][KC + 2];
  const int64_t nitems = g.nbox * g.nct;
  const int64_t item = tm_item(blockIdx.x, nitems);
  if (item >= nitems) return;
  const int64_t a = item / g.nct;
  const int c0 = (int)(item % g.nct) * COLS;
  const int ncol = min(COLS, g.NC - c0);         // valid columns of the tile
  const int r0 = blockIdx.y * NRT * 16;
  const int t = threadIdx.x, lane = t % TM_WAVE, w = t / TM_WAVE;
  const int ct = w % CT, rt0 = (w / CT) * RPW;
  const int K = g.K, M = g.M, NC = g.NC;
  const int mr2 = g.Mr / 2;
  const int kc0 = (K % KC) ? K % KC : KC;        // the partial chunk of every pair goes first
  const int nch = 1 + (K - kc0) / KC;            // chunks per pair
  const int jb = g.il_ptr[a], je = g.il_ptr[a + 1];
  const bool active = 16 * ct < ncol;
  // per-thread element offsets of a chunk (full chunks, and the partial chunk
  // with k clamped to its last step so that its loads stay inside the pair)
  int oa[NA], oap[NA], ob[NBT], obp[NBT];
  bool bok[NBT];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int e = t + i * TM_NT, k = e / HALF, rp = e % HALF;
    oa[i] = k * mr2 + rp;
    oap[i] = min(k, kc0 - 1) * mr2 + rp;
  }
#pragma unroll
  for (int i = 0; i < NBT; ++i) {
    const int e = t + i * TM_NT, col = e / KC, k = e % KC;
    const int cc = min(col, ncol - 1);
    ob[i] = cc * K + k;
    obp[i] = cc * K + min(k, kc0 - 1);
    bok[i] = col < ncol;
  }
  tm_f32x4 c1[RPW], c2[RPW], c3[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    c1[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
    c2[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
    c3[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float4 ra[NA];
  float2 rb[NBT];
  // chunk (pair j, chunk ci) into registers
  auto load = [&](int j, int ci) {
    const int slot = g.il_slot[j], src = g.il_src[j];
    const int kk = ci == 0 ? 0 : kc0 + (ci - 1) * KC;
    const float4* A4 = reinterpret_cast<const float4*>(g.D + (size_t)slot * g.a_stride + r0) + (size_t)kk * mr2;
    const float2* B = g.s + ((size_t)src * NC + c0) * K + kk;
    if (ci == 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) ra[i] = A4[oap[i]];
#pragma unroll
      for (int i = 0; i < NBT; ++i) rb[i] = B[obp[i]];
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) ra[i] = A4[oa[i]];
#pragma unroll
      for (int i = 0; i < NBT; ++i) rb[i] = B[ob[i]];
    }
  };
  // registers -> LDS; k past a partial chunk and empty columns become zeros
  auto stage = [&](int kc) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + i * TM_NT;
      As4[e / HALF][e % HALF] = (e / HALF < kc) ? ra[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      const int e = t + i * TM_NT;
      Bs[e / KC][e % KC] = (e % KC < kc && bok[i]) ? rb[i] : make_float2(0.f, 0.f);
    }
    __syncthreads();
  };
  const float2* As = reinterpret_cast<const float2*>(&As4[0][0]);
  auto step = [&](int ks) {
    const int kk = ks * 4 + lane / 16;
    const float2 b = Bs[ct * 16 + lane % 16][kk];
    const float bs = b.x + b.y;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const float2 av = As[kk * AST + (rt0 + r) * 16 + lane % 16];
      c1[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, b.x, c1[r], 0, 0, 0);
      c2[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, b.y, c2[r], 0, 0, 0);
      c3[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x + av.y, bs, c3[r], 0, 0, 0);
    }
  };
  if (jb < je) {
    load(jb, 0);
    for (int j = jb; j < je; ++j) {
      for (int ci = 0; ci < nch; ++ci) {
        const int kc = ci == 0 ? kc0 : KC;
        stage(kc);
        // the next chunk's loads stay in flight during this chunk's MFMAs
        if (ci + 1 < nch)
          load(j, ci + 1);
        else if (j + 1 < je)
          load(j + 1, 0);
        if (active) {
          if (kc == KC) {
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) step(ks);
          } else {
            for (int ks = 0; ks < (kc + 3) / 4; ++ks) step(ks);
          }
        }
      }
    }
  }
  // output through LDS ([column][row], row stride ROWS + 2), then runs of
  // consecutive rows of each column: o[a][c0 + col][r0 + row]
  constexpr int ROWS = NRT * 16;
  constexpr int RS = ROWS + 2;
  constexpr int ACAP = KC * (HALF + APAD) * 2;  // float2 in As4
  constexpr int PC = (ACAP / RS) >= COLS ? COLS : (ACAP / RS) / 16 * 16;
  static_assert(PC >= 16, "the LDS tile must hold one column tile");
  float2* otile = reinterpret_cast<float2*>(&As4[0][0]);
  const int mloc = min(ROWS, M - r0);
  float2* obase = g.o + ((size_t)a * NC + c0) * M + r0;
  for (int p0 = 0; p0 < COLS; p0 += PC) {
    __syncthreads();
    if (ct * 16 >= p0 && ct * 16 < p0 + PC) {
      const int lc = ct * 16 - p0 + lane % 16;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          otile[lc * RS + (rt0 + r) * 16 + 4 * (lane / 16) + i] =
              make_float2(c1[r][i] - c2[r][i], c3[r][i] - c1[r][i] - c2[r][i]);
      }
    }
    __syncthreads();
    const int nc = min(PC, ncol - p0);
    for (int e = t; e < nc * mloc; e += TM_NT) {
      const int lc = e / mloc, row = e % mloc;
      float2 v = otile[lc * RS + row];
      float2* out = obase + (size_t)(p0 + lc) * M + row;
      if (g.accumulate) {
        const float2 ov = *out;
        v.x += ov.x;
        v.y += ov.y;
      }
      *out = v;
    }
  }
}

template <int NRT, int CT>
__global__ __launch_bounds__(TM_NT) void k_translate_tm(TmArgs g) {
  translate_tm_body<NRT, CT>(g);
}


// Split form.  A (the translation matrices) arrives pre-split in six bf16
// planes [slot][plane][Mr][Kp] with k contiguous (Kp = K rounded up to 32,
// zero padded): re hi, re lo, im hi, im lo, (re + im) hi, (re + im) lo.  B (the
// FP32 sources) is split while it is staged: each thread takes 8 consecutive k
// of one column and writes them as 8 bf16 in each of six planes, which is the
// operand layout of the 16x16x32 instruction (lane l: row or column l % 16,
// k = 8 (l / 16) .. + 7).  Wave w owns column tile w and all row tiles.
// The 16-bit format F (split16.h) is bf16 or fp16; with fp16 the planes of A
// hold D x 2^a_exp, the sources are scaled by 2^split_shift(*bexp) before their
// split, and the results by 2^-(a_exp + shift).
typedef s16x8 tm_bf16x8;
__device__ __forceinline__ unsigned tm_pack(unsigned short a, unsigned short b) {
  return (unsigned)a | ((unsigned)b << 16);
}

template <int NRT, int F>
__device__ __forceinline__ void translate_tm_split_body(const TmArgs& g) {
  constexpr int KC = TM_KC;
  constexpr int ROWS = NRT * 16;
  constexpr int COLS = 64;
  constexpr int NAQ = 6 * ROWS * 4;               // uint4 of A per chunk (6 planes x rows x 4 quarters)
  constexpr int NAT = (NAQ + TM_NT - 1) / TM_NT;  // per thread
  static_assert(COLS * KC / 8 == TM_NT, "one column quarter of B per thread");
  // one LDS buffer: A planes [6][ROWS][5] and B planes [6][COLS][5] (uint4 of
  // 8 bf16; row stride 5 keeps a wave's 16-byte reads free of bank
  // conflicts), reused by the output tile at the end
  constexpr int AQ = 6 * ROWS * 5, BQ = 6 * COLS * 5;
  __shared__ uint4 lds[AQ + BQ];
  auto Al = [&](int pl, int row, int qu) -> uint4& { return lds[(pl * ROWS + row) * 5 + qu]; };
  auto Bl = [&](int pl, int col, int qu) -> uint4& { return lds[AQ + (pl * COLS + col) * 5 + qu]; };
  const int64_t nitems = g.nbox * g.nct;
  const int64_t item = tm_item(blockIdx.x, nitems);
  if (item >= nitems) return;
  const int64_t a = item / g.nct;
  const int c0 = (int)(item % g.nct) * COLS;
  const int ncol = min(COLS, g.NC - c0);
  const int r0 = blockIdx.y * ROWS;
  const int t = threadIdx.x, lane = t % TM_WAVE, w = t / TM_WAVE;
  const int K = g.K, M = g.M, NC = g.NC, Kp = g.Kp;
  const size_t plane = (size_t)g.Mr * Kp;
  const int nch = Kp / KC;
  const int jb = g.il_ptr[a], je = g.il_ptr[a + 1];
  const bool active = 16 * w < ncol;
  // A staging: element e = (plane, row, quarter) of the chunk
  int oa[NAT];
  bool aok[NAT];
#pragma unroll
  for (int i = 0; i < NAT; ++i) {
    const int e = t + i * TM_NT;
    aok[i] = e < NAQ;
    const int ee = aok[i] ? e : 0;
    const int pl = ee / (ROWS * 4), row = (ee / 4) % ROWS, qu = ee % 4;
    oa[i] = (int)(pl * plane / 8) + row * (Kp / 8) + qu;     // in uint4 (8 bf16)
  }
  // B staging: column t / 4 of the tile, quarter t % 4 (k = 8 (t % 4) .. + 7)
  const int bcol = t / 4, bq = t % 4;
  const bool bok = bcol < ncol;
  const int bcc = min(bcol, ncol - 1);
  tm_f32x4 c1[NRT], c2[NRT], c3[NRT];
#pragma unroll
  for (int r = 0; r < NRT; ++r) {
    c1[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
    c2[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
    c3[r] = tm_f32x4{0.f, 0.f, 0.f, 0.f};
  }
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // (see k_translate_tm_split2)
  u32x4 ra[NAT];
  float2 rb[8];
  auto load = [&](int j, int ci) {
    const int slot = g.il_slot[j], src = g.il_src[j];
    const int k0 = ci * KC;
    const u32x4* A = reinterpret_cast<const u32x4*>(g.Asplit + (size_t)slot * 6 * plane + (size_t)r0 * Kp + k0);
#pragma unroll
    for (int i = 0; i < NAT; ++i)
      if (aok[i]) ra[i] = A[oa[i]];
    const float2* B = g.s + ((size_t)src * NC + c0 + bcc) * K;
    const int kb = k0 + 8 * bq;
    if (k0 + KC <= K) {
#pragma unroll
      for (int u = 0; u < 8; ++u) rb[u] = B[kb + u];
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) rb[u] = B[min(kb + u, K - 1)];
    }
  };
  const int bshift = split_src_shift<F>(g.bexp);
  const int oexp = -(g.a_exp + bshift);
  auto stage = [&](int ci) {
    const int kv = K - ci * KC - 8 * bq;        // valid k of this thread's quarter
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NAT; ++i) {
      const int e = t + i * TM_NT;
      if (aok[i]) *reinterpret_cast<u32x4*>(&Al(e / (ROWS * 4), (e / 4) % ROWS, e % 4)) = ra[i];
    }
    unsigned short h[6][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      float2 v = rb[u];
      if (!(bok && u < kv)) v = make_float2(0.f, 0.f);
      if (F == SPLIT_FP16) v = make_float2(ldexpf(v.x, bshift), ldexpf(v.y, bshift));
      unsigned short hi, lo;
      split16<F>(v.x, hi, lo);
      h[0][u] = hi;
      h[1][u] = lo;
      split16<F>(v.y, hi, lo);
      h[2][u] = hi;
      h[3][u] = lo;
      split16<F>(v.x + v.y, hi, lo);
      h[4][u] = hi;
      h[5][u] = lo;
    }
#pragma unroll
    for (int pl = 0; pl < 6; ++pl)
      Bl(pl, bcol, bq) = make_uint4(tm_pack(h[pl][0], h[pl][1]), tm_pack(h[pl][2], h[pl][3]),
                                    tm_pack(h[pl][4], h[pl][5]), tm_pack(h[pl][6], h[pl][7]));
    __syncthreads();
  };
  auto mfma = [&]() {
    const int col = w * 16 + lane % 16, qu = lane / 16;
    const tm_bf16x8 brh = __builtin_bit_cast(tm_bf16x8, Bl(0, col, qu));
    const tm_bf16x8 brl = __builtin_bit_cast(tm_bf16x8, Bl(1, col, qu));
    const tm_bf16x8 bih = __builtin_bit_cast(tm_bf16x8, Bl(2, col, qu));
    const tm_bf16x8 bil = __builtin_bit_cast(tm_bf16x8, Bl(3, col, qu));
    const tm_bf16x8 bsh = __builtin_bit_cast(tm_bf16x8, Bl(4, col, qu));
    const tm_bf16x8 bsl = __builtin_bit_cast(tm_bf16x8, Bl(5, col, qu));
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
      const int row = r * 16 + lane % 16;
      const tm_bf16x8 arh = __builtin_bit_cast(tm_bf16x8, Al(0, row, qu));
      const tm_bf16x8 arl = __builtin_bit_cast(tm_bf16x8, Al(1, row, qu));
      const tm_bf16x8 aih = __builtin_bit_cast(tm_bf16x8, Al(2, row, qu));
      const tm_bf16x8 ail = __builtin_bit_cast(tm_bf16x8, Al(3, row, qu));
      const tm_bf16x8 ash = __builtin_bit_cast(tm_bf16x8, Al(4, row, qu));
      const tm_bf16x8 asl = __builtin_bit_cast(tm_bf16x8, Al(5, row, qu));
      c1[r] = mfma16x16x32<F>(arh, brh, c1[r]);
      c2[r] = mfma16x16x32<F>(aih, bih, c2[r]);
      c3[r] = mfma16x16x32<F>(ash, bsh, c3[r]);
      c1[r] = mfma16x16x32<F>(arh, brl, c1[r]);
      c2[r] = mfma16x16x32<F>(aih, bil, c2[r]);
      c3[r] = mfma16x16x32<F>(ash, bsl, c3[r]);
      c1[r] = mfma16x16x32<F>(arl, brh, c1[r]);
      c2[r] = mfma16x16x32<F>(ail, bih, c2[r]);
      c3[r] = mfma16x16x32<F>(asl, bsh, c3[r]);
    }
  };
  if (jb < je) {
    load(jb, 0);
    for (int j = jb; j < je; ++j) {
      for (int ci = 0; ci < nch; ++ci) {
        stage(ci);
        if (ci + 1 < nch)
          load(j, ci + 1);
        else if (j + 1 < je)
          load(j + 1, 0);
        if (active) mfma();
      }
    }
  }
  // output through LDS: o[a][c0 + col][r0 + row]
  constexpr int RS = ROWS + 2;
  static_assert((AQ + BQ) * 16 >= COLS * RS * 8, "LDS tile too small");
  float2* otile = reinterpret_cast<float2*>(&lds[0]);
  const int mloc = min(ROWS, M - r0);
  float2* obase = g.o + ((size_t)a * NC + c0) * M + r0;
  __syncthreads();
  {
    const int lc = w * 16 + lane % 16;
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        otile[lc * RS + r * 16 + 4 * (lane / 16) + i] =
            F == SPLIT_FP16 ? make_float2(ldexpf(c1[r][i] - c2[r][i], oexp),
                                          ldexpf(c3[r][i] - c1[r][i] - c2[r][i], oexp))
                            : make_float2(c1[r][i] - c2[r][i], c3[r][i] - c1[r][i] - c2[r][i]);
    }
  }
  __syncthreads();
  for (int e = t; e < ncol * mloc; e += TM_NT) {
    const int lc = e / mloc, row = e % mloc;
    float2 v = otile[lc * RS + row];
    float2* out = obase + (size_t)lc * M + row;
    if (g.accumulate) {
      const float2 ov = *out;
      v.x += ov.x;
      v.y += ov.y;
    }
    *out = v;
  }
}

template <int NRT, int F>
__global__ __launch_bounds__(TM_NT) void k_translate_tm_split(TmArgs g) {
  translate_tm_split_body<NRT, F>(g);
}

// ---------------------------------------------------------------------------
// Split form for 32 or more right-hand sides (NC >= 128 columns per box).
// These products move more bytes than the matrix cores can use (each source
// block serves one target's 64 rows per read), so the operands are kept at 8
// bytes per complex value: four bf16 planes (re hi, re lo, im hi, im lo) and
// complex products as four real ones (re = Ar Br - Ai Bi, im = Ar Bi + Ai Br),
// each hi hi + hi lo + lo hi: twelve MFMAs per k step.  The sources of a level
// are split once per product (k_split_sources) into s4[box][kc][plane][NC][16]
// (k chunks of 16), so that a workgroup stages them as plain copies; the
// products run on 32x32x16 bf16 MFMAs, each wave owning a 64 x 64 block (2 x 2
// tiles of 32 x 32) and the four waves side by side along the columns (a 64 x
// 256 workgroup tile).  A chunk of 16 k (both operands, four planes) is staged
// through registers into one of two LDS buffers while the MFMAs of the other
// buffer run: one barrier per chunk.  Operand layout of the instruction: lane l
// holds row (A) or column (B) l % 32 and k = 8 (l / 32) .. + 7; result value i
// of lane l is row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
typedef float tm_f32x16 __attribute__((ext_vector_type(16)));

template <int F>
__global__ __launch_bounds__(TM_NT) void k_split_sources(const float2* __restrict__ s, int64_t nbox, int NC, int K,
                                                         int Kp, uint4* __restrict__ s4, const int* __restrict__ bexp) {
  // one thread per (box, column, 8 consecutive k)
  const int per_box = NC * (Kp / 8);
  const int64_t i = (int64_t)blockIdx.x * TM_NT + threadIdx.x;
  if (i >= nbox * per_box) return;
  const int64_t box = i / per_box;
  const int r = (int)(i % per_box), c = r / (Kp / 8), k0 = 8 * (r % (Kp / 8));
  const float2* src = s + ((size_t)box * NC + c) * K;
  const int bshift = split_src_shift<F>(bexp);
  unsigned short h[4][8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    float2 v = (k0 + u < K) ? src[k0 + u] : make_float2(0.f, 0.f);
    if (F == SPLIT_FP16) v = make_float2(ldexpf(v.x, bshift), ldexpf(v.y, bshift));
    split16<F>(v.x, h[0][u], h[1][u]);
    split16<F>(v.y, h[2][u], h[3][u]);
  }
  const int kc = k0 / 16, half = (k0 % 16) / 8;
  uint4* dst = s4 + ((((size_t)box * (Kp / 16) + kc) * 4) * NC + c) * 2 + half;
#pragma unroll
  for (int pl = 0; pl < 4; ++pl)
    dst[(size_t)pl * NC * 2] = make_uint4(tm_pack(h[pl][0], h[pl][1]), tm_pack(h[pl][2], h[pl][3]),
                                          tm_pack(h[pl][4], h[pl][5]), tm_pack(h[pl][6], h[pl][7]));
}

__device__ __forceinline__ tm_bf16x8 tm_neg(tm_bf16x8 v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(tm_bf16x8, u);
}

template <int ROWS, int COLS, int F>
__global__ __launch_bounds__(TM_NT) __attribute__((amdgpu_waves_per_eu(2, COLS == 128 && ROWS == 64 ? 3 : 2))) void k_translate_tm_split2(TmArgs g) {
  constexpr int NP = 4;
  constexpr int WC = COLS / 4;                                 // columns per wave (64 or 32)
  constexpr int CTW = WC / 32;                                 // 32-column tiles per wave
  constexpr int RTW = ROWS / 32;                               // 32-row tiles per wave (every wave takes all rows)
  constexpr int AQ = NP * ROWS * 2, BQ = NP * COLS * 2;        // uint4 per buffer (8 bf16 each)
  constexpr int NAT = AQ / TM_NT, NBT = BQ / TM_NT;
  static_assert(AQ % TM_NT == 0 && BQ % TM_NT == 0, "staging must split evenly");
  static_assert(RTW * CTW <= 4, "at most four 32 x 32 accumulator tiles per wave");
  __shared__ uint4 lds[2 * (AQ + BQ)];
  const int64_t nitems = g.nbox * g.nct;
  // workgroup L (dispatch order) runs on XCD L % 8: each XCD takes a
  // contiguous eighth of the items, and the row blocks of an item one after
  // the other, so that they run side by side and read every source block of
  // the item once from the XCD's L2.  64 x 256 tiles: column tile major
  // (neighbouring targets of one column tile, whose sources overlap, follow each
  // other); 128 x 128 tiles: target major (the two column tiles of a target,
  // which read the same translation rows, follow each other)
  const int nrb = (int)gridDim.y;
  const int64_t lin = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  const int64_t per = (nitems + 7) / 8, seq = lin / 8;
  const int64_t item = (lin % 8) * per + seq / nrb;
  if (item >= nitems) return;
  const int64_t a = ROWS == 64 ? item % g.nbox : item / g.nct;
  const int c0 = (int)(ROWS == 64 ? item / g.nbox : item % g.nct) * COLS;
  const int ncol = min(COLS, g.NC - c0);
  const int r0 = (int)(seq % nrb) * ROWS;
  const int t = threadIdx.x, lane = t % TM_WAVE, w = t / TM_WAVE;
  const int NC = g.NC, M = g.M, Kp = g.Kp, KC = g.Kp / 16;
  const size_t plane = (size_t)g.Mr * Kp;
  const int jb = g.il_ptr[a], je = g.il_ptr[a + 1];
  const bool active = WC * w < ncol;
  // staging offsets (uint4 units): A element e = (plane, row, half), from the
  // pre-split matrix planes [slot][6][Mr][Kp] (planes 0-3); B element e =
  // (plane, column, half), from s4[box][kc][plane][NC][16]
  int oa[NAT], ob[NBT];
  bool bok[NBT];
#pragma unroll
  for (int i = 0; i < NAT; ++i) {
    const int e = t + i * TM_NT, pl = e / (ROWS * 2), row = (e / 2) % ROWS, hf = e % 2;
    oa[i] = (int)(pl * plane / 8) + row * (Kp / 8) + hf;
  }
#pragma unroll
  for (int i = 0; i < NBT; ++i) {
    const int e = t + i * TM_NT, pl = e / (COLS * 2), col = (e / 2) % COLS, hf = e % 2;
    bok[i] = col < ncol;
    ob[i] = (pl * NC + min(col, ncol - 1)) * 2 + hf;
  }
  tm_f32x16 cre[RTW][CTW], cim[RTW][CTW];
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int j = 0; j < CTW; ++j)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        cre[i][j][u] = 0.f;
        cim[i][j][u] = 0.f;
      }
  // staging registers as native vectors (copies of HIP's uint4 struct can
  // stay in private memory)
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 ra[NAT], rb[NBT];
  auto load = [&](int j, int kc) {
    const int slot = g.il_slot[j], src = g.il_src[j];
    const u32x4* A =
        reinterpret_cast<const u32x4*>(g.Asplit + (size_t)slot * 6 * plane + (size_t)r0 * Kp) + kc * 2;
    const u32x4* B = reinterpret_cast<const u32x4*>(g.s6) + (((size_t)src * KC + kc) * NP) * NC * 2 + (size_t)c0 * 2;
#pragma unroll
    for (int i = 0; i < NAT; ++i) ra[i] = A[oa[i]];
#pragma unroll
    for (int i = 0; i < NBT; ++i) rb[i] = B[ob[i]];
  };
  auto store = [&](int buf) {
    u32x4* Ab = reinterpret_cast<u32x4*>(lds) + buf * (AQ + BQ);
    u32x4* Bb = Ab + AQ;
#pragma unroll
    for (int i = 0; i < NAT; ++i) Ab[t + i * TM_NT] = ra[i];
#pragma unroll
    for (int i = 0; i < NBT; ++i) Bb[t + i * TM_NT] = bok[i] ? rb[i] : u32x4{0u, 0u, 0u, 0u};
  };
  auto mfma = [&](int buf) {
    const uint4* Ab = lds + buf * (AQ + BQ);
    const uint4* Bb = Ab + AQ;
    const int hf = lane / 32;
    tm_bf16x8 av[RTW][NP];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        av[rt][pl] = __builtin_bit_cast(tm_bf16x8, Ab[(pl * ROWS + rt * 32 + lane % 32) * 2 + hf]);
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
      tm_bf16x8 bv[NP];
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        bv[pl] = __builtin_bit_cast(tm_bf16x8, Bb[(pl * COLS + w * WC + ct * 32 + lane % 32) * 2 + hf]);
      const tm_bf16x8 nbih = tm_neg(bv[2]), nbil = tm_neg(bv[3]);
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) {
        // re += Ar Br - Ai Bi,  im += Ar Bi + Ai Br, each real product hi hi + hi lo + lo hi
        cre[rt][ct] = mfma32x32x16<F>(av[rt][0], bv[0], cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][0], bv[2], cim[rt][ct]);
        cre[rt][ct] = mfma32x32x16<F>(av[rt][0], bv[1], cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][0], bv[3], cim[rt][ct]);
        cre[rt][ct] = mfma32x32x16<F>(av[rt][1], bv[0], cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][1], bv[2], cim[rt][ct]);
        cre[rt][ct] = mfma32x32x16<F>(av[rt][2], nbih, cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][2], bv[0], cim[rt][ct]);
        cre[rt][ct] = mfma32x32x16<F>(av[rt][2], nbil, cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][2], bv[1], cim[rt][ct]);
        cre[rt][ct] = mfma32x32x16<F>(av[rt][3], nbih, cre[rt][ct]);
        cim[rt][ct] = mfma32x32x16<F>(av[rt][3], bv[0], cim[rt][ct]);
      }
    }
  };
  // chunks of 16 k over the pairs of the interaction list, in list order
  const int nchunk = (je - jb) * KC;
  if (nchunk > 0) {
    load(jb, 0);
    store(0);
    __syncthreads();
    for (int q = 0; q < nchunk; ++q) {
      const int buf = q & 1;
      const bool more = q + 1 < nchunk;
      if (more) load(jb + (q + 1) / KC, (q + 1) % KC);      // in flight during the MFMAs
      if (active) mfma(buf);
      if (more) store(buf ^ 1);                              // the other buffer: last read two chunks ago
      __syncthreads();
    }
  }
  // output through LDS in passes of PC columns ([column][row], stride ROWS + 2)
  constexpr int RS = ROWS + 2;
  constexpr int LB = 2 * (AQ + BQ) * 16;                                  // LDS bytes
  constexpr int PC = LB >= 128 * RS * 8 ? 128 : (LB >= 64 * RS * 8 ? 64 : 32);   // columns per output pass
  static_assert(LB >= PC * RS * 8 && PC >= WC, "LDS tile too small");
  float2* otile = reinterpret_cast<float2*>(&lds[0]);
  const int mloc = min(ROWS, M - r0);
  float2* obase = g.o + ((size_t)a * NC + c0) * M + r0;
  const int oexp = F == SPLIT_FP16 ? -(g.a_exp + split_shift(*g.bexp)) : 0;
  for (int p0 = 0; p0 < COLS; p0 += PC) {
    __syncthreads();
    if (w * WC >= p0 && w * WC < p0 + PC) {
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) {
          const int lc = w * WC - p0 + ct * 32 + lane % 32;
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int row = rt * 32 + 8 * (u / 4) + 4 * (lane / 32) + u % 4;
            otile[lc * RS + row] = F == SPLIT_FP16 ? make_float2(ldexpf(cre[rt][ct][u], oexp),
                                                                 ldexpf(cim[rt][ct][u], oexp))
                                                   : make_float2(cre[rt][ct][u], cim[rt][ct][u]);
          }
        }
    }
    __syncthreads();
    const int nc = min(PC, ncol - p0);
    for (int e = t; e < nc * mloc; e += TM_NT) {
      const int lc = e / mloc, row = e % mloc;
      float2 v = otile[lc * RS + row];
      float2* out = obase + (size_t)(p0 + lc) * M + row;
      if (g.accumulate) {
        const float2 ov = *out;
        v.x += ov.x;
        v.y += ov.y;
      }
      *out = v;
    }
  }
}

// Offset-major split products (groups = offset slots or octants, the pairs of a
// group sharing one matrix; up to 31 right-hand sides), with the operands of
// k_translate_tm_split2: A from the pre-split planes [g][6][Mr][Kp] (first
// four), B from the sources split once per level (s4[box][kc][plane][NC][16],
// k_split_sources), complex products as four real hi*hi + hi*lo + lo*hi
// products on 32x32x16 MFMAs.  A workgroup takes a tile of 128 (pair,
// channel) columns of one group (tile lists of width 128: col_src / col_dst
// hold the FP32 offsets (src NC + c) K and (dst NC + c) M of every column)
// and a block of ROWS rows; wave w owns columns 32 w .. 32 w + 31 and every
// row.  Chunks of 16 k are staged through registers into one of two LDS
// buffers while the MFMAs of the other run; the results leave through LDS in
// runs of consecutive rows of each column (one pair's NC columns are M
// contiguous rows each), written or added to the destination.
struct OmArgs {
  const unsigned short* Asplit;
  int Mr, Kp, M, K, NC;
  const uint4* s6;
  float2* dst;
  int accumulate;
  int64_t ntiles;
  const int32_t* tile_group;
  const int32_t* tile_ncols;
  const int64_t* col_src;
  const int64_t* col_dst;
  int a_exp;
  const int* bexp;
};

template <int ROWS, int F>
__global__ __launch_bounds__(TM_NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_om_split2(OmArgs g) {
  constexpr int NP = 4;
  constexpr int COLS = 128;                                    // 32 per wave
  constexpr int RTW = ROWS / 32;
  constexpr int AQ = NP * ROWS * 2, BQ = NP * COLS * 2;        // uint4 per buffer
  constexpr int NAT = AQ / TM_NT;
  static_assert(AQ % TM_NT == 0 && BQ == 4 * TM_NT, "staging must split evenly");
  __shared__ uint4 lds[2 * (AQ + BQ)];
  __shared__ int64_t cdst[COLS];
  const int nrb = (int)gridDim.y;
  const int64_t lin = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  const int64_t per = (g.ntiles + 7) / 8, seq = lin / 8;
  const int64_t tile = (lin % 8) * per + seq / nrb;
  if (tile >= g.ntiles) return;
  const int r0 = (int)(seq % nrb) * ROWS;
  const int t = threadIdx.x, lane = t % TM_WAVE, w = t / TM_WAVE;
  const int cnt = g.tile_ncols[tile];
  const int NC = g.NC, M = g.M, K = g.K, Kp = g.Kp, KC = g.Kp / 16;
  const size_t plane = (size_t)g.Mr * Kp;
  if (t < COLS) cdst[t] = g.col_dst[tile * COLS + t];
  const bool active = 32 * w < cnt;
  // A element e = t + i TM_NT of a chunk = (plane e / (2 ROWS), row
  // (e / 2) % ROWS, half e % 2): planes advance by TM_NT / (2 ROWS) per i, the
  // row and half are the thread's own; B: thread t takes column t / 2, half
  // t % 2 of every plane
  static_assert(TM_NT % (2 * ROWS) == 0, "A staging: whole planes per step");
  const int oa0 = (t / (2 * ROWS)) * (int)(plane / 8) + ((t / 2) % ROWS) * (Kp / 8) + t % 2;
  const int oastep = TM_NT / (2 * ROWS) * (int)(plane / 8);
  const int bcol = t / 2, bhf = t % 2;
  const bool bok = bcol < cnt;
  // (32-bit offsets in uint4: a level's split sources stay below 2^31 of
  // them, checked by the host)
  unsigned bbase;
  {
    const int64_t q = g.col_src[tile * COLS + min(bcol, cnt - 1)] / K;     // src NC + c
    const int64_t box = q / NC, c = q % NC;
    bbase = (unsigned)((box * KC * NP * NC + c) * 2 + bhf);
  }
  const unsigned bstep = (unsigned)(NP * NC * 2);                // uint4 per chunk of one box
  const uint4* A = reinterpret_cast<const uint4*>(g.Asplit + (size_t)g.tile_group[tile] * 6 * plane + (size_t)r0 * Kp);
  tm_f32x16 cre[RTW], cim[RTW];
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      cre[i][u] = 0.f;
      cim[i][u] = 0.f;
    }
  // staging registers as native vectors (HIP's uint4 struct copies kept them
  // in private memory)
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 ra[NAT], rb[NP];
  const u32x4* A4 = reinterpret_cast<const u32x4*>(A);
  const u32x4* S4 = reinterpret_cast<const u32x4*>(g.s6);
  u32x4* L4 = reinterpret_cast<u32x4*>(lds);
  auto load = [&](int kc) {
#pragma unroll
    for (int i = 0; i < NAT; ++i) ra[i] = (A4 + kc * 2)[oa0 + i * oastep];
    const u32x4* B = S4 + (size_t)kc * bstep;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) rb[pl] = B[bbase + (unsigned)(pl * NC * 2)];
  };
  auto store = [&](int buf) {
    u32x4* Ab = L4 + buf * (AQ + BQ);
    u32x4* Bb = Ab + AQ;
#pragma unroll
    for (int i = 0; i < NAT; ++i) Ab[t + i * TM_NT] = ra[i];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) Bb[t + pl * TM_NT] = bok ? rb[pl] : u32x4{0u, 0u, 0u, 0u};
  };
  auto mfma = [&](int buf) {
    const uint4* Ab = lds + buf * (AQ + BQ);
    const uint4* Bb = Ab + AQ;
    const int hf = lane / 32;
    tm_bf16x8 av[RTW][NP];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
        av[rt][pl] = __builtin_bit_cast(tm_bf16x8, Ab[(pl * ROWS + rt * 32 + lane % 32) * 2 + hf]);
    tm_bf16x8 bv[NP];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
      bv[pl] = __builtin_bit_cast(tm_bf16x8, Bb[(pl * COLS + w * 32 + lane % 32) * 2 + hf]);
    const tm_bf16x8 nbih = tm_neg(bv[2]), nbil = tm_neg(bv[3]);
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
      // re += Ar Br - Ai Bi,  im += Ar Bi + Ai Br, each real product hi hi + hi lo + lo hi
      cre[rt] = mfma32x32x16<F>(av[rt][0], bv[0], cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][0], bv[2], cim[rt]);
      cre[rt] = mfma32x32x16<F>(av[rt][0], bv[1], cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][0], bv[3], cim[rt]);
      cre[rt] = mfma32x32x16<F>(av[rt][1], bv[0], cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][1], bv[2], cim[rt]);
      cre[rt] = mfma32x32x16<F>(av[rt][2], nbih, cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][2], bv[0], cim[rt]);
      cre[rt] = mfma32x32x16<F>(av[rt][2], nbil, cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][2], bv[1], cim[rt]);
      cre[rt] = mfma32x32x16<F>(av[rt][3], nbih, cre[rt]);
      cim[rt] = mfma32x32x16<F>(av[rt][3], bv[0], cim[rt]);
    }
  };
  load(0);
  store(0);
  __syncthreads();
  for (int kc = 0; kc < KC; ++kc) {
    const int buf = kc & 1;
    const bool more = kc + 1 < KC;
    if (more) load(kc + 1);                                  // in flight during the MFMAs
    if (active) mfma(buf);
    if (more) store(buf ^ 1);                                // the other buffer: last read two chunks ago
    __syncthreads();
  }
  // output through LDS in passes of PC columns ([column][row], stride ROWS + 2)
  constexpr int RS = ROWS + 2;
  constexpr int LB = 2 * (AQ + BQ) * 16;
  constexpr int PC = LB >= 64 * RS * 8 ? 64 : 32;
  static_assert(LB >= PC * RS * 8, "LDS tile too small");
  float2* otile = reinterpret_cast<float2*>(&lds[0]);
  const int mloc = min(ROWS, M - r0);
  const int oexp = F == SPLIT_FP16 ? -(g.a_exp + split_shift(*g.bexp)) : 0;
  for (int p0 = 0; p0 < COLS; p0 += PC) {
    __syncthreads();
    if (w * 32 >= p0 && w * 32 < p0 + PC) {
      const int lc = w * 32 - p0 + lane % 32;
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int row = rt * 32 + 8 * (u / 4) + 4 * (lane / 32) + u % 4;
          otile[lc * RS + row] = F == SPLIT_FP16 ? make_float2(ldexpf(cre[rt][u], oexp), ldexpf(cim[rt][u], oexp))
                                                 : make_float2(cre[rt][u], cim[rt][u]);
        }
    }
    __syncthreads();
    const int nc = min(PC, cnt - p0);
    for (int e = t; e < nc * mloc; e += TM_NT) {
      const int lc = e / mloc, row = e % mloc;
      float2 v = otile[lc * RS + row];
      float2* out = g.dst + cdst[p0 + lc] + r0 + row;
      if (g.accumulate) {
        const float2 ov = *out;
        v.x += ov.x;
        v.y += ov.y;
      }
      *out = v;
    }
  }
}

// Largest binary exponent of a set of values (fp16 operand scale): a
// grid-stride loop keeps the maximum of frexp's exponent over the nonzero
// values, the workgroup reduces it, and one atomic maximum per workgroup
// updates the slot (integer maxima: the result does not depend on their
// order; few workgroups, since atomics on one address serialize).
template <typename R>
__global__ __launch_bounds__(TM_NT) void k_absmax_exp(const R* __restrict__ v, int64_t n, int* __restrict__ slot) {
  __shared__ int red[TM_NT / TM_WAVE];
  int e = EXP_NONE;
  for (int64_t i = (int64_t)blockIdx.x * TM_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * TM_NT) {
    const R x = v[i];
    if (x != R(0)) {
      int ex;
      frexp(x, &ex);
      e = max(e, ex);
    }
  }
#pragma unroll
  for (int o = TM_WAVE / 2; o > 0; o /= 2) e = max(e, __shfl_xor(e, o));
  if (threadIdx.x % TM_WAVE == 0) red[threadIdx.x / TM_WAVE] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < TM_NT / TM_WAVE; ++w) e = max(e, red[w]);
    if (e > EXP_NONE) atomicMax(slot, e);
  }
}

__global__ void k_exp_reset(int* __restrict__ slots, int n) {
  const int i = blockIdx.x * TM_NT + threadIdx.x;
  if (i < n) slots[i] = EXP_NONE;
}

// Device form of the host split of a grouped GEMM's A: FP64 column-major
// [g][K][Mr] -> bf16 planes [g][6][Mr][Kp] (k contiguous, zero for k >= K) and,
// when D32 is set, the FP32 copy [g][K][Mr].  One thread per (g, m, k < Kp).
template <int F>
__global__ void k_split_planes(const double2* __restrict__ D, int64_t total, int K, int Mr, int Kp,
                               float2* __restrict__ D32, unsigned short* __restrict__ P, int shift) {
  const int64_t i = (int64_t)blockIdx.x * TM_NT + threadIdx.x;
  if (i >= total) return;
  const int64_t per = (int64_t)Mr * Kp;
  const int64_t g = i / per;
  const int m = (int)((i / Kp) % Mr), k = (int)(i % Kp);
  double2 v = make_double2(0.0, 0.0);
  if (k < K) v = D[((size_t)g * K + k) * Mr + m];
  const float re = (float)v.x, im = (float)v.y;
  const float rs = F == SPLIT_FP16 ? ldexpf(re, shift) : re, is = F == SPLIT_FP16 ? ldexpf(im, shift) : im;
  unsigned short h[6];
  split16<F>(rs, h[0], h[1]);
  split16<F>(is, h[2], h[3]);
  split16<F>(rs + is, h[4], h[5]);
  unsigned short* o = P + (size_t)g * 6 * per + (size_t)m * Kp + k;
#pragma unroll
  for (int pl = 0; pl < 6; ++pl) o[pl * per] = h[pl];
  if (D32 && k < K) D32[((size_t)g * K + k) * Mr + m] = make_float2(re, im);
}

}  // namespace

void launch_split_planes(const void* D64, int64_t ngroups, int K, int Mr, int Kp, void* D32, void* planes, int fmt,
                         int shift, hipStream_t st) {
  const int64_t total = ngroups * Mr * (int64_t)Kp;
  if (total == 0) return;
  const unsigned nb = (unsigned)((total + TM_NT - 1) / TM_NT);
  if (fmt == SPLIT_FP16)
    k_split_planes<1><<<nb, TM_NT, 0, st>>>(static_cast<const double2*>(D64), total, K, Mr, Kp,
                                            static_cast<float2*>(D32), static_cast<unsigned short*>(planes), shift);
  else
    k_split_planes<0><<<nb, TM_NT, 0, st>>>(static_cast<const double2*>(D64), total, K, Mr, Kp,
                                            static_cast<float2*>(D32), static_cast<unsigned short*>(planes), 0);
}

void launch_absmax_exp(const void* v, int64_t n, bool fp64, int* slot, hipStream_t st) {
  if (n <= 0) return;
  const int64_t vals = 2 * n;
  // at least 16 values per thread, at most 64 workgroups (their atomics on
  // one address serialize: 512 of them took about 20 us)
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((vals + 16 * TM_NT - 1) / (16 * TM_NT), 64));
  if (fp64)
    k_absmax_exp<double><<<nb, TM_NT, 0, st>>>(static_cast<const double*>(v), vals, slot);
  else
    k_absmax_exp<float><<<nb, TM_NT, 0, st>>>(static_cast<const float*>(v), vals, slot);
}

void launch_exp_reset(int* slots, int n, hipStream_t st) {
  if (n <= 0) return;
  k_exp_reset<<<(unsigned)((n + TM_NT - 1) / TM_NT), TM_NT, 0, st>>>(slots, n);
}

// Row blocking of the target-major kernel: the fewest row tiles per workgroup
// (even when CT = 2) whose blocks stay inside the Mr allocated rows.
void tm_blocking(int M, int Mr, int NC, int& nrt, int& rblocks, int& ct) {
  ct = NC >= 64 ? 4 : 2;
  const int tiles = (M + 15) / 16;
  for (int blocks = 1;; ++blocks) {
    int n = (tiles + blocks - 1) / blocks;
    if (ct == 2 && n % 2) ++n;
    if (n <= 8 && blocks * n * 16 <= Mr) {
      nrt = n;
      rblocks = blocks;
      return;
    }
    if (blocks > tiles) break;
  }
  nrt = 0;
  rblocks = 0;
}

void launch_split_sources(const void* s, int64_t nbox, int NC, int K, int Kp, void* s6, int fmt, const int* bexp,
                          hipStream_t st) {
  const int64_t total = nbox * NC * (int64_t)(Kp / 8);
  if (total == 0) return;
  const unsigned nb = (unsigned)((total + TM_NT - 1) / TM_NT);
  if (fmt == SPLIT_FP16)
    k_split_sources<1><<<nb, TM_NT, 0, st>>>(static_cast<const float2*>(s), nbox, NC, K, Kp,
                                             static_cast<uint4*>(s6), bexp);
  else
    k_split_sources<0><<<nb, TM_NT, 0, st>>>(static_cast<const float2*>(s), nbox, NC, K, Kp,
                                             static_cast<uint4*>(s6), nullptr);
}

void launch_om_split2(const GemmPlan& p, const TileList& tl, int nrhs, const void* s6, void* dst, hipStream_t st) {
  if (tl.ntiles == 0) return;
  OmArgs g;
  g.Asplit = static_cast<const unsigned short*>(p.A_split);
  g.Mr = p.Mr;
  g.Kp = p.Kp;
  g.M = p.M;
  g.K = p.K;
  g.NC = 4 * nrhs;
  g.s6 = static_cast<const uint4*>(s6);
  g.dst = static_cast<float2*>(dst);
  g.accumulate = p.accumulate;
  g.ntiles = tl.ntiles;
  g.tile_group = tl.tile_group;
  g.tile_ncols = tl.tile_ncols;
  g.col_src = tl.col_src;
  g.col_dst = tl.col_dst;
  g.a_exp = p.a_exp;
  g.bexp = p.bexp;
  const bool h = p.split_fmt == SPLIT_FP16;
  const unsigned gx = (unsigned)((tl.ntiles + 7) / 8 * 8);
  if (p.M > 64) {
    const dim3 grid(gx, (unsigned)((p.M + 127) / 128));
    if (h)
      k_gemm_om_split2<128, 1><<<grid, TM_NT, 0, st>>>(g);
    else
      k_gemm_om_split2<128, 0><<<grid, TM_NT, 0, st>>>(g);
  } else {
    const dim3 grid(gx, 1);
    if (h)
      k_gemm_om_split2<64, 1><<<grid, TM_NT, 0, st>>>(g);
    else
      k_gemm_om_split2<64, 0><<<grid, TM_NT, 0, st>>>(g);
  }
}

void launch_translate_tm(const TmArgs& g, int nrt, int rblocks, int ct, hipStream_t st) {
  const int64_t nitems = g.nbox * g.nct;
  if (nitems == 0) return;
  if (g.Asplit && g.s6) {
    // 64 x 256, 64 x 128 or 128 x 128 workgroup tiles: nct counts the column
    // tiles; g.tm_rows = 128 selects the last
    const bool h = g.split_fmt == SPLIT_FP16;
    if (g.tm_rows == 128) {
      dim3 grid2((unsigned)((nitems + 7) / 8 * 8), (unsigned)((g.M + 127) / 128));
      if (h)
        k_translate_tm_split2<128, 128, 1><<<grid2, TM_NT, 0, st>>>(g);
      else
        k_translate_tm_split2<128, 128, 0><<<grid2, TM_NT, 0, st>>>(g);
      return;
    }
    dim3 grid2((unsigned)((nitems + 7) / 8 * 8), (unsigned)((g.M + 63) / 64));
    if (g.nct_cols == 128) {
      if (h)
        k_translate_tm_split2<64, 128, 1><<<grid2, TM_NT, 0, st>>>(g);
      else
        k_translate_tm_split2<64, 128, 0><<<grid2, TM_NT, 0, st>>>(g);
    } else if (h) {
      k_translate_tm_split2<64, 256, 1><<<grid2, TM_NT, 0, st>>>(g);
    } else {
      k_translate_tm_split2<64, 256, 0><<<grid2, TM_NT, 0, st>>>(g);
    }
    return;
  }
  dim3 grid((unsigned)((nitems + 7) / 8 * 8), (unsigned)rblocks);
  if (g.Asplit) {
#define NESA_TMS(N)                                        \
  case N:                                                  \
    if (g.split_fmt == SPLIT_FP16)                         \
      k_translate_tm_split<N, 1><<<grid, TM_NT, 0, st>>>(g); \
    else                                                   \
      k_translate_tm_split<N, 0><<<grid, TM_NT, 0, st>>>(g); \
    return;
    switch (nrt) {
      NESA_TMS(1) NESA_TMS(2) NESA_TMS(3) NESA_TMS(4) NESA_TMS(5) NESA_TMS(6) NESA_TMS(7) NESA_TMS(8)
      default: return;
    }
#undef NESA_TMS
  }
#define NESA_TM(N, C) \
  case N:             \
    k_translate_tm<N, C><<<grid, TM_NT, 0, st>>>(g); \
    return;
  if (ct == 4) {
    switch (nrt) {
      NESA_TM(1, 4) NESA_TM(2, 4) NESA_TM(3, 4) NESA_TM(4, 4) NESA_TM(5, 4) NESA_TM(6, 4) NESA_TM(7, 4)
      NESA_TM(8, 4)
      default: return;
    }
  } else {
    switch (nrt) {
      NESA_TM(2, 2) NESA_TM(4, 2) NESA_TM(6, 2) NESA_TM(8, 2)
      default: return;
    }
  }
#undef NESA_TM
}

}  // namespace nesa
