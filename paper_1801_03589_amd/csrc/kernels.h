// Device-side operator layout and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace nesa {

// Tiles of a grouped complex GEMM on the matrix cores (see cgemm_tiles_body):
// C_pair = A_group x_src(pair) for every channel, written to dst(pair) or added
// to it.  Pairs are listed group by group; a tile is up to 64 consecutive
// (pair, channel) columns of one group, so the tiling depends on the number of
// right-hand sides (channels = 4 x nrhs) and is built per nrhs on first use.
struct TileList {
  int nrt = 0, rblocks = 0;       // row tiles per workgroup and row blocks chosen by the autotuner (0: plan default)
  int tpw = 0, kt = 0;            // resident-A kernel: tiles per workgroup and its K capacity (0: chunked kernel)
  int regions = 1;                // tiles ordered by (region, group) when 8: each XCD takes one region
  int width = 64;                 // columns per tile (64; 32 for the chunked kernel on groups with few pairs;
                                  // 128: split form on the pre-split sources, k_gemm_om_split2)
  int m3 = 0;                     // chunked kernel: complex products with three real MFMAs
  int64_t ntiles = 0;
  int32_t* tile_group = nullptr;
  int32_t* tile_ncols = nullptr;
  int64_t* col_src = nullptr;     // [ntiles][64] source offsets
  int64_t* col_dst = nullptr;     // [ntiles][64] destination offsets
};
// 16-bit formats of the split products: bf16 (8-bit mantissa, FP32 range) or
// fp16 (11-bit mantissa, 5-bit exponent; operands carry a power-of-two scale)
enum SplitFmt { SPLIT_BF16 = 0, SPLIT_FP16 = 1 };

struct GemmPlan {
  const void* A = nullptr;       // [groups][K][Mr] column-major, rows padded with zeros
  const void* A_split = nullptr; // split precision: [groups][6 planes][Mr][Kp] 16-bit (re hi, re lo, im hi, im lo,
                                 // (re + im) hi, (re + im) lo)
  int Kp = 0;                    // K rounded up to 32
  int split_fmt = SPLIT_BF16;    // format of A_split and of the split sources
  int a_exp = 0;                 // fp16: A_split holds A x 2^a_exp
  const int* bexp = nullptr;     // fp16: device slot of the sources' largest binary exponent (see k_absmax_exp)
  int64_t a_stride = 0;
  int M = 0, K = 0, Mr = 0;      // Mr = rows of A allocated (row_alloc), >= rblocks x nrt x 16
  int nrt = 1;                    // default row tiles of 16 per workgroup (1..8)
  int rblocks = 1;                // default row blocks (grid y)
  int accumulate = 0;
  int ngroups = 0;
  std::vector<int32_t> group_count;   // host: pairs per group
  std::vector<int32_t> h_src, h_dst;  // host: pairs, group by group (by source inside a group)
  std::vector<int8_t> h_region;       // host: region (1/8 of the Morton order of the owner box) of every pair
  std::vector<TileList> by_nrhs;  // index nrhs
  const void* s6 = nullptr;       // split form: the pre-split planes of the source level (TileList::width 128)
};

// One level of the far-field hierarchy on the device.
struct DevLevel {
  int Q = 0;
  int64_t nbox = 0;
  int64_t s_off = 0;          // offset of box 0 in the s / o arrays (complex elements)
  int64_t npairs = 0;
  void* Ccm = nullptr;        // [8][Q_{l-1}] column blocks: Ccm[o][q][p] = C_o[p][q] (l > l0)
  void* Crm = nullptr;        // Crm[o][p][q] = C_o[p][q]
  void* D = nullptr;          // [nused][Q][Q] column-major: D[slot][q][p] = D_slot[p][q]
  int32_t* il_ptr = nullptr;  // [nbox + 1]
  int32_t* il_src = nullptr;
  int32_t* il_slot = nullptr; // compact slot index
  GemmPlan trans;               // translation tiles (complex64): groups = offset slots
  void* pair_out = nullptr;     // [npairs][4][Q] D s_b of every pair
  void* s6 = nullptr;           // split form with many right-hand sides: pre-split sources (TmArgs::s6, four planes)
  int32_t* up_ptr = nullptr;    // target-major source transfer into level l-1: children of every
  int32_t* up_src = nullptr;    //   box of level l-1 (CSR over those boxes), octant of each child
  int32_t* up_slot = nullptr;
  int32_t* dn_ptr = nullptr;    // target-major potential transfer into this level: the parent of
  int32_t* dn_src = nullptr;    //   every box (CSR, none for a body's top box), its octant
  int32_t* dn_slot = nullptr;
  GemmPlan up;                  // this level's children -> parents (groups = octants)
  void* child_out = nullptr;    // [nbox][4][Q_{l-1}] C s_child of every child
  GemmPlan down;                // parents -> this level's boxes (groups = octants, accumulate)
  int32_t* child_ptr = nullptr;  // [nbox] first child at level l+1
  int32_t* child_end = nullptr;  // [nbox] end of the children
  int32_t* parent = nullptr;     // [nbox] (l > l0)
  int32_t* octant = nullptr;     // [nbox] (l > l0)
};

template <typename T>
struct DevOp {
  int64_t n = 0, nleaf = 0;
  int L = 0, l0 = 0;
  int32_t* perm = nullptr;       // leaf position -> canonical index
  int32_t* leaf_ptr = nullptr;   // [nleaf + 1]
  int32_t* near_ptr = nullptr;
  int32_t* near_idx = nullptr;
  int64_t* zoff = nullptr;       // [nleaf + 1]
  void* Z = nullptr;             // near blocks, full (products of several right-hand sides)
  // near blocks in reciprocity half storage (products of one right-hand side):
  // leaf a keeps the blocks Z_ab of the near leaves b >= a, itself first
  int32_t* nh_ptr = nullptr;     // [nleaf] near-list entry of the leaf itself
  int64_t* zh_off = nullptr;     // [nleaf + 1]
  void* Zh = nullptr;
  int32_t* toff = nullptr;       // [nleaf] first slot of leaf a's outputs Z_ab^T x_a (b > a)
  int32_t* tsrc = nullptr;       // [near entries] entry (a, b < a): slot of Z_ba^T x_b
  void* tpart = nullptr;         // those outputs
  void* V = nullptr;             // [n][4][Q_L]
  void* s = nullptr;             // equivalent sources, all levels
  void* o = nullptr;             // equivalent potentials, all levels
  void* Minv = nullptr;          // block-diagonal preconditioner (inverse self blocks)
  int64_t* moff = nullptr;
  int32_t* near_order = nullptr; // leaves by decreasing half-storage near-field work (launch order)
  hipStream_t side = nullptr;    // non-blocking stream of the near field (untimed products)
  int near_wgs = 0;              // workgroups of the persistent near-field grid (0: 256)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t side2 = nullptr;   // second side stream: the finest level's translations (untimed products)
  hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;
  int max_nrhs = 1;              // right-hand sides the work buffers hold
  int pair_cap = 1;              // offset-major up to this many right-hand sides, target-major above
  double w[4] = {0, 0, 0, 0};    // channel weights: re/im of w_xyz, re/im of w_div
  int split_fmt = SPLIT_BF16;    // split form: 16-bit format
  bool om2 = false;              // split form: the pre-split offset-major kernel is an autotuner candidate
  int* bexp = nullptr;           // fp16 split form: [2 x levels] largest exponents of s_l (2 (l - l0)) and o_l (+1)
  std::vector<DevLevel> lev;
};



// Row blocking of a GEMM with M rows: tiles of 16, at most 8 per workgroup,
// every block the same size; returns (nrt, padded rows).
inline void row_blocking(int M, int& nrt, int& Mr) {
  const int tiles = (M + 15) / 16;
  const int blocks = (tiles + 7) / 8;
  nrt = (tiles + blocks - 1) / blocks;
  Mr = blocks * nrt * 16;
}

// Rows allocated for A of a grouped GEMM with M rows: 16 x (row tiles rounded
// up to 8), which holds every blocking with 1..8 row tiles per workgroup the
// autotuner may pick except those that pad beyond it.
inline int row_alloc(int M) {
  const int tiles = (M + 15) / 16;
  return 16 * ((tiles + 7) / 8 * 8);
}

// Target-major translations (translate_tm.hip): o_a = sum over the
// interaction list of D_{a-b} s_b for the 4 nrhs channel columns of every box,
// one workgroup per (box, tile of up to 64 columns, row block).  FP32 three-MFMA
// complex products, or split bf16x3 products when Asplit is set.
struct TmArgs {
  const float2* D = nullptr;              // [slot][K][Mr] column-major (FP32 form)
  const unsigned short* Asplit = nullptr; // [slot][6][Mr][Kp] bf16 planes (split form)
  int64_t a_stride = 0;                   // K * Mr
  int M = 0, K = 0, Mr = 0, Kp = 0;
  const float2* s = nullptr;              // this level's sources [box][NC][K]
  float2* o = nullptr;                    // this level's potentials [box][NC][M] (overwritten)
  const int32_t* il_ptr = nullptr;        // [nbox + 1]
  const int32_t* il_src = nullptr;
  const int32_t* il_slot = nullptr;       // compact slot of every pair
  int64_t nbox = 0;
  int NC = 0;                             // 4 x nrhs
  int nct = 0;                            // column tiles per box
  int accumulate = 0;                     // o += result (potential transfer) instead of o = result
  int nct_cols = 256;                     // split form from TM2_MIN_COLS: columns per workgroup tile (256 or 128)
  const uint4* s6 = nullptr;              // split form, NC >= TM2_MIN_COLS: sources pre-split
                                          // [box][Kp/16][4][NC][16] bf16 (rows of 64, 256-column tiles)
  int tm_rows = 64;                       // split form with s6: 128 for 128 x 128 workgroup tiles
                                          // (nct_cols must then be 128)
  int split_fmt = SPLIT_BF16;             // split form: 16-bit format of Asplit and s6
  int a_exp = 0;                          // fp16: Asplit holds D x 2^a_exp
  const int* bexp = nullptr;              // fp16: slot of the sources' largest exponent E (scaled by 2^split_shift(E))
};
// fp16 operand scale: a set of values whose largest magnitude m lies below 2^E
// (E from frexp, or EXP_NONE when every value is zero) is multiplied by
// 2^split_shift(E), which puts m below 2^14 (and the sum of a real and an
// imaginary part below 2^15, inside fp16's range); clamped so that the factor
// and its inverse stay finite in FP32.
constexpr int EXP_NONE = -1000;
__host__ __device__ inline int split_shift(int E) {
  const int s = 14 - E;
  return s < -120 ? -120 : (s > 120 ? 120 : s);
}
// columns per box (4 nrhs) from which the split translations use the pre-split
// sources and 64 x 256 workgroup tiles
constexpr int TM2_MIN_COLS = 128;
// Offset-major split product of a grouped GEMM plan on the pre-split sources
// s6 of its source level (tile list of width 128): dst(pair) = A_group
// x_src(pair), written or added (p.accumulate).
void launch_om_split2(const GemmPlan& p, const TileList& tl, int nrhs, const void* s6, void* dst, hipStream_t st);
// s6 = four bf16 planes (re hi, re lo, im hi, im lo) of the sources s
// [nbox][NC][K] (layout of TmArgs::s6)
// (fp16: scaled by 2^split_shift(*bexp) first)
void launch_split_sources(const void* s, int64_t nbox, int NC, int K, int Kp, void* s6, int fmt, const int* bexp,
                          hipStream_t st);
// *slot = max(*slot, largest binary exponent E (frexp) over the nonzero real
// and imaginary parts of n complex values); slots start at EXP_NONE
// (launch_exp_reset).  The maximum does not depend on the order of the
// atomic updates.
void launch_absmax_exp(const void* v, int64_t n, bool fp64, int* slot, hipStream_t st);
void launch_exp_reset(int* slots, int n, hipStream_t st);
// Products of up to DevOp::pair_cap right-hand sides run the translations and
// transfers offset-major (grouped GEMMs sharing each matrix over many pairs,
// partial results per pair or child summed in a fixed order); more right-hand
// sides run them target-major (no partial results).  pair_cap is at most
// PAIR_CAP_MAX and limited by the bytes of the partial-result buffers.
constexpr int PAIR_CAP_MAX = 31;
constexpr double PAIR_BUFFER_BUDGET = 12.0 * (1 << 30);
// row tiles per workgroup, row blocks and column tiles of 16 (4 or 2) for M
// rows inside Mr allocated rows and NC columns; nrt = 0 if none fits
void tm_blocking(int M, int Mr, int NC, int& nrt, int& rblocks, int& ct);
void launch_translate_tm(const TmArgs& g, int nrt, int rblocks, int ct, hipStream_t st);
// Split planes of a grouped GEMM's A on the device (the host's rounding):
// complex128 [ngroups][K][Mr] -> bf16 [ngroups][6][Mr][Kp] (re hi, re lo, im
// hi, im lo, (re + im) hi, (re + im) lo; zero for k >= K) and, if D32 is not
// null, its complex64 copy [ngroups][K][Mr].
// fmt = SPLIT_FP16: the planes hold the fp16 split of A x 2^shift.
void launch_split_planes(const void* D64, int64_t ngroups, int K, int Mr, int Kp, void* D32, void* planes, int fmt,
                         int shift, hipStream_t st);

// Leaf-level stages of products of LEAF_MFMA_MIN_R or more right-hand sides
// (complex64) as per-leaf GEMMs on the FP32 matrix cores (leaf_mfma.hip): the
// near field y = Z_near x (full blocks, zoff layout; y overwritten), the
// radiation s_L = V^T x (s in the [box][4 R][Q] layout) and the reception
// y += V (w o_L); 64 right-hand sides per workgroup.  w: the channel weights
// (re, im of w_xyz, re, im of w_div).
constexpr int LEAF_MFMA_MIN_R = 16;
void launch_near_mfma(const float2* Z, const int64_t* zoff, const int32_t* leaf_ptr, const int32_t* near_ptr,
                      const int32_t* near_idx, const float2* x, float2* y, int64_t nleaf, int R, int64_t n,
                      hipStream_t st);
void launch_radiate_mfma(const float2* V, const float2* x, const int32_t* leaf_ptr, float2* s, int64_t nleaf, int Q,
                         int R, int64_t n, hipStream_t st);
void launch_recv_mfma(const float2* V, const float2* o, const int32_t* leaf_ptr, float2* y, int64_t nleaf, int Q,
                      int R, int64_t n, const double* w, hipStream_t st);

// kernel kinds of the per-launch timing
enum { K_RADIATE = 1, K_UP_GEMM, K_UP_REDUCE, K_UP_VALU, K_TRANS_GEMM, K_TRANS_REDUCE, K_TRANS_VALU,
       K_DOWN_GEMM, K_DOWN_VALU, K_NEAR_RECV, K_RECV };

// hipEvent markers between the matvec stages (phase >= 0) and after every
// launch (kind > 0); events are recorded on the launch stream.
struct PhaseTimer {
  static constexpr int NMARK = 6;
  static constexpr int MAXEV = 128;
  hipEvent_t ev[MAXEV];
  int phase_ev[NMARK];
  int kind[MAXEV], level[MAXEV];
  int n = 0;
  bool overlap = false;   // time the launches of the overlapped form (near field on the side stream, untimed)
  void mark(hipStream_t st, int phase, int lev, int k) {
    if (n >= MAXEV) return;
    (void)hipEventRecord(ev[n], st);
    if (phase >= 0) phase_ev[phase] = n;
    kind[n] = k;
    level[n] = lev;
    ++n;
  }
};

// y = Z_NESA x for nrhs right-hand sides in leaf order, RHS-major ([nrhs][n]).
// The complex64 path needs the GEMM tiles of this nrhs (TileList) built.
template <typename T>
void launch_matvec_leaf(const DevOp<T>& d, const void* xl, void* yl, int nrhs, hipStream_t st, PhaseTimer* tm);
template <typename T>
void launch_gather(const void* x, void* xl, const int32_t* perm, int64_t n, hipStream_t st);
template <typename T>
void launch_scatter(const void* yl, void* y, const int32_t* perm, int64_t n, hipStream_t st);
template <typename T>
void launch_multidot(const void* basis, int64_t ld, int nvec, const void* w, int64_t n, double2* partial,
                     int nblocks, double2* out, int accumulate, hipStream_t st);
template <typename T>
void launch_combine(const void* basis, int64_t ld, int nvec, const double2* h, void* w, int64_t n, double sign,
                    hipStream_t st);
template <typename T>
void launch_scale(const void* x, void* y, int64_t n, double alpha, hipStream_t st);
// y = x / sqrt(nrm->x) (nrm on the device; zero vector for a zero norm)
template <typename T>
void launch_scale_norm(const void* x, void* y, int64_t n, const double2* nrm, hipStream_t st);
template <typename T>
void launch_sub(const void* a, const void* b, void* y, int64_t n, hipStream_t st);
template <typename T>
void launch_blockdiag(const DevOp<T>& d, const void* r, void* z, hipStream_t st);
// D_u[p][q] = g(E_p + off_u side - E_q) for the nused offsets off [nused][3]
// (cells) and the level's equivalent points E [Q][3] complex (re, im pairs),
// column-major [u][q][Qr] with zero rows p >= Q; FP64 math, stored as complex128
// (fp64) or complex64.  All pointers are device pointers.
void launch_fill_translation(const double* E, const int32_t* off, int nused, int Q, int Qr, double side, double k,
                             void* D, bool fp64, hipStream_t st);
// Geometry of the radiation matrices (device pointers): RWGs in leaf order via
// perm, their triangles (T+, T-), free vertices, edge lengths; triangle areas and
// 3-point quadrature points [nt][3][3]; vertices [nv][3]; leaf centres
// [nleaf][3]; check points X [M][3] around the origin; R_L^T [M][Q].
struct RadGeo {
  const int32_t* perm = nullptr;
  const int32_t* leaf_ptr = nullptr;
  const int32_t* tri = nullptr;
  const int32_t* freev = nullptr;
  const double* len = nullptr;
  const double* area = nullptr;
  const double* qp = nullptr;
  const double* v = nullptr;
  const double* centre = nullptr;
  const double* X = nullptr;
  const double2* Rt = nullptr;
  double k = 0;
  int Q = 0, M = 0;
};
// V [n leaf order][4][Q] (complex128 if fp64, else complex64) on `st`.
void launch_fill_radiation(const RadGeo& g, int64_t nleaf, void* V, bool fp64, hipStream_t st);
// one grouped GEMM plan for nrhs right-hand sides (autotuner timing)
void launch_plan(const GemmPlan& p, int nrhs, const void* src, void* dst, hipStream_t st, bool translation);
// y = arena x with an arena in the near-block layout (leaf order, one RHS)
template <typename T>
void launch_near_apply(const DevOp<T>& d, const void* arena, const void* x, void* y, hipStream_t st, int nrhs = 1);

}  // namespace nesa
