// Device-side operator layout and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace nesa {

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
  // translation as GEMMs grouped by offset (FP32 matrix cores): tiles of up to
  // TR_PAIRS pairs sharing one offset; results per pair, summed per target after
  int64_t ntiles = 0;
  int32_t* tile_slot = nullptr;  // [ntiles] compact offset slot
  int32_t* tile_start = nullptr; // [ntiles] first entry in pair_k
  int32_t* tile_count = nullptr; // [ntiles] pairs in the tile
  int32_t* pair_k = nullptr;     // [npairs] interaction-list positions grouped by slot
  void* pair_out = nullptr;      // [npairs][4][Q] D s_b of every pair
  int32_t* child_ptr = nullptr;  // [nbox + 1] children at level l+1
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
  void* Z = nullptr;             // near blocks
  void* V = nullptr;             // [n][4][Q_L]
  void* s = nullptr;             // equivalent sources, all levels
  void* o = nullptr;             // equivalent potentials, all levels
  void* Minv = nullptr;          // block-diagonal preconditioner (inverse self blocks)
  int64_t* moff = nullptr;
  double w[4] = {0, 0, 0, 0};    // channel weights: re/im of w_xyz, re/im of w_div
  std::vector<DevLevel> lev;
};

constexpr int TR_PAIRS = 16;   // pairs per translation tile (64 GEMM columns)

// hipEvent markers between the matvec phases
struct PhaseTimer {
  static constexpr int NMARK = 6;
  hipEvent_t ev[NMARK];
  void mark(hipStream_t st, int i) { (void)hipEventRecord(ev[i], st); }
};

template <typename T>
void launch_matvec_leaf(const DevOp<T>& d, const void* xl, void* yl, hipStream_t st, PhaseTimer* tm);
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
template <typename T>
void launch_sub(const void* a, const void* b, void* y, int64_t n, hipStream_t st);
template <typename T>
void launch_blockdiag(const DevOp<T>& d, const void* r, void* z, hipStream_t st);

}  // namespace nesa
