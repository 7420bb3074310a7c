// Host-side data structures of the NESA library: mesh, RWG basis, oct-tree,
// near-field blocks and far-field operators (all FP64, host memory).
#pragma once

#include <array>
#include <complex>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

namespace nesa {

using cd = std::complex<double>;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// RWG functions on the interior edges of a closed mesh (canonical order).
struct Rwg {
  int64_t n = 0, nt = 0;
  std::vector<double> v;            // [nv][3]
  std::vector<int32_t> t;           // [nt][3]
  std::vector<int64_t> edge;        // [n][2] (min, max) vertex ids
  std::vector<int64_t> tri;         // [n][2] (T+, T-)
  std::vector<int64_t> freev;       // [n][2] free vertex of T+, T-
  std::vector<double> len;          // [n]
  std::vector<double> area;         // [nt]
  std::vector<double> normal;       // [nt][3]
  std::vector<int64_t> tri_rwg;     // [nt][3] RWG on the edge opposite local vertex a
  std::vector<double> tri_sign;     // [nt][3] +1 (T+) / -1 (T-)
  std::vector<double> qp;           // [nt][3][3] quadrature points (3-point rule)
};

struct Level {
  int l = 0;
  double side = 0;
  int64_t nbox = 0;
  std::vector<std::array<int32_t, 3>> key;
  std::vector<int64_t> parent;      // box index at level l-1 (empty at l0; -1 for a body's top box)
  std::vector<int32_t> octant;      // position inside the parent (bit0 x, bit1 y, bit2 z)
  std::vector<int64_t> child_ptr;   // children at level l+1 start at child_ptr[b]
  std::vector<int64_t> child_end;   // ... and end at child_end[b] (= child_ptr[b+1] in one body;
                                    // in a forest other bodies' top boxes may follow)
  std::vector<int32_t> body;        // body of every box (forests of several meshes)
  std::vector<int64_t> il_ptr;      // interaction list (Sec. 3): CSR by target
  std::vector<int64_t> il_src;
  std::vector<int32_t> il_slot;     // offset slot of (target key - source key)
};

struct Tree {
  Rwg rwg;
  double leaf = 0.25;
  int L = 0, l0 = 0, buffer = 1;
  double lo[3] = {0, 0, 0};
  std::vector<Level> lev;           // lev[l - l0]
  std::vector<int64_t> perm;        // leaf-order position -> canonical RWG
  std::vector<int64_t> pos;         // canonical RWG -> leaf-order position
  std::vector<int64_t> leaf_ptr;    // RWGs of leaf b: positions [leaf_ptr[b], leaf_ptr[b+1])
  std::vector<int64_t> near_ptr, near_idx;   // leaf-level near lists
  // forest of several meshes: per-body grid origin and canonical RWG ranges
  // (empty for a single mesh); levels are aligned at the leaves
  std::vector<std::array<double, 3>> body_lo;
  std::vector<int64_t> body_rwg;    // [nbodies + 1]
  // offset slots of the translation tables: offsets in [-(W-1)/2, (W-1)/2] per
  // axis, W = max(4 buffer + 3, 2^(l0 + 1) - 1): the interaction lists below l0
  // reach 2 buffer + 1 boxes, the coarsest level's reach across its whole grid
  int slotw = 7;
  int slot_w() const { return slotw; }
  int nslot() const { return slot_w() * slot_w() * slot_w(); }
  const Level& level(int l) const { return lev[l - l0]; }
  Level& level(int l) { return lev[l - l0]; }
  std::array<double, 3> center(int l, int64_t b) const {
    const Level& lv = level(l);
    const double* o = body_lo.empty() ? lo : body_lo[lv.body[b]].data();
    return {o[0] + (lv.key[b][0] + 0.5) * lv.side, o[1] + (lv.key[b][1] + 0.5) * lv.side,
            o[2] + (lv.key[b][2] + 0.5) * lv.side};
  }
};

// Near-field blocks: for target leaf a, a dense S_a x W_a column-major block
// (W_a = sum of the sizes of the leaves in its near list, in list order).
struct Near {
  double k = 0, eta = 0;
  std::vector<int64_t> off;         // [nleaf + 1] offsets into z
  std::vector<cd> z;
  int64_t entries() const { return (int64_t)z.size(); }
};

struct FarLevel {
  int Q = 0, M = 0;
  double re = 0, rc = 0;
  std::vector<cd> E, X;             // [Q][3] on the complex radius re (1 + i eps), [M][3] on rc
  std::vector<cd> Cup;              // [8][Q_{l-1}][Q_l] row-major (l > l0)
  std::vector<uint8_t> slot_used;   // offset slots of the level's translations (D assembled on the device)
};

struct Far {
  double k = 0, eta = 0;
  int d0 = 3;
  double tau = 1e-8;
  double eps = 0.1;
  std::vector<FarLevel> lev;        // lev[l - l0]
  std::vector<cd> RLt;              // finest level's fitting operator R_L (Q_L x M), column-major
};

// thread pool helper: fn(i) for i in [0, n)
void parallel_for(int64_t n, const std::function<void(int64_t)>& fn);

Tree* build_tree(const double* verts, int64_t nv, const int32_t* tris, int64_t nt,
                 double leaf, int l0_max, int buffer);
// Several meshes in one tree structure: each body keeps its own grid, levels
// and lists; levels are aligned at the leaf level, boxes, RWGs and leaves are
// numbered body by body.
Tree* build_forest(int nbodies, const double* const* verts, const int64_t* nv, const int32_t* const* tris,
                   const int64_t* nt, double leaf, int l0_max, int buffer);
Near* assemble_near(const Tree& t, double k, double eta);
// the same blocks computed on the current device (FP64) and copied back
Near* assemble_near_device(const Tree& t, double k, double eta);
Far* assemble_far(const Tree& t, double k, double eta, int d0, int q_min, double tau, double eps);
// Transfer matrices of one pair of levels on the current device (FP64, Sec. 3,
// Eq. 11): cup[o][p][q] = sum_j R(p, j) g(X_j - delta_o - E_q) for the eight
// child octants o (delta_o = (+-a/2, +-a/2, +-a/2), a the child box side), R
// the parent's fitting operator column-major (Qp x Mp), X its Mp check points
// and E the child's Qc equivalent points ([n][3], complex); cup row-major
// [8][Qp][Qc].  Returns false, leaving cup untouched, when no device is present.
bool transfer_matrices_device(const std::vector<cd>& Rcm, int Qp, int Mp, const std::vector<cd>& X,
                              const std::vector<cd>& E, int Qc, double a, double k, std::vector<cd>& cup);
// Fitting operator of one level on the current device (FP64; Sec. 2 matches
// the equivalent sources to the field on a test surface, read here as the
// Tikhonov-regularised least-squares fit X = argmin ||G X - I_M||^2 +
// lam^2 ||X||^2), by Householder QR of [G; lam I]; G column-major (M x Q), X
// column-major (Q x M).  Returns false, leaving X untouched, when no device
// is present or Q exceeds 4096.
bool tikhonov_fit_device(const std::vector<cd>& G, int64_t M, int64_t Q, double lam, std::vector<cd>& X);
void plane_wave_rhs(const Tree& t, double k, const double* khat, const double* pol,
                    cd* b_canonical);
// Rows of the restricted near-field inverses (Schwarz preconditioner), in the
// layout of the near blocks; `single` computes the factorisations in FP32.
Near* near_schwarz(const Tree& t, const Near& near, bool single);

}  // namespace nesa
