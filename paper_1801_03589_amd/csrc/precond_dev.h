// Restricted additive Schwarz preconditioner assembled on the device
// (precond_dev.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nesa {

// near leaves of one leaf at most (its 3 x 3 x 3 neighbourhood)
constexpr int SCHWARZ_MAXN = 27;

// largest near-list width W handled on the device
constexpr int SCHWARZ_WMAX = 4096;

// Per-leaf tables (device, indexed by leaf) and the work arrays.
// For leaf a with near list N(a) = nb[0 .. na): off[i] is the first RWG of
// nb[i] inside N(a) (off[na] = W), rowa the one of a itself, and colpos[j][i]
// (-1 when nb[i] is not near nb[j]) the first column, inside the reciprocity
// half block of leaf x = min(nb[i], nb[j]), of leaf y = max(nb[i], nb[j]) (the
// half block of x holds Z_xz for its near leaves z >= x, S_x rows, columns in
// near-list order from x's own).
struct SchwarzWork {
  int nleaf = 0;
  const int32_t* order = nullptr;   // [nleaf] leaves in the order they are taken (largest W first)
  int32_t* counter = nullptr;       // next entry of order to take (zero at launch)
  const int32_t* na = nullptr;      // [nleaf]
  const int32_t* W = nullptr;       // [nleaf]
  const int32_t* rowa = nullptr;    // [nleaf]
  const int32_t* nb = nullptr;      // [nleaf][27]
  const int32_t* off = nullptr;     // [nleaf][28]
  const int32_t* colpos = nullptr;  // [nleaf][27][27]
  float2* ws = nullptr;             // [slots][ws_stride]: W x W matrix of the leaf a workgroup works on
  int64_t ws_stride = 0;
  int32_t* piv = nullptr;           // [slots][piv_stride]
  int64_t piv_stride = 0;
  int32_t* status = nullptr;        // set to 1 when a pivot is zero (singular Z_N)
};

// Workgroups of the persistent setup kernel that fit the device at once.
int schwarz_slots();

// Builds, factors and solves every leaf with `slots` persistent workgroups
// (slots <= schwarz_slots(); workgroup g works in ws + g ws_stride), each
// taking leaves from the counter until none is left: out (the preconditioner's
// arena, the layout of the full near blocks: leaf a at zoff[a], S_a x W_a
// column-major) gets the rows of Z_N^-1 of every leaf.  Zh: the near blocks in
// reciprocity half storage (complex64, leaf x at zh_off[x]); leaf_ptr
// [nleaf + 1].  The counter is cleared on the stream first.
void launch_schwarz(const float2* Zh, const int64_t* zh_off, const int64_t* zoff, const int32_t* leaf_ptr,
                    const SchwarzWork& w, int slots, float2* out, hipStream_t st);

}  // namespace nesa
