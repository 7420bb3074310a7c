// Device state and launchers of the learned per-leaf preconditioner network:
// u (4 s_max) -> relu(W1 u + c1) (H) -> relu(W2 h1 + c2) (H) -> W3 h2 + c3
// (2 s_max), FP16 weights and activations on the matrix cores with FP32
// accumulation, FP32 master weights and Adam state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nesa {

struct MlpRows {
  int64_t rows = 0, rows_pad = 0;   // rows = samples x leaves, padded to 64
  _Float16* U = nullptr;            // [rows_pad][4S]
  _Float16* UT = nullptr;           // [4S][rows_pad] (training only)
  float* scale = nullptr;           // [rows_pad] ||base_a||
  float* Tg = nullptr;              // [rows_pad][2S] targets (training only)
  int32_t* rowS = nullptr;          // [rows_pad] valid entries per half, 0 = row masked
  _Float16 *h1 = nullptr, *h2 = nullptr;     // [rows_pad][H]
  _Float16 *h1T = nullptr, *h2T = nullptr;   // [H][rows_pad] (training only)
  float* Y = nullptr;               // [rows_pad][2S]
  _Float16 *dY = nullptr, *dYT = nullptr;    // [rows_pad][2S], [2S][rows_pad]
  _Float16 *dp2 = nullptr, *dp2T = nullptr, *dp1T = nullptr;
};

struct MlpDev {
  int S = 0, H = 0;
  int64_t np = 0;
  int64_t off[7] = {0, 0, 0, 0, 0, 0, 0};   // W1, c1, W2, c2, W3, c3 offsets in theta, end
  float* theta = nullptr;           // FP32 master parameters
  float *m = nullptr, *v = nullptr; // Adam moments
  float* grad = nullptr;            // [np]
  _Float16 *W1h = nullptr, *W2h = nullptr, *W3h = nullptr;   // row-major FP16 copies
  _Float16 *W2t = nullptr, *W3t = nullptr;                   // transposed FP16 copies
  float* partial = nullptr;         // split-K partial weight gradients
  int64_t partial_elems = 0;
  double* loss_part = nullptr;      // per-block loss partial sums
  int64_t loss_blocks = 0;
  double* loss = nullptr;           // [1]
};

inline int64_t mlp_nparams(int S, int H) {
  return (int64_t)H * 4 * S + H + (int64_t)H * H + H + (int64_t)2 * S * H + 2 * S;
}

// features (and, with e != nullptr, targets) of nsamples vectors in leaf order
template <typename T>
void launch_mlp_features(const MlpDev& net, MlpRows& R, const void* r, const void* b, const void* e,
                         const int32_t* leaf_ptr, int64_t nleaf, int64_t n, int64_t nsamples, bool transposed,
                         hipStream_t st);
// y = network(u) for the rows; training keeps the transposed activations
void launch_mlp_forward(const MlpDev& net, MlpRows& R, bool training, hipStream_t st);
// masked squared error -> net.loss (device, unnormalised sum) and dY = 2 (y - t)
void launch_mlp_loss(const MlpDev& net, MlpRows& R, hipStream_t st);
// gradient (scaled by inv_count) into net.grad
void launch_mlp_backward(const MlpDev& net, MlpRows& R, float inv_count, hipStream_t st);
void launch_mlp_adam(const MlpDev& net, float lr, float b1, float b2, float eps, int t, hipStream_t st);
void launch_mlp_refresh(const MlpDev& net, hipStream_t st);
// z (leaf order) += ||b_a|| (y_a[0:S_a] + i y_a[S:S+S_a]) for every leaf
template <typename T>
void launch_mlp_combine(const MlpDev& net, const MlpRows& R, const int32_t* leaf_ptr, int64_t nleaf, void* z,
                        hipStream_t st);
// number of split-K partial elements the backward pass needs for rows_pad rows
int64_t mlp_partial_elems(int S, int H, int64_t rows_pad);

}  // namespace nesa
