// gfx950 kernels of the learned per-leaf preconditioner network (inference
// inside flexible GMRES, and training: loss, backpropagation, Adam).
//
// All three layers are NT products C[M][N] = A[M][K] B[N][K]^T with FP16
// operands (K contiguous) on v_mfma_f32_16x16x32_f16 and FP32 accumulation;
// the epilogues fuse bias + ReLU, the ReLU derivative, and the transposed
// copies the weight gradients need.  Weight gradients reduce over all rows:
// split-K partial tiles, then an ordered sum (no atomics, bitwise repeatable).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mlp.h"

namespace nesa {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct MC2;
template <> struct MC2<float> { using type = float2; };
template <> struct MC2<double> { using type = double2; };

enum { EPI_RELU = 0, EPI_OUT = 1, EPI_BWD = 2, EPI_PART = 3 };

// Block tile 64 x 64 (four waves of 32 x 32, 2 x 2 MFMA tiles each); M, N
// multiples of 64, K and kchunk multiples of 32.
//   EPI_RELU: C16 = relu(acc + bias), CT16 (optional) its transpose [N][M]
//   EPI_OUT : C32 = acc + bias
//   EPI_BWD : C16 / CT16 (each optional) = acc where hm > 0, else 0
//   EPI_PART: C32[z][M][N] = acc over the z-th K chunk
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const _Float16* __restrict__ A, const _Float16* __restrict__ B,
                                                 int M, int N, int K, int kchunk, const float* __restrict__ bias,
                                                 const _Float16* __restrict__ hm, _Float16* __restrict__ C16,
                                                 _Float16* __restrict__ CT16, float* __restrict__ C32) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  if (m0 >= M || n0 >= N) return;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int r = lane & 15, kq = (lane >> 4) * 8;
  const _Float16* a0 = A + (int64_t)(m0 + r) * K + kq;
  const _Float16* a1 = a0 + (int64_t)16 * K;
  const _Float16* b0 = B + (int64_t)(n0 + r) * K + kq;
  const _Float16* b1 = b0 + (int64_t)16 * K;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k = kb; k < ke; k += 32) {
    const f16x8 x0 = *reinterpret_cast<const f16x8*>(a0 + k);
    const f16x8 x1 = *reinterpret_cast<const f16x8*>(a1 + k);
    const f16x8 y0 = *reinterpret_cast<const f16x8*>(b0 + k);
    const f16x8 y1 = *reinterpret_cast<const f16x8*>(b1 + k);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x0, y0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x0, y1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x1, y0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x1, y1, acc[1][1], 0, 0, 0);
  }
  // accumulator layout: lane holds column r, rows 4 (lane / 16) + q
  for (int tm = 0; tm < 2; ++tm)
    for (int tn = 0; tn < 2; ++tn) {
      const int col = n0 + tn * 16 + r;
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + tm * 16 + (lane >> 4) * 4 + q;
        float v = acc[tm][tn][q];
        const int64_t ix = (int64_t)row * N + col;
        if (EPI == EPI_RELU) {
          v = fmaxf(v + bias[col], 0.f);
          C16[ix] = (_Float16)v;
          if (CT16) CT16[(int64_t)col * M + row] = (_Float16)v;
        } else if (EPI == EPI_OUT) {
          C32[ix] = v + bias[col];
        } else if (EPI == EPI_BWD) {
          v = ((float)hm[ix] > 0.f) ? v : 0.f;
          if (C16) C16[ix] = (_Float16)v;
          if (CT16) CT16[(int64_t)col * M + row] = (_Float16)v;
        } else {
          C32[((int64_t)blockIdx.z * M + row) * N + col] = v;
        }
      }
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// one wave per row (sample s = row / nleaf, leaf a = row % nleaf)
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_features(const typename MC2<T>::type* __restrict__ r,
                                                      const typename MC2<T>::type* __restrict__ b,
                                                      const typename MC2<T>::type* __restrict__ e,
                                                      const int32_t* __restrict__ leaf_ptr, int64_t nleaf,
                                                      int64_t n, int64_t rows, int64_t rows_pad, int S,
                                                      _Float16* __restrict__ U, _Float16* __restrict__ UT,
                                                      float* __restrict__ scale, float* __restrict__ Tg,
                                                      int32_t* __restrict__ rowS) {
  using V2 = typename MC2<T>::type;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows_pad) return;
  int Sa = 0;
  const V2 *rr = r, *bb = b, *ee = e;
  if (row < rows) {
    const int64_t s = row / nleaf, a = row % nleaf;
    const int64_t p0 = leaf_ptr[a];
    Sa = leaf_ptr[a + 1] - leaf_ptr[a];
    rr = r + s * n + p0;
    bb = b + s * n + p0;
    if (e) ee = e + s * n + p0;
  }
  T nr2 = 0, nb2 = 0;
  for (int j = lane; j < Sa; j += 64) {
    const V2 x = rr[j], y = bb[j];
    nr2 += x.x * x.x + x.y * x.y;
    nb2 += y.x * y.x + y.y * y.y;
  }
  nr2 = wave_sum(nr2);
  nb2 = wave_sum(nb2);
  const T nr = sqrt(nr2), nb = sqrt(nb2);
  const T ir = nr > 0 ? T(1) / nr : T(0), ib = nb > 0 ? T(1) / nb : T(0);
  for (int j = lane; j < 4 * S; j += 64) {
    const int sec = j / S, jj = j - sec * S;
    float v = 0.f;
    if (jj < Sa) {
      const V2 x = sec < 2 ? rr[jj] : bb[jj];
      v = (float)(((sec & 1) ? x.y : x.x) * (sec < 2 ? ir : ib));
    }
    U[row * 4 * S + j] = (_Float16)v;
    if (UT) UT[(int64_t)j * rows_pad + row] = (_Float16)v;
  }
  if (lane == 0) {
    scale[row] = (float)nb;
    if (rowS) rowS[row] = nb > 0 ? Sa : 0;
  }
  if (Tg) {
    for (int j = lane; j < 2 * S; j += 64) {
      const int jj = j < S ? j : j - S;
      float v = 0.f;
      if (jj < Sa && nb > 0) {
        const V2 x = ee[jj], y = bb[jj];
        v = (float)((j < S ? x.x - y.x : x.y - y.y) * ib);
      }
      Tg[row * 2 * S + j] = v;
    }
  }
}

// masked squared error per 4-row block; dY = 2 (y - t) on valid entries
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ Tg,
                                                  const int32_t* __restrict__ rowS, int64_t rows_pad, int S,
                                                  _Float16* __restrict__ dY, _Float16* __restrict__ dYT,
                                                  double* __restrict__ part) {
  __shared__ double red[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  const int Sa = rowS[row];
  double acc = 0;
  for (int j = lane; j < 2 * S; j += 64) {
    const int jj = j < S ? j : j - S;
    const float d = jj < Sa ? Y[row * 2 * S + j] - Tg[row * 2 * S + j] : 0.f;
    acc += (double)d * d;
    const _Float16 g = (_Float16)(2.f * d);
    dY[row * 2 * S + j] = g;
    dYT[(int64_t)j * rows_pad + row] = g;
  }
  acc = wave_sum(acc);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// out = sum of n doubles in a fixed order (one workgroup)
__global__ __launch_bounds__(256) void k_sum_ordered(const double* __restrict__ in, int64_t n,
                                                     double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += in[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// g[i] = inv * sum_z P[z][i], z in order
__global__ __launch_bounds__(256) void k_reduce_splits(const float* __restrict__ P, int64_t mn, int nz, float inv,
                                                       float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= mn) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += P[(int64_t)z * mn + i];
  g[i] = inv * s;
}

// g[c] = inv * sum_m XT[c][m] (one workgroup per c, fixed order)
__global__ __launch_bounds__(256) void k_colsum(const _Float16* __restrict__ XT, int64_t rows_pad, float inv,
                                                float* __restrict__ g) {
  __shared__ float red[256];
  const _Float16* x = XT + (int64_t)blockIdx.x * rows_pad;
  float s = 0.f;
  for (int64_t m = threadIdx.x; m < rows_pad; m += 256) s += (float)x[m];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[blockIdx.x] = inv * red[0];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t np, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// FP16 copies of the weights: W1, W2, W3 row-major, W2^T and W3^T
__global__ __launch_bounds__(256) void k_refresh(const float* __restrict__ th, int S, int H, int64_t o1, int64_t o2,
                                                 int64_t o3, _Float16* __restrict__ W1h, _Float16* __restrict__ W2h,
                                                 _Float16* __restrict__ W3h, _Float16* __restrict__ W2t,
                                                 _Float16* __restrict__ W3t) {
  const int64_t n1 = (int64_t)H * 4 * S, n2 = (int64_t)H * H, n3 = (int64_t)2 * S * H;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n1) {
    W1h[i] = (_Float16)th[o1 + i];
  } else if (i < n1 + n2) {
    const int64_t j = i - n1, row = j / H, col = j % H;   // W2[row][col]
    const _Float16 w = (_Float16)th[o2 + j];
    W2h[j] = w;
    W2t[col * H + row] = w;
  } else if (i < n1 + n2 + n3) {
    const int64_t j = i - n1 - n2, row = j / H, col = j % H;   // W3[row][col], row < 2S
    const _Float16 w = (_Float16)th[o3 + j];
    W3h[j] = w;
    W3t[col * 2 * S + row] = w;
  }
}

// z_a += ||b_a|| (y_a[0:S_a] + i y_a[S:S+S_a]); one wave per leaf
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_combine(const float* __restrict__ Y, const float* __restrict__ scale,
                                                     const int32_t* __restrict__ leaf_ptr, int64_t nleaf, int S,
                                                     typename MC2<T>::type* __restrict__ z) {
  const int64_t a = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a >= nleaf) return;
  const int64_t p0 = leaf_ptr[a];
  const int Sa = leaf_ptr[a + 1] - leaf_ptr[a];
  const T sc = scale[a];
  for (int j = lane; j < Sa; j += 64) {
    z[p0 + j].x += sc * (T)Y[a * 2 * S + j];
    z[p0 + j].y += sc * (T)Y[a * 2 * S + S + j];
  }
}

// ------------------------------------------------------------------ launchers
static int split_chunk(int64_t K, int64_t tiles) {
  int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>(1024 / std::max<int64_t>(1, tiles), K / 32));
  int64_t chunk = (K + nsplit - 1) / nsplit;
  chunk = (chunk + 31) / 32 * 32;
  return (int)chunk;
}

int64_t mlp_partial_elems(int S, int H, int64_t rows_pad) {
  auto need = [&](int64_t M, int64_t N) {
    const int64_t chunk = split_chunk(rows_pad, (M / 64) * (N / 64));
    return ((rows_pad + chunk - 1) / chunk) * M * N;
  };
  return std::max(need(2 * S, H), std::max(need(H, H), need(H, 4 * S)));
}

template <int EPI>
static void gemm(const _Float16* A, const _Float16* B, int M, int N, int K, int kchunk, const float* bias,
                 const _Float16* hm, _Float16* C16, _Float16* CT16, float* C32, hipStream_t st) {
  const int nz = (K + kchunk - 1) / kchunk;
  dim3 grid((unsigned)(M / 64), (unsigned)(N / 64), (unsigned)nz);
  k_gemm_nt<EPI><<<grid, 256, 0, st>>>(A, B, M, N, K, kchunk, bias, hm, C16, CT16, C32);
}

template <typename T>
void launch_mlp_features(const MlpDev& net, MlpRows& R, const void* r, const void* b, const void* e,
                         const int32_t* leaf_ptr, int64_t nleaf, int64_t n, int64_t nsamples, bool transposed,
                         hipStream_t st) {
  using V2 = typename MC2<T>::type;
  (void)nsamples;
  k_mlp_features<T><<<(unsigned)(R.rows_pad / 4), 256, 0, st>>>(
      static_cast<const V2*>(r), static_cast<const V2*>(b), static_cast<const V2*>(e), leaf_ptr, nleaf, n, R.rows,
      R.rows_pad, net.S, R.U, transposed ? R.UT : nullptr, R.scale, e ? R.Tg : nullptr, R.rowS);
}

void launch_mlp_forward(const MlpDev& net, MlpRows& R, bool training, hipStream_t st) {
  const int S = net.S, H = net.H;
  const int M = (int)R.rows_pad;
  gemm<EPI_RELU>(R.U, net.W1h, M, H, 4 * S, 4 * S, net.theta + net.off[1], nullptr, R.h1, training ? R.h1T : nullptr,
                 nullptr, st);
  gemm<EPI_RELU>(R.h1, net.W2h, M, H, H, H, net.theta + net.off[3], nullptr, R.h2, training ? R.h2T : nullptr,
                 nullptr, st);
  gemm<EPI_OUT>(R.h2, net.W3h, M, 2 * S, H, H, net.theta + net.off[5], nullptr, nullptr, nullptr, R.Y, st);
}

void launch_mlp_loss(const MlpDev& net, MlpRows& R, hipStream_t st) {
  const int64_t nb = R.rows_pad / 4;
  k_mlp_loss<<<(unsigned)nb, 256, 0, st>>>(R.Y, R.Tg, R.rowS, R.rows_pad, net.S, R.dY, R.dYT, net.loss_part);
  k_sum_ordered<<<1, 256, 0, st>>>(net.loss_part, nb, net.loss);
}

void launch_mlp_backward(const MlpDev& net, MlpRows& R, float inv, hipStream_t st) {
  const int S = net.S, H = net.H;
  const int M = (int)R.rows_pad;
  // dp2 = (dY W3) o relu'(h2); dp1 = (dp2 W2) o relu'(h1)
  gemm<EPI_BWD>(R.dY, net.W3t, M, H, 2 * S, 2 * S, nullptr, R.h2, R.dp2, R.dp2T, nullptr, st);
  gemm<EPI_BWD>(R.dp2, net.W2t, M, H, H, H, nullptr, R.h1, nullptr, R.dp1T, nullptr, st);
  auto wgrad = [&](const _Float16* AT, const _Float16* BT, int Mo, int No, int64_t off_w, int64_t off_c) {
    const int chunk = split_chunk(M, (int64_t)(Mo / 64) * (No / 64));
    const int nz = (M + chunk - 1) / chunk;
    gemm<EPI_PART>(AT, BT, Mo, No, M, chunk, nullptr, nullptr, nullptr, nullptr, net.partial, st);
    const int64_t mn = (int64_t)Mo * No;
    k_reduce_splits<<<(unsigned)((mn + 255) / 256), 256, 0, st>>>(net.partial, mn, nz, inv, net.grad + off_w);
    k_colsum<<<(unsigned)Mo, 256, 0, st>>>(AT, M, inv, net.grad + off_c);
  };
  wgrad(R.dYT, R.h2T, 2 * S, H, net.off[4], net.off[5]);
  wgrad(R.dp2T, R.h1T, H, H, net.off[2], net.off[3]);
  wgrad(R.dp1T, R.UT, H, 4 * S, net.off[0], net.off[1]);
}

void launch_mlp_adam(const MlpDev& net, float lr, float b1, float b2, float eps, int t, hipStream_t st) {
  const float bc1 = (float)(1.0 - std::pow((double)b1, t)), bc2 = (float)(1.0 - std::pow((double)b2, t));
  k_adam<<<(unsigned)((net.np + 255) / 256), 256, 0, st>>>(net.theta, net.m, net.v, net.grad, net.np, lr, b1, b2,
                                                          eps, bc1, bc2);
}

void launch_mlp_refresh(const MlpDev& net, hipStream_t st) {
  const int S = net.S, H = net.H;
  const int64_t tot = (int64_t)H * 4 * S + (int64_t)H * H + (int64_t)2 * S * H;
  k_refresh<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(net.theta, S, H, net.off[0], net.off[2], net.off[4],
                                                          net.W1h, net.W2h, net.W3h, net.W2t, net.W3t);
}

template <typename T>
void launch_mlp_combine(const MlpDev& net, const MlpRows& R, const int32_t* leaf_ptr, int64_t nleaf, void* z,
                        hipStream_t st) {
  using V2 = typename MC2<T>::type;
  k_mlp_combine<T><<<(unsigned)((nleaf + 3) / 4), 256, 0, st>>>(R.Y, R.scale, leaf_ptr, nleaf, net.S,
                                                                 static_cast<V2*>(z));
}

template void launch_mlp_features<float>(const MlpDev&, MlpRows&, const void*, const void*, const void*,
                                         const int32_t*, int64_t, int64_t, int64_t, bool, hipStream_t);
template void launch_mlp_features<double>(const MlpDev&, MlpRows&, const void*, const void*, const void*,
                                          const int32_t*, int64_t, int64_t, int64_t, bool, hipStream_t);
template void launch_mlp_combine<float>(const MlpDev&, const MlpRows&, const int32_t*, int64_t, void*, hipStream_t);
template void launch_mlp_combine<double>(const MlpDev&, const MlpRows&, const int32_t*, int64_t, void*, hipStream_t);

}  // namespace nesa
