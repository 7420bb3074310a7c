// C ABI of the NESA library (declared in include/nesa.h): handle management,
// device upload of the operators, the matvec driver and the GMRES driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/nesa.h"
#include "kernels.h"
#include "mlp.h"
#include "precond_dev.h"
#include "nesa_host.h"

using nesa::cd;
using nesa::Error;

struct nesa_tree {
  std::unique_ptr<nesa::Tree> t;
};
struct nesa_near {
  std::unique_ptr<nesa::Near> n;
};
struct nesa_far {
  std::unique_ptr<nesa::Far> f;
};

struct nesa_op {
  int precision = NESA_C64;
  const nesa::Tree* tree = nullptr;     // setup data for preconditioners built on demand
  const nesa::Near* near = nullptr;
  void* schwarz = nullptr;              // device arena of the Schwarz preconditioner (lazy)
  nesa_mlp* mlp = nullptr;              // network of NESA_PRECOND_LEARNED (not owned)
  std::vector<nesa_mlp*> nets;          // networks created for this op (detached when it is freed)
  int max_nrhs = 1;
  double k = 0, eta = 0;
  nesa::Tree geo;                       // copy of the RWG geometry (right-hand sides)
  nesa::DevOp<float> f;
  nesa::DevOp<double> d;
  std::vector<void*> allocs;
  void* xl = nullptr;                   // leaf-order work vectors
  void* yl = nullptr;
  size_t esize = 8;                     // bytes per complex element
  ~nesa_op();
};

static int64_t max_leaf(const nesa::Tree& t) {
  int64_t m = 0;
  for (size_t a = 0; a + 1 < t.leaf_ptr.size(); ++a) m = std::max(m, t.leaf_ptr[a + 1] - t.leaf_ptr[a]);
  return m;
}

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace nesa {
// error path shared with the 2D model module (sets nesa_last_error())
int report_failure(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace nesa

template <class F>
static int guarded(F&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(NESA_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(NESA_EINVAL, e.what());
  }
}

static void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Error(NESA_ENOMEM, std::string(what) + ": out of device memory");
    throw Error(NESA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

template <typename X>
static X* upload(nesa_op* op, const std::vector<X>& h) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(sizeof(X), h.size() * sizeof(X));
  hip_check(hipMalloc(&p, bytes), "hipMalloc");
  op->allocs.push_back(p);
  if (!h.empty()) hip_check(hipMemcpy(p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice), "hipMemcpy");
  return static_cast<X*>(p);
}

static void* dev_alloc(nesa_op* op, size_t bytes) {
  void* p = nullptr;
  hip_check(hipMalloc(&p, std::max<size_t>(bytes, 16)), "hipMalloc");
  op->allocs.push_back(p);
  return p;
}

template <typename T>
static void* upload_complex(nesa_op* op, const std::vector<cd>& h) {
  // conversion in chunks on the host's threads (near fields reach 10^9 entries)
  std::vector<T> buf(2 * h.size());
  constexpr int64_t CH = 1 << 20;
  const int64_t n = (int64_t)h.size();
  nesa::parallel_for((n + CH - 1) / CH, [&](int64_t c) {
    for (int64_t i = c * CH; i < std::min(n, (c + 1) * CH); ++i) {
      buf[2 * i] = (T)h[i].real();
      buf[2 * i + 1] = (T)h[i].imag();
    }
  });
  return upload(op, buf);
}

static std::vector<int32_t> to_i32(const std::vector<int64_t>& v) {
  std::vector<int32_t> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    if (v[i] > INT32_MAX || v[i] < INT32_MIN) throw Error(NESA_EINVAL, "index exceeds 32 bits");
    o[i] = (int32_t)v[i];
  }
  return o;
}

// Inverse of a dense complex matrix (column-major), Gauss-Jordan with partial pivoting.
static void invert(std::vector<cd>& A, int64_t S) {
  std::vector<cd> I(S * S, cd(0, 0));
  for (int64_t i = 0; i < S; ++i) I[i * S + i] = 1.0;
  for (int64_t c = 0; c < S; ++c) {
    int64_t piv = c;
    for (int64_t r = c + 1; r < S; ++r)
      if (std::abs(A[c * S + r]) > std::abs(A[c * S + piv])) piv = r;
    if (std::abs(A[c * S + piv]) == 0) throw Error(NESA_EINVAL, "singular near-field self block");
    if (piv != c)
      for (int64_t j = 0; j < S; ++j) {
        std::swap(A[j * S + c], A[j * S + piv]);
        std::swap(I[j * S + c], I[j * S + piv]);
      }
    cd inv = 1.0 / A[c * S + c];
    for (int64_t j = 0; j < S; ++j) {
      A[j * S + c] *= inv;
      I[j * S + c] *= inv;
    }
    for (int64_t r = 0; r < S; ++r) {
      if (r == c) continue;
      cd f = A[c * S + r];
      if (f == cd(0, 0)) continue;
      for (int64_t j = 0; j < S; ++j) {
        A[j * S + r] -= f * A[j * S + c];
        I[j * S + r] -= f * I[j * S + c];
      }
    }
  }
  A.swap(I);
}

// bf16 split planes of group matrices given column-major ([g][k][Mr]) on the host
static uint16_t bf16_rne_host(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
static float bf16_to_float(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}
static uint16_t f16_rne_host(float v) {
  const _Float16 h = (_Float16)v;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}
static float f16_to_float(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}
static bool is_split(int precision) { return precision == NESA_C64_SPLIT || precision == NESA_C64_SPLIT_FP16; }
static int split_fmt(int precision) {
  return precision == NESA_C64_SPLIT_FP16 ? nesa::SPLIT_FP16 : nesa::SPLIT_BF16;
}
// v = hi + lo in the 16-bit format (round to nearest even both times)
static void split_host(float v, int fmt, uint16_t& hi, uint16_t& lo) {
  if (fmt == nesa::SPLIT_FP16) {
    hi = f16_rne_host(v);
    lo = f16_rne_host(v - f16_to_float(hi));
  } else {
    hi = bf16_rne_host(v);
    lo = bf16_rne_host(v - bf16_to_float(hi));
  }
}
static void attach_split(nesa_op* op, nesa::GemmPlan& p, const std::vector<cd>& Acm, int ngroups, int fmt,
                         const int* bexp) {
  const int Kp = (p.K + 31) / 32 * 32;
  const size_t plane = (size_t)p.Mr * Kp;
  // fp16: one power-of-two scale for all groups (split_shift of the largest
  // exponent of the FP32 parts)
  int shift = 0;
  if (fmt == nesa::SPLIT_FP16) {
    int E = nesa::EXP_NONE;
    for (const cd& v : Acm)
      for (const float x : {(float)v.real(), (float)v.imag()})
        if (x != 0.f) {
          int ex;
          std::frexp(x, &ex);
          E = std::max(E, ex);
        }
    shift = nesa::split_shift(E);
  }
  std::vector<uint16_t> As((size_t)ngroups * 6 * plane, 0);
  nesa::parallel_for(ngroups, [&](int64_t gi) {
    for (int k = 0; k < p.K; ++k)
      for (int m = 0; m < p.Mr; ++m) {
        const cd v = Acm[((size_t)gi * p.K + k) * p.Mr + m];
        const float re = std::ldexp((float)v.real(), shift), im = std::ldexp((float)v.imag(), shift);
        const size_t base = (size_t)gi * 6 * plane + (size_t)m * Kp + k;
        split_host(re, fmt, As[base], As[base + plane]);
        split_host(im, fmt, As[base + 2 * plane], As[base + 3 * plane]);
        split_host(re + im, fmt, As[base + 4 * plane], As[base + 5 * plane]);
      }
  });
  p.A_split = upload(op, As);
  p.Kp = Kp;
  p.split_fmt = fmt;
  p.a_exp = shift;
  p.bexp = fmt == nesa::SPLIT_FP16 ? bexp : nullptr;
}

// Grouped pair lists of a GEMM plan (items in their given order inside a group);
// the tiles for a number of right-hand sides are made by build_tiles.
static nesa::GemmPlan make_plan(nesa_op* op, const void* A, int64_t a_stride, int M, int K, int Mr, int nrt,
                                int accumulate, const std::vector<int32_t>& group, int ngroups,
                                const std::vector<int32_t>& src, const std::vector<int32_t>& dst,
                                const std::vector<int8_t>& region) {
  nesa::GemmPlan p;
  p.A = A;
  p.a_stride = a_stride;
  p.M = M;
  p.K = K;
  p.Mr = Mr;
  p.nrt = nrt;
  p.rblocks = ((M + 15) / 16 + nrt - 1) / nrt;
  if (p.rblocks * nrt * 16 > Mr) throw Error(NESA_EINVAL, "row blocking exceeds the allocated rows");
  p.accumulate = accumulate;
  p.ngroups = ngroups;
  std::vector<std::vector<int32_t>> by(ngroups);
  for (size_t i = 0; i < group.size(); ++i) by[group[i]].push_back((int32_t)i);
  // inside a group, pairs ordered by source box (neighbouring tiles read
  // neighbouring source vectors)
  for (auto& v : by) std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) { return src[x] < src[y]; });
  std::vector<int32_t> ps, pd, gs(1, 0);
  std::vector<int8_t> pr;
  p.group_count.resize(ngroups);
  for (int u = 0; u < ngroups; ++u) {
    for (int32_t i : by[u]) {
      ps.push_back(src[i]);
      pd.push_back(dst[i]);
      pr.push_back(region[i]);
    }
    p.group_count[u] = (int32_t)by[u].size();
    gs.push_back((int32_t)ps.size());
  }
  p.h_src = ps;
  p.h_dst = pd;
  p.h_region = pr;
  p.by_nrhs.resize(op->max_nrhs + 1);
  return p;
}

// Tiles of up to 64 (pair, channel) columns of one group for nrhs right-hand
// sides, with the source / destination offset of every column precomputed.
static nesa::TileList build_tiles(nesa_op* op, const nesa::GemmPlan& p, int nrhs, int regions, int width) {
  nesa::TileList tl;
  const int NC = 4 * nrhs;
  std::vector<int32_t> tg, tn;
  std::vector<int64_t> cs, cdst;
  std::vector<int32_t> items;
  for (int reg = 0; reg < regions; ++reg) {
    int64_t pstart = 0;
    for (int u = 0; u < p.ngroups; ++u) {
      items.clear();
      for (int64_t i = pstart; i < pstart + p.group_count[u]; ++i)
        if (regions == 1 || p.h_region[i] == reg) items.push_back((int32_t)i);
      pstart += p.group_count[u];
      const int64_t ncols = (int64_t)items.size() * NC;
      for (int64_t c0 = 0; c0 < ncols; c0 += width) {
        const int64_t nc = std::min<int64_t>(width, ncols - c0);
        tg.push_back(u);
        tn.push_back((int32_t)nc);
        for (int j = 0; j < width; ++j) {
          const int64_t gc = c0 + std::min<int64_t>(j, nc - 1);
          const int64_t pi = items[gc / NC], c = gc % NC;
          cs.push_back(((int64_t)p.h_src[pi] * NC + c) * p.K);
          cdst.push_back(((int64_t)p.h_dst[pi] * NC + c) * p.M);
        }
      }
    }
  }
  tl.regions = regions;
  tl.width = width;
  tl.ntiles = (int64_t)tg.size();
  tl.tile_group = upload(op, tg);
  tl.tile_ncols = upload(op, tn);
  tl.col_src = upload(op, cs);
  tl.col_dst = upload(op, cdst);
  return tl;
}

// ------------------------------------------------------------------ autotuner
// The row blocking of every grouped GEMM (row tiles of 16 per workgroup,
// 1..8, and the row blocks that cover M) is picked by timing the candidates
// on the operator's own data the first time a plan runs for a number of
// right-hand sides.  Results do not depend on the choice (every output is
// one lane's sum in the same order).  Choices are kept per process, keyed by
// (kernel kind, precision, M, K, nrhs, tile count), and in the file named by
// NESA_TUNE_FILE when set; NESA_AUTOTUNE=0 keeps the default blocking.
struct TuneKey {
  int kind, split, M, K, nrhs;
  int64_t ntiles;
  bool operator<(const TuneKey& o) const {
    return std::tie(kind, split, M, K, nrhs, ntiles) < std::tie(o.kind, o.split, o.M, o.K, o.nrhs, o.ntiles);
  }
};
struct TuneChoice {
  int nrt, tpw, kt, regions, width, m3;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune;
static bool g_tune_loaded = false;

// NESA_AUTOTUNE: unset or "1" = all candidates, "0" = default blocking,
// "chunked" / "resident" / "direct" / "narrow" = only that kernel family
// (resident and direct where K <= 84, narrow = chunked with 32-column tiles
// where the row tiles split over the waves, gauss = chunked with three real
// MFMAs per complex product, presplit = split plans on the pre-split sources;
// else the plain chunked kernel)
static int autotune_mode() {
  const char* e = std::getenv("NESA_AUTOTUNE");
  if (!e) return 1;
  const std::string v(e);
  if (v == "0") return 0;
  if (v == "chunked") return 2;
  if (v == "resident") return 3;
  if (v == "direct") return 4;
  if (v == "narrow") return 5;
  if (v == "gauss") return 6;
  if (v == "presplit") return 7;
  return 1;
}

static void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* f = std::getenv("NESA_TUNE_FILE");
  if (!f) return;
  FILE* fp = std::fopen(f, "r");
  if (!fp) return;
  TuneKey k;
  long long nt;
  TuneChoice c;
  while (std::fscanf(fp, "%d %d %d %d %d %lld %d %d %d %d %d %d", &k.kind, &k.split, &k.M, &k.K, &k.nrhs, &nt,
                     &c.nrt, &c.tpw, &c.kt, &c.regions, &c.width, &c.m3) == 12) {
    k.ntiles = nt;
    if (c.nrt >= 1 && c.nrt <= 8 && (c.tpw <= 0 || c.kt == 52 || c.kt == 84) && (c.regions == 1 || c.regions == 8) &&
        (c.width == 32 || c.width == 64 || c.width == 128) && (c.m3 == 0 || c.m3 == 1))
      g_tune[k] = c;
  }
  std::fclose(fp);
}

static void tune_store_locked(const TuneKey& k, const TuneChoice& c) {
  g_tune[k] = c;
  const char* f = std::getenv("NESA_TUNE_FILE");
  if (!f) return;
  FILE* fp = std::fopen(f, "a");
  if (!fp) return;
  std::fprintf(fp, "%d %d %d %d %d %lld %d %d %d %d %d %d\n", k.kind, k.split, k.M, k.K, k.nrhs, (long long)k.ntiles,
               c.nrt, c.tpw, c.kt, c.regions, c.width, c.m3);
  std::fclose(fp);
}

// a choice is valid when its row blocks stay inside the allocated rows of A and
// (resident kernel) K fits its LDS capacity
// (tpw > 0: resident kernel; tpw = -13 / -21: direct kernel with that many k steps)
static bool set_blocking(nesa::GemmPlan& p, nesa::TileList& tl, const TuneChoice& c) {
  const int blocks = ((p.M + 15) / 16 + c.nrt - 1) / c.nrt;
  if (c.nrt < 1 || c.nrt > 8 || blocks * c.nrt * 16 > p.Mr) return false;
  // width 128: the split kernel on the pre-split sources (its own row blocks
  // of 64 or 128 rows)
  if (c.width == 128 && (!p.A_split || !p.s6 || c.tpw != 0 || c.m3 || c.nrt != (p.M > 64 ? 8 : 4))) return false;
  if (c.tpw > 0 && (p.A_split || (c.kt != 52 && c.kt != 84) || p.K > c.kt)) return false;
  if (c.tpw < 0 && (p.A_split || (c.tpw != -13 && c.tpw != -21) || p.K > -4 * c.tpw ||
                    (c.nrt != 1 && c.nrt != 2 && c.nrt != 4)))
    return false;
  if (c.width != (tl.width) || (c.width == 32 && (c.tpw != 0 || c.nrt % 2 || (p.A_split && c.m3)))) return false;
  if (c.m3 && (c.tpw != 0 || p.A_split)) return false;
  tl.nrt = c.nrt;
  tl.m3 = c.m3;
  tl.rblocks = blocks;
  tl.tpw = c.tpw;
  tl.kt = c.tpw > 0 ? c.kt : 0;
  return true;
}

// tile lists of both orderings are built on demand and kept per plan
static nesa::TileList& tiles_for(nesa_op* op, nesa::GemmPlan& p, int nrhs, int regions, int width,
                                 std::vector<nesa::TileList>& made) {
  for (auto& t : made)
    if (t.regions == regions && t.width == width) return t;
  made.push_back(build_tiles(op, p, nrhs, regions, width));
  return made.back();
}

static void tune_plan(nesa_op* op, nesa::GemmPlan& p, int nrhs, const void* src, void* dst, bool translation,
                      hipStream_t st) {
  nesa::TileList& out = p.by_nrhs[nrhs];
  if (out.tile_group) return;
  std::vector<nesa::TileList> made;
  made.reserve(4);
  const int mode = autotune_mode();
  const TuneChoice dflt{p.nrt, 0, 0, 1, 64, 0};
  if (mode == 0) {
    out = tiles_for(op, p, nrhs, 1, 64, made);
    set_blocking(p, out, dflt);
    return;
  }
  const int64_t base_tiles = tiles_for(op, p, nrhs, 1, 64, made).ntiles;
  if (base_tiles == 0) {
    out = made[0];
    return;
  }
  const bool res_ok = !p.A_split && p.K <= 84;
  // region ordering only pays when a group has many pairs per region
  const bool reg_ok = p.ngroups > 0 && (int64_t)p.h_src.size() / p.ngroups >= 64;
  // (split plans of either 16-bit format, with and without the pre-split
  // candidate, keep separate choices)
  const TuneKey key{(translation ? 1 : (p.accumulate ? 3 : 2)) + 10 * mode,
                    p.A_split ? 1 + (p.s6 ? 1 : 0) + 2 * p.split_fmt : 0, p.M, p.K, nrhs, base_tiles};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && (it->second.regions == 1 || reg_ok)) {
      nesa::TileList tl = tiles_for(op, p, nrhs, it->second.regions, it->second.width, made);
      if (set_blocking(p, tl, it->second)) {
        out = tl;
        return;
      }
    }
  }
  // candidates: chunked kernel with 1..8 row tiles (one per distinct row-block
  // count), resident kernel with 1..8 row tiles and 4 or 16 tiles per
  // workgroup; tiles in plain group order, and by region of the owner box
  std::vector<TuneChoice> cand;
  const int tiles = (p.M + 15) / 16;
  // the fewest row tiles per workgroup for every distinct number of row blocks
  std::vector<int> nrts;
  for (int blocks = 1; blocks <= tiles; ++blocks) {
    const int nrt = (tiles + blocks - 1) / blocks;
    if (nrt <= 8 && (nrts.empty() || nrts.back() != nrt)) nrts.push_back(nrt);
  }
  for (int regions : {1, 8}) {
    if (regions == 8 && !reg_ok) continue;
    for (int nrt : nrts) {
      for (int m3 : {0, 1}) {
        bool use;
        if (m3)
          use = !p.A_split && (mode == 1 || mode == 6);
        else
          use = mode == 1 || mode == 2 || mode == 5 || ((mode == 3 || mode == 4) && !res_ok) ||
                (mode == 6 && p.A_split);
        if (!use) continue;
        if (mode != 5) cand.push_back({nrt, 0, 0, regions, 64, m3});
        if ((!p.A_split || !m3) && nrt % 2 == 0) cand.push_back({nrt, 0, 0, regions, 32, m3});
      }
      if (res_ok && (mode == 1 || mode == 3))
        for (int tpw : {4, 16}) cand.push_back({nrt, tpw, p.K <= 52 ? 52 : 84, regions, 64, 0});
    }
    if (res_ok && (mode == 1 || mode == 4))
      for (int nrt : {1, 2, 4})
        if (nrt <= tiles) cand.push_back({nrt, p.K <= 52 ? -13 : -21, 0, regions, 64, 0});
  }
  // split plans: the kernel on the sources split once per level (tiles of
  // 128 columns, both orderings)
  if (p.A_split && p.s6 && (mode == 1 || mode == 7))
    for (int regions : {1, 8})
      if (regions == 1 || reg_ok) cand.push_back({p.M > 64 ? 8 : 4, 0, 0, regions, 128, 0});
  if (cand.empty()) cand.push_back(dflt);
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  TuneChoice best = dflt;
  float best_ms = 1e30f;
  for (const TuneChoice& c : cand) {
    nesa::TileList tl = tiles_for(op, p, nrhs, c.regions, c.width, made);
    if (!set_blocking(p, tl, c)) continue;
    p.by_nrhs[nrhs] = tl;
    nesa::launch_plan(p, nrhs, src, dst, st, translation);     // warm-up
    hip_check(hipEventRecord(e0, st), "hipEventRecord");
    for (int r = 0; r < 3; ++r) nesa::launch_plan(p, nrhs, src, dst, st, translation);
    hip_check(hipEventRecord(e1, st), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (const char* lf = std::getenv("NESA_TUNE_LOG")) {     // candidate timings, for inspection
      if (FILE* fp = std::fopen(lf, "a")) {
        std::fprintf(fp,
                     "kind %d M %d K %d nrhs %d tiles %lld : nrt %d tpw %d kt %d regions %d width %d m3 %d : %.4f ms\n",
                     key.kind, p.M, p.K, nrhs, (long long)tl.ntiles, c.nrt, c.tpw, c.kt, c.regions, c.width, c.m3,
                     ms / 3);
        std::fclose(fp);
      }
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  nesa::TileList tl = tiles_for(op, p, nrhs, best.regions, best.width, made);
  set_blocking(p, tl, best);
  out = tl;
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_store_locked(key, best);
}

template <typename T>
static void ensure_all_tiles(nesa_op* op, nesa::DevOp<T>& d, int nrhs, hipStream_t st = nullptr) {
  if (sizeof(T) != 4) return;
  using V2 = float2;
  V2* s = static_cast<V2*>(d.s);
  V2* o = static_cast<V2*>(d.o);
  for (size_t i = 0; i < d.lev.size(); ++i) {
    auto& dl = d.lev[i];
    // above pair_cap right-hand sides the translations run target-major
    // (no tiles, no per-pair outputs)
    if (dl.npairs > 0 && nrhs <= d.pair_cap) {
      tune_plan(op, dl.trans, nrhs, s + dl.s_off * nrhs, dl.pair_out, true, st);
    }
    if (i > 0 && nrhs <= d.pair_cap) {     // (target-major transfers above pair_cap)
      auto& pl = d.lev[i - 1];
      tune_plan(op, dl.up, nrhs, s + dl.s_off * nrhs, dl.child_out, false, st);
      tune_plan(op, dl.down, nrhs, o + pl.s_off * nrhs, o + dl.s_off * nrhs, false, st);
    }
  }
}

template <typename T>
static void build_dev(nesa_op* op, nesa::DevOp<T>& d, const nesa::Tree& t, const nesa::Near& nr,
                      const nesa::Far& fr) {
  const auto& LL = t.level(t.L);
  d.n = t.rwg.n;
  d.nleaf = LL.nbox;
  d.L = t.L;
  d.l0 = t.l0;
  const int QL = fr.lev[t.L - t.l0].Q;
  // limits of the kernels' fixed shapes
  int64_t smax = 0;
  for (int64_t b = 0; b < d.nleaf; ++b) smax = std::max(smax, t.leaf_ptr[b + 1] - t.leaf_ptr[b]);
  if (smax > 256) throw Error(NESA_EINVAL, "a leaf holds more than 256 RWGs; use a smaller leaf size");
  if (QL > 128) throw Error(NESA_EINVAL, "more than 128 equivalent sources per leaf");
  for (const auto& fl : fr.lev)
    if (fl.Q > 4096) throw Error(NESA_EINVAL, "more than 4096 equivalent sources per box");
  for (int64_t b = 0; b < d.nleaf; ++b)
    if (t.near_ptr[b + 1] - t.near_ptr[b] > 128) throw Error(NESA_EINVAL, "near list longer than 128");
  d.perm = upload(op, to_i32(t.perm));
  d.leaf_ptr = upload(op, to_i32(t.leaf_ptr));
  d.near_ptr = upload(op, to_i32(t.near_ptr));
  d.near_idx = upload(op, to_i32(t.near_idx));
  d.zoff = upload(op, nr.off);
  // the full blocks serve the products of several right-hand sides only
  if (op->max_nrhs > 1 && sizeof(T) == 4) d.Z = upload_complex<T>(op, nr.z);
  std::vector<int64_t> zh_off(d.nleaf + 1, 0);
  {
    // reciprocity half storage: leaf a keeps the columns of its near leaves
    // b >= a, i.e. the tail of its full block from its own columns on
    const int64_t nleaf = d.nleaf;
    std::vector<int32_t> nh(nleaf), tsrc(t.near_idx.size(), -1);
    std::vector<int64_t> col0(nleaf), toff(nleaf + 1, 0);
    for (int64_t a = 0; a < nleaf; ++a) {
      const int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      int64_t k = t.near_ptr[a], c = 0;
      while (k < t.near_ptr[a + 1] && t.near_idx[k] < a) {
        c += t.leaf_ptr[t.near_idx[k] + 1] - t.leaf_ptr[t.near_idx[k]];
        ++k;
      }
      if (k == t.near_ptr[a + 1] || t.near_idx[k] != a) throw Error(NESA_EINVAL, "leaf missing from its near list");
      const int64_t W = (nr.off[a + 1] - nr.off[a]) / S;
      nh[a] = (int32_t)k;
      col0[a] = c;
      zh_off[a + 1] = zh_off[a] + S * (W - c);
      toff[a + 1] = toff[a] + (W - c - S);
    }
    if (toff[nleaf] >= INT32_MAX) throw Error(NESA_EINVAL, "near field too large for 32-bit slot offsets");
    for (int64_t a = 0; a < nleaf; ++a) {
      const int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      int64_t col = S;
      for (int64_t k = nh[a] + 1; k < t.near_ptr[a + 1]; ++k) {
        const int64_t b = t.near_idx[k];
        const auto lo = t.near_idx.begin() + t.near_ptr[b], hi = t.near_idx.begin() + t.near_ptr[b + 1];
        const auto it = std::lower_bound(lo, hi, a);
        if (it == hi || *it != a) throw Error(NESA_EINVAL, "near lists are not symmetric");
        tsrc[it - t.near_idx.begin()] = (int32_t)(toff[a] + col - S);
        col += t.leaf_ptr[b + 1] - t.leaf_ptr[b];
      }
    }
    for (int64_t b = 0; b < nleaf; ++b)
      for (int64_t k = t.near_ptr[b]; k < nh[b]; ++k)
        if (tsrc[k] < 0) throw Error(NESA_EINVAL, "transposed near block without a slot");
    // the half blocks, converted to T on the way
    std::vector<T> zh(2 * zh_off[nleaf]);
    nesa::parallel_for(nleaf, [&](int64_t a) {
      const int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      const cd* z = nr.z.data() + nr.off[a] + col0[a] * S;
      T* o = zh.data() + 2 * zh_off[a];
      for (int64_t i = 0; i < zh_off[a + 1] - zh_off[a]; ++i) {
        o[2 * i] = (T)z[i].real();
        o[2 * i + 1] = (T)z[i].imag();
      }
    });
    d.nh_ptr = upload(op, nh);
    d.zh_off = upload(op, zh_off);
    d.Zh = upload(op, zh);
    std::vector<int32_t> to32(toff.begin(), toff.end() - 1);
    d.toff = upload(op, to32);
    d.tsrc = upload(op, tsrc);
    d.tpart = dev_alloc(op, (size_t)std::max<int64_t>(toff[nleaf], 1) * 2 * sizeof(T));
  }
  {
    // radiation matrices V = R_L G_src, assembled on the device
    const nesa::FarLevel& fl = fr.lev[t.L - t.l0];
    const nesa::Rwg& rw = t.rwg;
    nesa::RadGeo g;
    g.perm = d.perm;
    g.leaf_ptr = d.leaf_ptr;
    g.tri = upload(op, to_i32(rw.tri));
    g.freev = upload(op, to_i32(rw.freev));
    g.len = upload(op, rw.len);
    g.area = upload(op, rw.area);
    g.qp = upload(op, rw.qp);
    g.v = upload(op, rw.v);
    std::vector<double> cen(3 * d.nleaf), X(3 * fl.M), Rt(2 * fr.RLt.size());
    for (int64_t b = 0; b < d.nleaf; ++b) {
      const auto c = t.center(t.L, b);
      for (int e = 0; e < 3; ++e) cen[3 * b + e] = c[e];
    }
    for (int j = 0; j < 3 * fl.M; ++j) X[j] = fl.X[j].real();
    for (size_t i = 0; i < fr.RLt.size(); ++i) {
      Rt[2 * i] = fr.RLt[i].real();
      Rt[2 * i + 1] = fr.RLt[i].imag();
    }
    g.centre = upload(op, cen);
    g.X = upload(op, X);
    g.Rt = reinterpret_cast<const double2*>(upload(op, Rt));
    g.k = fr.k;
    g.Q = fl.Q;
    g.M = fl.M;
    if ((int64_t)fr.RLt.size() != (int64_t)fl.Q * fl.M) throw Error(NESA_EINVAL, "fitting operator size mismatch");
    d.V = dev_alloc(op, (size_t)d.n * 4 * fl.Q * 2 * sizeof(T));
    nesa::launch_fill_radiation(g, d.nleaf, d.V, sizeof(T) == 8, nullptr);
    hip_check(hipGetLastError(), "kernel launch");
  }
  d.w[0] = 0.0;
  d.w[1] = -fr.eta * fr.k;
  d.w[2] = 0.0;
  d.w[3] = fr.eta / fr.k;
  d.lev.resize(t.L - t.l0 + 1);
  d.split_fmt = split_fmt(op->precision);
  {
    // split operators run their offset-major products on the pre-split
    // sources (NESA_OM2=0: the kernels that split the sources themselves)
    const char* e = std::getenv("NESA_OM2");
    d.om2 = sizeof(T) == 4 && is_split(op->precision) && !(e && std::atoi(e) == 0);
    // (the kernel addresses a level's split sources with 32-bit offsets)
    for (int l = t.l0; l <= t.L; ++l) {
      const double kp = (fr.lev[l - t.l0].Q + 31) / 32 * 32;
      if ((double)t.level(l).nbox * kp * 2 * op->max_nrhs >= 2147483647.0) d.om2 = false;   // uint4 of s6
    }
  }
  if (op->precision == NESA_C64_SPLIT_FP16)
    d.bexp = static_cast<int*>(dev_alloc(op, (size_t)2 * (t.L - t.l0 + 1) * sizeof(int)));
  // exponent slot of a level's sources (which 0) or potentials (which 1)
  auto exp_slot = [&](int l, int which) -> const int* {
    return d.bexp ? d.bexp + 2 * (l - t.l0) + which : nullptr;
  };
  {
    // right-hand sides up to which the offset-major form (per-pair and
    // per-child partial results) runs: at most PAIR_CAP_MAX, and its partial
    // buffers within PAIR_BUFFER_BUDGET bytes
    double per_rhs = 0;
    for (int l = t.l0; l <= t.L; ++l) {
      const double Q = fr.lev[l - t.l0].Q;
      per_rhs += (double)t.level(l).il_src.size() * 4 * Q * 2 * sizeof(T);
      if (l > t.l0) per_rhs += (double)t.level(l).nbox * 4 * fr.lev[l - 1 - t.l0].Q * 2 * sizeof(T);
    }
    int cap = std::min(op->max_nrhs, nesa::PAIR_CAP_MAX);
    while (cap > 1 && cap * per_rhs > nesa::PAIR_BUFFER_BUDGET) --cap;
    if (const char* e = std::getenv("NESA_PAIR_CAP")) cap = std::max(1, std::min(cap, std::atoi(e)));   // tests
    d.pair_cap = sizeof(T) == 4 ? cap : 1;
  }
  int64_t soff = 0;
  for (int l = t.l0; l <= t.L; ++l) {
    const nesa::Level& lv = t.level(l);
    const nesa::FarLevel& fl = fr.lev[l - t.l0];
    nesa::DevLevel& dl = d.lev[l - t.l0];
    dl.Q = fl.Q;
    dl.nbox = lv.nbox;
    dl.s_off = soff;
    soff += lv.nbox * 4 * fl.Q;
    dl.npairs = (int64_t)lv.il_src.size();
    // compact translation table of the offset slots that occur, assembled on
    // the device: column-major, for complex64 the rows padded for the row blocking
    std::vector<int32_t> compact(t.nslot(), -1), offs;
    int nused = 0;
    const int SW = t.slot_w(), SH = SW / 2;
    for (int s = 0; s < t.nslot(); ++s) {
      if (!fl.slot_used[s]) continue;
      compact[s] = nused++;
      offs.push_back(s / (SW * SW) - SH);
      offs.push_back((s / SW) % SW - SH);
      offs.push_back(s % SW - SH);
    }
    const int Qr = sizeof(T) == 4 ? nesa::row_alloc(fl.Q) : fl.Q;
    void* d_split = nullptr;   // split precision: 16-bit planes of D made on the device
    int d_split_kp = 0, d_split_shift = 0;
    {
      std::vector<double> Eh(2 * fl.E.size());
      for (size_t i = 0; i < fl.E.size(); ++i) {
        Eh[2 * i] = fl.E[i].real();
        Eh[2 * i + 1] = fl.E[i].imag();
      }
      const double* Ed = upload(op, Eh);
      const int32_t* offd = offs.empty() ? nullptr : upload(op, offs);
      const size_t cnt = (size_t)nused * fl.Q * Qr;
      if (is_split(op->precision)) {
        // FP64 on the device, then its complex64 copy and the 16-bit planes of
        // the split products (no host round trip: the coarsest level of a
        // long body holds gigabytes); fp16 planes hold D x 2^shift, with the
        // shift from the largest exponent of the level's D
        dl.D = dev_alloc(op, std::max<size_t>(cnt, 1) * 2 * sizeof(T));
        d_split_kp = (fl.Q + 31) / 32 * 32;
        d_split = dev_alloc(op, std::max<size_t>((size_t)nused * 6 * Qr * d_split_kp, 1) * sizeof(uint16_t));
        if (cnt > 0) {
          void* tmp = nullptr;
          hip_check(hipMalloc(&tmp, cnt * sizeof(cd)), "hipMalloc");
          nesa::launch_fill_translation(Ed, offd, nused, fl.Q, Qr, lv.side, fr.k, tmp, true, nullptr);
          if (d.bexp) {
            int* e = static_cast<int*>(dev_alloc(op, sizeof(int)));
            nesa::launch_exp_reset(e, 1, nullptr);
            nesa::launch_absmax_exp(tmp, (int64_t)cnt, true, e, nullptr);
            int E = 0;
            hip_check(hipMemcpy(&E, e, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
            d_split_shift = nesa::split_shift(E);
          }
          nesa::launch_split_planes(tmp, nused, fl.Q, Qr, d_split_kp, dl.D, d_split, d.split_fmt, d_split_shift,
                                    nullptr);
          hip_check(hipGetLastError(), "kernel launch");
          hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
          hip_check(hipFree(tmp), "hipFree");
        }
      } else {
        dl.D = dev_alloc(op, std::max<size_t>(cnt, 1) * 2 * sizeof(T));
        nesa::launch_fill_translation(Ed, offd, nused, fl.Q, Qr, lv.side, fr.k, dl.D, sizeof(T) == 8, nullptr);
        hip_check(hipGetLastError(), "kernel launch");
      }
    }
    std::vector<int32_t> slot(lv.il_slot.size());
    for (size_t i = 0; i < slot.size(); ++i) slot[i] = compact[lv.il_slot[i]];
    dl.il_slot = upload(op, slot);
    if (sizeof(T) == 4 && dl.npairs > 0) {
      std::vector<int32_t> src(dl.npairs), dst(dl.npairs);
      for (int64_t k = 0; k < dl.npairs; ++k) {
        src[k] = (int32_t)lv.il_src[k];
        dst[k] = (int32_t)k;
      }
      int nrt = 1, Qdef = 0;
      nesa::row_blocking(fl.Q, nrt, Qdef);
      const int Qr = nesa::row_alloc(fl.Q);
      std::vector<int8_t> reg(dl.npairs);
      for (int64_t a = 0; a < lv.nbox; ++a)
        for (int64_t k = lv.il_ptr[a]; k < lv.il_ptr[a + 1]; ++k) reg[k] = (int8_t)(a * 8 / lv.nbox);
      dl.trans = make_plan(op, dl.D, (int64_t)fl.Q * Qr, fl.Q, fl.Q, Qr, nrt, 0, slot, nused, src, dst, reg);
      if (is_split(op->precision)) {
        dl.trans.A_split = d_split;
        dl.trans.Kp = d_split_kp;
        dl.trans.split_fmt = d.split_fmt;
        dl.trans.a_exp = d_split_shift;
        dl.trans.bexp = exp_slot(l, 0);
      }
      // per-pair outputs serve the offset-major form only (up to pair_cap)
      dl.pair_out = dev_alloc(op, (size_t)dl.npairs * 4 * d.pair_cap * fl.Q * 2 * sizeof(T));
    }
    // split form with many right-hand sides: the level's sources (and, in the
    // potential transfer, its potentials) split into four bf16 planes
    // (2 bytes x 4 x Kp x 4 max_nrhs per box, Kp = Q rounded up to 32)
    if (sizeof(T) == 4 && is_split(op->precision) && (d.om2 || 4 * op->max_nrhs >= nesa::TM2_MIN_COLS))
      dl.s6 = dev_alloc(op, (size_t)lv.nbox * ((fl.Q + 31) / 32 * 32) * 4 * 4 * op->max_nrhs * sizeof(uint16_t));
    // offset-major split products may read the pre-split sources (autotuner)
    if (d.om2) dl.trans.s6 = dl.s6;
    dl.il_ptr = upload(op, to_i32(lv.il_ptr));
    dl.il_src = upload(op, to_i32(lv.il_src));
    if (l < t.L) {
      dl.child_ptr = upload(op, to_i32(lv.child_ptr));
      dl.child_end = upload(op, to_i32(lv.child_end));
    }
    if (l > t.l0) {
      dl.parent = upload(op, to_i32(lv.parent));
      dl.octant = upload(op, lv.octant);
      const int Qp = fr.lev[l - 1 - t.l0].Q, Qc = fl.Q;
      std::vector<cd> ccm((size_t)8 * Qp * Qc);
      for (int o = 0; o < 8; ++o)
        for (int p = 0; p < Qp; ++p)
          for (int q = 0; q < Qc; ++q)
            ccm[((size_t)o * Qc + q) * Qp + p] = fl.Cup[((size_t)o * Qp + p) * Qc + q];
      dl.Ccm = upload_complex<T>(op, ccm);
      dl.Crm = upload_complex<T>(op, fl.Cup);
      if (sizeof(T) == 4) {
        // upward: A_o = C_o (Qp x Qc), column-major, rows padded to Qpr
        int nrt_u = 1, nrt_d = 1, Qdef = 0;
        nesa::row_blocking(Qp, nrt_u, Qdef);
        nesa::row_blocking(Qc, nrt_d, Qdef);
        const int Qpr = nesa::row_alloc(Qp), Qcr = nesa::row_alloc(Qc);
        std::vector<cd> au((size_t)8 * Qc * Qpr, cd(0, 0)), ad((size_t)8 * Qp * Qcr, cd(0, 0));
        for (int o = 0; o < 8; ++o)
          for (int p = 0; p < Qp; ++p)
            for (int q = 0; q < Qc; ++q) {
              const cd c = fl.Cup[((size_t)o * Qp + p) * Qc + q];
              au[((size_t)o * Qc + q) * Qpr + p] = c;      // C_o[p][q]
              ad[((size_t)o * Qp + p) * Qcr + q] = c;      // (C_o^T)[q][p]
            }
        // boxes with a parent (in a forest the top box of a body has none)
        std::vector<int32_t> grp, idx, par;
        std::vector<int8_t> reg;
        for (int64_t b = 0; b < lv.nbox; ++b) {
          if (lv.parent[b] < 0) continue;
          grp.push_back(lv.octant[b]);
          idx.push_back((int32_t)b);
          par.push_back((int32_t)lv.parent[b]);
          reg.push_back((int8_t)(b * 8 / lv.nbox));
        }
        dl.up = make_plan(op, upload_complex<T>(op, au), (int64_t)Qc * Qpr, Qp, Qc, Qpr, nrt_u, 0, grp, 8, idx, idx,
                           reg);
        if (is_split(op->precision)) attach_split(op, dl.up, au, 8, d.split_fmt, exp_slot(l, 0));
        if (d.om2) dl.up.s6 = dl.s6;           // this level's sources
        // per-child outputs serve the offset-major form only (up to pair_cap)
        dl.child_out = dev_alloc(op, (size_t)lv.nbox * 4 * d.pair_cap * Qp * 2 * sizeof(T));
        dl.down = make_plan(op, upload_complex<T>(op, ad), (int64_t)Qp * Qcr, Qc, Qp, Qcr, nrt_d, 1, grp, 8, par, idx,
                             reg);
        if (is_split(op->precision)) attach_split(op, dl.down, ad, 8, d.split_fmt, exp_slot(l - 1, 1));
        if (d.om2) dl.down.s6 = d.lev[l - 1 - t.l0].s6;     // the parent level's potentials
        // pair lists of the target-major transfers: the children of every box
        // of level l-1 in increasing index (CSR), and the parent of every box
        const int64_t np = t.level(l - 1).nbox;
        std::vector<int32_t> uptr(np + 1, 0), usrc, uslot, dptr(lv.nbox + 1, 0), dsrc, dslot;
        for (int64_t b = 0; b < lv.nbox; ++b)
          if (lv.parent[b] >= 0) ++uptr[lv.parent[b] + 1];
        for (int64_t P = 0; P < np; ++P) uptr[P + 1] += uptr[P];
        usrc.resize(uptr[np]);
        uslot.resize(uptr[np]);
        {
          std::vector<int32_t> fill(uptr.begin(), uptr.end() - 1);
          for (int64_t b = 0; b < lv.nbox; ++b) {
            if (lv.parent[b] < 0) continue;
            const int32_t e = fill[lv.parent[b]]++;
            usrc[e] = (int32_t)b;
            uslot[e] = lv.octant[b];
          }
        }
        for (int64_t b = 0; b < lv.nbox; ++b) {
          dptr[b + 1] = dptr[b];
          if (lv.parent[b] < 0) continue;
          dsrc.push_back((int32_t)lv.parent[b]);
          dslot.push_back(lv.octant[b]);
          ++dptr[b + 1];
        }
        dl.up_ptr = upload(op, uptr);
        dl.up_src = upload(op, usrc);
        dl.up_slot = upload(op, uslot);
        dl.dn_ptr = upload(op, dptr);
        dl.dn_src = upload(op, dsrc);
        dl.dn_slot = upload(op, dslot);
      }
    }
  }
  d.max_nrhs = op->max_nrhs;
  d.s = dev_alloc(op, (size_t)soff * op->max_nrhs * 2 * sizeof(T));
  d.o = dev_alloc(op, (size_t)soff * op->max_nrhs * 2 * sizeof(T));
  // block-diagonal preconditioner: inverses of the self blocks
  std::vector<int64_t> moff(d.nleaf + 1, 0);
  for (int64_t a = 0; a < d.nleaf; ++a) {
    int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
    moff[a + 1] = moff[a] + S * S;
  }
  std::vector<cd> minv(moff[d.nleaf]);
  nesa::parallel_for(d.nleaf, [&](int64_t a) {
    const int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
    int64_t col0 = 0;
    for (int64_t j = t.near_ptr[a]; j < t.near_ptr[a + 1]; ++j) {
      int64_t b = t.near_idx[j];
      if (b == a) break;
      col0 += t.leaf_ptr[b + 1] - t.leaf_ptr[b];
    }
    std::vector<cd> A(S * S);
    const cd* Z = &nr.z[nr.off[a]];
    for (int64_t c = 0; c < S; ++c)
      for (int64_t r = 0; r < S; ++r) A[c * S + r] = Z[(col0 + c) * S + r];
    invert(A, S);
    std::copy(A.begin(), A.end(), minv.begin() + moff[a]);
  });
  d.Minv = upload_complex<T>(op, minv);
  d.moff = upload(op, moff);
  {
    // launch order of the near-field workgroups: largest blocks first
    std::vector<int32_t> ord(d.nleaf);
    for (int64_t a = 0; a < d.nleaf; ++a) ord[a] = (int32_t)a;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
      return zh_off[x + 1] - zh_off[x] > zh_off[y + 1] - zh_off[y];
    });
    d.near_order = upload(op, ord);
  }
  op->xl = dev_alloc(op, (size_t)d.n * op->max_nrhs * 2 * sizeof(T));
  op->yl = dev_alloc(op, (size_t)d.n * op->max_nrhs * 2 * sizeof(T));
  // side stream (default priority, non-blocking so that it never serialises
  // with the legacy default stream) and the fork / join events of the product
  hip_check(hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  {
    // persistent near-field grid: one workgroup per CU (measured best beside the
    // far-field stages; NESA_NEAR_WGS overrides)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    }
    d.near_wgs = cus;
    if (const char* e = std::getenv("NESA_NEAR_WGS")) d.near_wgs = std::max(1, std::atoi(e));
  }
  hip_check(hipEventCreateWithFlags(&d.ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
  hip_check(hipEventCreateWithFlags(&d.ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
  hip_check(hipStreamCreateWithFlags(&d.side2, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  hip_check(hipEventCreateWithFlags(&d.ev_fork2, hipEventDisableTiming), "hipEventCreateWithFlags");
  hip_check(hipEventCreateWithFlags(&d.ev_join2, hipEventDisableTiming), "hipEventCreateWithFlags");
  ensure_all_tiles<T>(op, d, 1);
}

// device memory released at scope exit
struct DevTmp {
  void* p = nullptr;
  DevTmp() = default;
  DevTmp(const DevTmp&) = delete;
  DevTmp& operator=(const DevTmp&) = delete;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
  template <typename X>
  X* alloc(size_t count) {
    hip_check(hipMalloc(&p, std::max<size_t>(count * sizeof(X), 16)), "hipMalloc");
    return static_cast<X*>(p);
  }
  template <typename X>
  X* put(const std::vector<X>& h) {
    X* d = alloc<X>(h.size());
    if (!h.empty()) hip_check(hipMemcpy(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice), "hipMemcpy");
    return d;
  }
};

// Schwarz preconditioner of a complex64 operator assembled on the device
// (precond_dev.hip): per-leaf tables of the near lists on the host, then the
// matrices Z_N^T gathered from the device's near blocks (reciprocity half
// storage, the form the one-right-hand-side product applies), factored and
// solved by persistent workgroups, each with a workspace for the largest
// matrix (at most 32 GiB in all).  Returns false (nothing built) when a near
// list holds more than 27 leaves or more than SCHWARZ_WMAX RWGs.
static bool schwarz_device(nesa_op* op) {
  const nesa::Tree& t = *op->tree;
  const nesa::Near& nr = *op->near;
  const int64_t nleaf = t.level(t.L).nbox;
  constexpr int MX = nesa::SCHWARZ_MAXN;
  for (int64_t a = 0; a < nleaf; ++a)
    if (t.near_ptr[a + 1] - t.near_ptr[a] > MX) return false;
  std::vector<int32_t> na(nleaf), W(nleaf), rowa(nleaf, -1), nb((size_t)nleaf * MX, 0),
      off((size_t)nleaf * (MX + 1), 0), colpos((size_t)nleaf * MX * MX, -1);
  auto size_of = [&](int64_t b) { return (int32_t)(t.leaf_ptr[b + 1] - t.leaf_ptr[b]); };
  // npos[q]: first column of near-list entry q inside its leaf's full block
  std::vector<int32_t> npos(t.near_idx.size());
  nesa::parallel_for(nleaf, [&](int64_t x) {
    int32_t c = 0;
    for (int64_t q = t.near_ptr[x]; q < t.near_ptr[x + 1]; ++q) {
      npos[q] = c;
      c += size_of(t.near_idx[q]);
    }
  });
  // entry of leaf y in leaf x's (sorted) near list, -1 if absent
  auto entry = [&](int64_t x, int64_t y) -> int64_t {
    const int64_t* lo = t.near_idx.data() + t.near_ptr[x];
    const int64_t* hi = t.near_idx.data() + t.near_ptr[x + 1];
    const int64_t* it = std::lower_bound(lo, hi, y);
    return (it != hi && *it == y) ? it - t.near_idx.data() : -1;
  };
  nesa::parallel_for(nleaf, [&](int64_t a) {
    const int n = (int)(t.near_ptr[a + 1] - t.near_ptr[a]);
    int32_t* nba = &nb[(size_t)a * MX];
    int32_t* offa = &off[(size_t)a * (MX + 1)];
    for (int i = 0; i < n; ++i) {
      nba[i] = (int32_t)t.near_idx[t.near_ptr[a] + i];
      offa[i + 1] = offa[i] + size_of(nba[i]);
      if (nba[i] == a) rowa[a] = offa[i];
    }
    na[a] = n;
    W[a] = offa[n];
    for (int jb = 0; jb < n; ++jb)
      for (int ib = 0; ib < n; ++ib) {
        const int64_t x = std::min(nba[jb], nba[ib]), y = std::max(nba[jb], nba[ib]);
        const int64_t qy = entry(x, y), qx = entry(x, x);
        if (qy >= 0 && qx >= 0) colpos[(size_t)a * MX * MX + jb * MX + ib] = npos[qy] - npos[qx];
      }
  });
  for (int64_t a = 0; a < nleaf; ++a)
    if (rowa[a] < 0) throw Error(NESA_EINVAL, "a leaf is missing from its own near list");
  // persistent workgroups, each with a workspace for the largest W; leaves
  // taken largest first
  int32_t wmax = 0;
  for (int64_t a = 0; a < nleaf; ++a) wmax = std::max(wmax, W[a]);
  if (wmax > nesa::SCHWARZ_WMAX) return false;
  std::vector<int32_t> order(nleaf);
  for (int64_t a = 0; a < nleaf; ++a) order[a] = (int32_t)a;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return W[x] > W[y]; });
  size_t free_b = 0, total_b = 0;
  hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  const int64_t slot_bytes = (int64_t)wmax * wmax * (int64_t)sizeof(float2);
  const int64_t budget = std::min<int64_t>(int64_t(32) << 30, (int64_t)(free_b / 2));
  int64_t slots = std::min<int64_t>(nesa::schwarz_slots(), nleaf);
  slots = std::max<int64_t>(1, std::min<int64_t>(slots, budget / std::max<int64_t>(slot_bytes, 1)));
  nesa::DevOp<float>& d = op->f;
  DevTmp t_ord, t_cnt, t_na, t_w, t_rowa, t_nb, t_off, t_cp, t_ws, t_piv, t_st;
  nesa::SchwarzWork w;
  w.nleaf = (int)nleaf;
  w.order = t_ord.put(order);
  w.counter = t_cnt.alloc<int32_t>(1);
  w.na = t_na.put(na);
  w.W = t_w.put(W);
  w.rowa = t_rowa.put(rowa);
  w.nb = t_nb.put(nb);
  w.off = t_off.put(off);
  w.colpos = t_cp.put(colpos);
  w.ws_stride = (int64_t)wmax * wmax;
  w.ws = t_ws.alloc<float2>((size_t)(slots * w.ws_stride));
  w.piv_stride = std::max<int32_t>(wmax, 1);
  w.piv = t_piv.alloc<int32_t>((size_t)(slots * w.piv_stride));
  w.status = t_st.alloc<int32_t>(1);
  hip_check(hipMemset(w.status, 0, sizeof(int32_t)), "hipMemset");
  float2* out = static_cast<float2*>(dev_alloc(op, nr.z.size() * sizeof(float2)));
  nesa::launch_schwarz(static_cast<const float2*>(d.Zh), d.zh_off, d.zoff, d.leaf_ptr, w, (int)slots, out, nullptr);
  hip_check(hipGetLastError(), "kernel launch");
  int32_t status = 0;
  hip_check(hipMemcpy(&status, w.status, sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy");
  if (status) throw Error(-1, "singular near-field matrix in the Schwarz preconditioner");
  op->schwarz = out;
  return true;
}

// Schwarz preconditioner, built at first use in the near-block layout of the
// op's precision: on the device for complex64 operators (on the host in FP32
// when NESA_SCHWARZ_HOST=1), on the host in FP64 for complex128 ones
static void ensure_schwarz(nesa_op* op) {
  if (op->schwarz) return;
  const char* host = std::getenv("NESA_SCHWARZ_HOST");
  if (op->precision != NESA_C128 && !(host && std::atoi(host) == 1) && schwarz_device(op)) return;
  std::unique_ptr<nesa::Near> P(nesa::near_schwarz(*op->tree, *op->near, op->precision != NESA_C128));
  if (op->precision == NESA_C128)
    op->schwarz = upload_complex<double>(op, P->z);
  else
    op->schwarz = upload_complex<float>(op, P->z);
}

int nesa_precond_setup(nesa_op* op, int precond);

// ------------------------------------------------------------------ learned preconditioner
struct nesa_mlp {
  nesa_op* op = nullptr;
  int base = NESA_PRECOND_BLOCKDIAG;
  nesa::MlpDev net;
  nesa::MlpRows app;                    // one row per leaf (inference inside GMRES)
  nesa::MlpRows trn;                    // samples x leaves (training data)
  void* trn_vec = nullptr;              // leaf-order r, e, base output of the training samples
  int64_t trn_cap = 0;                  // samples the training buffers hold
  int64_t nsamples = 0, nvalid = 0;
  int t = 0;                            // Adam steps taken
  std::vector<void*> allocs;            // parameter and inference buffers
  std::vector<void*> trn_allocs;
  ~nesa_mlp() {
    for (void* p : allocs) (void)hipFree(p);
    for (void* p : trn_allocs) (void)hipFree(p);
  }
};

nesa_op::~nesa_op() {
  for (nesa_mlp* m : nets) m->op = nullptr;
  (void)hipDeviceSynchronize();
  for (auto* dv : {&f.side, &d.side, &f.side2, &d.side2})
    if (*dv) (void)hipStreamDestroy(*dv);
  for (auto* ev : {&f.ev_fork, &f.ev_join, &d.ev_fork, &d.ev_join, &f.ev_fork2, &f.ev_join2, &d.ev_fork2,
                   &d.ev_join2})
    if (*ev) (void)hipEventDestroy(*ev);
  for (void* p : allocs) (void)hipFree(p);
}

template <typename X>
static X* net_alloc(std::vector<void*>& list, int64_t count) {
  void* p = nullptr;
  hip_check(hipMalloc(&p, std::max<size_t>(256, (size_t)count * sizeof(X))), "hipMalloc");
  list.push_back(p);
  return static_cast<X*>(p);
}

// activation buffers of `rows` rows (training adds the transposed copies)
static void alloc_rows(std::vector<void*>& list, nesa::MlpRows& R, int S, int H, int64_t rows, bool training) {
  R.rows = rows;
  R.rows_pad = (rows + 63) / 64 * 64;
  const int64_t P = R.rows_pad;
  R.U = net_alloc<_Float16>(list, P * 4 * S);
  R.scale = net_alloc<float>(list, P);
  R.rowS = net_alloc<int32_t>(list, P);
  R.h1 = net_alloc<_Float16>(list, P * H);
  R.h2 = net_alloc<_Float16>(list, P * H);
  R.Y = net_alloc<float>(list, P * 2 * S);
  if (training) {
    R.UT = net_alloc<_Float16>(list, P * 4 * S);
    R.Tg = net_alloc<float>(list, P * 2 * S);
    R.h1T = net_alloc<_Float16>(list, P * H);
    R.h2T = net_alloc<_Float16>(list, P * H);
    R.dY = net_alloc<_Float16>(list, P * 2 * S);
    R.dYT = net_alloc<_Float16>(list, P * 2 * S);
    R.dp2 = net_alloc<_Float16>(list, P * H);
    R.dp2T = net_alloc<_Float16>(list, P * H);
    R.dp1T = net_alloc<_Float16>(list, P * H);
  }
}

template <typename T>
static void base_apply(nesa_op* op, nesa::DevOp<T>& d, int base, const void* r, void* z, hipStream_t st) {
  if (base == NESA_PRECOND_SCHWARZ)
    nesa::launch_near_apply<T>(d, op->schwarz, r, z, st);
  else
    nesa::launch_blockdiag<T>(d, r, z, st);
}

// z = M_base r + network correction (one vector, leaf order)
template <typename T>
static void learned_apply(nesa_mlp* h, nesa::DevOp<T>& d, const void* r, void* z, hipStream_t st) {
  base_apply<T>(h->op, d, h->base, r, z, st);
  nesa::launch_mlp_features<T>(h->net, h->app, r, z, nullptr, d.leaf_ptr, d.nleaf, d.n, 1, false, st);
  nesa::launch_mlp_forward(h->net, h->app, false, st);
  nesa::launch_mlp_combine<T>(h->net, h->app, d.leaf_ptr, d.nleaf, z, st);
}

// ------------------------------------------------------------------ GMRES driver
// Workgroups of the FP64 dot products (k_multidot): about four elements per
// thread, at most 512 workgroups (on the 201,720-unknown sphere a GMRES(50)
// iteration takes 1.156 ms with two or four elements per thread, 1.175 with
// eight and 1.191 with one).
static int dot_blocks(int64_t n) {
  return (int)std::min<int64_t>(512, std::max<int64_t>(1, (n + 4 * 256 - 1) / (4 * 256)));
}

// Device workspace of one GMRES(m) solve (bytes), carved in this order:
// basis V (m + 1 vectors), preconditioned basis Z (m vectors, flexible only),
// b, x, w, tmp in leaf order, the FP64 coefficients and the block partials.
static size_t gmres_workspace_bytes(int64_t n, int m, bool flex, size_t es) {
  auto r256 = [](size_t b) { return (std::max<size_t>(b, 16) + 255) / 256 * 256; };
  const int nblocks = dot_blocks(n);
  size_t b = r256((size_t)(m + 1) * n * es) + (flex ? r256((size_t)m * n * es) : 0) + 4 * r256(n * es);
  b += r256(sizeof(double2) * (2 * (m + 2) + 2)) + r256(sizeof(double2) * nblocks * (m + 2));
  return b;
}

// ws: caller-provided device workspace of gmres_workspace_bytes() and host
// scalars hws (2 (m + 2) + 2 values); null: both allocated here and freed on return
template <typename T>
static int gmres_one(nesa_op* op, nesa::DevOp<T>& d, const void* b_c, void* x_c, const nesa_gmres_params& prm,
                     nesa_gmres_report& rep, double* history, int64_t hist_len, hipStream_t st,
                     char* ws = nullptr, double2* hws = nullptr) {
  const int64_t n = d.n;
  const int m = prm.restart;
  const size_t es = 2 * sizeof(T);
  auto t0 = std::chrono::steady_clock::now();
  const bool flex = prm.precond != NESA_PRECOND_NONE;
  std::vector<void*> mine;
  size_t ws_used = 0;
  auto alloc = [&](size_t bytes) {
    void* p = nullptr;
    if (ws) {
      p = ws + ws_used;
      ws_used += (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
      return p;
    }
    hip_check(hipMalloc(&p, std::max<size_t>(bytes, 16)), "hipMalloc");
    mine.push_back(p);
    return p;
  };
  struct Free {
    std::vector<void*>& v;
    double2* host;
    ~Free() {
      for (void* p : v) (void)hipFree(p);
      if (host) (void)hipHostFree(host);
    }
  };
  const int nblocks = dot_blocks(n);
  char* Vb = static_cast<char*>(alloc((size_t)(m + 1) * n * es));
  char* Zb = flex ? static_cast<char*>(alloc((size_t)m * n * es)) : nullptr;
  void* bl = alloc(n * es);
  void* xl = alloc(n * es);
  void* w = alloc(n * es);
  void* tmp = alloc(n * es);
  double2* hd = static_cast<double2*>(alloc(sizeof(double2) * (2 * (m + 2) + 2)));
  double2* partial = static_cast<double2*>(alloc(sizeof(double2) * nblocks * (m + 2)));
  // Pipelined Arnoldi (the allocating form): the device normalises v_{j+1}
  // itself and step j + 1 is enqueued before the host reads step j's
  // coefficients back, so the GPU does not wait for the host's Givens
  // rotations; the read-backs alternate between two pinned slots, a third
  // carries the solution coefficients.  The form without allocation (caller's
  // workspace) keeps one slot and one synchronisation per step.
  const bool ahead = ws == nullptr;
  const int HS = 2 * (m + 2) + 2;
  double2* hh = hws;
  if (!hh) hip_check(hipHostMalloc((void**)&hh, sizeof(double2) * HS * (ahead ? 3 : 1)), "hipHostMalloc");
  Free guard{mine, hws ? nullptr : hh};
  double2* hslot[2] = {hh, ahead ? hh + HS : hh};
  double2* hy = ahead ? hh + 2 * HS : hh;
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{ev};
  if (ahead)
    for (int i = 0; i < 2; ++i) hip_check(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming), "hipEventCreate");
  auto vec = [&](char* base, int i) { return static_cast<void*>(base + (size_t)i * n * es); };
  auto matvec = [&](const void* src, void* dst) { nesa::launch_matvec_leaf<T>(d, src, dst, 1, st, nullptr); };
  auto norm = [&](const void* v) {
    nesa::launch_multidot<T>(v, n, 1, v, n, partial, nblocks, hd, 0, st);
    hip_check(hipMemcpyAsync(hh, hd, sizeof(double2), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return std::sqrt(std::max(0.0, hh[0].x));
  };
  // the learned preconditioner falls back to its base when a cycle yields a
  // non-finite value or does not reduce the true residual
  int active = prm.precond;
  auto precond = [&](const void* r, void* z) {
    if (active == NESA_PRECOND_LEARNED) {
      learned_apply<T>(op->mlp, d, r, z, st);
    } else if (active == NESA_PRECOND_SCHWARZ || active == NESA_PRECOND_BLOCKDIAG) {
      base_apply<T>(op, d, active, r, z, st);
    } else {
      hip_check(hipMemcpyAsync(z, r, n * es, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    }
  };
  nesa::launch_gather<T>(b_c, bl, d.perm, n, st);
  nesa::launch_gather<T>(x_c, xl, d.perm, n, st);
  const double nb = norm(bl);
  rep = nesa_gmres_report{0, 0, 0.0, 0.0, 0};
  if (nb == 0) {
    // x = 0: b gathered into leaf order is exactly zero; scattered back by a
    // kernel (no memset node when the caller captures the stream)
    nesa::launch_scatter<T>(bl, x_c, d.perm, n, st);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return NESA_OK;
  }
  int64_t nh = 0;
  auto push_hist = [&](double v) {
    if (history && nh < hist_len) history[nh] = v;
    ++nh;
  };
  matvec(xl, tmp);
  nesa::launch_sub<T>(bl, tmp, vec(Vb, 0), n, st);
  double beta = norm(vec(Vb, 0));
  push_hist(beta / nb);
  int iters = 0;
  std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m);
  std::vector<double> cs(m);
  int status = NESA_OK;
  while (beta / nb > prm.tol && iters < prm.max_iters) {
    rep.restarts++;
    bool discard = false;                 // learned cycle that produced a non-finite value
    nesa::launch_scale<T>(vec(Vb, 0), vec(Vb, 0), n, 1.0 / beta, st);
    std::fill(H.begin(), H.end(), cd(0, 0));
    std::fill(g.begin(), g.end(), cd(0, 0));
    g[0] = beta;
    int k = 0;
    // Arnoldi step j up to its coefficients (read back into hslot[j % 2]) and,
    // pipelined, v_{j+1} = w / ||w|| on the device
    auto enqueue = [&](int j) {
      const void* src = vec(Vb, j);
      if (flex) {
        precond(vec(Vb, j), vec(Zb, j));
        src = vec(Zb, j);
      }
      matvec(src, w);
      // two passes of classical Gram-Schmidt, FP64 dot products
      nesa::launch_multidot<T>(Vb, n, j + 1, w, n, partial, nblocks, hd, 0, st);
      nesa::launch_combine<T>(Vb, n, j + 1, hd, w, n, -1.0, st);
      nesa::launch_multidot<T>(Vb, n, j + 1, w, n, partial, nblocks, hd + (m + 2), 0, st);
      nesa::launch_combine<T>(Vb, n, j + 1, hd + (m + 2), w, n, -1.0, st);
      nesa::launch_multidot<T>(w, n, 1, w, n, partial, nblocks, hd + 2 * (m + 2), 0, st);
      hip_check(hipMemcpyAsync(hslot[j % 2], hd, sizeof(double2) * (2 * (m + 2) + 1), hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync");
      if (ahead) {
        hip_check(hipEventRecord(ev[j % 2], st), "hipEventRecord");
        nesa::launch_scale_norm<T>(w, vec(Vb, j + 1), n, hd + 2 * (m + 2), st);
      }
    };
    enqueue(0);
    for (int j = 0; j < m; ++j) {
      // (pipelined: step j + 1 runs while the host finishes step j; if the
      // cycle ends at j its result is not used)
      if (ahead && j + 1 < m) enqueue(j + 1);
      if (ahead)
        hip_check(hipEventSynchronize(ev[j % 2]), "hipEventSynchronize");
      else
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
      const double2* hc = hslot[j % 2];
      for (int i = 0; i <= j; ++i)
        H[(size_t)j * (m + 1) + i] = cd(hc[i].x + hc[m + 2 + i].x, hc[i].y + hc[m + 2 + i].y);
      const double hn = std::sqrt(std::max(0.0, hc[2 * (m + 2)].x));
      bool finite = std::isfinite(hn);
      for (int i = 0; i <= j && finite; ++i) finite = std::isfinite(std::abs(H[(size_t)j * (m + 1) + i]));
      if (!finite) {
        if (active == NESA_PRECOND_LEARNED) {
          active = op->mlp->base;
          rep.fell_back = 1;
          discard = true;
        } else {
          status = fail(NESA_EBREAKDOWN, "non-finite value in GMRES");
        }
        break;
      }
      H[(size_t)j * (m + 1) + j + 1] = hn;
      cd* Hj = &H[(size_t)j * (m + 1)];
      for (int i = 0; i < j; ++i) {
        cd t0v = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -std::conj(sn[i]) * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t0v;
      }
      cd a = Hj[j], bb = Hj[j + 1];
      double c;
      cd s, r;
      if (bb == cd(0, 0)) {
        c = 1;
        s = 0;
        r = a;
      } else if (a == cd(0, 0)) {
        c = 0;
        s = 1;
        r = bb;
      } else {
        double rho = std::hypot(std::abs(a), std::abs(bb));
        c = std::abs(a) / rho;
        s = a * std::conj(bb) / (std::abs(a) * rho);
        r = a * rho / std::abs(a);
      }
      cs[j] = c;
      sn[j] = s;
      Hj[j] = r;
      Hj[j + 1] = 0;
      g[j + 1] = -std::conj(s) * g[j];
      g[j] = c * g[j];
      ++iters;
      k = j + 1;
      push_hist(std::abs(g[j + 1]) / nb);
      if (std::abs(g[j + 1]) / nb <= prm.tol || iters >= prm.max_iters || hn == 0) break;
      if (!ahead && j + 1 < m) {
        nesa::launch_scale<T>(w, vec(Vb, j + 1), n, 1.0 / hn, st);
        enqueue(j + 1);
      }
    }
    if (status != NESA_OK) break;
    if (discard) {                        // restart from the same x with the base preconditioner
      nesa::launch_sub<T>(bl, tmp, vec(Vb, 0), n, st);
      continue;
    }
    std::vector<cd> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int c2 = i + 1; c2 < k; ++c2) acc -= H[(size_t)c2 * (m + 1) + i] * y[c2];
      y[i] = acc / H[(size_t)i * (m + 1) + i];
    }
    // (pipelined: a step enqueued past the end of the cycle may still be
    // copying into hslot; the coefficients go through their own slot)
    for (int i = 0; i < k; ++i) hy[i] = make_double2(y[i].real(), y[i].imag());
    hip_check(hipMemcpyAsync(hd, hy, sizeof(double2) * k, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    nesa::launch_combine<T>(flex ? Zb : Vb, n, k, hd, xl, n, +1.0, st);
    matvec(xl, tmp);
    nesa::launch_sub<T>(bl, tmp, vec(Vb, 0), n, st);
    const double beta_prev = beta;
    beta = norm(vec(Vb, 0));
    const double ratio = prm.fallback_ratio > 0 ? prm.fallback_ratio : 1.0;
    if (active == NESA_PRECOND_LEARNED && !(beta < ratio * beta_prev)) {
      active = op->mlp->base;
      rep.fell_back = 1;
    }
  }
  nesa::launch_scatter<T>(xl, x_c, d.perm, n, st);
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  rep.iters = iters;
  rep.true_rel_residual = beta / nb;
  rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status != NESA_OK) return status;
  if (beta / nb > prm.tol) return fail(NESA_ENOCONV, "GMRES reached max_iters above tolerance");
  return NESA_OK;
}

// Several right-hand sides in lock step (complex64).  Every right-hand side
// runs its own restarted (F)GMRES as in gmres_one, but each iteration all the
// unconverged ones take one Arnoldi step (each at its own position in its own
// restart cycle), their new vectors go through one multi-RHS product, and one
// host synchronisation serves all their Gram-Schmidt coefficients.  The true
// residuals that close the cycles are batched the same way.
static int gmres_batch(nesa_op* op, nesa::DevOp<float>& d, const void* b_c, void* x_c, int R,
                       const nesa_gmres_params& prm, nesa_gmres_report* rep, double* history, int64_t hist_len,
                       hipStream_t st) {
  using T = float;
  const int64_t n = d.n;
  const int m = prm.restart;
  const size_t es = 2 * sizeof(T);
  auto t0 = std::chrono::steady_clock::now();
  const bool flex = prm.precond != NESA_PRECOND_NONE;
  std::vector<void*> mine;
  auto alloc = [&](size_t bytes) {
    void* p = nullptr;
    hip_check(hipMalloc(&p, std::max<size_t>(bytes, 16)), "hipMalloc");
    mine.push_back(p);
    return p;
  };
  const int HS = 2 * (m + 2) + 2;                      // double2 slots per right-hand side
  double2* hh = nullptr;
  struct Free {
    std::vector<void*>& v;
    double2*& host;
    ~Free() {
      for (void* p : v) (void)hipFree(p);
      if (host) (void)hipHostFree(host);
    }
  } guard{mine, hh};
  hip_check(hipHostMalloc((void**)&hh, sizeof(double2) * HS * R), "hipHostMalloc");
  const int nblocks = dot_blocks(n);
  double2* hd = static_cast<double2*>(alloc(sizeof(double2) * HS * R));
  double2* partial = static_cast<double2*>(alloc(sizeof(double2) * nblocks * (m + 2)));
  // product input / output and preconditioned vectors, one slot per RHS; the
  // products always run R wide (slots of finished right-hand sides are ignored),
  // so the multi-RHS blockings are tuned once
  char* Xb = static_cast<char*>(alloc((size_t)R * n * es));
  char* Yb = static_cast<char*>(alloc((size_t)R * n * es));
  char* Pb = flex ? static_cast<char*>(alloc((size_t)R * n * es)) : nullptr;
  hip_check(hipMemsetAsync(Xb, 0, (size_t)R * n * es, st), "hipMemsetAsync");
  if (Pb) hip_check(hipMemsetAsync(Pb, 0, (size_t)R * n * es, st), "hipMemsetAsync");
  ensure_all_tiles<T>(op, d, R, st);
  struct Rhs {
    char *V, *Z;
    void *bl, *xl, *ax;                                             // b, x, A x (leaf order)
    double nb = 0, beta = 0, beta_prev = 0;
    int j = 0, iters = 0, active = 0;
    bool done = false, in_cycle = false, discard = false;
    std::vector<cd> H, g, sn;
    std::vector<double> cs;
  };
  std::vector<Rhs> rh(R);
  for (int r = 0; r < R; ++r) {
    Rhs& q = rh[r];
    q.V = static_cast<char*>(alloc((size_t)(m + 1) * n * es));
    q.Z = flex ? static_cast<char*>(alloc((size_t)m * n * es)) : nullptr;
    q.bl = alloc(n * es);
    q.xl = alloc(n * es);
    q.ax = alloc(n * es);
    q.H.assign((size_t)(m + 1) * m, cd(0, 0));
    q.g.assign(m + 1, cd(0, 0));
    q.sn.assign(m, cd(0, 0));
    q.cs.assign(m, 0.0);
    q.active = prm.precond;
    rep[r] = nesa_gmres_report{0, 0, 0.0, 0.0, 0};
  }
  auto vec = [&](char* base, int i) { return static_cast<void*>(base + (size_t)i * n * es); };
  auto slot = [&](char* base, int i) { return static_cast<void*>(base + (size_t)i * n * es); };
  auto hslot = [&](int r) { return hd + (size_t)r * HS; };
  auto fetch = [&]() {
    hip_check(hipMemcpyAsync(hh, hd, sizeof(double2) * HS * R, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  };
  auto precond = [&](Rhs& q, const void* r, void* z) {
    if (q.active == NESA_PRECOND_LEARNED)
      learned_apply<T>(op->mlp, d, r, z, st);
    else if (q.active == NESA_PRECOND_SCHWARZ || q.active == NESA_PRECOND_BLOCKDIAG)
      base_apply<T>(op, d, q.active, r, z, st);
    else
      hip_check(hipMemcpyAsync(z, r, n * es, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
  };
  // y = A x for the listed right-hand sides' vectors in one product (R wide)
  auto batched_matvec = [&](const std::vector<const void*>& src, const std::vector<void*>& dst) {
    const int ra = (int)src.size();
    if (ra == 0) return;
    for (int i = 0; i < ra; ++i)
      if (src[i] != slot(Xb, i))
        hip_check(hipMemcpyAsync(slot(Xb, i), src[i], n * es, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    nesa::launch_matvec_leaf<T>(d, Xb, Yb, R, st, nullptr);
    for (int i = 0; i < ra; ++i)
      if (dst[i] != slot(Yb, i))
        hip_check(hipMemcpyAsync(dst[i], slot(Yb, i), n * es, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
  };
  // true residuals of the listed right-hand sides: ax = A x, V0 = b - ax, beta
  auto residuals = [&](const std::vector<int>& list) {
    std::vector<const void*> src;
    std::vector<void*> dst;
    for (int r : list) {
      src.push_back(rh[r].xl);
      dst.push_back(rh[r].ax);
    }
    batched_matvec(src, dst);
    for (int r : list) {
      nesa::launch_sub<T>(rh[r].bl, rh[r].ax, vec(rh[r].V, 0), n, st);
      nesa::launch_multidot<T>(vec(rh[r].V, 0), n, 1, vec(rh[r].V, 0), n, partial, nblocks, hslot(r), 0, st);
    }
    fetch();
    for (int r : list) {
      rh[r].beta_prev = rh[r].beta;
      rh[r].beta = std::sqrt(std::max(0.0, hh[(size_t)r * HS].x));
    }
  };
  auto start_cycle = [&](int r) {
    Rhs& q = rh[r];
    nesa::launch_scale<T>(vec(q.V, 0), vec(q.V, 0), n, 1.0 / q.beta, st);
    std::fill(q.H.begin(), q.H.end(), cd(0, 0));
    std::fill(q.g.begin(), q.g.end(), cd(0, 0));
    q.g[0] = q.beta;
    q.j = 0;
    q.in_cycle = true;
    q.discard = false;
    rep[r].restarts++;
  };
  int64_t nh = 0;
  // right-hand side norms and initial residuals
  std::vector<int> all;
  for (int r = 0; r < R; ++r) {
    all.push_back(r);
    const char* br = static_cast<const char*>(b_c) + (size_t)r * n * es;
    char* xr = static_cast<char*>(x_c) + (size_t)r * n * es;
    nesa::launch_gather<T>(br, rh[r].bl, d.perm, n, st);
    nesa::launch_gather<T>(xr, rh[r].xl, d.perm, n, st);
    nesa::launch_multidot<T>(rh[r].bl, n, 1, rh[r].bl, n, partial, nblocks, hslot(r), 0, st);
  }
  fetch();
  std::vector<int> live;
  for (int r = 0; r < R; ++r) {
    rh[r].nb = std::sqrt(std::max(0.0, hh[(size_t)r * HS].x));
    if (rh[r].nb == 0) {
      rh[r].done = true;
      hip_check(hipMemsetAsync(static_cast<char*>(x_c) + (size_t)r * n * es, 0, n * es, st), "hipMemsetAsync");
    } else {
      live.push_back(r);
    }
  }
  residuals(live);
  if (!live.empty() && live[0] == 0 && history && nh < hist_len) history[nh] = rh[0].beta / rh[0].nb;
  if (!live.empty() && live[0] == 0) ++nh;
  for (int r : live) {
    if (rh[r].beta / rh[r].nb <= prm.tol || prm.max_iters <= 0)
      rh[r].done = true;
    else
      start_cycle(r);
  }
  int status = NESA_OK;
  for (;;) {
    std::vector<int> act;
    for (int r = 0; r < R; ++r)
      if (!rh[r].done) act.push_back(r);
    if (act.empty()) break;
    // one Arnoldi step for every active right-hand side: the basis vectors
    // (preconditioned together when every active one uses the Schwarz base)
    // go through one product
    std::vector<const void*> src;
    std::vector<void*> dst;
    bool all_schwarz = flex;
    for (int r : act) all_schwarz = all_schwarz && rh[r].active == NESA_PRECOND_SCHWARZ;
    for (size_t i = 0; i < act.size(); ++i) {
      Rhs& q = rh[act[i]];
      const void* v = vec(q.V, q.j);
      if (flex && !all_schwarz) {
        precond(q, v, vec(q.Z, q.j));
        v = vec(q.Z, q.j);
      }
      hip_check(hipMemcpyAsync(slot(Xb, (int)i), v, n * es, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
      src.push_back(slot(Xb, (int)i));
      dst.push_back(slot(Yb, (int)i));
    }
    if (all_schwarz) {
      nesa::launch_near_apply<T>(d, op->schwarz, Xb, Pb, st, R);
      for (size_t i = 0; i < act.size(); ++i) {
        Rhs& q = rh[act[i]];
        hip_check(hipMemcpyAsync(vec(q.Z, q.j), slot(Pb, (int)i), n * es, hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync");
        hip_check(hipMemcpyAsync(slot(Xb, (int)i), slot(Pb, (int)i), n * es, hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync");
      }
    }
    batched_matvec(src, dst);
    for (size_t i = 0; i < act.size(); ++i) {
      Rhs& q = rh[act[i]];
      void* w = slot(Yb, (int)i);
      double2* h = hslot(act[i]);
      // two passes of classical Gram-Schmidt, FP64 dot products
      nesa::launch_multidot<T>(q.V, n, q.j + 1, w, n, partial, nblocks, h, 0, st);
      nesa::launch_combine<T>(q.V, n, q.j + 1, h, w, n, -1.0, st);
      nesa::launch_multidot<T>(q.V, n, q.j + 1, w, n, partial, nblocks, h + (m + 2), 0, st);
      nesa::launch_combine<T>(q.V, n, q.j + 1, h + (m + 2), w, n, -1.0, st);
      nesa::launch_multidot<T>(w, n, 1, w, n, partial, nblocks, h + 2 * (m + 2), 0, st);
    }
    fetch();
    std::vector<int> ended;
    for (size_t i = 0; i < act.size(); ++i) {
      const int r = act[i];
      Rhs& q = rh[r];
      const double2* hr = hh + (size_t)r * HS;
      const int j = q.j;
      cd* Hj = &q.H[(size_t)j * (m + 1)];
      for (int k = 0; k <= j; ++k) Hj[k] = cd(hr[k].x + hr[m + 2 + k].x, hr[k].y + hr[m + 2 + k].y);
      const double hn = std::sqrt(std::max(0.0, hr[2 * (m + 2)].x));
      bool finite = std::isfinite(hn);
      for (int k = 0; k <= j && finite; ++k) finite = std::isfinite(std::abs(Hj[k]));
      if (!finite) {
        if (q.active == NESA_PRECOND_LEARNED) {
          q.active = op->mlp->base;
          rep[r].fell_back = 1;
          q.discard = true;
          ended.push_back(r);
          continue;
        }
        status = fail(NESA_EBREAKDOWN, "non-finite value in GMRES");
        q.done = true;
        continue;
      }
      Hj[j + 1] = hn;
      for (int k = 0; k < j; ++k) {
        cd t0v = q.cs[k] * Hj[k] + q.sn[k] * Hj[k + 1];
        Hj[k + 1] = -std::conj(q.sn[k]) * Hj[k] + q.cs[k] * Hj[k + 1];
        Hj[k] = t0v;
      }
      cd a = Hj[j], bb = Hj[j + 1];
      double c;
      cd sv, rr;
      if (bb == cd(0, 0)) {
        c = 1;
        sv = 0;
        rr = a;
      } else if (a == cd(0, 0)) {
        c = 0;
        sv = 1;
        rr = bb;
      } else {
        const double rho = std::hypot(std::abs(a), std::abs(bb));
        c = std::abs(a) / rho;
        sv = a * std::conj(bb) / (std::abs(a) * rho);
        rr = a * rho / std::abs(a);
      }
      q.cs[j] = c;
      q.sn[j] = sv;
      Hj[j] = rr;
      Hj[j + 1] = 0;
      q.g[j + 1] = -std::conj(sv) * q.g[j];
      q.g[j] = c * q.g[j];
      ++q.iters;
      if (r == 0) {
        if (history && nh < hist_len) history[nh] = std::abs(q.g[j + 1]) / q.nb;
        ++nh;
      }
      q.j = j + 1;
      if (std::abs(q.g[j + 1]) / q.nb <= prm.tol || q.iters >= prm.max_iters || hn == 0 || q.j == m) {
        ended.push_back(r);
      } else {
        nesa::launch_scale<T>(slot(Yb, (int)i), vec(q.V, q.j), n, 1.0 / hn, st);
      }
    }
    if (status != NESA_OK) break;
    if (ended.empty()) continue;
    // close the cycles: x += Z y (or V y), then the true residuals in one product
    std::vector<int> upd;
    for (int r : ended) {
      Rhs& q = rh[r];
      if (q.discard) continue;
      const int k = q.j;
      std::vector<cd> y(k);
      for (int i2 = k - 1; i2 >= 0; --i2) {
        cd acc = q.g[i2];
        for (int c2 = i2 + 1; c2 < k; ++c2) acc -= q.H[(size_t)c2 * (m + 1) + i2] * y[c2];
        y[i2] = acc / q.H[(size_t)i2 * (m + 1) + i2];
      }
      double2* yh = hh + (size_t)r * HS;
      for (int i2 = 0; i2 < k; ++i2) yh[i2] = make_double2(y[i2].real(), y[i2].imag());
      hip_check(hipMemcpyAsync(hslot(r), yh, sizeof(double2) * k, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      nesa::launch_combine<T>(flex ? q.Z : q.V, n, k, hslot(r), q.xl, n, +1.0, st);
      upd.push_back(r);
    }
    residuals(upd);
    for (int r : ended) {
      Rhs& q = rh[r];
      if (q.discard) {                        // restart from the same x with the base preconditioner
        nesa::launch_sub<T>(q.bl, q.ax, vec(q.V, 0), n, st);
        start_cycle(r);
        continue;
      }
      const double ratio = prm.fallback_ratio > 0 ? prm.fallback_ratio : 1.0;
      if (q.active == NESA_PRECOND_LEARNED && !(q.beta < ratio * q.beta_prev)) {
        q.active = op->mlp->base;
        rep[r].fell_back = 1;
      }
      if (q.beta / q.nb <= prm.tol || q.iters >= prm.max_iters)
        q.done = true;
      else
        start_cycle(r);
    }
  }
  int worst = status;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < R; ++r) {
    char* xr = static_cast<char*>(x_c) + (size_t)r * n * es;
    if (rh[r].nb != 0) nesa::launch_scatter<T>(rh[r].xl, xr, d.perm, n, st);
    rep[r].iters = rh[r].iters;
    rep[r].true_rel_residual = rh[r].nb != 0 ? rh[r].beta / rh[r].nb : 0.0;
    rep[r].seconds = secs;
    if (worst == NESA_OK && rh[r].nb != 0 && rep[r].true_rel_residual > prm.tol)
      worst = fail(NESA_ENOCONV, "GMRES reached max_iters above tolerance");
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  for (int r = 0; r < R; ++r) rep[r].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return worst;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* nesa_last_error(void) { return g_err.c_str(); }

int nesa_build_tree(const double* verts, int64_t nv, const int32_t* tris, int64_t nt,
                    const nesa_tree_params* params, nesa_tree** out) {
  return guarded([&]() {
    if (!verts || !tris || !params || !out) return fail(NESA_EINVAL, "null argument");
    std::unique_ptr<nesa_tree> h(new nesa_tree());
    h->t.reset(nesa::build_tree(verts, nv, tris, nt, params->leaf_size, params->l0_max, params->buffer));
    *out = h.release();
    return (int)NESA_OK;
  });
}

int nesa_build_forest(int nbodies, const double* const* verts, const int64_t* nv, const int32_t* const* tris,
                      const int64_t* nt, const nesa_tree_params* params, nesa_tree** out) {
  return guarded([&]() {
    if (nbodies < 1 || !verts || !nv || !tris || !nt || !params || !out) return fail(NESA_EINVAL, "null argument");
    for (int i = 0; i < nbodies; ++i)
      if (!verts[i] || !tris[i]) return fail(NESA_EINVAL, "null argument");
    std::unique_ptr<nesa_tree> h(new nesa_tree());
    h->t.reset(nesa::build_forest(nbodies, verts, nv, tris, nt, params->leaf_size, params->l0_max, params->buffer));
    *out = h.release();
    return (int)NESA_OK;
  });
}

int nesa_tree_bodies(const nesa_tree* tree, int64_t* rwg_ptr, int nmax, int* nbodies) {
  return guarded([&]() {
    if (!tree || !nbodies) return fail(NESA_EINVAL, "null argument");
    const auto& br = tree->t->body_rwg;
    const int nb = br.empty() ? 1 : (int)br.size() - 1;
    *nbodies = nb;
    if (rwg_ptr) {
      for (int i = 0; i <= nb && i < nmax; ++i) rwg_ptr[i] = br.empty() ? (i == 0 ? 0 : tree->t->rwg.n) : br[i];
    }
    return (int)NESA_OK;
  });
}

int nesa_tree_get_info(const nesa_tree* tree, nesa_tree_info* info) {
  return guarded([&]() {
    if (!tree || !info) return fail(NESA_EINVAL, "null argument");
    const nesa::Tree& t = *tree->t;
    std::memset(info, 0, sizeof(*info));
    info->n_rwg = t.rwg.n;
    info->n_tri = t.rwg.nt;
    info->L = t.L;
    info->l0 = t.l0;
    int64_t ne = 0, nh = 0, nt = 0;
    const auto& LL = t.level(t.L);
    for (int64_t a = 0; a < LL.nbox; ++a) {
      int64_t S = t.leaf_ptr[a + 1] - t.leaf_ptr[a], W = 0, Wh = 0;
      for (int64_t j = t.near_ptr[a]; j < t.near_ptr[a + 1]; ++j) {
        const int64_t b = t.near_idx[j], Sb = t.leaf_ptr[b + 1] - t.leaf_ptr[b];
        W += Sb;
        if (b >= a) Wh += Sb;
      }
      ne += S * W;
      nh += S * Wh;
      nt += Wh - S;
    }
    info->near_entries = ne;
    info->near_entries_half = nh;
    info->near_transposed = nt;
    info->max_leaf = max_leaf(t);
    for (int l = t.l0; l <= t.L && l - t.l0 < 32; ++l) {
      info->n_box[l - t.l0] = t.level(l).nbox;
      info->n_pairs[l - t.l0] = (int64_t)t.level(l).il_src.size();
    }
    return (int)NESA_OK;
  });
}

int nesa_tree_perm(const nesa_tree* tree, int64_t* perm) {
  return guarded([&]() {
    if (!tree || !perm) return fail(NESA_EINVAL, "null argument");
    std::copy(tree->t->perm.begin(), tree->t->perm.end(), perm);
    return (int)NESA_OK;
  });
}

int nesa_tree_leaf_sizes(const nesa_tree* tree, int64_t* S, int64_t* W) {
  return guarded([&]() {
    if (!tree) return fail(NESA_EINVAL, "null argument");
    const nesa::Tree& t = *tree->t;
    const int64_t nleaf = t.level(t.L).nbox;
    for (int64_t a = 0; a < nleaf; ++a) {
      if (S) S[a] = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      if (W) {
        int64_t w = 0;
        for (int64_t q = t.near_ptr[a]; q < t.near_ptr[a + 1]; ++q)
          w += t.leaf_ptr[t.near_idx[q] + 1] - t.leaf_ptr[t.near_idx[q]];
        W[a] = w;
      }
    }
    return (int)NESA_OK;
  });
}

void nesa_tree_free(nesa_tree* tree) { delete tree; }

int nesa_assemble_near(const nesa_tree* tree, const nesa_em_params* em, nesa_near** out) {
  return guarded([&]() {
    if (!tree || !em || !out) return fail(NESA_EINVAL, "null argument");
    if (!(em->k > 0) || !(em->eta > 0)) return fail(NESA_EINVAL, "k and eta must be positive");
    std::unique_ptr<nesa_near> h(new nesa_near());
    h->n.reset(nesa::assemble_near(*tree->t, em->k, em->eta));
    *out = h.release();
    return (int)NESA_OK;
  });
}

int nesa_assemble_near_device(const nesa_tree* tree, const nesa_em_params* em, nesa_near** out) {
  return guarded([&]() {
    if (!tree || !em || !out) return fail(NESA_EINVAL, "null argument");
    if (!(em->k > 0) || !(em->eta > 0)) return fail(NESA_EINVAL, "k and eta must be positive");
    std::unique_ptr<nesa_near> h(new nesa_near());
    h->n.reset(nesa::assemble_near_device(*tree->t, em->k, em->eta));
    *out = h.release();
    return (int)NESA_OK;
  });
}

int nesa_near_entries(const nesa_tree* tree, const nesa_near* near, const int64_t* rows, int64_t nrows,
                      const int64_t* cols, int64_t ncols, double* out) {
  return guarded([&]() {
    if (!tree || !near || !rows || !cols || !out) return fail(NESA_EINVAL, "null argument");
    const nesa::Tree& t = *tree->t;
    const nesa::Near& nr = *near->n;
    const int64_t n = t.rwg.n;
    // leaf of each leaf-order position
    std::vector<int64_t> leaf_of(n);
    const auto& LL = t.level(t.L);
    for (int64_t a = 0; a < LL.nbox; ++a)
      for (int64_t p = t.leaf_ptr[a]; p < t.leaf_ptr[a + 1]; ++p) leaf_of[p] = a;
    for (int64_t i = 0; i < nrows; ++i) {
      if (rows[i] < 0 || rows[i] >= n) return fail(NESA_EINVAL, "row index out of range");
      const int64_t pr = t.pos[rows[i]], a = leaf_of[pr], S = t.leaf_ptr[a + 1] - t.leaf_ptr[a];
      const int64_t ri = pr - t.leaf_ptr[a];
      for (int64_t j = 0; j < ncols; ++j) {
        if (cols[j] < 0 || cols[j] >= n) return fail(NESA_EINVAL, "column index out of range");
        const int64_t pc = t.pos[cols[j]], b = leaf_of[pc];
        cd v(0, 0);
        int64_t c0 = 0;
        for (int64_t q = t.near_ptr[a]; q < t.near_ptr[a + 1]; ++q) {
          const int64_t bb = t.near_idx[q];
          if (bb == b) {
            v = nr.z[nr.off[a] + (c0 + pc - t.leaf_ptr[b]) * S + ri];
            break;
          }
          c0 += t.leaf_ptr[bb + 1] - t.leaf_ptr[bb];
        }
        out[2 * (i * ncols + j)] = v.real();
        out[2 * (i * ncols + j) + 1] = v.imag();
      }
    }
    return (int)NESA_OK;
  });
}

void nesa_near_free(nesa_near* near) { delete near; }

int nesa_assemble_translations(const nesa_tree* tree, const nesa_em_params* em, const nesa_far_params* params,
                               nesa_far** out) {
  return guarded([&]() {
    if (!tree || !em || !params || !out) return fail(NESA_EINVAL, "null argument");
    if (!(em->k > 0) || !(em->eta > 0)) return fail(NESA_EINVAL, "k and eta must be positive");
    std::unique_ptr<nesa_far> h(new nesa_far());
    h->f.reset(nesa::assemble_far(*tree->t, em->k, em->eta, params->d0, params->q_min, params->tau,
                                          params->eps));
    *out = h.release();
    return (int)NESA_OK;
  });
}

int nesa_far_get_q(const nesa_far* far, int* Q, int nmax) {
  return guarded([&]() {
    if (!far || !Q) return fail(NESA_EINVAL, "null argument");
    for (int i = 0; i < nmax && i < (int)far->f->lev.size(); ++i) Q[i] = far->f->lev[i].Q;
    return (int)NESA_OK;
  });
}

void nesa_far_free(nesa_far* far) { delete far; }

int nesa_op_create(const nesa_tree* tree, const nesa_near* near, const nesa_far* far, int precision, int max_nrhs,
                   nesa_op** out) {
  return guarded([&]() {
    if (!tree || !near || !far || !out) return fail(NESA_EINVAL, "null argument");
    if (precision != NESA_C128 && precision != NESA_C64 && !is_split(precision))
      return fail(NESA_EINVAL, "unknown precision");
    if (max_nrhs < 1) return fail(NESA_EINVAL, "max_nrhs must be >= 1");
    std::unique_ptr<nesa_op> op(new nesa_op());
    op->precision = precision;
    op->max_nrhs = max_nrhs;
    if (max_nrhs > 1024) return fail(NESA_EINVAL, "max_nrhs above 1024");
    op->k = far->f->k;
    op->eta = far->f->eta;
    op->geo.rwg = tree->t->rwg;
    op->tree = tree->t.get();
    op->near = near->n.get();
    if (precision == NESA_C128) {
      op->esize = 16;
      build_dev<double>(op.get(), op->d, *tree->t, *near->n, *far->f);
    } else {
      op->esize = 8;
      build_dev<float>(op.get(), op->f, *tree->t, *near->n, *far->f);
    }
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    *out = op.release();
    return (int)NESA_OK;
  });
}

void nesa_op_free(nesa_op* op) {
  if (op) (void)hipDeviceSynchronize();
  delete op;
}

static int matvec_impl(nesa_op* op, const void* x, void* y, int64_t nrhs, void* stream, bool canonical) {
  return guarded([&]() {
    if (!op || !x || !y) return fail(NESA_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(NESA_EINVAL, "nrhs out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (op->precision == NESA_C128) {
      const int64_t n = op->d.n;
      for (int64_t r = 0; r < nrhs; ++r) {
        const char* xr = static_cast<const char*>(x) + (size_t)r * n * op->esize;
        char* yr = static_cast<char*>(y) + (size_t)r * n * op->esize;
        if (canonical) {
          nesa::launch_gather<double>(xr, op->xl, op->d.perm, n, st);
          nesa::launch_matvec_leaf<double>(op->d, op->xl, op->yl, 1, st, nullptr);
          nesa::launch_scatter<double>(op->yl, yr, op->d.perm, n, st);
        } else {
          nesa::launch_matvec_leaf<double>(op->d, xr, yr, 1, st, nullptr);
        }
      }
    } else {
      const int64_t n = op->f.n;
      ensure_all_tiles<float>(op, op->f, (int)nrhs, st);
      if (canonical) {
        for (int64_t r = 0; r < nrhs; ++r)
          nesa::launch_gather<float>(static_cast<const char*>(x) + (size_t)r * n * 8,
                                     static_cast<char*>(op->xl) + (size_t)r * n * 8, op->f.perm, n, st);
        nesa::launch_matvec_leaf<float>(op->f, op->xl, op->yl, (int)nrhs, st, nullptr);
        for (int64_t r = 0; r < nrhs; ++r)
          nesa::launch_scatter<float>(static_cast<const char*>(op->yl) + (size_t)r * n * 8,
                                      static_cast<char*>(y) + (size_t)r * n * 8, op->f.perm, n, st);
      } else {
        nesa::launch_matvec_leaf<float>(op->f, x, y, (int)nrhs, st, nullptr);
      }
    }
    hip_check(hipGetLastError(), "kernel launch");
    return (int)NESA_OK;
  });
}

// worker streams of nesa_matvec_batched (default priority, non-blocking),
// created once per device and kept until the process ends
static std::mutex g_batch_mu;
static std::map<int, std::vector<hipStream_t>> g_batch_streams;
static std::map<int, std::vector<hipEvent_t>> g_batch_events;     // fork, then one join per worker
static constexpr int BATCH_STREAMS = 4;

int nesa_matvec_batched(nesa_op* const* ops, int n_ops, const void* const* x_dev, void* const* y_dev,
                        const int64_t* nrhs, void* stream) {
  return guarded([&]() {
    if (n_ops < 0 || (n_ops > 0 && (!ops || !x_dev || !y_dev || !nrhs))) return fail(NESA_EINVAL, "null argument");
    for (int i = 0; i < n_ops; ++i) {
      if (!ops[i] || !x_dev[i] || !y_dev[i]) return fail(NESA_EINVAL, "null operator or vector");
      if (nrhs[i] < 1 || nrhs[i] > ops[i]->max_nrhs) return fail(NESA_EINVAL, "nrhs out of range");
      for (int j = 0; j < i; ++j)
        if (ops[j] == ops[i]) return fail(NESA_EINVAL, "an operator appears twice (its work buffers would race)");
    }
    if (n_ops == 0) return (int)NESA_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_ops == 1) return matvec_impl(ops[0], x_dev[0], y_dev[0], nrhs[0], stream, true);
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(g_batch_mu);      // one batched call at a time per process
    auto& ws = g_batch_streams[dev];
    auto& ev = g_batch_events[dev];
    while ((int)ws.size() < BATCH_STREAMS) {
      hipStream_t s2 = nullptr;
      hip_check(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking), "hipStreamCreateWithFlags");
      ws.push_back(s2);
    }
    while ((int)ev.size() < BATCH_STREAMS + 1) {
      hipEvent_t e = nullptr;
      hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
      ev.push_back(e);
    }
    // fork: every worker stream waits for the work queued on `stream`; the
    // products of different operators (independent buffers) then run side by
    // side, operator i on worker i mod BATCH_STREAMS; join back into `stream`
    hip_check(hipEventRecord(ev[0], st), "hipEventRecord");
    const int nw = std::min(n_ops, BATCH_STREAMS);
    for (int k = 0; k < nw; ++k) hip_check(hipStreamWaitEvent(ws[k], ev[0], 0), "hipStreamWaitEvent");
    int rc = NESA_OK;
    for (int i = 0; i < n_ops && rc == NESA_OK; ++i)
      rc = matvec_impl(ops[i], x_dev[i], y_dev[i], nrhs[i], ws[i % BATCH_STREAMS], true);
    for (int k = 0; k < nw; ++k) {
      hip_check(hipEventRecord(ev[k + 1], ws[k]), "hipEventRecord");
      hip_check(hipStreamWaitEvent(st, ev[k + 1], 0), "hipStreamWaitEvent");
    }
    return rc;
  });
}

int nesa_matvec(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream) {
  return matvec_impl(op, x_dev, y_dev, nrhs, stream, true);
}
int nesa_matvec_leaf(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream) {
  return matvec_impl(op, x_dev, y_dev, nrhs, stream, false);
}

int nesa_residual_error(nesa_op* op, const void* b_dev, const void* xs_dev, const void* x_dev, void* r_dev,
                        void* e_dev, void* stream) {
  const int rc = matvec_impl(op, x_dev, r_dev, 1, stream, true);
  if (rc != NESA_OK) return rc;
  return guarded([&]() {
    if (!b_dev || !xs_dev || !e_dev) return fail(NESA_EINVAL, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = op->geo.rwg.n;
    if (op->precision == NESA_C128) {
      nesa::launch_sub<double>(b_dev, r_dev, r_dev, n, st);
      nesa::launch_sub<double>(xs_dev, x_dev, e_dev, n, st);
    } else {
      nesa::launch_sub<float>(b_dev, r_dev, r_dev, n, st);
      nesa::launch_sub<float>(xs_dev, x_dev, e_dev, n, st);
    }
    hip_check(hipGetLastError(), "kernel launch");
    return (int)NESA_OK;
  });
}

static void timed_matvec(nesa_op* op, const void* x_dev, void* y_dev, hipStream_t st, nesa::PhaseTimer& tm,
                         int nrhs = 1) {
  for (auto& e : tm.ev) hip_check(hipEventCreate(&e), "hipEventCreate");
  if (op->precision == NESA_C128)
    nesa::launch_matvec_leaf<double>(op->d, x_dev, y_dev, 1, st, &tm);
  else
    nesa::launch_matvec_leaf<float>(op->f, x_dev, y_dev, nrhs, st, &tm);
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipEventSynchronize(tm.ev[tm.n - 1]), "hipEventSynchronize");
}

int nesa_matvec_phase_times(nesa_op* op, const void* x_dev, void* y_dev, void* stream, float* ms) {
  return guarded([&]() {
    if (!op || !x_dev || !y_dev || !ms) return fail(NESA_EINVAL, "null argument");
    nesa::PhaseTimer tm;
    timed_matvec(op, x_dev, y_dev, static_cast<hipStream_t>(stream), tm);
    for (int i = 0; i + 1 < nesa::PhaseTimer::NMARK; ++i)
      hip_check(hipEventElapsedTime(&ms[i], tm.ev[tm.phase_ev[i]], tm.ev[tm.phase_ev[i + 1]]),
                "hipEventElapsedTime");
    for (auto& e : tm.ev) (void)hipEventDestroy(e);
    return (int)NESA_OK;
  });
}

int nesa_matvec_launch_times(nesa_op* op, const void* x_dev, void* y_dev, void* stream, float* ms,
                             int32_t* kind, int32_t* level, int32_t max_launches, int32_t* count) {
  return nesa_matvec_launch_times_nrhs(op, x_dev, y_dev, 1, stream, ms, kind, level, max_launches, count);
}

int nesa_matvec_launch_times_nrhs(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream,
                                  float* ms, int32_t* kind, int32_t* level, int32_t max_launches, int32_t* count) {
  return guarded([&]() {
    if (!op || !x_dev || !y_dev || !ms || !kind || !level || !count) return fail(NESA_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(NESA_EINVAL, "nrhs out of range");
    if (nrhs > 1 && op->precision == NESA_C128) return fail(NESA_EINVAL, "complex128 products take one right-hand side");
    if (op->precision != NESA_C128 && nrhs > 1) ensure_all_tiles<float>(op, op->f, (int)nrhs, static_cast<hipStream_t>(stream));
    nesa::PhaseTimer tm;
    tm.overlap = true;       // the launches as the untimed product runs them
    timed_matvec(op, x_dev, y_dev, static_cast<hipStream_t>(stream), tm, (int)nrhs);
    int c = 0;
    for (int i = 1; i < tm.n && c < max_launches; ++i) {
      if (tm.kind[i] == 0) continue;
      hip_check(hipEventElapsedTime(&ms[c], tm.ev[i - 1], tm.ev[i]), "hipEventElapsedTime");
      kind[c] = tm.kind[i];
      level[c] = tm.level[i];
      ++c;
    }
    *count = c;
    for (auto& e : tm.ev) (void)hipEventDestroy(e);
    return (int)NESA_OK;
  });
}

int nesa_rhs_plane_wave_host(const nesa_tree* tree, double k, const double* khat, const double* pol,
                             int64_t nrhs, double* b) {
  return guarded([&]() {
    if (!tree || !khat || !pol || !b) return fail(NESA_EINVAL, "null argument");
    const int64_t n = tree->t->rwg.n;
    for (int64_t r = 0; r < nrhs; ++r)
      nesa::plane_wave_rhs(*tree->t, k, khat + 3 * r, pol + 3 * r, reinterpret_cast<cd*>(b) + r * n);
    return (int)NESA_OK;
  });
}

int nesa_rhs_plane_wave(nesa_op* op, const double* khat, const double* pol, int64_t nrhs, void* b_dev,
                        void* stream) {
  return guarded([&]() {
    if (!op || !khat || !pol || !b_dev) return fail(NESA_EINVAL, "null argument");
    if (nrhs < 1) return fail(NESA_EINVAL, "nrhs must be >= 1");
    const int64_t n = op->geo.rwg.n;
    std::vector<cd> b((size_t)n * nrhs);
    for (int64_t r = 0; r < nrhs; ++r) nesa::plane_wave_rhs(op->geo, op->k, khat + 3 * r, pol + 3 * r, &b[r * n]);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (op->precision == NESA_C128) {
      hip_check(hipMemcpyAsync(b_dev, b.data(), b.size() * 16, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    } else {
      std::vector<float> bf(2 * b.size());
      for (size_t i = 0; i < b.size(); ++i) {
        bf[2 * i] = (float)b[i].real();
        bf[2 * i + 1] = (float)b[i].imag();
      }
      hip_check(hipMemcpyAsync(b_dev, bf.data(), bf.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    }
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return (int)NESA_OK;
  });
}

int nesa_precond_setup(nesa_op* op, int precond) {
  return guarded([&]() {
    if (!op) return fail(NESA_EINVAL, "null argument");
    if (precond == NESA_PRECOND_SCHWARZ) ensure_schwarz(op);
    return (int)NESA_OK;
  });
}

int nesa_precond_apply(nesa_op* op, int precond, const void* r_dev, void* z_dev, void* stream) {
  return guarded([&]() {
    if (!op || !r_dev || !z_dev) return fail(NESA_EINVAL, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precond == NESA_PRECOND_SCHWARZ) {
      ensure_schwarz(op);
      if (op->precision == NESA_C128)
        nesa::launch_near_apply<double>(op->d, op->schwarz, r_dev, z_dev, st);
      else
        nesa::launch_near_apply<float>(op->f, op->schwarz, r_dev, z_dev, st);
    } else if (precond == NESA_PRECOND_BLOCKDIAG) {
      if (op->precision == NESA_C128)
        nesa::launch_blockdiag<double>(op->d, r_dev, z_dev, st);
      else
        nesa::launch_blockdiag<float>(op->f, r_dev, z_dev, st);
    } else {
      return fail(NESA_EINVAL, "preconditioner cannot be applied on its own");
    }
    hip_check(hipGetLastError(), "kernel launch");
    return (int)NESA_OK;
  });
}

int nesa_gmres_solve(nesa_op* op, const void* b_dev, void* x_dev, int64_t nrhs, const nesa_gmres_params* params,
                     nesa_gmres_report* report, double* history, int64_t history_len, void* stream) {
  return guarded([&]() {
    if (!op || !b_dev || !x_dev || !params || !report) return fail(NESA_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(NESA_EINVAL, "nrhs out of range");
    if (params->restart < 1 || params->restart > 250 || params->max_iters < 1 || !(params->tol > 0) ||
        !(params->fallback_ratio >= 0 && params->fallback_ratio <= 1))
      return fail(NESA_EINVAL, "bad GMRES parameters");
    if (params->precond < 0 || params->precond > 3) return fail(NESA_EINVAL, "unknown preconditioner");
    if (params->precond == NESA_PRECOND_SCHWARZ) ensure_schwarz(op);
    if (params->precond == NESA_PRECOND_LEARNED && !op->mlp)
      return fail(NESA_EINVAL, "no network attached for the learned preconditioner");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = op->geo.rwg.n;
    if (op->precision != NESA_C128 && nrhs > 1)
      return gmres_batch(op, op->f, b_dev, x_dev, (int)nrhs, *params, report, history, history_len, st);
    int worst = NESA_OK;
    for (int64_t r = 0; r < nrhs; ++r) {
      const char* br = static_cast<const char*>(b_dev) + (size_t)r * n * op->esize;
      char* xr = static_cast<char*>(x_dev) + (size_t)r * n * op->esize;
      int rc;
      if (op->precision == NESA_C128)
        rc = gmres_one<double>(op, op->d, br, xr, *params, report[r], r == 0 ? history : nullptr, history_len, st);
      else
        rc = gmres_one<float>(op, op->f, br, xr, *params, report[r], r == 0 ? history : nullptr, history_len, st);
      if (rc != NESA_OK && worst == NESA_OK) worst = rc;
    }
    return worst;
  });
}

// ------------------------------------------------------------------ GMRES without allocation
// Workspace of nesa_gmres_solve_noalloc: a fixed array in device memory (each
// device holds its own copy from library load to process end).  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, kept per device; the array's own name is a host-side stand-in.
static __device__ __align__(256) unsigned char scratch[NESA_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};
// host scalars of the solve (FP64 coefficients read back every iteration)
static thread_local double2 g_noalloc_host[2 * (250 + 2) + 2];

static char* scratch_for_current_device() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) throw Error(NESA_EINVAL, "device index above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (!p) throw Error(NESA_EHIP, "no device address for the GMRES scratch array");
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

int nesa_gmres_solve_noalloc(nesa_op* op, const void* b_dev, void* x_dev, int64_t nrhs,
                             const nesa_gmres_params* params, nesa_gmres_report* report, double* history,
                             int64_t history_len, void* stream) {
  return guarded([&]() {
    if (!op || !b_dev || !x_dev || !params || !report) return fail(NESA_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(NESA_EINVAL, "nrhs out of range");
    if (params->restart < 1 || params->restart > 250 || params->max_iters < 1 || !(params->tol > 0) ||
        !(params->fallback_ratio >= 0 && params->fallback_ratio <= 1))
      return fail(NESA_EINVAL, "bad GMRES parameters");
    if (params->precond < 0 || params->precond > 3) return fail(NESA_EINVAL, "unknown preconditioner");
    // preconditioners are built by nesa_precond_setup / nesa_op_set_mlp, which allocate
    if (params->precond == NESA_PRECOND_SCHWARZ && !op->schwarz)
      return fail(NESA_EINVAL, "Schwarz preconditioner not set up (call nesa_precond_setup first)");
    if (params->precond == NESA_PRECOND_LEARNED && !op->mlp)
      return fail(NESA_EINVAL, "no network attached for the learned preconditioner");
    const int64_t n = op->geo.rwg.n;
    const bool flex = params->precond != NESA_PRECOND_NONE;
    const size_t need = gmres_workspace_bytes(n, params->restart, flex, op->esize);
    if (need > NESA_NOALLOC_SCRATCH_BYTES)
      return fail(NESA_EINVAL, "GMRES workspace of " + std::to_string(need) + " bytes exceeds the " +
                                   std::to_string((size_t)NESA_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    char* ws = scratch_for_current_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    int worst = NESA_OK;
    // right-hand sides one after another, each through the same workspace
    for (int64_t r = 0; r < nrhs; ++r) {
      const char* br = static_cast<const char*>(b_dev) + (size_t)r * n * op->esize;
      char* xr = static_cast<char*>(x_dev) + (size_t)r * n * op->esize;
      int rc;
      if (op->precision == NESA_C128)
        rc = gmres_one<double>(op, op->d, br, xr, *params, report[r], r == 0 ? history : nullptr, history_len, st,
                               ws, g_noalloc_host);
      else
        rc = gmres_one<float>(op, op->f, br, xr, *params, report[r], r == 0 ? history : nullptr, history_len, st,
                              ws, g_noalloc_host);
      if (rc != NESA_OK && worst == NESA_OK) worst = rc;
    }
    return worst;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ learned preconditioner API
static void check_mlp_params(const nesa_mlp_params* p) {
  if (p->s_max < 32 || p->s_max > 512 || p->s_max % 32)
    throw Error(NESA_EINVAL, "s_max must be a multiple of 32 in [32, 512]");
  if (p->hidden < 64 || p->hidden > 512 || p->hidden % 64)
    throw Error(NESA_EINVAL, "hidden must be a multiple of 64 in [64, 512]");
  if (p->base != NESA_PRECOND_BLOCKDIAG && p->base != NESA_PRECOND_SCHWARZ)
    throw Error(NESA_EINVAL, "base must be BLOCKDIAG or SCHWARZ");
}

static void mlp_upload_params(nesa_mlp* h, const float* theta) {
  nesa::MlpDev& N = h->net;
  hip_check(hipMemcpy(N.theta, theta, N.np * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  std::vector<float> zero(N.np, 0.f);
  hip_check(hipMemcpy(N.m, zero.data(), N.np * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  hip_check(hipMemcpy(N.v, zero.data(), N.np * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  h->t = 0;
  nesa::launch_mlp_refresh(N, nullptr);
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
}

static void require_data(const nesa_mlp* h) {
  if (h->nsamples == 0) throw Error(NESA_EINVAL, "no training data set");
  if (h->nvalid == 0) throw Error(NESA_EINVAL, "training data has no leaf with a non-zero base output");
}

// forward (+ loss, + backward) over the training rows; returns the mean loss
static double mlp_pass(nesa_mlp* h, bool backward, hipStream_t st) {
  require_data(h);
  nesa::launch_mlp_forward(h->net, h->trn, true, st);
  nesa::launch_mlp_loss(h->net, h->trn, st);
  if (backward) nesa::launch_mlp_backward(h->net, h->trn, (float)(1.0 / (double)h->nvalid), st);
  hip_check(hipGetLastError(), "kernel launch");
  double loss = 0;
  hip_check(hipMemcpyAsync(&loss, h->net.loss, sizeof(double), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  return loss / (double)h->nvalid;
}

template <typename T>
static void mlp_set_data_t(nesa_mlp* h, nesa::DevOp<T>& d, const void* r, const void* e, int64_t ns,
                           hipStream_t st) {
  const int64_t n = d.n;
  const size_t es = 2 * sizeof(T);
  if (ns > h->trn_cap) {
    for (void* p : h->trn_allocs) (void)hipFree(p);
    h->trn_allocs.clear();
    h->trn_cap = 0;
    h->trn_vec = net_alloc<char>(h->trn_allocs, (int64_t)3 * ns * n * es);
    alloc_rows(h->trn_allocs, h->trn, h->net.S, h->net.H, ns * d.nleaf, true);
    h->net.partial_elems = nesa::mlp_partial_elems(h->net.S, h->net.H, h->trn.rows_pad);
    h->net.partial = net_alloc<float>(h->trn_allocs, h->net.partial_elems);
    h->net.loss_blocks = h->trn.rows_pad / 4;
    h->net.loss_part = net_alloc<double>(h->trn_allocs, h->net.loss_blocks);
    h->trn_cap = ns;
  } else {
    // rows of a smaller set inside the same buffers: keep rows_pad of the
    // allocation, the extra rows are masked by rowS = 0
    h->trn.rows = ns * d.nleaf;
  }
  char* rl = static_cast<char*>(h->trn_vec);
  char* el = rl + (size_t)h->trn_cap * n * es;
  char* bl = el + (size_t)h->trn_cap * n * es;
  for (int64_t s = 0; s < ns; ++s) {
    nesa::launch_gather<T>(static_cast<const char*>(r) + s * n * es, rl + s * n * es, d.perm, n, st);
    nesa::launch_gather<T>(static_cast<const char*>(e) + s * n * es, el + s * n * es, d.perm, n, st);
    base_apply<T>(h->op, d, h->base, rl + s * n * es, bl + s * n * es, st);
  }
  nesa::launch_mlp_features<T>(h->net, h->trn, rl, bl, el, d.leaf_ptr, d.nleaf, n, ns, true, st);
  hip_check(hipGetLastError(), "kernel launch");
  std::vector<int32_t> rowS(h->trn.rows_pad);
  hip_check(hipMemcpyAsync(rowS.data(), h->trn.rowS, rowS.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st),
            "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  h->nvalid = 0;
  for (int32_t v : rowS) h->nvalid += v > 0;
  h->nsamples = ns;
}

extern "C" {

int nesa_mlp_num_params(const nesa_mlp_params* params, int64_t* count) {
  return guarded([&]() {
    if (!params || !count) return fail(NESA_EINVAL, "null argument");
    check_mlp_params(params);
    *count = nesa::mlp_nparams(params->s_max, params->hidden);
    return (int)NESA_OK;
  });
}

int nesa_mlp_create(nesa_op* op, const nesa_mlp_params* params, const float* theta0, nesa_mlp** out) {
  return guarded([&]() {
    if (!op || !params || !theta0 || !out) return fail(NESA_EINVAL, "null argument");
    check_mlp_params(params);
    if (max_leaf(*op->tree) > params->s_max) return fail(NESA_EINVAL, "a leaf holds more RWGs than s_max");
    std::unique_ptr<nesa_mlp> h(new nesa_mlp());
    h->op = op;
    h->base = params->base;
    nesa::MlpDev& N = h->net;
    const int S = params->s_max, H = params->hidden;
    N.S = S;
    N.H = H;
    N.np = nesa::mlp_nparams(S, H);
    const int64_t sz[6] = {(int64_t)H * 4 * S, H, (int64_t)H * H, H, (int64_t)2 * S * H, 2 * S};
    N.off[0] = 0;
    for (int i = 0; i < 6; ++i) N.off[i + 1] = N.off[i] + sz[i];
    N.theta = net_alloc<float>(h->allocs, N.np);
    N.m = net_alloc<float>(h->allocs, N.np);
    N.v = net_alloc<float>(h->allocs, N.np);
    N.grad = net_alloc<float>(h->allocs, N.np);
    N.W1h = net_alloc<_Float16>(h->allocs, sz[0]);
    N.W2h = net_alloc<_Float16>(h->allocs, sz[2]);
    N.W3h = net_alloc<_Float16>(h->allocs, sz[4]);
    N.W2t = net_alloc<_Float16>(h->allocs, sz[2]);
    N.W3t = net_alloc<_Float16>(h->allocs, sz[4]);
    N.loss = net_alloc<double>(h->allocs, 1);
    const int64_t nleaf = (int64_t)op->tree->leaf_ptr.size() - 1;
    alloc_rows(h->allocs, h->app, S, H, nleaf, false);
    if (h->base == NESA_PRECOND_SCHWARZ) ensure_schwarz(op);
    mlp_upload_params(h.get(), theta0);
    op->nets.push_back(h.get());
    *out = h.release();
    return (int)NESA_OK;
  });
}

void nesa_mlp_free(nesa_mlp* net) {
  if (net && net->op) {
    if (net->op->mlp == net) net->op->mlp = nullptr;
    auto& v = net->op->nets;
    v.erase(std::remove(v.begin(), v.end(), net), v.end());
  }
  delete net;
}

int nesa_mlp_set_params(nesa_mlp* net, const float* theta) {
  return guarded([&]() {
    if (!net || !theta) return fail(NESA_EINVAL, "null argument");
    mlp_upload_params(net, theta);
    return (int)NESA_OK;
  });
}

int nesa_mlp_get_params(const nesa_mlp* net, float* theta) {
  return guarded([&]() {
    if (!net || !theta) return fail(NESA_EINVAL, "null argument");
    hip_check(hipMemcpy(theta, net->net.theta, net->net.np * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return (int)NESA_OK;
  });
}

// file layout: 8-byte tag "NESAMLP1", int32 s_max, hidden, base, int64 count,
// then count FP32 parameters (host byte order)
int nesa_mlp_save(const nesa_mlp* net, const char* path) {
  return guarded([&]() {
    if (!net || !path) return fail(NESA_EINVAL, "null argument");
    std::vector<float> th(net->net.np);
    hip_check(hipMemcpy(th.data(), net->net.theta, th.size() * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(NESA_EINVAL, std::string("cannot open for writing: ") + path);
    const int32_t hdr[3] = {net->net.S, net->net.H, net->base};
    const int64_t cnt = net->net.np;
    bool ok = std::fwrite("NESAMLP1", 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 &&
              std::fwrite(&cnt, sizeof(cnt), 1, fp) == 1 &&
              std::fwrite(th.data(), sizeof(float), th.size(), fp) == th.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(NESA_EINVAL, std::string("write failed: ") + path);
    return (int)NESA_OK;
  });
}

int nesa_mlp_load(nesa_op* op, const char* path, nesa_mlp** out) {
  return guarded([&]() {
    if (!op || !path || !out) return fail(NESA_EINVAL, "null argument");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(NESA_EINVAL, std::string("cannot open for reading: ") + path);
    char tag[8];
    int32_t hdr[3];
    int64_t cnt = 0;
    bool ok = std::fread(tag, 1, 8, fp) == 8 && std::memcmp(tag, "NESAMLP1", 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, fp) == 1 && std::fread(&cnt, sizeof(cnt), 1, fp) == 1;
    nesa_mlp_params prm{hdr[0], hdr[1], hdr[2]};
    std::vector<float> th;
    if (ok) {
      check_mlp_params(&prm);
      ok = cnt == nesa::mlp_nparams(prm.s_max, prm.hidden);
      if (ok) {
        th.resize(cnt);
        ok = std::fread(th.data(), sizeof(float), th.size(), fp) == th.size();
      }
    }
    std::fclose(fp);
    if (!ok) return fail(NESA_EINVAL, std::string("not a network file of this library: ") + path);
    return nesa_mlp_create(op, &prm, th.data(), out);
  });
}

int nesa_mlp_set_data(nesa_mlp* net, const void* r_dev, const void* e_dev, int64_t nsamples, void* stream) {
  return guarded([&]() {
    if (!net || !r_dev || !e_dev) return fail(NESA_EINVAL, "null argument");
    if (!net->op) return fail(NESA_EINVAL, "the operator of this network has been freed");
    if (nsamples < 1) return fail(NESA_EINVAL, "nsamples must be positive");
    nesa_op* op = net->op;
    const int64_t nleaf = (int64_t)op->tree->leaf_ptr.size() - 1;
    if (nsamples * nleaf > ((int64_t)1 << 31) / (4 * net->net.S))
      return fail(NESA_EINVAL, "too many training rows");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (op->precision == NESA_C128)
      mlp_set_data_t<double>(net, op->d, r_dev, e_dev, nsamples, st);
    else
      mlp_set_data_t<float>(net, op->f, r_dev, e_dev, nsamples, st);
    return (int)NESA_OK;
  });
}

int nesa_mlp_train(nesa_mlp* net, const nesa_adam_params* adam, int steps, double* loss_history, void* stream) {
  return guarded([&]() {
    if (!net || !adam) return fail(NESA_EINVAL, "null argument");
    if (steps < 0 || !(adam->lr > 0) || !(adam->beta1 >= 0 && adam->beta1 < 1) ||
        !(adam->beta2 >= 0 && adam->beta2 < 1) || !(adam->eps > 0))
      return fail(NESA_EINVAL, "bad Adam parameters");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int i = 0; i < steps; ++i) {
      const double loss = mlp_pass(net, true, st);
      if (loss_history) loss_history[i] = loss;
      net->t += 1;
      nesa::launch_mlp_adam(net->net, (float)adam->lr, (float)adam->beta1, (float)adam->beta2, (float)adam->eps,
                            net->t, st);
      nesa::launch_mlp_refresh(net->net, st);
      hip_check(hipGetLastError(), "kernel launch");
    }
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return (int)NESA_OK;
  });
}

int nesa_mlp_gradient(nesa_mlp* net, float* grad, double* loss) {
  return guarded([&]() {
    if (!net || !grad || !loss) return fail(NESA_EINVAL, "null argument");
    *loss = mlp_pass(net, true, nullptr);
    hip_check(hipMemcpy(grad, net->net.grad, net->net.np * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return (int)NESA_OK;
  });
}

int nesa_mlp_outputs(nesa_mlp* net, float* y) {
  return guarded([&]() {
    if (!net || !y) return fail(NESA_EINVAL, "null argument");
    if (!net->op) return fail(NESA_EINVAL, "the operator of this network has been freed");
    (void)mlp_pass(net, false, nullptr);
    const int64_t rows = net->nsamples * ((int64_t)net->op->tree->leaf_ptr.size() - 1);
    hip_check(hipMemcpy(y, net->trn.Y, (size_t)rows * 2 * net->net.S * sizeof(float), hipMemcpyDeviceToHost),
              "hipMemcpy");
    return (int)NESA_OK;
  });
}

int nesa_mlp_apply(nesa_mlp* net, const void* r_dev, void* z_dev, void* stream) {
  return guarded([&]() {
    if (!net || !r_dev || !z_dev) return fail(NESA_EINVAL, "null argument");
    if (!net->op) return fail(NESA_EINVAL, "the operator of this network has been freed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (net->op->precision == NESA_C128)
      learned_apply<double>(net, net->op->d, r_dev, z_dev, st);
    else
      learned_apply<float>(net, net->op->f, r_dev, z_dev, st);
    hip_check(hipGetLastError(), "kernel launch");
    return (int)NESA_OK;
  });
}

int nesa_op_set_mlp(nesa_op* op, nesa_mlp* net) {
  return guarded([&]() {
    if (!op) return fail(NESA_EINVAL, "null argument");
    if (net && net->op != op) return fail(NESA_EINVAL, "network belongs to another operator");
    op->mlp = net;
    return (int)NESA_OK;
  });
}

}  // extern "C"
