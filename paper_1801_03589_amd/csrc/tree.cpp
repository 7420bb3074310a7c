// RWG basis and oct-tree construction (host, FP64).
//
// Tree rules (Sec. 2: hierarchical oct-tree partition, near blocks stored and
// far blocks compressed, ascend while the ancestors do not touch; Sec. 3:
// coarsest level with four groups along the longest side, near groups are the
// adjacent ones including diagonal neighbours and the group itself, far pairs
// interact at the level where they are not neighbours but their parents are).
// The leaf side is a parameter; an RWG belongs to the leaf holding its edge
// midpoint; boxes are ordered by Morton code so that every box's RWGs, and
// every parent's children, are contiguous.
#include <algorithm>
#include <atomic>
#include <memory>
#include <cmath>
#include <thread>
#include <unordered_map>

#include "nesa_host.h"

namespace nesa {

void parallel_for(int64_t n, const std::function<void(int64_t)>& fn) {
  if (n <= 0) return;
  int nt = (int)std::min<int64_t>(n, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  if (nt == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next{0};
  std::vector<std::exception_ptr> err(nt);
  for (int w = 0; w < nt; ++w) {
    th.emplace_back([&, w]() {
      try {
        for (;;) {
          int64_t i = next.fetch_add(1);
          if (i >= n) break;
          fn(i);
        }
      } catch (...) {
        err[w] = std::current_exception();
        next.store(n);
      }
    });
  }
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

static uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}
static uint64_t morton(const std::array<int32_t, 3>& k) {
  return spread3((uint64_t)k[0]) | (spread3((uint64_t)k[1]) << 1) | (spread3((uint64_t)k[2]) << 2);
}
static uint64_t pack(const std::array<int32_t, 3>& k) {
  return ((uint64_t)(uint32_t)k[0] << 42) | ((uint64_t)(uint32_t)k[1] << 21) | (uint64_t)(uint32_t)k[2];
}
static int cheb(const std::array<int32_t, 3>& a, const std::array<int32_t, 3>& b) {
  return std::max({std::abs(a[0] - b[0]), std::abs(a[1] - b[1]), std::abs(a[2] - b[2])});
}

static void build_rwg(Rwg& r, const double* verts, int64_t nv, const int32_t* tris, int64_t nt) {
  r.v.assign(verts, verts + 3 * nv);
  r.t.assign(tris, tris + 3 * nt);
  r.nt = nt;
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (tris[i] < 0 || tris[i] >= nv) throw Error(-1, "triangle vertex index out of range");
  // (min, max, tri, local vertex) for every triangle edge; sorted, pairs form RWGs
  struct HE { int64_t a, b, t; int loc; };
  std::vector<HE> he;
  he.reserve(3 * nt);
  for (int64_t ti = 0; ti < nt; ++ti)
    for (int a = 0; a < 3; ++a) {
      int64_t p = tris[3 * ti + (a + 1) % 3], q = tris[3 * ti + (a + 2) % 3];
      if (p == q) throw Error(-4, "degenerate triangle");
      he.push_back({std::min(p, q), std::max(p, q), ti, a});
    }
  std::sort(he.begin(), he.end(), [](const HE& x, const HE& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.t < y.t;
  });
  r.tri_rwg.assign(3 * nt, -1);
  r.tri_sign.assign(3 * nt, 0.0);
  size_t i = 0;
  while (i < he.size()) {
    size_t j = i;
    while (j < he.size() && he[j].a == he[i].a && he[j].b == he[i].b) ++j;
    if (j - i != 2) throw Error(-4, "mesh is not a closed 2-manifold (edge shared by " +
                                        std::to_string(j - i) + " triangles)");
    int64_t n = (int64_t)r.len.size();
    const HE& P = he[i];
    const HE& M = he[i + 1];  // higher triangle index
    r.edge.push_back(P.a);
    r.edge.push_back(P.b);
    r.tri.push_back(P.t);
    r.tri.push_back(M.t);
    r.freev.push_back(tris[3 * P.t + P.loc]);
    r.freev.push_back(tris[3 * M.t + M.loc]);
    double d = 0;
    for (int c = 0; c < 3; ++c) {
      double x = verts[3 * P.a + c] - verts[3 * P.b + c];
      d += x * x;
    }
    r.len.push_back(std::sqrt(d));
    r.tri_rwg[3 * P.t + P.loc] = n;
    r.tri_sign[3 * P.t + P.loc] = 1.0;
    r.tri_rwg[3 * M.t + M.loc] = n;
    r.tri_sign[3 * M.t + M.loc] = -1.0;
    i = j;
  }
  r.n = (int64_t)r.len.size();
  r.area.resize(nt);
  r.normal.resize(3 * nt);
  r.qp.resize(9 * nt);
  const double bw[3][3] = {{2.0 / 3, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 2.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 2.0 / 3}};
  for (int64_t ti = 0; ti < nt; ++ti) {
    const double* A = verts + 3 * tris[3 * ti];
    const double* B = verts + 3 * tris[3 * ti + 1];
    const double* C = verts + 3 * tris[3 * ti + 2];
    double u[3], w[3], c[3];
    for (int k = 0; k < 3; ++k) { u[k] = B[k] - A[k]; w[k] = C[k] - A[k]; }
    c[0] = u[1] * w[2] - u[2] * w[1];
    c[1] = u[2] * w[0] - u[0] * w[2];
    c[2] = u[0] * w[1] - u[1] * w[0];
    double nn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(nn > 0)) throw Error(-4, "zero-area triangle");
    r.area[ti] = 0.5 * nn;
    for (int k = 0; k < 3; ++k) r.normal[3 * ti + k] = c[k] / nn;
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < 3; ++k)
        r.qp[9 * ti + 3 * q + k] = bw[q][0] * A[k] + bw[q][1] * B[k] + bw[q][2] * C[k];
  }
}

Tree* build_tree(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, double leaf,
                 int l0_max, int buffer) {
  if (!verts || !tris || nv < 3 || nt < 1) throw Error(-1, "empty mesh");
  if (!(leaf > 0) || l0_max < 0 || buffer < 1 || buffer > 3) throw Error(-1, "bad tree parameters");
  std::unique_ptr<Tree> T(new Tree());
  Tree& t = *T;
  build_rwg(t.rwg, verts, nv, tris, nt);
  t.leaf = leaf;
  t.buffer = buffer;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < nv; ++i)
    for (int c = 0; c < 3; ++c) {
      mn[c] = std::min(mn[c], verts[3 * i + c]);
      mx[c] = std::max(mx[c], verts[3 * i + c]);
    }
  double ext = std::max({mx[0] - mn[0], mx[1] - mn[1], mx[2] - mn[2]});
  t.L = ext > leaf ? (int)std::ceil(std::log2(ext / leaf)) : 0;
  if (t.L > 20) throw Error(-1, "tree deeper than 20 levels");
  t.l0 = std::min(l0_max, t.L);
  if (t.l0 > 6) throw Error(-1, "coarsest far level deeper than 6 (translation table too large)");
  t.slotw = std::max(4 * buffer + 3, (1 << (t.l0 + 1)) - 1);
  for (int c = 0; c < 3; ++c) t.lo[c] = mn[c] - 1e-9;
  const int64_t n = t.rwg.n;
  const int32_t nside = 1 << t.L;
  // leaf key of every RWG (edge midpoint)
  std::vector<std::array<int32_t, 3>> rkey(n);
  for (int64_t e = 0; e < n; ++e)
    for (int c = 0; c < 3; ++c) {
      double m = 0.5 * (verts[3 * t.rwg.edge[2 * e] + c] + verts[3 * t.rwg.edge[2 * e + 1] + c]);
      int64_t k = (int64_t)std::floor((m - t.lo[c]) / leaf);
      rkey[e][c] = (int32_t)std::min<int64_t>(std::max<int64_t>(k, 0), nside - 1);
    }
  // leaf order: by (Morton code of the leaf, canonical index)
  std::vector<uint64_t> code(n);
  for (int64_t e = 0; e < n; ++e) code[e] = morton(rkey[e]);
  t.perm.resize(n);
  for (int64_t e = 0; e < n; ++e) t.perm[e] = e;
  std::stable_sort(t.perm.begin(), t.perm.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
  t.pos.resize(n);
  for (int64_t i = 0; i < n; ++i) t.pos[t.perm[i]] = i;
  t.lev.resize(t.L - t.l0 + 1);
  Level& LL = t.level(t.L);
  LL.l = t.L;
  LL.side = leaf;
  for (int64_t i = 0; i < n; ++i) {
    const auto& k = rkey[t.perm[i]];
    if (LL.key.empty() || morton(LL.key.back()) != morton(k)) {
      LL.key.push_back(k);
      t.leaf_ptr.push_back(i);
    }
  }
  t.leaf_ptr.push_back(n);
  LL.nbox = (int64_t)LL.key.size();
  // coarser levels: parents of Morton-sorted children are Morton-sorted and
  // every parent's children are contiguous
  for (int l = t.L - 1; l >= t.l0; --l) {
    Level& C = t.level(l + 1);
    Level& P = t.level(l);
    P.l = l;
    P.side = leaf * (double)(1LL << (t.L - l));
    C.parent.resize(C.nbox);
    C.octant.resize(C.nbox);
    for (int64_t b = 0; b < C.nbox; ++b) {
      std::array<int32_t, 3> pk = {C.key[b][0] >> 1, C.key[b][1] >> 1, C.key[b][2] >> 1};
      if (P.key.empty() || P.key.back() != pk) {
        P.key.push_back(pk);
        P.child_ptr.push_back(b);
      }
      C.parent[b] = (int64_t)P.key.size() - 1;
      C.octant[b] = (C.key[b][0] & 1) | ((C.key[b][1] & 1) << 1) | ((C.key[b][2] & 1) << 2);
    }
    P.child_ptr.push_back(C.nbox);
    P.nbox = (int64_t)P.key.size();
    P.child_end.assign(P.child_ptr.begin() + 1, P.child_ptr.end());
  }
  // hash maps key -> box index per level
  std::vector<std::unordered_map<uint64_t, int64_t>> idx(t.lev.size());
  for (int l = t.l0; l <= t.L; ++l) {
    auto& mp = idx[l - t.l0];
    const Level& lv = t.level(l);
    mp.reserve(2 * lv.nbox);
    for (int64_t b = 0; b < lv.nbox; ++b) mp[pack(lv.key[b])] = b;
  }
  auto find = [&](int l, std::array<int32_t, 3> k) -> int64_t {
    if (k[0] < 0 || k[1] < 0 || k[2] < 0) return -1;
    auto& mp = idx[l - t.l0];
    auto it = mp.find(pack(k));
    return it == mp.end() ? -1 : it->second;
  };
  // near lists at the leaf level
  t.near_ptr.push_back(0);
  for (int64_t a = 0; a < LL.nbox; ++a) {
    std::vector<int64_t> nb;
    for (int dx = -buffer; dx <= buffer; ++dx)
      for (int dy = -buffer; dy <= buffer; ++dy)
        for (int dz = -buffer; dz <= buffer; ++dz) {
          int64_t j = find(t.L, {LL.key[a][0] + dx, LL.key[a][1] + dy, LL.key[a][2] + dz});
          if (j >= 0) nb.push_back(j);
        }
    std::sort(nb.begin(), nb.end());
    t.near_idx.insert(t.near_idx.end(), nb.begin(), nb.end());
    t.near_ptr.push_back((int64_t)t.near_idx.size());
  }
  // interaction lists
  const int W = t.slot_w(), H = W / 2;
  for (int l = t.l0; l <= t.L; ++l) {
    Level& lv = t.level(l);
    lv.il_ptr.assign(1, 0);
    for (int64_t a = 0; a < lv.nbox; ++a) {
      std::vector<int64_t> cand;
      if (l == t.l0) {
        for (int64_t b = 0; b < lv.nbox; ++b) cand.push_back(b);
      } else {
        const Level& pl = t.level(l - 1);
        int64_t p = lv.parent[a];
        for (int dx = -buffer; dx <= buffer; ++dx)
          for (int dy = -buffer; dy <= buffer; ++dy)
            for (int dz = -buffer; dz <= buffer; ++dz) {
              int64_t q = find(l - 1, {pl.key[p][0] + dx, pl.key[p][1] + dy, pl.key[p][2] + dz});
              if (q < 0) continue;
              for (int64_t c = pl.child_ptr[q]; c < pl.child_ptr[q + 1]; ++c) cand.push_back(c);
            }
      }
      std::sort(cand.begin(), cand.end());
      for (int64_t b : cand) {
        if (cheb(lv.key[a], lv.key[b]) <= buffer) continue;
        int dx = lv.key[a][0] - lv.key[b][0], dy = lv.key[a][1] - lv.key[b][1], dz = lv.key[a][2] - lv.key[b][2];
        if (std::abs(dx) > H || std::abs(dy) > H || std::abs(dz) > H)
          throw Error(-1, "interaction offset outside the translation table");
        lv.il_src.push_back(b);
        lv.il_slot.push_back(((dx + H) * W + (dy + H)) * W + (dz + H));
      }
      lv.il_ptr.push_back((int64_t)lv.il_src.size());
    }
  }
  return T.release();
}

static void append_rwg(Rwg& F, const Rwg& r) {
  const int64_t vo = (int64_t)F.v.size() / 3, to = F.nt, ro = F.n;
  F.v.insert(F.v.end(), r.v.begin(), r.v.end());
  for (int32_t x : r.t) F.t.push_back((int32_t)(x + vo));
  for (int64_t x : r.edge) F.edge.push_back(x + vo);
  for (int64_t x : r.tri) F.tri.push_back(x + to);
  for (int64_t x : r.freev) F.freev.push_back(x + vo);
  F.len.insert(F.len.end(), r.len.begin(), r.len.end());
  F.area.insert(F.area.end(), r.area.begin(), r.area.end());
  F.normal.insert(F.normal.end(), r.normal.begin(), r.normal.end());
  for (int64_t x : r.tri_rwg) F.tri_rwg.push_back(x + ro);
  F.tri_sign.insert(F.tri_sign.end(), r.tri_sign.begin(), r.tri_sign.end());
  F.qp.insert(F.qp.end(), r.qp.begin(), r.qp.end());
  F.n += r.n;
  F.nt += r.nt;
}

Tree* build_forest(int nbodies, const double* const* verts, const int64_t* nv, const int32_t* const* tris,
                   const int64_t* nt, double leaf, int l0_max, int buffer) {
  if (nbodies < 1) throw Error(-1, "a forest needs at least one body");
  std::vector<std::unique_ptr<Tree>> B(nbodies);
  parallel_for(nbodies, [&](int64_t i) {
    B[i].reset(build_tree(verts[i], nv[i], tris[i], nt[i], leaf, l0_max, buffer));
  });
  std::unique_ptr<Tree> F(new Tree());
  F->leaf = leaf;
  F->buffer = buffer;
  F->L = 0;
  for (auto& b : B) F->L = std::max(F->L, b->L);
  // body i's level li sits at forest level li + (L - L_i)
  F->l0 = F->L;
  for (auto& b : B) F->l0 = std::min(F->l0, b->l0 + F->L - b->L);
  // one slot encoding for all bodies: the widest of theirs
  F->slotw = 0;
  for (auto& b : B) F->slotw = std::max(F->slotw, b->slotw);
  const int FW = F->slotw, FH = FW / 2;
  for (int c = 0; c < 3; ++c) F->lo[c] = B[0]->lo[c];
  F->lev.resize(F->L - F->l0 + 1);
  for (int l = F->l0; l <= F->L; ++l) {
    F->level(l).l = l;
    F->level(l).side = leaf * (double)(1LL << (F->L - l));
  }
  F->body_rwg.push_back(0);
  // box offsets of every body at every forest level
  std::vector<std::vector<int64_t>> boff(F->lev.size(), std::vector<int64_t>(nbodies + 1, 0));
  for (int l = F->l0; l <= F->L; ++l)
    for (int i = 0; i < nbodies; ++i) {
      const int li = l - (F->L - B[i]->L);
      const int64_t nb = (li >= B[i]->l0) ? B[i]->level(li).nbox : 0;
      boff[l - F->l0][i + 1] = boff[l - F->l0][i] + nb;
    }
  int64_t leaf_off = 0;
  for (int i = 0; i < nbodies; ++i) {
    const Tree& b = *B[i];
    const int64_t ro = F->rwg.n;
    append_rwg(F->rwg, b.rwg);
    F->body_rwg.push_back(F->rwg.n);
    F->body_lo.push_back({b.lo[0], b.lo[1], b.lo[2]});
    for (int64_t p : b.perm) F->perm.push_back(p + ro);
    for (size_t a = 0; a + 1 < b.leaf_ptr.size(); ++a) F->leaf_ptr.push_back(b.leaf_ptr[a] + ro);
    for (size_t a = 0; a + 1 < b.near_ptr.size(); ++a) F->near_ptr.push_back(b.near_ptr[a] + (int64_t)F->near_idx.size() - b.near_ptr[0]);
    for (int64_t x : b.near_idx) F->near_idx.push_back(x + leaf_off);
    leaf_off += b.level(b.L).nbox;
    const int shift = F->L - b.L;
    for (int li = b.l0; li <= b.L; ++li) {
      const int l = li + shift;
      const Level& s = b.level(li);
      Level& d = F->level(l);
      const int64_t off = boff[l - F->l0][i];
      d.key.insert(d.key.end(), s.key.begin(), s.key.end());
      d.body.insert(d.body.end(), s.nbox, i);
      if (l > F->l0) {
        if (li > b.l0) {
          const int64_t poff = boff[l - 1 - F->l0][i];
          for (int64_t p : s.parent) d.parent.push_back(p + poff);
          d.octant.insert(d.octant.end(), s.octant.begin(), s.octant.end());
        } else {
          d.parent.insert(d.parent.end(), s.nbox, -1);
          d.octant.insert(d.octant.end(), s.nbox, 0);
        }
      }
      if (li < b.L) {
        const int64_t coff = boff[l + 1 - F->l0][i];
        for (int64_t k = 0; k < s.nbox; ++k) {
          d.child_ptr.push_back(s.child_ptr[k] + coff);
          d.child_end.push_back(s.child_ptr[k + 1] + coff);
        }
      }
      const int64_t io = (int64_t)d.il_src.size();
      for (int64_t k = 0; k < s.nbox; ++k) d.il_ptr.push_back(s.il_ptr[k] + io);
      for (int64_t x : s.il_src) d.il_src.push_back(x + off);
      const int BW = b.slotw, BH = BW / 2;
      for (int32_t x : s.il_slot) {
        const int dx = x / (BW * BW) - BH, dy = (x / BW) % BW - BH, dz = x % BW - BH;
        d.il_slot.push_back(((dx + FH) * FW + (dy + FH)) * FW + (dz + FH));
      }
    }
  }
  F->leaf_ptr.push_back(F->rwg.n);
  F->near_ptr.push_back((int64_t)F->near_idx.size());
  F->pos.resize(F->rwg.n);
  for (int64_t i = 0; i < F->rwg.n; ++i) F->pos[F->perm[i]] = i;
  for (int l = F->l0; l <= F->L; ++l) {
    Level& d = F->level(l);
    d.nbox = boff[l - F->l0][nbodies];
    d.il_ptr.push_back((int64_t)d.il_src.size());
    if (l < F->L) d.child_ptr.push_back(boff[l + 1 - F->l0][nbodies]);
  }
  return F.release();
}

}  // namespace nesa
