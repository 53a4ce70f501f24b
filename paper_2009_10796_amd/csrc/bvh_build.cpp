// Host BVH builder: binned-SAH two-wide BVH over float32 triangles, laid out
// for the GPU traversal (one 64-byte node = both child boxes and links; one
// 48-byte triangle record = three vertices plus id, object and material).
//
// Depth is bounded by kMaxDepth so that the traversal stack, which holds at
// most one entry per level, never overflows: SAH splits are used down to
// depth kSahDepth, object-median splits below it (each halves the count).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "irf_internal.h"

namespace irf {
namespace {

constexpr int kSahDepth = 24;
constexpr int kBins = 16;

struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const Box& b) {
    for (int a = 0; a < 3; a++) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow_pt(const float* p) {
    for (int a = 0; a < 3; a++) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double area() const {
    if (!(hi[0] >= lo[0])) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
  bool contains(const Box& b) const {
    for (int a = 0; a < 3; a++)
      if (b.lo[a] < lo[a] || b.hi[a] > hi[a]) return false;
    return true;
  }
};

struct Ref {
  Box b;
  float c[3];
  int32_t id;
};

struct Node {
  Box box[2];
  int32_t link[2];
};

struct Builder {
  std::vector<Ref> refs;
  std::vector<Node> nodes;
  std::vector<int32_t> order;
  int max_depth = 0;
  int64_t leaves = 0;
  double sah = 0.0;
  double root_area = 1.0;

  int32_t leaf(int first, int count, const Box& b) {
    leaves++;
    sah += b.area() / root_area * count;
    for (int i = 0; i < count; i++) order.push_back(refs[first + i].id);
    int32_t start = (int32_t)order.size() - count;
    return ~((start << 3) | (count - 1));
  }

  // Returns the link of the subtree over refs[first, first+count), sets its box.
  int32_t build(int first, int count, int depth, Box& out) {
    Box b, cb;
    for (int i = first; i < first + count; i++) {
      b.grow(refs[i].b);
      cb.grow_pt(refs[i].c);
    }
    out = b;
    if (depth > max_depth) max_depth = depth;
    if (count <= 2) return leaf(first, count, b);

    int split = -1;
    if (depth < kSahDepth) {
      double best = INFINITY;
      int best_axis = -1, best_bin = -1;
      for (int a = 0; a < 3; a++) {
        float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0f)) continue;
        Box bins[kBins];
        int cnt[kBins] = {0};
        for (int i = first; i < first + count; i++) {
          int k = std::min(kBins - 1, (int)((refs[i].c[a] - cb.lo[a]) / ext * kBins));
          cnt[k]++;
          bins[k].grow(refs[i].b);
        }
        Box rb[kBins];
        int rc[kBins];
        Box acc;
        int ac = 0;
        for (int k = kBins - 1; k > 0; k--) {
          acc.grow(bins[k]);
          ac += cnt[k];
          rb[k] = acc;
          rc[k] = ac;
        }
        Box lb;
        int lc = 0;
        for (int k = 0; k < kBins - 1; k++) {
          lb.grow(bins[k]);
          lc += cnt[k];
          if (lc == 0 || rc[k + 1] == 0) continue;
          double cost = lb.area() * lc + rb[k + 1].area() * rc[k + 1];
          if (cost < best) {
            best = cost;
            best_axis = a;
            best_bin = k;
          }
        }
      }
      double leaf_cost = b.area() * count;
      double split_cost = b.area() * 1.0 + best;
      if (count <= kLeafMax && (best_axis < 0 || leaf_cost <= split_cost)) return leaf(first, count, b);
      if (best_axis >= 0) {
        float ext = cb.hi[best_axis] - cb.lo[best_axis];
        auto mid = std::partition(refs.begin() + first, refs.begin() + first + count, [&](const Ref& r) {
          int k = std::min(kBins - 1, (int)((r.c[best_axis] - cb.lo[best_axis]) / ext * kBins));
          return k <= best_bin;
        });
        split = (int)(mid - refs.begin());
        if (split == first || split == first + count) split = -1;
      }
    } else if (count <= kLeafMax) {
      return leaf(first, count, b);
    }
    if (split < 0) {
      // object median on the widest centroid axis
      int a = 0;
      for (int k = 1; k < 3; k++)
        if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
      split = first + count / 2;
      std::nth_element(refs.begin() + first, refs.begin() + split, refs.begin() + first + count,
                       [a](const Ref& x, const Ref& y) { return x.c[a] < y.c[a] || (x.c[a] == y.c[a] && x.id < y.id); });
    }
    int32_t me = (int32_t)nodes.size();
    nodes.emplace_back();
    sah += b.area() / root_area;
    Box lb, rb;
    int32_t l = build(first, split - first, depth + 1, lb);
    int32_t r = build(split, first + count - split, depth + 1, rb);
    nodes[me].box[0] = lb;
    nodes[me].box[1] = rb;
    nodes[me].link[0] = l;
    nodes[me].link[1] = r;
    return me;
  }
};

inline float bits_f(int32_t x) {
  float f;
  std::memcpy(&f, &x, 4);
  return f;
}

}  // namespace

int build_bvh(const float* vertices, int64_t nv, const uint32_t* indices, int64_t nt,
              const uint32_t* tri_material, const uint32_t* tri_object, std::vector<float4>& out_nodes,
              std::vector<float4>& out_tris, double stats[5]) {
  (void)nv;
  Builder B;
  B.refs.resize((size_t)nt);
  Box root;
  for (int64_t t = 0; t < nt; t++) {
    Ref& r = B.refs[(size_t)t];
    for (int k = 0; k < 3; k++) r.b.grow_pt(vertices + (size_t)indices[t * 3 + k] * 3);
    for (int a = 0; a < 3; a++) r.c[a] = 0.5f * (r.b.lo[a] + r.b.hi[a]);
    r.id = (int32_t)t;
    root.grow(r.b);
  }
  B.root_area = std::max(root.area(), 1e-30);
  out_nodes.clear();
  out_tris.clear();
  if (nt > 0) {
    Box rb;
    B.nodes.reserve((size_t)(nt / 2 + 4));
    B.order.reserve((size_t)nt);
    int32_t link = B.build(0, (int)nt, 1, rb);
    if (link < 0) {
      // a single leaf: wrap it in a root whose two children are that leaf
      // (the traversal tests its triangles twice; harmless for nearest hit)
      Node n;
      n.box[0] = rb;
      n.box[1] = rb;
      n.link[0] = link;
      n.link[1] = link;
      B.nodes.insert(B.nodes.begin(), n);
    }
  }
  // layout
  out_nodes.resize(B.nodes.size() * 4);
  for (size_t i = 0; i < B.nodes.size(); i++) {
    const Node& n = B.nodes[i];
    const Box& a = n.box[0];
    const Box& b = n.box[1];
    out_nodes[i * 4 + 0] = make_float4(a.lo[0], a.lo[1], a.lo[2], a.hi[0]);
    out_nodes[i * 4 + 1] = make_float4(a.hi[1], a.hi[2], b.lo[0], b.lo[1]);
    out_nodes[i * 4 + 2] = make_float4(b.lo[2], b.hi[0], b.hi[1], b.hi[2]);
    out_nodes[i * 4 + 3] = make_float4(bits_f(n.link[0]), bits_f(n.link[1]), 0.0f, 0.0f);
  }
  out_tris.resize((size_t)nt * 3);
  for (size_t k = 0; k < B.order.size(); k++) {
    int32_t t = B.order[k];
    const float* v0 = vertices + (size_t)indices[t * 3 + 0] * 3;
    const float* v1 = vertices + (size_t)indices[t * 3 + 1] * 3;
    const float* v2 = vertices + (size_t)indices[t * 3 + 2] * 3;
    out_tris[k * 3 + 0] = make_float4(v0[0], v0[1], v0[2], bits_f(t));
    out_tris[k * 3 + 1] = make_float4(v1[0], v1[1], v1[2], bits_f(tri_object ? (int32_t)tri_object[t] : 0));
    out_tris[k * 3 + 2] = make_float4(v2[0], v2[1], v2[2], bits_f((int32_t)tri_material[t]));
  }
  // validation: every triangle once, every child box inside... (boxes are
  // exact unions of their contents, so check leaf contents against boxes)
  bool ok = B.order.size() == (size_t)nt;
  if (ok) {
    std::vector<char> seen((size_t)nt, 0);
    for (int32_t t : B.order) {
      if (t < 0 || t >= nt || seen[(size_t)t]) { ok = false; break; }
      seen[(size_t)t] = 1;
    }
  }
  for (size_t i = 0; ok && i < B.nodes.size(); i++) {
    const Node& n = B.nodes[i];
    for (int c = 0; c < 2 && ok; c++) {
      int32_t link = n.link[c];
      if (link >= 0) {
        const Node& ch = B.nodes[(size_t)link];
        Box u = ch.box[0];
        u.grow(ch.box[1]);
        if (!n.box[c].contains(u)) ok = false;
      } else {
        int32_t code = ~link;
        int32_t first = code >> 3, cnt = (code & 7) + 1;
        for (int32_t k = first; k < first + cnt && ok; k++) {
          Box tb;
          int32_t t = B.order[(size_t)k];
          for (int v = 0; v < 3; v++) tb.grow_pt(vertices + (size_t)indices[t * 3 + v] * 3);
          if (!n.box[c].contains(tb)) ok = false;
        }
      }
    }
  }
  stats[0] = (double)B.nodes.size();
  stats[1] = (double)B.leaves;
  stats[2] = (double)B.max_depth;
  stats[3] = B.sah;
  stats[4] = ok ? 1.0 : 0.0;
  return ok ? 0 : 1;
}

}  // namespace irf
