// Binned SAH construction (after Wald 2007) of a binary BVH, collapse to 4-wide
// nodes, and 8-bit quantization of child boxes in an FP32 parent frame (the
// compressed-node idea of Ylitie, Karras, Laine 2017, here with 4 children).
#include "bvh_build.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace rtq {

namespace {

constexpr float kInf = std::numeric_limits<float>::infinity();

struct Box {
  float lo[3] = {kInf, kInf, kInf};
  float hi[3] = {-kInf, -kInf, -kInf};
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  void grow_pt(float x, float y, float z) {
    const float p[3] = {x, y, z};
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  double area() const {
    if (!(lo[0] <= hi[0])) return 0.0;
    const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct Node2 {
  Box b;
  int32_t l = -1, r = -1;
  int32_t first = 0, count = 0;  // leaf when count > 0
};

struct Builder {
  const Aabb* in;
  const BuildParams& p;
  std::vector<float> cx, cy, cz;
  std::vector<uint32_t> idx;
  std::vector<Node2> nodes;
  Builder(const Aabb* boxes, int64_t n, const BuildParams& prm) : in(boxes), p(prm) {
    cx.resize(n);
    cy.resize(n);
    cz.resize(n);
    idx.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      cx[i] = 0.5f * (in[i].lo[0] + in[i].hi[0]);
      cy[i] = 0.5f * (in[i].lo[1] + in[i].hi[1]);
      cz[i] = 0.5f * (in[i].lo[2] + in[i].hi[2]);
      idx[i] = (uint32_t)i;
    }
  }
  float cen(uint32_t i, int k) const { return k == 0 ? cx[i] : (k == 1 ? cy[i] : cz[i]); }
  Box box_of(uint32_t i) const {
    Box b;
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = in[i].lo[k];
      b.hi[k] = in[i].hi[k];
    }
    return b;
  }

  void run() {
    const int64_t n = (int64_t)idx.size();
    nodes.reserve(2 * n / std::max(1, p.leaf_max) + 2);
    nodes.push_back(Node2{});
    struct Job {
      int32_t node;
      int64_t first, count;
      int depth;
    };
    std::vector<Job> jobs{{0, 0, n, 0}};
    const int B = p.bins;
    std::vector<Box> bb(B);
    std::vector<int64_t> bc(B);
    std::vector<double> right_area(B);
    std::vector<int64_t> right_count(B);
    while (!jobs.empty()) {
      const Job j = jobs.back();
      jobs.pop_back();
      Box b, cb;
      for (int64_t i = j.first; i < j.first + j.count; ++i) {
        const uint32_t q = idx[i];
        b.grow(box_of(q));
        cb.grow_pt(cx[q], cy[q], cz[q]);
      }
      nodes[j.node].b = b;
      const double A = std::max(b.area(), 1e-300);
      // best binned SAH split over the three axes
      int best_axis = -1, best_bin = -1;
      double best_cost = std::numeric_limits<double>::infinity();
      if (j.count > 1)
        for (int ax = 0; ax < 3; ++ax) {
          const float lo = cb.lo[ax], ext = cb.hi[ax] - cb.lo[ax];
          if (!(ext > 0.0f)) continue;
          const float scale = (float)B / ext;
          for (int k = 0; k < B; ++k) {
            bb[k] = Box{};
            bc[k] = 0;
          }
          for (int64_t i = j.first; i < j.first + j.count; ++i) {
            const uint32_t q = idx[i];
            const int k = std::min(B - 1, (int)((cen(q, ax) - lo) * scale));
            bb[k].grow(box_of(q));
            bc[k]++;
          }
          Box acc;
          int64_t cnt = 0;
          for (int k = B - 1; k > 0; --k) {
            acc.grow(bb[k]);
            cnt += bc[k];
            right_area[k] = acc.area();
            right_count[k] = cnt;
          }
          acc = Box{};
          cnt = 0;
          for (int k = 0; k < B - 1; ++k) {
            acc.grow(bb[k]);
            cnt += bc[k];
            const int64_t rc = right_count[k + 1];
            if (cnt == 0 || rc == 0) continue;
            const double cost = 1.0 + (acc.area() * (double)cnt + right_area[k + 1] * (double)rc) / A;
            if (cost < best_cost) {
              best_cost = cost;
              best_axis = ax;
              best_bin = k;
            }
          }
        }
      const bool can_leaf = j.count <= p.leaf_max;
      if (j.count == 1 || (can_leaf && (best_axis < 0 || (double)j.count <= best_cost))) {
        nodes[j.node].first = (int32_t)j.first;
        nodes[j.node].count = (int32_t)j.count;
        continue;
      }
      int64_t mid;
      if (best_axis >= 0 && j.depth < 48) {
        const float lo = cb.lo[best_axis], scale = (float)B / (cb.hi[best_axis] - cb.lo[best_axis]);
        auto it = std::partition(idx.begin() + j.first, idx.begin() + j.first + j.count, [&](uint32_t q) {
          return std::min(B - 1, (int)((cen(q, best_axis) - lo) * scale)) <= best_bin;
        });
        mid = it - idx.begin();
      } else {
        // no usable SAH split (identical centroids, or too deep): object median
        int ax = 0;
        float e = -1.0f;
        for (int k = 0; k < 3; ++k)
          if (cb.hi[k] - cb.lo[k] > e) {
            e = cb.hi[k] - cb.lo[k];
            ax = k;
          }
        mid = j.first + j.count / 2;
        std::nth_element(idx.begin() + j.first, idx.begin() + mid, idx.begin() + j.first + j.count,
                         [&](uint32_t a, uint32_t c) { return cen(a, ax) < cen(c, ax); });
      }
      if (mid == j.first || mid == j.first + j.count) mid = j.first + j.count / 2;
      const int32_t l = (int32_t)nodes.size();
      nodes.push_back(Node2{});
      nodes.push_back(Node2{});
      nodes[j.node].l = l;
      nodes[j.node].r = l + 1;
      jobs.push_back({l, j.first, mid - j.first, j.depth + 1});
      jobs.push_back({l + 1, mid, j.first + j.count - mid, j.depth + 1});
    }
  }
};

void set_child(NodeF32& n, int k, const Box& b, uint32_t ref) {
  n.lo_x[k] = b.lo[0];
  n.hi_x[k] = b.hi[0];
  n.lo_y[k] = b.lo[1];
  n.hi_y[k] = b.hi[1];
  n.lo_z[k] = b.lo[2];
  n.hi_z[k] = b.hi[2];
  n.child[k] = ref;
}

void empty_node(NodeF32& n) {
  for (int k = 0; k < 4; ++k) {
    n.lo_x[k] = n.lo_y[k] = n.lo_z[k] = kInf;
    n.hi_x[k] = n.hi_y[k] = n.hi_z[k] = -kInf;
    n.child[k] = kEmpty;
    n.pad[k] = 0;
  }
}

}  // namespace

float q8_decode(uint32_t q, int e, float origin) {
  return std::fma((float)q, std::ldexp(1.0f, e), origin);
}

NodeQ8 quantize_node(const NodeF32& n) {
  NodeQ8 o;
  std::memset(&o, 0, sizeof(o));
  const float* LO[3] = {n.lo_x, n.lo_y, n.lo_z};
  const float* HI[3] = {n.hi_x, n.hi_y, n.hi_z};
  float org[3];
  int ex[3];
  uint32_t qlo[3][4], qhi[3][4];
  for (int a = 0; a < 3; ++a) {
    float lo = kInf, hi = -kInf;
    for (int k = 0; k < 4; ++k)
      if (n.child[k] != kEmpty) {
        lo = std::min(lo, LO[a][k]);
        hi = std::max(hi, HI[a][k]);
      }
    if (!(lo <= hi)) lo = hi = 0.0f;  // no children at all
    org[a] = lo;
    const double ext = (double)hi - (double)lo;
    int e = -126;
    if (ext > 0.0) e = std::max(-126, (int)std::ceil(std::log2(ext / 255.0)));
    for (;;) {
      bool ok = true;
      for (int k = 0; k < 4 && ok; ++k) {
        if (n.child[k] == kEmpty) {
          qlo[a][k] = 255u;
          qhi[a][k] = 0u;
          continue;
        }
        const double s = std::ldexp(1.0, e);
        double fl = std::floor(((double)LO[a][k] - (double)lo) / s);
        double ce = std::ceil(((double)HI[a][k] - (double)lo) / s);
        int64_t ql = std::max<int64_t>(0, (int64_t)fl);
        int64_t qh = std::max<int64_t>(0, (int64_t)ce);
        while (ql > 0 && q8_decode((uint32_t)ql, e, lo) > LO[a][k]) --ql;
        while (qh <= 255 && q8_decode((uint32_t)qh, e, lo) < HI[a][k]) ++qh;
        if (ql > 255 || qh > 255 || q8_decode((uint32_t)ql, e, lo) > LO[a][k]) {
          ok = false;
          break;
        }
        qlo[a][k] = (uint32_t)ql;
        qhi[a][k] = (uint32_t)qh;
      }
      if (ok) break;
      ++e;
    }
    ex[a] = e;
  }
  o.ox = org[0];
  o.oy = org[1];
  o.oz = org[2];
  o.exps = (uint32_t)(uint8_t)(int8_t)ex[0] | ((uint32_t)(uint8_t)(int8_t)ex[1] << 8) |
           ((uint32_t)(uint8_t)(int8_t)ex[2] << 16);
  auto pack = [](const uint32_t q[4]) { return q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24); };
  o.lo_x = pack(qlo[0]);
  o.hi_x = pack(qhi[0]);
  o.lo_y = pack(qlo[1]);
  o.hi_y = pack(qhi[1]);
  o.lo_z = pack(qlo[2]);
  o.hi_z = pack(qhi[2]);
  for (int k = 0; k < 4; ++k) o.child[k] = n.child[k];
  return o;
}

void build_bvh4(const Aabb* boxes, int64_t n, const BuildParams& p, Bvh4& out) {
  out.f32.clear();
  out.q8.clear();
  out.order.clear();
  out.depth = 0;
  Builder bld(boxes, n, p);
  bld.run();
  out.order = bld.idx;
  const std::vector<Node2>& N = bld.nodes;
  const Box& rb = N[0].b;
  for (int k = 0; k < 3; ++k) {
    out.root_box.lo[k] = rb.lo[k];
    out.root_box.hi[k] = rb.hi[k];
  }
  // collapse: every 4-wide node adopts up to four BVH2 descendants, expanding
  // the internal child of largest surface area first
  struct Job {
    int32_t n2;      // BVH2 node whose subtree this 4-wide node covers
    uint32_t slot;   // 4-wide node index
    int depth;
  };
  out.f32.emplace_back();
  empty_node(out.f32[0]);
  std::vector<Job> jobs{{0, 0u, 1}};
  while (!jobs.empty()) {
    const Job j = jobs.back();
    jobs.pop_back();
    out.depth = std::max(out.depth, j.depth);
    int32_t kids[4];
    int nk = 0;
    if (N[j.n2].count > 0) {
      kids[nk++] = j.n2;  // a leaf root: one leaf child
    } else {
      kids[nk++] = N[j.n2].l;
      kids[nk++] = N[j.n2].r;
      while (nk < 4) {
        int best = -1;
        double ba = -1.0;
        for (int k = 0; k < nk; ++k)
          if (N[kids[k]].count == 0 && N[kids[k]].b.area() > ba) {
            ba = N[kids[k]].b.area();
            best = k;
          }
        if (best < 0) break;
        const int32_t c = kids[best];
        kids[best] = N[c].l;
        kids[nk++] = N[c].r;
      }
    }
    NodeF32 node;
    empty_node(node);
    for (int k = 0; k < nk; ++k) {
      const Node2& c = N[kids[k]];
      uint32_t ref;
      if (c.count > 0) {
        ref = make_leaf((uint32_t)c.first, (uint32_t)c.count);
      } else {
        ref = (uint32_t)out.f32.size();
        out.f32.emplace_back();
        jobs.push_back({kids[k], ref, j.depth + 1});
      }
      set_child(node, k, c.b, ref);
    }
    out.f32[j.slot] = node;
  }
  if (p.want_q8) {
    out.q8.resize(out.f32.size());
    for (size_t i = 0; i < out.f32.size(); ++i) out.q8[i] = quantize_node(out.f32[i]);
  }
}

float level_pmax(const Bvh4& b) {
  double m = 0.0;
  for (const NodeF32& n : b.f32)
    for (int k = 0; k < 4; ++k) {
      if (n.child[k] == kEmpty) continue;
      const float v[6] = {n.lo_x[k], n.hi_x[k], n.lo_y[k], n.hi_y[k], n.lo_z[k], n.hi_z[k]};
      for (float x : v) m = std::max(m, (double)std::fabs(x));
    }
  for (const NodeQ8& n : b.q8) {
    const float org[3] = {n.ox, n.oy, n.oz};
    for (int a = 0; a < 3; ++a) {
      const int e = (int)(int8_t)((n.exps >> (8 * a)) & 0xFFu);
      m = std::max(m, std::fabs((double)org[a]));
      m = std::max(m, std::fabs((double)org[a] + 255.0 * std::ldexp(1.0, e)));
    }
  }
  // round up so that the FP32 bound is not below the exact maximum
  const float f = (float)m;
  return (double)f >= m ? f : std::nextafter(f, std::numeric_limits<float>::infinity());
}

bool relocate(Bvh4& b, uint32_t node_base, uint32_t prim_base) {
  auto fix = [&](uint32_t& r) -> bool {
    if (r == kEmpty) return true;
    if (ref_is_leaf(r)) {
      const uint64_t f = (uint64_t)leaf_first(r) + prim_base;
      if (f > kMaxLeafFirst) return false;
      r = make_leaf((uint32_t)f, leaf_count(r));
    } else {
      const uint64_t v = (uint64_t)r + node_base;
      if (v >= kLeafBit) return false;
      r = (uint32_t)v;
    }
    return true;
  };
  for (auto& nd : b.f32)
    for (int k = 0; k < 4; ++k)
      if (!fix(nd.child[k])) return false;
  for (auto& nd : b.q8)
    for (int k = 0; k < 4; ++k)
      if (!fix(nd.child[k])) return false;
  return true;
}

}  // namespace rtq
