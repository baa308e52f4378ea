// Opening instances in the top level; see rebraid.h.
#include "rebraid.h"

#include <algorithm>
#include <cmath>
#include <queue>
#include <thread>
#include <utility>

namespace rtq {

namespace {

struct Box64 {
  double lo[3], hi[3];
};

double area(const Box64& b) {
  const double x = b.hi[0] - b.lo[0], y = b.hi[1] - b.lo[1], z = b.hi[2] - b.lo[2];
  return 2.0 * (x * y + y * z + z * x);
}

// World box of an object-space box under [A | t]: centre A c + t, half extent
// |A| e, evaluated in FP64 from FP32 inputs and widened by a bound on its
// rounding error (far below the pad added afterwards).
Box64 transform_box(const double* m, const float* lo, const float* hi) {
  Box64 w;
  for (int r = 0; r < 3; ++r) {
    double c = m[4 * r + 3], e = 0.0, mag = std::fabs(m[4 * r + 3]);
    for (int k = 0; k < 3; ++k) {
      const double ck = 0.5 * ((double)lo[k] + (double)hi[k]);
      const double ek = 0.5 * ((double)hi[k] - (double)lo[k]);
      c += m[4 * r + k] * ck;
      e += std::fabs(m[4 * r + k]) * ek;
      mag += std::fabs(m[4 * r + k]) * (std::fabs(ck) + ek);
    }
    // a few FP64 roundings, each within 2^-53 of the magnitudes involved:
    // widen by 2^-40 of them
    const double slack = std::ldexp(mag, -40);
    w.lo[r] = c - e - slack;
    w.hi[r] = c + e + slack;
  }
  return w;
}

float round_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}

float round_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

struct Child {
  uint32_t ref;
  float lo[3], hi[3];
};

int children(const std::vector<WideNode>& nodes, uint32_t ref, Child out[kMaxWidth]) {
  const WideNode& n = nodes[ref];
  int c = 0;
  for (int k = 0; k < kMaxWidth; ++k) {
    if (n.child[k] == kEmpty) continue;
    out[c].ref = n.child[k];
    for (int a = 0; a < 3; ++a) {
      out[c].lo[a] = n.lo[a][k];
      out[c].hi[a] = n.hi[a][k];
    }
    ++c;
  }
  return c;
}

}  // namespace

std::vector<TopEntry> open_instances(int64_t n, const float* xform, const int32_t* proto, const Aabb* inst_box,
                                     const double* pad, const std::vector<uint32_t>& proto_root,
                                     const std::vector<int32_t>& proto_qbase, const std::vector<int32_t>& proto_nq,
                                     const std::vector<WideNode>& nodes, const OpenParams& params) {
  std::vector<TopEntry> out((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t p = proto[i];
    out[i] = TopEntry{(uint32_t)i, proto_root[p], (uint32_t)proto_qbase[p], (uint32_t)proto_nq[p], inst_box[i]};
  }
  if (params.budget <= 0 || n == 0) return out;

  // quad range [lo, hi) of every bottom-level node: children follow their parent
  // in the node array, so one sweep from the back sees children first
  std::vector<uint32_t> q_lo(nodes.size()), q_hi(nodes.size());
  for (size_t j = nodes.size(); j-- > 0;) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int k = 0; k < kMaxWidth; ++k) {
      const uint32_t c = nodes[j].child[k];
      if (c == kEmpty) continue;
      uint32_t a, b;
      if (ref_is_leaf(c)) {
        a = leaf_first(c);
        b = a + leaf_count(c);
      } else {
        a = q_lo[c];
        b = q_hi[c];
      }
      lo = std::min(lo, a);
      hi = std::max(hi, b);
    }
    q_lo[j] = lo;
    q_hi[j] = hi;
  }

  // padded, clipped world box of one child of instance i
  auto child_box = [&](int64_t i, const double* m, const Child& c) {
    const Box64 w = transform_box(m, c.lo, c.hi);
    const Aabb& ib = inst_box[i];
    Aabb b;
    for (int r = 0; r < 3; ++r) {
      b.lo[r] = std::max(round_down(w.lo[r] - pad[i]), ib.lo[r]);
      b.hi[r] = std::min(round_up(w.hi[r] + pad[i]), ib.hi[r]);
      if (!(b.lo[r] <= b.hi[r])) return ib;  // both contain the subtree, so this cannot happen; stay conservative
    }
    return b;
  };
  auto box64 = [](const Aabb& a) {
    Box64 b;
    for (int r = 0; r < 3; ++r) {
      b.lo[r] = a.lo[r];
      b.hi[r] = a.hi[r];
    }
    return b;
  };
  auto load_m = [&](int64_t i, double* m) {
    for (int j = 0; j < 12; ++j) m[j] = (double)xform[12 * i + j];
  };
  // priority of opening an entry, or a negative value when it is not worth it
  auto priority = [&](const TopEntry& e) {
    if (ref_is_leaf(e.ref)) return -1.0;
    double m[12];
    load_m(e.inst, m);
    Child ch[kMaxWidth];
    const int nc = children(nodes, e.ref, ch);
    const double a = area(box64(e.box));
    double sum = 0.0;
    for (int k = 0; k < nc; ++k) sum += area(box64(child_box(e.inst, m, ch[k])));
    if (!(sum <= params.max_ratio * a)) return -1.0;
    return a - 0.5 * sum;
  };

  using Item = std::pair<double, uint32_t>;  // (priority, entry index)
  std::vector<double> g0(n);
  {
    const int T = n < 65536 ? 1 : std::max(1, params.threads);
    std::vector<std::thread> th;
    auto part = [&](int t) {
      for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) g0[i] = priority(out[i]);
    };
    for (int t = 1; t < T; ++t) th.emplace_back(part, t);
    part(0);
    for (auto& x : th) x.join();
  }
  std::vector<Item> init;
  for (int64_t i = 0; i < n; ++i)
    if (g0[i] > 0.0) init.push_back({g0[i], (uint32_t)i});
  g0 = std::vector<double>();
  std::priority_queue<Item> heap(std::less<Item>(), std::move(init));
  int64_t extra = 0;
  while (!heap.empty()) {
    const uint32_t ei = heap.top().second;
    heap.pop();
    const TopEntry e = out[ei];
    Child ch[kMaxWidth];
    const int nc = children(nodes, e.ref, ch);
    if (extra + nc - 1 > params.budget) break;
    double m[12];
    load_m(e.inst, m);
    for (int k = 0; k < nc; ++k) {
      TopEntry c;
      c.inst = e.inst;
      c.ref = ch[k].ref;
      if (ref_is_leaf(c.ref)) {
        c.q_first = leaf_first(c.ref);
        c.q_count = leaf_count(c.ref);
      } else {
        c.q_first = q_lo[c.ref];
        c.q_count = q_hi[c.ref] - q_lo[c.ref];
      }
      c.box = child_box(e.inst, m, ch[k]);
      uint32_t slot;
      if (k == 0) {
        slot = ei;
        out[ei] = c;
      } else {
        slot = (uint32_t)out.size();
        out.push_back(c);
      }
      const double g = priority(c);
      if (g > 0.0) heap.push({g, slot});
    }
    extra += nc - 1;
  }
  return out;
}

}  // namespace rtq
