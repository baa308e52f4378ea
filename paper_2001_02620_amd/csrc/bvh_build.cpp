// Binned SAH construction (after Wald 2007) of a binary BVH, collapse to W-wide
// nodes (W = 2, 4 or 8), and 8-bit quantization of child boxes in an FP32
// parent frame (the compressed-node idea of Ylitie, Karras, Laine 2017).
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

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

// Run fn(t) for t in [0, T) on T threads (the caller's thread takes t = 0).
template <class Fn>
void run_threads(int T, Fn&& fn) {
  if (T <= 1) {
    fn(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (int t = 1; t < T; ++t) th.emplace_back([&fn, t] { fn(t); });
  fn(0);
  for (auto& x : th) x.join();
}

// Top-down binned SAH build of a binary BVH.  Jobs with many primitives are
// split one at a time, each with its bounds, bins and partition computed on all
// threads; the remaining subtrees are built concurrently, one per thread, in
// node ranges reserved in advance.  Every partition is stable and every
// reduction is a min/max or an integer sum, so the tree does not depend on the
// thread count.
struct Builder {
  const Aabb* in;
  const BuildParams& p;
  int threads;
  std::vector<float> cx, cy, cz;
  std::vector<uint32_t> idx, tmp;
  std::vector<Node2> nodes;

  struct Job {
    int32_t node;
    int64_t first, count;
    int depth;
  };
  // bounds and per-axis bins of a range of primitives
  struct Bins {
    Box b, cb;
    std::vector<Box> bb;      // 3 x B
    std::vector<int64_t> bc;  // 3 x B
  };
  // per-thread scratch, reused across jobs
  struct Scratch {
    std::vector<Bins> part;
    std::vector<Box> bb;
    std::vector<int64_t> bc, right_count, nl;
    std::vector<double> right_area;
    std::vector<uint32_t> buf;
  };

  Builder(const Aabb* boxes, int64_t n, const BuildParams& prm, int nthreads)
      : in(boxes), p(prm), threads(std::max(1, nthreads)) {
    cx.resize(n);
    cy.resize(n);
    cz.resize(n);
    idx.resize(n);
    const int T = n < 65536 ? 1 : threads;
    run_threads(T, [&](int t) {
      const int64_t a = n * t / T, e = n * (t + 1) / T;
      for (int64_t i = a; i < e; ++i) {
        cx[i] = 0.5f * (in[i].lo[0] + in[i].hi[0]);
        cy[i] = 0.5f * (in[i].lo[1] + in[i].hi[1]);
        cz[i] = 0.5f * (in[i].lo[2] + in[i].hi[2]);
        idx[i] = (uint32_t)i;
      }
    });
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

  void bounds(int64_t a, int64_t e, Box& b, Box& cb) const {
    for (int64_t i = a; i < e; ++i) {
      const uint32_t q = idx[i];
      b.grow(box_of(q));
      cb.grow_pt(cx[q], cy[q], cz[q]);
    }
  }
  // bins for a job of c primitives: the configured count, but no more than
  // max(32, c) (more bins than primitives only cost time)
  int bins_for(int64_t c) const { return (int)std::min<int64_t>(p.bins, std::max<int64_t>(32, c)); }
  void bin(int64_t a, int64_t e, const Box& cb, int B, Bins& out) const {
    for (int ax = 0; ax < 3; ++ax) {
      const float lo = cb.lo[ax], ext = cb.hi[ax] - cb.lo[ax];
      if (!(ext > 0.0f)) continue;
      const float scale = (float)B / ext;
      for (int64_t i = a; i < e; ++i) {
        const uint32_t q = idx[i];
        const int k = std::min(B - 1, (int)((cen(q, ax) - lo) * scale));
        out.bb[ax * B + k].grow(box_of(q));
        out.bc[ax * B + k]++;
      }
    }
  }

  // Bounds, SAH split and partition of job j on T threads.  Returns the split
  // position, or -1 when j becomes a leaf.
  int64_t split(const Job& j, int T, Scratch& S) {
    const int64_t f = j.first, c = j.count;
    const int B = bins_for(c);
    if (c < 4096) T = 1;
    std::vector<Bins>& part = S.part;
    if ((int)part.size() < T) part.resize(T);
    for (int t = 0; t < T; ++t) {
      part[t].b = Box{};
      part[t].cb = Box{};
      part[t].bb.assign(3 * B, Box{});
      part[t].bc.assign(3 * B, 0);
    }
    run_threads(T, [&](int t) { bounds(f + c * t / T, f + c * (t + 1) / T, part[t].b, part[t].cb); });
    Box b, cb;
    for (int t = 0; t < T; ++t) {
      b.grow(part[t].b);
      cb.grow(part[t].cb);
    }
    nodes[j.node].b = b;
    const double A = std::max(b.area(), 1e-300);
    int best_axis = -1, best_bin = -1;
    double best_cost = std::numeric_limits<double>::infinity();
    if (c > 1) {
      run_threads(T, [&](int t) { bin(f + c * t / T, f + c * (t + 1) / T, cb, B, part[t]); });
      std::vector<double>& right_area = S.right_area;
      std::vector<int64_t>& right_count = S.right_count;
      right_area.resize(B);
      right_count.resize(B);
      for (int ax = 0; ax < 3; ++ax) {
        if (!(cb.hi[ax] - cb.lo[ax] > 0.0f)) continue;
        std::vector<Box>& bb = S.bb;
        std::vector<int64_t>& bc = S.bc;
        bb.assign(B, Box{});
        bc.assign(B, 0);
        for (int t = 0; t < T; ++t)
          for (int k = 0; k < B; ++k) {
            bb[k].grow(part[t].bb[ax * B + k]);
            bc[k] += part[t].bc[ax * B + k];
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
    }
    const bool can_leaf = c <= p.leaf_max;
    if (c == 1 || (can_leaf && (best_axis < 0 || (double)c <= best_cost))) {
      nodes[j.node].first = (int32_t)f;
      nodes[j.node].count = (int32_t)c;
      return -1;
    }
    int64_t mid;
    if (best_axis >= 0 && j.depth < 48) {
      const float lo = cb.lo[best_axis], scale = (float)B / (cb.hi[best_axis] - cb.lo[best_axis]);
      auto left = [&](uint32_t q) { return std::min(B - 1, (int)((cen(q, best_axis) - lo) * scale)) <= best_bin; };
      if (T == 1) {
        // stable: left elements compacted in place, right ones through S.buf
        S.buf.clear();
        int64_t w = f;
        for (int64_t i = f; i < f + c; ++i) {
          const uint32_t q = idx[i];
          if (left(q)) idx[w++] = q;
          else S.buf.push_back(q);
        }
        std::copy(S.buf.begin(), S.buf.end(), idx.begin() + w);
        mid = w;
      } else {
        // stable two-pass partition through tmp: count, then scatter
        std::vector<int64_t>& nl = S.nl;
        nl.assign(T + 1, 0);
        run_threads(T, [&](int t) {
          int64_t k = 0;
          for (int64_t i = f + c * t / T; i < f + c * (t + 1) / T; ++i) k += left(idx[i]) ? 1 : 0;
          nl[t + 1] = k;
        });
        for (int t = 0; t < T; ++t) nl[t + 1] += nl[t];
        const int64_t total_left = nl[T];
        run_threads(T, [&](int t) {
          const int64_t a = f + c * t / T, e = f + c * (t + 1) / T;
          int64_t wl = f + nl[t], wr = f + total_left + (a - f - nl[t]);
          for (int64_t i = a; i < e; ++i) {
            const uint32_t q = idx[i];
            if (left(q)) tmp[wl++] = q;
            else tmp[wr++] = q;
          }
        });
        run_threads(T, [&](int t) {
          std::copy(tmp.begin() + f + c * t / T, tmp.begin() + f + c * (t + 1) / T, idx.begin() + f + c * t / T);
        });
        mid = f + total_left;
      }
    } else {
      // no usable SAH split (identical centroids, or too deep): object median
      int ax = 0;
      float e = -1.0f;
      for (int k = 0; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > e) {
          e = cb.hi[k] - cb.lo[k];
          ax = k;
        }
      mid = f + c / 2;
      std::nth_element(idx.begin() + f, idx.begin() + mid, idx.begin() + f + c,
                       [&](uint32_t a, uint32_t d) { return cen(a, ax) < cen(d, ax); });
    }
    if (mid == f || mid == f + c) mid = f + c / 2;
    return mid;
  }

  // Depth-first build of the subtree of j on the calling thread; children take
  // node slots from *next.
  void subtree(const Job& root, int32_t* next) {
    Scratch S;
    std::vector<Job> jobs{root};
    while (!jobs.empty()) {
      const Job j = jobs.back();
      jobs.pop_back();
      const int64_t mid = split(j, 1, S);
      if (mid < 0) continue;
      const int32_t l = *next;
      *next += 2;
      nodes[j.node].l = l;
      nodes[j.node].r = l + 1;
      jobs.push_back({l, j.first, mid - j.first, j.depth + 1});
      jobs.push_back({l + 1, mid, j.first + j.count - mid, j.depth + 1});
    }
  }

  void run() {
    const int64_t n = (int64_t)idx.size();
    nodes.assign(2 * n + 1, Node2{});
    int32_t next = 1;
    if (threads == 1 || n < 65536) {
      subtree({0, 0, n, 0}, &next);
      nodes.resize(next);
      return;
    }
    tmp.resize(n);
    // large jobs, breadth first, each split on every thread
    const int64_t big = std::max<int64_t>(65536, n / (16 * threads));
    std::vector<Job> queue{{0, 0, n, 0}}, small;
    Scratch S;
    for (size_t h = 0; h < queue.size(); ++h) {
      const Job j = queue[h];
      const int64_t mid = split(j, threads, S);
      if (mid < 0) continue;
      const int32_t l = next;
      next += 2;
      nodes[j.node].l = l;
      nodes[j.node].r = l + 1;
      const Job kids[2] = {{l, j.first, mid - j.first, j.depth + 1}, {l + 1, mid, j.first + j.count - mid, j.depth + 1}};
      for (const Job& k : kids) (k.count >= big ? queue : small).push_back(k);
    }
    tmp = std::vector<uint32_t>();
    // the rest: one subtree per task; a subtree of c primitives has at most
    // 2c - 2 nodes below its root, reserved in list order
    std::vector<int32_t> base(small.size());
    int64_t at = next;
    for (size_t k = 0; k < small.size(); ++k) {
      base[k] = (int32_t)at;
      at += 2 * small[k].count - 2;
    }
    std::vector<size_t> order(small.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return small[a].count > small[b].count; });
    std::atomic<size_t> take{0};
    run_threads(threads, [&](int) {
      for (;;) {
        const size_t k = take.fetch_add(1);
        if (k >= order.size()) break;
        int32_t nx = base[order[k]];
        subtree(small[order[k]], &nx);
      }
    });
  }
};

float bit_float(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void set_child(WideNode& n, int k, const Box& b, uint32_t ref) {
  for (int a = 0; a < 3; ++a) {
    n.lo[a][k] = b.lo[a];
    n.hi[a][k] = b.hi[a];
  }
  n.child[k] = ref;
}

void empty_node(WideNode& n) {
  for (int k = 0; k < kMaxWidth; ++k) {
    for (int a = 0; a < 3; ++a) {
      n.lo[a][k] = kInf;
      n.hi[a][k] = -kInf;
    }
    n.child[k] = kEmpty;
  }
}

// Quantized planes of one axis over the first w children: the frame origin, the
// exponent and the byte planes (lower rounded down, upper up, each verified by
// decoding it the kernels' way).  Empty slots get lo = 255, hi = 0.
void quantize_axis(const WideNode& n, int w, int a, float* org, int* ex, uint32_t* qlo, uint32_t* qhi) {
  float lo = kInf, hi = -kInf;
  for (int k = 0; k < w; ++k)
    if (n.child[k] != kEmpty) {
      lo = std::min(lo, n.lo[a][k]);
      hi = std::max(hi, n.hi[a][k]);
    }
  if (!(lo <= hi)) lo = hi = 0.0f;  // no children at all
  *org = lo;
  const double ext = (double)hi - (double)lo;
  int e = -126;
  if (ext > 0.0) e = std::max(-126, (int)std::ceil(std::log2(ext / 255.0)));
  for (;;) {
    bool ok = true;
    for (int k = 0; k < w && ok; ++k) {
      if (n.child[k] == kEmpty) {
        qlo[k] = 255u;
        qhi[k] = 0u;
        continue;
      }
      const double sc = std::ldexp(1.0, e);
      const double fl = std::floor(((double)n.lo[a][k] - (double)lo) / sc);
      const double ce = std::ceil(((double)n.hi[a][k] - (double)lo) / sc);
      int64_t ql = std::max<int64_t>(0, (int64_t)fl);
      int64_t qh = std::max<int64_t>(0, (int64_t)ce);
      while (ql > 0 && q8_decode((uint32_t)ql, e, lo) > n.lo[a][k]) --ql;
      while (qh <= 255 && q8_decode((uint32_t)qh, e, lo) < n.hi[a][k]) ++qh;
      if (ql > 255 || qh > 255 || q8_decode((uint32_t)ql, e, lo) > n.lo[a][k]) {
        ok = false;
        break;
      }
      qlo[k] = (uint32_t)ql;
      qhi[k] = (uint32_t)qh;
    }
    if (ok) break;
    ++e;
  }
  *ex = e;
}

}  // namespace

float q8_decode(uint32_t q, int e, float origin) {
  return std::fma((float)q, std::ldexp(1.0f, e), origin);
}

NodeF32 pack_f32(const WideNode& n) {
  NodeF32 o;
  std::memset(&o, 0, sizeof(o));
  for (int k = 0; k < 4; ++k) {
    o.lo_x[k] = n.lo[0][k];
    o.hi_x[k] = n.hi[0][k];
    o.lo_y[k] = n.lo[1][k];
    o.hi_y[k] = n.hi[1][k];
    o.lo_z[k] = n.lo[2][k];
    o.hi_z[k] = n.hi[2][k];
    o.child[k] = n.child[k];
  }
  return o;
}

void quantize_node(const WideNode& n, int w, uint32_t* words) {
  float org[3];
  int ex[3];
  uint32_t qlo[3][kMaxWidth], qhi[3][kMaxWidth];
  for (int a = 0; a < 3; ++a) quantize_axis(n, w, a, &org[a], &ex[a], qlo[a], qhi[a]);
  std::memset(words, 0, 16 * q8_stride(w));
  std::memcpy(&words[0], &org[0], 4);
  std::memcpy(&words[1], &org[1], 4);
  std::memcpy(&words[2], &org[2], 4);
  words[3] = (uint32_t)(uint8_t)(int8_t)ex[0] | ((uint32_t)(uint8_t)(int8_t)ex[1] << 8) |
             ((uint32_t)(uint8_t)(int8_t)ex[2] << 16);
  auto pack4 = [](const uint32_t* q) { return q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24); };
  for (int a = 0; a < 3; ++a) {
    if (w == 4) {
      words[4 + 2 * a] = pack4(qlo[a]);
      words[5 + 2 * a] = pack4(qhi[a]);
    } else if (w == 8) {
      words[4 + 4 * a] = pack4(qlo[a]);
      words[5 + 4 * a] = pack4(qlo[a] + 4);
      words[6 + 4 * a] = pack4(qhi[a]);
      words[7 + 4 * a] = pack4(qhi[a] + 4);
    } else {
      words[4 + a] = qlo[a][0] | (qlo[a][1] << 8) | (qhi[a][0] << 16) | (qhi[a][1] << 24);
    }
  }
  for (int k = 0; k < w; ++k) words[q8_child_word(w) + k] = n.child[k];
}

void build_bvh(const Aabb* boxes, int64_t n, const BuildParams& p, Bvh& out) {
  const int W = p.width;
  out.nodes.clear();
  out.q8.clear();
  out.order.clear();
  out.depth = 0;
  out.width = W;
  Builder bld(boxes, n, p, p.threads);
  bld.run();
  out.order = bld.idx;
  const std::vector<Node2>& N = bld.nodes;
  const Box& rb = N[0].b;
  for (int k = 0; k < 3; ++k) {
    out.root_box.lo[k] = rb.lo[k];
    out.root_box.hi[k] = rb.hi[k];
  }
  // collapse: every W-wide node adopts up to W BVH2 descendants, expanding
  // the internal child of largest surface area first
  struct Job {
    int32_t n2;      // BVH2 node whose subtree this W-wide node covers
    uint32_t slot;   // W-wide node index
    int depth;
  };
  out.nodes.emplace_back();
  empty_node(out.nodes[0]);
  std::vector<Job> jobs{{0, 0u, 1}};
  while (!jobs.empty()) {
    const Job j = jobs.back();
    jobs.pop_back();
    out.depth = std::max(out.depth, j.depth);
    int32_t kids[kMaxWidth];
    int nk = 0;
    if (N[j.n2].count > 0) {
      kids[nk++] = j.n2;  // a leaf root: one leaf child
    } else {
      kids[nk++] = N[j.n2].l;
      kids[nk++] = N[j.n2].r;
      while (nk < W) {
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
    WideNode node;
    empty_node(node);
    for (int k = 0; k < nk; ++k) {
      const Node2& c = N[kids[k]];
      uint32_t ref;
      if (c.count > 0) {
        ref = make_leaf((uint32_t)c.first, (uint32_t)c.count);
      } else {
        ref = (uint32_t)out.nodes.size();
        out.nodes.emplace_back();
        jobs.push_back({kids[k], ref, j.depth + 1});
      }
      set_child(node, k, c.b, ref);
    }
    out.nodes[j.slot] = node;
  }
  if (p.want_q8) {
    const int st = q8_stride(W);
    out.q8.resize(out.nodes.size() * st);
    const int64_t m = (int64_t)out.nodes.size();
    const int T = m < 65536 ? 1 : std::max(1, p.threads);
    run_threads(T, [&](int t) {
      for (int64_t i = m * t / T; i < m * (t + 1) / T; ++i)
        quantize_node(out.nodes[i], W, reinterpret_cast<uint32_t*>(&out.q8[i * st]));
    });
  }
}

float level_pmax(const Bvh& b) {
  double m = 0.0;
  for (const WideNode& n : b.nodes)
    for (int k = 0; k < b.width; ++k) {
      if (n.child[k] == kEmpty) continue;
      for (int a = 0; a < 3; ++a)
        m = std::max(m, std::max(std::fabs((double)n.lo[a][k]), std::fabs((double)n.hi[a][k])));
    }
  const size_t st = q8_stride(b.width);
  for (size_t i = 0; i < b.q8.size(); i += st) {
    const uint4 h = b.q8[i];
    const float org[3] = {bit_float(h.x), bit_float(h.y), bit_float(h.z)};
    for (int a = 0; a < 3; ++a) {
      const int e = (int)(int8_t)((h.w >> (8 * a)) & 0xFFu);
      m = std::max(m, std::fabs((double)org[a]));
      m = std::max(m, std::fabs((double)org[a] + 255.0 * std::ldexp(1.0, e)));
    }
  }
  // round up so that the FP32 bound is not below the exact maximum
  const float f = (float)m;
  return (double)f >= m ? f : std::nextafter(f, std::numeric_limits<float>::infinity());
}

bool relocate(Bvh& b, uint32_t node_base, uint32_t prim_base) {
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
  for (auto& nd : b.nodes)
    for (int k = 0; k < b.width; ++k)
      if (!fix(nd.child[k])) return false;
  const size_t st = q8_stride(b.width);
  for (size_t i = 0; i < b.q8.size(); i += st) {
    uint32_t* w = reinterpret_cast<uint32_t*>(&b.q8[i]) + q8_child_word(b.width);
    for (int k = 0; k < b.width; ++k)
      if (!fix(w[k])) return false;
  }
  return true;
}

}  // namespace rtq
