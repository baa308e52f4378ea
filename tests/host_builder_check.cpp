// Host-side check of the scene builder, compiled by tests/test_host_sanitizers.py
// under AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer:
// 2-, 4- and 8-wide BVH builds over random boxes (duplicates, flat and point
// boxes, any leaf size, bin count and thread count) must give a permutation as
// leaf order;
// instance opening over random prototypes and transforms must stay within its
// budget, keep every entry's quads inside its prototype and its box inside the
// instance box, and cover each instance's quads exactly once.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "bvh_build.h"
#include "rebraid.h"
using namespace rtq;
static Aabb rand_box(std::mt19937_64& g, float spread) {
  std::uniform_real_distribution<float> U(-spread, spread), E(0.0f, 2.0f);
  Aabb b;
  for (int k = 0; k < 3; ++k) {
    float c = U(g), e = (g() % 10 == 0) ? 0.0f : E(g);
    b.lo[k] = c - e;
    b.hi[k] = c + e;
  }
  return b;
}
int main() {
  std::mt19937_64 g(11);
  long checks = 0;
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t n = 1 + (int64_t)(g() % (trial < 10 ? 20 : 40000));
    std::vector<Aabb> b(n);
    for (auto& x : b) x = rand_box(g, 100.0f);
    if (trial % 7 == 3) for (auto& x : b) x = b[0];
    BuildParams p;
    p.leaf_max = 1 + (int)(g() % 8);
    p.bins = 4 + (int)(g() % 60);
    p.threads = 1 + (int)(g() % 8);
    p.width = 2 << (trial % 3);
    Bvh out;
    build_bvh(b.data(), n, p, out);
    std::vector<int> seen(n, 0);
    for (uint32_t o : out.order) seen[o]++;
    for (int64_t i = 0; i < n; ++i)
      if (seen[i] != 1) { std::printf("order not a permutation\n"); return 1; }
    uint32_t words[24];
    for (const WideNode& nd : out.nodes) quantize_node(nd, p.width, words);
    if (p.width == 4)
      for (const WideNode& nd : out.nodes) (void)pack_f32(nd);
    ++checks;
  }
  // instance opening over a few prototypes
  for (int trial = 0; trial < 10; ++trial) {
    const int P = 1 + (int)(g() % 4);
    std::vector<WideNode> nodes;
    const int width = 2 << (trial % 3);
    std::vector<uint32_t> root(P);
    std::vector<int32_t> qbase(P), nq(P);
    std::vector<Aabb> pbox(P);
    uint32_t node_base = 0, quad_base = 0;
    for (int pi = 0; pi < P; ++pi) {
      const int64_t n = 1 + (int64_t)(g() % 5000);
      std::vector<Aabb> b(n);
      for (auto& x : b) x = rand_box(g, 5.0f);
      BuildParams bp;
      bp.threads = 2;
      bp.width = width;
      Bvh out;
      build_bvh(b.data(), n, bp, out);
      if (!relocate(out, node_base, quad_base)) { std::printf("relocate failed\n"); return 1; }
      root[pi] = node_base;
      qbase[pi] = (int32_t)quad_base;
      nq[pi] = (int32_t)n;
      pbox[pi] = out.root_box;
      nodes.insert(nodes.end(), out.nodes.begin(), out.nodes.end());
      node_base += (uint32_t)out.nodes.size();
      quad_base += (uint32_t)n;
    }
    const int64_t N = 1 + (int64_t)(g() % 3000);
    std::vector<float> xf(12 * N);
    std::vector<int32_t> proto(N);
    std::vector<Aabb> ibox(N);
    std::vector<double> pad(N, 1e-3);
    std::uniform_real_distribution<float> U(-50, 50), S(0.5f, 2.0f);
    for (int64_t i = 0; i < N; ++i) {
      const float s = S(g);
      float m[12] = {s, 0, 0, U(g), 0, s, 0, U(g), 0, 0, s, U(g)};
      for (int k = 0; k < 12; ++k) xf[12 * i + k] = m[k];
      proto[i] = (int32_t)(g() % P);
      const Aabb& pb = pbox[proto[i]];
      for (int r = 0; r < 3; ++r) {
        ibox[i].lo[r] = (float)(s * pb.lo[r] + m[4 * r + 3] - 1e-2);
        ibox[i].hi[r] = (float)(s * pb.hi[r] + m[4 * r + 3] + 1e-2);
      }
    }
    OpenParams op;
    op.budget = N * (int64_t)(g() % 200) / 100;
    op.threads = 1 + (int)(g() % 8);
    std::vector<TopEntry> e = open_instances(N, xf.data(), proto.data(), ibox.data(), pad.data(), root, qbase, nq,
                                             nodes, op);
    if ((int64_t)e.size() > N + op.budget) { std::printf("budget exceeded\n"); return 1; }
    std::vector<int64_t> quads(N, 0);
    for (const TopEntry& t : e) {
      const int pp = proto[t.inst];
      if ((int64_t)t.q_first < qbase[pp] || (int64_t)t.q_first + t.q_count > (int64_t)qbase[pp] + nq[pp]) {
        std::printf("quad range outside prototype\n");
        return 1;
      }
      for (int r = 0; r < 3; ++r)
        if (t.box.lo[r] < ibox[t.inst].lo[r] || t.box.hi[r] > ibox[t.inst].hi[r] || t.box.lo[r] > t.box.hi[r]) {
          std::printf("entry box outside instance box\n");
          return 1;
        }
      quads[t.inst] += t.q_count;
    }
    for (int64_t i = 0; i < N; ++i)
      if (quads[i] != nq[proto[i]]) { std::printf("entries of instance %lld do not cover its quads\n", (long long)i); return 1; }
    ++checks;
  }
  std::printf("ok %ld checks\n", checks);
  return 0;
}
