// Host-side BVH construction: binned SAH binary BVH, collapsed to 4-wide nodes,
// emitted as FP32 nodes and as 8-bit quantized nodes.
#pragma once
#include <stdint.h>

#include <vector>

#include "rtq_layout.h"

namespace rtq {

struct Aabb {
  float lo[3], hi[3];
};

struct Bvh4 {
  std::vector<NodeF32> f32;     // local child refs (node index within this BVH)
  std::vector<NodeQ8> q8;       // same topology, quantized boxes
  std::vector<uint32_t> order;  // leaf order -> input primitive index
  Aabb root_box;
  int depth = 0;                // 4-wide levels
};

struct BuildParams {
  int leaf_max = 4;  // primitives per leaf (1..8)
  int bins = 16;     // SAH bins per axis (a job of c primitives uses at most max(32, c))
  bool want_f32 = true;
  bool want_q8 = true;
  int threads = 1;   // host threads for this build (the tree does not depend on it)
};

// Build over n primitive boxes.  Leaves reference [first, first + count) of
// `order` with local indices; relocate() turns them into absolute references.
void build_bvh4(const Aabb* boxes, int64_t n, const BuildParams& p, Bvh4& out);

// Add node_base to every internal child reference and prim_base to every leaf's
// first index.  Returns false when an index overflows its encoding.
bool relocate(Bvh4& b, uint32_t node_base, uint32_t prim_base);

// Quantize one FP32 node into the 8-bit format; every decoded plane is
// verified to contain the FP32 plane (lower <=, upper >=).
NodeQ8 quantize_node(const NodeF32& n);

// Decoded quantized plane, correctly rounded.  The kernels take distances to the
// exact value origin + q 2^e, which lies within half an ulp of it; their slab
// error bound covers that half ulp.
float q8_decode(uint32_t q, int e, float origin);

// Largest |coordinate| any box plane of this BVH can take: finite FP32 child
// planes and, for quantized nodes, the node origin and origin + 255 2^e of every
// axis.  The kernels scale their slab error bound with it.
float level_pmax(const Bvh4& b);

// Plane bound above which the slab constants could overflow.
constexpr float kMaxPlaneAbs = 1152921504606846976.0f;  // 2^60

}  // namespace rtq
