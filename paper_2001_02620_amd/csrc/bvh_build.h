// Host-side BVH construction: binned SAH binary BVH, collapsed to W-wide nodes,
// kept as exact FP32 boxes and emitted as 8-bit quantized nodes (and, at W = 4,
// as device FP32 nodes).
#pragma once
#include <stdint.h>

#include <vector>

#include "rtq_layout.h"

namespace rtq {

struct Aabb {
  float lo[3], hi[3];
};

// Host form of a node of up to kMaxWidth children (slots beyond the tree's
// width stay empty): exact FP32 child boxes and child references.
struct WideNode {
  float lo[3][kMaxWidth], hi[3][kMaxWidth];
  uint32_t child[kMaxWidth];
};

struct Bvh {
  std::vector<WideNode> nodes;  // local child refs (node index within this BVH)
  std::vector<uint4> q8;        // same topology, quantized: q8_stride(width) uint4 per node
  std::vector<uint32_t> order;  // leaf order -> input primitive index
  Aabb root_box;
  int width = 4;
  int depth = 0;                // W-wide levels
};

struct BuildParams {
  int leaf_max = 4;  // primitives per leaf (1..8)
  int bins = 16;     // SAH bins per axis (a job of c primitives uses at most max(32, c))
  int width = 4;     // children per node: 2, 4 or 8
  bool want_q8 = true;
  int threads = 1;   // host threads for this build (the tree does not depend on it)
};

// Build over n primitive boxes.  Leaves reference [first, first + count) of
// `order` with local indices; relocate() turns them into absolute references.
void build_bvh(const Aabb* boxes, int64_t n, const BuildParams& p, Bvh& out);

// Add node_base to every internal child reference and prim_base to every leaf's
// first index (host nodes and quantized nodes).  Returns false when an index
// overflows its encoding.
bool relocate(Bvh& b, uint32_t node_base, uint32_t prim_base);

// The device FP32 node of a 4-wide host node.
NodeF32 pack_f32(const WideNode& n);

// Quantize the first w children of a node into the 8-bit format of width w
// (q8_stride(w) uint4 at `words`); every decoded plane is verified to contain
// the FP32 plane (lower <=, upper >=).
void quantize_node(const WideNode& n, int w, uint32_t* words);

// Decoded quantized plane, correctly rounded.  The kernels take distances to the
// exact value origin + q 2^e, which lies within half an ulp of it; their slab
// error bound covers that half ulp.
float q8_decode(uint32_t q, int e, float origin);

// Largest |coordinate| any box plane of this BVH can take: finite FP32 child
// planes and, for quantized nodes, the node origin and origin + 255 2^e of every
// axis.  The kernels scale their slab error bound with it.
float level_pmax(const Bvh& b);

// Plane bound above which the slab constants could overflow.
constexpr float kMaxPlaneAbs = 1152921504606846976.0f;  // 2^60

}  // namespace rtq
