// Device memory layout of a built scene, shared by the host builder and the kernels.
//
// Acceleration structure (Section 5.2 of the paper: one BVH per prototype object
// under a top-level BVH over the instances; quads are the primitives):
//   * top level (TLAS): W-wide nodes over instance world boxes; a leaf holds one
//     instance record index.
//   * bottom level (BLAS): W-wide nodes per prototype over its primitives (its
//     quads, or the capsules its curves are traced as); a leaf holds 1..8
//     consecutive primitives of the global leaf-ordered primitive array.
// The node width W (2, 4 or 8) is chosen per scene at build; FP32 nodes exist
// at W = 4 only, quantized nodes at every width.
// Child references are 32-bit offsets from one 64-bit array base per level (the
// GPU analogue of the 32-bit addressing from a uniform base that Section 5.5
// relies on: no object in these scenes needs 64-bit offsets).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtq {

// ---- child references ------------------------------------------------------
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // unused child slot
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kMaxLeafFirst = (1u << 28) - 1;  // 28-bit first index in a leaf

__host__ __device__ inline uint32_t make_leaf(uint32_t first, uint32_t count) {
  return kLeafBit | (first << 3) | (count - 1u);
}
__host__ __device__ inline bool ref_is_leaf(uint32_t r) { return (r & kLeafBit) != 0u; }
__host__ __device__ inline uint32_t leaf_first(uint32_t r) { return (r & 0x7FFFFFFFu) >> 3; }
__host__ __device__ inline uint32_t leaf_count(uint32_t r) { return (r & 7u) + 1u; }

// ---- FP32 4-wide node: 128 B, one cache line -------------------------------
// Planes are stored structure-of-arrays inside the node so that one 16-byte load
// fetches the same plane of all four children.
struct alignas(16) NodeF32 {
  float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
  uint32_t child[4];
  uint32_t pad[4];
};
static_assert(sizeof(NodeF32) == 128, "NodeF32 is 128 B");

// ---- quantized 4-wide node: 64 B ---------------------------------------------
// Child box planes are 8-bit integers q in a per-node FP32 frame:
//   plane = fmaf(q, 2^e_axis, origin_axis)
// The product q 2^e is exact, so each decoded plane is one correctly rounded
// FP32 value; the builder picks q (floor for lower, ceil for upper planes, then
// verified with this very expression) so every decoded box contains the exact
// FP32 child box.  An empty slot has lo = 255, hi = 0 and child = kEmpty.
struct alignas(16) NodeQ8 {
  float ox, oy, oz;
  uint32_t exps;  // byte k: int8 exponent of axis k (k = 0..2)
  uint32_t lo_x, hi_x, lo_y, hi_y;  // 4 x u8 each (child c in byte c)
  uint32_t lo_z, hi_z;
  uint32_t child[4];
  uint32_t pad[2];
};
static_assert(sizeof(NodeQ8) == 64, "NodeQ8 is 64 B");

// ---- quantized 8-wide node: 96 B ---------------------------------------------
// The 4-wide frame and decode with two words per plane set: children 0..3 in
// the first word of a pair, 4..7 in the second.
struct alignas(16) NodeQ8W8 {
  float ox, oy, oz;
  uint32_t exps;
  uint32_t lo_x[2], hi_x[2];
  uint32_t lo_y[2], hi_y[2];
  uint32_t lo_z[2], hi_z[2];
  uint32_t child[8];
};
static_assert(sizeof(NodeQ8W8) == 96, "NodeQ8W8 is 96 B");

// ---- quantized 2-wide node: 48 B ---------------------------------------------
// One word per axis: lower planes of children 0, 1 in bytes 0, 1 and upper
// planes in bytes 2, 3.
struct alignas(16) NodeQ8W2 {
  float ox, oy, oz;
  uint32_t exps;
  uint32_t x, y, z;
  uint32_t child[2];
  uint32_t pad[3];
};
static_assert(sizeof(NodeQ8W2) == 48, "NodeQ8W2 is 48 B");

constexpr int kMaxWidth = 8;

// Kernel node codecs: FP32 4-wide, and quantized 4-, 8- and 2-wide.
constexpr int kCodecF32 = 1, kCodecQ8 = 2, kCodecQ8W8 = 3, kCodecQ8W2 = 4;
// Flag added to the codec of a scene with curves: its kernels carry the capsule
// test beside the quad test, while scenes of quads alone run kernels without it
// (fewer registers, more waves per SIMD).
constexpr int kCodecCurves = 16;
constexpr int kCodecMask = 15;

// uint4 words per quantized node of width w, and the 32-bit word at which its
// child references start.
__host__ __device__ constexpr int q8_stride(int w) { return w == 8 ? 6 : (w == 2 ? 3 : 4); }
__host__ __device__ constexpr int q8_child_word(int w) { return w == 8 ? 16 : (w == 2 ? 7 : 10); }

// ---- instance record: 64 B ------------------------------------------------------
// r0..r2: rows of the inverse linear part A^-1 (xyz) and the translation t (w), so
// that the object-space ray is o' = A^-1 (o - t), d' = A^-1 d (t stays in the
// same units in both spaces).  The inverse is computed in FP64 at build.
struct alignas(16) InstRec {
  float r0[4], r1[4], r2[4];
  uint32_t blas_root;  // absolute index of the prototype's root node
  uint32_t inst_id;    // caller's instance index
  uint32_t face_base;  // first unique face of the prototype (albedo index base)
  uint32_t proto;      // prototype index, kProtoCurve set for a prototype of curves
};
static_assert(sizeof(InstRec) == 64, "InstRec is 64 B");

// Primitives are stored in leaf order as 3 x float4.  A quad:
//   (v0.x v0.y v0.z v1.x) (v1.y v1.z v2.x v2.y) (v2.z v3.x v3.y v3.z)
// A curve segment (a capsule of radius r = rb, or a ribbon of radius r at a
// and rb at b):
//   (a.x a.y a.z r) (b.x b.y b.z rb) (0 0 0 0)
constexpr int kQuadFloat4 = 3;

// Curves (Section 5.2): a cubic Bezier traced as kCapsPerCurve capsules; the
// capsules of curve c of a prototype are its primitives kCapsPerCurve c + j.
constexpr int kCapsPerCurve = 8;
constexpr uint32_t kProtoCurve = 0x80000000u;  // InstRec::proto flag: the prototype holds curves
constexpr uint32_t kProtoFlat = 0x40000000u;   // ... and they are flat ribbons (set with kProtoCurve)

// Traversal stack per lane: every W-wide level pushes at most W - 1 entries,
// so a scene needs (W - 1) (top depth + bottom depth) + 8 entries at most; the
// build rejects deeper trees.
constexpr int kStackTotal = 192;

// Work counters of one persistent launch: kClaimSlices counters, each on its own
// 128-byte line (kClaimStride 64-bit words apart).
constexpr int kClaimSlices = 8;
constexpr int kClaimStride = 16;
constexpr int kClaimWords = kClaimSlices * kClaimStride;

}  // namespace rtq
