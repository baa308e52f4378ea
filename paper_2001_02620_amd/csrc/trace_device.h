// Device-side closest-hit / any-hit traversal of the two-level quad BVH.
//
// One lane traces one ray.  The traversal stack lives in LDS (a column per lane,
// so lanes of a wave never conflict on a bank) with a private spill region for
// entries beyond the LDS depth.  Entries carry the child's entry distance so a
// popped subtree that lies behind the current closest hit is skipped without
// touching memory.
//
// Exactness rules that make every traversal variant return the same hit:
//   * the leaf test is one function used by every variant (FP32, watertight,
//     contraction off), and its result depends only on (ray, instance, quad);
//   * boxes are tested conservatively: robust slab test (Ize 2013: the far
//     distance is scaled by 1 + 2 gamma_3), quantized boxes contain the exact
//     boxes, instance world boxes are padded for the FP32 ray-transform error
//     and the ray origin is widened by a per-ray pad at the top level;
//   * a box is culled only when its entry distance exceeds t_best (1 + 2^-16);
//   * among hits the smallest key (t, instance id, primitive id, half) wins.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtq_layout.h"

#pragma clang fp contract(off)

namespace rtq {

struct SceneView {
  const uint4* tlas;          // TLAS nodes of the traced format
  const uint4* blas;          // BLAS nodes of the traced format
  const float4* quads;        // leaf-ordered quads, 3 float4 each
  const int32_t* quad_prim;   // leaf order -> quad index within its prototype
  const InstRec* inst;        // instance records in TLAS leaf order
  const int32_t* proto_qbase; // first leaf-ordered quad of each prototype
  const int32_t* proto_nq;    // quads per prototype
  const float* albedo;        // per unique face (prototype order)
  float pad_rel;              // top-level origin pad per unit of |o|_inf
  uint32_t n_inst;
};

// Far-plane scale of the robust slab test: with reciprocals from v_rcp_f32
// (at most 1 ulp) each slab distance carries four rounding factors, so the
// far distance is scaled by 1 + 2^-20 >= 1 + 2 gamma_4 (Ize 2013).
constexpr float kRobust = 1.0f + 9.5367431640625e-07f;
constexpr float kSlack = 1.0f + 1.52587890625e-05f;      // 1 + 2^-16
constexpr float kInfF = __builtin_huge_valf();

// Counter-free selection of component k (0, 1, 2) of (x, y, z).
__device__ __forceinline__ float pick3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

// Ray state of one lane.  Everything stays in registers.
struct Lane {
  // world ray
  float wox, woy, woz, wdx, wdy, wdz, tmin, tmax;
  // ray of the current level for box tests
  float onx, ony, onz;  // origin used for near planes (world level: widened)
  float ofx, ofy, ofz;  // origin used for far planes
  float ix, iy, iz;     // reciprocal direction
  // shear of the watertight leaf test (Woop, Benthin, Wald 2013); inside an
  // instance the leaf test uses the object-space origin (on*) as its origin
  float Sx, Sy, Sz;
  int kz;            // dominant axis of the object-space direction
  // traversal
  uint32_t cur;      // reference to process next, kEmpty = pop
  int sp;            // stack size
  int inst_sp;       // stack size when the current instance was entered, -1 at top level
  uint32_t rec;      // current instance record
  // best hit so far: record, leaf-ordered quad | half << 31
  float t_best, t_cull;
  uint32_t b_rec, b_qh;
  float b_u, b_v;
  // exclusion (spawning triangle): record, leaf-ordered quad | half << 31 (kEmpty: none)
  uint32_t ex_rec, ex_qh;
  bool any;   // any-hit query: stop at the first accepted hit
  bool done;  // traversal finished
};

// Hardware reciprocal (v_rcp_f32, 1 ulp): used for the slab test and the
// leaf test's shear and t.  Every traversal variant evaluates the same
// expressions, so the hits stay identical across variants.
__device__ __forceinline__ float rcp_fast(float d) { return __builtin_amdgcn_rcpf(d); }

// Set the box-test ray for the top level: the world ray with its origin widened
// by pad = pad_rel |o|_inf toward the near and far planes.
__device__ __forceinline__ void set_world_box_ray(Lane& L, float pad_rel) {
  L.ix = rcp_fast(L.wdx);
  L.iy = rcp_fast(L.wdy);
  L.iz = rcp_fast(L.wdz);
  const float m = fmaxf(fabsf(L.wox), fmaxf(fabsf(L.woy), fabsf(L.woz)));
  const float pad = pad_rel * m;
  // near plane of a positive-direction axis is lo: widen by moving the origin up
  L.onx = L.ix >= 0.0f ? L.wox + pad : L.wox - pad;
  L.ofx = L.ix >= 0.0f ? L.wox - pad : L.wox + pad;
  L.ony = L.iy >= 0.0f ? L.woy + pad : L.woy - pad;
  L.ofy = L.iy >= 0.0f ? L.woy - pad : L.woy + pad;
  L.onz = L.iz >= 0.0f ? L.woz + pad : L.woz - pad;
  L.ofz = L.iz >= 0.0f ? L.woz - pad : L.woz + pad;
}

// Enter instance `r`: transform the ray to object space, o' = A^-1 (o - t),
// d' = A^-1 d, and prepare the box test and the shear of the leaf test.
__device__ __forceinline__ void enter_instance(Lane& L, const InstRec* __restrict__ inst, uint32_t r,
                                               uint32_t* blas_root) {
  const float4 a = *reinterpret_cast<const float4*>(inst[r].r0);
  const float4 b = *reinterpret_cast<const float4*>(inst[r].r1);
  const float4 c = *reinterpret_cast<const float4*>(inst[r].r2);
  const uint4 m = *reinterpret_cast<const uint4*>(&inst[r].blas_root);
  const float px = L.wox - a.w, py = L.woy - b.w, pz = L.woz - c.w;
  const float ox = a.x * px + a.y * py + a.z * pz;
  const float oy = b.x * px + b.y * py + b.z * pz;
  const float oz = c.x * px + c.y * py + c.z * pz;
  const float dx = a.x * L.wdx + a.y * L.wdy + a.z * L.wdz;
  const float dy = b.x * L.wdx + b.y * L.wdy + b.z * L.wdz;
  const float dz = c.x * L.wdx + c.y * L.wdy + c.z * L.wdz;
  L.ix = rcp_fast(dx);
  L.iy = rcp_fast(dy);
  L.iz = rcp_fast(dz);
  L.onx = L.ofx = ox;
  L.ony = L.ofy = oy;
  L.onz = L.ofz = oz;
  const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  const int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  const int kx = kz == 2 ? 0 : kz + 1;
  const int ky = kx == 2 ? 0 : kx + 1;
  L.kz = kz;
  const float dkz = pick3(dx, dy, dz, kz);
  L.Sz = rcp_fast(dkz);
  L.Sx = pick3(dx, dy, dz, kx) * L.Sz;
  L.Sy = pick3(dx, dy, dz, ky) * L.Sz;
  L.rec = r;
  *blas_root = m.x;
}

// ---- leaf test -----------------------------------------------------------------
// Sheared vertex (Woop, Benthin, Wald 2013): X, Y in the plane orthogonal to the
// ray, Z along it.  The shear of a vertex depends only on (vertex, ray), so a
// vertex shared by two quads gets bit-identical coordinates in both.
struct Sv {
  float X, Y, Z;
};
// The two other axes follow kz cyclically; no swap is needed for a two-sided
// test (a swap only flips the sign of every edge function).
__device__ __forceinline__ Sv shear(const Lane& L, int kx, int ky, float vx, float vy, float vz) {
  const float ax = vx - L.onx, ay = vy - L.ony, az = vz - L.onz;
  const float akx = pick3(ax, ay, az, kx);
  const float aky = pick3(ax, ay, az, ky);
  const float akz = pick3(ax, ay, az, L.kz);
  Sv s;
  s.X = akx - L.Sx * akz;
  s.Y = aky - L.Sy * akz;
  s.Z = L.Sz * akz;
  return s;
}
// Edge function e(P, Q) = Qx Py - Qy Px.  With contraction off, e(Q, P) is the
// exact negative of e(P, Q): a shared edge gives the two triangles opposite
// signs bit for bit, which is what makes the test watertight.
__device__ __forceinline__ float edge(const Sv& P, const Sv& Q) { return Q.X * P.Y - Q.Y * P.X; }

struct TriResult {
  bool hit;
  float t, U, V, W, det;
};

// Edge function in FP64: both products of FP32 operands are exact, so the one
// rounding of the difference keeps the exact sign (and zero only when exact).
__device__ __forceinline__ double edge64(const Sv& P, const Sv& Q) {
  return (double)Q.X * (double)P.Y - (double)Q.Y * (double)P.X;
}

// Triangle (A, B, C) with precomputed edge functions U = e(B, C), V = e(C, A),
// W = e(A, B).  Two-sided: all three of one sign (zeros allowed), det != 0.
// Rounding is monotonic, so a non-zero FP32 edge value has the exact sign of the
// edge function of the sheared FP32 vertices; a zero may come from cancellation
// (for instance a distant triangle seen edge-on, whose edge lines all pass close
// to the ray) and is then re-evaluated in FP64, as Woop, Benthin and Wald
// prescribe.  Mixed strict signs are exact and reject at once.
__device__ __forceinline__ TriResult tri_finish(float U, float V, float W, const Sv& A, const Sv& B, const Sv& C,
                                                float tmin, float tmax) {
  TriResult r;
  r.hit = false;
  const bool neg = (U < 0.0f) || (V < 0.0f) || (W < 0.0f);
  const bool pos = (U > 0.0f) || (V > 0.0f) || (W > 0.0f);
  if (neg && pos) return r;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    const double u = edge64(B, C), v = edge64(C, A), w = edge64(A, B);
    const bool n64 = (u < 0.0) || (v < 0.0) || (w < 0.0);
    const bool p64 = (u > 0.0) || (v > 0.0) || (w > 0.0);
    const double det = u + v + w;
    if ((n64 && p64) || det == 0.0) return r;
    const double T = u * (double)A.Z + v * (double)B.Z + w * (double)C.Z;
    const float t = (float)(T / det);
    r.hit = (t > tmin) && (t <= tmax);
    r.t = t;
    // barycentrics already divided: u = V * rcp(det) with det = 1
    r.U = (float)(u / det);
    r.V = (float)(v / det);
    r.W = (float)(w / det);
    r.det = 1.0f;
    return r;
  }
  const float det = U + V + W;
  const float T = U * A.Z + V * B.Z + W * C.Z;
  const float t = T * rcp_fast(det);
  r.hit = (t > tmin) && (t <= tmax);
  r.t = t;
  r.U = U;
  r.V = V;
  r.W = W;
  r.det = det;
  return r;
}

// ---- stack ---------------------------------------------------------------------------
// LDS holds the top `depth` entries of every lane of a wave: references as
// [depth][64] u32 and entry distances as [depth][64] u16 (the upper half of the
// FP32 value, rounded toward -inf, so a popped entry is never culled wrongly).
// Deeper entries spill to a private array.
struct Stack {
  uint32_t* ref;
  uint16_t* tq;
  int depth;  // LDS entries per lane
  int lane;
};

constexpr int kStackEntryBytes = 6;

// Stack region of wave w in a block's dynamic LDS (6 bytes per entry and lane).
__device__ __forceinline__ Stack make_stack(void* lds, int depth) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  uint32_t* refs = reinterpret_cast<uint32_t*>(lds);
  uint16_t* ts = reinterpret_cast<uint16_t*>(refs + (size_t)waves * depth * 64);
  return Stack{refs + wave * depth * 64, ts + wave * depth * 64, depth, lane};
}

// FP32 -> upper 16 bits, rounded toward -inf.
__device__ __forceinline__ uint16_t t_down16(float t) {
  uint32_t b = __float_as_uint(t);
  if ((b & 0x80000000u) && (b & 0xFFFFu)) b += 0x10000u;  // negative: away from zero
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float t_up32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- box tests --------------------------------------------------------------------
// Ordered robust slab test of four children; returns entry distances (kInfF when
// missed).  lo/hi are the planes of axis x, y, z for each child.
__device__ __forceinline__ float slab1(const Lane& L, float nx, float fx, float ny, float fy, float nz, float fz,
                                       float t_lim) {
  const float tnx = (nx - L.onx) * L.ix, tfx = (fx - L.ofx) * L.ix;
  const float tny = (ny - L.ony) * L.iy, tfy = (fy - L.ofy) * L.iy;
  const float tnz = (nz - L.onz) * L.iz, tfz = (fz - L.ofz) * L.iz;
  const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, L.tmin));
  const float tf = fminf(fminf(tfx, tfy), tfz) * kRobust;
  return tn <= fminf(tf, t_lim) ? tn : kInfF;
}

template <int FMT>
struct NodeCodec;

// FP32 nodes: 8 x 16 B loads (planes SoA, children).
template <>
struct NodeCodec<1> {
  static constexpr int kStride = 8;  // uint4 per node
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[4], uint32_t ch[4]) {
    const uint4* p = base + (size_t)idx * kStride;
    const float4 lx = __builtin_bit_cast(float4, p[0]);
    const float4 hx = __builtin_bit_cast(float4, p[1]);
    const float4 ly = __builtin_bit_cast(float4, p[2]);
    const float4 hy = __builtin_bit_cast(float4, p[3]);
    const float4 lz = __builtin_bit_cast(float4, p[4]);
    const float4 hz = __builtin_bit_cast(float4, p[5]);
    const uint4 c = p[6];
    const bool sx = L.ix >= 0.0f, sy = L.iy >= 0.0f, sz = L.iz >= 0.0f;
    const float LX[4] = {lx.x, lx.y, lx.z, lx.w}, HX[4] = {hx.x, hx.y, hx.z, hx.w};
    const float LY[4] = {ly.x, ly.y, ly.z, ly.w}, HY[4] = {hy.x, hy.y, hy.z, hy.w};
    const float LZ[4] = {lz.x, lz.y, lz.z, lz.w}, HZ[4] = {hz.x, hz.y, hz.z, hz.w};
    ch[0] = c.x;
    ch[1] = c.y;
    ch[2] = c.z;
    ch[3] = c.w;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = slab1(L, sx ? LX[k] : HX[k], sx ? HX[k] : LX[k], sy ? LY[k] : HY[k], sy ? HY[k] : LY[k],
                            sz ? LZ[k] : HZ[k], sz ? HZ[k] : LZ[k], t_lim);
      tn[k] = ch[k] == kEmpty ? kInfF : t;
    }
  }
};

// Quantized nodes: 4 x 16 B loads; the near/far byte planes of all four children
// are selected with one select per axis before decoding.
template <>
struct NodeCodec<2> {
  static constexpr int kStride = 4;
  __device__ __forceinline__ static float scale_of(uint32_t e8) {
    const int e = (int)(int8_t)(e8 & 0xFFu);
    return __int_as_float((e + 127) << 23);
  }
  __device__ __forceinline__ static float ub(uint32_t w, int k) {
    return (float)((w >> (8 * k)) & 0xFFu);
  }
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[4], uint32_t ch[4]) {
    const uint4* p = base + (size_t)idx * kStride;
    const uint4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const float ox = __uint_as_float(q0.x), oy = __uint_as_float(q0.y), oz = __uint_as_float(q0.z);
    const float ex = scale_of(q0.w), ey = scale_of(q0.w >> 8), ez = scale_of(q0.w >> 16);
    const bool sx = L.ix >= 0.0f, sy = L.iy >= 0.0f, sz = L.iz >= 0.0f;
    const uint32_t nx = sx ? q1.x : q1.y, fx = sx ? q1.y : q1.x;
    const uint32_t ny = sy ? q1.z : q1.w, fy = sy ? q1.w : q1.z;
    const uint32_t nz = sz ? q2.x : q2.y, fz = sz ? q2.y : q2.x;
    ch[0] = q2.z;
    ch[1] = q2.w;
    ch[2] = q3.x;
    ch[3] = q3.y;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = slab1(L, fmaf(ub(nx, k), ex, ox), fmaf(ub(fx, k), ex, ox), fmaf(ub(ny, k), ey, oy),
                            fmaf(ub(fy, k), ey, oy), fmaf(ub(nz, k), ez, oz), fmaf(ub(fz, k), ez, oz), t_lim);
      tn[k] = ch[k] == kEmpty ? kInfF : t;
    }
  }
};

__device__ __forceinline__ void cswap(float& ta, uint32_t& ra, float& tb, uint32_t& rb) {
  const bool s = tb < ta;
  const float t0 = s ? tb : ta, t1 = s ? ta : tb;
  const uint32_t r0 = s ? rb : ra, r1 = s ? ra : rb;
  ta = t0;
  tb = t1;
  ra = r0;
  rb = r1;
}

__device__ __forceinline__ void push(Lane& L, const Stack& S, uint2* spill, uint32_t ref, float t) {
  if (L.sp < S.depth) {
    S.ref[L.sp * 64 + S.lane] = ref;
    S.tq[L.sp * 64 + S.lane] = t_down16(t);
  } else {
    spill[L.sp - S.depth] = make_uint2(ref, __float_as_uint(t));
  }
  ++L.sp;
}

// Pop the top entry: (reference, lower bound of its entry distance).
__device__ __forceinline__ uint2 pop(Lane& L, const Stack& S, const uint2* spill) {
  --L.sp;
  if (L.sp < S.depth)
    return make_uint2(S.ref[L.sp * 64 + S.lane], __float_as_uint(t_up32(S.tq[L.sp * 64 + S.lane])));
  return spill[L.sp - S.depth];
}

// Candidate hit (t, record, quad, half) against the best so far, by key
// (t, instance id, primitive id, half).  Ids are looked up only on exact ties.
__device__ __forceinline__ bool better(const Lane& L, const SceneView& sc, float t, uint32_t quad, uint32_t half) {
  if (L.b_rec == kEmpty) return true;  // the caller already checked t <= t_best (= tmax)
  if (t != L.t_best) return t < L.t_best;
  const uint32_t ia = sc.inst[L.rec].inst_id, ib = sc.inst[L.b_rec].inst_id;
  if (ia != ib) return ia < ib;
  const uint32_t bq = L.b_qh & 0x7FFFFFFFu;
  const int32_t pa = sc.quad_prim[quad], pb = sc.quad_prim[bq];
  if (pa != pb) return pa < pb;
  return half < (L.b_qh >> 31);
}

// Test quads [first, first + count) of the current instance.  Returns true if
// an any-hit query found a hit.
template <bool COUNT>
__device__ __forceinline__ bool leaf_quads(Lane& L, const SceneView& sc, uint32_t first, uint32_t count,
                                           uint32_t* ctr_quads) {
  const int kx = L.kz == 2 ? 0 : L.kz + 1;
  const int ky = kx == 2 ? 0 : kx + 1;
  for (uint32_t q = first; q < first + count; ++q) {
    if (COUNT) ++*ctr_quads;
    const float4 f0 = sc.quads[3 * (size_t)q + 0];
    const float4 f1 = sc.quads[3 * (size_t)q + 1];
    const float4 f2 = sc.quads[3 * (size_t)q + 2];
    const Sv s0 = shear(L, kx, ky, f0.x, f0.y, f0.z);
    const Sv s1 = shear(L, kx, ky, f0.w, f1.x, f1.y);
    const Sv s2 = shear(L, kx, ky, f1.z, f1.w, f2.x);
    const Sv s3 = shear(L, kx, ky, f2.y, f2.z, f2.w);
    // half A = (v0, v1, v3), half B = (v2, v3, v1); e(v1, v3) is shared (negated)
    const float e13 = edge(s1, s3);
    const float e30 = edge(s3, s0);
    const float e01 = edge(s0, s1);
    const float e31 = edge(s3, s1);
    const float e12 = edge(s1, s2);
    const float e23 = edge(s2, s3);
    const float t_lim = L.any ? L.tmax : L.t_best;
    const TriResult ra = tri_finish(e13, e30, e01, s0, s1, s3, L.tmin, t_lim);
    const TriResult rb = tri_finish(e31, e12, e23, s2, s3, s1, L.tmin, t_lim);
    const bool exq = L.rec == L.ex_rec;
    const bool oka = ra.hit && !(exq && L.ex_qh == q);
    const bool okb = rb.hit && !(exq && L.ex_qh == (q | 0x80000000u));
    if (L.any) {
      if (oka || okb) {
        L.t_best = oka ? ra.t : rb.t;
        L.b_rec = L.rec;
        L.b_qh = oka ? q : (q | 0x80000000u);
        return true;
      }
      continue;
    }
    if (oka && better(L, sc, ra.t, q, 0u)) {
      L.t_best = ra.t;
      L.b_rec = L.rec;
      L.b_qh = q;
      const float r = rcp_fast(ra.det);
      L.b_u = ra.V * r;
      L.b_v = ra.W * r;
    }
    if (okb && better(L, sc, rb.t, q, 1u)) {
      L.t_best = rb.t;
      L.b_rec = L.rec;
      L.b_qh = q | 0x80000000u;
      const float r = rcp_fast(rb.det);
      L.b_u = 1.0f - rb.V * r;
      L.b_v = 1.0f - rb.W * r;
    }
    L.t_cull = L.t_best * kSlack;
  }
  return false;
}

struct VisitCounters {
  uint32_t tlas, inst, blas, quads;
};

// Initialise a lane for world ray (o, d, tmin, tmax).  Returns false (miss) for
// non-finite input or a zero direction.
__device__ __forceinline__ bool lane_init(Lane& L, const SceneView& sc, float ox, float oy, float oz, float dx,
                                          float dy, float dz, float tmin, float tmax) {
  L.wox = ox;
  L.woy = oy;
  L.woz = oz;
  L.wdx = dx;
  L.wdy = dy;
  L.wdz = dz;
  L.tmin = tmin;
  L.tmax = tmax;
  L.t_best = tmax;
  L.t_cull = tmax * kSlack;
  L.b_rec = kEmpty;
  L.b_qh = kEmpty;
  L.b_u = 0.0f;
  L.b_v = 0.0f;
  L.sp = 0;
  L.inst_sp = -1;
  L.rec = kEmpty;
  L.cur = 0u;  // TLAS root
  L.any = false;
  L.done = false;
  const bool finite = __builtin_isfinite(ox) && __builtin_isfinite(oy) && __builtin_isfinite(oz) &&
                      __builtin_isfinite(dx) && __builtin_isfinite(dy) && __builtin_isfinite(dz) &&
                      !(dx == 0.0f && dy == 0.0f && dz == 0.0f) && !(tmin != tmin) && !(tmax != tmax);
  if (!finite || sc.n_inst == 0u) {
    L.cur = kEmpty;
    L.done = true;
    return false;
  }
  set_world_box_ray(L, sc.pad_rel);
  return true;
}

// Resolve an empty current reference: leave the instance when its subtree is
// exhausted, pop the next entry whose entry distance is not behind the closest
// hit, or finish.
__device__ __forceinline__ void advance(Lane& L, const SceneView& sc, const Stack& S, const uint2* spill) {
  while (L.cur == kEmpty) {
    if (L.inst_sp >= 0 && L.sp == L.inst_sp) {  // leave the instance
      L.inst_sp = -1;
      set_world_box_ray(L, sc.pad_rel);
    }
    if (L.sp == 0) {
      L.done = true;
      return;
    }
    const uint2 e = pop(L, S, spill);
    if (__uint_as_float(e.y) <= L.t_cull) L.cur = e.x;
  }
}

// Node step: test the four children, continue with the nearest, push the others
// (farthest first) with their entry distances.
template <int FMT, bool COUNT>
__device__ __forceinline__ void node_step(Lane& L, const SceneView& sc, const Stack& S, uint2* spill,
                                          VisitCounters& vc) {
  float tn[4];
  uint32_t ch[4];
  const bool top = L.inst_sp < 0;
  if (COUNT) {
    if (top) ++vc.tlas;
    else ++vc.blas;
  }
  NodeCodec<FMT>::test(L, top ? sc.tlas : sc.blas, L.cur, L.t_cull, tn, ch);
  cswap(tn[0], ch[0], tn[1], ch[1]);
  cswap(tn[2], ch[2], tn[3], ch[3]);
  cswap(tn[0], ch[0], tn[2], ch[2]);
  cswap(tn[1], ch[1], tn[3], ch[3]);
  cswap(tn[1], ch[1], tn[2], ch[2]);
  if (tn[3] < kInfF) push(L, S, spill, ch[3], tn[3]);
  if (tn[2] < kInfF) push(L, S, spill, ch[2], tn[2]);
  if (tn[1] < kInfF) push(L, S, spill, ch[1], tn[1]);
  L.cur = tn[0] < kInfF ? ch[0] : kEmpty;
  advance(L, sc, S, spill);
}

// Instance step: a top-level leaf -- transform the ray and descend into the
// prototype's bottom-level root.
template <bool COUNT>
__device__ __forceinline__ void inst_step(Lane& L, const SceneView& sc, VisitCounters& vc) {
  if (COUNT) ++vc.inst;
  uint32_t root;
  enter_instance(L, sc.inst, leaf_first(L.cur), &root);
  L.inst_sp = L.sp;
  L.cur = root;
}

// Quad step: test the first quad of the current bottom-level leaf.
template <bool COUNT>
__device__ __forceinline__ void quad_step(Lane& L, const SceneView& sc, const Stack& S, const uint2* spill,
                                          VisitCounters& vc) {
  const uint32_t first = leaf_first(L.cur), count = leaf_count(L.cur);
  if (leaf_quads<COUNT>(L, sc, first, 1u, &vc.quads)) {  // any-hit query answered
    L.cur = kEmpty;
    L.done = true;
    return;
  }
  L.cur = count > 1u ? make_leaf(first + 1u, count - 1u) : kEmpty;
  advance(L, sc, S, spill);
}

// Step kinds of a lane: 0 = traversal done, 1 = node test, 2 = instance entry,
// 3 = quad test.
__device__ __forceinline__ int step_kind(const Lane& L) {
  if (L.done) return 0;
  if (!ref_is_leaf(L.cur)) return 1;
  return L.inst_sp < 0 ? 2 : 3;
}

template <int FMT, bool COUNT>
__device__ __forceinline__ void run_step(int kind, Lane& L, const SceneView& sc, const Stack& S, uint2* spill,
                                         VisitCounters& vc) {
  if (kind == 1) node_step<FMT, COUNT>(L, sc, S, spill, vc);
  else if (kind == 2) inst_step<COUNT>(L, sc, vc);
  else quad_step<COUNT>(L, sc, S, spill, vc);
}

// Wave-uniform choice among the step kinds the participating lanes need: the
// kind with the most lanes (ties favour node, then quad, then instance).
__device__ __forceinline__ int vote_kind(int kind) {
  const int cn = __popcll(__ballot(kind == 1));
  const int ci = __popcll(__ballot(kind == 2));
  const int cq = __popcll(__ballot(kind == 3));
  if (cn >= ci && cn >= cq) return cn ? 1 : 0;
  return cq >= ci ? 3 : 2;
}

// One traversal step of the wave.  The lanes that take part vote: the wave runs
// only the step kind (node test, instance entry or quad test) that most of them
// need, the others wait.  Running one kind per iteration avoids paying for
// every branch whenever any lane needs it.  Returns true once this lane is done.
template <int FMT, bool COUNT>
__device__ __forceinline__ bool lane_step(Lane& L, const SceneView& sc, const Stack& S, uint2* spill,
                                          VisitCounters& vc) {
  const int kind = step_kind(L);
  const int chosen = vote_kind(kind);
  if (chosen != 0 && kind == chosen) run_step<FMT, COUNT>(kind, L, sc, S, spill, vc);
  return L.done;
}

}  // namespace rtq
