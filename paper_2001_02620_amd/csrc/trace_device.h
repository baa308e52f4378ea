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
//   * boxes are tested conservatively: every slab distance is one fused
//     multiply-add of a plane with per-level constants, and those constants are
//     moved by an absolute bound on every rounding error of that evaluation (near
//     distances down, far distances up); quantized boxes contain the exact boxes;
//     instance world boxes are padded for the FP32 ray-transform error and the
//     ray origin is widened by a per-ray pad at the top level;
//   * a box is culled only when its entry distance exceeds t_best (1 + 2^-16);
//   * among hits the smallest key (t, instance id, primitive id, half) wins.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtq_layout.h"

#pragma clang fp contract(off)

namespace rtq {

struct SceneView {
  const uint4* nodes;         // nodes of the traced format: every bottom level, then the top level
  const float4* quads;        // leaf-ordered quads, 3 float4 each
  const int32_t* quad_prim;   // leaf order -> quad index within its prototype
  const InstRec* inst;        // top-level entries in TLAS leaf order: an instance's record, entered
                              // at its bottom-level root or at one subtree of an opened instance
  const float* rec_pmax;      // per record: bound on |object coordinate| of its prototype's boxes
  const uint32_t* rec_qfirst; // per record: first leaf-ordered quad of the subtree it enters
  const uint32_t* rec_nq;     // per record: quads of that subtree
  const float* albedo;        // per unique face (prototype order)
  const float* tex;           // per unique face: tex_res x tex_res texels (row v, column u), or null
  int32_t tex_res;            // texels per side; 0 shades with `albedo`
  int32_t tex_ch;             // channels per texel (fastest): 1, or 3 for RGB base colours
  const float* env;           // environment map, env_w x env_h radiance values, or null
  int32_t env_w, env_h;       // 0: escaping rays see the constant sky
  const unsigned long long* env_T;  // its sampling table: texel k drawn with probability
                                    // (env_T[k] - env_T[k - 1]) / 2^32
  float pad_rel;              // top-level origin pad per unit of |o|_inf
  float p_world;              // bound on |world coordinate| of the top-level boxes
  uint32_t tlas_root;         // index of the top-level root in `nodes`
  uint32_t n_rec;             // records (0 for a scene without instances)
};

constexpr float kSlack = 1.0f + 1.52587890625e-05f;  // 1 + 2^-16

// Vote weights of the wave-voted traversal (a node-test lane counts 4): lanes
// waiting for an instance entry or a quad test count more, so those steps run
// at lower lane counts and return their lanes to node tests sooner.  Measured
// on the config-2 frame: weights (7, 10) against (4, 4) cut the traversal
// launches by 8 %.
#ifndef RTQ_VOTE_WI
#define RTQ_VOTE_WI 7
#endif
#ifndef RTQ_VOTE_WQ
#define RTQ_VOTE_WQ 10
#endif
constexpr float kInfF = __builtin_huge_valf();
// Slab-error bound per unit of (|plane| + |origin|) |1/d|: 2^-20 = 16 u covers
// the reciprocal (1 ulp), the fused multiply-add forming the level constants,
// the node-frame constant of quantized nodes, the fused multiply-add of the
// plane and the half-ulp by which a quantized plane may sit inside its decoded
// value.
constexpr float kDeltaRel = 9.5367431640625e-07f;
constexpr float kInvMax = 18446744073709551616.0f;         // 2^64
constexpr float kInvMaxArg = 5.42101086242752217e-20f;     // 2^-64

// Counter-free selection of component k (0, 1, 2) of (x, y, z).
__device__ __forceinline__ float pick3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

// Ray state of one lane.  Everything stays in registers.
struct Lane {
  // world ray
  float wox, woy, woz, wdx, wdy, wdz, tmin, tmax;
  // slab constants of the current level: the distance to a plane p of axis a is
  // fmaf(p, i_a, cn_a) for near planes (a lower bound) and fmaf(p, i_a, cf_a)
  // for far planes (an upper bound)
  float ix, iy, iz;
  float cnx, cny, cnz;
  float cfx, cfy, cfz;
  // the same constants of the top level, kept to restore them on leaving an
  // instance without recomputing the reciprocals
  float wix, wiy, wiz;
  float wcnx, wcny, wcnz;
  float wcfx, wcfy, wcfz;
  // leaf test inside an instance: object-space origin and the shear of the
  // watertight test (Woop, Benthin, Wald 2013)
  float lox, loy, loz;
  float Sx, Sy, Sz;
  int kz;            // dominant axis of the object-space direction
  bool curve;        // the current instance's prototype holds curves (capsule leaves)
  bool flat;         // ... flat ribbons (ribbon leaves)
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

// Reciprocal direction for the slab test.  Components below 2^-64 in magnitude
// (zero included) take +-2^64, which keeps every slab constant finite; the
// slab of such an axis then still brackets every distance the ray can reach
// inside the level's bounds, and the error bound widens it further.
__device__ __forceinline__ float slab_inv(float d) {
  return fabsf(d) < kInvMaxArg ? copysignf(kInvMax, d) : rcp_fast(d);
}

// Constants of one axis: origin `on` for near planes and `of` for far planes,
// `pmax` bounds |plane| over the level.
__device__ __forceinline__ void slab_axis(float i, float on, float of, float pmax, float& cn, float& cf) {
  const float delta = (pmax + fmaxf(fabsf(on), fabsf(of))) * fabsf(i) * kDeltaRel;
  cn = fmaf(-on, i, -delta);
  cf = fmaf(-of, i, delta);
}

// Box-test constants for the top level: the world ray with its origin widened
// by pad = pad_rel |o|_inf toward the near and far planes.
__device__ __forceinline__ void set_world_level(Lane& L, const SceneView& sc) {
  L.ix = slab_inv(L.wdx);
  L.iy = slab_inv(L.wdy);
  L.iz = slab_inv(L.wdz);
  const float m = fmaxf(fabsf(L.wox), fmaxf(fabsf(L.woy), fabsf(L.woz)));
  const float pad = sc.pad_rel * m;
  // near plane of a positive-direction axis is lo: widen by moving the origin up
  const float sx = L.ix >= 0.0f ? pad : -pad, sy = L.iy >= 0.0f ? pad : -pad, sz = L.iz >= 0.0f ? pad : -pad;
  slab_axis(L.ix, L.wox + sx, L.wox - sx, sc.p_world, L.cnx, L.cfx);
  slab_axis(L.iy, L.woy + sy, L.woy - sy, sc.p_world, L.cny, L.cfy);
  slab_axis(L.iz, L.woz + sz, L.woz - sz, sc.p_world, L.cnz, L.cfz);
}

// Enter instance `r`: transform the ray to object space, o' = A^-1 (o - t),
// d' = A^-1 d, and prepare the box test and the shear of the leaf test.
__device__ __forceinline__ void enter_instance(Lane& L, const SceneView& sc, uint32_t r, uint32_t* blas_root) {
  const float4 a = *reinterpret_cast<const float4*>(sc.inst[r].r0);
  const float4 b = *reinterpret_cast<const float4*>(sc.inst[r].r1);
  const float4 c = *reinterpret_cast<const float4*>(sc.inst[r].r2);
  const uint32_t root = sc.inst[r].blas_root;
  const uint32_t proto = sc.inst[r].proto;
  const float pmax = sc.rec_pmax[r];
  const float px = L.wox - a.w, py = L.woy - b.w, pz = L.woz - c.w;
  const float ox = fmaf(a.x, px, fmaf(a.y, py, a.z * pz));
  const float oy = fmaf(b.x, px, fmaf(b.y, py, b.z * pz));
  const float oz = fmaf(c.x, px, fmaf(c.y, py, c.z * pz));
  const float dx = fmaf(a.x, L.wdx, fmaf(a.y, L.wdy, a.z * L.wdz));
  const float dy = fmaf(b.x, L.wdx, fmaf(b.y, L.wdy, b.z * L.wdz));
  const float dz = fmaf(c.x, L.wdx, fmaf(c.y, L.wdy, c.z * L.wdz));
  L.ix = slab_inv(dx);
  L.iy = slab_inv(dy);
  L.iz = slab_inv(dz);
  slab_axis(L.ix, ox, ox, pmax, L.cnx, L.cfx);
  slab_axis(L.iy, oy, oy, pmax, L.cny, L.cfy);
  slab_axis(L.iz, oz, oz, pmax, L.cnz, L.cfz);
  L.lox = ox;
  L.loy = oy;
  L.loz = oz;
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
  L.curve = (proto & kProtoCurve) != 0u;
  L.flat = (proto & kProtoFlat) != 0u;
  *blas_root = root;
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
  const float ax = vx - L.lox, ay = vy - L.loy, az = vz - L.loz;
  const float akx = pick3(ax, ay, az, kx);
  const float aky = pick3(ax, ay, az, ky);
  const float akz = pick3(ax, ay, az, L.kz);
  Sv s;
  s.X = fmaf(-L.Sx, akz, akx);
  s.Y = fmaf(-L.Sy, akz, aky);
  s.Z = L.Sz * akz;
  return s;
}
// Edge function e(P, Q) = Qx Py - Qy Px.  With contraction off, e(Q, P) is the
// exact negative of e(P, Q): a shared edge gives the two triangles opposite
// signs bit for bit, which is what makes the test watertight.
__device__ __forceinline__ float edge(const Sv& P, const Sv& Q) { return Q.X * P.Y - Q.Y * P.X; }

struct TriResult {
  bool hit;
  bool f64;  // the edge values were re-evaluated in FP64
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
  r.f64 = false;
  const bool neg = (U < 0.0f) || (V < 0.0f) || (W < 0.0f);
  const bool pos = (U > 0.0f) || (V > 0.0f) || (W > 0.0f);
  if (neg && pos) return r;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    r.f64 = true;
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
  const float T = fmaf(U, A.Z, fmaf(V, B.Z, W * C.Z));
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
typedef __attribute__((address_space(3))) uint32_t LdsU32;  // LDS-qualified element types
typedef __attribute__((address_space(3))) uint16_t LdsU16;

struct Stack {
  LdsU32* ref;  // this lane's column: entry j at ref[64 j]
  LdsU16* tq;   // this lane's column of entry distances
  int depth;    // LDS entries per lane
};

constexpr int kStackEntryBytes = 6;

// Stack region of this lane in a block's dynamic LDS (6 bytes per entry and lane).
__device__ __forceinline__ Stack make_stack(void* lds, int depth) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  LdsU32* refs = (LdsU32*)lds;
  LdsU16* ts = (LdsU16*)(refs + (size_t)waves * depth * 64);
  return Stack{refs + wave * depth * 64 + lane, ts + wave * depth * 64 + lane, depth};
}

// FP32 -> upper 16 bits, rounded toward -inf: a negative value with a non-zero
// lower half rounds away from zero.
__device__ __forceinline__ uint16_t t_down16(float t) {
  const uint32_t b = __float_as_uint(t);
  return (uint16_t)((b + ((uint32_t)((int32_t)b >> 31) & 0xFFFFu)) >> 16);
}
__device__ __forceinline__ float t_up32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- box tests --------------------------------------------------------------------
// Slab test of one child: near planes (nx, ny, nz), far planes (fx, fy, fz).
// Returns the entry distance, or kInfF when the box is missed or lies beyond
// t_lim.
__device__ __forceinline__ float slab1(const Lane& L, float nx, float fx, float ny, float fy, float nz, float fz,
                                       float t_lim) {
  const float tn = fmaxf(fmaxf(fmaf(nx, L.ix, L.cnx), fmaf(ny, L.iy, L.cny)), fmaxf(fmaf(nz, L.iz, L.cnz), L.tmin));
  const float tf = fminf(fminf(fmaf(fx, L.ix, L.cfx), fmaf(fy, L.iy, L.cfy)), fmaf(fz, L.iz, L.cfz));
  return tn <= fminf(tf, t_lim) ? tn : kInfF;
}

template <int FMT>
struct NodeCodec;

// Near/far plane of an axis: lo when the reciprocal direction is non-negative.
__device__ __forceinline__ uint32_t sign_of(float i) { return __float_as_uint(i) >> 31; }

// FP32 nodes: the near and far plane vectors of each axis are chosen by address
// (6 x 16 B plane loads and the child references).  Empty slots have lo = +inf
// and hi = -inf and miss for every ray.
template <>
struct NodeCodec<kCodecF32> {
  static constexpr int kW = 4;
  static constexpr int kStride = 8;  // uint4 per node
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[4], uint32_t ch[4]) {
    const uint4* p = base + (size_t)idx * kStride;
    const uint32_t sx = sign_of(L.ix), sy = sign_of(L.iy), sz = sign_of(L.iz);
    const float4 nx = __builtin_bit_cast(float4, p[sx]);
    const float4 fx = __builtin_bit_cast(float4, p[sx ^ 1u]);
    const float4 ny = __builtin_bit_cast(float4, p[2u + sy]);
    const float4 fy = __builtin_bit_cast(float4, p[3u - sy]);
    const float4 nz = __builtin_bit_cast(float4, p[4u + sz]);
    const float4 fz = __builtin_bit_cast(float4, p[5u - sz]);
    const uint4 c = p[6];
    ch[0] = c.x;
    ch[1] = c.y;
    ch[2] = c.z;
    ch[3] = c.w;
    tn[0] = slab1(L, nx.x, fx.x, ny.x, fy.x, nz.x, fz.x, t_lim);
    tn[1] = slab1(L, nx.y, fx.y, ny.y, fy.y, nz.y, fz.y, t_lim);
    tn[2] = slab1(L, nx.z, fx.z, ny.z, fy.z, nz.z, fz.z, t_lim);
    tn[3] = slab1(L, nx.w, fx.w, ny.w, fy.w, nz.w, fz.w, t_lim);
  }
};

// Quantized nodes: 4 x 16 B loads.  A plane is origin + q 2^e, so its distance is
// fmaf(q, 2^e i, fmaf(origin, i, c)): two per-node constants per axis and one
// fused multiply-add per plane.  The near/far byte planes of all four children
// are selected with one select per axis.
template <>
struct NodeCodec<kCodecQ8> {
  static constexpr int kW = 4;
  static constexpr int kStride = 4;
  __device__ __forceinline__ static float ub(uint32_t w, int k) {
    return (float)((w >> (8 * k)) & 0xFFu);
  }
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[4], uint32_t ch[4]) {
    const uint4* p = base + (size_t)idx * kStride;
    const uint4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const float ox = __uint_as_float(q0.x), oy = __uint_as_float(q0.y), oz = __uint_as_float(q0.z);
    // 2^e i is exact (a power-of-two scaling)
    const float bx = __builtin_amdgcn_ldexpf(L.ix, (int)(int8_t)(q0.w & 0xFFu));
    const float by = __builtin_amdgcn_ldexpf(L.iy, (int)(int8_t)((q0.w >> 8) & 0xFFu));
    const float bz = __builtin_amdgcn_ldexpf(L.iz, (int)(int8_t)((q0.w >> 16) & 0xFFu));
    const float nax = fmaf(ox, L.ix, L.cnx), fax = fmaf(ox, L.ix, L.cfx);
    const float nay = fmaf(oy, L.iy, L.cny), fay = fmaf(oy, L.iy, L.cfy);
    const float naz = fmaf(oz, L.iz, L.cnz), faz = fmaf(oz, L.iz, L.cfz);
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
      const float n = fmaxf(fmaxf(fmaf(ub(nx, k), bx, nax), fmaf(ub(ny, k), by, nay)),
                            fmaxf(fmaf(ub(nz, k), bz, naz), L.tmin));
      const float f = fminf(fminf(fmaf(ub(fx, k), bx, fax), fmaf(ub(fy, k), by, fay)), fmaf(ub(fz, k), bz, faz));
      // no test for empty slots: their byte box is inverted (lo 255, hi 0), so
      // they miss unless the slab slack exceeds the node's whole extent, and a
      // pushed kEmpty is popped and dropped like a miss
      tn[k] = n <= fminf(f, t_lim) ? n : kInfF;
    }
  }
};

// Per-node constants of a quantized node: the exact 2^e / d per axis and the
// distances of the node origin (near and far constants).
struct Q8Frame {
  float bx, by, bz, nax, fax, nay, fay, naz, faz;
};
__device__ __forceinline__ Q8Frame q8_frame(const Lane& L, const uint4 q0) {
  Q8Frame f;
  const float ox = __uint_as_float(q0.x), oy = __uint_as_float(q0.y), oz = __uint_as_float(q0.z);
  f.bx = __builtin_amdgcn_ldexpf(L.ix, (int)(int8_t)(q0.w & 0xFFu));
  f.by = __builtin_amdgcn_ldexpf(L.iy, (int)(int8_t)((q0.w >> 8) & 0xFFu));
  f.bz = __builtin_amdgcn_ldexpf(L.iz, (int)(int8_t)((q0.w >> 16) & 0xFFu));
  f.nax = fmaf(ox, L.ix, L.cnx);
  f.fax = fmaf(ox, L.ix, L.cfx);
  f.nay = fmaf(oy, L.iy, L.cny);
  f.fay = fmaf(oy, L.iy, L.cfy);
  f.naz = fmaf(oz, L.iz, L.cnz);
  f.faz = fmaf(oz, L.iz, L.cfz);
  return f;
}
// Entry distance of one quantized child with near bytes (qnx, qny, qnz) and far
// bytes (qfx, qfy, qfz), or kInfF.
__device__ __forceinline__ float q8_child(const Lane& L, const Q8Frame& f, float qnx, float qfx, float qny, float qfy,
                                          float qnz, float qfz, float t_lim) {
  const float n = fmaxf(fmaxf(fmaf(qnx, f.bx, f.nax), fmaf(qny, f.by, f.nay)), fmaxf(fmaf(qnz, f.bz, f.naz), L.tmin));
  const float t = fminf(fminf(fmaf(qfx, f.bx, f.fax), fmaf(qfy, f.by, f.fay)), fmaf(qfz, f.bz, f.faz));
  return n <= fminf(t, t_lim) ? n : kInfF;
}

// Quantized 8-wide nodes: 6 x 16 B loads; per axis the lower and upper byte
// planes of children 0..3 and 4..7 sit in four words, and the near and far pair
// is chosen by the direction's sign.
template <>
struct NodeCodec<kCodecQ8W8> {
  static constexpr int kW = 8;
  static constexpr int kStride = 6;
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[8], uint32_t ch[8]) {
    const uint4* p = base + (size_t)idx * kStride;
    const uint4 q0 = p[0], qx = p[1], qy = p[2], qz = p[3], c0 = p[4], c1 = p[5];
    const Q8Frame f = q8_frame(L, q0);
    const bool sx = L.ix >= 0.0f, sy = L.iy >= 0.0f, sz = L.iz >= 0.0f;
    // (lo[0..3], lo[4..7], hi[0..3], hi[4..7]) per axis
    const uint32_t nx0 = sx ? qx.x : qx.z, nx1 = sx ? qx.y : qx.w, fx0 = sx ? qx.z : qx.x, fx1 = sx ? qx.w : qx.y;
    const uint32_t ny0 = sy ? qy.x : qy.z, ny1 = sy ? qy.y : qy.w, fy0 = sy ? qy.z : qy.x, fy1 = sy ? qy.w : qy.y;
    const uint32_t nz0 = sz ? qz.x : qz.z, nz1 = sz ? qz.y : qz.w, fz0 = sz ? qz.z : qz.x, fz1 = sz ? qz.w : qz.y;
    ch[0] = c0.x;
    ch[1] = c0.y;
    ch[2] = c0.z;
    ch[3] = c0.w;
    ch[4] = c1.x;
    ch[5] = c1.y;
    ch[6] = c1.z;
    ch[7] = c1.w;
    using C = NodeCodec<kCodecQ8>;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      tn[k] = q8_child(L, f, C::ub(nx0, k), C::ub(fx0, k), C::ub(ny0, k), C::ub(fy0, k), C::ub(nz0, k),
                       C::ub(fz0, k), t_lim);
      tn[k + 4] = q8_child(L, f, C::ub(nx1, k), C::ub(fx1, k), C::ub(ny1, k), C::ub(fy1, k), C::ub(nz1, k),
                           C::ub(fz1, k), t_lim);
    }
  }
};

// Quantized 2-wide nodes: 3 x 16 B loads; one word per axis holds the lower
// planes of both children in bytes 0, 1 and the upper planes in bytes 2, 3.
template <>
struct NodeCodec<kCodecQ8W2> {
  static constexpr int kW = 2;
  static constexpr int kStride = 3;
  __device__ __forceinline__ static void test(const Lane& L, const uint4* __restrict__ base, uint32_t idx,
                                              float t_lim, float tn[2], uint32_t ch[2]) {
    const uint4* p = base + (size_t)idx * kStride;
    const uint4 q0 = p[0], q1 = p[1];
    const uint32_t c1 = p[2].x;
    const Q8Frame f = q8_frame(L, q0);
    const bool sx = L.ix >= 0.0f, sy = L.iy >= 0.0f, sz = L.iz >= 0.0f;
    const uint32_t nx = sx ? q1.x : (q1.x >> 16), fx = sx ? (q1.x >> 16) : q1.x;
    const uint32_t ny = sy ? q1.y : (q1.y >> 16), fy = sy ? (q1.y >> 16) : q1.y;
    const uint32_t nz = sz ? q1.z : (q1.z >> 16), fz = sz ? (q1.z >> 16) : q1.z;
    ch[0] = q1.w;
    ch[1] = c1;
    using C = NodeCodec<kCodecQ8>;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      tn[k] = q8_child(L, f, C::ub(nx, k), C::ub(fx, k), C::ub(ny, k), C::ub(fy, k), C::ub(nz, k), C::ub(fz, k),
                       t_lim);
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

// Sort the children of a node by entry distance (misses, kInfF, go last).
// Sorting networks: 1 exchange for 2 children, 5 for 4, 19 for 8 (the optimal
// networks, Knuth TAOCP vol. 3, 5.3.4).
template <int W>
__device__ __forceinline__ void sort_children(float* tn, uint32_t* ch);
template <>
__device__ __forceinline__ void sort_children<2>(float* tn, uint32_t* ch) {
  cswap(tn[0], ch[0], tn[1], ch[1]);
}
template <>
__device__ __forceinline__ void sort_children<4>(float* tn, uint32_t* ch) {
  cswap(tn[0], ch[0], tn[1], ch[1]);
  cswap(tn[2], ch[2], tn[3], ch[3]);
  cswap(tn[0], ch[0], tn[2], ch[2]);
  cswap(tn[1], ch[1], tn[3], ch[3]);
  cswap(tn[1], ch[1], tn[2], ch[2]);
}
template <>
__device__ __forceinline__ void sort_children<8>(float* tn, uint32_t* ch) {
  constexpr int net[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                              {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int i = 0; i < 19; ++i) cswap(tn[net[i][0]], ch[net[i][0]], tn[net[i][1]], ch[net[i][1]]);
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

// Test quad q of the current instance on the lanes with `act` set; the other
// lanes evaluate the same instructions on quad q (any valid index) and keep their
// state.  Every update is a select, so no lane state is written under divergent
// control flow.  Returns true on the lanes where an any-hit query found its hit.
// *n64 (when given) counts this lane's FP64 edge re-evaluations.
__device__ __forceinline__ bool quad_test(Lane& L, const SceneView& sc, bool act, uint32_t q,
                                          uint32_t* n64 = nullptr) {
  const int kx = L.kz == 2 ? 0 : L.kz + 1;
  const int ky = kx == 2 ? 0 : kx + 1;
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
  if (n64) *n64 += (act && ra.f64 ? 1u : 0u) + (act && rb.f64 ? 1u : 0u);
  const bool exq = L.rec == L.ex_rec;
  const bool oka = act && ra.hit && !(exq && L.ex_qh == q);
  const bool okb = act && rb.hit && !(exq && L.ex_qh == (q | 0x80000000u));
  if (L.any) {
    // any-hit: the first accepted half answers the query
    const bool hit = oka || okb;
    L.t_best = hit ? (oka ? ra.t : rb.t) : L.t_best;
    L.b_rec = hit ? L.rec : L.b_rec;
    L.b_qh = hit ? (oka ? q : (q | 0x80000000u)) : L.b_qh;
    return hit;
  }
  const bool ua = oka && better(L, sc, ra.t, q, 0u);
  const float ra_r = rcp_fast(ra.det);
  L.t_best = ua ? ra.t : L.t_best;
  L.b_rec = ua ? L.rec : L.b_rec;
  L.b_qh = ua ? q : L.b_qh;
  L.b_u = ua ? ra.V * ra_r : L.b_u;
  L.b_v = ua ? ra.W * ra_r : L.b_v;
  const bool ub = okb && better(L, sc, rb.t, q, 1u);
  const float rb_r = rcp_fast(rb.det);
  L.t_best = ub ? rb.t : L.t_best;
  L.b_rec = ub ? L.rec : L.b_rec;
  L.b_qh = ub ? (q | 0x80000000u) : L.b_qh;
  L.b_u = ub ? 1.0f - rb.V * rb_r : L.b_u;
  L.b_v = ub ? 1.0f - rb.W * rb_r : L.b_v;
  L.t_cull = L.t_best * kSlack;
  return false;
}

// ---- capsule test -----------------------------------------------------------------
// Curves (Section 5.2) are traced as chains of capsules: a capsule is the set of
// points within r of the segment [a, b], entered from outside only.  The test
// runs in object space in FP32:
//   * the direction is recomputed from the instance record with the expressions
//     of enter_instance (bit-identical to the lane's leaf-test frame) and scaled
//     by a power of two so that |d|_inf lies in [0.5, 1) (exact; the squares
//     below stay in range for any ray);
//   * a ray starting inside the capsule misses it;
//   * the quadratics are solved from the ray's point of closest approach to the
//     axis midpoint, so their coefficients are formed next to the capsule, and
//     their roots are taken in the cancellation-free form
//     q = -(b + sign(b) sqrt(b^2 - a c)), roots q / a and c / q;
//   * the cylinder around the axis, |(b - a) x (p - a)|^2 = r^2 |b - a|^2, is
//     written with cross products (Lagrange's identity), which keeps its
//     leading coefficient exact in sign for a ray nearly parallel to the axis.
// A ray outside the infinite cylinder enters it at the smaller root; there it is
// on the capsule's body when the axial coordinate lies within the segment, else
// it can only enter through the end sphere on that side.  A ray starting inside
// the infinite cylinder (beyond an end) or parallel to the axis can only enter
// through an end sphere, the nearer one.
struct CapResult {
  float t;  // entry parameter in the world ray's units, kInfF for none at t >= 0
  float y;  // position of the entry along the axis, 0 at a and 1 at b
};

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// Smaller root s of |p + s d - c|^2 = r^2 (dd = d.d), or kInfF when the line
// misses the sphere.
__device__ __forceinline__ float sphere_root(float px, float py, float pz, float cx, float cy, float cz, float rr,
                                             float dx, float dy, float dz, float dd) {
  const float ox = px - cx, oy = py - cy, oz = pz - cz;
  const float b = dot3(ox, oy, oz, dx, dy, dz);
  const float c = dot3(ox, oy, oz, ox, oy, oz) - rr;
  const float disc = b * b - dd * c;
  if (!(disc >= 0.0f)) return kInfF;
  const float q = -(b + copysignf(sqrtf(disc), b));
  return fminf(q / dd, c / q);  // q = 0 only for a line touching the sphere at p: q / dd = 0
}

// Capsule q under instance record `rec` (both valid indices on every lane).
__device__ __forceinline__ CapResult cap_hit(const Lane& L, const SceneView& sc, uint32_t rec, uint32_t q) {
  CapResult res{kInfF, 0.0f};
  const float4 c0 = sc.quads[3 * (size_t)q + 0];
  const float4 c1 = sc.quads[3 * (size_t)q + 1];
  const float4 ra = *reinterpret_cast<const float4*>(sc.inst[rec].r0);
  const float4 rb = *reinterpret_cast<const float4*>(sc.inst[rec].r1);
  const float4 rc = *reinterpret_cast<const float4*>(sc.inst[rec].r2);
  float dx = fmaf(ra.x, L.wdx, fmaf(ra.y, L.wdy, ra.z * L.wdz));
  float dy = fmaf(rb.x, L.wdx, fmaf(rb.y, L.wdy, rb.z * L.wdz));
  float dz = fmaf(rc.x, L.wdx, fmaf(rc.y, L.wdy, rc.z * L.wdz));
  const float dm = fmaxf(fabsf(dx), fmaxf(fabsf(dy), fabsf(dz)));
  if (!(dm > 0.0f) || !(dm < kInfF)) return res;
  const int e = __builtin_amdgcn_frexp_expf(dm);
  dx = __builtin_amdgcn_ldexpf(dx, -e);
  dy = __builtin_amdgcn_ldexpf(dy, -e);
  dz = __builtin_amdgcn_ldexpf(dz, -e);
  const float ax = c0.x, ay = c0.y, az = c0.z, r = c0.w, rr = r * r;
  const float bax = c1.x - ax, bay = c1.y - ay, baz = c1.z - az;
  const float bb = dot3(bax, bay, baz, bax, bay, baz);
  // the origin inside the capsule: no entry
  const float wx = L.lox - ax, wy = L.loy - ay, wz = L.loz - az;
  const float s0 = bb > 0.0f ? fminf(fmaxf(dot3(wx, wy, wz, bax, bay, baz) / bb, 0.0f), 1.0f) : 0.0f;
  const float ex = fmaf(-s0, bax, wx), ey = fmaf(-s0, bay, wy), ez = fmaf(-s0, baz, wz);
  if (dot3(ex, ey, ez, ex, ey, ez) < rr) return res;
  // closest approach of the axis midpoint
  const float dd = dot3(dx, dy, dz, dx, dy, dz);
  const float mx = fmaf(0.5f, bax, ax), my = fmaf(0.5f, bay, ay), mz = fmaf(0.5f, baz, az);
  const float t0 = dot3(mx - L.lox, my - L.loy, mz - L.loz, dx, dy, dz) / dd;
  const float px = fmaf(t0, dx, L.lox), py = fmaf(t0, dy, L.loy), pz = fmaf(t0, dz, L.loz);
  // which end spheres to test: 1 = a, 2 = b, 3 = both (the nearer wins)
  int ends = 0;
  float s = kInfF, y = 0.0f;
  const float gx = bay * wz - baz * wy, gy = baz * wx - bax * wz, gz = bax * wy - bay * wx;  // ba x (o - a)
  const float ux = bay * dz - baz * dy, uy = baz * dx - bax * dz, uz = bax * dy - bay * dx;  // ba x d
  const float A = dot3(ux, uy, uz, ux, uy, uz);
  if (dot3(gx, gy, gz, gx, gy, gz) - rr * bb < 0.0f || !(A > 0.0f)) {
    ends = 3;
  } else {
    const float pax = px - ax, pay = py - ay, paz = pz - az;
    const float vx = bay * paz - baz * pay, vy = baz * pax - bax * paz, vz = bax * pay - bay * pax;  // ba x (p - a)
    const float B = dot3(vx, vy, vz, ux, uy, uz);
    const float C = dot3(vx, vy, vz, vx, vy, vz) - rr * bb;
    const float disc = B * B - A * C;
    if (disc >= 0.0f) {
      const float qq = -(B + copysignf(sqrtf(disc), B));
      const float sc_ = fminf(qq / A, C / qq);
      if (t0 + sc_ >= 0.0f) {
        const float ya = fmaf(sc_, dot3(bax, bay, baz, dx, dy, dz), dot3(bax, bay, baz, pax, pay, paz));
        if (ya >= 0.0f && ya <= bb) {
          s = sc_;
          y = ya / bb;
        } else {
          ends = ya < 0.0f ? 1 : 2;
        }
      }
    }
  }
  if (ends & 1) {
    const float sa = sphere_root(px, py, pz, ax, ay, az, rr, dx, dy, dz, dd);
    if (t0 + sa > 0.0f) s = sa;
  }
  if (ends & 2) {
    const float sb = sphere_root(px, py, pz, c1.x, c1.y, c1.z, rr, dx, dy, dz, dd);
    if (t0 + sb > 0.0f && !(sb >= s)) {
      s = sb;
      y = 1.0f;
    }
  }
  const float t = t0 + s;
  res.t = t < kInfF ? __builtin_amdgcn_ldexpf(t, -e) : kInfF;
  res.y = y;
  return res;
}

// Test capsule q of the current instance on the lanes with `act` set (the
// others evaluate the same instructions on record 0 -- a lane that has not
// entered an instance yet holds no record -- and keep their state); updates as
// quad_test.  No entry is t = +inf, which must not pass t <= t_best when
// t_best = tmax = +inf.  The hit's u holds its axis position y (the curve
// parameter is formed from it when the hit is stored), v = 0.
__device__ __forceinline__ bool cap_test(Lane& L, const SceneView& sc, bool act, uint32_t q) {
  const CapResult c = cap_hit(L, sc, act ? L.rec : 0u, q);
  const float t_lim = L.any ? L.tmax : L.t_best;
  const bool ok = act && c.t < kInfF && c.t > L.tmin && c.t <= t_lim && !(L.rec == L.ex_rec && L.ex_qh == q);
  if (L.any) {
    L.t_best = ok ? c.t : L.t_best;
    L.b_rec = ok ? L.rec : L.b_rec;
    L.b_qh = ok ? q : L.b_qh;
    return ok;
  }
  const bool u = ok && better(L, sc, c.t, q, 0u);
  L.t_best = u ? c.t : L.t_best;
  L.b_rec = u ? L.rec : L.b_rec;
  L.b_qh = u ? q : L.b_qh;
  L.b_u = u ? c.y : L.b_u;
  L.b_v = u ? 0.0f : L.b_v;
  L.t_cull = L.t_best * kSlack;
  return false;
}

// Flat ribbon segment q under record `rec` (Section 5.2 names flat ribbon
// curves): (a, ra) = c0, (b, rb) = c1, radius ra + u (rb - ra).  Seen along the
// ray it is the strip of points within that radius of its projection onto
// the plane orthogonal to the ray; the ray meets it when its line passes
// within the radius of the projected segment's point u closest to it, at the
// depth of that segment point.  In object space in FP32, the direction scaled
// by a power of two as in cap_hit, the origin moved to the ray's closest
// approach to the segment midpoint so every vector below is formed next to the
// segment.  y returns u.
__device__ __forceinline__ CapResult ribbon_hit(const Lane& L, const SceneView& sc, uint32_t rec, uint32_t q) {
  CapResult res{kInfF, 0.0f};
  const float4 c0 = sc.quads[3 * (size_t)q + 0];
  const float4 c1 = sc.quads[3 * (size_t)q + 1];
  const float4 ra = *reinterpret_cast<const float4*>(sc.inst[rec].r0);
  const float4 rb = *reinterpret_cast<const float4*>(sc.inst[rec].r1);
  const float4 rc = *reinterpret_cast<const float4*>(sc.inst[rec].r2);
  float dx = fmaf(ra.x, L.wdx, fmaf(ra.y, L.wdy, ra.z * L.wdz));
  float dy = fmaf(rb.x, L.wdx, fmaf(rb.y, L.wdy, rb.z * L.wdz));
  float dz = fmaf(rc.x, L.wdx, fmaf(rc.y, L.wdy, rc.z * L.wdz));
  const float dm = fmaxf(fabsf(dx), fmaxf(fabsf(dy), fabsf(dz)));
  if (!(dm > 0.0f) || !(dm < kInfF)) return res;
  const int e = __builtin_amdgcn_frexp_expf(dm);
  dx = __builtin_amdgcn_ldexpf(dx, -e);
  dy = __builtin_amdgcn_ldexpf(dy, -e);
  dz = __builtin_amdgcn_ldexpf(dz, -e);
  const float dd = dot3(dx, dy, dz, dx, dy, dz);
  const float bax = c1.x - c0.x, bay = c1.y - c0.y, baz = c1.z - c0.z;
  const float mx = fmaf(0.5f, bax, c0.x), my = fmaf(0.5f, bay, c0.y), mz = fmaf(0.5f, baz, c0.z);
  const float t0 = dot3(mx - L.lox, my - L.loy, mz - L.loz, dx, dy, dz) / dd;
  const float px = fmaf(t0, dx, L.lox), py = fmaf(t0, dy, L.loy), pz = fmaf(t0, dz, L.loz);
  const float Ax = c0.x - px, Ay = c0.y - py, Az = c0.z - pz;
  const float Bx = c1.x - px, By = c1.y - py, Bz = c1.z - pz;
  const float ka = dot3(Ax, Ay, Az, dx, dy, dz) / dd, kb = dot3(Bx, By, Bz, dx, dy, dz) / dd;
  const float apx = fmaf(-ka, dx, Ax), apy = fmaf(-ka, dy, Ay), apz = fmaf(-ka, dz, Az);
  const float ex = fmaf(-kb, dx, Bx) - apx, ey = fmaf(-kb, dy, By) - apy, ez = fmaf(-kb, dz, Bz) - apz;
  const float ee = dot3(ex, ey, ez, ex, ey, ez);
  const float u = ee > 0.0f ? fminf(fmaxf(-dot3(apx, apy, apz, ex, ey, ez) / ee, 0.0f), 1.0f) : 0.0f;
  const float qx = fmaf(u, ex, apx), qy = fmaf(u, ey, apy), qz = fmaf(u, ez, apz);
  const float r = fmaf(u, c1.w - c0.w, c0.w);
  if (!(dot3(qx, qy, qz, qx, qy, qz) <= r * r)) return res;
  const float t = t0 + fmaf(u, kb - ka, ka);
  res.t = t < kInfF ? __builtin_amdgcn_ldexpf(t, -e) : kInfF;
  res.y = u;
  return res;
}

// Test ribbon segment q of the current instance on the lanes with `act` set;
// updates as cap_test.  A ray that excludes a segment of a ribbon ignores every
// segment of that curve in that instance (a ribbon turns toward every ray, so
// the neighbours of the segment a ray leaves would face it next to its
// origin): compared by instance id and curve (primitive / 8), looked up only
// for a hit of a ray that has an exclusion.
__device__ __forceinline__ bool ribbon_test(Lane& L, const SceneView& sc, bool act, uint32_t q) {
  const CapResult c = ribbon_hit(L, sc, act ? L.rec : 0u, q);
  const float t_lim = L.any ? L.tmax : L.t_best;
  bool ok = act && c.t < kInfF && c.t > L.tmin && c.t <= t_lim;
  if (ok && L.ex_rec != kEmpty) {
    const bool same_curve =
        sc.inst[L.rec].inst_id == sc.inst[L.ex_rec].inst_id &&
        (uint32_t)sc.quad_prim[q] / (uint32_t)kCapsPerCurve ==
            (uint32_t)sc.quad_prim[L.ex_qh & 0x7FFFFFFFu] / (uint32_t)kCapsPerCurve;
    ok = !same_curve;
  }
  if (L.any) {
    L.t_best = ok ? c.t : L.t_best;
    L.b_rec = ok ? L.rec : L.b_rec;
    L.b_qh = ok ? q : L.b_qh;
    return ok;
  }
  const bool upd = ok && better(L, sc, c.t, q, 0u);
  L.t_best = upd ? c.t : L.t_best;
  L.b_rec = upd ? L.rec : L.b_rec;
  L.b_qh = upd ? q : L.b_qh;
  L.b_u = upd ? c.y : L.b_u;
  L.b_v = upd ? 0.0f : L.b_v;
  L.t_cull = L.t_best * kSlack;
  return false;
}

// Primitive test of the current instance: a quad, a capsule or a ribbon
// segment, by the instance's prototype.  Each test runs only when a lane of the
// wave needs it (wave-uniform branches).
__device__ __forceinline__ bool prim_test(Lane& L, const SceneView& sc, bool act, uint32_t q,
                                          uint32_t* n64 = nullptr) {
  bool answered = false;
  if (__any(act && !L.curve)) answered = quad_test(L, sc, act && !L.curve, q, n64);
  if (__any(act && L.curve && !L.flat)) answered = cap_test(L, sc, act && L.curve && !L.flat, q) || answered;
  if (__any(act && L.flat)) answered = ribbon_test(L, sc, act && L.flat, q) || answered;
  return answered;
}

// Test primitives [first, first + count) of the current instance on every lane.
// Returns true if an any-hit query found a hit.
__device__ __forceinline__ bool leaf_quads(Lane& L, const SceneView& sc, uint32_t first, uint32_t count) {
  for (uint32_t q = first; q < first + count; ++q)
    if (prim_test(L, sc, true, q)) return true;
  return false;
}

struct VisitCounters {
  uint32_t tlas, inst, blas, quads;
  uint32_t iters = 0;  // traversal iterations of its wave while the ray was not done
  uint32_t fp64 = 0;   // FP64 re-evaluations of zero edge values in its leaf tests
};

// ---- work claiming of the persistent kernels ------------------------------------
// The work indices [0, n) of a launch are dealt to kClaimSlices interleaved
// slices (index i belongs to slice i mod kClaimSlices), each with its own
// counter.  A wave claims from its home slice (its block index mod the slice
// count) and moves to the next slice once that one is used up, so the atomics of
// a launch spread over kClaimSlices counters instead of serialising on one, and
// every slice keeps the order of the indices.  Fields are wave-uniform.
struct ClaimState {
  int slice;  // slice claimed from
  int dry;    // consecutive slices found used up
};

__device__ __forceinline__ ClaimState claim_init() { return ClaimState{(int)(blockIdx.x % kClaimSlices), 0}; }

// Claim work for the idle lanes (mask `idle`, nidle >= 1 of them).  Returns this
// lane's work index, or -1 for a busy lane and when nothing was claimed for it;
// sets *exhausted once every slice is used up.
__device__ __forceinline__ int64_t claim_take(ClaimState& C, unsigned long long* ctr, int64_t n,
                                              unsigned long long idle, int nidle, bool* exhausted) {
  const int lane = threadIdx.x & 63;
  const bool is_idle = ((idle >> lane) & 1ull) != 0ull;
  const uint32_t rank =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
  const int leader = __ffsll((long long)__ballot(1)) - 1;
  while (C.dry < kClaimSlices) {
    const int h = C.slice;
    const int64_t len = n > h ? (n - h + kClaimSlices - 1) / kClaimSlices : 0;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(&ctr[h * kClaimStride], (unsigned long long)nidle);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)base, leader);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader);
    base = ((unsigned long long)hi << 32) | lo;
    if ((int64_t)base < len) {
      C.dry = 0;
      const int64_t j = (int64_t)base + rank;
      return (is_idle && j < len) ? j * kClaimSlices + h : -1;
    }
    C.slice = h + 1 == kClaimSlices ? 0 : h + 1;
    ++C.dry;
  }
  *exhausted = true;
  return -1;
}

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
  L.curve = false;
  L.flat = false;
  L.cur = sc.tlas_root;
  L.any = false;
  L.done = false;
  const bool finite = __builtin_isfinite(ox) && __builtin_isfinite(oy) && __builtin_isfinite(oz) &&
                      __builtin_isfinite(dx) && __builtin_isfinite(dy) && __builtin_isfinite(dz) &&
                      !(dx == 0.0f && dy == 0.0f && dz == 0.0f) && !(tmin != tmin) && !(tmax != tmax);
  if (!finite || sc.n_rec == 0u) {
    L.cur = kEmpty;
    L.done = true;
    return false;
  }
  set_world_level(L, sc);
  L.wix = L.ix;
  L.wiy = L.iy;
  L.wiz = L.iz;
  L.wcnx = L.cnx;
  L.wcny = L.cny;
  L.wcnz = L.cnz;
  L.wcfx = L.cfx;
  L.wcfy = L.cfy;
  L.wcfz = L.cfz;
  return true;
}

// Node step on the lanes with `act` set: test the W children, continue with
// the nearest, push the others (farthest first) with their entry distances.
// Lanes without `act` test the top-level root (any valid node) and keep their
// state; only the stack stores are predicated.  When no lane of the wave can
// reach the spill region the pushes go to LDS without a per-entry branch.
template <int FMT, bool COUNT>
__device__ __forceinline__ void node_step(bool act, Lane& L, const SceneView& sc, const Stack& S, uint2* spill,
                                          VisitCounters& vc) {
  constexpr int W = NodeCodec<FMT & kCodecMask>::kW;
  float tn[W];
  uint32_t ch[W];
  if (COUNT) {
    vc.tlas += (act && L.inst_sp < 0) ? 1u : 0u;
    vc.blas += (act && L.inst_sp >= 0) ? 1u : 0u;
  }
  NodeCodec<FMT & kCodecMask>::test(L, sc.nodes, act ? L.cur : sc.tlas_root, L.t_cull, tn, ch);
  sort_children<W>(tn, ch);
  // sorted: the hit children are a prefix; child k (k >= 1) goes to slot p[k],
  // the farthest to the bottom
  bool v[W];
  int pos[W];
  const int sp = L.sp;
#pragma unroll
  for (int k = 1; k < W; ++k) v[k] = act && tn[k] < kInfF;
  pos[W - 1] = sp;
#pragma unroll
  for (int k = W - 2; k >= 1; --k) pos[k] = pos[k + 1] + (v[k + 1] ? 1 : 0);
  if (!__any(act && sp + (W - 1) > S.depth)) {
#pragma unroll
    for (int k = W - 1; k >= 1; --k) {
      if (v[k]) {
        S.ref[64 * pos[k]] = ch[k];
        S.tq[64 * pos[k]] = t_down16(tn[k]);
      }
    }
  } else {
#pragma unroll
    for (int k = 1; k < W; ++k) {
      if (v[k]) {
        if (pos[k] < S.depth) {
          S.ref[64 * pos[k]] = ch[k];
          S.tq[64 * pos[k]] = t_down16(tn[k]);
        } else {
          spill[pos[k] - S.depth] = make_uint2(ch[k], __float_as_uint(tn[k]));
        }
      }
    }
  }
  L.sp = pos[1] + (v[1] ? 1 : 0);
  L.cur = act ? (tn[0] < kInfF ? ch[0] : kEmpty) : L.cur;
}

// Instance step on the lanes with `act` set: a top-level leaf -- transform the
// ray and descend into the prototype's bottom-level root.  Other lanes read
// record 0 and keep their state.
template <bool COUNT>
__device__ __forceinline__ void inst_step(bool act, Lane& L, const SceneView& sc, VisitCounters& vc) {
  if (COUNT) vc.inst += act ? 1u : 0u;
  Lane N = L;
  uint32_t root;
  enter_instance(N, sc, act ? leaf_first(L.cur) : 0u, &root);
  L.ix = act ? N.ix : L.ix;
  L.iy = act ? N.iy : L.iy;
  L.iz = act ? N.iz : L.iz;
  L.cnx = act ? N.cnx : L.cnx;
  L.cny = act ? N.cny : L.cny;
  L.cnz = act ? N.cnz : L.cnz;
  L.cfx = act ? N.cfx : L.cfx;
  L.cfy = act ? N.cfy : L.cfy;
  L.cfz = act ? N.cfz : L.cfz;
  L.lox = act ? N.lox : L.lox;
  L.loy = act ? N.loy : L.loy;
  L.loz = act ? N.loz : L.loz;
  L.Sx = act ? N.Sx : L.Sx;
  L.Sy = act ? N.Sy : L.Sy;
  L.Sz = act ? N.Sz : L.Sz;
  L.kz = act ? N.kz : L.kz;
  L.curve = act ? N.curve : L.curve;
  L.flat = act ? N.flat : L.flat;
  L.rec = act ? N.rec : L.rec;
  L.inst_sp = act ? L.sp : L.inst_sp;
  L.cur = act ? root : L.cur;
}

// Quad step on the lanes with `act` set: test the first quad of the current
// bottom-level leaf and keep the rest of the leaf as the current reference.
template <int FMT, bool COUNT>
__device__ __forceinline__ void quad_step(bool act, Lane& L, const SceneView& sc, VisitCounters& vc) {
  if (COUNT) vc.quads += act ? 1u : 0u;
  const uint32_t first = leaf_first(L.cur), count = leaf_count(L.cur);
  const uint32_t q = act ? first : 0u;
  uint32_t* n64 = COUNT ? &vc.fp64 : nullptr;
  bool answered;
  if constexpr ((FMT & kCodecCurves) != 0) answered = prim_test(L, sc, act, q, n64);
  else answered = quad_test(L, sc, act, q, n64);
  const uint32_t rest = count > 1u ? make_leaf(first + 1u, count - 1u) : kEmpty;
  L.cur = act ? (answered ? kEmpty : rest) : L.cur;
  L.done = L.done || answered;
}

// Pop step of the lanes whose current reference is empty: leave the instance
// when its subtree is exhausted, then take the top entry unless it lies behind
// the closest hit (the lane then pops again on its next step), or finish.
__device__ __forceinline__ void pop_step(Lane& L, const SceneView& sc, const Stack& S, const uint2* spill) {
  const bool need = !L.done && L.cur == kEmpty;
  const bool leave = need && L.sp == L.inst_sp;
  if (__any(leave)) {
    L.ix = leave ? L.wix : L.ix;
    L.iy = leave ? L.wiy : L.iy;
    L.iz = leave ? L.wiz : L.iz;
    L.cnx = leave ? L.wcnx : L.cnx;
    L.cny = leave ? L.wcny : L.cny;
    L.cnz = leave ? L.wcnz : L.cnz;
    L.cfx = leave ? L.wcfx : L.cfx;
    L.cfy = leave ? L.wcfy : L.cfy;
    L.cfz = leave ? L.wcfz : L.cfz;
    L.inst_sp = leave ? -1 : L.inst_sp;
  }
  const bool pop = need && L.sp > 0;
  L.done = L.done || (need && L.sp == 0);
  if (__any(pop)) {
    const int sp = L.sp - (pop ? 1 : 0);
    const int j = max(0, min(sp, S.depth - 1));
    // volatile keeps these LDS reads apart from the spill read below (merged,
    // they become one flat load that waits for vector memory)
    uint32_t ref = *(volatile LdsU32*)(S.ref + 64 * j);
    float t = t_up32(*(volatile LdsU16*)(S.tq + 64 * j));
    if (pop && sp >= S.depth) {
      const uint2 e = spill[sp - S.depth];
      ref = e.x;
      t = __uint_as_float(e.y);
    }
    L.sp = sp;
    L.cur = (pop && t <= L.t_cull) ? ref : L.cur;
  }
}

// Step kinds of a lane: 0 = traversal done, 1 = node test, 2 = instance entry,
// 3 = quad test, 4 = pop.
__device__ __forceinline__ int step_kind(const Lane& L) {
  if (L.done) return 0;
  if (L.cur == kEmpty) return 4;
  if (!ref_is_leaf(L.cur)) return 1;
  return L.inst_sp < 0 ? 2 : 3;
}

// Run the wave-uniform step kind `chosen` on the lanes whose own kind it is.  The
// dispatch on `chosen` is a scalar branch and the steps are predicated, so no
// lane state is merged through divergent control flow.
template <int FMT, bool COUNT>
__device__ __forceinline__ void run_step(int chosen, int kind, Lane& L, const SceneView& sc, const Stack& S,
                                         uint2* spill, VisitCounters& vc) {
  if (chosen == 2) inst_step<COUNT>(kind == 2, L, sc, vc);
  if (chosen == 1) node_step<FMT, COUNT>(kind == 1, L, sc, S, spill, vc);
  if (chosen == 3) quad_step<FMT, COUNT>(kind == 3, L, sc, vc);
}

// Wave-uniform choice among the step kinds the participating lanes need: the
// kind with the largest weighted lane count (ties favour node, then quad, then
// instance); 0 when no lane needs one of them.
__device__ __forceinline__ int vote_kind(int kind) {
  const int cn = __popcll(__ballot(kind == 1));
  const int ci = __popcll(__ballot(kind == 2));
  const int cq = __popcll(__ballot(kind == 3));
  const int sn = 4 * cn, si = RTQ_VOTE_WI * ci, sq = RTQ_VOTE_WQ * cq;
  if (sn >= si && sn >= sq) return cn ? 1 : 0;
  return sq >= si ? 3 : 2;
}

// One traversal step of the wave.  The lanes that take part vote: the wave runs
// only the step kind (node test, instance entry or quad test) that most of them
// need, the others wait.  Running one kind per iteration avoids paying for
// every branch whenever any lane needs it.  Afterwards every lane without a
// current reference pops one stack entry.  Returns true once this lane is done.
template <int FMT, bool COUNT>
__device__ __forceinline__ bool lane_step(Lane& L, const SceneView& sc, const Stack& S, uint2* spill,
                                          VisitCounters& vc) {
  const int kind = step_kind(L);
  if (COUNT) vc.iters += kind != 0 ? 1u : 0u;
  run_step<FMT, COUNT>(vote_kind(kind), kind, L, sc, S, spill, vc);
  pop_step(L, sc, S, spill);
  return L.done;
}

}  // namespace rtq
