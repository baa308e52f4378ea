// FP64 CPU oracle for instanced-quad closest-hit tracing and path tracing
// (Lambertian faces, or principled materials with RGB shading).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or helper with the HIP library; the two only read the same
// seeded input arrays.
//
// What it computes, and where each piece comes from:
//  * Scene: prototype quad meshes instanced by affine transforms (object-level
//    instancing, Section 5.2), quads rendered directly (Section 5.2 "Quads").
//  * Closest hit: by definition the smallest key (t, inst, prim, half) over ALL
//    (instance, quad, half) triangles whose hit satisfies tmin < t <= tmax.  The
//    quad v0..v3 is split on the diagonal v1-v3 into A = (v0, v1, v3) and
//    B = (v2, v3, v1); both sides count (no back-face culling).  Hits are
//    computed on world-space vertices w = A v + t (the oracle transforms the
//    vertices, never the rays) with a plain plane-then-inside test in FP64.
//    The BVH mode only culls which triangles get tested; the test itself is the
//    same function as in brute force, so both modes agree exactly whenever the
//    culling is conservative.
//  * Flags: rays whose FP32 answer may legitimately differ from this FP64 answer
//    (near ties, edge grazes, hits next to the origin, ill-conditioned t).
//  * Camera, counter-based RNG (Philox4x32-10, Salmon et al. 2011), cosine
//    sampling in the orthonormal basis of Duff et al. 2017, and the Lambertian
//    path loop with next-event estimation toward one directional light and a
//    constant sky.  Progressive 1 spp frames follow Section 5.4; the per-sample
//    average over spp is taken in sample order.
//  * Principled materials (Section 5.4, energy conserving and preserving; the
//    BSDF is written out where it is defined): RGB path values.
//  * Gradient of the image with respect to per-face albedo with every path held
//    fixed: path-replay form (each vertex's affine estimate and bounce weight,
//    with the radiance arriving along its bounce) and, independently,
//    forward-mode dual numbers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>
#include <vector>

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- vectors
struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return (1.0 / norm(a)) * a; }
inline double maxabs(V3 a) { return std::max(std::fabs(a.x), std::max(std::fabs(a.y), std::fabs(a.z))); }
inline double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// ---------------------------------------------------------------- flags
enum : uint32_t {
  F_NEAR_TIE = 1u,     // another (inst, prim) hit within the tie window
  F_GRAZE = 2u,        // the ray passes within the graze distance of a boundary edge
  F_NEAR_ORIGIN = 4u,  // the hit lies within the graze distance of the ray origin
  F_T_ILLCOND = 8u,    // FP32 t cannot be trusted to 1e-5 (grazing incidence)
  F_DIAG = 16u,        // the other half of the hit quad is hit within the tie window
  F_SHADE = 32u,       // render only: shading decision within rounding (n.d, n.l, n_z ~ 0)
};

// ---------------------------------------------------------------- scene
// A principled material (Section 5.4: the scene's materials all use Disney's
// principled BSDF, made energy conserving and preserving).  Base color
// c = tint x (the face's albedo or texel), per channel; alpha = roughness^2
// (GGX); metal in [0, 1]; spec in [0, 1] scales the dielectric Fresnel
// reflectance (Schlick, F0 = 0.04).
struct Material {
  double tint[3];
  double alpha, metal, spec;
  double coat = 0.0, calpha = 0.0;  // clearcoat weight and the coat's GGX alpha
};

struct Box {
  double lo[3] = {kInf, kInf, kInf};
  double hi[3] = {-kInf, -kInf, -kInf};
  void grow(V3 p) {
    lo[0] = std::min(lo[0], p.x); hi[0] = std::max(hi[0], p.x);
    lo[1] = std::min(lo[1], p.y); hi[1] = std::max(hi[1], p.y);
    lo[2] = std::min(lo[2], p.z); hi[2] = std::max(hi[2], p.z);
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], b.lo[k]); hi[k] = std::max(hi[k], b.hi[k]); }
  }
  double mag() const {
    double m = 0;
    for (int k = 0; k < 3; ++k) m = std::max(m, std::max(std::fabs(lo[k]), std::fabs(hi[k])));
    return m;
  }
};

struct Node {
  Box b;
  int32_t left = -1, right = -1;  // children (internal)
  int32_t start = 0, count = 0;   // item range (leaf when count > 0)
};

// Plain top-down BVH with an object-median split on the longest centroid axis.
struct Bvh {
  std::vector<Node> nodes;
  std::vector<int32_t> items;
  void build(const std::vector<Box>& boxes) {
    nodes.clear();
    items.resize(boxes.size());
    std::iota(items.begin(), items.end(), 0);
    if (boxes.empty()) return;
    std::vector<V3> cen(boxes.size());
    for (size_t i = 0; i < boxes.size(); ++i)
      cen[i] = {0.5 * (boxes[i].lo[0] + boxes[i].hi[0]), 0.5 * (boxes[i].lo[1] + boxes[i].hi[1]),
                0.5 * (boxes[i].lo[2] + boxes[i].hi[2])};
    nodes.reserve(2 * boxes.size() / 2 + 1);
    struct Job { int32_t node, start, count; };
    std::vector<Job> jobs;
    nodes.push_back(Node{});
    jobs.push_back({0, 0, (int32_t)boxes.size()});
    while (!jobs.empty()) {
      Job j = jobs.back();
      jobs.pop_back();
      Box b, cb;
      for (int32_t i = j.start; i < j.start + j.count; ++i) {
        b.grow(boxes[items[i]]);
        cb.grow(cen[items[i]]);
      }
      nodes[j.node].b = b;
      if (j.count <= 4) {
        nodes[j.node].start = j.start;
        nodes[j.node].count = j.count;
        continue;
      }
      int axis = 0;
      double ext = -1;
      for (int k = 0; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > ext) { ext = cb.hi[k] - cb.lo[k]; axis = k; }
      int32_t mid = j.start + j.count / 2;
      std::nth_element(items.begin() + j.start, items.begin() + mid, items.begin() + j.start + j.count,
                       [&](int32_t a, int32_t c) { return comp(cen[a], axis) < comp(cen[c], axis); });
      int32_t l = (int32_t)nodes.size();
      nodes.push_back(Node{});
      nodes.push_back(Node{});
      nodes[j.node].left = l;
      nodes[j.node].right = l + 1;
      jobs.push_back({l, j.start, mid - j.start});
      jobs.push_back({l + 1, mid, j.start + j.count - mid});
    }
  }
};

// One segment of a tessellated curve (object space).  Round curves: a capsule,
// the points within r of the segment [a, b] (rb = r).  Flat ribbons: the
// segment with radius r at a and rb at b, varying linearly.
struct Cap {
  V3 a, b;
  double r, rb;
};

struct Scene {
  int32_t P = 0;
  std::vector<V3> verts;           // object space, exact copies of the FP32 input
  std::vector<int32_t> quads;      // 4 per quad, local vertex index
  std::vector<int64_t> vo, qo;     // per-prototype offsets
  // curve prototypes (Section 5.2 "Curves"): pkind 1 round, 2 flat ribbons,
  // their curves tessellated into segments (kCapsPerCurve per curve, prototype
  // order) at co[p] .. co[p + 1]
  std::vector<int32_t> pkind;      // 0 quads, 1 round curves, 2 flat ribbons
  std::vector<int64_t> co;         // per-prototype capsule offsets
  std::vector<Cap> caps;
  std::vector<int64_t> fo;         // per-prototype face offsets: a face is a quad or a curve
  std::vector<double> albedo;      // per unique face
  // optional per-face textures: res x res values per unique quad, row v, column u
  std::vector<double> tex;
  int32_t tex_res = 0;
  int32_t tex_ch = 1;  // texel channels: 1 (a scalar albedo) or 3 (an RGB base color)
  // optional environment map: env_w x env_h radiance values, equirectangular
  std::vector<double> env;
  int32_t env_w = 0, env_h = 0;
  // its importance-sampling table: texel k (row-major) is drawn with
  // probability (env_T[k] - env_T[k - 1]) / 2^32 (see env_table)
  std::vector<uint64_t> env_T;
  // optional principled materials (RGB shading): a table and one entry per face;
  // without them every face is Lambertian with its scalar albedo
  std::vector<Material> mats;
  std::vector<int32_t> face_mat;
  int64_t N = 0;
  std::vector<int32_t> iproto;
  std::vector<double> X;           // 12 per instance: row-major [A | t] (FP32 values)
  std::vector<double> Xi;          // 12 per instance: FP64 inverse [A^-1 | -A^-1 t]
  std::vector<double> ainv_frob;   // Frobenius norm of A^-1 (bounds its spectral norm)
  std::vector<Box> proto_box;      // object space
  std::vector<Box> inst_box;       // world space
  std::vector<Bvh> proto_bvh;
  Bvh inst_bvh;
  double scene_mag = 1.0;
};

inline V3 xform_point(const double* X, V3 v) {
  return {X[0] * v.x + X[1] * v.y + X[2] * v.z + X[3], X[4] * v.x + X[5] * v.y + X[6] * v.z + X[7],
          X[8] * v.x + X[9] * v.y + X[10] * v.z + X[11]};
}
inline V3 xform_vec(const double* X, V3 v) {
  return {X[0] * v.x + X[1] * v.y + X[2] * v.z, X[4] * v.x + X[5] * v.y + X[6] * v.z,
          X[8] * v.x + X[9] * v.y + X[10] * v.z};
}

// FP64 inverse of the affine map by cofactors.  Returns false when singular.
bool invert_affine(const double* X, double* Y) {
  const double a = X[0], b = X[1], c = X[2], d = X[4], e = X[5], f = X[6], g = X[8], h = X[9], i = X[10];
  const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  const double det = a * A + b * B + c * C;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  const double r = 1.0 / det;
  double M[9] = {A * r, -(b * i - c * h) * r, (b * f - c * e) * r,
                 B * r, (a * i - c * g) * r, -(a * f - c * d) * r,
                 C * r, -(a * h - b * g) * r, (a * e - b * d) * r};
  for (int k = 0; k < 3; ++k) {
    Y[4 * k + 0] = M[3 * k + 0];
    Y[4 * k + 1] = M[3 * k + 1];
    Y[4 * k + 2] = M[3 * k + 2];
    Y[4 * k + 3] = -(M[3 * k + 0] * X[3] + M[3 * k + 1] * X[7] + M[3 * k + 2] * X[11]);
  }
  return true;
}

void quad_world(const Scene& S, int64_t inst, int64_t q_global, V3 w[4]) {
  const int32_t p = S.iproto[inst];
  const double* X = &S.X[12 * inst];
  for (int k = 0; k < 4; ++k) w[k] = xform_point(X, S.verts[S.vo[p] + S.quads[4 * q_global + k]]);
}

// ---------------------------------------------------------------- ray / triangle
struct Ray {
  V3 o, d;
  double tmin, tmax;
};

struct TriHit {
  bool hit = false;
  double t = kInf, l0 = 0, l1 = 0, l2 = 0;  // barycentric weights of w0, w1, w2
};

// Plane-then-inside test: t from the supporting plane, then the hit point must
// lie on the inner side of all three edges (boundary included).  Two-sided.
TriHit tri_test(const Ray& r, V3 w0, V3 w1, V3 w2, double tmax) {
  TriHit h;
  const V3 n = cross(w1 - w0, w2 - w0);
  const double nn = dot(n, n);
  if (!(nn > 0.0)) return h;
  const double den = dot(n, r.d);
  if (den == 0.0) return h;
  const double t = dot(n, w0 - r.o) / den;
  if (!(t > r.tmin && t <= tmax)) return h;
  const V3 p = r.o + t * r.d;
  const double c0 = dot(cross(w2 - w1, p - w1), n);
  const double c1 = dot(cross(w0 - w2, p - w2), n);
  const double c2 = dot(cross(w1 - w0, p - w0), n);
  if (c0 < 0 || c1 < 0 || c2 < 0) return h;
  h.hit = true;
  h.t = t;
  h.l0 = c0 / nn;
  h.l1 = c1 / nn;
  h.l2 = c2 / nn;
  return h;
}

struct Key {
  double t = kInf;
  int32_t inst = -1, prim = -1, half = -1;
  double u = 0, v = 0;
};
inline bool key_less(const Key& a, const Key& b) {
  if (a.t != b.t) return a.t < b.t;
  if (a.inst != b.inst) return a.inst < b.inst;
  if (a.prim != b.prim) return a.prim < b.prim;
  return a.half < b.half;
}

struct Excl {
  int32_t inst = -1, prim = -1, half = -1;
};

// Both halves of one quad.  u, v: v0 -> (0,0), v1 -> (1,0), v2 -> (1,1), v3 -> (0,1).
inline void quad_hits(const Ray& r, const V3 w[4], double tmax, TriHit hA_hB[2], Key k[2], int32_t inst,
                      int32_t prim) {
  hA_hB[0] = tri_test(r, w[0], w[1], w[3], tmax);
  hA_hB[1] = tri_test(r, w[2], w[3], w[1], tmax);
  k[0] = Key{hA_hB[0].t, inst, prim, 0, hA_hB[0].l1, hA_hB[0].l2};
  k[1] = Key{hA_hB[1].t, inst, prim, 1, 1.0 - hA_hB[1].l1, 1.0 - hA_hB[1].l2};
}

// Closest distance between the ray segment {o + s d, s in [s0, s1]} (s1 may be
// +inf) and the segment [a, b].  Closest points of two segments after Ericson,
// "Real-Time Collision Detection", Section 5.1.9.  Also returns the edge point.
double seg_dist(V3 o, V3 d, double s0, double s1, V3 a, V3 b, V3* q_out) {
  const V3 d2 = b - a;
  const V3 rr = o - a;
  const double A = dot(d, d), E = dot(d2, d2), F = dot(d2, rr);
  const double C = dot(d, rr), B = dot(d, d2);
  double s, t;
  if (E <= 0.0) {  // degenerate edge: point
    s = std::min(std::max(-C / A, s0), s1);
    t = 0.0;
  } else {
    const double den = A * E - B * B;
    s = den > 1e-300 * A * E ? std::min(std::max((B * F - C * E) / den, s0), s1) : s0;
    t = (B * s + F) / E;
    if (t < 0.0) {
      t = 0.0;
      s = std::min(std::max(-C / A, s0), s1);
    } else if (t > 1.0) {
      t = 1.0;
      s = std::min(std::max((B - C) / A, s0), s1);
    }
  }
  const V3 p = o + s * d;
  const V3 q = a + t * d2;
  if (q_out) *q_out = q;
  return norm(p - q);
}

// Distance from point p to triangle (a, b, c): the closest point is found by
// classifying p against the Voronoi regions of the vertices, edges and face
// (Ericson, "Real-Time Collision Detection", Section 5.1.5).
double point_tri_dist(V3 p, V3 a, V3 b, V3 c) {
  const V3 ab = b - a, ac = c - a, ap = p - a;
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) return norm(p - a);
  const V3 bp = p - b;
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) return norm(p - b);
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) return norm(p - (a + (d1 / (d1 - d3)) * ab));
  const V3 cp = p - c;
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) return norm(p - c);
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) return norm(p - (a + (d2 / (d2 - d6)) * ac));
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0)
    return norm(p - (b + ((d4 - d3) / ((d4 - d3) + (d5 - d6))) * (c - b)));
  const double den = va + vb + vc;
  if (!(den > 0)) return std::min(norm(p - a), std::min(norm(p - b), norm(p - c)));  // degenerate
  const double v = vb / den, w = vc / den;
  return norm(p - (a + v * ab + w * ac));
}

// ---------------------------------------------------------------- curves
// Section 5.2 renders the scene's curves (cubic Bezier, round) with Embree's
// curve primitives.  Reading: a curve with control points P0..P3 and radii
// r0..r3 is the chain of kCapsPerCurve capsules between its points at
// parameters j / kCapsPerCurve, each point the FP32 rounding of the Bezier
// evaluated in FP64 by de Casteljau's construction, each capsule's radius the
// FP32 rounding of the mean of the radii at its ends.  A capsule is hit from
// outside only (a ray starting inside it does not hit it).
constexpr int kCapsPerCurve = 8;

inline double lerp(double a, double b, double s) { return a + s * (b - a); }
// de Casteljau evaluation of a cubic Bezier component
double bez(double c0, double c1, double c2, double c3, double s) {
  const double a = lerp(c0, c1, s), b = lerp(c1, c2, s), c = lerp(c2, c3, s);
  const double d = lerp(a, b, s), e = lerp(b, c, s);
  return lerp(d, e, s);
}

// Segments of one curve: cp holds 4 control points (x, y, z, r), FP32 values.
// Round: capsules of the mean radius; flat: the radii at both ends.
void tessellate_curve(const float* cp, Cap out[kCapsPerCurve], bool flat) {
  V3 X[kCapsPerCurve + 1];
  double R[kCapsPerCurve + 1];
  for (int j = 0; j <= kCapsPerCurve; ++j) {
    const double s = (double)j / kCapsPerCurve;
    double v[4];
    for (int c = 0; c < 4; ++c) v[c] = (double)(float)bez(cp[c], cp[4 + c], cp[8 + c], cp[12 + c], s);
    X[j] = V3{v[0], v[1], v[2]};
    R[j] = v[3];
  }
  for (int j = 0; j < kCapsPerCurve; ++j) {
    const double rm = (double)(float)(0.5 * (R[j] + R[j + 1]));
    out[j] = flat ? Cap{X[j], X[j + 1], R[j], R[j + 1]} : Cap{X[j], X[j + 1], rm, rm};
  }
}

// Flat ribbons (Section 5.2 names flat ribbon curves for grass and palm
// fronds).  Reading: a ray-facing ribbon.  Segment c, seen along the ray
// (o, d), is the strip of points within r(u) = r + u (rb - r) of the segment's
// projection onto the plane orthogonal to the ray; the ray meets it when its
// line passes within r(u) of the projected segment's point u closest to it,
// at the depth of that segment point along the ray.  Returns t (+inf when the
// line passes farther), *u_out the segment parameter and *margin the
// distance minus r(u).
// ribbon_eval returns the depth whether or not the line passes within r(u).
double ribbon_eval(V3 o, V3 d, const Cap& c, double* u_out, double* margin) {
  const double dd = dot(d, d);
  const V3 A = c.a - o, B = c.b - o;
  const V3 Ap = A - (dot(A, d) / dd) * d, Bp = B - (dot(B, d) / dd) * d;
  const V3 E = Bp - Ap;
  const double ee = dot(E, E);
  const double u = ee > 0.0 ? std::min(1.0, std::max(0.0, -dot(Ap, E) / ee)) : 0.0;
  *margin = norm(Ap + u * E) - (c.r + u * (c.rb - c.r));
  *u_out = u;
  return dot(A + u * (B - A), d) / dd;
}
double ribbon_hit(V3 o, V3 d, const Cap& c, double* u_out) {
  double m;
  const double t = ribbon_eval(o, d, c, u_out, &m);
  return m > 0.0 ? kInf : t;
}
// The ribbon's normal there (not normalised): the reverse ray direction
// without its component along the segment, so the ribbon faces the ray.
inline V3 ribbon_normal(const Cap& c, V3 d) {
  const V3 T = c.b - c.a;
  const double tt = dot(T, T);
  return tt > 0.0 ? -1.0 * (d - (dot(d, T) / tt) * T) : -1.0 * d;
}

// Distance from point p to the segment [a, b].
double point_seg_dist(V3 p, V3 a, V3 b) {
  const V3 ab = b - a;
  const double e = dot(ab, ab);
  const double u = e > 0.0 ? std::min(1.0, std::max(0.0, dot(p - a, ab) / e)) : 0.0;
  return norm(p - (a + u * ab));
}

// Entry of ray (o, d) (object space, d not normalised) into capsule c: the
// smallest t >= 0 at which the ray reaches the capsule's surface from outside.
// A ray outside the infinite cylinder around the axis enters it at the smaller
// root of the cylinder's quadratic; there it is on the capsule's body if the
// axial coordinate lies within the segment, else it can only enter through the
// end sphere on that side.  A ray starting inside the infinite cylinder but
// beyond an end can only enter through that end's sphere.  Returns +inf when
// the ray misses the capsule or starts inside it; *n receives the outward
// normal (not normalised) and *y01 the axis parameter in [0, 1] of the hit.
double cap_entry(V3 o, V3 d, const Cap& c, V3* n, double* y01) {
  if (point_seg_dist(o, c.a, c.b) < c.r) return kInf;
  const V3 ba = c.b - c.a, oa = o - c.a;
  const double bb = dot(ba, ba), bd = dot(ba, d), bo = dot(ba, oa), dd = dot(d, d);
  const double rr = c.r * c.r;
  auto sphere = [&](V3 ctr, double y) {
    const V3 oc = o - ctr;
    const double b2 = dot(oc, d), c2 = dot(oc, oc) - rr;
    const double disc = b2 * b2 - dd * c2;
    if (disc < 0.0 || b2 >= 0.0) return kInf;  // missed, or moving away from it
    const double t = (-b2 - std::sqrt(disc)) / dd;
    *n = (o + t * d) - ctr;
    *y01 = y;
    return t;
  };
  if (bb <= 0.0) return sphere(c.a, 0.0);
  const double A = bb * dd - bd * bd;
  const double C = bb * dot(oa, oa) - bo * bo - rr * bb;
  if (A <= 1e-30 * bb * dd || C < 0.0) {
    // parallel to the axis, or inside the infinite cylinder beyond an end
    V3 na;
    double ya;
    const double ta = sphere(c.a, 0.0);
    na = *n;
    ya = *y01;
    const double tb = sphere(c.b, 1.0);
    if (ta <= tb) {
      *n = na;
      *y01 = ya;
      return ta;
    }
    return tb;
  }
  const double B = bb * dot(oa, d) - bo * bd;
  const double disc = B * B - A * C;
  if (disc < 0.0) return kInf;  // misses the infinite cylinder, hence the capsule
  const double t = (-B - std::sqrt(disc)) / A;
  if (t < 0.0) return kInf;  // both roots behind the origin
  const double y = bo + t * bd;
  if (y >= 0.0 && y <= bb) {
    *n = (o + t * d) - (c.a + (y / bb) * ba);
    *y01 = y / bb;
    return t;
  }
  return y < 0.0 ? sphere(c.a, 0.0) : sphere(c.b, 1.0);
}

// ---------------------------------------------------------------- traversal
inline bool slab(const Ray& r, const Box& b, double pad, double t_hi) {
  double tn = r.tmin, tf = t_hi;
  for (int k = 0; k < 3; ++k) {
    const double o = comp(r.o, k), d = comp(r.d, k);
    const double lo = b.lo[k] - pad, hi = b.hi[k] + pad;
    if (d == 0.0) {
      if (o < lo || o > hi) return false;
      continue;
    }
    double t0 = (lo - o) / d, t1 = (hi - o) / d;
    if (t0 > t1) std::swap(t0, t1);
    tn = std::max(tn, t0);
    tf = std::min(tf, t1);
  }
  return tn <= tf;
}

// Visit every (instance, quad) -- (instance, capsule) for a curve prototype --
// whose inflated boxes intersect the ray over [tmin, t_hi]; t_hi may shrink as
// the callback finds hits.  g_world is an extra world-space inflation (graze
// distance).  mode 0 visits all primitives.  The callback gets the global quad
// or capsule index.
template <class Fn>
void visit(const Scene& S, const Ray& r, int mode, double g_world, double& t_hi, Fn&& fn) {
  if (mode == 0) {
    for (int64_t i = 0; i < S.N; ++i) {
      const int32_t p = S.iproto[i];
      if (S.pkind[p])
        for (int64_t c = S.co[p]; c < S.co[p + 1]; ++c) fn(i, c);
      else
        for (int64_t q = S.qo[p]; q < S.qo[p + 1]; ++q) fn(i, q);
    }
    return;
  }
  if (S.inst_bvh.nodes.empty()) return;
  thread_local std::vector<int32_t> st, st2;
  st.clear();
  st.push_back(0);
  while (!st.empty()) {
    const Node& nd = S.inst_bvh.nodes[st.back()];
    st.pop_back();
    if (!slab(r, nd.b, g_world + 1e-9 * (nd.b.mag() + 1.0), t_hi)) continue;
    if (nd.count == 0) {
      st.push_back(nd.left);
      st.push_back(nd.right);
      continue;
    }
    for (int32_t k = nd.start; k < nd.start + nd.count; ++k) {
      const int64_t inst = S.inst_bvh.items[k];
      const Box& wb = S.inst_box[inst];
      if (!slab(r, wb, g_world + 1e-9 * (wb.mag() + 1.0), t_hi)) continue;
      const double* Y = &S.Xi[12 * inst];
      Ray ro{xform_point(Y, r.o), xform_vec(Y, r.d), r.tmin, r.tmax};
      const double gobj = g_world * S.ainv_frob[inst];
      const int32_t p = S.iproto[inst];
      const Bvh& pb = S.proto_bvh[p];
      if (pb.nodes.empty()) continue;
      st2.clear();
      st2.push_back(0);
      while (!st2.empty()) {
        const Node& pn = pb.nodes[st2.back()];
        st2.pop_back();
        if (!slab(ro, pn.b, gobj + 1e-9 * (pn.b.mag() + 1.0), t_hi)) continue;
        if (pn.count == 0) {
          st2.push_back(pn.left);
          st2.push_back(pn.right);
          continue;
        }
        const int64_t base = S.pkind[p] ? S.co[p] : S.qo[p];
        for (int32_t m = pn.start; m < pn.start + pn.count; ++m) fn(inst, base + pb.items[m]);
      }
    }
  }
}

// The ray in the object space of instance inst (same parameter t).
inline Ray obj_ray(const Scene& S, int64_t inst, const Ray& r) {
  const double* Y = &S.Xi[12 * inst];
  return Ray{xform_point(Y, r.o), xform_vec(Y, r.d), r.tmin, r.tmax};
}
// World coordinates' extent of capsule c of instance inst, seen from o.
double cap_extent(const Scene& S, int64_t inst, const Cap& c, V3 o) {
  const double* X = &S.X[12 * inst];
  const V3 a = xform_point(X, c.a), b = xform_point(X, c.b);
  return std::max(std::max(maxabs(a - o), maxabs(b - o)), std::max(maxabs(a), maxabs(b)));
}
// World normal (not normalised) of an object-space normal of instance inst: A^-T n.
inline V3 normal_to_world(const Scene& S, int64_t inst, V3 n) {
  const double* Y = &S.Xi[12 * inst];
  return {Y[0] * n.x + Y[4] * n.y + Y[8] * n.z, Y[1] * n.x + Y[5] * n.y + Y[9] * n.z,
          Y[2] * n.x + Y[6] * n.y + Y[10] * n.z};
}
// Outward normal (not normalised) of capsule c at object point p: p minus its
// closest point on the axis segment.
inline V3 cap_normal(const Cap& c, V3 p) {
  const V3 ab = c.b - c.a;
  const double e = dot(ab, ab);
  const double u = e > 0.0 ? std::min(1.0, std::max(0.0, dot(p - c.a, ab) / e)) : 0.0;
  return p - (c.a + u * ab);
}

// Uncertainty (radians) of a capsule's normal at the hit at parameter t along
// world ray r, as an FP32 renderer forms it: the normal follows the hit point,
// whose object-space coordinates carry rounding of about 2^-24 times the hit
// point's offset from the instance origin mapped by the inverse transform, the
// object-space hit point and the capsule's ends; 16 such units, plus a shift
// `t_shift` (world units) of the hit along the ray, over the radius.  One
// radian (no information) for a capsule of radius 0.
double cap_normal_uncertainty(const Scene& S, int64_t inst, const Cap& c, const Ray& r, double t, double t_shift) {
  if (!(c.r > 0.0)) return 1.0;
  const double* X = &S.X[12 * inst];
  const V3 tA{X[3], X[7], X[11]};
  const Ray ro = obj_ray(S, inst, r);
  const V3 ho = ro.o + t * ro.d;
  const V3 pw = r.o + t * r.d;
  const double e = 16.0 * std::ldexp(1.0, -24) * (norm(pw - tA) * S.ainv_frob[inst] + norm(ho) + norm(c.a) + norm(c.b));
  return std::min(1.0, (e + t_shift * S.ainv_frob[inst]) / c.r);
}

// A ray leaving a curve segment does not hit that segment; a ray leaving a flat
// ribbon does not hit any segment of that curve in that instance.  Reading: a
// ray-facing ribbon turns toward every ray, so the neighbouring segments of the
// curve a ray starts on would face it and be met next to its origin.
inline bool curve_excluded(const Scene& S, int32_t pr, int32_t inst, int32_t prim, const Excl& ex) {
  if (inst != ex.inst || ex.half != 0) return false;
  return S.pkind[pr] == 2 ? prim / kCapsPerCurve == ex.prim / kCapsPerCurve : prim == ex.prim;
}

struct TraceOut {
  Key best;
  uint32_t flags = 0;
  int32_t ncand = 0;
  int32_t cand[8];  // up to 4 (inst, prim) pairs hit within the tie window
  double cos_abs = 0;  // |n.d| / |d| at the best hit
  double S = 1;        // position scale of the answer: max(1, |o|, |p|, extent of the hit quad seen from o)
};

// Closest hit by key, then the flag pass over the same candidate triangles.
TraceOut trace_one(const Scene& S, const Ray& r, const Excl& ex, double r0, int mode, bool any_hit) {
  TraceOut out;
  const double dn = norm(r.d);
  if (!(dn > 0.0) || !std::isfinite(dn) || !std::isfinite(maxabs(r.o))) return out;  // miss
  // pass 1: the closest hit
  double t_hi = r.tmax;
  Key best;
  visit(S, r, mode, 0.0, t_hi, [&](int64_t inst, int64_t qg) {
    const int32_t pr0 = S.iproto[inst];
    if (S.pkind[pr0]) {
      // capsule or ribbon segment qg: in object space, key (t, inst, prim, half 0)
      const int32_t prim = (int32_t)(qg - S.co[pr0]);
      if (curve_excluded(S, pr0, (int32_t)inst, prim, ex)) return;
      const Ray ro = obj_ray(S, inst, r);
      V3 n;
      double y = 0.0;
      const double t = S.pkind[pr0] == 2 ? ribbon_hit(ro.o, ro.d, S.caps[qg], &y) : cap_entry(ro.o, ro.d, S.caps[qg], &n, &y);
      if (t < kInf && t > r.tmin && t <= t_hi) {
        const Key k{t, (int32_t)inst, prim, 0, ((prim % kCapsPerCurve) + y) / kCapsPerCurve, 0.0};
        if (key_less(k, best)) best = k;
      }
      if (best.t < t_hi) t_hi = best.t;
      return;
    }
    V3 w[4];
    quad_world(S, inst, qg, w);
    TriHit h[2];
    Key k[2];
    const int32_t prim = (int32_t)(qg - S.qo[S.iproto[inst]]);
    quad_hits(r, w, t_hi, h, k, (int32_t)inst, prim);
    for (int s = 0; s < 2; ++s) {
      if (!h[s].hit) continue;
      if (k[s].inst == ex.inst && k[s].prim == ex.prim && k[s].half == ex.half) continue;
      if (key_less(k[s], best)) best = k[s];
    }
    if (best.t < t_hi) t_hi = best.t;
  });
  out.best = best;
  const bool hit = best.inst >= 0;
  const V3 p = hit ? r.o + best.t * r.d : r.o;
  const double Sv = std::max(1.0, std::max(maxabs(r.o), maxabs(p)));
  // FP32 answers carry errors proportional to the coordinates they are computed
  // from: the ray origin, the hit point, and the vertices of the tested quad
  // relative to the origin (a large quad seen from close by).  Every threshold
  // below is 1e-6 times the largest of these.
  auto extent = [&](const V3 w[4]) {
    double e = 0.0;
    for (int k = 0; k < 4; ++k) e = std::max(e, maxabs(w[k] - r.o));
    return e;
  };
  double S_best = Sv;
  // pass 2: flags
  double t_end = std::isfinite(r.tmax) ? r.tmax + 1e-5 * r.tmax + 1e-6 * Sv / dn : kInf, win = 0;
  if (hit) {
    V3 n;
    const int32_t bp = S.iproto[best.inst];
    if (S.pkind[bp]) {
      const Cap& c = S.caps[S.co[bp] + best.prim];
      S_best = std::max(Sv, cap_extent(S, best.inst, c, r.o));
      const Ray ro = obj_ray(S, best.inst, r);
      n = normal_to_world(S, best.inst, S.pkind[bp] == 2 ? ribbon_normal(c, ro.d) : cap_normal(c, ro.o + best.t * ro.d));
    } else {
      V3 w[4];
      quad_world(S, best.inst, S.qo[bp] + best.prim, w);
      S_best = std::max(Sv, extent(w));
      n = best.half == 0 ? cross(w[1] - w[0], w[3] - w[0]) : cross(w[3] - w[2], w[1] - w[2]);
    }
    win = 1e-5 * best.t + 1e-6 * S_best / dn;
    t_end = best.t + win;
    if (best.t * dn < 1e-6 * S_best + r0) out.flags |= F_NEAR_ORIGIN;
    out.cos_abs = std::fabs(dot(n, r.d)) / (norm(n) * dn);
    if (16.0 * std::ldexp(1.0, -24) * S_best > 1e-5 * best.t * dn * out.cos_abs) out.flags |= F_T_ILLCOND;
  }
  out.S = S_best;
  const double s_hi = hit ? std::max(Sv, maxabs(r.o) + t_end * maxabs(r.d)) : std::max(Sv, S.scene_mag);
  const double g_cull = 1e-6 * 1.01 * (s_hi + maxabs(r.o) + S.scene_mag) + r0;
  const V3 o0 = r.o + r.tmin * r.d;
  double t_lim = t_end;
  visit(S, r, mode, g_cull, t_lim, [&](int64_t inst, int64_t qg) {
    const int32_t pr0 = S.iproto[inst];
    if (S.pkind[pr0] == 2) {
      // ribbon: near tie; graze when the line passes within the graze distance
      // of the strip's edge at a depth up to t_end; near origin when that
      // depth lies within it of tmin (object space, as for capsules)
      const int32_t prim = (int32_t)(qg - S.co[pr0]);
      if (curve_excluded(S, pr0, (int32_t)inst, prim, ex)) return;
      const Cap& c = S.caps[qg];
      const double Sq = std::max(Sv, cap_extent(S, inst, c, r.o));
      const double g = (1e-6 * Sq + r0) * S.ainv_frob[inst];
      const Ray ro = obj_ray(S, inst, r);
      double u, m;
      const double t = ribbon_eval(ro.o, ro.d, c, &u, &m);
      const double dlen = norm(ro.d);
      if (m < g && std::fabs(t - r.tmin) * dlen < g) out.flags |= F_NEAR_ORIGIN;
      const bool same = hit && inst == best.inst && prim == best.prim;
      if (m <= 0.0 && t > r.tmin && t <= t_end && !same) {
        out.flags |= F_NEAR_TIE;
        bool dup = false;
        for (int cc = 0; cc < out.ncand; ++cc)
          if (out.cand[2 * cc] == (int32_t)inst && out.cand[2 * cc + 1] == prim) dup = true;
        if (!dup && out.ncand < 4) {
          out.cand[2 * out.ncand] = (int32_t)inst;
          out.cand[2 * out.ncand + 1] = prim;
          out.ncand++;
        }
      }
      if (std::fabs(m) < g && t > r.tmin - g / dlen && t <= t_end) out.flags |= F_GRAZE;
      return;
    }
    if (S.pkind[pr0]) {
      // capsule: near origin, near tie and graze (the ray passing within the
      // graze distance of the capsule's surface), in object space with the
      // world distance scaled by |A^-1|
      const int32_t prim = (int32_t)(qg - S.co[pr0]);
      if (curve_excluded(S, pr0, (int32_t)inst, prim, ex)) return;
      const Cap& c = S.caps[qg];
      const double Sq = std::max(Sv, cap_extent(S, inst, c, r.o));
      const double g = (1e-6 * Sq + r0) * S.ainv_frob[inst];
      const Ray ro = obj_ray(S, inst, r);
      const V3 oo0 = ro.o + r.tmin * ro.d;
      if (std::fabs(point_seg_dist(oo0, c.a, c.b) - c.r) < g) out.flags |= F_NEAR_ORIGIN;
      V3 n;
      double y;
      const double t = cap_entry(ro.o, ro.d, c, &n, &y);
      const bool same = hit && inst == best.inst && prim == best.prim;
      if (t < kInf && t > r.tmin && t <= t_end && !same) {
        out.flags |= F_NEAR_TIE;
        bool dup = false;
        for (int cc = 0; cc < out.ncand; ++cc)
          if (out.cand[2 * cc] == (int32_t)inst && out.cand[2 * cc + 1] == prim) dup = true;
        if (!dup && out.ncand < 4) {
          out.cand[2 * out.ncand] = (int32_t)inst;
          out.cand[2 * out.ncand + 1] = prim;
          out.ncand++;
        }
      }
      // graze: the ray's closest approach to the axis (over t >= tmin, not cut
      // at t_end: the hit point itself lies on the surface) within g of the
      // radius, where the capsule could be entered no later than t_end (the
      // entry lies within the half-chord sqrt(2 r g + g^2) of that approach)
      V3 q;
      const double dist = seg_dist(ro.o, ro.d, r.tmin, kInf, c.a, c.b, &q);
      const double ddo = dot(ro.d, ro.d);
      const double s_q = dot(q - ro.o, ro.d) / ddo;
      const double half = std::sqrt(2.0 * c.r * g + g * g) / std::sqrt(ddo);
      if (std::fabs(dist - c.r) < g && s_q - half <= t_end) out.flags |= F_GRAZE;
      return;
    }
    V3 w[4];
    quad_world(S, inst, qg, w);
    const int32_t prim = (int32_t)(qg - S.qo[S.iproto[inst]]);
    const double Sq = std::max(Sv, extent(w));
    TriHit h[2];
    Key k[2];
    quad_hits(r, w, t_end, h, k, (int32_t)inst, prim);
    const bool same = hit && inst == best.inst && prim == best.prim;
    for (int s = 0; s < 2; ++s) {
      const bool excluded = (int32_t)inst == ex.inst && prim == ex.prim && s == ex.half;
      if (excluded) continue;
      // a triangle next to the ray origin may be hit at t ~ 0 in FP32
      const double dorg = s == 0 ? point_tri_dist(o0, w[0], w[1], w[3]) : point_tri_dist(o0, w[2], w[3], w[1]);
      if (dorg < 1e-6 * Sq + r0) out.flags |= F_NEAR_ORIGIN;
      if (!h[s].hit) continue;
      if (!same) {
        out.flags |= F_NEAR_TIE;
        bool dup = false;
        for (int c = 0; c < out.ncand; ++c)
          if (out.cand[2 * c] == (int32_t)inst && out.cand[2 * c + 1] == prim) dup = true;
        if (!dup && out.ncand < 4) {
          out.cand[2 * out.ncand] = (int32_t)inst;
          out.cand[2 * out.ncand + 1] = prim;
          out.ncand++;
        }
      } else if (s != best.half) {
        out.flags |= F_DIAG;
      }
    }
    static const int E[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
    for (int e = 0; e < 4; ++e) {
      V3 q;
      const double dist = seg_dist(r.o, r.d, r.tmin, t_end, w[E[e][0]], w[E[e][1]], &q);
      if (dist < 1e-6 * std::max(Sq, maxabs(q)) + r0) out.flags |= F_GRAZE;
    }
    {
      // the diagonal v1-v3 is a real boundary too: the two halves of a non-planar
      // quad overlap in projection on one side of it and leave an uncovered sliver
      // on the other, so a ray grazing it may hit this quad or miss it entirely
      V3 q;
      const double dist = seg_dist(r.o, r.d, r.tmin, t_end, w[1], w[3], &q);
      if (dist < 1e-6 * std::max(Sq, maxabs(q)) + r0) out.flags |= F_GRAZE;
    }
  });
  if (any_hit) out.flags &= ~(uint32_t)(F_NEAR_TIE | F_DIAG | F_T_ILLCOND);
  return out;
}

// ---------------------------------------------------------------- acceptance
// Every answer an FP32 traversal may legitimately give for one ray.  The FP32
// test of a triangle can disagree with the exact test only where rounding can
// move the ray across the triangle's boundary, or its hit across an end of the
// ray's interval:
//  * the ray passes within the graze distance of one of the triangle's edges,
//    measured in the plane orthogonal to the ray (the watertight test decides
//    inside/outside there, from edge functions of the projected vertices);
//  * the triangle lies within the graze distance of the ray's start point
//    (its FP32 t may fall on either side of tmin);
//  * its hit lies within the tie window of tmax.
// A triangle hit by the exact test with none of these near is a *certain*
// hit: every FP32 traversal finds it.  A triangle is a *possible* answer when
// rounding can make it a hit.  The closest certain hit C bounds the answer: a
// traversal reports C, or a possible answer no farther than C plus its tie
// window; without a certain hit a miss is acceptable too.  The graze distance
// is the one the flags use, 1e-6 of the position scale plus the origin
// uncertainty r0.

// Distance from the line {o + s d : s real} to the segment [a, b], measured in
// the plane orthogonal to d (equal to the 3D distance from the line).
double line_seg_dist(V3 o, V3 d, V3 a, V3 b) {
  const double dd = dot(d, d);
  const V3 qa = a - o, qb = b - o;
  const V3 pa = qa - (dot(qa, d) / dd) * d;
  const V3 pb = qb - (dot(qb, d) / dd) * d;
  const V3 e = pb - pa;
  const double ee = dot(e, e);
  const double u = ee > 0.0 ? std::min(1.0, std::max(0.0, -dot(pa, e) / ee)) : 0.0;
  return norm(pa + u * e);
}

struct Cand {
  Key k;           // t: where the ray meets the triangle's plane
  bool certain;    // hit by every FP32 traversal
  bool illcond;    // its FP32 t cannot be trusted to 1e-5
  double win;      // tie window at its t
  double tulp;     // change of t when the ray moves 2^-24 S along the normal: 2^-24 S / (|d| |cos|)
};

struct AcceptSet {
  bool ray_ok = true;      // finite origin and non-zero direction
  bool has_certain = false;
  Cand certain;            // the closest certain hit
  std::vector<Cand> cand;  // possible answers no farther than the certain hit's window
};

// One triangle (w0, w1, w2) of quad (inst, prim), half `half`, against ray r:
// whether it is a possible answer and whether it is a certain hit.
struct TriClass {
  bool possible = false, certain = false, illcond = false;
  double t = kInf, S = 1.0, tulp = kInf;
};
TriClass classify_tri(const Ray& r, double dn, double Sv, V3 w0, V3 w1, V3 w2, const V3 wq[4], double r0) {
  TriClass c;
  double ext = 0.0;
  for (int k = 0; k < 4; ++k) ext = std::max(ext, std::max(maxabs(wq[k] - r.o), maxabs(wq[k])));
  const double Sq = std::max(Sv, ext);
  c.S = Sq;
  const double thr = 1e-6 * Sq + r0;
  const V3 n = cross(w1 - w0, w2 - w0);
  const double nn = dot(n, n);
  if (!(nn > 0.0)) return c;  // degenerate: never hit (its edge functions sum to zero)
  const double den = dot(n, r.d);
  const V3 o0 = r.o + r.tmin * r.d;
  const bool near_org = point_tri_dist(o0, w0, w1, w2) < thr;
  const double g = std::min(line_seg_dist(r.o, r.d, w0, w1),
                            std::min(line_seg_dist(r.o, r.d, w1, w2), line_seg_dist(r.o, r.d, w2, w0)));
  const bool graze = g < thr;
  if (den == 0.0) {
    // parallel to the plane: only rounding can produce a hit
    c.possible = near_org;
    c.t = r.tmin;
    c.illcond = true;
    return c;
  }
  const double t = dot(n, w0 - r.o) / den;
  c.t = t;
  const V3 p = r.o + t * r.d;
  const double c0 = dot(cross(w2 - w1, p - w1), n);
  const double c1 = dot(cross(w0 - w2, p - w2), n);
  const double c2 = dot(cross(w1 - w0, p - w0), n);
  const bool inside = c0 >= 0 && c1 >= 0 && c2 >= 0;
  const bool in_iv = t > r.tmin && t <= r.tmax;
  const bool near_tmax = std::isfinite(r.tmax) && std::fabs(t - r.tmax) <= 1e-5 * r.tmax + 1e-6 * Sq / dn;
  const double cosv = std::fabs(den) / (std::sqrt(nn) * dn);
  c.illcond = 16.0 * std::ldexp(1.0, -24) * Sq > 1e-5 * std::fabs(t) * dn * cosv;
  c.tulp = std::ldexp(1.0, -24) * Sq / (dn * cosv);
  c.certain = inside && in_iv && !graze && !near_org && !near_tmax;
  c.possible = (inside || graze) && (in_iv || near_org || near_tmax);
  return c;
}

// Capsule c of instance inst against ray r (world) -- the same classes as a
// triangle: rounding can move the ray across the capsule's silhouette (the
// ray passes within the graze distance of its surface), its start point may
// lie within that distance of the surface, or the hit may lie next to tmax.
// Distances are taken in object space, the world graze distance scaled by
// |A^-1|.
// Ribbon segment c of instance inst against ray r: rounding can move the line
// across the strip's edge (graze), or the depth across tmin (near origin) or
// tmax.  t is ill-conditioned where the ray runs nearly along the segment
// (the closest point then moves fast along it): the sine of that angle plays
// the part of a triangle's |cos|.
TriClass classify_ribbon(const Scene& S, int64_t inst, const Cap& c, const Ray& r, double dn, double Sv, double r0) {
  TriClass k;
  const double Sq = std::max(Sv, cap_extent(S, inst, c, r.o));
  k.S = Sq;
  const double thr = (1e-6 * Sq + r0) * S.ainv_frob[inst];
  const Ray ro = obj_ray(S, inst, r);
  double u, m;
  const double t = ribbon_eval(ro.o, ro.d, c, &u, &m);
  const double dlen = norm(ro.d);
  const bool hit = m <= 0.0;
  const bool graze = std::fabs(m) < thr;
  const bool near_org = m < thr && std::fabs(t - r.tmin) * dlen < thr;
  const V3 T = c.b - c.a;
  const double tl = norm(T);
  const double cosv = tl > 0.0 ? norm(cross(T, ro.d)) / (tl * dlen) : 1.0;
  k.t = t;
  const bool in_iv = t > r.tmin && t <= r.tmax;
  const bool near_tmax = std::isfinite(r.tmax) && std::fabs(t - r.tmax) <= 1e-5 * r.tmax + 1e-6 * Sq / dn;
  k.illcond = !(cosv > 0.0) || 16.0 * std::ldexp(1.0, -24) * Sq > 1e-5 * std::fabs(t) * dn * cosv;
  k.tulp = cosv > 0.0 ? std::ldexp(1.0, -24) * Sq / (dn * cosv) : kInf;
  k.certain = hit && in_iv && !graze && !near_org && !near_tmax;
  k.possible = (hit || graze) && (in_iv || near_org || near_tmax);
  return k;
}

TriClass classify_cap(const Scene& S, int64_t inst, const Cap& c, const Ray& r, double dn, double Sv, double r0) {
  TriClass k;
  const double Sq = std::max(Sv, cap_extent(S, inst, c, r.o));
  k.S = Sq;
  const double thr = (1e-6 * Sq + r0) * S.ainv_frob[inst];
  const Ray ro = obj_ray(S, inst, r);
  const V3 o0 = ro.o + r.tmin * ro.d;
  const bool near_org = std::fabs(point_seg_dist(o0, c.a, c.b) - c.r) < thr;
  const double lg = line_seg_dist(ro.o, ro.d, c.a, c.b);
  const bool graze = std::fabs(lg - c.r) < thr;
  V3 n;
  double y;
  double t = cap_entry(ro.o, ro.d, c, &n, &y);
  const bool inside = t < kInf;
  double cosv = 0.0;
  if (inside) {
    cosv = std::fabs(dot(n, ro.d)) / (norm(n) * norm(ro.d));
  } else {
    // no exact hit: the parameter of the ray's closest approach to the axis
    const V3 ab = c.b - c.a, w0 = ro.o - c.a;
    const double a = dot(ro.d, ro.d), b = dot(ro.d, ab), e = dot(ab, ab);
    const double dd = dot(ro.d, w0), ee = dot(ab, w0);
    const double den = a * e - b * b;
    t = den > 1e-300 * a * e ? (b * ee - e * dd) / den : -dd / a;
    if (near_org && !(t > r.tmin)) t = r.tmin;
  }
  k.t = t;
  const bool in_iv = t > r.tmin && t <= r.tmax;
  const bool near_tmax = std::isfinite(r.tmax) && std::fabs(t - r.tmax) <= 1e-5 * r.tmax + 1e-6 * Sq / dn;
  k.illcond = !(cosv > 0.0) || 16.0 * std::ldexp(1.0, -24) * Sq > 1e-5 * std::fabs(t) * dn * cosv;
  k.tulp = cosv > 0.0 ? std::ldexp(1.0, -24) * Sq / (dn * cosv) : kInf;
  k.certain = inside && in_iv && !graze && !near_org && !near_tmax;
  k.possible = (inside || graze || near_org) && (in_iv || near_org || near_tmax);
  return k;
}

AcceptSet accept_set(const Scene& S, const Ray& r, const Excl& ex, double r0, int mode) {
  AcceptSet A;
  const double dn = norm(r.d);
  if (!(dn > 0.0) || !std::isfinite(dn) || !std::isfinite(maxabs(r.o))) {
    A.ray_ok = false;
    return A;
  }
  const double Sv = std::max(1.0, maxabs(r.o));
  auto each_tri = [&](int64_t inst, int64_t qg, auto&& fn) {
    const int32_t pr0 = S.iproto[inst];
    if (S.pkind[pr0]) {
      const int32_t prim = (int32_t)(qg - S.co[pr0]);
      if (curve_excluded(S, pr0, (int32_t)inst, prim, ex)) return;
      fn((int32_t)inst, prim, 0,
         S.pkind[pr0] == 2 ? classify_ribbon(S, inst, S.caps[qg], r, dn, Sv, r0)
                           : classify_cap(S, inst, S.caps[qg], r, dn, Sv, r0));
      return;
    }
    V3 w[4];
    quad_world(S, inst, qg, w);
    const int32_t prim = (int32_t)(qg - S.qo[S.iproto[inst]]);
    for (int h = 0; h < 2; ++h) {
      if ((int32_t)inst == ex.inst && prim == ex.prim && h == ex.half) continue;
      const TriClass c = h == 0 ? classify_tri(r, dn, Sv, w[0], w[1], w[3], w, r0)
                                : classify_tri(r, dn, Sv, w[2], w[3], w[1], w, r0);
      fn((int32_t)inst, prim, h, c);
    }
  };
  // pass 1: the closest certain hit (the search range shrinks only on certain hits)
  double t_hi = r.tmax;
  const double g_enum = 1e-6 * 1.01 * (std::max(Sv, S.scene_mag) + maxabs(r.o) + S.scene_mag) + r0;
  visit(S, r, mode, g_enum, t_hi, [&](int64_t inst, int64_t qg) {
    each_tri(inst, qg, [&](int32_t i, int32_t pr, int h, const TriClass& c) {
      if (!c.certain) return;
      Cand cd{Key{c.t, i, pr, h, 0, 0}, true, c.illcond, 1e-5 * c.t + 1e-6 * c.S / dn, c.tulp};
      if (!A.has_certain || key_less(cd.k, A.certain.k)) {
        A.certain = cd;
        A.has_certain = true;
      }
    });
    if (A.has_certain) t_hi = std::min(t_hi, A.certain.k.t + A.certain.win);
  });
  // pass 2: every possible answer up to the certain hit's window.  A triangle
  // whose edge grazes the ray may lie up to (graze distance) / |cos| beyond its
  // plane crossing; the enumeration reaches 1e-3 of the scene scale further.
  const double t_lim = A.has_certain ? A.certain.k.t + A.certain.win : r.tmax;
  double t_enum = std::isfinite(t_lim) ? t_lim + 1e-3 * std::max(Sv, S.scene_mag) / dn : kInf;
  visit(S, r, mode, g_enum, t_enum, [&](int64_t inst, int64_t qg) {
    each_tri(inst, qg, [&](int32_t i, int32_t pr, int h, const TriClass& c) {
      if (!c.possible || c.t > t_lim) return;
      A.cand.push_back(
          Cand{Key{c.t, i, pr, h, 0, 0}, c.certain, c.illcond, 1e-5 * std::fabs(c.t) + 1e-6 * c.S / dn, c.tulp});
    });
  });
  return A;
}

// Verdict on one closest-hit answer (inst, prim, half; half < 0 = either) at
// parameter t_gpu: 0 valid, 1 not a possible answer, 2 a miss while a certain
// hit exists, 3 t outside its tolerance (1e-5 relative plus the tie window's
// absolute term; where t is ill-conditioned, 16 units of 2^-24 S / (|d| |cos|)).
// *info: bit 1 the answer is the certain hit, bit 2 t is ill-conditioned (held
// to the FP32 bound).
int judge_closest(const AcceptSet& A, int32_t inst, int32_t prim, int32_t half, double t_gpu, int* info,
                  double* ulps = nullptr) {
  *info = 0;
  if (ulps) *ulps = 0.0;
  if (!A.ray_ok) return inst < 0 ? 0 : 1;
  if (inst < 0) return A.has_certain ? 2 : 0;
  const Cand* best = nullptr;
  for (const Cand& c : A.cand)
    if (c.k.inst == inst && c.k.prim == prim && (half < 0 || c.k.half == half)) {
      if (!best || std::fabs(c.k.t - t_gpu) < std::fabs(best->k.t - t_gpu)) best = &c;
    }
  if (!best) return 1;
  if (A.has_certain && A.certain.k.inst == inst && A.certain.k.prim == prim &&
      (half < 0 || A.certain.k.half == half))
    *info |= 1;
  const double err = std::fabs(t_gpu - best->k.t);
  if (ulps) *ulps = err / best->tulp;
  if (best->illcond) {
    // FP32 cannot resolve t to 1e-5 here: t is held to the FP32 bound instead,
    // 16 units of 2^-24 S along the normal, carried along the ray
    *info |= 2;
    return err <= 16.0 * best->tulp + best->win ? 0 : 3;
  }
  return err <= best->win ? 0 : 3;
}

// Verdict on one any-hit answer: 0 valid, 1 occluded without any possible
// occluder, 2 unoccluded while a certain occluder exists.
int judge_any(const AcceptSet& A, bool occluded) {
  if (!A.ray_ok) return occluded ? 1 : 0;
  if (occluded) return A.cand.empty() && !A.has_certain ? 1 : 0;
  return A.has_certain ? 2 : 0;
}

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw 2011).
void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
inline double unit(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

// ---------------------------------------------------------------- rendering
struct Params {
  int32_t spp, depth;
  uint64_t seed;
  uint32_t frame;
  double light[3];
  double E, L_sky;
  int n_area = 0;               // quad area lights
  const double* area = nullptr;  // 10 per light: corner, edge 1, edge 2, emitted radiance
  bool env_nee = false;          // next-event estimation toward the environment map
};

// pi: spp, depth, environment next-event estimation (0/1); pd: light
// direction (3), E, L_sky, number of area lights, then 10 per light.
Params make_params(const int32_t* pi, const uint64_t* pu, const double* pd) {
  Params P{pi[0], pi[1], pu[0], (uint32_t)pu[1], {pd[0], pd[1], pd[2]}, pd[3], pd[4]};
  P.n_area = (int)pd[5];
  P.area = pd + 6;
  P.env_nee = pi[2] != 0;
  return P;
}

// A pinhole view, or the rectangle (tx, ty, tw, th) of it that a call renders
// (Section 5.5 deals the tiles of a frame to the workers); its paths draw
// random numbers by (pixel of the whole view, sample, view id, bounce).
struct Cam {
  V3 eye, f, r, u;
  double tan_half, aspect;
  int64_t w, h, off;
  int64_t view_id, tx, ty, tw, th;
};

// ci: w, h, image offset of the rectangle, view id, tile x, y, width, height.
Cam make_cam(const double* cf, const int64_t* ci) {
  Cam c;
  c.eye = {cf[0], cf[1], cf[2]};
  const V3 look{cf[3], cf[4], cf[5]}, up{cf[6], cf[7], cf[8]};
  c.f = normalize(look - c.eye);
  c.r = normalize(cross(c.f, up));
  c.u = cross(c.r, c.f);
  c.tan_half = std::tan(0.5 * cf[9] * kPi / 180.0);
  c.w = ci[0];
  c.h = ci[1];
  c.off = ci[2];
  c.view_id = ci[3];
  c.tx = ci[4];
  c.ty = ci[5];
  c.tw = ci[6];
  c.th = ci[7];
  c.aspect = (double)c.w / (double)c.h;
  return c;
}

// ---------------------------------------------------------------- principled BSDF
// RGB triple (the three channels shade independently along one path).
struct C3 {
  double v[3] = {0.0, 0.0, 0.0};
};
inline C3 c3(double x) {
  C3 r;
  r.v[0] = r.v[1] = r.v[2] = x;
  return r;
}
inline C3 operator+(C3 a, C3 b) {
  for (int k = 0; k < 3; ++k) a.v[k] += b.v[k];
  return a;
}
inline C3 operator*(C3 a, C3 b) {
  for (int k = 0; k < 3; ++k) a.v[k] *= b.v[k];
  return a;
}
inline C3 operator*(double s, C3 a) {
  for (int k = 0; k < 3; ++k) a.v[k] *= s;
  return a;
}

// The BSDF (a reading of Section 5.4; the paper gives no formulas).  At a vertex
// with unit normal n on the viewer's side and unit direction wo to the viewer,
// mu_o = n . wo, the cosine-weighted BSDF toward wi (mu_i = n . wi > 0) is
//   f mu_i = (1 - m) [F_d p_s(wi) + (1 - F_d) c mu_i / pi] + m F_c p_s(wi)
// with F_d = spec (F0 + (1 - F0)(1 - mu_o)^5), F0 = 0.04, the dielectric
// Fresnel weight, and F_c = c + (1 - c)(1 - mu_o)^5 the metal's (Schlick, both at
// the macro-surface angle).  p_s is the density of the specular lobe: a GGX
// visible normal h is drawn (Heitz 2018; alpha = roughness^2, separable Smith
// masking), wo is reflected about it, and a reflection below the surface is
// mirrored above it (w - 2 (n . w) n), so p_s integrates to one over the upper
// hemisphere: the energy a single-scattering lobe loses below the horizon is
// returned in closed form.  Hence the albedo of the BSDF at wo is
// (1 - m)[F_d + (1 - F_d) c] + m F_c: at most one (energy conserving) and exactly
// one for c = 1 (energy preserving).  With m = spec = 0 it is Lambert's c / pi.
// The specular lobe is drawn with probability P_s = (1 - m) F_d + m (it does not
// depend on c, so a path's directions do not depend on the albedo), the cosine
// lobe otherwise; the weight of a sampled direction is f mu_i / pdf with
// pdf = P_s p_s + (1 - P_s) mu_i / pi.  f mu_i = A + B c is affine in c.
//
// A clearcoat of weight k (the principled model's coat layer) lies over that
// base: a second mirrored visible-normal lobe p_k of its own roughness with the
// Fresnel weight F_k = k (F0 + (1 - F0)(1 - mu_o)^5), and the base below it
// receives what the coat does not reflect:
//   f mu_i = F_k p_k(wi) + (1 - F_k) [base f mu_i],
// so the albedo is F_k + (1 - F_k) [base albedo]: still at most one, and one
// for c = 1.  The coat lobe is drawn with probability F_k, the base's lobes
// with the rest; the density is F_k p_k + (1 - F_k) [base density].  k = 0 is
// the base alone.
struct Shade {
  V3 n, wo, t1, t2;  // frame: t1, t2 the basis of Duff et al. 2017 about n
  double mo;         // n . wo
  double alpha, metal, Fd, k5, Ps;
  double calpha, Fk, Pn;  // the coat's alpha and weight F_k; Pn = F_k + (1 - F_k) P_s, a non-diffuse lobe's probability
  C3 tint;
};

inline double ggx_D(double a, double nh) {
  const double a2 = a * a, q = nh * nh * (a2 - 1.0) + 1.0;
  return a2 / (kPi * q * q);
}
inline double smith_G1(double a, double mu) { return 2.0 * mu / (mu + std::sqrt(a * a + (1.0 - a * a) * mu * mu)); }

// basis (t1, t2, n) of Duff et al. 2017; `flip` takes the other sign branch
void duff_basis(V3 n, bool flip, V3* t1, V3* t2) {
  double sg = n.z >= 0 ? 1.0 : -1.0;
  if (flip) sg = -sg;
  const double aa = -1.0 / (sg + n.z);
  const double bb = n.x * n.y * aa;
  *t1 = V3{1.0 + sg * n.x * n.x * aa, sg * bb, -sg * n.x};
  *t2 = V3{bb, sg + n.y * n.y * aa, -n.y};
}

Shade make_shade(const Material& M, V3 n, V3 wo, bool flip) {
  Shade s;
  s.n = n;
  s.wo = wo;
  duff_basis(n, flip, &s.t1, &s.t2);
  s.mo = dot(n, wo);
  const double om = std::max(0.0, 1.0 - s.mo);
  s.k5 = om * om * om * om * om;
  s.alpha = M.alpha;
  s.metal = M.metal;
  s.Fd = M.spec * (0.04 + 0.96 * s.k5);
  s.Ps = (1.0 - M.metal) * s.Fd + M.metal;
  s.calpha = M.calpha;
  s.Fk = M.coat * (0.04 + 0.96 * s.k5);
  s.Pn = s.Fk + (1.0 - s.Fk) * s.Ps;
  for (int k = 0; k < 3; ++k) s.tint.v[k] = M.tint[k];
  return s;
}

// density of the folded specular lobe toward wi (mu_i > 0): each preimage
// direction (the reflection itself and, when mu_o > mu_i, its mirror below the
// surface) contributes G1(mu_o) D(h) / (4 mu_o), h the half vector
double spec_pdf(const Shade& s, double alpha, V3 wi) {
  const double mi = dot(s.n, wi);
  if (!(mi > 0.0) || !(s.mo > 0.0)) return 0.0;
  const double g = smith_G1(alpha, s.mo) / (4.0 * s.mo);
  const V3 h1 = normalize(s.wo + wi);
  double p = g * ggx_D(alpha, dot(s.n, h1));
  if (s.mo > mi) {
    const V3 h2 = normalize(s.wo + (wi - 2.0 * mi * s.n));
    p += g * ggx_D(alpha, dot(s.n, h2));
  }
  return p;
}

// f mu_i = A + B c toward wi; returns false (and zeros) below the surface
bool eval_AB(const Shade& s, V3 wi, double* A, double* B) {
  const double mi = dot(s.n, wi);
  *A = *B = 0.0;
  if (!(mi > 0.0)) return false;
  const double ps = s.Ps > 0.0 ? spec_pdf(s, s.alpha, wi) : 0.0;
  *A = ((1.0 - s.metal) * s.Fd + s.metal * s.k5) * ps;
  *B = (1.0 - s.metal) * (1.0 - s.Fd) * mi / kPi + s.metal * (1.0 - s.k5) * ps;
  if (s.Fk > 0.0) {
    *A = s.Fk * spec_pdf(s, s.calpha, wi) + (1.0 - s.Fk) * *A;
    *B = (1.0 - s.Fk) * *B;
  }
  return true;
}

double bsdf_pdf(const Shade& s, V3 wi) {
  const double mi = dot(s.n, wi);
  if (!(mi > 0.0)) return 0.0;
  const double base = (s.Ps > 0.0 ? s.Ps * spec_pdf(s, s.alpha, wi) : 0.0) + (1.0 - s.Ps) * mi / kPi;
  return s.Fk > 0.0 ? s.Fk * spec_pdf(s, s.calpha, wi) + (1.0 - s.Fk) * base : base;
}

// A GGX visible normal for wo from (u1, u2) (Heitz 2018, "Sampling the GGX
// distribution of visible normals"), in the world frame of s.
V3 sample_vndf(const Shade& s, double alpha, double u1, double u2) {
  const double ox = dot(s.wo, s.t1), oy = dot(s.wo, s.t2), oz = s.mo;
  // stretch to the hemisphere configuration
  const V3 vh = normalize(V3{alpha * ox, alpha * oy, oz});
  const double l2 = vh.x * vh.x + vh.y * vh.y;
  const V3 T1 = l2 > 0.0 ? (1.0 / std::sqrt(l2)) * V3{-vh.y, vh.x, 0.0} : V3{1.0, 0.0, 0.0};
  const V3 T2 = cross(vh, T1);
  const double r = std::sqrt(u1), phi = 2.0 * kPi * u2;
  const double p1 = r * std::cos(phi);
  double p2 = r * std::sin(phi);
  const double sw = 0.5 * (1.0 + vh.z);
  p2 = (1.0 - sw) * std::sqrt(std::max(0.0, 1.0 - p1 * p1)) + sw * p2;
  const V3 nh = p1 * T1 + p2 * T2 + std::sqrt(std::max(0.0, 1.0 - p1 * p1 - p2 * p2)) * vh;
  // unstretch
  const V3 hl = normalize(V3{alpha * nh.x, alpha * nh.y, std::max(0.0, nh.z)});
  return hl.x * s.t1 + hl.y * s.t2 + hl.z * s.n;
}

// Lobes of the mixture: 0 the cosine lobe, 1 the base's specular lobe, 2 the coat.
enum { kLobeDiffuse = 0, kLobeSpec = 1, kLobeCoat = 2 };

// Direction of the bounce from the lobe word u0 and (u1, u2): the coat when
// u0 < F_k, the specular lobe when F_k <= u0 < Pn (each a reflection about a
// visible normal of its roughness, mirrored above the surface when below it),
// else the cosine lobe.  *ambiguous is set when u0 lies within 1e-6 of a
// threshold (FP32 may choose the neighbouring lobe).
V3 sample_bsdf(const Shade& s, double u0, double u1, double u2, int* lobe, bool* ambiguous) {
  *lobe = u0 < s.Fk ? kLobeCoat : (u0 < s.Pn ? kLobeSpec : kLobeDiffuse);
  if (ambiguous)
    *ambiguous = (s.Fk > 0.0 && std::fabs(u0 - s.Fk) < 1e-6) || (s.Pn > 0.0 && std::fabs(u0 - s.Pn) < 1e-6);
  if (*lobe != kLobeDiffuse) {
    const V3 h = sample_vndf(s, *lobe == kLobeCoat ? s.calpha : s.alpha, u1, u2);
    V3 wi = 2.0 * dot(s.wo, h) * h - s.wo;
    const double mi = dot(s.n, wi);
    if (mi < 0.0) wi = wi - 2.0 * mi * s.n;
    return wi;
  }
  const double rr = std::sqrt(u1), phi = 2.0 * kPi * u2;
  return (rr * std::cos(phi)) * s.t1 + (rr * std::sin(phi)) * s.t2 + std::sqrt(1.0 - u1) * s.n;
}

// A lobe word inside lobe l's interval, or -1 when l has probability 0.
double lobe_word(const Shade& s, int l) {
  if (l == kLobeCoat) return s.Fk > 0.0 ? 0.0 : -1.0;
  if (l == kLobeSpec) return s.Pn > s.Fk ? 0.5 * (s.Fk + s.Pn) : -1.0;
  return s.Pn < 1.0 ? 1.0 : -1.0;
}

// The material of a face (the Lambertian default without a table).
Material face_material(const Scene& S, int64_t face) {
  if (S.mats.empty()) return Material{{1.0, 1.0, 1.0}, 1.0, 0.0, 0.0};
  return S.mats[S.face_mat[face]];
}

// One sampled path, recorded vertex by vertex (for the image and both gradient forms).
struct Vertex {
  int64_t face;
  int64_t param;  // index of the shading parameter: the face, or its texel when the scene has textures
  double a;      // albedo (texel; an RGB texel's first channel) at the vertex
  C3 a3;         // per channel: the base color is the material's tint times a3
  C3 e, e1;      // next-event estimate at the vertex (visibility included) and its derivative in a
  C3 w, w1;      // weight f mu / pdf of the bounce leaving the vertex and its derivative in a (0: none)
  int32_t inst, prim, half;  // the hit
  double t;
  uint32_t flags, shadow_flags;
  int32_t shadow;  // -1 no shadow ray, 0 visible, 1 occluded
};
struct PathRec {
  int nv = 0;
  Vertex v[64];
  bool escaped = false;
  double L_esc = 0.0;  // radiance seen by the escaping ray (sky or environment map)
  uint32_t flags = 0;
  uint32_t esc_flags = 0;  // flags of the escaping ray (when the path escaped)
  int n_closest = 0, n_shadow = 0, n_incoherent = 0;
};

// Radiance of the environment toward direction d (Section 4.1 names the
// scene's textured environment light): an equirectangular map of env_w x env_h
// texels with u = (atan2(d_y, d_x) + pi) / (2 pi) along a row and
// v = acos(d_z) / pi down the rows (row 0 around +z), read at the nearest texel.
// Which texel a direction next to a texel boundary falls in depends on
// rounding: flag directions whose angular distance to a boundary, times
// sin(theta), is below 1e-5, and directions within 1e-3 of a pole.
double env_radiance(const Scene& S, V3 d, uint32_t* flags) {
  d = normalize(d);
  const double th = std::acos(std::min(1.0, std::max(-1.0, d.z)));
  const double st = std::sin(th);
  const double u = (std::atan2(d.y, d.x) + kPi) / (2.0 * kPi), v = th / kPi;
  const int W = S.env_w, H = S.env_h;
  const double gu = u * W, gv = v * H;
  const double du = std::fabs(gu - std::round(gu)) * (2.0 * kPi / W) * st;
  const double kv = std::round(gv);
  const double dv = (kv >= 1 && kv <= H - 1) ? std::fabs(gv - kv) * (kPi / H) * st : 1.0;
  if (du < 1e-5 || dv < 1e-5 || st < 1e-3) *flags |= F_SHADE;
  const int tx = std::min(std::max((int)std::floor(gu), 0), W - 1);
  const int ty = std::min(std::max((int)std::floor(gv), 0), H - 1);
  return S.env[(size_t)ty * W + tx];
}

// Importance sampling of the environment map (Section 4.1 names the scene's
// textured environment light; next-event estimation toward it).  Texel k = ty W
// + tx covers azimuths [-pi + 2 pi tx / W, -pi + 2 pi (tx + 1) / W) and polar
// angles [pi ty / H, pi (ty + 1) / H), a solid angle
// Omega_ty = (2 pi / W) (cos(pi ty / H) - cos(pi (ty + 1) / H)).  It is drawn
// with probability p_k proportional to L_k Omega_ty, quantised to 32 bits:
// T_k = floor(2^32 C_k / C_total), C the running sum of L Omega in texel order
// (FP64), p_k = (T_k - T_{k-1}) / 2^32, so the draw (the first k with a
// 32-bit word w < T_k) is an integer decision.  The direction is uniform in
// solid angle within the texel; its density is p_k / Omega_ty.
double env_omega(const Scene& S, int ty) {
  const double H = S.env_h;
  return (2.0 * kPi / S.env_w) * (std::cos(kPi * ty / H) - std::cos(kPi * (ty + 1) / H));
}

void env_table(Scene& S) {
  const int64_t n = (int64_t)S.env_w * S.env_h;
  S.env_T.assign(n, 0);
  double total = 0.0;
  for (int64_t k = 0; k < n; ++k) total += S.env[k] * env_omega(S, (int)(k / S.env_w));
  double cum = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    cum += S.env[k] * env_omega(S, (int)(k / S.env_w));
    S.env_T[k] = total > 0.0 ? (uint64_t)std::floor(std::ldexp(cum / total, 32)) : (uint64_t)((k + 1) * 4294967296.0 / n);
  }
  S.env_T[n - 1] = (uint64_t)1 << 32;
}

// probability of texel k
inline double env_p(const Scene& S, int64_t k) {
  return std::ldexp((double)(S.env_T[k] - (k > 0 ? S.env_T[k - 1] : 0)), -32);
}

// the texel a direction reads (nearest, as the escape lookup)
int64_t env_texel(const Scene& S, V3 d) {
  d = normalize(d);
  const double th = std::acos(std::min(1.0, std::max(-1.0, d.z)));
  const double u = (std::atan2(d.y, d.x) + kPi) / (2.0 * kPi), v = th / kPi;
  const int tx = std::min(std::max((int)std::floor(u * S.env_w), 0), S.env_w - 1);
  const int ty = std::min(std::max((int)std::floor(v * S.env_h), 0), S.env_h - 1);
  return (int64_t)ty * S.env_w + tx;
}

// density (per solid angle) of the environment sampling toward direction d
inline double env_pdf(const Scene& S, int64_t k) { return env_p(S, k) / env_omega(S, (int)(k / S.env_w)); }

// Power-heuristic weight of strategy a against b (Veach 1997).
inline double mis_power(double a, double b) { return a * a / (a * a + b * b); }

void trace_path(const Scene& S, const Params& P, const Cam& cam, int32_t view, int64_t pix, int32_t sample,
                int mode, PathRec& rec) {
  const uint32_t key[2] = {(uint32_t)(P.seed & 0xffffffffu), (uint32_t)(P.seed >> 32) ^ P.frame};
  const V3 L{P.light[0], P.light[1], P.light[2]};
  uint32_t w[4];
  uint32_t ctr[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0u};
  philox(ctr, key, w);
  const int64_t x = pix % cam.w, y = pix / cam.w;
  const double sx = (2.0 * ((double)x + unit(w[0])) / (double)cam.w - 1.0) * cam.tan_half * cam.aspect;
  const double sy = (1.0 - 2.0 * ((double)y + unit(w[1])) / (double)cam.h) * cam.tan_half;
  Ray ray{cam.eye, normalize(cam.f + sx * cam.r + sy * cam.u), 0.0, kInf};
  Excl ex;
  double r0 = 0.0;
  double pdf_bsdf = 0.0;  // BSDF density of the sample that produced the current ray (bounce >= 1)
  const bool env_light = P.env_nee && S.env_w > 0;
  const int nl = 1 + P.n_area + (env_light ? 1 : 0);
  for (int b = 0; b < P.depth; ++b) {
    TraceOut h = trace_one(S, ray, ex, r0, mode, false);
    rec.n_closest++;
    if (b >= 1) rec.n_incoherent++;
    rec.flags |= h.flags & ~(uint32_t)F_T_ILLCOND;
    if (h.best.inst < 0) {
      rec.escaped = true;
      rec.esc_flags = h.flags;
      rec.L_esc = S.env_w > 0 ? env_radiance(S, ray.d, &rec.esc_flags) : P.L_sky;
      // with next-event estimation toward the map, an escaping bounce ray is
      // the other strategy for the same light: weighted against it
      if (env_light && b >= 1) rec.L_esc *= mis_power(pdf_bsdf, env_pdf(S, env_texel(S, ray.d)) / nl);
      rec.flags |= rec.esc_flags & ~(uint32_t)F_T_ILLCOND;
      return;
    }
    V3 wq[4];
    const int32_t pr = S.iproto[h.best.inst];
    const bool is_cap = S.pkind[pr] != 0;
    const int64_t face = S.fo[pr] + (is_cap ? h.best.prim / kCapsPerCurve : h.best.prim);
    V3 n;
    if (is_cap) {
      // the capsule's outward normal at the hit, mapped by A^-T
      const Ray ro = obj_ray(S, h.best.inst, ray);
      const Cap& hc = S.caps[S.co[pr] + h.best.prim];
      n = normal_to_world(S, h.best.inst, S.pkind[pr] == 2 ? ribbon_normal(hc, ro.d) : cap_normal(hc, ro.o + h.best.t * ro.d));
    } else {
      quad_world(S, h.best.inst, S.qo[pr] + h.best.prim, wq);
      n = h.best.half == 0 ? cross(wq[1] - wq[0], wq[3] - wq[0]) : cross(wq[3] - wq[2], wq[1] - wq[2]);
    }
    n = normalize(n);
    const double nd = dot(n, ray.d);
    uint32_t vshade = 0;  // shading decisions of this vertex within rounding of a threshold
    if (std::fabs(nd) < 1e-3) vshade |= F_SHADE;
    if (is_cap && S.pkind[pr] == 1 && cap_normal_uncertainty(S, h.best.inst, S.caps[S.co[pr] + h.best.prim], ray, h.best.t,
                                         16.0 * std::ldexp(1.0, -24) * h.S / std::max(h.cos_abs, 1e-3)) > 1e-6)
      vshade |= F_SHADE;
    if (nd > 0) n = -1.0 * n;
    const V3 p = ray.o + h.best.t * ray.d;
    double a = S.albedo[face];
    C3 a3 = c3(a);
    int64_t param = face;
    uint32_t tex_flag = 0;
    if (S.tex_res > 0) {
      // the texel of (u, v): nearest, on a res x res grid over the quad.  Which
      // texel a hit near a texel edge lands on depends on rounding: flag hits
      // whose world distance to an inner texel edge is below 1e-5 S / |cos|
      // (the position error of an FP32 hit is about 1e-6 S, stretched by
      // 1 / |cos| across the face at grazing incidence)
      const int R = S.tex_res;
      const double lu = std::max(norm(wq[1] - wq[0]), norm(wq[2] - wq[3]));
      const double lv = std::max(norm(wq[3] - wq[0]), norm(wq[2] - wq[1]));
      const double gu = h.best.u * R, gv = h.best.v * R;
      const double tol = 1e-5 * h.S / std::max(std::fabs(nd), 1e-3);
      for (int k = 1; k < R; ++k)
        if (std::fabs(gu - k) * lu / R < tol || std::fabs(gv - k) * lv / R < tol) tex_flag = F_SHADE;
      rec.flags |= tex_flag;
      const int tx = std::min(std::max((int)std::floor(gu), 0), R - 1);
      const int ty = std::min(std::max((int)std::floor(gv), 0), R - 1);
      param = ((int64_t)face * R + ty) * R + tx;
      for (int ch = 0; ch < 3; ++ch) a3.v[ch] = S.tex[(size_t)param * S.tex_ch + (S.tex_ch == 3 ? ch : 0)];
      a = a3.v[0];
    }
    Vertex vx;
    vx.face = face;
    vx.param = param;
    vx.a = a;
    vx.a3 = a3;
    const Material M = face_material(S, face);
    const Shade sh = make_shade(M, n, -1.0 * normalize(ray.d), false);
    // next-event estimate e = X (A + B c) toward the light direction, X the
    // light's factor (nl, radiance, geometry, density, MIS weight)
    auto set_nee = [&](V3 wl_dir, double X) {
      double A, B;
      eval_AB(sh, wl_dir, &A, &B);
      for (int ch = 0; ch < 3; ++ch) {
        vx.e.v[ch] = X * (A + B * sh.tint.v[ch] * a3.v[ch]);
        vx.e1.v[ch] = X * B * sh.tint.v[ch];
      }
    };
    const double cl = dot(n, L);
    // next-event estimation (Section 4.1 names the scene's quad-shaped key
    // lights and its environment light): with area lights or a sampled
    // environment, one of the nl = 1 + n_area (+ 1) lights (0: the directional
    // light, last: the environment) is picked with equal probability from word
    // 0 of counter (pixel, sample, view, 2^31 + b), as an integer, and its
    // estimate is weighted by nl
    int j = 0;
    uint32_t wl[4] = {0u, 0u, 0u, 0u};
    if (nl > 1) {
      uint32_t ctr3[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0x80000000u | (uint32_t)b};
      philox(ctr3, key, wl);
      j = (int)(((uint64_t)(wl[0] >> 8) * (uint64_t)nl) >> 24);
    }
    if (j == 0 && std::fabs(cl) < 1e-6) vshade |= F_SHADE;
    // origin uncertainty of rays leaving p: the FP32 position error of this hit
    // plus the incoming ray's own origin uncertainty, both stretched along the
    // surface by the incidence angle
    const double r1 = (16.0 * std::ldexp(1.0, -24) * h.S + r0) / std::max(h.cos_abs, 1e-3);
    const Excl here{h.best.inst, h.best.prim, h.best.half};
    vx.inst = h.best.inst;
    vx.prim = h.best.prim;
    vx.half = h.best.half;
    vx.t = h.best.t;
    vx.flags = h.flags | tex_flag;
    vx.shadow = -1;
    vx.shadow_flags = 0;
    if (j == 0 && cl > 0) {
      Ray sr{p, L, 0.0, kInf};
      TraceOut o = trace_one(S, sr, here, r1, mode, true);
      rec.n_shadow++;
      rec.flags |= o.flags & ~(uint32_t)F_T_ILLCOND;
      vx.shadow = o.best.inst >= 0 ? 1 : 0;
      vx.shadow_flags = o.flags;
      if (o.best.inst < 0) set_nee(L, nl * P.E);
    } else if (env_light && j == nl - 1) {
      // the environment: texel k from word 1 (the first k with w1 < T_k), a
      // direction uniform in solid angle within it from words 2, 3; estimate
      // nl L_k cos_p w / (pi pdf), w the power-heuristic weight against the
      // cosine sample (density cos_p / pi)
      const int64_t nt = (int64_t)S.env_w * S.env_h;
      int64_t lo = 0, hi = nt - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((uint64_t)wl[1] < S.env_T[mid]) hi = mid;
        else lo = mid + 1;
      }
      const int tx = (int)(lo % S.env_w), ty = (int)(lo / S.env_w);
      const double phi = -kPi + 2.0 * kPi * (tx + unit(wl[2])) / S.env_w;
      const double z0 = std::cos(kPi * ty / S.env_h), z1 = std::cos(kPi * (ty + 1) / S.env_h);
      const double z = z0 - unit(wl[3]) * (z0 - z1);
      const double sr_ = std::sqrt(std::max(0.0, 1.0 - z * z));
      const V3 de{sr_ * std::cos(phi), sr_ * std::sin(phi), z};
      const double cp = dot(n, de);
      if (std::fabs(cp) < 1e-6) vshade |= F_SHADE;
      if (cp > 0) {
        Ray sr{p, de, 0.0, kInf};
        TraceOut o = trace_one(S, sr, here, r1, mode, true);
        rec.n_shadow++;
        rec.flags |= o.flags & ~(uint32_t)F_T_ILLCOND;
        vx.shadow = o.best.inst >= 0 ? 1 : 0;
        vx.shadow_flags = o.flags;
        const double pdf = env_pdf(S, lo);
        if (o.best.inst < 0) set_nee(de, nl * S.env[lo] * mis_power(pdf / nl, bsdf_pdf(sh, de)) / pdf);
      }
    } else if (j > 0) {
      // area light j - 1: the parallelogram c + s e1 + t e2, (s, t) uniform from
      // words 1, 2, emitting Le from the side e1 x e2 faces.  Its estimate of
      // the irradiance is Le A cos_p cos_l / d^2 for the sampled point x at
      // distance d; the shadow ray runs from p to x (direction x - p, tmax 1)
      const double* Lq = P.area + 10 * (j - 1);
      const V3 c0{Lq[0], Lq[1], Lq[2]}, e1{Lq[3], Lq[4], Lq[5]}, e2{Lq[6], Lq[7], Lq[8]};
      const V3 x = c0 + unit(wl[1]) * e1 + unit(wl[2]) * e2;
      const V3 wi = x - p;
      const double d2 = dot(wi, wi), dd = std::sqrt(d2);
      const V3 nlv = cross(e1, e2);
      const double A = norm(nlv);
      const double cp = dd > 0 ? dot(n, wi) / dd : 0.0;
      const double cq = dd > 0 && A > 0 ? -dot(nlv, wi) / (A * dd) : 0.0;
      if (std::fabs(cp) < 1e-6 || std::fabs(cq) < 1e-6 || dd < 1e-6 * h.S) vshade |= F_SHADE;
      if (cp > 0 && cq > 0) {
        Ray sr{p, wi, 0.0, 1.0};
        TraceOut o = trace_one(S, sr, here, r1, mode, true);
        rec.n_shadow++;
        rec.flags |= o.flags & ~(uint32_t)F_T_ILLCOND;
        vx.shadow = o.best.inst >= 0 ? 1 : 0;
        vx.shadow_flags = o.flags;
        if (o.best.inst < 0) set_nee((1.0 / dd) * wi, nl * Lq[9] * A * cq / d2);
      }
    }
    vx.flags |= vshade;
    rec.flags |= vshade;
    rec.v[rec.nv++] = vx;
    if (b == P.depth - 1) return;
    uint32_t ctr2[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, (uint32_t)b};
    philox(ctr2, key, w);
    const double u1 = unit(w[2]), u2 = unit(w[3]);
    if (std::fabs(n.z) < 1e-6) {
      rec.flags |= F_SHADE;
      rec.v[rec.nv - 1].flags |= F_SHADE;
    }
    // the lobe: word 0 of counter (pixel, sample, view, 2^30 + b), drawn only
    // when a specular or coat lobe has weight
    double u0 = 1.0;
    if (sh.Pn > 0.0) {
      uint32_t ctr4[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0x40000000u | (uint32_t)b};
      uint32_t wlob[4];
      philox(ctr4, key, wlob);
      u0 = unit(wlob[0]);
    }
    int lobe = 0;
    bool amb = false;
    const V3 dnew = sample_bsdf(sh, u0, u1, u2, &lobe, &amb);
    if (amb) {
      rec.flags |= F_SHADE;
      rec.v[rec.nv - 1].flags |= F_SHADE;
    }
    double A, B;
    if (!eval_AB(sh, dnew, &A, &B)) return;  // a direction on the surface (measure zero): the path ends
    pdf_bsdf = bsdf_pdf(sh, dnew);
    for (int ch = 0; ch < 3; ++ch) {
      rec.v[rec.nv - 1].w.v[ch] = (A + B * sh.tint.v[ch] * a3.v[ch]) / pdf_bsdf;
      rec.v[rec.nv - 1].w1.v[ch] = B * sh.tint.v[ch] / pdf_bsdf;
    }
    ray = Ray{p, dnew, 0.0, kInf};
    ex = here;
    r0 = r1;
  }
}

// Radiance of a recorded path, in the order the terms arise:
// L = sum_k T_k e_k (+ T_n L_esc), T_0 = 1, T_{k+1} = T_k w_k.
C3 path_value(const Params& P, const PathRec& rec) {
  (void)P;
  C3 L, T = c3(1.0);
  for (int k = 0; k < rec.nv; ++k) {
    L = L + T * rec.v[k].e;
    T = T * rec.v[k].w;
  }
  if (rec.escaped) L = L + rec.L_esc * T;
  return L;
}

// ---------------------------------------------------------------- path replay check
// A GPU path recorded vertex by vertex (the ray that found each vertex, the
// hit, the shadow-ray outcome, the shading value) is checked step by step
// along its own rays, so that no check depends on an earlier rounding choice:
//  * each recorded hit (or escape) is an acceptable answer for the recorded FP32
//    ray with the previous triangle excluded, and its t lies within tolerance;
//  * the next ray starts at the FP32 hit point o + t d, formed as the renderer
//    forms it (one rounding per operation), and points along the cosine sample
//    of the same random words about the exact normal of the hit triangle;
//  * shading decisions (normal side, whether a shadow ray is cast, texel,
//    environment texel) equal the exact ones unless they lie within rounding of
//    a threshold, where either side is accepted and the GPU's side is followed;
//  * each shadow outcome is acceptable for the shadow ray from the FP32 point;
//  * the path's radiance, re-evaluated in FP64 along these decisions, matches
//    the GPU's value to 1e-4 relative.
struct PathCheck {
  int code = 0;     // 0 valid; otherwise the first failed check (see orc_check_path)
  int vertex = -1;  // the vertex (or ray) where it failed
  double L = 0.0;   // FP64 radiance along the GPU's decisions (channel 0)
  double Lc[3] = {0.0, 0.0, 0.0};  // all three channels
  int n_vert = 0, n_certain = 0, n_waived = 0, n_ambiguous_shading = 0;  // n_waived: t ill-conditioned
  double max_ulps = 0.0;  // largest t error in units of 2^-24 S / (|d| |cos|)
};

inline float f32(double x) { return (float)x; }

// Environment texels a direction may read: the exact one, and its neighbours
// across a texel boundary within rounding (angular distance times sin(theta)
// below 1e-5) or near a pole (within 1e-3).
int env_candidates(const Scene& S, V3 d, double out[9], int64_t idx[9]) {
  d = normalize(d);
  const double th = std::acos(std::min(1.0, std::max(-1.0, d.z)));
  const double st = std::sin(th);
  const double u = (std::atan2(d.y, d.x) + kPi) / (2.0 * kPi), v = th / kPi;
  const int W = S.env_w, H = S.env_h;
  const double gu = u * W, gv = v * H;
  const int tx = std::min(std::max((int)std::floor(gu), 0), W - 1);
  const int ty = std::min(std::max((int)std::floor(gv), 0), H - 1);
  const double du = std::fabs(gu - std::round(gu)) * (2.0 * kPi / W) * st;
  const double dv = std::fabs(gv - std::round(gv)) * (kPi / H) * st;
  const bool pole = st < 1e-3;
  int xs[3] = {tx, tx, tx}, ys[3] = {ty, ty, ty};
  int nx = 1, ny = 1;
  if (du < 1e-5 || pole) {
    xs[nx++] = std::max(tx - 1, 0);
    xs[nx++] = std::min(tx + 1, W - 1);
  }
  if (dv < 1e-5 || pole) {
    ys[ny++] = std::max(ty - 1, 0);
    ys[ny++] = std::min(ty + 1, H - 1);
  }
  int n = 0;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b) {
      idx[n] = (int64_t)ys[b] * W + xs[a];
      out[n] = S.env[idx[n]];
      ++n;
    }
  return n;
}

// vi: 6 words per recorded ray (instance, primitive, half, shadow -1/0/1, face, 0);
// vf: 10 floats per recorded ray (t, shading value, cosine to the light,
// radiance so far, origin xyz, direction xyz).  Rays 0 .. nv-1 found vertices;
// when the path escaped, ray nv is the escaping ray (its words are ignored but
// origin and direction).
PathCheck check_path(const Scene& S, const Params& P, const Cam& cam, int32_t view, int64_t pix, int32_t sample,
                     int nv, const int32_t* vi, const float* vf, bool escaped, const float* radiance, int mode) {
  PathCheck R;
  auto fail = [&](int code, int k) {
    if (R.code == 0) {
      R.code = code;
      R.vertex = k;
    }
    return R;
  };
  const uint32_t key[2] = {(uint32_t)(P.seed & 0xffffffffu), (uint32_t)(P.seed >> 32) ^ P.frame};
  // the light direction as the device holds it (rounded to FP32)
  const V3 Lf{(double)f32(P.light[0]), (double)f32(P.light[1]), (double)f32(P.light[2])};
  const V3 L{P.light[0], P.light[1], P.light[2]};
  if (nv < 0 || nv > P.depth || (!escaped && nv != P.depth)) return fail(11, nv);
  auto ray_of = [&](int k) {
    const float* f = vf + 10 * k;
    return Ray{{(double)f[4], (double)f[5], (double)f[6]}, {(double)f[7], (double)f[8], (double)f[9]}, 0.0, kInf};
  };
  // camera ray: eye exactly, direction within FP32 rounding of the FP64 one
  {
    uint32_t w[4];
    uint32_t ctr[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0u};
    philox(ctr, key, w);
    const int64_t x = pix % cam.w, y = pix / cam.w;
    const double sx = (2.0 * ((double)x + unit(w[0])) / (double)cam.w - 1.0) * cam.tan_half * cam.aspect;
    const double sy = (1.0 - 2.0 * ((double)y + unit(w[1])) / (double)cam.h) * cam.tan_half;
    const V3 d = normalize(cam.f + sx * cam.r + sy * cam.u);
    const Ray r0 = ray_of(0);
    if (r0.o.x != (double)f32(cam.eye.x) || r0.o.y != (double)f32(cam.eye.y) || r0.o.z != (double)f32(cam.eye.z))
      return fail(1, 0);
    if (norm(r0.d - d) > 1e-5) return fail(1, 0);
  }
  Excl ex;
  C3 T = c3(1.0);
  C3 Lsum;
  // error budget of the radiance from capsule normals known only to their FP32
  // uncertainty: absolute per channel (Bsum), and the relative uncertainty of
  // the path weight T so far (rho)
  C3 Bsum;
  double rho = 0.0;
  bool unbounded = false;  // a capsule normal's uncertainty reaches a weight's support: no bound
  double pdf_bsdf = 0.0;  // BSDF density of the sample behind the current ray
  const bool env_light = P.env_nee && S.env_w > 0;
  const int nl = 1 + P.n_area + (env_light ? 1 : 0);
  std::vector<double> esc_vals;
  for (int k = 0; k <= nv; ++k) {
    if (k == nv && !escaped) break;
    const Ray ray = ray_of(k);
    const AcceptSet A = accept_set(S, ray, ex, 0.0, mode);
    if (k == nv) {
      // the escaping ray: a miss must be acceptable
      int info = 0;
      if (judge_closest(A, -1, -1, -1, kInf, &info)) return fail(3, k);
      if (S.env_w > 0) {
        double c[9];
        int64_t kk[9];
        const int n = env_candidates(S, ray.d, c, kk);
        for (int j = 0; j < n; ++j) {
          // with next-event estimation toward the map, an escaping bounce ray
          // is weighted against it (as the path loop does)
          const double w = env_light && k >= 1 ? mis_power(pdf_bsdf, env_pdf(S, kk[j]) / nl) : 1.0;
          esc_vals.push_back(c[j] * w);
        }
      } else {
        esc_vals.push_back(P.L_sky);
      }
      break;
    }
    const int32_t* I = vi + 6 * k;
    const float* F = vf + 10 * k;
    const int32_t inst = I[0], prim = I[1], half = I[2], shadow = I[3];
    if (inst < 0 || inst >= S.N || prim < 0 || half < 0 || half > 1) return fail(2, k);
    const int32_t pr = S.iproto[inst];
    const bool is_cap = S.pkind[pr] != 0;
    if (prim >= (is_cap ? S.co[pr + 1] - S.co[pr] : S.qo[pr + 1] - S.qo[pr]) || (is_cap && half != 0))
      return fail(2, k);
    int info = 0;
    double ulps = 0.0;
    const int jc = judge_closest(A, inst, prim, half, (double)F[0], &info, &ulps);
    R.max_ulps = std::max(R.max_ulps, ulps);
    if (jc == 1) return fail(2, k);
    if (jc == 3) return fail(4, k);
    R.n_vert++;
    if (info & 1) R.n_certain++;
    if (info & 2) R.n_waived++;
    const int64_t face = S.fo[pr] + (is_cap ? prim / kCapsPerCurve : prim);
    if (I[4] != (int32_t)face) return fail(5, k);
    V3 wq[4];
    V3 n;
    if (is_cap) {
      // the capsule's outward normal at the GPU's t along the recorded ray
      const Ray ro = obj_ray(S, inst, ray);
      const Cap& hc = S.caps[S.co[pr] + prim];
      n = normal_to_world(S, inst, S.pkind[pr] == 2 ? ribbon_normal(hc, ro.d) : cap_normal(hc, ro.o + (double)F[0] * ro.d));
    } else {
      quad_world(S, inst, S.qo[pr] + prim, wq);
      n = half == 0 ? cross(wq[1] - wq[0], wq[3] - wq[0]) : cross(wq[3] - wq[2], wq[1] - wq[2]);
    }
    n = normalize(n);
    const V3 dh = normalize(ray.d);
    const double nd = dot(n, dh);
    // the FP32 hit point, formed as the renderer forms it
    const float t32 = F[0];
    const V3 pg{(double)f32((double)F[4] + (double)f32((double)t32 * (double)F[7])),
                (double)f32((double)F[5] + (double)f32((double)t32 * (double)F[8])),
                (double)f32((double)F[6] + (double)f32((double)t32 * (double)F[9]))};
    const bool has_next = k + 1 < nv || (escaped && k + 1 == nv);
    // which side the normal faces: toward the incoming ray, unless the ray
    // grazes the surface; then the GPU's choice shows in its next direction or
    // in the sign of its cosine to the light
    double side = nd > 0 ? -1.0 : 1.0;
    if (std::fabs(nd) < 1e-3) {
      R.n_ambiguous_shading++;
      if (has_next) {
        const Ray nr = ray_of(k + 1);
        side = dot(n, nr.d) >= 0 ? 1.0 : -1.0;
      } else if (std::fabs((double)F[2]) > 1e-6) {
        side = ((double)F[2] * dot(n, L) >= 0) ? 1.0 : -1.0;
      }
    }
    n = side * n;
    // a capsule's normal follows the hit point: the GPU's is known to within
    // dn_unc of the exact normal at its t
    const double dn_unc = is_cap && S.pkind[pr] == 1
                              ? cap_normal_uncertainty(S, inst, S.caps[S.co[pr] + prim], ray, (double)F[0], 0.0)
                              : 0.0;
    // shading value: the face's albedo, or a texel at the hit's (u, v) (the
    // recorded value is an RGB texel's first channel)
    double a = S.albedo[face];
    C3 a3 = c3(a);
    if (S.tex_res > 0) {
      // barycentric (u, v) of the plane point along the recorded ray
      const V3 w0 = half == 0 ? wq[0] : wq[2], w1 = half == 0 ? wq[1] : wq[3], w2 = half == 0 ? wq[3] : wq[1];
      const V3 nt = cross(w1 - w0, w2 - w0);
      const double tt = dot(nt, w0 - ray.o) / dot(nt, ray.d);
      const V3 p = ray.o + tt * ray.d;
      const double nn = dot(nt, nt);
      const double l1 = dot(cross(w0 - w2, p - w2), nt) / nn, l2 = dot(cross(w1 - w0, p - w0), nt) / nn;
      const double u = half == 0 ? l1 : 1.0 - l1, v = half == 0 ? l2 : 1.0 - l2;
      const int Rr = S.tex_res;
      const double lu = std::max(norm(wq[1] - wq[0]), norm(wq[2] - wq[3]));
      const double lv = std::max(norm(wq[3] - wq[0]), norm(wq[2] - wq[1]));
      double Sq = std::max(1.0, std::max(maxabs(ray.o), maxabs(p)));
      for (int q = 0; q < 4; ++q) Sq = std::max(Sq, maxabs(wq[q] - ray.o));
      const double tol = 1e-5 * Sq / std::max(std::fabs(nd), 1e-3);
      const int tx = std::min(std::max((int)std::floor(u * Rr), 0), Rr - 1);
      const int ty = std::min(std::max((int)std::floor(v * Rr), 0), Rr - 1);
      bool found = false;
      for (int dx = -1; dx <= 1 && !found; ++dx)
        for (int dy = -1; dy <= 1 && !found; ++dy) {
          const int x2 = tx + dx, y2 = ty + dy;
          if (x2 < 0 || y2 < 0 || x2 >= Rr || y2 >= Rr) continue;
          // a neighbour is acceptable only across an edge within rounding
          if (dx != 0 && std::fabs(u * Rr - (dx > 0 ? tx + 1 : tx)) * lu / Rr >= tol) continue;
          if (dy != 0 && std::fabs(v * Rr - (dy > 0 ? ty + 1 : ty)) * lv / Rr >= tol) continue;
          const size_t ti = ((size_t)face * Rr + y2) * Rr + x2;
          const double val = S.tex[ti * S.tex_ch];
          if (f32(val) == F[1]) {
            for (int ch = 0; ch < 3; ++ch) a3.v[ch] = S.tex[ti * S.tex_ch + (S.tex_ch == 3 ? ch : 0)];
            a = val;
            found = true;
          }
        }
      if (!found) return fail(6, k);
    } else if (f32(a) != F[1]) {
      return fail(6, k);
    }
    const Material M = face_material(S, face);
    const Shade sh = make_shade(M, n, -1.0 * dh, false);
    // the shade with the normal turned by dn_unc about tangent axis q & 1, in
    // direction q & 2 (q = 0..3): the spread of every value that depends on
    // the normal over these four bounds its change to first order
    auto turned_shade = [&](int q) {
      const V3 tq = (q & 1) ? sh.t2 : sh.t1;
      return make_shade(M, normalize(n + (((q & 2) ? -1.0 : 1.0) * dn_unc) * tq), -1.0 * dh, false);
    };
    // next-event estimate
    int j = 0;
    uint32_t wl[4] = {0u, 0u, 0u, 0u};
    if (nl > 1) {
      uint32_t ctr3[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0x80000000u | (uint32_t)k};
      philox(ctr3, key, wl);
      j = (int)(((uint64_t)(wl[0] >> 8) * (uint64_t)nl) >> 24);
    }
    const Excl here{inst, prim, half};
    bool want_certain = false, skip_certain = false;
    Ray sr{pg, Lf, 0.0, kInf};
    V3 ldir = L;     // unit direction of the light sample
    double X = 0.0;  // the light's factor of the estimate X (A + B c)
    double env_L = 0.0, env_p = 0.0;  // an environment sample's radiance and density (its X depends on the BSDF)
    const double cth = 1e-6 + dn_unc;  // cosine thresholds of the light tests
    if (j == 0) {
      const double cl = dot(n, L);
      want_certain = cl > cth;
      skip_certain = cl < -cth;
      X = nl * P.E;
    } else if (env_light && j == nl - 1) {
      const int64_t nt = (int64_t)S.env_w * S.env_h;
      int64_t lo = 0, hi = nt - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((uint64_t)wl[1] < S.env_T[mid]) hi = mid;
        else lo = mid + 1;
      }
      const int tx = (int)(lo % S.env_w), ty = (int)(lo / S.env_w);
      const double phi = -kPi + 2.0 * kPi * (tx + unit(wl[2])) / S.env_w;
      const double z0 = std::cos(kPi * ty / S.env_h), z1 = std::cos(kPi * (ty + 1) / S.env_h);
      const double z = z0 - unit(wl[3]) * (z0 - z1);
      const double sr_ = std::sqrt(std::max(0.0, 1.0 - z * z));
      const V3 de{sr_ * std::cos(phi), sr_ * std::sin(phi), z};
      const double cp = dot(n, de);
      want_certain = cp > cth;
      skip_certain = cp < -cth;
      const double pdf = env_pdf(S, lo);
      X = nl * S.env[lo] * mis_power(pdf / nl, bsdf_pdf(sh, de)) / pdf;
      env_L = S.env[lo];
      env_p = pdf;
      ldir = de;
      sr = Ray{pg, de, 0.0, kInf};
    } else {
      const double* Lq = P.area + 10 * (j - 1);
      const V3 c0{Lq[0], Lq[1], Lq[2]}, e1{Lq[3], Lq[4], Lq[5]}, e2{Lq[6], Lq[7], Lq[8]};
      const V3 x = c0 + unit(wl[1]) * e1 + unit(wl[2]) * e2;
      const V3 wi = x - pg;
      const double d2 = dot(wi, wi), dd = std::sqrt(d2);
      const V3 nlv = cross(e1, e2);
      const double Ar = norm(nlv);
      const double cp = dot(n, wi) / dd, cq = -dot(nlv, wi) / (Ar * dd);
      want_certain = cp > cth && cq > 1e-6;
      skip_certain = cp < -cth || cq < -1e-6;
      X = nl * Lq[9] * Ar * cq / d2;
      ldir = (1.0 / dd) * wi;
      sr = Ray{pg, wi, 0.0, 1.0};
    }
    if (!want_certain && !skip_certain) R.n_ambiguous_shading++;
    if (shadow < 0 && want_certain) return fail(7, k);
    if (shadow >= 0 && skip_certain) return fail(7, k);
    if (shadow >= 0) {
      const AcceptSet As = accept_set(S, sr, here, 0.0, mode);
      if (judge_any(As, shadow == 1)) return fail(8, k);
      if (shadow == 0) {
        double fa, fb;
        eval_AB(sh, ldir, &fa, &fb);
        C3 e;
        for (int ch = 0; ch < 3; ++ch) e.v[ch] = X * (fa + fb * sh.tint.v[ch] * a3.v[ch]);
        Lsum = Lsum + T * e;
        for (int ch = 0; ch < 3; ++ch) Bsum.v[ch] += std::fabs(T.v[ch] * e.v[ch]) * rho;
        if (dn_unc > 0.0) {
          for (int q = 0; q < 4; ++q) {
            const Shade sq = turned_shade(q);
            const double Xq = env_p > 0.0 ? nl * env_L * mis_power(env_p / nl, bsdf_pdf(sq, ldir)) / env_p : X;
            double qa, qb;
            eval_AB(sq, ldir, &qa, &qb);
            for (int ch = 0; ch < 3; ++ch)
              Bsum.v[ch] += 0.5 * std::fabs(T.v[ch]) * std::fabs(Xq * (qa + qb * sq.tint.v[ch] * a3.v[ch]) - e.v[ch]);
          }
        }
      }
    }
    if (!has_next) break;
    // the next ray: from the FP32 hit point along the cosine sample
    const Ray nr = ray_of(k + 1);
    if (nr.o.x != pg.x || nr.o.y != pg.y || nr.o.z != pg.z) return fail(9, k + 1);
    uint32_t w2[4];
    uint32_t ctr2[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, (uint32_t)k};
    philox(ctr2, key, w2);
    double u0 = 1.0;
    if (sh.Pn > 0.0) {
      uint32_t ctr4[4] = {(uint32_t)pix, (uint32_t)sample, (uint32_t)view, 0x40000000u | (uint32_t)k};
      uint32_t wlob[4];
      philox(ctr4, key, wlob);
      u0 = unit(wlob[0]);
    }
    // the sampled direction, for every lobe when the lobe word lies within
    // rounding of a threshold, and for either basis branch when n_z ~ 0
    int lobe;
    bool amb;
    double err = norm(nr.d - sample_bsdf(sh, u0, unit(w2[2]), unit(w2[3]), &lobe, &amb));
    if (dn_unc > 0.0 && sh.Pn > 0.0) {
      // the lobe thresholds F_k and Pn are uncertain within their spread as well
      double dfk = 0.0, dpn = 0.0;
      for (int q = 0; q < 4; ++q) {
        const Shade sq = turned_shade(q);
        dfk = std::max(dfk, std::fabs(sq.Fk - sh.Fk));
        dpn = std::max(dpn, std::fabs(sq.Pn - sh.Pn));
      }
      amb = amb || (sh.Fk > 0.0 && std::fabs(u0 - sh.Fk) < 1e-6 + 2.0 * dfk) ||
            std::fabs(u0 - sh.Pn) < 1e-6 + 2.0 * dpn;
    }
    if (amb) {
      R.n_ambiguous_shading++;
      for (int l = 0; l < 3; ++l) {
        const double ul = lobe_word(sh, l);
        int ll;
        if (l != lobe && ul >= 0.0)
          err = std::min(err, norm(nr.d - sample_bsdf(sh, ul, unit(w2[2]), unit(w2[3]), &ll, nullptr)));
      }
    }
    if (std::fabs(n.z) < 1e-6) {
      R.n_ambiguous_shading++;
      const Shade sf = make_shade(M, n, -1.0 * dh, true);
      err = std::min(err, norm(nr.d - sample_bsdf(sf, u0, unit(w2[2]), unit(w2[3]), &lobe, nullptr)));
    }
    // a direction sampled about a normal turned by dn_unc turns by up to about
    // twice that (the specular lobe reflects about the microfacet normal)
    if (err > 1e-5 + 4.0 * dn_unc) return fail(10, k + 1);
    // the weight of the GPU's direction, in FP64
    const V3 dn = normalize(nr.d);
    double fa, fb;
    if (!eval_AB(sh, dn, &fa, &fb)) {
      // below the surface for the exact normal: acceptable only within the
      // normal's uncertainty, and the rest of the path then carries no bound
      if (!(dn_unc > 0.0) || dot(n, dn) < -2.0 * dn_unc) return fail(10, k + 1);
      unbounded = true;
    }
    pdf_bsdf = bsdf_pdf(sh, dn);
    C3 wgt;
    for (int ch = 0; ch < 3; ++ch) wgt.v[ch] = pdf_bsdf > 0.0 ? (fa + fb * sh.tint.v[ch] * a3.v[ch]) / pdf_bsdf : 0.0;
    if (dn_unc > 0.0 && !unbounded) {
      // relative spread of the weight and of the density (the environment's
      // MIS weight at an escape reads it) over the turned normals
      double dr = 0.0;
      for (int q = 0; q < 4; ++q) {
        const Shade sq = turned_shade(q);
        double qa, qb;
        const double pq = bsdf_pdf(sq, dn);
        if (!eval_AB(sq, dn, &qa, &qb) || !(pq > 0.0) || !(pdf_bsdf > 0.0)) {
          dr = kInf;
          break;
        }
        dr = std::max(dr, std::fabs(pq / pdf_bsdf - 1.0));
        for (int ch = 0; ch < 3; ++ch) {
          const double wq = (qa + qb * sq.tint.v[ch] * a3.v[ch]) / pq;
          if (wgt.v[ch] != 0.0) dr = std::max(dr, std::fabs(wq / wgt.v[ch] - 1.0));
        }
      }
      if (std::isfinite(dr)) rho += 2.0 * dr;
      else unbounded = true;
    }
    T = T * wgt;
    ex = here;
  }
  // radiance: the FP64 value along these decisions, for each environment
  // texel the escaping ray may read
  if (esc_vals.empty()) esc_vals.push_back(0.0);
  double best = kInf, Lbest = 0.0, scale = 0.0;
  C3 Lb;
  double budget = 0.0;  // of the chosen value, from uncertain capsule normals
  for (double e : esc_vals) {
    const C3 Lv = escaped ? Lsum + e * T : Lsum;
    double err = 0.0, mx = 0.0, bud = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      err = std::max(err, std::fabs((double)radiance[ch] - Lv.v[ch]));
      mx = std::max(mx, std::fabs(Lv.v[ch]));
      bud = std::max(bud, Bsum.v[ch] + (escaped ? std::fabs(e * T.v[ch]) * rho : 0.0));
    }
    if (err - bud < best - budget || best == kInf) {
      best = err;
      budget = bud;
      Lb = Lv;
      scale = mx;
    }
  }
  for (int ch = 0; ch < 3; ++ch) R.Lc[ch] = Lb.v[ch];
  R.L = Lb.v[0];
  (void)Lbest;
  // every channel within 1e-4 of the largest one (plus the budget of capsule normals)
  if (!unbounded && !(best <= 1e-4 * scale + 1e-7 + budget)) return fail(12, nv);
  return R;
}

template <class Fn>
void parallel_for(int64_t n, int nthreads, Fn&& fn) {
  if (nthreads <= 1 || n < 2) {
    for (int64_t i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  const int64_t chunk = 64;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t] {
      for (;;) {
        const int64_t s = next.fetch_add(chunk);
        if (s >= n) break;
        const int64_t e = std::min(n, s + chunk);
        for (int64_t i = s; i < e; ++i) fn(i, t);
      }
    });
  for (auto& x : th) x.join();
}

int g_threads = 0;
int threads() {
  if (g_threads > 0) return g_threads;
  const unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

// Packed image index g -> camera entry, pixel of the whole view (row-major).
void resolve_pixel(const std::vector<Cam>& cams, int64_t g, int32_t* cam, int64_t* pix) {
  for (size_t c = 0; c < cams.size(); ++c)
    if (g >= cams[c].off && g < cams[c].off + cams[c].tw * cams[c].th) {
      const int64_t local = g - cams[c].off;
      *cam = (int32_t)c;
      *pix = (cams[c].ty + local / cams[c].tw) * cams[c].w + cams[c].tx + local % cams[c].tw;
      return;
    }
  *cam = -1;
  *pix = -1;
}

// A material from its 8 parameters (tint r, g, b, roughness, metallic,
// specular, clearcoat, clearcoat roughness).
Material material_of(const double* m) { return Material{{m[0], m[1], m[2]}, m[3] * m[3], m[4], m[5], m[6], m[7] * m[7]}; }

}  // namespace

// =============================================================== C ABI
extern "C" {

void orc_set_threads(int n) { g_threads = n; }
int orc_get_threads() { return threads(); }

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

// A prototype holds quads or, when proto_curve_off gives it curves, only
// curves: 16 floats each (4 control points x, y, z, radius), tessellated into
// capsules here.  albedo: one per face (quad or curve) in prototype order.
void* orc_scene_create(const float* verts, int64_t n_verts, const int32_t* quads, int64_t n_quads,
                       const int64_t* proto_vert_off, const int64_t* proto_quad_off, int32_t n_protos,
                       const float* albedo, const int32_t* inst_proto, const float* inst_xform, int64_t n_inst,
                       const float* curves, const int64_t* proto_curve_off, const int32_t* proto_curve_flat) {
  Scene* S = new Scene;
  S->P = n_protos;
  S->verts.resize(n_verts);
  for (int64_t i = 0; i < n_verts; ++i) S->verts[i] = {verts[3 * i], verts[3 * i + 1], verts[3 * i + 2]};
  S->quads.assign(quads, quads + 4 * n_quads);
  S->vo.assign(proto_vert_off, proto_vert_off + n_protos + 1);
  S->qo.assign(proto_quad_off, proto_quad_off + n_protos + 1);
  S->pkind.assign(n_protos, 0);
  S->co.assign(n_protos + 1, 0);
  S->fo.assign(n_protos + 1, 0);
  for (int32_t p = 0; p < n_protos; ++p) {
    const int64_t nc = proto_curve_off ? proto_curve_off[p + 1] - proto_curve_off[p] : 0;
    if (nc > 0) {
      const bool flat = proto_curve_flat && proto_curve_flat[p] != 0;
      S->pkind[p] = flat ? 2 : 1;
      for (int64_t k = proto_curve_off[p]; k < proto_curve_off[p + 1]; ++k) {
        Cap cc[kCapsPerCurve];
        tessellate_curve(curves + 16 * k, cc, flat);
        for (int j = 0; j < kCapsPerCurve; ++j) S->caps.push_back(cc[j]);
      }
    }
    S->co[p + 1] = (int64_t)S->caps.size();
    S->fo[p + 1] = S->fo[p] + (nc > 0 ? nc : S->qo[p + 1] - S->qo[p]);
  }
  const int64_t n_faces = S->fo[n_protos];
  S->albedo.resize(n_faces);
  for (int64_t i = 0; i < n_faces; ++i) S->albedo[i] = albedo ? (double)albedo[i] : 0.5;
  S->N = n_inst;
  S->iproto.assign(inst_proto, inst_proto + n_inst);
  S->X.resize(12 * n_inst);
  S->Xi.resize(12 * n_inst);
  S->ainv_frob.resize(n_inst);
  for (int64_t i = 0; i < 12 * n_inst; ++i) S->X[i] = inst_xform[i];
  for (int64_t i = 0; i < n_inst; ++i) {
    if (!invert_affine(&S->X[12 * i], &S->Xi[12 * i])) {
      delete S;
      return nullptr;
    }
    double f = 0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) f += S->Xi[12 * i + 4 * r + c] * S->Xi[12 * i + 4 * r + c];
    S->ainv_frob[i] = std::sqrt(f);
  }
  // per-prototype object-space BVHs over quads (built in parallel over prototypes)
  S->proto_box.resize(n_protos);
  S->proto_bvh.resize(n_protos);
  parallel_for(n_protos, threads(), [&](int64_t p, int) {
    Box all;
    if (S->pkind[p]) {
      // capsule boxes: the segment's box grown by the radius
      std::vector<Box> cb(S->co[p + 1] - S->co[p]);
      for (int64_t c = S->co[p]; c < S->co[p + 1]; ++c) {
        const Cap& k = S->caps[c];
        const double rr = std::max(k.r, k.rb);
        Box b;
        b.grow(k.a - V3{rr, rr, rr});
        b.grow(k.a + V3{rr, rr, rr});
        b.grow(k.b - V3{rr, rr, rr});
        b.grow(k.b + V3{rr, rr, rr});
        cb[c - S->co[p]] = b;
        all.grow(b);
      }
      S->proto_box[p] = all;
      S->proto_bvh[p].build(cb);
      return;
    }
    std::vector<Box> qb(S->qo[p + 1] - S->qo[p]);
    for (int64_t q = S->qo[p]; q < S->qo[p + 1]; ++q) {
      Box b;
      for (int k = 0; k < 4; ++k) b.grow(S->verts[S->vo[p] + S->quads[4 * q + k]]);
      qb[q - S->qo[p]] = b;
      all.grow(b);
    }
    S->proto_box[p] = all;
    S->proto_bvh[p].build(qb);
  });
  // world boxes of instances: the 8 transformed corners of the prototype box
  S->inst_box.resize(n_inst);
  double mag = 1.0;
  for (int64_t i = 0; i < n_inst; ++i) {
    const Box& pb = S->proto_box[S->iproto[i]];
    Box wb;
    if (pb.lo[0] <= pb.hi[0])
      for (int c = 0; c < 8; ++c) {
        V3 v{(c & 1) ? pb.hi[0] : pb.lo[0], (c & 2) ? pb.hi[1] : pb.lo[1], (c & 4) ? pb.hi[2] : pb.lo[2]};
        wb.grow(xform_point(&S->X[12 * i], v));
      }
    S->inst_box[i] = wb;
    if (pb.lo[0] <= pb.hi[0]) mag = std::max(mag, wb.mag());
  }
  S->scene_mag = mag;
  S->inst_bvh.build(S->inst_box);
  return S;
}

void orc_scene_destroy(void* s) { delete static_cast<Scene*>(s); }

// The BSDF at one shading frame, for tests: material m (8 parameters), unit
// normal n, unit direction to the viewer wo.  For each of n directions wi
// (n x 3) writes (A, B, pdf, Pn): f mu_i = A + B c, the sampling density and the
// probability of a specular or coat lobe.
void orc_bsdf_eval(const double* m, const double* nrm, const double* wo, int64_t n, const double* wi, double* out) {
  const Material M = material_of(m);
  const Shade sh = make_shade(M, V3{nrm[0], nrm[1], nrm[2]}, V3{wo[0], wo[1], wo[2]}, false);
  for (int64_t i = 0; i < n; ++i) {
    const V3 w{wi[3 * i], wi[3 * i + 1], wi[3 * i + 2]};
    eval_AB(sh, w, &out[4 * i], &out[4 * i + 1]);
    out[4 * i + 2] = bsdf_pdf(sh, w);
    out[4 * i + 3] = sh.Pn;
  }
}

// Sampled bounce directions for (u0, u1, u2) triples (n x 3): writes the
// direction (n x 3) and, per sample, (lobe: 0 cosine, 1 specular, 2 coat; lobe
// word within rounding of a threshold).
void orc_bsdf_sample(const double* m, const double* nrm, const double* wo, int64_t n, const double* u, double* wi,
                     int32_t* info) {
  const Material M = material_of(m);
  const Shade sh = make_shade(M, V3{nrm[0], nrm[1], nrm[2]}, V3{wo[0], wo[1], wo[2]}, false);
  for (int64_t i = 0; i < n; ++i) {
    int lobe;
    bool amb;
    const V3 d = sample_bsdf(sh, u[3 * i], u[3 * i + 1], u[3 * i + 2], &lobe, &amb);
    wi[3 * i] = d.x;
    wi[3 * i + 1] = d.y;
    wi[3 * i + 2] = d.z;
    info[2 * i] = lobe;
    info[2 * i + 1] = amb ? 1 : 0;
  }
}

// The segments of every curve prototype, for tests: 8 doubles each (a, b,
// radius at a, radius at b; equal for round capsules), prototype order.
// Returns their count.
int64_t orc_scene_capsules(void* s, double* out) {
  const Scene& S = *static_cast<Scene*>(s);
  if (out)
    for (size_t k = 0; k < S.caps.size(); ++k) {
      const Cap& c = S.caps[k];
      const double v[8] = {c.a.x, c.a.y, c.a.z, c.b.x, c.b.y, c.b.z, c.r, c.rb};
      for (int j = 0; j < 8; ++j) out[8 * k + j] = v[j];
    }
  return (int64_t)S.caps.size();
}

// Principled materials (Section 5.4): n_mat entries of (tint r, g, b,
// roughness, metallic, specular) and one material index per unique quad; n_mat = 0
// removes them (every face Lambertian again).  Returns -1 on a bad argument.
int orc_scene_set_materials(void* s, const double* mats, int32_t n_mat, const int32_t* face_mat) {
  Scene* S = static_cast<Scene*>(s);
  if (n_mat < 0 || (n_mat > 0 && (!mats || !face_mat))) return -1;
  S->mats.clear();
  S->face_mat.clear();
  if (n_mat == 0) return 0;
  for (int32_t k = 0; k < n_mat; ++k) S->mats.push_back(material_of(mats + 8 * k));
  S->face_mat.assign(face_mat, face_mat + S->albedo.size());
  for (int32_t f : S->face_mat)
    if (f < 0 || f >= n_mat) return -1;
  return 0;
}

int orc_scene_set_albedo(void* s, const double* albedo) {
  Scene* S = static_cast<Scene*>(s);
  for (size_t i = 0; i < S->albedo.size(); ++i) S->albedo[i] = albedo[i];
  return 0;
}

// Per-face textures (Section 5.3: a Ptex lookup at the hit's face and (u, v)),
// here synthetic: res x res texels per unique quad in face order, row v, column
// u, each of `channels` values (1: an albedo; 3: an RGB base color, channel
// fastest); res = 0 removes them.
int orc_scene_set_textures(void* s, const double* texels, int32_t res, int32_t channels) {
  Scene* S = static_cast<Scene*>(s);
  if (res < 0 || (res > 0 && !texels) || (channels != 1 && channels != 3)) return -1;
  if (res > 0)
    for (int32_t k : S->pkind)
      if (k) return -1;  // textures are per quad face: a scene with curves has none
  S->tex_res = res;
  S->tex_ch = channels;
  S->tex.clear();
  if (res > 0) S->tex.assign(texels, texels + S->albedo.size() * (size_t)res * (size_t)res * (size_t)channels);
  return 0;
}

// Environment map (the scene's textured environment light, Section 4.1):
// w x h radiance values, row-major, row 0 around +z; w = 0 removes it and
// escaping rays see the constant sky again.
int orc_scene_set_environment(void* s, const double* texels, int32_t w, int32_t h) {
  Scene* S = static_cast<Scene*>(s);
  if (w < 0 || h < 0 || (w > 0 && (h < 1 || !texels))) return -1;
  S->env_w = w > 0 ? w : 0;
  S->env_h = w > 0 ? h : 0;
  S->env.clear();
  S->env_T.clear();
  if (w > 0) {
    S->env.assign(texels, texels + (size_t)w * (size_t)h);
    env_table(*S);
  }
  return 0;
}

// rays: n x 8 (ox oy oz dx dy dz tmin tmax), FP32 (read as exact doubles) or FP64.
// excl: n x 3 (inst, prim, half) or NULL; r0: per-ray origin uncertainty or NULL.
// cand: n x 8 int32 ((inst, prim) x 4) or NULL; scale: per-ray position scale of
// the answer (max of 1, |o|, |p| and the hit quad's extent from o) or NULL.
}  // extern "C"

template <class T>
static void trace_many(void* s, int64_t n, const T* rays, const int32_t* excl, const double* r0, int32_t mode,
                       int32_t any_hit, double* t, int32_t* inst, int32_t* prim, int32_t* half, double* u,
                       double* v, uint32_t* flags, int32_t* cand, int32_t* ncand, double* scale) {
  const Scene& S = *static_cast<Scene*>(s);
  parallel_for(n, threads(), [&](int64_t i, int) {
    const T* R = rays + 8 * i;
    Ray r{{(double)R[0], (double)R[1], (double)R[2]}, {(double)R[3], (double)R[4], (double)R[5]}, (double)R[6],
          (double)R[7]};
    Excl ex;
    if (excl) ex = {excl[3 * i], excl[3 * i + 1], excl[3 * i + 2]};
    TraceOut o = trace_one(S, r, ex, r0 ? r0[i] : 0.0, mode, any_hit != 0);
    t[i] = o.best.t;
    inst[i] = o.best.inst;
    prim[i] = o.best.prim;
    half[i] = o.best.half;
    u[i] = o.best.inst >= 0 ? o.best.u : 0.0;
    v[i] = o.best.inst >= 0 ? o.best.v : 0.0;
    flags[i] = o.flags;
    if (cand) {
      for (int c = 0; c < 8; ++c) cand[8 * i + c] = c < 2 * o.ncand ? o.cand[c] : -1;
    }
    if (ncand) ncand[i] = o.ncand;
    if (scale) scale[i] = o.S;
  });
}

extern "C" {

void orc_trace(void* s, int64_t n, const float* rays, const int32_t* excl, const double* r0, int32_t mode,
               int32_t any_hit, double* t, int32_t* inst, int32_t* prim, int32_t* half, double* u, double* v,
               uint32_t* flags, int32_t* cand, int32_t* ncand, double* scale) {
  trace_many(s, n, rays, excl, r0, mode, any_hit, t, inst, prim, half, u, v, flags, cand, ncand, scale);
}

void orc_trace_d(void* s, int64_t n, const double* rays, const int32_t* excl, const double* r0, int32_t mode,
                 int32_t any_hit, double* t, int32_t* inst, int32_t* prim, int32_t* half, double* u, double* v,
                 uint32_t* flags, int32_t* cand, int32_t* ncand, double* scale) {
  trace_many(s, n, rays, excl, r0, mode, any_hit, t, inst, prim, half, u, v, flags, cand, ncand, scale);
}

// Whether each GPU answer is one an FP32 traversal may give (see accept_set).
// rays: n x 8 FP32; excl: n x 3 or NULL; r0: per ray or NULL.  Closest hit
// (any_hit = 0): g_inst, g_prim (-1 = miss), g_half (NULL = either half), g_t.
// Any hit: g_inst[i] = 1 occluded, 0 not.  out[i]: 0 valid; closest: 1 not a
// possible answer, 2 a miss while a certain hit exists, 3 t outside its
// tolerance; any hit: 1 occluded without a possible occluder, 2 unoccluded
// while a certain occluder exists.  info[i] (may be NULL): bit 1 the answer is
// the certain hit, bit 2 its t is ill-conditioned (held to the FP32 bound), bit 4 the ray
// has possible answers other than the certain hit.  ulps[i] (may be NULL): the
// t error of a closest-hit answer in units of 2^-24 S / (|d| |cos|).
void orc_accept(void* s, int64_t n, const float* rays, const int32_t* excl, const double* r0, int32_t mode,
                int32_t any_hit, const int32_t* g_inst, const int32_t* g_prim, const int32_t* g_half,
                const float* g_t, int32_t* out, int32_t* info, double* ulps) {
  const Scene& S = *static_cast<Scene*>(s);
  parallel_for(n, threads(), [&](int64_t i, int) {
    const float* R = rays + 8 * i;
    Ray r{{(double)R[0], (double)R[1], (double)R[2]}, {(double)R[3], (double)R[4], (double)R[5]}, (double)R[6],
          (double)R[7]};
    Excl ex;
    if (excl) ex = {excl[3 * i], excl[3 * i + 1], excl[3 * i + 2]};
    const AcceptSet A = accept_set(S, r, ex, r0 ? r0[i] : 0.0, mode);
    int inf = 0;
    if (any_hit) {
      out[i] = judge_any(A, g_inst[i] != 0);
    } else {
      out[i] = judge_closest(A, g_inst[i], g_inst[i] < 0 ? -1 : g_prim[i], g_half ? g_half[i] : -1,
                             (double)g_t[i], &inf, ulps ? &ulps[i] : nullptr);
    }
    size_t others = 0;
    for (const Cand& c : A.cand)
      if (!A.has_certain || c.k.inst != A.certain.k.inst || c.k.prim != A.certain.k.prim) ++others;
    if (others || !A.has_certain) inf |= 4;
    if (info) info[i] = inf;
  });
}

// Flags by kind and bounce over the listed packed pixels (all samples): hist
// is [16 x 8] doubles; row b counts the closest-hit rays of bounce b (b >= 15
// folded into row 15): columns 0..5 those carrying F_NEAR_TIE, F_GRAZE,
// F_NEAR_ORIGIN, F_T_ILLCOND, F_DIAG, F_SHADE (the ray, its vertex's shading
// decisions, or the environment texel of an escaping ray), column 6 the
// bounce's shadow rays carrying any flag, column 7 every closest-hit ray.
void orc_flag_breakdown(void* s, const double* cam_f, const int64_t* cam_i, int32_t n_cams, const int32_t* pi,
                        const uint64_t* pu, const double* pd, const int64_t* pix, int64_t n_pix, double* hist) {
  const Scene& S = *static_cast<Scene*>(s);
  const Params P = make_params(pi, pu, pd);
  std::vector<Cam> cams;
  for (int c = 0; c < n_cams; ++c) cams.push_back(make_cam(cam_f + 10 * c, cam_i + 8 * c));
  const int nt = threads();
  std::vector<std::vector<double>> h(nt, std::vector<double>(16 * 8, 0.0));
  parallel_for(n_pix, nt, [&](int64_t i, int tid) {
    int32_t view;
    int64_t p;
    resolve_pixel(cams, pix[i], &view, &p);
    for (int32_t smp = 0; smp < P.spp; ++smp) {
      PathRec rec;
      trace_path(S, P, cams[view], (int32_t)cams[view].view_id, p, smp, 1, rec);
      auto add = [&](int b, uint32_t fl) {
        const int r = std::min(b, 15);
        for (int k = 0; k < 6; ++k)
          if (fl & (1u << k)) h[tid][8 * r + k] += 1;
        h[tid][8 * r + 7] += 1;
      };
      for (int k = 0; k < rec.nv; ++k) {
        add(k, rec.v[k].flags);
        if (rec.v[k].shadow >= 0 && rec.v[k].shadow_flags) h[tid][8 * std::min(k, 15) + 6] += 1;
      }
      if (rec.escaped) add(rec.nv, rec.esc_flags);
    }
  });
  for (int k = 0; k < 16 * 8; ++k) {
    hist[k] = 0;
    for (int t = 0; t < nt; ++t) hist[k] += h[t][k];
  }
}

// Check one GPU path (cam entry `cam`, pixel `local` of its rectangle, sample)
// against the scene along its own recorded rays (see check_path).  Returns 0
// when valid, else the first failed check: 1 camera ray, 2 a hit that is not a
// possible answer, 3 an escape while a certain hit exists, 4 t outside its
// tolerance, 5 face index, 6 shading value (albedo or texel), 7 shadow ray cast
// or not against a clear decision, 8 shadow outcome, 9 next origin is not the
// FP32 hit point, 10 next direction, 11 path length, 12 radiance.  stats
// (may be NULL): [failing ray, FP64 radiance, vertices, certain answers,
// t checks waived, shading decisions within rounding of a threshold, largest
// t error in units of 2^-24 S / (|d| |cos|)].
int32_t orc_check_path(void* s, const double* cam_f, const int64_t* cam_i, int32_t n_cams, const int32_t* pi,
                       const uint64_t* pu, const double* pd, int32_t cam, int64_t local, int32_t sample, int32_t nv,
                       const int32_t* vi, const float* vf, int32_t escaped, const float* radiance, double* stats) {
  const Scene& S = *static_cast<Scene*>(s);
  const Params P = make_params(pi, pu, pd);
  if (cam < 0 || cam >= n_cams) return -1;
  const Cam c = make_cam(cam_f + 10 * cam, cam_i + 8 * cam);
  if (local < 0 || local >= c.tw * c.th) return -1;
  const int64_t pix = (c.ty + local / c.tw) * c.w + c.tx + local % c.tw;
  const PathCheck R = check_path(S, P, c, (int32_t)c.view_id, pix, sample, nv, vi, vf, escaped != 0, radiance, 1);
  if (stats) {
    stats[0] = R.vertex;
    stats[1] = R.L;
    stats[2] = R.n_vert;
    stats[3] = R.n_certain;
    stats[4] = R.n_waived;
    stats[5] = R.n_ambiguous_shading;
    stats[6] = R.max_ulps;
    for (int ch = 0; ch < 3; ++ch) stats[7 + ch] = R.Lc[ch];
  }
  return R.code;
}

// Image (or listed pixels) of n_cams pinhole cameras, 3 channels per pixel
// (equal without materials).  cam_f: n x 10 (eye, look, up, vfov); cam_i: n x 8
// (w, h, offset of the view in the packed image, view id, tile).
// pix: global packed pixel indices, or NULL for every pixel.  stats (may be NULL):
// [closest rays, shadow rays, incoherent (bounce >= 1) rays, flagged pixels].
void orc_render(void* s, const double* cam_f, const int64_t* cam_i, int32_t n_cams, const int32_t* pi,
                const uint64_t* pu, const double* pd, const int64_t* pix, int64_t n_pix, int32_t mode,
                double* image, uint8_t* pflags, double* stats) {
  const Scene& S = *static_cast<Scene*>(s);
  const Params P = make_params(pi, pu, pd);
  std::vector<Cam> cams;
  int64_t total = 0;
  for (int c = 0; c < n_cams; ++c) {
    cams.push_back(make_cam(cam_f + 10 * c, cam_i + 8 * c));
    total += cams.back().w * cams.back().h;
  }
  const int64_t n = pix ? n_pix : total;
  const int nt = threads();
  std::vector<double> st(4 * nt, 0.0);
  parallel_for(n, nt, [&](int64_t i, int tid) {
    const int64_t g = pix ? pix[i] : i;
    int32_t view;
    int64_t p;
    resolve_pixel(cams, g, &view, &p);
    C3 sum;
    uint32_t fl = 0;
    for (int32_t smp = 0; smp < P.spp; ++smp) {
      PathRec rec;
      trace_path(S, P, cams[view], (int32_t)cams[view].view_id, p, smp, mode, rec);
      sum = sum + path_value(P, rec);
      fl |= rec.flags;
      st[4 * tid + 0] += rec.n_closest;
      st[4 * tid + 1] += rec.n_shadow;
      st[4 * tid + 2] += rec.n_incoherent;
    }
    for (int ch = 0; ch < 3; ++ch) image[3 * i + ch] = sum.v[ch] / P.spp;
    pflags[i] = (uint8_t)(fl != 0);
    st[4 * tid + 3] += fl != 0;
  });
  if (stats)
    for (int k = 0; k < 4; ++k) {
      stats[k] = 0;
      for (int t2 = 0; t2 < nt; ++t2) stats[k] += st[4 * t2 + k];
    }
}

// One path, vertex by vertex (debugging and tests): per hit k < *nv writes
// out_i[6k..6k+5] = (inst, prim, half, shadow state, flags, shadow flags) and
// out_d[2k..2k+1] = (t, albedo); *escaped = 1 if the path left the scene.
void orc_path(void* s, const double* cam_f, const int64_t* cam_i, int32_t n_cams, const int32_t* pi,
              const uint64_t* pu, const double* pd, int64_t g, int32_t sample, int32_t* nv, int32_t* out_i,
              double* out_d, int32_t* escaped, uint32_t* path_flags) {
  const Scene& S = *static_cast<Scene*>(s);
  const Params P = make_params(pi, pu, pd);
  std::vector<Cam> cams;
  for (int c = 0; c < n_cams; ++c) cams.push_back(make_cam(cam_f + 10 * c, cam_i + 8 * c));
  int32_t view;
  int64_t p;
  resolve_pixel(cams, g, &view, &p);
  PathRec rec;
  trace_path(S, P, cams[view], (int32_t)cams[view].view_id, p, sample, 1, rec);
  *nv = rec.nv;
  for (int k = 0; k < rec.nv; ++k) {
    const Vertex& v = rec.v[k];
    const int32_t vals[6] = {v.inst, v.prim, v.half, v.shadow, (int32_t)v.flags, (int32_t)v.shadow_flags};
    for (int j = 0; j < 6; ++j) out_i[6 * k + j] = vals[j];
    out_d[2 * k] = v.t;
    out_d[2 * k + 1] = v.a;
  }
  *escaped = rec.escaped ? 1 : 0;
  *path_flags = rec.flags;
}

// Gradient of sum_p g_p . I_p (RGB: g_p has 3 weights per pixel) with respect to
// the per-face albedo (or texel) a, paths held fixed.  Every vertex's estimate
// e_k and bounce weight w_k are affine in its own a (the base color is the
// material's tint times a), with derivatives e1_k, w1_k.  With RGB texels each
// channel of a texel is a parameter of its own (index 3 texel + channel), and
// channel c of a vertex's estimate and weight depends on channel c alone.
// mode 0: path replay, dI/da_j = (1/spp) sum over vertices k with parameter j
//         of T_k (e1_k + w1_k R_k), R_k = sum_{i>k} (w_{k+1} .. w_{i-1}) e_i
//         (+ the escape term) the radiance arriving along the bounce of k.
// mode 1: forward-mode dual numbers along `tangent` (per parameter); writes the
//         directional derivative of each listed pixel into dI (3 per pixel).
void orc_grad(void* s, const double* cam_f, const int64_t* cam_i, int32_t n_cams, const int32_t* pi,
              const uint64_t* pu, const double* pd, const int64_t* pix, int64_t n_pix, int32_t mode,
              const double* gpix, int32_t grad_mode, const double* tangent, double* grad_albedo, double* dI,
              uint8_t* pflags, uint8_t* face_tainted, int32_t taint_per_path) {
  const Scene& S = *static_cast<Scene*>(s);
  const Params P = make_params(pi, pu, pd);
  std::vector<Cam> cams;
  int64_t total = 0;
  for (int c = 0; c < n_cams; ++c) {
    cams.push_back(make_cam(cam_f + 10 * c, cam_i + 8 * c));
    total += cams.back().w * cams.back().h;
  }
  const int64_t n = pix ? n_pix : total;
  const int nt = threads();
  // shading parameters: per-face albedo, or every texel (channel) of every face
  const int nch = S.tex_res > 0 ? S.tex_ch : 1;
  const int64_t Q = (int64_t)S.albedo.size() * (S.tex_res > 0 ? (int64_t)S.tex_res * S.tex_res : 1) * nch;
  std::vector<std::vector<double>> gacc(grad_mode == 0 ? nt : 0, std::vector<double>(grad_mode == 0 ? Q : 0, 0.0));
  std::vector<std::vector<uint8_t>> taint(face_tainted ? nt : 0, std::vector<uint8_t>(face_tainted ? Q : 0, 0));
  parallel_for(n, nt, [&](int64_t i, int tid) {
    const int64_t g = pix ? pix[i] : i;
    int32_t view;
    int64_t p;
    resolve_pixel(cams, g, &view, &p);
    uint32_t fl = 0;
    C3 dsum;
    std::vector<int64_t> faces;  // every face on the pixel's paths
    for (int32_t smp = 0; smp < P.spp; ++smp) {
      PathRec rec;
      trace_path(S, P, cams[view], (int32_t)cams[view].view_id, p, smp, mode, rec);
      fl |= rec.flags;
      if (!taint_per_path || rec.flags)
        for (int k = 0; k < rec.nv; ++k) faces.push_back(rec.v[k].param);
      if (grad_mode == 0) {
        std::vector<C3> T(rec.nv + 1);
        T[0] = c3(1.0);
        for (int k = 0; k < rec.nv; ++k) T[k + 1] = T[k] * rec.v[k].w;
        C3 R = rec.escaped ? c3(rec.L_esc) : C3{};  // radiance arriving at the last vertex along its bounce
        for (int k = rec.nv - 1; k >= 0; --k) {
          const C3 d = T[k] * (rec.v[k].e1 + rec.v[k].w1 * R);
          if (nch == 3) {
            for (int ch = 0; ch < 3; ++ch) gacc[tid][3 * rec.v[k].param + ch] += gpix[3 * i + ch] * d.v[ch] / P.spp;
          } else {
            double gsum = 0.0;
            for (int ch = 0; ch < 3; ++ch) gsum += gpix[3 * i + ch] * d.v[ch];
            gacc[tid][rec.v[k].param] += gsum / P.spp;
          }
          R = rec.v[k].e + rec.v[k].w * R;
        }
      } else {
        // dual numbers (value, derivative) along the tangent direction
        C3 T = c3(1.0), dT, dL;
        for (int k = 0; k < rec.nv; ++k) {
          const int64_t q = rec.v[k].param;
          const C3 da = nch == 3 ? C3{{tangent[3 * q], tangent[3 * q + 1], tangent[3 * q + 2]}} : c3(tangent[q]);
          dL = dL + dT * rec.v[k].e + da * (T * rec.v[k].e1);
          dT = dT * rec.v[k].w + da * (T * rec.v[k].w1);
          T = T * rec.v[k].w;
        }
        if (rec.escaped) dL = dL + rec.L_esc * dT;
        dsum = dsum + dL;
      }
    }
    // per pixel: a flagged pixel's value may differ on the GPU, and it weights the
    // gradient of every face on every path through the pixel, so all of them are
    // tainted.  Per path (when both sides use the same pixel weights): only the
    // faces on flagged paths.
    if (face_tainted && fl)
      for (int64_t f : faces)
        for (int ch = 0; ch < nch; ++ch) taint[tid][nch * f + ch] = 1;
    if (grad_mode == 1)
      for (int ch = 0; ch < 3; ++ch) dI[3 * i + ch] = dsum.v[ch] / P.spp;
    if (pflags) pflags[i] = (uint8_t)(fl != 0);
  });
  if (grad_mode == 0)
    for (int64_t f = 0; f < Q; ++f) {
      double acc = 0;
      for (int t2 = 0; t2 < nt; ++t2) acc += gacc[t2][f];
      grad_albedo[f] = acc;
    }
  if (face_tainted)
    for (int64_t f = 0; f < Q; ++f) {
      uint8_t any = 0;
      for (int t2 = 0; t2 < nt; ++t2) any |= taint[t2][f];
      face_tainted[f] = any;
    }
}

}  // extern "C"
