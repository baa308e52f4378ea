// Device-side pieces of the path tracer shared by every scheduler:
// counter-based random numbers, pinhole camera rays, hit shading with next-event
// estimation, and bounces: cosine-distributed for Lambertian faces, drawn from
// the principled BSDF (RGB) when the scene has materials.
//
// Every scheduler calls exactly these functions in the same order per path, so
// the per-path radiance is bit-identical whichever kernel runs the path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trace_device.h"

#pragma clang fp contract(off)

namespace rtq {

// One view, or the rectangle of one that this call renders.  The basis
// (f, r, u) is computed on the host in FP64 and rounded.
struct CamDev {
  float eye[3];
  float f[3], r[3], u[3];
  float tan_half, aspect;
  int32_t w, h;        // the whole view
  int32_t view_id;     // the view's index in the RNG counter
  int32_t tx, ty;      // first column and row of the rendered rectangle
  int32_t tw, th;      // its size
  int64_t img_offset;  // first pixel of the rectangle in the packed image
  int64_t path_base;   // first path id of the rectangle; paths are sample-major: base + s * tw * th + local pixel
};

// A principled material (Section 5.4: the scene's materials use Disney's
// principled BSDF, made energy conserving and preserving): base color
// c = tint x (the face's albedo or texel), alpha = roughness^2 (GGX), metallic,
// and specular, which scales the dielectric Fresnel reflectance; a clearcoat of
// weight coat and GGX alpha calpha over that base.
struct MatDev {
  float tint[3];
  float alpha, metal, spec;
  float coat, calpha;
};

struct RenderParams {
  const CamDev* cams;
  int32_t n_cams;
  int32_t spp;
  int32_t depth;
  const uint32_t* keys; // device [3]: Philox key (seed_lo, seed_hi ^ frame) and the frames already
                        // averaged in the image, written at the start of each call
  float lx, ly, lz;     // unit direction toward the light
  float e_over_pi;      // E / pi
  float L_sky;
  int64_t n_paths;
  float* slots;         // per-path radiance
  const float* alights; // quad area lights, 10 floats each: corner, edge 1, edge 2, radiance
  int32_t n_alights;
  int32_t env_nee;      // next-event estimation toward the environment map (scene has one)
  const MatDev* mats;   // principled materials, or null: Lambertian faces, one channel
  const uint8_t* face_mat;  // material of each unique face
  float E;              // irradiance of the directional light
};

// Whether paths shade with the principled BSDF in three channels; radiance
// slots are then channel-major: slot of channel k of path p at k n_paths + p.
__device__ __forceinline__ bool rgb_mode(const RenderParams& rp) { return rp.mats != nullptr; }

// Whether next-event estimates sample light directions (area lights or the
// environment), so shadow rays carry their own direction and tmax.
__device__ __forceinline__ bool nee_sampled(const RenderParams& rp) { return rp.n_alights > 0 || rp.env_nee != 0; }

// Lights a next-event estimate chooses among: the directional one, the area
// lights and, when sampled, the environment (the last).
__device__ __forceinline__ uint32_t n_lights(const RenderParams& rp) {
  return 1u + (uint32_t)rp.n_alights + (rp.env_nee ? 1u : 0u);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw 2011): ten rounds of two 32x32->64
// multiplications with the round keys bumped by the Weyl constants in between.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Uniform in [0, 1): the top 24 bits, exactly representable in FP32.
__device__ __forceinline__ float u01(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }

// Where a path belongs: the camera entry of the call, the pixel within the
// rendered rectangle (its image slot), and the RNG coordinates (pixel of the
// whole view, sample, view id).
struct PathId {
  int cam;          // camera entry of the call
  uint32_t local;   // pixel index within the rendered rectangle
  uint32_t pixel;   // row * w + column within the whole view
  uint32_t sample;
  uint32_t view;    // view id of the RNG counter
};

// path id -> PathId by binary search over the cameras' path bases.
__device__ __forceinline__ PathId path_coords(const RenderParams& rp, int64_t pid) {
  int lo = 0, hi = rp.n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rp.cams[mid].path_base <= pid) lo = mid;
    else hi = mid - 1;
  }
  const CamDev& c = rp.cams[lo];
  const int64_t n = (int64_t)c.tw * c.th;
  const int64_t k = pid - c.path_base;
  PathId id;
  id.cam = lo;
  id.sample = (uint32_t)(k / n);
  id.local = (uint32_t)(k - (int64_t)id.sample * n);
  const uint32_t row = id.local / (uint32_t)c.tw, col = id.local - row * (uint32_t)c.tw;
  id.pixel = ((uint32_t)c.ty + row) * (uint32_t)c.w + (uint32_t)c.tx + col;
  id.view = (uint32_t)c.view_id;
  return id;
}

struct Ray3 {
  float ox, oy, oz, dx, dy, dz;
};

// Pinhole camera ray through pixel (x, y) (row 0 at the top) jittered by (xi0, xi1).
__device__ __forceinline__ Ray3 camera_ray(const CamDev& c, uint32_t pixel, float xi0, float xi1) {
  const uint32_t x = pixel % (uint32_t)c.w, y = pixel / (uint32_t)c.w;
  const float sx = (2.0f * ((float)x + xi0) / (float)c.w - 1.0f) * c.tan_half * c.aspect;
  const float sy = (1.0f - 2.0f * ((float)y + xi1) / (float)c.h) * c.tan_half;
  float dx = c.f[0] + sx * c.r[0] + sy * c.u[0];
  float dy = c.f[1] + sx * c.r[1] + sy * c.u[1];
  float dz = c.f[2] + sx * c.r[2] + sy * c.u[2];
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  return Ray3{c.eye[0], c.eye[1], c.eye[2], dx * inv, dy * inv, dz * inv};
}

struct Shade {
  float px, py, pz;  // hit point
  float nx, ny, nz;  // unit geometric normal facing the incoming ray
  float a;           // albedo
  float cosl;        // n . light
  uint32_t face;     // unique face index (albedo index)
  uint32_t param;    // the shading parameter read: the face, or its texel (f res + ty) res + tx
};

// Texel index of face `face` at (u, v) (Section 5.3: looked up by face id and
// the hit's coordinates on the face): the nearest of tex_res x tex_res texels
// over the face's unit square.  Clamping in float first keeps the index in
// range for any u, v (NaN included: fmaxf returns the other operand).
__device__ __forceinline__ uint32_t face_texel(const SceneView& sc, uint32_t face, float u, float v) {
  const int R = sc.tex_res;
  const float hi = (float)(R - 1);
  const int tx = (int)fminf(fmaxf(u * (float)R, 0.0f), hi);
  const int ty = (int)fminf(fmaxf(v * (float)R, 0.0f), hi);
  return (face * (uint32_t)R + (uint32_t)ty) * (uint32_t)R + (uint32_t)tx;
}

// Geometric normal of the hit in object space -- the hit half's for a quad; for
// a capsule the hit point minus its closest point on the axis; for a ribbon the
// reverse ray direction without its part along the segment -- mapped to world
// space by A^-T (columns of the stored inverse rows), normalised and turned to
// face the incoming ray; hit point p = o + t d; albedo of the unique prototype
// face (a quad, or the capsule's curve), or its texel at the hit's (u, v) when
// the scene has textures.
__device__ __forceinline__ Shade shade_hit(const SceneView& sc, const RenderParams& rp, const Ray3& r, float t,
                                           uint32_t rec, uint32_t quad, uint32_t half, float u, float v) {
  const float4 f0 = sc.quads[3 * (size_t)quad + 0];
  const float4 f1 = sc.quads[3 * (size_t)quad + 1];
  const float4 f2 = sc.quads[3 * (size_t)quad + 2];
  const InstRec& ir = sc.inst[rec];
  const float4 r0 = *reinterpret_cast<const float4*>(ir.r0);
  const float4 r1 = *reinterpret_cast<const float4*>(ir.r1);
  const float4 r2 = *reinterpret_cast<const float4*>(ir.r2);
  const bool cap = (ir.proto & kProtoCurve) != 0u;
  float onx, ony, onz;
  if ((ir.proto & kProtoFlat) != 0u) {
    // ribbon segment (a, b) = (f0, f1): it faces the ray, so its normal is the
    // reverse object-space direction without its part along the segment
    const float dx = fmaf(r0.x, r.dx, fmaf(r0.y, r.dy, r0.z * r.dz));
    const float dy = fmaf(r1.x, r.dx, fmaf(r1.y, r.dy, r1.z * r.dz));
    const float dz = fmaf(r2.x, r.dx, fmaf(r2.y, r.dy, r2.z * r.dz));
    const float tx = f1.x - f0.x, ty = f1.y - f0.y, tz = f1.z - f0.z;
    const float tt = fmaf(tx, tx, fmaf(ty, ty, tz * tz));
    const float k = tt > 0.0f ? fmaf(dx, tx, fmaf(dy, ty, dz * tz)) / tt : 0.0f;
    onx = fmaf(k, tx, -dx);
    ony = fmaf(k, ty, -dy);
    onz = fmaf(k, tz, -dz);
  } else if (cap) {
    // capsule (a, r) = f0, b = f1.xyz.  Its normal follows the hit point, so the
    // point is formed in FP64 from the FP32 ray and t (exact products, one
    // rounding per sum) relative to the instance origin, where it is small,
    // before the stored inverse rows map it to object space: the normal then
    // carries the rounding of those rows and of the capsule (about 2^-24 of the
    // object coordinates over the radius), not that of the ray's length
    const double hx = ((double)r.ox - (double)r0.w) + (double)t * (double)r.dx;
    const double hy = ((double)r.oy - (double)r1.w) + (double)t * (double)r.dy;
    const double hz = ((double)r.oz - (double)r2.w) + (double)t * (double)r.dz;
    const double px = (double)r0.x * hx + (double)r0.y * hy + (double)r0.z * hz;
    const double py = (double)r1.x * hx + (double)r1.y * hy + (double)r1.z * hz;
    const double pz = (double)r2.x * hx + (double)r2.y * hy + (double)r2.z * hz;
    const double bax = (double)f1.x - (double)f0.x, bay = (double)f1.y - (double)f0.y,
                 baz = (double)f1.z - (double)f0.z;
    const double wx = px - (double)f0.x, wy = py - (double)f0.y, wz = pz - (double)f0.z;
    const double bb = bax * bax + bay * bay + baz * baz;
    const double sa = bb > 0.0 ? fmin(fmax((wx * bax + wy * bay + wz * baz) / bb, 0.0), 1.0) : 0.0;
    onx = (float)(wx - sa * bax);
    ony = (float)(wy - sa * bay);
    onz = (float)(wz - sa * baz);
  } else {
    // v0 = f0.xyz, v1 = (f0.w, f1.x, f1.y), v2 = (f1.z, f1.w, f2.x), v3 = (f2.y, f2.z, f2.w)
    float ax, ay, az, bx, by, bz;
    if (half == 0u) {  // (v1 - v0) x (v3 - v0)
      ax = f0.w - f0.x; ay = f1.x - f0.y; az = f1.y - f0.z;
      bx = f2.y - f0.x; by = f2.z - f0.y; bz = f2.w - f0.z;
    } else {           // (v3 - v2) x (v1 - v2)
      ax = f2.y - f1.z; ay = f2.z - f1.w; az = f2.w - f2.x;
      bx = f0.w - f1.z; by = f1.x - f1.w; bz = f1.y - f2.x;
    }
    onx = ay * bz - az * by;
    ony = az * bx - ax * bz;
    onz = ax * by - ay * bx;
  }
  float nx = r0.x * onx + r1.x * ony + r2.x * onz;
  float ny = r0.y * onx + r1.y * ony + r2.y * onz;
  float nz = r0.z * onx + r1.z * ony + r2.z * onz;
  const float inv = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
  nx *= inv;
  ny *= inv;
  nz *= inv;
  if (nx * r.dx + ny * r.dy + nz * r.dz > 0.0f) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  Shade s;
  s.px = r.ox + t * r.dx;
  s.py = r.oy + t * r.dy;
  s.pz = r.oz + t * r.dz;
  s.nx = nx;
  s.ny = ny;
  s.nz = nz;
  const uint32_t prim = (uint32_t)sc.quad_prim[quad];
  s.face = ir.face_base + (cap ? prim / (uint32_t)kCapsPerCurve : prim);
  s.param = sc.tex_res > 0 ? face_texel(sc, s.face, u, v) : s.face;
  // (an RGB texel's first channel; principled_vertex reads the other two)
  s.a = sc.tex_res > 0 ? sc.tex[(size_t)s.param * sc.tex_ch] : sc.albedo[s.face];
  s.cosl = nx * rp.lx + ny * rp.ly + nz * rp.lz;
  return s;
}

constexpr float kPiF = 3.14159265358979323846f;

// Density (per solid angle) with which the environment's next-event estimate
// draws directions in texel (tx, ty): p_k / Omega_ty, p_k = (T_k - T_{k-1}) / 2^32,
// Omega_ty = (2 pi / W) (cos(pi ty / H) - cos(pi (ty + 1) / H)).
__device__ __forceinline__ float env_pdf(const SceneView& sc, int tx, int ty) {
  const size_t k = (size_t)ty * sc.env_w + tx;
  const float p = (float)(sc.env_T[k] - (k > 0 ? sc.env_T[k - 1] : 0ull)) * 2.3283064365386963e-10f;
  const float om = (2.0f * kPiF / (float)sc.env_w) * (cospif((float)ty / (float)sc.env_h) -
                                                      cospif((float)(ty + 1) / (float)sc.env_h));
  return p / om;
}

// Power-heuristic weight of strategy a against b (Veach 1997).
__device__ __forceinline__ float mis_power(float a, float b) { return a * a / (a * a + b * b); }

// Radiance seen by a ray leaving the scene along d: the constant sky, or the
// nearest texel of the environment map (Section 4.1 names the scene's textured
// environment light), an equirectangular map with u = (atan2(d_y, d_x) + pi) /
// (2 pi) along a row and v = acos(d_z) / pi down the rows (row 0 around +z).
// pdf_bsdf > 0 marks a ray drawn by a cosine bounce with that density: with
// next-event estimation toward the map, its radiance is weighted against that
// strategy by the power heuristic (camera rays pass 0 and keep weight 1).
__device__ __forceinline__ float escape_radiance(const SceneView& sc, const RenderParams& rp, float dx, float dy,
                                                 float dz, float pdf_bsdf) {
  if (sc.env_w == 0) return rp.L_sky;
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  const float z = fminf(fmaxf(dz * inv, -1.0f), 1.0f);
  const float u = (atan2f(dy, dx) + kPiF) / (2.0f * kPiF);
  const float v = acosf(z) / kPiF;
  // clamped in float first, so the index stays in range for any direction
  const int tx = (int)fminf(fmaxf(u * (float)sc.env_w, 0.0f), (float)(sc.env_w - 1));
  const int ty = (int)fminf(fmaxf(v * (float)sc.env_h, 0.0f), (float)(sc.env_h - 1));
  const float L = sc.env[(size_t)ty * sc.env_w + tx];
  if (!rp.env_nee || !(pdf_bsdf > 0.0f)) return L;
  return L * mis_power(pdf_bsdf, env_pdf(sc, tx, ty) / (float)n_lights(rp));
}

// Next-event contribution of a visible light: beta * (a / pi) * E * cos_L.
__device__ __forceinline__ float nee_term(float beta, float a, float cosl, const RenderParams& rp) {
  return beta * (a * rp.e_over_pi * cosl);
}
// The factor c = (E / pi) cos_L that multiplies beta * a (used by the adjoint).
__device__ __forceinline__ float nee_factor(float cosl, const RenderParams& rp) { return rp.e_over_pi * cosl; }

// The shadow ray of one next-event estimate and the factor c that multiplies
// beta * a when it is unoccluded.
struct NeeSample {
  bool want;           // a shadow ray is traced
  float dx, dy, dz;    // its direction (toward the directional light, or to the sampled point)
  float tmax;          // +inf, or 1 for an area-light sample (the ray ends at the point)
  float c;
  // for principled shading: the estimate is X (A + B c) toward the unit
  // direction (ux, uy, uz), times the power-heuristic weight against the BSDF
  // density when pdf_light > 0 (the environment)
  float X, ux, uy, uz, pdf_light;
};

// Next-event estimate at hit s of path (pixel, sample, view), bounce b.
// Without area lights: the directional light, c = (E / pi) cos_L.  With n area
// lights one of the nl = n + 1 lights is picked with equal probability (light
// 0 is the directional one) from word 0 of counter (pixel, sample, view,
// 2^31 + b), in integer arithmetic, and weighted by nl.  Area light j is the
// parallelogram x = c + s e1 + t e2, (s, t) uniform from words 1 and 2, emitting
// radiance Le from the side e1 x e2 faces: c = nl Le A cos_p cos_l / (pi d^2)
// for the sampled point at distance d, A = |e1 x e2|.
__device__ __forceinline__ NeeSample nee_sample(const SceneView& sc, const RenderParams& rp, const Shade& s,
                                                uint32_t pixel, uint32_t sample, uint32_t view, int b) {
  NeeSample r{s.cosl > 0.0f, rp.lx, rp.ly, rp.lz, kInfF, nee_factor(s.cosl, rp), rp.E, rp.lx, rp.ly, rp.lz, 0.0f};
  if (!nee_sampled(rp)) return r;
  const uint4 w = philox4x32_10(make_uint4(pixel, sample, view, 0x80000000u | (uint32_t)b), rp.keys[0], rp.keys[1]);
  const uint32_t nl = n_lights(rp);
  const uint32_t j = (uint32_t)(((uint64_t)(w.x >> 8) * nl) >> 24);
  if (j == 0u) {
    r.c = (float)nl * r.c;
    r.X = (float)nl * rp.E;
    return r;
  }
  if (rp.env_nee && j == nl - 1u) {
    // the environment: texel k = the first with w.y < T_k (binary search of the
    // table, an integer decision), a direction uniform in solid angle within
    // it from words 2, 3; c = nl L_k cos_p w / (pi pdf), w the power-heuristic
    // weight against the cosine bounce (density cos_p / pi)
    const int nt = sc.env_w * sc.env_h;
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((unsigned long long)w.y < sc.env_T[mid]) hi = mid;
      else lo = mid + 1;
    }
    const int ty = lo / sc.env_w, tx = lo - ty * sc.env_w;
    float sp, cp_;
    sincospif(2.0f * ((float)tx + u01(w.z)) / (float)sc.env_w - 1.0f, &sp, &cp_);
    const float z0 = cospif((float)ty / (float)sc.env_h), z1 = cospif((float)(ty + 1) / (float)sc.env_h);
    const float z = z0 - u01(w.w) * (z0 - z1);
    const float rr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    r.dx = rr * cp_;
    r.dy = rr * sp;
    r.dz = z;
    r.tmax = kInfF;
    const float cp = s.nx * r.dx + s.ny * r.dy + s.nz * r.dz;
    r.want = cp > 0.0f;
    const float pdf = env_pdf(sc, tx, ty);
    r.c = (float)nl * (sc.env[lo] * cp * mis_power(pdf / (float)nl, cp / kPiF) / (kPiF * pdf));
    r.X = (float)nl * sc.env[lo] / pdf;
    r.ux = r.dx;
    r.uy = r.dy;
    r.uz = r.dz;
    r.pdf_light = pdf / (float)nl;
    return r;
  }
  const float* q = rp.alights + 10 * (j - 1u);
  const float su = u01(w.y), sv = u01(w.z);
  const float wx = q[0] + su * q[3] + sv * q[6] - s.px;
  const float wy = q[1] + su * q[4] + sv * q[7] - s.py;
  const float wz = q[2] + su * q[5] + sv * q[8] - s.pz;
  const float d2 = wx * wx + wy * wy + wz * wz;
  const float inv_d = 1.0f / sqrtf(d2);
  const float nx = q[4] * q[8] - q[5] * q[7], ny = q[5] * q[6] - q[3] * q[8], nz = q[3] * q[7] - q[4] * q[6];
  const float A = sqrtf(nx * nx + ny * ny + nz * nz);
  const float cp = (s.nx * wx + s.ny * wy + s.nz * wz) * inv_d;
  const float cq = -(nx * wx + ny * wy + nz * wz) * inv_d / A;
  r.want = cp > 0.0f && cq > 0.0f;
  r.dx = wx;
  r.dy = wy;
  r.dz = wz;
  r.tmax = 1.0f;
  r.c = (float)nl * (q[9] * A * cp * cq / (3.14159265358979323846f * d2));
  r.X = (float)nl * (q[9] * A * cq / d2);
  r.ux = wx * inv_d;
  r.uy = wy * inv_d;
  r.uz = wz * inv_d;
  return r;
}

// beta * a * c, in the directional light's own rounding order when the scene
// has no area lights.
__device__ __forceinline__ float nee_contrib(float beta, const Shade& s, const NeeSample& ns,
                                             const RenderParams& rp) {
  return !nee_sampled(rp) ? nee_term(beta, s.a, s.cosl, rp) : beta * (s.a * ns.c);
}

// Cosine-distributed direction about n from (u1, u2): local
// (sqrt(u1) cos 2 pi u2, sqrt(u1) sin 2 pi u2, sqrt(1 - u1)) in the orthonormal
// basis of Duff et al. 2017.
__device__ __forceinline__ void cosine_dir(float nx, float ny, float nz, float u1, float u2, float* dx, float* dy,
                                           float* dz) {
  const float sg = nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sg + nz);
  const float b = nx * ny * a;
  const float t1x = 1.0f + sg * nx * nx * a, t1y = sg * b, t1z = -sg * nx;
  const float t2x = b, t2y = sg + ny * ny * a, t2z = -ny;
  const float rr = sqrtf(u1);
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  const float lx = rr * cs, ly = rr * sn, lz = sqrtf(1.0f - u1);
  *dx = lx * t1x + ly * t2x + lz * nx;
  *dy = lx * t1y + ly * t2y + lz * ny;
  *dz = lx * t1z + ly * t2z + lz * nz;
}

// ---------------------------------------------------------------- principled BSDF
// At a vertex with unit normal n (the viewer's side) and unit direction wo to
// the viewer, mu_o = n . wo, the cosine-weighted BSDF toward wi (mu_i = n . wi > 0)
// is f mu_i = (1 - m)[F_d p_s + (1 - F_d) c mu_i / pi] + m F_c p_s = A + B c, with
// the dielectric Fresnel weight F_d = spec (0.04 + 0.96 (1 - mu_o)^5) and the
// metal's F_c = c + (1 - c)(1 - mu_o)^5 (Schlick at the macro-surface angle).
// p_s is the density of the specular lobe: wo reflected about a GGX visible
// normal (Heitz 2018), a reflection below the surface mirrored above it, so p_s
// integrates to one and the albedo is (1 - m)[F_d + (1 - F_d) c] + m F_c: one
// for a white base (energy preserving), below one otherwise (conserving).  The
// specular lobe is drawn with probability P_s = (1 - m) F_d + m, independent of
// c; the density of a direction is P_s p_s + (1 - P_s) mu_i / pi.
// A clearcoat of weight k adds a second such lobe p_k with the coat's roughness
// and Fresnel weight F_k = k (0.04 + 0.96 (1 - mu_o)^5) over the base, which
// keeps the rest: f mu_i = F_k p_k + (1 - F_k) [base], albedo F_k + (1 - F_k)
// [base albedo].  The coat is drawn with probability F_k, the base's lobes with
// the rest; k = 0 is the base alone, bit for bit.
struct PShade {
  float nx, ny, nz;           // normal
  float ox, oy, oz;           // unit direction to the viewer
  float t1x, t1y, t1z, t2x, t2y, t2z;  // basis of Duff et al. 2017 about n
  float mo, alpha, metal, Fd, k5, Ps;
  float calpha, Fk, Pn;       // the coat's alpha and weight; Pn = F_k + (1 - F_k) P_s
  float tint[3];
};

__device__ __forceinline__ PShade make_pshade(const MatDev& m, const Shade& s, const Ray3& r) {
  PShade p;
  p.nx = s.nx;
  p.ny = s.ny;
  p.nz = s.nz;
  const float inv = 1.0f / sqrtf(r.dx * r.dx + r.dy * r.dy + r.dz * r.dz);
  p.ox = -r.dx * inv;
  p.oy = -r.dy * inv;
  p.oz = -r.dz * inv;
  const float sg = s.nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sg + s.nz);
  const float b = s.nx * s.ny * a;
  p.t1x = 1.0f + sg * s.nx * s.nx * a;
  p.t1y = sg * b;
  p.t1z = -sg * s.nx;
  p.t2x = b;
  p.t2y = sg + s.ny * s.ny * a;
  p.t2z = -s.ny;
  p.mo = p.nx * p.ox + p.ny * p.oy + p.nz * p.oz;
  const float om = fmaxf(0.0f, 1.0f - p.mo);
  const float om2 = om * om;
  p.k5 = om2 * om2 * om;
  p.alpha = m.alpha;
  p.metal = m.metal;
  p.Fd = m.spec * (0.04f + 0.96f * p.k5);
  p.Ps = (1.0f - m.metal) * p.Fd + m.metal;
  p.calpha = m.calpha;
  p.Fk = m.coat * (0.04f + 0.96f * p.k5);
  p.Pn = p.Fk + (1.0f - p.Fk) * p.Ps;
  p.tint[0] = m.tint[0];
  p.tint[1] = m.tint[1];
  p.tint[2] = m.tint[2];
  return p;
}

// GGX distribution with the cosine c = n . h and s2 = |n x h|^2 (the form
// 1 - c^2 (1 - alpha^2) = s2 + c^2 alpha^2 keeps its precision near the peak)
__device__ __forceinline__ float ggx_D(float alpha, float c, float s2) {
  const float a2 = alpha * alpha;
  const float q = s2 + c * c * a2;
  return a2 / (kPiF * q * q);
}
__device__ __forceinline__ float smith_G1(float alpha, float mu) {
  return 2.0f * mu / (mu + sqrtf(alpha * alpha + (1.0f - alpha * alpha) * mu * mu));
}
// D of the half vector of unit directions a and b about n
__device__ __forceinline__ float ggx_D_half(const PShade& p, float alpha, float ax, float ay, float az, float bx,
                                            float by, float bz) {
  float hx = ax + bx, hy = ay + by, hz = az + bz;
  const float inv = 1.0f / sqrtf(hx * hx + hy * hy + hz * hz);
  hx *= inv;
  hy *= inv;
  hz *= inv;
  const float c = p.nx * hx + p.ny * hy + p.nz * hz;
  const float cx = p.ny * hz - p.nz * hy, cy = p.nz * hx - p.nx * hz, cz = p.nx * hy - p.ny * hx;
  return ggx_D(alpha, c, cx * cx + cy * cy + cz * cz);
}

// density of a mirrored visible-normal lobe of GGX alpha toward unit wi
__device__ __forceinline__ float spec_pdf(const PShade& p, float alpha, float wx, float wy, float wz) {
  const float mi = p.nx * wx + p.ny * wy + p.nz * wz;
  if (!(mi > 0.0f) || !(p.mo > 0.0f)) return 0.0f;
  const float g = smith_G1(alpha, p.mo) / (4.0f * p.mo);
  float pdf = g * ggx_D_half(p, alpha, p.ox, p.oy, p.oz, wx, wy, wz);
  if (p.mo > mi) {
    const float mx = wx - 2.0f * mi * p.nx, my = wy - 2.0f * mi * p.ny, mz = wz - 2.0f * mi * p.nz;
    pdf += g * ggx_D_half(p, alpha, p.ox, p.oy, p.oz, mx, my, mz);
  }
  return pdf;
}

// f mu_i = A + B c toward unit wi (zero below the surface) and the density of
// drawing wi
__device__ __forceinline__ void pbsdf_eval(const PShade& p, float wx, float wy, float wz, float* A, float* B,
                                           float* pdf) {
  const float mi = p.nx * wx + p.ny * wy + p.nz * wz;
  if (!(mi > 0.0f)) {
    *A = *B = *pdf = 0.0f;
    return;
  }
  const float ps = p.Ps > 0.0f ? spec_pdf(p, p.alpha, wx, wy, wz) : 0.0f;
  *A = ((1.0f - p.metal) * p.Fd + p.metal * p.k5) * ps;
  *B = (1.0f - p.metal) * (1.0f - p.Fd) * mi / kPiF + p.metal * (1.0f - p.k5) * ps;
  *pdf = (p.Ps > 0.0f ? p.Ps * ps : 0.0f) + (1.0f - p.Ps) * mi / kPiF;
  if (p.Fk > 0.0f) {
    const float pk = spec_pdf(p, p.calpha, wx, wy, wz);
    *A = p.Fk * pk + (1.0f - p.Fk) * *A;
    *B = (1.0f - p.Fk) * *B;
    *pdf = p.Fk * pk + (1.0f - p.Fk) * *pdf;
  }
}

// Bounce direction from the lobe word u0 and (u1, u2): a GGX visible normal
// (Heitz 2018: stretch wo by alpha, sample the projected half disk, unstretch)
// and the reflection about it, mirrored above the surface, when u0 < Pn -- of
// the coat's alpha when u0 < F_k, else of the base's; the cosine lobe
// otherwise.
__device__ __forceinline__ void pbsdf_sample(const PShade& p, float u0, float u1, float u2, float* dx, float* dy,
                                             float* dz) {
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  if (!(u0 < p.Pn)) {
    const float rr = sqrtf(u1);
    const float lx = rr * cs, ly = rr * sn, lz = sqrtf(1.0f - u1);
    *dx = lx * p.t1x + ly * p.t2x + lz * p.nx;
    *dy = lx * p.t1y + ly * p.t2y + lz * p.ny;
    *dz = lx * p.t1z + ly * p.t2z + lz * p.nz;
    return;
  }
  const float alpha = u0 < p.Fk ? p.calpha : p.alpha;
  const float olx = p.ox * p.t1x + p.oy * p.t1y + p.oz * p.t1z;
  const float oly = p.ox * p.t2x + p.oy * p.t2y + p.oz * p.t2z;
  float vx = alpha * olx, vy = alpha * oly, vz = p.mo;
  const float vlen = sqrtf(vx * vx + vy * vy + vz * vz);
  const float iv = 1.0f / vlen;
  vx *= iv;
  vy *= iv;
  vz *= iv;
  const float l2 = vx * vx + vy * vy;
  float T1x = 1.0f, T1y = 0.0f;
  if (l2 > 0.0f) {
    const float il = 1.0f / sqrtf(l2);
    T1x = -vy * il;
    T1y = vx * il;
  }
  // T2 = v x T1 (T1 has no z component)
  const float T2x = -vz * T1y, T2y = vz * T1x, T2z = vx * T1y - vy * T1x;
  // a point of the unit disk, (p1, r sin phi), its second coordinate warped to
  // p2 = (1 - s) q + s r sin phi with q = sqrt(1 - p1^2), and its height
  // sqrt(1 - p1^2 - p2^2).  Near the rim, 1 - p1^2 - p2^2 cancels; written as
  // (q - p2)(q + p2) with q - p2 = s (q - r sin phi), q + p2 = 2 (1 - s) q +
  // s (q + r sin phi), and (q - r sin phi)(q + r sin phi) = 1 - u1 exactly, each
  // factor is formed without cancellation: the one of q -+ r sin phi whose terms
  // cancel as (1 - u1) over the other, and 1 - s = (1 - v_z) / 2 with
  // 1 - v_z = alpha^2 (1 - mu_o^2) / (|v| (|v| + mu_o)) from the unnormalised v.
  const float rr = sqrtf(u1);
  const float p1 = rr * cs, rs = rr * sn;
  const float osw = 0.5f * ((alpha * alpha * (olx * olx + oly * oly)) / (vlen * (vlen + p.mo)));  // 1 - s
  const float sw = 1.0f - osw;
  const float q = sqrtf((1.0f - u1) + u1 * (sn * sn));
  const float p2 = osw * q + sw * rs;
  const float qm = rs > 0.0f ? (1.0f - u1) / (q + rs) : q - rs;  // q - r sin phi
  const float qp = rs < 0.0f ? (1.0f - u1) / (q - rs) : q + rs;  // q + r sin phi
  const float pz = sqrtf(fmaxf(0.0f, sw * qm * (2.0f * osw * q + sw * qp)));
  const float nhx = p1 * T1x + p2 * T2x + pz * vx;
  const float nhy = p1 * T1y + p2 * T2y + pz * vy;
  const float nhz = p2 * T2z + pz * vz;
  float hx = alpha * nhx, hy = alpha * nhy, hz = fmaxf(0.0f, nhz);
  const float ih = 1.0f / sqrtf(hx * hx + hy * hy + hz * hz);
  hx *= ih;
  hy *= ih;
  hz *= ih;
  const float wx_h = hx * p.t1x + hy * p.t2x + hz * p.nx;
  const float wy_h = hx * p.t1y + hy * p.t2y + hz * p.ny;
  const float wz_h = hx * p.t1z + hy * p.t2z + hz * p.nz;
  const float oh = p.ox * wx_h + p.oy * wy_h + p.oz * wz_h;
  float rx = 2.0f * oh * wx_h - p.ox, ry = 2.0f * oh * wy_h - p.oy, rz = 2.0f * oh * wz_h - p.oz;
  const float mi = p.nx * rx + p.ny * ry + p.nz * rz;
  if (mi < 0.0f) {
    rx -= 2.0f * mi * p.nx;
    ry -= 2.0f * mi * p.ny;
    rz -= 2.0f * mi * p.nz;
  }
  *dx = rx;
  *dy = ry;
  *dz = rz;
}

// The principled vertex of hit s reached by ray r: its frame, and base color
// per channel in c: tint x s.a, or tint_k x channel k of an RGB texel.
__device__ __forceinline__ PShade principled_vertex(const SceneView& sc, const RenderParams& rp, const Shade& s,
                                                    const Ray3& r, float c[3]) {
  const PShade p = make_pshade(rp.mats[rp.face_mat[s.face]], s, r);
  const bool rgb_tex = sc.tex_res > 0 && sc.tex_ch == 3;
  c[0] = p.tint[0] * s.a;
  c[1] = p.tint[1] * (rgb_tex ? sc.tex[3 * (size_t)s.param + 1] : s.a);
  c[2] = p.tint[2] * (rgb_tex ? sc.tex[3 * (size_t)s.param + 2] : s.a);
  return p;
}

// Principled next-event estimate per channel (zero when no shadow ray is
// traced): X (A + B c_k) toward the sampled light direction, with the power
// heuristic against the BSDF density for the environment; e1 receives its
// derivative in the face's albedo.
__device__ __forceinline__ void pnee_estimate(const PShade& p, const float c[3], const NeeSample& ns, float e[3],
                                              float e1[3]) {
  float A, B, pdf;
  pbsdf_eval(p, ns.ux, ns.uy, ns.uz, &A, &B, &pdf);
  float X = ns.X;
  if (ns.pdf_light > 0.0f) X *= mis_power(ns.pdf_light, pdf);
  for (int k = 0; k < 3; ++k) {
    e[k] = ns.want ? X * (A + B * c[k]) : 0.0f;
    e1[k] = ns.want ? X * (B * p.tint[k]) : 0.0f;
  }
}

// Principled bounce after hit b: the lobe word (word 0 of counter (pixel,
// sample, view, 2^30 + b), drawn only when a specular or coat lobe has weight), the
// direction from words 2, 3 of counter (pixel, sample, view, b), its weight
// w_k = (A + B c_k) / pdf per channel and derivative w1_k = B tint_k / pdf.
// Returns the density (0: the direction lies on the surface and the path ends).
__device__ __forceinline__ float pbsdf_bounce(const RenderParams& rp, const PShade& p, const float c[3],
                                              uint32_t pixel, uint32_t sample, uint32_t view, int b, float* dx,
                                              float* dy, float* dz, float w[3], float w1[3]) {
  const uint4 wd = philox4x32_10(make_uint4(pixel, sample, view, (uint32_t)b), rp.keys[0], rp.keys[1]);
  float u0 = 1.0f;
  if (p.Pn > 0.0f) {
    const uint4 wl = philox4x32_10(make_uint4(pixel, sample, view, 0x40000000u | (uint32_t)b), rp.keys[0],
                                   rp.keys[1]);
    u0 = u01(wl.x);
  }
  pbsdf_sample(p, u0, u01(wd.z), u01(wd.w), dx, dy, dz);
  const float inv = 1.0f / sqrtf(*dx * *dx + *dy * *dy + *dz * *dz);
  float A, B, pdf;
  pbsdf_eval(p, *dx * inv, *dy * inv, *dz * inv, &A, &B, &pdf);
  for (int k = 0; k < 3; ++k) {
    w[k] = pdf > 0.0f ? (A + B * c[k]) / pdf : 0.0f;
    w1[k] = pdf > 0.0f ? B * p.tint[k] / pdf : 0.0f;
  }
  return pdf;
}

// Camera ray of path `pid` (jitter from words 0, 1 of the bounce-0 counter).
__device__ __forceinline__ Ray3 path_camera_ray(const RenderParams& rp, int64_t pid, PathId* id) {
  *id = path_coords(rp, pid);
  const uint4 w = philox4x32_10(make_uint4(id->pixel, id->sample, id->view, 0u), rp.keys[0], rp.keys[1]);
  return camera_ray(rp.cams[id->cam], id->pixel, u01(w.x), u01(w.y));
}

// Bounce direction after hit b of a path (words 2, 3 of counter (pixel, sample,
// view, b)); returns its density cos / pi.
__device__ __forceinline__ float bounce_dir(const RenderParams& rp, uint32_t pixel, uint32_t sample, uint32_t view,
                                            int b, const Shade& s, float* dx, float* dy, float* dz) {
  const uint4 w = philox4x32_10(make_uint4(pixel, sample, view, (uint32_t)b), rp.keys[0], rp.keys[1]);
  cosine_dir(s.nx, s.ny, s.nz, u01(w.z), u01(w.w), dx, dy, dz);
  return sqrtf(1.0f - u01(w.z)) / kPiF;
}

}  // namespace rtq
