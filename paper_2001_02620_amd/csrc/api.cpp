// C-ABI of the library: argument validation, scene construction and ownership,
// and the dispatch of every enqueued operation onto the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rtq.h"
#include "api_internal.h"
#include "bvh_build.h"
#include "kernels.h"
#include "rebraid.h"
#include "render_device.h"

using namespace rtq;

namespace {
thread_local std::string g_err = "no error";
}

namespace rtq {

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? RTQ_E_OOM : RTQ_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void* DeviceBuffers::alloc(size_t bytes, hipError_t* err) {
  void* p = nullptr;
  *err = hipMalloc(&p, std::max<size_t>(bytes, 16));
  if (*err != hipSuccess) return nullptr;
  ptrs.push_back(p);
  total += bytes;
  return p;
}

void DeviceBuffers::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  total = 0;
}

SceneView scene_view(const rtq_scene* s, int fmt) {
  SceneView v;
  v.nodes = reinterpret_cast<const uint4*>((fmt & kCodecMask) == kCodecF32 ? s->nodes_f32 : s->nodes_q8);
  v.rec_pmax = s->rec_pmax;
  v.p_world = s->p_world;
  v.tlas_root = s->tlas_root;
  v.quads = s->quads;
  v.quad_prim = s->quad_prim;
  v.inst = s->inst;
  v.rec_qfirst = s->rec_qfirst;
  v.rec_nq = s->rec_nq;
  v.albedo = s->albedo;
  v.tex = s->tex;
  v.tex_res = s->tex_res;
  v.tex_ch = s->tex_ch;
  v.env = s->env;
  v.env_w = s->env_w;
  v.env_h = s->env_h;
  v.env_T = s->env_T;
  v.pad_rel = s->pad_rel;
  v.n_rec = (uint32_t)s->n_rec;
  return v;
}

int resolve_format(const rtq_scene* s, int32_t req, int* fmt) {
  int f = req;
  if (f == 0) f = (s->formats & RTQ_NODE_Q8) ? RTQ_NODE_Q8 : RTQ_NODE_FP32;
  if (f != RTQ_NODE_FP32 && f != RTQ_NODE_Q8) return set_error(RTQ_E_INVALID_ARG, "unknown node format %d", req);
  if (!(s->formats & f)) return set_error(RTQ_E_INVALID_ARG, "node format %d was not built", f);
  if (f == RTQ_NODE_FP32) *fmt = kCodecF32;
  else *fmt = s->width == 8 ? kCodecQ8W8 : (s->width == 2 ? kCodecQ8W2 : kCodecQ8);
  if (s->n_curves > 0) *fmt |= kCodecCurves;
  return RTQ_OK;
}

int resolve_launch(const rtq_scene* s, int32_t sched, int32_t depth, int32_t block, int32_t waves, int32_t refill,
                   TraceLaunch* tl) {
  tl->persistent = sched;
  tl->stack_depth = depth ? depth : 20;
  tl->block = block ? block : 256;
  tl->refill = refill ? refill : 16;
  const int w = waves ? waves : 24;
  if (sched != RTQ_SCHED_PLAIN && sched != RTQ_SCHED_PERSISTENT)
    return set_error(RTQ_E_INVALID_ARG, "unknown scheduler %d", sched);
  if (tl->stack_depth < 4 || tl->stack_depth > 64)
    return set_error(RTQ_E_INVALID_ARG, "stack_depth %d outside [4, 64]", tl->stack_depth);
  if (tl->block < 64 || tl->block > 1024 || tl->block % 64)
    return set_error(RTQ_E_INVALID_ARG, "block %d must be a multiple of 64 in [64, 1024]", tl->block);
  if ((size_t)tl->block * tl->stack_depth * kStackEntryBytes > (size_t)s->max_lds)
    return set_error(RTQ_E_INVALID_ARG, "block %d x stack_depth %d needs %d B of LDS, the device allows %d",
                     tl->block, tl->stack_depth, tl->block * tl->stack_depth * kStackEntryBytes, s->max_lds);
  if (tl->refill < 1 || tl->refill > 64) return set_error(RTQ_E_INVALID_ARG, "refill %d outside [1, 64]", tl->refill);
  if (w < 1 || w > 32) return set_error(RTQ_E_INVALID_ARG, "waves_per_cu %d outside [1, 32]", w);
  const int waves_per_block = tl->block / 64;
  tl->grid = std::max(1, (s->n_cu * w + waves_per_block - 1) / waves_per_block);
  const uint32_t slot = s->counter_next.fetch_add(1) % rtq_scene::kCounterSlots;
  tl->counter = s->counters + (size_t)slot * kClaimWords;
  return RTQ_OK;
}

}  // namespace rtq

// =============================================================================
extern "C" {

const char* rtq_last_error(void) { return g_err.c_str(); }

const char* rtq_version(void) { return "rtq 0.1 (gfx950)"; }

// Extra top-level entries from opened instances, in percent of the instance
// count, when the caller leaves rtq_build_opts.open_pct at 0.
constexpr int32_t kDefaultOpenPct = 50;

// One segment of a curve: axis from a to b, radius r at a and rb at b (equal
// for the capsules of round curves; FP32 values).
struct Capsule {
  float a[3], b[3], r, rb;
};

// Curve -> kCapsPerCurve capsules (Section 5.2: curves rendered as chains of
// primitives).  The Bezier point at s = j / 8 is evaluated by de Casteljau's
// construction in FP64, which is exact here: every control value is an FP32
// number and s a dyadic fraction of 3 bits, so each of the three rounds of
// interpolation adds at most 3 bits to the operands' 24 (plus their exponent
// spread), well inside FP64's 53.  The exact point is then rounded once to FP32.
// A capsule's radius is the FP32 rounding of the mean of its end radii (exact
// in FP64 for the same reason); a ribbon segment keeps both end radii.
static void tessellate_curve(const float* cp, Capsule* out, bool flat) {
  double X[kCapsPerCurve + 1][4];
  for (int j = 0; j <= kCapsPerCurve; ++j) {
    const double s = (double)j / kCapsPerCurve;
    for (int c = 0; c < 4; ++c) {
      double v[4] = {cp[c], cp[4 + c], cp[8 + c], cp[12 + c]};
      for (int level = 3; level > 0; --level)
        for (int k = 0; k < level; ++k) v[k] = v[k] + s * (v[k + 1] - v[k]);
      X[j][c] = (double)(float)v[0];
    }
  }
  for (int j = 0; j < kCapsPerCurve; ++j) {
    Capsule& c = out[j];
    for (int k = 0; k < 3; ++k) {
      c.a[k] = (float)X[j][k];
      c.b[k] = (float)X[j + 1][k];
    }
    if (flat) {
      c.r = (float)X[j][3];
      c.rb = (float)X[j + 1][3];
    } else {
      c.r = c.rb = (float)(0.5 * (X[j][3] + X[j + 1][3]));
    }
  }
}

// Box of a capsule for the bottom-level build: the axis's box grown by r and by
// a margin of 2^-18 (max |coordinate| + r) for the FP32 capsule test, whose
// hits may lie that far outside the exact surface (the traversal must not cull
// a box whose capsule the same test would report hit), rounded outward.
static Aabb capsule_box(const Capsule& c) {
  const double rr = std::max((double)c.r, (double)c.rb);
  double m = rr;
  for (int k = 0; k < 3; ++k) m = std::max(m, std::max(std::fabs((double)c.a[k]), std::fabs((double)c.b[k])));
  const double g = rr + std::ldexp(m + rr, -18);
  Aabb b;
  for (int k = 0; k < 3; ++k) {
    const double lo = std::min((double)c.a[k], (double)c.b[k]) - g;
    const double hi = std::max((double)c.a[k], (double)c.b[k]) + g;
    float l = (float)lo, h = (float)hi;
    if ((double)l > lo) l = std::nextafter(l, -std::numeric_limits<float>::infinity());
    if ((double)h < hi) h = std::nextafter(h, std::numeric_limits<float>::infinity());
    b.lo[k] = l;
    b.hi[k] = h;
  }
  return b;
}

static int build_impl(const rtq_prototype* protos, int32_t n_protos, const rtq_instances* insts,
                      const rtq_build_opts* opts, rtq_scene** out) {
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  };
  if (!out) return set_error(RTQ_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!protos || n_protos < 1) return set_error(RTQ_E_INVALID_ARG, "need at least one prototype");
  if (n_protos >= (1 << 30)) return set_error(RTQ_E_LIMIT, "%d prototypes exceed 2^30", n_protos);
  if (!insts || insts->n < 0 || (insts->n > 0 && (!insts->proto || !insts->xform)))
    return set_error(RTQ_E_INVALID_ARG, "bad instance arrays");
  rtq_build_opts o{};
  if (opts) o = *opts;
  const int width = o.node_width ? o.node_width : 4;
  if (width != 2 && width != 4 && width != 8) return set_error(RTQ_E_INVALID_ARG, "node_width %d is not 2, 4 or 8", width);
  const int formats = o.formats ? o.formats : (width == 4 ? (RTQ_NODE_FP32 | RTQ_NODE_Q8) : RTQ_NODE_Q8);
  if (formats & ~(RTQ_NODE_FP32 | RTQ_NODE_Q8)) return set_error(RTQ_E_INVALID_ARG, "bad formats mask");
  if ((formats & RTQ_NODE_FP32) && width != 4)
    return set_error(RTQ_E_INVALID_ARG, "FP32 nodes are 4-wide only (node_width %d)", width);
  BuildParams bp;
  bp.width = width;
  bp.leaf_max = o.leaf_max ? o.leaf_max : 4;
  bp.bins = o.sah_bins ? o.sah_bins : 32;
  bp.want_q8 = true;  // the quantized nodes are cheap to derive; keep both topologies identical
  if (bp.leaf_max < 1 || bp.leaf_max > 8) return set_error(RTQ_E_INVALID_ARG, "leaf_max %d outside [1, 8]", bp.leaf_max);
  if (bp.bins < 4 || bp.bins > 64) return set_error(RTQ_E_INVALID_ARG, "sah_bins %d outside [4, 64]", bp.bins);
  if (o.open_area_pct != 0 && (o.open_area_pct < 100 || o.open_area_pct > 1000))
    return set_error(RTQ_E_INVALID_ARG, "open_area_pct %d outside [100, 1000]", o.open_area_pct);
  const int64_t N = insts->n;
  if (N > (int64_t)kMaxLeafFirst) return set_error(RTQ_E_LIMIT, "%lld instances exceed 2^28", (long long)N);

  // ---- validate prototypes: a quad mesh, or curves
  int64_t total_quads = 0, total_curves = 0, total_prims = 0, total_faces = 0;
  std::vector<int32_t> n_prim(n_protos);
  for (int32_t p = 0; p < n_protos; ++p) {
    const rtq_prototype& P = protos[p];
    if (P.n_curves < 0 || P.n_quads < 0) return set_error(RTQ_E_INVALID_ARG, "prototype %d: negative count", p);
    if ((P.n_quads > 0) == (P.n_curves > 0))
      return set_error(RTQ_E_INVALID_ARG, "prototype %d: needs quads or curves (one kind)", p);
    if (P.n_curves > 0) {
      if (!P.curves) return set_error(RTQ_E_INVALID_ARG, "prototype %d: NULL curves", p);
      if ((int64_t)P.n_curves * kCapsPerCurve > (int64_t)kMaxLeafFirst)
        return set_error(RTQ_E_LIMIT, "prototype %d: %d curves exceed 2^28 capsules", p, P.n_curves);
      for (int64_t i = 0; i < 16 * (int64_t)P.n_curves; ++i) {
        if (!std::isfinite(P.curves[i]))
          return set_error(RTQ_E_INVALID_ARG, "prototype %d: non-finite control point", p);
        if (i % 4 == 3 && P.curves[i] < 0.0f) return set_error(RTQ_E_INVALID_ARG, "prototype %d: negative radius", p);
      }
      n_prim[p] = P.n_curves * kCapsPerCurve;
      total_curves += P.n_curves;
      total_faces += P.n_curves;
    } else {
      if (!P.verts || !P.quads || P.n_verts < 1)
        return set_error(RTQ_E_INVALID_ARG, "prototype %d: empty or NULL arrays", p);
      for (int64_t i = 0; i < 3 * (int64_t)P.n_verts; ++i)
        if (!std::isfinite(P.verts[i])) return set_error(RTQ_E_INVALID_ARG, "prototype %d: non-finite vertex", p);
      for (int64_t i = 0; i < 4 * (int64_t)P.n_quads; ++i)
        if (P.quads[i] < 0 || P.quads[i] >= P.n_verts)
          return set_error(RTQ_E_INVALID_ARG, "prototype %d: quad index %d out of range", p, P.quads[i]);
      n_prim[p] = P.n_quads;
      total_quads += P.n_quads;
      total_faces += P.n_quads;
    }
    total_prims += n_prim[p];
    if (total_prims > (int64_t)kMaxLeafFirst)
      return set_error(RTQ_E_LIMIT, "more than 2^28 unique primitives (quads and capsules)");
  }
  for (int64_t i = 0; i < N; ++i)
    if (insts->proto[i] < 0 || insts->proto[i] >= n_protos)
      return set_error(RTQ_E_INVALID_ARG, "instance %lld: prototype %d out of range", (long long)i, insts->proto[i]);
  for (int64_t i = 0; i < 12 * N; ++i)
    if (!std::isfinite(insts->xform[i])) return set_error(RTQ_E_INVALID_ARG, "non-finite instance transform");

  int dev = o.device;
  hipError_t e;
  if (dev < 0) {
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  }
  e = hipSetDevice(dev);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");

  // ---- bottom level: one BVH per prototype, built on host threads
  std::vector<Bvh> blas(n_protos);
  std::vector<int32_t> order_p(n_protos);
  for (int32_t p = 0; p < n_protos; ++p) order_p[p] = p;
  std::sort(order_p.begin(), order_p.end(), [&](int a, int b) { return n_prim[a] > n_prim[b]; });
  const int nthreads_all =
      o.build_threads > 0 ? o.build_threads : (int)std::max(1u, std::thread::hardware_concurrency());
  // prototypes of kBigProto quads or more are built one at a time on every
  // thread (they come first in order_p); the rest concurrently, one per thread
  constexpr int32_t kBigProto = 1 << 18;
  int32_t n_big = 0;
  while (n_big < n_protos && n_prim[order_p[n_big]] >= kBigProto) ++n_big;
  const int nthreads = std::min(nthreads_all, std::max(1, n_protos - n_big));
  std::atomic<int32_t> next{n_big};
  // capsules of every curve prototype (empty for quad meshes), in curve order
  std::vector<std::vector<Capsule>> caps(n_protos);
  for (int32_t p = 0; p < n_protos; ++p) {
    if (protos[p].n_curves == 0) continue;
    caps[p].resize((size_t)n_prim[p]);
    for (int32_t c = 0; c < protos[p].n_curves; ++c)
      tessellate_curve(protos[p].curves + 16 * (int64_t)c, &caps[p][(size_t)c * kCapsPerCurve],
                       protos[p].curves_flat != 0);
  }
  auto build_proto = [&](int32_t p, int threads, std::vector<Aabb>& boxes) {
    const rtq_prototype& P = protos[p];
    boxes.resize(n_prim[p]);
    for (int32_t k = 0; k < (int32_t)caps[p].size(); ++k) boxes[k] = capsule_box(caps[p][k]);
    for (int32_t q = 0; q < P.n_quads; ++q) {
      Aabb b;
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::numeric_limits<float>::infinity();
        b.hi[a] = -std::numeric_limits<float>::infinity();
      }
      for (int c = 0; c < 4; ++c) {
        const float* v = P.verts + 3 * (int64_t)P.quads[4 * (int64_t)q + c];
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = std::min(b.lo[a], v[a]);
          b.hi[a] = std::max(b.hi[a], v[a]);
        }
      }
      boxes[q] = b;
    }
    BuildParams pp = bp;
    pp.threads = threads;
    build_bvh(boxes.data(), n_prim[p], pp, blas[p]);
  };
  {
    std::vector<Aabb> boxes;
    for (int32_t k = 0; k < n_big; ++k) build_proto(order_p[k], nthreads_all, boxes);
  }
  auto worker = [&]() {
    std::vector<Aabb> boxes;
    for (;;) {
      const int32_t k = next.fetch_add(1);
      if (k >= n_protos) break;
      build_proto(order_p[k], 1, boxes);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
  }

  // owned by `holder` until the build succeeds: every failure below (an early
  // return or a host allocation failure thrown out of the builders) frees the
  // scene and its device buffers, and `tmp` frees itself
  std::unique_ptr<rtq_scene> holder(new rtq_scene);
  rtq_scene* s = holder.get();
  s->build_phase[0] = since(t0);
  auto t1 = std::chrono::steady_clock::now();
  s->device = dev;
  s->formats = formats;
  s->width = width;
  s->n_protos = n_protos;
  s->n_inst = N;
  s->n_quads = total_quads;
  s->n_curves = total_curves;
  s->n_caps = total_prims - total_quads;
  s->n_faces = total_faces;
  (void)hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (s->n_cu <= 0) s->n_cu = 256;
  (void)hipDeviceGetAttribute(&s->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (s->max_lds <= 0) s->max_lds = 65536;

  // ---- concatenate the bottom levels with absolute references
  std::vector<uint32_t> proto_root(n_protos), face_base(n_protos), proto_flags(n_protos);
  std::vector<int32_t> proto_qbase(n_protos), proto_nq(n_protos);
  std::vector<float> proto_pmax(n_protos);
  uint64_t node_base = 0, quad_base = 0, fbase = 0;
  int max_blas_depth = 0;
  for (int32_t p = 0; p < n_protos; ++p) {
    if (node_base + blas[p].nodes.size() >= (uint64_t)kLeafBit) {
      return set_error(RTQ_E_LIMIT, "bottom-level node count exceeds 2^31");
    }
    if (!relocate(blas[p], (uint32_t)node_base, (uint32_t)quad_base)) {
      return set_error(RTQ_E_LIMIT, "reference overflow while relocating prototype %d", p);
    }
    proto_root[p] = (uint32_t)node_base;
    face_base[p] = (uint32_t)fbase;  // faces: quads, or curves, in prototype order
    proto_flags[p] = protos[p].n_curves > 0 ? (kProtoCurve | (protos[p].curves_flat ? kProtoFlat : 0u)) : 0u;
    proto_qbase[p] = (int32_t)quad_base;
    proto_nq[p] = n_prim[p];
    proto_pmax[p] = level_pmax(blas[p]);
    if (!(proto_pmax[p] < kMaxPlaneAbs)) {
      return set_error(RTQ_E_LIMIT, "prototype %d has coordinates beyond 2^60", p);
    }
    max_blas_depth = std::max(max_blas_depth, blas[p].depth);
    node_base += blas[p].nodes.size();
    quad_base += n_prim[p];
    fbase += protos[p].n_curves > 0 ? protos[p].n_curves : protos[p].n_quads;
  }
  const size_t n_blas_nodes = node_base;
  std::vector<float4> quads(3 * (size_t)total_prims);
  std::vector<int32_t> quad_prim(total_prims);
  std::vector<float> albedo(total_faces);
  // world boxes of curve instances bound the corners of their capsules' boxes
  std::vector<float> cap_corners;
  std::vector<int64_t> corner_off(n_protos + 1, 0);
  for (int32_t p = 0; p < n_protos; ++p) corner_off[p + 1] = corner_off[p] + 8 * (int64_t)caps[p].size();
  cap_corners.resize(3 * (size_t)corner_off[n_protos]);
  for (int32_t p = 0; p < n_protos; ++p) {
    const rtq_prototype& P = protos[p];
    const size_t qb = proto_qbase[p];
    for (int32_t j = 0; j < (int32_t)caps[p].size(); ++j) {
      const uint32_t k = blas[p].order[j];
      const Capsule& c = caps[p][k];
      quads[3 * (qb + j) + 0] = make_float4(c.a[0], c.a[1], c.a[2], c.r);
      quads[3 * (qb + j) + 1] = make_float4(c.b[0], c.b[1], c.b[2], c.rb);
      quads[3 * (qb + j) + 2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      quad_prim[qb + j] = (int32_t)k;
      const Aabb bx = capsule_box(c);
      float* out = &cap_corners[3 * (size_t)(corner_off[p] + 8 * (int64_t)k)];
      for (int m = 0; m < 8; ++m) {
        out[3 * m + 0] = (m & 1) ? bx.hi[0] : bx.lo[0];
        out[3 * m + 1] = (m & 2) ? bx.hi[1] : bx.lo[1];
        out[3 * m + 2] = (m & 4) ? bx.hi[2] : bx.lo[2];
      }
    }
    for (int32_t c = 0; c < P.n_curves; ++c) albedo[face_base[p] + c] = P.albedo ? P.albedo[c] : 0.5f;
    caps[p] = std::vector<Capsule>();
    for (int32_t j = 0; j < P.n_quads; ++j) {
      const uint32_t q = blas[p].order[j];
      const int32_t* iq = P.quads + 4 * (int64_t)q;
      float f[12];
      for (int c = 0; c < 4; ++c)
        for (int a = 0; a < 3; ++a) f[3 * c + a] = P.verts[3 * (int64_t)iq[c] + a];
      quads[3 * (qb + j) + 0] = make_float4(f[0], f[1], f[2], f[3]);
      quads[3 * (qb + j) + 1] = make_float4(f[4], f[5], f[6], f[7]);
      quads[3 * (qb + j) + 2] = make_float4(f[8], f[9], f[10], f[11]);
      quad_prim[qb + j] = (int32_t)q;
    }
    for (int32_t q = 0; q < P.n_quads; ++q) albedo[face_base[p] + q] = P.albedo ? P.albedo[q] : 0.5f;
  }

#define UPLOAD(dst, src, bytes)                                                   \
  do {                                                                            \
    dst = reinterpret_cast<decltype(dst)>(s->bufs.alloc((bytes), &e));            \
    if (!dst) return hip_error(e, "hipMalloc");                                   \
    e = hipMemcpy((void*)dst, (src), (bytes), hipMemcpyHostToDevice);             \
    if (e != hipSuccess) return hip_error(e, "hipMemcpy");                        \
  } while (0)

  // bottom levels first; the top level is appended once it is built.  The host
  // nodes (exact FP32 boxes) stay until the instances are opened, which reads
  // their boxes.
  std::vector<WideNode> nw;
  std::vector<uint4> nq;
  nw.reserve(n_blas_nodes);
  if (formats & RTQ_NODE_Q8) nq.reserve(n_blas_nodes * q8_stride(width));
  for (int32_t p = 0; p < n_protos; ++p) {
    nw.insert(nw.end(), blas[p].nodes.begin(), blas[p].nodes.end());
    if (formats & RTQ_NODE_Q8) nq.insert(nq.end(), blas[p].q8.begin(), blas[p].q8.end());
    blas[p] = Bvh{};  // release host memory early
  }
  UPLOAD(s->quads, quads.data(), quads.size() * sizeof(float4));
  UPLOAD(s->quad_prim, quad_prim.data(), quad_prim.size() * sizeof(int32_t));
  UPLOAD(s->albedo, albedo.data(), albedo.size() * sizeof(float));
  s->blas_nodes = (int64_t)n_blas_nodes;
  s->blas_depth = max_blas_depth;
  quads = std::vector<float4>();
  quad_prim = std::vector<int32_t>();

  // ---- instances: FP64 inverses and padded world boxes on the device
  const int64_t Nn = std::max<int64_t>(N, 1);
  float* d_x = nullptr;
  int32_t* d_proto = nullptr;
  uint32_t *d_root = nullptr, *d_face = nullptr;
  float *d_verts = nullptr, *d_cond = nullptr, *d_box = nullptr;
  int64_t* d_voff = nullptr;
  int32_t* d_status = nullptr;
  InstRec* d_rec = nullptr;
  DeviceBuffers tmp;
#define TALLOC(dst, bytes)                                                         \
  do {                                                                             \
    dst = reinterpret_cast<decltype(dst)>(tmp.alloc((bytes), &e));                 \
    if (!dst) return hip_error(e, "hipMalloc");                                    \
  } while (0)
#define TCHECK(expr, what)                                                         \
  do {                                                                             \
    e = (expr);                                                                    \
    if (e != hipSuccess) return hip_error(e, what);                                \
  } while (0)
  TALLOC(d_x, 12 * Nn * sizeof(float));
  TALLOC(d_proto, Nn * sizeof(int32_t));
  TALLOC(d_root, n_protos * sizeof(uint32_t));
  TALLOC(d_face, n_protos * sizeof(uint32_t));
  uint32_t* d_pflags = nullptr;
  TALLOC(d_pflags, n_protos * sizeof(uint32_t));
  // points whose transformed bounds give an instance's world box: the mesh's
  // vertices, or the corners of the capsules' boxes
  std::vector<int64_t> vert_off(n_protos + 1, 0);
  for (int32_t p = 0; p < n_protos; ++p)
    vert_off[p + 1] = vert_off[p] + (protos[p].n_curves > 0 ? corner_off[p + 1] - corner_off[p] : protos[p].n_verts);
  TALLOC(d_verts, std::max<int64_t>(3 * vert_off[n_protos], 1) * sizeof(float));
  TALLOC(d_voff, (n_protos + 1) * sizeof(int64_t));
  TALLOC(d_cond, Nn * sizeof(float));
  TALLOC(d_box, 6 * Nn * sizeof(float));
  TALLOC(d_status, Nn * sizeof(int32_t));
  TALLOC(d_rec, Nn * sizeof(InstRec));
  if (N > 0) {
    TCHECK(hipMemcpy(d_x, insts->xform, 12 * N * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    TCHECK(hipMemcpy(d_proto, insts->proto, N * sizeof(int32_t), hipMemcpyHostToDevice), "hipMemcpy");
  }
  TCHECK(hipMemcpy(d_root, proto_root.data(), n_protos * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
  TCHECK(hipMemcpy(d_face, face_base.data(), n_protos * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
  TCHECK(hipMemcpy(d_pflags, proto_flags.data(), n_protos * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
  for (int32_t p = 0; p < n_protos; ++p) {
    const int64_t nv = vert_off[p + 1] - vert_off[p];
    if (nv == 0) continue;
    const float* src = protos[p].n_curves > 0 ? &cap_corners[3 * (size_t)corner_off[p]] : protos[p].verts;
    TCHECK(hipMemcpy(d_verts + 3 * vert_off[p], src, 3 * (size_t)nv * sizeof(float), hipMemcpyHostToDevice),
           "hipMemcpy");
  }
  cap_corners = std::vector<float>();
  TCHECK(hipMemcpy(d_voff, vert_off.data(), (n_protos + 1) * sizeof(int64_t), hipMemcpyHostToDevice), "hipMemcpy");
  TCHECK(launch_invert_affine(d_x, d_proto, d_root, d_face, d_pflags, N, d_rec, d_cond, d_status, 0),
         "invert kernel");
  TCHECK(launch_instance_aabb(d_x, d_proto, d_verts, d_voff, d_cond, N, d_box, 0), "aabb kernel");
  std::vector<int32_t> status(N);
  std::vector<float> cond(N);
  std::vector<Aabb> boxes(N);
  if (N > 0) {
    TCHECK(hipMemcpy(status.data(), d_status, N * sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy");
    TCHECK(hipMemcpy(cond.data(), d_cond, N * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    TCHECK(hipMemcpy(boxes.data(), d_box, 6 * N * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  }
  float cond_max = 1.0f;
  for (int64_t i = 0; i < N; ++i) {
    if (status[i]) {
      const int code = set_error(RTQ_E_SINGULAR_XFORM, "instance %lld has a singular transform", (long long)i);
      return code;
    }
    cond_max = std::max(cond_max, cond[i]);
  }
  s->pad_rel = std::ldexp(1.0f, -17) * cond_max;

  s->build_phase[1] = since(t1);
  t1 = std::chrono::steady_clock::now();
  // ---- top-level entries: every instance, large ones opened into subtrees.
  // The host pad bound uses the padded box, so it is at least the device's.
  std::vector<TopEntry> entries;
  {
    std::vector<double> pad(N);
    for (int64_t i = 0; i < N; ++i) {
      const float* x = insts->xform + 12 * i;
      double mag = std::max(std::max(std::fabs((double)x[3]), std::fabs((double)x[7])), std::fabs((double)x[11]));
      for (int r = 0; r < 3; ++r)
        mag = std::max(mag, std::max(std::fabs((double)boxes[i].lo[r]), std::fabs((double)boxes[i].hi[r])));
      pad[i] = std::ldexp(1.0, -17) * (double)cond[i] * mag;
    }
    OpenParams op;
    const int32_t pct = o.open_pct == 0 ? kDefaultOpenPct : std::max(o.open_pct, 0);
    if (o.open_area_pct) op.max_ratio = o.open_area_pct / 100.0;
    op.budget = std::min<int64_t>(N * (int64_t)pct / 100, (int64_t)kMaxLeafFirst - N);
    op.threads = nthreads_all;
    entries = open_instances(N, insts->xform, insts->proto, boxes.data(), pad.data(), proto_root, proto_qbase,
                             proto_nq, nw, op);
  }
  const int64_t E = (int64_t)entries.size();
  s->n_rec = E;
  std::vector<NodeF32> nf;
  if (formats & RTQ_NODE_FP32) {
    nf.resize(nw.size());
    for (size_t i = 0; i < nw.size(); ++i) nf[i] = pack_f32(nw[i]);
  }
  nw = std::vector<WideNode>();
  s->build_phase[2] = since(t1);
  t1 = std::chrono::steady_clock::now();

  // ---- top level over the padded entry boxes (one entry per leaf)
  Bvh tlas;
  BuildParams tp = bp;
  tp.leaf_max = 1;
  // one box per entry: finer bins pay off at the top level (256 against 64:
  // 1.3 % off the config-2 frame); jobs smaller than that use fewer
  tp.bins = std::max(bp.bins, 256);
  tp.threads = nthreads_all;
  if (E > 0) {
    std::vector<Aabb> eb(E);
    for (int64_t k = 0; k < E; ++k) eb[k] = entries[k].box;
    boxes = std::vector<Aabb>();
    build_bvh(eb.data(), E, tp, tlas);
  } else {
    Aabb none;
    for (int a = 0; a < 3; ++a) none.lo[a] = none.hi[a] = 0.0f;
    build_bvh(&none, 1, tp, tlas);  // placeholder root; n_rec = 0 makes every ray miss first
  }
  if (n_blas_nodes + tlas.nodes.size() >= (uint64_t)kLeafBit)
    return set_error(RTQ_E_LIMIT, "node count exceeds 2^31");
  if (!relocate(tlas, (uint32_t)n_blas_nodes, 0u))
    return set_error(RTQ_E_LIMIT, "top-level reference overflow");
  if ((width - 1) * (tlas.depth + max_blas_depth) + 8 > kStackTotal)
    return set_error(RTQ_E_LIMIT, "BVH depth %d + %d exceeds the traversal stack", tlas.depth, max_blas_depth);
  s->p_world = level_pmax(tlas);
  if (!(s->p_world < kMaxPlaneAbs)) return set_error(RTQ_E_LIMIT, "instance boxes reach beyond 2^60");
  s->tlas_root = (uint32_t)n_blas_nodes;
  s->tlas_depth = tlas.depth;
  s->tlas_nodes = (int64_t)tlas.nodes.size();
  if (formats & RTQ_NODE_FP32) {
    for (const WideNode& w : tlas.nodes) nf.push_back(pack_f32(w));
    UPLOAD(s->nodes_f32, nf.data(), nf.size() * sizeof(NodeF32));
    nf = std::vector<NodeF32>();
  }
  if (formats & RTQ_NODE_Q8) {
    nq.insert(nq.end(), tlas.q8.begin(), tlas.q8.end());
    UPLOAD(s->nodes_q8, nq.data(), nq.size() * sizeof(uint4));
    nq = std::vector<uint4>();
  }
  // records in top-level leaf order
  const int64_t En = std::max<int64_t>(E, 1);
  {
    std::vector<float> rec_pmax(En, 0.0f);
    std::vector<uint32_t> rec_qfirst(En, 0u), rec_nq(En, 0u), order(En, 0u), root(En, 0u);
    for (int64_t r = 0; r < E; ++r) {
      const TopEntry& t = entries[tlas.order[r]];
      rec_pmax[r] = proto_pmax[insts->proto[t.inst]];
      rec_qfirst[r] = t.q_first;
      rec_nq[r] = t.q_count;
      order[r] = t.inst;
      root[r] = t.ref;
    }
    entries = std::vector<TopEntry>();
    UPLOAD(s->rec_pmax, rec_pmax.data(), rec_pmax.size() * sizeof(float));
    UPLOAD(s->rec_qfirst, rec_qfirst.data(), rec_qfirst.size() * sizeof(uint32_t));
    UPLOAD(s->rec_nq, rec_nq.data(), rec_nq.size() * sizeof(uint32_t));
    s->inst = reinterpret_cast<InstRec*>(s->bufs.alloc(En * sizeof(InstRec), &e));
    if (!s->inst) return hip_error(e, "hipMalloc");
    if (E > 0) {
      uint32_t *d_order, *d_eroot;
      TALLOC(d_order, E * sizeof(uint32_t));
      TALLOC(d_eroot, E * sizeof(uint32_t));
      TCHECK(hipMemcpy(d_order, order.data(), E * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
      TCHECK(hipMemcpy(d_eroot, root.data(), E * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy");
      TCHECK(launch_gather_inst(d_rec, d_order, d_eroot, E, s->inst, 0), "gather kernel");
    }
  }
  s->counters = reinterpret_cast<unsigned long long*>(
      s->bufs.alloc((size_t)rtq_scene::kCounterSlots * kClaimWords * sizeof(unsigned long long), &e));
  if (!s->counters) return hip_error(e, "hipMalloc");
  TCHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
  tmp.release();
  for (int64_t i = 0; i < N; ++i) s->n_instanced_quads += protos[insts->proto[i]].n_quads;  // quads only
  s->build_phase[3] = since(t1);
  s->build_seconds = since(t0);
  *out = holder.release();
  return RTQ_OK;
#undef UPLOAD
#undef TALLOC
#undef TCHECK
}

int rtq_scene_build(const rtq_prototype* protos, int32_t n_protos, const rtq_instances* insts,
                    const rtq_build_opts* opts, rtq_scene** out) {
  try {
    return build_impl(protos, n_protos, insts, opts, out);
  } catch (const std::bad_alloc&) {
    return set_error(RTQ_E_OOM, "host allocation failed during build");
  } catch (...) {
    return set_error(RTQ_E_HIP, "unexpected failure during build");
  }
}

void rtq_scene_destroy(rtq_scene* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  release_render_scratch(s);
  s->bufs.release();
  if (s->tex) (void)hipFree(s->tex);
  if (s->env) (void)hipFree(s->env);
  if (s->env_T) (void)hipFree(s->env_T);
  if (s->mats) (void)hipFree(s->mats);
  if (s->face_mat) (void)hipFree(s->face_mat);
  delete s;
}

int rtq_scene_get_info(const rtq_scene* s, rtq_scene_info* info) {
  if (!s || !info) return set_error(RTQ_E_INVALID_ARG, "NULL argument");
  info->n_instances = s->n_inst;
  info->n_prototypes = s->n_protos;
  info->n_unique_quads = s->n_quads;
  info->n_instanced_quads = s->n_instanced_quads;
  info->tlas_nodes = s->tlas_nodes;
  info->blas_nodes = s->blas_nodes;
  info->tlas_depth = s->tlas_depth;
  info->blas_depth_max = s->blas_depth;
  info->formats = s->formats;
  info->node_width = s->width;
  info->n_unique_curves = s->n_curves;
  info->n_unique_capsules = s->n_caps;
  info->n_faces = s->n_faces;
  info->device_bytes = (int64_t)(s->bufs.total + s->scratch.total + s->tex_bytes + s->env_bytes + s->mat_bytes);
  info->build_seconds = s->build_seconds;
  info->n_top_entries = s->n_rec;
  for (int k = 0; k < 4; ++k) info->build_phase_seconds[k] = s->build_phase[k];
  return RTQ_OK;
}

int rtq_scene_set_albedo(rtq_scene* s, const float* albedo_dev, int64_t n, hipStream_t stream) {
  if (!s || !albedo_dev) return set_error(RTQ_E_INVALID_ARG, "NULL argument");
  if (n != s->n_faces)
    return set_error(RTQ_E_INVALID_ARG, "albedo has %lld entries, scene has %lld faces", (long long)n,
                     (long long)s->n_faces);
  const hipError_t e = hipMemcpyAsync(s->albedo, albedo_dev, n * sizeof(float), hipMemcpyDeviceToDevice, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "hipMemcpyAsync");
}

int rtq_scene_set_materials(rtq_scene* s, const rtq_material* mats, int32_t n_mat, const uint8_t* face_mat_dev,
                            hipStream_t stream) {
  if (!s) return set_error(RTQ_E_INVALID_ARG, "NULL scene");
  if (n_mat < 0 || n_mat > RTQ_MAX_MATERIALS)
    return set_error(RTQ_E_INVALID_ARG, "%d materials outside [0, %d]", n_mat, RTQ_MAX_MATERIALS);
  if (n_mat > 0 && (!mats || !face_mat_dev)) return set_error(RTQ_E_INVALID_ARG, "NULL materials or face indices");
  std::vector<MatDev> md(n_mat);
  auto in01 = [](float x) { return x >= 0.0f && x <= 1.0f; };
  for (int32_t k = 0; k < n_mat; ++k) {
    const rtq_material& m = mats[k];
    if (!in01(m.tint[0]) || !in01(m.tint[1]) || !in01(m.tint[2]) || !(m.roughness >= 0.05f && m.roughness <= 1.0f) ||
        !in01(m.metallic) || !in01(m.specular) || !in01(m.clearcoat) ||
        (m.clearcoat > 0.0f && !(m.clearcoat_roughness >= 0.05f && m.clearcoat_roughness <= 1.0f)))
      return set_error(RTQ_E_INVALID_ARG, "material %d: parameter outside its range", k);
    md[k].tint[0] = m.tint[0];
    md[k].tint[1] = m.tint[1];
    md[k].tint[2] = m.tint[2];
    md[k].alpha = m.roughness * m.roughness;
    md[k].metal = m.metallic;
    md[k].spec = m.specular;
    md[k].coat = m.clearcoat;
    md[k].calpha = m.clearcoat > 0.0f ? m.clearcoat_roughness * m.clearcoat_roughness : 0.0f;
  }
  hipError_t e = hipSetDevice(s->device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  // renders already queued may still read the old materials
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  (void)stream;
  std::vector<uint8_t> fm;
  if (n_mat > 0) {
    fm.resize(s->n_faces);
    e = hipMemcpy(fm.data(), face_mat_dev, s->n_faces, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_error(e, "hipMemcpy");
    for (int64_t f = 0; f < s->n_faces; ++f)
      if (fm[f] >= n_mat) return set_error(RTQ_E_INVALID_ARG, "face %lld: material %d >= %d", (long long)f, fm[f], n_mat);
  }
  if (s->mats) (void)hipFree(s->mats);
  if (s->face_mat) (void)hipFree(s->face_mat);
  s->mats = nullptr;
  s->face_mat = nullptr;
  s->n_mat = 0;
  s->mat_bytes = 0;
  if (n_mat == 0) return RTQ_OK;
  void* dm = nullptr;
  void* df = nullptr;
  e = hipMalloc(&dm, n_mat * sizeof(MatDev));
  if (e == hipSuccess) e = hipMalloc(&df, (size_t)s->n_faces);
  if (e == hipSuccess) e = hipMemcpy(dm, md.data(), n_mat * sizeof(MatDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(df, fm.data(), (size_t)s->n_faces, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (dm) (void)hipFree(dm);
    if (df) (void)hipFree(df);
    return hip_error(e, "material upload");
  }
  s->mats = dm;
  s->face_mat = static_cast<uint8_t*>(df);
  s->n_mat = n_mat;
  s->mat_bytes = n_mat * sizeof(MatDev) + (size_t)s->n_faces;
  return RTQ_OK;
}

int rtq_scene_set_textures(rtq_scene* s, const float* texels_dev, int32_t res, int32_t channels,
                           hipStream_t stream) {
  if (!s) return set_error(RTQ_E_INVALID_ARG, "NULL scene");
  if (res < 0 || res > RTQ_MAX_TEX_RES)
    return set_error(RTQ_E_INVALID_ARG, "texture resolution %d outside [0, %d]", res, RTQ_MAX_TEX_RES);
  if (channels != 1 && channels != 3) return set_error(RTQ_E_INVALID_ARG, "%d texel channels (1 or 3)", channels);
  if (res > 0 && !texels_dev) return set_error(RTQ_E_INVALID_ARG, "NULL texels");
  if (res > 0 && s->n_curves > 0)
    return set_error(RTQ_E_INVALID_ARG, "textures need (u, v) squares: the scene has curves");
  hipError_t e = hipSetDevice(s->device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  // renders already queued may still read the old texels
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  const size_t bytes = (size_t)s->n_quads * (size_t)res * (size_t)res * (size_t)channels * sizeof(float);
  if (res == 0 || bytes != s->tex_bytes) {
    if (s->tex) (void)hipFree(s->tex);
    s->tex = nullptr;
    s->tex_res = 0;
    s->tex_ch = 1;
    s->tex_bytes = 0;
    if (res == 0) return RTQ_OK;
    e = hipMalloc(reinterpret_cast<void**>(&s->tex), bytes);
    if (e != hipSuccess) {
      s->tex = nullptr;
      return hip_error(e, "texture allocation");
    }
    s->tex_bytes = bytes;
  }
  e = hipMemcpyAsync(s->tex, texels_dev, bytes, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync");
  s->tex_res = res;
  s->tex_ch = channels;
  return RTQ_OK;
}

int rtq_scene_set_environment(rtq_scene* s, const float* texels_dev, int32_t w, int32_t h, hipStream_t stream) {
  if (!s) return set_error(RTQ_E_INVALID_ARG, "NULL scene");
  if (w < 0 || w > RTQ_MAX_ENV_SIDE || (w > 0 && (h < 1 || h > RTQ_MAX_ENV_SIDE)))
    return set_error(RTQ_E_INVALID_ARG, "environment map %d x %d outside [1, %d]^2", w, h, RTQ_MAX_ENV_SIDE);
  if (w > 0 && !texels_dev) return set_error(RTQ_E_INVALID_ARG, "NULL environment texels");
  hipError_t e = hipSetDevice(s->device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  // renders already queued may still read the old map
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  const size_t n = w > 0 ? (size_t)w * (size_t)h : 0;
  const size_t bytes = n * sizeof(float);
  if (s->env) (void)hipFree(s->env);
  if (s->env_T) (void)hipFree(s->env_T);
  s->env = nullptr;
  s->env_T = nullptr;
  s->env_w = s->env_h = 0;
  s->env_bytes = 0;
  if (w == 0) return RTQ_OK;
  // the sampling table of next-event estimation toward the map: texel
  // k = ty w + tx has weight L_k Omega_ty, Omega_ty = (2 pi / w)
  // (cos(pi ty / h) - cos(pi (ty + 1) / h)) its solid angle; T_k =
  // floor(2^32 C_k / C_total) with C the running FP64 sum in texel order, the
  // last entry 2^32; texel k is drawn with probability (T_k - T_{k-1}) / 2^32
  std::vector<float> host(n);
  e = hipMemcpy(host.data(), texels_dev, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "environment read-back");
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(host[k]) || host[k] < 0.0f)
      return set_error(RTQ_E_INVALID_ARG, "environment texel %zu is negative or not finite", k);
  std::vector<double> omega(h);
  for (int32_t ty = 0; ty < h; ++ty)
    omega[ty] = (2.0 * 3.14159265358979323846 / w) *
                (std::cos(3.14159265358979323846 * ty / h) - std::cos(3.14159265358979323846 * (ty + 1) / h));
  double total = 0.0;
  for (size_t k = 0; k < n; ++k) total += (double)host[k] * omega[k / w];
  std::vector<unsigned long long> T(n);
  double cum = 0.0;
  for (size_t k = 0; k < n; ++k) {
    cum += (double)host[k] * omega[k / w];
    T[k] = total > 0.0 ? (unsigned long long)std::floor(std::ldexp(cum / total, 32))
                       : (unsigned long long)((double)(k + 1) * 4294967296.0 / (double)n);
  }
  T[n - 1] = 1ull << 32;
  e = hipMalloc(reinterpret_cast<void**>(&s->env), bytes);
  if (e != hipSuccess) {
    s->env = nullptr;
    return hip_error(e, "environment allocation");
  }
  e = hipMalloc(reinterpret_cast<void**>(&s->env_T), n * sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipFree(s->env);
    s->env = nullptr;
    s->env_T = nullptr;
    return hip_error(e, "environment table allocation");
  }
  s->env_bytes = bytes + n * sizeof(unsigned long long);
  e = hipMemcpy(s->env, host.data(), bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->env_T, T.data(), n * sizeof(unsigned long long), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "environment upload");
  (void)stream;
  s->env_w = w;
  s->env_h = h;
  return RTQ_OK;
}

static int check_rays(const rtq_scene* s, const rtq_rays* r, int64_t n) {
  if (!s || !r) return set_error(RTQ_E_INVALID_ARG, "NULL scene or rays");
  if (n < 0) return set_error(RTQ_E_INVALID_ARG, "negative ray count");
  // a dispatch counts its work-items in 32 bits (one ray per lane in the plain kernels)
  if (n > (int64_t)0x7FFFFFFF) return set_error(RTQ_E_LIMIT, "%lld rays per call exceed 2^31 - 1", (long long)n);
  if (n > 0 && (!r->ox || !r->oy || !r->oz || !r->dx || !r->dy || !r->dz || !r->tmin || !r->tmax))
    return set_error(RTQ_E_INVALID_ARG, "NULL ray array");
  return RTQ_OK;
}

static RaysSoA soa(const rtq_rays* r) {
  return RaysSoA{r->ox, r->oy, r->oz, r->dx, r->dy, r->dz, r->tmin, r->tmax, r->exclude};
}

static int trace_common(const rtq_scene* s, const rtq_rays* rays, int64_t n, rtq_hits* hits, uint8_t* occ,
                        const rtq_trace_opts* opts, hipStream_t stream) {
  int rc = check_rays(s, rays, n);
  if (rc) return rc;
  rtq_trace_opts o{};
  if (opts) o = *opts;
  int fmt;
  if ((rc = resolve_format(s, o.node_format, &fmt))) return rc;
  TraceLaunch tl;
  if ((rc = resolve_launch(s, o.scheduler, o.stack_depth, o.block, o.waves_per_cu, o.refill, &tl))) return rc;
  tl.fmt = fmt;
  if (n == 0) return RTQ_OK;
  const SceneView sv = scene_view(s, fmt);
  HitsSoA h{};
  if (hits) h = HitsSoA{hits->t, hits->u, hits->v, hits->inst, hits->prim, hits->ref};
  const hipError_t e = launch_trace(sv, soa(rays), n, hits ? &h : nullptr, occ, o.visits, o.lane_stats, tl, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "trace launch");
}

int rtq_trace_closest(const rtq_scene* s, const rtq_rays* rays, int64_t n, rtq_hits* hits, const rtq_trace_opts* opts,
                      hipStream_t stream) {
  if (!hits) return set_error(RTQ_E_INVALID_ARG, "NULL hits");
  if (n > 0 && (!hits->t || !hits->u || !hits->v || !hits->inst || !hits->prim))
    return set_error(RTQ_E_INVALID_ARG, "NULL hit array");
  return trace_common(s, rays, n, hits, nullptr, opts, stream);
}

int rtq_trace_closest_noalloc(const rtq_scene* s, const rtq_rays* rays, int64_t n, rtq_hits* hits,
                              const rtq_trace_opts* opts, hipStream_t stream) {
  if (!hits) return set_error(RTQ_E_INVALID_ARG, "NULL hits");
  if (n > 0 && (!hits->t || !hits->u || !hits->v || !hits->inst || !hits->prim))
    return set_error(RTQ_E_INVALID_ARG, "NULL hit array");
  int rc = check_rays(s, rays, n);
  if (rc) return rc;
  rtq_trace_opts o{};
  if (opts) o = *opts;
  int fmt;
  if ((rc = resolve_format(s, o.node_format, &fmt))) return rc;
  TraceLaunch tl;
  if ((rc = resolve_launch(s, RTQ_SCHED_PERSISTENT, o.stack_depth, o.block, o.waves_per_cu, o.refill, &tl)))
    return rc;
  tl.fmt = fmt;
  unsigned long long* ctr = nullptr;
  hipError_t e = noalloc_counters(s->device, &ctr);
  if (e != hipSuccess) return hip_error(e, "claim counter address (hipGetSymbolAddress)");
  tl.counter = ctr;  // in place of the scene's counter ring; cleared by a fill kernel before the launch
  if (n == 0) return RTQ_OK;
  const SceneView sv = scene_view(s, fmt);
  const HitsSoA h{hits->t, hits->u, hits->v, hits->inst, hits->prim, hits->ref};
  e = launch_trace(sv, soa(rays), n, &h, nullptr, o.visits, o.lane_stats, tl, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "trace launch");
}

int rtq_trace_occluded(const rtq_scene* s, const rtq_rays* rays, int64_t n, uint8_t* occluded,
                       const rtq_trace_opts* opts, hipStream_t stream) {
  if (n > 0 && !occluded) return set_error(RTQ_E_INVALID_ARG, "NULL occluded array");
  return trace_common(s, rays, n, nullptr, occluded, opts, stream);
}

int rtq_host_bvh_build(const float* boxes, int64_t n, int32_t leaf_max, int32_t bins, int32_t threads,
                       int32_t width, rtq_host_bvh** out) {
  if (!out) return set_error(RTQ_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!boxes || n < 1) return set_error(RTQ_E_INVALID_ARG, "need at least one box");
  if (n > (int64_t)kMaxLeafFirst) return set_error(RTQ_E_LIMIT, "%lld boxes exceed 2^28", (long long)n);
  if (leaf_max < 1 || leaf_max > 8) return set_error(RTQ_E_INVALID_ARG, "leaf_max %d outside [1, 8]", leaf_max);
  if (bins < 4 || bins > 64) return set_error(RTQ_E_INVALID_ARG, "bins %d outside [4, 64]", bins);
  if (width != 2 && width != 4 && width != 8) return set_error(RTQ_E_INVALID_ARG, "width %d is not 2, 4 or 8", width);
  try {
    std::vector<Aabb> b(n);
    for (int64_t i = 0; i < n; ++i) {
      for (int a = 0; a < 3; ++a) {
        b[i].lo[a] = boxes[6 * i + a];
        b[i].hi[a] = boxes[6 * i + 3 + a];
        if (!std::isfinite(b[i].lo[a]) || !std::isfinite(b[i].hi[a]) || b[i].lo[a] > b[i].hi[a])
          return set_error(RTQ_E_INVALID_ARG, "box %lld is not finite or is inverted", (long long)i);
      }
    }
    BuildParams p;
    p.leaf_max = leaf_max;
    p.bins = bins;
    p.width = width;
    p.threads = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    std::unique_ptr<rtq_host_bvh> h(new rtq_host_bvh);
    build_bvh(b.data(), n, p, h->bvh);
    if (width == 4) {
      h->f32.resize(h->bvh.nodes.size());
      for (size_t i = 0; i < h->bvh.nodes.size(); ++i) h->f32[i] = pack_f32(h->bvh.nodes[i]);
    }
    *out = h.release();
    return RTQ_OK;
  } catch (const std::bad_alloc&) {
    return set_error(RTQ_E_OOM, "host allocation failed");
  }
}

int rtq_host_bvh_get(const rtq_host_bvh* h, const void** nodes_wide, const void** nodes_f32, const void** nodes_q8,
                     int64_t* n_nodes, const uint32_t** order, int32_t* depth) {
  if (!h) return set_error(RTQ_E_INVALID_ARG, "NULL bvh");
  if (nodes_wide) *nodes_wide = h->bvh.nodes.data();
  if (nodes_f32) *nodes_f32 = h->f32.empty() ? nullptr : h->f32.data();
  if (nodes_q8) *nodes_q8 = h->bvh.q8.data();
  if (n_nodes) *n_nodes = (int64_t)h->bvh.nodes.size();
  if (order) *order = h->bvh.order.data();
  if (depth) *depth = h->bvh.depth;
  return RTQ_OK;
}

void rtq_host_bvh_destroy(rtq_host_bvh* h) { delete h; }

int rtq_trace_brute(const rtq_scene* s, const rtq_rays* rays, int64_t n, rtq_hits* hits, hipStream_t stream) {
  int rc = check_rays(s, rays, n);
  if (rc) return rc;
  if (!hits || (n > 0 && (!hits->t || !hits->u || !hits->v || !hits->inst || !hits->prim)))
    return set_error(RTQ_E_INVALID_ARG, "NULL hit array");
  int fmt = 0;
  if ((rc = resolve_format(s, 0, &fmt))) return rc;
  const SceneView sv = scene_view(s, fmt);
  const HitsSoA h{hits->t, hits->u, hits->v, hits->inst, hits->prim, hits->ref};
  const hipError_t e = launch_trace_brute(sv, soa(rays), n, h, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "brute launch");
}

}  // extern "C"
