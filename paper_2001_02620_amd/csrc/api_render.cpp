// Rendering entry points of the C-ABI: camera set-up, scratch management and the
// dispatch to the plain (multi-kernel) or persistent (single-launch) scheduler,
// and the path-replay adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/rtq.h"
#include "api_internal.h"
#include "render_kernels.h"

using namespace rtq;

namespace {

// A captured render call: the graph of its launches and the claim counters its
// persistent launches use (its own, so replays never share counters with eager
// calls).
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  unsigned long long* counter = nullptr;
};

struct RenderScratch {
  DeviceBuffers bufs;
  int64_t paths_cap = 0;
  bool plain = false;
  bool rgb = false;  // three radiance slots per path and RGB queue channels
  int32_t cams_cap = 0;
  CamDev* cams = nullptr;
  float* slots = nullptr;
  uint32_t* keys = nullptr;  // [3] RNG key and accumulated frames of the current call
  float* alights = nullptr;  // RTQ_MAX_AREA_LIGHTS x 10: area lights of the current call
  PlainBuffers pb{};
  // captured calls, keyed by everything their launches bake in
  std::unordered_map<std::string, GraphEntry> graphs;
  DeviceBuffers graph_bufs;
  hipStream_t capture_stream = nullptr;
  void clear_graphs() {
    for (auto& kv : graphs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
    graph_bufs.release();
  }
};

}  // namespace

namespace rtq {
// Events recorded around the launches of timed render calls.  Events are pooled
// and reused after a query; the pool is capped so that a caller who never queries
// cannot grow it without bound.
struct StageLog {
  static constexpr size_t kMaxEvents = 4096;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> all, free_list;
  std::vector<Rec> recs;
  hipEvent_t call_first = nullptr, call_last = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> calls;
  int dropped = 0;
  hipEvent_t take() {
    if (!free_list.empty()) {
      hipEvent_t e = free_list.back();
      free_list.pop_back();
      return e;
    }
    if (all.size() >= kMaxEvents) return nullptr;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    all.push_back(e);
    return e;
  }
  ~StageLog() {
    for (hipEvent_t e : all) (void)hipEventDestroy(e);
  }
};

hipEvent_t stage_begin(StageLog* log, hipStream_t s) {
  if (!log) return nullptr;
  hipEvent_t e = log->take();
  if (!e) {
    ++log->dropped;
    return nullptr;
  }
  (void)hipEventRecord(e, s);
  if (!log->call_first) log->call_first = e;
  return e;
}

void stage_end(StageLog* log, int stage, hipEvent_t begin, hipStream_t s) {
  if (!log || !begin) return;
  hipEvent_t e = log->take();
  if (!e) {
    ++log->dropped;
    return;
  }
  (void)hipEventRecord(e, s);
  log->recs.push_back({stage, begin, e});
  log->call_last = e;
}
}  // namespace rtq

namespace {

RenderScratch* scratch_of(rtq_scene* s) {
  if (!s->render_state) s->render_state = new RenderScratch;
  return static_cast<RenderScratch*>(s->render_state);
}

// Grow the scene's render scratch to hold n_paths paths (and the plain
// scheduler's queues when asked).  Existing contents are not preserved.
int ensure_scratch(rtq_scene* s, int64_t n_paths, int32_t n_cams, bool plain, bool rgb) {
  RenderScratch* r = scratch_of(s);
  if (r->paths_cap >= n_paths && r->cams_cap >= n_cams && (r->plain || !plain) && (r->rgb || !rgb)) return RTQ_OK;
  (void)hipDeviceSynchronize();
  r->clear_graphs();  // their launches point into the buffers released here
  r->bufs.release();
  const int64_t P = std::max<int64_t>(std::max(n_paths, r->paths_cap), 64);
  const int32_t C = std::max(std::max(n_cams, r->cams_cap), 64);
  const bool want_plain = plain || r->plain;
  const bool want_rgb = rgb || r->rgb;
  hipError_t e;
  auto A = [&](size_t bytes) { return r->bufs.alloc(bytes, &e); };
#define RALLOC(dst, bytes)                                              \
  do {                                                                  \
    dst = reinterpret_cast<decltype(dst)>(A(bytes));                    \
    if (!dst) {                                                         \
      r->bufs.release();                                                \
      r->paths_cap = 0;                                                 \
      r->cams_cap = 0;                                                  \
      r->plain = false;                                                 \
      r->rgb = false;                                                   \
      return hip_error(e, "render scratch allocation");                 \
    }                                                                   \
  } while (0)
  RALLOC(r->cams, C * sizeof(CamDev));
  RALLOC(r->slots, (want_rgb ? 3 : 1) * P * sizeof(float));
  RALLOC(r->keys, 64);
  RALLOC(r->alights, RTQ_MAX_AREA_LIGHTS * 10 * sizeof(float));
  if (want_plain) {
    for (int k = 0; k < 2; ++k) {
      ExtQueue& q = r->pb.q[k];
      RALLOC(q.ox, P * 4);
      RALLOC(q.oy, P * 4);
      RALLOC(q.oz, P * 4);
      RALLOC(q.dx, P * 4);
      RALLOC(q.dy, P * 4);
      RALLOC(q.dz, P * 4);
      RALLOC(q.pid, P * 4);
      RALLOC(q.beta, P * 4);
      RALLOC(q.ex_rec, P * 4);
      RALLOC(q.ex_qh, P * 4);
      RALLOC(q.pdf, P * 4);
      if (want_rgb) {
        RALLOC(q.beta_g, P * 4);
        RALLOC(q.beta_b, P * 4);
      } else {
        q.beta_g = q.beta_b = nullptr;
      }
    }
    ShadowQueue& sq = r->pb.sq;
    RALLOC(sq.ox, P * 4);
    RALLOC(sq.oy, P * 4);
    RALLOC(sq.oz, P * 4);
    RALLOC(sq.pid, P * 4);
    RALLOC(sq.contrib, P * 4);
    RALLOC(sq.ex_rec, P * 4);
    RALLOC(sq.ex_qh, P * 4);
    RALLOC(sq.dx, P * 4);
    RALLOC(sq.dy, P * 4);
    RALLOC(sq.dz, P * 4);
    RALLOC(sq.tmax, P * 4);
    if (want_rgb) {
      RALLOC(sq.contrib_g, P * 4);
      RALLOC(sq.contrib_b, P * 4);
    } else {
      sq.contrib_g = sq.contrib_b = nullptr;
    }
    RALLOC(r->pb.hits.t, P * 4);
    RALLOC(r->pb.hits.rec, P * 4);
    RALLOC(r->pb.hits.qh, P * 4);
    RALLOC(r->pb.hits.u, P * 4);
    RALLOC(r->pb.hits.v, P * 4);
    RALLOC(r->pb.occ, P);
    RALLOC(r->pb.counts, (2 * kMaxDepth + 2) * sizeof(uint32_t));
    RALLOC(r->pb.work, (size_t)(kMaxDepth + 1) * kClaimWords * sizeof(unsigned long long));
  }
#undef RALLOC
  r->paths_cap = P;
  r->cams_cap = C;
  r->plain = want_plain;
  r->rgb = want_rgb;
  s->scratch.total = r->bufs.total;
  return RTQ_OK;
}

// Pixels of the rectangle a camera renders (prepare() has validated it).
int64_t rect_pixels(const rtq_camera& C) {
  return C.tile_w == 0 && C.tile_h == 0 ? (int64_t)C.w * C.h : (int64_t)C.tile_w * C.tile_h;
}

struct Prepared {
  RenderParams rp;
  int64_t n_pixels;
  std::string layout;  // every camera's size, rectangle, view id and image offset
  int fmt;
  TraceLaunch tl;
};

int prepare(const rtq_scene* cs, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
            const rtq_render_opts* opts, bool plain_buffers, hipStream_t stream, Prepared* out) {
  rtq_scene* s = const_cast<rtq_scene*>(cs);
  if (!s || !cams || !opts) return set_error(RTQ_E_INVALID_ARG, "NULL scene, cameras or options");
  if (n_cams < 1) return set_error(RTQ_E_INVALID_ARG, "need at least one camera");
  if (spp < 1) return set_error(RTQ_E_INVALID_ARG, "spp %d < 1", spp);
  if (depth < 1 || depth > kMaxDepth) return set_error(RTQ_E_INVALID_ARG, "depth %d outside [1, %d]", depth, kMaxDepth);
  if (opts->accumulate < 0) return set_error(RTQ_E_INVALID_ARG, "accumulate %d < 0", opts->accumulate);
  if (opts->scheduler != RTQ_SCHED_PLAIN && opts->scheduler != RTQ_SCHED_PERSISTENT &&
      opts->scheduler != RTQ_SCHED_MEGAKERNEL)
    return set_error(RTQ_E_INVALID_ARG, "unknown scheduler %d", opts->scheduler);
  int rc = resolve_format(s, opts->node_format, &out->fmt);
  if (rc) return rc;
  rc = resolve_launch(s, opts->scheduler == RTQ_SCHED_PLAIN ? RTQ_SCHED_PLAIN : RTQ_SCHED_PERSISTENT,
                      opts->stack_depth, opts->block, opts->waves_per_cu, opts->refill, &out->tl);
  if (rc) return rc;
  out->tl.fmt = out->fmt;
  const float L[3] = {opts->light_dir[0], opts->light_dir[1], opts->light_dir[2]};
  if (!std::isfinite(L[0]) || !std::isfinite(L[1]) || !std::isfinite(L[2]) || !std::isfinite(opts->E) ||
      !std::isfinite(opts->L_sky))
    return set_error(RTQ_E_INVALID_ARG, "non-finite light parameters");
  if (opts->n_area_lights < 0 || opts->n_area_lights > RTQ_MAX_AREA_LIGHTS)
    return set_error(RTQ_E_INVALID_ARG, "%d area lights outside [0, %d]", opts->n_area_lights, RTQ_MAX_AREA_LIGHTS);
  if (opts->n_area_lights > 0 && !opts->area_lights) return set_error(RTQ_E_INVALID_ARG, "NULL area lights");
  const bool rgb = s->mats != nullptr;
  if (s->tex_res > 0 && s->tex_ch == 3 && !rgb)
    return set_error(RTQ_E_INVALID_ARG, "RGB texels shade with materials: the scene has none");
  if (rgb ? opts->channels != 3 : (opts->channels != 0 && opts->channels != 1))
    return set_error(RTQ_E_INVALID_ARG, "channels %d: the scene %s", opts->channels,
                     rgb ? "has materials, so images have 3 channels" : "has no materials, so images have 1 channel");
  for (int32_t k = 0; k < 10 * opts->n_area_lights; ++k)
    if (!std::isfinite(opts->area_lights[k])) return set_error(RTQ_E_INVALID_ARG, "non-finite area light %d", k / 10);
  std::vector<CamDev> cd(n_cams);
  out->layout.clear();
  std::vector<std::pair<int64_t, int64_t>> ranges;
  int64_t path_base = 0, n_pixels = 0;
  for (int32_t c = 0; c < n_cams; ++c) {
    const rtq_camera& C = cams[c];
    if (C.w < 1 || C.h < 1 || C.img_offset < 0)
      return set_error(RTQ_E_INVALID_ARG, "camera %d: bad resolution or offset", c);
    if ((int64_t)C.w * C.h > (int64_t)0xFFFFFFFFll)
      return set_error(RTQ_E_LIMIT, "camera %d has more than 2^32 pixels", c);
    if (C.view_id < 0) return set_error(RTQ_E_INVALID_ARG, "camera %d: view_id %d < 0", c, C.view_id);
    const bool whole = C.tile_w == 0 && C.tile_h == 0;
    const int32_t tx = whole ? 0 : C.tile_x, ty = whole ? 0 : C.tile_y;
    const int32_t tw = whole ? C.w : C.tile_w, th = whole ? C.h : C.tile_h;
    if (tx < 0 || ty < 0 || tw < 1 || th < 1 || tw > C.w - tx || th > C.h - ty)
      return set_error(RTQ_E_INVALID_ARG, "camera %d: tile (%d, %d, %d x %d) outside the %d x %d view", c, tx, ty,
                       tw, th, C.w, C.h);
    const double ex = C.eye[0], ey = C.eye[1], ez = C.eye[2];
    double f[3] = {C.look[0] - ex, C.look[1] - ey, C.look[2] - ez};
    const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const double up[3] = {C.up[0], C.up[1], C.up[2]};
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(fn > 0.0) || !(rn > 0.0) || !(C.vfov_deg > 0.0f && C.vfov_deg < 180.0f))
      return set_error(RTQ_E_INVALID_ARG, "camera %d: degenerate view (eye == look, up parallel, or bad fov)", c);
    for (int k = 0; k < 3; ++k) {
      f[k] /= fn;
    }
    // r = normalize(f x up) computed from the normalised f
    double rr[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rrn = std::sqrt(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
    for (int k = 0; k < 3; ++k) rr[k] /= rrn;
    const double u[3] = {rr[1] * f[2] - rr[2] * f[1], rr[2] * f[0] - rr[0] * f[2], rr[0] * f[1] - rr[1] * f[0]};
    CamDev& d = cd[c];
    for (int k = 0; k < 3; ++k) {
      d.eye[k] = C.eye[k];
      d.f[k] = (float)f[k];
      d.r[k] = (float)rr[k];
      d.u[k] = (float)u[k];
    }
    d.tan_half = (float)std::tan(0.5 * (double)C.vfov_deg * 3.14159265358979323846 / 180.0);
    d.aspect = (float)((double)C.w / (double)C.h);
    d.w = C.w;
    d.h = C.h;
    d.view_id = C.view_id;
    d.tx = tx;
    d.ty = ty;
    d.tw = tw;
    d.th = th;
    d.img_offset = C.img_offset;
    d.path_base = path_base;
    const int64_t wh = (int64_t)tw * th;
    path_base += wh * spp;
    n_pixels = std::max(n_pixels, C.img_offset + wh);
    ranges.push_back({C.img_offset, C.img_offset + wh});
    char lay[128];
    std::snprintf(lay, sizeof(lay), "%d %d %d %d %d %d %d %lld;", C.w, C.h, C.view_id, tx, ty, tw, th,
                  (long long)C.img_offset);
    out->layout += lay;
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t k = 1; k < ranges.size(); ++k)
    if (ranges[k].first < ranges[k - 1].second) return set_error(RTQ_E_INVALID_ARG, "camera image ranges overlap");
  // the accumulation kernel walks views by increasing image offset
  for (int32_t c = 1; c < n_cams; ++c)
    if (cd[c].img_offset < cd[c - 1].img_offset)
      return set_error(RTQ_E_INVALID_ARG, "camera image offsets must increase with the camera index");
  // path ids are 32-bit, and a dispatch counts its work-items in 32 bits
  if (path_base > (int64_t)0x7FFFFFFF)
    return set_error(RTQ_E_LIMIT, "%lld paths per call exceed 2^31 - 1", (long long)path_base);
  {
    std::lock_guard<std::mutex> lock(s->scratch_mu);
    rc = ensure_scratch(s, path_base, n_cams, plain_buffers, rgb);
    if (rc) return rc;
  }
  RenderScratch* sc = scratch_of(s);
  const hipError_t e =
      hipMemcpyAsync(sc->cams, cd.data(), n_cams * sizeof(CamDev), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_error(e, "camera upload");
  if (opts->n_area_lights > 0) {
    const hipError_t ea = hipMemcpyAsync(sc->alights, opts->area_lights, 10 * sizeof(float) * opts->n_area_lights,
                                         hipMemcpyHostToDevice, stream);
    if (ea != hipSuccess) return hip_error(ea, "area light upload");
  }
  const hipError_t ek = launch_set_keys(sc->keys, (uint32_t)(opts->seed & 0xFFFFFFFFull),
                                         (uint32_t)(opts->seed >> 32) ^ opts->frame, (uint32_t)opts->accumulate,
                                         stream);
  if (ek != hipSuccess) return hip_error(ek, "key upload");
  RenderParams& rp = out->rp;
  rp.cams = sc->cams;
  rp.n_cams = n_cams;
  rp.spp = spp;
  rp.depth = depth;
  rp.keys = sc->keys;
  rp.lx = L[0];
  rp.ly = L[1];
  rp.lz = L[2];
  rp.e_over_pi = (float)((double)opts->E / 3.14159265358979323846);
  rp.L_sky = opts->L_sky;
  rp.n_paths = path_base;
  rp.slots = sc->slots;
  rp.alights = sc->alights;
  rp.n_alights = opts->n_area_lights;
  rp.env_nee = (opts->env_nee && s->env_w > 0) ? 1 : 0;
  rp.mats = static_cast<const MatDev*>(s->mats);
  rp.face_mat = s->face_mat;
  rp.E = opts->E;
  out->n_pixels = n_pixels;
  return RTQ_OK;
}

}  // namespace

namespace {

// Capture (first use) or replay the launches of one render call.  The key holds
// every value that the launches bake in: pointers, sizes, grid shapes, the
// render constants, the scene's texture and environment buffers and the number
// of area lights;
// the RNG key, the accumulated frame count and the area lights themselves are
// read from device memory, written before the graph runs, so frames with other
// seeds or moved lights replay the same graph.
int render_graph(rtq_scene* s, RenderScratch* r, const SceneView& sv, const Prepared& p, bool staged, float* images,
                 RenderExtras ex, hipStream_t stream) {
  char key[512];
  const RenderParams& rp = p.rp;
  std::snprintf(key, sizeof(key),
                "%d|%d|%d %d %d %d|%d %d %d|%lld %lld|%a %a %a %a %a|%p %p %p|%p %p %p %lld %p %p %p|%p|%p %d|%d|%p %d %d",
                staged ? 1 : 0,
                p.fmt, p.tl.persistent, p.tl.stack_depth, p.tl.block, p.tl.refill, p.tl.grid, rp.n_cams, rp.spp,
                (long long)rp.depth, (long long)rp.n_paths, rp.lx, rp.ly, rp.lz, rp.e_over_pi, rp.L_sky,
                (const void*)rp.cams, (const void*)rp.slots, (const void*)images, (void*)ex.counters,
                (void*)ex.visits, (void*)ex.dump, (long long)ex.dump_cap, (void*)ex.dump_count, (void*)ex.view_done,
                (void*)ex.start_tick, (void*)sv.nodes, (const void*)sv.tex, (int)(sv.tex_res * 4 + sv.tex_ch), (int)rp.n_alights,
                (const void*)sv.env, (int)sv.env_w, (int)sv.env_h);
  std::snprintf(key + std::strlen(key), sizeof(key) - std::strlen(key), "|%d %p|%p %p %a", (int)rp.env_nee,
                (const void*)sv.env_T, (const void*)rp.mats, (const void*)rp.face_mat, rp.E);
  // the accumulation grid and its bound bake in the packed image size, and the
  // camera layout decides which image pixels a replay writes
  const std::string k = std::string(key) + "|" + std::to_string((long long)p.n_pixels) + "|" + p.layout;
  auto it = r->graphs.find(k);
  if (it == r->graphs.end()) {
    hipError_t e;
    if (!r->capture_stream) {
      e = hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_error(e, "capture stream");
    }
    GraphEntry g;
    g.counter = reinterpret_cast<unsigned long long*>(
        r->graph_bufs.alloc(kClaimWords * sizeof(unsigned long long), &e));
    if (!g.counter) return hip_error(e, "graph counters");
    // captured work runs only when the graph is launched on the caller's
    // stream, after that stream's camera and key uploads
    TraceLaunch tl = p.tl;
    tl.counter = g.counter;
    RenderExtras cex = ex;
    cex.log = nullptr;  // no events inside a graph
    e = hipStreamBeginCapture(r->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "begin capture");
    hipError_t el = staged ? launch_render_wavefront(sv, rp, r->pb, p.fmt, tl, images, p.n_pixels, cex, r->capture_stream)
                           : launch_render_megakernel(sv, rp, p.fmt, tl, images, p.n_pixels, cex, r->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(r->capture_stream, &graph);
    if (el != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_error(el, "render capture");
    }
    if (e != hipSuccess) return hip_error(e, "end capture");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_error(e, "graph instantiate");
    it = r->graphs.emplace(k, g).first;
  }
  hipEvent_t ev = stage_begin(ex.log, stream);
  const hipError_t e = hipGraphLaunch(it->second.exec, stream);
  stage_end(ex.log, -1, ev, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "graph launch");
}

}  // namespace

namespace rtq {
void release_render_scratch(rtq_scene* s) {
  if (s->stage_log) {
    delete static_cast<StageLog*>(s->stage_log);
    s->stage_log = nullptr;
  }
  if (s->render_state) {
    RenderScratch* r = static_cast<RenderScratch*>(s->render_state);
    r->clear_graphs();
    if (r->capture_stream) (void)hipStreamDestroy(r->capture_stream);
    r->bufs.release();
    delete r;
    s->render_state = nullptr;
  }
  s->scratch.release();
}
}  // namespace rtq

extern "C" {

int rtq_render(const rtq_scene* s, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
               const rtq_render_opts* opts, float* images, hipStream_t stream) {
  if (!images) return set_error(RTQ_E_INVALID_ARG, "NULL image buffer");
  if (!opts) return set_error(RTQ_E_INVALID_ARG, "NULL options");
  const bool staged = opts->scheduler != RTQ_SCHED_MEGAKERNEL;
  Prepared p;
  int rc = prepare(s, cams, n_cams, spp, depth, opts, staged, stream, &p);
  if (rc) return rc;
  if (opts->dump_rays && (opts->dump_cap < 1 || !opts->dump_count))
    return set_error(RTQ_E_INVALID_ARG, "dump_rays needs dump_cap >= 1 and dump_count");
  const SceneView sv = scene_view(s, p.fmt);
  RenderExtras ex;
  ex.counters = reinterpret_cast<unsigned long long*>(opts->counters);
  ex.visits = reinterpret_cast<unsigned long long*>(opts->visits);
  ex.dump = opts->dump_rays;
  ex.dump_cap = opts->dump_cap;
  ex.dump_count = reinterpret_cast<unsigned long long*>(opts->dump_count);
  ex.view_done = reinterpret_cast<unsigned long long*>(opts->view_done);
  ex.start_tick = reinterpret_cast<unsigned long long*>(opts->start_tick);
  ex.log = nullptr;
  std::unique_lock<std::mutex> log_lock;
  if (opts->timing) {
    rtq_scene* ms = const_cast<rtq_scene*>(s);
    log_lock = std::unique_lock<std::mutex>(ms->scratch_mu);
    if (!ms->stage_log) ms->stage_log = new StageLog;
    ex.log = static_cast<StageLog*>(ms->stage_log);
    ex.log->call_first = ex.log->call_last = nullptr;
  }
  hipError_t e;
  RenderScratch* r = scratch_of(const_cast<rtq_scene*>(s));
  if (opts->graph) {
    std::unique_lock<std::mutex> graph_lock;
    if (!log_lock.owns_lock()) graph_lock = std::unique_lock<std::mutex>(const_cast<rtq_scene*>(s)->scratch_mu);
    int grc = render_graph(const_cast<rtq_scene*>(s), r, sv, p, staged, images, ex, stream);
    if (ex.log && ex.log->call_first && ex.log->call_last)
      ex.log->calls.push_back({ex.log->call_first, ex.log->call_last});
    return grc;
  }
  if (staged) {
    e = launch_render_wavefront(sv, p.rp, r->pb, p.fmt, p.tl, images, p.n_pixels, ex, stream);
  } else {
    e = launch_render_megakernel(sv, p.rp, p.fmt, p.tl, images, p.n_pixels, ex, stream);
  }
  if (ex.log && ex.log->call_first && ex.log->call_last)
    ex.log->calls.push_back({ex.log->call_first, ex.log->call_last});
  return e == hipSuccess ? RTQ_OK : hip_error(e, "render launch");
}

int rtq_render_timing(rtq_scene* s, float* ms, int32_t* launches) {
  if (!s) return set_error(RTQ_E_INVALID_ARG, "NULL scene");
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  int32_t cnt[4] = {0, 0, 0, 0};
  std::lock_guard<std::mutex> lock(s->scratch_mu);
  StageLog* log = static_cast<StageLog*>(s->stage_log);
  int rc = RTQ_OK;
  if (log) {
    for (const StageLog::Rec& r : log->recs) {
      if (r.stage < 0) continue;  // call marker of a graph launch
      float t = 0.0f;
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
      if (e != hipSuccess) {
        rc = hip_error(e, "stage event");
        break;
      }
      acc[r.stage] += t;
      ++cnt[r.stage];
    }
    for (const auto& c : log->calls) {
      float t = 0.0f;
      if (rc == RTQ_OK && hipEventSynchronize(c.second) == hipSuccess &&
          hipEventElapsedTime(&t, c.first, c.second) == hipSuccess) {
        acc[3] += t;
        ++cnt[3];
      }
    }
    log->free_list = log->all;
    log->recs.clear();
    log->calls.clear();
    log->dropped = 0;
  }
  if (ms)
    for (int k = 0; k < 4; ++k) ms[k] = acc[k];
  if (launches)
    for (int k = 0; k < 4; ++k) launches[k] = cnt[k];
  return rc;
}

int rtq_render_path(const rtq_scene* s, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
                    const rtq_render_opts* opts, int32_t view, int64_t pixel, int32_t sample, int32_t* vert_i,
                    float* vert_f, int32_t* n_vert, int32_t* escaped, float* radiance, hipStream_t stream) {
  if (!vert_i || !vert_f || !n_vert || !escaped || !radiance) return set_error(RTQ_E_INVALID_ARG, "NULL output");
  if (!cams || view < 0 || view >= n_cams) return set_error(RTQ_E_INVALID_ARG, "view %d outside [0, %d)", view, n_cams);
  Prepared p;
  int rc = prepare(s, cams, n_cams, spp, depth, opts, false, stream, &p);
  if (rc) return rc;
  const int64_t wh = rect_pixels(cams[view]);
  if (pixel < 0 || pixel >= wh || sample < 0 || sample >= spp)
    return set_error(RTQ_E_INVALID_ARG, "pixel or sample out of range");
  int64_t base = 0;
  for (int32_t c = 0; c < view; ++c) base += rect_pixels(cams[c]) * spp;
  const int64_t pid = base + (int64_t)sample * wh + pixel;
  hipError_t e;
  DeviceBuffers tmp;
  int32_t* d_i = reinterpret_cast<int32_t*>(tmp.alloc(6 * kMaxDepth * sizeof(int32_t) + 64, &e));
  float* d_f = reinterpret_cast<float*>(tmp.alloc((10 * kMaxDepth + 3) * sizeof(float), &e));
  int32_t* d_o = reinterpret_cast<int32_t*>(tmp.alloc(64, &e));
  if (!d_i || !d_f || !d_o) {
    tmp.release();
    return hip_error(e, "hipMalloc");
  }
  const SceneView sv = scene_view(s, p.fmt);
  e = launch_path_record(sv, p.rp, p.fmt, p.tl.stack_depth, pid, d_i, d_f, d_o, stream);
  int32_t ho[2] = {0, 0};
  float hf[10 * kMaxDepth + 3];
  if (e == hipSuccess) e = hipMemcpyAsync(vert_i, d_i, 6 * depth * sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hf, d_f, sizeof(hf), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ho, d_o, sizeof(ho), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  tmp.release();
  if (e != hipSuccess) return hip_error(e, "path record");
  for (int k = 0; k < 10 * depth; ++k) vert_f[k] = hf[k];
  *n_vert = ho[0];
  *escaped = ho[1];
  radiance[0] = hf[10 * kMaxDepth];
  if (s->mats) {
    radiance[1] = hf[10 * kMaxDepth + 1];
    radiance[2] = hf[10 * kMaxDepth + 2];
  }
  return RTQ_OK;
}

int rtq_render_backward(const rtq_scene* s, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
                        const rtq_render_opts* opts, const float* grad_images, float* grad_albedo,
                        hipStream_t stream) {
  if (!grad_images || !grad_albedo) return set_error(RTQ_E_INVALID_ARG, "NULL gradient buffer");
  Prepared p;
  int rc = prepare(s, cams, n_cams, spp, depth, opts, false, stream, &p);
  if (rc) return rc;
  const SceneView sv = scene_view(s, p.fmt);
  const hipError_t e =
      launch_adjoint(sv, p.rp, p.fmt, p.tl.stack_depth, p.tl.block, grad_images, grad_albedo, stream);
  return e == hipSuccess ? RTQ_OK : hip_error(e, "adjoint launch");
}

}  // extern "C"
