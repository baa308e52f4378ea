// Path-tracing kernels.
//
// Plain scheduler (a wavefront path tracer after Laine, Karras, Aila 2013, one
// kernel per stage, one ray per lane): raygen -> per bounce [closest-hit queue
// trace -> shade (appends shadow rays and extension rays with block-aggregated
// compaction) -> occlusion queue trace -> shadow resolve] -> accumulate.
//
// Persistent scheduler: the same stages, but each traversal launch is
// persistent (resident waves refill idle lanes from sliced claim counters) and
// traces the shadow rays of bounce b together with the extension rays of
// bounce b + 1.
//
// Megakernel: one launch.  Resident waves pull path ids from the claim
// counters; each lane runs one path, alternating extension and shadow rays in a
// single traversal loop, and finished lanes are refilled with new paths
// whenever enough of the wave is idle, across every view.
//
// All schedulers evaluate each path with the same device functions in the same
// order and write its radiance to its own slot; the image is the per-pixel mean
// over samples in sample order, so they produce bit-identical images.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "render_device.h"
#include "render_kernels.h"

namespace rtq {

// Threads per block of the shading kernel.
constexpr int kShadeBlock = 512;

// Block-aggregated append to two queues (one atomic per queue per block, since
// atomics on one counter serialise): sets *ja / *jb to this thread's slots where
// wa / wb hold.  Every thread of a kShadeBlock-thread block must call it.
__device__ __forceinline__ void block_append2(bool wa, bool wb, uint32_t* ca, uint32_t* cb, uint32_t* ja,
                                              uint32_t* jb) {
  constexpr int kWaves = kShadeBlock / 64;
  __shared__ uint32_t wcnt[2][kWaves];
  __shared__ uint32_t base[2];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const unsigned long long ma = __ballot(wa), mb = __ballot(wb);
  if (lane == 0) {
    wcnt[0][w] = (uint32_t)__popcll(ma);
    wcnt[1][w] = (uint32_t)__popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t tot = 0u;
    for (int k = 0; k < kWaves; ++k) tot += wcnt[threadIdx.x][k];
    base[threadIdx.x] = tot ? atomicAdd(threadIdx.x == 0 ? ca : cb, tot) : 0u;
  }
  __syncthreads();
  uint32_t pa = base[0], pb = base[1];
  for (int k = 0; k < w; ++k) {
    pa += wcnt[0][k];
    pb += wcnt[1][k];
  }
  *ja = pa + __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
  *jb = pb + __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
}

// Sum per-lane visit counters over the wave; one atomic per counter per wave.
// Must be reached by every lane of the wave.
__device__ __forceinline__ void wave_add_visits(const VisitCounters& vc, unsigned long long* visits) {
  unsigned long long v[4] = {vc.tlas, vc.inst, vc.blas, vc.quads};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(&visits[k], x);
  }
}

// Wave-aggregated append: returns this lane's slot (valid where want is true).
__device__ __forceinline__ unsigned long long wave_append64(bool want, unsigned long long* counter) {
  const unsigned long long m = __ballot(want);
  if (m == 0ull) return 0ull;
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0ull;
  if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader);
  const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  return (((unsigned long long)hi << 32) | lo) + rank;
}

// Per-view completion stamps: view_done[cam] = max over the view's paths of the
// wall-clock tick at which the path ended, so it holds the tick at which the
// view's last path finished.  One atomic per wave and distinct camera among the
// lanes whose path ends here.  Must be reached by every lane of the wave.
__device__ __forceinline__ void wave_stamp_views(bool ends, int cam, unsigned long long* view_done) {
  unsigned long long pend = __ballot(ends);
  if (pend == 0ull) return;
  const unsigned long long now = (unsigned long long)wall_clock64();
  const int lane = (int)(threadIdx.x & 63);
  while (pend != 0ull) {
    const int leader = __ffsll((long long)pend) - 1;
    const int c = __builtin_amdgcn_readlane(cam, leader);
    const unsigned long long same = __ballot(ends && cam == c);
    if (lane == leader) atomicMax(&view_done[c], now);
    pend &= ~same;
  }
}

// ---------------------------------------------------------------- plain scheduler
__global__ void k_raygen(RenderParams rp, ExtQueue q, uint32_t* counts) {
  const int64_t pid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pid == 0) counts[0] = (uint32_t)rp.n_paths;
  if (pid >= rp.n_paths) return;
  PathId id;
  const Ray3 r = path_camera_ray(rp, pid, &id);
  q.ox[pid] = r.ox;
  q.oy[pid] = r.oy;
  q.oz[pid] = r.oz;
  q.dx[pid] = r.dx;
  q.dy[pid] = r.dy;
  q.dz[pid] = r.dz;
  q.pid[pid] = (uint32_t)pid;
  q.beta[pid] = 1.0f;
  q.ex_rec[pid] = kEmpty;
  q.ex_qh[pid] = kEmpty;
  rp.slots[pid] = 0.0f;
  if (rgb_mode(rp)) {
    q.beta_g[pid] = 1.0f;
    q.beta_b[pid] = 1.0f;
    rp.slots[rp.n_paths + pid] = 0.0f;
    rp.slots[2 * rp.n_paths + pid] = 0.0f;
  }
}

// Load queue entry i into a lane: an extension ray (closest hit) or a shadow
// ray (any hit: toward the directional light, or, in a scene with area lights,
// along its stored direction up to its stored tmax), with its spawning triangle
// excluded.
template <bool ANY>
__device__ __forceinline__ bool load_queue_ray(Lane& L, const SceneView& sc, const RenderParams& rp,
                                               const ExtQueue& eq, const ShadowQueue& sq, int64_t i) {
  bool ok;
  if (ANY) {
    if (nee_sampled(rp))
      ok = lane_init(L, sc, sq.ox[i], sq.oy[i], sq.oz[i], sq.dx[i], sq.dy[i], sq.dz[i], 0.0f, sq.tmax[i]);
    else
      ok = lane_init(L, sc, sq.ox[i], sq.oy[i], sq.oz[i], rp.lx, rp.ly, rp.lz, 0.0f, kInfF);
    L.ex_rec = sq.ex_rec[i];
    L.ex_qh = sq.ex_qh[i];
    L.any = true;
  } else {
    ok = lane_init(L, sc, eq.ox[i], eq.oy[i], eq.oz[i], eq.dx[i], eq.dy[i], eq.dz[i], 0.0f, kInfF);
    L.ex_rec = eq.ex_rec[i];
    L.ex_qh = eq.ex_qh[i];
  }
  return ok;
}

// Optional scene features that select kernel variants: textures (closest hits
// carry (u, v)) and area lights (shadow rays carry a direction and a tmax).
constexpr int kFeatTex = 1;
constexpr int kFeatArea = 2;
static inline int scene_features(const SceneView& sc, const RenderParams& rp) {
  return (sc.tex_res > 0 ? kFeatTex : 0) | ((rp.n_alights > 0 || rp.env_nee) ? kFeatArea : 0);
}

template <bool ANY>
__device__ __forceinline__ void store_queue_result(const Lane& L, const QueueHits& qh, uint8_t* occ, int64_t i,
                                                   bool tex) {
  if (ANY) {
    occ[i] = L.b_rec != kEmpty ? 1 : 0;
  } else {
    qh.t[i] = L.t_best;
    qh.rec[i] = L.b_rec;
    qh.qh[i] = L.b_rec == kEmpty ? kEmpty : L.b_qh;
    if (tex) {
      qh.u[i] = L.b_u;
      qh.v[i] = L.b_v;
    }
  }
}

// Closest hit (ANY = false) of an extension queue, or occlusion (ANY = true) of a
// shadow queue, one lane per entry.  FEAT (scene_features): with kFeatTex the
// scene has textures, so closest hits also store (u, v); without it the
// compiler drops their arithmetic from the quad test.  Without kFeatArea every
// shadow ray goes to the directional light with tmax = +inf, a constant the
// compiler folds into the traversal.
template <int FMT, bool ANY, bool COUNT, int FEAT>
__global__ void k_trace_queue(SceneView sc, RenderParams rp, ExtQueue eq, ShadowQueue sq, const uint32_t* count,
                              QueueHits qh, uint8_t* occ, int depth, unsigned long long* visits) {
  constexpr bool TEX = (FEAT & kFeatTex) != 0;
  if (!(FEAT & kFeatArea)) {
    rp.n_alights = 0;
    rp.env_nee = 0;
  }
  extern __shared__ uint2 lds[];
  const Stack S = make_stack(lds, depth);
  uint2 spill[kStackTotal];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < (int64_t)*count;
  VisitCounters vc{0, 0, 0, 0};
  if (live) {
    Lane L;
    if (load_queue_ray<ANY>(L, sc, rp, eq, sq, i))
      while (!lane_step<FMT, COUNT>(L, sc, S, spill, vc)) {
      }
    store_queue_result<ANY>(L, qh, occ, i, TEX);
  }
  if (COUNT) wave_add_visits(vc, visits);
}

// Persistent traversal of an extension-ray queue (closest hits) and a shadow-ray
// queue (occlusion) in one launch: entries [0, n_ext) are extension rays,
// [n_ext, n_ext + n_sh) shadow rays.  Tracing the shadow rays of bounce b with
// the extension rays of bounce b + 1 halves the traversal launches of a frame
// and with them the drain at the end of each launch; the short any-hit rays
// come last, where the launch drains.
template <int FMT, bool COUNT, int FEAT>
__global__ void k_trace_queue_mixed(SceneView sc, RenderParams rp, ExtQueue eq, const uint32_t* count_ext,
                                    ShadowQueue sq, const uint32_t* count_sh, QueueHits qh, uint8_t* occ, int depth,
                                    int refill, unsigned long long* counter, unsigned long long* visits) {
  constexpr bool TEX = (FEAT & kFeatTex) != 0;
  if (!(FEAT & kFeatArea)) {
    rp.n_alights = 0;
    rp.env_nee = 0;
  }
  extern __shared__ uint2 lds[];
  const int lane = threadIdx.x & 63;
  const Stack S = make_stack(lds, depth);
  uint2 spill[kStackTotal];
  const int64_t n_ext = (int64_t)*count_ext;
  const int64_t n = n_ext + (int64_t)*count_sh;
  Lane L;
  VisitCounters vc{0, 0, 0, 0}, vc_cl{0, 0, 0, 0}, vc_sh{0, 0, 0, 0};
  bool has = false, exhausted = n == 0;
  ClaimState claim = claim_init();
  int64_t idx = -1;
  for (;;) {
    const unsigned long long idle = __ballot(!has);
    const int nidle = __popcll(idle);
    if (!exhausted && (nidle >= refill || nidle == 64)) {
      const int64_t k = claim_take(claim, counter, n, idle, nidle, &exhausted);
      if (k >= 0) {
        if (k < n_ext) {
          idx = k;
          if (load_queue_ray<false>(L, sc, rp, eq, sq, idx)) has = true;
          else store_queue_result<false>(L, qh, occ, idx, TEX);
        } else {
          idx = k - n_ext;
          if (load_queue_ray<true>(L, sc, rp, eq, sq, idx)) has = true;
          else store_queue_result<true>(L, qh, occ, idx, TEX);
        }
      }
    }
    if (!__any(has)) {
      if (exhausted) break;
      continue;
    }
    if (has) {
      for (;;) {
        if (lane_step<FMT, COUNT>(L, sc, S, spill, vc)) {
          if (L.any) store_queue_result<true>(L, qh, occ, idx, TEX);
          else store_queue_result<false>(L, qh, occ, idx, TEX);
          if (COUNT) {
            VisitCounters& acc = L.any ? vc_sh : vc_cl;
            acc.tlas += vc.tlas;
            acc.inst += vc.inst;
            acc.blas += vc.blas;
            acc.quads += vc.quads;
            vc = VisitCounters{0, 0, 0, 0};
          }
          has = false;
          break;
        }
        if (!exhausted && __popcll(__ballot(1)) <= 64 - refill) break;
      }
    }
  }
  if (COUNT) {
    wave_add_visits(vc_cl, visits);
    wave_add_visits(vc_sh, visits + 4);
  }
}

__global__ void k_shade(SceneView sc, RenderParams rp, int b, ExtQueue in, const uint32_t* count_in, QueueHits qh,
                        ExtQueue out, uint32_t* count_out, ShadowQueue sq, uint32_t* count_sq, float* dump,
                        long long dump_cap, unsigned long long* dump_count, unsigned long long* view_done) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < (int64_t)*count_in;
  bool want_shadow = false, want_next = false;
  float contrib = 0.0f, beta_next = 0.0f, ndx = 0.0f, ndy = 0.0f, ndz = 0.0f, pdf_next = 0.0f;
  float contrib3[3] = {0.0f, 0.0f, 0.0f}, beta3[3] = {0.0f, 0.0f, 0.0f};  // RGB: contribution, next throughput
  Shade s{};
  NeeSample ns{false, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  uint32_t pid = 0u, rec = kEmpty, qhv = kEmpty;
  const bool rgb = rgb_mode(rp);
  if (live) {
    pid = in.pid[i];
    const float beta = in.beta[i];
    rec = qh.rec[i];
    if (rec == kEmpty) {
      const float pdf = (b > 0 && rp.env_nee) ? in.pdf[i] : 0.0f;
      const float Le = escape_radiance(sc, rp, in.dx[i], in.dy[i], in.dz[i], pdf);
      rp.slots[pid] += beta * Le;  // escaped
      if (rgb) {
        rp.slots[rp.n_paths + pid] += in.beta_g[i] * Le;
        rp.slots[2 * rp.n_paths + pid] += in.beta_b[i] * Le;
      }
    } else if (rgb) {
      qhv = qh.qh[i];
      const Ray3 r{in.ox[i], in.oy[i], in.oz[i], in.dx[i], in.dy[i], in.dz[i]};
      const bool tex = sc.tex_res > 0;
      s = shade_hit(sc, rp, r, qh.t[i], rec, qhv & 0x7FFFFFFFu, qhv >> 31, tex ? qh.u[i] : 0.0f,
                    tex ? qh.v[i] : 0.0f);
      float c[3];
      const PShade ps = principled_vertex(sc, rp, s, r, c);
      const float bt[3] = {beta, in.beta_g[i], in.beta_b[i]};
      const bool next = b < rp.depth - 1;
      const PathId id = path_coords(rp, (int64_t)pid);
      ns = nee_sample(sc, rp, s, id.pixel, id.sample, id.view, b);
      if (ns.want) {
        float e[3], e1[3];
        pnee_estimate(ps, c, ns, e, e1);
        want_shadow = true;
        for (int k = 0; k < 3; ++k) contrib3[k] = bt[k] * e[k];
        contrib = contrib3[0];
      }
      if (next) {
        float w[3], w1[3];
        pdf_next = pbsdf_bounce(rp, ps, c, id.pixel, id.sample, id.view, b, &ndx, &ndy, &ndz, w, w1);
        for (int k = 0; k < 3; ++k) beta3[k] = bt[k] * w[k];
        beta_next = beta3[0];
        want_next = pdf_next > 0.0f;
      }
    } else {
      qhv = qh.qh[i];
      const Ray3 r{in.ox[i], in.oy[i], in.oz[i], in.dx[i], in.dy[i], in.dz[i]};
      const bool tex = sc.tex_res > 0;
      s = shade_hit(sc, rp, r, qh.t[i], rec, qhv & 0x7FFFFFFFu, qhv >> 31, tex ? qh.u[i] : 0.0f,
                    tex ? qh.v[i] : 0.0f);
      const bool next = b < rp.depth - 1;
      PathId id{0, 0u, 0u, 0u, 0u};
      if (next || nee_sampled(rp)) id = path_coords(rp, (int64_t)pid);
      ns = nee_sample(sc, rp, s, id.pixel, id.sample, id.view, b);
      if (ns.want) {
        want_shadow = true;
        contrib = nee_contrib(beta, s, ns, rp);
      }
      if (next) {
        pdf_next = bounce_dir(rp, id.pixel, id.sample, id.view, b, s, &ndx, &ndy, &ndz);
        beta_next = beta * s.a;
        want_next = true;
      }
    }
  }
  uint32_t js, jn;
  block_append2(want_shadow, want_next, count_sq, count_out, &js, &jn);
  if (want_shadow) {
    sq.ox[js] = s.px;
    sq.oy[js] = s.py;
    sq.oz[js] = s.pz;
    sq.pid[js] = pid;
    sq.contrib[js] = contrib;
    if (rgb) {
      sq.contrib_g[js] = contrib3[1];
      sq.contrib_b[js] = contrib3[2];
    }
    sq.ex_rec[js] = rec;
    sq.ex_qh[js] = qhv;
    if (nee_sampled(rp)) {
      sq.dx[js] = ns.dx;
      sq.dy[js] = ns.dy;
      sq.dz[js] = ns.dz;
      sq.tmax[js] = ns.tmax;
    }
  }
  if (want_next) {
    out.ox[jn] = s.px;
    out.oy[jn] = s.py;
    out.oz[jn] = s.pz;
    out.dx[jn] = ndx;
    out.dy[jn] = ndy;
    out.dz[jn] = ndz;
    out.pid[jn] = pid;
    out.beta[jn] = beta_next;
    if (rgb) {
      out.beta_g[jn] = beta3[1];
      out.beta_b[jn] = beta3[2];
    }
    out.ex_rec[jn] = rec;
    out.ex_qh[jn] = qhv;
    if (rp.env_nee) out.pdf[jn] = pdf_next;
  }
  if (view_done) {  // paths that end here: escaped, or past the last bounce without a shadow ray
    const bool ends = live && !want_next && !want_shadow;
    wave_stamp_views(ends, ends ? path_coords(rp, (int64_t)pid).cam : 0, view_done);
  }
  if (dump) {  // keep a copy of the incoherent (bounce >= 1) extension rays
    const unsigned long long jd = wave_append64(want_next, dump_count);
    if (want_next && jd < (unsigned long long)dump_cap) {
      const size_t c = (size_t)dump_cap;
      dump[0 * c + jd] = s.px;
      dump[1 * c + jd] = s.py;
      dump[2 * c + jd] = s.pz;
      dump[3 * c + jd] = ndx;
      dump[4 * c + jd] = ndy;
      dump[5 * c + jd] = ndz;
      dump[6 * c + jd] = 0.0f;
      dump[7 * c + jd] = kInfF;
      uint32_t* du = reinterpret_cast<uint32_t*>(dump);
      du[8 * c + jd] = rec;
      du[9 * c + jd] = qhv;
      du[10 * c + jd] = sc.inst[rec].inst_id;
      du[11 * c + jd] = (uint32_t)sc.quad_prim[qhv & 0x7FFFFFFFu] | (qhv & 0x80000000u);
    }
  }
}

// Shadow rays of bounce b: add the contributions of the unoccluded ones.  After
// the last bounce every path with a shadow ray ends here.
__global__ void k_shadow_resolve(RenderParams rp, ShadowQueue sq, const uint32_t* count, const uint8_t* occ, int b,
                                 unsigned long long* view_done) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < (int64_t)*count;
  if (live && !occ[i]) {
    const uint32_t pid = sq.pid[i];
    rp.slots[pid] += sq.contrib[i];
    if (rgb_mode(rp)) {
      rp.slots[rp.n_paths + pid] += sq.contrib_g[i];
      rp.slots[2 * rp.n_paths + pid] += sq.contrib_b[i];
    }
  }
  if (view_done && b == rp.depth - 1) {
    wave_stamp_views(live, live ? path_coords(rp, (int64_t)sq.pid[i]).cam : 0, view_done);
  }
}

// image[view pixel] = (sum over samples, in sample order) / spp
__global__ void k_accum(RenderParams rp, float* image, int64_t n_pixels) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_pixels) return;
  int lo = 0, hi = rp.n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rp.cams[mid].img_offset <= g) lo = mid;
    else hi = mid - 1;
  }
  const CamDev& c = rp.cams[lo];
  const int64_t wh = (int64_t)c.tw * c.th;
  const int64_t pixel = g - c.img_offset;
  // before the first view, or in a gap between views: not part of any image
  if (pixel < 0 || pixel >= wh) return;
  // progressive refinement: keys[2] frames are already averaged in the image
  const uint32_t k = rp.keys[2];
  const int nch = rgb_mode(rp) ? 3 : 1;
  for (int ch = 0; ch < nch; ++ch) {
    const float* sl = rp.slots + ch * rp.n_paths;
    float sum = 0.0f;
    for (int s = 0; s < rp.spp; ++s) sum += sl[c.path_base + s * wh + pixel];
    const float m = sum / (float)rp.spp;
    const int64_t o = nch * g + ch;  // RGB images interleave the channels per pixel
    image[o] = k == 0u ? m : image[o] + (m - image[o]) / (float)(k + 1u);
  }
}

// counters[0..3] += closest, shadow, incoherent (bounce >= 1), paths
__global__ void k_plain_stats(const uint32_t* counts, int depth, int64_t n_paths, unsigned long long* counters) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long ext = 0, sh = 0, inc = 0;
  for (int b = 0; b < depth; ++b) {
    ext += counts[b];
    if (b >= 1) inc += counts[b];
    sh += counts[kMaxDepth + 1 + b];
  }
  counters[0] += ext;
  counters[1] += sh;
  counters[2] += inc;
  counters[3] += (unsigned long long)n_paths;
}

__global__ void k_set_keys(uint32_t* keys, uint32_t k0, uint32_t k1, uint32_t acc) {
  if (threadIdx.x == 0) {
    keys[0] = k0;
    keys[1] = k1;
    keys[2] = acc;
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- persistent scheduler
// Per-lane path state of the persistent scheduler (pixel coordinates are
// re-derived from the path id when a bounce needs them).
struct PathLane {
  uint32_t pid;
  int b;
  float beta, radiance, pending, beta_next, ndx, ndy, ndz;
  float pdf, pdf_next;  // BSDF density of the current / next extension ray (0 for camera rays)
  // green and blue channels of beta, radiance, pending and beta_next (RGB shading)
  float beta_g, beta_b, rad_g, rad_b, pend_g, pend_b, bn_g, bn_b;
  bool shadow, have_next;
};

// At least four resident waves per SIMD (up to 128 registers per lane: the path
// state comes on top of the traversal state).
template <int FMT, bool TS, bool COUNT, int FEAT>
__global__ __attribute__((amdgpu_waves_per_eu(4))) void k_render_persistent(SceneView sc, RenderParams rp, int depth_lds, int refill,
                                    unsigned long long* counter, unsigned long long* counters,
                                    unsigned long long* view_done, unsigned long long* visits) {
  constexpr bool TEX = (FEAT & kFeatTex) != 0;
  if (!(FEAT & kFeatArea)) {
    rp.n_alights = 0;
    rp.env_nee = 0;
  }
  extern __shared__ uint2 lds[];
  const int lane = threadIdx.x & 63;
  const Stack S = make_stack(lds, depth_lds);
  uint2 spill[kStackTotal];
  Lane L;
  VisitCounters vc{0, 0, 0, 0};      // current traversal
  VisitCounters vc_sh{0, 0, 0, 0};   // finished shadow traversals (closest-hit ones stay in vc_cl)
  VisitCounters vc_cl{0, 0, 0, 0};
  PathLane P{};
  bool has = false, exhausted = rp.n_paths == 0;
  ClaimState claim = claim_init();
  uint32_t n_ext = 0, n_sh = 0, n_inc = 0, n_paths = 0;
  for (;;) {
    const unsigned long long idle = __ballot(!has);
    const int nidle = __popcll(idle);
    if (!exhausted && (nidle >= refill || nidle == 64)) {
      const int64_t pid = claim_take(claim, counter, rp.n_paths, idle, nidle, &exhausted);
      {
        if (pid >= 0) {
          P.pid = (uint32_t)pid;
          PathId id;
          const Ray3 r = path_camera_ray(rp, pid, &id);
          P.b = 0;
          P.beta = 1.0f;
          P.pdf = 0.0f;
          P.radiance = 0.0f;
          P.beta_g = P.beta_b = 1.0f;
          P.rad_g = P.rad_b = 0.0f;
          P.shadow = false;
          P.have_next = false;
          L.ex_rec = kEmpty;
          L.ex_qh = kEmpty;
          lane_init(L, sc, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, 0.0f, kInfF);
          ++n_ext;
          has = true;
        }
      }
    }
    if (!__any(has)) {
      if (exhausted) break;
      continue;
    }
    if (has) {
      for (;;) {
        // vote among the traversal step kinds and "shade" (the lane's ray is
        // finished): one kind per iteration, the most wanted
        const int kind = step_kind(L);
        const int cs = __popcll(__ballot(kind == 0));
        const int ct = vote_kind(kind);
        const int cmax = ct == 0 ? 0 : __popcll(__ballot(kind == ct));
        if (cs > 0 && cs >= cmax) {
          if (kind == 0) {
            if (COUNT) {
              VisitCounters& acc = P.shadow ? vc_sh : vc_cl;
              acc.tlas += vc.tlas;
              acc.inst += vc.inst;
              acc.blas += vc.blas;
              acc.quads += vc.quads;
              vc = VisitCounters{0, 0, 0, 0};
            }
            bool path_done = false;
            if (!P.shadow) {
              if (L.b_rec == kEmpty) {
                const float Le = escape_radiance(sc, rp, L.wdx, L.wdy, L.wdz, P.pdf);
                P.radiance += P.beta * Le;
                if (rgb_mode(rp)) {
                  P.rad_g += P.beta_g * Le;
                  P.rad_b += P.beta_b * Le;
                }
                path_done = true;
              } else {
                const Ray3 r{L.wox, L.woy, L.woz, L.wdx, L.wdy, L.wdz};
                const uint32_t hrec = L.b_rec, hqh = L.b_qh;
                const Shade s = shade_hit(sc, rp, r, L.t_best, hrec, hqh & 0x7FFFFFFFu, hqh >> 31,
                                          TEX ? L.b_u : 0.0f, TEX ? L.b_v : 0.0f);
                P.have_next = P.b < rp.depth - 1;
                PathId id{0, 0u, 0u, 0u, 0u};
                if (P.have_next || nee_sampled(rp) || rgb_mode(rp)) id = path_coords(rp, (int64_t)P.pid);
                const NeeSample ns = nee_sample(sc, rp, s, id.pixel, id.sample, id.view, P.b);
                if (rgb_mode(rp)) {
                  float c[3];
                  const PShade ps = principled_vertex(sc, rp, s, r, c);
                  if (P.have_next) {
                    float w[3], w1[3];
                    P.pdf_next = pbsdf_bounce(rp, ps, c, id.pixel, id.sample, id.view, P.b, &P.ndx, &P.ndy,
                                              &P.ndz, w, w1);
                    P.have_next = P.pdf_next > 0.0f;
                    P.beta_next = P.beta * w[0];
                    P.bn_g = P.beta_g * w[1];
                    P.bn_b = P.beta_b * w[2];
                  }
                  if (ns.want) {
                    float e[3], e1[3];
                    pnee_estimate(ps, c, ns, e, e1);
                    P.pending = P.beta * e[0];
                    P.pend_g = P.beta_g * e[1];
                    P.pend_b = P.beta_b * e[2];
                  }
                } else {
                  if (P.have_next) {
                    P.pdf_next = bounce_dir(rp, id.pixel, id.sample, id.view, P.b, s, &P.ndx, &P.ndy, &P.ndz);
                    P.beta_next = P.beta * s.a;
                  }
                  if (ns.want) P.pending = nee_contrib(P.beta, s, ns, rp);
                }
                L.ex_rec = hrec;
                L.ex_qh = hqh;
                if (ns.want) {
                  P.shadow = true;
                  lane_init(L, sc, s.px, s.py, s.pz, ns.dx, ns.dy, ns.dz, 0.0f, ns.tmax);
                  L.any = true;
                  ++n_sh;
                } else if (P.have_next) {
                  P.beta = P.beta_next;
                  P.beta_g = P.bn_g;
                  P.beta_b = P.bn_b;
                  P.pdf = P.pdf_next;
                  ++P.b;
                  lane_init(L, sc, s.px, s.py, s.pz, P.ndx, P.ndy, P.ndz, 0.0f, kInfF);
                  ++n_ext;
                  ++n_inc;
                } else {
                  path_done = true;
                }
              }
            } else {
              if (L.b_rec == kEmpty) {
                P.radiance += P.pending;
                if (rgb_mode(rp)) {
                  P.rad_g += P.pend_g;
                  P.rad_b += P.pend_b;
                }
              }
              P.shadow = false;
              if (P.have_next) {
                P.beta = P.beta_next;
                P.beta_g = P.bn_g;
                P.beta_b = P.bn_b;
                P.pdf = P.pdf_next;
                ++P.b;
                lane_init(L, sc, L.wox, L.woy, L.woz, P.ndx, P.ndy, P.ndz, 0.0f, kInfF);
                ++n_ext;
                ++n_inc;
              } else {
                path_done = true;
              }
            }
            if (path_done) {
              rp.slots[P.pid] = P.radiance;
              if (rgb_mode(rp)) {
                rp.slots[rp.n_paths + P.pid] = P.rad_g;
                rp.slots[2 * rp.n_paths + P.pid] = P.rad_b;
              }
              ++n_paths;
              if (TS) atomicMax(&view_done[path_coords(rp, (int64_t)P.pid).cam], (unsigned long long)wall_clock64());
              has = false;
              break;
            }
          }
        } else {
          run_step<FMT, COUNT>(ct, kind, L, sc, S, spill, vc);
        }
        pop_step(L, sc, S, spill);
        if (!exhausted && __popcll(__ballot(1)) <= 64 - refill) break;
      }
    }
  }
  if (COUNT) {
    wave_add_visits(vc_cl, visits);
    wave_add_visits(vc_sh, visits + 4);
  }
  if (counters) {
    // wave reduction, one atomic per counter per wave
    unsigned long long v[4] = {n_ext, n_sh, n_inc, n_paths};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      unsigned long long x = v[k];
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
      if (lane == 0) atomicAdd(&counters[k], x);
    }
  }
}

// One path traced by one lane with the device functions of the render kernels
// (camera ray, closest hit, shading, shadow ray, bounce), recording per vertex
// rec_i[6 k ..] = (instance id, primitive, half, shadow: -1 none / 0 visible /
// 1 occluded, unique face, 0) and rec_f[10 k ..] = (t, albedo, cos to the light,
// radiance after the vertex, origin xyz and direction xyz of the ray that found
// it); a path that escapes records its escaping ray after its last vertex (ids
// -1, t = +inf).  out[0] = vertices, out[1] = 1 if the path escaped, and
// rec_f[10 kMaxDepth ..] holds the final radiance (three channels with
// principled shading; rec_f[10 k + 3] then holds the red channel).
template <int FMT>
__global__ void k_path_record(SceneView sc, RenderParams rp, int64_t pid, int depth_lds, int32_t* rec_i,
                              float* rec_f, int32_t* out) {
  extern __shared__ uint2 lds[];
  const Stack S = make_stack(lds, depth_lds);
  uint2 spill[kStackTotal];
  if (threadIdx.x != 0) return;
  VisitCounters vc{0, 0, 0, 0};
  PathId id;
  Ray3 r = path_camera_ray(rp, pid, &id);
  float beta = 1.0f, radiance = 0.0f, pdf = 0.0f;
  float beta3[3] = {1.0f, 1.0f, 1.0f}, rad3[3] = {0.0f, 0.0f, 0.0f};  // RGB shading
  const bool rgb = rgb_mode(rp);
  uint32_t ex_rec = kEmpty, ex_qh = kEmpty;
  int n = 0, escaped = 0;
  for (int b = 0; b < rp.depth; ++b) {
    Lane L;
    L.ex_rec = ex_rec;
    L.ex_qh = ex_qh;
    if (lane_init(L, sc, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, 0.0f, kInfF))
      while (!lane_step<FMT, false>(L, sc, S, spill, vc)) {
      }
    if (L.b_rec == kEmpty) {
      const float Le = escape_radiance(sc, rp, r.dx, r.dy, r.dz, pdf);
      radiance += beta * Le;
      for (int k = 0; k < 3; ++k) rad3[k] += beta3[k] * Le;
      if (rgb) radiance = rad3[0];
      escaped = 1;
      // the escaping ray takes the next record (n < depth here)
      rec_i[6 * n + 0] = -1;
      rec_i[6 * n + 1] = -1;
      rec_i[6 * n + 2] = -1;
      rec_i[6 * n + 3] = -1;
      rec_i[6 * n + 4] = -1;
      rec_i[6 * n + 5] = 0;
      rec_f[10 * n + 0] = kInfF;
      rec_f[10 * n + 1] = 0.0f;
      rec_f[10 * n + 2] = 0.0f;
      rec_f[10 * n + 3] = radiance;
      rec_f[10 * n + 4] = r.ox;
      rec_f[10 * n + 5] = r.oy;
      rec_f[10 * n + 6] = r.oz;
      rec_f[10 * n + 7] = r.dx;
      rec_f[10 * n + 8] = r.dy;
      rec_f[10 * n + 9] = r.dz;
      break;
    }
    const uint32_t hqh = L.b_qh;
    const Shade sh = shade_hit(sc, rp, r, L.t_best, L.b_rec, hqh & 0x7FFFFFFFu, hqh >> 31, L.b_u, L.b_v);
    int shadow = -1;
    const NeeSample ns = nee_sample(sc, rp, sh, id.pixel, id.sample, id.view, b);
    float c3[3] = {0.0f, 0.0f, 0.0f};
    PShade ps{};
    if (rgb) ps = principled_vertex(sc, rp, sh, r, c3);
    if (ns.want) {
      float pend3[3] = {0.0f, 0.0f, 0.0f};
      if (rgb) {
        float e[3], e1[3];
        pnee_estimate(ps, c3, ns, e, e1);
        for (int k = 0; k < 3; ++k) pend3[k] = beta3[k] * e[k];
      }
      const float pending = rgb ? pend3[0] : nee_contrib(beta, sh, ns, rp);
      Lane Ls;
      Ls.ex_rec = L.b_rec;
      Ls.ex_qh = hqh;
      if (lane_init(Ls, sc, sh.px, sh.py, sh.pz, ns.dx, ns.dy, ns.dz, 0.0f, ns.tmax)) {
        Ls.any = true;
        while (!lane_step<FMT, false>(Ls, sc, S, spill, vc)) {
        }
      }
      shadow = Ls.b_rec != kEmpty ? 1 : 0;
      if (shadow == 0) {
        radiance += pending;
        for (int k = 0; k < 3; ++k) rad3[k] += pend3[k];
      }
    }
    rec_i[6 * n + 0] = (int32_t)sc.inst[L.b_rec].inst_id;
    rec_i[6 * n + 1] = sc.quad_prim[hqh & 0x7FFFFFFFu];
    rec_i[6 * n + 2] = (int32_t)(hqh >> 31);
    rec_i[6 * n + 3] = shadow;
    rec_i[6 * n + 4] = (int32_t)sh.face;
    rec_i[6 * n + 5] = 0;
    rec_f[10 * n + 0] = L.t_best;
    rec_f[10 * n + 1] = sh.a;
    rec_f[10 * n + 2] = sh.cosl;
    rec_f[10 * n + 3] = radiance;
    rec_f[10 * n + 4] = r.ox;
    rec_f[10 * n + 5] = r.oy;
    rec_f[10 * n + 6] = r.oz;
    rec_f[10 * n + 7] = r.dx;
    rec_f[10 * n + 8] = r.dy;
    rec_f[10 * n + 9] = r.dz;
    ++n;
    if (b == rp.depth - 1) break;
    float dx, dy, dz;
    if (rgb) {
      float w[3], w1[3];
      pdf = pbsdf_bounce(rp, ps, c3, id.pixel, id.sample, id.view, b, &dx, &dy, &dz, w, w1);
      if (!(pdf > 0.0f)) break;  // a direction on the surface: the path ends
      for (int k = 0; k < 3; ++k) beta3[k] *= w[k];
      beta = beta3[0];
    } else {
      pdf = bounce_dir(rp, id.pixel, id.sample, id.view, b, sh, &dx, &dy, &dz);
      beta = beta * sh.a;
    }
    r = Ray3{sh.px, sh.py, sh.pz, dx, dy, dz};
    ex_rec = L.b_rec;
    ex_qh = hqh;
  }
  out[0] = n;
  out[1] = escaped;
  rec_f[10 * kMaxDepth] = rgb ? rad3[0] : radiance;
  rec_f[10 * kMaxDepth + 1] = rgb ? rad3[1] : radiance;
  rec_f[10 * kMaxDepth + 2] = rgb ? rad3[2] : radiance;
}

__global__ void k_start_tick(unsigned long long* t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) t[0] = (unsigned long long)wall_clock64();
}

// ---------------------------------------------------------------- adjoint
// Principled (RGB) form of the adjoint: every vertex's next-event estimate e_k
// and bounce weight w_k are affine in its face's albedo (the base color is the
// material's tint times the albedo, and the sampled directions do not depend on
// it), with derivatives e1_k and w1_k.  With T_k the throughput before vertex k
// and R_k the radiance arriving at k along its bounce (R = e_{k+1} + w_{k+1}
// R_{k+1}, the escape's radiance after the last vertex), the derivative of the
// path value is T_k (e1_k + w1_k R_k), weighted per channel by the pixel's
// gradient.  Called by k_adjoint for scenes with materials.
template <int FMT>
__device__ __forceinline__ void adjoint_rgb(const SceneView& sc, const RenderParams& rp, const float* grad_img,
                                            float* grad_albedo, const Stack& S, uint2* spill, int64_t pid) {
  PathId id;
  Ray3 r = path_camera_ray(rp, pid, &id);
  const int64_t px = rp.cams[id.cam].img_offset + id.local;
  const float g[3] = {grad_img[3 * px] / (float)rp.spp, grad_img[3 * px + 1] / (float)rp.spp,
                      grad_img[3 * px + 2] / (float)rp.spp};
  if (g[0] == 0.0f && g[1] == 0.0f && g[2] == 0.0f) return;
  uint32_t face[kMaxDepth];
  float T[kMaxDepth][3], e[kMaxDepth][3], e1[kMaxDepth][3], w[kMaxDepth][3], w1[kMaxDepth][3];
  int K = 0;
  bool escaped = false;
  float beta[3] = {1.0f, 1.0f, 1.0f}, pdf = 0.0f;
  Lane L;
  VisitCounters vc{0, 0, 0, 0};
  L.ex_rec = kEmpty;
  L.ex_qh = kEmpty;
  for (int b = 0; b < rp.depth; ++b) {
    if (lane_init(L, sc, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, 0.0f, kInfF))
      while (!lane_step<FMT, false>(L, sc, S, spill, vc)) {
      }
    if (L.b_rec == kEmpty) {
      escaped = true;
      break;
    }
    const uint32_t hrec = L.b_rec, hqh = L.b_qh;
    const Shade s = shade_hit(sc, rp, r, L.t_best, hrec, hqh & 0x7FFFFFFFu, hqh >> 31, L.b_u, L.b_v);
    float c[3];
    const PShade ps = principled_vertex(sc, rp, s, r, c);
    NeeSample ns = nee_sample(sc, rp, s, id.pixel, id.sample, id.view, b);
    if (ns.want) {
      L.ex_rec = hrec;
      L.ex_qh = hqh;
      if (lane_init(L, sc, s.px, s.py, s.pz, ns.dx, ns.dy, ns.dz, 0.0f, ns.tmax)) {
        L.any = true;
        while (!lane_step<FMT, false>(L, sc, S, spill, vc)) {
        }
      }
      ns.want = L.b_rec == kEmpty;  // the estimate counts only when the light is visible
    }
    pnee_estimate(ps, c, ns, e[K], e1[K]);
    face[K] = s.param;
    for (int k = 0; k < 3; ++k) {
      T[K][k] = beta[k];
      w[K][k] = 0.0f;
      w1[K][k] = 0.0f;
    }
    ++K;
    if (b == rp.depth - 1) break;
    float dx, dy, dz;
    pdf = pbsdf_bounce(rp, ps, c, id.pixel, id.sample, id.view, b, &dx, &dy, &dz, w[K - 1], w1[K - 1]);
    if (!(pdf > 0.0f)) break;
    for (int k = 0; k < 3; ++k) beta[k] *= w[K - 1][k];
    r = Ray3{s.px, s.py, s.pz, dx, dy, dz};
    L.ex_rec = hrec;
    L.ex_qh = hqh;
  }
  const float Le = escaped ? escape_radiance(sc, rp, r.dx, r.dy, r.dz, pdf) : 0.0f;
  float R[3] = {Le, Le, Le};
  // per channel with RGB texels (parameter 3 texel + channel), summed otherwise
  const bool rgb_tex = sc.tex_res > 0 && sc.tex_ch == 3;
  for (int k = K - 1; k >= 0; --k) {
    float d = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
      const float dch = g[ch] * (T[k][ch] * (e1[k][ch] + w1[k][ch] * R[ch]));
      if (rgb_tex) unsafeAtomicAdd(&grad_albedo[3 * (size_t)face[k] + ch], dch);
      d += dch;
      R[ch] = e[k][ch] + w[k][ch] * R[ch];
    }
    if (!rgb_tex) unsafeAtomicAdd(&grad_albedo[face[k]], d);
  }
}

// One lane per path: replay the path from its RNG counters with the same device
// functions (identical hits), keep per vertex the face, beta_k and the NEE factor
// c_k = (E / pi) cos_L V_k, then walk back: with V_K the sky (or environment)
// radiance of the escaping ray if the path escaped
// (else 0) and V_k = a_k (c_k + V_{k+1}), the derivative of the path value with
// respect to the albedo at vertex k is beta_k (c_k + V_{k+1}).
template <int FMT>
__global__ void k_adjoint(SceneView sc, RenderParams rp, const float* grad_img, float* grad_albedo, int depth_lds) {
  extern __shared__ uint2 lds[];
  const int lane = threadIdx.x & 63;
  const Stack S = make_stack(lds, depth_lds);
  uint2 spill[kStackTotal];
  const int64_t pid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= rp.n_paths) return;
  if (rgb_mode(rp)) {
    adjoint_rgb<FMT>(sc, rp, grad_img, grad_albedo, S, spill, pid);
    return;
  }
  PathId id;
  Ray3 r = path_camera_ray(rp, pid, &id);
  // id.local < tw * th: the index stays inside the camera's image rectangle
  const float g = grad_img[rp.cams[id.cam].img_offset + id.local] / (float)rp.spp;
  if (g == 0.0f) return;
  uint32_t face[kMaxDepth];
  float betak[kMaxDepth], ck[kMaxDepth], ak[kMaxDepth];
  int K = 0;
  bool escaped = false;
  float beta = 1.0f, pdf = 0.0f;
  Lane L;
  VisitCounters vc{0, 0, 0, 0};
  L.ex_rec = kEmpty;
  L.ex_qh = kEmpty;
  for (int b = 0; b < rp.depth; ++b) {
    if (lane_init(L, sc, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz, 0.0f, kInfF))
      while (!lane_step<FMT, false>(L, sc, S, spill, vc)) {
      }
    if (L.b_rec == kEmpty) {
      escaped = true;
      break;
    }
    const uint32_t hrec = L.b_rec, hqh = L.b_qh;
    const Shade s = shade_hit(sc, rp, r, L.t_best, hrec, hqh & 0x7FFFFFFFu, hqh >> 31, L.b_u, L.b_v);
    float c = 0.0f;
    const NeeSample ns = nee_sample(sc, rp, s, id.pixel, id.sample, id.view, b);
    if (ns.want) {
      L.ex_rec = hrec;
      L.ex_qh = hqh;
      if (lane_init(L, sc, s.px, s.py, s.pz, ns.dx, ns.dy, ns.dz, 0.0f, ns.tmax)) {
        L.any = true;
        while (!lane_step<FMT, false>(L, sc, S, spill, vc)) {
        }
      }
      if (L.b_rec == kEmpty) c = ns.c;
    }
    face[K] = s.param;  // taken at shading, before the shadow ray reuses the lane's (u, v)
    betak[K] = beta;
    ck[K] = c;
    ak[K] = s.a;
    ++K;
    if (b == rp.depth - 1) break;
    float dx, dy, dz;
    pdf = bounce_dir(rp, id.pixel, id.sample, id.view, b, s, &dx, &dy, &dz);
    r = Ray3{s.px, s.py, s.pz, dx, dy, dz};
    beta = beta * s.a;
    L.ex_rec = hrec;
    L.ex_qh = hqh;
  }
  float V = escaped ? escape_radiance(sc, rp, r.dx, r.dy, r.dz, pdf) : 0.0f;
  for (int k = K - 1; k >= 0; --k) {
    const float cv = ck[k] + V;
    unsafeAtomicAdd(&grad_albedo[face[k]], g * (betak[k] * cv));
    V = ak[k] * cv;
  }
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Plain stages of bounce b: closest hits of its extension queue, shading,
// occlusion of its shadow queue, shadow resolution; one ray per lane.
template <int FMT, bool COUNT>
static void wavefront_bounce(const SceneView& sc, const RenderParams& rp, const PlainBuffers& pb, int b,
                             const TraceLaunch& tl, const RenderExtras& ex, hipStream_t s) {
  const unsigned gp = blocks(rp.n_paths, 256);
  const unsigned gs = blocks(rp.n_paths, kShadeBlock);
  const unsigned gt = blocks(rp.n_paths, tl.block);
  const size_t lds = (size_t)tl.block * tl.stack_depth * kStackEntryBytes;
  const ExtQueue& qin = pb.q[b & 1];
  const ExtQueue& qout = pb.q[(b + 1) & 1];
  uint32_t* cin = pb.counts + b;
  uint32_t* cout = pb.counts + b + 1;
  uint32_t* csq = pb.counts + kMaxDepth + 1 + b;
  unsigned long long* vis_sh = ex.visits ? ex.visits + 4 : nullptr;
  hipEvent_t ev = stage_begin(ex.log, s);
  const int feat = scene_features(sc, rp);
  if (feat & kFeatTex)
    hipLaunchKernelGGL((k_trace_queue<FMT, false, COUNT, kFeatTex>), dim3(gt), dim3(tl.block), lds, s, sc, rp, qin,
                       pb.sq, cin, pb.hits, pb.occ, tl.stack_depth, ex.visits);
  else
    hipLaunchKernelGGL((k_trace_queue<FMT, false, COUNT, 0>), dim3(gt), dim3(tl.block), lds, s, sc, rp, qin, pb.sq,
                       cin, pb.hits, pb.occ, tl.stack_depth, ex.visits);
  stage_end(ex.log, 0, ev, s);
  ev = stage_begin(ex.log, s);
  hipLaunchKernelGGL(k_shade, dim3(gs), dim3(kShadeBlock), 0, s, sc, rp, b, qin, cin, pb.hits, qout, cout, pb.sq, csq,
                     ex.dump, ex.dump_cap, ex.dump_count, ex.view_done);
  stage_end(ex.log, 2, ev, s);
  ev = stage_begin(ex.log, s);
  if (feat & kFeatArea)
    hipLaunchKernelGGL((k_trace_queue<FMT, true, COUNT, kFeatArea>), dim3(gt), dim3(tl.block), lds, s, sc, rp, qin,
                       pb.sq, csq, pb.hits, pb.occ, tl.stack_depth, vis_sh);
  else
    hipLaunchKernelGGL((k_trace_queue<FMT, true, COUNT, 0>), dim3(gt), dim3(tl.block), lds, s, sc, rp, qin, pb.sq, csq,
                       pb.hits, pb.occ, tl.stack_depth, vis_sh);
  stage_end(ex.log, 1, ev, s);
  ev = stage_begin(ex.log, s);
  hipLaunchKernelGGL(k_shadow_resolve, dim3(gp), dim3(256), 0, s, rp, pb.sq, csq, pb.occ, b, ex.view_done);
  stage_end(ex.log, 2, ev, s);
}

template <int FMT, bool COUNT>
static void mixed_launch(const SceneView& sc, const RenderParams& rp, const PlainBuffers& pb, const TraceLaunch& tl,
                         const RenderExtras& ex, const ExtQueue& eq, const uint32_t* cext, const uint32_t* csh,
                         int slot, hipStream_t s) {
  const size_t lds = (size_t)tl.block * tl.stack_depth * kStackEntryBytes;
  hipEvent_t ev = stage_begin(ex.log, s);
  unsigned long long* work = pb.work + (size_t)slot * kClaimWords;
#define RTQ_MIXED(F)                                                                                             \
  hipLaunchKernelGGL((k_trace_queue_mixed<FMT, COUNT, F>), dim3(tl.grid), dim3(tl.block), lds, s, sc, rp, eq, cext, \
                     pb.sq, csh, pb.hits, pb.occ, tl.stack_depth, tl.refill, work, ex.visits)
  switch (scene_features(sc, rp)) {
    case 0: RTQ_MIXED(0); break;
    case kFeatTex: RTQ_MIXED(kFeatTex); break;
    case kFeatArea: RTQ_MIXED(kFeatArea); break;
    default: RTQ_MIXED(kFeatTex | kFeatArea); break;
  }
#undef RTQ_MIXED
  stage_end(ex.log, 0, ev, s);
}

// Persistent stages: traverse(extension 0); then per bounce b: shade(b),
// traverse(shadow b + extension b + 1), resolve(b).
template <int FMT, bool COUNT>
static void wavefront_persistent(const SceneView& sc, const RenderParams& rp, const PlainBuffers& pb,
                                 const TraceLaunch& tl, const RenderExtras& ex, hipStream_t s) {
  const unsigned gp = blocks(rp.n_paths, 256);
  const unsigned gs = blocks(rp.n_paths, kShadeBlock);
  const uint32_t* zero = pb.counts + 2 * kMaxDepth + 1;  // cleared, never written
  mixed_launch<FMT, COUNT>(sc, rp, pb, tl, ex, pb.q[0], pb.counts, zero, 0, s);
  for (int b = 0; b < rp.depth; ++b) {
    const ExtQueue& qin = pb.q[b & 1];
    const ExtQueue& qout = pb.q[(b + 1) & 1];
    uint32_t* cin = pb.counts + b;
    uint32_t* cout = pb.counts + b + 1;
    uint32_t* csq = pb.counts + kMaxDepth + 1 + b;
    hipEvent_t ev = stage_begin(ex.log, s);
    hipLaunchKernelGGL(k_shade, dim3(gs), dim3(kShadeBlock), 0, s, sc, rp, b, qin, cin, pb.hits, qout, cout, pb.sq,
                       csq, ex.dump, ex.dump_cap, ex.dump_count, ex.view_done);
    stage_end(ex.log, 2, ev, s);
    // after the last bounce the extension count stays zero: shadow rays only
    mixed_launch<FMT, COUNT>(sc, rp, pb, tl, ex, qout, cout, csq, b + 1, s);
    ev = stage_begin(ex.log, s);
    hipLaunchKernelGGL(k_shadow_resolve, dim3(gp), dim3(256), 0, s, rp, pb.sq, csq, pb.occ, b, ex.view_done);
    stage_end(ex.log, 2, ev, s);
  }
}

hipError_t launch_render_wavefront(const SceneView& sc, const RenderParams& rp, const PlainBuffers& pb, int fmt,
                                   const TraceLaunch& tl, float* image, int64_t n_pixels, const RenderExtras& ex,
                                   hipStream_t s) {
  const unsigned gp = blocks(rp.n_paths, 256);
  hipEvent_t ev = stage_begin(ex.log, s);
  if (ex.start_tick) hipLaunchKernelGGL(k_start_tick, dim3(1), dim3(64), 0, s, ex.start_tick);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, pb.counts, 2 * kMaxDepth + 2);
  hipError_t e = launch_zero_u64(pb.work, (kMaxDepth + 1) * kClaimWords, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_raygen, dim3(gp), dim3(256), 0, s, rp, pb.q[0], pb.counts);
  stage_end(ex.log, 2, ev, s);
  const bool cnt = ex.visits != nullptr;
  with_codec(fmt, [&](auto c) {
    constexpr int F = decltype(c)::value;
    if (tl.persistent) {
      if (cnt) wavefront_persistent<F, true>(sc, rp, pb, tl, ex, s);
      else wavefront_persistent<F, false>(sc, rp, pb, tl, ex, s);
    } else {
      for (int b = 0; b < rp.depth; ++b) {
        if (cnt) wavefront_bounce<F, true>(sc, rp, pb, b, tl, ex, s);
        else wavefront_bounce<F, false>(sc, rp, pb, b, tl, ex, s);
      }
    }
  });
  ev = stage_begin(ex.log, s);
  hipLaunchKernelGGL(k_accum, dim3(blocks(n_pixels, 256)), dim3(256), 0, s, rp, image, n_pixels);
  if (ex.counters)
    hipLaunchKernelGGL(k_plain_stats, dim3(1), dim3(64), 0, s, pb.counts, rp.depth, rp.n_paths, ex.counters);
  stage_end(ex.log, 2, ev, s);
  return hipGetLastError();
}

template <int FMT, bool TS, bool COUNT>
static void persistent_launch(const SceneView& sc, const RenderParams& rp, const TraceLaunch& tl,
                              const RenderExtras& ex, hipStream_t s) {
  const size_t lds = (size_t)tl.block * tl.stack_depth * kStackEntryBytes;
#define RTQ_MEGA(F)                                                                                        \
  hipLaunchKernelGGL((k_render_persistent<FMT, TS, COUNT, F>), dim3(tl.grid), dim3(tl.block), lds, s, sc, rp, \
                     tl.stack_depth, tl.refill, tl.counter, ex.counters, ex.view_done, ex.visits)
  switch (scene_features(sc, rp)) {
    case 0: RTQ_MEGA(0); break;
    case kFeatTex: RTQ_MEGA(kFeatTex); break;
    case kFeatArea: RTQ_MEGA(kFeatArea); break;
    default: RTQ_MEGA(kFeatTex | kFeatArea); break;
  }
#undef RTQ_MEGA
}

hipError_t launch_render_megakernel(const SceneView& sc, const RenderParams& rp, int fmt, const TraceLaunch& tl,
                                    float* image, int64_t n_pixels, const RenderExtras& ex, hipStream_t s) {
  hipEvent_t ev = stage_begin(ex.log, s);
  hipError_t e = launch_zero_u64(tl.counter, kClaimWords, s);
  if (e != hipSuccess) return e;
  if (ex.start_tick) hipLaunchKernelGGL(k_start_tick, dim3(1), dim3(64), 0, s, ex.start_tick);
  stage_end(ex.log, 2, ev, s);
  ev = stage_begin(ex.log, s);
  const bool ts = ex.view_done != nullptr, cnt = ex.visits != nullptr;
  with_codec(fmt, [&](auto c) {
    constexpr int F = decltype(c)::value;
    if (cnt) {
      if (ts) persistent_launch<F, true, true>(sc, rp, tl, ex, s);
      else persistent_launch<F, false, true>(sc, rp, tl, ex, s);
    } else {
      if (ts) persistent_launch<F, true, false>(sc, rp, tl, ex, s);
      else persistent_launch<F, false, false>(sc, rp, tl, ex, s);
    }
  });
  stage_end(ex.log, 0, ev, s);
  ev = stage_begin(ex.log, s);
  hipLaunchKernelGGL(k_accum, dim3(blocks(n_pixels, 256)), dim3(256), 0, s, rp, image, n_pixels);
  stage_end(ex.log, 2, ev, s);
  return hipGetLastError();
}

hipError_t launch_path_record(const SceneView& sc, const RenderParams& rp, int fmt, int stack_depth, int64_t pid,
                              int32_t* rec_i, float* rec_f, int32_t* out, hipStream_t s) {
  const size_t lds = (size_t)64 * stack_depth * kStackEntryBytes;
  with_codec(fmt, [&](auto c) {
    hipLaunchKernelGGL((k_path_record<decltype(c)::value>), dim3(1), dim3(64), lds, s, sc, rp, pid, stack_depth,
                       rec_i, rec_f, out);
  });
  return hipGetLastError();
}

hipError_t launch_set_keys(uint32_t* keys, uint32_t k0, uint32_t k1, uint32_t acc, hipStream_t s) {
  hipLaunchKernelGGL(k_set_keys, dim3(1), dim3(64), 0, s, keys, k0, k1, acc);
  return hipGetLastError();
}

hipError_t launch_adjoint(const SceneView& sc, const RenderParams& rp, int fmt, int stack_depth, int block,
                          const float* grad_img, float* grad_albedo, hipStream_t s) {
  const size_t lds = (size_t)block * stack_depth * kStackEntryBytes;
  const unsigned g = blocks(rp.n_paths, block);
  with_codec(fmt, [&](auto c) {
    hipLaunchKernelGGL((k_adjoint<decltype(c)::value>), dim3(g), dim3(block), lds, s, sc, rp, grad_img, grad_albedo,
                       stack_depth);
  });
  return hipGetLastError();
}

}  // namespace rtq
