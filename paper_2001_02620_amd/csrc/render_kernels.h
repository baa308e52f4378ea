// Internal interface of the path-tracing kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "render_device.h"

namespace rtq {

constexpr int kMaxDepth = 16;  // closest-hit rays per path

// Extension-ray queue (structure of arrays).  ex_qh packs the spawning
// triangle's leaf-ordered quad (bits 0..30) and half (bit 31); kEmpty = none.
struct ExtQueue {
  float *ox, *oy, *oz, *dx, *dy, *dz;
  uint32_t* pid;
  float* beta;
  uint32_t *ex_rec, *ex_qh;
  float* pdf;  // density of the bounce that drew the ray (written when the
               // environment is sampled by next-event estimation)
  float *beta_g, *beta_b;  // green and blue throughput (RGB shading; beta holds red)
};

// Shadow-ray queue: direction is the light direction.
struct ShadowQueue {
  float *ox, *oy, *oz;
  uint32_t* pid;
  float* contrib;
  uint32_t *ex_rec, *ex_qh;
  float *dx, *dy, *dz, *tmax;  // written only for a scene with area lights
  float *contrib_g, *contrib_b;  // green and blue contributions (RGB shading; contrib holds red)
};

// Closest hits of an extension queue (internal form).
struct QueueHits {
  float* t;
  uint32_t* rec;
  uint32_t* qh;
  float *u, *v;  // written only for a scene with textures
};

struct PlainBuffers {
  ExtQueue q[2];
  ShadowQueue sq;
  QueueHits hits;
  uint8_t* occ;
  uint32_t* counts;  // [0, kMaxDepth]: extension queue sizes; [kMaxDepth + 1, ...): shadow queue sizes
  unsigned long long* work;  // [(kMaxDepth + 1) kClaimWords]: claim counters of the persistent traversal launches
};

// Host-side log of HIP events around a render call's launches (owned by the
// scene).  stage_begin returns nullptr when log is nullptr or full; stage_end
// records the matching end event and files the pair under `stage`
// (0 closest-hit traversal, 1 shadow traversal, 2 other).
struct StageLog;
hipEvent_t stage_begin(StageLog* log, hipStream_t s);
void stage_end(StageLog* log, int stage, hipEvent_t begin, hipStream_t s);

// Optional instrumentation of a render call.
struct RenderExtras {
  unsigned long long* counters;    // [4] closest, shadow, incoherent rays, paths
  unsigned long long* visits;      // [8] top nodes, instances, bottom nodes, quads: closest-hit rays, then shadow rays
  float* dump;                     // 8 x dump_cap SoA
  long long dump_cap;
  unsigned long long* dump_count;
  unsigned long long* view_done;
  unsigned long long* start_tick;
  StageLog* log;                   // event log of a timed call, or nullptr
};

// Multi-kernel wavefront frame; tl.persistent selects lane-refilling traversal stages.
hipError_t launch_render_wavefront(const SceneView& sc, const RenderParams& rp, const PlainBuffers& pb, int fmt,
                                   const TraceLaunch& tl, float* image, int64_t n_pixels, const RenderExtras& ex,
                                   hipStream_t s);
// Single persistent launch per frame.
hipError_t launch_render_megakernel(const SceneView& sc, const RenderParams& rp, int fmt, const TraceLaunch& tl,
                                    float* image, int64_t n_pixels, const RenderExtras& ex, hipStream_t s);
hipError_t launch_adjoint(const SceneView& sc, const RenderParams& rp, int fmt, int stack_depth, int block,
                          const float* grad_img, float* grad_albedo, hipStream_t s);
// Trace path `pid` alone and record its vertices (see k_path_record).
hipError_t launch_path_record(const SceneView& sc, const RenderParams& rp, int fmt, int stack_depth, int64_t pid,
                              int32_t* rec_i, float* rec_f, int32_t* out, hipStream_t s);
// Write the call's RNG key to device memory (kept outside captured graphs, so a
// replayed frame picks up the key of its own call).
hipError_t launch_set_keys(uint32_t* keys, uint32_t k0, uint32_t k1, uint32_t acc, hipStream_t s);

}  // namespace rtq
