// Host-callable launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "rtq_layout.h"
#include "trace_device.h"

namespace rtq {

// Call f with std::integral_constant<int, CODEC> for the run-time node codec id
// (kCodecF32, kCodecQ8, kCodecQ8W8, kCodecQ8W2, each with or without
// kCodecCurves), so a launcher instantiates its kernels once per codec.
template <class F>
decltype(auto) with_codec(int fmt, F&& f) {
  constexpr int C = kCodecCurves;
  switch (fmt) {
    case kCodecQ8: return f(std::integral_constant<int, kCodecQ8>{});
    case kCodecQ8W8: return f(std::integral_constant<int, kCodecQ8W8>{});
    case kCodecQ8W2: return f(std::integral_constant<int, kCodecQ8W2>{});
    case kCodecF32 | C: return f(std::integral_constant<int, kCodecF32 | C>{});
    case kCodecQ8 | C: return f(std::integral_constant<int, kCodecQ8 | C>{});
    case kCodecQ8W8 | C: return f(std::integral_constant<int, kCodecQ8W8 | C>{});
    case kCodecQ8W2 | C: return f(std::integral_constant<int, kCodecQ8W2 | C>{});
    default: return f(std::integral_constant<int, kCodecF32>{});
  }
}

hipError_t launch_invert_affine(const float* X, const int32_t* proto, const uint32_t* proto_root,
                                const uint32_t* face_base, const uint32_t* proto_flags, int64_t n, InstRec* out,
                                float* cond, int32_t* status, hipStream_t s);
hipError_t launch_instance_aabb(const float* X, const int32_t* proto, const float* verts, const int64_t* vert_off,
                                const float* cond, int64_t n, float* box, hipStream_t s);
// out[k] = in[order[k]] with its bottom-level entry reference replaced by root[k].
hipError_t launch_gather_inst(const InstRec* in, const uint32_t* order, const uint32_t* root, int64_t n, InstRec* out,
                              hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);

struct RaysSoA {
  const float *ox, *oy, *oz, *dx, *dy, *dz, *tmin, *tmax;
  const uint32_t* exclude;  // optional: per ray (record, quad | half << 31) of the triangle it leaves
};
struct HitsSoA {
  float *t, *u, *v;
  int32_t *inst, *prim;
  uint32_t* ref;  // optional: per ray (record, quad | half << 31) of the hit
};

struct TraceLaunch {
  int fmt;          // node codec: kCodecF32, kCodecQ8, kCodecQ8W8 or kCodecQ8W2, | kCodecCurves
  int persistent;   // 0 plain, 1 persistent with refill
  int stack_depth;  // LDS entries per lane
  int block;        // threads per block
  int grid;         // persistent: blocks
  int refill;       // persistent: refill threshold (idle lanes)
  unsigned long long* counter;  // persistent: device ray counter (zeroed by the launcher)
};

hipError_t launch_trace(const SceneView& sc, const RaysSoA& rays, int64_t n, const HitsSoA* hits, uint8_t* occ,
                        uint32_t* visits, uint32_t* lane_stats, const TraceLaunch& tl, hipStream_t s);
// Device address of the allocation-free query's claim counters (kClaimWords
// words, a static device array) on `device`; looked up once per device.
hipError_t noalloc_counters(int device, unsigned long long** out);
hipError_t launch_trace_brute(const SceneView& sc, const RaysSoA& rays, int64_t n, const HitsSoA& hits,
                              hipStream_t s);

}  // namespace rtq
