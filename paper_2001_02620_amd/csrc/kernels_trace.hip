// Ray-query kernels: closest hit and occlusion over the two-level quad BVH, in a
// plain schedule (one ray per lane for its whole traversal) and a persistent
// schedule (resident waves pull rays from a shared counter and refill lanes
// whose ray has finished, so the SIMD stays busy on incoherent rays).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "kernels.h"
#include "trace_device.h"

namespace rtq {

template <bool ANY>
__device__ __forceinline__ void store_result(const Lane& L, const SceneView& sc, int64_t i, const HitsSoA& h,
                                             uint8_t* occ) {
  const bool hit = L.b_rec != kEmpty;
  if (ANY) {
    occ[i] = hit ? 1 : 0;
    return;
  }
  const int32_t prim = hit ? sc.quad_prim[L.b_qh & 0x7FFFFFFFu] : -1;
  // a capsule hit carries its axis position y: u is the curve parameter (j + y) / 8
  const bool cap = hit && (sc.inst[L.b_rec].proto & kProtoCurve) != 0u;
  h.t[i] = hit ? L.t_best : kInfF;
  h.u[i] = hit ? (cap ? ((float)(prim % kCapsPerCurve) + L.b_u) * (1.0f / kCapsPerCurve) : L.b_u) : 0.0f;
  h.v[i] = hit ? L.b_v : 0.0f;
  h.inst[i] = hit ? (int32_t)sc.inst[L.b_rec].inst_id : -1;
  h.prim[i] = prim;
  if (h.ref) reinterpret_cast<uint2*>(h.ref)[i] = hit ? make_uint2(L.b_rec, L.b_qh) : make_uint2(kEmpty, kEmpty);
}

template <bool ANY>
__device__ __forceinline__ bool load_ray(Lane& L, const SceneView& sc, const RaysSoA& r, int64_t i) {
  const uint2 ex = r.exclude ? reinterpret_cast<const uint2*>(r.exclude)[i] : make_uint2(kEmpty, kEmpty);
  L.ex_rec = ex.x;
  L.ex_qh = ex.y;
  const bool ok = lane_init(L, sc, r.ox[i], r.oy[i], r.oz[i], r.dx[i], r.dy[i], r.dz[i], r.tmin[i], r.tmax[i]);
  L.any = ANY;
  return ok;
}

template <bool COUNT>
__device__ __forceinline__ void store_visits(uint32_t* visits, uint32_t* lane_stats, int64_t i,
                                             const VisitCounters& vc) {
  if (COUNT) {
    if (visits) reinterpret_cast<uint4*>(visits)[i] = make_uint4(vc.tlas, vc.inst, vc.blas, vc.quads);
    if (lane_stats) reinterpret_cast<uint2*>(lane_stats)[i] = make_uint2(vc.iters, vc.fp64);
  }
}

template <int FMT, bool ANY, bool COUNT>
__global__ void k_trace_plain(SceneView sc, RaysSoA rays, int64_t n, HitsSoA hits, uint8_t* occ, uint32_t* visits,
                              uint32_t* lane_stats, int depth) {
  extern __shared__ uint2 lds[];
  const int lane = threadIdx.x & 63;
  const Stack S = make_stack(lds, depth);
  uint2 spill[kStackTotal];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Lane L;
  VisitCounters vc{0, 0, 0, 0};
  if (load_ray<ANY>(L, sc, rays, i))
    while (!lane_step<FMT, COUNT>(L, sc, S, spill, vc)) {
    }
  store_result<ANY>(L, sc, i, hits, occ);
  store_visits<COUNT>(visits, lane_stats, i, vc);
}

template <int FMT, bool ANY, bool COUNT>
__global__ void k_trace_persistent(SceneView sc, RaysSoA rays, int64_t n, HitsSoA hits, uint8_t* occ,
                                   uint32_t* visits, uint32_t* lane_stats, int depth, int refill,
                                   unsigned long long* counter) {
  extern __shared__ uint2 lds[];
  const int lane = threadIdx.x & 63;
  const Stack S = make_stack(lds, depth);
  uint2 spill[kStackTotal];
  Lane L;
  VisitCounters vc{0, 0, 0, 0};
  bool has = false;
  bool exhausted = n == 0;  // wave-uniform
  ClaimState claim = claim_init();
  int64_t idx = -1;
  for (;;) {
    const unsigned long long idle = __ballot(!has);
    const int nidle = __popcll(idle);
    if (!exhausted && (nidle >= refill || nidle == 64)) {
      const int64_t k = claim_take(claim, counter, n, idle, nidle, &exhausted);
      if (k >= 0) {
        idx = k;
        vc = VisitCounters{0, 0, 0, 0};
        if (load_ray<ANY>(L, sc, rays, idx)) {
          has = true;
        } else {
          store_result<ANY>(L, sc, idx, hits, occ);
          store_visits<COUNT>(visits, lane_stats, idx, vc);
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
          store_result<ANY>(L, sc, idx, hits, occ);
          store_visits<COUNT>(visits, lane_stats, idx, vc);
          has = false;
          break;
        }
        if (!exhausted && __popcll(__ballot(1)) <= 64 - refill) break;
      }
    }
  }
}

// Reference: every instance, every quad or capsule, the same leaf code.
__global__ void k_trace_brute(SceneView sc, RaysSoA rays, int64_t n, HitsSoA hits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Lane L;
  if (load_ray<false>(L, sc, rays, i)) {
    for (uint32_t r = 0; r < sc.n_rec; ++r) {
      uint32_t root;
      enter_instance(L, sc, r, &root);
      leaf_quads(L, sc, sc.rec_qfirst[r], sc.rec_nq[r]);
    }
  }
  store_result<false>(L, sc, i, hits, nullptr);
}

template <int FMT, bool ANY, bool COUNT>
static hipError_t launch3(const SceneView& sc, const RaysSoA& r, int64_t n, const HitsSoA& h, uint8_t* occ,
                          uint32_t* visits, uint32_t* lane_stats, const TraceLaunch& tl, hipStream_t s) {
  const size_t lds = (size_t)tl.block * tl.stack_depth * kStackEntryBytes;
  if (tl.persistent) {
    hipError_t e = launch_zero_u64(tl.counter, kClaimWords, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_trace_persistent<FMT, ANY, COUNT>), dim3(tl.grid), dim3(tl.block), lds, s, sc, r, n, h,
                       occ, visits, lane_stats, tl.stack_depth, tl.refill, tl.counter);
  } else {
    const unsigned g = (unsigned)((n + tl.block - 1) / tl.block);
    hipLaunchKernelGGL((k_trace_plain<FMT, ANY, COUNT>), dim3(g), dim3(tl.block), lds, s, sc, r, n, h, occ, visits,
                       lane_stats, tl.stack_depth);
  }
  return hipGetLastError();
}

template <int FMT>
static hipError_t launch2(const SceneView& sc, const RaysSoA& r, int64_t n, const HitsSoA* h, uint8_t* occ,
                          uint32_t* visits, uint32_t* lane_stats, const TraceLaunch& tl, hipStream_t s) {
  const HitsSoA hh = h ? *h : HitsSoA{};
  const bool cnt = visits || lane_stats;
  if (occ) {
    return cnt ? launch3<FMT, true, true>(sc, r, n, hh, occ, visits, lane_stats, tl, s)
               : launch3<FMT, true, false>(sc, r, n, hh, occ, visits, lane_stats, tl, s);
  }
  return cnt ? launch3<FMT, false, true>(sc, r, n, hh, occ, visits, lane_stats, tl, s)
             : launch3<FMT, false, false>(sc, r, n, hh, occ, visits, lane_stats, tl, s);
}

hipError_t launch_trace(const SceneView& sc, const RaysSoA& rays, int64_t n, const HitsSoA* hits, uint8_t* occ,
                        uint32_t* visits, uint32_t* lane_stats, const TraceLaunch& tl, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return with_codec(tl.fmt, [&](auto c) {
    return launch2<decltype(c)::value>(sc, rays, n, hits, occ, visits, lane_stats, tl, s);
  });
}

// Claim counters of the allocation-free ray query (rtq_trace_closest_noalloc):
// one persistent launch's worth, kClaimWords 64-bit words (1 KiB), held by every
// device the library runs on until the process ends.  Host code never uses
// this name as an address: noalloc_counters() returns the device's own address
// of the array.
static __device__ __align__(256) unsigned long long scratch[kClaimWords];

hipError_t noalloc_counters(int device, unsigned long long** out) {
  static std::mutex mu;
  static std::map<int, unsigned long long*> addr;  // per device, looked up once
  std::lock_guard<std::mutex> lock(mu);
  const auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  addr[device] = static_cast<unsigned long long*>(p);
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_trace_brute(const SceneView& sc, const RaysSoA& rays, int64_t n, const HitsSoA& hits,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_brute, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, sc, rays, n, hits);
  return hipGetLastError();
}

}  // namespace rtq
