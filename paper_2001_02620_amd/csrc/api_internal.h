// Library-internal state behind the opaque rtq_scene handle.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/rtq.h"
#include "bvh_build.h"
#include "kernels.h"
#include "rtq_layout.h"
#include "trace_device.h"

namespace rtq {

// Device allocations owned together; freed by release() or on destruction, so
// an early return or an exception on a failure path leaks nothing.
struct DeviceBuffers {
  std::vector<void*> ptrs;
  size_t total = 0;
  DeviceBuffers() = default;
  DeviceBuffers(const DeviceBuffers&) = delete;
  DeviceBuffers& operator=(const DeviceBuffers&) = delete;
  ~DeviceBuffers() { release(); }
  void* alloc(size_t bytes, hipError_t* err);
  void release();
};

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);

}  // namespace rtq

struct rtq_host_bvh {
  rtq::Bvh bvh;
  std::vector<rtq::NodeF32> f32;  // the device FP32 nodes (4-wide trees only)
};

struct rtq_scene {
  static constexpr int kCounterSlots = 256;
  int device = 0;
  int formats = 0;
  int width = 4;  // children per node (2, 4 or 8), every level
  int n_cu = 256;
  int max_lds = 65536;  // bytes of LDS one block may use
  int32_t n_protos = 0;
  int64_t n_inst = 0, n_quads = 0, n_instanced_quads = 0;
  int64_t n_curves = 0, n_caps = 0;  // unique curves and their capsules
  int64_t n_faces = 0;               // unique faces: quads and curves
  int64_t n_rec = 0;  // top-level entries (instances, opened ones counted per subtree)
  int64_t tlas_nodes = 0, blas_nodes = 0;
  int tlas_depth = 0, blas_depth = 0;
  double build_seconds = 0.0;
  double build_phase[4] = {0.0, 0.0, 0.0, 0.0};  // see rtq_scene_info.build_phase_seconds
  float pad_rel = 0.0f;
  // device data (owned by bufs)
  float p_world = 0.0f;    // bound on |world coordinate| of every top-level plane
  uint32_t tlas_root = 0;  // top-level root: the nodes after every bottom level
  void* nodes_f32 = nullptr;  // [bottom levels | top level], FP32 nodes
  void* nodes_q8 = nullptr;   // same topology, quantized nodes
  float* rec_pmax = nullptr;  // per instance record: bound on |object coordinate| of its prototype's planes
  float4* quads = nullptr;      // leaf-ordered primitives: quads and capsules, 3 float4 each
  int32_t* quad_prim = nullptr; // leaf order -> primitive index within its prototype
  rtq::InstRec* inst = nullptr;
  uint32_t* rec_qfirst = nullptr;  // per record: quad range of the subtree it enters
  uint32_t* rec_nq = nullptr;
  float* albedo = nullptr;
  float* tex = nullptr;  // per-face textures (own allocation, rtq_scene_set_textures)
  int32_t tex_res = 0;
  int32_t tex_ch = 1;  // channels per texel: 1 or 3
  size_t tex_bytes = 0;
  float* env = nullptr;  // environment map (own allocation, rtq_scene_set_environment)
  int32_t env_w = 0, env_h = 0;
  size_t env_bytes = 0;
  unsigned long long* env_T = nullptr;  // its sampling table (own allocation)
  void* mats = nullptr;        // principled materials (rtq::MatDev, own allocation), or null
  uint8_t* face_mat = nullptr; // material of each unique face (own allocation)
  int32_t n_mat = 0;
  size_t mat_bytes = 0;
  unsigned long long* counters = nullptr;  // ring of persistent-kernel work counters
  mutable std::atomic<uint32_t> counter_next{0};
  rtq::DeviceBuffers bufs;
  // render scratch, grown on demand (guarded by scratch_mu)
  std::mutex scratch_mu;
  rtq::DeviceBuffers scratch;
  size_t scratch_paths = 0;
  void* render_state = nullptr;
  void* stage_log = nullptr;  // HIP events of timed render calls (rtq_render_timing)
};

namespace rtq {
SceneView scene_view(const rtq_scene* s, int fmt);
int resolve_format(const rtq_scene* s, int32_t req, int* fmt);
int resolve_launch(const rtq_scene* s, int32_t sched, int32_t depth, int32_t block, int32_t waves, int32_t refill,
                   TraceLaunch* tl);
void release_render_scratch(rtq_scene* s);
}  // namespace rtq
