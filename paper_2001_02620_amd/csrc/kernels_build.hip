// Build-time kernels: FP64 inversion of instance transforms and padded world
// boxes.  These are the only FP64 computations on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"
#include "rtq_layout.h"

namespace rtq {

// Inverse of the affine map w = A v + t, in FP64 by cofactors.  Writes the FP32
// rounding of A^-1 and t into the instance record, and cond = ||A||_F ||A^-1||_F
// (an upper bound of the 2-norm condition number).  status: 0 ok, 1 singular or
// non-finite.
__global__ void k_invert_affine_fp64(const float* __restrict__ X, const int32_t* __restrict__ proto,
                                     const uint32_t* __restrict__ proto_root, const uint32_t* __restrict__ face_base,
                                     const uint32_t* __restrict__ proto_flags, int64_t n, InstRec* __restrict__ out, float* __restrict__ cond,
                                     int32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* x = X + 12 * i;
  const double a = x[0], b = x[1], c = x[2], d = x[4], e = x[5], f = x[6], g = x[8], h = x[9], k = x[10];
  const double C00 = e * k - f * h, C01 = -(d * k - f * g), C02 = d * h - e * g;
  const double det = a * C00 + b * C01 + c * C02;
  double m = 0.0, fa = 0.0;
  const double A9[9] = {a, b, c, d, e, f, g, h, k};
  for (int j = 0; j < 9; ++j) {
    m = fmax(m, fabs(A9[j]));
    fa += A9[j] * A9[j];
  }
  bool ok = isfinite(det) && fabs(det) > 1e-12 * m * m * m && isfinite(x[3]) && isfinite(x[7]) && isfinite(x[11]);
  const double r = 1.0 / det;
  const double M[9] = {C00 * r, -(b * k - c * h) * r, (b * f - c * e) * r,
                       C01 * r, (a * k - c * g) * r,  -(a * f - c * d) * r,
                       C02 * r, -(a * h - b * g) * r, (a * e - b * d) * r};
  double fi = 0.0;
  for (int j = 0; j < 9; ++j) {
    fi += M[j] * M[j];
    ok = ok && isfinite(M[j]);
  }
  InstRec rec;
  for (int j = 0; j < 3; ++j) {
    rec.r0[j] = (float)M[j];
    rec.r1[j] = (float)M[3 + j];
    rec.r2[j] = (float)M[6 + j];
  }
  rec.r0[3] = x[3];
  rec.r1[3] = x[7];
  rec.r2[3] = x[11];
  const int32_t p = proto[i];
  rec.blas_root = proto_root[p];
  rec.inst_id = (uint32_t)i;
  rec.face_base = face_base[p];
  rec.proto = (uint32_t)p | proto_flags[p];
  out[i] = rec;
  cond[i] = ok ? (float)(sqrt(fa) * sqrt(fi)) : 0.0f;
  status[i] = ok ? 0 : 1;
}

// World box of each instance: the exact bounds of its prototype's vertices mapped
// through the FP64 transform (one block per instance at a time; every quad lies
// in the convex hull of its vertices), padded by 2^-17 cond (|t| + |box|) for the
// FP32 ray-transform error and rounded outward to FP32.  For rotated instances
// this is much tighter than the box of the eight transformed corners of the
// prototype's object box.  Blocks stride over the instances: a dispatch counts
// its work-items in 32 bits, so one block per instance would stop at 2^24
// instances of 256 lanes.
__device__ __forceinline__ void instance_aabb_one(const float* __restrict__ X, const int32_t* __restrict__ proto,
                                                  const float* __restrict__ verts,
                                                  const int64_t* __restrict__ vert_off,
                                                  const float* __restrict__ cond, int64_t i,
                                                  float* __restrict__ box, double (*red)[6]) {
  const float* x = X + 12 * i;
  double m[12];
  for (int j = 0; j < 12; ++j) m[j] = (double)x[j];
  const int32_t p = proto[i];
  const int64_t v0 = vert_off[p], v1 = vert_off[p + 1];
  double lo[3] = {1e308, 1e308, 1e308}, hi[3] = {-1e308, -1e308, -1e308};
  for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    const double a = verts[3 * v], b = verts[3 * v + 1], c = verts[3 * v + 2];
    for (int r = 0; r < 3; ++r) {
      const double w = m[4 * r] * a + m[4 * r + 1] * b + m[4 * r + 2] * c + m[4 * r + 3];
      lo[r] = fmin(lo[r], w);
      hi[r] = fmax(hi[r], w);
    }
  }
  // block reduction: wave shuffles, then one value per wave in LDS
  for (int o = 32; o > 0; o >>= 1)
    for (int r = 0; r < 3; ++r) {
      lo[r] = fmin(lo[r], __shfl_xor(lo[r], o));
      hi[r] = fmax(hi[r], __shfl_xor(hi[r], o));
    }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int r = 0; r < 3; ++r) {
      red[wave][r] = lo[r];
      red[wave][3 + r] = hi[r];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      for (int r = 0; r < 3; ++r) {
        lo[r] = fmin(lo[r], red[w][r]);
        hi[r] = fmax(hi[r], red[w][3 + r]);
      }
    double mag = fmax(fmax(fabs(m[3]), fabs(m[7])), fabs(m[11]));
    for (int r = 0; r < 3; ++r) mag = fmax(mag, fmax(fabs(lo[r]), fabs(hi[r])));
    const double pad = ldexp(1.0, -17) * (double)cond[i] * mag;
    for (int r = 0; r < 3; ++r) {
      box[6 * i + r] = __double2float_rd(lo[r] - pad);
      box[6 * i + 3 + r] = __double2float_ru(hi[r] + pad);
    }
  }
  __syncthreads();  // red is reused by the block's next instance
}

__global__ void __launch_bounds__(256) k_instance_aabb(const float* __restrict__ X, const int32_t* __restrict__ proto,
                                                       const float* __restrict__ verts,
                                                       const int64_t* __restrict__ vert_off,
                                                       const float* __restrict__ cond, int64_t n,
                                                       float* __restrict__ box) {
  __shared__ double red[4][6];
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) instance_aabb_one(X, proto, verts, vert_off, cond, i, box, red);
}

__global__ void k_gather_inst(const InstRec* __restrict__ in, const uint32_t* __restrict__ order,
                              const uint32_t* __restrict__ root, int64_t n, InstRec* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  InstRec r = in[order[i]];
  r.blas_root = root[i];
  out[i] = r;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

static inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_invert_affine(const float* X, const int32_t* proto, const uint32_t* proto_root,
                                const uint32_t* face_base, const uint32_t* proto_flags, int64_t n, InstRec* out,
                                float* cond, int32_t* status, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_invert_affine_fp64, dim3(grid_for(n, 256)), dim3(256), 0, s, X, proto, proto_root, face_base,
                     proto_flags, n, out, cond, status);
  return hipGetLastError();
}

hipError_t launch_instance_aabb(const float* X, const int32_t* proto, const float* verts, const int64_t* vert_off,
                                const float* cond, int64_t n, float* box, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(n, 65536);
  hipLaunchKernelGGL(k_instance_aabb, dim3(grid), dim3(256), 0, s, X, proto, verts, vert_off, cond, n, box);
  return hipGetLastError();
}

hipError_t launch_gather_inst(const InstRec* in, const uint32_t* order, const uint32_t* root, int64_t n, InstRec* out,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_inst, dim3(grid_for(n, 256)), dim3(256), 0, s, in, order, root, n, out);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace rtq
