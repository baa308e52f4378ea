/*
 * rtq — closest-hit tracing of instanced quad meshes and Lambertian path tracing
 * on AMD Instinct MI355X (gfx950).
 *
 * The problem this library solves is the one posed by the Moana Island Scene in
 * "Digesting the Elephant" (Wald et al., TOG 2020): millions of affinely
 * transformed instances of prototype quad meshes (object-level instancing and
 * quads rendered directly, Section 5.2), traced by a path tracer whose time goes
 * mostly into traversal and intersection (Section 6, Table 1), and whose texture
 * lookup needs the hit's primitive ID and barycentrics (Section 5.3).
 *
 * Conventions shared by every call
 *  - All functions return 0 (RTQ_OK) or a negative RTQ_E_* code.  No C++
 *    exception crosses this boundary.  rtq_last_error() returns a message for
 *    the last failure on the calling thread.
 *  - "device" pointers are HIP device memory on the scene's device; "host"
 *    pointers are ordinary process memory.  Inputs are read only during the call
 *    (build) or by the work enqueued on the stream (trace, render); the caller
 *    keeps them alive until that work completes.
 *  - Enqueuing calls (trace, render, backward, set_albedo) are asynchronous on
 *    the given stream and never synchronize the device; set_textures and
 *    set_environment wait for the device first (they may free memory that
 *    queued work reads).  Argument errors are reported synchronously, before
 *    anything is enqueued.
 *  - A quad is (v0, v1, v2, v3), counter-clockwise.  It is traced as the two
 *    triangles A = (v0, v1, v3) and B = (v2, v3, v1), both sides visible.  The hit
 *    parameterisation is v0 -> (u, v) = (0, 0), v1 -> (1, 0), v2 -> (1, 1),
 *    v3 -> (0, 1).
 *  - A curve (Section 5.2: the scene's curves, rendered as chains of
 *    primitives) is a cubic Bezier of four control points (x, y, z, radius).  It
 *    is traced as 8 capsules: capsule j joins the curve's points at parameters
 *    j/8 and (j+1)/8 (each the FP32 rounding of the exact Bezier point) with the
 *    FP32 rounding of the mean of the two points' radii.  A capsule is a
 *    cylinder with a hemisphere on each end, hit from outside only (a ray that
 *    starts inside a capsule does not hit it).  Capsule j of curve c of a
 *    prototype is its primitive 8 c + j; the hit's u is the curve parameter
 *    (j + y) / 8, y in [0, 1] the position along the capsule's axis, and v = 0.
 *    A prototype may instead hold flat (ray-facing) ribbons: the same 8
 *    segments with radius varying linearly from one point's radius to the
 *    next, each seen along the ray as the strip of points within that radius
 *    of its projection; a ray meets it when its line passes within the radius
 *    of the projected segment's closest point, at the depth of that segment
 *    point (u then holds that point's curve parameter).  A ray that excludes
 *    a ribbon segment (rtq_rays.exclude) ignores every segment of that curve
 *    in that instance: a ribbon turns toward every ray, so the neighbours of
 *    the segment a ray leaves would face it next to its origin.
 *  - An instance transform is a row-major 3x4 FP32 matrix [A | t] mapping object
 *    to world space, w = A v + t.
 *  - A hit is accepted when tmin < t <= tmax; among accepted hits the one with
 *    the smallest key (t, instance id, primitive id, half) wins, so the result
 *    does not depend on traversal order, node format or node width.
 */
#ifndef RTQ_H
#define RTQ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define RTQ_OK 0
#define RTQ_E_INVALID_ARG (-1)    /* bad pointer, size, index, NaN vertex, ... */
#define RTQ_E_SINGULAR_XFORM (-2) /* an instance transform cannot be inverted */
#define RTQ_E_OOM (-3)            /* device or host allocation failed */
#define RTQ_E_HIP (-4)            /* a HIP runtime call failed */
#define RTQ_E_LIMIT (-5)          /* a size exceeds an encoding or dispatch limit */

/* Message describing the last error on this thread (never NULL). */
const char* rtq_last_error(void);
/* Library version string. */
const char* rtq_version(void);

/* ------------------------------------------------------------- host BVH */
/*
 * The scene builder's bottom-level construction on its own, on the host, over
 * arbitrary boxes (Section 5.2: one BVH per object; here binned SAH, collapsed
 * to `width`-wide nodes, emitted as exact FP32 boxes and as 8-bit quantized
 * nodes).  For inspecting the acceleration structure and for host-side checks;
 * no device is touched.
 *   boxes: host, n x 6 FP32 (lo x y z, hi x y z); n >= 1.
 *   leaf_max: primitives per leaf, 1..8.  bins: SAH bins per axis, 4..64.
 *   threads: host threads, 0 = all; the result does not depend on it.
 *   width: children per node, 2, 4 or 8.
 * Node layouts (little-endian, node 0 is the root):
 *   wide, 224 B (every width; slots >= width empty):
 *                float lo[3][8], hi[3][8] (axis-major); uint32 child[8].
 *   FP32, 128 B (width 4 only, else NULL): float lo_x[4], hi_x[4], lo_y[4],
 *                hi_y[4], lo_z[4], hi_z[4]; uint32 child[4]; uint32 pad[4].
 *   Q8, 64 B (width 4): float origin[3]; uint32 exps (byte a: int8 exponent of
 *                axis a); uint32 lo_x, hi_x, lo_y, hi_y, lo_z, hi_z (byte c:
 *                child c); uint32 child[4]; uint32 pad[2].
 *   Q8, 96 B (width 8): origin and exps as above; uint32 lo_x[2], hi_x[2],
 *                lo_y[2], hi_y[2], lo_z[2], hi_z[2] (byte c of word j: child
 *                4 j + c); uint32 child[8].
 *   Q8, 48 B (width 2): origin and exps; uint32 x, y, z (bytes 0, 1: lower
 *                planes of children 0, 1; bytes 2, 3: upper planes);
 *                uint32 child[2]; uint32 pad[3].
 *   A quantized plane decodes to fmaf(q, 2^e, origin), which contains the
 *   FP32 plane; an empty slot has lower byte 255 and upper byte 0.
 *   child: 0xFFFFFFFF empty; bit 31 set: leaf of primitives
 *          order[first .. first + count) with first = (c >> 3) & 0x0FFFFFFF and
 *          count = (c & 7) + 1; otherwise the index of an internal node.
 * *out owns the arrays; rtq_host_bvh_get returns pointers into it, valid until
 * rtq_host_bvh_destroy.  Errors: INVALID_ARG (NULL, n < 1, non-finite or
 * inverted box, parameter out of range), LIMIT (n >= 2^28), OOM.
 */
typedef struct rtq_host_bvh rtq_host_bvh;
int rtq_host_bvh_build(const float* boxes, int64_t n, int32_t leaf_max, int32_t bins, int32_t threads,
                       int32_t width, rtq_host_bvh** out);
int rtq_host_bvh_get(const rtq_host_bvh* bvh, const void** nodes_wide, const void** nodes_f32,
                     const void** nodes_q8, int64_t* n_nodes, const uint32_t** order, int32_t* depth);
void rtq_host_bvh_destroy(rtq_host_bvh* bvh);

/* ------------------------------------------------------------------ scene */
typedef struct rtq_scene rtq_scene;

/* One prototype (host memory): a quad mesh, or a set of curves.  Its faces
 * (the units that carry an albedo, a material or a gradient) are its quads, or
 * its curves. */
typedef struct {
  const float* verts;   /* n_verts x 3 FP32, object space (quad meshes) */
  const int32_t* quads; /* n_quads x 4 vertex indices into verts (CCW) */
  int32_t n_verts;
  int32_t n_quads;      /* >= 1 for a quad mesh, 0 for curves */
  const float* albedo;  /* one per face (n_quads, or n_curves), or NULL for 0.5 */
  const float* curves;  /* n_curves x 16 FP32: 4 control points (x, y, z, radius), radius >= 0;
                           NULL for a quad mesh */
  int32_t n_curves;     /* >= 1 for curves (then n_quads = 0 and verts, quads may be NULL), else 0 */
  int32_t curves_flat;  /* nonzero: the curves are flat ray-facing ribbons; 0: round */
} rtq_prototype;

/* Object-level instances (host memory): instance i draws prototype proto[i]
 * through the transform xform[12 i .. 12 i + 11]. */
typedef struct {
  int64_t n;
  const int32_t* proto; /* n prototype indices */
  const float* xform;   /* n x 12, row-major [A | t], world <- object */
} rtq_instances;

/* Node formats (bit mask for building, single value for tracing). */
#define RTQ_NODE_FP32 1 /* 4-wide nodes with FP32 child boxes, 128 B (4-wide scenes only) */
#define RTQ_NODE_Q8 2   /* nodes with 8-bit child boxes in an FP32 parent frame: 48 B (2-wide),
                           64 B (4-wide), 96 B (8-wide) */

typedef struct {
  int32_t formats;       /* RTQ_NODE_* mask to build; 0 = both */
  int32_t leaf_max;      /* quads per bottom-level leaf, 1..8; 0 = 4 */
  int32_t sah_bins;      /* binned-SAH bins of the bottom levels, 4..64; 0 = 32 (the top level uses 64) */
  int32_t build_threads; /* host threads for the bottom-level builds; 0 = all */
  int32_t device;        /* HIP device ordinal; -1 = current */
  int32_t open_pct;      /* top-level entries added by opening instances into subtrees of their
                            bottom-level BVH (partial re-braiding), in percent of the instance
                            count; 0 = default (50), negative = none.  Hits do not depend on it. */
  int32_t node_width;    /* children per node at both levels: 2, 4 or 8; 0 = 4.  Widths other
                            than 4 build quantized nodes only (formats 0 or RTQ_NODE_Q8).  Hits
                            do not depend on it. */
  int32_t open_area_pct; /* an instance subtree is opened only if its children's world boxes
                            cover at most this percentage of its own box's surface area,
                            100..1000; 0 = 150.  Hits do not depend on it. */
} rtq_build_opts;

/*
 * Build the acceleration structures of a scene (Section 5.2: per-object BVHs
 * under a top-level BVH over instances, quads and curves' capsules as
 * primitives).
 *   protos[0..n_protos), insts: host memory, read during the call only.
 *   opts: may be NULL for defaults.
 *   *out: receives a handle owning all device memory of the scene.
 * Instance inverses and world boxes are computed on the device in FP64; the
 * BVHs are built on the host (binned SAH) and uploaded.  The call
 * synchronizes the device it builds on.
 * Errors: INVALID_ARG (NULL pointer, a prototype with neither or both of quads
 * and curves, vertex index out of range, non-finite vertex, control point or
 * transform, negative radius, proto index out of range), SINGULAR_XFORM, LIMIT
 * (more than 2^28 unique primitives or instances, 2^31 nodes, or BVHs deeper
 * than the traversal stack allows), OOM, HIP.
 */
int rtq_scene_build(const rtq_prototype* protos, int32_t n_protos, const rtq_instances* insts,
                    const rtq_build_opts* opts, rtq_scene** out);

/* Free every device allocation of the scene.  NULL-safe.  Synchronizes. */
void rtq_scene_destroy(rtq_scene* scene);

typedef struct {
  int64_t n_instances, n_prototypes, n_unique_quads, n_instanced_quads;
  int64_t tlas_nodes, blas_nodes;
  int32_t tlas_depth, blas_depth_max; /* node levels */
  int32_t formats;                    /* RTQ_NODE_* built */
  int64_t device_bytes;               /* all device memory held by the scene (textures included) */
  double build_seconds;               /* wall time of rtq_scene_build */
  int64_t n_top_entries;              /* top-level leaves: instances plus the subtrees opened ones add */
  double build_phase_seconds[4];      /* bottom levels (host); instance inverses and boxes (device) and
                                         bottom-level upload; opening instances (host); top level
                                         (host) and its upload */
  int32_t node_width;                 /* children per node */
  int64_t n_unique_curves, n_unique_capsules;
  int64_t n_faces;                    /* unique faces: quads and curves */
} rtq_scene_info;

int rtq_scene_get_info(const rtq_scene* scene, rtq_scene_info* info);

/*
 * Replace the per-face albedo (device memory, n = total unique faces -- quads
 * and curves --, in prototype order) without rebuilding.  Enqueued on `stream` (a device copy).
 * Not part of the paper's system (its colours come from Ptex textures, Section
 * 5.3): this library's addition for gradient-driven loops over the albedo
 * (rtq_render_backward).
 */
int rtq_scene_set_albedo(rtq_scene* scene, const float* albedo_dev, int64_t n, hipStream_t stream);

/*
 * Per-face textures (Section 5.3: the diffuse colour of nearly every face comes
 * from a Ptex texture, looked up by face id and the hit's coordinates on the
 * face).  Here each unique quad carries res x res texels, read at the nearest
 * texel of the hit's (u, v) (v0 -> (0, 0), v1 -> (1, 0), v2 -> (1, 1),
 * v3 -> (0, 1)), in every scheduler and node format.  A texel of one channel
 * replaces the face's albedo in shading; a texel of three (an RGB colour, for
 * scenes with materials) gives channel k of the base colour as the material's
 * tint_k times texel channel k.  No filtering, no mip levels, no borders shared
 * with adjacent faces.
 *
 * texels_dev: device memory, n_unique_quads * res * res * channels floats,
 * face-major in prototype order, then row v, then column u, channel fastest:
 * channel k of texel (tx, ty) of face f at [((f * res + ty) * res + tx) *
 * channels + k]; it is copied into memory the scene owns (freed by
 * rtq_scene_destroy), the caller keeps its buffer.  channels: 1 or 3.  res = 0
 * (texels_dev may be NULL) removes the textures.  Waits for all work on the
 * device, then enqueues the copy on `stream`; renders on other streams are
 * ordered by the caller.
 * Errors: RTQ_E_INVALID_ARG for res outside [0, RTQ_MAX_TEX_RES], channels
 * other than 1 or 3, NULL texels with res > 0, or res > 0 in a scene with
 * curves (they have no (u, v) square); RTQ_E_HIP when the allocation or copy
 * fails.  A render of a scene with RGB texels and no materials fails with
 * RTQ_E_INVALID_ARG.
 * rtq_render_backward then differentiates with respect to the texels (every
 * channel of an RGB texel separately, at index texel * 3 + channel).
 */
#define RTQ_MAX_TEX_RES 64
int rtq_scene_set_textures(rtq_scene* scene, const float* texels_dev, int32_t res, int32_t channels,
                           hipStream_t stream);

/*
 * Environment map (Section 4.1: the scene has a textured environment light):
 * the radiance a path sees when its ray leaves the scene, in place of the
 * constant sky L_sky, and, with rtq_render_opts.env_nee, a light sampled by
 * next-event estimation.  An equirectangular map of w x h values: direction d
 * (normalised) has u = (atan2(d_y, d_x) + pi) / (2 pi) along a row and
 * v = acos(d_z) / pi down the rows (row 0 around +z), read at the nearest
 * texel.  The call also builds the map's sampling table (texel k drawn with
 * probability (T_k - T_{k-1}) / 2^32, T_k = floor(2^32 C_k / C_total), C the
 * running sum in texel order of radiance x solid angle).
 *
 * texels_dev: device memory, h rows of w floats, copied into memory the scene
 * owns (freed by rtq_scene_destroy); w = 0 (texels_dev may be NULL) removes the
 * map.  Waits for all work on the device, then copies the map synchronously.
 * Errors: RTQ_E_INVALID_ARG for w or h outside [1, RTQ_MAX_ENV_SIDE] (w = 0
 * aside), NULL texels, or a negative or non-finite texel; RTQ_E_HIP when the
 * allocation or copy fails.
 */
#define RTQ_MAX_ENV_SIDE 16384
int rtq_scene_set_environment(rtq_scene* scene, const float* texels_dev, int32_t w, int32_t h, hipStream_t stream);

/*
 * Principled materials (Section 5.4: every material of the scene uses Disney's
 * principled BSDF, which the paper made energy conserving and preserving; it
 * gives no formulas, so this is a reading).  A face's base color is its
 * material's tint times its albedo (or texel), per channel, and it shades with
 *   f mu_i = (1 - m)[F_d p_s + (1 - F_d) c mu_i / pi] + m F_c p_s,
 * F_d = specular (0.04 + 0.96 (1 - mu_o)^5) and F_c = c + (1 - c)(1 - mu_o)^5
 * (Schlick at the macro-surface angle), p_s the density of the outgoing
 * direction reflected about a GGX visible normal (alpha = roughness^2, separable
 * Smith masking, Heitz 2018), a reflection below the surface mirrored above it.
 * The albedo is (1 - m)[F_d + (1 - F_d) c] + m F_c: one for c = 1, at most one
 * otherwise; metallic = specular = 0 is Lambert's c / pi.  A clearcoat of weight
 * k (the principled model's coat layer) lies over that base: a second such lobe
 * p_k of its own roughness with the Fresnel weight F_k = k (0.04 + 0.96
 * (1 - mu_o)^5), the base keeping the rest,
 *   f mu_i = F_k p_k + (1 - F_k) [base f mu_i],
 * albedo F_k + (1 - F_k) [base albedo]; clearcoat = 0 is the base alone.  Bounces
 * draw, from word 0 u of Philox counter (pixel, sample, view, 2^30 + bounce),
 * the coat when u < F_k, the base's specular lobe when u < F_k + (1 - F_k) P_s
 * with P_s = (1 - m) F_d + m, the cosine lobe otherwise, and weigh the
 * direction by f mu_i over the mixture's density.  With materials every
 * path carries three channels: images and image gradients hold 3 floats per
 * pixel (interleaved RGB) and rtq_render_opts.channels must be 3.  Lights stay
 * white.
 *
 * mats: host memory, n_mat entries (copied); face_mat_dev: device memory, one
 * material index per unique face (quad or curve) in prototype order (copied
 * into memory the scene owns).  n_mat = 0 (both may be NULL) removes the materials.  Waits for
 * all work on the device, then copies synchronously.
 * Errors: RTQ_E_INVALID_ARG for n_mat outside [0, RTQ_MAX_MATERIALS], NULL
 * arrays, a tint outside [0, 1], roughness outside [0.05, 1], metallic,
 * specular or clearcoat outside [0, 1], a clearcoat roughness outside
 * [0.05, 1] where clearcoat > 0 (it is ignored where clearcoat = 0), or a face
 * index >= n_mat; RTQ_E_HIP when the allocation or copy fails.
 */
typedef struct {
  float tint[3];
  float roughness, metallic, specular;
  float clearcoat, clearcoat_roughness;
} rtq_material;
#define RTQ_MAX_MATERIALS 256
int rtq_scene_set_materials(rtq_scene* scene, const rtq_material* mats, int32_t n_mat, const uint8_t* face_mat_dev,
                            hipStream_t stream);

/* ------------------------------------------------------------------ tracing */
/* Rays and hits are structure-of-arrays in device memory, one element per ray. */
typedef struct {
  const float *ox, *oy, *oz; /* origin */
  const float *dx, *dy, *dz; /* direction, need not be normalised; t is in its units */
  const float *tmin, *tmax;  /* accepted interval tmin < t <= tmax */
  const uint32_t* exclude;   /* optional (NULL: none), 2 words per ray: the hit reference
                                (rtq_hits.ref) of a triangle the ray must not hit -- the one a
                                secondary or shadow ray leaves; the pair 0xFFFFFFFF 0xFFFFFFFF
                                excludes nothing */
} rtq_rays;

typedef struct {
  float *t, *u, *v;      /* miss: t = +inf, u = v = 0 */
  int32_t *inst, *prim;  /* miss: -1, -1; prim is the quad (or capsule) index within its prototype */
  uint32_t* ref;         /* optional (NULL: not written), 2 words per ray: an opaque reference of the
                            hit triangle (top-level entry; leaf-ordered quad, and the half in bit 31)
                            valid for this scene, for rtq_rays.exclude of rays that leave it; a miss
                            writes 0xFFFFFFFF 0xFFFFFFFF */
} rtq_hits;

#define RTQ_SCHED_PLAIN 0      /* one ray per lane for its whole traversal */
#define RTQ_SCHED_PERSISTENT 1 /* resident waves refill finished lanes from a shared ray counter */
#define RTQ_SCHED_MEGAKERNEL 2 /* rendering only: the whole frame in one persistent launch */

typedef struct {
  int32_t node_format; /* RTQ_NODE_FP32 or RTQ_NODE_Q8; 0 = Q8 if built, else FP32 */
  int32_t scheduler;   /* RTQ_SCHED_* */
  int32_t stack_depth; /* LDS stack entries per lane, 4..64 (deeper entries spill); 0 = 20 */
  int32_t block;       /* threads per block, multiple of 64, 64..1024; 0 = 256 */
  int32_t waves_per_cu;/* persistent scheduler: resident waves per CU; 0 = 24 */
  int32_t refill;      /* persistent scheduler: refill when this many lanes are idle, 1..64; 0 = 16 */
  uint32_t* visits;    /* optional device n x 4 counters: top nodes, instances entered,
                          bottom nodes, quads tested (slower kernel variant) */
  uint32_t* lane_stats;/* optional device n x 2 counters (same kernel variant): traversal
                          iterations of the ray's wave while the ray was not done (its
                          visits over this is the fraction of its live iterations in
                          which its lane did useful work), and FP64 re-evaluations of
                          zero edge values in its leaf tests */
} rtq_trace_opts;

/*
 * Closest hit of n rays (device SoA in, device SoA out), enqueued on `stream`:
 * the ray query of the path tracer's camera and bounce rays (Section 5.2:
 * instances of quad meshes traced directly; Section 5.3: the hit carries the
 * primitive id and the coordinates on the quad that a texture lookup needs).
 * opts may be NULL.  Zero-length or NaN directions miss.  n may be 0.
 * Errors: LIMIT when n exceeds 2^31 - 1 (a dispatch counts its work-items in
 * 32 bits); INVALID_ARG for NULL arrays or options out of range.
 */
int rtq_trace_closest(const rtq_scene* scene, const rtq_rays* rays, int64_t n, rtq_hits* hits,
                      const rtq_trace_opts* opts, hipStream_t stream);

/*
 * rtq_trace_closest with the persistent scheduler, allocating nothing: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid it).  Same arguments, results and
 * errors as rtq_trace_closest; opts.scheduler is ignored (always persistent).
 * The persistent launch's claim counters (1 KiB) live in a static device array
 * the library holds on each device it runs on until the process ends, instead
 * of the scene's counter ring; the call clears them with a kernel before its
 * launch.  Every call on one device shares that array: calls that overlap in
 * time on one device race and must be ordered by the caller (one stream, or
 * events).  The first call on a device looks the array's address up
 * (hipGetSymbolAddress, no allocation).  Errors as rtq_trace_closest, plus
 * RTQ_E_HIP if the address lookup fails.
 */
int rtq_trace_closest_noalloc(const rtq_scene* scene, const rtq_rays* rays, int64_t n, rtq_hits* hits,
                              const rtq_trace_opts* opts, hipStream_t stream);

/*
 * Occlusion: occluded[i] = 1 if any hit with tmin < t <= tmax exists, else 0 --
 * the shadow-ray query of next-event estimation (Section 5.4 samples the
 * scene's lights at every path vertex).  Arguments and errors as
 * rtq_trace_closest.
 */
int rtq_trace_occluded(const rtq_scene* scene, const rtq_rays* rays, int64_t n, uint8_t* occluded,
                       const rtq_trace_opts* opts, hipStream_t stream);

/*
 * Reference traversal for tests: every instance and every quad (or capsule) of
 * its prototype is tested with the same leaf code as rtq_trace_closest (no
 * acceleration structure).  Meant for tiny scenes only.
 */
int rtq_trace_brute(const rtq_scene* scene, const rtq_rays* rays, int64_t n, rtq_hits* hits, hipStream_t stream);

/* ------------------------------------------------------------------ rendering */
/*
 * One pinhole view, or a rectangle of one (Section 5.5: image-parallel
 * rendering deals the tiles of a frame to the workers).  The random-number
 * counter of a path is (pixel of the whole view, sample, view_id, bounce), so a
 * view rendered whole in one call, or tile by tile in several calls (or on
 * several devices), gives bit-identical pixels as long as view_id, the view's
 * parameters and the render options are the same.
 */
typedef struct {
  float eye[3], look[3], up[3];
  float vfov_deg;
  int32_t w, h;        /* resolution of the whole view */
  int64_t img_offset;  /* first pixel of the rendered rectangle in the packed image buffer */
  int32_t view_id;     /* the view's index in the random-number counter, >= 0.  Cameras of one call
                          need distinct ids unless they are tiles of one view. */
  int32_t tile_x, tile_y, tile_w, tile_h; /* rendered rectangle: columns [tile_x, tile_x + tile_w),
                          rows [tile_y, tile_y + tile_h); tile_w = tile_h = 0 renders the whole view.
                          Its pixels are stored row by row from img_offset (tile_w per row). */
} rtq_camera;

typedef struct {
  uint64_t seed;       /* RNG key (Philox4x32-10 key = (seed_lo, seed_hi ^ frame)) */
  uint32_t frame;      /* progressive frame index (Section 5.4: 1 spp per frame) */
  float light_dir[3];  /* unit direction toward the directional light */
  float E;             /* light irradiance */
  float L_sky;         /* constant sky radiance */
  int32_t node_format; /* as rtq_trace_opts */
  int32_t scheduler;   /* RTQ_SCHED_PLAIN: wavefront of one kernel per stage and bounce
                          (queues of extension and shadow rays), one ray per lane;
                          RTQ_SCHED_PERSISTENT: the same wavefront with persistent,
                          lane-refilling traversal stages, each tracing one
                          bounce's shadow rays with the next bounce's extension rays;
                          RTQ_SCHED_MEGAKERNEL: one persistent launch per frame whose
                          lanes run whole paths and are refilled with new paths */
  int32_t stack_depth, block, waves_per_cu, refill; /* as rtq_trace_opts */
  uint64_t* counters;  /* optional device [4]: closest rays, shadow rays, incoherent
                          (bounce >= 1) rays, paths; accumulated (caller zeroes) */
  uint64_t* view_done; /* optional device [n_cams], zeroed by the caller: the
                          wall-clock tick (the device's constant-rate clock,
                          s_memrealtime) at which each camera entry's last path
                          finished, in every scheduler (per-view latency of a
                          batch of views, Section 6 reports per-view frame times) */
  uint64_t* start_tick;/* optional device [1]: wall-clock tick at the start of the
                          call's first kernel */
  uint64_t* visits;    /* optional device [8]: top-level nodes, instances entered,
                          bottom-level nodes and quads tested, summed over the
                          closest-hit rays ([0..3]) and over the shadow rays
                          ([4..7]) (accumulated; selects a slower counting variant) */
  float* dump_rays;    /* optional device 12 x dump_cap 32-bit words, structure of
                          arrays: ox, oy, oz, dx, dy, dz, tmin, tmax (FP32), then the
                          two words of the hit reference of the triangle the ray
                          leaves (uint32, as rtq_hits.ref, for rtq_rays.exclude),
                          then that triangle's instance id and primitive | half << 31:
                          extension rays of bounce >= 1 (plain and persistent
                          schedulers) */
  int64_t dump_cap;    /* capacity of dump_rays in rays */
  uint64_t* dump_count;/* device [1]: rays appended to dump_rays (accumulated; the
                          count may exceed dump_cap, rays beyond it are dropped) */
  int32_t timing;      /* nonzero: record HIP events around the call's kernel
                          launches on `stream` (no synchronisation); read them
                          with rtq_render_timing (with graph set: the whole
                          graph launch, reported under calls only) */
  int32_t graph;       /* nonzero: capture the call's launches into a HIP graph
                          on first use and replay it on later calls with the same
                          configuration (cameras, sizes, buffers, options; the
                          seed and frame may change).  Graphs are kept in the
                          scene and dropped when its render scratch grows.
                          Replays of one scene must not overlap in time. */
  int32_t accumulate;  /* progressive refinement (Section 5.4: one sample per pixel
                          per frame, frames accumulated over time): the number k
                          of frames already averaged in `images`.  0 writes this
                          call's mean m; k > 0 blends it in as
                          images += (m - images) / (k + 1), so frames rendered with
                          accumulate = 0, 1, ..., K - 1 (and different `frame`
                          values) leave the running mean of their K images.  It
                          changes nothing but that blend (graphs replay with any
                          k).  Ignored by rtq_render_backward and rtq_render_path. */
  int32_t n_area_lights;     /* quad area lights (Section 4.1: besides an environment
                                light the scene has 23 quad-shaped key lights),
                                0..RTQ_MAX_AREA_LIGHTS */
  const float* area_lights;  /* host, 10 floats per light: corner xyz, edge-1 xyz, edge-2
                                xyz, emitted radiance Le; the light is the parallelogram
                                corner + s e1 + t e2, s, t in [0, 1), emitting from the
                                side e1 x e2 faces, and is not seen by camera or bounce
                                rays.  With n > 0 lights, each hit's next-event estimate
                                picks one of the n + 1 lights (the directional one
                                included) with equal probability, weighted by n + 1; an
                                area light is sampled uniformly over its area and its
                                shadow ray ends at the sampled point.  Copied to the
                                device during the call. */
  int32_t env_nee;           /* nonzero, with an environment map set: the map becomes one
                                more light of the next-event choice (Section 4.1: the
                                scene's textured environment light).  A texel is drawn
                                with probability proportional to radiance x solid angle
                                (a 32-bit table built by rtq_scene_set_environment), a
                                direction uniformly in solid angle within it; that
                                estimate and the radiance an escaping bounce ray reads
                                are weighted against each other by the power heuristic.
                                Unbiased either way; lower variance for small bright
                                regions of the map. */
  int32_t channels;          /* floats per image pixel: 0 or 1 without materials, 3 with
                                them (rtq_scene_set_materials); any other value is an
                                error, so buffers are sized for the scene's layout */
} rtq_render_opts;

#define RTQ_MAX_AREA_LIGHTS 64

/*
 * Path-trace n_cams pinhole views (Section 5.4: progressive 1 spp frames; here
 * spp samples per call, frames averaged with opts.accumulate) with a
 * Lambertian BSDF (albedo per face, or a texel of the face's texture when the
 * scene has textures; a curve's normal is the capsule's) or, with materials, the principled BSDF in three
 * channels (rtq_scene_set_materials), next-event estimation toward one directional light
 * (and optional quad area lights, opts.area_lights), and a constant sky (or an
 * environment map, rtq_scene_set_environment).  depth counts closest-hit rays per path including the
 * camera ray.  `images` is a packed FP32 device buffer; view
 * c occupies pixels [img_offset, img_offset + w h), row 0 at the top, one float
 * per pixel (three, interleaved RGB, with materials).  Each pixel is
 * the mean over its spp samples, summed in sample order, so every scheduler
 * produces bit-identical images.  cams: host memory.  Scratch memory is
 * allocated on first use and kept in the scene handle.
 * Errors: INVALID_ARG (spp < 1, depth < 1 or > 16, w or h < 1, NULL images,
 * accumulate < 0, area-light count outside [0, RTQ_MAX_AREA_LIGHTS], NULL or
 * non-finite area lights); LIMIT when the call has more than 2^31 - 1 paths
 * (sum of w h spp).
 */
int rtq_render(const rtq_scene* scene, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
               const rtq_render_opts* opts, float* images, hipStream_t stream);

/*
 * Kernel time of the render calls made with opts->timing set since the previous
 * query, by stage: ms[0] traversal launches (RTQ_SCHED_PLAIN: closest hits of
 * each bounce; RTQ_SCHED_PERSISTENT: the depth + 1 launches that each trace one
 * bounce's shadow rays together with the next bounce's extension rays;
 * RTQ_SCHED_MEGAKERNEL: the megakernel), ms[1] shadow-ray traversal launches of
 * RTQ_SCHED_PLAIN, ms[2] every other launch (ray generation, shading, shadow
 * resolve, accumulation), ms[3] whole calls (first to last recorded event).  launches[k] counts the launches
 * in ms[k] (launches[3] = calls).  Waits for the recorded events, then forgets
 * them.  ms, launches: host arrays of 4, either may be NULL.  The event log
 * holds at most 4096 events; calls beyond it are not timed (launches tells).
 */
int rtq_render_timing(rtq_scene* scene, float* ms, int32_t* launches);

/*
 * One path of rtq_render traced alone (same RNG counters, hits and shading as
 * the render kernels; node format and stack depth from opts), for path-level
 * checks: path (view, pixel, sample) with view the camera entry and pixel the
 * index within its rendered rectangle (row * width + column).  Per vertex
 * k < *n_vert: vert_i[6k..6k+5] = (instance id, primitive, half, shadow: -1 no
 * shadow ray / 0 light visible / 1 occluded, unique face, 0) and
 * vert_f[10k..10k+9] = (t, albedo or texel, cosine to the light, radiance after the
 * vertex, origin xyz and direction xyz of the ray that found the vertex);
 * *escaped = 1 if the path left the scene, and then record *n_vert holds the
 * escaping ray (ids -1, t = +inf, its origin and direction); *radiance = the
 * path's total (radiance[0..2], the three channels, with materials; then the
 * radiance after each vertex is the red channel).
 * vert_i: host, 6 depth int32; vert_f: host, 10 depth floats; radiance: host,
 * 1 float (3 with materials).  Synchronises
 * `stream`.  Errors: INVALID_ARG (view, pixel or sample out of range, NULL
 * outputs), as rtq_render otherwise.
 */
int rtq_render_path(const rtq_scene* scene, const rtq_camera* cams, int32_t n_cams, int32_t spp, int32_t depth,
                    const rtq_render_opts* opts, int32_t view, int64_t pixel, int32_t sample, int32_t* vert_i,
                    float* vert_f, int32_t* n_vert, int32_t* escaped, float* radiance, hipStream_t stream);

/*
 * Not part of the paper's system: this library's addition, a path-replay
 * adjoint (after Vicini, Speierer and Jakob 2021) of the renderer above.
 * Adjoint of rtq_render with respect to per-face albedo, paths held fixed:
 * grad_albedo[f] += sum over pixels p of grad_images[p] * dI_p / d albedo[f].
 * Each path is replayed from its RNG counters (same hits as the forward pass).
 * With textures the gradient is per texel (the parameter a hit reads):
 * grad_albedo then holds n_unique_quads * res * res floats in the texture's
 * layout (rtq_scene_set_textures).  With materials, grad_images holds 3 floats per pixel (as the image) and each
 * vertex's estimate and bounce weight, affine in its albedo, are differentiated
 * per channel.
 * grad_albedo: device, n_faces floats (n_unique_quads times res^2 with textures), zeroed by the caller, accumulated
 * with atomics (summation order is not fixed).  Errors: as rtq_render.
 */
int rtq_render_backward(const rtq_scene* scene, const rtq_camera* cams, int32_t n_cams, int32_t spp,
                        int32_t depth, const rtq_render_opts* opts, const float* grad_images, float* grad_albedo,
                        hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RTQ_H */
