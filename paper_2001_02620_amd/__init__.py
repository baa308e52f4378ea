"""Python binding of librtq (the HIP library behind ``include/rtq.h``).

This module only marshals arguments: torch tensors provide device memory and
the current HIP stream; every step of tracing, shading and differentiation runs
in the library's kernels.  There is no CPU fallback: importing the binding
without the built library, or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtq.so")

RTQ_NODE_FP32 = 1
RTQ_NODE_Q8 = 2
SCHED_PLAIN = 0
SCHED_PERSISTENT = 1
SCHED_MEGAKERNEL = 2

ERRORS = {-1: "INVALID_ARG", -2: "SINGULAR_XFORM", -3: "OOM", -4: "HIP", -5: "LIMIT"}


class RtqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rtq error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


# ----------------------------------------------------------------------------- C structs
class _Proto(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("quads", ctypes.c_void_p), ("n_verts", ctypes.c_int32),
                ("n_quads", ctypes.c_int32), ("albedo", ctypes.c_void_p), ("curves", ctypes.c_void_p),
                ("n_curves", ctypes.c_int32), ("curves_flat", ctypes.c_int32)]


class _Insts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("proto", ctypes.c_void_p), ("xform", ctypes.c_void_p)]


class _BuildOpts(ctypes.Structure):
    _fields_ = [("formats", ctypes.c_int32), ("leaf_max", ctypes.c_int32), ("sah_bins", ctypes.c_int32),
                ("build_threads", ctypes.c_int32), ("device", ctypes.c_int32), ("open_pct", ctypes.c_int32),
                ("node_width", ctypes.c_int32), ("open_area_pct", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int64), ("n_prototypes", ctypes.c_int64),
                ("n_unique_quads", ctypes.c_int64), ("n_instanced_quads", ctypes.c_int64),
                ("tlas_nodes", ctypes.c_int64), ("blas_nodes", ctypes.c_int64), ("tlas_depth", ctypes.c_int32),
                ("blas_depth_max", ctypes.c_int32), ("formats", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("n_top_entries", ctypes.c_int64),
                ("build_phase_seconds", ctypes.c_double * 4), ("node_width", ctypes.c_int32),
                ("n_unique_curves", ctypes.c_int64), ("n_unique_capsules", ctypes.c_int64), ("n_faces", ctypes.c_int64)]


class _Rays(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("ox", "oy", "oz", "dx", "dy", "dz", "tmin", "tmax", "exclude")]


class _Hits(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("t", "u", "v", "inst", "prim", "ref")]


class _TraceOpts(ctypes.Structure):
    _fields_ = [("node_format", ctypes.c_int32), ("scheduler", ctypes.c_int32), ("stack_depth", ctypes.c_int32),
                ("block", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("refill", ctypes.c_int32),
                ("visits", ctypes.c_void_p), ("lane_stats", ctypes.c_void_p)]


class _Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("look", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("vfov_deg", ctypes.c_float), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("img_offset", ctypes.c_int64), ("view_id", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


class _RenderOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("frame", ctypes.c_uint32), ("light_dir", ctypes.c_float * 3),
                ("E", ctypes.c_float), ("L_sky", ctypes.c_float), ("node_format", ctypes.c_int32),
                ("scheduler", ctypes.c_int32), ("stack_depth", ctypes.c_int32), ("block", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("refill", ctypes.c_int32), ("counters", ctypes.c_void_p),
                ("view_done", ctypes.c_void_p), ("start_tick", ctypes.c_void_p), ("visits", ctypes.c_void_p),
                ("dump_rays", ctypes.c_void_p), ("dump_cap", ctypes.c_int64), ("dump_count", ctypes.c_void_p),
                ("timing", ctypes.c_int32), ("graph", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("n_area_lights", ctypes.c_int32), ("area_lights", ctypes.c_void_p), ("env_nee", ctypes.c_int32),
                ("channels", ctypes.c_int32)]


class _Material(ctypes.Structure):
    _fields_ = [("tint", ctypes.c_float * 3), ("roughness", ctypes.c_float), ("metallic", ctypes.c_float),
                ("specular", ctypes.c_float), ("clearcoat", ctypes.c_float), ("clearcoat_roughness", ctypes.c_float)]


# ----------------------------------------------------------------------------- loading
_lib = None

EXPORTS = ["rtq_last_error", "rtq_version", "rtq_scene_build", "rtq_scene_destroy", "rtq_scene_get_info",
           "rtq_scene_set_albedo", "rtq_trace_closest", "rtq_trace_occluded", "rtq_trace_brute", "rtq_render",
           "rtq_render_backward", "rtq_render_timing", "rtq_render_path", "rtq_host_bvh_build", "rtq_host_bvh_get",
           "rtq_host_bvh_destroy", "rtq_scene_set_textures", "rtq_scene_set_environment",
           "rtq_trace_closest_noalloc", "rtq_scene_set_materials"]


def load_library():
    """Load librtq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"librtq.so is not built ({LIB_PATH}); run paper_2001_02620_amd/build.py")
    # torch carries its own HIP runtime (same SONAME as ROCm's).  Loading torch
    # first makes librtq bind to that runtime, so both share one device context,
    # one allocator view and the same streams.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.rtq_last_error.restype = ctypes.c_char_p
    L.rtq_version.restype = ctypes.c_char_p
    L.rtq_scene_build.argtypes = [P, ctypes.c_int32, P, P, P]
    L.rtq_scene_destroy.argtypes = [P]
    L.rtq_scene_get_info.argtypes = [P, P]
    L.rtq_scene_set_albedo.argtypes = [P, P, ctypes.c_int64, P]
    L.rtq_scene_set_textures.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P]
    L.rtq_scene_set_environment.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P]
    L.rtq_scene_set_materials.argtypes = [P, P, ctypes.c_int32, P, P]
    L.rtq_trace_closest.argtypes = [P, P, ctypes.c_int64, P, P, P]
    L.rtq_trace_occluded.argtypes = [P, P, ctypes.c_int64, P, P, P]
    L.rtq_trace_closest_noalloc.argtypes = [P, P, ctypes.c_int64, P, P, P]
    L.rtq_trace_brute.argtypes = [P, P, ctypes.c_int64, P, P]
    L.rtq_host_bvh_build.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, P]
    L.rtq_host_bvh_get.argtypes = [P, P, P, P, P, P, P]
    L.rtq_host_bvh_destroy.argtypes = [P]
    L.rtq_host_bvh_destroy.restype = None
    L.rtq_render.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    L.rtq_render_backward.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
    L.rtq_render_timing.argtypes = [P, P, P]
    L.rtq_render_path.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P]
    for f in EXPORTS:
        if f not in ("rtq_last_error", "rtq_version", "rtq_scene_destroy", "rtq_host_bvh_destroy"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise RtqError(rc, load_library().rtq_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("rtq needs a HIP GPU (torch.cuda is not available)")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ----------------------------------------------------------------------------- scene
class Scene:
    """Built acceleration structures of a generator scene (``scenegen.Scene`` arrays)."""

    def __init__(self, s, formats: int = 0, leaf_max: int = 0, sah_bins: int = 0, build_threads: int = 0,
                 device: int = -1, open_pct: int = 0, node_width: int = 0, open_area_pct: int = 0):
        L = load_library()
        _torch()
        self.n_quads = int(s.quads.shape[0])
        curves = getattr(s, "curves", None)
        self.n_curves = 0 if curves is None else int(curves.shape[0])
        self.n_faces = self.n_quads + self.n_curves  # shading faces: quads, then curves, in prototype order
        verts = np.ascontiguousarray(s.verts, dtype=np.float32)
        quads = np.ascontiguousarray(s.quads, dtype=np.int32)
        albedo = np.ascontiguousarray(s.albedo, dtype=np.float32)
        assert albedo.shape[0] == self.n_faces
        cv = np.ascontiguousarray(curves if curves is not None else np.zeros((0, 16)), dtype=np.float32)
        co = s.proto_curve_off if curves is not None else np.zeros(s.n_protos + 1, np.int64)
        flat = getattr(s, "proto_curve_flat", None)
        P = s.n_protos
        protos = (_Proto * P)()
        vb = verts.ctypes.data
        qb = quads.ctypes.data
        ab = albedo.ctypes.data
        f0 = 0
        for p in range(P):
            v0, v1 = int(s.proto_vert_off[p]), int(s.proto_vert_off[p + 1])
            q0, q1 = int(s.proto_quad_off[p]), int(s.proto_quad_off[p + 1])
            c0, c1 = int(co[p]), int(co[p + 1])
            protos[p].verts = vb + 12 * v0
            protos[p].quads = qb + 16 * q0
            protos[p].n_verts = v1 - v0
            protos[p].n_quads = q1 - q0
            protos[p].albedo = ab + 4 * f0
            protos[p].curves = cv.ctypes.data + 64 * c0 if c1 > c0 else None
            protos[p].n_curves = c1 - c0
            protos[p].curves_flat = int(flat[p]) if flat is not None else 0
            f0 += (q1 - q0) + (c1 - c0)
        ip = np.ascontiguousarray(s.inst_proto, dtype=np.int32)
        ix = np.ascontiguousarray(s.inst_xform, dtype=np.float32)
        insts = _Insts(ip.shape[0], ip.ctypes.data, ix.ctypes.data)
        opts = _BuildOpts(formats, leaf_max, sah_bins, build_threads, device, open_pct, node_width, open_area_pct)
        h = ctypes.c_void_p()
        _check(L.rtq_scene_build(ctypes.cast(protos, ctypes.c_void_p), P, ctypes.byref(insts), ctypes.byref(opts),
                                 ctypes.byref(h)))
        self._h = h
        self.rgb = False
        self.tex_res = 0
        self.tex_ch = 1

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("scene is closed")
        return self._h

    def info(self) -> dict:
        i = _Info()
        _check(load_library().rtq_scene_get_info(self.handle, ctypes.byref(i)))
        out = {k: getattr(i, k) for k, _ in _Info._fields_}
        out["build_phase_seconds"] = list(i.build_phase_seconds)
        return out

    def set_albedo(self, albedo) -> None:
        assert albedo.dtype.is_floating_point and albedo.numel() == self.n_faces and albedo.is_cuda
        a = albedo.contiguous().float()
        _check(load_library().rtq_scene_set_albedo(self.handle, a.data_ptr(), a.numel(), _stream()))
        self._albedo_keep = a

    def set_textures(self, texels) -> None:
        """Per-face textures: a device tensor [n_quads, res, res] (row v, column u),
        read at the nearest texel of each hit's (u, v) in place of the face's
        albedo, or [n_quads, res, res, 3]: RGB texels, each channel scaling the
        material's tint (scenes with materials); None removes them."""
        if texels is None:
            _check(load_library().rtq_scene_set_textures(self.handle, None, 0, 1, _stream()))
            self._tex_keep = None
            self.tex_res = 0
            self.tex_ch = 1
            return
        assert texels.is_cuda and texels.dim() in (3, 4) and texels.shape[0] == self.n_quads
        assert texels.shape[1] == texels.shape[2] and (texels.dim() == 3 or texels.shape[3] == 3)
        ch = 3 if texels.dim() == 4 else 1
        t = texels.contiguous().float()
        _check(load_library().rtq_scene_set_textures(self.handle, t.data_ptr(), int(t.shape[1]), ch, _stream()))
        self._tex_keep = t
        self.tex_res = int(t.shape[1])
        self.tex_ch = ch

    def set_materials(self, mats, face_mat=None) -> None:
        """Principled materials: rows (tint r, g, b, roughness, metallic,
        specular[, clearcoat, clearcoat roughness]; rows of 6 have no coat) and
        one material index per unique face (uint8, device tensor or host
        array); None removes them.  With materials, images and image gradients
        have three channels per pixel (interleaved RGB)."""
        L = load_library()
        if mats is None:
            _check(L.rtq_scene_set_materials(self.handle, None, 0, None, _stream()))
            self.rgb = False
            return
        torch = _torch()
        m = np.asarray(mats, dtype=np.float32)
        m = m.reshape(-1, m.shape[-1])
        if m.shape[1] not in (6, 8):
            raise ValueError(f"material rows have 6 or 8 parameters, not {m.shape[1]}")
        arr = (_Material * m.shape[0])()
        for k, row in enumerate(m):
            arr[k].tint[:] = [float(x) for x in row[:3]]
            arr[k].roughness, arr[k].metallic, arr[k].specular = (float(x) for x in row[3:6])
            if m.shape[1] == 8:
                arr[k].clearcoat, arr[k].clearcoat_roughness = float(row[6]), float(row[7])
        fm = face_mat if isinstance(face_mat, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(face_mat, dtype=np.uint8))
        fm = fm.to(device="cuda", dtype=torch.uint8).contiguous()
        assert fm.numel() == self.n_faces
        _check(L.rtq_scene_set_materials(self.handle, ctypes.cast(arr, ctypes.c_void_p), m.shape[0], fm.data_ptr(),
                                         _stream()))
        self.rgb = True

    def set_environment(self, texels) -> None:
        """Environment map seen by escaping rays: a device tensor [h, w] (row 0
        around +z, columns from azimuth -pi), or None for the constant sky."""
        if texels is None:
            _check(load_library().rtq_scene_set_environment(self.handle, None, 0, 0, _stream()))
            self._env_keep = None
            return
        assert texels.is_cuda and texels.dim() == 2
        t = texels.contiguous().float()
        _check(load_library().rtq_scene_set_environment(self.handle, t.data_ptr(), int(t.shape[1]), int(t.shape[0]),
                                                        _stream()))
        self._env_keep = t

    def close(self):
        if getattr(self, "_h", None):
            load_library().rtq_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Hits:
    t: object
    u: object
    v: object
    inst: object
    prim: object
    ref: object = None  # [n, 2] int32 view of the opaque hit references, when asked for


def _rays_struct(rays, exclude=None, soa_in=False):
    """rays: CUDA float32 tensor [n, 8] (ox oy oz dx dy dz tmin tmax) -> SoA copy + struct,
    or, with soa_in, a contiguous float32 tensor [8, n] used in place (no copy);
    exclude: optional CUDA int32 tensor [n, 2] of hit references (Hits.ref) not to hit."""
    torch = _torch()
    if soa_in:
        assert rays.is_cuda and rays.dim() == 2 and rays.shape[0] == 8 and rays.dtype == torch.float32
        assert rays.is_contiguous()
        soa = rays
    else:
        assert rays.is_cuda and rays.dim() == 2 and rays.shape[1] == 8
        soa = rays.to(torch.float32).t().contiguous()
    n = soa.shape[1]
    ex = None
    if exclude is not None:
        assert exclude.is_cuda and exclude.shape == (n, 2) and exclude.dtype == torch.int32
        ex = exclude.contiguous()
    st = _Rays(*[soa[k].data_ptr() for k in range(8)], _ptr(ex))
    return (soa, ex), st


def _trace_opts(node_format=0, scheduler=SCHED_PLAIN, stack_depth=0, block=0, waves_per_cu=0, refill=0,
                visits=None, lane_stats=None):
    return _TraceOpts(node_format, scheduler, stack_depth, block, waves_per_cu, refill, _ptr(visits),
                      _ptr(lane_stats))


def trace_closest(scene: Scene, rays, exclude=None, want_ref: bool = False, soa_in: bool = False, **opts) -> Hits:
    """Closest hits of rays [n, 8] (or [8, n] structure of arrays with soa_in);
    exclude: optional [n, 2] int32 hit references of triangles the rays leave;
    want_ref: also return each hit's reference."""
    torch = _torch()
    n = rays.shape[1] if soa_in else rays.shape[0]
    soa, st = _rays_struct(rays, exclude, soa_in)
    dev = rays.device
    h = Hits(torch.empty(n, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev),
             torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
             torch.empty((n, 2), dtype=torch.int32, device=dev) if want_ref else None)
    hs = _Hits(h.t.data_ptr(), h.u.data_ptr(), h.v.data_ptr(), h.inst.data_ptr(), h.prim.data_ptr(), _ptr(h.ref))
    o = _trace_opts(**opts)
    _check(load_library().rtq_trace_closest(scene.handle, ctypes.byref(st), n, ctypes.byref(hs), ctypes.byref(o),
                                            _stream()))
    h._keep = (soa, o)
    return h


def trace_occluded(scene: Scene, rays, exclude=None, **opts):
    torch = _torch()
    n = rays.shape[0]
    soa, st = _rays_struct(rays, exclude)
    occ = torch.empty(n, dtype=torch.uint8, device=rays.device)
    o = _trace_opts(**opts)
    _check(load_library().rtq_trace_occluded(scene.handle, ctypes.byref(st), n, occ.data_ptr(), ctypes.byref(o),
                                             _stream()))
    occ._keep = soa
    return occ


def trace_brute(scene: Scene, rays, exclude=None) -> Hits:
    torch = _torch()
    n = rays.shape[0]
    soa, st = _rays_struct(rays, exclude)
    dev = rays.device
    h = Hits(torch.empty(n, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev),
             torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    hs = _Hits(h.t.data_ptr(), h.u.data_ptr(), h.v.data_ptr(), h.inst.data_ptr(), h.prim.data_ptr(), None)
    _check(load_library().rtq_trace_brute(scene.handle, ctypes.byref(st), n, ctypes.byref(hs), _stream()))
    h._keep = soa
    return h


# ----------------------------------------------------------------------------- rendering
def camera_structs(cams) -> tuple:
    """C cameras packed one after the other in the image buffer; a camera's
    view id defaults to its position in the list, its rectangle to the whole
    view.  Returns (array, total pixels)."""
    arr = (_Camera * len(cams))()
    off = 0
    for k, c in enumerate(cams):
        arr[k].eye[:] = list(c.eye)
        arr[k].look[:] = list(c.look)
        arr[k].up[:] = list(c.up)
        arr[k].vfov_deg = c.vfov_deg
        arr[k].w = c.w
        arr[k].h = c.h
        arr[k].img_offset = off
        vid = getattr(c, "view_id", None)
        arr[k].view_id = k if vid is None else int(vid)
        tile = getattr(c, "tile", None)
        if tile is None:
            tile = (0, 0, 0, 0)
        arr[k].tile_x, arr[k].tile_y, arr[k].tile_w, arr[k].tile_h = (int(x) for x in tile)
        off += (c.w * c.h) if tile[2] == 0 and tile[3] == 0 else tile[2] * tile[3]
    return arr, off


def render_opts(settings, node_format=0, scheduler=SCHED_PLAIN, stack_depth=0, block=0, waves_per_cu=0, refill=0,
                counters=None, view_done=None, start_tick=None, visits=None, dump_rays=None, dump_count=None,
                timing=False, graph=False, accumulate=0):
    o = _RenderOpts()
    o.seed = int(settings.seed)
    o.frame = int(settings.frame)
    o.light_dir[:] = [float(x) for x in settings.light_dir]
    o.E = float(settings.E)
    o.L_sky = float(settings.L_sky)
    o.node_format = node_format
    o.scheduler = scheduler
    o.stack_depth = stack_depth
    o.block = block
    o.waves_per_cu = waves_per_cu
    o.refill = refill
    o.counters = _ptr(counters)
    o.view_done = _ptr(view_done)
    o.start_tick = _ptr(start_tick)
    o.visits = _ptr(visits)
    o.dump_rays = _ptr(dump_rays)
    o.dump_cap = 0 if dump_rays is None else dump_rays.numel() // 12
    o.dump_count = _ptr(dump_count)
    o.timing = 1 if timing else 0
    o.graph = 1 if graph else 0
    o.accumulate = int(accumulate)
    al = np.ascontiguousarray(np.asarray(getattr(settings, "area_lights", ()), dtype=np.float32).reshape(-1, 10))
    o.n_area_lights = al.shape[0]
    o._area_keep = al  # the library reads it during the call
    o.area_lights = al.ctypes.data if al.shape[0] else None
    o.env_nee = 1 if getattr(settings, "env_nee", False) else 0
    return o


def _channels(scene) -> int:
    return 3 if getattr(scene, "rgb", False) else 1


def render(scene: Scene, cams, settings, images=None, **opts):
    """Packed FP32 image of all views (view c at its offset, row 0 at the top);
    [pixels, 3] (RGB) for a scene with materials."""
    torch = _torch()
    arr, total = camera_structs(cams)
    ch = _channels(scene)
    if images is None:
        images = torch.empty((total, 3) if ch == 3 else total, device="cuda", dtype=torch.float32)
    assert images.is_cuda and images.dtype == torch.float32 and images.numel() >= ch * total
    assert images.is_contiguous()
    o = render_opts(settings, **opts)
    o.channels = ch
    _check(load_library().rtq_render(scene.handle, ctypes.cast(arr, ctypes.c_void_p), len(cams), settings.spp,
                                     settings.depth, ctypes.byref(o), images.data_ptr(), _stream()))
    return images


def render_timing(scene: Scene) -> dict:
    """Kernel milliseconds and launch counts, by stage, of the render calls made
    with timing=True since the previous query (waits for their events)."""
    ms = (ctypes.c_float * 4)()
    n = (ctypes.c_int32 * 4)()
    _check(load_library().rtq_render_timing(scene.handle, ctypes.cast(ms, ctypes.c_void_p),
                                            ctypes.cast(n, ctypes.c_void_p)))
    names = ("closest", "shadow", "other", "call")
    return {k: {"ms": float(ms[i]), "launches": int(n[i])} for i, k in enumerate(names)}


def render_path(scene: Scene, cams, settings, view: int, pixel: int, sample: int, **opts):
    """One path traced alone: (vertices, escaped, radiance); each vertex a dict
    (inst, prim, half, shadow, face, t, albedo, cosl, radiance, origin and
    direction of the ray that found it)."""
    arr, _ = camera_structs(cams)
    o = render_opts(settings, **opts)
    o.channels = _channels(scene)
    d = settings.depth
    vi = (ctypes.c_int32 * (6 * d))()
    vf = (ctypes.c_float * (10 * d))()
    nv, esc, rad = ctypes.c_int32(), ctypes.c_int32(), (ctypes.c_float * 3)()
    _check(load_library().rtq_render_path(scene.handle, ctypes.cast(arr, ctypes.c_void_p), len(cams), settings.spp,
                                          d, ctypes.byref(o), view, pixel, sample, ctypes.cast(vi, ctypes.c_void_p),
                                          ctypes.cast(vf, ctypes.c_void_p), ctypes.byref(nv), ctypes.byref(esc),
                                          ctypes.cast(rad, ctypes.c_void_p), _stream()))
    verts = [dict(inst=vi[6 * k], prim=vi[6 * k + 1], half=vi[6 * k + 2], shadow=vi[6 * k + 3], face=vi[6 * k + 4],
                  t=vf[10 * k], albedo=vf[10 * k + 1], cosl=vf[10 * k + 2], radiance=vf[10 * k + 3],
                  origin=tuple(vf[10 * k + 4:10 * k + 7]), direction=tuple(vf[10 * k + 7:10 * k + 10]))
             for k in range(nv.value)]
    return verts, bool(esc.value), (tuple(rad) if o.channels == 3 else float(rad[0]))


def render_path_raw(scene: Scene, cams, settings, view: int, pixel: int, sample: int, **opts):
    """One path traced alone, as recorded by the library: (n_vert, vi [depth, 6]
    int32, vf [depth, 10] float32, escaped, radiance: a float32, or 3 for a scene
    with materials); when the path escaped, row n_vert holds the escaping ray."""
    arr, _ = camera_structs(cams)
    o = render_opts(settings, **opts)
    o.channels = _channels(scene)
    d = settings.depth
    vi = np.zeros((d, 6), np.int32)
    vf = np.zeros((d, 10), np.float32)
    nv, esc = ctypes.c_int32(), ctypes.c_int32()
    rad = np.zeros(3, np.float32)
    _check(load_library().rtq_render_path(scene.handle, ctypes.cast(arr, ctypes.c_void_p), len(cams), settings.spp,
                                          d, ctypes.byref(o), view, pixel, sample, vi.ctypes.data, vf.ctypes.data,
                                          ctypes.byref(nv), ctypes.byref(esc), rad.ctypes.data, _stream()))
    return nv.value, vi, vf, bool(esc.value), (rad if o.channels == 3 else np.float32(rad[0]))


def render_backward(scene: Scene, cams, settings, grad_images, grad_albedo=None, **opts):
    torch = _torch()
    arr, total = camera_structs(cams)
    g = grad_images.contiguous().float()
    ch = _channels(scene)
    assert g.numel() == ch * total and g.is_cuda
    if grad_albedo is None:
        # one entry per shading parameter: per face, or per texel (and channel
        # of an RGB texel) with textures
        n_par = scene.n_faces * max(1, getattr(scene, "tex_res", 0)) ** 2
        if getattr(scene, "tex_res", 0) > 0:
            n_par *= getattr(scene, "tex_ch", 1)
        grad_albedo = torch.zeros(n_par, device=g.device, dtype=torch.float32)
    o = render_opts(settings, **opts)
    o.channels = ch
    _check(load_library().rtq_render_backward(scene.handle, ctypes.cast(arr, ctypes.c_void_p), len(cams),
                                              settings.spp, settings.depth, ctypes.byref(o), g.data_ptr(),
                                              grad_albedo.data_ptr(), _stream()))
    return grad_albedo


# ----------------------------------------------------------------------------- host BVH
NODE_WIDE = np.dtype([("lo", "<f4", (3, 8)), ("hi", "<f4", (3, 8)), ("child", "<u4", 8)])
NODE_F32 = np.dtype([("lo_x", "<f4", 4), ("hi_x", "<f4", 4), ("lo_y", "<f4", 4), ("hi_y", "<f4", 4),
                     ("lo_z", "<f4", 4), ("hi_z", "<f4", 4), ("child", "<u4", 4), ("pad", "<u4", 4)])
NODE_Q8 = np.dtype([("origin", "<f4", 3), ("exps", "<u4"), ("lo_x", "<u4"), ("hi_x", "<u4"), ("lo_y", "<u4"),
                    ("hi_y", "<u4"), ("lo_z", "<u4"), ("hi_z", "<u4"), ("child", "<u4", 4), ("pad", "<u4", 2)])
NODE_Q8W8 = np.dtype([("origin", "<f4", 3), ("exps", "<u4"), ("lo_x", "<u4", 2), ("hi_x", "<u4", 2),
                      ("lo_y", "<u4", 2), ("hi_y", "<u4", 2), ("lo_z", "<u4", 2), ("hi_z", "<u4", 2),
                      ("child", "<u4", 8)])
NODE_Q8W2 = np.dtype([("origin", "<f4", 3), ("exps", "<u4"), ("x", "<u4"), ("y", "<u4"), ("z", "<u4"),
                      ("child", "<u4", 2), ("pad", "<u4", 3)])
_Q8_DTYPE = {2: NODE_Q8W2, 4: NODE_Q8, 8: NODE_Q8W8}


def host_bvh(boxes, leaf_max: int = 4, bins: int = 32, threads: int = 0, width: int = 4) -> dict:
    """The scene builder's W-wide BVH over host boxes ([n, 6] lo xyz, hi xyz),
    built on the host (no device): dict of exact FP32 boxes ("wide"), device
    FP32 nodes ("f32", width 4 only, else None), quantized nodes ("q8") as
    numpy structured arrays, leaf order, depth and width."""
    L = load_library()
    b = np.ascontiguousarray(boxes, dtype=np.float32).reshape(-1, 6)
    h = ctypes.c_void_p()
    _check(L.rtq_host_bvh_build(b.ctypes.data, b.shape[0], int(leaf_max), int(bins), int(threads), int(width),
                                ctypes.byref(h)))
    try:
        pw, pf, pq, po = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        nn, depth = ctypes.c_int64(), ctypes.c_int32()
        _check(L.rtq_host_bvh_get(h, ctypes.byref(pw), ctypes.byref(pf), ctypes.byref(pq), ctypes.byref(nn),
                                  ctypes.byref(po), ctypes.byref(depth)))
        n = nn.value
        qd = _Q8_DTYPE[int(width)]
        wide = np.frombuffer(ctypes.string_at(pw.value, n * NODE_WIDE.itemsize), dtype=NODE_WIDE).copy()
        f32 = (np.frombuffer(ctypes.string_at(pf.value, n * NODE_F32.itemsize), dtype=NODE_F32).copy()
               if pf.value else None)
        q8 = np.frombuffer(ctypes.string_at(pq.value, n * qd.itemsize), dtype=qd).copy()
        order = np.frombuffer(ctypes.string_at(po.value, 4 * b.shape[0]), dtype=np.uint32).copy()
    finally:
        L.rtq_host_bvh_destroy(h)
    return {"wide": wide, "f32": f32, "q8": q8, "order": order, "depth": depth.value, "width": int(width)}


def version() -> str:
    return load_library().rtq_version().decode()
