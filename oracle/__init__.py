"""ctypes wrapper of the FP64 CPU oracle (``oracle/oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this module and this module never imports the product package; both consume
the same seeded input arrays (numpy) and nothing else.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# Ray flag bits (see oracle.cpp)
F_NEAR_TIE = 1
F_GRAZE = 2
F_NEAR_ORIGIN = 4
F_T_ILLCOND = 8
F_DIAG = 16
F_SHADE = 32
ID_FLAGS = F_NEAR_TIE | F_GRAZE | F_NEAR_ORIGIN

# verdicts of OracleScene.accept (closest hit) and OracleScene.check_path
ACCEPT_CODES = {1: "not a possible answer", 2: "miss while a certain hit exists", 3: "t outside its tolerance"}
PATH_CODES = {1: "camera ray", 2: "hit is not a possible answer", 3: "escape while a certain hit exists",
              4: "t outside its tolerance", 5: "face index", 6: "shading value", 7: "shadow ray cast or not",
              8: "shadow outcome", 9: "next origin is not the FP32 hit point", 10: "next direction",
              11: "path length", 12: "radiance", -1: "bad arguments"}


def build(force: bool = True) -> str:
    """Compile the oracle: plain C++17, -O3, no fast-math, std::thread."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O3", "-march=x86-64-v3", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
           "-pthread",
           "-Wall", "-o", tmp, _SRC]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        L.orc_scene_create.restype = P
        L.orc_scene_create.argtypes = [P, i64, P, i64, P, P, i32, P, P, P, i64, P, P, P]
        L.orc_scene_destroy.argtypes = [P]
        L.orc_scene_set_albedo.argtypes = [P, P]
        L.orc_scene_set_textures.argtypes = [P, P, i32, i32]
        L.orc_scene_set_environment.argtypes = [P, P, i32, i32]
        L.orc_scene_set_materials.argtypes = [P, P, i32, P]
        L.orc_bsdf_eval.argtypes = [P, P, P, i64, P, P]
        L.orc_scene_capsules.argtypes = [P, P]
        L.orc_scene_capsules.restype = i64
        L.orc_bsdf_sample.argtypes = [P, P, P, i64, P, P, P]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_philox.argtypes = [P, P, P]
        L.orc_trace.argtypes = [P, i64, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P]
        L.orc_trace_d.argtypes = [P, i64, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P]
        L.orc_render.argtypes = [P, P, P, i32, P, P, P, P, i64, i32, P, P, P]
        L.orc_grad.argtypes = [P, P, P, i32, P, P, P, P, i64, i32, P, i32, P, P, P, P, P, i32]
        L.orc_path.argtypes = [P, P, P, i32, P, P, P, i64, i32, P, P, P, P, P]
        L.orc_flag_breakdown.argtypes = [P, P, P, i32, P, P, P, P, i64, P]
        L.orc_accept.argtypes = [P, i64, P, P, P, i32, i32, P, P, P, P, P, P, P]
        L.orc_check_path.argtypes = [P, P, P, i32, P, P, P, i32, i64, i32, i32, P, P, i32, P, P]
        L.orc_check_path.restype = i32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(out))
    return out


def _mat8(mat) -> np.ndarray:
    """Material rows of 8 parameters (tint r, g, b, roughness, metallic,
    specular, clearcoat, clearcoat roughness); rows of 6 have no clearcoat."""
    m = np.asarray(mat, dtype=np.float64)
    if m.shape[-1] == 6:
        m = np.concatenate([m, np.zeros(m.shape[:-1] + (2,))], axis=-1)
    assert m.shape[-1] == 8, m.shape
    return np.ascontiguousarray(m)


def bsdf_eval(mat, n, wo, wi):
    """The oracle's BSDF at one frame (tests): mat = (tint r, g, b, roughness,
    metallic, specular[, clearcoat, clearcoat roughness]), unit n and wo,
    directions wi [k, 3].  Returns [k, 4]: (A, B, pdf, Pn) with f mu_i = A + B c
    for base color c, Pn the probability of a specular or coat lobe."""
    m = _mat8(mat)
    nn = np.ascontiguousarray(n, dtype=np.float64)
    o = np.ascontiguousarray(wo, dtype=np.float64)
    w = np.ascontiguousarray(np.asarray(wi, dtype=np.float64).reshape(-1, 3))
    out = np.zeros((w.shape[0], 4))
    lib().orc_bsdf_eval(_p(m), _p(nn), _p(o), w.shape[0], _p(w), _p(out))
    return out


def bsdf_sample(mat, n, wo, u):
    """Sampled bounce directions for lobe and direction words u [k, 3] in [0, 1):
    (directions [k, 3], lobe [k] (0 cosine, 1 specular, 2 coat), lobe word
    within rounding of a threshold [k])."""
    m = _mat8(mat)
    nn = np.ascontiguousarray(n, dtype=np.float64)
    o = np.ascontiguousarray(wo, dtype=np.float64)
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1, 3))
    wi = np.zeros_like(uu)
    info = np.zeros((uu.shape[0], 2), np.int32)
    lib().orc_bsdf_sample(_p(m), _p(nn), _p(o), uu.shape[0], _p(uu), _p(wi), _p(info))
    return wi, info[:, 0].copy(), info[:, 1].astype(bool)


@dataclass
class Hits:
    t: np.ndarray
    inst: np.ndarray
    prim: np.ndarray
    half: np.ndarray
    u: np.ndarray
    v: np.ndarray
    flags: np.ndarray
    cand: np.ndarray
    ncand: np.ndarray
    scale: np.ndarray  # position scale of each answer (max of 1, |o|, |p|, hit-quad extent from o)


class OracleScene:
    """FP64 oracle view of a scene given as the generator's arrays."""

    def __init__(self, scene):
        self._keep = dict(
            verts=np.ascontiguousarray(scene.verts, dtype=np.float32),
            quads=np.ascontiguousarray(scene.quads, dtype=np.int32),
            vo=np.ascontiguousarray(scene.proto_vert_off, dtype=np.int64),
            qo=np.ascontiguousarray(scene.proto_quad_off, dtype=np.int64),
            albedo=np.ascontiguousarray(scene.albedo, dtype=np.float32),
            ip=np.ascontiguousarray(scene.inst_proto, dtype=np.int32),
            x=np.ascontiguousarray(scene.inst_xform, dtype=np.float32),
        )
        curves = getattr(scene, "curves", None)
        if curves is not None:
            self._keep["curves"] = np.ascontiguousarray(curves, dtype=np.float32)
            self._keep["co"] = np.ascontiguousarray(scene.proto_curve_off, dtype=np.int64)
            flat = getattr(scene, "proto_curve_flat", None)
            if flat is not None:
                self._keep["flat"] = np.ascontiguousarray(flat, dtype=np.int32)
        k = self._keep
        # shading faces: every quad and every curve (in prototype order)
        self.n_quads = int(k["albedo"].shape[0])
        self.tex_res = 0
        self.tex_ch = 1
        self.rgb = False
        self.h = lib().orc_scene_create(_p(k["verts"]), k["verts"].shape[0], _p(k["quads"]), k["quads"].shape[0],
                                        _p(k["vo"]), _p(k["qo"]), k["qo"].shape[0] - 1, _p(k["albedo"]),
                                        _p(k["ip"]), _p(k["x"]), k["ip"].shape[0], _p(k.get("curves")),
                                        _p(k.get("co")), _p(k.get("flat")))
        if not self.h:
            raise ValueError("oracle: singular instance transform")

    def close(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_albedo(self, albedo: np.ndarray) -> None:
        a = np.ascontiguousarray(albedo, dtype=np.float64)
        assert a.shape == (self.n_quads,)
        lib().orc_scene_set_albedo(self.h, _p(a))

    @property
    def n_params(self) -> int:
        """Shading parameters that gradients refer to: one albedo per face, or,
        with textures, every texel (face-major, then row v, column u), and with
        RGB texels every channel of every texel (channel fastest)."""
        return self.n_quads * (self.tex_res * self.tex_res * self.tex_ch if self.tex_res > 0 else 1)

    def set_materials(self, mats: Optional[np.ndarray], face_mat: Optional[np.ndarray] = None) -> None:
        """Principled materials: [n_mat, 6] or [n_mat, 8] rows (tint r, g, b,
        roughness, metallic, specular[, clearcoat, clearcoat roughness]; FP32
        values read exactly; 6 columns: no clearcoat) and one material index per
        face; None returns to Lambertian faces.  With materials, images and
        gradient weights have three channels."""
        if mats is None:
            assert lib().orc_scene_set_materials(self.h, None, 0, None) == 0
            self.rgb = False
            return
        m32 = np.asarray(mats, dtype=np.float32)
        m = _mat8(m32.reshape(-1, m32.shape[-1]).astype(np.float64))
        f = np.ascontiguousarray(face_mat, dtype=np.int32)
        assert f.shape == (self.n_quads,)
        assert lib().orc_scene_set_materials(self.h, _p(m), int(m.shape[0]), _p(f)) == 0
        self._mats = (m, f)
        self.rgb = True

    def capsules(self) -> np.ndarray:
        """The segments the curves are tessellated into: [n, 8] (a, b, radius at
        a, radius at b; equal for the capsules of round curves)."""
        n = int(lib().orc_scene_capsules(self.h, None))
        out = np.zeros((n, 8))
        lib().orc_scene_capsules(self.h, _p(out))
        return out

    def set_textures(self, texels: Optional[np.ndarray]) -> None:
        """Per-face textures [n_quads, res, res] (row v, column u; FP32 values read
        exactly) or [n_quads, res, res, 3] (RGB base colors, for scenes with
        materials), or None to shade with the per-face albedo again.  With
        textures the gradient functions refer to the texels (and channels)."""
        if texels is None:
            assert lib().orc_scene_set_textures(self.h, None, 0, 1) == 0
            self.tex_res = 0
            self.tex_ch = 1
            return
        t = np.ascontiguousarray(np.asarray(texels, dtype=np.float32), dtype=np.float64)
        ch = 3 if t.ndim == 4 else 1
        assert t.ndim in (3, 4) and t.shape[0] == self.n_quads and t.shape[1] == t.shape[2] >= 1
        assert ch == 1 or t.shape[3] == 3
        assert lib().orc_scene_set_textures(self.h, _p(t), int(t.shape[1]), ch) == 0
        self._tex = t
        self.tex_res = int(t.shape[1])
        self.tex_ch = ch

    def set_environment(self, texels: Optional[np.ndarray]) -> None:
        """Environment map [h, w] (row 0 around +z; FP32 values read exactly)
        seen by escaping rays in place of the constant sky, or None."""
        if texels is None:
            assert lib().orc_scene_set_environment(self.h, None, 0, 0) == 0
            return
        t = np.ascontiguousarray(np.asarray(texels, dtype=np.float32), dtype=np.float64)
        assert t.ndim == 2 and t.shape[0] >= 1 and t.shape[1] >= 1
        assert lib().orc_scene_set_environment(self.h, _p(t), int(t.shape[1]), int(t.shape[0])) == 0
        self._env = t

    def trace(self, rays: np.ndarray, excl: Optional[np.ndarray] = None, r0: Optional[np.ndarray] = None,
              brute: bool = False, any_hit: bool = False) -> Hits:
        """Closest hit (or, with any_hit, the first-hit occlusion flags) of n rays given
        as [n, 8] (ox oy oz dx dy dz tmin tmax): FP32 rays are read exactly, FP64 rays
        are used as they are."""
        f64 = rays.dtype == np.float64
        rays = np.ascontiguousarray(rays, dtype=np.float64 if f64 else np.float32)
        n = rays.shape[0]
        ex = None if excl is None else np.ascontiguousarray(excl, dtype=np.int32)
        rr = None if r0 is None else np.ascontiguousarray(r0, dtype=np.float64)
        out = Hits(t=np.zeros(n), inst=np.zeros(n, np.int32), prim=np.zeros(n, np.int32),
                   half=np.zeros(n, np.int32), u=np.zeros(n), v=np.zeros(n), flags=np.zeros(n, np.uint32),
                   cand=np.zeros((n, 8), np.int32), ncand=np.zeros(n, np.int32), scale=np.zeros(n))
        fn = lib().orc_trace_d if f64 else lib().orc_trace
        fn(self.h, n, _p(rays), _p(ex), _p(rr), 0 if brute else 1, 1 if any_hit else 0, _p(out.t),
                        _p(out.inst), _p(out.prim), _p(out.half), _p(out.u), _p(out.v), _p(out.flags),
                        _p(out.cand), _p(out.ncand), _p(out.scale))
        return out

    def accept(self, rays: np.ndarray, inst: np.ndarray, prim: Optional[np.ndarray] = None,
               t: Optional[np.ndarray] = None, half: Optional[np.ndarray] = None,
               excl: Optional[np.ndarray] = None, r0: Optional[np.ndarray] = None, any_hit: bool = False,
               brute: bool = False, want_ulps: bool = False):
        """Whether each answer (closest: inst, prim, t and optionally half, inst -1 for a
        miss; any_hit: inst = 1 occluded / 0 not) is one an FP32 traversal may give
        for the FP32 ray.  Returns (code [n] int32, 0 = valid, see ACCEPT_CODES;
        info [n] int32 bits: 1 the certain hit, 2 t ill-conditioned (held to the FP32 bound of
        16 units of 2^-24 S / (|d| |cos|) instead of 1e-5 relative), 4 other answers possible;
        with want_ulps also the t error of each answer in units of 2^-24 S / (|d| |cos|))."""
        rays = np.ascontiguousarray(rays, dtype=np.float32)
        n = rays.shape[0]
        gi = np.ascontiguousarray(inst, dtype=np.int32)
        gp = None if prim is None else np.ascontiguousarray(prim, dtype=np.int32)
        gh = None if half is None else np.ascontiguousarray(half, dtype=np.int32)
        gt = None if t is None else np.ascontiguousarray(t, dtype=np.float32)
        if not any_hit:
            assert gp is not None and gt is not None
        ex = None if excl is None else np.ascontiguousarray(excl, dtype=np.int32)
        rr = None if r0 is None else np.ascontiguousarray(r0, dtype=np.float64)
        out = np.zeros(n, np.int32)
        info = np.zeros(n, np.int32)
        ul = np.zeros(n) if want_ulps else None
        lib().orc_accept(self.h, n, _p(rays), _p(ex), _p(rr), 0 if brute else 1, 1 if any_hit else 0, _p(gi),
                         _p(gp), _p(gh), _p(gt), _p(out), _p(info), _p(ul))
        return (out, info, ul) if want_ulps else (out, info)

    def flag_breakdown(self, cams, settings, pixels: np.ndarray) -> np.ndarray:
        """Flags by kind and bounce over the listed packed pixels (every sample):
        [16, 8] counts; row b = closest-hit rays of bounce b; columns: near tie,
        graze, near origin, ill-conditioned t, diagonal, shading within
        rounding, flagged shadow rays, all closest-hit rays."""
        cf, ci, _ = self._cams(cams)
        pi, pu, pd = self._params(settings)
        px = np.ascontiguousarray(pixels, dtype=np.int64)
        out = np.zeros(16 * 8)
        lib().orc_flag_breakdown(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), _p(px), px.shape[0],
                                 _p(out))
        return out.reshape(16, 8)

    def check_path(self, cams, settings, cam: int, local: int, sample: int, nv: int, vi: np.ndarray,
                   vf: np.ndarray, escaped: bool, radiance):
        """Check a GPU path record (rtq_render_path: vi 6 int32 and vf 10 float32 per
        recorded ray, the escaping ray last) step by step along its own rays.
        Returns (code, stats): code 0 = valid, else PATH_CODES[code]; stats: failing
        ray, FP64 radiance along the path, vertices, certain answers, vertices
        whose t is ill-conditioned (held to the FP32 bound), shading decisions
        within rounding of a threshold, largest t error in units of
        2^-24 S / (|d| |cos|), and the FP64 radiance of every channel ("Lc").
        radiance: the GPU's value (a float, or 3 with materials)."""
        cf, ci, _ = self._cams(cams)
        pi, pu, pd = self._params(settings)
        vi = np.ascontiguousarray(vi, dtype=np.int32)
        vf = np.ascontiguousarray(vf, dtype=np.float32)
        st = np.zeros(10)
        rad = np.zeros(3, np.float32)
        rad[:] = np.asarray(radiance, dtype=np.float32).ravel()  # a scalar fills all three channels
        code = lib().orc_check_path(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), int(cam), int(local),
                                    int(sample), int(nv), _p(vi), _p(vf), 1 if escaped else 0, _p(rad), _p(st))
        return int(code), dict(ray=int(st[0]), L=float(st[1]), vertices=int(st[2]), certain=int(st[3]),
                               t_waived=int(st[4]), ambiguous_shading=int(st[5]), max_t_ulps=float(st[6]),
                               Lc=st[7:10].copy())

    @staticmethod
    def _params(settings):
        pi = np.array([settings.spp, settings.depth, 1 if getattr(settings, "env_nee", False) else 0],
                      dtype=np.int32)
        pu = np.array([settings.seed, settings.frame], dtype=np.uint64)
        al = np.asarray(settings.area_lights, dtype=np.float32).reshape(-1, 10).astype(np.float64)
        pd = np.array(list(settings.light_dir) + [settings.E, settings.L_sky, al.shape[0]] + al.ravel().tolist(),
                      dtype=np.float64)
        if not (1 <= settings.depth <= 64):
            raise ValueError("depth must be in [1, 64]")
        return pi, pu, pd

    @staticmethod
    def _cams(cams):
        cf = np.array([list(c.eye) + list(c.look) + list(c.up) + [c.vfov_deg] for c in cams], dtype=np.float64)
        off = 0
        ci = []
        for k, c in enumerate(cams):
            vid = getattr(c, "view_id", None)
            tile = getattr(c, "tile", None) or (0, 0, c.w, c.h)
            ci.append([c.w, c.h, off, k if vid is None else vid] + [int(x) for x in tile])
            off += tile[2] * tile[3]
        return np.ascontiguousarray(cf), np.array(ci, dtype=np.int64).reshape(-1, 8), off

    def render(self, cams, settings, pixels: Optional[np.ndarray] = None, brute: bool = False):
        """Returns (image or per-listed-pixel radiance [f64]: [n] without materials,
        [n, 3] with them; pixel flags [u8]; stats dict)."""
        if self.tex_res > 0 and self.tex_ch == 3 and not self.rgb:
            raise ValueError("RGB textures shade a scene with materials")
        cf, ci, total = self._cams(cams)
        pi, pu, pd = self._params(settings)
        px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
        n = total if px is None else px.shape[0]
        img = np.zeros((n, 3))
        fl = np.zeros(n, np.uint8)
        st = np.zeros(4)
        lib().orc_render(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), _p(px),
                         0 if px is None else n, 0 if brute else 1, _p(img), _p(fl), _p(st))
        stats = dict(closest=st[0], shadow=st[1], incoherent=st[2], flagged_pixels=st[3])
        return (img if self.rgb else img[:, 0].copy()), fl, stats

    def grad(self, cams, settings, gpix: np.ndarray, pixels: Optional[np.ndarray] = None, brute: bool = False,
             taint: str = "pixel"):
        """Path-replay gradient of sum_p gpix[p] * I_p w.r.t. the shading
        parameters (per-face albedo, or the texels of a textured scene).
        Returns (grad [n_params] f64, pixel flags, tainted-parameter mask).  taint="pixel" marks
        every face on any path of a flagged pixel; taint="path" only the faces on
        flagged paths (valid when both sides use these same pixel weights)."""
        cf, ci, total = self._cams(cams)
        pi, pu, pd = self._params(settings)
        px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
        n = total if px is None else px.shape[0]
        g = self._gpix(gpix, n)
        out = np.zeros(self.n_params)
        fl = np.zeros(n, np.uint8)
        tmask = np.zeros(self.n_params, np.uint8)
        lib().orc_grad(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), _p(px), 0 if px is None else n,
                       0 if brute else 1, _p(g), 0, None, _p(out), None, _p(fl), _p(tmask),
                       1 if taint == "path" else 0)
        return out, fl, tmask

    def tangent(self, cams, settings, tangent: np.ndarray, pixels: Optional[np.ndarray] = None):
        """Forward-mode (dual number) derivative of each pixel along a tangent of
        the shading parameters (per face, or per texel with textures)."""
        cf, ci, total = self._cams(cams)
        pi, pu, pd = self._params(settings)
        px = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
        n = total if px is None else px.shape[0]
        tg = np.ascontiguousarray(tangent, dtype=np.float64)
        assert tg.shape == (self.n_params,)
        dI = np.zeros((n, 3))
        fl = np.zeros(n, np.uint8)
        lib().orc_grad(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), _p(px), 0 if px is None else n,
                       1, None, 1, _p(tg), None, _p(dI), _p(fl), None, 0)
        return (dI if self.rgb else dI[:, 0].copy()), fl

    def _gpix(self, gpix, n):
        """Pixel weights as [n, 3]: [n] weights (no materials) go to channel 0
        (the three channels are equal there), [n, 3] with materials."""
        g = np.asarray(gpix, dtype=np.float64)
        out = np.zeros((n, 3))
        if self.rgb:
            assert g.shape == (n, 3)
            out[:] = g
        else:
            assert g.shape == (n,)
            out[:, 0] = g
        return np.ascontiguousarray(out)

    def path(self, cams, settings, pixel: int, sample: int):
        """The vertices of one path: list of dicts (inst, prim, half, t, albedo,
        shadow: -1 none / 0 visible / 1 occluded, flags, shadow_flags), escaped, path flags."""
        cf, ci, _ = self._cams(cams)
        pi, pu, pd = self._params(settings)
        nv = np.zeros(1, np.int32)
        oi = np.zeros(6 * 64, np.int32)
        od = np.zeros(2 * 64)
        esc = np.zeros(1, np.int32)
        pf = np.zeros(1, np.uint32)
        lib().orc_path(self.h, _p(cf), _p(ci), len(cams), _p(pi), _p(pu), _p(pd), int(pixel), int(sample), _p(nv),
                       _p(oi), _p(od), _p(esc), _p(pf))
        verts = []
        for k in range(int(nv[0])):
            verts.append(dict(inst=int(oi[6 * k]), prim=int(oi[6 * k + 1]), half=int(oi[6 * k + 2]),
                              shadow=int(oi[6 * k + 3]), flags=int(oi[6 * k + 4]) & 0xFFFFFFFF,
                              shadow_flags=int(oi[6 * k + 5]) & 0xFFFFFFFF, t=float(od[2 * k]),
                              albedo=float(od[2 * k + 1])))
        return verts, bool(esc[0]), int(pf[0])
