"""Seeded synthetic scenes, cameras and render settings.

This module only *produces inputs*: prototype quad meshes, instance transforms,
per-face albedo, cameras and light settings.  It contains none of the
arithmetic of the rendering method itself (no ray tests, no traversal, no
shading), so both the HIP library and the CPU oracle can consume the very same
arrays.

The scenes stand in for the Moana Island Scene, which is not available here.
They reproduce the properties the paper singles out as what makes that scene
hard (Section 4.2): many small prototypes instanced many times with heavy
overlap, instances sitting on a coarse terrain, long thin quads, and a huge
range of tessellation densities.  The instancing is object-level (one instance
= one prototype), as adopted in Section 5.2, and the geometry is quads
(Section 5.2, "Quads").

Conventions
-----------
* A quad is four vertex indices (v0, v1, v2, v3), counter-clockwise.  Indices
  are local to the prototype's vertex block.
* An instance transform is a row-major 3x4 FP32 matrix [A | t] mapping object
  space to world space: w = A v + t.
* Albedo is one FP32 value per unique prototype quad.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple, Callable

import numpy as np

SEED_BASE = 2001026200


@dataclass
class Scene:
    verts: np.ndarray          # float32 [V, 3], all prototypes concatenated
    quads: np.ndarray          # int32 [Q, 4], indices local to the prototype
    proto_vert_off: np.ndarray  # int64 [P + 1]
    proto_quad_off: np.ndarray  # int64 [P + 1]
    albedo: np.ndarray         # float32 [F]: one per face (quad, or curve) in prototype order
    inst_proto: np.ndarray     # int32 [N]
    inst_xform: np.ndarray     # float32 [N, 12]
    # curves (a prototype holds quads or curves): 4 control points (x, y, z,
    # radius) per cubic Bezier curve, and per-prototype offsets
    curves: Optional[np.ndarray] = None           # float32 [C, 16]
    proto_curve_off: Optional[np.ndarray] = None  # int64 [P + 1]
    # per prototype of curves: 0 round curves, 1 flat (ray-facing) ribbons
    proto_curve_flat: Optional[np.ndarray] = None  # int32 [P]

    @property
    def n_protos(self) -> int:
        return int(self.proto_quad_off.shape[0] - 1)

    @property
    def n_quads(self) -> int:
        return int(self.quads.shape[0])

    @property
    def n_instances(self) -> int:
        return int(self.inst_proto.shape[0])

    @property
    def n_curves(self) -> int:
        return 0 if self.curves is None else int(self.curves.shape[0])

    @property
    def n_faces(self) -> int:
        """Shading faces: every quad and every curve."""
        return self.n_quads + self.n_curves

    def proto_face_off(self) -> np.ndarray:
        """First face of each prototype (its quads, or its curves)."""
        nq = np.diff(self.proto_quad_off)
        nc = np.diff(self.proto_curve_off) if self.proto_curve_off is not None else np.zeros_like(nq)
        return np.concatenate([[0], np.cumsum(nq + nc)]).astype(np.int64)

    def instanced_quads(self) -> int:
        counts = np.diff(self.proto_quad_off)
        return int(counts[self.inst_proto].sum())

    def validate(self) -> None:
        P = self.n_protos
        assert self.verts.dtype == np.float32 and self.verts.ndim == 2 and self.verts.shape[1] == 3
        assert self.quads.dtype == np.int32 and self.quads.shape[1] == 4
        assert self.albedo.dtype == np.float32 and self.albedo.shape[0] == self.n_faces
        if self.curves is not None:
            assert self.curves.dtype == np.float32 and self.curves.ndim == 2 and self.curves.shape[1] == 16
            assert self.proto_curve_off[-1] == self.curves.shape[0]
            nq, nc = np.diff(self.proto_quad_off), np.diff(self.proto_curve_off)
            assert ((nq > 0) != (nc > 0)).all(), "a prototype holds quads or curves"
            assert (self.curves[:, 3::4] >= 0).all()
            if self.proto_curve_flat is not None:
                assert self.proto_curve_flat.shape == (P,) and ((self.proto_curve_flat == 0) | (nc > 0)).all()
        assert self.proto_vert_off[-1] == self.verts.shape[0]
        assert self.proto_quad_off[-1] == self.quads.shape[0]
        assert self.inst_proto.dtype == np.int32 and self.inst_xform.dtype == np.float32
        assert self.inst_xform.shape == (self.inst_proto.shape[0], 12)
        assert (self.inst_proto >= 0).all() and (self.inst_proto < P).all()


@dataclass
class Camera:
    eye: Tuple[float, float, float]
    look: Tuple[float, float, float]
    up: Tuple[float, float, float]
    vfov_deg: float
    w: int
    h: int
    # index of the view in the random-number counter (None: its position in the
    # camera list of the call), and the rectangle (x, y, w, h) of the view that
    # is rendered (None: all of it) -- a tile of an image-parallel split
    view_id: Optional[int] = None
    tile: Optional[Tuple[int, int, int, int]] = None

    def rect(self) -> Tuple[int, int, int, int]:
        return self.tile if self.tile is not None else (0, 0, self.w, self.h)

    def n_pixels(self) -> int:
        r = self.rect()
        return r[2] * r[3]


@dataclass
class RenderSettings:
    spp: int = 1
    depth: int = 3
    seed: int = SEED_BASE + 1
    frame: int = 0
    light_dir: Tuple[float, float, float] = field(
        default_factory=lambda: tuple((np.array([1.0, -1.0, 2.0]) / math.sqrt(6.0)).tolist()))
    E: float = math.pi
    L_sky: float = 0.25
    # quad area lights: (corner xyz, edge-1 xyz, edge-2 xyz, emitted radiance)
    # each, emitting from the side that edge 1 x edge 2 faces
    area_lights: Tuple[Tuple[float, ...], ...] = ()
    # next-event estimation toward the environment map (when the scene has one)
    env_nee: bool = False


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def _concat(protos: List[Tuple[np.ndarray, np.ndarray]], albedo_rng: np.random.Generator,
            inst_proto: np.ndarray, inst_xform: np.ndarray,
            albedo_lo: float = 0.2, albedo_hi: float = 0.8) -> Scene:
    vo = [0]
    qo = [0]
    for v, q in protos:
        vo.append(vo[-1] + v.shape[0])
        qo.append(qo[-1] + q.shape[0])
    verts = np.concatenate([v for v, _ in protos]).astype(np.float32, copy=False)
    quads = np.concatenate([q for _, q in protos]).astype(np.int32, copy=False)
    albedo = albedo_rng.uniform(albedo_lo, albedo_hi, size=quads.shape[0]).astype(np.float32)
    s = Scene(verts=np.ascontiguousarray(verts), quads=np.ascontiguousarray(quads),
              proto_vert_off=np.array(vo, dtype=np.int64), proto_quad_off=np.array(qo, dtype=np.int64),
              albedo=albedo, inst_proto=np.ascontiguousarray(inst_proto.astype(np.int32)),
              inst_xform=np.ascontiguousarray(inst_xform.astype(np.float32)))
    s.validate()
    return s


def grid_quads(nx: int, ny: int) -> np.ndarray:
    """Quad indices of an nx x ny grid of (nx+1)(ny+1) vertices laid out row by row."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v0 = j * (nx + 1) + i
    q = np.stack([v0, v0 + 1, v0 + 1 + (nx + 1), v0 + (nx + 1)], axis=-1)
    return q.reshape(-1, 4).astype(np.int32)


def grid_proto(rng: np.random.Generator, nx: int, ny: int, half_x: float, half_y: float,
               z_amp: float) -> Tuple[np.ndarray, np.ndarray]:
    """Height-displaced grid on [-half_x, half_x] x [-half_y, half_y], z ~ U[-z_amp, z_amp]."""
    xs = np.linspace(-half_x, half_x, nx + 1)
    ys = np.linspace(-half_y, half_y, ny + 1)
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    Z = rng.uniform(-z_amp, z_amp, size=X.shape)
    v = np.stack([X, Y, Z], axis=-1).reshape(-1, 3).astype(np.float32)
    return v, grid_quads(nx, ny)


def shell_proto(rng: np.random.Generator, n: int, radius: float, noise: float) -> Tuple[np.ndarray, np.ndarray]:
    """Closed cube-sphere quad shell: 6 n^2 quads, vertices shared along cube edges.

    Every lattice point of the cube surface becomes exactly one vertex, so the
    shell is closed (no cracks by construction).  Quads face outward.
    """
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a = a.ravel()
    b = b.ravel()
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]
    keys = []
    for axis in range(3):
        for side in (0, n):
            u_ax, v_ax = [(1, 2), (2, 0), (0, 1)][axis]
            if side == 0:
                u_ax, v_ax = v_ax, u_ax
            face = []
            for du, dv in corners:
                ijk = np.zeros((a.shape[0], 3), dtype=np.int64)
                ijk[:, axis] = side
                ijk[:, u_ax] = a + du
                ijk[:, v_ax] = b + dv
                face.append(ijk)
            keys.append(np.stack(face, axis=1))  # [n^2, 4, 3]
    ijk = np.concatenate(keys, axis=0)  # [6 n^2, 4, 3]
    m = n + 1
    key = (ijk[..., 0] * m + ijk[..., 1]) * m + ijk[..., 2]
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    quads = inv.reshape(-1, 4).astype(np.int32)
    k = uniq
    ii = k // (m * m)
    jj = (k // m) % m
    kk = k % m
    p = np.stack([ii, jj, kk], axis=-1).astype(np.float64) * (2.0 / n) - 1.0
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    r = radius * (1.0 + rng.uniform(-noise, noise, size=(p.shape[0], 1)))
    return (p * r).astype(np.float32), quads


def shoemake_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed random rotations (Shoemake 1992), [n, 3, 3] float64."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    s1, s2 = np.sqrt(1.0 - u1), np.sqrt(u1)
    x = s1 * np.sin(2 * np.pi * u2)
    y = s1 * np.cos(2 * np.pi * u2)
    z = s2 * np.sin(2 * np.pi * u3)
    w = s2 * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def compose_xforms(R: np.ndarray, scale: np.ndarray, trans: np.ndarray) -> np.ndarray:
    """[A | t] with A = scale * R, row-major 3x4, float32 [n, 12]."""
    A = R * scale[:, None, None]
    X = np.concatenate([A, trans[:, :, None]], axis=2)
    return X.reshape(-1, 12).astype(np.float32)


class FBm:
    """Value-noise fractional Brownian motion height field over [-half, half]^2."""

    def __init__(self, rng: np.random.Generator, half: float, amp: float, octaves: int = 8, base_cells: int = 4):
        self.half = half
        self.amp = amp
        self.lattices = []
        for o in range(octaves):
            r = base_cells * (2 ** o)
            self.lattices.append(rng.uniform(-1.0, 1.0, size=(r + 1, r + 1)))
        self.norm = sum(0.5 ** o for o in range(octaves))

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        h = np.zeros(np.broadcast(x, y).shape)
        for o, lat in enumerate(self.lattices):
            r = lat.shape[0] - 1
            fx = np.clip((x + self.half) / (2 * self.half) * r, 0, r - 1e-9)
            fy = np.clip((y + self.half) / (2 * self.half) * r, 0, r - 1e-9)
            ix = np.floor(fx).astype(np.int64)
            iy = np.floor(fy).astype(np.int64)
            tx = fx - ix
            ty = fy - iy
            tx = tx * tx * (3 - 2 * tx)
            ty = ty * ty * (3 - 2 * ty)
            v00 = lat[iy, ix]
            v10 = lat[iy, ix + 1]
            v01 = lat[iy + 1, ix]
            v11 = lat[iy + 1, ix + 1]
            h += (0.5 ** o) * ((v00 * (1 - tx) + v10 * tx) * (1 - ty) + (v01 * (1 - tx) + v11 * tx) * ty)
        return h * (self.amp / self.norm)


def terrain_proto(fbm: FBm, n: int) -> Tuple[np.ndarray, np.ndarray]:
    """n x n quad height field over [-half, half]^2 (identity-instanced)."""
    xs = np.linspace(-fbm.half, fbm.half, n + 1)
    Y, X = np.meshgrid(xs, xs, indexing="ij")
    Z = fbm(X, Y)
    v = np.stack([X, Y, Z], axis=-1).reshape(-1, 3).astype(np.float32)
    return v, grid_quads(n, n)


# ----------------------------------------------------------------------------
# the configurations
# ----------------------------------------------------------------------------

def light_settings(spp: int, depth: int, seed: int) -> RenderSettings:
    return RenderSettings(spp=spp, depth=depth, seed=seed)


def config1(seed: Optional[int] = None, n_inst: int = 1000, n_protos: int = 16, res: int = 128):
    """16 prototypes of 32x32 quads on [-1,1]^2 (z ~ U[-0.1,0.1]), 1000 instances with
    random rotation, uniform scale in [0.5, 2] and translation in [-50, 50]^3."""
    seed = SEED_BASE + 1 if seed is None else seed
    rng = np.random.default_rng(seed)
    protos = [grid_proto(rng, 32, 32, 1.0, 1.0, 0.1) for _ in range(n_protos)]
    inst_proto = rng.integers(0, n_protos, size=n_inst)
    R = shoemake_rotations(rng, n_inst)
    s = rng.uniform(0.5, 2.0, size=n_inst)
    t = rng.uniform(-50.0, 50.0, size=(n_inst, 3))
    scene = _concat(protos, rng, inst_proto, compose_xforms(R, s, t))
    cams = [Camera((0.0, -160.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 40.0, res, res)]
    return scene, cams, light_settings(1, 3, seed)


def config4(seed: Optional[int] = None):
    """The config-1 scene at 512x512, 4 spp, depth 4 (differentiation workload)."""
    seed = SEED_BASE + 1 if seed is None else seed
    scene, cams, _ = config1(seed, res=512)
    return scene, cams, light_settings(4, 4, SEED_BASE + 4)


def _log_uniform_int(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)).round().astype(np.int64)


def island(seed: int, n_protos: int, n_inst: int, quad_lo: int = 2000, quad_hi: int = 200000,
           terrain_n: int = 2048, half: float = 1000.0, amp: float = 100.0,
           cluster_frac: float = 0.0, n_clusters: int = 0, target_quads: Optional[int] = None,
           progress: Optional[Callable[[str], None]] = None):
    """Prototype zoo instanced over a procedural terrain (configs 2, 3 and 5).

    Half the prototypes are noise-displaced grids with quad aspect U[1, 8] (long
    thin quads), half are closed cube-sphere shells; prototype size is
    log-uniform in [0.2, 20] m.  The terrain is the last prototype, instanced
    once with the identity.  With ``target_quads`` the prototype count grows
    until the unique quad total reaches it.  ``progress`` (optional) receives a
    line every 512 prototypes.
    """
    rng = np.random.default_rng(seed)
    counts = list(_log_uniform_int(rng, quad_lo, quad_hi, n_protos))
    if target_quads is not None:
        while sum(counts) < target_quads:
            counts.extend(_log_uniform_int(rng, quad_lo, quad_hi, 64))
    P = len(counts)
    protos = []
    for p in range(P):
        if progress is not None and p % 512 == 0:
            progress(f"generating prototype {p} of {P}")
        size = math.exp(rng.uniform(math.log(0.2), math.log(20.0)))
        c = int(counts[p])
        if p % 2 == 0:
            aspect = rng.uniform(1.0, 8.0)
            nx = max(1, int(round(math.sqrt(c * aspect))))
            ny = max(1, int(round(c / nx)))
            protos.append(grid_proto(rng, nx, ny, 0.5 * size, 0.5 * size, 0.02 * size))
        else:
            n = max(1, int(round(math.sqrt(c / 6.0))))
            protos.append(shell_proto(rng, n, 0.5 * size, 0.05))
    fbm = FBm(rng, half, amp)
    protos.append(terrain_proto(fbm, terrain_n))
    terrain_id = P
    # instances: uniform over the terrain, optionally a fraction in tight clusters
    n_obj = n_inst - 1
    xy = rng.uniform(-half, half, size=(n_obj, 2))
    if cluster_frac > 0.0 and n_clusters > 0:
        nc = int(round(cluster_frac * n_obj))
        centres = rng.uniform(-half, half, size=(n_clusters, 2))
        which = rng.integers(0, n_clusters, size=nc)
        xy[:nc] = np.clip(centres[which] + rng.normal(0.0, 3.0, size=(nc, 2)), -half, half)
    z = fbm(xy[:, 0], xy[:, 1])
    trans = np.concatenate([xy, z[:, None]], axis=1)
    R = shoemake_rotations(rng, n_obj)
    s = rng.uniform(0.5, 2.0, size=n_obj)
    X = compose_xforms(R, s, trans)
    ident = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], dtype=np.float32)
    inst_xform = np.concatenate([ident, X], axis=0)
    inst_proto = np.concatenate([[terrain_id], rng.integers(0, P, size=n_obj)])
    scene = _concat(protos, rng, inst_proto, inst_xform)
    return scene, fbm


def config2(seed: Optional[int] = None, scale: float = 1.0, res: Tuple[int, int] = (1920, 1080)):
    """256 prototypes (2k-200k quads), 1M instances on a 2 km terrain of 4M quads;
    two views (overview and ground level), 1 spp, depth 8.  ``scale`` shrinks the
    instance and prototype counts for quick tests (1.0 = the full configuration)."""
    seed = SEED_BASE + 2 if seed is None else seed
    n_protos = max(4, int(round(256 * scale)))
    n_inst = max(8, int(round(1_000_000 * scale)))
    terrain_n = 2048 if scale >= 1.0 else max(16, int(2048 * math.sqrt(scale)))
    qhi = 200000 if scale >= 1.0 else max(2000, int(200000 * scale))
    scene, fbm = island(seed, n_protos, n_inst, quad_hi=qhi, terrain_n=terrain_n)
    w, h = res
    g_eye = (-900.0, -900.0, float(fbm(-900.0, -900.0)) + 20.0)
    g_look = (0.0, 0.0, float(fbm(0.0, 0.0)))
    cams = [Camera((0.0, -1500.0, 800.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, w, h),
            Camera(g_eye, g_look, (0.0, 0.0, 1.0), 50.0, w, h)]
    return scene, cams, light_settings(1, 8, seed)


def config3(seed: Optional[int] = None, scale: float = 1.0, clustered: bool = True,
            progress: Optional[Callable[[str], None]] = None):
    """Config-2 generator grown to 20M instances / ~100M unique quads, 30% of the
    instances in tight clusters; 1920x1080 ground view, 4 spp, depth 8."""
    seed = SEED_BASE + 3 if seed is None else seed
    n_inst = max(8, int(round(20_000_000 * scale)))
    target = int(96_000_000 * scale)
    scene, fbm = island(seed, 256, n_inst, target_quads=target,
                        cluster_frac=0.3 if clustered else 0.0, n_clusters=max(1, int(10000 * scale)),
                        progress=progress)
    g_eye = (-900.0, -900.0, float(fbm(-900.0, -900.0)) + 20.0)
    g_look = (0.0, 0.0, float(fbm(0.0, 0.0)))
    cams = [Camera(g_eye, g_look, (0.0, 0.0, 1.0), 50.0, 1920, 1080)]
    return scene, cams, light_settings(4, 8, seed)


def config5_cameras(rng: np.random.Generator, fbm: FBm, n_views: int = 64):
    sides = np.exp(rng.uniform(math.log(64), math.log(1024), size=n_views)).round().astype(int)
    cams = []
    for k in range(n_views):
        ex, ey, lx, ly = rng.uniform(-900, 900, size=4)
        eye = (float(ex), float(ey), float(fbm(ex, ey)) + float(rng.uniform(2, 50)))
        look = (float(lx), float(ly), float(fbm(lx, ly)))
        cams.append(Camera(eye, look, (0.0, 0.0, 1.0), 50.0, int(sides[k]), int(sides[k])))
    return cams


def config5(seed: Optional[int] = None, scale: float = 1.0, progress: Optional[Callable[[str], None]] = None):
    """40M instances, 250M unique quads, 64 square views of side log-uniform in
    [64, 1024], 1 spp, depth 6, all views in one launch."""
    seed = SEED_BASE + 5 if seed is None else seed
    n_inst = max(8, int(round(40_000_000 * scale)))
    target = int(246_000_000 * scale)
    scene, fbm = island(seed, 256, n_inst, target_quads=target,
                        cluster_frac=0.3, n_clusters=max(1, int(20000 * scale)), progress=progress)
    cams = config5_cameras(np.random.default_rng(seed + 1), fbm)
    return scene, cams, light_settings(1, 6, seed)


def make_config(k: int, **kw):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[k](**kw)


# ----------------------------------------------------------------------------
# small scenes for tests and the smoke run
# ----------------------------------------------------------------------------

def tiny_scene(seed: int, n_inst: int = 4, n_protos: int = 2, nq: int = 4, spread: float = 2.0) -> Scene:
    """A few instances of nq x nq displaced grids packed tightly (heavy overlap)."""
    rng = np.random.default_rng(seed)
    protos = [grid_proto(rng, nq, nq, 1.0, 1.0, 0.2) for _ in range(n_protos)]
    inst_proto = rng.integers(0, n_protos, size=n_inst)
    R = shoemake_rotations(rng, n_inst)
    s = rng.uniform(0.5, 2.0, size=n_inst)
    t = rng.uniform(-spread, spread, size=(n_inst, 3))
    return _concat(protos, rng, inst_proto, compose_xforms(R, s, t))


def blade_curves(rng: np.random.Generator, n: int, height: float, radius: float, spread: float) -> np.ndarray:
    """n grass-blade curves rooted on a disk of the given spread: cubic Beziers
    rising to `height` with a random lean, radius tapering from `radius` at the
    root to a tenth of it at the tip: float32 [n, 16]."""
    c = np.zeros((n, 16), np.float64)
    root = np.c_[rng.uniform(-spread, spread, (n, 2)), np.zeros(n)]
    lean = rng.normal(size=(n, 2)) * 0.35 * height
    for k in range(4):
        f = k / 3.0
        c[:, 4 * k + 0] = root[:, 0] + lean[:, 0] * f * f
        c[:, 4 * k + 1] = root[:, 1] + lean[:, 1] * f * f
        c[:, 4 * k + 2] = height * f * rng.uniform(0.8, 1.2, n)
        c[:, 4 * k + 3] = radius * (1.0 - 0.9 * f)
    return c.astype(np.float32)


def curve_scene(seed: int, n_inst: int = 6, n_curves: int = 24, spread: float = 2.5, with_ground: bool = True,
                flat: Tuple[bool, bool] = (False, False)) -> Scene:
    """Tufts of curves (Section 5.2: the scene's curves) instanced over a small
    quad ground: prototype 0 the ground grid (when asked), the others curve
    tufts, each tuft instance rotated about z and scaled uniformly; `flat`
    makes the first or second tuft flat ribbons instead of round curves."""
    rng = np.random.default_rng(seed)
    protos_q = [grid_proto(rng, 6, 6, spread + 1.0, spread + 1.0, 0.05)] if with_ground else []
    tufts = [blade_curves(rng, n_curves, rng.uniform(0.6, 1.2), rng.uniform(0.02, 0.05), 0.4) for _ in range(2)]
    verts = [v for v, _ in protos_q]
    quads = [q for _, q in protos_q]
    vo = np.cumsum([0] + [v.shape[0] for v in verts] + [0] * len(tufts)).astype(np.int64)
    qo = np.cumsum([0] + [q.shape[0] for q in quads] + [0] * len(tufts)).astype(np.int64)
    co = np.cumsum([0] * (len(protos_q) + 1) + [t.shape[0] for t in tufts]).astype(np.int64)
    P = len(protos_q) + len(tufts)
    n_faces = int(qo[-1] + co[-1])
    albedo = rng.uniform(0.2, 0.8, n_faces).astype(np.float32)
    inst_proto = list(range(len(protos_q))) + list(rng.integers(len(protos_q), P, n_inst))
    xf = []
    for k, p in enumerate(inst_proto):
        if p < len(protos_q):
            xf.append([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0])
            continue
        a = rng.uniform(0, 2 * math.pi)
        sc = rng.uniform(0.7, 1.4)
        tx, ty = rng.uniform(-spread, spread, 2)
        ca, sa = math.cos(a) * sc, math.sin(a) * sc
        xf.append([ca, -sa, 0, tx, sa, ca, 0, ty, 0, 0, sc, 0])
    s = Scene(verts=np.concatenate(verts).astype(np.float32) if verts else np.zeros((0, 3), np.float32),
              quads=np.concatenate(quads).astype(np.int32) if quads else np.zeros((0, 4), np.int32),
              proto_vert_off=vo, proto_quad_off=qo, albedo=albedo,
              inst_proto=np.asarray(inst_proto, np.int32), inst_xform=np.asarray(xf, np.float32),
              curves=np.concatenate(tufts).astype(np.float32), proto_curve_off=co,
              proto_curve_flat=np.array([0] * len(protos_q) + [int(f) for f in flat], np.int32))
    s.validate()
    return s


def identity_xform(n: int = 1) -> np.ndarray:
    return np.tile(np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float32), (n, 1))


def single_mesh_scene(verts: np.ndarray, quads: np.ndarray, albedo: Optional[np.ndarray] = None,
                      xforms: Optional[np.ndarray] = None) -> Scene:
    """One prototype, instanced by the given transforms (identity by default)."""
    verts = np.asarray(verts, dtype=np.float32)
    quads = np.asarray(quads, dtype=np.int32)
    if xforms is None:
        xforms = identity_xform(1)
    xforms = np.asarray(xforms, dtype=np.float32).reshape(-1, 12)
    if albedo is None:
        albedo = np.full(quads.shape[0], 0.5, dtype=np.float32)
    s = Scene(verts=verts, quads=quads, proto_vert_off=np.array([0, verts.shape[0]], dtype=np.int64),
              proto_quad_off=np.array([0, quads.shape[0]], dtype=np.int64),
              albedo=np.asarray(albedo, dtype=np.float32),
              inst_proto=np.zeros(xforms.shape[0], dtype=np.int32), inst_xform=xforms)
    s.validate()
    return s


def random_rays(rng: np.random.Generator, n: int, box_lo, box_hi, target_lo, target_hi) -> np.ndarray:
    """Rays from points in one box toward points in another: float32 [n, 8]
    (ox oy oz dx dy dz tmin tmax), tmin = 0, tmax = +inf, d not normalised."""
    o = rng.uniform(box_lo, box_hi, size=(n, 3))
    p = rng.uniform(target_lo, target_hi, size=(n, 3))
    d = p - o
    r = np.zeros((n, 8), dtype=np.float32)
    r[:, 0:3] = o
    r[:, 3:6] = d
    r[:, 6] = 0.0
    r[:, 7] = np.inf
    return r


def camera_arrays(cams: List[Camera]):
    """Packed camera parameters (float64 [n, 10]: eye, look, up, vfov) and int64 [n, 3]
    (w, h, image offset in pixels)."""
    f = np.array([list(c.eye) + list(c.look) + list(c.up) + [c.vfov_deg] for c in cams], dtype=np.float64)
    off = 0
    ii = []
    for c in cams:
        ii.append([c.w, c.h, off])
        off += c.w * c.h
    return f, np.array(ii, dtype=np.int64)
