"""Pins of the oracle's flag predicates and of its acceptance check: what an FP32
answer may legitimately be where the exact answer is within rounding of a
decision.  Each predicate is tied to the property that justifies it, computed
here independently (numpy ray-triangle tests, perturbed rays, closed forms), so
that a dropped term, an inverted inequality or a wrong threshold in the oracle
fails one of these tests."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts

U24 = 2.0 ** -24


def _rays(o, d, tmin=0.0, tmax=np.inf):
    o = np.atleast_2d(np.asarray(o, np.float64))
    d = np.atleast_2d(np.asarray(d, np.float64))
    r = np.zeros((max(o.shape[0], d.shape[0]), 8))
    r[:, 0:3] = o
    r[:, 3:6] = d
    r[:, 6] = tmin
    r[:, 7] = tmax
    return r


def _mt(o, d, a, b, c):
    """Moller-Trumbore, vectorised over rays: (hit, t) against triangle (a, b, c)."""
    e1, e2 = b - a, c - a
    pv = np.cross(d, e2)
    det = pv @ e1
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        tv = o - a
        bu = (tv * pv).sum(1) * inv
        qv = np.cross(tv, e1)
        bv = (d * qv).sum(1) * inv
        tt = (qv @ e2) * inv
    ok = (det != 0) & (bu >= 0) & (bv >= 0) & (bu + bv <= 1)
    return ok, tt


def _world_tris(scene):
    """[(inst, prim, half, a, b, c)] world-space triangles in FP64."""
    out = []
    for i in range(scene.n_instances):
        X = scene.inst_xform[i].astype(np.float64).reshape(3, 4)
        p = scene.inst_proto[i]
        vs = scene.verts[scene.proto_vert_off[p]:scene.proto_vert_off[p + 1]].astype(np.float64)
        W = vs @ X[:, :3].T + X[:, 3]
        for q in range(scene.proto_quad_off[p + 1] - scene.proto_quad_off[p]):
            idx = scene.quads[scene.proto_quad_off[p] + q]
            for half, tri in ((0, (0, 1, 3)), (1, (2, 3, 1))):
                out.append((i, q, half, W[idx[tri[0]]], W[idx[tri[1]]], W[idx[tri[2]]]))
    return out


# --------------------------------------------------------------------- F_T_ILLCOND
def test_t_illcond_matches_t_sensitivity(ora):
    """F_T_ILLCOND marks hits whose t is not determined to 1e-5 relative by the
    positions the FP32 path computes with: moving the ray origin by 16 units of
    2^-24 of the position scale S (the error scale the FP32 transform and leaf
    test accumulate) along the surface normal changes the plane parameter t by
    16 2^-24 S / (|d| |cos|).  The flag must be set exactly when that change
    exceeds 1e-5 t (with a 2 % band around the threshold left out): head-on hits
    near the origin unflagged, grazing or distant ones flagged."""
    quad = ts.axis_quad(-50.0, 50.0, -50.0, 50.0, 0.0)
    scene = ts.multi_mesh_scene([quad])
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(7)
    n = 20000
    # targets on the floor, origins at log-uniform distances and elevations
    tgt = np.stack([rng.uniform(-40, 40, n), rng.uniform(-40, 40, n), np.zeros(n)], 1)
    dist = np.exp(rng.uniform(math.log(0.05), math.log(3000.0), n))
    elev = np.exp(rng.uniform(math.log(1e-4), math.log(math.pi / 2), n))
    az = rng.uniform(0, 2 * math.pi, n)
    dirs = np.stack([np.cos(elev) * np.cos(az), np.cos(elev) * np.sin(az), np.sin(elev)], 1)
    org = tgt + dist[:, None] * dirs
    d = -dirs * rng.uniform(0.3, 3.0, (n, 1))
    r = _rays(org, d).astype(np.float32)
    h = o.trace(r)
    hit = (h.inst >= 0) & ((h.flags & oracle.ID_FLAGS) == 0)
    assert hit.mean() > 0.9
    # sensitivity, computed from the geometry: t of the plane z = 0 for the
    # origin moved by eps along the normal
    r64 = r.astype(np.float64)
    eps = 16 * U24 * h.scale
    t0 = -r64[:, 2] / r64[:, 5]
    t1 = -(r64[:, 2] + eps) / r64[:, 5]
    rel = np.abs(t1 - t0) / np.abs(t0)
    ill = (h.flags & oracle.F_T_ILLCOND) != 0
    clear = hit & (np.abs(rel / 1e-5 - 1.0) > 0.02)
    np.testing.assert_array_equal(ill[clear], rel[clear] > 1e-5)
    # both kinds occur; a head-on hit 10 m away (the quad reaches 50 m from the
    # ray's origin, which sets S) is not flagged, a grazing one is
    assert ill[clear].any() and (~ill[clear]).any()
    hh = o.trace(_rays([[1.0, 2.0, 10.0]], [[0, 0, -1.0]]).astype(np.float32))
    assert hh.inst[0] == 0 and not (hh.flags[0] & oracle.F_T_ILLCOND)
    hg = o.trace(_rays([[-40.0, 2.0, 1e-3]], [[1.0, 0, -1e-4]]).astype(np.float32))
    assert hg.inst[0] == 0 and (hg.flags[0] & oracle.F_T_ILLCOND)


# --------------------------------------------------------------------- F_NEAR_TIE, F_DIAG
def _folded_scene(h):
    """One quad folded along its diagonal: half A in z = 0, v2 lifted to height h."""
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, h], [0, 1, 0]], np.float32)
    return ts.multi_mesh_scene([(v, np.array([[0, 1, 2, 3]], np.int32))])


@pytest.mark.parametrize("h", [0.3, -0.3])
def test_diag_flag_is_both_halves_within_the_window(ora, h):
    """F_DIAG marks rays that hit both halves of the quad they hit with t within
    the tie window (1e-5 t + 1e-6 S / |d|), computed here with numpy: rays
    aimed at points near the fold of a ridge and of a valley, from many
    directions, some exactly on the diagonal."""
    scene = _folded_scene(h)
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(3)
    n = 6000
    s_ = rng.uniform(0.1, 0.9, n)
    off = np.where(rng.random(n) < 0.3, 0.0, rng.normal(0, 1e-5, n) * 10 ** rng.uniform(-2, 2, n))
    tgt = np.stack([s_ + off, 1 - s_ + off, np.zeros(n)], 1)
    dirs = rng.normal(size=(n, 3))
    dirs[:, 2] = np.abs(dirs[:, 2]) * np.sign(rng.uniform(-0.2, 1, n))
    org = tgt + dirs * rng.uniform(0.5, 5, (n, 1))
    r = _rays(org, tgt - org)  # FP64 rays: the targets keep their offsets from the diagonal
    hh = o.trace(r)
    r64 = r
    tris = _world_tris(scene)
    ok_a, t_a = _mt(r64[:, 0:3], r64[:, 3:6], *tris[0][3:])
    ok_b, t_b = _mt(r64[:, 0:3], r64[:, 3:6], *tris[1][3:])
    ok_a &= t_a > 0
    ok_b &= t_b > 0
    t1 = np.minimum(np.where(ok_a, t_a, np.inf), np.where(ok_b, t_b, np.inf))
    dn = np.linalg.norm(r64[:, 3:6], axis=1)
    win = 1e-5 * t1 + 1e-6 * hh.scale / dn
    both = ok_a & ok_b & (np.abs(t_a - t_b) <= win)
    margin = ok_a & ok_b & (np.abs(np.abs(t_a - t_b) / win - 1) < 0.05)
    diag = (hh.flags & oracle.F_DIAG) != 0
    # exactly on the diagonal the FP64 roundings of the two tests decide the
    # shared boundary differently; the predicate is checked off it
    sel = ~margin & (off != 0) & (hh.inst >= 0)
    np.testing.assert_array_equal(diag[sel], both[sel])
    assert both[sel].sum() > 50 and (~both[sel]).sum() > 50


def test_near_tie_flag_is_another_quad_within_the_window(ora):
    """F_NEAR_TIE marks rays for which another (instance, quad) is hit within the
    tie window of the closest hit: two parallel quads at small separations, the
    flag compared with numpy hits of every triangle."""
    rng = np.random.default_rng(5)
    for gap in (0.0, 1e-7, 1e-6, 1e-5, 1e-3):
        q0 = ts.axis_quad(-1, 1, -1, 1, 0.0)
        q1 = ts.axis_quad(-0.5, 1.5, -0.5, 1.5, np.float32(gap))
        scene = ts.multi_mesh_scene([q0, q1])
        o = oracle.OracleScene(scene)
        n = 3000
        tgt = np.stack([rng.uniform(-0.4, 0.9, n), rng.uniform(-0.4, 0.9, n), np.zeros(n)], 1)
        dirs = rng.normal(size=(n, 3))
        dirs[:, 2] = np.abs(dirs[:, 2]) + 0.2
        org = tgt + dirs * rng.uniform(1, 10, (n, 1))
        r = _rays(org, tgt - org).astype(np.float32)
        hh = o.trace(r)
        r64 = r.astype(np.float64)
        ts_ = []
        for (i, q, half, a, b, c) in _world_tris(scene):
            ok, t = _mt(r64[:, 0:3], r64[:, 3:6], a, b, c)
            ts_.append(np.where(ok & (t > 0), t, np.inf))
        ts_ = np.array(ts_).reshape(2, 2, n).min(axis=1)  # per instance
        tb = ts_.min(0)
        other = ts_.max(0)
        dn = np.linalg.norm(r64[:, 3:6], axis=1)
        win = 1e-5 * tb + 1e-6 * hh.scale / dn
        tie = np.isfinite(other) & (other - tb <= win)
        grz = (hh.flags & oracle.F_GRAZE) != 0
        margin = np.abs((other - tb) / win - 1) < 0.05
        sel = np.isfinite(tb) & ~grz & ~margin
        np.testing.assert_array_equal((hh.flags[sel] & oracle.F_NEAR_TIE) != 0, tie[sel])


# --------------------------------------------------------------------- F_GRAZE
def test_unflagged_answers_survive_perturbation(ora):
    """Rays without an identity flag keep their (instance, quad) answer when the
    ray is moved by up to 0.9 of the graze distance (1e-6 S, S the position
    scale), in origin and in direction: the flags cover every ray whose answer
    rounding can change.  Rays aimed at quad edges are flagged."""
    scene = sg.tiny_scene(9, n_inst=4, n_protos=2, nq=3, spread=1.0)
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(17)
    rays = sg.random_rays(rng, 3000, -4, 4, -1.5, 1.5).astype(np.float64)
    h = o.trace(rays)
    clean = (h.flags & oracle.ID_FLAGS) == 0
    assert clean.mean() > 0.9
    dn = np.linalg.norm(rays[:, 3:6], axis=1)
    for k in range(6):
        u = rng.normal(size=(rays.shape[0], 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        v = rng.normal(size=(rays.shape[0], 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        p = rays.copy()
        g = 0.9e-6 * h.scale
        p[:, 0:3] += 0.5 * g[:, None] * u
        # a direction change that moves the far end of the ray by the rest
        far = np.where(np.isfinite(h.t), h.t, 10.0) * dn
        p[:, 3:6] += (0.5 * g / np.maximum(far, 1e-9))[:, None] * dn[:, None] * v
        hp = o.trace(p)
        np.testing.assert_array_equal(hp.inst[clean], h.inst[clean])
        np.testing.assert_array_equal(hp.prim[clean], h.prim[clean])
    # aimed exactly at edge midpoints: flagged, unless something nearer hides the
    # edge (the ray's closest hit lies before it)
    tris = _world_tris(scene)
    tgt = np.array([0.5 * (a + b) for (_, _, _, a, b, c) in tris])
    org = tgt + rng.normal(size=tgt.shape) * 3
    he = o.trace(_rays(org, tgt - org))
    seen = ~(he.t < 1.0 - 1e-6)
    assert seen.sum() > 40
    assert ((he.flags[seen] & oracle.F_GRAZE) != 0).all()
    # the diagonal of a folded quad is a boundary too: the halves leave a sliver
    # (or overlap) along it, so a ray aimed at it may hit either half or neither
    for h_ in (0.3, -0.3):
        fo = oracle.OracleScene(_folded_scene(h_))
        s_ = rng.uniform(0.1, 0.9, 200)
        tg = np.stack([s_, 1 - s_, np.zeros(200)], 1)
        og = tg + np.abs(rng.normal(size=(200, 3))) * 3
        hd = fo.trace(_rays(og, tg - og))
        assert ((hd.flags & oracle.F_GRAZE) != 0).all()


# --------------------------------------------------------------------- F_SHADE thresholds
def _aim(eye, target, w=1, h=1, vfov=1e-6, up=(0.0, 0.0, 1.0)):
    """A camera whose every ray leaves `eye` within 1e-8 rad of the direction to
    `target` (vfov 1e-6 degrees), so a path's first hit is placed at will."""
    return [sg.Camera(tuple(float(x) for x in eye), tuple(float(x) for x in target), up, vfov, w, h)]


def _path_flags(o, cams, st):
    _, _, pf = o.path(cams, st, 0, 0)
    return pf


def test_shade_flag_normal_side_threshold(ora):
    """|n . d| < 1e-3 flags a hit (the side the normal faces is decided within
    rounding): a ray meeting the floor at cos 5e-4 is flagged, at 2e-3 not."""
    scene = ts.floor_scene(albedo=0.5)
    o = oracle.OracleScene(scene)
    st = sg.RenderSettings(spp=1, depth=1, seed=3)
    for c, want in ((5e-4, True), (2e-3, False)):
        dist = 100.0
        eye = (0.0, -dist * math.sqrt(1 - c * c), dist * c)
        pf = _path_flags(o, _aim(eye, (0.0, 0.0, 0.0)), st)
        assert bool(pf & oracle.F_SHADE) == want, (c, pf)


def test_shade_flag_light_side_threshold(ora):
    """|n . w_L| < 1e-6 flags a hit (whether the light is above the surface is
    decided within rounding): a floor lit at cos 1e-7 is flagged, at 1e-5 not."""
    scene = ts.floor_scene(albedo=0.5)
    o = oracle.OracleScene(scene)
    for c, want in ((1e-7, True), (1e-5, False)):
        L = (math.sqrt(1 - c * c), 0.0, c)
        st = sg.RenderSettings(spp=1, depth=1, seed=3, light_dir=L)
        pf = _path_flags(o, _aim((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)), st)
        assert bool(pf & oracle.F_SHADE) == want, (c, pf)


def test_shade_flag_basis_branch_threshold(ora):
    """|n_z| < 1e-6 flags a bounce (the orthonormal basis picks its branch by the
    sign of n_z): a vertical wall is flagged at depth 2, a wall tilted to
    n_z = 1e-4 is not, and neither is flagged at depth 1 (no bounce)."""
    for tilt, depth, want in ((0.0, 2, True), (1e-4, 2, False), (0.0, 1, False)):
        v = np.array([[0, -50, -50 - 50 * tilt], [0, 50, -50 - 50 * tilt], [0, 50, 50 + 50 * tilt],
                      [0, -50, 50 + 50 * tilt]], np.float32)
        # rotate the tilt into x: wall plane x = tilt * z
        v[:, 0] = (tilt * v[:, 2]).astype(np.float32)
        scene = ts.multi_mesh_scene([(v, np.array([[0, 1, 2, 3]], np.int32))])
        o = oracle.OracleScene(scene)
        st = sg.RenderSettings(spp=1, depth=depth, seed=3, light_dir=(-0.6, 0.0, 0.8))
        pf = _path_flags(o, _aim((-10.0, 0.3, 0.2), (0.0, 0.3, 0.2)), st)
        assert bool(pf & oracle.F_SHADE) == want, (tilt, depth, pf)


def test_texel_flag_threshold(ora):
    """A textured hit is flagged when its world distance to an inner texel edge
    is below 1e-5 S / max(|cos|, 1e-3): a head-on hit on a 4 x 4-texel floor
    0.3 of that distance from the edge x = 0 is flagged, 3 times it is not."""
    half = 2.0
    scene = ts.multi_mesh_scene([ts.axis_quad(-half, half, -half, half, 0.0)])
    o = oracle.OracleScene(scene)
    res = 4
    o.set_textures(np.linspace(0.2, 0.8, res * res).reshape(1, res, res))
    st = sg.RenderSettings(spp=1, depth=1, seed=3)
    S = 10.0  # the eye's height is the largest coordinate
    tol = 1e-5 * S
    for dx, want in ((0.3 * tol, True), (3.0 * tol, False)):
        pf = _path_flags(o, _aim((dx, 0.3, S), (dx, 0.3, 0.0), up=(0.0, 1.0, 0.0)), st)
        assert bool(pf & oracle.F_SHADE) == want, (dx, pf)


# --------------------------------------------------------------------- acceptance
def test_acceptance_single_quad_closed_form(ora):
    """An interior hit of an axis-aligned quad: the right (quad, half) at the
    closed-form t is the only acceptable answer; the other half, another quad,
    a miss or a t off by 1e-4 are rejected."""
    scene = ts.multi_mesh_scene([ts.axis_quad(0, 1, 0, 1, 0.0), ts.axis_quad(5, 6, 0, 1, 0.0)])
    o = oracle.OracleScene(scene)
    r = _rays([[0.3, 0.6, 2.0]], [[0.0, 0.0, -1.0]]).astype(np.float32)
    t = np.float32(2.0)

    def acc(inst, prim, half, tt):
        code, info = o.accept(r, [inst], [prim], [tt], half=[half])
        return int(code[0]), int(info[0])

    assert acc(0, 0, 0, t) == (0, 1)                 # x + y < 1: half A, the certain hit
    assert acc(0, 0, 1, t)[0] == 1                   # the other half
    assert acc(1, 0, 0, t)[0] == 1                   # another quad
    assert acc(-1, -1, -1, np.inf)[0] == 2           # a miss
    assert acc(0, 0, 0, np.float32(2.0 * (1 + 1e-4)))[0] == 3
    assert acc(0, 0, 0, np.float32(2.0 * (1 + 2e-6)))[0] == 0
    # an ill-conditioned t (a grazing hit far from the origin) is held to the
    # FP32 bound, 16 units of 2^-24 S / (|d| |cos|), not waived
    rg = _rays([[-399.5, 0.5, 0.04]], [[1.0, 0.0, -1e-4]]).astype(np.float32)
    r64 = rg.astype(np.float64)
    tg = -r64[0, 2] / r64[0, 5]
    hg = o.trace(rg)
    assert hg.inst[0] == 0 and (hg.flags[0] & oracle.F_T_ILLCOND)
    unit = 2.0 ** -24 * hg.scale[0] / abs(r64[0, 5])  # |d| |cos| = |d_z| on the floor
    for k, want in ((0.0, 0), (8.0, 0), (40.0, 3)):
        code, info = o.accept(rg, [0], [0], [np.float32(tg + k * unit)])
        assert code[0] == want and (info[0] & 2), (k, code, info)


def test_acceptance_shared_edge_and_ties(ora):
    """A ray along the edge shared by two quads may report either quad (or, as
    far as this check can tell, neither: watertightness is pinned separately);
    1e-3 inside one quad only that quad; two overlapping coplanar quads at the
    same t accept both; a closer quad excludes a farther one."""
    v = np.array([[-1, -1, 0], [0, -1, 0], [0, 1, 0], [-1, 1, 0], [1, -1, 0], [1, 1, 0]], np.float32)
    qd = np.array([[0, 1, 2, 3], [1, 4, 5, 2]], np.int32)
    strip = ts.multi_mesh_scene([(v, qd)])
    o = oracle.OracleScene(strip)
    r = _rays([[0.0, 0.3, 1.0], [1e-3, 0.3, 1.0]], [[0, 0, -1.0]] * 2).astype(np.float32)
    t = np.float32([1.0, 1.0])
    for prim in (0, 1):
        code, _ = o.accept(r[:1], [0], [prim], t[:1])
        assert code[0] == 0, prim
    code, _ = o.accept(r[:1], [-1], [-1], [np.inf])
    assert code[0] == 0
    code, _ = o.accept(r[1:], [0], [0], t[1:])
    assert code[0] == 1
    code, _ = o.accept(r[1:], [0], [1], t[1:])
    assert code[0] == 0
    code, _ = o.accept(r[1:], [-1], [-1], [np.inf])
    assert code[0] == 2
    # passing 1e-7 outside a quad's outer edge: rounding may report it (or not)
    ro = _rays([[1.0 + 1e-7, 0.3, 1.0], [1.0 + 1e-3, 0.3, 1.0]], [[0, 0, -1.0]] * 2)
    for row, want in ((0, 0), (1, 1)):
        code, _ = o.accept(ro[row:row + 1].astype(np.float32), [0], [1], [np.float32(1.0)])
        assert code[0] == want, row
        code, _ = o.accept(ro[row:row + 1].astype(np.float32), [-1], [-1], [np.inf])
        assert code[0] == 0, row
    # coplanar overlap: both instances acceptable
    quad = ts.axis_quad(-1, 1, -1, 1, 0.0)
    twin = ts.multi_mesh_scene([quad], xforms=sg.identity_xform(2), protos=[0, 0])
    ot = oracle.OracleScene(twin)
    r1 = _rays([[0.3, 0.2, 1.0]], [[0, 0, -1.0]]).astype(np.float32)
    for inst in (0, 1):
        code, info = ot.accept(r1, [inst], [0], [np.float32(1.0)])
        assert code[0] == 0 and (info[0] & 4)
    # stacked quads: the closer one wins, the farther one is not acceptable
    stack = ts.multi_mesh_scene([ts.axis_quad(-1, 1, -1, 1, 0.0), ts.axis_quad(-1, 1, -1, 1, 1.0)])
    os_ = oracle.OracleScene(stack)
    r2 = _rays([[0.3, 0.2, 5.0]], [[0, 0, -1.0]]).astype(np.float32)
    assert os_.accept(r2, [1], [0], [np.float32(4.0)])[0][0] == 0
    assert os_.accept(r2, [0], [0], [np.float32(5.0)])[0][0] == 1
    # ... unless the farther one lies within the tie window (1e-5 t + 1e-6 S / |d|)
    near = ts.multi_mesh_scene([ts.axis_quad(-1, 1, -1, 1, 0.0), ts.axis_quad(-1, 1, -1, 1, 2e-5)])
    on = oracle.OracleScene(near)
    assert on.accept(r2, [0], [0], [np.float32(5.0)])[0][0] == 0
    assert on.accept(r2, [1], [0], [np.float32(5.0 - 2e-5)])[0][0] == 0


def test_acceptance_near_origin_and_any_hit(ora):
    """A ray starting on a quad may or may not report it (FP32 t either side of
    tmin); shadow rays: a certain occluder must be reported, a clear segment
    must not, a grazed occluder may be either."""
    strip = ts.multi_mesh_scene([ts.axis_quad(-1, 1, -1, 1, 0.0), ts.axis_quad(-1, 1, -1, 1, 2.0)])
    o = oracle.OracleScene(strip)
    r = _rays([[0.3, 0.2, 1e-9]], [[0.0, 0.0, 1.0]]).astype(np.float32)
    assert o.accept(r, [0], [0], [np.float32(1e-9)])[0][0] == 0     # the quad it starts on
    assert o.accept(r, [1], [0], [np.float32(2.0)])[0][0] == 0      # the next one up
    r_sh = _rays([[0.3, 0.2, 1.0], [0.3, 0.2, 1.0], [1.0, 0.2, 1.0]],
                 [[0, 0, 1.0], [0, 0, -1.0], [0, 0, 1.0]]).astype(np.float32)
    r_sh[1, 7] = 0.5  # segment ending above the floor
    occ = np.array([1, 0, 1], np.int32)
    code, _ = o.accept(r_sh, occ, any_hit=True)
    assert list(code) == [0, 0, 0]
    code, _ = o.accept(r_sh, 1 - occ, any_hit=True)
    assert list(code) == [2, 1, 0]  # the third ray grazes the occluder's edge: either is acceptable


def test_acceptance_accepts_the_oracle_answer_and_rejects_wrong_ones(ora):
    """Over random rays in a heavily overlapping scene, the oracle's own closest
    hit (half included) is always acceptable; answering with the second-closest
    (instance, quad) is rejected unless it lies within the tie window; answering
    a miss is rejected whenever the oracle's hit is unflagged."""
    scene = sg.tiny_scene(9, n_inst=4, n_protos=2, nq=4, spread=1.0)
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(23)
    rays = sg.random_rays(rng, 4000, -4, 4, -1.5, 1.5)
    h = o.trace(rays)
    code, info = o.accept(rays, h.inst, h.prim, h.t.astype(np.float32), half=h.half)
    assert (code == 0).all(), np.unique(code, return_counts=True)
    clean = (h.flags & oracle.ID_FLAGS) == 0
    assert (info[clean & (h.inst >= 0)] & 1).all()  # an unflagged hit is the certain one
    miss_code, _ = o.accept(rays, np.full(rays.shape[0], -1), np.full(rays.shape[0], -1),
                            np.full(rays.shape[0], np.inf, np.float32))
    assert (miss_code[clean & (h.inst >= 0)] == 2).all()
    # second-closest distinct quad, from numpy hits of every triangle
    r64 = rays.astype(np.float64)
    T, K = [], []
    for (i, q, half, a, b, c) in _world_tris(scene):
        ok, t = _mt(r64[:, 0:3], r64[:, 3:6], a, b, c)
        T.append(np.where(ok & (t > 0), t, np.inf))
        K.append((i, q, half))
    T = np.array(T)
    order = np.argsort(T, axis=0)
    n_rej = 0
    for j in np.nonzero(clean & (h.inst >= 0))[0][:1500]:
        first = K[order[0, j]]
        for k in order[1:, j]:
            if not np.isfinite(T[k, j]):
                break
            i2, q2, h2 = K[k]
            if (i2, q2) != first[:2]:
                c2, _ = o.accept(rays[j:j + 1], [i2], [q2], [np.float32(T[k, j])], half=[h2])
                assert c2[0] == 1, (j, K[k], T[k, j], h.t[j])
                n_rej += 1
                break
    assert n_rej > 200


# --------------------------------------------------------------------- path replay check
def _u01(w):
    return float(int(w) >> 8) * 2.0 ** -24


def _model_path(o, scene, tris, cam, st, pix, sample):
    """A path built here the way an FP32 renderer builds it: each ray is traced
    by the oracle's closest hit (the ray's own FP32 values, the previous triangle
    excluded), the hit point is o + t d rounded to FP32 per operation, the next
    direction is the cosine sample about the hit triangle's normal (numpy),
    rounded to FP32.  Returns the record in rtq_render_path's layout."""
    f32 = np.float32
    key = (st.seed & 0xFFFFFFFF, (st.seed >> 32) ^ st.frame)
    eye = np.array(cam.eye, np.float64)
    fw = np.array(cam.look, np.float64) - eye
    fw /= np.linalg.norm(fw)
    rt = np.cross(fw, cam.up)
    rt /= np.linalg.norm(rt)
    up = np.cross(rt, fw)
    th = math.tan(math.radians(cam.vfov_deg) / 2)
    w = oracle.philox([pix, sample, 0, 0], key)
    x, y = pix % cam.w, pix // cam.w
    sx = (2 * (x + _u01(w[0])) / cam.w - 1) * th * cam.w / cam.h
    sy = (1 - 2 * (y + _u01(w[1])) / cam.h) * th
    d = fw + sx * rt + sy * up
    d /= np.linalg.norm(d)
    ray_o, ray_d = eye.astype(f32), d.astype(f32)
    L = np.array(st.light_dir)
    vi, vf = [], []
    excl = None
    beta, rad = 1.0, 0.0
    for b in range(st.depth):
        r = np.zeros((1, 8), np.float32)
        r[0, 0:3], r[0, 3:6], r[0, 7] = ray_o, ray_d, np.inf
        hh = o.trace(r, excl=None if excl is None else np.array([excl], np.int32))
        rec_f = [np.inf, 0, 0, 0, *ray_o, *ray_d]
        if hh.inst[0] < 0:
            rad += beta * st.L_sky
            vi.append([-1, -1, -1, -1, -1, 0])
            vf.append(rec_f)
            return len(vi) - 1, np.array(vi), np.array(vf, np.float32), True, f32(rad)
        key3 = (int(hh.inst[0]), int(hh.prim[0]), int(hh.half[0]))
        a_, b_, c_ = tris[key3]
        n = np.cross(b_ - a_, c_ - a_)
        n /= np.linalg.norm(n)
        if n @ ray_d.astype(np.float64) > 0:
            n = -n
        t32 = f32(hh.t[0])
        p = np.array([f32(f32(ray_o[k]) + f32(t32 * ray_d[k])) for k in range(3)], np.float32)
        face = int(scene.proto_quad_off[scene.inst_proto[key3[0]]] + key3[1])
        alb = float(scene.albedo[face])
        cl = float(n @ L)
        shadow = -1
        if cl > 0:
            rs = np.zeros((1, 8), np.float32)
            rs[0, 0:3], rs[0, 3:6], rs[0, 7] = p, np.array(L, np.float32), np.inf
            occ = o.trace(rs, excl=np.array([key3], np.int32), any_hit=True)
            shadow = 1 if occ.inst[0] >= 0 else 0
            if shadow == 0:
                rad += beta * alb * (st.E / math.pi) * cl
        vi.append([key3[0], key3[1], key3[2], shadow, face, 0])
        rec_f[0], rec_f[1], rec_f[2], rec_f[3] = t32, alb, cl, rad
        vf.append(rec_f)
        if b == st.depth - 1:
            break
        w2 = oracle.philox([pix, sample, 0, b], key)
        u1, u2 = _u01(w2[2]), _u01(w2[3])
        sg_ = 1.0 if n[2] >= 0 else -1.0
        aa = -1.0 / (sg_ + n[2])
        bb = n[0] * n[1] * aa
        t1 = np.array([1 + sg_ * n[0] ** 2 * aa, sg_ * bb, -sg_ * n[0]])
        t2 = np.array([bb, sg_ + n[1] ** 2 * aa, -n[1]])
        dn = (math.sqrt(u1) * math.cos(2 * math.pi * u2)) * t1 + (math.sqrt(u1) * math.sin(2 * math.pi * u2)) * t2 \
            + math.sqrt(1 - u1) * n
        ray_o, ray_d = p, dn.astype(np.float32)
        beta *= alb
        excl = key3
    return len(vi), np.array(vi), np.array(vf, np.float32), False, f32(rad)


def test_path_check_accepts_model_paths_and_rejects_mistakes(ora):
    """The replay check accepts paths an FP32 renderer builds step by step (here:
    a numpy model on top of the oracle's ray queries), and rejects each planted
    mistake with the check it violates: another quad, a flipped shadow outcome,
    a wrong albedo, a moved origin, a turned direction, a dropped vertex, a wrong
    radiance."""
    scene = sg.tiny_scene(21, n_inst=24, n_protos=3, nq=8, spread=3.0)
    cams = [sg.Camera((0.0, -12.0, 2.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 45.0, 37, 23)]
    st = sg.RenderSettings(spp=1, depth=3, seed=77, frame=2)
    o = oracle.OracleScene(scene)
    tris = {(i, q, h): (a, b, c) for (i, q, h, a, b, c) in _world_tris(scene)}
    cam = cams[0]
    rng = np.random.default_rng(2)
    n_ok = n_vert = 0
    muts = {k: 0 for k in ("prim", "shadow", "albedo", "origin", "direction", "length", "radiance")}
    for pix in rng.choice(cam.w * cam.h, 300, replace=False):
        nv, vi, vf, esc, rad = _model_path(o, scene, tris, cam, st, int(pix), 0)
        code, stats = o.check_path(cams, st, 0, int(pix), 0, nv, vi, vf, esc, rad)
        assert code == 0, (pix, oracle.PATH_CODES.get(code), stats, vi, vf)
        n_ok += 1
        n_vert += stats["vertices"]
        if nv == 0:
            continue
        m = vi.copy()
        m[0, 1] = (m[0, 1] + 1) % 64
        m[0, 4] = vi[0, 4] - vi[0, 1] + m[0, 1]
        muts["prim"] += o.check_path(cams, st, 0, int(pix), 0, nv, m, vf, esc, rad)[0] == 2
        if vi[0, 3] >= 0:
            m = vi.copy()
            m[0, 3] = 1 - vi[0, 3]
            c = o.check_path(cams, st, 0, int(pix), 0, nv, m, vf, esc, rad)[0]
            muts["shadow"] += c in (8, 12)
        f = vf.copy()
        f[0, 1] = np.float32(vf[0, 1] * 1.01)
        muts["albedo"] += o.check_path(cams, st, 0, int(pix), 0, nv, vi, f, esc, rad)[0] == 6
        if vf.shape[0] > 1:
            f = vf.copy()
            f[1, 4] = np.nextafter(vf[1, 4], np.float32(np.inf))
            muts["origin"] += o.check_path(cams, st, 0, int(pix), 0, nv, vi, f, esc, rad)[0] == 9
            f = vf.copy()
            f[1, 7:10] = (vf[1, 7:10] + np.float32(1e-3) * rng.normal(size=3)).astype(np.float32)
            c = o.check_path(cams, st, 0, int(pix), 0, nv, vi, f, esc, rad)[0]
            muts["direction"] += c == 10
        if not esc:
            muts["length"] += o.check_path(cams, st, 0, int(pix), 0, nv - 1, vi, vf, esc, rad)[0] == 11
        muts["radiance"] += o.check_path(cams, st, 0, int(pix), 0, nv, vi, vf, esc, np.float32(rad * 1.001 + 1e-3))[0] == 12
    assert n_ok == 300 and n_vert > 100, n_vert
    assert all(v >= 10 for v in muts.values()), muts
