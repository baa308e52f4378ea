"""Pins of the oracle's curves (Section 5.2 "Curves": cubic Bezier curves with
a radius, rendered as chains of capsules) against closed forms, brute force
and invariants."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg

K = 8  # capsules per curve


def _curve_scene(curves, xforms=None, albedo=0.5, flat=False):
    """Curve prototype(s) only: one prototype holding `curves` [n, 16], round
    capsule chains or (flat) ray-facing ribbons."""
    curves = np.asarray(curves, np.float32).reshape(-1, 16)
    if xforms is None:
        xforms = sg.identity_xform(1)
    xforms = np.asarray(xforms, np.float32).reshape(-1, 12)
    s = sg.Scene(verts=np.zeros((0, 3), np.float32), quads=np.zeros((0, 4), np.int32),
                 proto_vert_off=np.array([0, 0], np.int64), proto_quad_off=np.array([0, 0], np.int64),
                 albedo=np.full(curves.shape[0], albedo, np.float32),
                 inst_proto=np.zeros(xforms.shape[0], np.int32), inst_xform=xforms, curves=curves,
                 proto_curve_off=np.array([0, curves.shape[0]], np.int64),
                 proto_curve_flat=np.array([1 if flat else 0], np.int32))
    s.validate()
    return s


def _straight(x0=-2.0, x1=2.0, r=0.25, y=0.0, z=0.0):
    """A straight curve along x with evenly spaced control points and a
    constant radius (the Bezier is then linear in its parameter)."""
    xs = np.linspace(x0, x1, 4)
    return [v for x in xs for v in (x, y, z, r)]


def _rays(o, d):
    o = np.atleast_2d(np.asarray(o, np.float64))
    d = np.atleast_2d(np.asarray(d, np.float64))
    r = np.zeros((o.shape[0], 8), np.float64)
    r[:, 0:3] = o
    r[:, 3:6] = d
    r[:, 7] = np.inf
    return r


def test_tessellation_points_lie_on_the_bezier():
    """Capsule ends are the Bezier's points at j / 8 (rounded to FP32): for a
    straight curve with evenly spaced control points they are evenly spaced on
    the line; for the standard cubic approximation of a quarter circle (handle
    length 0.5523 R) they lie within its known radial error (2.7e-4 R) of the
    circle; the curve's ends are the end control points exactly."""
    o = oracle.OracleScene(_curve_scene(_straight()))
    c = o.capsules()
    assert c.shape == (K, 8)
    xs = np.concatenate([c[:, 0], c[-1:, 3]])
    np.testing.assert_allclose(xs, np.linspace(-2, 2, K + 1), atol=1e-6)
    assert (c[:, 6] == np.float32(0.25)).all()
    R, h = 3.0, 0.5523 * 3.0
    arc = [R, 0, 0, 0.1, R, h, 0, 0.1, h, R, 0, 0.1, 0, R, 0, 0.1]
    c = oracle.OracleScene(_curve_scene(arc)).capsules()
    pts = np.concatenate([c[:, 0:3], c[-1:, 3:6]])
    rad = np.linalg.norm(pts[:, :2], axis=1)
    assert (np.abs(rad - R) < 2.8e-4 * R + 1e-6).all(), rad - R
    assert tuple(pts[0]) == (R, 0, 0) and tuple(pts[-1]) == (0, R, 0)
    # radii: the FP32 mean of the radius at the ends; a tapered curve decreases
    taper = [0, 0, 0, 0.4, 1, 0, 0, 0.3, 2, 0, 0, 0.2, 3, 0, 0, 0.1]
    cr = oracle.OracleScene(_curve_scene(taper)).capsules()[:, 6]
    # radii 0.4 .. 0.1 at evenly spaced control points: r(s) = 0.4 - 0.3 s, so
    # the first capsule's radius is the mean of r(0) and r(1/8), 0.38125
    assert (np.diff(cr) < 0).all() and abs(cr[0] - 0.38125) < 1e-7


def test_capsule_closed_forms():
    """Straight curve of radius r along x: a ray toward the axis at offset h
    meets the body at t = D - sqrt(r^2 - h^2); a ray along the axis meets the
    end sphere at D - r; a ray passing at h > r misses; a ray starting inside
    the capsule does not hit it (capsules are entered from outside only), also
    when it runs along the axis toward the last capsule's end sphere."""
    r = 0.25
    o = oracle.OracleScene(_curve_scene(_straight(r=r)))
    hs = np.array([0.0, 0.1, 0.2, 0.249])
    rays = _rays([[0.3, h, 5.0] for h in hs], [[0, 0, -1.0]] * len(hs))
    out = o.trace(rays)
    expect = 5.0 - np.sqrt(r * r - hs ** 2)
    np.testing.assert_allclose(out.t, expect, rtol=1e-12)
    assert (out.inst == 0).all() and (out.half == 0).all()
    # the hit capsule is the one covering x = 0.3 (each spans 0.5 along x)
    assert (out.prim == int((0.3 + 2.0) / 0.5)).all()
    end = o.trace(_rays([[-6.0, 0.05, 0.0]], [[1.0, 0, 0]]))
    np.testing.assert_allclose(end.t, [-2.0 - math.sqrt(r * r - 0.05 ** 2) + 6.0], rtol=1e-12)
    assert end.prim[0] == 0
    miss = o.trace(_rays([[0.3, 0.26, 5.0], [0.3, 0.0, 0.1]], [[0, 0, -1.0], [0, 0, 1.0]]))
    assert (miss.inst == -1).all() and np.isinf(miss.t).all()
    # a ray along +z from the axis point at x = 0.3: inside capsule 4 and
    # nowhere else near it
    inside = o.trace(_rays([[0.3, 0.0, 0.0], [1.7, 0.0, 0.0], [1.7, 0.1, 0.0]],
                           [[0, 0, 1.0], [1.0, 0, 0], [1.0, 0.0, 0.0]]))
    assert (inside.inst == -1).all()


@pytest.mark.parametrize("flat", [False, True])
def test_curve_bvh_equals_brute_force_and_instances(flat):
    """Over a tuft scene with ground (one tuft prototype of flat ribbons when
    asked), the BVH traversal equals brute force bit for bit (flags
    included); an instanced straight curve's hits equal the prototype's hits
    under the FP64 inverse transform."""
    scene = sg.curve_scene(3, flat=(False, flat))
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(5)
    rays = sg.random_rays(rng, 4000, [-3, -3, 0.05], [3, 3, 1.5], [-3, -3, 0.0], [3, 3, 1.2])
    a, b = o.trace(rays), o.trace(rays, brute=True)
    for f in ("t", "inst", "prim", "half", "flags"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    cap_hits = (a.inst >= 1).sum()
    assert cap_hits > 200, cap_hits
    # instance invariance: rotation about z by 30 degrees, scale 1.5, translation
    c, s_ = math.cos(math.pi / 6) * 1.5, math.sin(math.pi / 6) * 1.5
    X = np.array([[c, -s_, 0, 1.0, s_, c, 0, -2.0, 0, 0, 1.5, 0.5]], np.float32)
    o1 = oracle.OracleScene(_curve_scene(_straight(), xforms=X, flat=flat))
    o0 = oracle.OracleScene(_curve_scene(_straight(), flat=flat))
    A = X.reshape(3, 4).astype(np.float64)
    Ainv = np.linalg.inv(A[:, :3])
    rw = sg.random_rays(rng, 2000, [-4, -5, -2], [6, 2, 3], [-1, -4, 0], [3, 0, 1])
    ro = rw.astype(np.float64).copy()
    ro[:, 0:3] = (rw[:, 0:3].astype(np.float64) - A[:, 3]) @ Ainv.T
    ro[:, 3:6] = rw[:, 3:6].astype(np.float64) @ Ainv.T
    hw, h0 = o1.trace(rw), o0.trace(ro)
    assert np.array_equal(hw.inst, h0.inst) and (hw.inst >= 0).sum() > 100
    m = hw.inst >= 0
    np.testing.assert_allclose(hw.t[m], h0.t[m], rtol=1e-12)


def test_curve_flags():
    """A ray passing the capsule's surface within the graze distance is
    flagged GRAZE; rays through the body, head-on or at a shallow angle, are
    not flagged; a ray starting on the surface is flagged NEAR_ORIGIN."""
    r = 0.25
    o = oracle.OracleScene(_curve_scene(_straight(r=r)))
    rays = _rays([[0.3, r * (1 + 1e-9), 5.0], [0.3, r * (1 - 1e-9), 5.0], [0.3, 0.0, 5.0],
                  [0.3, 0.0, r]], [[0, 0, -1.0], [0, 0, -1.0], [0, 0, -1.0], [0, 1.0, 1.0]])
    out = o.trace(rays)
    assert out.flags[0] & oracle.F_GRAZE and out.flags[1] & oracle.F_GRAZE
    assert out.flags[2] == 0 and out.inst[2] == 0
    assert out.flags[3] & oracle.F_NEAR_ORIGIN
    # a ray nearly parallel to the axis enters the body at a shallow angle
    # (cos 0.02) and passes far from the surface afterwards: not a graze
    shallow = o.trace(_rays([[-1.3, 0.0, r + 0.01]], [[1.0, 0.0, -0.02]]))
    assert shallow.inst[0] == 0 and shallow.prim[0] == 2 and (shallow.flags[0] & oracle.ID_FLAGS) == 0
    np.testing.assert_allclose(shallow.t, [0.5], rtol=1e-12)
    # the acceptance check: the grazing ray may hit or miss, the central ray must hit
    code, info = o.accept(rays[:3].astype(np.float32), np.array([-1, 0, -1]), np.array([-1, 4, -1]),
                          np.array([np.inf, out.t[1], np.inf], np.float32))
    assert code[0] == 0 and code[1] == 0 and code[2] == 2


def test_curve_sky_closed_form():
    """A curve floating under the constant sky, no sun, depth 2: a convex
    capsule never sees itself, so every camera sample that hits a capsule
    carries a L_sky and every other one L_sky; a pixel of two samples is one
    of L_sky, (1 + a) L_sky / 2 and a L_sky."""
    a = float(np.float32(0.6))
    o = oracle.OracleScene(_curve_scene(_straight(r=0.3), albedo=a))
    cams = [sg.Camera((0.0, -6.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 40.0, 32, 24)]
    st = sg.RenderSettings(spp=2, depth=2, seed=3)
    st.E = 0.0
    img, _, _ = o.render(cams, st)
    L = st.L_sky
    k = np.rint((L - img) / ((1.0 - a) * L / 2)).astype(int)  # samples on a capsule
    assert set(np.unique(k)) <= {0, 1, 2} and (k == 2).sum() > 50 and (k == 1).sum() > 0
    np.testing.assert_allclose(img, ((2 - k) * L + k * a * L) / 2, rtol=1e-12)


@pytest.mark.parametrize("flat", [False, True])
def test_curve_gradient_forms_agree(flat):
    """Curves are faces of their own (one albedo per curve): PRB = dual
    numbers = central differences on a tuft scene with ground."""
    scene = sg.curve_scene(4, n_inst=4, n_curves=12, flat=(flat, False))
    o = oracle.OracleScene(scene)
    cams = [sg.Camera((0.0, -6.0, 1.5), (0.0, 0.0, 0.4), (0.0, 0.0, 1.0), 45.0, 24, 24)]
    st = sg.RenderSettings(spp=2, depth=3, seed=5)
    rng = np.random.default_rng(2)
    alb = scene.albedo.astype(np.float64)
    o.set_albedo(alb + rng.uniform(-0.1, 0.1, alb.shape))
    T, _, _ = o.render(cams, st)
    o.set_albedo(alb)
    I, _, _ = o.render(cams, st)
    gp = 2 * (I - T) / I.size
    g, _, _ = o.grad(cams, st, gp)
    nq = scene.n_quads
    assert np.abs(g[nq:]).max() > 0, "no curve face has a gradient"
    e = rng.normal(size=alb.shape)
    dI, _ = o.tangent(cams, st, e)
    assert abs((g * e).sum() - (gp * dI).sum()) <= 1e-10 * abs((gp * dI).sum())

    def loss(x):
        o.set_albedo(x)
        Ix, _, _ = o.render(cams, st)
        return ((Ix - T) ** 2).sum() / I.size

    h = 1e-5
    f = nq + int(np.argmax(np.abs(g[nq:])))
    ef = np.zeros_like(alb)
    ef[f] = 1.0
    fd = (loss(alb + h * ef) - loss(alb - h * ef)) / (2 * h)
    assert abs(fd - g[f]) <= 1e-6 * abs(g[f])


def test_curve_scene_rejects_textures():
    o = oracle.OracleScene(sg.curve_scene(1))
    with pytest.raises(AssertionError):
        o.set_textures(np.zeros((o.n_quads, 2, 2), np.float32))


@pytest.mark.parametrize("turned", [False, True])
def test_curve_sun_shading_closed_form(turned):
    """A straight curve along x seen from high above, the sun overhead: a
    sample on the capsule carries a L_sky + a E cos / pi with cos the z part of
    the outward normal, so cos lies in (0, 1] and its mean over the footprint is
    the area-weighted mean of sqrt(1 - (y / r)^2) over the body (pi / 4) and of
    n_z over the two end half-disks (2 / 3).  Turned: the same curve built
    along y and placed by a quarter turn about x and one about y, so the world
    normal depends on the instance transform."""
    a, r, L = float(np.float32(0.5)), 0.3, 0.25
    if turned:
        # object y -> world x: a quarter turn about x (y -> z), then about y (z -> x)
        proto = [v for y in np.linspace(-2, 2, 4) for v in (0.0, y, 0.0, r)]
        Rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float64)
        Ry = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], np.float64)
        M = Ry @ Rx
        assert np.allclose(M @ [0, 1, 0], [1, 0, 0])
        X = np.concatenate([M, np.zeros((3, 1))], axis=1).reshape(1, 12)
        o = oracle.OracleScene(_curve_scene(proto, xforms=X, albedo=a))
    else:
        o = oracle.OracleScene(_curve_scene(_straight(r=r), albedo=a))
    # far away with a narrow field, so the camera rays are nearly parallel
    cams = [sg.Camera((0.0, 0.0, 200.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 1.5, 128, 128)]
    st = sg.RenderSettings(spp=1, depth=2, seed=9, light_dir=(0.0, 0.0, 1.0), E=math.pi, L_sky=L)
    img, fl, _ = o.render(cams, st)
    hit = np.abs(img - L) > 1e-9
    cos = (img[hit] - a * L) / a
    assert hit.sum() > 1000 and (cos > 0).all() and (cos <= 1 + 1e-12).all()
    body, disks = 4.0 * 2 * r, math.pi * r * r
    expect = (body * math.pi / 4 + disks * 2 / 3) / (body + disks)
    # 1600 samples: the mean's standard error is about 0.003
    assert abs(cos.mean() - expect) < 0.009, (cos.mean(), expect)


def _u01(w):
    return float(int(w) >> 8) * 2.0 ** -24


def _curve_model_path(o, scene, caps, cam, st, pix, sample, turn=0.0, rng=None):
    """A path over a scene with curves built the way an FP32 renderer builds
    it: rays traced by the oracle's closest hit (the previous primitive
    excluded), hit points o + t d rounded to FP32 per operation, a capsule's
    normal formed from the hit point relative to the instance origin through
    the FP32-rounded inverse transform, a quad's from its vertices, the next
    direction the cosine sample about the normal (rounded to FP32).  turn > 0
    turns every capsule normal by that angle about a random tangent first.
    Returns the record in rtq_render_path's layout."""
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
    fo = scene.proto_face_off()
    curve_proto = np.diff(scene.proto_curve_off) > 0
    flat_proto = (scene.proto_curve_flat if scene.proto_curve_flat is not None
                  else np.zeros(scene.n_protos, np.int32)) != 0
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
        inst, prim, half = int(hh.inst[0]), int(hh.prim[0]), int(hh.half[0])
        p_ = scene.inst_proto[inst]
        X = scene.inst_xform[inst].astype(np.float64).reshape(3, 4)
        t32 = f32(hh.t[0])
        if curve_proto[p_] and flat_proto[p_]:
            # a ribbon faces the ray: the reverse object-space direction without
            # its part along the segment
            c = caps[8 * scene.proto_curve_off[p_] + prim]
            Ai = np.linalg.inv(X[:, :3]).astype(np.float32).astype(np.float64)
            do = Ai @ ray_d.astype(np.float64)
            T = c[3:6] - c[0:3]
            no = -(do - (do @ T) / (T @ T) * T)
            n = Ai.T @ no.astype(np.float32).astype(np.float64)
            face = int(fo[p_] + prim // 8)
        elif curve_proto[p_]:
            c = caps[8 * scene.proto_curve_off[p_] + prim]
            Ai = np.linalg.inv(X[:, :3]).astype(np.float32).astype(np.float64)
            h = (ray_o.astype(np.float64) - X[:, 3].astype(np.float32)) + float(t32) * ray_d.astype(np.float64)
            ho = Ai @ h
            ba = c[3:6] - c[0:3]
            s_ = np.clip((ho - c[0:3]) @ ba / (ba @ ba), 0, 1)
            no = (ho - (c[0:3] + s_ * ba)).astype(np.float32).astype(np.float64)
            n = Ai.T @ no
            face = int(fo[p_] + prim // 8)
        else:
            q = scene.quads[scene.proto_quad_off[p_] + prim] + scene.proto_vert_off[p_]
            V = scene.verts[q].astype(np.float64) @ X[:, :3].T + X[:, 3]
            n = np.cross(V[1] - V[0], V[3] - V[0]) if half == 0 else np.cross(V[3] - V[2], V[1] - V[2])
            face = int(fo[p_] + prim)
        n /= np.linalg.norm(n)
        if n @ ray_d.astype(np.float64) > 0:
            n = -n
        if turn > 0 and curve_proto[p_]:
            tv = np.cross(n, rng.normal(size=3))
            tv /= np.linalg.norm(tv)
            n = math.cos(turn) * n + math.sin(turn) * tv
        p = np.array([f32(f32(ray_o[k]) + f32(t32 * ray_d[k])) for k in range(3)], np.float32)
        alb = float(scene.albedo[face])
        cl = float(n @ L)
        shadow = -1
        key3 = (inst, prim, half)
        if cl > 0:
            rs = np.zeros((1, 8), np.float32)
            rs[0, 0:3], rs[0, 3:6], rs[0, 7] = p, np.array(L, np.float32), np.inf
            occ = o.trace(rs, excl=np.array([key3], np.int32), any_hit=True)
            shadow = 1 if occ.inst[0] >= 0 else 0
            if shadow == 0:
                rad += beta * alb * (st.E / math.pi) * cl
        vi.append([inst, prim, half, shadow, face, 0])
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


@pytest.mark.parametrize("flat", [False, True])
def test_path_check_on_curves(flat):
    """The replay check accepts paths over curves whose normals carry an FP32
    renderer's rounding (through the FP32 inverse transform), and rejects
    paths whose curve normals are turned by 0.05 rad, and a wrong radiance;
    with flat ribbons (one tuft prototype) as well."""
    scene = sg.curve_scene(4, n_inst=8, n_curves=24, flat=(flat, flat))
    o = oracle.OracleScene(scene)
    caps = o.capsules()
    cams = [sg.Camera((0.0, -5.5, 1.4), (0.0, 0.0, 0.4), (0.0, 0.0, 1.0), 45.0, 48, 40)]
    st = sg.RenderSettings(spp=1, depth=3, seed=17, frame=1)
    cam = cams[0]
    rng = np.random.default_rng(3)
    curve_proto = np.diff(scene.proto_curve_off) > 0
    n_ok = n_cap = n_turn = n_rad = 0
    for pix in rng.choice(cam.w * cam.h, 400, replace=False):
        nv, vi, vf, esc, rad = _curve_model_path(o, scene, caps, cam, st, int(pix), 0)
        code, stats = o.check_path(cams, st, 0, int(pix), 0, nv, vi, vf, esc, rad)
        assert code == 0, (pix, oracle.PATH_CODES.get(code), stats, vi, vf)
        n_ok += 1
        on_cap = [k for k in range(nv) if curve_proto[scene.inst_proto[vi[k, 0]]]]
        if not on_cap or on_cap[0] == nv - 1:
            continue
        n_cap += 1
        nv2, vi2, vf2, esc2, rad2 = _curve_model_path(o, scene, caps, cam, st, int(pix), 0, turn=0.05,
                                                      rng=np.random.default_rng(int(pix)))
        c = o.check_path(cams, st, 0, int(pix), 0, nv2, vi2, vf2, esc2, rad2)[0]
        n_turn += c != 0
        n_rad += o.check_path(cams, st, 0, int(pix), 0, nv, vi, vf, esc, np.float32(rad * 1.01 + 1e-3))[0] == 12
    assert n_ok == 400 and n_cap > 30, n_cap
    assert n_turn == n_cap and n_rad == n_cap, (n_turn, n_rad, n_cap)


def test_ribbon_closed_forms():
    """A flat ribbon faces the ray: a ray toward a straight ribbon of radius r
    along x meets it at the depth of the axis point closest to the ray's line
    whenever the line passes within r of the axis (t = D for a ray straight
    down from height D at any offset h < r; t = 5 for a ray crossing the axis
    5 units away at 53 degrees), and misses beyond r; a ray along the axis
    meets the first segment at its start; a tapered ribbon's half-width at a
    segment end is that end's radius."""
    r = 0.25
    o = oracle.OracleScene(_curve_scene(_straight(r=r), flat=True))
    c = o.capsules()
    assert (c[:, 6] == np.float32(r)).all() and (c[:, 7] == np.float32(r)).all()
    hs = np.array([0.0, 0.1, 0.2, 0.249, -0.249])
    out = o.trace(_rays([[0.3, h, 5.0] for h in hs], [[0, 0, -1.0]] * len(hs)))
    np.testing.assert_allclose(out.t, 5.0, rtol=1e-12)
    assert (out.prim == 4).all()
    obl = o.trace(_rays([[0.3, -3.0, 4.0], [0.3, -3.2, 4.0]], [[0, 0.6, -0.8], [0, 0.6, -0.8]]))
    np.testing.assert_allclose(obl.t[0], 5.0, rtol=1e-12)
    # shifted 0.2 in y: the line passes the axis at distance 0.2 * 0.8 = 0.16 < r,
    # closest to the axis point x = 0.3; depth (3.2 * 0.6 + 4 * 0.8) = 5.12
    np.testing.assert_allclose(obl.t[1], 5.12, rtol=1e-12)
    miss = o.trace(_rays([[0.3, 0.26, 5.0], [0.3, -0.26, 5.0]], [[0, 0, -1.0], [0, 0, -1.0]]))
    assert (miss.inst == -1).all()
    along = o.trace(_rays([[-6.0, 0.05, 0.0]], [[1.0, 0, 0]]))
    assert along.prim[0] == 0
    np.testing.assert_allclose(along.t, [4.0], rtol=1e-12)
    taper = [0, 0, 0, 0.4, 1, 0, 0, 0.3, 2, 0, 0, 0.2, 3, 0, 0, 0.1]
    ot = oracle.OracleScene(_curve_scene(taper, flat=True))
    ct = ot.capsules()
    assert (ct[:-1, 7] == ct[1:, 6]).all() and ct[4, 6] == np.float32(0.25)
    # at x = 1.5 (the start of segment 4) the half-width is 0.25
    near = ot.trace(_rays([[1.5, 0.25 * (1 - 1e-6), 5.0], [1.5, 0.25 * (1 + 1e-6), 5.0]], [[0, 0, -1.0]] * 2))
    assert near.inst[0] == 0 and near.inst[1] == -1


@pytest.mark.parametrize("turned", [False, True])
def test_ribbon_sun_shading_closed_form(turned):
    """A flat ribbon faces the ray: seen from far away at 45 degrees along its
    axis, its normal is the reverse ray direction without the part along the
    axis, i.e. straight up up to the ray's sideways tilt beta (the ribbon's
    half-width 0.3 at distance 200, over the 45-degree ray's vertical part:
    |beta| < 2.3e-3).  With the sun at angle alpha from the zenith across the
    axis, a camera sample on it carries a L_sky + a E cos(alpha - beta) / pi:
    within a sin(alpha) 2.3e-3 of a L_sky + a E cos(alpha) / pi, and cos(alpha) on
    average over the symmetric footprint.  (The reverse ray direction itself
    would give cos(alpha) / sqrt(2).)"""
    a, r, L, alpha = float(np.float32(0.5)), 0.3, 0.25, 0.6
    if turned:
        proto = [v for y in np.linspace(-2, 2, 4) for v in (0.0, y, 0.0, r)]
        Rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float64)
        Ry = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], np.float64)
        X = np.concatenate([Ry @ Rx, np.zeros((3, 1))], axis=1).reshape(1, 12)
        o = oracle.OracleScene(_curve_scene(proto, xforms=X, albedo=a, flat=True))
    else:
        o = oracle.OracleScene(_curve_scene(_straight(r=r), albedo=a, flat=True))
    D = 200.0 / math.sqrt(2.0)
    cams = [sg.Camera((-D, 0.0, D), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 1.5, 96, 96)]
    st = sg.RenderSettings(spp=1, depth=2, seed=9, light_dir=(0.0, math.sin(alpha), math.cos(alpha)), E=math.pi,
                           L_sky=L)
    img, fl, _ = o.render(cams, st)
    hit = np.abs(img - L) > 1e-9
    assert hit.sum() > 300
    cosv = (img[hit] - a * L) / a
    assert (np.abs(cosv - math.cos(alpha)) <= math.sin(alpha) * 2.3e-3).all(), np.abs(cosv - math.cos(alpha)).max()
    assert abs(cosv.mean() - math.cos(alpha)) < 1e-4, cosv.mean() - math.cos(alpha)


def test_ribbon_flags():
    """A ray passing a flat ribbon's edge within the graze distance is flagged
    GRAZE and either answer is acceptable; a ray through the middle of a
    segment is not flagged and must hit.  (Segments 0.5 long with radius 0.2,
    rays at x = 0.25, the middle of segment 4: the neighbouring segments' ends
    lie 0.25 away, beyond their radius.  Where the round ends of neighbouring
    segments overlap a segment seen face-on, both lie at the same depth: a
    tie.)"""
    r = 0.2
    o = oracle.OracleScene(_curve_scene(_straight(r=r), flat=True))
    rays = _rays([[0.25, r * (1 + 1e-9), 5.0], [0.25, r * (1 - 1e-9), 5.0], [0.25, 0.0, 5.0]], [[0, 0, -1.0]] * 3)
    out = o.trace(rays)
    assert out.flags[0] & oracle.F_GRAZE and out.flags[1] & oracle.F_GRAZE
    assert (out.flags[2] & oracle.ID_FLAGS) == 0 and out.inst[2] == 0
    code, info = o.accept(rays.astype(np.float32), np.array([-1, 0, -1]), np.array([-1, 4, -1]),
                          np.array([np.inf, out.t[1], np.inf], np.float32))
    assert code[0] == 0 and code[1] == 0 and code[2] == 2
