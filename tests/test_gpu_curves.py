"""Curves on the GPU (Section 5.2: the scene's curves, traced as chains of
capsules) against brute force and the oracle: every traversal variant and node
width returns the brute-force hits bit for bit; unflagged hits match the
oracle's FP64 answers and every ray's answer passes the acceptance check;
frames are bit-identical across schedulers and match the oracle (flagged
pixels replayed path by path); the adjoint is the transpose of the renderer's
own derivative and matches the oracle's gradient on the faces no flagged path
reaches; a closed form holds; argument errors are reported."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import (assert_hits_identical, camera_rays, compare_with_oracle, hits_np, log,
                            replay_check_pixels, to_dev)

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

VARIANTS = [dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
            dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
            dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PERSISTENT),
            dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
            dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT, stack_depth=4, refill=1, block=64)]
FRAME_KINDS = [dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
               dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
               dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
               dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL)]


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def capsule_rays(scene, osc, rng, n):
    """Rays aimed at points within 1.6 radii of random capsules' axes (hits,
    grazes and near misses), from 0.3 to 4 units away, with direction lengths
    spread over 2^-10 .. 2^10: [n, 8] FP32."""
    caps = osc.capsules()
    co = 8 * scene.proto_curve_off
    ci = np.nonzero(np.diff(scene.proto_curve_off)[scene.inst_proto] > 0)[0]
    inst = rng.choice(ci, n)
    p = scene.inst_proto[inst]
    k = co[p] + (rng.random(n) * (co[p + 1] - co[p])).astype(np.int64)
    c = caps[k]
    X = scene.inst_xform[inst].astype(np.float64).reshape(-1, 3, 4)
    a = np.einsum("nij,nj->ni", X[:, :, :3], c[:, 0:3]) + X[:, :, 3]
    b = np.einsum("nij,nj->ni", X[:, :, :3], c[:, 3:6]) + X[:, :, 3]
    scale = np.abs(np.linalg.det(X[:, :, :3])) ** (1 / 3)
    off = rng.normal(size=(n, 3))
    off *= (rng.uniform(0, 1.6, n) * c[:, 6] * scale / np.linalg.norm(off, axis=1))[:, None]
    target = a + rng.uniform(-0.1, 1.1, n)[:, None] * (b - a) + off
    dirn = rng.normal(size=(n, 3))
    dirn /= np.linalg.norm(dirn, axis=1)[:, None]
    o = target - rng.uniform(0.3, 4.0, n)[:, None] * dirn
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3:6] = dirn * np.exp2(rng.integers(-10, 11, n))[:, None]
    rays[:, 7] = np.inf
    return rays


def _curve_case(seed=3, flat=(False, False)):
    scene = sg.curve_scene(seed, n_inst=8, n_curves=24, flat=flat)
    osc = oracle.OracleScene(scene)
    rng = np.random.default_rng(seed + 100)
    rays = np.concatenate([capsule_rays(scene, osc, rng, 30000),
                           sg.random_rays(rng, 10000, [-3, -3, 0.05], [3, 3, 1.5], [-3, -3, -0.5], [3, 3, 1.2])])
    return scene, osc, rays


@pytest.mark.parametrize("width,flat", [(4, False), (2, False), (8, False), (4, True), (2, True)])
def test_curve_hits_bvh_brute_and_oracle(width, flat):
    """Round capsule chains, or one tuft prototype of each kind (flat: the
    second tuft is ribbons)."""
    log(f"case: curves, closest hits and occlusion, width {width}, flat ribbons {flat}")
    scene, osc, rays = _curve_case(flat=(False, flat))
    R = to_dev(rays)
    fmts = 0 if width == 4 else rtq.RTQ_NODE_Q8
    S = rtq.Scene(scene, node_width=width, formats=fmts)
    info = S.info()
    assert info["n_unique_curves"] == scene.n_curves and info["n_unique_capsules"] == 8 * scene.n_curves
    assert info["n_faces"] == scene.n_faces
    ref = hits_np(rtq.trace_brute(S, R))
    ncap = int((np.diff(scene.proto_curve_off)[scene.inst_proto[np.maximum(ref["inst"], 0)]] > 0)[ref["inst"] >= 0].sum())
    log(f"  {rays.shape[0]} rays, {int((ref['inst'] >= 0).sum())} hits, {ncap} on capsules")
    assert ncap > 5000
    for var in VARIANTS:
        if width != 4 and var["node_format"] == rtq.RTQ_NODE_FP32:
            continue
        assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), f"width {width} {var}")
        occ = _np(rtq.trace_occluded(S, R, **var))
        assert np.array_equal(occ != 0, ref["inst"] >= 0), f"width {width} {var}: occlusion differs"
    o = osc.trace(rays)
    st = {}
    frac = compare_with_oracle(scene, rays, ref, o, ora_scene=osc, stats=st)
    log(f"  flagged fraction {frac:.4f}, t error max {st['max_t_ulps']:.2f} units")
    assert frac < 0.05
    S.close()


@pytest.mark.parametrize("flat", [False, True])
def test_curve_secondary_rays_with_exclusion(flat):
    """Bounce rays leaving capsule, ribbon (and ground) hits exclude the
    primitive they leave (a ribbon: its whole curve): variants equal brute
    force, and the oracle, given the same exclusions, accepts every answer."""
    import torch
    log(f"case: curves, secondary rays with exclusion, flat ribbons {flat}")
    scene, osc, rays = _curve_case(5, flat=(flat, flat))
    S = rtq.Scene(scene)
    h0 = rtq.trace_closest(S, to_dev(rays), want_ref=True, node_format=rtq.RTQ_NODE_Q8,
                           scheduler=rtq.SCHED_PERSISTENT)
    torch.cuda.synchronize()
    hit = (h0.inst >= 0).cpu().numpy()
    t = h0.t.cpu().numpy()
    p = (rays[:, 0:3] + t[:, None] * rays[:, 3:6]).astype(np.float32)
    rng = np.random.default_rng(9)
    d = rng.normal(size=(rays.shape[0], 3)).astype(np.float32)
    sec = np.zeros((int(hit.sum()), 8), np.float32)
    sec[:, 0:3] = p[hit]
    sec[:, 3:6] = d[hit]
    sec[:, 7] = np.inf
    ref = h0.ref[torch.from_numpy(hit).cuda()].contiguous()
    R = to_dev(sec)
    base = hits_np(rtq.trace_brute(S, R, exclude=ref))
    for var in VARIANTS:
        assert_hits_identical(base, hits_np(rtq.trace_closest(S, R, exclude=ref, **var)), str(var))
    src_inst = h0.inst.cpu().numpy()[hit]
    src_prim = h0.prim.cpu().numpy()[hit]
    src_half = (ref[:, 1].cpu().numpy().view(np.uint32) >> 31).astype(np.int32)
    excl = np.stack([src_inst, src_prim, src_half], 1)
    o = osc.trace(sec, excl=excl)
    frac = compare_with_oracle(scene, sec, base, o, excl=excl, ora_scene=osc)
    log(f"  {sec.shape[0]} rays, flagged fraction {frac:.4f}")
    S.close()


def _frame_setup(seed=4, flat=(False, False)):
    scene = sg.curve_scene(seed, n_inst=8, n_curves=24, flat=flat)
    cams = [sg.Camera((0.0, -5.5, 1.4), (0.0, 0.0, 0.4), (0.0, 0.0, 1.0), 45.0, 48, 40),
            sg.Camera((3.0, 3.0, 2.0), (0.0, 0.0, 0.3), (0.0, 0.0, 1.0), 50.0, 40, 32)]
    st = sg.RenderSettings(spp=2, depth=4, seed=17, frame=1)
    return scene, cams, st


@pytest.mark.parametrize("mode,flat", [("lambert", False), ("principled+lights", False), ("lambert", True),
                                       ("principled+lights", True)])
def test_curve_frames_schedulers_and_oracle(mode, flat):
    import torch
    log(f"case: curve frames, {mode}, flat ribbons {flat}")
    scene, cams, st = _frame_setup(flat=(flat, flat))
    S = rtq.Scene(scene)
    osc = oracle.OracleScene(scene)
    if mode != "lambert":
        mats = np.array([(0.9, 0.6, 0.3, 0.5, 0.0, 0.8), (0.4, 0.7, 0.9, 0.35, 0.7, 0.2),
                         (0.3, 0.5, 0.2, 1.0, 0.0, 0.0)], np.float32)
        fm = np.random.default_rng(3).integers(0, 3, scene.n_faces).astype(np.uint8)
        S.set_materials(mats, torch.from_numpy(fm).cuda())
        osc.set_materials(mats, fm.astype(np.int32))
        st.area_lights = ((-3.0, -3.0, 5.0, 0.0, 6.0, 0.0, 6.0, 0.0, 0.0, 2.0),)
        env = np.random.default_rng(4).uniform(0.0, 1.0, size=(16, 32)).astype(np.float32)
        S.set_environment(torch.from_numpy(env).cuda())
        osc.set_environment(env)
        st.env_nee = True
    imgs = [_np(rtq.render(S, cams, st, **kw)) for kw in FRAME_KINDS]
    g1 = _np(rtq.render(S, cams, st, graph=True, **FRAME_KINDS[2]))
    g2 = _np(rtq.render(S, cams, st, graph=True, **FRAME_KINDS[2]))
    ref_img = imgs[0]
    for img, kw in zip(imgs[1:] + [g1, g2], FRAME_KINDS[1:] + ["graph", "graph replay"]):
        assert (img.view(np.uint32) == ref_img.view(np.uint32)).all(), f"frame differs for {kw}"
    ref, fl, _ = osc.render(cams, st)
    rgb = ref_img.ndim == 2
    ok = fl == 0
    err = np.abs(ref_img.astype(np.float64) - ref)
    scale = np.abs(ref).max(axis=1, keepdims=True) if rgb else np.abs(ref)
    bad = ok[:, None] & (err > 1e-4 * scale + 1e-7) if rgb else ok & (err > 1e-4 * scale + 1e-7)
    if bad.any():
        k = np.nonzero(bad.any(axis=1) if rgb else bad)[0][:8]
        raise AssertionError(f"unflagged pixels differ: idx {k} gpu {ref_img[k]} oracle {ref[k]}")
    idx = np.nonzero(~ok)[0]
    tot = replay_check_pixels(rtq, osc, S, cams, st, idx, ref_img, **FRAME_KINDS[2])
    log(f"  flagged pixels {idx.size} of {ok.size}, replayed: {tot}")
    # a path that meets a capsule is flagged for its normal's FP32 uncertainty
    assert idx.size < 0.6 * ok.size
    # every path of a few pixels that see curves, replayed as well
    pix = np.arange(0, ok.size, 97)
    replay_check_pixels(rtq, osc, S, cams, st, pix, ref_img, **FRAME_KINDS[2])
    S.close()


def test_curve_frames_equal_across_widths():
    log("case: curve frames, node widths")
    scene, cams, st = _frame_setup(6, flat=(False, True))
    S4 = rtq.Scene(scene)
    ref = _np(rtq.render(S4, cams, st, node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN))
    S4.close()
    for w in (2, 8):
        S = rtq.Scene(scene, node_width=w)
        for kw in FRAME_KINDS[1:]:
            img = _np(rtq.render(S, cams, st, **kw))
            assert (img.view(np.uint32) == ref.view(np.uint32)).all(), f"width {w} {kw}"
        S.close()


def test_curve_adjoint():
    """Curves are faces of their own.  (a) The adjoint is the transpose of the
    renderer's own derivative: with paths held fixed a Lambertian path's value
    is a polynomial in the albedos it meets, so g . e equals the central
    difference of sum(gp I) along e, on the curve faces and on the ground
    faces (the GPU's own paths, so this holds whatever the normals' rounding).
    (b) Against the oracle's gradient with the pixel weights of flagged pixels
    -- every path that meets a capsule is flagged for its normal's FP32
    uncertainty -- set to zero: the faces no flagged path reaches agree."""
    import torch
    log("case: curve adjoint")
    scene, cams, st = _frame_setup(7, flat=(True, False))
    st.depth = 3
    S = rtq.Scene(scene)
    kw = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    n_pix = sum(c.w * c.h for c in cams)
    rng = np.random.default_rng(2)
    gp = rng.normal(size=n_pix).astype(np.float32)
    g = _np(rtq.render_backward(S, cams, st, torch.from_numpy(gp).cuda(), **kw)).astype(np.float64)
    assert g.shape == (scene.n_faces,)
    curves = np.zeros(scene.n_faces, bool)
    curves[scene.n_quads:] = True
    assert (np.abs(g[curves]) > 0).sum() > 20
    alb = torch.from_numpy(scene.albedo).cuda()
    h = 1e-3
    for part in (curves, ~curves):
        e = np.where(part, rng.normal(size=scene.n_faces), 0.0)
        et = torch.from_numpy(e.astype(np.float32)).cuda()
        S.set_albedo(alb + h * et)
        Ip = _np(rtq.render(S, cams, st, **kw)).astype(np.float64)
        S.set_albedo(alb - h * et)
        Im = _np(rtq.render(S, cams, st, **kw)).astype(np.float64)
        S.set_albedo(alb)
        # the perturbation as the device holds it (FP32 albedos)
        ep = ((scene.albedo + h * e.astype(np.float32)).astype(np.float32).astype(np.float64)
              - (scene.albedo - h * e.astype(np.float32)).astype(np.float32).astype(np.float64)) / (2 * h)
        fd = (gp.astype(np.float64) * (Ip - Im)).sum() / (2 * h)
        ge = (g * ep).sum()
        log(f"  {'curve' if part[-1] else 'ground'} faces: g.e {ge:.6g}, central difference {fd:.6g}")
        assert abs(ge - fd) <= 1e-3 * abs(fd) + 2e-2, (ge, fd)
    osc = oracle.OracleScene(scene)
    ref, fl, _ = osc.render(cams, st)
    gq = rng.normal(size=ref.shape)
    gq[fl != 0] = 0.0
    g_ref, _, taint = osc.grad(cams, st, gq, taint="path")
    g2 = _np(rtq.render_backward(S, cams, st, torch.from_numpy(gq.astype(np.float32)).cuda(), **kw))
    keep = taint == 0
    scale = np.abs(g_ref[keep]).max()
    err = np.abs(g2[keep] - g_ref[keep])
    log(f"  oracle: faces kept {keep.sum()} of {keep.size}, max error {err.max():.3g} of {scale:.3g}")
    assert (err <= 2e-4 * scale + 1e-4 * np.abs(g_ref[keep])).all()
    S.close()


def test_curve_sun_closed_form_gpu():
    """A straight curve along x seen from far above with the sun overhead: a
    sample on a capsule carries a L_sky + a E cos / pi, cos the z part of the
    normal, so every such pixel lies in (a L_sky, a (L_sky + E / pi)] and the
    mean cos over the footprint is the closed form of the body (pi / 4) and
    the end half-disks (2 / 3)."""
    log("case: curve closed form on the GPU")
    a, r, L = float(np.float32(0.5)), 0.3, 0.25
    curve = [v for x in np.linspace(-2, 2, 4) for v in (x, 0.0, 0.0, r)]
    scene = sg.Scene(verts=np.zeros((0, 3), np.float32), quads=np.zeros((0, 4), np.int32),
                     proto_vert_off=np.array([0, 0], np.int64), proto_quad_off=np.array([0, 0], np.int64),
                     albedo=np.array([a], np.float32), inst_proto=np.zeros(1, np.int32),
                     inst_xform=sg.identity_xform(1), curves=np.array([curve], np.float32),
                     proto_curve_off=np.array([0, 1], np.int64))
    scene.validate()
    S = rtq.Scene(scene)
    cams = [sg.Camera((0.0, 0.0, 200.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 1.5, 128, 128)]
    st = sg.RenderSettings(spp=1, depth=2, seed=9, light_dir=(0.0, 0.0, 1.0), E=math.pi, L_sky=L)
    img = _np(rtq.render(S, cams, st)).astype(np.float64)
    hit = np.abs(img - L) > 1e-6
    cos = (img[hit] - a * L) / a
    body, disks = 4.0 * 2 * r, math.pi * r * r
    expect = (body * math.pi / 4 + disks * 2 / 3) / (body + disks)
    log(f"  {hit.sum()} samples on the curve, mean cos {cos.mean():.4f} (closed form {expect:.4f})")
    assert hit.sum() > 1000 and (cos > 0).all() and (cos <= 1 + 1e-6).all()
    assert abs(cos.mean() - expect) < 0.009
    S.close()


def test_curve_argument_errors():
    import torch
    scene = sg.curve_scene(1, n_inst=2, n_curves=4)
    S = rtq.Scene(scene)
    with pytest.raises(rtq.RtqError):
        S.set_textures(torch.zeros((scene.n_quads, 2, 2), device="cuda"))
    S.close()
    for bad in ("nan", "radius"):
        c = scene.curves.copy()
        if bad == "nan":
            c[1, 5] = np.nan
        else:
            c[2, 7] = -0.1
        s2 = sg.Scene(verts=scene.verts, quads=scene.quads, proto_vert_off=scene.proto_vert_off,
                      proto_quad_off=scene.proto_quad_off, albedo=scene.albedo, inst_proto=scene.inst_proto,
                      inst_xform=scene.inst_xform, curves=c, proto_curve_off=scene.proto_curve_off)
        with pytest.raises(rtq.RtqError):
            rtq.Scene(s2)


def test_ribbon_sun_closed_form_gpu():
    """A flat ribbon seen from far away at 45 degrees along its axis faces up
    to within the ray's sideways tilt (|beta| < 2.3e-3): with the sun at
    alpha = 0.6 from the zenith across the axis, every camera sample on it
    carries a L_sky + a E cos(alpha - beta) / pi (the reverse ray direction
    as the normal would give cos(alpha) / sqrt(2))."""
    log("case: ribbon closed form on the GPU")
    a, r, L, alpha = float(np.float32(0.5)), 0.3, 0.25, 0.6
    curve = [v for x in np.linspace(-2, 2, 4) for v in (x, 0.0, 0.0, r)]
    scene = sg.Scene(verts=np.zeros((0, 3), np.float32), quads=np.zeros((0, 4), np.int32),
                     proto_vert_off=np.array([0, 0], np.int64), proto_quad_off=np.array([0, 0], np.int64),
                     albedo=np.array([a], np.float32), inst_proto=np.zeros(1, np.int32),
                     inst_xform=sg.identity_xform(1), curves=np.array([curve], np.float32),
                     proto_curve_off=np.array([0, 1], np.int64), proto_curve_flat=np.array([1], np.int32))
    scene.validate()
    S = rtq.Scene(scene)
    D = 200.0 / math.sqrt(2.0)
    cams = [sg.Camera((-D, 0.0, D), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 1.5, 96, 96)]
    st = sg.RenderSettings(spp=1, depth=2, seed=9, light_dir=(0.0, math.sin(alpha), math.cos(alpha)), E=math.pi,
                           L_sky=L)
    img = _np(rtq.render(S, cams, st)).astype(np.float64)
    hit = np.abs(img - L) > 1e-6
    cosv = (img[hit] - a * L) / a
    log(f"  {hit.sum()} samples on the ribbon, cos spread {cosv.min():.6f} .. {cosv.max():.6f} "
        f"(cos(alpha) {math.cos(alpha):.6f})")
    assert hit.sum() > 300
    assert (np.abs(cosv - math.cos(alpha)) <= math.sin(alpha) * 2.3e-3 + 2e-6).all()
    S.close()
