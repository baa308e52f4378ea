"""Parity of the HIP ray queries (through the C-ABI) with the oracle, and
bit-identity of every traversal variant with the brute-force reference."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import assert_hits_identical, compare_with_oracle, hits_np, log, to_dev

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

VARIANTS = [
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PERSISTENT),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT, stack_depth=4, refill=1, block=64),
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN, stack_depth=4, block=128),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT, stack_depth=32, refill=48, block=256,
         waves_per_cu=4),
]


def _tiny_rays(seed, n):
    rng = np.random.default_rng(seed)
    return np.concatenate([sg.random_rays(rng, n // 2, -5, 5, -2, 2), sg.random_rays(rng, n - n // 2, -1, 1, -3, 3)])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bvh_variants_equal_brute_force_tiny(seed):
    log(f"case: tiny scene seed {seed}")
    rng = np.random.default_rng(seed)
    scene = sg.tiny_scene(seed, n_inst=4, n_protos=2, nq=int(rng.integers(2, 9)), spread=1.5)
    S = rtq.Scene(scene)
    rays = _tiny_rays(seed, 20000)
    R = to_dev(rays)
    ref = hits_np(rtq.trace_brute(S, R))
    assert (ref["inst"] >= 0).mean() > 0.2
    for var in VARIANTS:
        log("  variant", var)
        assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), str(var))
    o = oracle.OracleScene(scene).trace(rays)
    frac = compare_with_oracle(scene, rays, ref, o)
    log(f"  flagged fraction {frac:.4f}")
    assert frac < 0.05


def test_bvh_variants_equal_brute_force_config1():
    log("case: config 1 scene, random rays")
    scene, cams, _ = sg.config1()
    S = rtq.Scene(scene)
    rng = np.random.default_rng(4)
    rays = sg.random_rays(rng, 20000, -80, 80, -50, 50)
    R = to_dev(rays)
    ref = hits_np(rtq.trace_brute(S, R))
    assert (ref["inst"] >= 0).mean() > 0.05
    for var in VARIANTS:
        log("  variant", var)
        assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), str(var))
    o = oracle.OracleScene(scene).trace(rays)
    frac = compare_with_oracle(scene, rays, ref, o)
    log(f"  flagged fraction {frac:.4f}")


def test_edge_on_sliver_rays_config1():
    """Two rays of the config-1 scene pass far from quads that they see edge-on:
    in FP32 two edge functions of such a quad cancel to exactly zero and the
    third is one ulp, which a test accepting zeros as inside takes for a vertex
    hit tens of units from the ray.  The FP64 re-evaluation of zero edge values
    must reject them, in the brute-force reference and in every variant."""
    log("case: config 1 scene, edge-on sliver rays")
    scene, cams, _ = sg.config1()
    S = rtq.Scene(scene)
    rays = sg.random_rays(np.random.default_rng(4), 20000, -80, 80, -50, 50)[[162, 3709]]
    o = oracle.OracleScene(scene).trace(rays)
    assert list(o.inst) == [626, -1] and (o.flags == 0).all()
    R = to_dev(rays)
    ref = hits_np(rtq.trace_brute(S, R))
    assert list(ref["inst"]) == [626, -1] and list(ref["prim"]) == [464, -1]
    for var in VARIANTS:
        assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), str(var))


def test_camera_rays_config1_vs_oracle():
    log("case: config 1 camera rays through pixel centres")
    scene, cams, _ = sg.config1()
    c = cams[0]
    W, H = 256, 256
    f = np.array(c.look) - np.array(c.eye)
    f /= np.linalg.norm(f)
    r = np.cross(f, c.up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(c.vfov_deg) / 2)
    ys, xs = np.mgrid[0:H, 0:W]
    sx = (2 * (xs + 0.5) / W - 1) * th
    sy = (1 - 2 * (ys + 0.5) / H) * th
    d = f + sx[..., None] * r + sy[..., None] * u
    d = d.reshape(-1, 3)
    rays = np.zeros((d.shape[0], 8), np.float32)
    rays[:, 0:3] = c.eye
    rays[:, 3:6] = d
    rays[:, 7] = np.inf
    S = rtq.Scene(scene)
    g = hits_np(rtq.trace_closest(S, to_dev(rays), node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT))
    o = oracle.OracleScene(scene).trace(rays)
    frac = compare_with_oracle(scene, rays, g, o)
    log(f"  hit fraction {(o.inst >= 0).mean():.3f} flagged {frac:.4f}")
    assert (o.inst >= 0).mean() > 0.05


def test_analytic_quad_gpu():
    log("case: axis-aligned quad closed form")
    x0, x1, y0, y1, c = -1.5, 2.0, -0.5, 1.25, 0.75
    scene = ts.multi_mesh_scene([ts.axis_quad(x0, x1, y0, y1, c)])
    S = rtq.Scene(scene)
    rng = np.random.default_rng(11)
    n = 20000
    org = np.stack([rng.uniform(-4, 4, n), rng.uniform(-4, 4, n), rng.choice([-3.0, 4.0], n)], 1)
    tgt = np.stack([rng.uniform(x0 - 1, x1 + 1, n), rng.uniform(y0 - 1, y1 + 1, n), np.full(n, c)], 1)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = org
    rays[:, 3:6] = tgt - org
    rays[:, 7] = np.inf
    r64 = rays.astype(np.float64)
    g = hits_np(rtq.trace_closest(S, to_dev(rays)))
    t_exp = (c - r64[:, 2]) / r64[:, 5]
    p = r64[:, 0:3] + t_exp[:, None] * r64[:, 3:6]
    uu = (p[:, 0] - x0) / (x1 - x0)
    vv = (p[:, 1] - y0) / (y1 - y0)
    m = 1e-4
    inside = (uu > m) & (uu < 1 - m) & (vv > m) & (vv < 1 - m)
    outside = (uu < -m) | (uu > 1 + m) | (vv < -m) | (vv > 1 + m)
    assert (g["inst"][inside] == 0).all() and (g["inst"][outside] == -1).all()
    np.testing.assert_allclose(g["t"][inside], t_exp[inside], rtol=1e-6)
    np.testing.assert_allclose(g["u"][inside], uu[inside], atol=2e-5)
    np.testing.assert_allclose(g["v"][inside], vv[inside], atol=2e-5)


@pytest.mark.parametrize("fmt", [1, 2])
def test_watertight_closed_shell(fmt):
    """Rays from inside a closed quad shell aimed exactly at every vertex and every
    edge midpoint never escape (FP32, watertight leaf test)."""
    log(f"case: closed shell, format {fmt}")
    for seed, n in ((3, 6), (5, 17)):
        scene, v, q = ts.shell_scene(seed=seed, n=n)
        S = rtq.Scene(scene)
        tg = [v.astype(np.float64)]
        for a, b in ((0, 1), (1, 2), (2, 3), (3, 0)):
            tg.append(0.5 * (v[q[:, a]].astype(np.float64) + v[q[:, b]].astype(np.float64)))
        tg = np.concatenate(tg)
        for centre in (np.zeros(3), np.array([0.1, -0.05, 0.2])):
            rays = np.zeros((tg.shape[0], 8), np.float32)
            rays[:, 0:3] = centre
            rays[:, 3:6] = tg - centre
            rays[:, 7] = np.inf
            g = hits_np(rtq.trace_closest(S, to_dev(rays), node_format=fmt))
            assert (g["inst"] == 0).all(), f"{(g['inst'] < 0).sum()} rays escaped the shell"


def test_occluded_matches_closest_and_edge_cases():
    log("case: occlusion and degenerate rays")
    import torch
    scene = sg.tiny_scene(7, n_inst=4, n_protos=2, nq=6, spread=1.5)
    S = rtq.Scene(scene)
    rays = _tiny_rays(7, 5000)
    rays[0, 3:6] = 0.0          # zero direction
    rays[1, 3] = np.nan         # NaN direction
    rays[2, 7] = 1e-3           # tiny tmax
    rays[3, 6] = 1e9            # tmin beyond everything
    R = to_dev(rays)
    g = hits_np(rtq.trace_closest(S, R))
    for var in VARIANTS:
        occ = rtq.trace_occluded(S, R, **var).cpu().numpy()
        np.testing.assert_array_equal(occ.astype(bool), g["inst"] >= 0)
    assert g["inst"][0] == -1 and g["inst"][1] == -1 and g["inst"][3] == -1
    assert np.isinf(g["t"][0]) and g["prim"][0] == -1 and g["u"][0] == 0
    # empty launch
    e = rtq.trace_closest(S, torch.zeros((0, 8), device="cuda"))
    assert e.t.numel() == 0


def test_argument_errors():
    import torch
    scene = sg.tiny_scene(1)
    S = rtq.Scene(scene)
    R = torch.zeros((4, 8), device="cuda")
    with pytest.raises(rtq.RtqError):
        rtq.trace_closest(S, R, stack_depth=2)
    with pytest.raises(rtq.RtqError):
        rtq.trace_closest(S, R, block=96)
    bad = sg.tiny_scene(1)
    bad.inst_xform[0, :] = 0.0
    with pytest.raises(rtq.RtqError) as ei:
        rtq.Scene(bad)
    assert ei.value.code == -2
    bad2 = sg.tiny_scene(1)
    bad2.quads[0, 0] = 10 ** 6
    with pytest.raises(rtq.RtqError) as ei:
        rtq.Scene(bad2)
    assert ei.value.code == -1
    # more rays per call than a dispatch can count: LIMIT, before anything runs
    import ctypes
    soa, rs = rtq._rays_struct(R)
    out = torch.zeros((5, 4), device="cuda")
    hits = rtq._Hits(*[out[k].data_ptr() for k in range(5)])
    L = rtq.load_library()
    rc = L.rtq_trace_closest(S.handle, ctypes.byref(rs), 2 ** 31, ctypes.byref(hits), None, None)
    assert rc == -5, rc
    rc = L.rtq_trace_occluded(S.handle, ctypes.byref(rs), 2 ** 31, out.data_ptr(), None, None)
    assert rc == -5, rc
    torch.cuda.synchronize()


def test_config2_sampled_rays_vs_oracle():
    """Full-size config 2 scene (1M instances on a 4M-quad terrain): camera rays of
    both views on a sampled pixel grid, plus incoherent rays, against the oracle."""
    log("case: config 2 full size, sampled rays")
    scene, cams, _ = sg.config2()
    S = rtq.Scene(scene)
    log("  built", S.info())
    rng = np.random.default_rng(9)
    rays = []
    for c in cams:
        f = np.array(c.look) - np.array(c.eye)
        f /= np.linalg.norm(f)
        r = np.cross(f, c.up)
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        th = math.tan(math.radians(c.vfov_deg) / 2)
        xs = rng.uniform(0, c.w, 4000)
        ys = rng.uniform(0, c.h, 4000)
        d = f + ((2 * xs / c.w - 1) * th * c.w / c.h)[:, None] * r + ((1 - 2 * ys / c.h) * th)[:, None] * u
        rr = np.zeros((4000, 8), np.float32)
        rr[:, 0:3] = c.eye
        rr[:, 3:6] = d
        rr[:, 7] = np.inf
        rays.append(rr)
    inc = sg.random_rays(rng, 4000, [-1000, -1000, 0], [1000, 1000, 150], [-1000, -1000, -50], [1000, 1000, 100])
    rays.append(inc)
    rays = np.concatenate(rays)
    R = to_dev(rays)
    ref = hits_np(rtq.trace_closest(S, R, node_format=rtq.RTQ_NODE_FP32))
    for var in VARIANTS[1:4]:
        assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), str(var))
    o = oracle.OracleScene(scene).trace(rays)
    frac = compare_with_oracle(scene, rays, ref, o)
    log(f"  hit fraction {(o.inst >= 0).mean():.3f} flagged {frac:.4f}")


@pytest.mark.parametrize("cfg", ["tiny", "config1", "config2_small"])
def test_opened_instances_keep_hits_and_images(cfg):
    """Opening instances into subtrees in the top level (rtq_build_opts.open_pct)
    changes which entries a ray visits, never its hits: closest hits of every
    opening budget equal the unopened scene's and the brute-force reference bit
    for bit, and so do rendered frames."""
    import torch
    log(f"case: opened instances, {cfg}")
    rng = np.random.default_rng(17)
    if cfg == "tiny":
        scene = sg.tiny_scene(8, n_inst=5, n_protos=2, nq=8, spread=1.2)
        cams = [sg.Camera((0.0, -9.0, 1.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 50.0, 40, 30)]
        st = sg.RenderSettings(spp=2, depth=4, seed=3)
        rays = _tiny_rays(8, 20000)
    elif cfg == "config1":
        scene, cams, st = sg.config1()
        rays = sg.random_rays(rng, 20000, -80, 80, -50, 50)
    else:
        scene, cams, st = sg.config2(scale=0.01, res=(96, 64))
        rays = sg.random_rays(rng, 20000, [-1000, -1000, 0], [1000, 1000, 150], [-1000, -1000, -50],
                              [1000, 1000, 100])
    R = to_dev(rays)
    ref = img = None
    for pct in (-1, 0, 400, 100000):
        S = rtq.Scene(scene, open_pct=pct)
        info = S.info()
        log(f"  open_pct {pct}: {info['n_top_entries']} top-level entries for {info['n_instances']} instances")
        if pct == -1:
            assert info["n_top_entries"] == info["n_instances"]
        if pct == 100000:
            assert info["n_top_entries"] > info["n_instances"]
        h = hits_np(rtq.trace_closest(S, R, node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT))
        hb = hits_np(rtq.trace_brute(S, R))
        assert_hits_identical(hb, h, f"open_pct {pct} vs its brute force")
        st.frame = 1
        im = rtq.render(S, cams, st, node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
        torch.cuda.synchronize()
        im = im.cpu().numpy()
        if ref is None:
            ref, img = h, im
        else:
            assert_hits_identical(ref, h, f"open_pct {pct} vs unopened")
            assert np.array_equal(img.view(np.uint32), im.view(np.uint32)), f"open_pct {pct}: image differs"
        S.close()


def test_secondary_rays_with_exclusion_config1():
    """Secondary rays leaving a surface (Section 5.4's bounce and shadow rays):
    camera-ray hits return their references, rays from the FP32 hit points in
    random directions exclude the triangle they leave; every traversal variant
    equals the brute-force reference bit for bit, no ray reports its own
    triangle, and the hits match the oracle given the same exclusions."""
    import torch
    log("case: secondary rays with exclusion, config 1")
    scene, cams, _ = sg.config1()
    S = rtq.Scene(scene)
    rng = np.random.default_rng(31)
    from tests.gpu_util import camera_rays
    cr = camera_rays(cams, rng, 30000)
    h0 = rtq.trace_closest(S, to_dev(cr), want_ref=True, node_format=rtq.RTQ_NODE_Q8,
                           scheduler=rtq.SCHED_PERSISTENT)
    torch.cuda.synchronize()
    hit = (h0.inst >= 0).cpu().numpy()
    t = h0.t.cpu().numpy()
    p = (cr[:, 0:3] + t[:, None] * cr[:, 3:6]).astype(np.float32)  # FP32 hit points, as the renderer forms them
    d = rng.normal(size=(cr.shape[0], 3)).astype(np.float32)
    rays = np.zeros((int(hit.sum()), 8), np.float32)
    rays[:, 0:3] = p[hit]
    rays[:, 3:6] = d[hit]
    rays[:, 7] = np.inf
    ref = h0.ref[torch.from_numpy(hit).cuda()].contiguous()
    R = to_dev(rays)
    base = hits_np(rtq.trace_brute(S, R, exclude=ref))
    for var in VARIANTS:
        assert_hits_identical(base, hits_np(rtq.trace_closest(S, R, exclude=ref, **var)), str(var))
    src_inst = h0.inst.cpu().numpy()[hit]
    src_prim = h0.prim.cpu().numpy()[hit]
    src_half = (ref[:, 1].cpu().numpy().view(np.uint32) >> 31).astype(np.int32)
    # rays that hit their own quad hit its other half (the excluded half is never reported)
    own = (base["inst"] == src_inst) & (base["prim"] == src_prim)
    log(f"  {rays.shape[0]} rays, {own.sum()} hit the other half of the quad they leave")
    excl = np.stack([src_inst, src_prim, src_half], 1)
    o = oracle.OracleScene(scene).trace(rays, excl=excl)
    frac = compare_with_oracle(scene, rays, base, o, excl=excl)
    log(f"  flagged fraction {frac:.4f}")
    # without the exclusion the same rays often re-hit the triangle they leave
    plain = hits_np(rtq.trace_closest(S, R, node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT))
    again = (plain["inst"] == src_inst) & (plain["prim"] == src_prim) & (plain["t"] < 1e-3)
    log(f"  without exclusion {again.sum()} rays re-hit their own quad at t < 1e-3")
