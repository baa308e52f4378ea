"""Parity of the HIP path tracer and its adjoint (through the C-ABI) with the
oracle, and bit-identity of the two schedulers."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import log, replay_check_pixels

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

SCHEDS = [
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PERSISTENT),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
    dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_MEGAKERNEL),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT, stack_depth=4, refill=1, block=64,
         waves_per_cu=2),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL, stack_depth=4, refill=1, block=64,
         waves_per_cu=2),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL, stack_depth=24, refill=40, block=128),
]


def _render(S, cams, st, **kw):
    import torch
    img = rtq.render(S, cams, st, **kw)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def _compare_image(gpu, ref, flags, rel=1e-4, replay=None, pixels=None):
    """Unflagged pixels: the oracle's free-running FP64 value to `rel`.  Flagged
    pixels: with replay = (S, osc, cams, st, render options), every sample path
    of each one is traced alone on the GPU and checked step by step along its
    own rays (replay_check_pixels), so no pixel goes unchecked.  `pixels` maps
    the compared entries to packed image indices (default: all).  Returns the
    flagged fraction."""
    ok = flags == 0
    err = np.abs(gpu.astype(np.float64) - ref)
    bad = ok & (err > rel * np.abs(ref) + 1e-7)
    if bad.any():
        k = np.nonzero(bad)[0][:8]
        raise AssertionError(f"{bad.sum()} unflagged pixels differ: idx {k} gpu {gpu[k]} oracle {ref[k]}")
    if replay is not None:
        S, osc, cams, st, kw = replay
        idx = np.nonzero(~ok)[0]
        full = np.zeros(int(np.max(pixels)) + 1 if pixels is not None else gpu.size, np.float32)
        gidx = idx if pixels is None else np.asarray(pixels)[idx]
        full[gidx] = gpu[idx]
        tot = replay_check_pixels(rtq, osc, S, cams, st, gidx, full, **kw)
        log(f"  replayed {idx.size} flagged pixels: {tot}")
    return 1.0 - ok.mean()


def _multi_view_scene():
    scene = sg.tiny_scene(21, n_inst=24, n_protos=3, nq=8, spread=3.0)
    cams = [sg.Camera((0.0, -12.0, 2.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 45.0, 37, 23),
            sg.Camera((9.0, 4.0, 6.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 64, 64),
            sg.Camera((-3.0, 2.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 5, 70)]
    return scene, cams


@pytest.mark.parametrize("cfg", ["config1", "multiview"])
def test_schedulers_bit_identical_and_match_oracle(cfg):
    log(f"case: render {cfg}")
    if cfg == "config1":
        scene, cams, st = sg.config1()
    else:
        scene, cams = _multi_view_scene()
        st = sg.RenderSettings(spp=3, depth=5, seed=77, frame=2)
    S = rtq.Scene(scene)
    import torch
    imgs = []
    for kw in SCHEDS:
        log("  scheduler", kw)
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        imgs.append((_render(S, cams, st, counters=cnt, **kw), cnt.cpu().numpy()))
    ref_img, ref_cnt = imgs[0]
    for (img, cnt), kw in zip(imgs[1:], SCHEDS[1:]):
        assert (img.view(np.uint32) == ref_img.view(np.uint32)).all(), f"image differs for {kw}"
        assert (cnt == ref_cnt).all(), f"ray counts differ for {kw}: {cnt} vs {ref_cnt}"
    o = oracle.OracleScene(scene)
    ref, fl, stats = o.render(cams, st)
    frac = _compare_image(ref_img, ref, fl, replay=(S, o, cams, st, SCHEDS[3]))
    log(f"  flagged pixels {frac:.4f}; gpu rays {ref_cnt}; oracle {stats}")
    assert frac < 0.1
    n_paths = sum(c.w * c.h for c in cams) * st.spp
    assert ref_cnt[3] == n_paths
    if frac == 0.0:
        assert ref_cnt[0] == stats["closest"] and ref_cnt[1] == stats["shadow"]


def test_closed_form_images_gpu():
    log("case: closed-form images")
    a = float(np.float32(0.35))
    st = sg.RenderSettings(spp=2, depth=2, seed=9)
    cams = [sg.Camera((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 16, 16)]
    for kw in SCHEDS[:4]:
        img = _render(rtq.Scene(ts.floor_scene(albedo=a)), cams, st, **kw)
        cosl = st.light_dir[2]
        np.testing.assert_allclose(img, a * cosl + a * st.L_sky, rtol=2e-6)
        empty = ts.multi_mesh_scene([ts.axis_quad(-1, 1, -1, 1, 0.0)], xforms=[[1, 0, 0, 0, 0, 1, 0, 500, 0, 0, 1, 0]])
        img = _render(rtq.Scene(empty), cams, st, **kw)
        assert (img == np.float32(st.L_sky)).all()


def test_cosine_sampling_form_factor_gpu():
    """The view-factor scene of the oracle pin: per-pixel parity with the oracle
    on unflagged pixels, and the mean escape fraction of cosine-sampled bounces
    equal to 1 - F within 5 sigma."""
    log("case: cosine sampling view factor")
    a_f, h, half = 0.5, 1.0, 0.4
    ceil = ts.axis_quad(-half, half, -half, half, h)
    scene = ts.floor_scene(albedo=a_f, half=50.0, extra=[(ceil, 0.5)])
    cams = [sg.Camera((0.0, 0.0, 0.5), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.01, 64, 64)]
    st = sg.RenderSettings(spp=64, depth=2, seed=78)
    S = rtq.Scene(scene)
    img = _render(S, cams, st, scheduler=rtq.SCHED_MEGAKERNEL).astype(np.float64)
    o = oracle.OracleScene(scene)
    ref, fl, _ = o.render(cams, st)
    frac = _compare_image(img.astype(np.float32), ref, fl, replay=(S, o, cams, st, {}))
    assert frac < 0.05
    F = 4 * ts.form_factor_corner(half, half, h)
    cosl = 2 / math.sqrt(6.0)
    escape = (img - a_f * cosl) / (a_f * st.L_sky)
    n = img.size * st.spp
    assert abs(escape.mean() - (1 - F)) < 5 * math.sqrt(F * (1 - F) / n)


def _fd_faces(rng, g_or, taint, k=64):
    mx = np.abs(g_or).max()
    cand = np.nonzero((np.abs(g_or) > 1e-6 * mx) & (taint == 0))[0]
    return rng.choice(cand, size=min(k, cand.size), replace=False)


def test_adjoint_config4_vs_oracle_and_fd():
    """Config 4: L2 loss against a target rendered with albedo + U[-0.1, 0.1].
    (i) The adjoint kernel against the oracle's FP64 path-replay gradient, both
    fed the same pixel weights 2 (I - T) / N with flagged pixels weighted zero,
    on 64 random faces with a non-negligible gradient (1e-3 relative).  (ii) The whole differentiable render (the
    torch.autograd.Function on the GPU's own loss) against central finite
    differences of the GPU renderer (h = 1e-2, 1e-3 relative)."""
    import torch
    from paper_2001_02620_amd.autograd import RenderAlbedo
    log("case: config 4 adjoint")
    scene, cams, st = sg.config4()
    S = rtq.Scene(scene)
    rng = np.random.default_rng(2001026204)
    alb = scene.albedo.astype(np.float32)
    tgt_alb = (alb + rng.uniform(-0.1, 0.1, alb.shape)).astype(np.float32)
    opts = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    o = oracle.OracleScene(scene)
    o.set_albedo(tgt_alb.astype(np.float64))
    T_or, _, _ = o.render(cams, st)
    o.set_albedo(alb.astype(np.float64))
    I_or, fl, _ = o.render(cams, st)
    N = I_or.size
    # pixel weights of the loss, zero on flagged pixels: every path that then
    # contributes is unflagged, so both sides replay identical hits
    gpix = (2 * (I_or - T_or) / N).astype(np.float32).astype(np.float64)
    gpix[fl != 0] = 0.0
    g_or, _, _ = o.grad(cams, st, gpix)
    S.set_albedo(torch.from_numpy(alb).cuda())
    g_gpu = rtq.render_backward(S, cams, st, torch.from_numpy(gpix.astype(np.float32)).cuda(), **opts)
    g_gpu = g_gpu.cpu().numpy().astype(np.float64)
    faces = _fd_faces(rng, g_or, np.zeros_like(g_or, dtype=np.uint8))
    log(f"  flagged pixels {fl.mean():.3f}, faces with gradient {int((g_or != 0).sum())}")
    assert faces.size >= 32
    rel = np.abs(g_gpu[faces] - g_or[faces]) / np.abs(g_or[faces])
    log(f"  adjoint vs oracle: max rel {rel.max():.2e} over {faces.size} faces")
    assert (rel <= 1e-3).all()
    # the differentiable render on the GPU's own loss vs central differences
    a_t = torch.from_numpy(tgt_alb).cuda()
    with torch.no_grad():
        T = RenderAlbedo.apply(a_t, S, cams, st, opts).clone()
    a = torch.from_numpy(alb).cuda().requires_grad_(True)
    I = RenderAlbedo.apply(a, S, cams, st, opts)
    loss = ((I.double() - T.double()) ** 2).sum() / N
    loss.backward()
    g_ad = a.grad.cpu().numpy().astype(np.float64)
    h = 1e-2

    def loss_at(av):
        with torch.no_grad():
            Iv = RenderAlbedo.apply(torch.from_numpy(av).cuda(), S, cams, st, opts)
            return float(((Iv.double() - T.double()) ** 2).sum() / N)

    big = np.argsort(-np.abs(g_ad))[:200]
    worst = 0.0
    for f in rng.choice(big, 16, replace=False):
        ap = alb.copy()
        am = alb.copy()
        ap[f] += h
        am[f] -= h
        fd = (loss_at(ap) - loss_at(am)) / (2 * h)
        worst = max(worst, abs(fd - g_ad[f]) / abs(g_ad[f]))
    log(f"  autograd vs GPU finite differences: max rel {worst:.2e}")
    assert worst <= 1e-3


@pytest.mark.parametrize("sched", [rtq.SCHED_PERSISTENT, rtq.SCHED_MEGAKERNEL, rtq.SCHED_PLAIN])
def test_graph_replays_match_eager(sched):
    """Captured render calls (uneven views in one call): every replay, with other
    eager work and synchronisations between replays, equals the eager frame bit
    for bit; a new frame index changes the image; new cameras capture anew."""
    import torch
    log(f"case: graph replay, scheduler {sched}")
    scene, cams = _multi_view_scene()
    S = rtq.Scene(scene)
    st = sg.light_settings(2, 4, 77)
    kw = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=sched)
    eager = {}
    for f in range(4):
        st.frame = f
        eager[f] = _render(S, cams, st, **kw)
    assert not np.array_equal(eager[0], eager[1])
    other = sg.light_settings(1, 2, 5)
    n = sum(c.w * c.h for c in cams)
    img = torch.empty(n, device="cuda")
    for rep in range(3):
        for f in (0, 1, 2, 3, 1):
            st.frame = f
            rtq.render(S, cams, st, images=img, graph=True, **kw)
            torch.cuda.synchronize()
            got = img.cpu().numpy()
            assert np.array_equal(got.view(np.uint32), eager[f].view(np.uint32)), (rep, f)
            _render(S, cams[:1], other, **kw)  # eager work between replays
    # another camera set: a second graph, still equal to eager
    cams2 = cams[1:]
    st.frame = 2
    ref2 = _render(S, cams2, st, **kw)
    for _ in range(2):
        img2 = rtq.render(S, cams2, st, graph=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(img2.cpu().numpy().view(np.uint32), ref2.view(np.uint32))
    # timing of graph calls: whole calls only
    rtq.render_timing(S)
    for f in range(3):
        st.frame = f
        rtq.render(S, cams, st, images=img, graph=True, timing=True, **kw)
    t = rtq.render_timing(S)
    assert t["call"]["launches"] == 3 and t["call"]["ms"] > 0.0 and t["closest"]["launches"] == 0


def test_path_records_match_frame_and_oracle():
    """rtq_render_path traces one path alone: its radiance equals the frame's pixel
    bit for bit (1 spp), and its vertices (instance, primitive, half, shadow)
    equal the oracle's FP64 path up to the first vertex the oracle flags."""
    import torch
    log("case: path records, config 1")
    scene, cams, st = sg.config1()
    S = rtq.Scene(scene)
    o = oracle.OracleScene(scene)
    kw = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    st.frame = 3
    img = _render(S, cams, st, **kw)
    rng = np.random.default_rng(9)
    n_pix = cams[0].w * cams[0].h
    compared = 0
    pix = rng.choice(n_pix, size=256, replace=False)
    for p in pix:
        gv, gesc, grad = rtq.render_path(S, cams, st, 0, int(p), 0, **kw)
        assert np.float32(grad).view(np.uint32) == img[p].view(np.uint32), (p, grad, img[p])
        ov, oesc, pflags = o.path(cams, st, int(p), 0)
        if pflags:
            continue  # checked by the replay below
        assert len(gv) == len(ov) and gesc == oesc, (p, gv, ov)
        for x, y in zip(gv, ov):
            assert (x["inst"], x["prim"], x["half"], x["shadow"]) == (y["inst"], y["prim"], y["half"], y["shadow"])
            assert abs(x["t"] - y["t"]) <= 1e-5 * y["t"] or (y["flags"] & oracle.F_T_ILLCOND), (p, x, y)
            compared += 1
    log(f"  {compared} vertices of unflagged paths equal the oracle's")
    assert compared >= 64
    tot = replay_check_pixels(rtq, o, S, cams, st, pix, img, **kw)
    log(f"  every sampled path replayed and checked: {tot}")


def test_render_argument_errors():
    import torch
    scene, cams, st = sg.config1(n_inst=10)
    S = rtq.Scene(scene)
    bad = sg.RenderSettings(spp=1, depth=0)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, bad)
    bad = sg.RenderSettings(spp=0, depth=2)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, bad)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, [sg.Camera((0, 0, 0), (0, 0, 0), (0, 0, 1), 40.0, 8, 8)], st)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, sg.RenderSettings(spp=1, depth=17))
    # 2^31 paths in one call: LIMIT, checked before any scratch is allocated
    import ctypes
    big = [sg.Camera((0.0, -160.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 40.0, 65536, 32768)]
    arr, total = rtq.camera_structs(big)
    assert total == 2 ** 31
    img = torch.zeros(1, device="cuda")
    o = rtq.render_opts(st)
    rc = rtq.load_library().rtq_render(S.handle, ctypes.cast(arr, ctypes.c_void_p), 1, 1, 2, ctypes.byref(o),
                                       img.data_ptr(), None)
    assert rc == -5, rc
    torch.cuda.synchronize()


def test_config2_full_frame_bench_launch_vs_oracle():
    """The full-size config-2 frame (1M instances, two 1920x1080 views, depth 8)
    rendered the way the benchmark times it (quantized nodes, persistent
    wavefront, default launch, stage timing on): bit-identical to the FP32 plain
    frame and to a captured-graph replay; 256 sampled pixels match the oracle's
    FP64 paths; 64 sampled paths match the oracle vertex by vertex."""
    import torch
    log("case: config 2 full size, benchmark launch")
    scene, cams, st = sg.config2()
    S = rtq.Scene(scene)
    q8 = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    st.frame = 2
    a = _render(S, cams, st, timing=True, **q8)
    rtq.render_timing(S)
    b = _render(S, cams, st, node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "Q8 persistent and FP32 plain frames differ"
    g1 = _render(S, cams, st, graph=True, **q8)
    g2 = _render(S, cams, st, graph=True, **q8)
    assert np.array_equal(a.view(np.uint32), g1.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), g2.view(np.uint32))
    log("  frames bit-identical")
    o = oracle.OracleScene(scene)
    rng = np.random.default_rng(12)
    n_pix = sum(c.w * c.h for c in cams)
    pix = np.sort(rng.choice(n_pix, size=256, replace=False))
    ref, fl, _ = o.render(cams, st, pixels=pix)
    frac = _compare_image(a[pix], ref, fl)
    log(f"  256 sampled pixels, flagged {frac:.4f}")
    assert frac < 0.4
    tot = replay_check_pixels(rtq, o, S, cams, st, pix, a, **q8)
    log(f"  all 256 sampled pixels replayed and checked: {tot}")
    assert tot["vertices"] >= 256


def test_autotuner_quick_grid_keeps_images():
    """The autotuner times launch configurations and refuses any whose image
    differs from the FP32 plain one; on the quick grid every candidate passes
    and each (format, scheduler) pair gets a configuration."""
    from paper_2001_02620_amd.autotune import QUICK_GRID, autotune_render
    log("case: autotuner, quick grid, config 1")
    scene, cams, st = sg.config1()
    S = rtq.Scene(scene)
    res = autotune_render(S, cams, st, formats=(rtq.RTQ_NODE_Q8, rtq.RTQ_NODE_FP32),
                          schedulers=(rtq.SCHED_PERSISTENT, rtq.SCHED_PLAIN), grid=QUICK_GRID, reps=1, cache=None)
    for fmt in (rtq.RTQ_NODE_Q8, rtq.RTQ_NODE_FP32):
        for sch in (rtq.SCHED_PERSISTENT, rtq.SCHED_PLAIN):
            best = res[f"{fmt}/{sch}"]
            assert best["opts"]["node_format"] == fmt and best["opts"]["scheduler"] == sch and best["ms"] > 0
    assert len(res["table"]) >= 8
    log(f"  {len(res['table'])} candidates, all bit-identical")


@pytest.mark.parametrize("sched", [rtq.SCHED_PLAIN, rtq.SCHED_PERSISTENT, rtq.SCHED_MEGAKERNEL])
def test_view_completion_stamps_every_scheduler(sched):
    """Per-view completion stamps (the tick at which a view's last path ended)
    in every scheduler: each view gets a stamp after the call's start tick and
    no later than the end of the call, and the stamps do not change the image."""
    import torch
    log(f"case: view completion stamps, scheduler {sched}")
    scene, cams = _multi_view_scene()
    S = rtq.Scene(scene)
    st = sg.RenderSettings(spp=2, depth=5, seed=7)
    kw = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=sched)
    ref = _render(S, cams, st, **kw)
    done = torch.zeros(len(cams), dtype=torch.uint64, device="cuda")
    start = torch.zeros(1, dtype=torch.uint64, device="cuda")
    img = _render(S, cams, st, view_done=done, start_tick=start, **kw)
    after = torch.zeros(1, dtype=torch.uint64, device="cuda")
    _render(S, cams[:1], st, start_tick=after, **kw)  # a later call's start
    d = done.cpu().numpy().astype(np.int64)
    t0, t1 = int(start.cpu().item()), int(after.cpu().item())
    assert (d > t0).all() and (d <= t1).all(), (t0, d, t1)
    assert np.array_equal(img.view(np.uint32), ref.view(np.uint32))
    log(f"  view completion ticks after start: {d - t0}")
