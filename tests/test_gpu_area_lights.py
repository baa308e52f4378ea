"""Quad area lights in next-event estimation on the HIP path: every scheduler
and node format gives the same image, equal to the oracle's on the pixels it
does not flag; paths (hits and shadow outcomes) match the oracle's; the
view-factor closed form and the shadow segment hold on the GPU; the adjoint
matches the oracle's path-replay gradient with area lights on."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import log, replay_check_pixels
from tests.test_gpu_render import SCHEDS, _compare_image, _multi_view_scene, _render
from tests.test_oracle_pins import AREA_LIGHTS, _area_setup

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

LIGHTS = ((-3.0, -3.0, 6.0, 0.0, 6.0, 0.0, 6.0, 0.0, 0.0, 1.5),
          (5.0, -2.0, -2.0, 0.0, 0.0, 4.0, 0.0, 4.0, 0.0, 3.0),
          (-1.0, -9.0, 3.0, 2.0, 0.0, 0.0, 0.0, 0.0, 1.0, 4.0))


def test_area_lights_schedulers_bit_identical_and_match_oracle():
    import torch
    log("case: area lights, multiview")
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=3, depth=5, seed=77, frame=2, area_lights=LIGHTS)
    S = rtq.Scene(scene)
    imgs = []
    for kw in SCHEDS:
        log("  scheduler", kw)
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        imgs.append((_render(S, cams, st, counters=cnt, **kw), cnt.cpu().numpy()))
    for (img, cnt), kw in zip(imgs[1:], SCHEDS[1:]):
        assert (img.view(np.uint32) == imgs[0][0].view(np.uint32)).all(), f"image differs for {kw}"
        assert (cnt == imgs[0][1]).all(), kw
    g = _render(S, cams, st, graph=True, **SCHEDS[3])
    assert (g.view(np.uint32) == imgs[0][0].view(np.uint32)).all()
    o = oracle.OracleScene(scene)
    ref, fl, stats = o.render(cams, st)
    frac = _compare_image(imgs[0][0], ref, fl, replay=(S, o, cams, st, SCHEDS[3]))
    log(f"  flagged pixels {frac:.4f}; gpu rays {imgs[0][1]}; oracle {stats}")
    assert frac < 0.1
    if frac == 0.0:
        assert imgs[0][1][1] == stats["shadow"]
    plain, _, _ = o.render(cams, dataclasses.replace(st, area_lights=()))
    assert np.abs(ref - plain).mean() > 1e-2 * np.abs(plain).mean()
    rng = np.random.default_rng(5)
    pix = rng.choice(ref.size, 256, replace=False)
    for kw in (SCHEDS[0], SCHEDS[3]):
        # many pixels of these views see no geometry: 256 pixels give a few hundred vertices
        tot = replay_check_pixels(rtq, o, S, cams, st, pix, imgs[0][0], **kw)
        log(f"  256 pixels replayed and checked: {tot}")
        assert tot["vertices"] > 80


def test_area_light_floor_closed_form_and_segment_gpu():
    log("case: area light closed form")
    half, h = 0.4, 1.0
    for E in (0.0, math.pi):
        scene, cams, st, a_f = _area_setup(E, half, h)
        S = rtq.Scene(scene)
        img = np.concatenate([_render(S, cams, dataclasses.replace(st, seed=st.seed + k), **SCHEDS[3])
                              for k in range(4)])
        F = 4 * ts.form_factor_corner(half, half, h)
        expect = a_f * ((E / math.pi) * st.light_dir[2] + F)
        se = img.std() / math.sqrt(img.size)
        assert abs(img.mean() - expect) < 5 * se, (E, img.mean(), expect, se)
    below = ts.axis_quad(-3.0, 3.5, -3.0, 4.0, 0.75)
    scene, cams, st, _ = _area_setup(0.0, extra=[(below, 0.5)])
    for kw in (SCHEDS[0], SCHEDS[3], SCHEDS[5]):
        assert (_render(rtq.Scene(scene), cams, st, **kw) == 0.0).all(), kw


def test_area_light_adjoint_vs_oracle():
    import torch
    log("case: area light adjoint")
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 48, 48)]
    st = sg.RenderSettings(spp=4, depth=3, seed=31, area_lights=AREA_LIGHTS)
    rng = np.random.default_rng(7)
    alb = scene.albedo.astype(np.float32)
    tgt = (alb + rng.uniform(-0.1, 0.1, alb.shape)).astype(np.float32)
    o = oracle.OracleScene(scene)
    o.set_albedo(tgt.astype(np.float64))
    T, _, _ = o.render(cams, st)
    o.set_albedo(alb.astype(np.float64))
    I, fl, _ = o.render(cams, st)
    gpix = (2 * (I - T) / I.size).astype(np.float32).astype(np.float64)
    gpix[fl != 0] = 0.0
    g_or, _, _ = o.grad(cams, st, gpix)
    S = rtq.Scene(scene)
    for kw in (SCHEDS[0], SCHEDS[3]):
        g = rtq.render_backward(S, cams, st, torch.from_numpy(gpix.astype(np.float32)).cuda(), **kw)
        g = g.cpu().numpy().astype(np.float64)
        mx = np.abs(g_or).max()
        faces = np.nonzero(np.abs(g_or) > 1e-3 * mx)[0]
        assert faces.size >= 8
        # FP32 atomics against FP64 sums: 1e-3 relative, plus 1e-5 of the largest
        # gradient for faces whose terms cancel
        err = np.abs(g[faces] - g_or[faces])
        log(f"  {kw}: {faces.size} faces, max rel {(err / np.abs(g_or[faces])).max():.2e}")
        assert (err <= 1e-3 * np.abs(g_or[faces]) + 1e-5 * mx).all()


def test_area_light_argument_errors():
    import torch
    scene, cams = _multi_view_scene()
    S = rtq.Scene(scene)
    bad = ((0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, float("nan")),)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, sg.RenderSettings(spp=1, depth=2, area_lights=bad))
    many = tuple((0.0, 0.0, 1.0 + k, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 1.0) for k in range(65))
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, sg.RenderSettings(spp=1, depth=2, area_lights=many))
    torch.cuda.synchronize()
