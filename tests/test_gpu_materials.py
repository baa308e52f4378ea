"""Principled materials in three channels on the GPU (Section 5.4: Disney's
principled BSDF, energy conserving and preserving), against the oracle:
every scheduler and graph replay give bit-identical RGB images; unflagged
pixels match the oracle's FP64 values and every flagged pixel is replayed path
by path; the adjoint matches the oracle's gradient; a white furnace stays at
the sky radiance; argument errors are reported."""
import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import log, replay_check_pixels

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

SCHEDS = [dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
          dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
          dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL),
          dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)]

# rough and smooth dielectrics, metals, a Lambertian one
MATS = np.array([(0.9, 0.6, 0.3, 0.5, 0.0, 0.8), (0.4, 0.7, 0.9, 0.35, 0.7, 0.2),
                 (0.8, 0.8, 0.8, 0.9, 0.2, 0.5), (0.95, 0.85, 0.6, 0.08, 1.0, 0.0),
                 (0.3, 0.5, 0.2, 1.0, 0.0, 0.0), (1.0, 1.0, 1.0, 0.15, 0.0, 1.0)], np.float32)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _materials(n_quads, seed=3):
    return np.random.default_rng(seed).integers(0, MATS.shape[0], n_quads).astype(np.uint8)


def _compare_rgb(gpu, ref, flags, replay, rel=1e-4):
    """Unflagged pixels: every channel within rel of the pixel's largest FP64
    channel; flagged pixels: replayed path by path."""
    ok = flags == 0
    err = np.abs(gpu.astype(np.float64) - ref)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    bad = ok[:, None] & (err > rel * scale + 1e-7)
    if bad.any():
        k = np.nonzero(bad.any(axis=1))[0][:8]
        raise AssertionError(f"{bad.any(axis=1).sum()} unflagged pixels differ: idx {k} gpu {gpu[k]} oracle {ref[k]}")
    S, osc, cams, st, kw = replay
    idx = np.nonzero(~ok)[0]
    tot = replay_check_pixels(rtq, osc, S, cams, st, idx, gpu, **kw)
    log(f"  replayed {idx.size} flagged pixels: {tot}")
    return 1.0 - ok.mean()


def _setup(cfg):
    if cfg == "config1":
        scene, cams, st = sg.config1()
    else:
        scene = sg.tiny_scene(21, n_inst=24, n_protos=3, nq=8, spread=3.0)
        cams = [sg.Camera((0.0, -12.0, 2.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 45.0, 37, 23),
                sg.Camera((9.0, 4.0, 6.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 64, 64)]
        st = sg.RenderSettings(spp=3, depth=5, seed=77, frame=2)
    return scene, cams, st


@pytest.mark.parametrize("cfg,lights", [("config1", "sun"), ("multiview", "area+env")])
def test_materials_schedulers_bit_identical_and_match_oracle(cfg, lights):
    import torch
    log(f"case: principled materials, {cfg}, {lights}")
    scene, cams, st = _setup(cfg)
    fm = _materials(scene.n_quads)
    S = rtq.Scene(scene)
    S.set_materials(MATS, torch.from_numpy(fm).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(MATS, fm.astype(np.int32))
    if lights == "area+env":
        st.area_lights = ((-4.0, -4.0, 8.0, 0.0, 8.0, 0.0, 8.0, 0.0, 0.0, 3.0),)
        env = np.random.default_rng(4).uniform(0.0, 1.0, size=(16, 32)).astype(np.float32)
        S.set_environment(torch.from_numpy(env).cuda())
        o.set_environment(env)
        st.env_nee = True
    imgs = []
    for kw in SCHEDS:
        imgs.append(_np(rtq.render(S, cams, st, **kw)))
    g = _np(rtq.render(S, cams, st, graph=True, **SCHEDS[3]))
    g2 = _np(rtq.render(S, cams, st, graph=True, **SCHEDS[3]))
    ref_img = imgs[0]
    assert ref_img.shape == (sum(c.w * c.h for c in cams), 3)
    for img, kw in zip(imgs[1:] + [g, g2], SCHEDS[1:] + ["graph", "graph replay"]):
        assert (img.view(np.uint32) == ref_img.view(np.uint32)).all(), f"image differs for {kw}"
    assert not np.allclose(ref_img[:, 0], ref_img[:, 2])
    ref, fl, _ = o.render(cams, st)
    frac = _compare_rgb(ref_img, ref, fl, (S, o, cams, st, SCHEDS[3]))
    log(f"  flagged pixels {frac:.4f}")
    assert frac < 0.15


def test_materials_white_furnace_floor():
    """A white floor (c = 1) of each material under the sky, no sun: every
    path's weight is one, so every pixel and channel is L_sky to FP32 rounding."""
    import torch
    scene = ts.floor_scene(albedo=1.0)
    cams = [sg.Camera((1.0, -2.0, 10.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 24, 24)]
    st = sg.RenderSettings(spp=2, depth=3, seed=7)
    st.E = 0.0
    S = rtq.Scene(scene)
    for m in MATS:
        white = np.array([(1.0, 1.0, 1.0) + tuple(m[3:])], np.float32)
        S.set_materials(white, torch.zeros(scene.n_quads, dtype=torch.uint8, device="cuda"))
        img = _np(rtq.render(S, cams, st, **SCHEDS[3]))
        np.testing.assert_allclose(img, st.L_sky, rtol=2e-6)


@pytest.mark.parametrize("env", [False, True])
def test_materials_adjoint_vs_oracle(env):
    """The RGB adjoint (per-vertex estimates and bounce weights, affine in the
    face's albedo) against the oracle's path-replay gradient, with RGB pixel
    weights; flagged pixels carry zero weight on both sides."""
    import torch
    log(f"case: principled adjoint, environment {env}")
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 48, 48)]
    st = sg.RenderSettings(spp=2, depth=4, seed=31)
    fm = _materials(scene.n_quads, seed=9)
    S = rtq.Scene(scene)
    S.set_materials(MATS, torch.from_numpy(fm).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(MATS, fm.astype(np.int32))
    if env:
        emap = np.random.default_rng(8).uniform(0.0, 1.0, size=(8, 16)).astype(np.float32)
        S.set_environment(torch.from_numpy(emap).cuda())
        o.set_environment(emap)
        st.env_nee = True
    ref, fl, _ = o.render(cams, st)
    rng = np.random.default_rng(2)
    gp = rng.normal(size=ref.shape)
    gp[fl != 0] = 0.0
    g_ref, _, taint = o.grad(cams, st, gp, taint="path")
    gpu_g = _np(rtq.render_backward(S, cams, st, torch.from_numpy(gp.astype(np.float32)).cuda(), **SCHEDS[3]))
    keep = taint == 0
    scale = np.abs(g_ref[keep]).max()
    err = np.abs(gpu_g[keep] - g_ref[keep])
    log(f"  faces {keep.sum()} of {keep.size}, max |grad| {scale:.4g}, max error {err.max():.3g}")
    assert (err <= 2e-4 * scale + 1e-4 * np.abs(g_ref[keep])).all(), err.max()
    assert np.abs(g_ref[keep]).max() > 0


def test_materials_argument_errors():
    import torch
    scene = sg.tiny_scene(2, n_inst=2, n_protos=1, nq=4, spread=1.0)
    S = rtq.Scene(scene)
    fm = torch.zeros(scene.n_quads, dtype=torch.uint8, device="cuda")
    for bad in ([(1.2, 0.5, 0.5, 0.5, 0.0, 0.0)], [(0.5, 0.5, 0.5, 0.01, 0.0, 0.0)],
                [(0.5, 0.5, 0.5, 0.5, 1.5, 0.0)], [(0.5, 0.5, 0.5, 0.5, 0.0, -0.1)]):
        with pytest.raises(rtq.RtqError):
            S.set_materials(np.array(bad, np.float32), fm)
    with pytest.raises(rtq.RtqError):
        S.set_materials(MATS[:2], torch.full((scene.n_quads,), 2, dtype=torch.uint8, device="cuda"))
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 8, 8)]
    st = sg.RenderSettings(spp=1, depth=2, seed=1)
    img1 = _np(rtq.render(S, cams, st))
    assert img1.shape == (64,)
    S.set_materials(MATS, fm)
    # a one-channel buffer for a scene with materials is refused by the library
    o = rtq.render_opts(st)
    arr, _ = rtq.camera_structs(cams)
    buf = torch.empty(64 * 3, device="cuda")
    import ctypes
    rc = rtq.load_library().rtq_render(S.handle, ctypes.cast(arr, ctypes.c_void_p), 1, 1, 2, ctypes.byref(o),
                                       buf.data_ptr(), rtq._stream())
    assert rc != 0
    img3 = _np(rtq.render(S, cams, st))
    assert img3.shape == (64, 3)
    S.set_materials(None)
    assert _np(rtq.render(S, cams, st)).shape == (64,)
