"""RGB per-face textures on the HIP path (Section 5.3: the scene's Ptex textures
hold the materials' colors): with materials, channel k of the base color is
the material's tint_k times channel k of the nearest texel.  Every scheduler
and graph replay give bit-identical images that match the oracle (flagged
pixels replayed path by path); texels with three equal channels render as the
scalar texture bit for bit; the adjoint is per texel channel and matches the
oracle; RGB texels without materials and other channel counts are refused."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import log
from tests.test_gpu_materials import SCHEDS, _compare_rgb, _materials, _np, _setup
from tests.test_gpu_clearcoat import COAT_MATS

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")


def _rgb_texels(n_faces, res, seed):
    return np.random.default_rng(seed).uniform(0.05, 0.95, size=(n_faces, res, res, 3)).astype(np.float32)


@pytest.mark.parametrize("cfg,lights,res", [("config1", "sun", 2), ("multiview", "area+env", 4)])
def test_rgb_textures_schedulers_bit_identical_and_match_oracle(cfg, lights, res):
    import torch
    log(f"case: RGB textures, {cfg}, {lights}, res {res}")
    scene, cams, st = _setup(cfg)
    fm = _materials(scene.n_quads)
    tex = _rgb_texels(scene.n_quads, res, 50 + res)
    S = rtq.Scene(scene)
    S.set_materials(COAT_MATS, torch.from_numpy(fm).cuda())
    S.set_textures(torch.from_numpy(tex).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(COAT_MATS, fm.astype(np.int32))
    o.set_textures(tex)
    if lights == "area+env":
        st.area_lights = ((-4.0, -4.0, 8.0, 0.0, 8.0, 0.0, 8.0, 0.0, 0.0, 3.0),)
        env = np.random.default_rng(4).uniform(0.0, 1.0, size=(16, 32)).astype(np.float32)
        S.set_environment(torch.from_numpy(env).cuda())
        o.set_environment(env)
        st.env_nee = True
    imgs = [_np(rtq.render(S, cams, st, **kw)) for kw in SCHEDS]
    g = _np(rtq.render(S, cams, st, graph=True, **SCHEDS[3]))
    g2 = _np(rtq.render(S, cams, st, graph=True, **SCHEDS[3]))
    ref_img = imgs[0]
    for img, kw in zip(imgs[1:] + [g, g2], SCHEDS[1:] + ["graph", "graph replay"]):
        assert (img.view(np.uint32) == ref_img.view(np.uint32)).all(), f"image differs for {kw}"
    ref, fl, _ = o.render(cams, st)
    frac = _compare_rgb(ref_img, ref, fl, (S, o, cams, st, SCHEDS[3]))
    log(f"  flagged pixels {frac:.4f}")
    assert frac < 0.15
    # the channels differ from the scalar texture of any one channel
    S.set_textures(torch.from_numpy(tex[..., 0].copy()).cuda())
    assert not np.array_equal(_np(rtq.render(S, cams, st, **SCHEDS[3])), ref_img)


def test_equal_channels_render_as_the_scalar_texture():
    import torch
    scene, cams, st = _setup("multiview")
    fm = torch.from_numpy(_materials(scene.n_quads)).cuda()
    scalar = _rgb_texels(scene.n_quads, 3, 8)[..., 2].copy()
    S = rtq.Scene(scene)
    S.set_materials(COAT_MATS, fm)
    S.set_textures(torch.from_numpy(scalar).cuda())
    a = _np(rtq.render(S, cams, st, **SCHEDS[3]))
    S.set_textures(torch.from_numpy(np.repeat(scalar[..., None], 3, axis=-1)).cuda())
    b = _np(rtq.render(S, cams, st, **SCHEDS[3]))
    assert (a.view(np.uint32) == b.view(np.uint32)).all()


def test_rgb_texel_adjoint_vs_oracle():
    """The adjoint of an RGB-textured scene is per texel channel (index
    3 texel + channel) and matches the oracle's path-replay gradient, flagged
    paths carrying zero pixel weight on both sides."""
    import torch
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 64, 64)]
    st = sg.RenderSettings(spp=2, depth=4, seed=31)
    R = 3
    fm = _materials(scene.n_quads, seed=9)
    tex = _rgb_texels(scene.n_quads, R, 6)
    S = rtq.Scene(scene)
    S.set_materials(COAT_MATS, torch.from_numpy(fm).cuda())
    S.set_textures(torch.from_numpy(tex).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(COAT_MATS, fm.astype(np.int32))
    o.set_textures(tex)
    ref, fl, _ = o.render(cams, st)
    gp = np.random.default_rng(3).normal(size=ref.shape)
    gp[fl != 0] = 0.0
    g_ref, _, taint = o.grad(cams, st, gp, taint="path")
    g = _np(rtq.render_backward(S, cams, st, torch.from_numpy(gp.astype(np.float32)).cuda(), **SCHEDS[3]))
    g = g.astype(np.float64)
    assert g.shape == g_ref.shape == (scene.n_quads * R * R * 3,)
    keep = taint == 0
    scale = np.abs(g_ref[keep]).max()
    err = np.abs(g[keep] - g_ref[keep])
    log(f"  texel channels {keep.sum()} of {keep.size}, max |grad| {scale:.4g}, max error {err.max():.3g}")
    assert scale > 0 and (err <= 2e-4 * scale + 1e-4 * np.abs(g_ref[keep])).all(), err.max()
    assert (g[keep & (g_ref == 0)] == 0).all()


def test_rgb_texture_errors():
    import torch
    scene = sg.tiny_scene(2, n_inst=2, n_protos=1, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 8, 8)]
    st = sg.RenderSettings(spp=1, depth=2, seed=1)
    S = rtq.Scene(scene)
    tex = torch.full((scene.n_quads, 2, 2, 3), 0.5, device="cuda")
    S.set_textures(tex)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, st)
    S.set_materials(COAT_MATS[:1], torch.zeros(scene.n_quads, dtype=torch.uint8, device="cuda"))
    assert _np(rtq.render(S, cams, st)).shape == (64, 3)
    L = rtq.load_library()
    assert L.rtq_scene_set_textures(S.handle, ctypes.c_void_p(tex.data_ptr()), 2, 2, rtq._stream()) != 0
