"""The clearcoat layer of the principled BSDF on the GPU (Section 5.4: the
scene's materials use Disney's principled BSDF; its coat is read as a second
mirrored visible-normal lobe over the base, weighted by the coat's Fresnel
term), against the oracle: every scheduler and graph replay give bit-identical
RGB images that match the oracle (flagged pixels replayed path by path); a
zero coat leaves images bit for bit as without it; a white coated floor stays
at the sky radiance; the adjoint matches the oracle's gradient; out-of-range
coat parameters are refused."""
import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import log
from tests.test_gpu_materials import MATS, SCHEDS, _compare_rgb, _materials, _np, _setup

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

# the base materials with a coat each: full and smooth, half and rough, none,
# a light one over a smooth metal, a full one over Lambert, a rough one
COATS = np.array([(1.0, 0.2), (0.5, 0.6), (0.0, 0.0), (0.3, 0.1), (1.0, 0.35), (0.8, 0.9)], np.float32)
COAT_MATS = np.concatenate([MATS, COATS], axis=1)


@pytest.mark.parametrize("cfg,lights", [("config1", "sun"), ("multiview", "area+env")])
def test_clearcoat_schedulers_bit_identical_and_match_oracle(cfg, lights):
    import torch
    log(f"case: clearcoat materials, {cfg}, {lights}")
    scene, cams, st = _setup(cfg)
    fm = _materials(scene.n_quads)
    S = rtq.Scene(scene)
    S.set_materials(COAT_MATS, torch.from_numpy(fm).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(COAT_MATS, fm.astype(np.int32))
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
    # the coat changes the image
    S.set_materials(MATS, torch.from_numpy(fm).cuda())
    assert not np.array_equal(_np(rtq.render(S, cams, st, **SCHEDS[3])), ref_img)


def test_zero_coat_is_bit_identical_to_no_coat():
    """Rows with clearcoat = 0 (any coat roughness) render bit for bit as the
    six-parameter rows."""
    import torch
    scene, cams, st = _setup("multiview")
    fm = torch.from_numpy(_materials(scene.n_quads)).cuda()
    S = rtq.Scene(scene)
    S.set_materials(MATS, fm)
    a = _np(rtq.render(S, cams, st, **SCHEDS[3]))
    zero = np.concatenate([MATS, np.tile(np.float32([0.0, 0.7]), (MATS.shape[0], 1))], axis=1)
    S.set_materials(zero, fm)
    b = _np(rtq.render(S, cams, st, **SCHEDS[3]))
    assert (a.view(np.uint32) == b.view(np.uint32)).all()


def test_clearcoat_white_furnace_floor():
    """A white coated floor under the sky, no sun: every path's weight is one,
    so every pixel and channel is L_sky to FP32 rounding."""
    import torch
    scene = ts.floor_scene(albedo=1.0)
    cams = [sg.Camera((1.0, -2.0, 10.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 24, 24)]
    st = sg.RenderSettings(spp=2, depth=3, seed=7)
    st.E = 0.0
    S = rtq.Scene(scene)
    for m in COAT_MATS:
        white = np.array([(1.0, 1.0, 1.0) + tuple(m[3:])], np.float32)
        S.set_materials(white, torch.zeros(scene.n_quads, dtype=torch.uint8, device="cuda"))
        img = _np(rtq.render(S, cams, st, **SCHEDS[3]))
        np.testing.assert_allclose(img, st.L_sky, rtol=2e-6)


def test_clearcoat_adjoint_vs_oracle():
    """The RGB adjoint with coated materials (the coat's lobe choice does not
    depend on the albedo, so each vertex stays affine in it) against the
    oracle's path-replay gradient; flagged pixels carry zero weight."""
    import torch
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 48, 48)]
    st = sg.RenderSettings(spp=2, depth=4, seed=31)
    fm = _materials(scene.n_quads, seed=9)
    S = rtq.Scene(scene)
    S.set_materials(COAT_MATS, torch.from_numpy(fm).cuda())
    o = oracle.OracleScene(scene)
    o.set_materials(COAT_MATS, fm.astype(np.int32))
    ref, fl, _ = o.render(cams, st)
    gp = np.random.default_rng(2).normal(size=ref.shape)
    gp[fl != 0] = 0.0
    g_ref, _, taint = o.grad(cams, st, gp, taint="path")
    gpu_g = _np(rtq.render_backward(S, cams, st, torch.from_numpy(gp.astype(np.float32)).cuda(), **SCHEDS[3]))
    keep = taint == 0
    scale = np.abs(g_ref[keep]).max()
    err = np.abs(gpu_g[keep] - g_ref[keep])
    log(f"  faces {keep.sum()} of {keep.size}, max |grad| {scale:.4g}, max error {err.max():.3g}")
    assert (err <= 2e-4 * scale + 1e-4 * np.abs(g_ref[keep])).all(), err.max()


def test_clearcoat_argument_errors():
    import torch
    scene = sg.tiny_scene(2, n_inst=2, n_protos=1, nq=4, spread=1.0)
    S = rtq.Scene(scene)
    fm = torch.zeros(scene.n_quads, dtype=torch.uint8, device="cuda")
    for bad in ([(0.5, 0.5, 0.5, 0.5, 0.0, 0.0, 1.2, 0.5)], [(0.5, 0.5, 0.5, 0.5, 0.0, 0.0, -0.1, 0.5)],
                [(0.5, 0.5, 0.5, 0.5, 0.0, 0.0, 0.5, 0.01)], [(0.5, 0.5, 0.5, 0.5, 0.0, 0.0, 0.5, 1.5)]):
        with pytest.raises(rtq.RtqError):
            S.set_materials(np.array(bad, np.float32), fm)
    with pytest.raises(ValueError):
        S.set_materials(np.zeros((1, 7), np.float32), fm)
    # without a coat its roughness is not read
    S.set_materials(np.array([(0.5, 0.5, 0.5, 0.5, 0.0, 0.0, 0.0, 0.0)], np.float32), fm)
