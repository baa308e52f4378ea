"""Per-face textures (Section 5.3) on the HIP path: every scheduler and node
format gives the same image, which matches the oracle's textured render on the
pixels it does not flag; a constant texture reproduces the per-face albedo
image bit for bit; removing textures restores it; the adjoint of a textured
scene is per texel and matches the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import log
from tests.test_gpu_render import SCHEDS, _compare_image, _multi_view_scene, _render

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")


def _texels(n_faces, res, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 0.95, size=(n_faces, res, res)).astype(np.float32)


@pytest.mark.parametrize("cfg,res", [("config1", 2), ("multiview", 4), ("multiview", 1)])
def test_textured_schedulers_bit_identical_and_match_oracle(cfg, res):
    import torch
    log(f"case: textured render {cfg} res {res}")
    if cfg == "config1":
        scene, cams, st = sg.config1()
    else:
        scene, cams = _multi_view_scene()
        st = sg.RenderSettings(spp=3, depth=5, seed=77, frame=2)
    tex = _texels(scene.albedo.shape[0], res, 40 + res)
    S = rtq.Scene(scene)
    S.set_textures(torch.from_numpy(tex).cuda())
    imgs = []
    for kw in SCHEDS:
        log("  scheduler", kw)
        imgs.append(_render(S, cams, st, **kw))
    for img, kw in zip(imgs[1:], SCHEDS[1:]):
        assert (img.view(np.uint32) == imgs[0].view(np.uint32)).all(), f"textured image differs for {kw}"
    o = oracle.OracleScene(scene)
    o.set_textures(tex)
    ref, fl, _ = o.render(cams, st)
    frac = _compare_image(imgs[0], ref, fl)
    log(f"  flagged pixels {frac:.4f}")
    assert frac < 0.1
    # the texture changes the image (the texels are not the albedo)
    plain, _, _ = oracle.OracleScene(scene).render(cams, st)
    assert np.abs(ref - plain).mean() > 1e-3


def test_constant_textures_and_removal_keep_the_albedo_image():
    import torch
    log("case: constant textures")
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=2, depth=4, seed=5)
    S = rtq.Scene(scene)
    kws = [SCHEDS[0], SCHEDS[3], SCHEDS[5]]
    ref = [_render(S, cams, st, **kw) for kw in kws]
    for res in (1, 3):
        const = np.repeat(scene.albedo[:, None], res * res, axis=1).reshape(-1, res, res)
        S.set_textures(torch.from_numpy(const).cuda())
        for r, kw in zip(ref, kws):
            assert (_render(S, cams, st, **kw).view(np.uint32) == r.view(np.uint32)).all(), (res, kw)
    # a graph captured before the textures changed is not replayed after
    g0 = _render(S, cams, st, graph=True, **kws[1])
    assert (g0.view(np.uint32) == ref[1].view(np.uint32)).all()
    S.set_textures(torch.from_numpy(_texels(scene.albedo.shape[0], 2, 3)).cuda())
    eager = _render(S, cams, st, **kws[1])
    assert not np.array_equal(eager, ref[1])
    for _ in range(2):
        assert (_render(S, cams, st, graph=True, **kws[1]).view(np.uint32) == eager.view(np.uint32)).all()
    S.set_textures(None)
    for r, kw in zip(ref, kws):
        assert (_render(S, cams, st, **kw).view(np.uint32) == r.view(np.uint32)).all(), kw
    assert (_render(S, cams, st, graph=True, **kws[1]).view(np.uint32) == ref[1].view(np.uint32)).all()


def test_textured_path_records_and_errors():
    import torch
    log("case: textured path records and errors")
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=1, depth=3, seed=8)
    tex = _texels(scene.albedo.shape[0], 4, 9)
    S = rtq.Scene(scene)
    S.set_textures(torch.from_numpy(tex).cuda())
    o = oracle.OracleScene(scene)
    o.set_textures(tex)
    # a path's recorded shading value is a texel of the face it hit, the
    # oracle's texel wherever the oracle does not flag the vertex
    checked = exact = 0
    for g in range(0, cams[0].w * cams[0].h, 5):
        verts, _, _ = rtq.render_path(S, cams, st, 0, g, 0)
        ov, _, _ = o.path(cams, st, g, 0)
        for k, v in enumerate(verts):
            assert np.float32(v["albedo"]) in tex[v["face"]].ravel(), v
            checked += 1
            if k >= len(ov) or ov[k]["flags"] or ov[k]["shadow_flags"]:
                break
            assert (v["inst"], v["prim"], v["half"]) == (ov[k]["inst"], ov[k]["prim"], ov[k]["half"]), (g, k)
            assert v["albedo"] == ov[k]["albedo"], (g, k, v, ov[k])
            exact += 1
    assert checked > 10 and exact > 10
    from paper_2001_02620_amd.autograd import RenderAlbedo
    n = scene.albedo.shape[0]
    grad = torch.ones(sum(c.w * c.h for c in cams), device="cuda")
    assert rtq.render_backward(S, cams, st, grad).numel() == S.n_params == n * 16
    with pytest.raises(AssertionError):  # a per-face buffer is too small for texel gradients
        rtq.render_backward(S, cams, st, grad, grad_albedo=torch.zeros(n, device="cuda"))
    with pytest.raises(ValueError):
        RenderAlbedo.apply(torch.from_numpy(scene.albedo).cuda(), S, cams, st)
    with pytest.raises(rtq.RtqError):
        S.set_textures(torch.zeros((n, 65, 65), device="cuda"))
    S.set_textures(None)
    assert rtq.render_backward(S, cams, st, grad).numel() == n
    torch.cuda.synchronize()


def test_texel_adjoint_vs_oracle():
    """The adjoint of a textured scene accumulates per texel: against the
    oracle's path-replay texel gradient, both fed the same pixel weights with
    flagged pixels weighted zero."""
    import torch
    log("case: texel adjoint")
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 48, 48)]
    st = sg.RenderSettings(spp=4, depth=3, seed=31)
    R = 3
    tex = _texels(scene.albedo.shape[0], R, 13)
    rng = np.random.default_rng(9)
    o = oracle.OracleScene(scene)
    o.set_textures((tex + rng.uniform(-0.1, 0.1, tex.shape)).astype(np.float32))
    T, _, _ = o.render(cams, st)
    o.set_textures(tex)
    I, fl, _ = o.render(cams, st)
    gpix = (2 * (I - T) / I.size).astype(np.float32).astype(np.float64)
    gpix[fl != 0] = 0.0
    g_or, _, _ = o.grad(cams, st, gpix)
    S = rtq.Scene(scene)
    S.set_textures(torch.from_numpy(tex).cuda())
    for kw in (SCHEDS[0], SCHEDS[3]):
        g = rtq.render_backward(S, cams, st, torch.from_numpy(gpix.astype(np.float32)).cuda(), **kw)
        g = g.cpu().numpy().astype(np.float64)
        assert g.shape == g_or.shape
        mx = np.abs(g_or).max()
        big = np.nonzero(np.abs(g_or) > 1e-3 * mx)[0]
        assert big.size >= 16
        err = np.abs(g - g_or)
        log(f"  {kw}: {big.size} texels, max rel {(err[big] / np.abs(g_or[big])).max():.2e}")
        assert (err <= 1e-3 * np.abs(g_or) + 1e-5 * mx).all()
