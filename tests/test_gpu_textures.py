"""Per-face textures (Section 5.3) on the HIP path: every scheduler and node
format gives the same image, which matches the oracle's textured render on the
pixels it does not flag; a constant texture reproduces the per-face albedo
image bit for bit; removing textures restores it; the adjoint refuses a
textured scene."""
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
    frac = _compare_image(imgs[0], ref, fl, replay=(S, o, cams, st, SCHEDS[3]))
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
    grad = torch.ones(sum(c.w * c.h for c in cams), device="cuda")
    assert rtq.render_backward(S, cams, st, grad).numel() == scene.albedo.shape[0] * 16  # one entry per texel
    with pytest.raises(rtq.RtqError):
        S.set_textures(torch.zeros((scene.albedo.shape[0], 65, 65), device="cuda"))
    S.set_textures(None)
    rtq.render_backward(S, cams, st, grad)
    torch.cuda.synchronize()


def test_texel_adjoint_vs_oracle():
    """The adjoint of a textured scene is per texel: the GPU kernel takes each
    vertex's texel index at shading (before the shadow ray reuses the lane's
    (u, v)) and matches the oracle's pinned per-texel path-replay gradient,
    with flagged paths carrying zero pixel weight on both sides."""
    import torch
    log("case: per-texel adjoint")
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 64, 64)]
    st = sg.RenderSettings(spp=2, depth=4, seed=31)
    R = 4
    tex = _texels(scene.albedo.shape[0], R, 5)
    S = rtq.Scene(scene)
    S.set_textures(torch.from_numpy(tex).cuda())
    o = oracle.OracleScene(scene)
    o.set_textures(tex)
    ref, fl, _ = o.render(cams, st)
    gp = np.random.default_rng(3).normal(size=ref.shape)
    gp[fl != 0] = 0.0
    g_ref, _, taint = o.grad(cams, st, gp, taint="path")
    g = rtq.render_backward(S, cams, st, torch.from_numpy(gp.astype(np.float32)).cuda(),
                            node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    assert g.shape == g_ref.shape == (scene.albedo.shape[0] * R * R,)
    keep = taint == 0
    scale = np.abs(g_ref[keep]).max()
    err = np.abs(g[keep] - g_ref[keep])
    log(f"  texels {keep.sum()} of {keep.size}, {int((g_ref[keep] != 0).sum())} with a gradient, max |grad| "
        f"{scale:.4g}, max error {err.max():.3g}")
    assert scale > 0 and (err <= 2e-4 * scale + 1e-4 * np.abs(g_ref[keep])).all(), err.max()
    # texels no path reads get exactly zero on both sides
    assert (g[keep & (g_ref == 0)] == 0).all()
