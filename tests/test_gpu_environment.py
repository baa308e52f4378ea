"""Environment map seen by escaping rays on the HIP path, and sampled as a light
by next-event estimation: every scheduler and node format gives the same
image, equal to the oracle's on the pixels it does not flag (flagged ones
replayed path by path); texel orientation as the oracle's hand-worked cases; a
constant map is the constant sky bit for bit; the adjoint matches the oracle's
gradient with the map on, sampled or not."""
import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.gpu_util import log
from tests.test_gpu_render import SCHEDS, _compare_image, _multi_view_scene, _render

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")


def _env(w, h, seed):
    return np.random.default_rng(seed).uniform(0.05, 1.0, size=(h, w)).astype(np.float32)


@pytest.mark.parametrize("nee", [False, True])
def test_environment_schedulers_bit_identical_and_match_oracle(nee):
    """With and without next-event estimation toward the map (texels drawn from
    the 32-bit table, weighted against escaping bounce rays): every scheduler
    and node format gives the same image, equal to the oracle's where it flags
    nothing; flagged pixels are replayed and checked path by path."""
    import torch
    log(f"case: environment map, multiview, next-event estimation {nee}")
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=3, depth=5, seed=77, frame=2, env_nee=nee)
    env = _env(64, 32, 11)
    if nee:
        env[5:8, 20:26] = 30.0  # a small bright region the sampling finds
    S = rtq.Scene(scene)
    S.set_environment(torch.from_numpy(env).cuda())
    imgs = [_render(S, cams, st, **kw) for kw in SCHEDS]
    for img, kw in zip(imgs[1:], SCHEDS[1:]):
        assert (img.view(np.uint32) == imgs[0].view(np.uint32)).all(), f"image differs for {kw}"
    for _ in range(2):
        g = _render(S, cams, st, graph=True, **SCHEDS[3])
        assert (g.view(np.uint32) == imgs[0].view(np.uint32)).all()
    o = oracle.OracleScene(scene)
    o.set_environment(env)
    ref, fl, _ = o.render(cams, st)
    frac = _compare_image(imgs[0], ref, fl, replay=(S, o, cams, st, SCHEDS[3]))
    log(f"  flagged pixels {frac:.4f}")
    assert frac < 0.1
    plain, _, _ = oracle.OracleScene(scene).render(cams, st)
    assert np.abs(ref - plain).mean() > 1e-2 * np.abs(plain).mean()


def test_environment_orientation_and_constant_map_gpu():
    import torch
    log("case: environment orientation")
    empty = ts.multi_mesh_scene([ts.axis_quad(-1, 1, -1, 1, 0.0)], xforms=[[1, 0, 0, 0, 0, 1, 0, 500, 0, 0, 1, 0]])
    env = (np.arange(32, dtype=np.float32) + 1.0).reshape(4, 8)
    S = rtq.Scene(empty)
    S.set_environment(torch.from_numpy(env).cuda())
    st = sg.RenderSettings(spp=2, depth=2, seed=3)
    cases = [((1.0, 0.2, 0.3), (4, 1)), ((-1.0, -0.2, -0.3), (0, 2)), ((0.2, 1.0, -0.3), (5, 2)),
             ((0.05, -0.1, 1.0), (2, 0))]
    for d, (tx, ty) in cases:
        up = (0.0, 0.0, 1.0) if abs(d[2]) < 0.9 else (0.0, 1.0, 0.0)
        cams = [sg.Camera((0.0, 0.0, 0.0), d, up, 0.01, 4, 4)]
        for kw in (SCHEDS[0], SCHEDS[5]):
            assert (_render(S, cams, st, **kw) == env[ty, tx]).all(), (d, kw)
    # a constant map equal to L_sky is the constant sky, bit for bit
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=2, depth=4, seed=5)
    S = rtq.Scene(scene)
    ref = [_render(S, cams, st, **kw) for kw in (SCHEDS[0], SCHEDS[3], SCHEDS[5])]
    S.set_environment(torch.full((5, 9), st.L_sky, device="cuda"))
    for r, kw in zip(ref, (SCHEDS[0], SCHEDS[3], SCHEDS[5])):
        assert (_render(S, cams, st, **kw).view(np.uint32) == r.view(np.uint32)).all(), kw
    S.set_environment(None)
    assert (_render(S, cams, st, **SCHEDS[3]).view(np.uint32) == ref[1].view(np.uint32)).all()
    with pytest.raises(rtq.RtqError):
        S.set_environment(torch.zeros((2, 16385), device="cuda"))


@pytest.mark.parametrize("nee", [False, True])
def test_environment_adjoint_vs_oracle(nee):
    import torch
    log(f"case: environment adjoint, next-event estimation {nee}")
    scene = sg.tiny_scene(31, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 48, 48)]
    st = sg.RenderSettings(spp=4, depth=3, seed=31, env_nee=nee)
    env = _env(32, 16, 12)
    rng = np.random.default_rng(8)
    alb = scene.albedo.astype(np.float32)
    tgt = (alb + rng.uniform(-0.1, 0.1, alb.shape)).astype(np.float32)
    o = oracle.OracleScene(scene)
    o.set_environment(env)
    o.set_albedo(tgt.astype(np.float64))
    T, _, _ = o.render(cams, st)
    o.set_albedo(alb.astype(np.float64))
    I, fl, _ = o.render(cams, st)
    gpix = (2 * (I - T) / I.size).astype(np.float32).astype(np.float64)
    gpix[fl != 0] = 0.0
    g_or, _, _ = o.grad(cams, st, gpix)
    S = rtq.Scene(scene)
    S.set_environment(torch.from_numpy(env).cuda())
    for kw in (SCHEDS[0], SCHEDS[3]):
        g = rtq.render_backward(S, cams, st, torch.from_numpy(gpix.astype(np.float32)).cuda(), **kw)
        g = g.cpu().numpy().astype(np.float64)
        mx = np.abs(g_or).max()
        faces = np.nonzero(np.abs(g_or) > 1e-3 * mx)[0]
        assert faces.size >= 8
        err = np.abs(g[faces] - g_or[faces])
        log(f"  {kw}: {faces.size} faces, max rel {(err / np.abs(g_or[faces])).max():.2e}")
        assert (err <= 1e-3 * np.abs(g_or[faces]) + 1e-5 * mx).all()
