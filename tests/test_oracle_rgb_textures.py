"""Pins of the oracle's RGB per-face textures (Section 5.3: the scene's Ptex
textures hold the materials' colors; here synthetic res x res texels of three
channels per quad, read at the nearest texel of the hit's (face, u, v)).  With
materials, channel c of the base color is the material's tint times channel c
of the texel; each texel channel is a shading parameter of its own."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts

MATS = np.array([(0.9, 0.6, 0.3, 0.5, 0.0, 0.8, 0.5, 0.4), (0.4, 0.7, 0.9, 0.35, 0.7, 0.2, 0.0, 0.0),
                 (0.8, 0.8, 0.8, 0.9, 0.2, 0.5, 1.0, 0.3)], np.float32)


def _setup(seed=31, res=3):
    scene = sg.tiny_scene(seed, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 12, 12)]
    st = sg.RenderSettings(spp=2, depth=4, seed=seed)
    fm = (np.arange(scene.n_quads) % 3).astype(np.int32)
    o = oracle.OracleScene(scene)
    o.set_materials(MATS, fm)
    tex = np.random.default_rng(seed).uniform(0.05, 0.95, size=(scene.n_quads, res, res, 3)).astype(np.float32)
    return scene, cams, st, o, tex


def test_equal_channels_render_as_the_scalar_texture():
    """RGB texels whose three channels hold one value render exactly as the
    scalar texture of that value, and so does their gradient."""
    scene, cams, st, o, tex = _setup()
    scalar = tex[..., 1]
    o.set_textures(scalar)
    a, fa, _ = o.render(cams, st)
    g = np.random.default_rng(4).normal(size=a.shape)
    ga, _, _ = o.grad(cams, st, g)
    o.set_textures(np.repeat(scalar[..., None], 3, axis=-1))
    b, fb, _ = o.render(cams, st)
    gb, _, _ = o.grad(cams, st, g)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    # the scalar texel's gradient is the sum over its three channels
    assert o.n_params == 3 * ga.shape[0]
    np.testing.assert_allclose(gb.reshape(-1, 3).sum(axis=1), ga, rtol=1e-12, atol=1e-15)


def test_channels_are_independent():
    """Changing one channel of every texel changes that channel of the image
    and leaves the other two bit for bit."""
    scene, cams, st, o, tex = _setup(seed=7)
    o.set_textures(tex)
    a, _, _ = o.render(cams, st)
    t2 = tex.copy()
    t2[..., 1] = np.float32(0.5) * t2[..., 1]
    o.set_textures(t2)
    b, _, _ = o.render(cams, st)
    assert np.array_equal(a[:, 0], b[:, 0]) and np.array_equal(a[:, 2], b[:, 2])
    assert np.abs(a[:, 1] - b[:, 1]).max() > 1e-3


def test_rgb_texture_floor_closed_form():
    """A Lambertian white-tint floor with one RGB color t in every texel, under
    the sun and the sky, depth 2: channel k of every pixel is
    t_k (E / pi) cos_L + t_k L_sky."""
    scene = ts.floor_scene(albedo=0.5)
    o = oracle.OracleScene(scene)
    o.set_materials(np.array([(1.0, 1.0, 1.0, 0.5, 0.0, 0.0)], np.float32), np.zeros(scene.n_quads, np.int32))
    color = np.float32([0.9, 0.5, 0.2])
    o.set_textures(np.broadcast_to(color, (scene.n_quads, 4, 4, 3)).copy())
    cams = [sg.Camera((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 8, 8)]
    st = sg.RenderSettings(spp=2, depth=2, seed=9)
    img, _, _ = o.render(cams, st)
    t = color.astype(np.float64)
    expect = t * (st.E / math.pi) * st.light_dir[2] + t * st.L_sky
    np.testing.assert_allclose(img, np.broadcast_to(expect, img.shape), rtol=1e-12)


def test_rgb_texel_gradient_forms_agree():
    """Path replay, forward-mode dual numbers and central differences of the
    rendered loss agree for the per-channel texel gradient."""
    scene, cams, st, o, tex = _setup(seed=13)
    rng = np.random.default_rng(2)
    base = tex.astype(np.float64)
    o.set_textures(base + rng.uniform(-0.03, 0.03, base.shape))
    T, _, _ = o.render(cams, st)
    o.set_textures(base)
    I, _, _ = o.render(cams, st)
    N = I.size
    gpix = 2 * (I - T) / N
    g, _, _ = o.grad(cams, st, gpix)
    assert g.shape == (base.size,)
    e = rng.normal(size=g.shape)
    dI, _ = o.tangent(cams, st, e)
    fwd = (gpix * dI).sum()
    prb = (g * e).sum()
    assert abs(prb - fwd) <= 1e-10 * abs(fwd)

    def loss(t):
        o.set_textures(t.reshape(base.shape))
        Ia, _, _ = o.render(cams, st)
        return ((Ia - T) ** 2).sum() / N

    # texels are read as FP32: steps of 2^-16 keep them exact
    h = 2.0 ** -16
    fd = (loss(base.ravel() + h * np.sign(e)) - loss(base.ravel() - h * np.sign(e))) / (2 * h)
    assert abs(fd - (g * np.sign(e)).sum()) <= 1e-6 * abs(fd)
    for q in np.argsort(-np.abs(g))[:3]:
        eq = np.zeros(g.shape)
        eq[q] = 1.0
        fdq = (loss(base.ravel() + h * eq) - loss(base.ravel() - h * eq)) / (2 * h)
        assert abs(fdq - g[q]) <= 1e-6 * abs(g[q])


def test_rgb_textures_need_materials():
    scene = sg.tiny_scene(3, n_inst=2, n_protos=1, nq=4, spread=1.0)
    o = oracle.OracleScene(scene)
    o.set_textures(np.full((scene.n_quads, 2, 2, 3), 0.5, np.float32))
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 4, 4)]
    with pytest.raises(ValueError):
        o.render(cams, sg.RenderSettings(spp=1, depth=2, seed=1))
