"""Pins of the oracle's principled BSDF (Section 5.4: Disney's principled BSDF,
made energy conserving and preserving) and of its RGB path values, against
closed forms, quadrature and invariants that do not reuse the oracle's code.

The reading under test: f mu_i = (1 - m)[F_d p_s + (1 - F_d) c mu_i / pi] +
m F_c p_s, with p_s the density of a GGX visible-normal reflection mirrored
above the surface, F_d = spec (0.04 + 0.96 (1 - mu_o)^5) and
F_c = c + (1 - c)(1 - mu_o)^5.  Its albedo is (1 - m)[F_d + (1 - F_d) c] + m F_c
in closed form."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts

MATS = [(1.0, 1.0, 1.0, 0.8, 0.0, 1.0),   # white dielectric, rough, full specular
        (0.7, 0.3, 0.2, 0.5, 0.3, 0.6),   # colored, partly metallic
        (1.0, 1.0, 1.0, 0.3, 1.0, 0.0),   # white metal
        (0.9, 0.5, 0.1, 1.0, 0.6, 0.4),
        (0.2, 0.8, 0.4, 0.4, 0.0, 0.0)]   # Lambertian (no specular, no metal)


def _albedo_terms(mat, mo):
    """Closed-form albedo A_int + B_int c of the reading at mu_o."""
    m, s = mat[4], mat[5]
    k5 = (1.0 - mo) ** 5
    fd = s * (0.04 + 0.96 * k5)
    return (1 - m) * fd + m * k5, (1 - m) * (1 - fd) + m * (1 - k5)


def _frame(n):
    t1 = np.cross(n, [0.3, 0.5, 0.8])
    t1 /= np.linalg.norm(t1)
    return t1, np.cross(n, t1)


def _hemi_quadrature(mat, n, wo, nmu=800, nphi=1600):
    """Integrals of A and B over the hemisphere of n: Gauss-Legendre in mu_i,
    split at mu_o (the mirrored branch of the specular density starts there),
    midpoint rule in phi (periodic)."""
    mo = float(np.dot(n, wo))
    t1, t2 = _frame(n)
    tot = np.zeros(2)
    x, wx = np.polynomial.legendre.leggauss(nmu)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    for a, b in ((0.0, mo), (mo, 1.0)):
        mu = 0.5 * (b - a) * x + 0.5 * (b + a)
        wmu = 0.5 * (b - a) * wx
        M, PH = np.meshgrid(mu, phi, indexing="ij")
        st = np.sqrt(1 - M ** 2)
        d = (st * np.cos(PH))[..., None] * t1 + (st * np.sin(PH))[..., None] * t2 + M[..., None] * n
        out = oracle.bsdf_eval(mat, n, wo, d.reshape(-1, 3)).reshape(nmu, nphi, 4)
        w = wmu[:, None] * (2 * np.pi / nphi)
        tot += [(out[..., 0] * w).sum(), (out[..., 1] * w).sum()]
    return tot


def _dir(n, mo, az=0.7):
    t1, t2 = _frame(n)
    so = math.sqrt(1 - mo * mo)
    return so * math.cos(az) * t1 + so * math.sin(az) * t2 + mo * n


@pytest.mark.parametrize("mat", MATS[:4])
@pytest.mark.parametrize("mo", [0.9, 0.45, 0.2])
def test_albedo_closed_form_by_quadrature(mat, mo):
    """Energy conservation and preservation: the hemisphere integral of f mu_i
    equals (1 - m)[F_d + (1 - F_d) c] + m F_c (so it is 1 for c = 1).  A dropped
    mirrored branch, masking term, Jacobian or Fresnel factor moves it by
    percents."""
    n = np.array([0.36, -0.48, 0.8])
    wo = _dir(n, mo)
    A, B = _hemi_quadrature(mat, n, wo)
    ea, eb = _albedo_terms(mat, mo)
    assert abs(A - ea) < 5e-5 and abs(B - eb) < 5e-5, (A, ea, B, eb)


def test_lambert_limit():
    """metallic = specular = 0 is Lambert's c / pi: A = 0, B = mu_i / pi, the
    density is mu_i / pi and the specular lobe is never drawn."""
    mat = MATS[4]
    n = np.array([0.0, 0.6, 0.8])
    wo = _dir(n, 0.3)
    rng = np.random.default_rng(3)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d[d @ n < 0] *= -1
    out = oracle.bsdf_eval(mat, n, wo, d)
    mu = d @ n
    assert (out[:, 0] == 0).all() and (out[:, 3] == 0).all()
    np.testing.assert_allclose(out[:, 1], mu / math.pi, rtol=1e-14)
    np.testing.assert_allclose(out[:, 2], mu / math.pi, rtol=1e-14)
    wi, spec, _ = oracle.bsdf_sample(mat, n, wo, rng.uniform(size=(500, 3)))
    assert not spec.any()


@pytest.mark.parametrize("mat", MATS[:4])
def test_white_base_gives_unit_weights(mat):
    """Energy preservation path by path: with c = 1 every sampled direction's
    weight (A + B) / pdf is exactly one, whatever lobe drew it."""
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(4)
    for mo in (0.95, 0.5, 0.1):
        wo = _dir(n, mo, az=1.9)
        wi, spec, _ = oracle.bsdf_sample(mat, n, wo, rng.uniform(size=(4000, 3)))
        out = oracle.bsdf_eval(mat, n, wo, wi)
        w = (out[:, 0] + out[:, 1]) / out[:, 2]
        np.testing.assert_allclose(w, 1.0, rtol=1e-12)
        if mat[4] > 0 or mat[5] > 0:
            assert spec.any()


@pytest.mark.parametrize("mat", MATS[:4])
def test_sampler_follows_its_density(mat):
    """Chi-square of sampled directions in (mu_i, phi) bins against the
    density integrated per bin by quadrature: a sampler that does not draw
    from the density it reports (a missing mirror, a wrong stretch of the
    visible-normal sampling) fails by hundreds of standard deviations."""
    n = np.array([0.0, 0.0, 1.0])
    wo = _dir(n, 0.35, az=0.0)
    rng = np.random.default_rng(5)
    N = 400_000
    wi, _, _ = oracle.bsdf_sample(mat, n, wo, rng.uniform(size=(N, 3)))
    t1, t2 = _frame(n)
    mu = np.clip(wi @ n, 0, 1)
    ph = np.mod(np.arctan2(wi @ t2, wi @ t1), 2 * np.pi)
    nb_mu, nb_ph = 12, 16
    cnt, _, _ = np.histogram2d(mu, ph, bins=[nb_mu, nb_ph], range=[[0, 1], [0, 2 * np.pi]])
    # expected probability per bin: Gauss-Legendre 12 x 12 inside each bin
    x, wx = np.polynomial.legendre.leggauss(12)
    exp = np.zeros((nb_mu, nb_ph))
    for i in range(nb_mu):
        m0, m1 = i / nb_mu, (i + 1) / nb_mu
        mm = 0.5 * (m1 - m0) * x + 0.5 * (m1 + m0)
        for j in range(nb_ph):
            p0, p1 = 2 * np.pi * j / nb_ph, 2 * np.pi * (j + 1) / nb_ph
            pp = 0.5 * (p1 - p0) * x + 0.5 * (p1 + p0)
            M, P = np.meshgrid(mm, pp, indexing="ij")
            st = np.sqrt(1 - M ** 2)
            d = (st * np.cos(P))[..., None] * t1 + (st * np.sin(P))[..., None] * t2 + M[..., None] * n
            pdf = oracle.bsdf_eval(mat, n, wo, d.reshape(-1, 3))[:, 2].reshape(12, 12)
            exp[i, j] = (pdf * np.outer(wx, wx)).sum() * 0.25 * (m1 - m0) * (p1 - p0)
    assert abs(exp.sum() - 1.0) < 2e-3, exp.sum()
    e = N * exp
    keep = e > 20
    chi2 = ((cnt[keep] - e[keep]) ** 2 / e[keep]).sum()
    dof = int(keep.sum()) - 1
    # mean dof, sd sqrt(2 dof): allow 6 standard deviations
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_mirror_limit():
    """A smooth metal (roughness 0.05, alpha 0.0025) reflects about the mirror
    direction 2 mu_o n - wo: GGX half vectors have tan(theta_h) = alpha
    sqrt(u / (1 - u)), so the reflection's median angle is about 2 alpha and
    its 99th percentile about 20 alpha."""
    mat = (0.9, 0.9, 0.9, 0.05, 1.0, 0.0)
    n = np.array([0.0, 0.0, 1.0])
    wo = _dir(n, 0.6, az=0.3)
    mirror = 2 * 0.6 * n - wo
    wi, spec, _ = oracle.bsdf_sample(mat, n, wo, np.random.default_rng(6).uniform(size=(2000, 3)))
    assert spec.all()
    ang = np.arccos(np.clip(wi @ mirror, -1, 1))
    assert np.median(ang) < 4 * 0.0025 and np.percentile(ang, 99) < 25 * 0.0025


def _floor_rgb(mat, res=10):
    scene = ts.floor_scene(albedo=1.0)
    o = oracle.OracleScene(scene)
    o.set_materials(np.array([mat], np.float32), np.zeros(scene.n_quads, np.int32))
    cams = [sg.Camera((1.0, -2.0, 10.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, res, res)]
    return o, cams


@pytest.mark.parametrize("mat", MATS[:4])
def test_white_furnace_floor(mat):
    """A white floor (c = 1) under the constant sky, no sun: every path leaves
    the floor with weight exactly one, so every pixel and channel is L_sky."""
    mat = (1.0, 1.0, 1.0) + tuple(mat[3:])
    o, cams = _floor_rgb(mat)
    st = sg.RenderSettings(spp=3, depth=3, seed=7)
    st.E = 0.0
    img, _, _ = o.render(cams, st)
    assert img.shape == (100, 3)
    np.testing.assert_allclose(img, st.L_sky, rtol=1e-12)


def test_lambert_rgb_floor_closed_form():
    """Lambertian RGB floor (tint per channel, specular = metallic = 0) under
    the sun and the sky: channel k is tint_k a (E / pi) cos_L + tint_k a L_sky."""
    tint = (0.9, 0.5, 0.2)
    a = float(np.float32(0.7))
    scene = ts.floor_scene(albedo=a)
    o = oracle.OracleScene(scene)
    o.set_materials(np.array([tint + (0.5, 0.0, 0.0)], np.float32), np.zeros(scene.n_quads, np.int32))
    cams = [sg.Camera((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 8, 8)]
    st = sg.RenderSettings(spp=2, depth=2, seed=9)
    img, _, _ = o.render(cams, st)
    c = np.float32(tint).astype(np.float64) * a
    expect = c * (st.E / math.pi) * st.light_dir[2] + c * st.L_sky
    np.testing.assert_allclose(img, np.broadcast_to(expect, img.shape), rtol=1e-12)


def test_principled_floor_mean_albedo():
    """A colored principled floor under the sky (no sun, one bounce): a pixel's
    expected value is L_sky times the closed-form albedo at its mu_o; the mean
    ratio over many pixels and samples is one within its sampling error."""
    mat = (0.8, 0.4, 0.2, 0.45, 0.4, 0.7)
    o, cams = _floor_rgb(mat, res=48)
    st = sg.RenderSettings(spp=16, depth=2, seed=11)
    st.E = 0.0
    img, _, _ = o.render(cams, st)
    c = cams[0]
    f = np.array(c.look) - np.array(c.eye)
    f /= np.linalg.norm(f)
    r = np.cross(f, c.up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(c.vfov_deg) / 2)
    ys, xs = np.mgrid[0:c.h, 0:c.w]
    d = f + ((2 * (xs.ravel() + 0.5) / c.w - 1) * th)[:, None] * r + ((1 - 2 * (ys.ravel() + 0.5) / c.h) * th)[:, None] * u
    mo = (-d[:, 2]) / np.linalg.norm(d, axis=1)  # the floor's normal is +z
    A, B = _albedo_terms(mat, mo)
    tint = np.float32(mat[:3]).astype(np.float64)
    expect = st.L_sky * (A[:, None] + B[:, None] * tint[None, :])
    ratio = img / expect
    # pixel jitter moves mu_o slightly; the bias is far below the sampling error
    se = ratio.std(axis=0) / math.sqrt(ratio.shape[0])
    assert (np.abs(ratio.mean(axis=0) - 1.0) < 5 * se + 2e-3).all(), (ratio.mean(axis=0), se)


def _grad_setup_rgb(seed=31):
    scene = sg.tiny_scene(seed, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 12, 12)]
    st = sg.RenderSettings(spp=2, depth=4, seed=seed)
    mats = np.array([(0.9, 0.6, 0.3, 0.5, 0.0, 0.8), (0.4, 0.7, 0.9, 0.35, 0.7, 0.2),
                     (0.8, 0.8, 0.8, 0.9, 0.2, 0.5)], np.float32)
    fm = (np.arange(scene.n_quads) % 3).astype(np.int32)
    return scene, cams, st, mats, fm


@pytest.mark.parametrize("env", [False, True])
def test_rgb_gradient_replay_forward_mode_and_fd_agree(env):
    """Principled RGB shading keeps each path's value affine in every vertex's
    albedo (the base color is tint x albedo and the sampled directions do not
    depend on it), so the path-replay gradient, forward-mode dual numbers and
    central differences of the rendered loss agree, with RGB pixel weights."""
    scene, cams, st, mats, fm = _grad_setup_rgb()
    o = oracle.OracleScene(scene)
    o.set_materials(mats, fm)
    if env:
        rng0 = np.random.default_rng(8)
        o.set_environment(rng0.uniform(0.0, 1.0, size=(8, 16)).astype(np.float32))
        st.env_nee = True
    rng = np.random.default_rng(2)
    alb = scene.albedo.astype(np.float64)
    o.set_albedo(alb + rng.uniform(-0.1, 0.1, alb.shape))
    T, _, _ = o.render(cams, st)
    o.set_albedo(alb)
    I, _, _ = o.render(cams, st)
    assert I.shape == (144, 3) and not np.allclose(I[:, 0], I[:, 1])
    N = I.size
    gpix = 2 * (I - T) / N
    g, _, _ = o.grad(cams, st, gpix)
    e = rng.normal(size=alb.shape)
    dI, _ = o.tangent(cams, st, e)
    fwd = (gpix * dI).sum()
    prb = (g * e).sum()
    assert abs(prb - fwd) <= 1e-10 * abs(fwd)

    def loss(a):
        o.set_albedo(a)
        Ia, _, _ = o.render(cams, st)
        return ((Ia - T) ** 2).sum() / N

    h = 1e-5
    fd = (loss(alb + h * e) - loss(alb - h * e)) / (2 * h)
    assert abs(fd - prb) <= 1e-6 * abs(prb)
    for f in np.argsort(-np.abs(g))[:4]:
        ef = np.zeros_like(alb)
        ef[f] = 1.0
        fdf = (loss(alb + h * ef) - loss(alb - h * ef)) / (2 * h)
        assert abs(fdf - g[f]) <= 1e-6 * abs(g[f])
