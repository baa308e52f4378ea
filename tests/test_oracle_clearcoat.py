"""Pins of the clearcoat layer of the oracle's principled BSDF (Section 5.4: the
scene's materials use Disney's principled BSDF, made energy conserving and
preserving; its coat layer is read here as a second mirrored visible-normal lobe
over the base).

The reading under test: f mu_i = F_k p_k + (1 - F_k) [base f mu_i] with
F_k = k (0.04 + 0.96 (1 - mu_o)^5) and p_k the density of a GGX visible-normal
reflection of the coat's roughness, mirrored above the surface.  Its albedo is
F_k + (1 - F_k) [base albedo] in closed form: one for a white base.  The coat
lobe is drawn with probability F_k, the base's lobes with the rest."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests import scenes as ts
from tests.test_oracle_bsdf import _albedo_terms, _dir, _frame, _hemi_quadrature

# (tint r, g, b, roughness, metallic, specular, clearcoat, clearcoat roughness)
COAT = [(1.0, 1.0, 1.0, 0.8, 0.0, 1.0, 1.0, 0.3),   # white rough dielectric, full coat
        (0.7, 0.3, 0.2, 0.5, 0.3, 0.6, 0.5, 0.45),  # colored, partly metallic, half coat
        (1.0, 1.0, 1.0, 0.3, 1.0, 0.0, 0.8, 0.6),   # white metal under a coat
        (0.0, 0.0, 0.0, 0.5, 0.0, 0.0, 1.0, 0.35)]  # black Lambertian base: the coat alone


def _coat_terms(mat, mo):
    """Closed-form albedo A_int + B_int c with the coat over the base."""
    k5 = (1.0 - mo) ** 5
    fk = mat[6] * (0.04 + 0.96 * k5)
    a, b = _albedo_terms(mat, mo)
    return fk + (1 - fk) * a, (1 - fk) * b


@pytest.mark.parametrize("mat", COAT)
@pytest.mark.parametrize("mo", [0.9, 0.45, 0.2])
def test_coat_albedo_closed_form_by_quadrature(mat, mo):
    """Energy conservation and preservation with the coat: the hemisphere
    integral of f mu_i is F_k + (1 - F_k) [base albedo].  For the black base it
    is F_k alone.  A coat that does not attenuate the base, a coat lobe with
    the base's roughness folded in, or a wrong coat Fresnel factor moves it by
    percents."""
    n = np.array([0.36, -0.48, 0.8])
    wo = _dir(n, mo)
    A, B = _hemi_quadrature(mat, n, wo)
    ea, eb = _coat_terms(mat, mo)
    assert abs(A - ea) < 5e-5 and abs(B - eb) < 5e-5, (A, ea, B, eb)


def test_zero_coat_is_the_base_bit_for_bit():
    """clearcoat = 0 leaves the BSDF, its density and its sampler exactly as the
    base alone, whatever the coat roughness."""
    base = (0.7, 0.3, 0.2, 0.5, 0.3, 0.6)
    n = np.array([0.0, 0.6, 0.8])
    wo = _dir(n, 0.4)
    rng = np.random.default_rng(12)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    u = rng.uniform(size=(300, 3))
    e6 = oracle.bsdf_eval(base, n, wo, d)
    e8 = oracle.bsdf_eval(base + (0.0, 0.7), n, wo, d)
    assert np.array_equal(e6, e8)
    w6, l6, a6 = oracle.bsdf_sample(base, n, wo, u)
    w8, l8, a8 = oracle.bsdf_sample(base + (0.0, 0.7), n, wo, u)
    assert np.array_equal(w6, w8) and np.array_equal(l6, l8) and np.array_equal(a6, a8)
    assert set(np.unique(l6)) <= {0, 1}


@pytest.mark.parametrize("mat", COAT[:3])
def test_coat_white_base_gives_unit_weights(mat):
    """Energy preservation path by path: with c = 1 every sampled direction's
    weight (A + B) / pdf is one, whichever of the three lobes drew it."""
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(14)
    for mo in (0.95, 0.5, 0.1):
        wo = _dir(n, mo, az=1.9)
        wi, lobe, _ = oracle.bsdf_sample(mat, n, wo, rng.uniform(size=(4000, 3)))
        out = oracle.bsdf_eval(mat, n, wo, wi)
        np.testing.assert_allclose((out[:, 0] + out[:, 1]) / out[:, 2], 1.0, rtol=1e-12)
        assert (lobe == 2).any() and (lobe != 2).any()


def test_coat_lobe_choice_follows_its_fresnel_weight():
    """The lobe word picks the coat exactly when it lies below F_k, the base's
    specular lobe up to Pn = F_k + (1 - F_k) P_s, the cosine lobe above."""
    mat = COAT[1]
    n = np.array([0.0, 0.0, 1.0])
    mo = 0.3
    wo = _dir(n, mo)
    k5 = (1 - mo) ** 5
    fk = mat[6] * (0.04 + 0.96 * k5)
    fd = mat[5] * (0.04 + 0.96 * k5)
    pn = fk + (1 - fk) * ((1 - mat[4]) * fd + mat[4])
    u = np.random.default_rng(15).uniform(size=(5000, 3))
    _, lobe, _ = oracle.bsdf_sample(mat, n, wo, u)
    want = np.where(u[:, 0] < fk, 2, np.where(u[:, 0] < pn, 1, 0))
    assert np.array_equal(lobe, want)
    assert abs(oracle.bsdf_eval(mat, n, wo, n[None])[0, 3] - pn) < 1e-15


@pytest.mark.parametrize("mat", COAT[1:])
def test_coat_sampler_follows_its_density(mat):
    """Chi-square of sampled directions in (mu_i, phi) bins against the
    reported density integrated per bin: the three-lobe sampler draws from the
    mixture density it reports."""
    n = np.array([0.0, 0.0, 1.0])
    wo = _dir(n, 0.35, az=0.0)
    N = 400_000
    wi, _, _ = oracle.bsdf_sample(mat, n, wo, np.random.default_rng(16).uniform(size=(N, 3)))
    t1, t2 = _frame(n)
    mu = np.clip(wi @ n, 0, 1)
    ph = np.mod(np.arctan2(wi @ t2, wi @ t1), 2 * np.pi)
    nb_mu, nb_ph = 12, 16
    cnt, _, _ = np.histogram2d(mu, ph, bins=[nb_mu, nb_ph], range=[[0, 1], [0, 2 * np.pi]])
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
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_smooth_coat_mirror_limit():
    """A smooth coat (roughness 0.05, alpha 0.0025) over a rough base reflects
    about the mirror direction, while the base's specular lobe stays wide."""
    mat = (0.9, 0.9, 0.9, 0.9, 1.0, 0.0, 1.0, 0.05)
    n = np.array([0.0, 0.0, 1.0])
    wo = _dir(n, 0.6, az=0.3)
    mirror = 2 * 0.6 * n - wo
    wi, lobe, _ = oracle.bsdf_sample(mat, n, wo, np.random.default_rng(17).uniform(size=(4000, 3)))
    ang = np.arccos(np.clip(wi @ mirror, -1, 1))
    assert (lobe == 2).sum() > 50 and (lobe == 1).sum() > 1000
    assert np.median(ang[lobe == 2]) < 4 * 0.0025 and np.percentile(ang[lobe == 2], 99) < 25 * 0.0025
    assert np.median(ang[lobe == 1]) > 0.1


@pytest.mark.parametrize("mat", COAT[:3])
def test_coat_white_furnace_floor(mat):
    """A white coated floor under the constant sky, no sun: every path leaves
    the floor with weight exactly one, so every pixel and channel is L_sky."""
    mat = (1.0, 1.0, 1.0) + tuple(mat[3:])
    scene = ts.floor_scene(albedo=1.0)
    o = oracle.OracleScene(scene)
    o.set_materials(np.array([mat], np.float32), np.zeros(scene.n_quads, np.int32))
    cams = [sg.Camera((1.0, -2.0, 10.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 10, 10)]
    st = sg.RenderSettings(spp=3, depth=3, seed=7)
    st.E = 0.0
    img, _, _ = o.render(cams, st)
    np.testing.assert_allclose(img, st.L_sky, rtol=1e-12)


def test_coat_gradient_replay_forward_mode_and_fd_agree():
    """The coat's lobe choice depends on mu_o and the coat weight only, so a
    path's value stays affine in each vertex's albedo: the path-replay
    gradient, forward-mode dual numbers and central differences agree."""
    scene = sg.tiny_scene(33, n_inst=4, n_protos=2, nq=4, spread=1.0)
    cams = [sg.Camera((0.0, -8.0, 1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 35.0, 12, 12)]
    st = sg.RenderSettings(spp=2, depth=4, seed=33)
    mats = np.array([(0.9, 0.6, 0.3, 0.5, 0.0, 0.8, 1.0, 0.3), (0.4, 0.7, 0.9, 0.35, 0.7, 0.2, 0.6, 0.5),
                     (0.8, 0.8, 0.8, 0.9, 0.2, 0.5, 0.0, 0.0)], np.float32)
    fm = (np.arange(scene.n_quads) % 3).astype(np.int32)
    o = oracle.OracleScene(scene)
    o.set_materials(mats, fm)
    rng = np.random.default_rng(3)
    alb = scene.albedo.astype(np.float64)
    o.set_albedo(alb + rng.uniform(-0.1, 0.1, alb.shape))
    T, _, _ = o.render(cams, st)
    o.set_albedo(alb)
    I, _, _ = o.render(cams, st)
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
