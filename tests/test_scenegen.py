"""The seeded input generators produce the workloads the design's input recipe
states (sizes, structure, value ranges), deterministically."""
import numpy as np
import pytest

from paper_2001_02620_amd import scenegen as sg


def test_config1_recipe():
    s, cams, st = sg.config1()
    assert s.n_protos == 16 and s.n_instances == 1000 and s.n_quads == 16 * 32 * 32
    assert (s.albedo >= 0.2).all() and (s.albedo <= 0.8).all()
    x = s.inst_xform.reshape(-1, 3, 4).astype(np.float64)
    A, t = x[:, :, :3], x[:, :, 3]
    # rotation x uniform scale in [0.5, 2]: A^T A = s^2 I
    ata = np.einsum("nij,nik->njk", A, A)
    sc2 = ata[:, 0, 0]
    assert np.allclose(ata, sc2[:, None, None] * np.eye(3), atol=1e-5)
    assert (np.sqrt(sc2) >= 0.5 - 1e-6).all() and (np.sqrt(sc2) <= 2.0 + 1e-6).all()
    assert (np.abs(t) <= 50.0).all()
    assert len(cams) == 1 and (cams[0].w, cams[0].h) == (128, 128) and st.depth == 3


def test_config2_recipe_and_determinism():
    s, cams, st = sg.config2()
    assert s.n_instances == 1_000_000 and s.n_protos == 257  # 256 prototypes + the terrain
    assert 14.0e6 < s.n_quads < 14.2e6
    assert [(c.w, c.h) for c in cams] == [(1920, 1080), (1920, 1080)] and st.spp == 1 and st.depth == 8
    sizes = np.diff(s.proto_quad_off)
    assert sizes.max() == 2048 * 2048  # the terrain
    other = np.sort(sizes)[:-1]
    # log-uniform in [2k, 200k]; a cube-sphere shell holds 6 n^2 quads, the
    # nearest such count to the one drawn
    assert other.min() >= 0.9 * 2000 and other.max() <= 200_000
    s2, _, _ = sg.config2()
    assert np.array_equal(s.verts, s2.verts) and np.array_equal(s.inst_xform, s2.inst_xform)


def test_config4_recipe():
    s, cams, st = sg.config4()
    assert s.n_quads == 16 * 32 * 32 and s.n_instances == 1000
    assert [(c.w, c.h) for c in cams] == [(512, 512)] and st.spp == 4 and st.depth == 4
