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


def test_shoemake_rotations_are_uniform_rotations():
    R = sg.shoemake_rotations(np.random.default_rng(3), 20000)
    assert np.allclose(np.einsum("nji,njk->nik", R, R), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # Haar measure: E[R] = 0 and E[R_ij^2] = 1/3
    assert np.abs(R.mean(axis=0)).max() < 0.02
    assert np.abs((R ** 2).mean(axis=0) - 1.0 / 3.0).max() < 0.02


@pytest.mark.parametrize("n", [1, 2, 7])
def test_shell_is_closed_and_faces_outward(n):
    v, q = sg.shell_proto(np.random.default_rng(n), n, 1.0, 0.05)
    assert q.shape == (6 * n * n, 4) and v.shape[0] == 6 * n * n + 2  # Euler: V - E + F = 2
    edges = np.sort(np.stack([q, np.roll(q, -1, axis=1)], axis=-1).reshape(-1, 2), axis=1)
    _, counts = np.unique(edges, axis=0, return_counts=True)
    assert (counts == 2).all(), "an edge is not shared by exactly two quads"
    # directed edges appear once each way: consistent orientation
    directed = np.stack([q, np.roll(q, -1, axis=1)], axis=-1).reshape(-1, 2)
    assert np.unique(directed, axis=0).shape[0] == directed.shape[0]
    c = v[q].astype(np.float64)
    nrm = np.cross(c[:, 1] - c[:, 0], c[:, 3] - c[:, 0])
    assert (np.einsum("ij,ij->i", nrm, c.mean(axis=1)) > 0).all(), "a quad faces inward"


def test_grid_topology():
    q = sg.grid_quads(5, 3)
    assert q.shape == (15, 4) and q.min() == 0 and q.max() == 6 * 4 - 1
    edges = np.sort(np.stack([q, np.roll(q, -1, axis=1)], axis=-1).reshape(-1, 2), axis=1)
    _, counts = np.unique(edges, axis=0, return_counts=True)
    # interior edges shared by two quads, boundary edges (2 (5 + 3)) by one
    assert (counts <= 2).all() and (counts == 1).sum() == 2 * (5 + 3)


def test_scaled_big_configs():
    s3, c3, st3 = sg.config3(scale=0.0005)
    assert s3.n_instances == 10_000 and len(c3) == 1 and (st3.spp, st3.depth) == (4, 8)
    s5, c5, st5 = sg.config5(scale=0.0002)
    assert s5.n_instances == 8_000 and len(c5) == 64 and (st5.spp, st5.depth) == (1, 6)
    sides = np.array([c.w for c in c5])
    assert (sides >= 64).all() and (sides <= 1024).all() and all(c.w == c.h for c in c5)
