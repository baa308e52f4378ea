"""Helpers shared by the GPU tests: tensors in and out of the binding, and the
comparison of GPU hits with the oracle under the flag rules."""
import sys

import numpy as np

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(rays: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rays, dtype=np.float32)).cuda()


def hits_np(h):
    import torch
    torch.cuda.synchronize()
    return dict(t=h.t.cpu().numpy(), u=h.u.cpu().numpy(), v=h.v.cpu().numpy(), inst=h.inst.cpu().numpy(),
                prim=h.prim.cpu().numpy())


def assert_hits_identical(a, b, what=""):
    for k in ("t", "u", "v", "inst", "prim"):
        x, y = a[k], b[k]
        if k in ("t", "u", "v"):
            same = (x.view(np.uint32) == y.view(np.uint32))
        else:
            same = x == y
        if not same.all():
            bad = np.nonzero(~same)[0]
            raise AssertionError(f"{what}: field {k} differs on {bad.size} rays, first {bad[:5]}: "
                                 f"{x[bad[:5]]} vs {y[bad[:5]]}")


def world_quads(scene, inst, prim):
    """World-space vertices [n, 4, 3] (FP64) of (instance, prim) pairs."""
    p = scene.inst_proto[inst]
    q = scene.proto_quad_off[p] + prim
    idx = scene.quads[q] + scene.proto_vert_off[p][:, None]
    v = scene.verts[idx].astype(np.float64)
    X = scene.inst_xform[inst].astype(np.float64).reshape(-1, 3, 4)
    return np.einsum("nij,nkj->nki", X[:, :, :3], v) + X[:, None, :, 3]


def compare_with_oracle(scene, rays, g, o, uv_factor=64.0):
    """Assert GPU hits g agree with oracle hits o (oracle.Hits) under the flag rules.

    * unflagged rays (no near tie, graze or near-origin flag): identical
      (instance, primitive); t within 1e-5 relative unless t is ill-conditioned;
      u, v within uv_factor * 2^-24 * S / (shortest world edge * |cos|), the FP32
      position error carried into the quad's parameterisation, with S the
      oracle's position scale of the answer;
    * flagged rays: a hit reported by the GPU is one of the oracle's candidates.
    Returns the fraction of flagged rays.
    """
    flagged = (o.flags & oracle.ID_FLAGS) != 0
    ok = ~flagged
    gi, gp = g["inst"], g["prim"]
    bad = ok & ((gi != o.inst) | (gp != o.prim))
    if bad.any():
        k = np.nonzero(bad)[0][:8]
        raise AssertionError(f"{bad.sum()} unflagged rays differ in (inst, prim): idx {k} gpu "
                             f"{list(zip(gi[k], gp[k]))} oracle {list(zip(o.inst[k], o.prim[k]))} t {g['t'][k]} "
                             f"{o.t[k]} flags {o.flags[k]}")
    hit = ok & (o.inst >= 0)
    tcheck = hit & ((o.flags & oracle.F_T_ILLCOND) == 0)
    rel = np.abs(g["t"][tcheck].astype(np.float64) - o.t[tcheck]) / o.t[tcheck]
    assert (rel <= 1e-5).all(), f"t relative error {rel.max()} > 1e-5"
    miss = ok & (o.inst < 0)
    assert np.isinf(g["t"][miss]).all() and (g["u"][miss] == 0).all() and (g["v"][miss] == 0).all()
    if hit.any():
        W = world_quads(scene, o.inst[hit], o.prim[hit])
        r = rays[hit].astype(np.float64)
        edges = np.stack([np.linalg.norm(W[:, (k + 1) % 4] - W[:, k], axis=1) for k in range(4)], 1)
        half = o.half[hit]
        A = np.where(half[:, None] == 0, W[:, 1] - W[:, 0], W[:, 3] - W[:, 2])
        B = np.where(half[:, None] == 0, W[:, 3] - W[:, 0], W[:, 1] - W[:, 2])
        n = np.cross(A, B)
        cos = np.abs((n * r[:, 3:6]).sum(1)) / (np.linalg.norm(n, axis=1) * np.linalg.norm(r[:, 3:6], axis=1))
        tol = uv_factor * 2.0 ** -24 * o.scale[hit] / (edges.min(1) * np.maximum(cos, 1e-3))
        du = np.abs(g["u"][hit] - o.u[hit])
        dv = np.abs(g["v"][hit] - o.v[hit])
        assert (du <= tol).all() and (dv <= tol).all(), f"uv error {max(du.max(), dv.max())}"
    # flagged rays: any hit the GPU reports must be a candidate of the oracle
    fl = np.nonzero(flagged & (gi >= 0))[0]
    for i in fl:
        cands = {(int(o.inst[i]), int(o.prim[i]))} | {(int(o.cand[i, 2 * c]), int(o.cand[i, 2 * c + 1]))
                                                      for c in range(int(o.ncand[i]))}
        if (o.flags[i] & (oracle.F_GRAZE | oracle.F_NEAR_ORIGIN)) == 0:
            assert (int(gi[i]), int(gp[i])) in cands, f"ray {i}: gpu hit not among the oracle candidates"
    return flagged.mean()
