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


def camera_rays(cams, rng, n_per_cam):
    """FP32 rays from each camera's eye through uniformly jittered image points
    (pinhole model of the render), tmin 0, tmax +inf: [n, 8]."""
    import math
    out = []
    for c in cams:
        f = np.array(c.look, dtype=np.float64) - np.array(c.eye, dtype=np.float64)
        f /= np.linalg.norm(f)
        r = np.cross(f, c.up)
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        th = math.tan(math.radians(c.vfov_deg) / 2)
        xs = rng.uniform(0, c.w, n_per_cam)
        ys = rng.uniform(0, c.h, n_per_cam)
        d = f + ((2 * xs / c.w - 1) * th * c.w / c.h)[:, None] * r + ((1 - 2 * ys / c.h) * th)[:, None] * u
        rr = np.zeros((n_per_cam, 8), np.float32)
        rr[:, 0:3] = c.eye
        rr[:, 3:6] = d
        rr[:, 7] = np.inf
        out.append(rr)
    return np.concatenate(out)


def compare_paths(rtq, oracle, S, o, cams, st, rng, n_paths, **kw):
    """Paths traced alone on the GPU (rtq_render_path) against the oracle's FP64
    paths: instance, primitive, half, shadow outcome and t of every vertex up to
    the first vertex the oracle flags.  Returns the number of vertices compared."""
    offs = np.cumsum([0] + [c.w * c.h for c in cams])
    compared = 0
    for g in rng.choice(int(offs[-1]), size=n_paths, replace=False):
        view = int(np.searchsorted(offs, g, side="right") - 1)
        p = int(g - offs[view])
        s_ = int(rng.integers(0, st.spp))
        gv, gesc, _ = rtq.render_path(S, cams, st, view, p, s_, **kw)
        ov, oesc, pflags = o.path(cams, st, int(g), s_)
        for k, y in enumerate(ov):
            if (y["flags"] & oracle.ID_FLAGS) or y["shadow_flags"]:
                break
            assert k < len(gv), (g, s_, k, "gpu path ended early")
            x = gv[k]
            assert (x["inst"], x["prim"], x["half"]) == (y["inst"], y["prim"], y["half"]), (g, s_, k, x, y)
            assert abs(x["t"] - y["t"]) <= 1e-5 * y["t"] or (y["flags"] & oracle.F_T_ILLCOND), (g, s_, k, x, y)
            compared += 1
            if y["flags"] & oracle.F_SHADE:
                break
            assert x["shadow"] == y["shadow"], (g, s_, k, x, y)
        else:
            assert gesc == oesc or pflags, (g, s_, gesc, oesc)
    return compared
