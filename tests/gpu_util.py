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


def compare_with_oracle(scene, rays, g, o, uv_factor=64.0, excl=None, ora_scene=None, stats=None):
    """Assert GPU hits g agree with oracle hits o (oracle.Hits) under the flag rules.

    * unflagged rays (no near tie, graze or near-origin flag): identical
      (instance, primitive); t within 1e-5 relative unless t is ill-conditioned;
      u, v within uv_factor * 2^-24 * S / (shortest world edge * |cos|), the FP32
      position error carried into the quad's parameterisation, with S the
      oracle's position scale of the answer (a capsule hit: u, the curve
      parameter, within that error over 8 axis lengths, and v = 0);
    * flagged rays: the GPU's answer (hit or miss) is one an FP32 traversal may
      give (the oracle's acceptance check over every triangle near the ray),
      with its t within tolerance unless ill-conditioned -- every flagged ray is
      checked.
    Where t is ill-conditioned (FP32 cannot resolve it to 1e-5) it is held to
    the FP32 bound, 16 units of 2^-24 S / (|d| |cos|), by the acceptance check.
    Returns the fraction of flagged rays; `stats` (a dict, optional) receives
    counts and the largest t error in those units.
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
    osc = ora_scene if ora_scene is not None else oracle.OracleScene(scene)
    # hits on the capsules of curves (Section 5.2) carry u = curve parameter, v = 0
    caph = np.zeros_like(hit)
    if getattr(scene, "curves", None) is not None:
        curve_proto = np.diff(scene.proto_curve_off) > 0
        caph = hit & curve_proto[scene.inst_proto[np.maximum(o.inst, 0)]]
        hit = hit & ~caph
    if caph.any():
        caps = osc.capsules()
        pi = scene.inst_proto[o.inst[caph]]
        c = caps[8 * scene.proto_curve_off[pi] + o.prim[caph]]
        X = scene.inst_xform[o.inst[caph]].astype(np.float64).reshape(-1, 3, 4)
        a = np.einsum("nij,nj->ni", X[:, :, :3], c[:, 0:3]) + X[:, :, 3]
        b = np.einsum("nij,nj->ni", X[:, :, :3], c[:, 3:6]) + X[:, :, 3]
        r = rays[caph].astype(np.float64)
        P = r[:, 0:3] + o.t[caph][:, None] * r[:, 3:6]
        ba = b - a
        Lc = np.linalg.norm(ba, axis=1)
        s_ = np.clip(((P - a) * ba).sum(1) / np.maximum(Lc * Lc, 1e-300), 0, 1)
        nrm = P - (a + s_[:, None] * ba)
        cos = np.abs((nrm * r[:, 3:6]).sum(1)) / (np.linalg.norm(nrm, axis=1) * np.linalg.norm(r[:, 3:6], axis=1))
        flat = getattr(scene, "proto_curve_flat", None)
        if flat is not None:
            # a ribbon's u follows the projected segment: the sine of the angle
            # between the ray and the segment takes the part of |cos|
            fl_ = flat[pi] != 0
            sin = np.linalg.norm(np.cross(ba, r[:, 3:6]), axis=1) / (np.maximum(Lc, 1e-300) *
                                                                     np.linalg.norm(r[:, 3:6], axis=1))
            cos = np.where(fl_, sin, cos)
        tol = uv_factor * 2.0 ** -24 * o.scale[caph] / (8 * np.maximum(Lc, 1e-30) * np.maximum(cos, 1e-3)) + 2.0 ** -21
        du = np.abs(g["u"][caph] - o.u[caph])
        assert (du <= tol).all() and (g["v"][caph] == 0).all(), f"capsule u error {du.max()}"
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
    # every ray (flagged ones included): the GPU's answer must be acceptable for
    # the FP32 ray; its t error is measured in units of 2^-24 S / (|d| |cos|)
    fl = np.nonzero(flagged)[0]
    code, info, ulps = osc.accept(rays, gi, gp, g["t"], excl=excl, want_ulps=True)
    bad = code != 0
    if bad.any():
        k = np.nonzero(bad)[0][:8]
        raise AssertionError(f"{bad.sum()} rays ({flagged[bad].sum()} flagged) have an answer no FP32 traversal "
                             f"may give: idx {k} codes {[oracle.ACCEPT_CODES[c] for c in code[bad][:8]]} gpu "
                             f"{list(zip(gi[k], gp[k], g['t'][k]))} oracle {list(zip(o.inst[k], o.prim[k], o.t[k]))}")
    waived = (info & 2) != 0
    u = ulps[gi >= 0]
    log(f"    rays {rays.shape[0]}: flagged {fl.size}, t ill-conditioned (FP32 bound) {int(waived.sum())}, t error in "
        f"2^-24 S/(|d||cos|): p99 {np.percentile(u, 99) if u.size else 0:.2f} max {u.max() if u.size else 0:.2f}")
    if stats is not None:
        stats["t_waived"] = stats.get("t_waived", 0) + int(waived.sum())
        stats["rays"] = stats.get("rays", 0) + int(rays.shape[0])
        stats["flagged"] = stats.get("flagged", 0) + int(fl.size)
        stats["max_t_ulps"] = max(stats.get("max_t_ulps", 0.0), float(u.max()) if u.size else 0.0)
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


def replay_check_pixels(rtq, osc, S, cams, st, pixels, img, **kw):
    """Every sample path of the listed packed pixels, traced alone on the GPU
    (rtq_render_path) and checked by the oracle step by step along its own rays
    (acceptable hits and escapes, shadow outcomes, shading decisions, next rays,
    FP64 radiance to 1e-4).  The pixel must equal the mean of its recorded
    paths' radiance bit for bit (FP32 sum in sample order over spp, as the
    accumulation forms it) and the mean of the oracle's replay values to 1e-4.
    img: [n] floats, or [n, 3] (RGB) for a scene with materials, compared per
    channel.  Returns counts (paths, vertices, certain answers, vertices whose t
    is ill-conditioned and held to the FP32 bound, shading decisions near a
    threshold) and the largest t error in units of 2^-24 S / (|d| |cos|)."""
    offs = np.cumsum([0] + [c.n_pixels() if hasattr(c, "n_pixels") else c.w * c.h for c in cams])
    tot = dict(paths=0, vertices=0, certain=0, t_waived=0, ambiguous_shading=0, max_t_ulps=0.0)
    rgb = np.ndim(img) == 2
    nch = 3 if rgb else 1
    for g in np.asarray(pixels):
        view = int(np.searchsorted(offs, g, side="right") - 1)
        p = int(g - offs[view])
        acc = np.zeros(nch, np.float32)
        ref = np.zeros(nch)
        for s_ in range(st.spp):
            nv, vi, vf, esc, rad = rtq.render_path_raw(S, cams, st, view, p, s_, **kw)
            code, info = osc.check_path(cams, st, view, p, s_, nv, vi, vf, esc, rad)
            assert code == 0, (f"pixel {g} sample {s_}: {oracle.PATH_CODES.get(code)} at ray {info['ray']}",
                               nv, vi[:nv + 1].tolist(), vf[:nv + 1].tolist(), esc, rad, info)
            acc = (acc + np.asarray(rad, np.float32).reshape(nch)).astype(np.float32)
            ref += info["Lc"] if rgb else info["L"]
            tot["paths"] += 1
            for k in ("vertices", "certain", "t_waived", "ambiguous_shading"):
                tot[k] += info[k]
            tot["max_t_ulps"] = max(tot["max_t_ulps"], info["max_t_ulps"])
        mean = (acc / np.float32(st.spp)).astype(np.float32)
        gv = np.asarray(img[g], np.float32).reshape(nch)
        assert (mean.view(np.uint32) == gv.view(np.uint32)).all(), (g, mean, gv)
        ref /= st.spp
        assert (np.abs(gv - ref) <= 1e-4 * np.abs(ref).max() + 1e-7).all(), (g, gv, ref)
    return tot
