"""Hand-built scenes for the pins (closed forms, conventions, watertightness)."""
import math

import numpy as np

from paper_2001_02620_amd import scenegen as sg


def axis_quad(x0, x1, y0, y1, c):
    """Quad in the plane z = c: v0=(x0,y0) v1=(x1,y0) v2=(x1,y1) v3=(x0,y1)."""
    v = np.array([[x0, y0, c], [x1, y0, c], [x1, y1, c], [x0, y1, c]], dtype=np.float32)
    return v, np.array([[0, 1, 2, 3]], dtype=np.int32)


def multi_mesh_scene(meshes, albedos=None, xforms=None, protos=None):
    """Several prototypes (list of (verts, quads)); instance k uses protos[k] (default k)
    with transform xforms[k] (default identity)."""
    vo, qo = [0], [0]
    for v, q in meshes:
        vo.append(vo[-1] + v.shape[0])
        qo.append(qo[-1] + q.shape[0])
    verts = np.concatenate([v for v, _ in meshes]).astype(np.float32)
    quads = np.concatenate([q for _, q in meshes]).astype(np.int32)
    if albedos is None:
        albedo = np.full(quads.shape[0], 0.5, dtype=np.float32)
    else:
        albedo = np.concatenate([np.broadcast_to(np.asarray(a, np.float32), (q.shape[0],))
                                 for a, (_, q) in zip(albedos, meshes)]).astype(np.float32)
    n_inst = len(meshes) if protos is None else len(protos)
    if protos is None:
        protos = list(range(len(meshes)))
    if xforms is None:
        xforms = sg.identity_xform(n_inst)
    s = sg.Scene(verts=verts, quads=quads, proto_vert_off=np.array(vo, np.int64),
                 proto_quad_off=np.array(qo, np.int64), albedo=albedo,
                 inst_proto=np.asarray(protos, np.int32), inst_xform=np.asarray(xforms, np.float32).reshape(-1, 12))
    s.validate()
    return s


def floor_scene(albedo=0.5, half=5000.0, extra=None):
    """Large floor quad at z = 0, shifted by half/2 along x and y so that its
    diagonal (x + y = half) stays far from the origin, where the test cameras look
    (a bounce ray leaving next to the diagonal may meet the other half at t ~ 0)."""
    c = 0.5 * half
    meshes = [axis_quad(-half + c, half + c, -half + c, half + c, 0.0)]
    albs = [albedo]
    if extra is not None:
        for m, a in extra:
            meshes.append(m)
            albs.append(a)
    return multi_mesh_scene(meshes, albs)


def rotation(seed):
    return sg.shoemake_rotations(np.random.default_rng(seed), 1)[0]


def rotate_scene(scene, R):
    """Apply the world rotation R (3x3) to every instance transform."""
    X = scene.inst_xform.astype(np.float64).reshape(-1, 3, 4)
    Y = np.einsum("ij,njk->nik", R, X)
    s = sg.Scene(verts=scene.verts, quads=scene.quads, proto_vert_off=scene.proto_vert_off,
                 proto_quad_off=scene.proto_quad_off, albedo=scene.albedo, inst_proto=scene.inst_proto,
                 inst_xform=Y.reshape(-1, 12).astype(np.float32))
    return s


def form_factor_corner(a, b, c):
    """Differential area to a parallel a x b rectangle at distance c whose corner lies on
    the element's normal (standard radiative view-factor catalogue closed form)."""
    X, Y = a / c, b / c
    return (1.0 / (2 * math.pi)) * (X / math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X))
                                    + Y / math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y)))


def shell_scene(seed=3, n=6, radius=1.0, noise=0.05):
    rng = np.random.default_rng(seed)
    v, q = sg.shell_proto(rng, n, radius, noise)
    return sg.single_mesh_scene(v, q), v, q
