"""Node width (2, 4 or 8 children per node, chosen per scene at build) never
changes a hit: the box test stays conservative at every width and the leaf test
and the tie-break are the same code, so closest hits, occlusion answers and
rendered frames of 2- and 8-wide quantized trees equal the 4-wide FP32 trees
and the brute-force reference bit for bit, in every scheduler."""
import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import assert_hits_identical, compare_with_oracle, hits_np, log, to_dev

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

WIDTHS = (2, 8)
Q8_VARIANTS = [
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
    # shallow LDS stack: most pushes go to the private spill region
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT, stack_depth=4, refill=1, block=64),
    dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN, stack_depth=8, block=128),
]
FRAME_KINDS = [dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT),
               dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN),
               dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL)]


def _case(cfg):
    rng = np.random.default_rng(23)
    if cfg == "tiny":
        scene = sg.tiny_scene(5, n_inst=6, n_protos=2, nq=9, spread=1.3)
        cams = [sg.Camera((0.0, -9.0, 1.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 50.0, 40, 30)]
        st = sg.RenderSettings(spp=2, depth=4, seed=3)
        rays = np.concatenate([sg.random_rays(rng, 10000, -5, 5, -2, 2), sg.random_rays(rng, 10000, -1, 1, -3, 3)])
    elif cfg == "config1":
        scene, cams, st = sg.config1()
        rays = sg.random_rays(rng, 20000, -80, 80, -50, 50)
    else:
        scene, cams, st = sg.config2(scale=0.01, res=(96, 64))
        rays = sg.random_rays(rng, 20000, [-1000, -1000, 0], [1000, 1000, 150], [-1000, -1000, -50],
                              [1000, 1000, 100])
    return scene, cams, st, rays


def _np(img):
    import torch
    torch.cuda.synchronize()
    return img.cpu().numpy()


@pytest.mark.parametrize("cfg", ["tiny", "config1", "config2_small"])
def test_node_widths_keep_hits_and_frames(cfg):
    log(f"case: node widths, {cfg}")
    scene, cams, st, rays = _case(cfg)
    R = to_dev(rays)
    S4 = rtq.Scene(scene)
    assert S4.info()["node_width"] == 4
    ref = hits_np(rtq.trace_brute(S4, R))
    assert_hits_identical(ref, hits_np(rtq.trace_closest(S4, R, node_format=rtq.RTQ_NODE_FP32,
                                                         scheduler=rtq.SCHED_PLAIN)), "width 4 FP32")
    occ_ref = rtq.trace_occluded(S4, R, node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)
    occ_ref = _np(occ_ref)
    assert np.array_equal(occ_ref != 0, ref["inst"] >= 0)
    st.frame = 1
    img_ref = _np(rtq.render(S4, cams, st, node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN))
    info4 = S4.info()
    S4.close()
    for w in WIDTHS:
        S = rtq.Scene(scene, node_width=w)
        info = S.info()
        log(f"  width {w}: depth {info['tlas_depth']} + {info['blas_depth_max']} levels, "
            f"{info['tlas_nodes'] + info['blas_nodes']} nodes (width 4: {info4['tlas_nodes'] + info4['blas_nodes']})")
        assert info["node_width"] == w and info["formats"] == rtq.RTQ_NODE_Q8
        if w == 8:
            assert info["blas_nodes"] < info4["blas_nodes"]
        else:
            assert info["blas_nodes"] > info4["blas_nodes"]
        assert_hits_identical(ref, hits_np(rtq.trace_brute(S, R)), f"width {w} brute force")
        for var in Q8_VARIANTS:
            assert_hits_identical(ref, hits_np(rtq.trace_closest(S, R, **var)), f"width {w} {var}")
            occ = _np(rtq.trace_occluded(S, R, **var))
            assert np.array_equal(occ, occ_ref), f"width {w} {var}: occlusion differs"
        for kind in FRAME_KINDS:
            st.frame = 1
            img = _np(rtq.render(S, cams, st, **kind))
            assert np.array_equal(img.view(np.uint32), img_ref.view(np.uint32)), f"width {w} {kind}: frame differs"
        S.close()
    o = oracle.OracleScene(scene).trace(rays)
    frac = compare_with_oracle(scene, rays, ref, o)
    log(f"  flagged fraction {frac:.4f}")


def test_node_width_secondary_rays_with_exclusion():
    """Bounce rays that exclude the triangle they leave: the exclusion keys come
    from each scene's own hits (top-level records differ between widths, since
    opened instances follow the tree), the hits do not."""
    import torch
    from tests.gpu_util import camera_rays
    log("case: node widths, secondary rays with exclusion, config 1")
    scene, cams, _ = sg.config1()
    rng = np.random.default_rng(41)
    cr = camera_rays(cams, rng, 20000)
    d = rng.normal(size=(cr.shape[0], 3)).astype(np.float32)
    base = None
    for w in (4, 2, 8):
        S = rtq.Scene(scene, node_width=w)
        h0 = rtq.trace_closest(S, to_dev(cr), want_ref=True, node_format=rtq.RTQ_NODE_Q8,
                               scheduler=rtq.SCHED_PERSISTENT)
        torch.cuda.synchronize()
        hit = (h0.inst >= 0).cpu().numpy()
        t = h0.t.cpu().numpy()
        p = (cr[:, 0:3] + t[:, None] * cr[:, 3:6]).astype(np.float32)
        rays = np.zeros((int(hit.sum()), 8), np.float32)
        rays[:, 0:3] = p[hit]
        rays[:, 3:6] = d[hit]
        rays[:, 7] = np.inf
        ex = h0.ref[torch.from_numpy(hit).cuda()].contiguous()
        R = to_dev(rays)
        hb = hits_np(rtq.trace_brute(S, R, exclude=ex))
        for var in Q8_VARIANTS[:3]:
            assert_hits_identical(hb, hits_np(rtq.trace_closest(S, R, exclude=ex, **var)), f"width {w} {var}")
        if base is None:
            base = (hits_np(h0), hb)
        else:
            assert_hits_identical(base[0], hits_np(h0), f"width {w} camera rays")
            assert_hits_identical(base[1], hb, f"width {w} bounce rays")
        S.close()


def test_node_width_argument_errors():
    scene = sg.tiny_scene(2, n_inst=2, n_protos=1, nq=4, spread=1.0)
    with pytest.raises(rtq.RtqError):
        rtq.Scene(scene, node_width=3)
    with pytest.raises(rtq.RtqError):
        rtq.Scene(scene, node_width=8, formats=rtq.RTQ_NODE_FP32)
    S = rtq.Scene(scene, node_width=8)
    with pytest.raises(rtq.RtqError):
        rtq.trace_closest(S, to_dev(sg.random_rays(np.random.default_rng(1), 10, -1, 1, -1, 1)),
                          node_format=rtq.RTQ_NODE_FP32)
    S.close()


def test_autotuner_chooses_a_width_at_equal_frames():
    """autotune_width builds the scene at each width, refuses a width whose
    frame or hits differ from the 4-wide FP32 reference, and returns the
    fastest with its launch options."""
    import torch
    from paper_2001_02620_amd.autotune import autotune_width
    log("case: width autotuner, config 1")
    scene, cams, st = sg.config1()
    rays = to_dev(sg.random_rays(np.random.default_rng(5), 20000, -80, 80, -50, 50))
    grid = {rtq.SCHED_PERSISTENT: dict(stack_depth=[16], waves_per_cu=[24], block=[256], refill=[16])}
    res = autotune_width(scene, cams, st, widths=(4, 8, 2), grid=grid, reps=1, rays=rays, log=log)
    assert res["best"]["node_width"] in (2, 4, 8)
    assert set(res["widths"]) == {2, 4, 8}
    assert res["best"]["ms"] == min(v["ms"] for v in res["widths"].values())
    torch.cuda.synchronize()


def test_autotuner_chooses_the_opening():
    """autotune_build also tries top-level openings (none, the default, twice
    the instance count), keeps the frames bit-identical and returns the
    fastest pair."""
    from paper_2001_02620_amd.autotune import autotune_build
    log("case: build autotuner (opening), config 1")
    scene, cams, st = sg.config1()
    grid = {rtq.SCHED_PERSISTENT: dict(stack_depth=[16], waves_per_cu=[24], block=[256], refill=[16])}
    res = autotune_build(scene, cams, st, widths=(4,), open_pcts=(-1, 0, 200), grid=grid, reps=1, log=log)
    assert set(res["builds"]) == {(4, -1), (4, 0), (4, 200)}
    ent = {p: v["top_entries"] for (_, p), v in res["builds"].items()}
    assert ent[-1] == scene.n_instances and ent[-1] < ent[0] < ent[200]
    assert res["best"]["ms"] == min(v["ms"] for v in res["builds"].values())
