"""Image-parallel decomposition on one GPU (Section 5.5: the frame's tiles, or
views, are dealt to workers that each render their share, and the shares are
gathered into the frame).  Every path draws its random numbers by (pixel of the
whole view, sample, view id, bounce), so rendering disjoint tile or view sets in
separate calls and gathering them must reproduce the single call bit for bit --
the property a multi-GPU split relies on.  Also: the accumulation kernel leaves
pixels outside every view untouched, and graph replays follow a moved view."""
import ctypes
import dataclasses

import numpy as np
import pytest

from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

Q8P = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
KINDS = [Q8P, dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN),
         dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_MEGAKERNEL)]


def _np(img):
    import torch
    torch.cuda.synchronize()
    return img.cpu().numpy()


def _tiles(w, h, tw, th):
    """Row-major tiles of a w x h view; the last column and row are ragged."""
    return [(x, y, min(tw, w - x), min(th, h - y)) for y in range(0, h, th) for x in range(0, w, tw)]


def _gather_tiles(full_w, full_h, parts):
    """parts: list of (tile list, packed image of those tiles) -> full image."""
    out = np.full(full_w * full_h, np.nan, np.float32)
    for tiles, img in parts:
        off = 0
        for (x, y, tw, th) in tiles:
            blk = img[off:off + tw * th].reshape(th, tw)
            v = out.reshape(full_h, full_w)[y:y + th, x:x + tw]
            assert np.isnan(v).all(), "tiles overlap"
            out.reshape(full_h, full_w)[y:y + th, x:x + tw] = blk
            off += tw * th
    assert not np.isnan(out).any(), "tiles do not cover the view"
    return out


@pytest.mark.parametrize("k", [2, 3, 8])
def test_tile_shards_equal_single_call_config1(k):
    """Config 1 (one 128 x 128 view, depth 3): 24 x 20 tiles (ragged at the right
    and bottom) dealt round-robin to k workers, each worker one render call of
    all its tiles; the gathered frame equals the single call bit for bit for
    three schedulers, and so do the path counts."""
    import torch
    log(f"case: tile shards, config 1, k = {k}")
    scene, cams, st = sg.config1()
    st.frame = 5
    S = rtq.Scene(scene)
    c = cams[0]
    tiles = _tiles(c.w, c.h, 24, 20)
    for kw in KINDS:
        full = _np(rtq.render(S, cams, st, **kw))
        parts = []
        total = np.zeros(4, np.uint64)
        for j in range(k):
            mine = tiles[j::k]
            tc = [dataclasses.replace(c, view_id=0, tile=t) for t in mine]
            cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
            parts.append((mine, _np(rtq.render(S, tc, st, counters=cnt, **kw))))
            total += cnt.cpu().numpy()
        got = _gather_tiles(c.w, c.h, parts)
        assert np.array_equal(got.view(np.uint32), full.view(np.uint32)), (k, kw)
        cnt1 = torch.zeros(4, dtype=torch.uint64, device="cuda")
        rtq.render(S, cams, st, counters=cnt1, **kw)
        assert np.array_equal(total, cnt1.cpu().numpy()), (kw, total, cnt1)
    log(f"  {len(tiles)} tiles over {k} calls: gathered frame bit-identical")


def _config5_small():
    scene, cams, st = sg.config5(scale=0.001)
    return scene, cams, st


@pytest.mark.parametrize("k", [2, 3, 8])
def test_view_shards_equal_single_call_config5_views(k):
    """Config 5's 64 uneven square views (sides 64..1024, depth 6) over a
    40 000-instance island: the views split into k sets by a greedy balance of
    pixel counts, each set one call with the views' global ids; the gathered
    views equal the single 64-view call bit for bit."""
    log(f"case: view shards, config-5 views, k = {k}")
    scene, cams, st = _config5_small()
    S = rtq.Scene(scene)
    full = _np(rtq.render(S, cams, st, **Q8P))
    offs = np.cumsum([0] + [c.w * c.h for c in cams])
    # greedy: largest view first onto the least loaded set
    load = [0] * k
    sets = [[] for _ in range(k)]
    for v in sorted(range(len(cams)), key=lambda v: -cams[v].w * cams[v].h):
        j = int(np.argmin(load))
        sets[j].append(v)
        load[j] += cams[v].w * cams[v].h
    got = np.full(full.shape, np.nan, np.float32)
    for views in sets:
        views = sorted(views)
        sub = [dataclasses.replace(cams[v], view_id=v) for v in views]
        img = _np(rtq.render(S, sub, st, **Q8P))
        o = 0
        for v in views:
            n = cams[v].w * cams[v].h
            got[offs[v]:offs[v] + n] = img[o:o + n]
            o += n
    assert not np.isnan(got).any()
    assert np.array_equal(got.view(np.uint32), full.view(np.uint32))
    log(f"  loads {load}: gathered views bit-identical")


def _render_structs(S, arr, n, st, images, **kw):
    o = rtq.render_opts(st, **kw)
    rc = rtq.load_library().rtq_render(S.handle, ctypes.cast(arr, ctypes.c_void_p), n, st.spp, st.depth,
                                       ctypes.byref(o), images.data_ptr(), rtq._stream())
    if rc != 0:
        raise rtq.RtqError(rc, rtq.load_library().rtq_last_error().decode())


def test_image_gaps_stay_untouched_and_graphs_follow_offsets():
    """Regression: views placed after a gap (the first view at an offset > 0,
    another gap between views) -- the accumulation writes only the views' own
    pixels, each equal bit for bit to the view rendered at offset 0; a captured
    graph replayed after a view's offset moved writes the moved view (the
    replay is keyed by the camera layout), equal to the eager call."""
    import torch
    log("case: image gaps and graph keys")
    scene = sg.tiny_scene(21, n_inst=24, n_protos=3, nq=8, spread=3.0)
    S = rtq.Scene(scene)
    cams = [sg.Camera((0.0, -12.0, 2.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 45.0, 37, 23),
            sg.Camera((9.0, 4.0, 6.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 60.0, 64, 64)]
    st = sg.light_settings(2, 4, 77)
    ref = _np(rtq.render(S, cams, st, **Q8P))
    n0, n1 = cams[0].w * cams[0].h, cams[1].w * cams[1].h
    # one buffer for every layout: a replay keyed only by the buffers and the
    # path count would accumulate the first layout's pixel range
    img = torch.empty(1000 + n0 + 333 + n1 + 50, device="cuda")
    for graph in (False, True):
        for gap0, gap1 in ((77, 5), (1000, 333)):
            arr, _ = rtq.camera_structs(cams)
            arr[0].img_offset = gap0
            arr[1].img_offset = gap0 + n0 + gap1
            img.fill_(-7.5)
            _render_structs(S, arr, 2, st, img, graph=graph, **Q8P)
            got = _np(img)
            assert (got[:gap0] == -7.5).all() and (got[gap0 + n0:gap0 + n0 + gap1] == -7.5).all()
            assert (got[gap0 + n0 + gap1 + n1:] == -7.5).all()
            assert np.array_equal(got[gap0:gap0 + n0].view(np.uint32), ref[:n0].view(np.uint32))
            assert np.array_equal(got[gap0 + n0 + gap1:gap0 + n0 + gap1 + n1].view(np.uint32),
                                  ref[n0:].view(np.uint32))
    log("  gaps untouched; eager and replayed views equal the packed render")
