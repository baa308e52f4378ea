"""Progressive refinement (Section 5.4: one sample per pixel per frame, frames
accumulated over time): K frames rendered with accumulate = 0..K-1 leave the
mean of the K frame images, equal in every scheduler and under graph replay,
and equal to the mean of the oracle's frames on the pixels it flags in none."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import log, replay_check_pixels
from tests.test_gpu_render import SCHEDS, _multi_view_scene

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")

K = 4


def _progressive(S, cams, st, **kw):
    import torch
    total = sum(c.w * c.h for c in cams)
    img = torch.full((total,), float("nan"), device="cuda")
    for f in range(K):
        rtq.render(S, cams, dataclasses.replace(st, frame=f), images=img, accumulate=f, **kw)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def test_progressive_frames_match_mean_of_oracle_frames():
    log("case: progressive accumulation")
    scene, cams = _multi_view_scene()
    st = sg.RenderSettings(spp=1, depth=4, seed=31)
    S = rtq.Scene(scene)
    kws = [SCHEDS[0], SCHEDS[3], SCHEDS[5], dict(SCHEDS[3], graph=True)]
    imgs = [_progressive(S, cams, st, **kw) for kw in kws]
    for img, kw in zip(imgs[1:], kws[1:]):
        assert (img.view(np.uint32) == imgs[0].view(np.uint32)).all(), kw
    o = oracle.OracleScene(scene)
    frames, flags = [], []
    for f in range(K):
        img, fl, _ = o.render(cams, dataclasses.replace(st, frame=f))
        frames.append(img)
        flags.append(fl != 0)
    ref = np.mean(frames, axis=0)
    ok = ~np.any(flags, axis=0)
    assert ok.mean() > 0.9
    err = np.abs(imgs[0].astype(np.float64) - ref)
    bad = ok & (err > 1e-4 * np.abs(ref) + 1e-6)
    assert not bad.any(), (np.nonzero(bad)[0][:8], imgs[0][bad][:8], ref[bad][:8])
    # pixels flagged in some frame: each frame's paths are traced alone and
    # checked along their own rays (replay_check_pixels), and the running mean
    # is re-formed in FP32 from them exactly as the accumulation forms it
    idx = np.nonzero(~ok)[0]
    run = np.zeros(idx.size, np.float32)
    for f in range(K):
        stf = dataclasses.replace(st, frame=f)
        m = np.zeros(ref.size, np.float32)
        for j, g in enumerate(idx):
            offs = np.cumsum([0] + [c.w * c.h for c in cams])
            view = int(np.searchsorted(offs, g, side="right") - 1)
            nv, vi, vf, esc, rad = rtq.render_path_raw(S, cams, stf, view, int(g - offs[view]), 0, **SCHEDS[3])
            m[g] = rad
        tot = replay_check_pixels(rtq, o, S, cams, stf, idx, m, **SCHEDS[3])
        mf = m[idx]
        run = mf if f == 0 else (run + (mf - run) / np.float32(f + 1)).astype(np.float32)
    assert np.array_equal(run.view(np.uint32), imgs[0][idx].view(np.uint32))
    log(f"  {idx.size} pixels flagged in some frame: replayed, checked and re-accumulated bit for bit")
    # the frames differ (independent samples per frame), so the mean is not one frame
    assert np.abs(frames[0] - frames[1]).max() > 1e-3


def test_accumulate_argument_error():
    import torch
    scene, cams = _multi_view_scene()
    S = rtq.Scene(scene)
    with pytest.raises(rtq.RtqError):
        rtq.render(S, cams, sg.RenderSettings(spp=1, depth=2), accumulate=-1)
    torch.cuda.synchronize()
