"""The allocation-free ray query (rtq_trace_closest_noalloc, claim counters in a
static device array) called through the C-ABI: its hits equal those of
rtq_trace_closest with the persistent scheduler bit for bit, on two calls in a
row, the second with fewer rays (the shared counters are cleared per call)."""
import ctypes

import numpy as np
import pytest

from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import assert_hits_identical, camera_rays, log

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")


def _noalloc(S, rays_np, **opts):
    import torch
    n = rays_np.shape[0]
    R = torch.from_numpy(np.ascontiguousarray(rays_np, dtype=np.float32)).cuda()
    (soa, ex), st = rtq._rays_struct(R)
    out = [torch.full((n,), -3.0, device="cuda") for _ in range(3)] + \
          [torch.full((n,), -7, dtype=torch.int32, device="cuda") for _ in range(2)]
    hs = rtq._Hits(*[t.data_ptr() for t in out], None)
    o = rtq._trace_opts(**opts)
    rc = rtq.load_library().rtq_trace_closest_noalloc(S.handle, ctypes.byref(st), n, ctypes.byref(hs),
                                                      ctypes.byref(o), rtq._stream())
    assert rc == 0, rtq.load_library().rtq_last_error()
    torch.cuda.synchronize()
    return dict(t=out[0].cpu().numpy(), u=out[1].cpu().numpy(), v=out[2].cpu().numpy(),
                inst=out[3].cpu().numpy(), prim=out[4].cpu().numpy())


def _ref(S, rays_np, **opts):
    import torch
    h = rtq.trace_closest(S, torch.from_numpy(np.ascontiguousarray(rays_np, dtype=np.float32)).cuda(),
                          scheduler=rtq.SCHED_PERSISTENT, **opts)
    torch.cuda.synchronize()
    return dict(t=h.t.cpu().numpy(), u=h.u.cpu().numpy(), v=h.v.cpu().numpy(), inst=h.inst.cpu().numpy(),
                prim=h.prim.cpu().numpy())


def test_noalloc_trace_equals_persistent_trace():
    log("case: allocation-free ray query, config 1")
    scene, cams, _ = sg.config1()
    S = rtq.Scene(scene)
    rng = np.random.default_rng(41)
    big = np.concatenate([camera_rays(cams, rng, 60000), sg.random_rays(rng, 40000, -80, 80, -50, 50)])
    small = big[rng.choice(big.shape[0], 3001, replace=False)]
    for opts in (dict(node_format=rtq.RTQ_NODE_Q8), dict(node_format=rtq.RTQ_NODE_FP32, refill=1, block=64)):
        for rays in (big, small):
            a = _noalloc(S, rays, **opts)
            b = _ref(S, rays, **opts)
            assert_hits_identical(b, a, f"noalloc {opts} n={rays.shape[0]}")
            assert (a["inst"] >= 0).mean() > 0.05
        log(f"  {opts}: {big.shape[0]} then {small.shape[0]} rays, hits bit-identical")
    # argument errors are reported before anything is enqueued
    import torch
    (soa, ex), st = rtq._rays_struct(torch.zeros((4, 8), device="cuda"))
    assert rtq.load_library().rtq_trace_closest_noalloc(S.handle, ctypes.byref(st), 4, None, None, None) == -1
    # 2^31 rays: LIMIT, returned before any array is read (these pointers are never used)
    dummy = rtq._Hits(1, 1, 1, 1, 1, None)
    assert rtq.load_library().rtq_trace_closest_noalloc(S.handle, ctypes.byref(st), 2 ** 31, ctypes.byref(dummy),
                                                        None, None) == -5
