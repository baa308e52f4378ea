"""A scene build that fails after it has allocated device memory releases all of
it (regression: the failure paths once left the bottom-level arrays and the
build's temporaries allocated)."""
import numpy as np
import pytest

from paper_2001_02620_amd import scenegen as sg
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

rtq = pytest.importorskip("paper_2001_02620_amd")


def test_failed_builds_release_device_memory():
    import torch
    log("case: failed builds release device memory")
    rng = np.random.default_rng(3)
    verts, quads = sg.grid_proto(rng, 256, 256, 1.0, 1.0, 0.05)
    n = 200_000
    R = sg.shoemake_rotations(rng, n)
    X = sg.compose_xforms(R, rng.uniform(0.5, 2.0, n), rng.uniform(-50, 50, (n, 3)))
    X[n // 2, :] = 0.0  # a singular transform: detected after the instance kernels ran
    scene = sg._concat([(verts, quads)], rng, np.zeros(n, np.int32), X)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(4):
        with pytest.raises(rtq.RtqError) as ei:
            rtq.Scene(scene)
        assert ei.value.code == -2, ei.value
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log(f"  free device memory before {free0 / 2**20:.1f} MiB, after four failed builds {free1 / 2**20:.1f} MiB")
    # each failed build held about 40 MB of device memory when it failed
    assert free1 >= free0 - (16 << 20), (free0, free1)
