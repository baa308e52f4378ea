"""Host-side behaviour of bench.py that needs no GPU: it refuses more than one
GPU with a message, and the profile lookup returns the committed counters only
for the kernel sources they were taken from."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_counters_follow_the_kernel_sources():
    """Counters are read only under the source hash recorded with them."""
    import re
    b = _bench()
    txt = open(os.path.join(ROOT, "profiles", b.TRAFFIC_FILE)).read()
    recorded = re.search(r"sources_hash:\s*(\w+)", txt).group(1)
    traffic, valu = b.measured_counters(recorded)
    assert traffic is not None and traffic > 0 and valu is not None and 0 < valu <= 1
    assert b.measured_counters("0000000000000000") == (None, None)
    assert len(b.kernel_sources_hash()) == len(recorded)
