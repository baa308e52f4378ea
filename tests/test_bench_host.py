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
    assert b.committed_counters("no_such_file.md", b.kernel_sources_hash()) == (None,) * 5
    for name in (b.COUNTERS_FILE, b.COUNTERS_FRAME_FILE):
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        recorded = re.search(r"sources_hash:\s*(\w+)", open(path).read()).group(1)
        traffic, valu, hbm, insts, lanes = b.committed_counters(name, recorded)
        assert traffic is not None and traffic > 0 and valu is not None and 0 < valu < 2 and hbm > 0
        assert insts is None or insts > 0
        assert lanes is None or 0 < lanes <= 64
        assert b.committed_counters(name, "0000000000000000") == (None,) * 5
        assert len(b.kernel_sources_hash()) == len(recorded)


def test_roofline_names_the_measured_bound():
    """The roofline's bound is the larger of the measured HBM fraction and the
    VALU issue fraction; without counters it is the HBM roofline of the
    algorithmic bytes."""
    b = _bench()
    r = b.roofline(4e9, 1.0, (None,) * 5, "k")
    assert r["bound"] == "hbm" and abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - 0.5) < 1e-9
    r = b.roofline(4e9, 1.0, (2e9, 0.9, 2000.0, None, None), "k")
    assert r["bound"] == "alu" and abs(r["frac"] - 0.9) < 1e-9 and r["peak"] == round(b.VALU_PEAK_TOPS, 2)
    assert abs(r["algorithmic_hbm"]["frac"] - 0.5) < 1e-9
    # with the launch's instruction count: lane-operations over the live time
    insts = 0.45 * b.VALU_PEAK_TOPS * 1e12 * 1e-3 / 64
    r = b.roofline(4e9, 1.0, (2e9, 0.9, 2000.0, insts, 40.0), "k")
    assert r["valu_active_lanes_per_inst"] == 40.0
    assert r["bound"] == "alu" and abs(r["frac"] - 0.45) < 1e-9
    r = b.roofline(4e9, 1.0, (6e9, 0.5, 6000.0, None, None), "k")
    assert r["bound"] == "hbm" and r["measured_hbm_frac"] == 0.75
