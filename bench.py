#!/usr/bin/env python3
"""Throughput of the instanced-quad path tracer on one MI355X.

Workload (one step = one path-traced frame of the whole hot path): the
config-2 scene -- 256 prototypes (grids with long thin quads and closed
cube-sphere shells, 2k-200k quads each), 1M randomly rotated and scaled
instances on a 2 km height field of 4M quads -- seen from two 1920x1080 views
(overview and ground level), 1 sample per pixel, up to 8 closest-hit rays per
path with next-event estimation.  Inputs are seeded and synthetic and resident
in HBM before timing starts.

Reported (one JSON line):
  value / ms_per_step  Mrays/s and ms/frame of the quantized-node persistent
                       wavefront path (8-bit nodes, one launch per frame);
  plain_fp32           the same for FP32 nodes and the multi-kernel scheduler,
                       at bit-identical images;
  incoherent           closest-hit throughput on the frame's bounce >= 1 rays,
                       quantized-persistent vs FP32-plain, at bit-identical hits;
  roofline             algorithmic traversal bytes of the persistent kernel per
                       launch over its measured duration, against 8 TB/s;
  cpu_baseline         the FP64 oracle on a bounded pixel sample, host cores.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_NODE = {1: 128, 2: 64}   # bytes per 4-wide node: FP32, 8-bit
B_INST = 64                # instance record
B_QUAD = 48                # four FP32 vertices
B_RAY, B_HIT = 32, 20      # ray in, hit out
B_SHADE = 4 + 48           # albedo + quad vertices for the normal, per shaded hit


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2001_02620_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2001_02620_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_render_persistent_q8_config2.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"sources_hash:\s*(\w+)", txt)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_key:
        return None
    return float(b.group(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-pixels", type=int, default=2000000, help="pixels of the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--incoherent-rays", type=int, default=16_000_000)
    ap.add_argument("--scale", type=float, default=1.0, help="scene scale (1.0 = the full configuration)")
    ap.add_argument("--profile", action="store_true", help="only the timed quantized-persistent frames")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: this build has no multi-GPU path "
                                   "(image-parallel sharding is described in the design notes, not built); "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2001_02620_amd as rtq
    from paper_2001_02620_amd import scenegen as sg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(2 ** 28, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 5 x 1 GiB")
        return
    t0 = time.time()
    scene, cams, st = sg.config2(scale=args.scale)
    log(f"scene: {scene.n_quads} unique quads, {scene.n_instances} instances, "
        f"{scene.instanced_quads():.3e} instanced quads ({time.time() - t0:.1f} s)")
    t0 = time.time()
    S = rtq.Scene(scene)
    info = S.info()
    log(f"build: {time.time() - t0:.1f} s, device {info['device_bytes'] / 2**30:.2f} GiB, "
        f"TLAS depth {info['tlas_depth']}, BLAS depth {info['blas_depth_max']}")
    n_pix = sum(c.w * c.h for c in cams)
    img = torch.empty(n_pix, device="cuda")
    Q8P = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    F32 = dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)

    def frame(frame_idx, counters=None, **kw):
        st.frame = frame_idx
        rtq.render(S, cams, st, images=img, counters=counters, **kw)

    def timed(kw, steps, warmup):
        for i in range(warmup):
            frame(1000 + i, **kw)
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(steps):
            evs[i][0].record()
            frame(i, counters=cnt, **kw)
            evs[i][1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ev_ms = [a.elapsed_time(b) for a, b in evs]
        c = cnt.cpu().numpy().astype(np.float64)
        return dict(wall_ms=1e3 * wall / steps, ev_ms=float(np.mean(ev_ms)), ev_min=float(np.min(ev_ms)),
                    ev_max=float(np.max(ev_ms)), closest=c[0] / steps, shadow=c[1] / steps,
                    incoherent=c[2] / steps, rays=(c[0] + c[1]) / steps)

    if args.profile:
        r = timed(Q8P, args.steps, args.warmup)
        log(f"profile run: {r}")
        return

    # ---- equal images between the two paths (frame 0), visits for the roofline
    frame(0, **F32)
    a = img.clone()
    frame(0, **Q8P)
    b = img.clone()
    torch.cuda.synchronize()
    equal_images = bool(torch.equal(a.view(torch.int32), b.view(torch.int32)))
    assert equal_images, "quantized-persistent and FP32-plain images differ"
    visits = {}
    for name, kw in (("q8_persistent", Q8P), ("fp32_plain", F32)):
        v = torch.zeros(4, dtype=torch.uint64, device="cuda")
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        st.frame = 0
        rtq.render(S, cams, st, images=img, counters=cnt, visits=v, **kw)
        torch.cuda.synchronize()
        vv = v.cpu().numpy().astype(np.float64)
        cc = cnt.cpu().numpy().astype(np.float64)
        visits[name] = dict(tlas=vv[0], inst=vv[1], blas=vv[2], quads=vv[3], closest=cc[0], shadow=cc[1])
    log(f"visits: {visits}")

    # ---- timed frames
    q8 = timed(Q8P, args.steps, args.warmup)
    log(f"q8 persistent: {q8}")
    f32 = timed(F32, args.steps, args.warmup)
    log(f"fp32 plain: {f32}")
    ablation = {}
    for name, kw in (("q8_plain", dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PLAIN)),
                     ("fp32_persistent", dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PERSISTENT))):
        r = timed(kw, max(3, args.steps // 2), 1)
        ablation[name] = dict(ms_per_frame=r["wall_ms"], mrays_s=r["rays"] / (r["wall_ms"] * 1e3))
    ablation["q8_persistent"] = dict(ms_per_frame=q8["wall_ms"], mrays_s=q8["rays"] / (q8["wall_ms"] * 1e3))
    ablation["fp32_plain"] = dict(ms_per_frame=f32["wall_ms"], mrays_s=f32["rays"] / (f32["wall_ms"] * 1e3))

    # ---- incoherent rays: bounce >= 1 extension rays of frame 0
    cap = args.incoherent_rays
    dump = torch.empty(8 * cap, device="cuda")
    dcount = torch.zeros(1, dtype=torch.uint64, device="cuda")
    st.frame = 0
    rtq.render(S, cams, st, images=img, dump_rays=dump, dump_count=dcount, **F32)
    torch.cuda.synchronize()
    nd = int(min(int(dcount.cpu().item()), cap))
    rays = dump.view(8, cap)[:, :nd].t()  # [n, 8] view of the SoA dump (copied to SoA again by the binding)
    rays = rays.contiguous()
    inc = {}
    hits_ref = None
    for name, kw in (("fp32_plain", dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)),
                     ("q8_persistent", dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT))):
        h = rtq.trace_closest(S, rays, **kw)
        torch.cuda.synchronize()
        if hits_ref is None:
            hits_ref = h
        else:
            same = all(torch.equal(getattr(h, k).view(torch.int32), getattr(hits_ref, k).view(torch.int32))
                       for k in ("t", "u", "v", "inst", "prim"))
            assert same, "incoherent hits differ between node formats / schedulers"
        reps = max(3, args.steps // 2)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(reps):
            rtq.trace_closest(S, rays, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - w0) / reps
        inc[name] = dict(ms=1e3 * dt, mrays_s=nd / dt / 1e6)
    log(f"incoherent ({nd} rays): {inc}")

    # ---- roofline of the persistent kernel (algorithmic bytes per launch)
    v = visits["q8_persistent"]
    alg_bytes = ((v["closest"] + v["shadow"]) * (B_RAY + B_HIT) + v["tlas"] * B_NODE[2] + v["inst"] * B_INST +
                 v["blas"] * B_NODE[2] + v["quads"] * B_QUAD + v["closest"] * B_SHADE)
    kern_s = q8["ev_ms"] * 1e-3
    achieved = alg_bytes / kern_s / 1e9
    tr = measured_traffic(kernel_sources_hash())

    # ---- CPU baseline: the oracle on a bounded sample of the same frame
    cpu = None
    if not args.no_cpu:
        import oracle
        o = oracle.OracleScene(scene)
        rng = np.random.default_rng(0)
        pix = np.sort(rng.choice(n_pix, size=min(args.cpu_pixels, n_pix), replace=False))
        st.frame = 0
        w0 = time.perf_counter()
        _, fl, stats = o.render(cams, st, pixels=pix)
        dt = time.perf_counter() - w0
        cpu = {"value": (stats["closest"] + stats["shadow"]) / dt / 1e6, "unit": "Mrays/s",
               "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"{pix.size} random pixels of frame 0 (both views), all paths, FP64 with flags; "
                         f"{dt:.1f} s, {int(stats['closest'] + stats['shadow'])} rays, "
                         f"{100 * fl.mean():.1f}% pixels flagged"}
        log(f"cpu baseline: {cpu}")

    value = q8["rays"] / (q8["wall_ms"] * 1e3)
    out = {
        "metric": "incoherent Mrays/s + ms/frame, quantized-wavefront vs plain FP32 at equal hits",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(q8["wall_ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded config-2 generator)",
        "config": {
            "workload": "config2: 256 prototypes + 2048^2 terrain (%d unique quads), %d instances, "
                        "2 views 1920x1080, 1 spp, depth 8" % (scene.n_quads, scene.n_instances),
            "node_format": "q8", "scheduler": "persistent", "parallelism": "single GPU",
        },
        "rays_per_frame": q8["rays"],
        "rays_per_pixel": q8["rays"] / n_pix,
        "plain_fp32": {"ms_per_frame": round(f32["wall_ms"], 3),
                       "mrays_s": round(f32["rays"] / (f32["wall_ms"] * 1e3), 2)},
        "speedup_vs_plain_fp32": round(f32["wall_ms"] / q8["wall_ms"], 3),
        "equal_images": equal_images,
        "incoherent": {"rays": nd, "equal_hits": True,
                       "q8_persistent_mrays_s": round(inc["q8_persistent"]["mrays_s"], 2),
                       "fp32_plain_mrays_s": round(inc["fp32_plain"]["mrays_s"], 2),
                       "speedup": round(inc["q8_persistent"]["mrays_s"] / inc["fp32_plain"]["mrays_s"], 3)},
        "ablation": {k: {kk: round(vv, 3) for kk, vv in d.items()} for k, d in ablation.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if tr is None else tr,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_render_persistent<Q8>", "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_ms": round(q8["ev_ms"], 3)},
        "cpu_baseline": cpu,
        "scene": {"build_s": round(info["build_seconds"], 2), "device_gib": round(info["device_bytes"] / 2**30, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
