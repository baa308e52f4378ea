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
  value / ms_per_step  Mrays/s and ms/frame of the quantized wavefront (8-bit
                       nodes; ray generation, shading and shadow resolution as
                       kernels per bounce; closest-hit and shadow traversal as
                       persistent lane-refilling kernels);
  frame_ms_percentiles p10 / p50 / p90 of the timed frames (HIP events);
  plain_fp32           the same for FP32 nodes and one-ray-per-lane traversal
                       kernels, at bit-identical images;
  ablation             node format x scheduler (plain, persistent stages,
                       single persistent megakernel);
  graph_replay         the headline path replayed from a captured HIP graph;
  textured             the headline path with per-face 4x4 textures in place
                       of per-face albedo (equal images in both paths checked);
  area_lights          the headline path with four quad area lights besides
                       the sun (equal images in both paths checked);
  environment          the headline path under a 2048x1024 environment map in
                       place of the constant sky (equal images checked);
  incoherent           closest-hit throughput on the frame's bounce >= 1 rays,
                       quantized-persistent vs FP32-plain, at bit-identical hits;
  roofline             the frame's dominant kernel (the traversal launches, each
                       tracing a bounce's shadow rays with the next bounce's
                       extension rays): algorithmic bytes per launch over its
                       average launch time from HIP events, against 8 TB/s,
                       with the committed counters' HBM traffic and VALU issue
                       rate while the kernel sources are unchanged;
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
# algorithmic bytes per ray of a traversal: ray in, hit out, and per visit
B_NODE = {1: 128, 2: 64}   # 4-wide node: FP32, 8-bit
B_INST = 56                # instance entry: FP32 inverse 3x4, BLAS root, prototype
B_QUAD = 48                # four FP32 vertices
B_RAY, B_HIT = 32, 20
DOMINANT = "k_trace_queue_mixed<Q8> (shadow rays of bounce b + extension rays of bounce b+1)"
TRAFFIC_FILE = "traffic_trace_queue_mixed_q8_config2.md"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2001_02620_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2001_02620_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel_key):
    """HBM bytes per launch and VALU issue rate from the committed rocprofv3
    counter summary: (bytes, VALU wave-instructions per CU-cycle), each None when
    absent or when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    if not os.path.exists(path):
        return None, None
    txt = open(path).read()
    m = re.search(r"sources_hash:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_key:
        return None, None
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    v = re.search(r"valu_issue_per_cu_cycle:\s*([0-9.eE+]+)", txt)
    return (float(b.group(1)) if b else None), (float(v.group(1)) if v else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=16.0, help="target length of the oracle's timed sample")
    ap.add_argument("--cpu-pilot", type=int, default=4096, help="pixels of the pilot that sizes the oracle sample")
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

    def timed(kw, steps, warmup, stage_timing=False):
        for i in range(warmup):
            frame(1000 + i, **kw)
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        if stage_timing:
            rtq.render_timing(S)  # forget earlier timed calls
        w0 = time.perf_counter()
        for i in range(steps):
            evs[i][0].record()
            frame(i, counters=cnt, timing=stage_timing, **kw)
            evs[i][1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ev_ms = [a.elapsed_time(b) for a, b in evs]
        c = cnt.cpu().numpy().astype(np.float64)
        r = dict(wall_ms=1e3 * wall / steps, ev_ms=float(np.mean(ev_ms)), ev_min=float(np.min(ev_ms)),
                 ev_max=float(np.max(ev_ms)), ev_pct={f"p{q}": float(np.percentile(ev_ms, q)) for q in (10, 50, 90)},
                 closest=c[0] / steps, shadow=c[1] / steps,
                 incoherent=c[2] / steps, rays=(c[0] + c[1]) / steps)
        if stage_timing:
            r["stages"] = rtq.render_timing(S)
        return r

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
        v = torch.zeros(8, dtype=torch.uint64, device="cuda")
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        st.frame = 0
        rtq.render(S, cams, st, images=img, counters=cnt, visits=v, **kw)
        torch.cuda.synchronize()
        vv = v.cpu().numpy().astype(np.float64)
        cc = cnt.cpu().numpy().astype(np.float64)
        visits[name] = dict(closest=dict(zip(("tlas", "inst", "blas", "quads"), vv[:4]), rays=cc[0]),
                            shadow=dict(zip(("tlas", "inst", "blas", "quads"), vv[4:]), rays=cc[1]))
    log(f"visits: {visits}")

    # ---- timed frames (the quantized wavefront with HIP events around its stages)
    q8 = timed(Q8P, args.steps, args.warmup, stage_timing=True)
    log(f"q8 persistent: {q8}")
    f32 = timed(F32, args.steps, args.warmup)
    log(f"fp32 plain: {f32}")
    ablation = {}
    for fname, fmt in (("q8", rtq.RTQ_NODE_Q8), ("fp32", rtq.RTQ_NODE_FP32)):
        for sname, sch in (("plain", rtq.SCHED_PLAIN), ("persistent", rtq.SCHED_PERSISTENT),
                           ("megakernel", rtq.SCHED_MEGAKERNEL)):
            key = f"{fname}_{sname}"
            if key == "q8_persistent":
                r = q8
            elif key == "fp32_plain":
                r = f32
            else:
                r = timed(dict(node_format=fmt, scheduler=sch), max(3, args.steps // 2), 1)
            ablation[key] = dict(ms_per_frame=r["wall_ms"], mrays_s=r["rays"] / (r["wall_ms"] * 1e3))
    log(f"ablation: {ablation}")
    # the headline path replayed from a captured HIP graph (same launches)
    g = timed(dict(Q8P, graph=True), args.steps, args.warmup)
    graph_replay = dict(ms_per_frame=g["wall_ms"], mrays_s=g["rays"] / (g["wall_ms"] * 1e3))
    log(f"graph replay: {graph_replay}")

    # ---- the same frame shaded from per-face textures (4 x 4 texels per face,
    # nearest texel at the hit's (u, v)) instead of per-face albedo
    tex_res = 4
    gen = torch.Generator(device="cuda").manual_seed(1234)
    S.set_textures(torch.rand((S.n_quads, tex_res, tex_res), device="cuda", generator=gen) * 0.9 + 0.05)
    frame(0, **F32)
    a = img.clone()
    frame(0, **Q8P)
    torch.cuda.synchronize()
    tex_equal = bool(torch.equal(a.view(torch.int32), img.view(torch.int32)))
    assert tex_equal, "textured images differ between the two paths"
    t = timed(Q8P, max(3, args.steps // 2), 1)
    S.set_textures(None)
    textured = dict(tex_res=tex_res, ms_per_frame=t["wall_ms"], mrays_s=t["rays"] / (t["wall_ms"] * 1e3))
    log(f"textured: {textured}")

    # ---- the same frame with four 100 m x 100 m area lights 400 m above the
    # terrain (besides the sun): one of the five lights sampled per hit
    st.area_lights = tuple((cx - 50.0, cy - 50.0, 400.0, 0.0, 100.0, 0.0, 100.0, 0.0, 0.0, 16.0)
                           for cx in (-400.0, 400.0) for cy in (-400.0, 400.0))
    frame(0, **F32)
    a = img.clone()
    frame(0, **Q8P)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), img.view(torch.int32)), "area-light images differ between the two paths"
    t = timed(Q8P, max(3, args.steps // 2), 1)
    st.area_lights = ()
    area = dict(n_lights=4, ms_per_frame=t["wall_ms"], mrays_s=t["rays"] / (t["wall_ms"] * 1e3))
    log(f"area lights: {area}")

    # ---- the same frame under a 2048 x 1024 environment map instead of the sky
    S.set_environment(torch.rand((1024, 2048), device="cuda", generator=gen) * 0.5)
    frame(0, **F32)
    a = img.clone()
    frame(0, **Q8P)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), img.view(torch.int32)), "environment images differ between the two paths"
    t = timed(Q8P, max(3, args.steps // 2), 1)
    S.set_environment(None)
    envmap = dict(w=2048, h=1024, ms_per_frame=t["wall_ms"], mrays_s=t["rays"] / (t["wall_ms"] * 1e3))
    log(f"environment: {envmap}")

    # ---- incoherent rays: bounce >= 1 extension rays of frame 0
    log("incoherent rays: dumping bounce >= 1 rays")
    cap = args.incoherent_rays
    dump = torch.empty(8 * cap, device="cuda")
    dcount = torch.zeros(1, dtype=torch.uint64, device="cuda")
    st.frame = 0
    rtq.render(S, cams, st, images=img, dump_rays=dump, dump_count=dcount, **F32)
    torch.cuda.synchronize()
    nd = int(min(int(dcount.cpu().item()), cap))
    rays = dump.view(8, cap)[:, :nd].t().contiguous()
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
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            rtq.trace_closest(S, rays, **kw)
        ev1.record()
        torch.cuda.synchronize()
        dt = ev0.elapsed_time(ev1) * 1e-3 / reps
        inc[name] = dict(ms=1e3 * dt, mrays_s=nd / dt / 1e6)
    log(f"incoherent ({nd} rays): {inc}")

    # ---- roofline of the dominant kernel: the traversal launches of the frame
    # (depth + 1 per frame, each tracing one bounce's shadow rays and the next
    # bounce's extension rays); per launch = per frame / launches per frame
    frame_bytes = 0.0
    for kind in ("closest", "shadow"):
        v = visits["q8_persistent"][kind]
        frame_bytes += (v["rays"] * (B_RAY + B_HIT) + v["tlas"] * B_NODE[2] + v["inst"] * B_INST +
                        v["blas"] * B_NODE[2] + v["quads"] * B_QUAD)
    stg = q8["stages"]["closest"]
    launches_per_frame = stg["launches"] / args.steps
    alg_bytes = frame_bytes / launches_per_frame
    kern_ms = stg["ms"] / stg["launches"]
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    tr, valu = measured_counters(kernel_sources_hash())

    # ---- CPU baseline: the oracle on a bounded sample of the same frame, sized
    # from a short pilot so that the timed sample takes about cpu_seconds
    cpu = None
    if not args.no_cpu:
        import oracle
        log("cpu baseline: building the oracle scene")
        o = oracle.OracleScene(scene)
        rng = np.random.default_rng(0)
        order = rng.permutation(n_pix)
        st.frame = 0
        # untimed warm-up of the pilot pixels (pages the oracle's scene in), then
        # the timed pilot
        pilot = np.sort(order[:min(args.cpu_pilot, n_pix)])
        o.render(cams, st, pixels=pilot)
        w0 = time.perf_counter()
        o.render(cams, st, pixels=pilot)
        dt0 = time.perf_counter() - w0
        n_cpu = int(min(n_pix, max(pilot.size, pilot.size * args.cpu_seconds / max(dt0, 1e-3))))
        log(f"cpu baseline: pilot {pilot.size} px in {dt0:.1f} s; timing {n_cpu} px")
        # per-pixel cost varies a lot, so a small pilot drains unevenly over the
        # host threads and underestimates the rate: re-size once if the sample
        # came out well short of its target length
        for attempt in range(2):
            pix = np.sort(order[:n_cpu])
            w0 = time.perf_counter()
            _, fl, stats = o.render(cams, st, pixels=pix)
            dt = time.perf_counter() - w0
            if attempt == 1 or dt >= 0.7 * args.cpu_seconds or n_cpu == n_pix:
                break
            n_cpu = int(min(n_pix, n_cpu * args.cpu_seconds / max(dt, 1e-3)))
            log(f"cpu baseline: {pix.size} px took {dt:.1f} s; timing {n_cpu} px")
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
        "frame_ms_percentiles": {k: round(v, 3) for k, v in q8["ev_pct"].items()},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded config-2 generator)",
        "config": {
            "workload": "config2: 256 prototypes + 2048^2 terrain (%d unique quads), %d instances, "
                        "2 views 1920x1080, 1 spp, depth 8" % (scene.n_quads, scene.n_instances),
            "node_format": "q8", "scheduler": "wavefront, persistent traversal stages",
            "parallelism": "single GPU",
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
        "graph_replay": {k: round(v, 3) for k, v in graph_replay.items()},
        "textured": {k: round(v, 3) if isinstance(v, float) else v for k, v in textured.items()},
        "area_lights": {k: round(v, 3) if isinstance(v, float) else v for k, v in area.items()},
        "environment": {k: round(v, 3) if isinstance(v, float) else v for k, v in envmap.items()},
        "stages_ms_per_frame": {("traversal" if k == "closest" else k): round(d["ms"] / args.steps, 3)
                                for k, d in q8["stages"].items() if k != "shadow"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if tr is None else tr,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": DOMINANT, "algorithmic_bytes_per_launch": alg_bytes,
                     "launches_per_frame": launches_per_frame, "kernel_ms": round(kern_ms, 3),
                     # the launch is bound by VALU issue, not HBM: the measured issue rate
                     "valu_issue": None if valu is None else {
                         "achieved": valu, "peak": 1.0, "frac": valu,
                         "unit": "VALU wave-instructions per CU-cycle (rocprofv3 SQ_INSTS_VALU / GRBM_GUI_ACTIVE)"}},
        "cpu_baseline": cpu,
        "scene": {"build_s": round(info["build_seconds"], 2), "device_gib": round(info["device_bytes"] / 2**30, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
