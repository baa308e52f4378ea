#!/usr/bin/env python3
"""Throughput of the instanced-quad path tracer on one MI355X: incoherent-ray
Mrays/s and ms/frame, quantized-BVH persistent wavefront against plain FP32, at
equal hits.

Workload: configuration 3 -- the island generator grown to 20M randomly
rotated and scaled instances (30 % of them in tight clusters) of 2304
prototypes (noise-displaced grids with long thin quads and closed cube-sphere
shells) over a 2 km height field, 101M unique quads; one 1920x1080 ground-level
view, 4 samples per pixel, up to 8 closest-hit rays per path with next-event
estimation.  Inputs are seeded, synthetic and resident in HBM before timing.

One timed step = one closest-hit query of the frame's incoherent rays: the
first 16M cosine-sampled extension rays of bounce >= 1 of frame 0, each
excluding the triangle it leaves, traced by the quantized-node persistent
kernel (value = those rays per second).  The same rays traced by the FP32-node
one-ray-per-lane kernel must give bit-identical hits before any number is
printed.  Beside it (same JSON line):
  frame                ms/frame (p10/p50/p90) and Mrays/s of whole config-3
                       frames (every stage: ray generation, traversal, shading,
                       shadow rays, accumulation), quantized persistent
                       wavefront vs FP32 plain wavefront, bit-identical images;
  ablation             node format x scheduler frames;
  graph_replay         the headline frame replayed from a captured HIP graph;
  textured, area_lights, environment, principled
                       the headline frame with per-face 4x4 textures, four quad
                       area lights, a 2048x1024 environment map, eight
                       principled materials in three channels;
  config4_adjoint      forward frame and path-replay backward pass at config 4;
  curves               a grass field of 100k tufts of cubic Bezier curves (51M
                       instanced segments) over a quad ground, round (capsule
                       chains) and flat (ray-facing ribbons): frames of both
                       paths (bit-identical) and its bounce rays' closest hits;
  config2              the smaller 1M-instance configuration: frames and
                       incoherent rays, both paths, and node widths 2, 4 and 8
                       (quantized persistent, equal hits and images);
  roofline             the timed kernel: algorithmic bytes per launch (visit
                       counts of the same rays) over its launch time from HIP
                       events, against 8 TB/s; the bound named by the committed
                       rocprofv3 counters (HBM bytes against VALU issue);
  roofline_frame       the same for the frame's dominant kernel;
  cpu_baseline         the FP64 oracle tracing a bounded sample of the same
                       incoherent rays on the host's cores (and on one core).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak with packed FP32 instructions off: one 64-lane instruction per
# SIMD every 4 cycles, 4 SIMDs per CU, 256 CUs at 2.4 GHz (lane-operations/s)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic bytes per ray of a traversal: ray in, hit out, and per visit
B_NODE = {1: 128, 2: 64}   # 4-wide node: FP32, 8-bit
B_NODE_Q8_W = {2: 48, 4: 64, 8: 96}  # quantized node by width
B_INST = 56                # instance entry: FP32 inverse 3x4, BLAS root, prototype
B_QUAD = 48                # four FP32 vertices
B_RAY, B_HIT = 32, 20
DOMINANT = "k_trace_persistent<Q8, closest>"
DOMINANT_FRAME = "k_trace_queue_mixed<Q8> (shadow rays of bounce b + extension rays of bounce b+1)"
COUNTERS_FILE = "counters_trace_persistent_q8_incoherent_config3.md"
COUNTERS_FRAME_FILE = "counters_trace_queue_mixed_q8_config3.md"
METRIC = "incoherent Mrays/s + ms/frame, quantized-wavefront vs plain FP32 at equal hits"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2001_02620_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2001_02620_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_counters(name, kernel_key):
    """Per-launch HBM bytes, VALU issue rate, measured HBM GB/s, VALU
    wave-instructions per launch and enabled lanes per VALU instruction from a
    committed rocprofv3 counter summary, or Nones when absent or taken from
    other sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, None, None, None, None
    txt = open(path).read()
    m = re.search(r"sources_hash:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_key:
        return None, None, None, None, None

    def num(key):
        x = re.search(key + r":\s*([0-9.eE+-]+)", txt)
        return float(x.group(1)) if x else None
    return (num("traffic_bytes_per_launch"), num("valu_issue_per_cu_cycle"), num("hbm_gbs"),
            num("valu_insts_per_launch"), num("valu_active_lanes_per_inst"))


def roofline(alg_bytes, kern_ms, counters, kernel):
    """Roofline object: algorithmic GB/s against HBM peak; the bound is the
    larger of the measured HBM fraction and the VALU issue fraction (committed
    counters of the same sources), and is reported against its own peak."""
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    tr, valu, hbm, insts, lanes = counters
    hbm_frac = None if hbm is None else hbm / HBM_PEAK_GBS
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
           "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
           "kernel": kernel, "algorithmic_bytes_per_launch": alg_bytes, "kernel_ms": round(kern_ms, 4)}
    if valu is not None:
        out["valu_issue_frac"] = valu
        out["measured_hbm_frac"] = None if hbm_frac is None else round(hbm_frac, 4)
        if hbm_frac is None or valu > hbm_frac:
            # issue-bound: VALU lane-operations per second against the issue peak,
            # the launch's wave-instructions (counted by rocprofv3) x 64 lanes over
            # its duration measured here
            lane_ops = insts * 64 / (kern_ms * 1e-3) / 1e12 if insts else valu * VALU_PEAK_TOPS
            out.update({"bound": "alu", "achieved": round(lane_ops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "T VALU lane-ops/s", "frac": round(lane_ops / VALU_PEAK_TOPS, 4),
                        "valu_insts_per_launch": insts, "valu_active_lanes_per_inst": lanes,
                        "algorithmic_hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": round(achieved / HBM_PEAK_GBS, 4)}})
    return out


def visit_bytes(v, rays, fmt=2):
    return rays * (B_RAY + B_HIT) + v[0] * B_NODE[fmt] + v[1] * B_INST + v[2] * B_NODE[fmt] + v[3] * B_QUAD


def compare_widths(rtq, scene, cams, st, cap, log, steps=5, frames=5):
    """Node widths 2, 4 and 8 on one workload: one build per width, the
    quantized persistent kernels.  Frames must equal the 4-wide build's bit for
    bit, and so must the closest hits of the 4-wide frame's first million
    bounce rays (traced without exclusions, whose keys name each build's own
    top-level records).  Each width is timed on the bounce >= 1 rays of its own
    frame 0 with their exclusions (the same rays in its own queue order).
    Returns per width: nodes, depths, incoherent Mrays/s, ms/frame and visits
    per ray."""
    import torch
    q8p = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    n_pix = sum(c.w * c.h for c in cams)
    out, ref = {}, None
    for w in (4, 8, 2):
        torch.cuda.empty_cache()
        t0 = time.time()
        S = rtq.Scene(scene, node_width=w)
        info = S.info()
        build_s = time.time() - t0
        img = torch.empty(n_pix, device="cuda")
        d = torch.empty(12 * cap, device="cuda")
        c = torch.zeros(1, dtype=torch.uint64, device="cuda")
        st.frame = 0
        rtq.render(S, cams, st, images=img, dump_rays=d, dump_count=c, **q8p)
        torch.cuda.synchronize()
        m = int(min(int(c.cpu().item()), cap))
        pl = d.view(12, cap)[:, :m]
        r, e = pl[:8].contiguous(), pl[8:10].view(torch.int32).t().contiguous()
        if ref is None:
            probe = r[:, :min(m, 1 << 20)].contiguous()
            ref = (img.clone(), probe, rtq.trace_closest(S, probe, soa_in=True, **q8p))
        else:
            assert torch.equal(ref[0].view(torch.int32), img.view(torch.int32)), f"width {w}: frame differs"
            h = rtq.trace_closest(S, ref[1], soa_in=True, **q8p)
            torch.cuda.synchronize()
            for k in ("t", "u", "v", "inst", "prim"):
                assert torch.equal(getattr(ref[2], k).view(torch.int32), getattr(h, k).view(torch.int32)), \
                    f"width {w}: hits differ ({k})"
            del h
        v = torch.zeros((m, 4), dtype=torch.int32, device="cuda")
        rtq.trace_closest(S, r, exclude=e, soa_in=True, visits=v, **q8p)
        torch.cuda.synchronize()
        vis = v.to(torch.float64).sum(0).cpu().numpy() / m
        del v
        for _ in range(2):
            rtq.trace_closest(S, r, exclude=e, soa_in=True, **q8p)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(steps):
            rtq.trace_closest(S, r, exclude=e, soa_in=True, **q8p)
        torch.cuda.synchronize()
        inc_ms = (time.perf_counter() - w0) / steps * 1e3
        for i in range(2):
            st.frame = 1000 + i
            rtq.render(S, cams, st, images=img, **q8p)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(frames):
            st.frame = i
            rtq.render(S, cams, st, images=img, **q8p)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - w0) / frames * 1e3
        bn = B_NODE_Q8_W[w]
        out[w] = {"nodes": info["tlas_nodes"] + info["blas_nodes"], "node_bytes": bn,
                  "depth": [info["tlas_depth"], info["blas_depth_max"]], "build_s": round(build_s, 1),
                  "incoherent_rays": m, "incoherent_mrays_s": round(m / inc_ms / 1e3, 2),
                  "incoherent_ms": round(inc_ms, 3), "ms_per_frame": round(fms, 3),
                  "visits_per_ray": [round(float(x), 2) for x in vis],
                  "algorithmic_bytes_per_ray": round(float(B_RAY + B_HIT + (vis[0] + vis[2]) * bn + vis[1] * B_INST
                                                           + vis[3] * B_QUAD), 1)}
        log(f"node width {w}: {out[w]}")
        del S, r, e, pl, d, img
    del ref
    torch.cuda.empty_cache()
    return {"widths": {str(k): v for k, v in out.items()},
            "fastest_incoherent": min(out, key=lambda k: out[k]["incoherent_ms"]),
            "fastest_frame": min(out, key=lambda k: out[k]["ms_per_frame"])}


def curve_field(rtq, sg, args, log, flat=False):
    """Curves (Section 5.2: the scene's curves): a grass field of tuft
    instances -- cubic Beziers traced as chains of capsules -- over a ground
    grid, one 1280x720 view at 4 spp, depth 4.  FP32-plain and
    quantized-persistent frames must be bit-identical; then timed frames, and
    the closest-hit rate of the frame's bounce rays (with the primitive each
    leaves excluded)."""
    import numpy as np
    import torch
    t0 = time.time()
    scene = sg.curve_scene(11, n_inst=args.curve_instances, n_curves=64, spread=40.0, flat=(flat, flat))
    S = rtq.Scene(scene)
    build_s = time.time() - t0
    info = S.info()
    cams = [sg.Camera((0.0, -46.0, 4.0), (0.0, 0.0, 0.3), (0.0, 0.0, 1.0), 50.0, 1280, 720)]
    st = sg.RenderSettings(spp=4, depth=4, seed=7)
    n_pix = 1280 * 720
    img = torch.empty(n_pix, device="cuda")
    Q8P = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    F32 = dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)
    log(f"curves: {scene.n_instances} instances, {info['n_unique_curves']} unique curves "
        f"({info['n_unique_capsules']} capsules), {build_s:.1f} s to generate and build")

    def timed(kw, steps, warmup):
        for i in range(warmup):
            st.frame = 100 + i
            rtq.render(S, cams, st, images=img, **kw)
        cnt = torch.zeros(4, dtype=torch.uint64, device="cuda")
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(steps):
            st.frame = i
            rtq.render(S, cams, st, images=img, counters=cnt, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        c = cnt.cpu().numpy().astype(np.float64)
        return dict(ms_per_frame=round(1e3 * wall / steps, 3), mrays_s=round((c[0] + c[1]) / wall / 1e6, 2),
                    rays_per_frame=(c[0] + c[1]) / steps)

    if args.profile in ("curves", "ribbons"):
        log(f"profile run ({args.profile} frames): {timed(Q8P, args.steps, args.warmup)}")
        return None
    st.frame = 0
    rtq.render(S, cams, st, images=img, **F32)
    ref = img.clone()
    rtq.render(S, cams, st, images=img, **Q8P)
    torch.cuda.synchronize()
    equal = bool(torch.equal(ref.view(torch.int32), img.view(torch.int32)))
    assert equal, "curve frames differ between the quantized-persistent and FP32-plain paths"
    q8 = timed(Q8P, max(3, args.steps // 2), 2)
    f32 = timed(F32, 3, 1)
    # bounce rays of frame 0, traced alone
    cap = 8_000_000
    dump = torch.empty(12 * cap, device="cuda")
    dcount = torch.zeros(1, dtype=torch.uint64, device="cuda")
    st.frame = 0
    rtq.render(S, cams, st, images=img, dump_rays=dump, dump_count=dcount, **F32)
    torch.cuda.synchronize()
    nd = int(min(int(dcount.cpu().item()), cap))
    planes = dump.view(12, cap)[:, :nd]
    rays = planes[:8].contiguous()
    excl = planes[8:10].view(torch.int32).t().contiguous()
    h = rtq.trace_closest(S, rays, exclude=excl, soa_in=True, **Q8P)
    torch.cuda.synchronize()
    on_cap = (np.diff(scene.proto_curve_off) > 0)[scene.inst_proto[np.maximum(h.inst.cpu().numpy(), 0)]]
    hit = h.inst.cpu().numpy() >= 0
    for _ in range(2):
        rtq.trace_closest(S, rays, exclude=excl, soa_in=True, **Q8P)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    w0 = time.perf_counter()
    for _ in range(steps):
        rtq.trace_closest(S, rays, exclude=excl, soa_in=True, **Q8P)
    torch.cuda.synchronize()
    inc = nd * steps / (time.perf_counter() - w0) / 1e6
    kind = "flat ribbons" if flat else "round curves (capsule chains)"
    out = {"workload": f"grass field of {kind}: {scene.n_instances - 1} tufts of 64 curves (2 prototypes, rotated and "
                       f"scaled) over a 6x6 quad ground, {info['n_unique_capsules']} unique segments, "
                       f"{8 * 64 * (scene.n_instances - 1):.3e} instanced segments; 1280x720, 4 spp, depth 4",
           "equal_images": equal, "q8_persistent": q8, "fp32_plain": f32,
           "speedup": round(f32["ms_per_frame"] / q8["ms_per_frame"], 3),
           "incoherent": {"rays": nd, "q8_persistent_mrays_s": round(inc, 2),
                          "hit_fraction": round(float(hit.mean()), 4),
                          "capsule_hit_fraction": round(float((hit & on_cap).mean()), 4)},
           "build_s": round(info["build_seconds"], 2), "device_gib": round(info["device_bytes"] / 2**30, 3)}
    log(f"curves: {out}")
    S.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-config2", action="store_true")
    ap.add_argument("--incoherent-rays", type=int, default=16_000_000)
    ap.add_argument("--scale", type=float, default=1.0, help="scene scale (1.0 = the full configuration)")
    ap.add_argument("--curve-instances", type=int, default=100_000, help="tufts of the curve field")
    ap.add_argument("--no-curves", action="store_true")
    ap.add_argument("--open-area-pct", type=int, default=0,
                    help="config 3's build: area limit of opened subtrees in percent (0: the library's 150)")
    ap.add_argument("--open-pct", type=int, default=200,
                    help="config 3's build: top-level entries added by opening instances, in percent of the instance "
                         "count (the library's default is 50; at config 3, 25/50/100/200/400 measured 27.0/22.7/"
                         "21.4/20.3/21.4 ms per incoherent query, and frames of 56.7 ms at 50, 50.6 at 200, 52.8 at "
                         "400 -- the pick of autotune_build; config 2 keeps the default, its best)")
    ap.add_argument("--profile", choices=("incoherent", "frame", "curves", "ribbons"), default=None,
                    help="only the timed incoherent queries, or only timed frames (for rocprofv3)")
    ap.add_argument("--widths", action="store_true",
                    help="only compare node widths 2, 4 and 8 on the configuration-3 workload (one build each)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: this build has no multi-GPU path "
                                   "(image-parallel sharding is described in the design notes and shown on one "
                                   "GPU by the shard tests); run with --gpus 1"}))
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
    if args.profile in ("curves", "ribbons"):
        curve_field(rtq, sg, args, log, flat=args.profile == "ribbons")
        return
    t0 = time.time()
    scene, cams, st = sg.config3(scale=args.scale)
    log(f"config 3: {scene.n_quads} unique quads, {scene.n_instances} instances, "
        f"{scene.instanced_quads():.3e} instanced quads ({time.time() - t0:.1f} s)")
    if args.widths:
        print(json.dumps({"config3_node_width": compare_widths(rtq, scene, cams, st, args.incoherent_rays, log,
                                                             steps=args.steps, frames=args.steps)}))
        return
    t0 = time.time()
    S = rtq.Scene(scene, open_pct=args.open_pct, open_area_pct=args.open_area_pct)
    info = S.info()
    log(f"build: {time.time() - t0:.1f} s, device {info['device_bytes'] / 2**30:.2f} GiB, "
        f"{info['n_top_entries']} top-level entries")
    n_pix = sum(c.w * c.h for c in cams)
    img = torch.empty(n_pix, device="cuda")
    Q8P = dict(node_format=rtq.RTQ_NODE_Q8, scheduler=rtq.SCHED_PERSISTENT)
    F32 = dict(node_format=rtq.RTQ_NODE_FP32, scheduler=rtq.SCHED_PLAIN)

    # ---- the incoherent rays: bounce >= 1 extension rays of frame 0, with the
    # triangle each leaves (the images of both paths are bit-identical, so are
    # their rays)
    cap = args.incoherent_rays
    dump = torch.empty(12 * cap, device="cuda")
    dcount = torch.zeros(1, dtype=torch.uint64, device="cuda")
    st.frame = 0
    rtq.render(S, cams, st, images=img, dump_rays=dump, dump_count=dcount, **F32)
    torch.cuda.synchronize()
    nd = int(min(int(dcount.cpu().item()), cap))
    planes = dump.view(12, cap)[:, :nd]
    rays = planes[:8].contiguous()  # structure of arrays [8, n], traced in place
    excl = planes[8:10].view(torch.int32).t().contiguous()
    log(f"incoherent rays: {nd} of {int(dcount.cpu().item())} bounce >= 1 rays of frame 0")

    def query(kw):
        return rtq.trace_closest(S, rays, exclude=excl, soa_in=True, **kw)

    def timed_queries(kw, steps, warmup):
        for _ in range(warmup):
            query(kw)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(steps):
            evs[i][0].record()
            query(kw)
            evs[i][1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = [a.elapsed_time(b) for a, b in evs]
        return dict(wall_ms=1e3 * wall / steps, ev_ms=float(np.mean(ms)),
                    ev_pct={f"p{q}": float(np.percentile(ms, q)) for q in (10, 50, 90)},
                    mrays_s=nd * steps / wall / 1e6)

    if args.profile == "incoherent":
        r = timed_queries(Q8P, args.steps, args.warmup)
        log(f"profile run (incoherent): {r}")
        return

    def frame(frame_idx, counters=None, **kw):
        st.frame = frame_idx
        rtq.render(S, cams, st, images=img, counters=counters, **kw)

    def timed_frames(kw, steps, warmup, stage_timing=False):
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
        ms = [a.elapsed_time(b) for a, b in evs]
        c = cnt.cpu().numpy().astype(np.float64)
        r = dict(wall_ms=1e3 * wall / steps, ev_pct={f"p{q}": float(np.percentile(ms, q)) for q in (10, 50, 90)},
                 closest=c[0] / steps, shadow=c[1] / steps, incoherent=c[2] / steps, rays=(c[0] + c[1]) / steps)
        r["mrays_s"] = r["rays"] / (r["wall_ms"] * 1e3)
        if stage_timing:
            r["stages"] = rtq.render_timing(S)
        return r

    if args.profile == "frame":
        r = timed_frames(Q8P, args.steps, args.warmup)
        log(f"profile run (frames): {r}")
        return

    # ---- equal hits on the incoherent rays (before any number), visit counts
    h_f32 = query(F32)
    h_q8 = query(Q8P)
    torch.cuda.synchronize()
    equal_hits = all(torch.equal(getattr(h_f32, k).view(torch.int32), getattr(h_q8, k).view(torch.int32))
                     for k in ("t", "u", "v", "inst", "prim"))
    assert equal_hits, "incoherent hits differ between the quantized-persistent and FP32-plain kernels"
    hit_frac = float((h_q8.inst >= 0).float().mean().item())
    del h_f32, h_q8
    inc_visits, lane = {}, {}
    for name, fmt in (("q8", rtq.RTQ_NODE_Q8), ("fp32", rtq.RTQ_NODE_FP32)):
        v = torch.zeros((nd, 4), dtype=torch.int32, device="cuda")
        ls = torch.zeros((nd, 2), dtype=torch.int32, device="cuda")
        rtq.trace_closest(S, rays, exclude=excl, soa_in=True, node_format=fmt, scheduler=rtq.SCHED_PERSISTENT,
                          visits=v, lane_stats=ls)
        torch.cuda.synchronize()
        inc_visits[name] = v.to(torch.float64).sum(0).cpu().numpy()
        lsum = ls.to(torch.float64).sum(0).cpu().numpy()
        # a lane does useful work in an iteration when the wave runs its step kind
        # (one visit); live iterations also include waiting and pop-only ones
        lane[name] = {"useful_fraction_of_live_iterations": round(float(inc_visits[name].sum() / lsum[0]), 4),
                      "fp64_edge_reevaluations_per_triangle_test": float(lsum[1] / (2 * inc_visits[name][3])),
                      "fp64_edge_reevaluations": int(lsum[1])}
        del v, ls
    log(f"incoherent visits (per ray): q8 {inc_visits['q8'] / nd}")

    # ---- the timed steps: the quantized persistent kernel on the incoherent rays
    q8_inc = timed_queries(Q8P, args.steps, args.warmup)
    log(f"incoherent, q8 persistent: {q8_inc}")
    f32_inc = timed_queries(F32, max(3, args.steps // 2), 2)
    log(f"incoherent, fp32 plain: {f32_inc}")

    # ---- whole frames: equal images, then timed frames of both paths
    frame(0, **F32)
    a = img.clone()
    frame(0, **Q8P)
    torch.cuda.synchronize()
    equal_images = bool(torch.equal(a.view(torch.int32), img.view(torch.int32)))
    assert equal_images, "quantized-persistent and FP32-plain frames differ"
    fv = torch.zeros(8, dtype=torch.uint64, device="cuda")
    fc = torch.zeros(4, dtype=torch.uint64, device="cuda")
    st.frame = 0
    rtq.render(S, cams, st, images=img, counters=fc, visits=fv, **Q8P)
    torch.cuda.synchronize()
    fvv = fv.cpu().numpy().astype(np.float64)
    fcc = fc.cpu().numpy().astype(np.float64)
    q8f = timed_frames(Q8P, args.steps, args.warmup, stage_timing=True)
    log(f"frames, q8 persistent: {q8f}")
    f32f = timed_frames(F32, max(3, args.steps // 2), 2)
    log(f"frames, fp32 plain: {f32f}")
    ablation = {}
    for fname, fmt in (("q8", rtq.RTQ_NODE_Q8), ("fp32", rtq.RTQ_NODE_FP32)):
        for sname, sch in (("plain", rtq.SCHED_PLAIN), ("persistent", rtq.SCHED_PERSISTENT),
                           ("megakernel", rtq.SCHED_MEGAKERNEL)):
            key = f"{fname}_{sname}"
            r = q8f if key == "q8_persistent" else f32f if key == "fp32_plain" else \
                timed_frames(dict(node_format=fmt, scheduler=sch), 3, 1)
            ablation[key] = dict(ms_per_frame=round(r["wall_ms"], 3), mrays_s=round(r["mrays_s"], 2))
    log(f"ablation: {ablation}")
    g = timed_frames(dict(Q8P, graph=True), max(3, args.steps // 2), 2)
    graph_replay = dict(ms_per_frame=round(g["wall_ms"], 3), mrays_s=round(g["mrays_s"], 2))

    def variant(setup, teardown, name, **extra):
        setup()
        frame(0, **F32)
        ref = img.clone()
        frame(0, **Q8P)
        torch.cuda.synchronize()
        assert torch.equal(ref.view(torch.int32), img.view(torch.int32)), f"{name}: images differ between paths"
        r = timed_frames(Q8P, 3, 1)
        teardown()
        out = dict(extra, ms_per_frame=round(r["wall_ms"], 3), mrays_s=round(r["mrays_s"], 2))
        log(f"{name}: {out}")
        return out

    gen = torch.Generator(device="cuda").manual_seed(1234)
    textured = variant(lambda: S.set_textures(torch.rand((S.n_quads, 4, 4), device="cuda", generator=gen) * 0.9
                                              + 0.05), lambda: S.set_textures(None), "textured", tex_res=4)
    lights = tuple((cx - 50.0, cy - 50.0, 400.0, 0.0, 100.0, 0.0, 100.0, 0.0, 0.0, 16.0)
                   for cx in (-400.0, 400.0) for cy in (-400.0, 400.0))

    def set_lights(v):
        st.area_lights = v
    area = variant(lambda: set_lights(lights), lambda: set_lights(()), "area lights", n_lights=4)
    envmap = variant(lambda: S.set_environment(torch.rand((1024, 2048), device="cuda", generator=gen) * 0.5),
                     lambda: S.set_environment(None), "environment", w=2048, h=1024)
    # principled materials in three channels: 8 random materials over the faces,
    # the last four under a clearcoat
    mat_rng = np.random.default_rng(7)
    mats = np.concatenate([mat_rng.uniform(0.05, 0.95, (8, 3)), mat_rng.uniform(0.1, 1.0, (8, 1)),
                           mat_rng.uniform(0.0, 1.0, (8, 2))], axis=1)
    coats = np.stack([np.r_[np.zeros(4), mat_rng.uniform(0.3, 1.0, 4)], mat_rng.uniform(0.1, 0.6, 8)], axis=1)
    mats = np.concatenate([mats, coats], axis=1).astype(np.float32)
    face_mat = torch.randint(0, 8, (S.n_quads,), device="cuda", generator=gen, dtype=torch.int64).to(torch.uint8)

    def set_mats():
        S.set_materials(mats, face_mat)
        img.resize_(n_pix, 3)

    def unset_mats():
        S.set_materials(None)
        img.resize_(n_pix)
    principled = variant(set_mats, unset_mats, "principled", n_materials=8, coated=4, channels=3)

    # the same materials over RGB per-face textures (4 x 4 texels of 3 channels)
    def set_rgb_tex():
        set_mats()
        S.set_textures(torch.rand((S.n_quads, 4, 4, 3), device="cuda", generator=gen) * 0.9 + 0.05)

    def unset_rgb_tex():
        S.set_textures(None)
        unset_mats()
    rgb_textured = variant(set_rgb_tex, unset_rgb_tex, "principled, RGB textures", n_materials=8, tex_res=4,
                           channels=3)

    # ---- rooflines: the timed kernel and the frame's dominant kernel
    key = kernel_sources_hash()
    inc_bytes = visit_bytes(inc_visits["q8"], nd)
    roof = roofline(inc_bytes, q8_inc["ev_ms"], committed_counters(COUNTERS_FILE, key), DOMINANT)
    stg = q8f["stages"]["closest"]
    launches_per_frame = stg["launches"] / args.steps
    frame_bytes = visit_bytes(fvv[:4], fcc[0]) + visit_bytes(fvv[4:], fcc[1])
    roof_frame = roofline(frame_bytes / launches_per_frame, stg["ms"] / stg["launches"],
                          committed_counters(COUNTERS_FRAME_FILE, key), DOMINANT_FRAME)
    roof_frame["launches_per_frame"] = launches_per_frame

    # ---- config 2 (1M instances, two 1080p views, 1 spp, depth 8), both paths
    cfg2 = None
    if not args.no_config2:
        del S
        torch.cuda.empty_cache()
        scene2, cams2, st2 = sg.config2(scale=args.scale)
        S2 = rtq.Scene(scene2)
        n2 = sum(c.w * c.h for c in cams2)
        img2 = torch.empty(n2, device="cuda")
        d2 = torch.empty(12 * cap, device="cuda")
        c2 = torch.zeros(1, dtype=torch.uint64, device="cuda")
        st2.frame = 0
        rtq.render(S2, cams2, st2, images=img2, dump_rays=d2, dump_count=c2, **F32)
        torch.cuda.synchronize()
        m2 = int(min(int(c2.cpu().item()), cap))
        pl2 = d2.view(12, cap)[:, :m2]
        r2, e2 = pl2[:8].contiguous(), pl2[8:10].view(torch.int32).t().contiguous()
        out2 = {"workload": "config2: 1M instances, 14M unique quads, 2 views 1920x1080, 1 spp, depth 8",
                "incoherent_rays": m2}
        for name, kw in (("q8_persistent", Q8P), ("fp32_plain", F32)):
            for _ in range(2):
                rtq.trace_closest(S2, r2, exclude=e2, soa_in=True, **kw)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for _ in range(5):
                rtq.trace_closest(S2, r2, exclude=e2, soa_in=True, **kw)
            torch.cuda.synchronize()
            inc_ms = (time.perf_counter() - w0) / 5 * 1e3
            for i in range(3):
                st2.frame = 1000 + i
                rtq.render(S2, cams2, st2, images=img2, **kw)
            cnt2 = torch.zeros(4, dtype=torch.uint64, device="cuda")
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for i in range(10):
                st2.frame = i
                rtq.render(S2, cams2, st2, images=img2, counters=cnt2, **kw)
            torch.cuda.synchronize()
            fms = (time.perf_counter() - w0) / 10 * 1e3
            rays2 = float(cnt2[0].item() + cnt2[1].item()) / 10
            out2[name] = dict(incoherent_mrays_s=round(m2 / inc_ms / 1e3, 2), ms_per_frame=round(fms, 3),
                              frame_mrays_s=round(rays2 / fms / 1e3, 2))
        del S2, r2, e2, pl2, d2, img2
        out2["node_width"] = compare_widths(rtq, scene2, cams2, st2, cap, log)
        log(f"config 2: {out2}")
        cfg2 = out2

    # ---- the adjoint at config 4 (the config-1 scene at 512 x 512, 4 spp, depth
    # 4): forward frame and one path-replay backward pass, quantized nodes
    scene4, cams4, st4 = sg.config4()
    S4 = rtq.Scene(scene4)
    n4 = sum(c.w * c.h for c in cams4)
    g4 = torch.full((n4,), 1.0 / n4, device="cuda")
    adj = {}
    for name, fn in (("forward", lambda: rtq.render(S4, cams4, st4, **Q8P)),
                     ("backward", lambda: rtq.render_backward(S4, cams4, st4, g4, **Q8P))):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        adj[name + "_ms"] = round((time.perf_counter() - w0) / 5 * 1e3, 3)
    adj["paths"] = n4 * st4.spp
    adj["workload"] = "config4: config-1 scene (1000 instances, 16384 unique quads), 512x512, 4 spp, depth 4"
    log(f"config 4 adjoint: {adj}")
    del S4
    curves = None if args.no_curves else {"round": curve_field(rtq, sg, args, log),
                                          "flat": curve_field(rtq, sg, args, log, flat=True)}

    # ---- CPU baseline: the FP64 oracle tracing a bounded random sample of the
    # same incoherent rays (same exclusions), sized by a pilot to about
    # cpu_seconds; the rate includes the oracle's flag pass
    cpu = None
    if not args.no_cpu:
        import oracle
        log("cpu baseline: building the oracle scene")
        o = oracle.OracleScene(scene)
        rs = rays.t().contiguous().cpu().numpy()
        ex_pub = planes[10:12].view(torch.int32).t().contiguous().cpu().numpy()
        excl3 = np.stack([ex_pub[:, 0], ex_pub[:, 1] & 0x7FFFFFFF, (ex_pub[:, 1].view(np.uint32) >> 31)
                          .astype(np.int32)], 1)
        rng = np.random.default_rng(0)
        order = rng.permutation(nd)

        def run(n, threads):
            oracle.set_threads(threads)
            idx = np.sort(order[:n])
            w0 = time.perf_counter()
            o.trace(rs[idx], excl=excl3[idx])
            return time.perf_counter() - w0

        all_threads = os.cpu_count() or 1
        run(2000, all_threads)  # pages the oracle's scene in
        dt0 = run(4000, all_threads)
        n_cpu = int(min(nd, max(4000, 4000 * args.cpu_seconds / max(dt0, 1e-3))))
        dt = run(n_cpu, all_threads)
        used = oracle.get_threads()
        n_one = int(max(500, n_cpu / max(used, 1) / 2))
        dt1 = run(n_one, 1)
        oracle.set_threads(all_threads)
        cpu = {"value": round(n_cpu / dt / 1e6, 5), "unit": "Mrays/s", "cores": used, "kind": "oracle",
               "sample": f"{n_cpu} of the {nd} incoherent rays (random, with their exclusions), FP64 closest "
                         f"hit with the oracle's flag pass, {dt:.1f} s on {used} threads",
               "one_core": {"value": round(n_one / dt1 / 1e6, 5), "unit": "Mrays/s",
                            "sample": f"{n_one} rays, {dt1:.1f} s on 1 thread"}}
        log(f"cpu baseline: {cpu}")

    value = q8_inc["mrays_s"]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(q8_inc["wall_ms"], 3),
        "step": f"one closest-hit query of {nd} incoherent rays (bounce >= 1 extension rays of a config-3 frame)",
        "step_ms_percentiles": {k: round(v, 3) for k, v in q8_inc["ev_pct"].items()},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded config-3 generator)",
        "config": {
            "workload": "config3: 20M instances (30% clustered) of 2304 prototypes + 2048^2 terrain, "
                        f"{scene.n_quads} unique quads, 1 view 1920x1080, 4 spp, depth 8",
            "node_format": "q8", "scheduler": "persistent (lane refill)", "parallelism": "single GPU",
        },
        "incoherent": {"rays": nd, "equal_hits": equal_hits, "hit_fraction": round(hit_frac, 4),
                       "q8_persistent_mrays_s": round(value, 2),
                       "fp32_plain_mrays_s": round(f32_inc["mrays_s"], 2),
                       "speedup": round(value / f32_inc["mrays_s"], 3),
                       "visits_per_ray_q8": [round(x / nd, 2) for x in inc_visits["q8"]],
                       "visits_per_ray_fp32": [round(x / nd, 2) for x in inc_visits["fp32"]],
                       "lanes_q8": lane["q8"], "lanes_fp32": lane["fp32"]},
        "frame": {"equal_images": equal_images,
                  "q8_persistent": {"ms_per_frame": round(q8f["wall_ms"], 3), "mrays_s": round(q8f["mrays_s"], 2),
                                    "ms_percentiles": {k: round(v, 3) for k, v in q8f["ev_pct"].items()}},
                  "fp32_plain": {"ms_per_frame": round(f32f["wall_ms"], 3), "mrays_s": round(f32f["mrays_s"], 2)},
                  "speedup": round(f32f["wall_ms"] / q8f["wall_ms"], 3),
                  "rays_per_frame": q8f["rays"], "rays_per_pixel": q8f["rays"] / n_pix,
                  "incoherent_rays_per_frame": q8f["incoherent"],
                  "stages_ms_per_frame": {("traversal" if k == "closest" else k): round(d["ms"] / args.steps, 3)
                                          for k, d in q8f["stages"].items() if k != "shadow"}},
        "ablation": ablation,
        "graph_replay": graph_replay,
        "textured": textured,
        "area_lights": area,
        "environment": envmap,
        "principled": principled,
        "principled_rgb_textures": rgb_textured,
        "config2": cfg2,
        "config4_adjoint": adj,
        "curves": curves,
        "roofline": roof,
        "roofline_frame": roof_frame,
        "cpu_baseline": cpu,
        "scene": {"build_s": round(info["build_seconds"], 2), "device_gib": round(info["device_bytes"] / 2**30, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
