"""Throughput benchmark of the decolorization + global tone-map hot path on one
MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
``dc_tonemap_global`` on 16 binary16 linear-RGB images of 4096 x 4096 (the
statistics pass fused with the decolorization of Eqs. (1)-(6), the fixed-order
combine, and the curve pass that writes FP32 T). Inputs are resident in HBM
before timing starts. The same run also times the plain decolorization of the
64-frame video batch (32 x 1920x1080 + 32 x 3840x2160, 8-bit in, 8-bit + FP32
out) in one batched launch, reported in the same JSON line.

Prints one JSON line (see the keys below). ``--gpus`` above 1 is refused: the
benchmark measures one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
METRIC = "Gpixels/s + % of HBM peak (decolorize+tonemap); p50/p99 latency served"


ROOT = os.path.dirname(os.path.abspath(__file__))


def profiled_counters(kind="traffic_bytes"):
    """Per-launch counter figures measured with rocprofv3, from the summaries
    under profiles/ that were taken on the current kernel source (an empty dict
    when none matches, i.e. the kernels changed since): kind "traffic_bytes"
    (calibrated HBM bytes per launch) or "valu_slots_per_px" (VALU issue slots
    per pixel from the SQ counters)."""
    import glob
    import hashlib
    import re
    found = {}
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(fn).read()
        m = re.search(r"source sha256 \((\S+)\): ([0-9a-f]+)", text)
        src = os.path.join(ROOT, m.group(1)) if m else None
        if not src or not os.path.exists(src):
            continue
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(2):
            continue
        for key, val in re.findall(r"^%s (\S+) ([0-9.]+)$" % kind, text, re.M):
            found[key] = float(val) if "." in val else int(val)
    return found


def profiled_traffic():
    return profiled_counters("traffic_bytes")


# VALU issue: a wave64 instruction holds one of the 1024 SIMDs (256 CUs x 4)
# for 4 cycles at 2.4 GHz, so slots / px x px take slots x px / (16 x 1024 x
# 2.4e9) seconds of the whole chip.
def valu_issue_ms(slots_per_px, px):
    return slots_per_px * px / (16.0 * 1024 * 2.4e9) * 1e3


def add_traffic_rates(obj):
    """In every roofline object with a measured `traffic`, adds the counter
    rate beside the algorithmic one: traffic_gbs = traffic bytes / kernel time
    (kernel time = algorithmic_bytes / achieved) and its fraction of peak."""
    if isinstance(obj, dict):
        if obj.get("traffic") and obj.get("achieved") and obj.get("algorithmic_bytes"):
            secs = obj["algorithmic_bytes"] / (obj["achieved"] * 1e9)
            obj["traffic_gbs"] = round(obj["traffic"] / secs / 1e9, 1)
            obj["traffic_frac"] = round(obj["traffic_gbs"] / obj["peak"], 4)
        for v in obj.values():
            add_traffic_rates(v)
    return obj


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--images", type=int, default=16, help="HDR images per step")
    ap.add_argument("--size", type=int, default=4096, help="HDR image side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-images", type=int, default=16)
    ap.add_argument("--skip-video", action="store_true")
    ap.add_argument("--skip-uneven", action="store_true")
    ap.add_argument("--no-per-image", action="store_true",
                    help="skip the per-image-launch and gray-channel comparisons (profiler runs)")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--requests", type=int, default=10000, help="serving trace length")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="serving memory budget")
    ap.add_argument("--serve-log", default=None,
                    help="append one JSON line per served request (times, size, format, bytes)")
    ap.add_argument("--no-h2d", action="store_true",
                    help="skip the serving variant with pinned host inputs")
    ap.add_argument("--skip-colour", action="store_true")
    ap.add_argument("--skip-local", action="store_true")
    ap.add_argument("--only", choices=["tonemap", "colour", "local", "video", "uneven", "serve",
                                       "sweep", "channels", "ceilings"],
                    default=None,
                    help="time one workload only (for profiler runs)")
    ap.add_argument("--tuning", default=None,
                    help="JSON launch shapes to use instead of autotuning (written by --save-tuning)")
    ap.add_argument("--save-tuning", default=None, help="write the autotuned shapes here")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shapes")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


WORKERS = min(16, os.cpu_count() or 1)
# Host cores the CPU legs may use: the affinity mask, at most 16 (one GPU's
# share of a shared host).
HOST_CORES = max(1, min(16, len(os.sched_getaffinity(0))))


def gen_hdr(n, size):
    import synth
    return synth.hdr_images(count=n, shape=(size, size), workers=WORKERS)


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per step


def kernel_times(fn, reps, P, dev):
    """Per-kernel durations (ms) from the library's own HIP events."""
    import torch
    P.set_profiling(True, dev)
    acc = None
    for _ in range(reps):
        fn()
        t = P.last_timings(dev)
        acc = t if acc is None else [a + b for a, b in zip(acc, t)]
    P.set_profiling(False, dev)
    torch.cuda.synchronize()
    return [a / reps for a in acc]


def channels_leg(P, dev, stream, frames, o32, reps):
    """Same-GPU comparison with the gray channels the paper compares its L
    against: the video frames, u8 in, f32 out, Gpx/s from the kernel time of
    the library's events."""
    import torch
    vpx = sum(f.shape[0] * f.shape[1] for f in frames)
    comp = {}
    with torch.cuda.stream(stream):
        cplan = P.Plan(P.PLAN_DECOLORIZE, frames, o32)
        cplan.run(stream)  # warm-up
        comp["decolor_L"] = vpx / (kernel_times(lambda: cplan.run(stream), reps, P, dev)[0]
                                   * 1e-3) / 1e9
        cplan.close()
        for ch in ("y601", "hsv_v", "cielab_l"):
            P.channel_batch(frames, ch, outs=o32, stream=stream)  # warm-up
            t = kernel_times(lambda: P.channel_batch(frames, ch, outs=o32, stream=stream), reps,
                             P, dev)[0]
            comp[ch] = vpx / (t * 1e-3) / 1e9
    comp = {k: round(v, 1) for k, v in comp.items()}
    log("same-GPU gray channels, u8 -> f32, Gpx/s: %s" % comp)
    return comp


def sweep_leg(P, dev, stream, frame, reps, traffic):
    """Weight sweep (Fig. 4's explorer): one 3840x2160 u8 frame under 20
    (beta_R, beta_k) pairs, 20 FP32 outputs from one launch that reads the
    frame once."""
    import torch
    betas = [(br, bk) for br in (0.0, 0.3, 0.55, 0.8, 1.0) for bk in (0.2, 0.5, 0.8, 1.0)]
    sw = torch.empty((len(betas),) + tuple(frame.shape[:2]), dtype=torch.float32, device=dev)
    with torch.cuda.stream(stream):
        P.beta_sweep(frame, betas, out=sw, stream=stream)  # warm-up
        swt = kernel_times(lambda: P.beta_sweep(frame, betas, out=sw, stream=stream), reps,
                           P, dev)[0]
    spx = len(betas) * frame.shape[0] * frame.shape[1]
    # algorithmic bytes: the frame read once, 20 FP32 planes written
    sbytes = frame.shape[0] * frame.shape[1] * 3 + spx * 4
    ach = sbytes / (swt * 1e-3) / 1e9
    sweep = {"workload": "beta_sweep_3840x2160_u8_x20", "pairs": len(betas),
             "kernel_ms": round(swt, 4),
             "output_gpx_s": round(spx / (swt * 1e-3) / 1e9, 1),
             "roofline": {"bound": "hbm", "kernel": "sweep", "achieved": round(ach, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                          "traffic": traffic.get("sweep"), "algorithmic_bytes": sbytes}}
    log("beta sweep: %d pairs on one 4K frame in %.3f ms (%.0f Gpx/s of outputs, %.0f GB/s)" %
        (len(betas), swt, sweep["output_gpx_s"], ach))
    del sw
    return sweep


# Streams whose ceilings are measured: (name, 16-B reads : writes per trip,
# read bytes, written bytes). Read:write ratios of the passes: statistics pass
# read-only, curve pass 6:4 (binary16 in, FP32 T out), video 3:5 (8-bit in,
# 8-bit + FP32 out), a copy 1:1, and a pure write.
# (name, reads, writes per thread and tile, read bytes, write bytes, access
# size): 16-byte vectors, and the hot path's 12-byte unit loads with 8-byte
# stores (the curve pass's binary16 unit in, two FP32 values out).
CEILING_STREAMS = [("read", 8, 0, 1610612736, 0, 16),
                   ("write", 0, 8, 0, 1073741824, 16),
                   ("read6_write4", 6, 4, 1610612736, 1073741824, 16),
                   ("read3_write5", 3, 5, 995328000, 1658880000, 16),
                   ("copy", 4, 4, 1073741824, 1073741824, 16),
                   ("read_12B_units", 8, 0, 1610612736, 0, 12),
                   ("read6_write4_12B_units", 6, 6, 1610612736, 1073741824, 12)]


def ceilings_leg(dev, reps=7, grids=(0, 4, 8, 16, 32)):
    """What HBM sustains for plain streams (libdc_ceilings.so: no arithmetic,
    nontemporal 16-byte loads and stores): per stream, the best grid's median
    pass time over `reps` passes, as bytes moved / time. Grids are workgroups
    per CU, 0 = one workgroup per tile."""
    import ctypes
    import torch
    from paper_2108_13656_amd import build as B
    if not os.path.exists(B.CEIL_LIB):
        return None
    L = ctypes.CDLL(B.CEIL_LIB)
    L.dcx_stream.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                             ctypes.c_void_p]
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    big = max(c[3] for c in CEILING_STREAMS)
    bigw = max(c[4] for c in CEILING_STREAMS)
    src = torch.ones(big, dtype=torch.uint8, device=dev)
    dst = torch.empty(bigw, dtype=torch.uint8, device=dev)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {}
    L.dcx_stream12.argtypes = L.dcx_stream.argtypes
    for name, vr, vw, rb, wb, unit in CEILING_STREAMS:
        fn = L.dcx_stream if unit == 16 else L.dcx_stream12
        best = None
        for gpc in grids:
            ts = []
            for _ in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc = fn(src.data_ptr(), rb, dst.data_ptr(), wb, vr, vw, gpc * ncu,
                        sink.data_ptr(), stream.cuda_stream)
                e1.record(stream)
                if rc != 0:
                    raise RuntimeError("dcx_stream failed: %d" % rc)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts[1:]))
            if best is None or ms < best[0]:
                best = (ms, gpc)
        gbs = (rb + wb) / (best[0] * 1e-3) / 1e9
        out[name] = {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "ms": round(best[0], 4), "grid_per_cu": best[1], "read_bytes": rb,
                     "write_bytes": wb}
        log("ceiling %-22s %7.1f GB/s (%.1f %% of peak) at %d workgroups/CU" %
            (name, gbs, 100 * gbs / HBM_PEAK_GBS, best[1]))
    del src, dst
    torch.cuda.empty_cache()
    # The tone map's two-pass traffic with no arithmetic, 16 x 4096^2 binary16
    # -> FP32 (24 KiB in / 16 KiB out per 4096-px tile): batch order (read all,
    # then re-read all and write) and the lagged order (image s read beside
    # image s - 1's re-read and write, one launch per stage).
    L.dcx_stage.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    nimg, tpi = 16, 4096
    inb, outb = nimg * tpi * 24576, nimg * tpi * 16384
    src = torch.ones(inb, dtype=torch.uint8, device=dev)
    dst = torch.empty(outb, dtype=torch.uint8, device=dev)
    px = nimg * tpi * 4096

    def batch(gpc):
        rc = L.dcx_stream(src.data_ptr(), inb, 0, 0, 8, 0, gpc * ncu, sink.data_ptr(),
                          stream.cuda_stream)
        rc = rc or L.dcx_stream(src.data_ptr(), inb, dst.data_ptr(), outb, 6, 4, gpc * ncu,
                                sink.data_ptr(), stream.cuda_stream)
        return rc

    def lagged(gpc):
        rc = 0
        for s in range(nimg + 1):
            rc = rc or L.dcx_stage(src.data_ptr(), dst.data_ptr(), s, nimg, tpi, gpc * ncu,
                                   sink.data_ptr(), stream.cuda_stream)
        return rc

    # The same two passes parking a 4-byte intermediate (x2 of the statistics
    # pass in the FP32 output) instead of re-reading the input: 6 B read and
    # 4 B written, then 4 B read and 4 B written per pixel (18 B/px).
    L.dcx_stage_parked.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]
    mid = torch.empty(outb, dtype=torch.uint8, device=dev)

    def parked_batch(gpc):
        rc = L.dcx_stream(src.data_ptr(), inb, mid.data_ptr(), outb, 6, 4, gpc * ncu,
                          sink.data_ptr(), stream.cuda_stream)
        rc = rc or L.dcx_stream(mid.data_ptr(), outb, dst.data_ptr(), outb, 4, 4, gpc * ncu,
                                sink.data_ptr(), stream.cuda_stream)
        return rc

    def parked_lagged(gpc):
        rc = 0
        for s in range(nimg + 1):
            rc = rc or L.dcx_stage_parked(src.data_ptr(), mid.data_ptr(), dst.data_ptr(), s, nimg,
                                          tpi, gpc * ncu, sink.data_ptr(), stream.cuda_stream)
        return rc

    for name, fn in (("tonemap_two_pass_batch", batch), ("tonemap_two_pass_lagged", lagged),
                     ("tonemap_parked_batch", parked_batch),
                     ("tonemap_parked_lagged", parked_lagged)):
        best = None
        for gpc in grids:
            ts = []
            for _ in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc = fn(gpc)
                e1.record(stream)
                if rc != 0:
                    raise RuntimeError("%s failed: %d" % (name, rc))
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts[1:]))
            if best is None or ms < best[0]:
                best = (ms, gpc)
        bpp = 18 if "parked" in name else 16
        out[name] = {"ms": round(best[0], 4), "grid_per_cu": best[1], "bytes_per_px": bpp,
                     "gbs": round(px * bpp / (best[0] * 1e-3) / 1e9, 1),
                     "frac_of_peak_at_10_bytes_per_px":
                         round(px * 10 / (best[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("%s: %.3f ms (%.1f GB/s of %d B/px traffic; %.1f %% of peak at 10 B/px)" %
            (name, best[0], px * bpp / (best[0] * 1e-3) / 1e9, bpp,
             100 * px * 10 / (best[0] * 1e-3) / 1e9 / HBM_PEAK_GBS))
    del src, dst, mid
    torch.cuda.empty_cache()
    return out


POOL_W = 8192          # serving: source pools read as images this many pixels wide
UNALIGNED_EVERY = 10   # serving: one request in this many starts at any pixel


def serve_leg(args, P, dev):
    """Poisson trace through the native continuous-batching server: saturated
    throughput first, then arrivals at 0.7 of it; FIFO one-image-per-launch
    baseline on the same trace."""
    import torch
    import synth
    log("serving: building device-resident source pools")
    rng = np.random.default_rng(synth.SERVING_SEED)
    pool_bytes = 2 << 30
    pools = {}
    for fmt, base, dt in (("u8", synth.sdr_pixels(rng, 4096, 4096), P.DC_U8),
                          ("f16", synth.hdr_pixels(rng, 4096, 4096), P.DC_F16)):
        flat = torch.from_numpy(base).to(dev).view(-1)
        reps = -(-pool_bytes // (flat.numel() * flat.element_size()))
        pool = flat.repeat(reps)
        pools[fmt] = (pool, dt, 3 * pool.element_size(), pool.numel() // 3)
    trace = synth.serving_trace(n_requests=args.requests, rate_per_s=1.0)
    # Each pool is read as a POOL_W-pixel-wide image (row pitch POOL_W * bpp
    # bytes) and every request is a crop of it: its rows lie POOL_W pixels
    # apart, wider than the crop, so the kernels walk pitched rows. Crops start
    # at a multiple of 16 pixels except one in UNALIGNED_EVERY, which starts
    # anywhere (a row start that is not 16-byte aligned takes the per-pixel walk).
    reqs, px, unaligned = [], [], 0
    for r in trace:
        pool, dt, bpp, npx = pools[r["fmt"]]
        rows = npx // POOL_W
        y0 = int(rng.integers(0, rows - r["h"] + 1))
        if r["id"] % UNALIGNED_EVERY == UNALIGNED_EVERY - 1:
            x0 = int(rng.integers(0, POOL_W - r["w"] + 1))
        else:
            x0 = int(rng.integers(0, (POOL_W - r["w"]) // 16 + 1)) * 16
        unaligned += (x0 * bpp) % 16 != 0
        off = y0 * POOL_W + x0
        reqs.append(P.make_request(r["id"], pool.data_ptr() + off * bpp, dt, r["w"], r["h"],
                                   POOL_W * bpp, P.DC_U8 if r["fmt"] == "u8" else P.DC_F32))
        px.append(r["w"] * r["h"])
    px = np.array(px, np.float64)
    unit_arrivals = np.array([r["arrival"] for r in trace])
    budget = int(args.budget_gib * (1 << 30))
    torch.cuda.synchronize()

    def run(max_batch, max_inflight, arrivals, name):
        srv = P.Server(budget, max_batch=max_batch, max_inflight=max_inflight, device=dev)
        srv.replay(reqs[:64], [0.0] * 64)  # warm-up (workspace growth)
        h0, n0 = srv.host_stats()
        done = srv.replay(reqs, list(arrivals))
        h1, n1 = srv.host_stats()
        srv.close()
        if args.serve_log:
            # one JSON object per request: times on the server clock, size, format, bytes
            meta = {r["id"]: r for r in trace}
            with open(args.serve_log, "a") as f:
                for c in done:
                    r = meta[c.id]
                    f.write(json.dumps({
                        "run": name, "id": c.id, "status": c.status, "batch": c.batch_size,
                        "t_submit": c.t_submit, "t_admit": c.t_admit, "t_launch": c.t_launch,
                        "t_done": c.t_done, "w": r["w"], "h": r["h"], "fmt": r["fmt"],
                        "in_bytes": r["w"] * r["h"] * (3 if r["fmt"] == "u8" else 6),
                        "out_bytes": r["w"] * r["h"] * (1 if r["fmt"] == "u8" else 4)}) + "\n")
        ok = [c for c in done if c.status == P.DC_OK]
        lat = np.array([c.t_done - c.t_submit for c in ok])
        t_first = min(c.t_submit for c in done)
        t_last = max(c.t_done for c in done)
        sizes = np.array([c.batch_size for c in ok])
        log("serving: %d requests in %.3f s (max_batch %d, lanes %d)" %
            (len(done), t_last - t_first, max_batch, max_inflight))
        return {"gpx_s": round(float(px.sum()) / (t_last - t_first) / 1e9, 2),
                "p50_ms": round(1e3 * float(np.median(lat)), 3),
                "p99_ms": round(1e3 * float(np.quantile(lat, 0.99)), 3),
                "mean_batch": round(float(sizes.mean()), 2), "rejected": len(done) - len(ok),
                "wall_s": round(t_last - t_first, 4),
                "host_us_per_launch": round(1e6 * (h1 - h0) / max(1, n1 - n0), 2)}

    sat = run(64, 4, np.zeros(len(reqs)), "saturated")
    rate = 0.7 * sat["gpx_s"] * 1e9 / px.mean()
    arrivals = unit_arrivals / rate
    served = run(64, 4, arrivals, "served")
    fifo = run(1, 1, arrivals, "fifo_per_image")
    # The same trace with inputs in pinned host memory: the server copies each
    # request's crop into its budget (DC_IMG_HOST_SRC) on the lane's stream,
    # so PCIe transfers of one lane overlap kernels of the others.
    h2d = None
    if not args.no_h2d:
        log("serving: building pinned host source pools")
        dev_reqs = reqs
        hpools = {fmt: torch.empty(pool.numel(), dtype=pool.dtype).pin_memory()
                  for fmt, (pool, _, _, _) in pools.items()}
        for fmt, (pool, _, _, _) in pools.items():
            hpools[fmt].copy_(pool)
        reqs = []
        for r, q in zip(trace, dev_reqs):
            pool, dt, bpp, _ = pools[r["fmt"]]
            off = q.img.src - pool.data_ptr()
            reqs.append(P.make_request(r["id"], hpools[r["fmt"]].data_ptr() + off, dt, r["w"],
                                       r["h"], POOL_W * bpp, q.img.dst_dtype,
                                       flags=P.DC_IMG_HOST_SRC))
        hsat = run(64, 4, np.zeros(len(reqs)), "host_saturated")
        hrate = 0.7 * hsat["gpx_s"] * 1e9 / px.mean()
        hserved = run(64, 4, unit_arrivals / hrate, "host_served")
        in_bytes = sum(r["w"] * r["h"] * (3 if r["fmt"] == "u8" else 6) for r in trace)
        h2d = {"saturated_gpx_s": hsat["gpx_s"],
               "saturated_h2d_gbs": round(in_bytes / hsat["wall_s"] / 1e9, 1),
               "rate_req_s": round(hrate, 1), "gpx_s": hserved["gpx_s"],
               "p50_ms": hserved["p50_ms"], "p99_ms": hserved["p99_ms"],
               "mean_batch": hserved["mean_batch"], "rejected": hserved["rejected"]}
        log("serving, host inputs: saturated %.1f Gpx/s (%.1f GB/s of inputs over PCIe); at %.0f "
            "req/s: %.1f Gpx/s p50 %.3f ms p99 %.3f ms" %
            (hsat["gpx_s"], h2d["saturated_h2d_gbs"], hrate, hserved["gpx_s"], hserved["p50_ms"],
             hserved["p99_ms"]))
        reqs = dev_reqs
        del hpools
    out = {"workload": "serving_tonemap", "requests": len(reqs),
           "mix": "70% u8 SDR -> u8 T, 30% f16 HDR -> f32 T",
           "sizes": "w log-uniform 256..7680, h log-uniform 256..4320",
           "sources": "crops of %d-px-wide device pools (row pitch > row bytes); %d of %d "
                      "start at a row offset that is not 16-byte aligned" %
                      (POOL_W, unaligned, len(reqs)),
           "mean_mpx": round(px.mean() / 1e6, 3), "budget_gib": args.budget_gib,
           "saturated_gpx_s": sat["gpx_s"], "rate_req_s": round(rate, 1),
           "gpx_s": served["gpx_s"], "p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"],
           "mean_batch": served["mean_batch"], "rejected": served["rejected"],
           "host_us_per_launch": served["host_us_per_launch"],
           "fifo_per_image": fifo, "host_inputs": h2d}
    log("serving: saturated %.1f Gpx/s; at %.0f req/s: %.1f Gpx/s p50 %.3f ms p99 %.3f ms "
        "(mean batch %.1f, %.1f us of host time per launch); FIFO per-image: %.1f Gpx/s "
        "p50 %.3f ms p99 %.3f ms" %
        (sat["gpx_s"], rate, served["gpx_s"], served["p50_ms"], served["p99_ms"],
         served["mean_batch"], served["host_us_per_launch"], fifo["gpx_s"], fifo["p50_ms"],
         fifo["p99_ms"]))
    del pools
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2108_13656_amd as P
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    result = {}
    traffic = profiled_traffic()
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n, "copies": 3}), flush=True)
        return
    ceilings = None
    if args.only in (None, "ceilings"):
        ceilings = ceilings_leg(dev)
        if args.only == "ceilings":
            print(json.dumps({"ceilings": ceilings, "peak_gbs": HBM_PEAK_GBS}), flush=True)
            return
    fixed = None
    if args.tuning:
        with open(args.tuning) as f:
            fixed = json.load(f)
    saved = {}

    def tune(kind, *bufs):
        if fixed is not None:
            P.set_tuning(fixed, dev)
            return P.get_tuning(dev)
        if args.no_autotune:
            return P.get_tuning(dev)
        t = P.autotune(kind, *bufs, stream=stream)
        saved.update(t)
        return t

    # ---------------------------------------------------- HDR tone map (headline)
    n_img, size = args.images, args.size
    hdr_px = n_img * size * size
    run_gray = args.only in (None, "tonemap")
    run_colour = args.only in (None, "colour") and not args.skip_colour
    run_local = args.only in (None, "local") and not args.skip_local
    if run_gray or run_colour or run_local:
        log("generating %d HDR images %dx%d" % (n_img, size, size))
        t0 = time.time()
        imgs = gen_hdr(n_img, size)
        log("generated in %.1f s" % (time.time() - t0))
        xs = [torch.from_numpy(a).to(dev) for a in imgs]
        torch.cuda.synchronize()
    tuning = None
    if run_gray:
        outs = [torch.empty((size, size), dtype=torch.float32, device=dev) for _ in xs]
        stats = torch.empty((n_img, P.STATS_BYTES), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()

        with torch.cuda.stream(stream):
            tuning = tune(P.PLAN_TONEMAP, xs, outs)
            log("autotuned tone-map shape: %s" % tuning)
            plan = P.Plan(P.PLAN_TONEMAP, xs, outs, stats=stats, graph=True)

            def step():
                plan.run(stream)

            # The untimed measurements of this leg come first: per-kernel
            # durations from the batch schedule (three kernels on one stream,
            # events between them; the same kernels the step runs) and the
            # per-call API path. The MI355X's power management slows the first
            # few dozen steps after the GPU has idled, so they also keep the
            # GPU busy until the W warm-up steps and the K timed steps; the
            # breakdown is taken again after the timed block.
            P.set_tuning(dict(tuning, tonemap_pipeline=0), dev)
            plan_ev = P.Plan(P.PLAN_TONEMAP, xs, outs, stats=stats, graph=False)
            kernel_times(lambda: plan_ev.run(stream), max(5, args.steps // 2), P, dev)
            P.set_tuning(tuning, dev)
            dyn_ms = time_steps(lambda: P.tonemap_global(xs, outs=outs, stats=stats, stream=stream),
                                max(3, args.steps // 2), 1, stream)
            ms = time_steps(step, args.steps, args.warmup, stream)
            # The same step kept running (five more blocks of K steps, not part
            # of the timed result): the steady state beside the timed block,
            # and the per-kernel breakdown taken again there (the one reported).
            steady = [time_steps(step, args.steps, 0, stream) for _ in range(5)]
            ktimes = kernel_times(lambda: plan_ev.run(stream), max(5, args.steps // 2), P, dev)
        log("tonemap step %.3f ms (steady %.3f); kernels (pass1, combine, pass2) %s ms" %
            (ms, float(np.median(steady)), ", ".join("%.3f" % t for t in ktimes)))
        gpx = hdr_px / (ms * 1e-3) / 1e9
        step_bytes = hdr_px * (6 + 4)  # read RGB f16 once, write T f32 once
        # Dominant kernel: the curve pass (re-reads the input, writes T).
        k_pass1, k_comb, k_pass2 = ktimes
        dom = ("tonemap_pass2", k_pass2, hdr_px * 10) if k_pass2 >= k_pass1 else \
              ("tonemap_pass1", k_pass1, hdr_px * 6)
        ach = dom[2] / (dom[1] * 1e-3) / 1e9
        result.update({
            "metric": METRIC, "value": round(gpx, 3), "unit": "Gpixels/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "hdr_tonemap", "images": n_img, "height": size,
                       "width": size, "src": "f16 linear RGB", "dst": "f32 T",
                       "hot_path": "decolorize + stats + combine + curve"},
            "hbm_frac_step": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_ms": {"tonemap_pass1": round(k_pass1, 4), "tonemap_combine": round(k_comb, 4),
                          "tonemap_pass2": round(k_pass2, 4)},
            "launch": {"plan": "hip graph replay, %s schedule" %
                               ("two-stream pipeline, groups of %d images" %
                                tuning["tonemap_pipeline"] if tuning.get("tonemap_pipeline") else
                                "batch"),
                       "tuning": {k: v for k, v in tuning.items() if "pass" in k or "tonemap" in k},
                       "per_call_api_ms_per_step": round(dyn_ms, 4),
                       "steady_ms_per_step": round(float(np.median(steady)), 4)},
            "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": traffic.get(dom[0]), "algorithmic_bytes": dom[2]},
        })
        roof = result["roofline"]
        if ceilings:
            pat = "read6_write4" if dom[0] == "tonemap_pass2" else "read"
            c = ceilings[pat]["gbs"]
            roof["stream_ceiling"] = {"pattern": pat, "gbs": c, "frac_of_peak": round(c / HBM_PEAK_GBS, 4),
                                      "achieved_frac_of_ceiling": round(ach / c, 4)}
        # The whole step against its limits: algorithmic bytes (input read
        # once, T written once), the counted HBM bytes of both passes, the
        # same traffic with no arithmetic (the ceilings leg's two-pass batch
        # order), and the VALU issue time of both passes from the SQ counters.
        slots = profiled_counters("valu_slots_per_px")
        step = {"ms": round(ms, 4), "algorithmic_bytes": step_bytes,
                "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if "tonemap_pass1" in traffic and "tonemap_pass2" in traffic:
            tb = traffic["tonemap_pass1"] + traffic["tonemap_pass2"]
            step.update({"traffic_bytes": tb, "traffic_ratio": round(tb / step_bytes, 4),
                         "traffic_gbs": round(tb / (ms * 1e-3) / 1e9, 1),
                         "traffic_frac": round(tb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        if ceilings:
            fl = ceilings["tonemap_two_pass_batch"]["ms"]
            step.update({"traffic_floor_ms": fl, "frac_of_traffic_floor": round(fl / ms, 4),
                         "lagged_order_floor_ms": ceilings["tonemap_two_pass_lagged"]["ms"],
                         "parked_intermediate_floor_ms": {
                             "batch": ceilings["tonemap_parked_batch"]["ms"],
                             "lagged": ceilings["tonemap_parked_lagged"]["ms"]}})
        if "tonemap_pass1" in slots and "tonemap_pass2" in slots:
            v1 = valu_issue_ms(slots["tonemap_pass1"], hdr_px)
            v2 = valu_issue_ms(slots["tonemap_pass2"], hdr_px)
            step.update({"valu_slots_per_px": {"pass1": slots["tonemap_pass1"],
                                               "pass2": slots["tonemap_pass2"]},
                         "valu_issue_ms": {"pass1": round(v1, 4), "pass2": round(v2, 4)},
                         "valu_issue_frac_of_kernel": {"pass1": round(v1 / k_pass1, 4),
                                                       "pass2": round(v2 / k_pass2, 4)},
                         "valu_floor_ms": round(v1 + v2, 4),
                         "frac_of_valu_floor": round((v1 + v2) / ms, 4)})
            step["limiter"] = (
                "pass 1 issue-bound (VALU issue %.0f %% of its time, reading 6 B/px at %.0f GB/s); "
                "pass 2 at the 6:4 stream ceiling (%.0f GB/s)" %
                (100 * v1 / k_pass1, hdr_px * 6 / (k_pass1 * 1e-3) / 1e9,
                 hdr_px * 10 / (k_pass2 * 1e-3) / 1e9))
        roof["step"] = step

        # CPU baseline: the FP64 oracle, single thread, on a sample of images.
        if not args.no_cpu_baseline:
            import oracle
            k = min(args.cpu_sample_images, n_img)
            log("cpu baseline: oracle on %d image(s), 1 thread" % k)
            dt = 0.0
            worst = 0.0
            for i in range(k):
                t0 = time.time()
                t_ref, _, _ = oracle.tonemap(imgs[i], nthreads=1)
                dt += time.time() - t0
                worst = max(worst, float(np.max(np.abs(outs[i].cpu().numpy() - t_ref))))
            cpu_gpx = k * size * size / dt / 1e9
            result["cpu_baseline"] = {"value": round(cpu_gpx, 6), "unit": "Gpixels/s", "cores": 1,
                                      "kind": "oracle",
                                      "sample": "%d of the %d images (%dx%d f16), full tone map in "
                                                "FP64, one thread" % (k, n_img, size, size)}
            # the same image's T against the oracle on the radiance it stores
            # before binary16 rounding (the storage error, bounded in the tests)
            import synth
            exact = synth.hdr_image(0, shape=(size, size), exact=True).astype(np.float32)
            t_exact, _, _ = oracle.tonemap(exact, nthreads=HOST_CORES)
            err_exact = float(np.max(np.abs(outs[0].cpu().numpy() - t_exact)))
            del exact, t_exact
            result["parity_sample"] = {"images": k, "max_abs_err_T": worst,
                                       "max_abs_err_T_vs_unrounded_radiance": err_exact}
            log("cpu baseline %.4f Gpx/s; GPU vs oracle max |dT| %.2e" % (cpu_gpx, worst))
            # Eqs. (1)-(6) alone, as in the paper's run-time table: one thread,
            # and the oracle's row split over every host core this process may
            # use, at most 16: the CPU share that goes with one GPU on a shared
            # host (nproc and the affinity mask are reported beside it).
            ncores = HOST_CORES
            t0 = time.time()
            oracle.decolorize(imgs[0], nthreads=1)
            one = size * size / (time.time() - t0) / 1e9
            t0 = time.time()
            for i in range(k):
                oracle.decolorize(imgs[i], nthreads=ncores)
            allc = k * size * size / (time.time() - t0) / 1e9
            model = None
            try:
                with open("/proc/cpuinfo") as f:
                    model = next((ln.split(":", 1)[1].strip() for ln in f
                                  if ln.startswith("model name")), None)
            except OSError:
                pass
            result["cpu_baseline"]["decolorize_only"] = {
                "one_thread_gpx": round(one, 6), "all_cores_gpx": round(allc, 6),
                "cores": ncores, "sample": "Eqs. (1)-(6) in FP64 on 1 and %d of the images" % k}
            result["cpu_baseline"]["host"] = {"cpu_model": model, "nproc": os.cpu_count(),
                                              "affinity_cores": len(os.sched_getaffinity(0)),
                                              "cores_used_all_cores_leg": ncores,
                                              "cap": "16 threads, one GPU's share of the host"}
            log("cpu oracle, decolorization only: %.4f Gpx/s on 1 thread, %.4f on %d (%s)" %
                (one, allc, ncores, model))
        plan.close()
        plan_ev.close()
        del outs
        torch.cuda.empty_cache()

    # ------------------------------------- HDR tone map with re-coloured RGB output
    if run_colour:
        # Same images and launch shapes as the gray tone map; the curve pass
        # writes min(1, T (C / L)^s) per channel as 8-bit RGB.
        couts = [torch.empty((size, size, 3), dtype=torch.uint8, device=dev) for _ in xs]
        with torch.cuda.stream(stream):
            if tuning is None:
                tuning = tune(P.PLAN_TONEMAP, xs, couts)
        legs = {}
        for sat in (1.0, 0.6):
            with torch.cuda.stream(stream):
                cplan = P.Plan(P.PLAN_TONEMAP, xs, couts, graph=True, saturation=sat)
                P.set_tuning(dict(tuning, tonemap_pipeline=0), dev)
                cev = P.Plan(P.PLAN_TONEMAP, xs, couts, graph=False, saturation=sat)
                kernel_times(lambda: cev.run(stream), max(5, args.steps // 2), P, dev)
                P.set_tuning(tuning, dev)
                cms = time_steps(lambda: cplan.run(stream), args.steps, args.warmup, stream)
                ck = kernel_times(lambda: cev.run(stream), max(5, args.steps // 2), P, dev)
                cplan.close()
                cev.close()
            key = "tonemap_colour_s1" if sat == 1.0 else "tonemap_colour_pow"
            cach = hdr_px * 9 / (ck[2] * 1e-3) / 1e9
            legs["s=%g" % sat] = {
                "ms_per_step": round(cms, 4), "value": round(hdr_px / (cms * 1e-3) / 1e9, 3),
                "unit": "Gpixels/s",
                "kernel_ms": {"tonemap_pass1": round(ck[0], 4), "tonemap_combine": round(ck[1], 4),
                              "tonemap_colour": round(ck[2], 4)},
                "roofline": {"bound": "hbm", "kernel": key, "achieved": round(cach, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(cach / HBM_PEAK_GBS, 4), "traffic": traffic.get(key),
                             "algorithmic_bytes": hdr_px * 9}}
            # The curve pass with colour output issues VALU work for most of its
            # time (SQ counters in profiles/): its HBM rate is set by that.
            cslots = profiled_counters("valu_slots_per_px").get(key)
            if cslots:
                vi = valu_issue_ms(cslots, hdr_px)
                legs["s=%g" % sat]["roofline"].update({
                    "valu_slots_per_px": cslots, "valu_issue_ms": round(vi, 4),
                    "valu_issue_frac_of_kernel": round(vi / ck[2], 4),
                    "limiter": "VALU issue (%.0f %% of the curve pass's time)" % (100 * vi / ck[2])})
            log("colour tone map s=%g: step %.3f ms (%.1f Gpx/s); kernels %s ms; curve pass %.0f GB/s"
                % (sat, cms, legs["s=%g" % sat]["value"], ", ".join("%.3f" % t for t in ck), cach))
        colour = {"workload": "hdr_tonemap_colour", "images": n_img, "height": size, "width": size,
                  "src": "f16 linear RGB", "dst": "u8 RGB, min(1, T (C / L)^s) per channel",
                  "legs": legs}
        if result:
            result["colour_tonemap"] = colour
        else:
            first = legs["s=1"]
            result.update({"metric": METRIC, "value": first["value"], "unit": "Gpixels/s",
                           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                           "ms_per_step": first["ms_per_step"], "higher_is_better": True,
                           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                           "data": "synthetic", "config": {"workload": "hdr_tonemap_colour"},
                           "roofline": first["roofline"], "colour_tonemap": colour})
        del couts

    # ------------------------------------------ local tone map (Sec. III-B.2)
    if run_local:
        # Same images; 64 x 64-pixel tiles, strength 0.5, FP32 T (staged form:
        # the statistics pass parks log2 luminance in the output for the curve
        # pass). Kernel intervals: statistics + histograms, combine + tables,
        # curve pass.
        louts = [torch.empty((size, size), dtype=torch.float32, device=dev) for _ in xs]
        with torch.cuda.stream(stream):
            lplan = P.Plan(P.PLAN_LOCAL, xs, louts, graph=True)
            lev = P.Plan(P.PLAN_LOCAL, xs, louts, graph=False)
            kernel_times(lambda: lev.run(stream), max(5, args.steps // 2), P, dev)
            lms = time_steps(lambda: lplan.run(stream), args.steps, args.warmup, stream)
            lk = kernel_times(lambda: lev.run(stream), max(5, args.steps // 2), P, dev)
            lplan.close()
            lev.close()
        b1, b2 = hdr_px * (6 + 4), hdr_px * (4 + 4)
        dom = ("ltm_pass1", lk[0], b1) if lk[0] >= lk[2] else ("ltm_pass2", lk[2], b2)
        lach = dom[2] / (dom[1] * 1e-3) / 1e9
        local = {"workload": "hdr_tonemap_local", "images": n_img, "height": size, "width": size,
                 "src": "f16 linear RGB", "dst": "f32 T", "strength": 0.5, "tile": 64, "bins": 64,
                 "ms_per_step": round(lms, 4), "value": round(hdr_px / (lms * 1e-3) / 1e9, 3),
                 "unit": "Gpixels/s",
                 "kernel_ms": {"ltm_pass1": round(lk[0], 4), "combine_tables": round(lk[1], 4),
                               "ltm_pass2": round(lk[2], 4)},
                 "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(lach, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(lach / HBM_PEAK_GBS, 4), "traffic": traffic.get(dom[0]),
                              "algorithmic_bytes": dom[2]}}
        log("local tone map: step %.3f ms (%.1f Gpx/s); kernels %s ms" %
            (lms, local["value"], ", ".join("%.3f" % t for t in lk)))
        if result:
            result["local_tonemap"] = local
        else:
            result.update({"metric": METRIC, "value": local["value"], "unit": "Gpixels/s",
                           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                           "ms_per_step": local["ms_per_step"], "higher_is_better": True,
                           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                           "data": "synthetic", "config": {"workload": "hdr_tonemap_local"},
                           "roofline": local["roofline"], "local_tonemap": local})
        del louts
    if run_gray or run_colour or run_local:
        del xs
        torch.cuda.empty_cache()

    # ---------------------------------------------------- video batch decolorize
    if args.only in (None, "video") and not args.skip_video:
        import synth
        log("generating 64 video frames")
        t0 = time.time()
        frames = [torch.from_numpy(f).to(dev) for f in synth.video_frames(workers=WORKERS)]
        log("generated in %.1f s" % (time.time() - t0))
        vpx = sum(f.shape[0] * f.shape[1] for f in frames)
        o8 = [torch.empty(f.shape[:2], dtype=torch.uint8, device=dev) for f in frames]
        o32 = [torch.empty(f.shape[:2], dtype=torch.float32, device=dev) for f in frames]
        torch.cuda.synchronize()

        with torch.cuda.stream(stream):
            vtune = tune(P.PLAN_DECOLORIZE, frames, o8, o32)
            log("autotuned decolorize shape: %s" % vtune)
            vplan = P.Plan(P.PLAN_DECOLORIZE, frames, o8, o32, graph=True)
            vplan_ev = P.Plan(P.PLAN_DECOLORIZE, frames, o8, o32, graph=False)
            # plain per-image launches: one kernel per frame, no host marshalling
            singles = [P.Plan(P.PLAN_DECOLORIZE, [f], [a], [b]) for f, a, b in zip(frames, o8, o32)]

            def vstep_single():
                for sp in singles:
                    sp.run(stream)

            kernel_times(lambda: vplan_ev.run(stream), max(5, args.steps // 2), P, dev)
            vms = time_steps(lambda: vplan.run(stream), args.steps, args.warmup, stream)
            vk = kernel_times(lambda: vplan_ev.run(stream), max(5, args.steps // 2), P, dev)[0]
            vms_single = None if args.no_per_image else \
                time_steps(vstep_single, max(3, args.steps // 2), 1, stream)
            vplan.close()
            vplan_ev.close()
            for sp in singles:
                sp.close()
            comp = sweep = None
            if not args.no_per_image:
                comp = channels_leg(P, dev, stream, frames, o32, 10)
                sweep = sweep_leg(P, dev, stream, frames[-1], 10, traffic)
        # 8-bit and FP32 parity on 4 of the frames against the oracle's value of
        # every 24-bit colour (the LSB-mismatch fraction of the u8 output)
        parity = None
        if not args.no_cpu_baseline:
            import oracle
            lut = oracle.all_colours()
            off = total = 0
            worst = 0.0
            for i in (0, 1, 32, 33):
                # the frame again through dc_decolorize (bit-identical to the
                # batch): the comparison legs above reused the FP32 outputs
                g8, g32 = P.decolorize(frames[i], torch.uint8, torch.float32)
                f = frames[i].cpu().numpy().astype(np.int64)
                want = lut[(f[..., 0] << 16) | (f[..., 1] << 8) | f[..., 2]] / 255.0
                d = np.abs(g8.cpu().numpy().astype(np.int32) -
                           oracle.encode_u8(want).astype(np.int32))
                off += int(np.count_nonzero(d))
                total += d.size
                worst = max(worst, float(np.max(np.abs(g32.cpu().numpy() - want))))
            parity = {"frames": 4, "pixels": total, "u8_lsb_mismatch_fraction": off / total,
                      "max_abs_err_f32": worst}
            del lut
        vbytes = vpx * 8
        vach = vbytes / (vk * 1e-3) / 1e9
        video = {"workload": "video_decolorize", "frames": "32x1920x1080 + 32x3840x2160",
                 "src": "u8 sRGB", "dst": "u8 + f32", "ms_per_step": round(vms, 4),
                 "value": round(vpx / (vms * 1e-3) / 1e9, 3), "unit": "Gpixels/s",
                 "per_image_launches_gpx": round(vpx / (vms_single * 1e-3) / 1e9, 3)
                 if vms_single else None,
                 "tuning": {"groups_u8": vtune["groups"][0],
                            "grid_per_cu": vtune["decolor_grid_per_cu"]},
                 "gray_channels_u8_to_f32_gpx": comp,
                 "parity_sample": parity,
                 "beta_sweep": sweep,
                 "roofline": {"bound": "hbm", "kernel": "decolor_table", "achieved": round(vach, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(vach / HBM_PEAK_GBS, 4),
                              "traffic": traffic.get("decolor_table"),
                              "algorithmic_bytes": vbytes}}
        log("video step %.3f ms (%.1f Gpx/s), kernel %.3f ms, %.0f GB/s; per-image launches %s "
            "Gpx/s" % (vms, video["value"], vk, vach, video["per_image_launches_gpx"]))
        if not result:
            result.update({"metric": METRIC, "value": video["value"], "unit": "Gpixels/s",
                           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                           "ms_per_step": video["ms_per_step"], "higher_is_better": True,
                           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                           "data": "synthetic", "config": {"workload": "video_decolorize"},
                           "roofline": video["roofline"]})
        else:
            result["video_decolorize"] = video
    # ---------------------------------------------------- gray channels alone
    if args.only == "channels":
        import synth
        frames = [torch.from_numpy(f).to(dev) for f in synth.video_frames(workers=WORKERS)]
        o32 = [torch.empty(f.shape[:2], dtype=torch.float32, device=dev) for f in frames]
        comp = channels_leg(P, dev, stream, frames, o32, max(args.steps, 1))
        result.update({"metric": METRIC, "value": comp["decolor_L"], "unit": "Gpixels/s",
                       "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                       "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                       "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                       "config": {"workload": "video_gray_channels_u8_to_f32"},
                       "gray_channels_u8_to_f32_gpx": comp})
        del frames, o32
    # ---------------------------------------------------- weight sweep alone
    if args.only == "sweep":
        import synth
        frame = torch.from_numpy(synth.video_frame(63)).to(dev)
        sweep = sweep_leg(P, dev, stream, frame, max(args.steps, 1), traffic)
        result.update({"metric": METRIC, "value": sweep["output_gpx_s"], "unit": "Gpixels/s",
                       "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                       "ms_per_step": sweep["kernel_ms"], "higher_is_better": True,
                       "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                       "data": "synthetic", "config": {"workload": sweep["workload"]},
                       "roofline": sweep["roofline"], "beta_sweep": sweep})
        del frame
    # ---------------------------------------------------- uneven batch decolorize
    if args.only in (None, "uneven") and not args.skip_uneven:
        import synth
        log("generating the uneven 256-image batch")
        t0 = time.time()
        imgs = [torch.from_numpy(a).to(dev) for a in synth.uneven_batch(workers=WORKERS)]
        log("generated in %.1f s" % (time.time() - t0))
        upx = sum(a.shape[0] * a.shape[1] for a in imgs)
        ubytes = sum(a.shape[0] * a.shape[1] * (3 * a.element_size() + 4) for a in imgs)
        uo = [torch.empty(a.shape[:2], dtype=torch.float32, device=dev) for a in imgs]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            utune = tune(P.PLAN_DECOLORIZE, imgs, uo)
            log("autotuned uneven-batch shape: %s" % utune)
            uplan = P.Plan(P.PLAN_DECOLORIZE, imgs, uo, graph=True)
            uplan_ev = P.Plan(P.PLAN_DECOLORIZE, imgs, uo, graph=False)
            singles = [P.Plan(P.PLAN_DECOLORIZE, [a], [o]) for a, o in zip(imgs, uo)]

            def ustep_single():
                for sp in singles:
                    sp.run(stream)

            kernel_times(lambda: uplan_ev.run(stream), max(5, args.steps // 2), P, dev)
            ums = time_steps(lambda: uplan.run(stream), args.steps, args.warmup, stream)
            uk = kernel_times(lambda: uplan_ev.run(stream), max(5, args.steps // 2), P, dev)[0]
            # Graph replay against the same launch made directly, in alternating
            # blocks: the step's time outside the kernel.
            ug, ud = [], []
            for _ in range(3):
                ud.append(time_steps(lambda: uplan_ev.run(stream), args.steps, 0, stream))
                ug.append(time_steps(lambda: uplan.run(stream), args.steps, 0, stream))
            ums_direct = float(np.median(ud))
            ums_single = None if args.no_per_image else \
                time_steps(ustep_single, max(3, args.steps // 2), 1, stream)
            for pl in [uplan, uplan_ev] + singles:
                pl.close()
        uach = ubytes / (uk * 1e-3) / 1e9
        uneven = {"workload": "uneven_batch_decolorize", "images": len(imgs), "pixels": upx,
                  "src": "128 u8 + 128 f16, sides log-uniform 64..4096", "dst": "f32",
                  "ms_per_step": round(ums, 4), "value": round(upx / (ums * 1e-3) / 1e9, 3),
                  "unit": "Gpixels/s", "kernel_ms": round(uk, 4),
                  "steady_ms_per_step": {"graph": round(float(np.median(ug)), 4),
                                         "direct_launch": round(ums_direct, 4)},
                  "per_image_launches_gpx": round(upx / (ums_single * 1e-3) / 1e9, 3)
                  if ums_single else None,
                  "tuning": {"mixed_groups": utune["mixed_groups"],
                             "grid_per_cu": utune["mixed_grid_per_cu"]},
                  "roofline": {"bound": "hbm", "kernel": "decolor_table (mixed)",
                               "achieved": round(uach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(uach / HBM_PEAK_GBS, 4),
                               "traffic": traffic.get("decolor_table_mixed"),
                               "algorithmic_bytes": ubytes}}
        log("uneven step %.3f ms (%.1f Gpx/s), kernel %.3f ms, %.0f GB/s; per-image launches %s"
            " Gpx/s" % (ums, uneven["value"], uk, uach, uneven["per_image_launches_gpx"]))
        if result:
            result["uneven_batch"] = uneven
        else:
            result.update({"metric": METRIC, "value": uneven["value"], "unit": "Gpixels/s",
                           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                           "ms_per_step": uneven["ms_per_step"], "higher_is_better": True,
                           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                           "data": "synthetic", "config": {"workload": "uneven_batch_decolorize"},
                           "roofline": uneven["roofline"]})
        del imgs, uo
        torch.cuda.empty_cache()

    # ---------------------------------------------------- one small image (latency)
    if args.only is None:
        import synth
        x = torch.from_numpy(synth.gradient_rects()).to(dev)
        o = torch.empty(x.shape[:2], dtype=torch.float32, device=dev)
        with torch.cuda.stream(stream):
            sp = P.Plan(P.PLAN_DECOLORIZE, [x], [o], graph=False)
            lat_ms = time_steps(lambda: sp.run(stream), 200, 20, stream)
            sp.close()
            call_ms = time_steps(lambda: P.decolorize(x, out=o, stream=stream), 200, 20, stream)
        small = {"workload": "gradient_rects_512x512_u8_to_f32", "pixels": 512 * 512,
                 "plan_launch_us": round(lat_ms * 1e3, 2), "per_call_api_us": round(call_ms * 1e3, 2)}
        log("512x512 u8 -> f32: %.2f us per plan launch, %.2f us per dc_decolorize call" %
            (small["plan_launch_us"], small["per_call_api_us"]))
        result["small_image"] = small

    # ---------------------------------------------------- serving loop
    if args.only in (None, "serve") and not args.skip_serve:
        result_serve = serve_leg(args, P, dev)
        if result:
            result["serving"] = result_serve
        else:
            result.update({"metric": METRIC, "value": result_serve["gpx_s"], "unit": "Gpixels/s",
                           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None,
                           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                           "dtype": "f32", "data": "synthetic",
                           "config": {"workload": "serving_tonemap"}, "serving": result_serve})

    if ceilings and result:
        result["ceilings"] = ceilings
    if args.save_tuning and saved:
        with open(args.save_tuning, "w") as f:
            json.dump(P.get_tuning(dev), f)
    print(json.dumps(add_traffic_rates(result)), flush=True)


if __name__ == "__main__":
    main()
