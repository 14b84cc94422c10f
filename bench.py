"""Benchmark: dynamic urban scene, coherent refit tracing against full re-trace.

Workload (one GPU): 8x8-block Manhattan grid, 32,002 triangles, 40 moving metal
vehicles, one rooftop transmitter, 256 receivers, 2^20 Fibonacci rays per frame,
up to 4 reflections, 28 GHz, 60 frames at 10 Hz.  A step is one frame of the
whole hot path: object transforms, BVH refit (or rebuild), ray shooting with
capture, candidate de-duplication, FP64 path refinement, per-receiver power,
and (coherent mode) the revalidation pass.  Inputs are resident on the GPU
before the timed region; the per-frame host calls are part of the step.  The
frame loop is software-pipelined: the next frame's transforms and BVH update
are enqueued before the current frame's powers are read back (each timed step
still does one geometry update and one trace).

Prints one JSON line.  `value` is delivered Mrays/s of the coherent mode
(rays whose result the frame delivers, traced or reused).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=59)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rays", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["both", "coherent", "full"], default="both")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-scene batched workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--variants-only", choices=["all", "visited_series", "backward", "transmission"],
                    help="time only the paper's variant workloads (one JSON object; for profiling them)")
    ap.add_argument("--large-only", action="store_true",
                    help="time only the large dynamic workload (one JSON object; for profiling it)")
    return ap.parse_args()


def run_mode(scene, mode, warmup, steps, n_rays, torch, instrumented):
    """Warmup + steps frames on a fresh context; returns the wall time of the
    timed frames, their powers and (instrumented: per-stage HIP event timings
    on, per-frame statistics collected) their frame statistics."""
    from paper_2112_07115_amd import dcem
    ctx = dcem.Context(0)
    ctx.scene_upload(scene)
    nf = scene.n_frames
    coherent = mode == "coherent"
    # per-frame object transforms, resident on the GPU before timing starts
    xfs = torch.tensor(np.stack([scene.transforms(f) for f in range(nf)]), device="cuda")
    xf_views = [xfs[f] for f in range(nf)]   # one device view per frame, made before timing

    def geometry(f):
        ctx.set_object_transforms(xf_views[f % nf])
        ctx.refit_bvh(force_rebuild=not coherent)

    def frame(f):
        # frame f's geometry is in place; the next frame's transforms and
        # refit are enqueued behind this frame before its powers are read
        # back, so the device does not wait for the host between frames
        ctx.trace_frame(scene.tx, scene.rx, scene.rx_radius, n_rays, max_reflections=scene.max_reflections,
                        freqs_hz=scene.freqs_hz, tx_power_w=scene.tx_power_w,
                        mode=dcem.MODE_COHERENT if coherent else dcem.MODE_FULL)
        geometry(f + 1)
        return ctx.received_power()

    ctx.set_timing(instrumented)
    geometry(0)
    for f in range(warmup):
        frame(f)
    outs, stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(warmup, warmup + steps):
        pc, _ = frame(f)
        outs.append(pc.copy())
        if instrumented:
            stats.append(ctx.stats())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return dt, outs, stats


def gradient_timing(scene, n_rays, calls=20):
    """Mean wall time of dcem_power_gradients on one traced frame (the derivative
    pass, its wait and the read-back of the results)."""
    from paper_2112_07115_amd import dcem
    ctx = dcem.Context(0)
    ctx.scene_upload(scene)
    ctx.set_object_transforms(scene.transforms(1))
    ctx.refit_bvh()
    ctx.trace_frame(scene.tx, scene.rx, scene.rx_radius, n_rays, max_reflections=scene.max_reflections,
                    freqs_hz=scene.freqs_hz, tx_power_w=scene.tx_power_w)
    ctx.received_power()
    ctx.power_gradients()
    t0 = time.perf_counter()
    for _ in range(calls):
        ctx.power_gradients()
    dt = (time.perf_counter() - t0) / calls
    st = ctx.stats()
    ctx.close()
    return {"ms_per_call": dt * 1e3, "calls": calls, "valid_paths": st["valid_paths"],
            "paths_per_s": st["valid_paths"] / dt,
            "outputs": "dP/d eps_r and dP/d sigma of %d materials, dP/dP_t and dP/dw of the 16 transmit "
                       "pattern weights for %d receivers, frame 1"
                       % (scene.materials.shape[0], scene.rx.shape[0])}


def batched_bench(torch, steps=3, n_scenes=64):
    """The ragged batch workload: 64 independent cities (10k-500k triangles,
    1-8 transmitters, 256k-4M rays, 2-6 reflections, 64-1024 receivers, 28 or
    60 GHz), one frame of each per step.  Timed three ways, each step from the
    object transforms to every scene's powers read back: one batched frame
    (one persistent trace launch for all scenes, shape from the autotuner),
    the same captured as one HIP graph, and the 64 scenes traced one after
    the other with their own launches."""
    from paper_2112_07115_amd import dcem, scenes
    ws = scenes.batched_workload(n_scenes, seed=3)
    stream = torch.cuda.Stream()
    out = {"scenes": n_scenes, "triangles": int(sum(s.n_tris for s in ws)),
           "rays_per_frame": int(sum(s.n_rays * s.tx.shape[0] for s in ws))}
    with torch.cuda.stream(stream):
        ctxs = [dcem.Context(0, stream=stream.cuda_stream) for _ in ws]
        xfs = []
        for c, s in zip(ctxs, ws):
            c.scene_upload(s)
            xfs.append(torch.tensor(np.stack([s.transforms(f) for f in range(s.n_frames)]), device="cuda"))
        frames = [dcem.scene_frame_args(s) for s in ws]
        batch = dcem.Batch(ctxs)

        def place(f):
            for c, s, x in zip(ctxs, ws, xfs):
                c.set_object_transforms(x[f % s.n_frames])
                c.refit_bvh()

        def read():
            for c in ctxs:
                c.received_power()

        place(0)
        t0 = time.perf_counter()
        out["tuning"] = batch.tune(frames, repeats=1)
        out["tuning"]["s"] = time.perf_counter() - t0
        read()

        def timed(step_fn):
            step_fn(1)   # warm-up (buffers, graph instantiation)
            stream.synchronize()
            t0 = time.perf_counter()
            for f in range(2, 2 + steps):
                step_fn(f)
            stream.synchronize()
            return (time.perf_counter() - t0) / steps

        def batched(f):
            place(f)
            batch.trace(frames)
            read()

        def single(f):
            place(f)
            for c, fa in zip(ctxs, frames):
                c.trace_frame(**fa)
            read()

        t_b = timed(batched)
        batch.set_graph(True)
        t_g = timed(batched)
        graph_frames = batch.info()["graph_frames"]
        batch.set_graph(False)
        t_s = timed(single)
        batch.close()
        for c in ctxs:
            c.close()
    n = out["rays_per_frame"]
    out.update({"steps": steps, "ms_per_frame_batched": t_b * 1e3, "ms_per_frame_batched_graph": t_g * 1e3,
                "graph_frames": graph_frames, "ms_per_frame_single": t_s * 1e3,
                "mrays_per_s_batched": n / t_b / 1e6, "mrays_per_s_batched_graph": n / t_g / 1e6,
                "mrays_per_s_single": n / t_s / 1e6, "batched_speedup": t_s / t_b})
    return out


def large_bench(torch, frames=6):
    """The large dynamic workload: a 6 km highway corridor beside a 16x16
    block city (2.04M triangles), 200 vehicles at 15-35 m/s carrying 4096
    receivers, 4 roadside transmitters x 4M Fibonacci rays (16.8M rays per
    frame), 6 reflections, 28 and 60 GHz from one trace.  Coherent frames
    (refit, revalidation, re-capture of the kept segments at the moved
    receivers, re-trace of the invalidated rays) against full frames
    (rebuild, trace every ray); both equal bitwise.  Frame 0 is the
    first full trace of each context and is not timed.  Also the power
    gradients of one frame (8 derivatives per receiver and band: the 3
    materials' eps_r and sigma, P_t; plus 16 pattern weights)."""
    from paper_2112_07115_amd import dcem, scenes
    s = scenes.highway_city()
    out = {"triangles": s.n_tris, "vehicles": s.n_objects, "receivers": int(s.rx.shape[0]), "tx": int(s.tx.shape[0]),
           "rays_per_frame": int(s.n_rays * s.tx.shape[0]), "max_reflections": s.max_reflections,
           "bands_ghz": [f / 1e9 for f in s.freqs_hz]}
    res = {}
    for mode in ("coherent", "full"):
        ctx = dcem.Context(0)
        ctx.set_capture_capacity(1 << 24)
        ctx.scene_upload(s)
        last = None
        dcem.trace_scene_frame(ctx, s, frame=0, mode=dcem.MODE_COHERENT if mode == "coherent" else dcem.MODE_FULL,
                               rebuild=mode == "full")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        traced = 0
        for f in range(1, frames + 1):
            last = dcem.trace_scene_frame(ctx, s, frame=f, rebuild=mode == "full",
                                          mode=dcem.MODE_COHERENT if mode == "coherent" else dcem.MODE_FULL)
            traced += ctx.stats()["rays_traced"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / frames
        st = ctx.stats()
        res[mode] = {"ms_per_frame": dt * 1e3, "frames_per_s": 1.0 / dt,
                     "mrays_per_s": out["rays_per_frame"] / dt / 1e6,
                     "rays_traced_fraction": traced / (frames * out["rays_per_frame"]),
                     "captures": st["captures"], "valid_paths": st["valid_paths"]}
        if mode == "coherent":
            g0 = time.perf_counter()
            for _ in range(5):
                ctx.power_gradients()
            gdt = (time.perf_counter() - g0) / 5
            res["power_gradients"] = {"ms_per_call": gdt * 1e3, "valid_paths": st["valid_paths"],
                                      "paths_per_s": st["valid_paths"] / gdt,
                                      "receiver_bands_per_s": out["receivers"] * out["tx"] * len(s.freqs_hz) / gdt}
            coh_power = last.p_coh.copy()
        else:
            res["coherent_vs_full_bitwise_equal"] = bool(np.array_equal(coh_power, last.p_coh))
        ctx.close()
    out.update(res)
    out["coherent_speedup"] = res["full"]["ms_per_frame"] / res["coherent"]["ms_per_frame"]
    return out


def variants_bench(torch, frames=4, only=None):
    """The paper's variants of the frame algorithm (Sec. III), each at its
    workload, full frames timed after one untimed frame (wall clock over the
    frames, the host round trips of visited-series discovery included):
      visited_series  dynamic_urban (2^20 Fibonacci rays, K = 4, 256 Rx):
                      every distinct series of faces the rays visit tried
                      against every receiver, against capture spheres;
      backward        the same scene traced from the 256 receivers (4096
                      rays each, 2^20 in all), visited series;
      transmission    the indoor office (396 triangles, 336 Rx, 30 GHz),
                      2^18 rays, K = 2 reflections and 2 transmissions
                      through walls (20 dB) and glass (5 dB): 11 branches
                      per ray, visited series and capture spheres."""
    from paper_2112_07115_amd import dcem, scenes

    def timed(s, label, **kw):
        ctx = dcem.Context(0)
        ctx.set_capture_capacity(1 << 24)
        ctx.scene_upload(s)
        dcem.trace_scene_frame(ctx, s, frame=0, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(1, frames + 1):
            dcem.trace_scene_frame(ctx, s, frame=f if s.n_frames > 1 else 0, **kw)
            ctx.received_power()
        dt = (time.perf_counter() - t0) / frames
        st = ctx.stats()
        ctx.close()
        work = st["rays_total"]
        return {"case": label, "ms_per_frame": dt * 1e3, "work_items_per_frame": int(work),
                "mrays_per_s": work / dt / 1e6, "candidates": int(st["unique_candidates"]),
                "valid_paths": int(st["valid_paths"])}

    urban = scenes.dynamic_urban()
    office = scenes.indoor_office()
    cases = {"visited_series": lambda: [timed(urban, "capture spheres"),
                                        timed(urban, "visited series", discovery=dcem.DISCOVER_VISITED)],
             "backward": lambda: [timed(urban, "from the receivers, visited series", trace_from_rx=True,
                                        discovery=dcem.DISCOVER_VISITED, n_rays=4096)],
             "transmission": lambda: [timed(office, "visited series", discovery=dcem.DISCOVER_VISITED),
                                      timed(office, "capture spheres")]}
    return {k: f() for k, f in cases.items() if only in (None, "all", k)}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def cpu_baseline(scene):
    """The oracle (plain FP64 brute force, no BVH) on the host cores: frames 0,
    1 and 59 of the urban workload on every 16th Fibonacci ray with all its
    threads (`value`), frame 1 on every 256th ray with one thread, and the
    static toy frame in full (4096 rays, K = 2) with both."""
    from oracle import oracle
    from paper_2112_07115_amd import scenes
    threads = oracle.default_threads()
    fib = oracle.fibonacci(scene.n_rays)
    legs = []

    def leg(name, sc, frame_index, dirs, nthreads):
        t0 = time.perf_counter()
        oracle.frame(sc, frame_index=frame_index, dirs=dirs, nthreads=nthreads)
        dt = time.perf_counter() - t0
        legs.append({"leg": name, "frame": frame_index, "rays": int(dirs.shape[0]), "threads": nthreads,
                     "s": dt, "mrays_per_s": dirs.shape[0] / dt / 1e6})
        return dt

    sub = fib[::16].copy()
    total = sum(leg("dynamic_urban 1/16 rays", scene, f, sub, threads) for f in (0, 1, 59))
    leg("dynamic_urban 1/256 rays", scene, 1, fib[::256].copy(), 1)
    toy = scenes.static_toy()
    tdirs = oracle.fibonacci(toy.n_rays)
    leg("static_toy full frame", toy, 0, tdirs, threads)
    leg("static_toy full frame", toy, 0, tdirs, 1)
    return {"value": 3 * sub.shape[0] / total / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": "dynamic_urban frames 0, 1, 59 on every 16th of the 2^20 Fibonacci rays (%d rays each), "
                      "full frame (trace, candidates, refinement, power), %.1f s wall on %d threads"
                      % (sub.shape[0], total, threads),
            "cpu": cpu_info(), "legs": legs}


# Algorithmic bytes of one closest-hit launch (what the traversal must read
# and write, counted once per use; nothing assumed cached):
#   per-thread kernel: 128 B per 4-wide node fetched from memory (the top
#     three levels are read from LDS and not counted), 48 B per triangle test,
#     per ray 13 B (direction, order entry, state), per segment 4 B (face log)
#     + 32 B when the segment cache is kept, 8 B per capture record;
#   group kernel: per node visit its four 32-byte slots (a leaf slot reads its
#     48-byte triangle instead: +16 B per triangle test), per ray 42 B (list
#     entry, restart, cached segment, face, state), per segment 84 B (face log,
#     segment cache, reflecting triangle), 8 B per capture record.
def trace_bytes(s, kernel_cache):
    if s["trace_kernel"] == 1:
        return 128 * s["nodes_visited"] + 16 * s["tri_tests"] + 42 * s["rays_traced"] + 84 * s["segments"] \
            + 8 * s["captures"]
    return 128 * s["nodes_visited"] + 48 * s["tri_tests"] + 13 * s["rays_traced"] \
        + (4 + (32 if kernel_cache else 0)) * s["segments"] + 8 * s["captures"]


PROFILE = os.path.join(ROOT, "profiles", "dynamic_urban_bench_kernels.md")
KERNEL_SOURCES = ["paper_2112_07115_amd/csrc/dcem_internal.h", "paper_2112_07115_amd/csrc/bvh.hip",
                  "paper_2112_07115_amd/csrc/trace.hip", "paper_2112_07115_amd/csrc/refit.h"]


def measured_traffic(kernel, mode):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        lines = open(PROFILE).read().splitlines()
    except OSError:
        return None
    for line in lines:
        if not line.startswith("traffic-record:"):
            continue
        kv = dict(x.split("=", 1) for x in line.split()[1:])
        if kv.get("kernel") == kernel and kv.get("mode") == mode and kv.get("sources") == h.hexdigest()[:16]:
            return float(kv["bytes"])
    return None


def roofline(stats, mode):
    """Achieved algorithmic GB/s of the closest-hit kernel against HBM peak;
    kernel time from the HIP events around the launch on the library's stream."""
    sel = [s for s in stats if s["ms_trace"] > 0]
    kinds = [s["trace_kernel"] for s in sel]
    kind = max(set(kinds), key=kinds.count) if kinds else 0   # the traversal most frames used
    sel = [s for s in sel if s["trace_kernel"] == kind]
    name = "k_trace_wave" if kind == 1 else "k_trace"
    ms = float(np.mean([s["ms_trace"] for s in sel]))
    by = float(np.mean([trace_bytes(s, mode == "coherent") for s in sel]))
    segs = float(sum(s["segments"] for s in sel))
    achieved = by / (ms * 1e-3) / 1e9
    traffic = measured_traffic(name, "coh" if mode == "coherent" else "full")
    out = {"bound": "hbm", "kernel": name + (" (coherent frame re-trace)" if kind == 1 else " (%s frame)" % mode),
           "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
           "traffic": traffic, "bytes_per_launch": by, "ms_per_launch": ms,
           "traced_mseg_per_s": segs / max(len(sel), 1) / (ms * 1e-3) / 1e6,
           "nodes_per_segment": float(sum(s["nodes_visited"] for s in sel)) / max(segs, 1.0),
           "tris_per_segment": float(sum(s["tri_tests"] for s in sel)) / max(segs, 1.0),
           "segments_per_launch": segs / max(len(sel), 1), "launches": len(sel)}
    if traffic:
        # what HBM actually moved (rocprofv3 counters) against the peak: the
        # traversal is bound by dependent round trips, not by bandwidth
        out["hbm_measured"] = {"gbps": traffic / (ms * 1e-3) / 1e9, "frac": traffic / (ms * 1e-3) / 1e9 / 8000.0}
    return out



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2112_07115_amd import dcem, scenes
    if args.variants_only:
        print(json.dumps({"variants": variants_bench(torch, only=args.variants_only)}))
        return
    if args.large_only:
        print(json.dumps({"large_dynamic": large_bench(torch)}))
        return
    scene = scenes.dynamic_urban(n_rays=args.rays)
    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    res = {}
    # per mode: the timed run (no instrumentation: it gives `value`), then the
    # same frames again on a fresh context with stage timings and statistics
    for mode in (["coherent", "full"] if args.mode == "both" else [args.mode]):
        dt, outs, _ = run_mode(scene, mode, args.warmup, args.steps, args.rays, torch, False)
        _, _, stats = run_mode(scene, mode, args.warmup, args.steps, args.rays, torch, True)
        res[mode] = (dt, outs, stats)
    main_mode = "coherent" if "coherent" in res else "full"
    dt, outs, stats = res[main_mode]
    steps = args.steps
    n = args.rays
    out = {
        "metric": "Mrays/s and frames/s, coherent-refit vs full retrace, at <=0.01 dB power error",
        "value": n * steps / dt / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dynamic_urban: 8x8 grid, 32002 tris, 40 moving vehicles, 1 rooftop Tx, "
                               "256 Rx, %d Fibonacci rays/frame, K=4, 28 GHz, frames %d..%d of 60 at 10 Hz"
                               % (n, args.warmup, args.warmup + steps - 1),
                   "mode": main_mode, "geometry": "f32", "paths": "f64"},
    }
    out["frames_per_s"] = steps / dt
    if "full" in res:
        dtf, outsf, statsf = res["full"]
        out["full_retrace"] = {"mrays_per_s": n * steps / dtf / 1e6, "frames_per_s": steps / dtf,
                               "ms_per_step": dtf / steps * 1e3,
                               "ms_trace_kernel": float(np.mean([s["ms_trace"] for s in statsf])),
                               "ms_rebuild": float(np.mean([s["ms_refit"] for s in statsf]))}
        if "coherent" in res:
            out["coherent_speedup"] = dtf / dt
            worst, nbitdiff = 0.0, 0
            for a, b in zip(outs, outsf):
                nbitdiff += int(np.sum(a != b))
                m = (a > 0) & (b > 0)
                if m.any():
                    worst = max(worst, float(np.max(np.abs(10 * np.log10(a[m] / b[m])))))
                worst = max(worst, float(np.inf) if np.any((a > 0) != (b > 0)) else 0.0)
            out["coherent_vs_full"] = {"max_abs_db": worst, "elements_not_bitwise_equal": nbitdiff}
    traced = np.array([s["rays_traced"] for s in stats], float)
    out["rays_traced_fraction"] = float(traced.sum() / (n * steps))
    out["ms_refit"] = float(np.mean([s["ms_refit"] for s in stats]))
    out["ms_stages"] = {k: float(np.mean([s[k] for s in stats])) for k in
                        ["ms_coherence", "ms_trace", "ms_candidates", "ms_refine", "ms_reduce"]}
    # roofline of the closest-hit kernel, the largest kernel of both steps:
    # the group re-trace in coherent frames, the per-thread trace in full ones
    out["roofline"] = roofline(stats, "coherent" if main_mode == "coherent" else "full")
    if "full" in res and main_mode != "full":
        out["roofline_full_trace"] = roofline(res["full"][2], "full")
    out["power_gradients"] = gradient_timing(scene, n)
    if not args.no_batch and args.mode == "both":
        out["batched"] = batched_bench(torch)
        out["large_dynamic"] = large_bench(torch)
        out["variants"] = variants_bench(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
