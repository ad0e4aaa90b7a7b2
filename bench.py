#!/usr/bin/env python3
"""Shading samples/s and cache hit rate of progressive material caching on one MI355X.

One step = one progressive render of the workload from an empty table: every
frame (one batch of hits, one sample per pixel) goes through material sort,
key computation, probes, the node interpreter on misses and lock-free inserts
(the paper's GPU update, Sec. 3.3).  Inputs are generated on the host, seeded,
and resident in HBM before timing starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shading samples/s + cache hit rate, cached/surrogate vs uncached, 1 MI355X"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes of the shade kernel (per unit of work)
B_HIT_IN = 40          # material 4, uv 8, duv 16, normal 12
B_HIT_OUT = 28         # base colour 12, roughness 4, normal 12
B_PERM = 4             # sorted index read
B_PROBE = 128          # one N_e x 16 B cell scanned per lookup
B_INSERT = 16          # one entry written per miss that inserts
B_TEXEL = 16           # four RGBA8 texels per evaluated image-texture node


def kernel_bytes(st, n_hits):
    """Algorithmic bytes of one step of the shade kernel (all its launches)."""
    return (n_hits * (B_HIT_IN + B_PERM + B_HIT_OUT) +
            (st["probes"] + st["probes_deferred"]) * B_PROBE +
            st["deferred"] * (B_HIT_IN + 4) +
            st["insert_attempts"] * B_INSERT + st["texture_evals"] * B_TEXEL)


KERNEL_SOURCES = ("shade.hip", "shade.h", "device_common.h", "program.h")


def measured_traffic(workload_name, best, late_frame=0, late=None):
    """HBM bytes per launch of the shade kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy calibration), or None
    when the kernel sources or the launch settings differ from the profiled ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "shade_%s_traffic.json" % workload_name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_07238_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    def same(rec, want):
        return (rec.get("waves_per_block", 4) == (want.get("waves_per_block", 0) or 4) and
                all(rec[k] == want[k] for k in ("flags", "chunk_waves", "defer_max")))
    for rec in recs:
        if h.hexdigest() != rec["source_sha256"] or not same(rec, best):
            continue
        if rec.get("late_frame", 0) != late_frame:
            continue
        if late_frame and not same(rec["late"], late):
            continue
        return rec["traffic_bytes_per_launch"]
    return None


def shade_kernel_name(mode, flags):
    """Name of the shade kernel a timed step launches (template arguments: mode,
    kind (1 = probe first with deferral), counters, networks)."""
    from paper_2305_07238_amd import binding as B
    m = {"uncached": 0, "cached": 1, "snapshot": 2}[mode]
    kind = 1 if (m != 0 and flags & B.PMC_FLAG_DEFER) else 0
    base = "k_shade_persistent" if flags & B.PMC_FLAG_PERSISTENT else "k_shade_flat"
    if m != 0:
        base += "_w4"
    return "%s<%d, %d, false, false>" % (base, m, kind)


def scenes_concat(sc):
    from paper_2305_07238_amd import scenes
    return scenes.Hits.concat([sc.frame(f) for f in range(sc.frames)])


def workload(name, frames=None):
    from paper_2305_07238_amd import scenes
    if name == "mid":
        sc = scenes.mid_scene(frames=frames or 16)
        desc = ("mid: 64 materials (8-64 nodes: image texture 1024^2 RGBA8, Perlin 4 oct, mix, "
                "math, ramp, normal map), 1920x1080 x %d progressive frames, Zipf(1.1) materials, "
                "table 2^22 slots x 16 B (N_c=524288, N_e=8), keep-first" % sc.frames)
    elif name == "tiny":
        sc = scenes.tiny_scene()
        desc = "tiny: 1 material, 8 nodes, 64x64 px x 4 spp, table 2^16 slots x 16 B"
    elif name == "batching":
        sc = scenes.batching_scene(frames=frames or 64)
        desc = ("batching: 1000 materials (lognormal sizes 4-400 nodes), 1920x1080 x %d frames, "
                "table 2^24 slots x 16 B" % sc.frames)
    elif name == "scale":
        sc = scenes.scale_scene(frames=frames or 128)
        desc = ("scale: 4096 materials (lognormal sizes 8-400 nodes), 3840x2160 x %d frames, "
                "table 2^26 slots x 16 B (1 GiB), overwrite-oldest" % sc.frames)
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


SURR_FLOP_PER_POINT = 2 * (32 * 64 + 64 * 64 + 64 * 4)     # 12,800 per network evaluation
FP16_PEAK_TFLOPS = 2500.0
TRAIN = dict(steps=8000, batch=1024, lr=2e-2, lr_end=1e-5, seed=0)


def _median_ms(fn, reps=5):
    import torch
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn(pre=True)
        e0.record()
        fn(pre=False)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _errors_vs_uncached(results):
    """Max and mean absolute error of every BSDF output of each variant against the
    variant "uncached" (the same hits, plain evaluation on the GPU)."""
    ref = results["uncached"]["_out"]
    for r in results.values():
        got = r["_out"]
        errs = np.concatenate([np.abs(got[k] - ref[k]).ravel()
                               for k in ("base_color", "roughness", "normal")])
        r["max_abs_err_vs_uncached"] = float(errs.max())
        r["mean_abs_err_vs_uncached"] = float(errs.mean())
    for r in results.values():
        del r["_out"]


def surrogate_leg(ctx, sc, frame_views, out, cache, best, log):
    """Learned surrogate (the mid scene after its progressive render): train every
    network on the insert log the render collected, then shade the next pass
    (its first 2^20 hits) from the render's final table: uncached, cache only,
    and networks + cache; errors of every output against the uncached GPU path (the
    plain evaluation, which the parity tests hold to the FP64 graph within 1e-5)."""
    import torch
    from paper_2305_07238_amd import binding as B
    n_slots = ctx.surrogate_setup(seed=0)
    flags = best["flags"] & ~(B.PMC_FLAG_LOG | B.PMC_FLAG_SURROGATE)
    kw = dict(chunk_waves=best["chunk_waves"], defer_max=best["defer_max"],
              blocks_per_cu=best["blocks_per_cu"], waves_per_block=best["waves_per_block"])
    cache.clear()
    ctx.log_clear()
    for f in range(sc.frames):
        ctx.shade(frame_views[f], out, cache, mode=B.PMC_MODE_CACHED, frame=f,
                  flags=flags | B.PMC_FLAG_LOG, **kw)
    torch.cuda.synchronize()
    n_log = len(ctx.log_read())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.surrogate_train(**TRAIN)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    rep = ctx.surrogate_report()
    trained = [r for r in rep if r["steps"] > 0]
    trusted = [k for k, r in enumerate(rep) if r["trusted"]]
    log(f"surrogate: {n_slots} slots, {len(trained)} trained on {n_log} log records in "
        f"{train_ms:.1f} ms, {len(trusted)} trusted")
    train_flop = 3.0 * SURR_FLOP_PER_POINT * TRAIN["batch"] * TRAIN["steps"] * len(trained)

    table = cache.export()
    n17 = min(1 << 20, sc.hits_per_frame)
    h17 = sc.frame(sc.frames).take(np.arange(n17))
    d17 = B.hits_to_device(h17)
    o17 = B.alloc_outputs(n17)
    results = {}
    for name, use_cache, f in (("uncached", False, 0), ("cache_only", True, 0),
                               ("surrogate_cache", True, B.PMC_FLAG_SURROGATE)):
        def run(pre, use_cache=use_cache, f=f):
            if pre:
                if use_cache:
                    cache.import_(table)
                for k in trusted:
                    ctx.surrogate_set_trust(k, True)
                torch.cuda.synchronize()
                return
            ctx.shade(d17, o17, cache if use_cache else None,
                      mode=B.PMC_MODE_CACHED if use_cache else B.PMC_MODE_UNCACHED,
                      frame=sc.frames, flags=flags | f, **kw)
        ms = _median_ms(run)
        got = {k: v.cpu().numpy().astype(np.float64) for k, v in o17.items()}
        results[name] = {"samples_per_s": n17 / (ms * 1e-3), "ms": ms, "_out": got}
    _errors_vs_uncached(results)
    # network inference on the matrix cores: 2^20 points through one slot
    uv = d17["uv"]
    y = torch.empty((n17, 4), dtype=torch.float32, device="cuda")
    # back-to-back launches, so the host's launch time does not enter the figure
    reps = 20

    def infer_batch(pre):
        if not pre:
            for _ in range(reps):
                ctx.surrogate_infer(0, uv, y)
    ms_inf = _median_ms(infer_batch) / reps
    inf_tflops = SURR_FLOP_PER_POINT * n17 / (ms_inf * 1e-3) / 1e12
    return {
        "slots": n_slots, "trusted": len(trusted), "log_records": n_log,
        "train": dict(TRAIN, ms=train_ms, slots_trained=len(trained),
                      tflops=train_flop / (train_ms * 1e-3) / 1e12),
        "heldout_max_err": [r["max_err"] for r in rep],
        "heldout_mean_err": [r["mean_err"] for r in rep],
        "pass_hits": n17, "pass": results,
        "gain_vs_cache_only": results["cache_only"]["ms"] / results["surrogate_cache"]["ms"],
        "infer": {"points": n17, "ms": ms_inf, "tflops": inf_tflops,
                  "roofline": {"bound": "mfma", "achieved": inf_tflops,
                               "peak": FP16_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": inf_tflops / FP16_PEAK_TFLOPS}},
    }


def surrogate_smooth_leg(log):
    """The networks where they can be trusted: a 1920x1080 scene of 4 materials whose
    deep sub-graphs are expensive but low-frequency functions of UV (12 Perlin layers
    averaged).  Snapshot frames with the log on collect training pairs; every network
    is trained (one launch) and trusted when its held-out maximum error is at most
    5e-3; then the first frame alone (cold table) and a 4-frame progressive render, each
    from an empty table, are timed uncached, cache only, and networks + cache; errors
    of the last frame's outputs against the uncached GPU path."""
    import torch
    from paper_2305_07238_amd import binding as B
    from paper_2305_07238_amd import scenes
    sc = scenes.smooth_scene(width=1920, height=1080, frames=4, slots=1 << 22)
    n = sc.hits_per_frame
    frames = [B.hits_to_device(sc.frame(f)) for f in range(sc.frames)]
    out = B.alloc_outputs(n)
    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials)
    n_slots = ctx.surrogate_setup(seed=0, max_err=5e-3)
    cache = ctx.cache(sc.cache.n_cells, 8, 16)
    ctx.log_clear()
    for f in range(sc.frames):
        ctx.shade(frames[f], out, cache, mode=B.PMC_MODE_SNAPSHOT, frame=f,
                  flags=B.PMC_FLAG_SORT | B.PMC_FLAG_LOG)
    torch.cuda.synchronize()
    n_log = len(ctx.log_read())
    train = dict(steps=48000, batch=512, lr=2e-2, lr_end=2e-6, seed=0, min_records=256)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.surrogate_train(**train)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    rep = ctx.surrogate_report()
    trusted = [k for k, r in enumerate(rep) if r["trusted"]]
    log(f"smooth scene: {len(trusted)} of {n_slots} networks trusted after {train_ms:.0f} ms")
    results, cold = {}, {}
    for name, use_cache, f in (("uncached", False, 0), ("cache_only", True, 0),
                               ("surrogate_cache", True, B.PMC_FLAG_SURROGATE),
                               ("surrogate_insert_cache", True,
                                B.PMC_FLAG_SURROGATE | B.PMC_FLAG_SURROGATE_INSERT)):
        def run(pre, use_cache=use_cache, f=f, n_frames=sc.frames):
            if pre:
                for k in trusted:
                    ctx.surrogate_set_trust(k, True)
                if use_cache:
                    cache.clear()
                torch.cuda.synchronize()
                return
            for fr in range(n_frames):
                ctx.shade(frames[fr], out, cache if use_cache else None,
                          mode=B.PMC_MODE_CACHED if use_cache else B.PMC_MODE_UNCACHED,
                          frame=fr, flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER | f)
        ms1 = _median_ms(lambda pre, run=run: run(pre, n_frames=1))
        cold[name] = {"samples_per_s": n / (ms1 * 1e-3), "ms": ms1}
        ms = _median_ms(run)
        last = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        results[name] = {"samples_per_s": n * sc.frames / (ms * 1e-3), "ms": ms, "_out": last}
    _errors_vs_uncached(results)
    # texels 8x finer than the footprints (level bias +3): the table reuses far
    # less, so more lookups miss, and a miss of a trusted output costs one
    # network evaluation instead of the sub-graph
    fine = ctx.cache(sc.cache.n_cells, 8, 16, level_bias=3)
    fine_res = {}
    for name, f in (("cache_only", 0), ("surrogate_cache", B.PMC_FLAG_SURROGATE)):
        st = B.new_stats()

        def run_fine(pre, f=f, st=st):
            if pre:
                for k in trusted:
                    ctx.surrogate_set_trust(k, True)
                fine.clear()
                st.zero_()
                torch.cuda.synchronize()
                return
            for fr in range(sc.frames):
                ctx.shade(frames[fr], out, fine, mode=B.PMC_MODE_CACHED, frame=fr,
                          flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER | f, stats=st)
        ms = _median_ms(run_fine)
        sd = B.stats_dict(st)
        fine_res[name] = {"samples_per_s": n * sc.frames / (ms * 1e-3), "ms": ms,
                          "hit_rate": sd["cache_hits"] / max(sd["probes"], 1),
                          "surrogate_used": sd["surrogate_used"]}
    ctx.close()
    return {"workload": "smooth: 4 materials of 38 nodes (12 low-frequency Perlin layers averaged, "
                        "MUL/POW chain), 1920x1080 x 4 progressive frames, table 2^22 slots, "
                        "trust at held-out max error 5e-3",
            "log_records": n_log, "train": dict(train, ms=train_ms), "trusted": len(trusted),
            "slots": n_slots, "heldout_max_err": [r["max_err"] for r in rep],
            "render": results, "cold_first_frame": cold,
            "cold_gain_vs_cache_only": cold["cache_only"]["ms"] / cold["surrogate_cache"]["ms"],
            "gain_vs_cache_only": results["cache_only"]["ms"] / results["surrogate_cache"]["ms"],
            "insert_gain_vs_cache_only": (results["cache_only"]["ms"] /
                                          results["surrogate_insert_cache"]["ms"]),
            "gain_vs_uncached": results["uncached"]["ms"] / results["surrogate_cache"]["ms"],
            "fine_texels": dict(fine_res, level_bias=3,
                                gain_vs_cache_only=(fine_res["cache_only"]["ms"] /
                                                    fine_res["surrogate_cache"]["ms"]))}


def cpu_baseline(sc, sample_hits=786432, frames=3):
    """The FP64 oracle (snapshot-mode progressive shading) on a bounded sample."""
    from oracle import render, table
    t = table.Table(sc.cache.n_cells, sc.cache.n_entries, sc.cache.entry_bytes)
    batches = [sc.frame(f).take(np.arange(min(sample_hits, sc.hits_per_frame)))
               for f in range(min(frames, sc.frames))]
    t0 = time.perf_counter()
    render.shade_snapshot(sc.materials, sc.textures, batches, t)
    dt = time.perf_counter() - t0
    n = sum(len(b) for b in batches)
    return {"value": n / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"first {len(batches[0])} hits (screen order) of frames 0-{len(batches)-1}, "
                      f"snapshot-mode shading in FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--frames", type=int, default=0)
    ap.add_argument("--mode", default="cached", choices=["cached", "snapshot", "uncached"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--uncached-steps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the launch-parameter search (use sort + deferral, 4-chunk runs)")
    ap.add_argument("--min-subgraph", type=int, default=0,
                    help="smallest cacheable sub-graph in nodes (compile option; 0 = library default 2)")
    ap.add_argument("--flags", type=int, default=-1,
                    help="with --no-autotune: pmc_flags bits (default sort, plus deferral cached)")
    ap.add_argument("--chunk-waves", type=int, default=0,
                    help="with --no-autotune: chunks per wave run (default 4 cached, 1 uncached)")
    ap.add_argument("--defer-max", type=int, default=0,
                    help="with --no-autotune: deferral threshold (default 48)")
    ap.add_argument("--waves-per-block", type=int, default=0,
                    help="with --no-autotune: waves per workgroup of the flat grid (default 4)")
    ap.add_argument("--late-frame", type=int, default=0,
                    help="with --no-autotune: frames from this one on use the --late-* setting")
    ap.add_argument("--late-flags", type=int, default=-1)
    ap.add_argument("--late-chunk-waves", type=int, default=0)
    ap.add_argument("--late-defer-max", type=int, default=0)
    ap.add_argument("--tune-json", default=None,
                    help="write every autotuner candidate and its time to this file")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate leg (training on the insert log)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)

    import torch
    from paper_2305_07238_amd import binding as B

    if args.calibrate_copy:
        n = 1 << 28                                    # 2^28 int32 = 1 GiB each way
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    sc, desc = workload(args.workload, args.frames or None)
    log(f"workload {args.workload}: {sc.frames} frames x {sc.hits_per_frame} hits")
    n_frame = sc.hits_per_frame
    n_step = n_frame * sc.frames
    hits = B.hits_to_device(scenes_concat(sc))
    frame_views = [{k: v[f * n_frame:(f + 1) * n_frame] for k, v in hits.items()}
                   for f in range(sc.frames)]
    out = B.alloc_outputs(n_frame)          # the renderer consumes each frame's BSDF inputs

    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials, min_subgraph_nodes=args.min_subgraph)
    cc = sc.cache
    policy = B.PMC_POLICY_OVERWRITE if cc.policy == "OVERWRITE" else B.PMC_POLICY_FIRST
    cache = ctx.cache(cc.n_cells, cc.n_entries, cc.entry_bytes, policy)
    mode = {"cached": B.PMC_MODE_CACHED, "snapshot": B.PMC_MODE_SNAPSHOT,
            "uncached": B.PMC_MODE_UNCACHED}[args.mode]
    use_cache = cache if mode != B.PMC_MODE_UNCACHED else None
    log("inputs resident; autotuning launch parameters on the first frames")

    tune_frames = min(4, sc.frames)
    if args.no_autotune:
        best = dict(flags=args.flags if args.flags >= 0 else
                    B.PMC_FLAG_SORT | (B.PMC_FLAG_DEFER if use_cache else 0),
                    chunk_waves=args.chunk_waves or (4 if use_cache else 1),
                    defer_max=args.defer_max or 48, blocks_per_cu=0,
                    waves_per_block=args.waves_per_block)
    else:
        tune = ctx.autotune(use_cache, ctx.frame_plan(hits, n_frame, tune_frames, out, mode=mode),
                            args.tune_json)
        b = tune.best
        best = dict(flags=b.flags, chunk_waves=b.chunk_waves, defer_max=b.defer_max,
                    blocks_per_cu=b.blocks_per_cu, waves_per_block=b.waves_per_block)
        log(f"autotune: {best} {tune.best_ms:.3f} ms vs defaults {tune.default_ms:.3f} ms "
            f"({tune.n_tried} settings, {tune_frames} frames)")
    # frames from late_frame on may use another setting: once the table holds
    # most values, chunks miss rarely and the best launch shape changes
    late_frame, late = 0, None
    if args.no_autotune:
        if args.late_frame:
            late_frame = args.late_frame
            late = dict(flags=args.late_flags if args.late_flags >= 0 else best["flags"],
                        chunk_waves=args.late_chunk_waves, defer_max=args.late_defer_max,
                        blocks_per_cu=0, waves_per_block=0)
    elif use_cache and sc.frames >= 2 * tune_frames:
        late_frame = tune_frames
        lt = ctx.autotune(use_cache, ctx.frame_plan(hits, n_frame, 2 * tune_frames, out,
                                                    mode=mode, late_frame=late_frame, **best),
                          args.tune_json + ".late" if args.tune_json else None)
        b = lt.best
        late = dict(flags=b.flags, chunk_waves=b.chunk_waves, defer_max=b.defer_max,
                    blocks_per_cu=b.blocks_per_cu, waves_per_block=b.waves_per_block)
        log(f"autotune, frames {late_frame}+: {late} ({lt.n_tried} settings, frames "
            f"{late_frame}..{2 * tune_frames - 1} after {late_frame} with the first setting)")
    graph = ctx.frame_graph(use_cache, ctx.frame_plan(hits, n_frame, sc.frames, out, mode=mode,
                                                      clear_cache=True, late_frame=late_frame,
                                                      late=late, **best))
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()

    # timed region: whole progressive renders, each from an empty table
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        graph.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"{ms_step:.3f} ms/step (graph replay)")
    graph.close()

    # the same work launched per frame with HIP-event phase timing on the stream
    def step(m=mode, stats=None):
        if m != B.PMC_MODE_UNCACHED:
            cache.clear()
        for f in range(sc.frames):
            kw = late if (late_frame and f >= late_frame) else best
            ctx.shade(frame_views[f], out, use_cache if m != B.PMC_MODE_UNCACHED else None,
                      mode=m, frame=f, stats=stats, **kw)

    prof_steps = 3
    ctx.profile_enable(True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    log(f"phases over {prof_steps} steps: {prof}")

    # one more step with counters (same work) for hit rate and algorithmic bytes
    stats = B.new_stats()
    step(stats=stats)
    torch.cuda.synchronize()
    st = B.stats_dict(stats)
    kb = kernel_bytes(st, n_step)
    shade_ms, shade_launches = prof["shade"]
    achieved = kb / (shade_ms / prof_steps * 1e-3) / 1e9

    # uncached reference on the same inputs, also replayed as a graph; the last
    # frame's BSDF inputs of both give the error of the cached values
    unc, err = None, None
    if mode != B.PMC_MODE_UNCACHED and args.uncached_steps > 0:
        cached_last = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        g_u = ctx.frame_graph(None, ctx.frame_plan(hits, n_frame, sc.frames, out,
                                                   mode=B.PMC_MODE_UNCACHED))
        g_u.launch()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.uncached_steps):
            g_u.launch()
        ev1.record()
        torch.cuda.synchronize()
        unc = ev0.elapsed_time(ev1) / args.uncached_steps
        log(f"uncached {unc:.3f} ms/step")
        g_u.close()
        e = np.concatenate([np.abs(out[k].cpu().numpy().astype(np.float64) - cached_last[k]).ravel()
                            for k in ("base_color", "roughness", "normal")])
        err = {"max_abs": float(e.max()), "mean_abs": float(e.mean()),
               "sample": "every BSDF input of the last frame, cached vs uncached GPU path"}

    value = n_step / (ms_step * 1e-3)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "hits_per_step": n_step, "frames": sc.frames,
                   "mode": args.mode, "launch": "one HIP graph per step (table clear + frames)",
                   "autotuned": best, "late_frame": late_frame, "autotuned_late": late},
        "cache_hit_rate": st["cache_hits"] / max(st["probes"], 1),
        "found_per_sample": st["cache_hits"] / max(st["hits_shaded"], 1),
        "deferred_fraction": st["deferred"] / max(st["hits_shaded"], 1),
        "nodes_executed_fraction": st["nodes_executed"] / max(st["nodes_total"], 1),
        "uncached_samples_per_s": (n_step / (unc * 1e-3)) if unc else None,
        "speedup_vs_uncached": (unc / ms_step) if unc else None,
        "bsdf_err_vs_uncached": err,
        "stats": st,
        "phase_ms_per_step": {k: v[0] / prof_steps for k, v in prof.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, best, late_frame, late),
                     "kernel": shade_kernel_name(args.mode, best["flags"]) + (
                         "" if not late_frame or shade_kernel_name(args.mode, late["flags"]) ==
                         shade_kernel_name(args.mode, best["flags"]) else
                         " (frames < %d), %s (later frames)" % (
                             late_frame, shade_kernel_name(args.mode, late["flags"]))),
                     "bytes_per_launch": kb / sc.frames,
                     "avg_launch_ms": shade_ms / max(shade_launches, 1)},
    }
    if not args.no_surrogate and use_cache and args.workload == "mid":
        res["surrogate"] = surrogate_leg(ctx, sc, frame_views, out, cache, best, log)
        res["surrogate_smooth"] = surrogate_smooth_leg(log)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
