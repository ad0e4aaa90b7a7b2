#!/usr/bin/env python3
"""Shading samples/s and cache hit rate of progressive material caching on one MI355X.

One step = one progressive render of the workload from an empty table: every
frame (one batch of hits, one sample per pixel) goes through material sort,
key computation, probes, the node interpreter on misses and lock-free inserts
(the paper's GPU update, Sec. 3.3), all frames replayed as one HIP graph.
Inputs are generated on the host, seeded, and resident in HBM before timing
starts.  The headline is the scale workload (4096 materials, 3840x2160 x 128
frames, 1 GiB overwrite table); the batching workload (1000 materials,
1920x1080 x 64 frames), the mid workload with the learned surrogate, and the
table-size and level-offset sweeps (Sec. 4) run as further legs.  Prints one
JSON line.
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

# algorithmic bytes of the shade kernel (per unit of the method's work)
B_HIT_IN = 40          # material 4, uv 8, duv 16, normal 12
B_HIT_OUT = 28         # base colour 12, roughness 4, normal 12
B_PERM = 4             # sorted index read
B_PROBE = 128          # one N_e x 16 B cell scanned per lookup
B_INSERT = 16          # one entry written per stored value
B_TEXEL = 16           # four RGBA8 texels per evaluated image-texture node
B_DEFER = B_HIT_IN + B_PERM   # a deferred hit's data read again for its dense pass


def kernel_bytes(st, n_hits):
    """Algorithmic bytes of the method in the shade kernel (all its launches):
    hit data in and out, the sorted index, one cell per lookup, one entry per
    value stored, four texels per image-texture evaluation."""
    return (n_hits * (B_HIT_IN + B_PERM + B_HIT_OUT) + st["probes"] * B_PROBE +
            (st["inserts"] + st["overwrites"]) * B_INSERT + st["texture_evals"] * B_TEXEL)


def overhead_bytes(st):
    """Bytes the implementation adds to the method's: lookups repeated for
    deferred hits, deferred hits' data read twice, insert attempts that stored
    nothing (lost races, full cells, keys already present)."""
    failed = max(st["insert_attempts"] - st["inserts"] - st["overwrites"], 0)
    return st["probes_deferred"] * B_PROBE + st["deferred"] * B_DEFER + failed * B_INSERT


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
        # the deferral threshold only matters with deferral on
        keys = ("flags", "chunk_waves", "defer_max") if want["flags"] & 4 else \
            ("flags", "chunk_waves")
        return (rec.get("waves_per_block", 4) == (want.get("waves_per_block", 0) or 4) and
                all(rec[k] == want[k] for k in keys))
    for rec in recs:
        if h.hexdigest() != rec["source_sha256"] or not same(rec, best):
            continue
        if rec.get("late_frame", 0) != late_frame:
            continue
        if late_frame and not same(rec["late"], late):
            continue
        return rec
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
                "Zipf(1.1) materials on 40-px objects, table 2^24 slots x 16 B, keep-first"
                % sc.frames)
    elif name == "scale":
        sc = scenes.scale_scene(frames=frames or 128)
        desc = ("scale: 4096 materials (lognormal sizes 8-400 nodes), 3840x2160 x %d frames, "
                "Zipf(1.1) materials on 40-px objects, table 2^26 slots x 16 B (1 GiB), "
                "overwrite-oldest" % sc.frames)
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------ CPU baseline ---

_CPU = {}          # scene and hits shared with forked workers


def _cpu_uncached_chunk(rows):
    from oracle import render
    sc, h = _CPU["scene"], _CPU["hits"]
    t0 = time.perf_counter()
    out = render.shade_uncached(sc.materials, sc.textures, h.take(rows))
    return rows, out, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, frame, n_parallel=1 << 19, n_single=65536, n_snapshot=8192,
                 workers=None):
    """The FP64 oracle timed on the host, on a bounded sample of the workload.
    Runs before the process touches the GPU (the worker pool forks).

    * uncached, one worker process per core (at most 16, the host share of one
      GPU): the first n_parallel hits of ``frame``;
    * uncached, one process: the first n_single hits of that frame;
    * snapshot-mode progressive shading (lookups, evaluation on misses,
      Algorithm 1 inserts into the full-size table), one process: the first
      n_snapshot hits of frames 0 and 1.
    Returns the cpu_baseline record and the FP64 outputs of the parallel sample
    (the reference for the GPU outputs of the same hits)."""
    import multiprocessing as mp
    from oracle import render, table
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    h = sc.frame(frame)
    n_parallel = min(n_parallel, len(h))
    _CPU["scene"], _CPU["hits"] = sc, h
    chunks = np.array_split(np.arange(n_parallel), workers * 4)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_cpu_uncached_chunk, chunks)
    t_par = time.perf_counter() - t0
    ref = dict(base_color=np.zeros((n_parallel, 3)), roughness=np.zeros(n_parallel),
               normal=np.zeros((n_parallel, 3)))
    for rows, out, _ in parts:
        for k in ref:
            ref[k][rows] = out[k]
    t0 = time.perf_counter()
    render.shade_uncached(sc.materials, sc.textures, h.take(np.arange(n_single)))
    t_single = time.perf_counter() - t0
    t = table.Table(sc.cache.n_cells, sc.cache.n_entries, sc.cache.entry_bytes)
    batches = [sc.frame(f).take(np.arange(n_snapshot)) for f in range(2)]
    t0 = time.perf_counter()
    res = render.shade_snapshot(sc.materials, sc.textures, batches, t,
                                policy=sc.cache.policy)
    t_snap = time.perf_counter() - t0
    probes = sum(r.stats["probes"] for r in res)
    hits = sum(r.stats["hits"] for r in res)
    rec = {"value": n_parallel / t_par, "unit": "samples/s", "cores": workers, "kind": "oracle",
           "cpu": cpu_model(), "mode": "uncached (FP64 graph evaluation)",
           "sample": f"first {n_parallel} hits (screen order) of frame {frame}, "
                     f"{workers} worker processes, {t_par:.1f} s wall",
           "single_process_uncached": {"value": n_single / t_single, "cores": 1,
                                       "sample": f"first {n_single} hits of frame {frame}, "
                                                 f"{t_single:.1f} s"},
           "single_process_snapshot": {"value": 2 * n_snapshot / t_snap, "cores": 1,
                                       "hit_rate": hits / max(probes, 1),
                                       "sample": f"first {n_snapshot} hits of frames 0-1, "
                                                 f"table {sc.cache.n_cells} x "
                                                 f"{sc.cache.n_entries}, {t_snap:.1f} s"}}
    _CPU.clear()
    return rec, ref


# --------------------------------------------------------------- GPU legs ---

def device_frames(sc, n_frames, first=0):
    """Hits of frames first .. first + n_frames - 1, frame-major, generated one
    frame at a time straight into device buffers."""
    import torch
    n = sc.hits_per_frame
    N = n * n_frames
    d = {"material": torch.empty(N, dtype=torch.int32, device="cuda"),
         "uv": torch.empty((N, 2), dtype=torch.float32, device="cuda"),
         "duv": torch.empty((N, 4), dtype=torch.float32, device="cuda"),
         "normal": torch.empty((N, 3), dtype=torch.float32, device="cuda")}
    for f in range(n_frames):
        h = sc.frame(first + f)
        s = slice(f * n, (f + 1) * n)
        d["material"][s].copy_(torch.from_numpy(np.ascontiguousarray(h.material).view(np.int32)))
        d["uv"][s].copy_(torch.from_numpy(h.uv))
        d["duv"][s].copy_(torch.from_numpy(h.duv))
        d["normal"][s].copy_(torch.from_numpy(h.normal))
    return d


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


def _abs_err(got, ref, rows=None):
    e = np.concatenate([np.abs(np.asarray(got[k], np.float64)[rows if rows is not None else
                                                              slice(None)] - ref[k]).ravel()
                        for k in ("base_color", "roughness", "normal")])
    return {"max_abs": float(e.max()), "mean_abs": float(e.mean())}


def tune_settings(ctx, cache, mode, sc, args, n_tune=4):
    """Launch settings from the autotuner, run on a warm-up scene (the same
    materials on another screen layout and jitter): one setting for the first
    n_tune frames, one for the later frames tuned on a table the first ones
    filled."""
    import torch
    from paper_2305_07238_amd import binding as B, scenes
    use_cache = cache if mode != B.PMC_MODE_UNCACHED else None
    if args.no_autotune:
        best = dict(flags=args.flags if args.flags >= 0 else
                    B.PMC_FLAG_SORT | (B.PMC_FLAG_DEFER if use_cache else 0),
                    chunk_waves=args.chunk_waves or (4 if use_cache else 1),
                    defer_max=args.defer_max or 48, blocks_per_cu=0,
                    waves_per_block=args.waves_per_block)
        late_frame, late = 0, None
        if args.late_frame:
            late_frame = args.late_frame
            late = dict(flags=args.late_flags if args.late_flags >= 0 else best["flags"],
                        chunk_waves=args.late_chunk_waves, defer_max=args.late_defer_max,
                        blocks_per_cu=0, waves_per_block=0)
        return best, late_frame, late, None
    warm = scenes.relayout(sc, seed=sc.seed + 1) if sc.layout is not None else sc
    n_frames = min(2 * n_tune, sc.frames)
    wh = device_frames(warm, n_frames)
    n = sc.hits_per_frame
    out = B.alloc_outputs(n)
    tune = ctx.autotune(use_cache, ctx.frame_plan(wh, n, min(n_tune, n_frames), out, mode=mode),
                        args.tune_json)
    b = tune.best
    best = dict(flags=b.flags, chunk_waves=b.chunk_waves, defer_max=b.defer_max,
                blocks_per_cu=b.blocks_per_cu, waves_per_block=b.waves_per_block)
    info = {"warmup_scene": warm.name, "early_ms": tune.best_ms, "default_ms": tune.default_ms,
            "tried": tune.n_tried}
    late_frame, late = 0, None
    if use_cache and sc.frames >= 2 * n_tune:
        late_frame = n_tune
        lt = ctx.autotune(use_cache, ctx.frame_plan(wh, n, 2 * n_tune, out, mode=mode,
                                                    late_frame=late_frame, **best),
                          args.tune_json + ".late" if args.tune_json else None)
        b = lt.best
        late = dict(flags=b.flags, chunk_waves=b.chunk_waves, defer_max=b.defer_max,
                    blocks_per_cu=b.blocks_per_cu, waves_per_block=b.waves_per_block)
        info["late_tried"] = lt.n_tried
    del wh
    torch.cuda.synchronize()
    return best, late_frame, late, info


def path_leg(name, sc, desc, args, steps, warmup, ref=None, ref_frame=None,
             uncached_steps=3, prof_steps=3):
    """Progressive renders of one workload: HIP-graph replays of all frames
    (timed), the same frames launched one by one with phase timing (the shade
    kernel's own launch time), one render with counters (hit rate, bytes), and
    the uncached path on the same inputs."""
    import torch
    from paper_2305_07238_amd import binding as B
    mode = {"cached": B.PMC_MODE_CACHED, "snapshot": B.PMC_MODE_SNAPSHOT,
            "uncached": B.PMC_MODE_UNCACHED}[args.mode]
    n_frame = sc.hits_per_frame
    n_step = n_frame * sc.frames
    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials, min_subgraph_nodes=args.min_subgraph)
    cc = sc.cache
    policy = {"FIRST": B.PMC_POLICY_FIRST, "OVERWRITE": B.PMC_POLICY_OVERWRITE,
              "PRIORITY": B.PMC_POLICY_PRIORITY}[cc.policy]
    cache = ctx.cache(cc.n_cells, cc.n_entries, cc.entry_bytes, policy)
    use_cache = cache if mode != B.PMC_MODE_UNCACHED else None
    best, late_frame, late, tune_info = tune_settings(ctx, cache, mode, sc, args)
    log(f"{name}: launch settings {best}, from frame {late_frame}: {late} ({tune_info})")
    t0 = time.perf_counter()
    hits = device_frames(sc, sc.frames)
    log(f"{name}: {sc.frames} frames x {n_frame} hits resident in HBM "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    out = B.alloc_outputs(n_frame)          # the renderer consumes each frame's BSDF inputs
    graph = ctx.frame_graph(use_cache, ctx.frame_plan(hits, n_frame, sc.frames, out, mode=mode,
                                                      clear_cache=True, late_frame=late_frame,
                                                      late=late, **best))
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        graph.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    log(f"{name}: {ms_step:.3f} ms/step (graph replay), {n_step / ms_step / 1e6:.3f} G samples/s")
    graph.close()
    # the same render with the statistics counters on (every shade launch counts,
    # and each frame ends with the reduction of its counters)
    st_g = B.new_stats()
    graph_s = ctx.frame_graph(use_cache, ctx.frame_plan(hits, n_frame, sc.frames, out, mode=mode,
                                                        clear_cache=True, stats=st_g,
                                                        late_frame=late_frame, late=late, **best))
    graph_s.launch()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        graph_s.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms_stats = ev0.elapsed_time(ev1) / steps
    graph_s.close()
    log(f"{name}: {ms_stats:.3f} ms/step with statistics")
    views = [{k: v[f * n_frame:(f + 1) * n_frame] for k, v in hits.items()}
             for f in range(sc.frames)]

    def step(stats=None):
        if mode != B.PMC_MODE_UNCACHED:
            cache.clear()
        for f in range(sc.frames):
            kw = late if (late_frame and f >= late_frame) else best
            ctx.shade(views[f], out, use_cache, mode=mode, frame=f, stats=stats, **kw)

    prof = None
    if prof_steps:
        ctx.profile_enable(True)
        for _ in range(prof_steps):
            step()
        torch.cuda.synchronize()
        prof = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
    stats = B.new_stats()
    step(stats=stats)
    torch.cuda.synchronize()
    st = B.stats_dict(stats)
    cached_last = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    res = {"workload": desc, "samples_per_s": n_step / (ms_step * 1e-3), "ms_per_step": ms_step,
           "ms_per_step_with_stats": ms_stats,
           "hits_per_step": n_step, "frames": sc.frames, "mode": args.mode,
           "launch": {"autotuned": best, "late_frame": late_frame, "autotuned_late": late,
                      "tuning": tune_info},
           "cache_hit_rate": st["cache_hits"] / max(st["probes"], 1),
           "found_per_sample": st["cache_hits"] / max(st["hits_shaded"], 1),
           "deferred_fraction": st["deferred"] / max(st["hits_shaded"], 1),
           "nodes_executed_fraction": st["nodes_executed"] / max(st["nodes_total"], 1),
           "stats": st}
    if prof:
        kb = kernel_bytes(st, n_step)
        ob = overhead_bytes(st)
        shade_ms, shade_launches = prof["shade"]
        avg_ms = shade_ms / max(shade_launches, 1)
        achieved = kb / (shade_ms / prof_steps * 1e-3) / 1e9
        trec = measured_traffic(name, best, late_frame, late)
        kname = shade_kernel_name(args.mode, best["flags"])
        if late_frame and shade_kernel_name(args.mode, late["flags"]) != kname:
            kname += " (frames < %d), %s (later frames)" % (
                late_frame, shade_kernel_name(args.mode, late["flags"]))
        res["phase_ms_per_step"] = {k: v[0] / prof_steps for k, v in prof.items()}
        res["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": trec["traffic_bytes_per_launch"] if trec else None,
            "kernel": kname, "bytes_per_launch": kb / sc.frames,
            "overhead_bytes_per_launch": ob / sc.frames,
            "avg_launch_ms": avg_ms, "launches_timed": shade_launches}
        if trec:
            res["roofline"]["traffic_source"] = trec.get("summary")
    # uncached path on the same inputs (also a graph); last-frame outputs of both
    if mode != B.PMC_MODE_UNCACHED and uncached_steps > 0:
        g_u = ctx.frame_graph(None, ctx.frame_plan(hits, n_frame, sc.frames, out,
                                                   mode=B.PMC_MODE_UNCACHED))
        g_u.launch()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(uncached_steps):
            g_u.launch()
        ev1.record()
        torch.cuda.synchronize()
        unc = ev0.elapsed_time(ev1) / uncached_steps
        g_u.close()
        unc_last = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        res["uncached_samples_per_s"] = n_step / (unc * 1e-3)
        res["uncached_ms_per_step"] = unc
        res["speedup_vs_uncached"] = unc / ms_step
        res["bsdf_err_vs_uncached_gpu"] = dict(
            _abs_err(cached_last, unc_last),
            sample="every BSDF input of the last frame, cached vs the uncached GPU path")
        log(f"{name}: uncached {unc:.3f} ms/step, speedup {unc / ms_step:.2f}x")
    if ref is not None and ref_frame == sc.frames - 1:
        rows = np.arange(len(ref["roughness"]))
        res["bsdf_err_vs_fp64_oracle"] = dict(
            _abs_err(cached_last, ref, rows),
            sample=f"first {len(rows)} hits of the last frame, cached GPU outputs vs the FP64 "
                   "oracle's plain evaluation (the CPU baseline's sample)")
    del views, hits
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def sweeps_leg(args, steps=3):
    """The paper's two experiments (Sec. 4) on the mid workload: table sizes
    N_c x N_e (16-byte entries) and the level offset (an integer bias on
    floor(lambda), finer texels for positive values).  Samples/s of the
    progressive render (one graph, 16 frames), hit rate, and the BSDF error of
    the last frame against the uncached GPU path (held within 1e-5 of the FP64
    graph by the parity tests)."""
    import torch
    from paper_2305_07238_amd import binding as B
    sc, _ = workload("mid")
    n = sc.hits_per_frame
    hits = device_frames(sc, sc.frames)
    out = B.alloc_outputs(n)
    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials)
    early = dict(flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, chunk_waves=4, defer_max=48)
    late = dict(flags=B.PMC_FLAG_SORT, chunk_waves=1, defer_max=0)
    g_u = ctx.frame_graph(None, ctx.frame_plan(hits, n, sc.frames, out,
                                               mode=B.PMC_MODE_UNCACHED))
    g_u.launch()
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    ms_u = _median_ms(lambda pre: None if pre else g_u.launch(), reps=steps)
    g_u.close()

    def point(n_cells, n_entries, bias):
        cache = ctx.cache(n_cells, n_entries, 16, level_bias=bias)
        st_t = B.new_stats()
        g = ctx.frame_graph(cache, ctx.frame_plan(hits, n, sc.frames, out, clear_cache=True,
                                                  late_frame=4, late=late, **early))
        g.launch()
        ms = _median_ms(lambda pre: None if pre else g.launch(), reps=steps)
        g.close()
        last = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        gs = ctx.frame_graph(cache, ctx.frame_plan(hits, n, sc.frames, out, clear_cache=True,
                                                   stats=st_t, late_frame=4, late=late, **early))
        gs.launch()
        torch.cuda.synchronize()
        gs.close()
        sd = B.stats_dict(st_t)
        cache.close()
        return dict(n_cells=n_cells, n_entries=n_entries, level_bias=bias,
                    table_mib=n_cells * n_entries * 16 / 2 ** 20,
                    samples_per_s=n * sc.frames / (ms * 1e-3), ms=ms,
                    hit_rate=sd["cache_hits"] / max(sd["probes"], 1),
                    found_per_sample=sd["cache_hits"] / max(sd["hits_shaded"], 1),
                    cell_full=sd["cell_full"], inserts=sd["inserts"],
                    speedup_vs_uncached=ms_u / ms, err_vs_uncached=_abs_err(last, ref))

    grid = []
    for n_entries in (4, 8, 16):
        for slots in (1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24):
            grid.append(point(slots // n_entries, n_entries, 0))
            log("sweep N_c x N_e: %d x %d: %.2f G samples/s, hit rate %.3f" % (
                slots // n_entries, n_entries, grid[-1]["samples_per_s"] / 1e9,
                grid[-1]["hit_rate"]))
    bias = []
    for b in (-1, 0, 1, 2, 3):
        bias.append(point((1 << 22) // 8, 8, b))
        log("sweep level bias %+d: %.2f G samples/s, hit rate %.3f, err max %.3g mean %.3g" % (
            b, bias[-1]["samples_per_s"] / 1e9, bias[-1]["hit_rate"],
            bias[-1]["err_vs_uncached"]["max_abs"], bias[-1]["err_vs_uncached"]["mean_abs"]))
    ctx.close()
    del hits
    torch.cuda.empty_cache()
    return {"workload": "mid (64 materials, 1920x1080 x 16 frames), keep-first",
            "uncached_samples_per_s": n * sc.frames / (ms_u * 1e-3),
            "table_size": grid, "level_bias": bias}


def cones_leg(args, n=3840 * 2160, reps=20):
    """Ray-cone footprints (Sec. 3.1) for one 3840x2160 frame of hits: the
    kernel reads 56 bytes per hit (direction, radius, triangle and UV edges)
    and writes the 16-byte gradients; HBM-bound elementwise work."""
    import torch
    from paper_2305_07238_amd import binding as B
    from paper_2305_07238_amd import scenes
    c = {k: torch.from_numpy(v).cuda() for k, v in scenes.cone_hits(0, n).items()}
    duv = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    ctx = B.Context(0)

    def run(pre):
        if not pre:
            for _ in range(reps):
                ctx.ray_cone_gradients(c, duv)
    ms = _median_ms(run) / reps
    gbs = n * 72 / (ms * 1e-3) / 1e9
    ctx.close()
    return {"hits": n, "ms": ms, "samples_per_s": n / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_hit": 72}}


def policies_leg(args, frames=8, n_cells=1 << 17):
    """Priority insertion (after Sec. 5: prefer directly visible samples when
    storage is short) on a path tracer's hits: each frame holds the mid
    workload's 2,073,600 camera hits (depth 0) and as many secondary hits
    (depth 1-3, footprints 2-16x wider), on a table of 2^17 cells x 8 entries
    (2^20 slots, far fewer than the render's keys), cached mode.  Per policy:
    the 8-frame render's samples/s, and the last frame's hit rates of the
    depth-0 and the deeper lookups."""
    import torch
    from paper_2305_07238_amd import binding as B
    from paper_2305_07238_amd import scenes
    sc, _ = workload("mid", frames)
    fr = [scenes.with_indirect(sc.frame(f), f) for f in range(frames)]
    bounce = fr[-1].bounce.astype(np.int64)
    dev = [B.hits_to_device(h) for h in fr]
    n = len(fr[0])
    out = B.alloc_outputs(n)
    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials)
    res = {"workload": "mid materials, %d frames x %d hits (camera + secondary), table "
                       "2^17 cells x 8 entries x 16 B" % (frames, n)}
    for name, pol in (("FIRST", B.PMC_POLICY_FIRST), ("OVERWRITE", B.PMC_POLICY_OVERWRITE),
                      ("PRIORITY", B.PMC_POLICY_PRIORITY)):
        cache = ctx.cache(n_cells, 8, 16, pol)

        def run(pre, cache=cache):
            if pre:
                cache.clear()
                torch.cuda.synchronize()
                return
            for f in range(frames):
                ctx.shade(dev[f], out, cache, mode=B.PMC_MODE_CACHED, frame=f,
                          flags=B.PMC_FLAG_SORT)
        ms = _median_ms(run)
        run(True)
        for f in range(frames - 1):
            ctx.shade(dev[f], out, cache, mode=B.PMC_MODE_CACHED, frame=f, flags=B.PMC_FLAG_SORT)
        state = torch.full((n, 8), 255, dtype=torch.uint8, device="cuda")
        st = B.new_stats()
        ctx.shade(dev[-1], out, cache, mode=B.PMC_MODE_CACHED, frame=frames - 1,
                  flags=B.PMC_FLAG_SORT, stats=st, debug={"state": state})
        torch.cuda.synchronize()
        s_np = state.cpu().numpy()
        probed = (s_np == 0) | (s_np == 1)
        found = s_np == 1
        d0 = bounce == 0
        res[name] = {"samples_per_s": n * frames / (ms * 1e-3), "ms": ms,
                     "hit_rate_depth0": float(found[d0].sum() / max(probed[d0].sum(), 1)),
                     "hit_rate_deeper": float(found[~d0].sum() / max(probed[~d0].sum(), 1)),
                     "overwrites_last_frame": int(B.stats_dict(st)["overwrites"])}
        log(f"policies: {name} {res[name]}")
        cache.close()
    ctx.close()
    return res


def spatial_leg(args, frames=16):
    """World-position descriptors (Sec. 3.1's other shading-point information):
    the mid material mix with 35% of its UV leaves replaced by 3D value noise of
    the world position, 1920x1080 x 16 frames of hits on planar patches in the
    world carrying position and footprint width, table 2^24 slots.  Uncached;
    cached with texel descriptors only (outputs of the world position are then
    always evaluated); cached with world-cell descriptors as well.  Samples/s,
    hit rate, interpreter work, the share of lookups keyed by world cells, and
    the last frame's error against the uncached path."""
    import torch
    from paper_2305_07238_amd import binding as B
    from paper_2305_07238_amd import scenes
    sc = scenes.spatial_scene(width=1920, height=1080, frames=frames, slots=1 << 24)
    fr = [sc.frame(f) for f in range(frames)]
    dev = [B.hits_to_device(h) for h in fr]
    n = len(fr[0])
    out = B.alloc_outputs(n)
    res = {"workload": "spatial: 64 materials (35%% of UV leaves -> world-position noise), "
                       "1920x1080 x %d frames, table 2^24 slots x 16 B" % frames}
    outs = {}
    cnt = np.bincount(fr[-1].material, minlength=len(sc.materials))
    for name, texel_only, cached in (("uncached", False, False), ("texel_keys", True, True),
                                     ("world_cells", False, True)):
        ctx = B.Context(0)
        ctx.set_textures(sc.textures)
        ctx.compile(sc.materials, texel_keys_only=texel_only)
        cache = ctx.cache(sc.cache.n_cells, 8, 16) if cached else None
        mode = B.PMC_MODE_CACHED if cached else B.PMC_MODE_UNCACHED

        def run(pre, cache=cache, ctx=ctx, mode=mode):
            if pre:
                if cache is not None:
                    cache.clear()
                torch.cuda.synchronize()
                return
            for f in range(frames):
                ctx.shade(dev[f], out, cache, mode=mode, frame=f, flags=B.PMC_FLAG_SORT)
        ms = _median_ms(run)
        outs[name] = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        r = {"samples_per_s": n * frames / (ms * 1e-3), "ms": ms}
        if cached:
            st = B.new_stats()
            run(True)
            for f in range(frames):
                ctx.shade(dev[f], out, cache, mode=mode, frame=f, flags=B.PMC_FLAG_SORT, stats=st)
            torch.cuda.synchronize()
            sd = B.stats_dict(st)
            infos = [ctx.material_info(m) for m in range(len(sc.materials))]
            cell = np.array([sum(i.cacheable_key[c] for c in range(i.n_cacheable)) for i in infos])
            allk = np.array([i.n_cacheable for i in infos])
            r.update(cache_hit_rate=sd["cache_hits"] / max(sd["probes"], 1),
                     nodes_executed_fraction=sd["nodes_executed"] / max(sd["nodes_total"], 1),
                     world_cell_share_of_lookups=float((cnt * cell).sum() /
                                                       max((cnt * allk).sum(), 1)))
        res[name] = r
        ctx.close()
    for name in ("texel_keys", "world_cells"):
        res[name]["speedup_vs_uncached"] = res["uncached"]["ms"] / res[name]["ms"]
        res[name]["err_vs_uncached"] = _abs_err(outs[name], outs["uncached"])
    res["world_cells_vs_texel_keys"] = res["texel_keys"]["ms"] / res["world_cells"]["ms"]
    log(f"spatial: {res}")
    return res


SURR_FLOP_PER_POINT = 2 * (32 * 64 + 64 * 64 + 64 * 4)     # 12,800 per network evaluation
FP16_PEAK_TFLOPS = 2500.0
TRAIN = dict(steps=8000, batch=1024, lr=2e-2, lr_end=1e-5, seed=0)
LOG_TARGET = (1 << 20) - 64 * 64       # the log's 2^20 records, less a partly filled row of regions


def surrogate_leg(args):
    """Learned surrogate on the mid workload: a progressive render (16 frames,
    cached mode, insert log on) collects training pairs, topped up to the log's
    2^20 records by the first frames of the same materials on other layouts;
    every network is trained (one launch) and trusted by its own held-out
    error; then the next
    pass (its first 2^20 hits) is shaded from the render's final table:
    uncached, cache only, and networks + cache.  Errors of every output
    against the uncached GPU path (held within 1e-5 of the FP64 graph by the
    parity tests)."""
    import torch
    from paper_2305_07238_amd import binding as B
    from paper_2305_07238_amd import scenes
    sc, _ = workload("mid")
    n = sc.hits_per_frame
    hits = device_frames(sc, sc.frames)
    views = [{k: v[f * n:(f + 1) * n] for k, v in hits.items()} for f in range(sc.frames)]
    out = B.alloc_outputs(n)
    ctx = B.Context(0)
    ctx.set_textures(sc.textures)
    ctx.compile(sc.materials)
    cache = ctx.cache(sc.cache.n_cells, 8, 16)
    n_slots = ctx.surrogate_setup(seed=0)
    kw = dict(flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, chunk_waves=4, defer_max=48)
    ctx.log_clear()
    for f in range(sc.frames):
        k = dict(kw) if f < 4 else dict(flags=B.PMC_FLAG_SORT, chunk_waves=1, defer_max=0)
        k["flags"] |= B.PMC_FLAG_LOG
        ctx.shade(views[f], out, cache, mode=B.PMC_MODE_CACHED, frame=f, **k)
    torch.cuda.synchronize()
    table = cache.export()
    n_log_render = n_log = len(ctx.log_read())
    # more training pairs, up to the log's 2^20 records: the first frames of the
    # same materials on other screen layouts, each from an empty table
    extra_frames = 0
    for seed in range(1, 4):
        if n_log >= LOG_TARGET:
            break
        sc2 = scenes.relayout(sc, seed)
        cache.clear()
        for f in range(4):
            h2 = B.hits_to_device(sc2.frame(f))
            ctx.shade(h2, out, cache, mode=B.PMC_MODE_CACHED, frame=f,
                      flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER | B.PMC_FLAG_LOG,
                      chunk_waves=4, defer_max=48)
            extra_frames += 1
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
    n17 = min(1 << 20, n)
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
                      frame=sc.frames, flags=B.PMC_FLAG_SORT | f)
        ms = _median_ms(run)
        got = {k: v.cpu().numpy().astype(np.float64) for k, v in o17.items()}
        results[name] = {"samples_per_s": n17 / (ms * 1e-3), "ms": ms, "_out": got}
    ref = results["uncached"]["_out"]
    for r in results.values():
        r["err_vs_uncached"] = _abs_err(r["_out"], ref)
    for r in results.values():
        del r["_out"]
    uv = d17["uv"]
    y = torch.empty((n17, 4), dtype=torch.float32, device="cuda")
    reps = 20

    def infer_batch(pre):
        if not pre:
            for _ in range(reps):
                ctx.surrogate_infer(0, uv, y)
    ms_inf = _median_ms(infer_batch) / reps
    inf_tflops = SURR_FLOP_PER_POINT * n17 / (ms_inf * 1e-3) / 1e12
    res = {
        "workload": "mid after its 16-frame render; next pass, first 2^20 hits",
        "slots": n_slots, "trusted": len(trusted),
        "trusted_materials": [int(rep[k]["material"]) for k in trusted], "log_records": n_log,
        "log_records_render": n_log_render, "log_extra_frames": extra_frames,
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
    ctx.close()
    del hits, views
    torch.cuda.empty_cache()
    return res


def surrogate_smooth_leg(args):
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
    ref = results["uncached"]["_out"]
    for r in results.values():
        r["err_vs_uncached"] = _abs_err(r["_out"], ref)
    for r in results.values():
        del r["_out"]
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


LEGS = ("batching", "mid", "surrogate", "sweeps", "cones", "policies", "spatial")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scale",
                    help="headline workload: scale (default), batching, mid or tiny")
    ap.add_argument("--frames", type=int, default=0)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="further legs, comma separated (%s) or 'none'" % ", ".join(LEGS))
    ap.add_argument("--mode", default="cached", choices=["cached", "snapshot", "uncached"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--uncached-steps", type=int, default=3)
    ap.add_argument("--prof-steps", type=int, default=3,
                    help="renders launched frame by frame with HIP-event phase timing")
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
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the path is shown on "
                                   "one GPU's share of the work); --gpus must be 1",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    for leg in legs:
        if leg not in LEGS:
            raise SystemExit(f"unknown leg {leg}")

    if args.calibrate_copy:
        import torch
        n = 1 << 28                                    # 2^28 int32 = 1 GiB each way
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    sc, desc = workload(args.workload, args.frames or None)
    log(f"workload {args.workload}: {sc.frames} frames x {sc.hits_per_frame} hits")
    cpu, ref, ref_frame = None, None, None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the oracle's worker pool forks
        ref_frame = sc.frames - 1
        log("timing the CPU oracle on a bounded sample")
        cpu, ref = cpu_baseline(sc, ref_frame)
        log(f"CPU oracle: {cpu['value']:.0f} samples/s on {cpu['cores']} cores")

    import torch  # noqa: F401
    from paper_2305_07238_amd import binding as B  # noqa: F401  (fails loudly if not built)

    head = path_leg(args.workload, sc, desc, args, args.steps, args.warmup, ref, ref_frame,
                    args.uncached_steps, args.prof_steps)
    del sc
    out_legs = {}
    for leg in legs:
        t0 = time.perf_counter()
        if leg in ("batching", "mid") and leg != args.workload:
            lsc, ldesc = workload(leg)
            out_legs[leg] = path_leg(leg, lsc, ldesc, args, 3, 1, None, None, 2, 2)
            del lsc
        elif leg == "surrogate":
            out_legs["surrogate"] = surrogate_leg(args)
            out_legs["surrogate_smooth"] = surrogate_smooth_leg(args)
        elif leg == "sweeps":
            out_legs["sweeps"] = sweeps_leg(args)
        elif leg == "cones":
            out_legs["cones"] = cones_leg(args)
        elif leg == "policies":
            out_legs["policies"] = policies_leg(args)
        elif leg == "spatial":
            out_legs["spatial"] = spatial_leg(args)
        log(f"leg {leg}: {time.perf_counter() - t0:.0f} s")

    res = {
        "metric": METRIC,
        "value": head["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "hits_per_step": head["hits_per_step"],
                   "frames": head["frames"], "mode": args.mode,
                   "launch": "one HIP graph per step (table clear + every frame)",
                   **head["launch"]},
    }
    for k in ("ms_per_step_with_stats", "cache_hit_rate", "found_per_sample", "deferred_fraction",
              "nodes_executed_fraction", "uncached_samples_per_s", "speedup_vs_uncached",
              "bsdf_err_vs_fp64_oracle", "bsdf_err_vs_uncached_gpu", "stats",
              "phase_ms_per_step", "roofline"):
        if k in head:
            res[k] = head[k]
    res["legs"] = out_legs
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
