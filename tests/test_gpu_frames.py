"""Progressive frames captured in a HIP graph, and the autotuner, against
stream launches and the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import render, table
from paper_2305_07238_amd import scenes
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2305_07238_amd import binding as B  # noqa: E402


def _frames_on_device(sc, n_frames):
    return B.hits_to_device(scenes.Hits.concat([sc.frame(f) for f in range(n_frames)]))


def _slice(d, f, n):
    return {k: v[f * n:(f + 1) * n] for k, v in d.items()}


# 3 frames: groups {0}, {1, 2}; 11 frames: {0}, {1..4}, {5..8}, {9, 10}, so frames
# 8..10 reuse the workspace sets of frames 0..2 and the sorts wait for shading
# late: frames from 5 on use another setting (another kernel variant; with
# unsorted late frames the sorts do not run on their own stream)
@pytest.mark.parametrize("mode,F,late", [
    (B.PMC_MODE_SNAPSHOT, 3, None), (B.PMC_MODE_UNCACHED, 3, None),
    (B.PMC_MODE_SNAPSHOT, 11, None),
    (B.PMC_MODE_SNAPSHOT, 11, dict(flags=B.PMC_FLAG_SORT, chunk_waves=1)),
    (B.PMC_MODE_SNAPSHOT, 7, dict(flags=0, chunk_waves=2))])
def test_frame_graph_replays_match_stream_launches(mode, F, late):
    """A captured render (sorts pipelined on a second stream) equals the same
    frames launched one by one, bit for bit, on every replay."""
    sc = G.small_mid_scene(frames=F)
    ctx = G.setup(sc)
    n = sc.hits_per_frame
    hits = _frames_on_device(sc, F)
    out_g = B.alloc_outputs(n * F)
    out_s = B.alloc_outputs(n * F)
    cache_g, cache_s = ctx.cache(1 << 13), ctx.cache(1 << 13)
    stats_g = B.new_stats()
    plan = ctx.frame_plan(hits, n, F, out_g, mode=mode, out_per_frame=True, clear_cache=True,
                          stats=stats_g, flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER,
                          late_frame=5 if late else 0, late=late)
    graph = ctx.frame_graph(cache_g if mode != B.PMC_MODE_UNCACHED else None, plan)
    # eager reference
    stats_s = B.new_stats()
    for f in range(F):
        kw = late if (late and f >= 5) else dict(flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER)
        ctx.shade(_slice(hits, f, n), _slice(out_s, f, n), cache_s if mode else None, mode=mode,
                  frame=f, stats=stats_s, **kw)
    torch.cuda.synchronize()
    ref = G.to_numpy(out_s)
    ref_table = cache_s.export()
    st_ref = B.stats_dict(stats_s)
    for rep in range(3):
        stats_g.zero_()
        for v in out_g.values():
            v.fill_(-1.0)
        graph.launch()
        torch.cuda.synchronize()
        got = G.to_numpy(out_g)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (rep, k)
        if mode != B.PMC_MODE_UNCACHED:
            assert np.array_equal(cache_g.export(), ref_table), rep
        st = B.stats_dict(stats_g)
        for k in ("hits_shaded", "probes", "cache_hits", "inserts", "present", "cell_full",
                  "nodes_total"):
            assert st[k] == st_ref[k], (rep, k)
        # eager work between replays
        ctx.shade(_slice(hits, 0, n), _slice(out_s, 0, n), None, mode=B.PMC_MODE_UNCACHED)
        torch.cuda.synchronize()


def test_frame_graph_tiny_snapshot_matches_oracle():
    sc = scenes.tiny_scene()
    ctx = G.setup(sc)
    n, F = sc.hits_per_frame, 4
    hits = _frames_on_device(sc, F)
    out = B.alloc_outputs(n)                            # every frame writes the same buffer
    cache = ctx.cache(sc.cache.n_cells)
    stats = B.new_stats()
    graph = ctx.frame_graph(cache, ctx.frame_plan(hits, n, F, out, mode=B.PMC_MODE_SNAPSHOT,
                                                  stats=stats))
    graph.launch()
    torch.cuda.synchronize()
    ref_t = table.Table(sc.cache.n_cells, 8, 16)
    res = render.shade_snapshot(sc.materials, sc.textures, [sc.frame(f) for f in range(F)], ref_t)
    assert B.stats_dict(stats)["cache_hits"] == sum(r.stats["hits"] for r in res) == 24576
    w = cache.words()
    assert np.array_equal(w[:, 0] >> np.uint64(32), ref_t.words() >> np.uint64(32))
    assert np.array_equal((w[:, 1] & np.uint64(0xFFFFFFFF)).astype(np.uint32), ref_t.stamps())


def test_autotune_picks_a_valid_setting(tmp_path):
    sc = G.small_mid_scene(frames=2)
    ctx = G.setup(sc)
    n, F = sc.hits_per_frame, 2
    hits = _frames_on_device(sc, F)
    out = B.alloc_outputs(n)
    cache = ctx.cache(1 << 13)
    plan = ctx.frame_plan(hits, n, F, out, mode=B.PMC_MODE_SNAPSHOT)
    path = str(tmp_path / "tune.json")
    res = ctx.autotune(cache, plan, path)
    assert res.n_tried >= 10 and res.best_ms > 0 and res.best_ms <= res.default_ms * 1.5
    rec = json.load(open(path))
    assert len(rec["candidates"]) == res.n_tried
    assert np.count_nonzero(cache.export()) == 0          # left cleared
    # the chosen setting gives the same snapshot results as the defaults
    b = res.best
    out2 = B.alloc_outputs(n)
    cache2 = ctx.cache(1 << 13)
    for f in range(F):
        h = _slice(hits, f, n)
        ctx.shade(h, out, cache, mode=B.PMC_MODE_SNAPSHOT, frame=f)
        ctx.shade(h, out2, cache2, mode=B.PMC_MODE_SNAPSHOT, frame=f, flags=b.flags,
                  chunk_waves=b.chunk_waves, defer_max=b.defer_max, blocks_per_cu=b.blocks_per_cu,
                  waves_per_block=b.waves_per_block)
    torch.cuda.synchronize()
    assert np.array_equal(cache.export(), cache2.export())
    for k in out:
        assert torch.equal(out[k], out2[k])


def test_frame_graph_keeps_what_it_uses():
    """While a graph exists the context refuses to change what the graph replays
    (program, textures, surrogate slots) or to replace a workspace buffer (a batch
    larger than any reserved); destroying the table it replays into is deferred,
    so a later replay still gives the same results; destroying the graph lifts
    both."""
    sc = G.small_mid_scene(frames=2)
    ctx = G.setup(sc)
    n, F = sc.hits_per_frame, 2
    hits = _frames_on_device(sc, F)
    out = B.alloc_outputs(n)
    cache = ctx.cache(1 << 13)
    graph = ctx.frame_graph(cache, ctx.frame_plan(hits, n, F, out, mode=B.PMC_MODE_SNAPSHOT,
                                                  clear_cache=True))
    graph.launch()
    torch.cuda.synchronize()
    first = G.to_numpy(out)
    for call in (lambda: ctx.compile(sc.materials), lambda: ctx.set_textures(sc.textures),
                 lambda: ctx.surrogate_setup(seed=0)):
        with pytest.raises(B.PmcError) as e:
            call()
        assert e.value.code == B.PMC_ERR_STATE
    out_big = B.alloc_outputs(n * F)
    with pytest.raises(B.PmcError) as e:
        ctx.shade(hits, out_big, cache, mode=B.PMC_MODE_SNAPSHOT)
    assert e.value.code == B.PMC_ERR_STATE
    # within the reservation, eager calls still run
    ctx.shade(_slice(hits, 0, n), _slice(out_big, 0, n), None, mode=B.PMC_MODE_UNCACHED)
    torch.cuda.synchronize()
    cache.close()
    for v in out.values():
        v.fill_(-1.0)
    graph.launch()
    torch.cuda.synchronize()
    got = G.to_numpy(out)
    for k in first:
        assert np.array_equal(got[k], first[k]), k
    graph.close()
    ctx.compile(sc.materials)
    ctx.shade(hits, out_big, None, mode=B.PMC_MODE_UNCACHED)
    torch.cuda.synchronize()


def test_autotune_of_the_late_frames():
    """With late_frame set the candidates replace the late setting only; the pick is
    valid and the table is left cleared."""
    sc = G.small_mid_scene(frames=4)
    ctx = G.setup(sc)
    n, F = sc.hits_per_frame, 4
    hits = _frames_on_device(sc, F)
    out = B.alloc_outputs(n)
    cache = ctx.cache(1 << 13)
    plan = ctx.frame_plan(hits, n, F, out, mode=B.PMC_MODE_CACHED, late_frame=2,
                          flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, chunk_waves=4)
    res = ctx.autotune(cache, plan)
    assert res.n_tried >= 10 and 0 < res.best_ms <= res.default_ms * 1.5
    assert res.best.flags & B.PMC_FLAG_SORT
    assert np.count_nonzero(cache.export()) == 0
    bad = ctx.frame_plan(hits, n, F, out, mode=B.PMC_MODE_CACHED, late_frame=F)
    with pytest.raises(B.PmcError):
        ctx.autotune(cache, bad)


def test_frame_graph_carries_path_depths():
    """PRIORITY over frames of camera and secondary hits: a captured snapshot
    render (each frame's path depths taken at the frame's offset) equals the
    frames launched one by one, bit for bit."""
    F = 3
    sc = G.small_mid_scene(frames=F)
    ctx = G.setup(sc)
    fr = [scenes.with_indirect(sc.frame(f), f) for f in range(F)]
    n = len(fr[0])
    hits = B.hits_to_device(scenes.Hits.concat(fr))
    assert "bounce" in hits
    out_g, out_s = B.alloc_outputs(n * F), B.alloc_outputs(n * F)
    cache_g = ctx.cache(1 << 12, 8, 16, B.PMC_POLICY_PRIORITY)
    cache_s = ctx.cache(1 << 12, 8, 16, B.PMC_POLICY_PRIORITY)
    plan = ctx.frame_plan(hits, n, F, out_g, mode=B.PMC_MODE_SNAPSHOT, out_per_frame=True,
                          clear_cache=True, flags=B.PMC_FLAG_SORT)
    graph = ctx.frame_graph(cache_g, plan)
    st = B.new_stats()
    for f in range(F):
        ctx.shade(_slice(hits, f, n), _slice(out_s, f, n), cache_s, mode=B.PMC_MODE_SNAPSHOT,
                  frame=f, flags=B.PMC_FLAG_SORT, stats=st)
    torch.cuda.synchronize()
    assert B.stats_dict(st)["overwrites"] > 0          # the table overflows: depths decide
    ref = G.to_numpy(out_s)
    ref_table = cache_s.export()
    graph.launch()
    torch.cuda.synchronize()
    got = G.to_numpy(out_g)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(cache_g.export(), ref_table)
    graph.close()
