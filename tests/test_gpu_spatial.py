"""GPU parity of world-position descriptors: graphs with POSITION_NOISE leaves
(3D value noise of the hit's world position), whose position-only outputs the
table keys by a world-space cell instead of a UV texel (the paper's descriptor
may use other shading-point information than UV, Sec. 3.1).

Keys bit-exact with the oracle's (texel and cell keys alike); uncached outputs
at the value bar; a snapshot-mode progressive render with hit pattern, table
and found values matching the oracle."""
import numpy as np
import pytest

from oracle import graph, keys as K, render, table
from paper_2305_07238_amd import scenes
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2305_07238_amd import binding as B  # noqa: E402


def _scene(frames=2):
    return scenes.spatial_scene(frames=frames)


def test_spatial_keys_bit_exact():
    sc = _scene(1)
    h = sc.frame(0)
    n_cells = 99991
    ctx = G.setup(sc)
    cache = ctx.cache(n_cells)
    out = torch.zeros(len(h) * 8 * 6, dtype=torch.int32, device="cuda")
    ctx.debug_keys(cache, B.hits_to_device(h), out)
    torch.cuda.synchronize()
    rec = out.cpu().numpy().view(B.KEY_RECORD_DTYPE).reshape(len(h), 8)
    mat = h.material.astype(np.int64)
    n_cell_keys = 0
    for m in np.unique(mat):
        idx = np.nonzero(mat == m)[0]
        for c, (node, sock) in enumerate(graph.cacheable_outputs(sc.materials[m])):
            ky = K.keys_for(sc.materials[m], int(m), node, sock, h, idx, n_cells)
            r = rec[idx, c]
            assert np.array_equal(r["bypass"].astype(bool), ky.bypass), (m, c)
            ok = ~ky.bypass
            for f in ("cell", "hash2", "level", "tx", "ty"):
                assert np.array_equal(r[f][ok], getattr(ky, f)[ok].astype(r[f].dtype)), (m, c, f)
            if graph.key_kind(sc.materials[m], node) == graph.POS:
                n_cell_keys += int(ok.sum())
    assert n_cell_keys > len(h) // 10


def test_spatial_uncached_matches_oracle():
    sc = _scene(1)
    ctx = G.setup(sc)
    h = sc.frame(0)
    ref = render.shade_uncached(sc.materials, sc.textures, h)
    for flags in (0, B.PMC_FLAG_SORT):
        out, _, _, st = G.shade(ctx, h, None, mode=B.PMC_MODE_UNCACHED, flags=flags)
        errs = G.assert_outputs(out, ref)
        print("spatial uncached error / bar", flags, errs)
        assert st["hits_shaded"] == len(h)


def test_spatial_snapshot_two_frames_match_oracle():
    sc = _scene(2)
    ctx = G.setup(sc)
    n_cells = 1 << 16
    cache = ctx.cache(n_cells, 8, 16)
    ref_t = table.Table(n_cells, 8, 16)
    for f in range(2):
        h = sc.frame(f)
        ref = render.shade_snapshot_frame(sc.materials, sc.textures, h, ref_t, f)
        out, state, value, st = G.shade(ctx, h, cache, mode=B.PMC_MODE_SNAPSHOT, frame=f,
                                        flags=B.PMC_FLAG_SORT, debug=True)
        assert np.array_equal(state == 1, ref.found)
        assert np.array_equal(state == 2, ref.bypass & ref.valid)
        G.found_values_parity(sc.materials, h, state, value, ref.found_value)
        o = G.substituted_outputs(sc.materials, sc.textures, h, state, value)
        G.assert_outputs(out, o)
        assert st["cache_hits"] == ref.stats["hits"]
        assert st["inserts"] == ref.stats.get("inserted", 0)
        G.table_parity(cache.words(), ref_t, sc.materials)
    assert st["cache_hits"] > 0


def test_spatial_cached_outputs_within_the_bar_of_substitution():
    """Racing (cached) mode: whatever the device found, the outputs equal the FP64
    graph with those values substituted."""
    sc = _scene(2)
    ctx = G.setup(sc)
    cache = ctx.cache(sc.cache.n_cells)
    for f in range(2):
        h = sc.frame(f)
        out, state, value, st = G.shade(ctx, h, cache, mode=B.PMC_MODE_CACHED, frame=f,
                                        flags=B.PMC_FLAG_SORT, debug=True)
        o = G.substituted_outputs(sc.materials, sc.textures, h, state, value)
        G.assert_outputs(out, o)
    assert st["cache_hits"] > 0


def test_position_required_when_the_graphs_read_it():
    sc = _scene(1)
    ctx = G.setup(sc)
    h = sc.frame(0)
    d = B.hits_to_device(h)
    d.pop("width")
    out = B.alloc_outputs(len(h))
    with pytest.raises(B.PmcError) as e:
        ctx.shade(d, out, None, mode=B.PMC_MODE_UNCACHED)
    assert e.value.code == B.PMC_ERR_INVALID
    d.pop("position")
    with pytest.raises(B.PmcError) as e:
        ctx.shade(d, out, None, mode=B.PMC_MODE_UNCACHED)
    assert "world position" in str(e.value)


def test_texel_keys_only_snapshot_matches_oracle():
    """Descriptors restricted to UV texels (the comparison the benchmark draws):
    the compiler's cacheable outputs equal the oracle's texel-only ones, and a
    two-frame snapshot render matches the oracle with those outputs."""
    sc = _scene(2)
    ctx = G.setup(sc, texel_keys_only=True)
    cach = [graph.cacheable_outputs(m, texel_only=True) for m in sc.materials]
    for mi in range(len(sc.materials)):
        assert ctx.cacheables(mi) == cach[mi], mi
    n_cells = 1 << 16
    cache = ctx.cache(n_cells, 8, 16)
    ref_t = table.Table(n_cells, 8, 16)
    for f in range(2):
        h = sc.frame(f)
        ref = render.shade_snapshot_frame(sc.materials, sc.textures, h, ref_t, f, cacheables=cach)
        out, state, value, st = G.shade(ctx, h, cache, mode=B.PMC_MODE_SNAPSHOT, frame=f,
                                        flags=B.PMC_FLAG_SORT, debug=True)
        assert np.array_equal(state == 1, ref.found)
        assert np.array_equal(state == 2, ref.bypass & ref.valid)
        G.found_values_parity(sc.materials, h, state, value, ref.found_value, cacheables=cach)
        o = G.substituted_outputs(sc.materials, sc.textures, h, state, value, cacheables=cach)
        G.assert_outputs(out, o)
        assert st["cache_hits"] == ref.stats["hits"]
        assert st["inserts"] == ref.stats.get("inserted", 0)
        G.table_parity(cache.words(), ref_t, sc.materials)
    assert st["cache_hits"] > 0


def test_frame_graph_carries_positions():
    """A captured snapshot render of the spatial scene (each frame's positions
    and widths taken at the frame's offset) equals the frames launched one by
    one, bit for bit, on two replays."""
    F = 3
    sc = _scene(F)
    ctx = G.setup(sc)
    n = sc.hits_per_frame
    hits = B.hits_to_device(scenes.Hits.concat([sc.frame(f) for f in range(F)]))
    assert "position" in hits and "width" in hits
    out_g, out_s = B.alloc_outputs(n * F), B.alloc_outputs(n * F)
    cache_g, cache_s = ctx.cache(1 << 14), ctx.cache(1 << 14)
    plan = ctx.frame_plan(hits, n, F, out_g, mode=B.PMC_MODE_SNAPSHOT, out_per_frame=True,
                          clear_cache=True, flags=B.PMC_FLAG_SORT)
    graph = ctx.frame_graph(cache_g, plan)
    for f in range(F):
        sl = {k: v[f * n:(f + 1) * n] for k, v in hits.items()}
        ctx.shade(sl, {k: v[f * n:(f + 1) * n] for k, v in out_s.items()}, cache_s,
                  mode=B.PMC_MODE_SNAPSHOT, frame=f, flags=B.PMC_FLAG_SORT)
    torch.cuda.synchronize()
    ref = G.to_numpy(out_s)
    ref_table = cache_s.export()
    for rep in range(2):
        for v in out_g.values():
            v.fill_(-1.0)
        graph.launch()
        torch.cuda.synchronize()
        got = G.to_numpy(out_g)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (rep, k)
        assert np.array_equal(cache_g.export(), ref_table), rep
    graph.close()


def test_surrogates_beside_world_keys():
    """Networks (untrained, trusted by a huge threshold) on graphs that also
    hold world-keyed outputs: no network stands for a world-keyed output (they
    read UV only), and in racing mode every output equals the FP64 graph with
    the device's found and network values substituted."""
    sc = _scene(2)
    ctx = G.setup(sc)
    n_slots = ctx.surrogate_setup(min_subgraph_nodes=4, seed=3, max_err=1e6)
    assert n_slots > 0
    for k in range(n_slots):
        sl = ctx.surrogate_slot(k)
        info = ctx.material_info(sl["material"])
        assert all(info.cacheable_key[c] == 0 for c in range(8) if (sl["ordinal_mask"] >> c) & 1)
        ctx.surrogate_set_trust(k, True)
    cache = ctx.cache(1 << 16, 8, 16)
    used = 0
    for f in range(2):
        h = sc.frame(f)
        out, state, value, st = G.shade(ctx, h, cache, mode=B.PMC_MODE_CACHED, frame=f,
                                        flags=B.PMC_FLAG_SORT | B.PMC_FLAG_SURROGATE, debug=True)
        o = G.substituted_outputs(sc.materials, sc.textures, h, state, value, states=(1, 4))
        G.assert_outputs(out, o)
        used += st["surrogate_used"]
    assert used > 0
