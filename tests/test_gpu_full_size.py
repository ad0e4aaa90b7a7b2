"""Full-size parity on the batching workload (1000 materials of 4-400 nodes,
1920x1080, table 2^24 slots) and the scale workload (4096 materials,
3840x2160, table 2^26 slots = 1 GiB, OVERWRITE), in the launch settings the
benchmark uses, checked on sampled hits.

Snapshot mode makes every frame's table unique, so at full size the oracle
can check sampled outputs one by one:
  frame 0  the table is empty: no lookup hits, and each sampled output equals
           the FP64 graph (value bar: 1e-5 |ref| + 1e-6 per scalar, 1e-5 for
           the unit normal);
  frame 1  every sampled lookup hits iff its (cell, hash2) is in the exported
           table after frame 0 (same scan as Algorithm 1); a key absent from
           that table was either never seen in frame 0 or met a full cell; a
           found value is the code of the key's first writer in frame 0 (the
           lowest (hit, ordinal) sequence number with that key), re-evaluated
           in FP64 (within one RGB9E5 step, or the scalar bar for raw floats); every
           sampled output equals the FP64 graph with the GPU's found values
           substituted (value bar).
"""
import numpy as np
import pytest

from oracle import codec, graph, keys as K, render
from paper_2305_07238_amd import scenes
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2305_07238_amd import binding as B  # noqa: E402


def _table_lookup(words, n_entries, cell, hash2):
    """Algorithm 1's scan on an exported table: (found, code, cell full of other keys)."""
    row = words[cell * n_entries:(cell + 1) * n_entries]
    for w in row:
        h = int(w) >> 32
        if h == hash2:
            return True, int(w) & 0xFFFFFFFF, False
        if int(w) == 0:
            return False, 0, False
    return False, 0, True


def _run(sc, flags, policy, n_sample=1500, seed=0):
    ctx = G.setup(sc)
    cc = sc.cache
    cache = ctx.cache(cc.n_cells, cc.n_entries, cc.entry_bytes, policy)
    kw = dict(mode=B.PMC_MODE_SNAPSHOT, flags=flags, chunk_waves=4, defer_max=48, debug=True)
    h0, h1 = sc.frame(0), sc.frame(1)
    rng = np.random.default_rng(seed)

    # ---- frame 0: empty table
    out0, state0, _, st0 = G.shade(ctx, h0, cache, frame=0, **kw)
    assert st0["cache_hits"] == 0 and st0["hits_shaded"] == len(h0)
    assert not np.any(state0 == 1)
    s0 = np.sort(rng.choice(len(h0), n_sample, replace=False))
    ref0 = render.shade_uncached(sc.materials, sc.textures, h0.take(s0))
    G.assert_outputs(out0, ref0, s0, "frame 0")
    words = cache.words()[:, 0].copy()
    del out0, state0

    # ---- frame 1: lookups see the table of frame 0
    out1, state1, value1, st1 = G.shade(ctx, h1, cache, frame=1, **kw)
    s1 = np.sort(rng.choice(len(h1), n_sample, replace=False))
    n_found = n_absent_full = 0
    for m in np.unique(h1.material[s1]):
        m = int(m)
        mat = sc.materials[m]
        cach = graph.cacheable_outputs(mat)
        mine1 = s1[h1.material[s1] == m]
        mine0 = np.nonzero(h0.material == m)[0]
        subst = {}
        for c, (node, sock) in enumerate(cach):
            otype = graph.output_type(mat, node, sock)
            k1 = K.compute_keys(m, node, sock, h1.uv[mine1], h1.duv[mine1], cc.n_cells)
            k0 = K.compute_keys(m, node, sock, h0.uv[mine0], h0.duv[mine0], cc.n_cells)
            ok0 = ~k0.bypass
            key0 = (k0.cell[ok0].astype(np.uint64) << np.uint64(32)) | k0.hash2[ok0].astype(np.uint64)
            uniq, first = np.unique(key0, return_index=True)
            writer = mine0[np.nonzero(ok0)[0][first]]
            found_rows, writers = [], []
            for j, h in enumerate(mine1):
                st = state1[h, c]
                if k1.bypass[j]:
                    assert st == 2
                    continue
                cell, h2 = int(k1.cell[j]), int(k1.hash2[j])
                hit, code, full = _table_lookup(words, cc.n_entries, cell, h2)
                assert (st == 1) == hit, (m, c, h)
                kk = np.uint64((cell << 32) | h2)
                pos = np.searchsorted(uniq, kk)
                seen = pos < len(uniq) and uniq[pos] == kk
                if hit:
                    assert seen
                    found_rows.append(j)
                    writers.append(int(writer[pos]))
                elif seen:
                    assert full                       # seen in frame 0, dropped by a full cell
                    n_absent_full += 1
            if found_rows:
                n_found += len(found_rows)
                w = np.array(writers)
                _, vals = graph.evaluate(mat, h0.uv[w], h0.normal[w], sc.textures)
                ref = render.decode(render.encode(vals[(node, sock)], otype), otype)
                got = value1[mine1[found_rows], c]
                if otype == "COLOR":
                    step = codec.rgb9e5_step(codec.rgb9e5_encode(ref))
                    assert np.all(np.abs(got - ref) <= step[:, None] + 1e-12), (m, c)
                else:
                    assert G.scalar_ok(got[:, 0], ref), (m, c)
            sel = state1[mine1, c] == 1
            if sel.any():
                v = value1[mine1, c, :3] if otype == "COLOR" else value1[mine1, c, 0]
                subst[(node, sock)] = (sel, np.nan_to_num(v.astype(np.float64)))
        o, _ = graph.evaluate(mat, h1.uv[mine1], h1.normal[mine1], sc.textures, subst)
        G.assert_outputs(out1, o, mine1, m)
    print(f"{sc.name}: frame-1 stats {st1}; sampled found {n_found}, dropped by full cells "
          f"{n_absent_full}")
    assert n_found > n_sample // 4
    ctx.close()


def test_batching_workload_full_size():
    sc = scenes.batching_scene(frames=2)
    _run(sc, B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, B.PMC_POLICY_FIRST)


def test_scale_workload_full_size():
    sc = scenes.scale_scene(frames=2)
    _run(sc, B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER | B.PMC_FLAG_PERSISTENT, B.PMC_POLICY_OVERWRITE,
         seed=1)


def test_scale_workload_overwrite_evicts_like_the_oracle():
    """OVERWRITE evictions at the scale workload's size: a 2^22-slot table
    (2^19 cells of 8, a sixteenth of the benchmark's) overflows in frame 0, so
    frame 1's misses displace frame-0 entries.  On sampled cells the table
    after frame 1 equals the oracle's sequential apply of frame 1's candidates
    (in (hit, ordinal) order) to the device's own table after frame 0: hash
    halves and stamps bit-exact, value codes within one RGB9E5 step or the
    scalar bar of the FP64 value at the entry's writer.

    A key's writer in frame 1 is its first candidate: entries stamped in the
    current frame are never displaced, so later candidates of the key find it
    present or its cell full.  The candidates' values are all finite (the
    device counts no non-finite value), so the simulation needs the FP64 values
    of the writers only; a writer's value is its graph with the outputs it
    found in the table (upstream of the written one, if any) substituted."""
    from oracle import table as T
    sc = scenes.scale_scene(frames=2)
    n_cells, n_e = 1 << 19, 8
    ctx = G.setup(sc)
    cache = ctx.cache(n_cells, n_e, 16, B.PMC_POLICY_OVERWRITE)
    kw = dict(mode=B.PMC_MODE_SNAPSHOT, flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, chunk_waves=4,
              defer_max=48)
    _, _, _, st0 = G.shade(ctx, sc.frame(0), cache, frame=0, **kw)
    w0 = cache.words().copy()
    h1 = sc.frame(1)
    _, _, _, st1 = G.shade(ctx, h1, cache, frame=1, **kw)
    w1 = cache.words().copy()
    ctx.close()
    print("scale, 2^19 x 8 table: frame 0", st0, "frame 1", st1)
    assert st0["cell_full"] > 0 and st1["overwrites"] > 10_000
    assert st1["nonfinite"] == 0

    rng = np.random.default_rng(3)
    cells = np.sort(rng.choice(n_cells, 1000, replace=False))
    slot_of = np.full(n_cells, -1, np.int64)
    slot_of[cells] = np.arange(len(cells))
    rows = (cells[:, None] * n_e + np.arange(n_e)).ravel()
    ref = T.Table(len(cells), n_e, 16)
    ref.word = [int(x) for x in w0[rows, 0]]
    ref.stamp = [int(x) & 0xFFFFFFFF for x in w0[rows, 1]]
    ref.aux = [int(x) >> 32 for x in w0[rows, 1]]

    # frame 1's candidates in the sampled cells: keys that miss in the table after frame 0
    order = np.argsort(h1.material, kind="stable")
    bounds = np.searchsorted(h1.material[order], np.arange(len(sc.materials) + 1))
    cand = []                                     # (hit, ordinal, slot, hash2, key, m, node, sock)
    for m in range(len(sc.materials)):
        idx = order[bounds[m]:bounds[m + 1]]
        if len(idx) == 0:
            continue
        for c, (node, sock) in enumerate(graph.cacheable_outputs(sc.materials[m])):
            ky = K.compute_keys(m, node, sock, h1.uv[idx], h1.duv[idx], n_cells)
            for j in np.nonzero(~ky.bypass & (slot_of[ky.cell] >= 0))[0]:
                hit, _, _ = _table_lookup(w0[:, 0], n_e, int(ky.cell[j]), int(ky.hash2[j]))
                if not hit:
                    cand.append((int(idx[j]), c, int(slot_of[ky.cell[j]]), int(ky.hash2[j]),
                                 (int(ky.k0[j]), int(ky.k1[j])), m, node, sock))
    cand.sort(key=lambda t: (t[0], t[1]))
    first = {}
    outcome = {}
    for h, c, slot, h2, key, m, node, sock in cand:
        first.setdefault(key, (h, m, node, sock))
        r = ref.insert(slot, h2, 0, T.OVERWRITE, 1, key=key)
        outcome[r] = outcome.get(r, 0) + 1
    # the codes of the entries written in frame 1, from their writers' FP64 values
    by_mat = {}
    for e in range(len(ref.word)):
        if ref.stamp[e] == 2:
            h, m, node, sock = first[ref.key[e]]
            by_mat.setdefault(m, []).append((e, h, node, sock))
    for m, ents in by_mat.items():
        mat = sc.materials[m]
        hh = np.array(sorted({h for _, h, _, _ in ents}))
        # the writer's other outputs found in the table after frame 0 stand in
        # for their sub-graphs, as in the shading of frame 1
        subst = {}
        for node, sock in graph.cacheable_outputs(mat):
            otype = graph.output_type(mat, node, sock)
            ky = K.compute_keys(m, node, sock, h1.uv[hh], h1.duv[hh], n_cells)
            found = np.zeros(len(hh), bool)
            v = np.zeros((len(hh), 3)) if otype == "COLOR" else np.zeros(len(hh))
            for j in np.nonzero(~ky.bypass)[0]:
                hit, code, _ = _table_lookup(w0[:, 0], n_e, int(ky.cell[j]), int(ky.hash2[j]))
                if hit:
                    found[j] = True
                    v[j] = render.decode(np.array([code], np.uint64), otype)[0]
            if found.any():
                subst[(node, sock)] = (found, v)
        _, vals = graph.evaluate(mat, h1.uv[hh], h1.normal[hh], sc.textures, subst)
        for e, h, node, sock in ents:
            v = np.asarray(vals[(node, sock)][np.searchsorted(hh, h)])
            enc = int(render.encode(v[None], graph.output_type(mat, node, sock))[0])
            ref.word[e] = (ref.word[e] >> 32 << 32) | enc
    print("sampled cells:", len(cells), "candidates", len(cand), outcome)
    assert outcome.get("overwritten", 0) > 10
    n_diff = G.table_parity(w1[rows], ref, sc.materials)
    print("value codes differing within the bar:", n_diff)
