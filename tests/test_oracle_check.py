"""Pins of the oracle's invariant checker, its false-hit accounting and the
priority policy (CPU only).

The checker (oracle/check.py) judges every nondeterministic-mode GPU test, so
it is pinned here by mutation: it must accept a result that the oracle itself
produced, and report each kind of corruption a wrong device result could
carry (a found value of another key, an output off by 1e-4, a hole in a
cell, a duplicate verification hash, a stored word changed between frames,
a live entry no descriptor produced, a wrong bypass decision).

False hits (Sec. 3.2: verification collisions cannot be avoided) are counted
by the oracle's full-descriptor shadow map; a mask on the verification hash
forces them, and the closed forms below fix how many there must be.
"""
import itertools

import numpy as np
import pytest

from oracle import check, codec, graph, keys as K, render, table
from paper_2305_07238_amd import scenes


def _as_device_result(sc, hits, res, kmax=8):
    """An oracle FrameResult in the layout the device debug export uses."""
    n = len(hits)
    state = np.full((n, kmax), 3, np.uint8)
    state[res.valid] = 0
    state[res.valid & res.found] = 1
    state[res.valid & res.bypass] = 2
    value = res.found_value.astype(np.float32)
    out = {k: v.copy() for k, v in res.outputs.items()}
    return state, value, out


def _run_checker(sc, frames, n_cells, n_entries=8, mutate=None):
    """Snapshot-render ``frames`` with the oracle and run every checker function
    on each frame; ``mutate(f, hits, state, value, out, words, prev)`` may corrupt
    the device-layout result before the checks.  Returns all violations."""
    t = table.Table(n_cells, n_entries, 16)
    log, vals = check.KeyLog(), {}
    prev = None
    bad = []
    for f, h in enumerate(frames):
        res = render.shade_snapshot_frame(sc.materials, sc.textures, h, t, f)
        state, value, out = _as_device_result(sc, h, res)
        words = t.words().copy()
        if mutate is not None:
            mutate(f, h, state, value, out, words, prev)
        bad += check.check_frame(sc.materials, sc.textures, h, f, state, value, out, n_cells,
                                 log, vals)
        bad += check.table_structure(words, n_entries, prev)
        bad += check.check_entries_come_from_keys(words, n_entries, log)
        prev = words
    return bad


@pytest.fixture(scope="module")
def tiny():
    sc = scenes.tiny_scene()
    return sc, [sc.frame(f) for f in range(2)]


@pytest.fixture(scope="module")
def mid():
    sc = scenes.mid_scene(width=480, height=240, frames=2)
    sel = np.arange(0, sc.hits_per_frame, 8)             # 14,400 hits over 8 objects
    return sc, [sc.frame(f).take(sel) for f in range(2)]


def _recompute_outputs(sc, h, state, value, out, rows):
    """Outputs of ``rows`` re-evaluated with the (possibly corrupted) found values,
    as a device that used those values consistently would write them."""
    mat = h.material.astype(np.int64)
    for m in np.unique(mat[rows]):
        idx = np.nonzero(mat == m)[0]
        material = sc.materials[m]
        subst = {}
        for c, (node, sock) in enumerate(graph.cacheable_outputs(material)):
            otype = graph.output_type(material, node, sock)
            hit = state[idx, c] == 1
            if hit.any():
                v = value[idx, c, :3] if otype == "COLOR" else value[idx, c, 0]
                subst[(node, sock)] = (hit, np.nan_to_num(v.astype(np.float64)))
        o, _ = graph.evaluate(material, h.uv[idx], h.normal[idx], sc.textures, subst)
        for k in out:
            out[k][idx] = o[k]


@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_checker_accepts_the_oracles_own_run(which, request):
    sc, frames = request.getfixturevalue(which)
    n_cells = sc.cache.n_cells if which == "tiny" else 1 << 10
    assert _run_checker(sc, frames, n_cells) == []


def test_checker_flags_found_value_of_another_key(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f != 1:
            return
        # a FLOAT ordinal that hit: give hit j the value another key stored
        for c in range(8):
            rows = np.nonzero(state[:, c] == 1)[0]
            if len(rows) < 2:
                continue
            m = h.material[rows[0]]
            otype = graph.output_type(sc.materials[m], *graph.cacheable_outputs(sc.materials[m])[c])
            if otype != "FLOAT":
                continue
            same = rows[h.material[rows] == m]
            v = value[same, c, 0]
            far = np.nonzero(np.abs(v - v[0]) > 1e-2)[0]
            if len(far) == 0:
                continue
            value[same[0], c, 0] = v[far[0]]
            _recompute_outputs(sc, h, state, value, out, same[:1])
            return
        raise AssertionError("no FLOAT hit to corrupt")

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("matches no sample of its key" in b for b in bad), bad


def test_checker_flags_output_off_by_1e4(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 1:
            out["roughness"][123] += 1e-4

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("roughness" in b for b in bad), bad


def test_checker_flags_normal_off_by_2e5(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 0:
            out["normal"][77] += np.array([2e-5, 0.0, 0.0])

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("normal" in b for b in bad), bad


def _live_cell(words, n_entries, at_least):
    w = words.reshape(-1, n_entries)
    cells = np.nonzero((w != 0).sum(1) >= at_least)[0]
    assert len(cells), "no cell with enough live entries"
    return int(cells[0])


def test_checker_flags_hole_in_cell(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 0:
            c = _live_cell(words, 8, 2)
            words[c * 8] = 0

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("holes" in b for b in bad), bad


def test_checker_flags_duplicate_hash2(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 0:
            c = _live_cell(words, 8, 2)
            hi = words[c * 8] & np.uint64(0xFFFFFFFF00000000)
            words[c * 8 + 1] = hi | (words[c * 8 + 1] & np.uint64(0xFFFFFFFF))

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("duplicate hash2" in b for b in bad), bad


def test_checker_flags_word_changed_between_frames(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 1:
            c = _live_cell(prev, 8, 1)
            words[c * 8] ^= np.uint64(1)                 # value bits of a kept entry

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("stored words changed" in b for b in bad), bad


def test_checker_flags_entry_no_key_produced(mid):
    sc, frames = mid

    def mutate(f, h, state, value, out, words, prev):
        if f == 0:
            w = words.reshape(-1, 8)
            c = int(np.nonzero((w != 0).sum(1) < 8)[0][0])
            k = int((w[c] != 0).sum())
            words[c * 8 + k] = np.uint64((0xDEADBEEF << 32) | 5)

    bad = _run_checker(sc, frames, 1 << 10, mutate=mutate)
    assert any("no matching descriptor" in b for b in bad), bad


def test_checker_flags_wrong_bypass_decision(tiny):
    sc, frames = tiny

    def mutate(f, h, state, value, out, words, prev):
        if f == 0:
            state[5, 0] = 2

    bad = _run_checker(sc, frames, sc.cache.n_cells, mutate=mutate)
    assert any("bypass" in b for b in bad), bad


def test_tolerance_bars():
    # scalar: |d| <= 1e-5 |ref| + 1e-6
    assert check.scalar_ratio([1.0 + 1.05e-5], [1.0]) < 1.0
    assert check.scalar_ratio([1.0 + 1.2e-5], [1.0]) > 1.0
    assert check.scalar_ratio([0.01 + 1.0e-6], [0.01]) < 1.0
    assert check.scalar_ratio([0.01 + 2.0e-6], [0.01]) > 1.0        # small values: tighter
    assert check.scalar_ratio([np.nan], [0.5]) == np.inf
    # unit normal: Euclidean length of the difference
    n = np.array([[0.0, 0.6, 0.8]])
    assert check.normal_ratio(n + [[6e-6, 6e-6, 0.0]], n) < 1.0
    assert check.normal_ratio(n + [[8e-6, 8e-6, 0.0]], n) > 1.0


# ----------------------------------------------------------- false hits -------

def test_full_hash_gives_no_false_hits_on_tiny(tiny):
    sc, frames = tiny
    t = table.Table(sc.cache.n_cells, 8, 16)
    res = render.shade_snapshot(sc.materials, sc.textures, frames, t)
    assert sum(r.stats["false_hits"] for r in res) == 0
    assert res[1].stats["hits"] == res[1].stats["probes"] == 8192


def test_one_bit_verification_hash_forces_closed_form_false_hits(tiny):
    """One cell and a 1-bit mask: every verification hash is 1.  Frame 0 stores
    exactly its first candidate (the others find hash 1 present); in frame 1
    every probe hits that entry, and it is a false hit exactly when the probe's
    descriptor differs from the first candidate's."""
    sc, frames = tiny
    t = table.Table(1, 8, 16)
    res = render.shade_snapshot(sc.materials, sc.textures, frames, t, hash2_mask=0x1)
    assert t.occupancy() == 1
    assert res[0].stats["inserted"] == 1
    assert res[0].stats["present"] == res[0].stats["candidates"] - 1
    mat = sc.materials[0]
    cach = graph.cacheable_outputs(mat)
    k0 = [K.compute_keys(0, n, s, frames[0].uv, frames[0].duv, 1) for n, s in cach]
    first = (int(k0[0].k0[0]), int(k0[0].k1[0]))            # seq 0: hit 0, ordinal 0
    k1 = [K.compute_keys(0, n, s, frames[1].uv, frames[1].duv, 1) for n, s in cach]
    same = sum(int(np.sum((k.k0 == first[0]) & (k.k1 == first[1]))) for k in k1)
    probes = sum(len(k.k0) for k in k1)
    assert res[1].stats["hits"] == probes
    assert res[1].stats["false_hits"] == probes - same
    assert res[1].stats["false_hits"] > 0
    # every frame-1 lookup returned the one stored code
    code = t.word[0] & 0xFFFFFFFF
    f = res[1].found_value
    assert np.all(f[:, 1, 0] == codec.float_decode(np.array([code], np.uint64))[0]) or \
        np.all(f[:, 0, :] == codec.rgb9e5_decode(np.array([code], np.uint64))[0])


class _KeyedListModel:
    """Cells as ordered lists of [hash, value, stamp, bounce, key]; no indexing.
    Counts a lookup as false when the hash matches but the key does not."""

    def __init__(self, n_cells, cap):
        self.cells = [[] for _ in range(n_cells)]
        self.cap = cap
        self.false_hits = 0

    def insert(self, cell, h, v, policy, frame, key, bounce):
        lst = self.cells[cell]
        if any(e[0] == h for e in lst):
            return "present"
        if len(lst) < self.cap:
            lst.append([h, v, frame + 1, bounce if policy == "PRIORITY" else 0, key])
            return "inserted"
        if policy == "FIRST":
            return "full"
        if policy == "OVERWRITE":
            order = sorted(range(len(lst)), key=lambda i: (lst[i][2], i))
            k = order[0]
            if lst[k][2] < frame + 1:
                lst[k] = [h, v, frame + 1, 0, key]
                return "overwritten"
            return "full"
        # PRIORITY: the most-bounced entry goes first, then the oldest
        worst = max(e[3] for e in lst)
        cands = [i for i in range(len(lst)) if lst[i][3] == worst]
        k = min(cands, key=lambda i: (lst[i][2], i))
        if worst > bounce or (worst == bounce and lst[k][2] < frame + 1):
            lst[k] = [h, v, frame + 1, bounce, key]
            return "overwritten"
        return "full"

    def lookup(self, cell, h, key):
        for e in self.cells[cell]:
            if e[0] == h:
                if e[4] != key:
                    self.false_hits += 1
                return True, e[1]
        return False, 0


@pytest.mark.parametrize("policy", ["FIRST", "OVERWRITE", "PRIORITY"])
def test_table_matches_keyed_list_model_all_orders(policy):
    """Colliding hashes (several keys share a hash), bounce counts and two
    frames, over every insert order of 6 keys, against a model with no arrays."""
    n_cells, cap = 2, 2
    # key k: cell k % 2, hash 1 + k % 3 (keys 0 and 3 share cell 0? no: 0,2,4 -> cell 0)
    keys_ = [(k % n_cells, 1 + (k // 2) % 2, 100 + k, ("key", k), k % 3) for k in range(6)]
    for perm in itertools.permutations(range(6)):
        t = table.Table(n_cells, cap, 16)
        m = _KeyedListModel(n_cells, cap)
        for pos, k in enumerate(perm):
            cell, h, v, key, b = keys_[k]
            frame = 0 if pos < 3 else 1
            got = t.insert(cell, h, v, policy, frame, key=key, bounce=b)
            want = m.insert(cell, h, v, policy, frame, key, b)
            assert got == want, (perm, pos)
        for cell in range(n_cells):
            words = t.word[cell * cap:(cell + 1) * cap]
            live = sorted((w >> 32, w & 0xFFFFFFFF) for w in words if w)
            assert live == sorted((e[0], e[1]) for e in m.cells[cell])
        for cell, h, v, key, b in keys_:
            assert t.lookup(cell, h, key) == m.lookup(cell, h, key)
        assert t.false_hits == m.false_hits


def test_priority_hand_trace():
    """One cell of two entries; bounce counts in brackets.
    frame 0: A[1] -> e0, B[1] -> e1 (cell full);
             C[0] displaces the most-bounced, oldest, lowest entry: A (e0);
             D[1] same frame, ties with B[1] but B is not older: full;
             E[2] may not displace anything of fewer bounces: full.
    frame 1: F[1] displaces B[1] (same bounces, older); G[0] displaces F[1] (more
             bounces, although written in this frame); H[0] ties on bounces and
             displaces C[0], the older; I[0] then finds only bounce-0 entries of
             this frame: full."""
    t = table.Table(1, 2, 16)
    P = table.PRIORITY
    assert t.insert(0, 10, 1, P, 0, bounce=1) == "inserted"
    assert t.insert(0, 11, 2, P, 0, bounce=1) == "inserted"
    assert t.insert(0, 12, 3, P, 0, bounce=0) == "overwritten"
    assert t.word[0] >> 32 == 12 and t.aux[0] == 0
    assert t.insert(0, 13, 4, P, 0, bounce=1) == "full"
    assert t.insert(0, 14, 5, P, 0, bounce=2) == "full"
    assert t.insert(0, 15, 6, P, 1, bounce=1) == "overwritten"
    assert t.word[1] >> 32 == 15 and t.stamp[1] == 2 and t.aux[1] == 1
    assert t.insert(0, 16, 7, P, 1, bounce=0) == "overwritten"      # displaces F[1] (more bounces)
    assert t.word[1] >> 32 == 16 and t.aux[1] == 0
    assert t.insert(0, 17, 8, P, 1, bounce=0) == "overwritten"      # C[0], stamp 1 < 2
    assert t.word[0] >> 32 == 17
    assert t.insert(0, 18, 9, P, 1, bounce=0) == "full"
    # OVERWRITE and FIRST leave aux at 0
    t2 = table.Table(1, 1, 16)
    t2.insert(0, 5, 1, table.OVERWRITE, 0, bounce=3)
    assert t2.aux[0] == 0


def test_priority_keeps_direct_samples_findable():
    """What the policy is for (Sec. 5: prefer directly visible samples when
    storage is limited): each frame's direct hits are followed by as many
    indirect ones, scattered over the scene with wider footprints.  On a table
    too small for all of them, directly visible samples of the last frame find
    their values more often under PRIORITY than under OVERWRITE or FIRST (same
    inputs, deterministic snapshot runs)."""
    sc = scenes.mid_scene(width=480, height=240, frames=3)
    sel = np.arange(0, sc.hits_per_frame, 6)
    frames = [scenes.with_indirect(sc.frame(f).take(sel), f) for f in range(3)]
    rate = {}
    for policy in (table.FIRST, table.OVERWRITE, table.PRIORITY):
        t = table.Table(4096, 8, 16)
        res = render.shade_snapshot(sc.materials, sc.textures, frames, t, policy=policy)
        last = res[-1]
        direct = frames[-1].bounce == 0
        probed = last.valid & ~last.bypass
        rate[policy] = float(last.found[direct][probed[direct]].mean())
    print("direct-sample hit rate of the last frame", rate)
    assert rate[table.PRIORITY] > rate[table.OVERWRITE] + 0.1, rate
    assert rate[table.PRIORITY] > rate[table.FIRST], rate
