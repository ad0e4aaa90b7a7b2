"""Invariants that a lock-free (nondeterministic) cached run must satisfy.

Sec. 3.3: several threads may shade samples with the same descriptor at once
and insert with a compare-and-swap, so which sample's value a later lookup
returns, and whether a lookup hits at all, depends on timing.  Many results
are then correct.  A run is accepted when:
  (i)   every value returned by a lookup is the encoded value of the same
        cacheable output computed at some sample with the same descriptor
        (Sec. 3: the stored value is a sub-graph result at an earlier sample);
  (ii)  every live table entry carries the hash2 of a descriptor that was
        inserted into that cell;
  (iii) FIRST policy (Sec. 3.2): no hash2 appears twice in a cell, the live
        entries of each cell form a prefix, and a stored word never changes
        in later frames;
  (iv)  the BSDF outputs equal plain evaluation with the returned values
        substituted at the cacheable outputs.
The functions return lists of violations (empty = accepted).

Value tolerance (FP32 device arithmetic against this FP64 model): a scalar
channel (a colour component, roughness, a FLOAT node value) passes when
|got - ref| <= 1e-5 |ref| + 1e-6; the unit normal when the Euclidean length
of got - ref is at most 1e-5.  A value taken from the table may also sit one
RGB9E5 step from the re-evaluated one (an FP32 input on the other side of a
rounding boundary of the encoding).
"""
from collections import defaultdict

import numpy as np

from . import codec, graph, keys as K


RTOL, ATOL, NTOL = 1e-5, 1e-6, 1e-5
OUTPUT_KEYS = ("base_color", "roughness", "normal")


def scalar_ratio(got, ref, rtol=RTOL, atol=ATOL) -> float:
    """Largest |got - ref| / (rtol |ref| + atol) over the elements (<= 1 passes;
    NaN in either array counts as a failure unless both are NaN)."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    if g.size == 0:
        return 0.0
    both_nan = np.isnan(g) & np.isnan(r)
    q = np.abs(g - r) / (rtol * np.abs(r) + atol)
    q = np.where(both_nan, 0.0, np.where(np.isnan(q), np.inf, q))
    return float(q.max())


def normal_ratio(got, ref, ntol=NTOL) -> float:
    """Largest Euclidean |got - ref| / ntol over rows of 3-vectors."""
    g = np.asarray(got, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    if g.shape[0] == 0:
        return 0.0
    d = np.sqrt(np.sum((g - r) ** 2, axis=1)) / ntol
    return float(np.where(np.isnan(d), np.inf, d).max())


def output_ratios(got: dict, ref: dict, rows=None) -> dict:
    """Per BSDF output, the largest error relative to its bar (<= 1 passes)."""
    sel = (lambda a: a) if rows is None else (lambda a: np.asarray(a)[rows])
    return {"base_color": scalar_ratio(sel(got["base_color"]), ref["base_color"]),
            "roughness": scalar_ratio(sel(got["roughness"]), ref["roughness"]),
            "normal": normal_ratio(sel(got["normal"]), ref["normal"])}


def decoded_candidates(values, out_type):
    """Decode(Encode(v)) of FP64 values: what the table can hold for them."""
    if out_type == "COLOR":
        return codec.rgb9e5_decode(codec.rgb9e5_encode(values))
    return codec.float_decode(codec.float_encode(values))


def table_structure(words, n_entries, previous=None):
    """(iii): prefix occupancy, unique hash2 per cell, and monotonic growth."""
    bad = []
    w = np.asarray(words, dtype=np.uint64).reshape(-1, n_entries)
    live = w != 0
    # prefix: once an entry is empty, the rest of the cell is empty
    after_gap = np.cumsum(~live, axis=1) > 0
    if np.any(live & after_gap):
        bad.append(f"{int(np.sum(np.any(live & after_gap, axis=1)))} cells with holes")
    h = (w >> np.uint64(32)).astype(np.int64)
    for cell in np.nonzero(live.sum(1) > 1)[0]:
        hs = h[cell][live[cell]]
        if len(set(hs.tolist())) != len(hs):
            bad.append(f"cell {cell}: duplicate hash2")
            break
    if previous is not None:
        p = np.asarray(previous, dtype=np.uint64).reshape(-1, n_entries)
        changed = (p != 0) & (p != w)
        if np.any(changed):
            bad.append(f"{int(changed.sum())} stored words changed")
    return bad


class KeyLog:
    """Every sample that could have stored a value so far (a lookup that missed):
    descriptor -> list of (frame, hit id, ordinal), and its (cell, hash2)."""

    def __init__(self):
        self.by_key = defaultdict(list)      # (k0, k1) -> [(frame, local hit, c)]
        self.cellhash = set()                # (cell, hash2) of every such sample

    def add(self, frame, mat, c, local_idx, ky, rows=None):
        """Log the samples ``rows`` (positions into local_idx; default all) that
        were not bypassed."""
        rows = range(len(local_idx)) if rows is None else rows
        for j in rows:
            if ky.bypass[j]:
                continue
            self.by_key[(int(ky.k0[j]), int(ky.k1[j]))].append((frame, int(local_idx[j]), c))
            self.cellhash.add((int(ky.cell[j]), int(ky.hash2[j])))


def check_frame(materials, textures, hits, frame, state, value, outputs, n_cells,
                log: KeyLog, values_by_frame, level_bias=0, level_max=K.LEVEL_MAX_DEFAULT,
                rtol=1e-5, min_subgraph_nodes=2):
    """Check (i) and (iv) for one frame of GPU results and extend the key log.

    state [n, 8] uint8 (0 miss, 1 hit, 2 bypass, 3 none), value [n, 8, 3]
    (decoded value on a hit), outputs dict of [n, ...] arrays.  values_by_frame
    collects, per frame, the oracle's per-(hit, c) values for (i).
    Returns a list of violations."""
    bad = []
    n = len(hits)
    mat = hits.material.astype(np.int64)
    frame_vals = {}
    pending_hits = []                      # (h, c, key, type, gpu value)
    for m in np.unique(mat):
        idx = np.nonzero(mat == m)[0]
        if m >= len(materials):
            continue
        material = materials[m]
        cach = graph.cacheable_outputs(material, min_subgraph_nodes)
        subst = {}
        kys = []
        for c, (node, sock) in enumerate(cach):
            ky = K.keys_for(material, int(m), node, sock, hits, idx, n_cells, level_bias,
                            level_max)
            kys.append(ky)
            otype = graph.output_type(material, node, sock)
            st = state[idx, c]
            if np.any((st == 2) != ky.bypass):
                bad.append(f"material {m} ordinal {c}: bypass decisions differ")
            hit = st == 1
            if hit.any():
                v = value[idx, c, :3] if otype == "COLOR" else value[idx, c, 0]
                subst[(node, sock)] = (hit, v.astype(np.float64))
                for j in np.nonzero(hit)[0]:
                    pending_hits.append((int(idx[j]), c, (int(ky.k0[j]), int(ky.k1[j])), otype,
                                         v[j]))
        pos = None if getattr(hits, "position", None) is None else hits.position[idx]
        out, vals = graph.evaluate(material, hits.uv[idx], hits.normal[idx], textures, subst,
                                   position=pos)
        ratios = output_ratios(outputs, out, idx)
        for k, q in ratios.items():
            if not q <= 1.0:
                bad.append(f"material {m}: {k} error {q:.3g} x its bar")
        # what a sample that missed ordinal c computed and may have stored: the
        # sub-graph of c with the sample's other found values in place (its own
        # ordinal is not substituted: it missed)
        for c, (node, sock) in enumerate(cach):
            otype = graph.output_type(material, node, sock)
            missed = np.nonzero(state[idx, c] == 0)[0]
            if len(missed) == 0:
                continue
            own = vals
            if (node, sock) in subst:
                others = {k: v for k, v in subst.items() if k != (node, sock)}
                _, own = graph.evaluate(material, hits.uv[idx], hits.normal[idx], textures,
                                        others, position=pos)
            dv = decoded_candidates(own[(node, sock)], otype)
            for j in missed:
                frame_vals[(int(idx[j]), c)] = dv[j]
            log.add(frame, int(m), c, idx, kys[c], missed)
    values_by_frame[frame] = frame_vals
    # (i): a found value equals the stored value of some sample with the same key
    for h, c, key, otype, gv in pending_hits:
        ok = False
        for (f, li, cc) in log.by_key.get(key, []):
            cand = values_by_frame[f].get((li, cc))
            if cand is None:
                continue
            cand = np.atleast_1d(cand)
            g = np.atleast_1d(gv).astype(np.float64)[:cand.shape[0]]
            if otype == "COLOR":
                step = codec.rgb9e5_step(codec.rgb9e5_encode(np.reshape(cand, (1, 3))))[0]
                if np.all(np.abs(g - cand) <= step * 1.0001):
                    ok = True
                    break
            elif scalar_ratio(g, cand, rtol) <= 1.0:
                ok = True
                break
        if not ok:
            bad.append(f"hit {h} ordinal {c}: found value matches no sample of its key")
            if len(bad) > 20:
                break
    return bad


def check_entries_come_from_keys(words, n_entries, log: KeyLog):
    """(ii): every live entry's (cell, hash2) belongs to a keyed sample."""
    w = np.asarray(words, dtype=np.uint64).reshape(-1, n_entries)
    cells, ents = np.nonzero(w != 0)
    missing = 0
    for cell, e in zip(cells, ents):
        if (int(cell), int(w[cell, e] >> np.uint64(32))) not in log.cellhash:
            missing += 1
    return [f"{missing} live entries with no matching descriptor"] if missing else []
