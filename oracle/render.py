"""Shading a batch of hits: uncached, and cached in deterministic snapshot mode.

Sec. 3: at a cacheable node the cache is looked up first; on a hit the cached
value is used and the sub-graph is skipped; otherwise the sub-graph is
evaluated in the standard way and its value stored.  Sec. 1 and 3.2: values
are inserted progressively while frames are rendered, and the table persists
across frames.

Snapshot semantics (a deterministic reading of the concurrent update of
Sec. 3.3): a frame is one batch of hits.  Every lookup of frame f sees the
table as it was after frame f - 1; the frame's insert candidates are then
applied in ascending sequence number seq = (hit index, cacheable ordinal)
with Algorithm 1, stamping writes with f + 1.
"""
from collections import Counter
from typing import List, Optional

import numpy as np

from . import codec, graph, keys as K, mlp
from .table import FIRST, Table


def decode(enc, out_type):
    if out_type == "COLOR":
        return codec.rgb9e5_decode(np.asarray(enc, dtype=np.uint64))
    return codec.float_decode(np.asarray(enc, dtype=np.uint64))


def encode(value, out_type):
    if out_type == "COLOR":
        return codec.rgb9e5_encode(value)
    return codec.float_encode(value)


def _pos(hits, idx):
    p = getattr(hits, "position", None)
    return None if p is None else p[idx]


def shade_uncached(materials, textures, hits):
    """Plain evaluation of every hit (cache disabled).  Returns dict of FP64 arrays."""
    n = len(hits)
    out = dict(base_color=np.zeros((n, 3)), roughness=np.zeros(n), normal=np.zeros((n, 3)))
    mat = hits.material.astype(np.int64)
    for m in np.unique(mat):
        idx = np.nonzero(mat == m)[0]
        if m >= len(materials):
            o = graph.default_outputs(hits.normal[idx])
        else:
            o, _ = graph.evaluate(materials[m], hits.uv[idx], hits.normal[idx], textures,
                                  position=_pos(hits, idx))
        for k in out:
            out[k][idx] = o[k]
    return out


class FrameResult:
    def __init__(self, n, kmax):
        self.outputs = dict(base_color=np.zeros((n, 3)), roughness=np.zeros(n),
                            normal=np.zeros((n, 3)))
        self.found = np.zeros((n, kmax), dtype=bool)        # cache hit per (hit, ordinal)
        self.false_hit = np.zeros((n, kmax), dtype=bool)    # hit on another descriptor's entry
        self.bypass = np.zeros((n, kmax), dtype=bool)
        self.valid = np.zeros((n, kmax), dtype=bool)        # ordinal exists for the hit's material
        self.found_value = np.full((n, kmax, 3), np.nan)    # decoded value on a cache hit
        self.surrogate = np.zeros((n, kmax), dtype=bool)    # value taken from the network
        self.surrogate_value = np.full((n, kmax, 3), np.nan)
        self.audited = np.zeros((n, kmax), dtype=bool)      # eligible, evaluated by the graph
        self.live_err = {}                                  # material -> max audited error
        self.log = []                                       # (material, ordinal, u, v, value)
        self.stats = Counter()


def shade_snapshot_frame(materials, textures, hits, table: Table, frame: int,
                         policy: str = FIRST, level_bias: int = 0,
                         level_max: int = K.LEVEL_MAX_DEFAULT, min_subgraph_nodes: int = 2,
                         kmax: int = 8, cacheables: Optional[list] = None,
                         surrogate: Optional[dict] = None,
                         surrogate_values: Optional[np.ndarray] = None,
                         surrogate_insert: bool = False,
                         hash2_mask: int = 0xFFFFFFFF) -> FrameResult:
    """One snapshot-mode frame; mutates ``table`` into T_f and returns the frame's results.

    surrogate: optional {material: dict(params=[W1, b1, W2, b2, W3, b3],
    ordmap={ordinal: (first channel, width)}, trusted=bool)} of the materials
    that have a network.  For a trusted one, a missed surrogated output that
    is not audited takes the network's value (FP16 rounding points of
    mlp.forward) and is not inserted; for every one, the inserts of its
    surrogated outputs are logged.  surrogate_values [n, kmax, 3], if given,
    replaces the network's values at the substituted entries (to check what
    follows them against another implementation's network outputs).
    surrogate_insert: the substituted values are inserted too (as candidates of
    their hits, like graph values).
    hash2_mask: bits of the verification hash kept (forces collisions; see keys).
    Lookups pass the full descriptor, so ``stats["false_hits"]`` counts hits on
    entries written for another descriptor (Sec. 3.2).  Under the PRIORITY
    policy each candidate carries its hit's bounce count (``hits.bounce``,
    0 when absent).
    """
    n = len(hits)
    res = FrameResult(n, kmax)
    mat = hits.material.astype(np.int64)
    if cacheables is None:
        cacheables = [graph.cacheable_outputs(m, min_subgraph_nodes) for m in materials]
    candidates = []                                  # (hit, ordinal, cell, hash2, enc, key)
    false0 = table.false_hits
    for m in np.unique(mat):
        idx = np.nonzero(mat == m)[0]
        if m >= len(materials):
            o = graph.default_outputs(hits.normal[idx])
            res.stats["invalid_material"] += len(idx)
            for k in res.outputs:
                res.outputs[k][idx] = o[k]
            continue
        material = materials[m]
        cach = cacheables[m]
        subst = {}
        key_list = []
        for c, (node, sock) in enumerate(cach):
            ky = K.keys_for(material, int(m), node, sock, hits, idx, table.n_cells,
                            level_bias, level_max, hash2_mask)
            key_list.append(ky)
            otype = graph.output_type(material, node, sock)
            found = np.zeros(len(idx), dtype=bool)
            encs = np.zeros(len(idx), dtype=np.uint64)
            for j in range(len(idx)):
                if ky.bypass[j]:
                    continue
                f0 = table.false_hits
                hit, enc = table.lookup(int(ky.cell[j]), int(ky.hash2[j]),
                                        (int(ky.k0[j]), int(ky.k1[j])))
                found[j] = hit
                encs[j] = enc
                if table.false_hits != f0:
                    res.false_hit[idx[j], c] = True
            res.valid[idx, c] = True
            res.bypass[idx, c] = ky.bypass
            res.found[idx, c] = found
            res.stats["bypasses"] += int(ky.bypass.sum())
            res.stats["probes"] += int((~ky.bypass).sum())
            res.stats["hits"] += int(found.sum())
            if found.any():
                dv = decode(encs[found], otype)
                if otype == "COLOR":
                    res.found_value[idx[found], c, :] = dv
                else:
                    res.found_value[idx[found], c, 0] = dv
                subst[(node, sock)] = (found, np.zeros((len(idx), 3)) if otype == "COLOR"
                                       else np.zeros(len(idx)))
                full = subst[(node, sock)][1]
                full[found] = dv
        sinfo = surrogate.get(int(m)) if surrogate else None
        y_net = None
        if sinfo is not None and sinfo["trusted"]:
            y_net, _ = mlp.forward(sinfo["params"], mlp.features(hits.uv[idx]), round16=True)
            aud = mlp.audited(frame, idx)
            for c, (base, width) in sinfo["ordmap"].items():
                node, sock = cach[c]
                otype = graph.output_type(material, node, sock)
                eligible = ~res.found[idx, c] & ~res.bypass[idx, c]
                sm = eligible & ~aud
                res.audited[idx, c] = eligible & aud
                if not sm.any():
                    continue
                vals = y_net[:, base:base + width].copy()
                if surrogate_values is not None:
                    vals[sm] = surrogate_values[idx[sm], c, :width]
                res.surrogate[idx, c] = sm
                res.surrogate_value[idx[sm], c, :width] = vals[sm]
                res.stats["surrogate_used"] += int(sm.sum())
                prev = subst.get((node, sock))
                if prev is None:
                    prev = (np.zeros(len(idx), dtype=bool),
                            np.zeros((len(idx), 3)) if otype == "COLOR" else np.zeros(len(idx)))
                mask, full = prev
                if otype == "COLOR":
                    full[sm] = vals[sm]
                else:
                    full[sm] = vals[sm, 0]
                subst[(node, sock)] = (mask | sm, full)
        out, values = graph.evaluate(material, hits.uv[idx], hits.normal[idx], textures, subst,
                                     position=_pos(hits, idx))
        for k in res.outputs:
            res.outputs[k][idx] = out[k]
        for c, (node, sock) in enumerate(cach):
            ky = key_list[c]
            otype = graph.output_type(material, node, sock)
            v = values[(node, sock)]
            miss = np.nonzero(~res.found[idx, c] & ~ky.bypass & ~res.surrogate[idx, c])[0]
            vals = v[miss]
            fin = np.isfinite(vals) if vals.ndim == 1 else np.all(np.isfinite(vals), axis=1)
            res.stats["nonfinite"] += int((~fin).sum())
            miss, vals = miss[fin], vals[fin]
            encs = encode(vals, otype)
            for j, enc in zip(miss, encs):
                candidates.append((int(idx[j]), c, int(ky.cell[j]), int(ky.hash2[j]), int(enc),
                                   (int(ky.k0[j]), int(ky.k1[j]))))
            if surrogate_insert:
                sub_rows = np.nonzero(res.surrogate[idx, c])[0]
                if len(sub_rows):
                    sv = res.surrogate_value[idx[sub_rows], c, :3 if otype == "COLOR" else 1]
                    sv = sv if otype == "COLOR" else sv[:, 0]
                    fin = np.isfinite(sv) if sv.ndim == 1 else np.all(np.isfinite(sv), axis=1)
                    for j, enc in zip(sub_rows[fin], encode(sv[fin], otype)):
                        candidates.append((int(idx[j]), c, int(ky.cell[j]), int(ky.hash2[j]),
                                           int(enc), (int(ky.k0[j]), int(ky.k1[j]))))
            if sinfo is not None and c in sinfo["ordmap"]:
                base, width = sinfo["ordmap"][c]
                for j, val in zip(miss, vals):
                    vv = np.zeros(4)
                    vv[:width] = np.atleast_1d(val)[:width]
                    res.log.append((int(m), c, float(hits.uv[idx[j], 0]),
                                    float(hits.uv[idx[j], 1]), vv))
                if y_net is not None:
                    au = np.nonzero(res.audited[idx, c])[0]
                    if len(au):
                        g = np.asarray(v[au], dtype=np.float64).reshape(len(au), -1)[:, :width]
                        e = np.abs(g - y_net[au, base:base + width]).max()
                        res.live_err[int(m)] = max(res.live_err.get(int(m), 0.0), float(e))
    res.stats["misses"] = res.stats["probes"] - res.stats["hits"]
    res.stats["candidates"] = len(candidates)
    res.stats["false_hits"] = table.false_hits - false0
    candidates.sort(key=lambda t: (t[0], t[1]))
    bounce = getattr(hits, "bounce", None)
    for h, c, cell, h2, enc, key in candidates:
        b = int(bounce[h]) if bounce is not None else 0
        res.stats[table.insert(cell, h2, enc, policy, frame, key=key, bounce=b)] += 1
    return res


def shade_snapshot(materials, textures, frames: List, table: Table, policy: str = FIRST,
                   level_bias: int = 0, level_max: int = K.LEVEL_MAX_DEFAULT,
                   min_subgraph_nodes: int = 2, kmax: int = 8, first_frame: int = 0,
                   surrogate: Optional[dict] = None, hash2_mask: int = 0xFFFFFFFF):
    """Progressive snapshot render of a list of hit batches; returns one FrameResult each."""
    cach = [graph.cacheable_outputs(m, min_subgraph_nodes) for m in materials]
    return [shade_snapshot_frame(materials, textures, h, table, first_frame + f, policy,
                                 level_bias, level_max, min_subgraph_nodes, kmax, cach, surrogate,
                                 hash2_mask=hash2_mask)
            for f, h in enumerate(frames)]
