"""Helpers shared by the GPU tests: run scenes through the C ABI, fetch results,
and compare them with the FP64 oracle.

Value bar (FP32 device arithmetic against FP64): a scalar channel passes when
|gpu - ref| <= 1e-5 |ref| + 1e-6, the unit normal when |gpu - ref| (Euclidean)
<= 1e-5 (``oracle.check``).  A value read from the table may also sit one
RGB9E5 step from the oracle's (COLOR codes: an FP32 input on the other side of
a rounding boundary of the encoding)."""
import numpy as np

from oracle import check, codec, graph
from paper_2305_07238_amd import scenes

RTOL, ATOL, NTOL = check.RTOL, check.ATOL, check.NTOL


def output_ratios(got, ref, rows=None):
    """Per BSDF output, the largest error in units of its bar (<= 1 passes)."""
    return check.output_ratios(got, ref, rows)


def assert_outputs(got, ref, rows=None, what=""):
    r = output_ratios(got, ref, rows)
    assert all(q <= 1.0 for q in r.values()), (what, r)
    return r


def scalar_ok(got, ref):
    return check.scalar_ratio(got, ref) <= 1.0


def max_abs(gpu, ref):
    d = np.abs(np.asarray(gpu, np.float64) - np.asarray(ref, np.float64))
    return float(np.nanmax(d)) if d.size else 0.0


def setup(scene, device=0, **compile_kw):
    from paper_2305_07238_amd import binding as B
    ctx = B.Context(device)
    ctx.set_textures(scene.textures)
    ctx.compile(scene.materials, **compile_kw)
    return ctx


def to_numpy(out):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in out.items()}


def shade(ctx, hits_np, cache=None, debug=False, **kw):
    """Shade a numpy Hits batch; returns (outputs numpy, state, value, stats dict)."""
    import torch
    from paper_2305_07238_amd import binding as B
    n = len(hits_np)
    hits = B.hits_to_device(hits_np)
    out = B.alloc_outputs(n)
    stats = B.new_stats()
    dbg = None
    if debug:
        dbg = {"state": torch.full((n, 8), 255, dtype=torch.uint8, device="cuda"),
               "value": torch.full((n, 8, 3), float("nan"), dtype=torch.float32, device="cuda")}
    ctx.shade(hits, out, cache, stats=stats, debug=dbg, **kw)
    torch.cuda.synchronize()
    res = to_numpy(out)
    st = B.stats_dict(stats)
    if debug:
        return res, dbg["state"].cpu().numpy(), dbg["value"].cpu().numpy(), st
    return res, None, None, st


def small_mid_scene(seed=0, frames=2, **kw):
    """The mid workload's material set (64 graphs of 8-64 nodes, 16 textures of
    1024^2) on a 480 x 240 screen: spans many waves and every material class."""
    return scenes.mid_scene(seed=seed, width=480, height=240, frames=frames, **kw)


def crossed_chains(n_tex):
    """n_tex textures read by a forward MIX chain and again by a reverse one:
    whichever texture any order computes last, every texture is still awaited
    by one of the chains then, so at least 3 n_tex registers are live
    (3 n_tex + 6 as compiled).  Textures 0-3 of the scene."""
    N, L, Cn = scenes.Node, scenes.Input.link, scenes.Input.const
    nodes = [N("UV_INPUT")] + [N("IMAGE_TEXTURE", [L(0)], texture=t % 4) for t in range(n_tex)]
    fwd = 1
    for t in range(2, n_tex + 1):
        nodes.append(N("MIX", [Cn(0.5), L(fwd), L(t)]))
        fwd = len(nodes) - 1
    rev = n_tex
    for t in range(n_tex - 1, 0, -1):
        nodes.append(N("MIX", [Cn(0.25), L(rev), L(t)]))
        rev = len(nodes) - 1
    nodes.append(N("MIX", [Cn(0.5), L(fwd), L(rev)]))
    nodes.append(N("BSDF_OUTPUT", [L(len(nodes) - 1), Cn(0.5), Cn()]))
    return scenes.Material(nodes)


def found_values_parity(materials, hits, state, value, ref_found_value, min_subgraph_nodes=2,
                        cacheables=None):
    """Values the device found in the table against the oracle's found values:
    COLOR within one RGB9E5 step of the oracle's decoded code, FLOAT at the
    scalar bar.  Returns the number of (hit, ordinal) pairs compared."""
    mat = hits.material.astype(np.int64)
    n_cmp = 0
    for m in np.unique(mat):
        if m >= len(materials):
            continue
        idx = np.nonzero(mat == m)[0]
        cach = (cacheables[m] if cacheables is not None
                else graph.cacheable_outputs(materials[m], min_subgraph_nodes))
        for c, (node, sock) in enumerate(cach):
            rows = idx[state[idx, c] == 1]
            if len(rows) == 0:
                continue
            n_cmp += len(rows)
            ref = ref_found_value[rows, c]
            got = value[rows, c]
            if graph.output_type(materials[m], node, sock) == "COLOR":
                step = codec.rgb9e5_step(codec.rgb9e5_encode(ref))
                assert np.all(np.abs(got - ref) <= step[:, None] * 1.0001), (m, c)
            else:
                assert scalar_ok(got[:, 0], ref[:, 0]), (m, c, max_abs(got[:, 0], ref[:, 0]))
    return n_cmp


def substituted_outputs(materials, textures, hits, state, value, min_subgraph_nodes=2,
                        states=(1,), cacheables=None):
    """FP64 evaluation of every hit with the device's values substituted at the
    cacheable outputs whose state is in ``states`` (1 = found in the table,
    4 = supplied by a network)."""
    n = len(hits)
    out = dict(base_color=np.zeros((n, 3)), roughness=np.zeros(n), normal=np.zeros((n, 3)))
    mat = hits.material.astype(np.int64)
    for m in np.unique(mat):
        idx = np.nonzero(mat == m)[0]
        if m >= len(materials):
            o = graph.default_outputs(hits.normal[idx])
        else:
            subst = {}
            cach = (cacheables[m] if cacheables is not None
                    else graph.cacheable_outputs(materials[m], min_subgraph_nodes))
            for c, (node, sock) in enumerate(cach):
                rows = np.isin(state[idx, c], states)
                if rows.any():
                    if graph.output_type(materials[m], node, sock) == "COLOR":
                        v = value[idx, c, :3].astype(np.float64)
                    else:
                        v = value[idx, c, 0].astype(np.float64)
                    subst[(node, sock)] = (rows, v)
            pos = None if getattr(hits, "position", None) is None else hits.position[idx]
            o, _ = graph.evaluate(materials[m], hits.uv[idx], hits.normal[idx], textures, subst,
                                  position=pos)
        for k in out:
            out[k][idx] = o[k]
    return out


def table_parity(gpu_words, ref, materials):
    """Snapshot tables: hash halves, positions, stamps and the aux field
    bit-exact; value codes that differ are within one RGB9E5 step (COLOR) or
    the scalar bar (FLOAT).  Returns the number of differing value codes."""
    gw = gpu_words[:, 0]
    rw = ref.words()
    assert np.array_equal(gw >> np.uint64(32), rw >> np.uint64(32))
    if gpu_words.shape[1] == 2:
        stamps = (gpu_words[:, 1] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        assert np.array_equal(stamps, ref.stamps())
        assert np.array_equal((gpu_words[:, 1] >> np.uint64(32)).astype(np.uint32), ref.auxes())
    diff = np.nonzero(gw != rw)[0]
    for i in diff:
        k0 = ref.key[int(i)][0]
        m, node, sock = k0 >> 32, (k0 >> 16) & 0xFFFF, (k0 >> 8) & 0xFF
        g = np.uint64(gw[i] & np.uint64(0xFFFFFFFF))
        r = np.uint64(rw[i] & np.uint64(0xFFFFFFFF))
        if graph.output_type(materials[m], node, sock) == "COLOR":
            gv = codec.rgb9e5_decode(np.array([g]))[0]
            rv = codec.rgb9e5_decode(np.array([r]))[0]
            step = codec.rgb9e5_step(np.array([r]))[0]
            assert np.all(np.abs(gv - rv) <= step * 1.0001), (int(i), gv, rv)
        else:
            gv = codec.float_decode(np.array([g]))[0]
            rv = codec.float_decode(np.array([r]))[0]
            assert scalar_ok(gv, rv), (int(i), gv, rv)
    return len(diff)
