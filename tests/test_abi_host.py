"""Host-side checks of the C ABI: exports, struct layouts, and the graph
compiler (host-only context, no GPU) against the oracle's independent
cacheable marking."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import graph
from paper_2305_07238_amd import binding as B
from paper_2305_07238_amd import scenes
from tests import gpu_util as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pmc_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(B.lib, n), n
        assert n in B.EXPORTED, f"binding lacks {n}"


def test_struct_layouts_match_the_header():
    assert B.pmc_abi_version() == 6
    for i, st in enumerate([B.pmc_node_desc, B.pmc_input, B.pmc_texture_desc, B.pmc_compile_opts,
                            B.pmc_material_info, B.pmc_cache_params, B.pmc_shade_params,
                            B.pmc_stats, B.pmc_hits, B.pmc_bsdf_out, B.pmc_debug_out,
                            B.pmc_key_record, B.pmc_frame_plan, B.pmc_tune_result,
                            B.pmc_profile, B.pmc_surrogate_opts, B.pmc_surrogate_slot,
                            None, B.pmc_train_params, B.pmc_surrogate_stat,
                            B.pmc_cone_hits]):
        if st is None:                      # pmc_log_record: 32 bytes, numpy dtype
            assert B.pmc_abi_sizeof(i) == B.LOG_RECORD_DTYPE.itemsize == 32
            continue
        assert B.pmc_abi_sizeof(i) == C.sizeof(st), st.__name__
    assert B.pmc_abi_sizeof(99) == 0
    assert C.sizeof(B.pmc_node_desc) == 244
    assert C.sizeof(B.pmc_stats) == 256
    assert C.sizeof(B.pmc_surrogate_stat) == 48


def test_host_only_context_refuses_device_work():
    ctx = B.Context(-1)
    with pytest.raises(B.PmcError) as e:
        ctx.set_textures([np.zeros((4, 4, 4), np.uint8)])
    assert e.value.code == B.PMC_ERR_STATE
    ctx.close()


def _compile(mats, **kw):
    ctx = B.Context(-1)
    ctx.compile(mats, **kw)
    return ctx


def test_compiler_marking_matches_oracle_tiny():
    m = scenes.tiny_material()
    ctx = _compile([m])
    assert ctx.cacheables(0) == graph.cacheable_outputs(m) == [(4, 0), (6, 0)]
    info = ctx.material_info(0)
    assert info.n_nodes == 8 and info.n_live == 8 and info.n_folded == 0
    assert info.n_instr == 6                       # UV input and sink are not instructions
    assert list(info.cacheable_type)[:2] == [1, 0]  # ramp colour (RGB9E5), roughness (float)
    assert list(info.subgraph_nodes)[:2] == [4, 6]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_compiler_marking_matches_oracle_random(seed):
    sc = scenes.mid_scene(seed=seed, width=120, height=120, frames=1, tex_size=8)
    ctx = _compile(sc.materials)
    for mi, m in enumerate(sc.materials):
        assert ctx.cacheables(mi) == graph.cacheable_outputs(m), mi
        info = ctx.material_info(mi)
        assert info.n_regs <= 64
        assert info.n_live == sum(graph.reachable(m))


def test_large_networks_fit_the_register_file():
    sc_rng = np.random.default_rng(5)
    mats = [scenes.random_material(sc_rng, 400, 4) for _ in range(20)]
    ctx = _compile(mats)
    for mi in range(len(mats)):
        assert ctx.cacheables(mi) == graph.cacheable_outputs(mats[mi])
        assert ctx.material_info(mi).n_regs <= 64
    # the order search (materials above 24 registers) is deterministic: a second
    # compile in a new context gives the same register counts
    regs = [ctx.material_info(mi).n_regs for mi in range(len(mats))]
    assert max(regs) > 24
    ctx2 = _compile(mats)
    assert [ctx2.material_info(mi).n_regs for mi in range(len(mats))] == regs


def test_constant_folding_and_min_subgraph_option():
    N, L, Cn = scenes.Node, scenes.Input.link, scenes.Input.const
    m = scenes.Material([
        N("UV_INPUT"),
        N("MATH", [Cn(0.25), Cn(0.5)], math_op="ADD"),                  # folds to 0.75
        N("MATH", [L(1), Cn(2.0)], math_op="MUL", clamp=True),          # folds to 1.0
        N("PERLIN_NOISE", [L(0)], freq=4, octaves=2, seed=3),
        N("MIX", [L(2), L(3, 0), Cn(0.1, 0.2, 0.3)]),
        N("BSDF_OUTPUT", [L(4), L(3), Cn()]),
    ])
    ctx = _compile([m])
    info = ctx.material_info(0)
    assert info.n_folded == 2 and info.n_instr == 2
    assert ctx.cacheables(0) == graph.cacheable_outputs(m) == [(4, 0)]
    ctx2 = _compile([m], no_fold=True)
    assert ctx2.material_info(0).n_instr == 4
    ctx3 = _compile([m], min_subgraph_nodes=1)
    assert ctx3.cacheables(0) == graph.cacheable_outputs(m, 1) == [(3, 0), (4, 0)]


def test_a_result_takes_the_register_its_operand_frees():
    """A chain noise -> 8 MATH nodes -> roughness: each MATH node reads the one
    before it for the last time, so its result can take that register (the
    interpreter reads all operands before it writes).  The chain's end is the
    cacheable output, held from the start for a found value: two registers in
    all, where a rule that keeps the operand's register busy through its last
    reader needs three."""
    N, L, Cn = scenes.Node, scenes.Input.link, scenes.Input.const
    nodes = [N("UV_INPUT"), N("PERLIN_NOISE", [L(0)], freq=4, octaves=2, seed=3)]
    for k in range(8):
        nodes.append(N("MATH", [L(len(nodes) - 1), Cn(0.5 + k)], math_op="ADD" if k % 2 else "MUL"))
    nodes.append(N("BSDF_OUTPUT", [Cn(0.2, 0.3, 0.4), L(len(nodes) - 1), Cn()]))
    m = scenes.Material(nodes)
    ctx = _compile([m])
    assert ctx.cacheables(0) == graph.cacheable_outputs(m) == [(9, 0)]
    info = ctx.material_info(0)
    assert info.n_instr == 9 and info.n_regs == 2


def test_register_need_beyond_the_limit_is_refused():
    ctx = _compile([G.crossed_chains(16)])
    assert 48 <= ctx.material_info(0).n_regs <= 64
    ctx.close()
    ctx = B.Context(-1)
    with pytest.raises(B.PmcError) as e:
        ctx.compile([G.crossed_chains(24)])
    assert e.value.code == B.PMC_ERR_UNSUPPORTED
    assert "registers" in str(e.value)
    ctx.compile([scenes.tiny_material()])      # the context stays usable
    assert ctx.material_info(0).n_regs > 0
    ctx.close()


@pytest.mark.parametrize("bad", ["cycle", "type", "no_sink", "link", "ramp"])
def test_compiler_rejects_bad_graphs(bad):
    N, L, Cn = scenes.Node, scenes.Input.link, scenes.Input.const
    pos = tuple(np.linspace(0, 1, 8))
    rgba = tuple((0.5, 0.5, 0.5, 1.0) for _ in range(8))
    if bad == "cycle":
        nodes = [N("MATH", [L(1), Cn(1)]), N("MATH", [L(0), Cn(1)]), N("BSDF_OUTPUT", [Cn(), L(0), Cn()])]
    elif bad == "type":
        nodes = [N("UV_INPUT"), N("MATH", [L(0), Cn(1)]), N("BSDF_OUTPUT", [Cn(), L(1), Cn()])]
    elif bad == "no_sink":
        nodes = [N("UV_INPUT")]
    elif bad == "link":
        nodes = [N("UV_INPUT"), N("BSDF_OUTPUT", [L(7), Cn(), Cn()])]
    else:
        nodes = [N("COLOR_RAMP", [Cn(0.5)], ramp_pos=pos[::-1], ramp_rgba=rgba),
                 N("BSDF_OUTPUT", [L(0), Cn(), Cn()])]
    ctx = B.Context(-1)
    with pytest.raises(B.PmcError) as e:
        ctx.compile([scenes.Material(nodes)])
    assert e.value.code == B.PMC_ERR_GRAPH
    assert "material 0" in str(e.value)


def test_surrogate_slots_follow_the_subgraph_rule():
    """Slot selection on a host-only context: outputs whose sub-graph (UV inputs
    excluded, as the oracle counts it) has more than 32 nodes, packed in
    ordinal order into 4 channels (COLOR 3, FLOAT 1)."""
    sc = scenes.mid_scene(frames=1, width=64, height=32)
    ctx = _compile(sc.materials)
    n = ctx.surrogate_setup()
    expect = []
    for m, mat in enumerate(sc.materials):
        mask, chans, used = 0, {}, 0
        for c, (node, sock) in enumerate(graph.cacheable_outputs(mat)):
            size = sum(1 for j in graph.subgraph(mat, node) if mat.nodes[j].op != "UV_INPUT")
            w = 3 if graph.output_type(mat, node, sock) == "COLOR" else 1
            if size > 32 and used + w <= 4:
                mask |= 1 << c
                chans[c] = used
                used += w
        if mask:
            expect.append((m, mask, chans, used))
    assert n == len(expect) > 0
    for k, (m, mask, chans, used) in enumerate(expect):
        sl = ctx.surrogate_slot(k)
        assert sl["material"] == m and sl["ordinal_mask"] == mask and sl["n_channels"] == used
        for c, ch in chans.items():
            assert sl["channel"][c] == ch
    ctx.close()


def test_compiler_marks_world_keyed_outputs_like_the_oracle():
    """Graphs with POSITION_NOISE leaves: the same cacheable outputs as the
    oracle, keyed by a world cell exactly where the oracle's dependency class
    is the world position, and no surrogate network over such an output."""
    sc = scenes.spatial_scene(width=96, height=48, frames=1, n_mats=24)
    ctx = _compile(sc.materials)
    kinds = set()
    for mi, m in enumerate(sc.materials):
        cach = graph.cacheable_outputs(m)
        assert ctx.cacheables(mi) == cach, mi
        info = ctx.material_info(mi)
        want = [1 if graph.key_kind(m, node) == graph.POS else 0 for node, _ in cach]
        assert list(info.cacheable_key)[:len(cach)] == want, mi
        kinds.update(want)
    assert kinds == {0, 1}
    n = ctx.surrogate_setup()
    for k in range(n):
        sl = ctx.surrogate_slot(k)
        key = list(ctx.material_info(sl.material).cacheable_key)
        assert all(key[c] == 0 for c in range(8) if (sl.ordinal_mask >> c) & 1)


def test_texel_keys_only_drops_the_world_keyed_outputs():
    """With descriptors restricted to UV texels, the outputs of the world
    position are not cached; the UV-keyed ones stay (where the 8-output cap
    did not cut the list)."""
    sc = scenes.spatial_scene(width=96, height=48, frames=1, n_mats=24)
    ctx = _compile(sc.materials)
    ctx2 = B.Context(-1)
    ctx2.compile(sc.materials, texel_keys_only=True)
    dropped = 0
    for mi, m in enumerate(sc.materials):
        cach = graph.cacheable_outputs(m)
        uv_only = [c for c in cach if graph.key_kind(m, c[0]) != graph.POS]
        info = ctx2.material_info(mi)
        assert list(info.cacheable_key)[:info.n_cacheable] == [0] * info.n_cacheable
        assert ctx2.cacheables(mi) == graph.cacheable_outputs(m, texel_only=True), mi
        if len(cach) < 8:
            assert ctx2.cacheables(mi) == uv_only, mi
        dropped += len(cach) - len(uv_only)
    assert dropped > 0
