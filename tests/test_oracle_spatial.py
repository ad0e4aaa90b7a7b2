"""Pins of the world-position descriptors (Sec. 3.1: other shading-point
information such as the world position can key cacheable nodes): the
position-noise node at lattice points, position-class marking on hand-built
graphs, spatial keys in closed form, and the cached values of a snapshot run
against brute-force key matching."""
import numpy as np

from oracle import graph, hashing as H, keys as K, nodes as N, render, table
from paper_2305_07238_amd import scenes


def _h3(i, j, k, seed):
    sg = np.uint64(((seed & 0xFFFFFFFF) * 0x9E3779B97F4A7C15) & (2 ** 64 - 1))
    kz = H.mix64(np.uint64(k & 0xFFFFFFFF) ^ sg)
    ij = np.uint64(((i & 0xFFFFFFFF) << 32) | (j & 0xFFFFFFFF))
    return float(H.mix64(ij ^ kz) & np.uint64(0xFFFFFFFF)) * 2.0 ** -32


def test_position_noise_at_lattice_points():
    pts = [(0, 0, 0), (1, 2, 3), (-3, 4, -5), (7, -1, 2)]
    p = np.array(pts, np.float64)
    v1 = N.position_noise(p, 1.0, 1, 11)
    assert np.allclose(v1, [_h3(*q, 11) for q in pts], rtol=0, atol=1e-15)
    # two octaves on lattice points of both (frequency 1 and 2): the weighted mean
    v2 = N.position_noise(p, 1.0, 2, 11)
    want = [(_h3(*q, 11) + 0.5 * _h3(*(2 * np.array(q)), 12)) / 1.5 for q in pts]
    assert np.allclose(v2, want, rtol=0, atol=1e-15)
    # between lattice points: inside the range of the eight corners
    q = np.array([[0.3, 0.6, 0.9]])
    corners = [_h3(i, j, k, 11) for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    v = N.position_noise(q, 1.0, 1, 11)[0]
    assert min(corners) <= v <= max(corners)


def _mat(nodes):
    return scenes.Material(nodes)


def test_position_class_marking():
    Nd, L, C = scenes.Node, scenes.Input.link, scenes.Input.const
    ramp = dict(ramp_pos=tuple(np.linspace(0, 1, 8)),
                ramp_rgba=tuple((k / 7, 0.5, 0.2, 1.0) for k in range(8)))
    m = _mat([Nd("UV_INPUT"),                                               # 0
              Nd("PERLIN_NOISE", [L(0)], freq=2, octaves=1),                # 1  UV
              Nd("COLOR_RAMP", [L(1)], **ramp),                             # 2  UV
              Nd("POSITION_NOISE", [], freq=1, octaves=1, seed=3),          # 3  POS
              Nd("MATH", [L(3), C(0.5)], math_op="MUL"),                    # 4  POS
              Nd("MIX", [L(4), L(2, 0), C(0.1, 0.2, 0.3)]),                 # 5  UV|POS
              Nd("MATH", [L(4), C(0.1)], math_op="ADD", clamp=True),        # 6  POS
              Nd("BSDF_OUTPUT", [L(5), L(6), C()])])                        # 7
    cls = graph.dependency_classes(m)
    assert cls[:7] == [graph.UV, graph.UV, graph.UV, graph.POS, graph.POS,
                       graph.UV | graph.POS, graph.POS]
    # the ramp (UV) and the MUL (POS) feed the mixed MIX; the ADD (POS) feeds the
    # sink and holds the MUL: the highest POS level there is the ADD
    assert graph.cacheable_outputs(m) == [(2, 0), (4, 0), (6, 0)]
    assert [graph.key_kind(m, n) for n, _ in graph.cacheable_outputs(m)] == \
        [graph.UV, graph.POS, graph.POS]


def test_spatial_keys_closed_form():
    p = np.array([[0.5, 0.25, 0.75], [-0.5, 3.0, 1.0 / 128]], np.float32)
    w = np.array([1.0 / 64, 1.0 / 64], np.float32)
    ky = K.compute_keys_spatial(5, 3, 0, p, w, 1 << 20)
    assert list(ky.level) == [6, 6]
    assert not ky.bypass.any()
    assert list(ky.tx) == [32, -32] and list(ky.ty) == [16, 192]
    U = np.uint64
    M = (1 << 21) - 1
    k1 = (32 << 42) | (16 << 21) | 48
    assert int(ky.k1[0]) == k1
    assert int(ky.k1[1]) == (((-32) & M) << 42) | (192 << 21) | 0
    assert int(ky.k0[0]) == (5 << 32) | (3 << 16) | 0x80 | 6
    # the same node keyed by UV has another descriptor (no 0x80 flag)
    kuv = K.compute_keys(5, 3, 0, p[:, :2], np.tile(np.float32([1 / 64, 0, 0, 1 / 64]), (2, 1)),
                         1 << 20)
    assert int(kuv.k0[0]) != int(ky.k0[0])
    # cell indices wrap every 2^21 cells (a reading: 21 bits per axis in k1)
    p2 = p.copy()
    p2[0, 0] += np.float32(2 ** 21 / 64)
    ky2 = K.compute_keys_spatial(5, 3, 0, p2, w, 1 << 20)
    assert int(ky2.k1[0]) == int(ky.k1[0]) and ky2.cell[0] == ky.cell[0]
    # width 0: finest level; non-finite: bypass; beyond int32: bypass
    e = K.compute_keys_spatial(0, 1, 0, np.array([[0.1, 0.2, 0.3], [np.nan, 0, 0], [1e10, 0, 0]],
                                                 np.float32),
                               np.array([0.0, 0.1, 0.1], np.float32), 97)
    assert e.level[0] == 20 and list(e.bypass) == [False, True, True]


def test_spatial_snapshot_values_are_earlier_samples():
    """Snapshot mode on the spatial scene: every value found for a POS-class
    output in frame 1 is the encoded value of a frame-0 sample with the same
    world-space descriptor (brute force over keys); the cache disabled gives the
    uncached outputs."""
    sc = scenes.spatial_scene()
    sel = np.arange(0, sc.hits_per_frame, 8)
    f0, f1 = sc.frame(0).take(sel), sc.frame(1).take(sel)
    t = table.Table(1 << 14, 8, 16)
    r0 = render.shade_snapshot_frame(sc.materials, sc.textures, f0, t, 0)
    r1 = render.shade_snapshot_frame(sc.materials, sc.textures, f1, t, 1)
    checked = 0
    for m in np.unique(f1.material):
        mat = sc.materials[m]
        i0 = np.nonzero(f0.material == m)[0]
        i1 = np.nonzero(f1.material == m)[0]
        for c, (node, sock) in enumerate(graph.cacheable_outputs(mat)):
            if graph.key_kind(mat, node) != graph.POS:
                continue
            k0 = K.keys_for(mat, int(m), node, sock, f0, i0, t.n_cells)
            k1 = K.keys_for(mat, int(m), node, sock, f1, i1, t.n_cells)
            _, v0 = graph.evaluate(mat, f0.uv[i0], f0.normal[i0], sc.textures,
                                   position=f0.position[i0])
            otype = graph.output_type(mat, node, sock)
            dec = render.decode(render.encode(v0[(node, sock)], otype), otype)
            dec = dec.reshape(len(i0), -1)
            by_key = {}
            for j in range(len(i0)):
                by_key.setdefault((int(k0.k0[j]), int(k0.k1[j])), set()).add(tuple(dec[j]))
            w = dec.shape[1]
            for j in np.nonzero(r1.found[i1, c])[0]:
                key = (int(k1.k0[j]), int(k1.k1[j]))
                assert key in by_key
                assert tuple(r1.found_value[i1[j], c, :w]) in by_key[key]
                checked += 1
    assert checked > 1000
    unc = render.shade_uncached(sc.materials, sc.textures, f1)
    assert r0.stats["hits"] == 0 and checked > 0
    assert np.all(np.isfinite(unc["base_color"]))


def test_texel_only_marking():
    """Texel-only descriptors drop exactly the outputs of the world position
    (while the 8-output cap does not bind) and change nothing where no node
    reads the position."""
    from paper_2305_07238_amd import scenes as S
    sc = S.spatial_scene(width=96, height=48, frames=1, n_mats=24)
    for m in sc.materials:
        full = graph.cacheable_outputs(m)
        tex = graph.cacheable_outputs(m, texel_only=True)
        assert all(graph.key_kind(m, node) == graph.UV for node, _ in tex)
        if len(full) < graph.MAX_CACHEABLE:
            assert tex == [c for c in full if graph.key_kind(m, c[0]) == graph.UV]
    mid = S.mid_scene(frames=1, width=64, height=32)
    for m in mid.materials:
        assert graph.cacheable_outputs(m, texel_only=True) == graph.cacheable_outputs(m)
