"""Seeded synthetic scenes: material graph sets, textures and per-frame hit batches.

This module only produces inputs.  It contains none of the caching method's
arithmetic (no node evaluation, no key quantisation, no hashing of
descriptors, no encoding): both the HIP path and the CPU oracle consume what
it returns.  Every random draw goes through ``numpy.random.default_rng`` with
an explicit seed sequence, so a (config, purpose, frame) triple always yields
the same bytes.

The paper's production scenes are not available; the workloads below stand in
for them with the shapes the paper describes: thousands of node-based
materials, networks of up to a few hundred nodes (Sec. 2), 1920x1080 frames
rendered progressively at one sample per pixel per pass (Sec. 4).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# graph data model (plain data; the C-ABI mirrors it in pmc_node_desc)
# ----------------------------------------------------------------------------

OPS = ("UV_INPUT", "IMAGE_TEXTURE", "VALUE_NOISE", "PERLIN_NOISE", "MIX",
       "MATH", "COLOR_RAMP", "NORMAL_MAP", "BSDF_OUTPUT", "POSITION_NOISE")
MATH_OPS = ("ADD", "MUL", "POW")

# socket types of each op: inputs and outputs
IN_TYPES = {
    "UV_INPUT": (),
    "IMAGE_TEXTURE": ("UV",),
    "VALUE_NOISE": ("UV",),
    "PERLIN_NOISE": ("UV",),
    "MIX": ("FLOAT", "COLOR", "COLOR"),
    "MATH": ("FLOAT", "FLOAT"),
    "COLOR_RAMP": ("FLOAT",),
    "NORMAL_MAP": ("COLOR", "FLOAT"),
    "BSDF_OUTPUT": ("COLOR", "FLOAT", "VECTOR"),
    "POSITION_NOISE": (),
}
OUT_TYPES = {
    "UV_INPUT": ("UV",),
    "IMAGE_TEXTURE": ("COLOR", "FLOAT"),
    "VALUE_NOISE": ("FLOAT",),
    "PERLIN_NOISE": ("FLOAT",),
    "MIX": ("COLOR",),
    "MATH": ("FLOAT",),
    "COLOR_RAMP": ("COLOR", "FLOAT"),
    "NORMAL_MAP": ("VECTOR",),
    "BSDF_OUTPUT": (),
    "POSITION_NOISE": ("FLOAT",),
}


@dataclasses.dataclass
class Input:
    """One input socket: a link to (node, socket) of the same material, or a constant."""
    node: int = -1                      # -1 = unconnected (use ``value``)
    socket: int = 0
    value: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @staticmethod
    def link(node: int, socket: int = 0) -> "Input":
        return Input(node=node, socket=socket)

    @staticmethod
    def const(*v: float) -> "Input":
        vals = tuple(float(x) for x in v) + (0.0,) * (3 - len(v))
        return Input(node=-1, socket=0, value=vals[:3])


@dataclasses.dataclass
class Node:
    op: str
    inputs: List[Input] = dataclasses.field(default_factory=list)
    math_op: str = "ADD"                # MATH
    clamp: bool = False                 # MATH
    texture: int = 0                    # IMAGE_TEXTURE: index into the scene's texture list
    freq: float = 0.0                   # noise base frequency f0
    octaves: int = 1                    # noise octave count
    seed: int = 0                       # noise seed
    ramp_pos: Tuple[float, ...] = ()    # COLOR_RAMP: 8 ascending positions
    ramp_rgba: Tuple[Tuple[float, float, float, float], ...] = ()  # COLOR_RAMP: 8 stops


@dataclasses.dataclass
class Material:
    nodes: List[Node]

    @property
    def sink(self) -> int:
        return next(i for i, n in enumerate(self.nodes) if n.op == "BSDF_OUTPUT")


@dataclasses.dataclass
class Hits:
    """A batch of shading points (structure of arrays, host memory)."""
    material: np.ndarray                # uint32 [n]
    uv: np.ndarray                      # float32 [n, 2]
    duv: np.ndarray                     # float32 [n, 4]: g1.x, g1.y, g2.x, g2.y
    normal: np.ndarray                  # float32 [n, 3]
    bounce: Optional[np.ndarray] = None  # uint32 [n]: path depth of the hit (0 = camera ray)
    position: Optional[np.ndarray] = None  # float32 [n, 3]: world position
    width: Optional[np.ndarray] = None     # float32 [n]: world-space footprint width

    OPTIONAL = ("bounce", "position", "width")

    def __len__(self) -> int:
        return int(self.material.shape[0])

    def take(self, idx) -> "Hits":
        opt = {k: (None if getattr(self, k) is None else getattr(self, k)[idx])
               for k in self.OPTIONAL}
        return Hits(self.material[idx], self.uv[idx], self.duv[idx], self.normal[idx], **opt)

    @staticmethod
    def concat(parts: Sequence["Hits"]) -> "Hits":
        opt = {}
        for k in Hits.OPTIONAL:
            if all(getattr(p, k) is None for p in parts):
                opt[k] = None
            elif k == "bounce":
                opt[k] = np.concatenate([p.bounce if p.bounce is not None
                                         else np.zeros(len(p), np.uint32) for p in parts])
            else:
                opt[k] = np.concatenate([getattr(p, k) for p in parts])
        return Hits(np.concatenate([p.material for p in parts]),
                    np.concatenate([p.uv for p in parts]),
                    np.concatenate([p.duv for p in parts]),
                    np.concatenate([p.normal for p in parts]), **opt)


@dataclasses.dataclass
class CacheConfig:
    slots: int                          # N_c * N_e
    n_entries: int = 8                  # N_e
    entry_bytes: int = 16
    policy: str = "FIRST"               # FIRST (keep first value) or OVERWRITE

    @property
    def n_cells(self) -> int:
        return self.slots // self.n_entries


@dataclasses.dataclass
class Scene:
    name: str
    materials: List[Material]
    textures: List[np.ndarray]          # each uint8 [H, W, 4] (RGBA8, row 0 at v = 0)
    frames: int
    hits_per_frame: int
    cache: CacheConfig
    seed: int
    _frame_fn: object = dataclasses.field(repr=False, default=None)
    layout: Optional[dict] = None       # _object_screen arguments of the screen layout

    def frame(self, f: int) -> Hits:
        """Hits of progressive pass ``f`` (deterministic)."""
        return self._frame_fn(f)

    def all_hits(self) -> Hits:
        return Hits.concat([self.frame(f) for f in range(self.frames)])


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(k) & 0xFFFFFFFF for k in key]))


# purpose tags for seed sequences
_P_GRAPH, _P_TEX, _P_OBJ, _P_JITTER, _P_MLP, _P_BOUNCE = 1, 2, 3, 4, 5, 6


# ----------------------------------------------------------------------------
# tiny scene: one 8-node material, 64x64 px x 4 spp
# ----------------------------------------------------------------------------

def checker_texture(size: int = 256, block_shift: int = 5) -> np.ndarray:
    """Grey checker: 230 where ((x>>5) ^ (y>>5)) is odd, else 26; alpha 255."""
    y, x = np.mgrid[0:size, 0:size]
    on = ((x >> block_shift) ^ (y >> block_shift)) & 1
    img = np.empty((size, size, 4), np.uint8)
    img[..., :3] = np.where(on, 230, 26)[..., None]
    img[..., 3] = 255
    return img


def _ramp_stops(rng: np.random.Generator, min_gap: float = 0.08, max_slope=1.5):
    """8 ascending stops (first at 0, last at 1) whose colours change smoothly.

    Each colour step is bounded by ``max_slope`` times the position gap, which
    keeps the ramp's Lipschitz constant small (FP32 vs FP64 round-off is not
    amplified by steep ramps).  ``max_slope=None`` draws every stop colour
    independently in [0, 1] (steep ramps where stops are close)."""
    while True:
        inner = np.sort(rng.uniform(0.0, 1.0, 6))
        pos = np.concatenate([[0.0], inner, [1.0]])
        if np.all(np.diff(pos) >= min_gap):
            break
    rgba = np.empty((8, 4))
    rgba[0] = rng.uniform(0.1, 0.9, 4)
    if max_slope is None:
        rgba = rng.uniform(0.0, 1.0, (8, 4))
    for k in range(1, 8 if max_slope is not None else 1):
        step = rng.uniform(-1, 1, 4) * max_slope * (pos[k] - pos[k - 1])
        rgba[k] = np.clip(rgba[k - 1] + step, 0.0, 1.0)
    pos32 = tuple(float(np.float32(p)) for p in pos)
    rgba32 = tuple(tuple(float(np.float32(c)) for c in row) for row in rgba)
    return pos32, rgba32


def tiny_material(seed: int = 0) -> Material:
    rng = _rng(seed, _P_GRAPH, 1)
    pos, rgba = _ramp_stops(rng)
    L, C = Input.link, Input.const
    nodes = [
        Node("UV_INPUT"),                                                      # n0
        Node("IMAGE_TEXTURE", [L(0)], texture=0),                              # n1 checker
        Node("VALUE_NOISE", [L(0)], freq=8.0, octaves=2, seed=7),             # n2
        Node("MIX", [L(2, 0), L(1, 0), C(0.9, 0.6, 0.2)]),                     # n3
        Node("COLOR_RAMP", [L(3, 0)], ramp_pos=pos, ramp_rgba=rgba),          # n4
        Node("MATH", [L(4, 1), C(0.9)], math_op="MUL", clamp=True),           # n5
        Node("MATH", [L(5, 0), C(0.05)], math_op="ADD", clamp=True),          # n6
        Node("BSDF_OUTPUT", [L(4, 0), L(6, 0), C()]),                         # n7
    ]
    return Material(nodes)


def tiny_scene(seed: int = 0, px: int = 64, spp: int = 4, slots: int = 1 << 16) -> Scene:
    """1 material, 8 nodes, px x px pixels x spp samples (sample-major: frame = sample)."""
    mat = tiny_material(seed)
    tex = [checker_texture(256)]

    def frame(f: int) -> Hits:
        rng = _rng(seed, _P_JITTER, 1, f)
        r = rng.integers(0, 1 << 16, size=(px, px, 2), dtype=np.int64)
        py, pxx = np.mgrid[0:px, 0:px]
        # u = (px + r * 2^-16) / px: exact in float32 (23 fractional bits suffice)
        u = (pxx + r[..., 0] / 65536.0) / px
        v = (py + r[..., 1] / 65536.0) / px
        n = px * px
        uv = np.stack([u.ravel(), v.ravel()], 1).astype(np.float32)
        duv = np.tile(np.array([1.0 / px, 0.0, 0.0, 1.0 / px], np.float32), (n, 1))
        normal = np.tile(np.array([0.0, 0.0, 1.0], np.float32), (n, 1))
        return Hits(np.zeros(n, np.uint32), uv, duv, normal)

    return Scene("tiny", [mat], tex, spp, px * px, CacheConfig(slots), seed, frame)


# ----------------------------------------------------------------------------
# random material networks
# ----------------------------------------------------------------------------

# target mix of body node types (the paper's networks are Blender-like node
# graphs; these proportions are this workload's stand-in)
_BODY_MIX = (("IMAGE_TEXTURE", 0.20), ("PERLIN_NOISE", 0.20), ("MIX", 0.20),
             ("MATH", 0.25), ("COLOR_RAMP", 0.10), ("VALUE_NOISE", 0.05))
_LEAVES = ("IMAGE_TEXTURE", "PERLIN_NOISE", "VALUE_NOISE")
_INNER = ("MIX", "MATH", "COLOR_RAMP")


# Constant ranges of the random networks.  "narrow" (the default of every
# workload) keeps ramps gentle (stop gaps >= 0.08, colour slope <= 1.5) and
# MATH constants at MUL in [0.5, 1], POW in [1, 2]; "wide" draws ramps with
# stop gaps >= 1e-3 and independent stop colours, MUL in [0.5, 1.5] and POW in
# [0.5, 2].  Wide ramps can be steep (slope up to ~1/gap), which amplifies the
# difference between FP32 and FP64 evaluation of their input.
RANGES = {
    "narrow": dict(ramp_gap=0.08, ramp_slope=1.5,
                   math={"ADD": (0.0, 0.5), "MUL": (0.5, 1.0), "POW": (1.0, 2.0)}),
    "wide": dict(ramp_gap=1e-3, ramp_slope=None,
                 math={"ADD": (0.0, 0.5), "MUL": (0.5, 1.5), "POW": (0.5, 2.0)}),
}


def random_material(rng: np.random.Generator, n_nodes: int, n_textures: int,
                    p_normal_map: float = 0.5, p_share: float = 0.15,
                    ranges: str = "narrow", p_position: float = 0.0) -> Material:
    """A random node network with exactly ``n_nodes`` nodes, all reachable from the sink.

    Built top-down from the BSDF sink: every open input slot is filled by a new
    node while the node budget lasts, else by an existing node created later
    than the slot's owner (sharing, which keeps the graph acyclic) or a
    constant.  The creation order reversed is a topological order, so the
    returned node list has every input before its consumers (UV_INPUT first,
    BSDF_OUTPUT last)."""
    n_nodes = max(int(n_nodes), 4)
    budget = n_nodes - 2                        # minus UV_INPUT and the sink
    created: List[dict] = []                    # creation order; index = creation id

    def new(op, **kw):
        created.append(dict(op=op, slots={}, **kw))
        return len(created) - 1

    sink = new("BSDF_OUTPUT")
    open_slots: List[Tuple[int, int]] = [(sink, 0), (sink, 1)]
    if budget >= 3 and rng.random() < p_normal_map:
        nm = new("NORMAL_MAP", strength=float(np.float32(rng.uniform(0.5, 1.0))))
        budget -= 1
        created[sink]["slots"][2] = ("node", nm, 0)
        open_slots.append((nm, 0))
    else:
        created[sink]["slots"][2] = ("const", (0.0, 0.0, 0.0))

    types = [t for t, _ in _BODY_MIX]
    probs = np.array([p for _, p in _BODY_MIX])
    probs = probs / probs.sum()
    inner_probs = np.array([p for t, p in _BODY_MIX if t in _INNER])
    inner_probs = inner_probs / inner_probs.sum()
    leaf_probs = np.array([p for t, p in _BODY_MIX if t in _LEAVES])
    leaf_probs = leaf_probs / leaf_probs.sum()

    def make_node(op):
        kw = {}
        if p_position > 0.0 and op in _LEAVES and rng.random() < p_position:
            op = "POSITION_NOISE"                   # a leaf reading the world position
            kw["freq"] = float(rng.choice([0.5, 1.0, 2.0, 4.0]))
            kw["octaves"] = 2
            kw["seed"] = int(rng.integers(0, 1 << 30))
        elif op == "IMAGE_TEXTURE":
            kw["texture"] = int(rng.integers(0, n_textures))
        elif op in ("PERLIN_NOISE", "VALUE_NOISE"):
            kw["freq"] = float(rng.choice([2.0, 4.0, 8.0, 16.0]))
            kw["octaves"] = 4 if op == "PERLIN_NOISE" else 2
            kw["seed"] = int(rng.integers(0, 1 << 30))
        elif op == "MATH":
            mop = str(rng.choice(MATH_OPS))
            lo, hi = RANGES[ranges]["math"][mop]
            kw["math_op"] = mop
            kw["b"] = float(np.float32(rng.uniform(lo, hi)))
        elif op == "COLOR_RAMP":
            kw["ramp"] = _ramp_stops(rng, RANGES[ranges]["ramp_gap"], RANGES[ranges]["ramp_slope"])
        idx = new(op, **kw)
        if op == "MIX":
            open_slots.extend([(idx, 0), (idx, 1), (idx, 2)])
        elif op in ("MATH", "COLOR_RAMP"):
            open_slots.append((idx, 0))
        return idx

    def out_socket(op):
        if op in ("IMAGE_TEXTURE", "COLOR_RAMP"):
            return int(rng.random() < 0.3)          # mostly colour, sometimes alpha
        return 0

    while open_slots:
        k = int(rng.integers(0, len(open_slots)))
        owner, slot = open_slots.pop(k)
        later = [i for i in range(owner + 1, len(created))
                 if created[i]["op"] not in ("BSDF_OUTPUT", "NORMAL_MAP")]
        if budget > 0:
            if later and open_slots and rng.random() < p_share:
                src = int(rng.choice(later))
                created[owner]["slots"][slot] = ("node", src, out_socket(created[src]["op"]))
                continue
            if len(open_slots) == 0 and budget > 1:
                op = str(rng.choice(_INNER, p=inner_probs))     # keep the graph growing
            elif len(open_slots) >= budget:
                op = str(rng.choice(_LEAVES, p=leaf_probs))     # close slots in time
            else:
                op = str(rng.choice(types, p=probs))
            budget -= 1
            src = make_node(op)
            created[owner]["slots"][slot] = ("node", src, out_socket(created[src]["op"]))
        else:
            if later and rng.random() < 0.7:
                src = int(rng.choice(later))
                created[owner]["slots"][slot] = ("node", src, out_socket(created[src]["op"]))
            else:
                created[owner]["slots"][slot] = ("const", tuple(
                    float(np.float32(x)) for x in rng.uniform(0.1, 0.9, 3)))
    uv_id = new("UV_INPUT")

    # reverse creation order -> topological order
    n = len(created)
    order = list(range(n - 1, -1, -1))
    remap = {c: i for i, c in enumerate(order)}
    nodes: List[Node] = []
    for c in order:
        d = created[c]
        op = d["op"]
        if op in ("IMAGE_TEXTURE", "PERLIN_NOISE", "VALUE_NOISE"):
            ins = [Input.link(remap[uv_id], 0)]
        elif op in ("UV_INPUT", "POSITION_NOISE"):
            ins = []
        else:
            n_in = len(IN_TYPES[op])
            ins = []
            for s in range(n_in):
                sv = d["slots"].get(s)
                if op == "MATH" and s == 1:
                    ins.append(Input.const(d["b"]))
                elif op == "NORMAL_MAP" and s == 1:
                    ins.append(Input.const(d["strength"]))
                elif sv is None:
                    ins.append(Input.const(0.5, 0.5, 0.5))
                elif sv[0] == "node":
                    ins.append(Input.link(remap[sv[1]], sv[2]))
                else:
                    ins.append(Input.const(*sv[1]))
        node = Node(op, ins)
        if op == "IMAGE_TEXTURE":
            node.texture = d["texture"]
        elif op in ("PERLIN_NOISE", "VALUE_NOISE", "POSITION_NOISE"):
            node.freq, node.octaves, node.seed = d["freq"], d["octaves"], d["seed"]
        elif op == "MATH":
            node.math_op, node.clamp = d["math_op"], True
        elif op == "COLOR_RAMP":
            node.ramp_pos, node.ramp_rgba = d["ramp"]
        nodes.append(node)
    assert nodes[-1].op == "BSDF_OUTPUT" and nodes[0].op == "UV_INPUT"
    return Material(nodes)


def texture_pool(seed: int, count: int, size: int = 1024) -> List[np.ndarray]:
    """Procedural RGBA8 textures: checkers, stripes and blocky random noise."""
    pool = []
    y, x = np.mgrid[0:size, 0:size]
    for t in range(count):
        rng = _rng(seed, _P_TEX, t)
        kind = t % 3
        c0 = rng.integers(0, 256, 4)
        c1 = rng.integers(0, 256, 4)
        if kind == 0:
            sh = int(rng.integers(3, 8))
            on = (((x >> sh) ^ (y >> sh)) & 1)[..., None]
            img = np.where(on, c1, c0)
        elif kind == 1:
            period = int(rng.integers(16, 128))
            ang = rng.uniform(0, np.pi)
            ph = (x * np.cos(ang) + y * np.sin(ang)) * (2 * np.pi / period)
            w = (0.5 + 0.5 * np.sin(ph))[..., None]
            img = np.rint(c0 + (c1.astype(np.float64) - c0) * w)
        else:
            sh = int(rng.integers(2, 6))
            blocks = rng.integers(0, 256, ((size >> sh) + 1, (size >> sh) + 1, 4))
            img = blocks[y >> sh, x >> sh]
        pool.append(np.ascontiguousarray(img.astype(np.uint8)))
    return pool


def _zipf_choice(rng: np.random.Generator, n_items: int, size: int, s: float = 1.1) -> np.ndarray:
    """Items drawn with P(rank r) proportional to r^-s; ranks mapped through a random permutation."""
    w = np.arange(1, n_items + 1, dtype=np.float64) ** (-s)
    rank = rng.choice(n_items, size=size, p=w / w.sum())
    perm = rng.permutation(n_items)
    return perm[rank]


def _object_screen(seed: int, n_mats: int, width: int, height: int, obj: int, frames: int,
                   scale=(1.0, 8.0), name: str = "scene", world: bool = False):
    """Screen split into obj x obj pixel objects; each object has one material,
    a UV scale and offset, an anisotropy and a normal.  Returns the frame function."""
    gx, gy = width // obj, height // obj
    n_obj = gx * gy
    rng = _rng(seed, _P_OBJ, n_mats, width)
    mat = _zipf_choice(rng, n_mats, n_obj).astype(np.uint32)
    s = rng.uniform(scale[0], scale[1], n_obj)
    off = rng.uniform(0.0, 1.0, (n_obj, 2))
    aniso = rng.uniform(1.0, 2.0, n_obj)
    # uniform direction on the upper hemisphere
    z = rng.uniform(0.0, 1.0, n_obj)
    phi = rng.uniform(0.0, 2 * np.pi, n_obj)
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    nrm = np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)

    py, px = np.mgrid[0:gy * obj, 0:gx * obj]
    oid = (py // obj) * gx + (px // obj)
    xl = (px % obj).astype(np.float64)
    yl = (py % obj).astype(np.float64)
    oid = oid.ravel(); xl = xl.ravel(); yl = yl.ravel()
    n = oid.shape[0]
    # per-hit constants that do not change between frames
    mat_h = mat[oid]
    s_h = s[oid]
    duv = np.zeros((n, 4), np.float32)
    duv[:, 0] = s_h / obj
    duv[:, 3] = aniso[oid] * s_h / obj
    nrm_h = nrm[oid].astype(np.float32)

    if world:
        # each object a planar patch in the world: an origin in [-8, 8]^3, two
        # orthonormal in-plane axes, a pixel size U[0.005, 0.04] world units
        # (drawn from a stream of their own, so the screen layout is unchanged)
        wr = _rng(seed, _P_OBJ, n_mats, width, 7)
        origin = wr.uniform(-8.0, 8.0, (n_obj, 3))
        ax = wr.normal(size=(n_obj, 3))
        ax /= np.linalg.norm(ax, axis=1)[:, None]
        ay = np.cross(nrm, ax)
        ay /= np.linalg.norm(ay, axis=1)[:, None]
        ax = np.cross(ay, nrm)
        px = wr.uniform(0.005, 0.04, n_obj)
        width_h = px[oid].astype(np.float32)

    def frame(f: int) -> Hits:
        jr = _rng(seed, _P_JITTER, n_mats, f)
        j = jr.random((n, 2))
        uv = np.empty((n, 2), np.float32)
        uv[:, 0] = off[oid, 0] + s_h * (xl + j[:, 0]) / obj
        uv[:, 1] = off[oid, 1] + s_h * (yl + j[:, 1]) / obj
        if not world:
            return Hits(mat_h.copy(), uv, duv.copy(), nrm_h.copy())
        p = origin[oid] + (px[oid] * (xl + j[:, 0]))[:, None] * ax[oid] + \
            (px[oid] * (yl + j[:, 1]))[:, None] * ay[oid]
        return Hits(mat_h.copy(), uv, duv.copy(), nrm_h.copy(), position=p.astype(np.float32),
                    width=width_h.copy())

    return frame, n


def mid_scene(seed: int = 0, n_mats: int = 64, width: int = 1920, height: int = 1080,
              frames: int = 16, slots: int = 1 << 22, n_textures: int = 16,
              tex_size: int = 1024, nodes=(8, 64), ranges: str = "narrow") -> Scene:
    """64 materials of U{8..64} nodes, 120x120-px objects, Zipf(1.1) materials."""
    rng = _rng(seed, _P_GRAPH, 2)
    mats = [random_material(rng, int(rng.integers(nodes[0], nodes[1] + 1)), n_textures,
                            ranges=ranges)
            for _ in range(n_mats)]
    tex = texture_pool(seed, n_textures, tex_size)
    frame_fn, n = _object_screen(seed, n_mats, width, height, 120, frames, name="mid")
    return Scene("mid", mats, tex, frames, n, CacheConfig(slots), seed, frame_fn,
                 dict(n_mats=n_mats, width=width, height=height, obj=120))


def spatial_scene(seed: int = 0, n_mats: int = 64, width: int = 480, height: int = 240,
                  frames: int = 2, slots: int = 1 << 18, n_textures: int = 16,
                  tex_size: int = 1024, nodes=(8, 64), p_position: float = 0.35) -> Scene:
    """The mid material mix with a share ``p_position`` of its leaves reading the
    world position (3D value noise), on 120-px objects that are planar patches
    in the world; hits carry world positions and one pixel's world width."""
    rng = _rng(seed, _P_GRAPH, 11)
    mats = [random_material(rng, int(rng.integers(nodes[0], nodes[1] + 1)), n_textures,
                            p_position=p_position)
            for _ in range(n_mats)]
    tex = texture_pool(seed, n_textures, tex_size)
    frame_fn, n = _object_screen(seed, n_mats, width, height, 120, frames, name="spatial",
                                 world=True)
    return Scene("spatial", mats, tex, frames, n, CacheConfig(slots), seed, frame_fn,
                 dict(n_mats=n_mats, width=width, height=height, obj=120))


def lognormal_sizes(rng, n, lo, hi, mu=3.0, sigma=1.0):
    return np.clip(np.rint(rng.lognormal(mu, sigma, n)), lo, hi).astype(int)


def smooth_material(seed: int, m: int, groups: int = 2, n_noise: int = 12,
                    perlin_freq: float = 0.25, perlin_octaves: int = 2,
                    value_freq: float = 0.25) -> Material:
    """A material whose deep sub-graphs are expensive but smooth functions of UV:
    n_noise low-frequency Perlin layers averaged (ADD chain, then a scale), then
    4 * groups MUL/POW nodes that undo each other pairwise, mixing a value-noise
    colour.  Base colour (COLOR) and roughness (FLOAT) are cacheable outputs of
    more than 32 nodes each, which a small network can represent."""
    rng = _rng(seed, _P_GRAPH, 7, m)
    L, C = Input.link, Input.const
    ca, cb, cc = (tuple(float(x) for x in rng.uniform(0.1, 0.9, 3)) for _ in range(3))
    nodes = [
        Node("UV_INPUT"),                                                        # 0
        Node("VALUE_NOISE", [L(0)], freq=value_freq, octaves=1,
             seed=int(rng.integers(1 << 30))),                                   # 1
        Node("MIX", [L(1), C(*ca), C(*cb)]),                                     # 2
    ]
    layers = []
    for _ in range(n_noise):
        f = perlin_freq * float(rng.uniform(0.75, 1.25))
        nodes.append(Node("PERLIN_NOISE", [L(0)], freq=f, octaves=perlin_octaves,
                          seed=int(rng.integers(1 << 30))))
        layers.append(len(nodes) - 1)
    x = layers[0]
    for q in layers[1:]:
        nodes.append(Node("MATH", [L(x), L(q)], math_op="ADD"))
        x = len(nodes) - 1
    nodes.append(Node("MATH", [L(x), C(1.0 / n_noise)], math_op="MUL"))
    x = len(nodes) - 1
    for _ in range(groups):
        c = float(rng.uniform(0.8, 1.25))
        e = float(rng.uniform(0.8, 1.25))
        for op, k in (("MUL", c), ("MUL", 1.0 / c), ("POW", e), ("POW", 1.0 / e)):
            nodes.append(Node("MATH", [L(x), C(k)], math_op=op))
            x = len(nodes) - 1
    nodes.append(Node("MIX", [L(x), L(2), C(*cc)]))                              # base colour
    base = len(nodes) - 1
    nodes.append(Node("MATH", [L(x), C(0.8)], math_op="MUL", clamp=True))       # roughness
    rough = len(nodes) - 1
    nodes.append(Node("BSDF_OUTPUT", [L(base), L(rough), C()]))
    return Material(nodes)


def smooth_scene(seed: int = 0, n_mats: int = 4, width: int = 480, height: int = 240,
                 frames: int = 4, slots: int = 1 << 18, **material_kw) -> Scene:
    """Scene of smooth_material graphs on 40-px objects with UV scale U[0.5, 1]."""
    mats = [smooth_material(seed, m, **material_kw) for m in range(n_mats)]
    frame, n = _object_screen(seed, n_mats, width, height, 40, frames, scale=(0.5, 1.0),
                              name="smooth")
    return Scene("smooth", mats, [], frames, n, CacheConfig(slots), seed, frame)


def batching_scene(seed: int = 0, n_mats: int = 1000, width: int = 1920, height: int = 1080,
                   frames: int = 64, slots: int = 1 << 24, n_textures: int = 64,
                   tex_size: int = 1024) -> Scene:
    """1000 materials with lognormal(3, 1) sizes in [4, 400], 40x40-px objects."""
    rng = _rng(seed, _P_GRAPH, 3)
    sizes = lognormal_sizes(rng, n_mats, 4, 400)
    mats = [random_material(rng, int(k), n_textures) for k in sizes]
    tex = texture_pool(seed + 1, n_textures, tex_size)
    frame_fn, n = _object_screen(seed, n_mats, width, height, 40, frames, name="batching")
    return Scene("batching", mats, tex, frames, n, CacheConfig(slots), seed, frame_fn,
                 dict(n_mats=n_mats, width=width, height=height, obj=40))


def scale_scene(seed: int = 0, n_mats: int = 4096, width: int = 3840, height: int = 2160,
                frames: int = 128, slots: int = 1 << 26, n_textures: int = 64,
                tex_size: int = 1024) -> Scene:
    """4096 materials with lognormal sizes in [8, 400], 3840x2160, OVERWRITE table."""
    rng = _rng(seed, _P_GRAPH, 5)
    sizes = lognormal_sizes(rng, n_mats, 8, 400)
    mats = [random_material(rng, int(k), n_textures) for k in sizes]
    tex = texture_pool(seed + 2, n_textures, tex_size)
    frame_fn, n = _object_screen(seed, n_mats, width, height, 40, frames, name="scale")
    return Scene("scale", mats, tex, frames, n, CacheConfig(slots, policy="OVERWRITE"), seed,
                 frame_fn, dict(n_mats=n_mats, width=width, height=height, obj=40))


def mlp_init(seed: int, n_mats: int, fan=((32, 64), (64, 64), (64, 4))) -> List[List[np.ndarray]]:
    """He-uniform initial weights (float32) per material: [W1, b1, W2, b2, W3, b3], W as [out, in]."""
    out = []
    for m in range(n_mats):
        rng = _rng(seed, _P_MLP, m)
        layers = []
        for fi, fo in fan:
            lim = np.sqrt(6.0 / fi)
            layers.append(rng.uniform(-lim, lim, (fo, fi)).astype(np.float32))
            layers.append(np.zeros(fo, np.float32))
        out.append(layers)
    return out


def with_indirect(direct: Hits, frame: int, seed: int = 0, widen=(2.0, 16.0),
                  max_bounce: int = 3) -> Hits:
    """A frame of a path tracer: the camera hits ``direct`` (bounce 0) followed
    by as many hits of secondary rays (bounce 1 .. max_bounce).  A secondary
    hit lands on a random point of the scene (a random direct hit's material,
    normal and UV, moved by up to a few footprints) and its footprint is wider
    by a random factor in ``widen`` (a ray cone that has spread over a longer
    path), so it keys coarser texels than the camera rays there."""
    n = len(direct)
    rng = _rng(seed, _P_BOUNCE, frame, n)
    pick = rng.integers(0, n, n)
    ind = direct.take(pick)
    k = np.exp(rng.uniform(np.log(widen[0]), np.log(widen[1]), n))
    duv = (ind.duv.astype(np.float64) * k[:, None]).astype(np.float32)
    shift = rng.uniform(-2.0, 2.0, (n, 2)) * np.abs(duv[:, [0, 3]])
    uv = (ind.uv.astype(np.float64) + shift).astype(np.float32)
    bounce = rng.integers(1, max_bounce + 1, n).astype(np.uint32)
    ind = Hits(ind.material.copy(), uv, duv, ind.normal.copy(), bounce)
    d = Hits(direct.material, direct.uv, direct.duv, direct.normal, np.zeros(n, np.uint32))
    return Hits.concat([d, ind])


def relayout(sc: Scene, seed: int) -> Scene:
    """The same materials, textures and table on another screen layout: objects,
    their materials, UV scales and normals, and the per-frame jitter all drawn
    from ``seed`` (a warm-up scene for tuning launch settings)."""
    if sc.layout is None:
        raise ValueError(f"scene {sc.name} has no object layout")
    L = sc.layout
    frame_fn, n = _object_screen(seed, L["n_mats"], L["width"], L["height"], L["obj"], sc.frames)
    return Scene(sc.name + "-layout%d" % seed, sc.materials, sc.textures, sc.frames, n, sc.cache,
                 seed, frame_fn, dict(L))


def cone_hits(seed: int, n: int, min_sin: float = 0.1, min_cos: float = 0.05,
              head_on: float = 0.01) -> Dict[str, np.ndarray]:
    """Hit geometry of a path tracer for the ray-cone footprint: per hit a ray
    direction, the cone radius at the hit, the hit triangle's edges and UV
    edges (float32).  Triangles of scale log-uniform in [1e-3, 1] with angles
    whose sine is at least ``min_sin``; rays at least ``min_cos`` from grazing;
    a ``head_on`` fraction exactly along the triangle normal; radii
    log-uniform in [1e-4, 1e-1] times the triangle scale; UV edges of lengths
    log-uniform in [1e-3, 10]."""
    rng = _rng(seed, _P_BOUNCE, 7, n)
    out = {"dir": np.zeros((n, 3), np.float32), "radius": np.zeros(n, np.float32),
           "edge": np.zeros((n, 6), np.float32), "uv_edge": np.zeros((n, 4), np.float32)}
    done = 0
    while done < n:
        k = 2 * (n - done) + 16
        s = np.exp(rng.uniform(np.log(1e-3), 0.0, k))
        e1 = rng.normal(size=(k, 3)) * s[:, None]
        e2 = rng.normal(size=(k, 3)) * s[:, None]
        nrm = np.cross(e1, e2)
        sin = np.linalg.norm(nrm, axis=1) / (np.linalg.norm(e1, axis=1) * np.linalg.norm(e2, axis=1))
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        m = nrm / np.linalg.norm(nrm, axis=1)[:, None]
        cos = np.abs(np.sum(d * m, axis=1))
        on = rng.random(k) < head_on
        e1f, e2f = e1.astype(np.float32), e2.astype(np.float32)
        # exactly along the normal of the float32 triangle
        nf = np.cross(e1f.astype(np.float64), e2f.astype(np.float64))
        d = np.where(on[:, None], -nf / np.linalg.norm(nf, axis=1)[:, None], d)
        ok = (sin >= min_sin) & ((cos >= min_cos) | on)
        sel = np.nonzero(ok)[0][:n - done]
        m_ = len(sel)
        r = np.exp(rng.uniform(np.log(1e-4), np.log(1e-1), k)) * s
        uvl = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), (k, 2)))
        ang = rng.uniform(0, 2 * np.pi, (k, 2))
        t = np.stack([uvl[:, 0] * np.cos(ang[:, 0]), uvl[:, 0] * np.sin(ang[:, 0]),
                      uvl[:, 1] * np.cos(ang[:, 1]), uvl[:, 1] * np.sin(ang[:, 1])], 1)
        out["dir"][done:done + m_] = d[sel]
        out["radius"][done:done + m_] = r[sel]
        out["edge"][done:done + m_] = np.concatenate([e1f[sel], e2f[sel]], 1)
        out["uv_edge"][done:done + m_] = t[sel]
        done += m_
    return out
