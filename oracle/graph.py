"""Material networks: validation, dependency classes, cacheable outputs, evaluation.

Sec. 2: a material is a node network evaluated at each shading point.
Sec. 3: cacheable nodes are found by traversing the network from the inputs
up ("bottom to top") and taking the highest nodes whose sub-graph depends on
no shading-point information other than UV; a material may have several.
Sec. 3.1: a sub-graph that reads any other shading-point datum is not
cacheable.

Readings used here (the paper gives no formal rule):
  * dependency class of a node: the set of shading-point data its value
    depends on, among UV, POS (the world position, read by the position-noise
    node: Sec. 3.1 names world position as other shading-point information a
    descriptor can use) and SP (any other datum: the normal-map node reads the
    hit normal); CONST is the empty set;
  * an output socket (node, socket) is cacheable when the node's class is
    exactly UV or exactly POS, the node is not the UV input itself, its
    sub-graph holds at least ``min_subgraph_nodes`` nodes besides UV inputs,
    and at least one consumer of that socket has another class or is the BSDF
    sink, i.e. the socket is the highest level of its class; a UV-class output
    is keyed by a UV texel, a POS-class output by a world-space cell;
  * only nodes reachable from the sink take part;
  * a multi-output node gets one descriptor per cacheable output socket;
  * ordinals c = 0..K-1 follow ascending (node index, socket).

Evaluation is memoised recursion from the sink in FP64, with no constant
folding (folding is an optimisation of the evaluator, Sec. 2, and must not
change values beyond FP32 round-off).
"""
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import nodes as N

IN_TYPES = {
    "UV_INPUT": (), "IMAGE_TEXTURE": ("UV",), "VALUE_NOISE": ("UV",), "PERLIN_NOISE": ("UV",),
    "MIX": ("FLOAT", "COLOR", "COLOR"), "MATH": ("FLOAT", "FLOAT"), "COLOR_RAMP": ("FLOAT",),
    "NORMAL_MAP": ("COLOR", "FLOAT"), "BSDF_OUTPUT": ("COLOR", "FLOAT", "VECTOR"),
    "POSITION_NOISE": (),
}
OUT_TYPES = {
    "UV_INPUT": ("UV",), "IMAGE_TEXTURE": ("COLOR", "FLOAT"), "VALUE_NOISE": ("FLOAT",),
    "PERLIN_NOISE": ("FLOAT",), "MIX": ("COLOR",), "MATH": ("FLOAT",),
    "COLOR_RAMP": ("COLOR", "FLOAT"), "NORMAL_MAP": ("VECTOR",), "BSDF_OUTPUT": (),
    "POSITION_NOISE": ("FLOAT",),
}
CONST, UV, POS, SP = 0, 1, 2, 4          # class = union (bitwise or) of these flags

DEFAULT_BASE = (0.8, 0.8, 0.8)
DEFAULT_ROUGHNESS = 0.5


class GraphError(ValueError):
    pass


def _convertible(src: str, dst: str) -> bool:
    if src == dst:
        return True
    return {src, dst} == {"FLOAT", "COLOR"}


def validate(material) -> None:
    nodes = material.nodes
    sinks = [i for i, n in enumerate(nodes) if n.op == "BSDF_OUTPUT"]
    if len(sinks) != 1:
        raise GraphError("exactly one BSDF_OUTPUT node is required")
    for i, n in enumerate(nodes):
        if n.op not in IN_TYPES:
            raise GraphError(f"node {i}: unknown op {n.op}")
        if len(n.inputs) > len(IN_TYPES[n.op]):
            raise GraphError(f"node {i}: too many inputs")
        for k, inp in enumerate(n.inputs):
            if inp.node < 0:
                continue
            if inp.node >= len(nodes):
                raise GraphError(f"node {i}: input {k} links past the end")
            src_types = OUT_TYPES[nodes[inp.node].op]
            if inp.socket >= len(src_types):
                raise GraphError(f"node {i}: input {k} names a missing socket")
            if not _convertible(src_types[inp.socket], IN_TYPES[n.op][k]):
                raise GraphError(f"node {i}: input {k} type mismatch")
    # acyclic: depth-first search with colours
    state = [0] * len(nodes)

    def visit(i):
        if state[i] == 1:
            raise GraphError("cycle")
        if state[i] == 2:
            return
        state[i] = 1
        for inp in nodes[i].inputs:
            if inp.node >= 0:
                visit(inp.node)
        state[i] = 2

    for i in range(len(nodes)):
        visit(i)


def reachable(material) -> List[bool]:
    nodes = material.nodes
    seen = [False] * len(nodes)
    stack = [material.sink]
    while stack:
        i = stack.pop()
        if seen[i]:
            continue
        seen[i] = True
        stack.extend(inp.node for inp in nodes[i].inputs if inp.node >= 0)
    return seen


def dependency_classes(material) -> List[int]:
    nodes = material.nodes
    memo: Dict[int, int] = {}

    def cls(i):
        if i in memo:
            return memo[i]
        n = nodes[i]
        c = {"UV_INPUT": UV, "IMAGE_TEXTURE": UV, "VALUE_NOISE": UV, "PERLIN_NOISE": UV,
             "POSITION_NOISE": POS, "NORMAL_MAP": SP}.get(n.op, CONST)
        for inp in n.inputs:
            if inp.node >= 0:
                c |= cls(inp.node)
        memo[i] = c
        return c

    return [cls(i) for i in range(len(nodes))]


def subgraph(material, i) -> set:
    nodes = material.nodes
    out, stack = set(), [i]
    while stack:
        j = stack.pop()
        if j in out:
            continue
        out.add(j)
        stack.extend(inp.node for inp in nodes[j].inputs if inp.node >= 0)
    return out


MAX_CACHEABLE = 8


def cacheable_outputs(material, min_subgraph_nodes: int = 2,
                      texel_only: bool = False) -> List[Tuple[int, int]]:
    """Ordered list of cacheable (node, socket) pairs (ordinal = list index); at
    most MAX_CACHEABLE per material, the first in (node, socket) order (the
    rest are evaluated every time, as if not cacheable).  texel_only: the
    descriptor is the UV texel alone, as Sec. 3.1 defines it, so outputs of
    the world position are not cacheable."""
    nodes = material.nodes
    live = reachable(material)
    cls = dependency_classes(material)
    keyed = (UV,) if texel_only else (UV, POS)
    out = []
    for i, n in enumerate(nodes):
        if not live[i] or cls[i] not in keyed or n.op == "UV_INPUT" or n.op == "BSDF_OUTPUT":
            continue
        size = sum(1 for j in subgraph(material, i) if nodes[j].op != "UV_INPUT")
        if size < min_subgraph_nodes:
            continue
        for s in range(len(OUT_TYPES[n.op])):
            boundary = False
            for q, m in enumerate(nodes):
                if not live[q]:
                    continue
                for inp in m.inputs:
                    if inp.node == i and inp.socket == s and (m.op == "BSDF_OUTPUT" or
                                                              cls[q] != cls[i]):
                        boundary = True
            if boundary and len(out) < MAX_CACHEABLE:
                out.append((i, s))
    return out


def output_type(material, node, socket) -> str:
    return OUT_TYPES[material.nodes[node].op][socket]


def key_kind(material, node) -> int:
    """UV for a UV-texel descriptor, POS for a world-space cell (cacheable outputs)."""
    return dependency_classes(material)[node]


def _convert(val, src: str, dst: str):
    if src == dst:
        return val
    if src == "COLOR" and dst == "FLOAT":
        return (val[:, 0] + val[:, 1] + val[:, 2]) / 3.0
    if src == "FLOAT" and dst == "COLOR":
        return np.repeat(val[:, None], 3, axis=1)
    raise GraphError(f"cannot convert {src} to {dst}")


def evaluate(material, uv, normal, textures, subst: Optional[dict] = None, position=None):
    """Evaluate one material at n shading points.

    uv: [n, 2], normal: [n, 3] (float arrays; promoted to FP64).
    position: [n, 3] world positions (needed when the material reads them).
    subst: optional {(node, socket): (mask [n] bool, value array)}; where the
    mask is set, that output takes the given value instead of its computed
    one (this is how a cache hit replaces a sub-graph's result, Sec. 3).

    Returns (outputs, values) with outputs = dict(base_color [n,3],
    roughness [n], normal [n,3]) and values = {(node, socket): array} of every
    output socket that was computed (substituted values included).
    """
    nodes = material.nodes
    uv = np.asarray(uv, dtype=np.float64)
    normal = np.asarray(normal, dtype=np.float64)
    n = uv.shape[0]
    subst = subst or {}
    memo: Dict[int, tuple] = {}

    def read(i, k, want):
        inp = nodes[i].inputs[k] if k < len(nodes[i].inputs) else None
        if inp is None or inp.node < 0:
            if want == "UV":
                return uv
            if want == "VECTOR":
                return normal
            v = inp.value if inp is not None else (0.0, 0.0, 0.0)
            if want == "FLOAT":
                return np.full(n, float(v[0]))
            return np.tile(np.asarray(v[:3], dtype=np.float64), (n, 1))
        src_t = OUT_TYPES[nodes[inp.node].op][inp.socket]
        return _convert(outs(inp.node)[inp.socket], src_t, want)

    def outs(i):
        if i in memo:
            return memo[i]
        nd = nodes[i]
        op = nd.op
        if op == "UV_INPUT":
            r = (uv,)
        elif op == "IMAGE_TEXTURE":
            r = N.image_texture(textures[nd.texture], read(i, 0, "UV"))
        elif op == "VALUE_NOISE":
            r = (N.value_noise(read(i, 0, "UV"), nd.freq, nd.octaves, nd.seed),)
        elif op == "PERLIN_NOISE":
            r = (N.perlin_noise(read(i, 0, "UV"), nd.freq, nd.octaves, nd.seed),)
        elif op == "MIX":
            r = (N.mix(read(i, 0, "FLOAT"), read(i, 1, "COLOR"), read(i, 2, "COLOR")),)
        elif op == "MATH":
            r = (N.math_op(nd.math_op, read(i, 0, "FLOAT"), read(i, 1, "FLOAT"), nd.clamp),)
        elif op == "COLOR_RAMP":
            r = N.color_ramp(read(i, 0, "FLOAT"), nd.ramp_pos, nd.ramp_rgba)
        elif op == "NORMAL_MAP":
            r = (N.normal_map(read(i, 0, "COLOR"), read(i, 1, "FLOAT"), normal),)
        elif op == "POSITION_NOISE":
            if position is None:
                raise GraphError("the material reads the world position, none given")
            r = (N.position_noise(np.asarray(position, dtype=np.float64), nd.freq, nd.octaves,
                                  nd.seed),)
        else:
            raise GraphError(f"cannot evaluate {op}")
        r = list(r)
        for s in range(len(r)):
            if (i, s) in subst:
                mask, val = subst[(i, s)]
                val = np.asarray(val, dtype=np.float64)
                if r[s].ndim == 2:
                    r[s] = np.where(mask[:, None], val, r[s])
                else:
                    r[s] = np.where(mask, val, r[s])
        memo[i] = tuple(r)
        return memo[i]

    sink = material.sink
    outputs = dict(base_color=read(sink, 0, "COLOR"), roughness=read(sink, 1, "FLOAT"),
                   normal=read(sink, 2, "VECTOR"))
    values = {(i, s): v for i, r in memo.items() for s, v in enumerate(r)}
    return outputs, values


def default_outputs(normal):
    n = normal.shape[0]
    return dict(base_color=np.tile(np.asarray(DEFAULT_BASE), (n, 1)),
                roughness=np.full(n, DEFAULT_ROUGHNESS),
                normal=np.asarray(normal, dtype=np.float64).copy())
