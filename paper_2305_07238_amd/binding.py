"""ctypes binding of libpmc (include/pmc.h).

Argument marshalling only: every step of shading runs in the library's HIP
kernels.  The module refuses to import when ``libpmc.so`` has not been built
(there is no fallback path).  Functions carry the C names; ``Context`` and
``Cache`` are thin owners of the opaque handles that raise on error codes.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmc.so")

# torch ships its own HIP runtime libraries; load them before libpmc.so so that
# both find the device (loaded the other way round, one of them sees none)
try:
    import torch  # noqa: F401
except ImportError:
    pass

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(python -c 'import __graft_entry__ as g; g.build()')")
lib = C.CDLL(LIB_PATH)

# ----------------------------------------------------------------- constants --
PMC_OK, PMC_ERR_INVALID, PMC_ERR_GRAPH, PMC_ERR_OOM, PMC_ERR_HIP, PMC_ERR_UNSUPPORTED, \
    PMC_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
OPS = {"UV_INPUT": 0, "IMAGE_TEXTURE": 1, "VALUE_NOISE": 2, "PERLIN_NOISE": 3, "MIX": 4,
       "MATH": 5, "COLOR_RAMP": 6, "NORMAL_MAP": 7, "BSDF_OUTPUT": 8, "POSITION_NOISE": 9}
MATH_OPS = {"ADD": 0, "MUL": 1, "POW": 2}
PMC_NODE_CLAMP = 1
PMC_POLICY_FIRST, PMC_POLICY_OVERWRITE, PMC_POLICY_PRIORITY = 0, 1, 2
PMC_MODE_UNCACHED, PMC_MODE_CACHED, PMC_MODE_SNAPSHOT = 0, 1, 2
PMC_FLAG_SORT, PMC_FLAG_PERSISTENT, PMC_FLAG_DEFER, PMC_FLAG_LOG, PMC_FLAG_SURROGATE = 1, 2, 4, 8, 16
PMC_FLAG_SURROGATE_INSERT = 32
PMC_STATIC_SCRATCH_BYTES, PMC_STATIC_MAX_HITS = 16 << 20, 1 << 20
N_PARAMS = 6532
MAX_CACHEABLE = 8


# ----------------------------------------------------------------- structs ----
class pmc_input(C.Structure):
    _fields_ = [("node", C.c_int32), ("socket", C.c_uint32), ("value", C.c_float * 3)]


class pmc_node_desc(C.Structure):
    _fields_ = [("op", C.c_uint32), ("variant", C.c_uint32), ("flags", C.c_uint32),
                ("seed", C.c_uint32), ("freq", C.c_float), ("octaves", C.c_uint32),
                ("inp", pmc_input * 3), ("ramp_pos", C.c_float * 8),
                ("ramp_rgba", (C.c_float * 4) * 8)]


class pmc_texture_desc(C.Structure):
    _fields_ = [("texels", C.c_void_p), ("width", C.c_uint32), ("height", C.c_uint32)]


class pmc_compile_opts(C.Structure):
    _fields_ = [("min_subgraph_nodes", C.c_uint32), ("no_fold", C.c_uint32),
                ("texel_keys_only", C.c_uint32), ("reserved", C.c_uint32 * 5)]


class pmc_material_info(C.Structure):
    _fields_ = [("n_nodes", C.c_uint32), ("n_live", C.c_uint32), ("n_folded", C.c_uint32),
                ("n_instr", C.c_uint32), ("n_regs", C.c_uint32), ("n_cacheable", C.c_uint32),
                ("cacheable_node", C.c_uint32 * MAX_CACHEABLE),
                ("cacheable_socket", C.c_uint32 * MAX_CACHEABLE),
                ("subgraph_nodes", C.c_uint32 * MAX_CACHEABLE),
                ("cacheable_type", C.c_uint32 * MAX_CACHEABLE),
                ("cacheable_key", C.c_uint32 * MAX_CACHEABLE)]


class pmc_cache_params(C.Structure):
    _fields_ = [("n_cells", C.c_uint64), ("n_entries", C.c_uint32), ("entry_bytes", C.c_uint32),
                ("policy", C.c_uint32), ("level_bias", C.c_int32), ("level_max", C.c_uint32),
                ("hash2_mask", C.c_uint32)]


class pmc_hits(C.Structure):
    _fields_ = [("material", C.c_void_p), ("uv", C.c_void_p), ("duv", C.c_void_p),
                ("normal", C.c_void_p), ("n", C.c_uint64), ("bounce", C.c_void_p),
                ("position", C.c_void_p), ("width", C.c_void_p)]


class pmc_cone_hits(C.Structure):
    _fields_ = [("dir", C.c_void_p), ("radius", C.c_void_p), ("edge", C.c_void_p),
                ("uv_edge", C.c_void_p), ("n", C.c_uint64)]


class pmc_bsdf_out(C.Structure):
    _fields_ = [("base_color", C.c_void_p), ("roughness", C.c_void_p), ("normal", C.c_void_p)]


class pmc_debug_out(C.Structure):
    _fields_ = [("state", C.c_void_p), ("value", C.c_void_p)]


class pmc_shade_params(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("flags", C.c_uint32), ("frame", C.c_uint32),
                ("chunk_waves", C.c_uint32), ("blocks_per_cu", C.c_uint32),
                ("defer_max", C.c_uint32), ("waves_per_block", C.c_uint32),
                ("reserved", C.c_uint32)]


class pmc_frame_plan(C.Structure):
    _fields_ = [("hits", pmc_hits), ("hits_per_frame", C.c_uint64), ("n_frames", C.c_uint32),
                ("first_frame", C.c_uint32), ("out", pmc_bsdf_out), ("out_per_frame", C.c_uint32),
                ("clear_cache", C.c_uint32), ("params", pmc_shade_params), ("stats", C.c_void_p),
                ("late_frame", C.c_uint32), ("reserved", C.c_uint32),
                ("late_params", pmc_shade_params)]


class pmc_tune_result(C.Structure):
    _fields_ = [("best", pmc_shade_params), ("best_ms", C.c_double), ("default_ms", C.c_double),
                ("n_tried", C.c_uint32), ("reserved", C.c_uint32)]


STAT_FIELDS = ("hits_shaded", "probes", "cache_hits", "bypasses", "inserts", "cas_failures",
               "present", "cell_full", "overwrites", "nonfinite", "candidates",
               "nodes_executed", "nodes_total", "invalid_material", "texture_evals",
               "deferred", "insert_attempts", "texture_evals_deferred",
               "insert_attempts_deferred", "probes_deferred", "surrogate_used", "logged",
               "audited")


class pmc_stats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in STAT_FIELDS] + [("reserved", C.c_uint64 * 9)]


class pmc_surrogate_opts(C.Structure):
    _fields_ = [("min_subgraph_nodes", C.c_uint32), ("log_capacity", C.c_uint32),
                ("seed", C.c_uint64), ("max_err", C.c_float), ("reserved", C.c_uint32 * 3)]


class pmc_surrogate_slot(C.Structure):
    _fields_ = [("material", C.c_uint32), ("ordinal_mask", C.c_uint32),
                ("n_channels", C.c_uint32), ("channel", C.c_uint32 * 8),
                ("reserved", C.c_uint32)]


class pmc_train_params(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("batch", C.c_uint32), ("lr", C.c_float),
                ("holdout", C.c_uint32), ("min_records", C.c_uint32), ("lr_end", C.c_float),
                ("seed", C.c_uint64), ("workgroups", C.c_uint32), ("reserved", C.c_uint32)]


SURROGATE_STAT_FIELDS = ("material", "trusted", "n_train", "n_heldout", "max_err", "mean_err",
                         "loss", "live_max_err", "steps", "live_checked")


class pmc_surrogate_stat(C.Structure):
    _fields_ = [("material", C.c_uint32), ("trusted", C.c_uint32), ("n_train", C.c_uint32),
                ("n_heldout", C.c_uint32), ("max_err", C.c_float), ("mean_err", C.c_float),
                ("loss", C.c_float), ("live_max_err", C.c_float), ("steps", C.c_uint32),
                ("live_checked", C.c_uint32), ("reserved", C.c_uint32 * 2)]


LOG_RECORD_DTYPE = np.dtype([("material", "<u4"), ("ordinal", "<u4"), ("u", "<f4"),
                             ("v", "<f4"), ("value", "<f4", (4,))])


PROFILE_PHASES = ("sort", "shade", "snapshot", "stats")


class pmc_profile(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_uint64 * 4)]


class pmc_key_record(C.Structure):
    _fields_ = [("cell", C.c_uint32), ("hash2", C.c_uint32), ("level", C.c_int32),
                ("tx", C.c_int32), ("ty", C.c_int32), ("bypass", C.c_uint32)]


KEY_RECORD_DTYPE = np.dtype([("cell", "<u4"), ("hash2", "<u4"), ("level", "<i4"),
                             ("tx", "<i4"), ("ty", "<i4"), ("bypass", "<u4")])

# ------------------------------------------------------------- prototypes -----
_P = C.c_void_p
_S = C.c_int32
_proto = {
    "pmc_abi_version": (C.c_uint32, []),
    "pmc_abi_sizeof": (C.c_size_t, [C.c_uint32]),
    "pmc_create": (_S, [C.c_int, C.POINTER(C.c_void_p)]),
    "pmc_destroy": (None, [_P]),
    "pmc_last_error": (C.c_char_p, [_P]),
    "pmc_set_textures": (_S, [_P, C.POINTER(pmc_texture_desc), C.c_uint32]),
    "pmc_compile_materials": (_S, [_P, C.POINTER(pmc_node_desc), C.POINTER(C.c_uint32),
                                   C.c_uint32, C.POINTER(pmc_compile_opts)]),
    "pmc_get_material_info": (_S, [_P, C.c_uint32, C.POINTER(pmc_material_info)]),
    "pmc_cache_create": (_S, [_P, C.POINTER(pmc_cache_params), _P, C.POINTER(C.c_void_p)]),
    "pmc_cache_destroy": (None, [_P]),
    "pmc_cache_clear": (_S, [_P, _P]),
    "pmc_cache_device_ptr": (_S, [_P, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)]),
    "pmc_cache_export": (_S, [_P, _P, C.c_size_t, _P]),
    "pmc_cache_import": (_S, [_P, _P, C.c_size_t, _P]),
    "pmc_shade": (_S, [_P, _P, C.POINTER(pmc_hits), C.POINTER(pmc_bsdf_out),
                       C.POINTER(pmc_shade_params), _P, C.POINTER(pmc_debug_out), _P]),
    "pmc_shade_static": (_S, [_P, _P, C.POINTER(pmc_hits), C.POINTER(pmc_bsdf_out),
                              C.POINTER(pmc_shade_params), _P, C.POINTER(pmc_debug_out), _P]),
    "pmc_debug_keys": (_S, [_P, _P, C.POINTER(pmc_hits), _P, _P]),
    "pmc_ray_cone_gradients": (_S, [_P, C.POINTER(pmc_cone_hits), _P, _P]),
    "pmc_cache_insert_raw": (_S, [_P, _P, _P, _P, C.c_uint64, C.c_uint32, _P, _P]),
    "pmc_cache_lookup_raw": (_S, [_P, _P, _P, C.c_uint64, _P, _P, _P]),
    "pmc_frame_graph_create": (_S, [_P, _P, C.POINTER(pmc_frame_plan), C.POINTER(C.c_void_p)]),
    "pmc_frame_graph_launch": (_S, [_P, _P]),
    "pmc_frame_graph_destroy": (None, [_P]),
    "pmc_autotune": (_S, [_P, _P, C.POINTER(pmc_frame_plan), C.POINTER(pmc_tune_result),
                          C.c_char_p]),
    "pmc_profile_enable": (_S, [_P, C.c_int]),
    "pmc_profile_read": (_S, [_P, C.POINTER(pmc_profile), C.c_int]),
    "pmc_surrogate_setup": (_S, [_P, C.POINTER(pmc_surrogate_opts), C.POINTER(C.c_uint32)]),
    "pmc_surrogate_get_slot": (_S, [_P, C.c_uint32, C.POINTER(pmc_surrogate_slot)]),
    "pmc_log_clear": (_S, [_P, _P]),
    "pmc_log_read": (_S, [_P, _P, C.c_uint64, C.POINTER(C.c_uint64), _P]),
    "pmc_surrogate_set_params": (_S, [_P, C.c_uint32, _P]),
    "pmc_surrogate_get_params": (_S, [_P, C.c_uint32, _P]),
    "pmc_surrogate_set_trust": (_S, [_P, C.c_uint32, C.c_int, _P]),
    "pmc_surrogate_train": (_S, [_P, C.POINTER(pmc_train_params), _P]),
    "pmc_surrogate_train_records": (_S, [_P, C.c_uint32, _P, C.c_uint32,
                                         C.POINTER(pmc_train_params), _P]),
    "pmc_surrogate_grad": (_S, [_P, C.c_uint32, _P, C.c_uint32, _P, _P, _P]),
    "pmc_surrogate_infer": (_S, [_P, C.c_uint32, _P, C.c_uint32, _P, _P]),
    "pmc_surrogate_report": (_S, [_P, C.POINTER(pmc_surrogate_stat), C.c_uint32, _P]),
}
for _name, (_res, _args) in _proto.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

EXPORTED = tuple(_proto)

ABI_VERSION = 6                     # the layouts above follow this version of include/pmc.h
if pmc_abi_version() != ABI_VERSION:
    raise ImportError(f"{LIB_PATH} has ABI {pmc_abi_version()}, the binding expects "
                      f"{ABI_VERSION}: rebuild it with __graft_entry__.build()")


class PmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pmc error {code}: {msg}")
        self.code = code


# --------------------------------------------------------------- marshalling --

def node_array(materials) -> tuple:
    """scenes.Material list -> (pmc_node_desc array, uint32 offsets array)."""
    total = sum(len(m.nodes) for m in materials)
    arr = (pmc_node_desc * max(total, 1))()
    offsets = (C.c_uint32 * (len(materials) + 1))()
    k = 0
    for mi, m in enumerate(materials):
        offsets[mi] = k
        for nd in m.nodes:
            d = arr[k]
            d.op = OPS[nd.op]
            if nd.op == "MATH":
                d.variant = MATH_OPS[nd.math_op]
            elif nd.op == "IMAGE_TEXTURE":
                d.variant = nd.texture
            d.flags = PMC_NODE_CLAMP if nd.clamp else 0
            d.seed = nd.seed & 0xFFFFFFFF
            d.freq = nd.freq
            d.octaves = nd.octaves
            for s in range(3):
                if s < len(nd.inputs):
                    inp = nd.inputs[s]
                    d.inp[s].node = inp.node
                    d.inp[s].socket = inp.socket
                    for c in range(3):
                        d.inp[s].value[c] = inp.value[c]
                else:
                    d.inp[s].node = -1
            if nd.op == "COLOR_RAMP":
                for c in range(8):
                    d.ramp_pos[c] = nd.ramp_pos[c]
                    for q in range(4):
                        d.ramp_rgba[c][q] = nd.ramp_rgba[c][q]
            k += 1
    offsets[len(materials)] = k
    return arr, offsets


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


class Context:
    """Owner of a pmc_ctx (device >= 0) or a host-only one (device = -1)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = pmc_create(device, C.byref(h))
        if st != PMC_OK:
            raise PmcError(st, f"pmc_create({device}) failed")
        self.h = h
        self.device = device
        self.n_mats = 0
        self._caches = weakref.WeakSet()

    def close(self):
        # caches and graphs first: a context must outlive them (the cyclic garbage
        # collector may finalise a context before the objects that refer to it)
        for c in list(self._caches):
            c.close()
        if self.h:
            pmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != PMC_OK:
            raise PmcError(st, (pmc_last_error(self.h) or b"").decode())

    def set_textures(self, textures: Sequence[np.ndarray]):
        descs = (pmc_texture_desc * max(len(textures), 1))()
        keep = []
        for i, t in enumerate(textures):
            a = np.ascontiguousarray(t, dtype=np.uint8)
            keep.append(a)
            descs[i].texels = a.ctypes.data
            descs[i].height, descs[i].width = a.shape[0], a.shape[1]
        self.check(pmc_set_textures(self.h, descs, len(textures)))

    def compile(self, materials, min_subgraph_nodes: int = 0, no_fold: bool = False,
                texel_keys_only: bool = False):
        arr, offs = node_array(materials)
        opts = pmc_compile_opts(min_subgraph_nodes, 1 if no_fold else 0,
                                1 if texel_keys_only else 0)
        self.check(pmc_compile_materials(self.h, arr, offs, len(materials), C.byref(opts)))
        self.n_mats = len(materials)

    def material_info(self, m: int) -> pmc_material_info:
        info = pmc_material_info()
        self.check(pmc_get_material_info(self.h, m, C.byref(info)))
        return info

    def cacheables(self, m: int):
        info = self.material_info(m)
        return [(info.cacheable_node[c], info.cacheable_socket[c]) for c in range(info.n_cacheable)]

    def cache(self, n_cells: int, n_entries: int = 8, entry_bytes: int = 16,
              policy: int = PMC_POLICY_FIRST, level_bias: int = 0, level_max: int = 0,
              device_mem=None, hash2_mask: int = 0) -> "Cache":
        return Cache(self, n_cells, n_entries, entry_bytes, policy, level_bias, level_max,
                     device_mem, hash2_mask)

    def shade(self, hits: dict, out: dict, cache: Optional["Cache"] = None,
              mode: int = PMC_MODE_CACHED, flags: int = PMC_FLAG_SORT, frame: int = 0,
              stats=None, debug: Optional[dict] = None, chunk_waves: int = 0,
              blocks_per_cu: int = 0, defer_max: int = 0, waves_per_block: int = 0,
              stream=None, static: bool = False):
        """hits: dict of torch CUDA tensors material/uv/duv/normal (and optionally bounce);
        out: base_color/roughness/normal."""
        h = pmc_hits(_ptr(hits["material"]), _ptr(hits["uv"]), _ptr(hits["duv"]),
                     _ptr(hits["normal"]), int(hits["material"].numel()), _ptr(hits.get("bounce")),
                     _ptr(hits.get("position")), _ptr(hits.get("width")))
        o = pmc_bsdf_out(_ptr(out["base_color"]), _ptr(out["roughness"]), _ptr(out["normal"]))
        p = pmc_shade_params(mode, flags, frame, chunk_waves, blocks_per_cu, defer_max,
                             waves_per_block)
        dbg = None
        if debug is not None:
            dbg = C.byref(pmc_debug_out(_ptr(debug.get("state")), _ptr(debug.get("value"))))
        fn = pmc_shade_static if static else pmc_shade
        self.check(fn(self.h, cache.h if cache else None, C.byref(h), C.byref(o),
                      C.byref(p), _ptr(stats), dbg, _stream_ptr(stream)))

    def profile_enable(self, on: bool = True):
        self.check(pmc_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, reset: bool = True) -> dict:
        p = pmc_profile()
        self.check(pmc_profile_read(self.h, C.byref(p), 1 if reset else 0))
        return {ph: (p.ms[i], int(p.launches[i])) for i, ph in enumerate(PROFILE_PHASES)}

    def frame_plan(self, hits: dict, hits_per_frame: int, n_frames: int, out: dict,
                   mode: int = PMC_MODE_CACHED, flags: int = PMC_FLAG_SORT, first_frame: int = 0,
                   out_per_frame: bool = False, clear_cache: bool = True, stats=None,
                   chunk_waves: int = 0, blocks_per_cu: int = 0,
                   defer_max: int = 0, waves_per_block: int = 0, late_frame: int = 0,
                   late: Optional[dict] = None) -> pmc_frame_plan:
        """hits: torch tensors holding n_frames * hits_per_frame hits, frame-major."""
        h = pmc_hits(_ptr(hits["material"]), _ptr(hits["uv"]), _ptr(hits["duv"]),
                     _ptr(hits["normal"]), 0, _ptr(hits.get("bounce")),
                     _ptr(hits.get("position")), _ptr(hits.get("width")))
        o = pmc_bsdf_out(_ptr(out["base_color"]), _ptr(out["roughness"]), _ptr(out["normal"]))
        prm = pmc_shade_params(mode, flags, 0, chunk_waves, blocks_per_cu, defer_max,
                               waves_per_block)
        lp = pmc_shade_params()
        if late_frame:
            lk = dict(flags=flags, chunk_waves=0, blocks_per_cu=0, defer_max=0,
                      waves_per_block=0)
            lk.update(late or {})
            lp = pmc_shade_params(mode, lk["flags"], 0, lk["chunk_waves"], lk["blocks_per_cu"],
                                  lk["defer_max"], lk["waves_per_block"])
        plan = pmc_frame_plan(h, hits_per_frame, n_frames, first_frame, o, int(out_per_frame),
                              int(clear_cache), prm, _ptr(stats), late_frame, 0, lp)
        plan._keep = (hits, out, stats)
        return plan

    def frame_graph(self, cache: Optional["Cache"], plan: pmc_frame_plan) -> "FrameGraph":
        return FrameGraph(self, cache, plan)

    def autotune(self, cache: Optional["Cache"], plan: pmc_frame_plan,
                 json_path: Optional[str] = None) -> pmc_tune_result:
        res = pmc_tune_result()
        self.check(pmc_autotune(self.h, cache.h if cache else None, C.byref(plan), C.byref(res),
                                json_path.encode() if json_path else None))
        return res

    # ---------------------------------------------------------- surrogate --
    def surrogate_setup(self, min_subgraph_nodes: int = 0, log_capacity: int = 0, seed: int = 0,
                        max_err: float = 0.0) -> int:
        o = pmc_surrogate_opts(min_subgraph_nodes, log_capacity, seed, max_err)
        n = C.c_uint32()
        self.check(pmc_surrogate_setup(self.h, C.byref(o), C.byref(n)))
        self.n_slots = n.value
        return n.value

    def surrogate_slot(self, slot: int) -> dict:
        s = pmc_surrogate_slot()
        self.check(pmc_surrogate_get_slot(self.h, slot, C.byref(s)))
        return {"material": s.material, "ordinal_mask": s.ordinal_mask,
                "n_channels": s.n_channels, "channel": list(s.channel)}

    def log_clear(self, stream=None):
        self.check(pmc_log_clear(self.h, _stream_ptr(stream)))

    def log_read(self, max_records: int = 1 << 26, stream=None) -> np.ndarray:
        n = C.c_uint64()
        self.check(pmc_log_read(self.h, None, 0, C.byref(n), _stream_ptr(stream)))
        k = min(n.value, max_records)
        buf = np.zeros(k, LOG_RECORD_DTYPE)
        if k:
            self.check(pmc_log_read(self.h, buf.ctypes.data, k, C.byref(n),
                                    _stream_ptr(stream)))
        return buf

    def surrogate_set_params(self, slot: int, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == N_PARAMS
        self.check(pmc_surrogate_set_params(self.h, slot, p.ctypes.data))

    def surrogate_get_params(self, slot: int) -> np.ndarray:
        p = np.zeros(N_PARAMS, np.float32)
        self.check(pmc_surrogate_get_params(self.h, slot, p.ctypes.data))
        return p

    def surrogate_set_trust(self, slot: int, trusted: bool, stream=None):
        self.check(pmc_surrogate_set_trust(self.h, slot, 1 if trusted else 0,
                                           _stream_ptr(stream)))

    def surrogate_train(self, steps: int = 0, batch: int = 0, lr: float = 0.0, holdout: int = 0,
                        min_records: int = 0, seed: int = 0, lr_end: float = 0.0,
                        workgroups: int = 0, stream=None):
        p = pmc_train_params(steps, batch, lr, holdout, min_records, lr_end, seed, workgroups)
        self.check(pmc_surrogate_train(self.h, C.byref(p), _stream_ptr(stream)))

    def surrogate_train_records(self, slot: int, records, steps: int = 0, batch: int = 0,
                                lr: float = 0.0, seed: int = 0, lr_end: float = 0.0,
                                workgroups: int = 0, stream=None):
        """records: torch uint8/int32 CUDA tensor holding n packed pmc_log_record."""
        n = records.numel() * records.element_size() // 32
        p = pmc_train_params(steps, batch, lr, 0, 0, lr_end, seed, workgroups)
        self.check(pmc_surrogate_train_records(self.h, slot, _ptr(records), n, C.byref(p),
                                               _stream_ptr(stream)))

    def surrogate_grad(self, slot: int, records, grads, loss, stream=None):
        n = records.numel() * records.element_size() // 32
        self.check(pmc_surrogate_grad(self.h, slot, _ptr(records), n, _ptr(grads), _ptr(loss),
                                      _stream_ptr(stream)))

    def surrogate_infer(self, slot: int, uv, y, stream=None):
        self.check(pmc_surrogate_infer(self.h, slot, _ptr(uv), int(uv.shape[0]), _ptr(y),
                                       _stream_ptr(stream)))

    def surrogate_report(self, stream=None) -> List[dict]:
        n = getattr(self, "n_slots", 0)
        arr = (pmc_surrogate_stat * max(n, 1))()
        self.check(pmc_surrogate_report(self.h, arr, n, _stream_ptr(stream)))
        return [{f: getattr(arr[k], f) for f in SURROGATE_STAT_FIELDS} for k in range(n)]

    def ray_cone_gradients(self, cone: dict, duv, stream=None):
        """cone: torch CUDA tensors dir [n, 3], radius [n], edge [n, 6], uv_edge [n, 4];
        duv: float32 [n, 4] output (the layout of the hits' duv)."""
        h = pmc_cone_hits(_ptr(cone["dir"]), _ptr(cone["radius"]), _ptr(cone["edge"]),
                          _ptr(cone["uv_edge"]), int(cone["radius"].numel()))
        self.check(pmc_ray_cone_gradients(self.h, C.byref(h), _ptr(duv), _stream_ptr(stream)))

    def debug_keys(self, cache: "Cache", hits: dict, out, stream=None):
        h = pmc_hits(_ptr(hits["material"]), _ptr(hits["uv"]), _ptr(hits["duv"]),
                     _ptr(hits["normal"]), int(hits["material"].numel()), _ptr(hits.get("bounce")),
                     _ptr(hits.get("position")), _ptr(hits.get("width")))
        self.check(pmc_debug_keys(self.h, cache.h, C.byref(h), _ptr(out), _stream_ptr(stream)))


class FrameGraph:
    """A progressive render captured into one HIP graph (pmc_frame_graph_*)."""

    def __init__(self, ctx: Context, cache: Optional["Cache"], plan: pmc_frame_plan):
        self.ctx, self.cache, self.plan = ctx, cache, plan
        h = C.c_void_p()
        ctx.check(pmc_frame_graph_create(ctx.h, cache.h if cache else None, C.byref(plan),
                                         C.byref(h)))
        self.h = h
        ctx._caches.add(self)           # released before the context

    def launch(self, stream=None):
        self.ctx.check(pmc_frame_graph_launch(self.h, _stream_ptr(stream)))

    def close(self):
        if self.h:
            pmc_frame_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cache:
    def __init__(self, ctx: Context, n_cells, n_entries, entry_bytes, policy, level_bias,
                 level_max, device_mem=None, hash2_mask=0):
        self.ctx = ctx
        self.params = pmc_cache_params(int(n_cells), n_entries, entry_bytes, policy, level_bias,
                                       level_max, int(hash2_mask) & 0xFFFFFFFF)
        h = C.c_void_p()
        ctx.check(pmc_cache_create(ctx.h, C.byref(self.params), _ptr(device_mem), C.byref(h)))
        self.h = h
        ctx._caches.add(self)
        ptr, nbytes = C.c_void_p(), C.c_size_t()
        ctx.check(pmc_cache_device_ptr(self.h, C.byref(ptr), C.byref(nbytes)))
        self.nbytes = nbytes.value
        self.n_cells, self.n_entries, self.entry_bytes = int(n_cells), n_entries, entry_bytes

    def close(self):
        if self.h:
            pmc_cache_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        self.ctx.check(pmc_cache_clear(self.h, _stream_ptr(stream)))

    def export(self, stream=None) -> np.ndarray:
        buf = np.zeros(self.nbytes, np.uint8)
        self.ctx.check(pmc_cache_export(self.h, buf.ctypes.data, self.nbytes, _stream_ptr(stream)))
        return buf

    def import_(self, raw: np.ndarray, stream=None):
        raw = np.ascontiguousarray(raw, dtype=np.uint8)
        self.ctx.check(pmc_cache_import(self.h, raw.ctypes.data, raw.nbytes, _stream_ptr(stream)))

    def words(self, stream=None) -> np.ndarray:
        """Table as (n_cells * n_entries, entry_bytes // 8) uint64 (word first)."""
        return self.export(stream).view(np.uint64).reshape(-1, self.entry_bytes // 8)

    def insert_raw(self, k0, k1, enc, frame=0, stats=None, stream=None):
        self.ctx.check(pmc_cache_insert_raw(self.h, _ptr(k0), _ptr(k1), _ptr(enc), int(k0.numel()),
                                            frame, _ptr(stats), _stream_ptr(stream)))

    def lookup_raw(self, k0, k1, enc_out, hit_out, stream=None):
        self.ctx.check(pmc_cache_lookup_raw(self.h, _ptr(k0), _ptr(k1), int(k0.numel()),
                                            _ptr(enc_out), _ptr(hit_out), _stream_ptr(stream)))


# ------------------------------------------------------------ torch helpers ---

def hits_to_device(hits, device="cuda"):
    """scenes.Hits (numpy) -> dict of torch tensors on the device."""
    import torch
    d = {
        "material": torch.from_numpy(np.ascontiguousarray(hits.material, np.uint32).view(np.int32)).to(device),
        "uv": torch.from_numpy(np.ascontiguousarray(hits.uv, np.float32)).to(device),
        "duv": torch.from_numpy(np.ascontiguousarray(hits.duv, np.float32)).to(device),
        "normal": torch.from_numpy(np.ascontiguousarray(hits.normal, np.float32)).to(device),
    }
    if getattr(hits, "bounce", None) is not None:
        d["bounce"] = torch.from_numpy(
            np.ascontiguousarray(hits.bounce, np.uint32).view(np.int32)).to(device)
    if getattr(hits, "position", None) is not None:
        d["position"] = torch.from_numpy(np.ascontiguousarray(hits.position, np.float32)).to(device)
        d["width"] = torch.from_numpy(np.ascontiguousarray(hits.width, np.float32)).to(device)
    return d


def alloc_outputs(n: int, device="cuda"):
    import torch
    return {"base_color": torch.empty((n, 3), dtype=torch.float32, device=device),
            "roughness": torch.empty((n,), dtype=torch.float32, device=device),
            "normal": torch.empty((n, 3), dtype=torch.float32, device=device)}


def records_to_device(records: np.ndarray, device="cuda"):
    """LOG_RECORD_DTYPE array -> torch int32 tensor of the packed 32-byte records."""
    import torch
    raw = np.ascontiguousarray(records, LOG_RECORD_DTYPE).view(np.int32).reshape(-1, 8)
    return torch.from_numpy(raw.copy()).to(device)


def new_stats(device="cuda"):
    import torch
    return torch.zeros(32, dtype=torch.int64, device=device)


def stats_dict(t) -> dict:
    v = t.cpu().numpy().astype(np.uint64)
    return {f: int(v[i]) for i, f in enumerate(STAT_FIELDS)}
