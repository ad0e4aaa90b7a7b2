"""Helpers shared by the GPU tests: run scenes through the C ABI, fetch results."""
import numpy as np

from paper_2305_07238_amd import scenes

# FP32 vs the FP64 oracle: |gpu - ref| <= RTOL * max(|ref|, 1).  BSDF inputs are
# unit-scale quantities (colours and roughness in [0, 1], unit normals), so the
# 1e-5 relative bound is taken relative to max(|ref|, 1).
RTOL = 1e-5


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1.0)


def max_rel(gpu, ref):
    e = rel_err(gpu, ref)
    return float(np.nanmax(e)) if e.size else 0.0


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


def small_mid_scene(seed=0, frames=2):
    """The mid workload's material set (64 graphs of 8-64 nodes, 16 textures of
    1024^2) on a 480 x 240 screen: spans many waves and every material class."""
    return scenes.mid_scene(seed=seed, width=480, height=240, frames=frames)
