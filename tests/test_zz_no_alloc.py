"""pmc_shade_static (the entry point that allocates nothing) against pmc_shade.

Two calls in a row on the same device, the second with a smaller batch, in
several launch settings: outputs and counters equal those of pmc_shade bit
for bit (same kernels, workspace in the fixed device array).  CACHED mode runs
on copies of a table that already holds every key of the batch, so no insert
races and the results are unique.  Requests beyond the array are refused
before anything is enqueued."""
import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2305_07238_amd import binding as B  # noqa: E402

SETTINGS = {
    "flat": dict(flags=0),
    "sorted": dict(flags=B.PMC_FLAG_SORT),
    "sorted_defer": dict(flags=B.PMC_FLAG_SORT | B.PMC_FLAG_DEFER, chunk_waves=4),
    "persistent": dict(flags=B.PMC_FLAG_SORT | B.PMC_FLAG_PERSISTENT, chunk_waves=2),
}


def _run(ctx, hits_np, cache, static, **kw):
    import torch as T
    n = len(hits_np)
    hits = B.hits_to_device(hits_np)
    out = B.alloc_outputs(n)
    for v in out.values():
        v.fill_(float("nan"))
    stats = B.new_stats()
    ctx.shade(hits, out, cache, stats=stats, static=static, **kw)
    T.cuda.synchronize()
    return G.to_numpy(out), B.stats_dict(stats)


@pytest.mark.parametrize("setting", list(SETTINGS))
@pytest.mark.parametrize("mode", ["uncached", "cached"])
def test_static_entry_point_matches_pmc_shade(mode, setting):
    sc = G.small_mid_scene(frames=2)
    ctx = G.setup(sc)
    batches = [sc.frame(0), sc.frame(1).take(np.arange(7, 40007))]   # second call smaller
    kw = dict(SETTINGS[setting])
    if mode == "cached":
        # a table holding every key of both batches (snapshot frames, no full cells)
        base = ctx.cache(1 << 18, 8, 16)
        for f, h in enumerate(batches):
            _run(ctx, h, base, False, mode=B.PMC_MODE_SNAPSHOT, frame=f, flags=B.PMC_FLAG_SORT)
        raw = base.export()
        kw["mode"] = B.PMC_MODE_CACHED
        kw["frame"] = 2
    else:
        kw["mode"] = B.PMC_MODE_UNCACHED
    for i, h in enumerate(batches):
        ca = cb = None
        if mode == "cached":
            ca, cb = ctx.cache(1 << 18, 8, 16), ctx.cache(1 << 18, 8, 16)
            ca.import_(raw)
            cb.import_(raw)
        ref, st_ref = _run(ctx, h, ca, False, **kw)
        got, st_got = _run(ctx, h, cb, True, **kw)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (i, k)
        assert st_got == st_ref, i
        assert st_got["hits_shaded"] == len(h)
        if mode == "cached":
            assert st_got["cache_hits"] == st_got["probes"] > 0       # every key present
            assert st_got["inserts"] == 0
            assert np.array_equal(cb.export(), ca.export())


def test_static_entry_point_refuses_what_does_not_fit():
    sc = G.small_mid_scene(frames=1)
    ctx = G.setup(sc)
    h = sc.frame(0)
    hits = B.hits_to_device(h)
    out = B.alloc_outputs(len(h))
    cache = ctx.cache(1 << 12, 8, 16)
    with pytest.raises(B.PmcError) as e:
        ctx.shade(hits, out, cache, mode=B.PMC_MODE_SNAPSHOT, static=True)
    assert e.value.code == B.PMC_ERR_UNSUPPORTED
    # more hits than the array is sized for: refused on the host (the arrays are
    # never read: the size check comes first)
    big = {k: v for k, v in hits.items()}
    n_big = B.PMC_STATIC_MAX_HITS + 1
    p = B.pmc_hits(B._ptr(big["material"]), B._ptr(big["uv"]), B._ptr(big["duv"]),
                   B._ptr(big["normal"]), n_big, None)
    o = B.pmc_bsdf_out(B._ptr(out["base_color"]), B._ptr(out["roughness"]),
                       B._ptr(out["normal"]))
    prm = B.pmc_shade_params(B.PMC_MODE_UNCACHED, B.PMC_FLAG_SORT, 0, 0, 0, 0, 0)
    import ctypes as C
    st = B.pmc_shade_static(ctx.h, None, C.byref(p), C.byref(o), C.byref(prm), None, None,
                            None)
    assert st == B.PMC_ERR_UNSUPPORTED
    assert b"at most" in B.pmc_last_error(ctx.h)
