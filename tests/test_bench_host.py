"""Host logic of the benchmark: the algorithmic-bytes model, the kernel name of
a launch setting, and the lookup of measured HBM traffic (valid only for the
profiled kernel sources and launch settings)."""
import hashlib
import json
import os
import shutil

import bench
from paper_2305_07238_amd import binding as B

SORT, DEFER = B.PMC_FLAG_SORT, B.PMC_FLAG_DEFER


def test_kernel_bytes_model():
    """Method bytes: hit data, sorted index, one cell per first lookup, one entry
    per stored value, four texels per image-texture evaluation; the rest
    (repeated lookups and hit reads of deferred hits, attempts that stored
    nothing) is overhead."""
    st = dict(probes=10, probes_deferred=2, deferred=3, insert_attempts=9, inserts=4,
              overwrites=1, texture_evals=7)
    n = 100
    assert bench.kernel_bytes(st, n) == n * (40 + 4 + 28) + 10 * 128 + 5 * 16 + 7 * 16
    assert bench.overhead_bytes(st) == 2 * 128 + 3 * 44 + 4 * 16


def test_kernel_names_follow_the_launch_setting():
    assert bench.shade_kernel_name("cached", SORT | DEFER) == "k_shade_flat_w4<1, 1, false, false>"
    assert bench.shade_kernel_name("cached", SORT) == "k_shade_flat_w4<1, 0, false, false>"
    assert bench.shade_kernel_name("snapshot", SORT | DEFER | B.PMC_FLAG_PERSISTENT) == \
        "k_shade_persistent_w4<2, 1, false, false>"
    # deferral needs a table: the uncached kernel never probes first
    assert bench.shade_kernel_name("uncached", SORT | DEFER) == "k_shade_flat<0, 0, false, false>"


def _tree(tmp_path, records):
    """A copy of the kernel sources and a traffic file under tmp_path."""
    src = os.path.join(bench.ROOT, "paper_2305_07238_amd", "csrc")
    dst = tmp_path / "paper_2305_07238_amd" / "csrc"
    dst.mkdir(parents=True)
    h = hashlib.sha256()
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, name), dst / name)
        h.update((dst / name).read_bytes())
    for r in records:
        r.setdefault("source_sha256", h.hexdigest())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "shade_w_traffic.json").write_text(json.dumps(records))
    return dst


def test_traffic_only_for_the_profiled_sources_and_settings(tmp_path, monkeypatch):
    early = dict(flags=SORT | DEFER, chunk_waves=4, defer_max=48, waves_per_block=0)
    late = dict(flags=SORT, chunk_waves=1, defer_max=0, waves_per_block=0)
    recs = [dict(flags=SORT | DEFER, chunk_waves=4, defer_max=48, waves_per_block=4,
                 traffic_bytes_per_launch=1.0),
            dict(flags=SORT | DEFER, chunk_waves=4, defer_max=48, waves_per_block=4, late_frame=4,
                 late=dict(flags=SORT, chunk_waves=1, defer_max=0, waves_per_block=4),
                 traffic_bytes_per_launch=2.0)]
    dst = _tree(tmp_path, recs)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", early)["traffic_bytes_per_launch"] == 1.0
    assert bench.measured_traffic("w", early, 4, late)["traffic_bytes_per_launch"] == 2.0
    assert bench.measured_traffic("w", dict(early, defer_max=32)) is None
    assert bench.measured_traffic("w", dict(early, waves_per_block=1)) is None
    assert bench.measured_traffic("w", early, 5, late) is None
    assert bench.measured_traffic("w", early, 4, dict(late, chunk_waves=2)) is None
    assert bench.measured_traffic("other", early) is None
    # any change to the kernel sources invalidates the record
    with open(dst / "shade.hip", "a") as f:
        f.write("\n")
    assert bench.measured_traffic("w", early) is None
