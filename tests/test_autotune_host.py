"""Host-side checks of the update-form autotuner: its tables agree with each other and with the
library's tile ids, every id it can choose has launch names for the profile summaries, and the cache
keeps a choice only for the kernel sources it was timed on."""
import json
import os

import pytest

from paper_1509_02572_amd import autotune as A

STREAM_IDS = sorted(A.STREAM_CHUNK)


def test_stream_tables_agree():
    assert STREAM_IDS == list(range(21, 30))
    assert sorted(A.STREAM_NBAR) == STREAM_IDS
    for t in STREAM_IDS:
        ty, tz = A.TILE_IDS[t]
        assert ty * tz in (128, 256, 512)
        assert A.STREAM_CHUNK[t] in (32, 64) and A.STREAM_NBAR[t] in (1, 2)
    # every batch candidate is a batch tile or a streaming form
    for t in A.BATCH_CANDIDATES:
        assert t in A.BATCH_TILES or t in STREAM_IDS
    for t in A.REFINED_CANDIDATES:
        assert t in A.BATCH_TILES


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_kernel_names_cover_every_choice(prec):
    t = "float" if prec == "f32" else "double"
    for tid in [0] + list(A.TILE_IDS):
        names = A.kernel_names(tid, prec)
        assert len(names) == 2 and all(n.startswith("cc::k_") and t in n for n in names)
    # the two-pass form: its prepare pass and point pass
    assert A.kernel_names(20, prec) == (f"cc::k_prepare<{t}>", f"cc::k_stage_points<{t}, 0>")
    # streaming forms: the template arguments of the launch (threads, chunk, waves, barriers)
    w = 4 if prec == "f32" else 1
    for tid in STREAM_IDS:
        ty, tz = A.TILE_IDS[tid]
        reg, band = A.kernel_names(tid, prec)
        assert reg == f"cc::k_stage_stream<{t}, {ty}, {tz}, {A.STREAM_CHUNK[tid]}, {w}, {A.STREAM_NBAR[tid]}>"
        assert band == f"cc::k_stage_tiled<{t}, 8, 8, 1, 0, 1, 1, false, 2>"
    assert A.kernel_names(21, prec, small=True)[1] == f"cc::k_stage_tiled<{t}, 4, 4, 4, 0, 1, 1, false, 2>"


def test_cache_keyed_by_source_hash(tmp_path):
    path = str(tmp_path / "cache.json")
    A._store("grid:f32:8x8x8", 22, {21: 1.5, 22: 1.25}, path)
    ent = A._lookup("grid:f32:8x8x8", path)
    assert ent["tile"] == 22 and ent["ms"] == {"21": 1.5, "22": 1.25}
    assert ent["source_hash"] == A.source_hash()
    # a choice timed on other kernel sources is not reused
    cache = json.load(open(path))
    cache["grid:f32:8x8x8"]["source_hash"] = "0" * 16
    json.dump(cache, open(path, "w"))
    assert A._lookup("grid:f32:8x8x8", path) is None
    assert A._lookup("grid:f32:8x8x8", None) is None


def test_committed_cache_is_well_formed():
    if not os.path.exists(A.CACHE):
        pytest.skip("no tuning cache")
    cache = A.load_cache()
    for k, ent in cache.items():
        kind = k.split(":")[0]
        assert kind in ("grid", "batch", "refined"), k
        assert str(ent["tile"]) in ent["ms"], k
        assert ent["ms"][str(ent["tile"])] == min(ent["ms"].values()), k
        allowed = {"grid": [0] + list(A.TILE_IDS), "batch": A.BATCH_CANDIDATES,
                   "refined": A.REFINED_CANDIDATES}[kind]
        assert ent["tile"] in allowed, k
