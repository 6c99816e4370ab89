"""Autotuner table lookups (host logic only; the timing sweep itself needs a GPU)."""
import json
import os

import numpy as np

from paper_1612_01506_amd import autotune

TABLE = os.path.join(autotune.TABLE_DIR, "gfx950.json")


def test_alphabet_class_boundaries():
    for nsym, want in ((1, 2), (2, 2), (3, 4), (4, 4), (5, 20), (32, 20), (33, 95), (256, 95)):
        h = np.zeros(256, dtype=np.uint64)
        h[:nsym] = 7
        assert autotune.alphabet_class(h) == want, nsym


def test_buckets():
    assert [autotune._bucket(m, autotune.M_BUCKETS) for m in (1, 8, 9, 64, 65, 512, 513, 4096, 10**6)] == \
        [0, 0, 1, 1, 2, 2, 3, 3, 3]
    assert [autotune._bucket(n, autotune.N_BUCKETS) for n in (1, 16 << 20, (16 << 20) + 1, 1 << 40)] == [0, 0, 1, 1]


def test_committed_table_is_complete_and_inside_its_grid():
    tab = json.load(open(TABLE))
    grid = tab["grid"]
    bm = grid["bitmap"]
    assert bm["classes"] == list(autotune.BM_CLASSES)
    for c in autotune.CLASSES:
        for mi in range(len(autotune.M_BUCKETS)):
            for ni in range(len(autotune.N_BUCKETS)):
                e = tab["cells"][f"{c}/{mi}/{ni}"]
                g = bm if e.get("bitmap") else grid
                assert e["tile_kib"] in g["tile_kib"] and e["wgs_per_cu"] in g["wgs_per_cu"]
                assert e["peel"] in g["peel"]
                assert not e.get("bitmap") or c in bm["classes"]
                # the kept setting is the fastest timing of its cell, over both compare modes
                pre = f"{c}/{mi}/{ni}/"
                byte_t = {k: v for k, v in tab["timings_us"].items() if k.startswith(pre) and "/bm/" not in k}
                bm_t = {k: v for k, v in tab["timings_us"].items() if k.startswith(pre + "bm/")}
                assert len(byte_t) == len(grid["tile_kib"]) * len(grid["wgs_per_cu"]) * len(grid["peel"])
                want_bm = len(bm["tile_kib"]) * len(bm["wgs_per_cu"]) * len(bm["peel"]) if c in bm["classes"] else 0
                assert len(bm_t) == want_bm
                assert e["us"] == min(list(byte_t.values()) + list(bm_t.values()))
                key = f"{pre}{'bm/' if e.get('bitmap') else ''}{e['tile_kib']}/{e['wgs_per_cu']}/{e['peel']}"
                assert tab["timings_us"][key] == e["us"]
    assert grid["peel"] == list(autotune.PEELS)


def test_params_for_reads_the_device_table(monkeypatch):
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx950", "test"))
    monkeypatch.setattr(autotune, "_table_key", None)
    tab = json.load(open(TABLE))
    h = np.zeros(256, dtype=np.uint64)
    h[:4] = 1000
    got = autotune.params_for(h, 100, 1 << 30)
    e = tab["cells"]["4/2/1"]
    assert got == {"tile_kib": e["tile_kib"], "wgs_per_cu": e["wgs_per_cu"], "peel": e["peel"],
                   "bitmap": bool(e.get("bitmap"))}
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx000", "test"))   # no table for this device
    assert autotune.params_for(h, 100, 1 << 30) is None


def test_committed_batch_section_is_complete_and_its_choices_are_the_fastest():
    b = json.load(open(TABLE))["batch"]
    tm = b["timings_us"]
    for ci, c in enumerate(autotune.CLASSES):
        # bitmap threshold: the first tried query count at which the bitmap mode was not slower
        ks = [k for k in autotune.BM_KS if tm[f"{c}/threshold/{k}"]["bitmap"] <= tm[f"{c}/threshold/{k}"]["byte_tiles"]]
        assert b["bm_min"][ci] == (ks[0] if ks else 2 * autotune.BM_KS[-1])
        chunk = tm[f"{c}/chunk"]
        assert b["bm_chunk"][ci] == int(min(chunk, key=chunk.get))
        peel = tm[f"{c}/peel"]
        assert b["peel"][ci] == int(min(peel, key=peel.get)) and 0 <= b["peel"][ci] <= 8
    deals = tm["deals"]
    assert f"{b['tile_kib']}/{b['deal_wgs_per_cu']}" == min(deals, key=deals.get)
    chunks = tm["chunks"]
    assert f"{b['tile_kib']}/{b['wgs_per_cu']}" == min(chunks, key=chunks.get)


def test_batch_params_record(monkeypatch):
    """The binding turns the table's batch section into the sm_batch_tune record it passes."""
    import paper_1612_01506_amd as sm
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx950", "test"))
    monkeypatch.setattr(autotune, "_table_key", None)
    b = json.load(open(TABLE))["batch"]
    p = sm._batch_params()._obj          # the sm_params behind the byref handed to the library
    rec = p.batch.contents
    assert list(rec.bm_min) == b["bm_min"] and list(rec.bm_chunk) == b["bm_chunk"] and list(rec.peel) == b["peel"]
    assert (rec.tile_kib, rec.wgs_per_cu, rec.deal_wgs_per_cu) == (b["tile_kib"], b["wgs_per_cu"], b["deal_wgs_per_cu"])
    assert sm._batch_params(peel=3) is not None and sm._batch_params(tune=False) is None
    custom = sm._batch_params(tune={"bm_min": [1] * 4})._obj
    assert list(custom.batch.contents.bm_min) == [1] * 4 and list(custom.batch.contents.peel) == [0] * 4


def test_tuned_params_carry_the_compare_mode(monkeypatch):
    """A cell that chose the bitmap compares sets SM_BITMAP with its bitmap tile size; asking for the
    other mode drops the cell's tile size (it is in the other mode's units)."""
    import paper_1612_01506_amd as sm
    from paper_1612_01506_amd import _lib

    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx950", "test"))
    monkeypatch.setattr(autotune, "_table_key", None)
    tab = json.load(open(TABLE))
    bm_cells = [k for k, e in tab["cells"].items() if e.get("bitmap")]
    byte_cells = [k for k, e in tab["cells"].items() if not e.get("bitmap")]
    assert bm_cells and byte_cells

    class FakeText(sm.Text):
        def __init__(self, hist, n):
            self._hist, self._n = hist, n

        @property
        def n(self):
            return self._n

    for key in (bm_cells[0], byte_cells[0]):
        c, mi, ni = (int(x) for x in key.split("/"))
        e = tab["cells"][key]
        h = np.zeros(256, dtype=np.uint64)
        h[:c] = 1
        m = autotune.M_BUCKETS[mi]
        n = autotune.N_BUCKETS[0] if ni == 0 else 1 << 30
        p = sm._params(text=FakeText(h, n), m=m)._obj
        assert bool(p.flags & _lib.SM_BITMAP) == bool(e.get("bitmap"))
        assert (p.peel, p.tile_kib, p.wgs_per_cu) == (e["peel"], e["tile_kib"], e["wgs_per_cu"])
        flipped = sm._params(text=FakeText(h, n), m=m, bitmap=not e.get("bitmap"))._obj
        assert bool(flipped.flags & _lib.SM_BITMAP) != bool(e.get("bitmap")) and flipped.tile_kib == 0


def test_table_of_the_running_hip_version_is_preferred(monkeypatch, tmp_path):
    """tuning/<arch>-hip<version>.json beats tuning/<arch>.json; either is reported with its version."""
    monkeypatch.setattr(autotune, "TABLE_DIR", str(tmp_path))
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfxT", "9.9.1"))
    for name in ("_table", "_table_key", "_table_path"):     # restored with the cache they form
        monkeypatch.setattr(autotune, name, None)
    assert autotune.load_table() is None
    assert autotune.table_status() == {"table": None, "runtime_hip": "9.9.1"}
    (tmp_path / "gfxT.json").write_text(json.dumps({"hip": "9.8.0", "cells": {}, "tag": "any"}))
    monkeypatch.setattr(autotune, "_table_key", None)
    assert autotune.load_table()["tag"] == "any"
    assert autotune.table_status() == {"table": "gfxT.json", "table_hip": "9.8.0", "runtime_hip": "9.9.1",
                                       "same_hip": False}
    (tmp_path / "gfxT-hip9.9.1.json").write_text(json.dumps({"hip": "9.9.1", "cells": {}, "tag": "exact"}))
    monkeypatch.setattr(autotune, "_table_key", None)
    assert autotune.load_table()["tag"] == "exact"
    assert autotune.table_status()["same_hip"] is True
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfxT", "9.7.0"))   # another runtime version
    assert autotune.load_table()["tag"] == "any"
