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
    for c in autotune.CLASSES:
        for mi in range(len(autotune.M_BUCKETS)):
            for ni in range(len(autotune.N_BUCKETS)):
                e = tab["cells"][f"{c}/{mi}/{ni}"]
                assert e["tile_kib"] in grid["tile_kib"] and e["wgs_per_cu"] in grid["wgs_per_cu"]
                assert e["peel"] in grid["peel"]
                # the kept setting is the fastest timing of its cell
                cell = {k: v for k, v in tab["timings_us"].items() if k.startswith(f"{c}/{mi}/{ni}/")}
                assert len(cell) == len(grid["tile_kib"]) * len(grid["wgs_per_cu"]) * len(grid["peel"])
                assert e["us"] == min(cell.values())
    assert grid["peel"] == list(autotune.PEELS)


def test_params_for_reads_the_device_table(monkeypatch):
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx950", "test"))
    monkeypatch.setattr(autotune, "_table_key", None)
    tab = json.load(open(TABLE))
    h = np.zeros(256, dtype=np.uint64)
    h[:4] = 1000
    got = autotune.params_for(h, 100, 1 << 30)
    e = tab["cells"]["4/2/1"]
    assert got == {"tile_kib": e["tile_kib"], "wgs_per_cu": e["wgs_per_cu"], "peel": e["peel"]}
    monkeypatch.setattr(autotune, "_device_key", lambda: ("gfx000", "test"))   # no table for this device
    assert autotune.params_for(h, 100, 1 << 30) is None
