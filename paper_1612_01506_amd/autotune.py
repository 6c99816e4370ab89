"""Launch-parameter autotuner for single searches.

For every cell (alphabet class, pattern-length bucket, text-size bucket) the
tuner times count searches of substring patterns on a seeded synthetic text
over a grid of tile size, workgroups per compute unit and peel factor r, and
keeps the fastest setting.  None of these parameters changes a result.  The
grid holds every compiled peel factor r = 1..8, which includes the paper's
choices with frequency order: r = 2 for large alphabets, r = 3 for protein
and r = 5 for DNA (Section 3).

The table is one JSON file per GPU architecture (`tuning/<arch>.json` next to
this module), which records the HIP version it was measured with.  The
binding consults it for searches on texts whose histogram it knows (`Text`
objects) when the caller gives no explicit parameters; with no table for the
current device it passes nothing and the library's defaults apply.

    python -m paper_1612_01506_amd.autotune --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_DIR = os.path.join(_HERE, "tuning")

CLASSES = (2, 4, 20, 95)            # alphabet classes (symbols present)
M_BUCKETS = (8, 64, 512, 4096)       # upper bounds of pattern-length buckets
N_BUCKETS = (16 << 20, 1 << 62)      # upper bounds of text-size buckets
TILE_KIB = (4, 8, 16)
WGS_PER_CU = (4, 5, 6, 8)
PEELS = (1, 2, 3, 4, 5, 6, 7, 8)     # every compiled peel factor
GRID = [(tk, w, r) for tk in TILE_KIB for w in WGS_PER_CU for r in PEELS]

_table = None
_table_key = None
_device_keys: dict = {}   # device index -> (architecture, HIP version)


def alphabet_class(hist) -> int:
    nsym = int(np.count_nonzero(np.asarray(hist)))
    return 2 if nsym <= 2 else 4 if nsym <= 4 else 20 if nsym <= 32 else 95


def _bucket(v: int, bounds) -> int:
    for i, b in enumerate(bounds):
        if v <= b:
            return i
    return len(bounds) - 1


def _device_key():
    import torch

    dev = torch.cuda.current_device()
    key = _device_keys.get(dev)
    if key is None:
        props = torch.cuda.get_device_properties(dev)
        key = (props.gcnArchName.split(":")[0], torch.version.hip or "unknown")
        _device_keys[dev] = key
    return key


def load_table(path: str | None = None):
    global _table, _table_key
    if path is None:
        try:
            arch, hip = _device_key()
        except Exception:  # noqa: BLE001 - no device: no table
            return None
        path = os.path.join(TABLE_DIR, f"{arch}.json")
        key = (arch, hip)
    else:
        key = ("file", path)
    if _table_key == key:
        return _table
    _table_key = key
    _table = None
    if os.path.exists(path):
        with open(path) as f:
            _table = json.load(f)
    return _table


def params_for(hist, m: int, n: int) -> dict | None:
    """Tuned launch parameters for a pattern of length m in a text of n bytes with this histogram."""
    tab = load_table()
    if not tab:
        return None
    key = f"{alphabet_class(hist)}/{_bucket(m, M_BUCKETS)}/{_bucket(n, N_BUCKETS)}"
    e = tab["cells"].get(key)
    if e is None:
        return None
    return {"tile_kib": e["tile_kib"], "wgs_per_cu": e["wgs_per_cu"], "peel": e["peel"]}


def tune(sizes=(8 << 20, 1 << 30), patterns_per_cell: int = 4, rounds: int = 3, log=print) -> dict:
    """Every setting of a cell is timed once per round, the rounds interleaved over the grid so that
    slow drifts of the device hit all settings alike; a setting's time is its median over the rounds."""
    import torch

    from . import Patterns, Text
    import synth

    dev = torch.device("cuda:0")
    arch, hip = _device_key()
    cells = {}
    timings = {}
    for ni, n in enumerate(sizes):
        for sigma in CLASSES:
            if sigma == 95:
                t_host = synth.zipf_text(n, 95, 1.0, family=7, stream=ni)
            else:
                t_host = synth.uniform_text(n, sigma, family=7, stream=10 * ni + sigma)
            t = Text(torch.from_numpy(t_host).to(dev))
            g = synth.rng(7, 100 + sigma + ni)
            lo = 1
            for mi, mhi in enumerate(M_BUCKETS):
                ms = [int(x) for x in np.linspace(lo, mhi, patterns_per_cell).round()]
                lo = mhi + 1
                pats = [synth.substring_pattern(t_host, min(m, n), g)[0] for m in ms]
                ps = Patterns(pats, "freq", t.hist)
                out = torch.zeros(1, dtype=torch.int64, device=dev)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                samples = {cfg: [] for cfg in GRID}
                for rnd in range(rounds + 1):          # round 0 warms up (attributes, caches) and is not kept
                    for tk, w, r in GRID:
                        e0.record()
                        for i in range(len(pats)):
                            ps.count_async(i, t.t, out, peel=r, tile_kib=tk, wgs_per_cu=w)
                        e1.record()
                        torch.cuda.synchronize()
                        if rnd:
                            samples[(tk, w, r)].append(e0.elapsed_time(e1) * 1e3 / len(pats))
                best = None
                for (tk, w, r), v in samples.items():
                    us = float(np.median(v))
                    timings[f"{sigma}/{mi}/{ni}/{tk}/{w}/{r}"] = round(us, 2)
                    if best is None or us < best[0]:
                        best = (us, tk, w, r)
                ps.close()
                key = f"{sigma}/{mi}/{ni}"
                cells[key] = {"tile_kib": best[1], "wgs_per_cu": best[2], "peel": best[3],
                              "us": round(best[0], 2), "text_bytes": n, "m": ms}
                log(f"[autotune] class {sigma} m<={mhi} n={n}: {cells[key]}")
            del t
            torch.cuda.empty_cache()
    return {"arch": arch, "hip": hip, "created": time.strftime("%Y-%m-%d"),
            "grid": {"tile_kib": list(TILE_KIB), "wgs_per_cu": list(WGS_PER_CU), "peel": list(PEELS)},
            "classes": list(CLASSES), "m_buckets": list(M_BUCKETS), "n_buckets": list(N_BUCKETS),
            "cells": cells, "timings_us": timings}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--rounds", type=int, default=3)
    args = ap.parse_args()
    tab = tune(rounds=args.rounds)
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
    print(f"wrote {args.out}: {len(tab['cells'])} cells")


if __name__ == "__main__":
    main()
