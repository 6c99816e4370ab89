"""Launch-parameter autotuner for single searches and batches.

For every cell (alphabet class, pattern-length bucket, text-size bucket) the
tuner times count searches of substring patterns on a seeded synthetic text
over a grid of tile size, workgroups per compute unit and peel factor r, and
keeps the fastest setting.  None of these parameters changes a result.  The
grid holds every compiled peel factor r = 1..8, which includes the paper's
choices with frequency order: r = 2 for large alphabets, r = 3 for protein
and r = 5 for DNA (Section 3).  Cells of texts over at most 4 symbols also
time the bitmap compares (SM_BITMAP: bitmap tile size, workgroups per CU and
r), and a cell records which mode won.

The table is a JSON file per GPU architecture and HIP version next to this
module: `tuning/<arch>-hip<version>.json` when one was measured with the
running HIP version, else `tuning/<arch>.json` (any version; `table_status()`
says which file is in use and whether its recorded HIP version matches).  The
binding consults it for searches on texts whose histogram it knows (`Text`
objects) when the caller gives no explicit parameters; with no table for the
current device it passes nothing and the library's defaults apply.

Batches are tuned as a separate section (`tune_batch`): per alphabet class the
query count from which the bitmap mode beats byte tiles, the bitmap work item's
query chunk and the batch peel; for byte-tile batches the tile size and the
workgroups per compute unit of single-query deals and of multi-query chunks.
The binding passes that section with every batched call that gives no explicit
launch parameters.

    python -m paper_1612_01506_amd.autotune --out tuned.json [--only single|batch|both]
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
BM_CLASSES = (2, 4)                  # classes whose cells also time the bitmap compares
BM_TILE_KIB = (8, 16, 32)
BM_WGS_PER_CU = (4, 6, 8)
BM_PEELS = (1, 2, 3, 4)
BM_GRID = [(tk, w, r) for tk in BM_TILE_KIB for w in BM_WGS_PER_CU for r in BM_PEELS]

_table = None
_table_key = None
_table_path = None
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


def table_paths(arch: str, hip: str) -> list:
    """Candidate table files for a device, most specific first."""
    return [os.path.join(TABLE_DIR, f"{arch}-hip{hip}.json"), os.path.join(TABLE_DIR, f"{arch}.json")]


def load_table(path: str | None = None):
    global _table, _table_key, _table_path
    if path is None:
        try:
            arch, hip = _device_key()
        except Exception:  # noqa: BLE001 - no device: no table
            return None
        key = (arch, hip)
        if _table_key == key:
            return _table
        path = next((c for c in table_paths(arch, hip) if os.path.exists(c)), None)
    else:
        key = ("file", path)
        if _table_key == key:
            return _table
    _table_key = key
    _table = None
    _table_path = None
    if path is not None and os.path.exists(path):
        with open(path) as f:
            _table = json.load(f)
        _table_path = path
    return _table


def table_status() -> dict:
    """The tuning table in use for the current device: its file, the HIP version it records and
    whether that is the running one (a table from another version still applies: its settings
    only change speed)."""
    tab = load_table()
    try:
        hip = _device_key()[1]
    except Exception:  # noqa: BLE001 - no device
        hip = None
    if not tab:
        return {"table": None, "runtime_hip": hip}
    return {"table": os.path.basename(_table_path), "table_hip": tab.get("hip"), "runtime_hip": hip,
            "same_hip": tab.get("hip") == hip}


def params_for(hist, m: int, n: int) -> dict | None:
    """Tuned launch parameters for a pattern of length m in a text of n bytes with this histogram."""
    tab = load_table()
    if not tab:
        return None
    key = f"{alphabet_class(hist)}/{_bucket(m, M_BUCKETS)}/{_bucket(n, N_BUCKETS)}"
    e = tab["cells"].get(key)
    if e is None:
        return None
    return {"tile_kib": e["tile_kib"], "wgs_per_cu": e["wgs_per_cu"], "peel": e["peel"],
            "bitmap": bool(e.get("bitmap", False))}


def batch_tune() -> dict | None:
    """The tuning table's batch section for this device (per alphabet class: bitmap threshold,
    bitmap chunk and peel; byte-tile tile size and workgroups per CU), or None."""
    tab = load_table()
    if not tab:
        return None
    return tab.get("batch")


def tune(sizes=(8 << 20, 1 << 30), patterns_per_cell: int = 4, rounds: int = 3, log=print,
         classes=CLASSES) -> dict:
    """Every setting of a cell is timed once per round, the rounds interleaved over the grid so that
    slow drifts of the device hit all settings alike; a setting's time is its median over the rounds.
    classes: the alphabet classes to tune (the others are left out of the result)."""
    import torch

    from . import Patterns, Text
    import synth

    dev = torch.device("cuda:0")
    arch, hip = _device_key()
    cells = {}
    timings = {}
    for ni, n in enumerate(sizes):
        for sigma in classes:
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
                grid = [(False,) + g for g in GRID]
                if sigma in BM_CLASSES:
                    grid += [(True,) + g for g in BM_GRID]
                samples = {cfg: [] for cfg in grid}
                for rnd in range(rounds + 1):          # round 0 warms up (attributes, caches) and is not kept
                    for bm, tk, w, r in grid:
                        e0.record()
                        for i in range(len(pats)):
                            ps.count_async(i, t.t, out, peel=r, tile_kib=tk, wgs_per_cu=w, bitmap=bm)
                        e1.record()
                        torch.cuda.synchronize()
                        if rnd:
                            samples[(bm, tk, w, r)].append(e0.elapsed_time(e1) * 1e3 / len(pats))
                best = None
                for (bm, tk, w, r), v in samples.items():
                    us = float(np.median(v))
                    timings[f"{sigma}/{mi}/{ni}/{'bm/' if bm else ''}{tk}/{w}/{r}"] = round(us, 2)
                    if best is None or us < best[0]:
                        best = (us, tk, w, r, bm)
                ps.close()
                key = f"{sigma}/{mi}/{ni}"
                cells[key] = {"tile_kib": best[1], "wgs_per_cu": best[2], "peel": best[3], "bitmap": best[4],
                              "us": round(best[0], 2), "text_bytes": n, "m": ms}
                log(f"[autotune] class {sigma} m<={mhi} n={n}: {cells[key]}")
            del t
            torch.cuda.empty_cache()
    return {"arch": arch, "hip": hip, "created": time.strftime("%Y-%m-%d"),
            "grid": {"tile_kib": list(TILE_KIB), "wgs_per_cu": list(WGS_PER_CU), "peel": list(PEELS),
                     "bitmap": {"classes": list(BM_CLASSES), "tile_kib": list(BM_TILE_KIB),
                                "wgs_per_cu": list(BM_WGS_PER_CU), "peel": list(BM_PEELS)}},
            "classes": list(CLASSES), "m_buckets": list(M_BUCKETS), "n_buckets": list(N_BUCKETS),
            "cells": cells, "timings_us": timings}


def _time_plans(plans, out, rounds: int, reps: int = 3) -> list[float]:
    """Median device time (us) of each plan's run, rounds interleaved over the plans."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    samples = [[] for _ in plans]
    for rnd in range(rounds + 1):                  # round 0 warms up and is not kept
        for k, pl in enumerate(plans):
            e0.record()
            for _ in range(reps):
                pl.run(out)
            e1.record()
            torch.cuda.synchronize()
            if rnd:
                samples[k].append(e0.elapsed_time(e1) * 1e3 / reps)
    return [float(np.median(v)) for v in samples]


BM_KS = (4, 8, 16, 32, 64, 128)          # queries per text tried for the bitmap / byte-tile threshold
BM_CHUNKS = (256, 512, 1024)
BATCH_PEELS = (0, 1, 2, 3, 4, 5)        # 0: the library's frequency model
BT_TILES = (4, 8, 16)
BT_WGS = (8, 12, 16, 24, 32)
DEAL_WGS = (12, 16, 24, 32, 48)


def tune_batch(n: int = 512 << 20, rounds: int = 3, log=print) -> dict:
    """The batched path's launch parameters.  Per alphabet class on an n-byte text: the number of
    queries from which the bitmap mode is faster than byte tiles, the bitmap work item's query
    chunk, and the peel of batched queries (the frequency model or a fixed r); then, on many
    texts of 4 KiB - 4 MiB, the tile size and workgroups per CU of single-query deals and of
    chunks of several queries.  Every setting is a plan timed over interleaved rounds (median);
    none changes a count, which each setting's first run is checked for."""
    import torch

    from . import BatchPlan, PackedTexts, Text
    import synth

    dev = torch.device("cuda:0")
    sec = {"bm_min": [0] * 4, "bm_chunk": [0] * 4, "peel": [0] * 4, "timings_us": {}}
    out = torch.empty(4096, dtype=torch.int64, device=dev)
    for ci, sigma in enumerate(CLASSES):
        t_host = (synth.zipf_text(n, 95, 1.0, family=8, stream=ci) if sigma == 95 else
                  synth.uniform_text(n, sigma, family=8, stream=ci))
        text = Text(torch.from_numpy(t_host).to(dev))
        g = synth.rng(8, 50 + ci)
        ms = synth.loguniform_ints(2, 1024, 1024, g)
        pats = [synth.substring_pattern(t_host, int(m), g)[0] if k % 2 == 0 else
                synth.random_pattern(synth.ALPHABETS[sigma], int(m), g) for k, m in enumerate(ms)]

        def plans_for(qs, variants):
            pl = [BatchPlan([text], [(0, p) for p in qs], tune=v) for v in variants]
            ref = None
            for x in pl:
                x.run(out)
                torch.cuda.synchronize()
                got = out[:len(qs)].clone()
                assert ref is None or torch.equal(got, ref), "a tuning setting changed a count"
                ref = got
            return pl

        # threshold: bitmap (bm_min 1) against byte tiles (bm_min huge) at k queries
        best_k = None
        for k in BM_KS:
            qs = pats[:k]
            pl = plans_for(qs, [{"bm_min": [1] * 4}, {"bm_min": [1 << 30] * 4}])
            tb, tt = _time_plans(pl, out, rounds)
            for x in pl:
                x.close()
            sec["timings_us"][f"{sigma}/threshold/{k}"] = {"bitmap": round(tb, 1), "byte_tiles": round(tt, 1)}
            if best_k is None and tb <= tt:
                best_k = k
        sec["bm_min"][ci] = best_k if best_k is not None else 2 * BM_KS[-1]
        # bitmap chunk and peel on all 1024 queries
        pl = plans_for(pats, [{"bm_min": [1] * 4, "bm_chunk": [c] * 4} for c in BM_CHUNKS])
        tc = _time_plans(pl, out, rounds)
        for x in pl:
            x.close()
        sec["bm_chunk"][ci] = BM_CHUNKS[int(np.argmin(tc))]
        sec["timings_us"][f"{sigma}/chunk"] = {str(c): round(v, 1) for c, v in zip(BM_CHUNKS, tc)}
        pl = plans_for(pats, [{"bm_min": [1] * 4, "bm_chunk": [sec["bm_chunk"][ci]] * 4, "peel": [r] * 4}
                              for r in BATCH_PEELS])
        tp = _time_plans(pl, out, rounds)
        for x in pl:
            x.close()
        sec["peel"][ci] = BATCH_PEELS[int(np.argmin(tp))]
        sec["timings_us"][f"{sigma}/peel"] = {str(r): round(v, 1) for r, v in zip(BATCH_PEELS, tp)}
        log(f"[autotune] batch class {sigma}: bm_min {sec['bm_min'][ci]} chunk {sec['bm_chunk'][ci]} "
            f"peel {sec['peel'][ci]} (0 = model)")
        del text
        torch.cuda.empty_cache()
    # byte tiles on many texts: single-query deals, then chunks of 8 queries per text
    texts_h, pats2 = synth.batched_many_texts_workload(ntexts=1024)
    hists = np.stack([np.bincount(t, minlength=256).astype(np.uint64) for t in texts_h])
    total = sum(t.size for t in texts_h)
    buf = torch.empty(total, dtype=torch.uint8, device=dev)
    offs = np.cumsum([0] + [t.size for t in texts_h[:-1]])
    for o, t in zip(offs, texts_h):
        buf[int(o):int(o) + t.size].copy_(torch.from_numpy(t))
    packed = PackedTexts(buf, offs, [t.size for t in texts_h], hists)
    solo_q = [(i, p) for i, p in enumerate(pats2)]
    g = synth.rng(8, 99)
    multi_q = [(i, synth.substring_pattern(texts_h[i], int(synth.loguniform_ints(4, 256, 1, g)[0]), g)[0])
               for i in range(0, 1024, 4) for _ in range(8)]
    base = {k: list(sec[k]) for k in ("bm_min", "bm_chunk", "peel")}
    grid = [(tk, w) for tk in BT_TILES for w in DEAL_WGS]
    byte = dict(base, bm_min=[1 << 30] * 4)          # byte tiles whatever the query count
    pl = [BatchPlan(packed, solo_q, tune=dict(byte, tile_kib=tk, deal_wgs_per_cu=w)) for tk, w in grid]
    td = _time_plans(pl, out, rounds)
    for x in pl:
        x.close()
    tk_best, dw_best = grid[int(np.argmin(td))]
    sec["timings_us"]["deals"] = {f"{tk}/{w}": round(v, 1) for (tk, w), v in zip(grid, td)}
    grid2 = [(tk_best, w) for w in BT_WGS]
    pl = [BatchPlan(packed, multi_q, tune=dict(byte, tile_kib=tk, deal_wgs_per_cu=dw_best, wgs_per_cu=w))
          for tk, w in grid2]
    tm = _time_plans(pl, out, rounds)
    for x in pl:
        x.close()
    sec["timings_us"]["chunks"] = {f"{tk}/{w}": round(v, 1) for (tk, w), v in zip(grid2, tm)}
    sec.update(tile_kib=tk_best, deal_wgs_per_cu=dw_best, wgs_per_cu=grid2[int(np.argmin(tm))][1])
    log(f"[autotune] batch byte tiles: tile {tk_best} KiB, deals {dw_best}/CU, chunks {sec['wgs_per_cu']}/CU")
    return sec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--rounds", type=int, default=3)
    ap.add_argument("--only", choices=["single", "batch", "both"], default="both")
    ap.add_argument("--base", help="table whose other section is kept (with --only), and whose cells of "
                                   "the classes not tuned (with --classes)")
    ap.add_argument("--classes", type=int, nargs="+", default=list(CLASSES),
                    help="alphabet classes whose single-search cells are tuned")
    args = ap.parse_args()
    tab = json.load(open(args.base)) if args.base else {}
    if args.only in ("single", "both"):
        new = tune(rounds=args.rounds, classes=tuple(args.classes))
        pre = tuple(f"{c}/" for c in args.classes)
        cells = {k: v for k, v in tab.get("cells", {}).items() if not k.startswith(pre)}
        timings = {k: v for k, v in tab.get("timings_us", {}).items() if not k.startswith(pre)}
        cells.update(new.pop("cells"))
        timings.update(new.pop("timings_us"))
        tab.update(new, cells=cells, timings_us=timings)
    if args.only in ("batch", "both"):
        tab["batch"] = tune_batch(rounds=args.rounds)
        if "arch" not in tab:
            arch, hip = _device_key()
            tab.update(arch=arch, hip=hip)
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
    print(f"wrote {args.out}: {len(tab.get('cells', {}))} single-search cells, "
          f"batch section {'yes' if 'batch' in tab else 'no'}")


if __name__ == "__main__":
    main()
