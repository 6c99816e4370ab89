#!/usr/bin/env python3
"""Benchmark of the MI355X exact-string-matching path (libsm).

Default workload (one "step" = one pass of the whole search path over one
batch of synthetic input): a 1 GiB order-0 Zipf(1.0) text over the 95
printable bytes, 100 substring patterns for each m in {2, 4, ..., 1024}:
symbol histogram of the text, frequency compare order of every pattern, one
count search per pattern and, for m >= 64, the reporting search (positions).
`value` is whole-job text throughput: bytes of text scanned by all searches
of a step divided by the step time (GB/s, 1e9 B/s), inputs resident in HBM.
After the timed steps the same line also reports, each measured on its own:
the count kernel's roofline, the CPU baselines (the oracle on this GPU's host
threads and on one thread, the paper's Algorithm 4 with AVX2), the batched
forms (10,000 patterns on a 2 GiB text; 4,096 texts) against the sequential
single-search form, and the serving loop's p50/p99 latency at a few offered
loads (--no-extras skips the last two).

Other workloads (--workload) print their own JSON line: single (8 MiB ACGT),
small (sigma 2/4 and periodic texts), batched (10,000 patterns on a 2 GiB
text; 4,096 texts), serve (continuous batching, p50/p99 latency).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload zipf]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1612_01506_amd", "csrc", "sm_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "count_staged_zipf95_1GiB_pmc.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def traffic_from_profile(n_bytes: int, kernel: str):
    """HBM bytes per count launch from the committed rocprofv3 --pmc summary, or None.

    The summary stores FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of one count
    kernel instance and of a plain copy of known size; it is used only if it
    was taken on the current kernel source and for the instance named.
    """
    if not os.path.exists(PMC_SUMMARY):
        return None
    rec = None
    for line in open(PMC_SUMMARY):
        if line.startswith("JSON "):
            rec = json.loads(line[5:])
    if not rec or rec.get("kernel_source_sha") != kernel_sha() or rec.get("kernel") != kernel:
        return None
    fscale = rec["copy_bytes"] / (rec["copy_fetch_kib"] * 1024.0)
    wscale = rec["copy_bytes"] / (rec["copy_write_kib"] * 1024.0)
    per = (rec["count_fetch_kib"] * fscale + rec["count_write_kib"] * wscale) * 1024.0
    return int(round(per * n_bytes / rec["count_text_bytes"]))


def cpu_info() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------------ zipf
def run_zipf(args):
    import torch

    import paper_1612_01506_amd as sm
    import synth

    n = args.n
    t0 = time.time()
    t_host, pats = synth.zipf_workload(n=n, per_m=args.per_m)
    log(f"[bench] text {n} B + {len(pats)} patterns generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    t_dev = torch.from_numpy(t_host).to(dev)
    torch.cuda.synchronize()
    patterns = [p for p, _ in pats]
    rep_idx = [i for i, (_, r) in enumerate(pats) if r]
    cap = 4096  # positions kept per reporting search (substrings of m >= 64 occur about once)
    posbuf = torch.empty((len(rep_idx), cap), dtype=torch.int64, device=dev)
    totals_dev = torch.empty(len(rep_idx), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    # the count kernel's launch duration is timed with HIP events on every tenth launch (ten per
    # pattern length); an event pair between two launches idles the GPU for a few microseconds
    timed_idx = set(range(0, len(patterns), 10))
    ev = {i: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for i in timed_idx}

    state = {}

    def step(timed: bool):
        # the resident text; its symbol frequencies (one histogram pass) are computed once per step and
        # select the autotuner's launch parameters for each search
        text = sm.Text(t_dev)
        ps = sm.Patterns(patterns, "freq", text.hist)             # compare orders pi + step tables -> HBM
        counts = torch.zeros(len(patterns), dtype=torch.int64, device=dev)
        for i in range(len(patterns)):
            if i in timed_idx:
                ev[i][0].record(stream)
                ps.count_async(i, text, counts[i:i + 1], stream=stream)
                ev[i][1].record(stream)
            else:
                ps.count_async(i, text, counts[i:i + 1], stream=stream)
        for k, i in enumerate(rep_idx):                                             # reporting version
            ps.report_async(i, text, posbuf[k], totals_dev[k:k + 1], stream=stream)
        state["hist"] = text.hist
        torch.cuda.synchronize()
        ps.close()
        state["counts"] = counts.cpu().numpy()
        state["totals"] = totals_dev.cpu().numpy()
        state["plist"] = [posbuf[k, :min(int(tot), cap)] for k, tot in enumerate(state["totals"])]
        if timed:
            state.setdefault("kern_ms", []).extend((i, a.elapsed_time(b)) for i, (a, b) in ev.items())

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_step = elapsed * 1e3 / args.steps
    searches = len(patterns) + len(rep_idx)
    value = searches * n / (elapsed / args.steps) / 1e9

    # ---- checks outside the timed region
    counts = state["counts"]
    for k, i in enumerate(rep_idx):
        assert state["totals"][k] == counts[i], (i, state["totals"][k], counts[i])
        pos = state["plist"][k].cpu().numpy()
        m = len(patterns[i])
        assert np.all(np.diff(pos) > 0)
        for s in pos[:64]:
            assert bytes(t_host[s:s + m]) == patterns[i]
    # histogram pass alone, launched back to back (device time; each step above also runs it once)
    hev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    sm.histogram(t_dev)
    hev[0].record(stream)
    for _ in range(5):
        sm.histogram(t_dev)
    hev[1].record(stream)
    torch.cuda.synchronize()
    hist_ms = hev[0].elapsed_time(hev[1]) / 5
    from paper_1612_01506_amd import autotune
    launch_by_m = {len(patterns[i]): autotune.params_for(state["hist"], len(patterns[i]), n)
                   for i in range(0, len(patterns), args.per_m)}
    # the dominant kernel: the (tile, peel) instance that most pattern lengths launch; its sampled
    # launches give the roofline's average duration
    def inst(m):
        tp = launch_by_m[m] or {"tile_kib": 8, "peel": 2}
        return tp["tile_kib"], min(tp["peel"], m)
    insts = [inst(len(p)) for p in patterns]
    dom = max(set(insts), key=insts.count)
    kern = np.array([ms for i, ms in state["kern_ms"] if insts[i] == dom])
    avg_ms = float(kern.mean())
    stream = str(n >= (512 << 20)).lower()   # the library streams tile loads for texts of 512 MiB and more
    traffic = traffic_from_profile(n, f"void smk::k_count_staged<{dom[0] // 4}, {dom[1]}, {stream}>(smk::CountArgs)")
    achieved = n / (avg_ms * 1e-3) / 1e9

    if args.copy_probe:
        # plain copy of known size (n bytes read, n written) for scaling the HBM counters
        dst = torch.empty_like(t_dev)
        dst.copy_(t_dev)
        torch.cuda.synchronize()
        del dst

    import cpu_alg4
    import oracle  # CPU baseline and sampled parity: the oracle as it stands
    # the host threads of this GPU's share of the box (OMP_NUM_THREADS when set), and all it has
    nproc = os.cpu_count() or 1
    ncores = max(1, min(nproc, int(os.environ.get("OMP_NUM_THREADS") or nproc)))
    # one pattern of each length in turn (the first of each, then the second, ...) until the time
    # budget is spent: a bounded sample of the same workload
    nlen = len(patterns) // args.per_m
    sample_idx = [k * args.per_m + j for j in range(args.per_m) for k in range(nlen)]

    def cpu_leg(fn, seconds):
        nb, tt, nchk = 0, 0.0, 0
        for i in sample_idx:
            if tt >= seconds:
                break
            t2 = time.perf_counter()
            want = fn(i)
            tt += time.perf_counter() - t2
            nb += n
            nchk += 1
            assert want == counts[i], ("parity", i, len(patterns[i]), want, counts[i])
        return (round(nb / tt / 1e9, 3) if tt else None), nchk, tt

    cpu_gbs, checked, cpu_t = cpu_leg(lambda i: oracle.count(patterns[i], t_host, ncores), args.cpu_seconds)
    cpu1_gbs, checked1, cpu1_t = cpu_leg(lambda i: oracle.count(patterns[i], t_host, 1), args.cpu_seconds / 3)
    alg4 = None
    if cpu_alg4.available() and args.cpu_seconds > 0:
        orders = {}

        def a4(i, th):
            if i not in orders:
                orders[i] = cpu_alg4.freq_order(patterns[i], state["hist"])
            return cpu_alg4.count(patterns[i], t_host, orders[i], min(2, len(patterns[i])), th)

        a1, c1, s1 = cpu_leg(lambda i: a4(i, 1), args.cpu_seconds / 3)
        an, cn, sn = cpu_leg(lambda i: a4(i, ncores), args.cpu_seconds / 3)
        alg4 = {"value_1_thread": a1, "value_all_threads": an, "threads": ncores, "unit": "GB/s",
                "method": "Algorithm 4 with AVX2 (32 starts per vector), frequency order from the text's "
                          "histogram, peel r = 2 (Section 3's value for large alphabets)",
                "sample": f"{c1} patterns on 1 thread ({s1:.1f} s) and {cn} on {ncores} threads ({sn:.1f} s), "
                          "lengths taken in turn, full text; every count equal to the GPU's"}
    if args.cpu_seconds > 0:
        i0 = rep_idx[0]
        assert np.array_equal(state["plist"][0].cpu().numpy().astype(np.uint64), oracle.report(patterns[i0], t_host))
    log(f"[bench] sampled parity vs oracle OK on {checked} + {checked1} patterns; report lists verified")

    extras = {}
    if not args.no_extras:
        del t_dev, posbuf, totals_dev
        state.clear()
        torch.cuda.empty_cache()
        from paper_1612_01506_amd import autotune
        bt = autotune.batch_tune() or {}
        extras["batched"] = {
            "one_text": batched_one_text(args, args.nq, 2),
            "many_texts": batched_many_texts(args, args.ntexts, 3),
            "tuning": {k: v for k, v in bt.items() if k != "timings_us"} or "library defaults",
        }
        points, info = serve_points(args, args.serve_rates, args.serve_seconds, args.max_requests)
        extras["serve"] = dict(info, points=points)
        torch.cuda.empty_cache()
        small = run_small(args)
        extras["small_alphabets"] = {
            ln["config"]["workload"].split(",")[0]: {k: v for k, v in ln["config"].items() if k.endswith("_by_m")}
            for ln in small[:2]}
        extras["small_alphabets"]["periodic_a^255b_freq_us"] = small[2]["config"]["results"]["a^255b/freq"]["us"]

    return {
        "metric": "text GB/s per search (% HBM peak)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded order-0 Zipf text and substring patterns; no corpus files)",
        "config": {
            "workload": "zipf95_1GiB: histogram + freq order + count of 100 substrings for each "
                        "m in {2..1024} + report for m >= 64",
            "text_bytes": n, "sigma": 95, "zipf_s": 1.0, "patterns": len(patterns),
            "report_searches": len(rep_idx), "searches_per_step": searches,
            "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 1),
            "launch_by_m": launch_by_m,
            "tuning_table": autotune.table_status(),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"k_count_staged<{dom[0] // 4},{dom[1]},{stream}> ({dom[0]} KiB tiles, "
                      f"peel {dom[1]})",
            "avg_launch_us": round(avg_ms * 1e3, 2),
            "median_launch_us": round(float(np.median(kern)) * 1e3, 2),
            "timed_launches": len(kern),
            "algorithmic_bytes_per_launch": n,
        },
        "histogram": {"avg_us": round(hist_ms * 1e3, 1), "GBps": round(n / (hist_ms * 1e-3) / 1e9, 1),
                      "kernel": "k_hist (per-lane LDS bin copies)"},
        "cpu_baseline": {
            "value": cpu_gbs, "unit": "GB/s", "cores": ncores, "kind": "oracle",
            "sample": f"oracle count (Algorithm 1, OpenMP over starts) of {checked} patterns "
                      f"(lengths taken in turn) over the full {n}-byte text, {cpu_t:.1f} s on {ncores} threads "
                      f"(this GPU's share of the host, OMP_NUM_THREADS); host: {cpu_info()}, {nproc} hardware threads",
            "host_nproc": nproc,
            "single_thread": {"value": cpu1_gbs, "unit": "GB/s",
                              "sample": f"{checked1} patterns, {cpu1_t:.1f} s, 1 thread"},
            "alg4_avx2": alg4,
        },
        **extras,
    }


# --------------------------------------------------------------------- batched
def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def _plan_times(sm, texts, queries, out_len, reps, want):
    """(create seconds, eager run seconds, graph replay seconds) of a BatchPlan; counts checked."""
    import torch

    t0 = time.perf_counter()
    plan = sm.BatchPlan(texts, queries)
    t_create = time.perf_counter() - t0
    out = torch.empty(out_len, dtype=torch.int64, device=want.device)
    plan.run(out)
    torch.cuda.synchronize()
    assert torch.equal(out[:len(queries)], want), "plan counts differ from the one-shot batch"
    t_run, _ = _timed(lambda: plan.run(out), reps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(out)
    out.fill_(-1)
    t_graph, _ = _timed(g.replay, reps)
    assert torch.equal(out[:len(queries)], want), "graph replay counts differ"
    del g
    plan.close()
    return t_create, t_run, t_graph


def batched_one_text(args, nq: int, reps: int):
    """10,000 patterns on one 2 GiB Zipf text: the sequential single-search form (one count launch
    per query, one final sync) against one sm_count_batch call, a plan run and a graph replay."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    dev = torch.device("cuda:0")
    n = args.n if args.n != (1 << 30) else (2 << 30)
    t0 = time.time()
    t_host, pats = synth.batched_one_text_workload(n=n, nq=nq)
    log(f"[bench] batched: {n} B text, {len(pats)} patterns in {time.time() - t0:.1f}s")
    t_dev = torch.from_numpy(t_host).to(dev)
    text = sm.Text(t_dev)
    hist = text.hist
    queries = [(0, p) for p in pats]

    def sequential():
        ps = sm.Patterns(pats, "freq", hist)
        out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
        for i in range(len(pats)):
            ps.count_async(i, t_dev, out[i:i + 1])
        torch.cuda.synchronize()
        ps.close()
        return out

    enq = []

    def batched():
        t_e = time.perf_counter()
        out = sm.count_batch([text], queries)
        enq.append(time.perf_counter() - t_e)
        return out

    batched()
    tb, cb = min((_timed(batched) for _ in range(reps)), key=lambda x: x[0])
    sequential()
    ts, cs = _timed(sequential)
    assert torch.equal(cb, cs), "batched and sequential counts differ"
    cb = cb.cpu().numpy()
    pc, pr, pg = _plan_times(sm, [text], queries, len(pats), max(reps, 3), torch.from_numpy(cb).to(dev))
    del t_dev, text
    torch.cuda.empty_cache()
    return {"patterns": len(pats), "text_bytes": n, "mean_m": round(float(np.mean([len(p) for p in pats])), 1),
            "sequential_s": round(ts, 4), "batched_s": round(tb, 4), "batched_host_enqueue_s": round(min(enq), 4),
            "plan_create_s": round(pc, 4), "plan_run_s": round(pr, 4), "plan_graph_replay_s": round(pg, 4),
            "searches_per_s": round(len(pats) / tb, 1), "sequential_searches_per_s": round(len(pats) / ts, 1),
            "speedup_vs_sequential": round(ts / tb, 2),
            "sequential_text_GBps": round(len(pats) * n / ts / 1e9, 1),
            "logical_text_GBps_batched": round(len(pats) * n / tb / 1e9, 1),
            "checked": "batched == sequential single searches, every count (oracle parity at full size: tests/)"}


def batched_many_texts(args, ntexts: int, reps: int):
    """4,096 resident texts of 4 KiB - 4 MiB with one pattern each: sequential against one batch."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    dev = torch.device("cuda:0")
    texts_h, pats2 = synth.batched_many_texts_workload(ntexts=ntexts)
    total = sum(t.size for t in texts_h)
    big = torch.empty(total + 16 * len(texts_h), dtype=torch.uint8, device=dev)
    views, off = [], 0
    for i, th in enumerate(texts_h):
        off += i % 16   # mixed alignments
        v = big[off:off + th.size]
        v.copy_(torch.from_numpy(th))
        views.append(v)
        off += th.size
    q2 = [(i, p) for i, p in enumerate(pats2)]
    # resident texts keep their symbol histograms (computed once, outside the timed region)
    t_h = time.perf_counter()
    hists = torch.stack([sm.histogram(v) for v in views]).cpu().numpy().view(np.uint64)
    hist_s = time.perf_counter() - t_h
    packed = sm.PackedTexts(big, [v.data_ptr() - big.data_ptr() for v in views], [v.numel() for v in views], hists)

    def sequential2():
        ps = sm.Patterns(pats2)
        out = torch.zeros(len(pats2), dtype=torch.int64, device=dev)
        for i in range(len(pats2)):
            ps.count_async(i, views[i], out[i:i + 1])
        torch.cuda.synchronize()
        ps.close()
        return out

    enq2 = []

    def batched2():
        t_e = time.perf_counter()
        out = sm.count_batch(packed, q2)
        enq2.append(time.perf_counter() - t_e)
        return out

    batched2()
    tb2, cb2 = min((_timed(batched2) for _ in range(reps)), key=lambda x: x[0])
    sequential2()
    ts2, cs2 = _timed(sequential2)
    assert torch.equal(cb2, cs2), "batched and sequential counts differ (many texts)"
    cb2 = cb2.cpu().numpy()
    pc2, pr2, pg2 = _plan_times(sm, packed, q2, len(pats2), max(reps, 10), torch.from_numpy(cb2).to(dev))
    del big, views, packed
    torch.cuda.empty_cache()
    return {"texts": len(pats2), "text_bytes": total, "sequential_s": round(ts2, 5), "batched_s": round(tb2, 5),
            "batched_host_enqueue_s": round(min(enq2), 5), "plan_create_s": round(pc2, 4),
            "plan_run_s": round(pr2, 5), "plan_graph_replay_s": round(pg2, 5),
            "text_GBps_plan_replay": round(total / pg2 / 1e9, 1), "histograms_once_s": round(hist_s, 4),
            "searches_per_s": round(len(pats2) / tb2, 1), "speedup_vs_sequential": round(ts2 / tb2, 2),
            "text_GBps_batched": round(total / tb2 / 1e9, 1),
            "checked": "batched == sequential single searches, every count"}


def run_batched(args):
    """Both batched workloads as JSON lines of their own."""
    one = batched_one_text(args, args.nq, args.steps)
    many = batched_many_texts(args, args.ntexts, args.steps)
    common = {"n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "u8", "metric": "batched searches/s", "unit": "searches/s"}
    return [
        dict(common, value=one["searches_per_s"], ms_per_step=round(one["batched_s"] * 1e3, 3),
             data="synthetic (seeded Zipf text; half substring, half random patterns)",
             config=dict(one, workload=f"batched_one_text: {one['patterns']} patterns, m log-uniform [2,1024], "
                                       f"{one['text_bytes']}-byte Zipf(1.0) sigma=95 text")),
        dict(common, value=many["searches_per_s"], ms_per_step=round(many["batched_s"] * 1e3, 3),
             data="synthetic (seeded texts sigma 4/20/95, one substring pattern each)",
             config=dict(many, workload=f"batched_many_texts: {many['texts']} texts, {many['text_bytes']} bytes "
                                        "in all, lengths log-uniform [4 KiB, 4 MiB], m log-uniform [4,256]")),
    ]


# ---------------------------------------------------------------------- single
def run_single(args):
    """8 MiB ACGT text, one m=16 substring: plain synchronous search, asynchronous loop and graph
    replay, in left-to-right and frequency order.  Small enough to stay cache resident, so this is a
    latency figure, not an HBM figure."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    n = args.n if args.n != (1 << 30) else (8 << 20)
    t_host, p = synth.single_count_workload(n=n, m=16)
    dev = torch.device("cuda:0")
    t_dev = torch.from_numpy(t_host).to(dev)
    text = sm.Text(t_dev)
    # every timed form must agree with the position list (full oracle parity: tests/)
    want = int(sm.report(text, p).numel())
    lines = []
    reps = args.reps
    for order in ("ltr", "freq"):
        # plain form: one synchronous call per search
        for _ in range(10):
            assert sm.count(text, p, order=order) == want
        t0 = time.perf_counter()
        for _ in range(reps):
            c = sm.count(text, p, order=order)
        sync_us = (time.perf_counter() - t0) / reps * 1e6
        assert c == want
        # asynchronous loop over a prepared pattern
        ps = sm.Patterns([p], [sm.order(order, p, text.hist) if order == "freq" else None])
        out = torch.zeros(reps, dtype=torch.int64, device=dev)
        for i in range(min(reps, 10)):
            ps.count_async(0, t_dev, out[i:i + 1])
        out.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            ps.count_async(0, t_dev, out[i:i + 1])
        torch.cuda.synchronize()
        async_us = (time.perf_counter() - t0) / reps * 1e6
        assert bool((out == want).all())
        # graph replay: `per_graph` searches captured once, replayed; every replay checked
        per_graph = 100
        gout = torch.zeros(per_graph, dtype=torch.int64, device=dev)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for i in range(per_graph):
                ps.count_async(0, t_dev, gout[i:i + 1])     # warm-up outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            gout.zero_()
            for i in range(per_graph):
                ps.count_async(0, t_dev, gout[i:i + 1])
        nrep = max(1, reps // per_graph)
        for k in range(3):          # replays with eager work in between
            g.replay()
            torch.cuda.synchronize()
            assert bool((gout == want).all()), "graph replay differs from eager"
            assert sm.count(text, p, order=order) == want
        t0 = time.perf_counter()
        for _ in range(nrep):
            g.replay()
        torch.cuda.synchronize()
        graph_us = (time.perf_counter() - t0) / (nrep * per_graph) * 1e6
        assert bool((gout == want).all())
        ps.close()
        lines.append({
            "metric": "single-search latency", "value": round(graph_us, 2), "unit": "us/search (graph replay)",
            "n_gpus": 1, "steps": reps, "warmup": 10, "ms_per_step": round(graph_us / 1e3, 5),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic (seeded uniform ACGT text, substring pattern)",
            "config": {"workload": f"single: {n}-byte uniform ACGT text, m=16 substring, order={order}",
                       "count": want, "sync_call_us": round(sync_us, 2), "async_loop_us": round(async_us, 2),
                       "graph_replay_us": round(graph_us, 2),
                       "text_GBps_graph": round(n / (graph_us * 1e-6) / 1e9, 1)},
        })
    return lines


# ----------------------------------------------------------------------- small
def run_small(args):
    """Small alphabets (sigma 2 and 4, 1 GiB) with m in {8, 64, 512, 4096}, and periodic a^n texts."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    dev = torch.device("cuda:0")
    lines = []
    n = args.n
    for sigma in (2, 4):
        t_host, pats = synth.small_alphabet_workload(n=n, sigma=sigma)
        t_dev = torch.from_numpy(t_host).to(dev)
        text = sm.Text(t_dev)
        if args.copy_probe and sigma == 2:
            # plain copy of known size (n bytes read, n written) for scaling the HBM counters
            dst = torch.empty_like(t_dev)
            dst.copy_(t_dev)
            torch.cuda.synchronize()
            del dst
        res = {}
        per_peel = []
        # peel 2 and 5 (the paper's values for large and DNA alphabets) as given, then the launch
        # parameters the autotuner's table gives a resident text with a histogram (the default)
        for peel in (2, 5, "tuned"):
            ps = sm.Patterns(pats, "freq", text.hist)
            out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
            tgt, kw = (text, {}) if peel == "tuned" else (t_dev, {"peel": peel})
            for i in range(len(pats)):
                ps.count_async(i, tgt, out[i:i + 1], **kw)
            out.zero_()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in pats]
            for i in range(len(pats)):
                ev[i][0].record()
                ps.count_async(i, tgt, out[i:i + 1], **kw)
                ev[i][1].record()
            torch.cuda.synchronize()
            counts = out.cpu().numpy()
            per_peel.append(counts)
            per_m = {}
            for i, p in enumerate(pats):
                per_m.setdefault(len(p), []).append(ev[i][0].elapsed_time(ev[i][1]))
            key = "tuned_GBps_by_m" if peel == "tuned" else f"peel{peel}_GBps_by_m"
            res[key] = {m: round(n / (np.mean(v) * 1e-3) / 1e9, 1) for m, v in per_m.items()}
            ps.close()
        for c in per_peel[1:]:
            assert np.array_equal(per_peel[0], c), "launch parameters changed a count"  # oracle parity: tests/
        res["counts_first_per_m"] = {len(p): int(counts[i]) for i, p in enumerate(pats) if i % 11 == 0}
        lines.append({
            "metric": "text GB/s per search (% HBM peak)", "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "value": round(float(np.mean([v for v in res["tuned_GBps_by_m"].values()])), 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic (seeded uniform text; 10 substrings + 1 random pattern per m)",
            "ms_per_step": None,
            "config": dict({"workload": f"small_alphabet: {n}-byte uniform sigma={sigma} text, "
                                        "m in {8,64,512,4096}, frequency order"}, **res),
        })
        del t_dev, text
        torch.cuda.empty_cache()
    # periodic a^n with a^(k-1)b and a^k
    np_ = min(n, 256 << 20)
    t_dev = torch.full((np_,), ord("a"), dtype=torch.uint8, device=dev)
    text = sm.Text(t_dev)
    per = {}
    for k in (16, 256):
        for name, p, want in ((f"a^{k}", b"a" * k, np_ - k + 1), (f"a^{k - 1}b", b"a" * (k - 1) + b"b", 0)):
            for order in ("ltr", "freq"):
                ps = sm.Patterns([p], "freq" if order == "freq" else "ltr", text.hist)
                out = torch.zeros(1, dtype=torch.int64, device=dev)
                ps.count_async(0, t_dev, out)
                out.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ps.count_async(0, t_dev, out)
                e1.record()
                torch.cuda.synchronize()
                assert int(out.item()) == want, (name, order)
                per[f"{name}/{order}"] = {"us": round(e0.elapsed_time(e1) * 1e3, 1),
                                          "GBps": round(np_ / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)}
                ps.close()
    lines.append({
        "metric": "text GB/s per search (% HBM peak)", "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "value": per["a^256/freq"]["GBps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (a^n)", "ms_per_step": None,
        "config": {"workload": f"periodic: a^n, n={np_}, patterns a^k and a^(k-1)b, k in {{16,256}}; "
                               "counts equal the closed forms n-k+1 and 0", "results": per},
    })
    return lines


# ---------------------------------------------------------------------- bigram
def run_bigram(args):
    """Compare orders on a correlated text: an order-1 Markov text over 26 letters and space (1 GiB),
    20 substring patterns for each m in {4, 8, 16, 32, 64}; count-kernel time per order."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    dev = torch.device("cuda:0")
    n = args.n
    t0 = time.time()
    t_host = synth.markov_text(n, family=8, stream=0)
    log(f"[bench] markov text {n} B in {time.time() - t0:.1f}s")
    t_dev = torch.from_numpy(t_host).to(dev)
    text = sm.Text(t_dev)
    bg_dev = sm.bigram(t_dev, text.hist)                       # pair counts (first call also warms up)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        sm.bigram(t_dev, text.hist)
    e1.record()
    torch.cuda.synchronize()
    bigram_us = e0.elapsed_time(e1) * 1e3 / 3
    text._bigram = bg_dev.cpu().numpy().view(np.uint64).copy()
    g = synth.rng(8, 1)
    ms = (4, 8, 16, 32, 64)
    pats = [synth.substring_pattern(t_host, m, g)[0] for m in ms for _ in range(20)]
    res = {}
    counts_by_order = {}
    for kind in ("ltr", "h", "freq", "bigram"):
        if kind == "ltr":
            orders = None
        elif kind == "bigram":
            orders = [sm.order("bigram", p, text.hist, text.bigram) for p in pats]
        else:
            orders = [sm.order(kind, p, text.hist) for p in pats]
        ps = sm.Patterns(pats, orders)
        out = torch.zeros(len(pats), dtype=torch.int64, device=dev)
        for i in range(len(pats)):
            ps.count_async(i, t_dev, out[i:i + 1], peel=2)
        out.zero_()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in pats]
        for i in range(len(pats)):
            ev[i][0].record()
            ps.count_async(i, t_dev, out[i:i + 1], peel=2)
            ev[i][1].record()
        torch.cuda.synchronize()
        counts_by_order[kind] = out.cpu().numpy()
        per_m = {}
        for i, p in enumerate(pats):
            per_m.setdefault(len(p), []).append(ev[i][0].elapsed_time(ev[i][1]))
        res[kind] = {m: round(n / (np.mean(v) * 1e-3) / 1e9, 1) for m, v in per_m.items()}
        ps.close()
    for kind in counts_by_order:
        assert np.array_equal(counts_by_order[kind], counts_by_order["ltr"]), kind
    mean = {k: round(float(np.mean(list(v.values()))), 1) for k, v in res.items()}
    return [{
        "metric": "text GB/s per search (% HBM peak)", "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "value": mean["bigram"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded order-1 Markov text over 26 letters and space; substring patterns)",
        "ms_per_step": None,
        "config": {"workload": f"bigram: {n}-byte order-1 Markov text, 20 substrings for each m in {{4..64}}, "
                               "peel 2, count kernel time per compare order",
                   "GBps_by_order_and_m": res, "mean_GBps_by_order": mean,
                   "bigram_table_us": round(bigram_us, 1)},
    }]


# ------------------------------------------------------------------ nonoverlap
def run_nonoverlap(args):
    """Disjoint-occurrence counts (greedy leftmost) beside the all-starts counts: the 1 GiB Zipf text
    with short substrings (many overlapping occurrences), and a^n (every start an occurrence)."""
    import torch

    import paper_1612_01506_amd as sm
    import synth

    dev = torch.device("cuda:0")
    n = args.n
    t_host = synth.zipf_text(n, 95, 1.0, family=2, stream=0)
    t_bytes = t_host.tobytes()
    t_dev = torch.from_numpy(t_host).to(dev)
    text = sm.Text(t_dev)
    g = synth.rng(6, 1)
    res = {}

    def wall(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        return (time.perf_counter() - t0) / reps, r

    for m in (2, 4, 8, 64):
        p = synth.substring_pattern(t_host, m, g)[0]
        t_all, c_all = wall(lambda: sm.count(text, p, order="freq"))
        t_no, c_no = wall(lambda: sm.count(text, p, order="freq", overlap=False))
        assert c_no == t_bytes.count(p), ("bytes.count", m)   # Python's count is disjoint, leftmost first
        assert c_all == int(sm.report(text, p).numel()), ("report length", m)
        res[f"zipf m={m}"] = {"occurrences": c_all, "disjoint": c_no, "all_ms": round(t_all * 1e3, 3),
                              "disjoint_ms": round(t_no * 1e3, 3),
                              "disjoint_GBps": round(n / t_no / 1e9, 1)}
    del t_dev, text
    torch.cuda.empty_cache()
    na = min(n, 256 << 20)
    a_dev = torch.full((na,), ord("a"), dtype=torch.uint8, device=dev)
    for k in (16, 256):
        t_no, c_no = wall(lambda: sm.count(a_dev, b"a" * k, overlap=False), reps=1)
        assert c_no == na // k, ("closed form", k)
        res[f"a^n a^{k}"] = {"occurrences": na - k + 1, "disjoint": c_no, "disjoint_ms": round(t_no * 1e3, 3)}
    del a_dev
    torch.cuda.empty_cache()
    head = res["zipf m=8"]
    return [{
        "metric": "text GB/s per search (% HBM peak)", "unit": "GB/s", "n_gpus": 1, "steps": 3, "warmup": 1,
        "value": head["disjoint_GBps"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic (seeded Zipf text, substring patterns; a^n)", "ms_per_step": head["disjoint_ms"],
        "config": {"workload": f"nonoverlap: disjoint-occurrence counts (synchronous calls, wall clock) on a "
                               f"{n}-byte Zipf(1.0) sigma=95 text and a^n (n={na}); value = the m=8 search",
                   "results": res},
    }]


# ----------------------------------------------------------------------- serve
def serve_points(args, rates, seconds: float, max_requests: int):
    """Open-loop Poisson requests against 8 resident 1 GiB texts at each offered load in `rates`;
    returns one summary per load point.  Results are checked outside the clock: reported positions
    are occurrences, and a sample of counts equals the same search alone."""
    import torch

    import paper_1612_01506_amd as sm
    import synth
    from paper_1612_01506_amd.serve import GpuExecutor, Server

    n = args.n
    mixes = [("uniform", 2), ("uniform", 4), ("zipf", 4), ("uniform", 20), ("zipf", 20), ("uniform", 95),
             ("zipf", 95), ("zipf", 95)]
    t0 = time.time()
    texts_h = []
    for i, (kind, sigma) in enumerate(mixes):
        if kind == "zipf":
            texts_h.append(synth.zipf_text(n, sigma, 1.0, family=5, stream=i))
        else:
            texts_h.append(synth.uniform_text(n, sigma, family=5, stream=i))
    log(f"[bench] serve: 8 texts of {n} B generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ex = GpuExecutor([torch.from_numpy(t).to(dev) for t in texts_h], nstreams=args.streams)
    alphabets = [bytes(np.unique(t[:1 << 20])) for t in texts_h]
    g = synth.rng(5, 100)
    budget_us = args.batch_budget_ms * 1e3 if args.batch_budget_ms > 0 else None

    def make_requests(count):
        tid = g.integers(0, len(texts_h), size=count)
        ms = synth.loguniform_ints(2, 512, count, g)
        rep = g.random(count) < 0.05
        out = []
        for k in range(count):
            t = texts_h[tid[k]]
            p = (synth.substring_pattern(t, int(ms[k]), g)[0] if k % 2 else
                 synth.random_pattern(alphabets[tid[k]], int(ms[k]), g))
            out.append((int(tid[k]), p, bool(rep[k])))
        return out

    # warm-up (kernel attributes, allocator, histograms)
    adaptive = not args.fixed_budget
    srv = Server(ex, hbm_budget=args.hbm_budget, on_done=lambda r: None, batch_budget_us=budget_us,
                 adaptive=adaptive)
    for t, p, r in make_requests(256):
        srv.submit(t, p, r)
    srv.drain()

    points = []
    last = None
    for rate in rates:
        nreq = int(min(max_requests, max(1000, rate * seconds)))
        reqs = make_requests(nreq)
        arrivals = np.cumsum(g.exponential(1.0 / rate, size=nreq))
        checks = []

        def consume(r):  # the client takes the result; the server frees the positions after this
            if r.report and len(checks) < 20 and 0 < r.count < (1 << 20):
                checks.append((r.text_id, r.pattern, r.positions[:64].cpu().numpy()))

        srv = Server(ex, hbm_budget=args.hbm_budget, on_done=consume, batch_budget_us=budget_us,
                     adaptive=adaptive)
        clock = srv.clock
        start = clock()
        k = 0
        handles = []
        while k < nreq or not srv.idle():
            now = clock() - start
            while k < nreq and arrivals[k] <= now:
                t, p, r = reqs[k]
                handles.append(srv.submit(t, p, r, t_submit=start + arrivals[k]))
                k += 1
            srv.step()
        elapsed = clock() - start
        st = srv.stats()
        done = st["completed"]
        pt = {"offered_req_per_s": rate, "achieved_req_per_s": round(done / elapsed, 1), "requests": nreq,
              "p50_ms": round(st.get("p50_ms", float("nan")), 3), "p99_ms": round(st.get("p99_ms", float("nan")), 3),
              "count_p50_ms": round(st.get("count_p50_ms", float("nan")), 3),
              "count_p99_ms": round(st.get("count_p99_ms", float("nan")), 3),
              "report_p50_ms": round(st.get("report_p50_ms", float("nan")), 3),
              "report_p99_ms": round(st.get("report_p99_ms", float("nan")), 3),
              "mean_batch": None if st.get("mean_batch") is None else round(st["mean_batch"], 1),
              "max_batch_model_us": None if st.get("max_batch_cost_us") is None else round(st["max_batch_cost_us"], 1),
              "batches": st["batches"], "rejected": st["rejected"],
              "peak_reserved_bytes": st["peak_reserved_bytes"], "seconds": round(elapsed, 2)}
        log(f"[bench] serve rate {rate}/s: {json.dumps(pt)}")
        points.append(pt)
        last = handles
        for tid, p, pos in checks:   # the positions reported in the mix are occurrences of p
            for q in pos:
                assert bytes(texts_h[tid][int(q):int(q) + len(p)]) == p
    # each result in the mix equals the same search alone
    for r in last[:: max(1, len(last) // 200)]:
        if r.status == "done":
            assert r.count == sm.count(ex.texts[r.text_id], r.pattern), ("mix != alone", r.rid)
    del ex
    torch.cuda.empty_cache()
    return points, {"texts": f"8 resident texts of {n} B (sigma 2/4/4/20/20/95/95/95, uniform or Zipf)",
                    "patterns": "m log-uniform [2,512], half substring, half random", "report_fraction": 0.05,
                    "hbm_budget_bytes": args.hbm_budget, "batch_budget_ms": args.batch_budget_ms,
                    "batch_budget": "fixed" if args.fixed_budget else "adaptive (the budget or the oldest wait)",
                    "streams": args.streams,
                    "checked": "reported positions are occurrences; sampled counts equal the search alone"}


def run_serve(args):
    """Open-loop Poisson requests against 8 resident texts, swept offered load: one line per load."""
    points, info = serve_points(args, args.rates, args.seconds, args.max_requests)
    lines = []
    for pt in points:
        lines.append({"metric": "served p50/p99 latency", "value": pt["p99_ms"], "unit": "ms (p99)", "n_gpus": 1,
                      "steps": 1, "warmup": 1, "ms_per_step": round(pt["seconds"] * 1e3, 1),
                      "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
                      "data": "synthetic (8 seeded texts; Poisson arrivals; half substring, half random patterns)",
                      "config": dict(pt, workload=f"serve: {info['texts']}, {info['patterns']}, 5% report",
                                     hbm_budget_bytes=info["hbm_budget_bytes"],
                                     batch_budget_ms=info["batch_budget_ms"], batch_budget=info["batch_budget"],
                                     streams=info["streams"])})
    return lines


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zipf", choices=["zipf", "batched", "serve", "single", "small", "nonoverlap", "bigram"])
    ap.add_argument("--reps", type=int, default=1000, help="single: searches timed per form")
    ap.add_argument("--rates", type=float, nargs="+", default=[200, 1000, 5000, 20000, 50000, 100000],
                    help="serve: offered loads in requests/s")
    ap.add_argument("--seconds", type=float, default=2.0, help="serve: seconds of arrivals per load point")
    ap.add_argument("--max-requests", type=int, default=20000, dest="max_requests")
    ap.add_argument("--streams", type=int, default=2, help="serve: device streams (in-flight batches)")
    ap.add_argument("--hbm-budget", type=int, default=1 << 30, dest="hbm_budget",
                    help="serve: bytes of HBM for report position buffers")
    ap.add_argument("--batch-budget-ms", type=float, default=10.0, dest="batch_budget_ms",
                    help="serve: modelled device time per batch (0: no bound)")
    ap.add_argument("--fixed-budget", action="store_true", dest="fixed_budget",
                    help="serve: no batch exceeds --batch-budget-ms (default: adaptive, up to the oldest wait)")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[1000, 5000, 12000], dest="serve_rates",
                    help="default workload: offered loads of the serve object")
    ap.add_argument("--serve-seconds", type=float, default=1.5, dest="serve_seconds",
                    help="default workload: seconds of arrivals per serve load point")
    ap.add_argument("--no-extras", action="store_true", dest="no_extras",
                    help="default workload: skip the batched and serve objects")
    ap.add_argument("--nq", type=int, default=10_000, help="batched: patterns on the one text")
    ap.add_argument("--ntexts", type=int, default=4096, help="batched: texts with one pattern each")
    ap.add_argument("--n", type=int, default=1 << 30, help="text bytes (default 1 GiB)")
    ap.add_argument("--per-m", type=int, default=100, dest="per_m")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, dest="cpu_seconds",
                    help="wall-time budget of the oracle CPU baseline (0 skips it)")
    ap.add_argument("--copy-probe", action="store_true", dest="copy_probe",
                    help="also run one plain device copy of the text (HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the search has no multi-GPU path (the design notes "
              "describe how it would shard: start positions split with an (m-1)-byte halo, counts "
              "summed by an all-reduce)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    res = {"zipf": run_zipf, "batched": run_batched, "serve": run_serve, "single": run_single,
           "small": run_small, "nonoverlap": run_nonoverlap, "bigram": run_bigram}[args.workload](args)
    for r in (res if isinstance(res, list) else [res]):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
