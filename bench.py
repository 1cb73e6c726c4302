"""Benchmark of exact fixed-radius neighbour search on one MI355X.

Default run (about two minutes):
  * headline: the 300,000-point tracking event (D=8, r=0.1, K=256,
    self-join); one step = build + count + fill of the whole event, inputs
    resident in HBM; value = neighbour pairs/s.
  * roofline of the dominant kernel, timed live with HIP events on the
    library's stream, against the MI355X VALU peak for its op mix;
  * the CPU oracle timed on a bounded sample of the same event;
  * paper-shaped: the 271,663-point 12-D self-join (r=0.12, K=1000, self
    pairs excluded) standing in for the paper's measured event;
  * density: 1,000,000 12-D references, 200,000 separate queries, K=64;
  * batched: 64 uneven tracking events in one batched call (one launch per
    pipeline step over all events; also replayed as HIP graphs) vs 64 plain
    per-event build+query calls (identical output checked);
  * serving: Poisson arrivals of log-normal-size events through the
    continuous-batching server vs a FIFO of plain per-event calls, with a
    load sweep, paired rounds and a tight memory budget.
A/B comparisons follow the paper's protocol (Sec. 4.2): warm-ups, paired
rounds in random order, medians with 95% bootstrap intervals, sign tests.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "neighbour pairs/s + events/s (batched vs per-event); p50/p99 event latency"
# Vector ALU rate for the op mix of the distance evaluation on MI355X: the
# published FP32 vector peak, 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 256 flops
# per CU per clock, counts each fused multiply-add as two flops; the
# distance's subtract, multiply and add are one operation each and may not
# be fused, so their peak is half of it, 128 per CU per clock (78.6 T op/s).
# The microkernel of frnn_measure_valu_rate measures the same chain on the
# device and is reported beside it.
VALU_PEAK_OPS = 256 * 128 * 2.4e9
HBM_PEAK_GBS = 8000.0


def counter_traffic():
    """HBM bytes per launch of the count kernel, from the committed counter
    summary (two rocprofv3 passes, FETCH_SIZE and WRITE_SIZE, each scaled by
    what the counter reads for a plain kernel of known size).  None when that
    summary was taken on a different kernel source than the one built here."""
    import hashlib
    src = os.path.join(ROOT, "paper_2609_31980_amd", "csrc", "frnn_kernels.hip")
    md = os.path.join(ROOT, "profiles", "hbm_traffic_tracks300k_d8.md")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        line = next(l for l in open(md) if l.startswith("count-kernel-counters:"))
    except (OSError, StopIteration):
        return None
    f = dict(kv.split("=", 1) for kv in line.split(":", 1)[1].split())
    if f.get("source_sha256") != sha:
        return None
    return (float(f["fetch_kib"]) * float(f["fetch_factor"])
            + float(f["write_kib"]) * float(f["write_factor"])) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


# ------------------------------------------------------ statistics (Sec. 4.2)
# The paper's protocol: warm-ups, paired rounds in randomised order with a
# synchronisation before and after each timed call, outputs verified first,
# medians with 95 % percentile-bootstrap intervals from 10,000 resamples, and
# an exact two-sided sign test on the paired differences.
def boot_ci(x, n_boot=10_000, seed=0):
    """Median and its 95 % percentile-bootstrap interval."""
    x = np.asarray(x, dtype=np.float64)
    rng = np.random.default_rng(seed)
    meds = np.median(x[rng.integers(0, len(x), size=(n_boot, len(x)))], axis=1)
    return {"median": float(np.median(x)), "ci95": [float(np.percentile(meds, 2.5)), float(np.percentile(meds, 97.5))],
            "n": int(len(x))}


def sign_test(a, b):
    """Exact two-sided sign test of paired samples a vs b (ties dropped)."""
    from math import comb
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    pos, neg = int(np.sum(d > 0)), int(np.sum(d < 0))
    n, k = pos + neg, min(pos, neg)
    p = min(1.0, 2.0 * sum(comb(n, i) for i in range(k + 1)) / 2.0 ** n) if n else 1.0
    return {"a_slower_rounds": pos, "b_slower_rounds": neg, "p_two_sided": p}


def paired_rounds(fns, rounds=30, seed=1):
    """Time each function once per round, in a seeded random order per round,
    with a device synchronisation before and after each call."""
    rng = np.random.default_rng(seed)
    times = {k: [] for k in fns}
    names = list(fns)
    for _ in range(rounds):
        for k in rng.permutation(names):
            sync()
            t0 = time.perf_counter()
            fns[k]()
            sync()
            times[k].append(time.perf_counter() - t0)
    return times


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


# ------------------------------------------------------------ single event
def time_steps(step, steps, warmup):
    for _ in range(warmup):
        nnz = step()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        nnz = step()
    sync()
    return time.perf_counter() - t0, nnz


def bench_single(frnn, x, r, K, steps, warmup):
    """One step = the whole path for one event (bin, count, fill), input
    resident in HBM.  Headline: the batched call on one event (its launch
    sequence, one synchronisation for the counts).  Beside it: the same
    launch sequence replayed as a HIP graph (the graphs option), and the
    same kernels through the build + query API (two synchronisations)."""
    og = frnn.default_opts(graphs=1)

    def step_batch():
        c = frnn.query_batch([x], r, K)[0]
        n = c.nnz
        c.release()
        return n

    def step_graph():
        c = frnn.query_batch([x], r, K, opts=og)[0]
        n = c.nnz
        c.release()
        return n

    def step_api():
        ix = frnn.build(x, r)
        c = ix.query(None, r, K)
        n = c.nnz
        c.release()
        ix.close()
        return n

    dt, nnz = time_steps(step_batch, steps, warmup)
    stats = frnn.last_stats()
    dt_graph, nnz_graph = time_steps(step_graph, steps, warmup)
    assert nnz_graph == nnz
    dt_api, nnz_api = time_steps(step_api, steps, warmup)
    assert nnz_api == nnz
    # a fourth pass with per-launch HIP events for the kernel durations of
    # the same work
    frnn.profile_enable(True)
    frnn.profile_read(reset=True)
    for _ in range(steps):
        step_batch()
    sync()
    prof = frnn.profile_read(reset=True)
    frnn.profile_enable(False)
    return dt, dt_graph, dt_api, nnz, stats, prof


# ------------------------------------------------------------ CPU baseline
def cpu_baseline(points, r, K, budget_s=12.0):
    import oracle
    o = oracle.get()
    n = len(points)
    rows = np.sort(np.random.default_rng(5).choice(n, size=min(n, 400), replace=False))
    t0 = time.perf_counter()
    c = o.frnn(points, r, K, Q=points[rows])
    t1 = time.perf_counter() - t0
    m = int(min(n, max(400, 400 * budget_s / max(t1, 1e-3))))
    rows = np.sort(np.random.default_rng(6).choice(n, size=m, replace=False))
    t0 = time.perf_counter()
    c = o.frnn(points, r, K, Q=points[rows])
    dt = time.perf_counter() - t0
    # one thread, on a sample that takes about a quarter of that time
    m1 = max(100, m // (4 * max(1, o.threads())))
    rows1 = np.sort(np.random.default_rng(7).choice(n, size=min(n, m1), replace=False))
    t0 = time.perf_counter()
    c1 = o.frnn(points, r, K, Q=points[rows1], nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": c.nnz / dt, "unit": "neighbour pairs/s", "cores": o.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{m} of {n} queries of the same event against all {n} references "
                      f"({c.nnz} pairs, {dt:.1f} s); full-event rate scales linearly in queries",
            "seconds": dt, "events_per_s_equiv": (m / n) / dt,
            "pair_evaluations_per_s": m * n / dt,
            "one_thread": {"value": c1.nnz / dt1, "unit": "neighbour pairs/s", "queries": int(len(rows1)),
                           "seconds": dt1, "pair_evaluations_per_s": len(rows1) * n / dt1}}


# ------------------------------------------------------------ batched
def bench_edges(frnn, x, r, K, steps=10):
    """Undirected edge export (frnn_csr_edges) from the headline event's CSR:
    upper-triangle and symmetrised lists, milliseconds per export."""
    ix = frnn.build(x, r)
    c = ix.query(None, r, K)
    out = {}
    for name, sym in (("upper", False), ("symmetrized", True)):
        e = c.edges(symmetrized=sym)
        n = e.n
        e.release()
        sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            e = c.edges(symmetrized=sym)
            e.release()
        sync()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"edges": n, "ms": dt * 1e3, "edges_per_s": n / dt}
    c.release()
    ix.close()
    return out


def bench_host(frnn, pts, r, K, steps=10, warmup=2):
    """The synchronous host-array call (frnn_query_host) on the headline
    event: host float32 in, compact host CSR out, so the host-to-device copy
    of the points and the device-to-host copy of the CSR are inside each call
    (the PCIe-inclusive rate; never the headline value)."""
    def step():
        c = frnn.query_host(pts, r, K)
        n = c.nnz
        c.release()
        return n
    dt, nnz = time_steps(step, steps, warmup)
    out_bytes = 8 * (len(pts) + 1) + 8 * nnz
    return {"ms_per_call": dt / steps * 1e3, "pairs_per_s": nnz * steps / dt,
            "bytes_in": int(pts.nbytes), "bytes_out": int(out_bytes)}


# settings for dense rows, timed beside the defaults (every setting gives the
# same output; the larger stashes cost 8 bytes per query and key)
DENSE_SETTINGS = {"stash128": dict(stash_cap=128), "stash256": dict(stash_cap=256),
                  "stash256_one_cell_window16": dict(stash_cap=256, cells_per_item=1, queries_per_item=16)}


def bench_paper_shaped(frnn, steps=20, warmup=5, tune=True):
    """The paper-shaped self-join (271,663 points, D=12, r=0.12, K=1000, self
    pairs excluded): the same batched step and build + query API as the headline.  The
    paper's own per-event times on its GPU are quoted as context only."""
    import torch
    from paper_2609_31980_amd import inputs
    w = inputs.paper_shaped()
    x = torch.from_numpy(w.points).cuda()

    def step_batch(opts=None):
        c = frnn.query_batch([x], w.r, w.K, exclude_self=True, opts=opts)[0]
        n = c.nnz
        c.release()
        return n

    def step_api():
        ix = frnn.build(x, w.r)
        c = ix.query(None, w.r, w.K, exclude_self=True)
        n = c.nnz
        c.release()
        ix.close()
        return n

    dt, nnz = time_steps(step_batch, steps, warmup)
    stats = frnn.last_stats()   # (the default options adapt to dense rows after the first run)
    dense = {}
    for name, kw in DENSE_SETTINGS.items():
        od = frnn.default_opts(**kw)
        dtd, nnzd = time_steps(lambda: step_batch(od), steps, warmup)
        assert nnzd == nnz
        dense[name] = {"options": kw, "ms_per_step": dtd / steps * 1e3}
    # the autotuner on this event (a self-query of its points; its parity
    # gate compares every candidate with the default setting's output)
    tuned = None
    if tune:
        otun, rep = frnn.tune(x, w.r, w.K)
        dtt, nnzt = time_steps(lambda: step_batch(otun), steps, warmup)
        assert nnzt == nnz
        tuned = {"ms_per_step": dtt / steps * 1e3, "options": otun.as_dict(),
                 "tuner_default_ms": rep["default_ms"], "tuner_best_ms": rep["best_ms"],
                 "tried": rep["candidates_tried"], "density_class": rep["density_class"]}
    dt_api, nnz_api = time_steps(step_api, steps, warmup)
    assert nnz_api == nnz
    # per-launch HIP events for the kernel durations
    frnn.profile_enable(True)
    frnn.profile_read(reset=True)
    for _ in range(5):
        step_batch()
    sync()
    prof = frnn.profile_read(reset=True)
    frnn.profile_enable(False)
    del x
    return {"workload": "paper-shaped-271663-d12: Zipf-sized Gaussian clusters in [-1,1]^12, "
                        "sigma 0.0305 (calibrated to the paper's mean non-self degree), r=0.12, "
                        "K=1000, self pairs excluded",
            "ms_per_step": dt / steps * 1e3, "pairs_per_step": nnz,
            "pairs_per_s": nnz * steps / dt, "events_per_s": steps / dt,
            "api_ms_per_step": dt_api / steps * 1e3,
            "default_run": {"stash_cap": stats["stash_cap"], "adapted": stats["adapted"]},
            "dense_settings": dense,
            "tuned": tuned,
            "candidates_per_pair": stats["candidates"] / max(nnz, 1),
            "kernels_us": {k: round(v[1] / max(v[0], 1) * 1e3, 1) for k, v in prof.items()},
            "paper_context": {"exact_device_p50_ms": 267.829, "rerun_device_p50_ms": 207.299,
                              "gpu": "RTX 2070 SUPER", "pairs": 9279672,
                              "note": "different hardware and the real event; context, not a target"}}


def bench_batched(frnn, rounds=30, tuned=None):
    import torch
    from paper_2609_31980_amd import inputs
    log("batched: generating 64 events")
    evs = inputs.c3_events()
    xs = [torch.from_numpy(e).cuda() for e in evs]
    npts = sum(len(e) for e in evs)
    r, K = 0.1, 256

    def per_event():
        outs = []
        for x in xs:
            ix = frnn.build(x, r)
            outs.append(ix.query(None, r, K))
            ix.close()
        return outs

    og = frnn.default_opts(graphs=1)

    def per_event_batch_call():
        return [frnn.query_batch([x], r, K)[0] for x in xs]

    def batched():
        return frnn.query_batch(xs, r, K)

    def batched_graphs():
        return frnn.query_batch(xs, r, K, opts=og)

    def batched_tuned():
        return frnn.query_batch(xs, r, K, opts=tuned)

    # parity: batched == per-event, event by event, before any timing
    a, b = per_event(), batched()
    for e in range(len(xs)):
        oa, ia, da = a[e].torch()
        ob, ib, db = b[e].torch()
        assert torch.equal(oa, ob) and torch.equal(ia, ib) and torch.equal(da.view(torch.int32), db.view(torch.int32)), \
            f"batched output differs from per-event on event {e}"
    nnz = sum(o.nnz for o in b)
    for o in a + b:
        o.release()
    del a, b
    sync()
    c = batched_graphs()
    for e in range(len(xs)):   # graph replay == default batched output, event by event
        ob, ib, db = c[e].torch()
        oa, ia, da = frnn.query_batch([xs[e]], r, K)[0].torch()
        assert torch.equal(oa, ob) and torch.equal(ia, ib) and torch.equal(da.view(torch.int32), db.view(torch.int32))
    for o in c:
        o.release()
    fns = {"per_event": per_event, "per_event_batch_call": per_event_batch_call, "batched": batched,
           "batched_graphs": batched_graphs}
    if tuned is not None:
        c = batched_tuned()
        for e in range(len(xs)):   # tuned == default batched output, event by event
            ob, ib, db = c[e].torch()
            oa, ia, da = frnn.query_batch([xs[e]], r, K)[0].torch()
            assert torch.equal(oa, ob) and torch.equal(ia, ib) and torch.equal(da.view(torch.int32), db.view(torch.int32))
        for o in c:
            o.release()
        fns["batched_tuned"] = batched_tuned

    def run(fn):
        return lambda: [o.release() for o in fn()]
    for _ in range(10):      # warm-up (graph capture, pools)
        for fn in fns.values():
            run(fn)()
    times = paired_rounds({k: run(f) for k, f in fns.items()}, rounds=rounds)
    E = len(xs)
    tp, tg, tb, tbg = (float(np.median(times[k]))
                       for k in ("per_event", "per_event_batch_call", "batched", "batched_graphs"))
    ms = {k: {kk: (v * 1e3 if kk == "median" else [u * 1e3 for u in v] if kk == "ci95" else v)
              for kk, v in boot_ci(times[k]).items()} for k in fns}
    res = {"events": E, "points": npts, "pairs": nnz,
           "per_event_ms": tp * 1e3, "per_event_batch_call_ms": tg * 1e3, "batched_ms": tb * 1e3,
           "batched_graphs_ms": tbg * 1e3,
           "per_event_events_per_s": E / tp, "per_event_batch_call_events_per_s": E / tg,
           "batched_events_per_s": E / tb, "batched_pairs_per_s": nnz / tb,
           "speedup_vs_per_event": tp / tb, "speedup_vs_per_event_batch_call": tg / tb,
           "ms_median_ci95": ms,
           "sign_test_per_event_vs_batched": sign_test(times["per_event"], times["batched"]),
           "sign_test_per_event_batch_call_vs_batched": sign_test(times["per_event_batch_call"], times["batched"]),
           "sign_test_batched_vs_graphs": sign_test(times["batched"], times["batched_graphs"]),
           **({"batched_tuned_ms": float(np.median(times["batched_tuned"])) * 1e3,
               "batched_tuned_events_per_s": E / float(np.median(times["batched_tuned"])),
               "tuned_options": tuned.as_dict(),
               "sign_test_batched_vs_tuned": sign_test(times["batched"], times["batched_tuned"])}
              if tuned is not None else {}),
           "protocol": f"10 warm-up rounds, then {rounds} rounds each timing every path once in a seeded "
                       "random order, synchronised before and after each call; medians with 95% percentile "
                       "bootstrap intervals (10,000 resamples); exact two-sided sign tests",
           "identical_output": "batched == per-event API on the device, every event; every event also equals "
                               "the CPU oracle's CSR in the GPU tests (stored digests)",
           "per_event": "64 x (build + query API calls)",
           "per_event_batch_call": "64 x single-event batched calls",
           "batched": "one launch sequence over all 64 events (kernels launched one by one)",
           "batched_graphs": "the same launch sequence replayed as HIP graphs (graphs option)"}
    del xs
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------ serving
def bench_serving(frnn, n_events=600, load=0.7, pool=96, sweep_events=300, rounds=30):
    """Open-loop Poisson arrivals of log-normal-size events through the
    continuous-batching server vs a FIFO of plain per-event calls on the same
    trace: at 0.7x the batched capacity (headline), a load sweep that also
    covers loads the plain path can sustain, paired rounds at 0.7x the plain
    capacity, and a run under a tight memory budget."""
    import torch
    from paper_2609_31980_amd import inputs
    log("serving: generating event pool")
    probe = inputs.c5_trace(pool, rate=1.0)
    evs = [inputs.c5_event(a) for a in probe]        # distinct events, reused cyclically
    mean_n = float(np.mean([len(e) for e in evs]))
    r, K = 0.1, 256
    # capacity of the plain path (events/s) on this pool
    xs = [torch.from_numpy(e).cuda() for e in evs[:16]]
    sync()
    t0 = time.perf_counter()
    for x in xs:
        ix = frnn.build(x, r)
        ix.query(None, r, K).release()
        ix.close()
    sync()
    plain_rate = len(xs) / (time.perf_counter() - t0)
    del xs

    def server(budget=64 << 30):
        return frnn.Server(8, r, K, hbm_budget_bytes=budget, max_batch_events=64, max_inflight=2)

    # batched capacity: the server with everything queued at once
    srv = server()
    t0 = time.perf_counter()
    tick = [srv.submit(evs[i % pool]) for i in range(128)]
    for t in tick:
        c, _ = srv.wait(t)
        c.release()
    cap = 128 / (time.perf_counter() - t0)
    log(f"serving: plain capacity {plain_rate:.0f}/s, batched capacity {cap:.0f}/s")

    def run_server(srv, trace):
        n = len(trace)
        lat, bid = [], set()
        done = [0.0]
        tickets = [None] * n
        start = time.perf_counter() + 0.02

        def submitter():
            for i, a in enumerate(trace):
                dl = start + a.t - time.perf_counter()
                if dl > 0:
                    time.sleep(dl)
                tickets[i] = srv.submit(evs[i % pool])

        th = threading.Thread(target=submitter)
        th.start()
        for i, a in enumerate(trace):
            while tickets[i] is None:
                time.sleep(0.0002)
            c, tm = srv.wait(tickets[i])
            c.release()
            lat.append(tm["done_s"] - (start + a.t))
            bid.add(tm["batch_id"])
            done[0] = tm["done_s"]
        th.join()
        return lat, n / (done[0] - start), len(bid)

    def run_plain(trace):
        n = len(trace)
        lat = []
        start = time.perf_counter() + 0.02
        last = start
        for i, a in enumerate(trace):
            dl = start + a.t - time.perf_counter()
            if dl > 0:
                time.sleep(dl)
            x = torch.from_numpy(evs[i % pool]).cuda()
            ix = frnn.build(x, r)
            ix.query(None, r, K).release()
            ix.close()
            sync()
            last = time.perf_counter()
            lat.append(last - (start + a.t))
        return lat, n / (last - start)

    def both(rate, n, seed=inputs.SEED_C5):
        trace = inputs.c5_trace(n, rate=rate, seed=seed)
        ls, rs, nb = run_server(srv, trace)
        lp, rp = run_plain(trace)
        return {"offered_events_per_s": rate, "events": n, "batches": nb,
                "served_events_per_s": rs, "served_p50_ms": pct(ls, 50) * 1e3, "served_p99_ms": pct(ls, 99) * 1e3,
                "plain_fifo_events_per_s": rp, "plain_p50_ms": pct(lp, 50) * 1e3, "plain_p99_ms": pct(lp, 99) * 1e3}

    head = both(load * cap, n_events)
    log("serving: load sweep")
    sweep = {}
    for f in (0.3, 0.5, 0.7, 0.9):
        sweep[f"{f}x_batched_capacity"] = both(f * cap, sweep_events, seed=inputs.SEED_C5 + 10)
    sweep["0.7x_plain_capacity"] = both(0.7 * plain_rate, sweep_events, seed=inputs.SEED_C5 + 11)
    # paired rounds at a load both paths sustain: per-round median latency
    log("serving: paired rounds")
    rng = np.random.default_rng(2)
    p50s = {"served": [], "plain": []}
    for i in range(rounds):
        trace = inputs.c5_trace(60, rate=0.7 * plain_rate, seed=inputs.SEED_C5 + 100 + i)
        for which in rng.permutation(["served", "plain"]):
            lat = run_server(srv, trace)[0] if which == "served" else run_plain(trace)[0]
            p50s[which].append(pct(lat, 50) * 1e3)
    srv.close()
    paired = {"load": "0.7x the plain capacity, 60-event traces, a fresh trace per round",
              "served_p50_ms": boot_ci(p50s["served"]), "plain_p50_ms": boot_ci(p50s["plain"]),
              "sign_test_plain_vs_served": sign_test(p50s["plain"], p50s["served"])}
    # a budget that holds only a few events' work at once: admission waits
    log("serving: tight budget")
    tight = 512 << 20
    srv = server(tight)
    trace = inputs.c5_trace(sweep_events, rate=0.9 * cap, seed=inputs.SEED_C5 + 12)
    lt, rt, nbt = run_server(srv, trace)
    held, peak = srv.memory()
    srv.close()
    tight_res = {"hbm_budget_bytes": tight, "offered_events_per_s": 0.9 * cap, "events": sweep_events,
                 "batches": nbt, "served_events_per_s": rt, "served_p50_ms": pct(lt, 50) * 1e3,
                 "served_p99_ms": pct(lt, 99) * 1e3, "server_peak_bytes": peak}
    return {"events": n_events, "mean_points": mean_n, "load_fraction_of_batched_capacity": load,
            **head,
            "plain_capacity_events_per_s": plain_rate, "batched_capacity_events_per_s": cap,
            "load_sweep": sweep, "paired_rounds": paired, "tight_budget": tight_res,
            "latency": "completion on the device minus scheduled arrival; H2D of the event included"}


def hbm_kernels(kern, N, D, nnz, cells, cells_cleared):
    """Algorithmic HBM bytes per launch of the memory-bound kernels of one
    event (read + written once each), their rate and fraction of the 8 TB/s
    peak at the measured per-launch times."""
    Dp = (D + 3) & ~3
    alg = {"extent": 4 * D * N + 4 * cells_cleared,            # read X, clear the cell table
           "keys": (4 * D + 8 + 4) * N,                          # read X, write key and rank, one counter update
           "scatter": (4 * D + 12) * N + (4 * Dp + 8) * N,       # read X, key, rank, cell start; write row, perm, key
           "short_rows": 16 * nnz + 16 * N,                      # stash keys in, (index, dist2) out, offsets
           "scan_cells": 8 * cells,                              # counts in, starts out
           "scan_rows": 20 * N}                                  # degree in, two offsets out
    out = {}
    for k, b in alg.items():
        if k in kern and kern[k]["avg_ms"] > 0:
            gbs = b / (kern[k]["avg_ms"] * 1e-3) / 1e9
            out[k] = {"algorithmic_bytes": int(b), "avg_us": kern[k]["avg_ms"] * 1e3, "GB_per_s": gbs,
                      "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    return out


def bench_tuning(frnn):
    """The autotuner (frnn_tune) on one event of each tracking-shaped
    workload: the 300,000-point event, the median-size event of the batch of
    64, and a median-size served event; chosen options, the default's and the
    best time (batched single-event path, best of three), the density class."""
    import torch
    from paper_2609_31980_amd import inputs
    evs = {"tracks-300k-d8": inputs.c2().points,
           "batch64-median-event": None, "serving-median-event": None}
    sizes = inputs.c3_sizes()
    k = int(np.argsort(sizes)[len(sizes) // 2])
    # event k of the batch, generated alone (its own spawned seed, as c3_events does)
    evs["batch64-median-event"] = inputs.tracks(
        int(sizes[k]), 8, seed=np.random.SeedSequence(inputs.SEED_C3).spawn(1 + len(sizes))[1 + k])
    tr = inputs.c5_trace(96, rate=1.0)
    med = sorted(tr, key=lambda a: a.n)[48]
    evs["serving-median-event"] = inputs.c5_event(med)
    out = {}
    for name, pts in evs.items():
        x = torch.from_numpy(pts).cuda()
        best, rep = frnn.tune(x, 0.1, 256)
        out[name] = {"N": int(len(pts)), "chosen": best.as_dict(), "default_ms": rep["default_ms"],
                     "best_ms": rep["best_ms"], "gain": rep["default_ms"] / max(rep["best_ms"], 1e-9),
                     "tried": rep["candidates_tried"], "rejected": rep["candidates_rejected"],
                     "density_class": rep["density_class"], "from_cache": bool(rep["from_cache"])}
        del x
    return out


def bench_density(frnn, steps=10, warmup=3, tune=True):
    """The density workload: 1,000,000 12-D references in Zipf-sized
    clusters, 200,000 separate queries, r=0.15 (mean degree about 100), K=64;
    one step = bin the references and the queries, count, fill."""
    import torch
    from paper_2609_31980_amd import inputs
    log("density: generating 1M x 200k")
    w = inputs.c4()
    x = torch.from_numpy(w.points).cuda()
    q = torch.from_numpy(w.queries).cuda()

    def step(opts=None):
        c = frnn.query_batch([x], w.r, w.K, queries=[q], opts=opts)[0]
        n = c.nnz
        c.release()
        return n
    dt, nnz = time_steps(step, steps, warmup)
    stats = frnn.last_stats()   # (the default options adapt to dense rows after the first run)
    dense = {}
    for name, kw in DENSE_SETTINGS.items():
        od = frnn.default_opts(**kw)
        dtd, nnzd = time_steps(lambda: step(od), steps, warmup)
        assert nnzd == nnz
        dense[name] = {"options": kw, "ms_per_step": dtd / steps * 1e3}
    # the autotuner on the references (it times self-queries; the queries
    # are drawn from the same clusters), applied to the query step
    tuned = None
    if tune:
        log("density: tuning on the references")
        otun, rep = frnn.tune(x, w.r, w.K)
        dtt, nnzt = time_steps(lambda: step(otun), steps, warmup)
        assert nnzt == nnz
        tuned = {"ms_per_step": dtt / steps * 1e3, "options": otun.as_dict(),
                 "tuned_on": "self-query of the 1,000,000 references",
                 "tuner_default_ms": rep["default_ms"], "tuner_best_ms": rep["best_ms"],
                 "tried": rep["candidates_tried"], "density_class": rep["density_class"]}
    frnn.profile_enable(True)
    frnn.profile_read(reset=True)
    for _ in range(3):
        step()
    sync()
    prof = frnn.profile_read(reset=True)
    frnn.profile_enable(False)
    kus = {k: round(v[1] / max(v[0], 1) * 1e3, 1) for k, v in prof.items()}
    cand = stats["candidates"]
    ops = cand * 3 * w.points.shape[1]
    cnt_s = kus.get("count", 0.0) * 1e-6
    del x, q
    return {"workload": "zipf-clusters-1m-200k-d12: 1,000,000 references in Zipf(1.5)-sized Gaussian clusters "
                        "(sigma 0.03) in [-1,1]^12, 200,000 queries drawn from the clusters, r=0.15, K=64",
            "ms_per_step": dt / steps * 1e3, "pairs_per_step": nnz, "pairs_per_s": nnz * steps / dt,
            "queries_per_s": 200_000 * steps / dt, "candidates_per_pair": cand / max(nnz, 1),
            "kernels_us": kus,
            "default_run": {"stash_cap": stats["stash_cap"], "adapted": stats["adapted"]},
            "dense_settings": dense,
            "tuned": tuned,
            "count_roofline": {"achieved": ops / cnt_s / 1e12 if cnt_s else None, "peak": VALU_PEAK_OPS / 1e12,
                               "unit": "TFLOP/s", "frac": (ops / cnt_s) / VALU_PEAK_OPS if cnt_s else None,
                               "ops_per_launch": ops, "candidates": cand}}


# ------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-density", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--paper-only", action="store_true",
                    help="run only the paper-shaped self-join and print its JSON (a profiling aid)")
    ap.add_argument("--only", choices=["density", "batched", "serving"], default=None,
                    help="run only this section and print its JSON (a profiling aid)")
    ap.add_argument("--serve-events", type=int, default=600)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also write and then read this many MiB with plain kernels (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the benchmark measures one GPU only; multi-GPU runs are not supported "
              "(events would shard across GPUs, one process each, with no collectives)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_31980_amd import frnn, inputs

    if args.paper_only:
        print(json.dumps({"paper_shaped": bench_paper_shaped(frnn, args.steps, args.warmup, not args.no_tune)}),
              flush=True)
        return
    if args.only:
        fn = {"density": lambda: bench_density(frnn, args.steps, args.warmup, not args.no_tune),
              "batched": lambda: bench_batched(frnn, rounds=args.steps),
              "serving": lambda: bench_serving(frnn, args.serve_events, sweep_events=100, rounds=3)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    if args.calib_copy_mib:
        # a plain write kernel and a plain read kernel of known size, to
        # scale the HBM byte counters (FETCH_SIZE, WRITE_SIZE)
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        sync()
        s = a.sum()
        sync()
        del a, s
    w = inputs.c2()
    x = torch.from_numpy(w.points).cuda()
    D = w.points.shape[1]
    log("single event: timing")
    dt, dt_graph, dt_api, nnz, stats, prof = bench_single(frnn, x, w.r, w.K, args.steps, args.warmup)
    ms = dt / args.steps * 1e3
    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1), "total_ms": v[1]} for k, v in prof.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    cand = stats["candidates"]
    ops = cand * 3 * D            # D subtracts, D multiplies, D adds per candidate pair
    avg_s = kern[dom]["avg_ms"] * 1e-3
    achieved = ops / avg_s / 1e12
    log("valu rate microkernel")
    measured = frnn.measure_valu_rate() / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / (VALU_PEAK_OPS / 1e12), "traffic": counter_traffic() if dom == "count" else None,
            "kernel": dom, "kernel_avg_ms": kern[dom]["avg_ms"],
            "algorithmic_ops_per_launch": ops, "candidates_per_launch": cand,
            "candidates_per_pair": cand / max(nnz, 1),
            "peak_measured": measured, "frac_of_measured": achieved / measured,
            "peak_published_fp32": 157.3, "frac_of_published_fp32": achieved / 157.3,
            "peak_note": "peak: the published 157.3 TFLOP/s FP32 vector peak halved (it counts a fused "
                         "multiply-add as two flops; the distance's subtract, multiply and add are one op each "
                         "and are never fused): 256 CUs x 128 ops x 2.4 GHz; peak_measured: that operation "
                         "chain timed on this GPU (frnn_measure_valu_rate)"}
    # per-step distribution (Sec. 4.2 protocol: 30 synchronised timed steps)
    def one():
        c = frnn.query_batch([x], w.r, w.K)[0]
        c.release()
    st30 = paired_rounds({"step": one}, rounds=30)["step"]
    step_stats = {k: ([u * 1e3 for u in v] if k == "ci95" else v * 1e3 if k == "median" else v)
                  for k, v in boot_ci(st30).items()}
    step_stats["unit"] = "ms"
    # the event's grid cells and the cell table the batched path clears (its
    # capacity class: 2 cells per point of 2^k x {1, 1.25, 1.5, 1.75} points)
    ix = frnn.build(x, w.r)
    cells = int(ix.info()["cells"])
    ix.close()
    pts_cap = 4096
    while pts_cap * 2 <= w.points.shape[0]:
        pts_cap *= 2
    pts_cap = next(pts_cap + pts_cap * q // 4 for q in range(5) if pts_cap + pts_cap * q // 4 >= w.points.shape[0])
    out = {"metric": METRIC, "value": nnz * args.steps / dt, "unit": "neighbour pairs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "tracks-300k-d8: one tracking-shaped event, N=300000, D=8, "
                                  "25000 tracks x 12 (sigma 0.02) + 10% uniform noise, r=0.1, "
                                  "K=256, queries = references", "N": 300000, "D": 8, "r": 0.1, "K": 256,
                      "parallelism": "1 GPU"},
           "events_per_s": args.steps / dt, "pairs_per_step": nnz,
           "graphs_option": {"ms_per_step": dt_graph / args.steps * 1e3,
                             "pairs_per_s": nnz * args.steps / dt_graph,
                             "note": "the same step with its launch sequence replayed as a HIP graph"},
           "api_build_query": {"ms_per_step": dt_api / args.steps * 1e3,
                               "pairs_per_s": nnz * args.steps / dt_api,
                               "events_per_s": args.steps / dt_api},
           "step_ms_median_ci95": step_stats,
           "roofline": roof, "kernels": kern,
           "hbm_kernels": hbm_kernels(kern, w.points.shape[0], D, nnz, cells, 2 * pts_cap + 2),
           "edge_export": bench_edges(frnn, x, w.r, w.K),
           "host_interface": bench_host(frnn, w.points, w.r, w.K)}
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w.points, w.r, w.K)
    del x
    torch.cuda.empty_cache()
    if not args.no_paper:
        log("paper-shaped")
        out["paper_shaped"] = bench_paper_shaped(frnn, tune=not args.no_tune)
        torch.cuda.empty_cache()
    if not args.no_density:
        log("density")
        out["density"] = bench_density(frnn, tune=not args.no_tune)
        torch.cuda.empty_cache()
    tuned = None
    if not args.no_tune:
        log("tuning")
        out["tuning"] = bench_tuning(frnn)
        tuned = frnn.default_opts(**out["tuning"]["batch64-median-event"]["chosen"])
        torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched")
        out["batched"] = bench_batched(frnn, tuned=tuned)
    if not args.no_serving:
        log("serving")
        out["serving"] = bench_serving(frnn, args.serve_events)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
