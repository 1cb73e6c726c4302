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
  * batched: 64 uneven tracking events, one graph-replayed batch (one
    launch per pipeline step over all events) vs 64 plain per-event
    build+query calls (identical output checked);
  * serving: Poisson arrivals of log-normal-size events through the
    continuous-batching server vs a FIFO of plain per-event calls.

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
# Dense VALU rate for the op mix of the distance evaluation on MI355X:
# 256 CUs x 64 FP32 lanes x 2.4 GHz, one subtract, multiply or add per lane
# per clock (no FMA: the canonical sum forbids contraction; packed FP32 is
# not used).
VALU_PEAK_OPS = 256 * 64 * 2.4e9
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
    resident in HBM.  Headline: the single-event launch sequence replayed as
    a HIP graph (one synchronisation).  Beside it: the same kernels through
    the build + query API (two synchronisations, eager launches)."""
    def step_graph():
        c = frnn.query_batch([x], r, K)[0]
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

    dt, nnz = time_steps(step_graph, steps, warmup)
    stats = frnn.last_stats()
    dt_api, nnz_api = time_steps(step_api, steps, warmup)
    assert nnz_api == nnz
    # a third pass with per-launch HIP events (eager launches) for the
    # kernel durations of the same work
    frnn.profile_enable(True)
    frnn.profile_read(reset=True)
    for _ in range(steps):
        step_graph()
    sync()
    prof = frnn.profile_read(reset=True)
    frnn.profile_enable(False)
    return dt, dt_api, nnz, stats, prof


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
    return {"value": c.nnz / dt, "unit": "neighbour pairs/s", "cores": o.threads(),
            "kind": "oracle",
            "sample": f"{m} of {n} queries of the same event against all {n} references "
                      f"({c.nnz} pairs, {dt:.1f} s); full-event rate scales linearly in queries",
            "seconds": dt, "events_per_s_equiv": (m / n) / dt}


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


def bench_paper_shaped(frnn, steps=20, warmup=5):
    """The paper-shaped self-join (271,663 points, D=12, r=0.12, K=1000, self
    pairs excluded): the same graph step and eager API as the headline.  The
    paper's own per-event times on its GPU are quoted as context only."""
    import torch
    from paper_2609_31980_amd import inputs
    w = inputs.paper_shaped()
    x = torch.from_numpy(w.points).cuda()

    def step_graph():
        c = frnn.query_batch([x], w.r, w.K, exclude_self=True)[0]
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

    dt, nnz = time_steps(step_graph, steps, warmup)
    stats = frnn.last_stats()
    dt_api, nnz_api = time_steps(step_api, steps, warmup)
    assert nnz_api == nnz
    # per-launch HIP events (eager launches) for the kernel durations
    frnn.profile_enable(True)
    frnn.profile_read(reset=True)
    for _ in range(5):
        step_graph()
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
            "candidates_per_pair": stats["candidates"] / max(nnz, 1),
            "kernels_us": {k: round(v[1] / max(v[0], 1) * 1e3, 1) for k, v in prof.items()},
            "paper_context": {"exact_device_p50_ms": 267.829, "rerun_device_p50_ms": 207.299,
                              "gpu": "RTX 2070 SUPER", "pairs": 9279672,
                              "note": "different hardware and the real event; context, not a target"}}


def bench_batched(frnn, rounds=3):
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

    def per_event_graph():
        return [frnn.query_batch([x], r, K)[0] for x in xs]

    def batched():
        return frnn.query_batch(xs, r, K)

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
    times = {per_event: [], per_event_graph: [], batched: []}
    fns = [per_event, per_event_graph, batched]
    for fn in fns:          # warm-up (graph capture, pools)
        [o.release() for o in fn()]
    for i in range(rounds):
        order = fns if i % 2 == 0 else fns[::-1]
        for fn in order:
            sync()
            t0 = time.perf_counter()
            outs = fn()
            sync()
            times[fn].append(time.perf_counter() - t0)
            for o in outs:
                o.release()
    E = len(xs)
    tp, tg, tb = (float(np.median(times[f])) for f in fns)
    res = {"events": E, "points": npts, "pairs": nnz,
           "per_event_ms": tp * 1e3, "per_event_graph_ms": tg * 1e3, "batched_ms": tb * 1e3,
           "per_event_events_per_s": E / tp, "per_event_graph_events_per_s": E / tg,
           "batched_events_per_s": E / tb, "batched_pairs_per_s": nnz / tb,
           "speedup_vs_per_event": tp / tb, "speedup_vs_per_event_graph": tg / tb,
           "identical_output": True,
           "per_event": "64 x (build + query API calls)",
           "per_event_graph": "64 x single-event graph-replayed calls",
           "batched": "one graph-replayed launch sequence over all 64 events"}
    del xs
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------ serving
def bench_serving(frnn, n_events=600, load=0.7, pool=96):
    import torch
    from paper_2609_31980_amd import inputs
    log("serving: generating event pool")
    probe = inputs.c5_trace(pool, rate=1.0)
    evs = [inputs.c5_event(a) for a in probe]        # distinct events, reused cyclically
    mean_n = float(np.mean([len(e) for e in evs]))
    r, K = 0.1, 256
    # capacity of the plain path (events/s) on this pool, to set the load
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
    # batched capacity: the server with everything queued at once
    srv = frnn.Server(8, r, K, hbm_budget_bytes=64 << 30, max_batch_events=64, max_inflight=2)
    t0 = time.perf_counter()
    tick = [srv.submit(evs[i % pool]) for i in range(128)]
    for t in tick:
        c, _ = srv.wait(t)
        c.release()
    cap = 128 / (time.perf_counter() - t0)
    rate = load * cap
    trace = inputs.c5_trace(n_events, rate=rate)
    log(f"serving: plain capacity {plain_rate:.0f}/s, batched capacity {cap:.0f}/s, offered {rate:.0f}/s")

    def run_server():
        lat = []
        done = [0.0]
        tickets = [None] * n_events
        start = time.perf_counter() + 0.05

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
            done[0] = tm["done_s"]
        th.join()
        return lat, n_events / (done[0] - start)

    def run_plain():
        lat = []
        start = time.perf_counter() + 0.05
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
        return lat, n_events / (last - start)

    ls, rs = run_server()
    srv.close()
    lp, rp = run_plain()
    return {"events": n_events, "mean_points": mean_n, "offered_events_per_s": rate,
            "load_fraction_of_batched_capacity": load,
            "served_events_per_s": rs, "served_p50_ms": pct(ls, 50) * 1e3, "served_p99_ms": pct(ls, 99) * 1e3,
            "plain_fifo_events_per_s": rp, "plain_p50_ms": pct(lp, 50) * 1e3, "plain_p99_ms": pct(lp, 99) * 1e3,
            "plain_capacity_events_per_s": plain_rate, "batched_capacity_events_per_s": cap,
            "latency": "completion on the device minus scheduled arrival; H2D of the event included"}


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
    ap.add_argument("--paper-only", action="store_true",
                    help="run only the paper-shaped self-join and print its JSON (a profiling aid)")
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
        print(json.dumps({"paper_shaped": bench_paper_shaped(frnn, args.steps, args.warmup)}), flush=True)
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
    dt, dt_api, nnz, stats, prof = bench_single(frnn, x, w.r, w.K, args.steps, args.warmup)
    ms = dt / args.steps * 1e3
    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1), "total_ms": v[1]} for k, v in prof.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    cand = stats["candidates"]
    ops = cand * 3 * D            # D subtracts, D multiplies, D adds per candidate pair
    avg_s = kern[dom]["avg_ms"] * 1e-3
    achieved = ops / avg_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_OPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / (VALU_PEAK_OPS / 1e12), "traffic": counter_traffic() if dom == "count" else None,
            "kernel": dom, "kernel_avg_ms": kern[dom]["avg_ms"],
            "algorithmic_ops_per_launch": ops, "candidates_per_launch": cand,
            "candidates_per_pair": cand / max(nnz, 1)}
    out = {"metric": METRIC, "value": nnz * args.steps / dt, "unit": "neighbour pairs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "tracks-300k-d8: one tracking-shaped event, N=300000, D=8, "
                                  "25000 tracks x 12 (sigma 0.02) + 10% uniform noise, r=0.1, "
                                  "K=256, queries = references", "N": 300000, "D": 8, "r": 0.1, "K": 256,
                      "parallelism": "1 GPU"},
           "events_per_s": args.steps / dt, "pairs_per_step": nnz,
           "api_build_query": {"ms_per_step": dt_api / args.steps * 1e3,
                               "pairs_per_s": nnz * args.steps / dt_api,
                               "events_per_s": args.steps / dt_api},
           "roofline": roof, "kernels": kern,
           "edge_export": bench_edges(frnn, x, w.r, w.K),
           "host_interface": bench_host(frnn, w.points, w.r, w.K)}
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w.points, w.r, w.K)
    del x
    torch.cuda.empty_cache()
    if not args.no_paper:
        log("paper-shaped")
        out["paper_shaped"] = bench_paper_shaped(frnn)
        torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched")
        out["batched"] = bench_batched(frnn)
    if not args.no_serving:
        log("serving")
        out["serving"] = bench_serving(frnn, args.serve_events)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
