"""Bit-exact parity at full size on the multi-event workloads: every event of
the 64-event uneven batch and every event of a 40-event served stream
against digests of the CPU oracle's complete CSR (written once by
tests/golden/write_event_hashes.py, which calls only the oracle and the
seeded generators).  The digest covers offsets, indices and dist2 bits, so a
match is the oracle's CSR bit for bit; on a mismatch the event's rows are
compared with a live oracle run to name the first differing row."""
import json
import os
import time

import numpy as np
import pytest

import pinlib
from golden.write_event_hashes import K, R, csr_digest
from gpu_util import dev, say
from paper_2609_31980_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name, n):
    with open(os.path.join(GOLDEN, name)) as f:
        doc = json.load(f)
    ev = {e["event"]: e for e in doc["events"]}
    assert sorted(ev) == list(range(n)), f"{name} holds {len(ev)} of {n} events"
    return ev


@pytest.fixture(scope="module")
def frnn():
    import torch
    assert torch.cuda.is_available()
    from paper_2609_31980_amd import frnn as f
    return f


def explain(orc, x, got, what):
    """Name the first row that differs from a live oracle run."""
    pinlib.assert_csr_equal(got, pinlib.as_tuple(orc.frnn(x, R, K)), what)


def check_event(orc, x, got, want, what):
    off, idx, d2 = got
    assert len(off) == want["N"] + 1, f"{what}: {len(off) - 1} rows, want {want['N']}"
    if int(off[-1]) != want["nnz"] or csr_digest(off, idx, d2) != want["sha256"]:
        explain(orc, x, got, what)
        raise AssertionError(f"{what}: digest differs from the oracle's")


@pytest.fixture(scope="module")
def batch64():
    say("batch of 64: generating")
    return inputs.c3_events()


@pytest.mark.parametrize("persistent,graphs", [(0, 0), (1, 1)], ids=["grid", "persistent-graphs"])
def test_batch64_every_event_bit_exact(orc, frnn, batch64, persistent, graphs):
    """All 64 events (about 14.4 million points) in one batched call, twice,
    every event's CSR equal to the oracle's: with the default launch
    (kernels launched one by one), and with the persistent work queue
    replayed as HIP graphs (the second run replays the recorded graphs)."""
    import torch
    want = load("batch64_hashes.json", 64)
    xs = [dev(x) for x in batch64]
    opts = frnn.default_opts(persistent=persistent, graphs=graphs)
    for rep in range(2):
        say(f"batch of 64 (persistent={persistent}, graphs={graphs}): run {rep}")
        outs = frnn.query_batch(xs, R, K, opts=opts)
        for e, o in enumerate(outs):
            check_event(orc, batch64[e], o.numpy(), want[e], f"batch64 event {e} run {rep}")
            o.release()
        torch.cuda.synchronize()


def test_stream40_served_events_bit_exact(orc, frnn):
    """A 40-event stream of log-normal sizes (median 100,000 points) through
    the continuous-batching server: events arrive in bursts while earlier
    batches are on the device, and every served CSR equals the oracle's."""
    want = load("stream40_hashes.json", 40)
    tr = inputs.c5_trace(40, rate=1.0)
    say("stream of 40: generating")
    evs = [inputs.c5_event(a) for a in tr]
    srv = frnn.Server(8, R, K, hbm_budget_bytes=64 << 30, max_batch_events=16, max_inflight=2)
    try:
        tickets = []
        for i, x in enumerate(evs):
            tickets.append(srv.submit(x))
            if i % 7 == 6:
                time.sleep(0.002)   # let a batch start before the next burst
        batches = set()
        for i, t in enumerate(tickets):
            c, tm = srv.wait(t)
            batches.add(tm["batch_id"])
            check_event(orc, evs[i], c.numpy(), want[i], f"served event {i} (batch {tm['batch_id']})")
            c.release()
        say(f"stream of 40: {len(batches)} batches")
        assert len(batches) > 1
    finally:
        srv.close()


def test_stream40_served_under_tight_budget_bit_exact(orc, frnn):
    """The same stream under a 512 MiB budget with two workers: admission
    waits, idle workers drop their contexts and new ones are recorded into
    graphs (the graphs option) while the other worker runs and the client
    copies and releases results; every served CSR still equals the
    oracle's."""
    want = load("stream40_hashes.json", 40)
    tr = inputs.c5_trace(40, rate=1.0)
    say("stream of 40, tight budget: generating")
    evs = [inputs.c5_event(a) for a in tr]
    budget = 512 << 20
    srv = frnn.Server(8, R, K, hbm_budget_bytes=budget, max_batch_events=64, max_inflight=2,
                      opts=frnn.default_opts(graphs=1))
    try:
        tickets = [srv.submit(x) for x in evs]
        batches = set()
        for i, t in enumerate(tickets):
            c, tm = srv.wait(t)
            batches.add(tm["batch_id"])
            check_event(orc, evs[i], c.numpy(), want[i], f"tight-budget event {i} (batch {tm['batch_id']})")
            c.release()
        held, peak = srv.memory()
        say(f"stream of 40, tight budget: {len(batches)} batches, peak {peak >> 20} MiB")
        assert len(batches) > 2
    finally:
        srv.close()
