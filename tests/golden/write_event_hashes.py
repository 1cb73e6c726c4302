"""Write per-event digests of the CPU oracle's CSR for the multi-event
workloads, so that GPU tests can compare every event bit for bit without
re-running a brute force of several trillion pair evaluations.

    python tests/golden/write_event_hashes.py batch64     # 64 uneven tracking events
    python tests/golden/write_event_hashes.py stream40    # 40 log-normal served events

Each event's digest is the SHA-256 of its oracle CSR, serialised as
offsets (int64, little endian) || indices (int32) || dist2 bit patterns
(uint32), the same byte layout the tests hash the GPU output in.  The file
also records each event's size, pair count and uncapped degree sum.  Only
the oracle and the seeded generators are called; the output is written
after every event, and an interrupted run resumes where it stopped.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2609_31980_amd import inputs  # noqa: E402

R = float(np.float32(0.1))
K = 256
STREAM_EVENTS = 40


def csr_digest(offsets, indices, dist2) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(indices, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(dist2, dtype=np.float32).view("<u4").tobytes())
    return h.hexdigest()


def batch64_events():
    sizes = inputs.c3_sizes()
    for e, x in enumerate(inputs.c3_events(sizes=sizes)):
        yield e, x


def stream40_events():
    tr = inputs.c5_trace(STREAM_EVENTS, rate=1.0)
    for e, a in enumerate(tr):
        yield e, inputs.c5_event(a)


WORKLOADS = {
    "batch64": ("batch64_hashes.json", batch64_events,
                "inputs.c3_events(): 64 tracking events, N ~ U{50000..400000}, D=8, seed 1003"),
    "stream40": ("stream40_hashes.json", stream40_events,
                 f"inputs.c5_event(a) for a in inputs.c5_trace({STREAM_EVENTS}, rate=1.0): "
                 "log-normal sizes (median 100000, sigma 0.6, clipped to [10000, 500000]), D=8, seed 1005"),
}


def main(which: str, nthreads: int = 0):
    fname, gen, desc = WORKLOADS[which]
    path = os.path.join(HERE, fname)
    doc = {"workload": desc, "r": R, "K": K, "self_join": True, "exclude_self": False,
           "digest": "sha256(offsets int64 LE || indices int32 LE || dist2 bits uint32 LE)",
           "events": []}
    if os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
    done = {ev["event"] for ev in doc["events"]}
    o = oracle.get()
    for e, x in gen():
        if e in done:
            continue
        t0 = time.perf_counter()
        c = o.frnn(x, R, K, nthreads=nthreads)
        dt = time.perf_counter() - t0
        doc["events"].append({"event": e, "N": int(len(x)), "nnz": int(c.nnz),
                              "degree_sum": int(c.degree.sum()),
                              "sha256": csr_digest(c.offsets, c.indices, c.dist2)})
        doc["events"].sort(key=lambda v: v["event"])
        with open(path + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(path + ".tmp", path)
        print(f"{which} event {e}: N={len(x)} nnz={c.nnz} ({dt:.1f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
