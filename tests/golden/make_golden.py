"""Write the full-size expected match lists' digests, using only the CPU oracle.

    python tests/golden/make_golden.py [dna256m] [protein1g]

For each plain workload it regenerates the seeded text and pattern set
(synth.plain_workload), runs the failure-link oracle over the whole text, and
stores the match count, the SHA-256 of the sorted keys (little-endian uint64)
and the first and last keys in tests/golden/<workload>.json. Nothing here
touches the GPU library.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import plain_workload  # noqa: E402


def digest(keys: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(keys, dtype="<u8").tobytes()).hexdigest()


def make(name: str) -> dict:
    t0 = time.time()
    w = plain_workload(name)
    t1 = time.time()
    ac = oracle.OracleAC(w.patterns)
    t2 = time.time()
    keys = ac.scan(w.text)
    t3 = time.time()
    rec = {
        "workload": name,
        "source": "CPU oracle (failure-link Aho-Corasick) over the seeded workload; "
                  "written by tests/golden/make_golden.py",
        "n": int(len(w.text)),
        "n_patterns": len(w.patterns),
        "oracle_states": ac.n_states,
        "count": int(keys.size),
        "sha256": digest(keys),
        "first": [int(k) for k in keys[:64]],
        "last": [int(k) for k in keys[-64:]],
        "seconds": {"generate": round(t1 - t0, 1), "build": round(t2 - t1, 1),
                    "scan": round(t3 - t2, 1)},
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json"), "w") as f:
        json.dump(rec, f, indent=1)
    return rec


if __name__ == "__main__":
    for name in sys.argv[1:] or ["dna256m", "protein1g"]:
        r = make(name)
        print(name, r["count"], r["sha256"][:16], r["seconds"], flush=True)
