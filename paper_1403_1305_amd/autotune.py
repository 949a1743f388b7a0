"""Autotuner for the batched scan.

Picks the matcher (the gated failure-less scan when every automaton has the
class gate, or the chunked DFA), and for the DFA the table placement (LDS
image + global cold rows, or global table), the number of chunks each lane
walks (1 to 4) and the chunk length, for the gated scan the task length, by
timing candidate plans on the device with HIP events. The winner is cached
under a key of (GPU architecture, byte-class scheme, largest automaton's
state count, total text bytes, number of texts), each size rounded to a
power of two.

The input split follows the paper's data-parallel reading (§III: the input
is divided among workers, and several machines may serve the same input,
§IV.A); the choice of split length and of where the machine lives is this
library's, measured rather than fixed.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import ac

CACHE_ENV = "AC_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1403_1305_amd", "batch_tune.json")
CHUNKS = (0, 128, 256, 512, 1024, 2048, 4096)  # 0 = the plan's own choice
WALKERS = (1, 2, 3, 4)
GATED_TASKS = (0, 256 * 1008, 4096 * 1008)  # gated plans: start positions per task, 0 = the plan's choice


def _log2_bucket(x: int) -> int:
    return int(math.ceil(math.log2(max(1, int(x)))))


def tune_key(autos, text_len, arch: str | None = None) -> str:
    infos = [ac.ac_info(a) for a in autos]
    arch = arch or torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    scheme = f"h{infos[0]['class_hashed']}c{infos[0]['n_cols']}"
    states = max(i["n_states"] for i in infos)
    total = int(np.sum(np.asarray(text_len, dtype=np.uint64)))
    return (f"{arch}|{scheme}|S{_log2_bucket(states)}|T{_log2_bucket(total)}"
            f"|n{_log2_bucket(len(text_len))}|v2")


def candidates(autos):
    """(algo, placement, walkers, chunk) tuples valid for these automata."""
    infos = [ac.ac_info(a) for a in autos]
    images = all(i["hot_states"] > 0 for i in infos)
    places = [ac.AC_PLACE_LDS_HOT, ac.AC_PLACE_GLOBAL] if images else [ac.AC_PLACE_GLOBAL]
    cands = [(ac.AC_ALGO_DFA, p, w, c) for p in places for w in WALKERS for c in CHUNKS]
    if all(i["has_gate"] == 1 for i in infos):
        cands += [(ac.AC_ALGO_GATED, 0, 0, c) for c in GATED_TASKS]
    return cands


def make_tune(algo: int, placement: int, walkers: int, chunk: int) -> ac.ac_batch_tune:
    t = ac.ac_batch_tune()
    t.algo, t.placement, t.walkers, t.chunk = algo, placement, walkers, chunk
    return t


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(batch: ac.Batch, d_text, out, cap, count, reps: int, stream, use_graph=True) -> float:
    """Median milliseconds of one ac_batch_scan (counter reset + launch)."""
    stream = stream or torch.cuda.current_stream()
    ac.ac_batch_scan(batch, d_text, out, cap, count, use_graph, stream)  # warm-up, graph capture
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        ac.ac_batch_scan(batch, d_text, out, cap, count, use_graph, stream)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def tune_batch(autos, d_text, text_off, text_len, text_auto, out, cap, count, reps: int = 3,
               stream=None, cache_path: str | None = None, use_cache: bool = True):
    """Best plan for this batch.

    Returns (batch, tune, report): the plan built with the winning
    ac_batch_tune, that tune, and a dict with the key, whether it came from
    the cache, the tuning time and every candidate's median time.
    """
    path = cache_path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    key = tune_key(autos, text_len)
    cache = _load_cache(path) if use_cache else {}
    t0 = time.perf_counter()
    if key in cache:
        g, p, w, c = cache[key]["choice"]
        tune = make_tune(g, p, w, c)
        batch = ac.ac_batch_create(autos, text_off, text_len, text_auto, tune=tune, stream=stream)
        return batch, tune, {"key": key, "cached": True, "tune_s": time.perf_counter() - t0,
                             "choice": [g, p, w, c]}
    timings = []
    best = None
    for g, p, w, c in candidates(autos):
        tune = make_tune(g, p, w, c)
        batch = ac.ac_batch_create(autos, text_off, text_len, text_auto, tune=tune, stream=stream)
        ms = time_plan(batch, d_text, out, cap, count, reps, stream)
        info = ac.ac_batch_info(batch)
        timings.append({"algo": g, "placement": p, "walkers": w, "chunk": info["chunk"], "ms": round(ms, 4)})
        if best is None or ms < best[0]:
            best = (ms, (g, p, w, c))
        ac.ac_batch_free(batch)
    g, p, w, c = best[1]
    tune = make_tune(g, p, w, c)
    batch = ac.ac_batch_create(autos, text_off, text_len, text_auto, tune=tune, stream=stream)
    if use_cache:
        cache = _load_cache(path)
        cache[key] = {"choice": [g, p, w, c], "ms": round(best[0], 4)}
        _store_cache(path, cache)
    return batch, tune, {"key": key, "cached": False, "tune_s": time.perf_counter() - t0,
                         "choice": [g, p, w, c], "candidates": timings}
