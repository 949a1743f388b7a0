"""Benchmark: scanned text GB/s of the plain scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dna256m]

One step = one ac_scan with the matcher AC_ALGO_AUTO picks (the gated
failure-less scan for the headline workloads) over the whole text, which is
already resident in HBM. Three copies of the text are scanned in rotation so
that no step can be served from the previous step's cache contents (3 x 256
MiB exceeds the 256 MB MALL). Machine construction, the device sort of the
match list, the chunked full-DFA scan and the failure-less (PFAC) kernel are
timed separately and reported beside the headline, as are the 1 GiB protein
configuration and the batched and served forms.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# The served form runs one HIP stream per slot; kernels on streams that share
# a hardware queue run one after another, so give the process as many queues
# as the server has slots (set before the HIP runtime starts).
SERVE_SLOTS = 16
os.environ["GPU_MAX_HW_QUEUES"] = str(max(SERVE_SLOTS, int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4)))

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOAD_DESC = {
    "dna1m": "1 MiB i.i.d. uniform ACGT text; 100 patterns of length 8-16, half planted",
    "dna256m": "256 MiB i.i.d. uniform ACGT text; 10,000 patterns of length 20-32, 10% planted",
    "protein1g": "1 GiB 20-letter text, letter p ~ rank^-0.8; 50,000 patterns of length 6-20, 20% planted",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, stream, torch, pre=None):
    """Per-step HIP event pairs on `stream` (the stream the kernels run on);
    pre(i), when given, runs in each step before its first event."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if pre is not None:
            pre(i)
        evs[i][0].record(stream)
        fn(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in evs]
    return wall, ms


# per scan kernel: its rocprofv3 counter summary and the sources it is built from
PROFILES = {
    "dfa": ("dfa_scan_dna256m.md", ["paper_1403_1305_amd/csrc/dfa_kernel.h",
                                    "paper_1403_1305_amd/csrc/device_common.h",
                                    "paper_1403_1305_amd/csrc/dfa.hip"]),
    "gated": ("gate_scan_dna256m.md", ["paper_1403_1305_amd/csrc/gate.hip",
                                       "paper_1403_1305_amd/csrc/device_common.h",
                                       "paper_1403_1305_amd/csrc/machine.h"]),
    "qgated": ("qgate_scan_protein1g.md", ["paper_1403_1305_amd/csrc/qgate.hip",
                                           "paper_1403_1305_amd/csrc/device_common.h",
                                           "paper_1403_1305_amd/csrc/machine.h"]),
}
ALGOS = {"auto": 0, "dfa": 1, "pfac": 2, "gated": 3}
ALGO_NAMES = {1: "dfa", 2: "pfac", 3: "gated"}


def kernel_source_sha256(kind):
    import hashlib
    h = hashlib.sha256()
    for f in PROFILES[kind][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pfac_lookups_per_byte(auto, sample):
    """Goto lookups the failure-less scan makes per text byte: from every
    start of `sample`, one lookup per byte until a missing edge (or a byte in
    no pattern), counted on the automaton's host tables."""
    import numpy as np

    from paper_1403_1305_amd import ac

    go = ac.ac_get_table(auto, ac.AC_TABLE_GO)
    cols = ac.ac_info(auto)["n_cols"]
    cmap = ac.ac_get_table(auto, ac.AC_TABLE_CMAP).astype(np.int64)
    cls = cmap[np.asarray(sample, dtype=np.uint8)]
    n = len(cls)
    # all starts advance together: one vectorised lookup per step
    state = np.zeros(n, dtype=np.int64)
    pos = np.arange(n, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    lookups = 0
    while alive.any():
        idx = np.nonzero(alive)[0]
        p = pos[idx]
        ok = p < n
        idx, p = idx[ok], p[ok]
        c = cls[p]
        known = c < cols  # 255 (or 256): a byte in no pattern ends the walk without a lookup
        lookups += int(known.sum())
        idx, p, c = idx[known], p[known], c[known]
        e = go[state[idx] * cols + c]
        edge = e != 0
        alive[:] = False
        alive[idx[edge]] = True
        state[idx[edge]] = (e[edge] & 0x7FFFFFFF).astype(np.int64)
        pos[idx[edge]] += 1
    return round(lookups / n, 3)


def profiled_traffic(workload, kind):
    """HBM bytes per scan launch from the committed rocprofv3 counter summary,
    or None when the summary is for another workload or the kernel sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", PROFILES[kind][0]) if kind in PROFILES else ""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("workload") != workload or fields.get("kernel_source_sha256") != kernel_source_sha256(kind):
        return None
    return int(fields["traffic_bytes_per_launch"])


def resolved_algo(ac, auto, algo):
    """The matcher ac_scan runs for `algo` (AUTO resolved as the library does)."""
    if algo != 0:
        return algo
    info = ac.ac_info(auto)
    if info["has_gate"] and info["gate_pass"] <= 0.05:
        return 3
    return 2 if info["goto_only"] else 1


def cpu_baseline(w, sample_bytes, min_s=10.0, max_passes=3):
    """The oracle (single-threaded failure-link scan) over the first
    sample_bytes of the same text, repeated until at least min_s seconds of
    CPU work (at most max_passes passes)."""
    import oracle
    ac_cpu = oracle.OracleAC(w.patterns)
    sample = w.text[:sample_bytes]
    passes, dt, count = 0, 0.0, 0
    while passes < max_passes and (passes == 0 or dt < min_s):
        t0 = time.perf_counter()
        count = ac_cpu.scan(sample).size
        dt += time.perf_counter() - t0
        passes += 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(passes * len(sample) / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "host_threads": os.cpu_count(), "host_cpu": model,
            "sample": f"{passes} pass(es) over the first {len(sample) >> 20} MiB of the same text, full pattern "
                      f"set, single-threaded failure-link scan ({dt:.1f} s); build not timed"}, (ac_cpu, sample, count)


def cpu_all_cores(ac_cpu, sample, count, m_max, min_s=2.0, max_passes=5):
    """The same oracle on every host thread (at most 16): the sample is cut
    into one slice per thread, each read from m_max - 1 bytes before its
    start and keeping the matches that end inside it (the chunk rule of the
    GPU scan). Its match count must equal the single-threaded pass."""
    import threading
    import numpy as np
    T = max(1, min(os.cpu_count() or 1, 16))
    n = len(sample)
    bounds = [n * t // T for t in range(T + 1)]
    got = [None] * T

    def work(t):
        lo, hi = bounds[t], bounds[t + 1]
        start = max(0, lo - (m_max - 1))
        keys = ac_cpu.scan(sample[start:hi])
        ends = (keys >> np.uint64(32)).astype(np.int64) + start
        got[t] = keys[ends >= lo]

    passes, dt = 0, 0.0
    while passes < max_passes and (passes == 0 or dt < min_s):
        threads = [threading.Thread(target=work, args=(t,)) for t in range(T)]
        t0 = time.perf_counter()
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        dt += time.perf_counter() - t0
        passes += 1
    total = int(sum(g.size for g in got))
    return {"value": round(passes * n / dt / 1e9, 6), "unit": "GB/s", "cores": T, "kind": "oracle, text slices",
            "exact_count": total == count,
            "sample": f"{passes} pass(es) over the same {n >> 20} MiB, one slice per thread with an m_max - 1 "
                      f"byte lead-in ({dt:.1f} s)"}


BATCHED_DESC = ("4,096 i.i.d. uniform ACGT texts, lengths log-uniform in [1 KiB, 4 MiB]; 16 resident "
                 "pattern sets of 100-20,000 patterns (lengths 8-32), each text naming one at random")


def bench_batched(args, torch, ac, stream):
    """The batched form: one autotuned persistent launch over every text
    (hipGraph-captured submission), against per-text plain ac_scan launches of
    the same texts; both lists must agree exactly."""
    import numpy as np

    from paper_1403_1305_amd import autotune
    from synth import batched_workload

    log("generate batched")
    texts, sets, text_set = batched_workload()
    buf, offs, lens = ac.pack_texts(texts)
    del texts
    total = int(lens.sum())
    t0 = time.perf_counter()
    autos = []
    for s in sets:
        d, o = ac.patterns_csr(s)
        autos.append(ac.ac_build(d, o, opts=ac._opts(placement=ac.AC_PLACE_LDS_HOT)))
    build_s = time.perf_counter() - t0
    states = [ac.ac_info(a)["n_states"] for a in autos]
    d_text = torch.from_numpy(buf).to("cuda")
    del buf
    cap = 1 << 25
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    log("tune batched")
    batch, tune, report = autotune.tune_batch(autos, d_text, offs, lens, text_set, out, cap, count,
                                              stream=stream, use_cache=False)
    info = ac.ac_batch_info(batch)
    log("batched plan", info, report["choice"])

    def step(i, graph=True):
        ac.ac_batch_scan(batch, d_text, out, cap, count, graph, stream)

    for i in range(args.warmup):
        step(i)
    steps = max(3, args.steps // 2)
    wall, ms = time_steps(step, steps, stream, torch)
    _, ms_eager = time_steps(lambda i: step(i, False), steps, stream, torch)
    matches = int(count.item())
    assert matches <= cap, "batched output buffer too small"
    keys = np.sort(ac.keys_to_numpy(out[:matches]))

    # per-text plain launches of the same texts, each into its own slice
    pos = (keys >> np.uint64(32)).astype(np.int64)
    per_text = np.diff(np.searchsorted(pos, np.append(offs.astype(np.int64), np.int64(1) << 40)))
    slot = np.concatenate([[0], np.cumsum(per_text)]).astype(np.int64)
    counts = torch.zeros(len(offs), dtype=torch.int64, device="cuda")
    out2 = torch.empty(max(1, matches), dtype=torch.int64, device="cuda")
    popts = ac._scan_opts(ac.AC_ALGO_AUTO, 0, 0, 0)  # each text with the matcher AUTO picks for it

    def plain(i):
        for t in range(len(offs)):
            o, n = int(offs[t]), int(lens[t])
            if n:
                ac.ac_scan(autos[int(text_set[t])], d_text[o:o + n], n, out2[int(slot[t]):],
                           int(per_text[t]), counts[t:t + 1], popts, stream)

    plain(0)
    pwall, pms = time_steps(plain, 2, stream, torch)
    got = counts.cpu().numpy()
    exact = bool(np.array_equal(got, per_text))
    if exact:
        k2 = ac.keys_to_numpy(out2[:matches]).copy()
        for t in range(len(offs)):  # positions relative to each text -> batch buffer
            k2[slot[t]:slot[t + 1]] += np.uint64(int(offs[t])) << np.uint64(32)
        exact = bool(np.array_equal(np.sort(k2), keys))
    kernel_ms = float(np.mean(ms))
    achieved = (total + 8 * matches) / (kernel_ms * 1e-3) / 1e9
    return {
        "value": round(total * steps / wall / 1e9, 3), "unit": "GB/s",
        "workload": f"batched: {BATCHED_DESC}",
        "n_texts": len(offs), "text_bytes": total, "automata": len(autos),
        "states_min_max": [min(states), max(states)], "matches": matches,
        "graph_ms": round(kernel_ms, 4), "eager_ms": round(float(np.mean(ms_eager)), 4),
        "plan": {k: info[k] for k in ("algo", "placement", "walkers", "chunk", "threads", "grid", "n_tasks")},
        "autotune": {"choice": report["choice"], "tune_s": round(report["tune_s"], 2),
                     "candidates": len(report.get("candidates", []))},
        "plain_per_text": {"value": round(total * len(pms) / pwall / 1e9, 3), "unit": "GB/s",
                           "ms": round(float(np.mean(pms)), 3), "launches": int((lens > 0).sum())},
        "speedup_vs_plain": round(float(np.mean(pms)) / kernel_ms, 2),
        "exact_vs_plain": exact,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "build_s": round(build_s, 2),
    }


SERVED_DESC = ("scan requests with lengths log-uniform in [1 KiB, 64 MiB], half DNA and half skewed protein; "
               "8 resident automata of 1,000-50,000 patterns (4 DNA, lengths 8-32; 4 protein, 6-20); "
               "Poisson arrivals at a fixed rate; HBM-budget admission")


def bench_protein(args, torch, ac, stream):
    """The 1 GiB skewed-protein configuration beside the headline: the matcher
    AUTO picks for it (the hashed-gate scan), timed like the headline (HIP
    events on the scan stream, each step appending into a counter of its own),
    its last timed list checked against the oracle's digest."""
    import hashlib

    import numpy as np

    from synth import plain_workload

    name = "protein1g"
    log("generate", name)
    w = plain_workload(name)
    n = len(w.text)
    d, o = ac.patterns_csr(w.patterns)
    auto = ac.ac_build(d, o)
    info = ac.ac_info(auto)
    text = torch.from_numpy(w.text).to("cuda")
    algo = resolved_algo(ac, auto, ALGOS[args.algo])
    kind = ALGO_NAMES[algo]
    if kind == "gated" and info["has_gate"] == 2:
        kind = "qgated"
    cap = 1 << 24
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    warm = torch.zeros(1, dtype=torch.int64, device="cuda")
    steps = max(3, args.steps // 2)
    counts = torch.zeros(steps, dtype=torch.int64, device="cuda")
    opts = ac._scan_opts(algo, 0, 0, 0, 0, append=1)
    for _ in range(2):
        warm.zero_()
        ac.ac_scan(auto, text, n, out, cap, warm, opts, stream)
    torch.cuda.synchronize()
    log("timed", name, kind)
    wall, ms = time_steps(lambda i: ac.ac_scan(auto, text, n, out, cap, counts[i:i + 1], opts, stream),
                          steps, stream, torch)
    per = counts.cpu().numpy()
    matches = int(per[-1])
    assert (per == matches).all(), "every timed step must report the same match count"
    golden_ok = None
    gpath = os.path.join(ROOT, "tests", "golden", name + ".json")
    if os.path.exists(gpath) and matches <= cap:
        g = json.load(open(gpath))
        got = np.sort(ac.keys_to_numpy(out[:matches]))
        golden_ok = bool(got.size == g["count"] and
                         hashlib.sha256(np.ascontiguousarray(got, dtype="<u8").tobytes()).hexdigest() == g["sha256"])
    kernel_ms = float(np.mean(ms))
    achieved = (n + 8 * matches) / (kernel_ms * 1e-3) / 1e9
    return {"workload": f"{name}: {WORKLOAD_DESC[name]}", "value": round(n * steps / wall / 1e9, 3),
            "unit": "GB/s", "steps": steps, "kernel": f"{kind}_scan", "matches": matches,
            "kernel_ms": round(kernel_ms, 4), "kernel_ms_median": round(float(np.median(ms)), 4),
            "exact_vs_oracle_digest": golden_ok, "gate_pass": round(info["gate_pass"], 5),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(name, kind)}}


def bench_served(args, torch, ac, stream, rhos=(0.5, 0.8)):
    """The served form: requests replayed through ac_serve_* (continuous
    batching, budget admission, pieces with carried state) against the same
    requests as serial plain ac_scan launches on one stream."""
    import numpy as np

    from synth import served_workload

    log("generate served")
    w = served_workload()
    R = len(w.length)
    total = int(w.length.sum())
    d_texts = [torch.from_numpy(t).to("cuda") for t in w.texts]
    t0 = time.perf_counter()
    autos = []
    for s in w.sets:
        d, o = ac.patterns_csr(s)
        autos.append(ac.ac_build(d, o))
    build_s = time.perf_counter() - t0
    views = [d_texts[int(w.alpha[i])][int(w.offset[i]):int(w.offset[i] + w.length[i])] for i in range(R)]

    # serial plain scans: one after another on one stream
    cap = 1 << 26
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    counts = torch.zeros(R, dtype=torch.int64, device="cuda")

    def serial(_):
        for i in range(R):
            ac.ac_scan(autos[int(w.automaton[i])], views[i], int(w.length[i]), out, cap, counts[i:i + 1],
                       None, stream)

    serial(0)
    torch.cuda.synchronize()
    swall, sms = time_steps(serial, 2, stream, torch)
    plain_counts = counts.cpu().numpy()
    serial_gbs = total * len(sms) / swall / 1e9
    serial_ms = swall / len(sms) * 1e3
    del out
    torch.cuda.empty_cache()

    budget = 4 << 30
    srv = ac.Server(autos, hbm_budget=budget, max_inflight=args.slots, max_large=args.max_large)

    def replay(arrivals_ns):
        base = srv.now_ns() + 50_000_000  # submissions finish well before the first arrival
        tickets = [srv.submit(int(w.automaton[i]), views[i], n=int(w.length[i]), on_device=True,
                              arrival_ns=base + int(arrivals_ns[i])) for i in range(R)]
        res = []
        for t in tickets:
            r = srv.wait(t, 120_000)  # an error, not a silent hang, if a request never finishes
            res.append((r.t_submit_ns, r.t_admit_ns, r.t_done_ns, r.n_matches, r.rescans))
            srv.release(t)
        a = np.array(res, dtype=np.float64)
        lat = (a[:, 2] - a[:, 0]) / 1e6
        span = (a[:, 2].max() - a[:, 0].min()) / 1e9
        return {"value": round(total / span / 1e9, 3), "unit": "GB/s",
                "p50_ms": round(float(np.percentile(lat, 50)), 4),
                "p99_ms": round(float(np.percentile(lat, 99)), 4),
                "mean_ms": round(float(lat.mean()), 4), "makespan_ms": round(span * 1e3, 3),
                "rescans": int(a[:, 4].sum())}, a[:, 3].astype(np.int64)

    log("served: saturated")
    replay(np.zeros(R))  # warm-up: rates learnt, kernels loaded
    sat, got = replay(np.zeros(R))
    exact = bool(np.array_equal(got, plain_counts))
    sat["running_peak"] = srv.stats()["running_peak"]
    rng = np.random.default_rng(6)
    poisson = []
    for rho in rhos:
        lam = rho * serial_gbs * 1e9 / (total / R)  # requests per second
        arr = np.cumsum(rng.exponential(1.0 / lam, size=R)) * 1e9
        arr -= arr[0]
        log(f"served: poisson rho={rho}")
        rec, got = replay(arr)
        exact &= bool(np.array_equal(got, plain_counts))
        rec.update({"rho": rho, "rate_per_s": round(lam, 1)})
        poisson.append(rec)

    # full lists of a sample of requests: served vs plain
    sample = np.argsort(w.length)[:: max(1, R // 12)]
    for i in sample:
        t = srv.submit(int(w.automaton[i]), views[i], n=int(w.length[i]), on_device=True)
        r = srv.wait(t, 120_000)
        a = np.sort(srv.keys(r))
        srv.release(t)
        b = np.sort(ac.keys_to_numpy(ac.scan_text(autos[int(w.automaton[i])], views[i])))
        exact &= bool(np.array_equal(a, b))
    st = srv.stats()
    srv.close()
    return {
        "workload": f"served: {SERVED_DESC}", "requests": R, "text_bytes": total, "automata": len(autos),
        "slots": args.slots, "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]), "hbm_budget": budget,
        "max_large": args.max_large,
        "piece_bytes": 16 << 20,
        "serial_plain": {"value": round(serial_gbs, 3), "unit": "GB/s", "ms": round(serial_ms, 3)},
        "saturated": sat, "poisson": poisson,
        "exact_vs_plain": exact, "pool_peak": st["pool_peak"], "build_s": round(build_s, 2),
    }


BUILD_DESC = ("total-time throughput, eq. (1): input bytes / (machine build + scan), DNA pattern sets of "
              "0.5M / 1M / 1.5M random patterns of 16-24 bytes (10 / 20 / 30 MB) and i.i.d. DNA inputs "
              "of 70 KB and 100 KB")


def bench_build(args, torch, ac, stream, sizes=(500_000, 1_000_000, 1_500_000), inputs=(70_000, 100_000)):
    """Build time and total-time throughput (eq. 1): the full machine (goto,
    failure, output, DFA) with the DFA scan against the failure-less machine
    (goto and own outputs only) with the PFAC scan, for growing pattern sets.
    Builds run on the host and include the upload of the tables."""
    import numpy as np

    from synth import DNA, dna_text, random_pattern_csr

    texts = {n: torch.from_numpy(dna_text(n, 77)).to("cuda") for n in inputs}
    out = torch.empty(1 << 22, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    rows = []
    for n_pat in sizes:
        pat, off = random_pattern_csr(n_pat, 16, 24, DNA, 4000 + n_pat // 1000)
        rec = {"patterns": n_pat, "pattern_mb": round(int(off[-1]) / 1e6, 1)}
        for kind, flags, algo in (("dfa", 0, ac.AC_ALGO_DFA), ("pfac_goto_only", ac.AC_BUILD_GOTO_ONLY,
                                                                   ac.AC_ALGO_PFAC)):
            log(f"build {n_pat} {kind}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a = ac.ac_build(pat, off, opts=ac._opts(flags=flags), stream=stream)
            build_s = time.perf_counter() - t0
            info = ac.ac_info(a)
            sub = {"build_s": round(build_s, 3), "host_build_s": round(info["build_ms"] / 1e3, 3),
                   "states": info["n_states"]}
            opts = ac._scan_opts(algo)
            for n in inputs:
                ac.ac_scan(a, texts[n], n, out, out.numel(), count, opts, stream)  # warm-up
                _, ms = time_steps(lambda i: ac.ac_scan(a, texts[n], n, out, out.numel(), count, opts, stream),
                                   5, stream, torch)
                scan_s = float(np.median(ms)) / 1e3
                sub[f"scan_ms_{n // 1000}k"] = round(scan_s * 1e3, 4)
                sub[f"throughput_Bps_{n // 1000}k"] = round(n / (build_s + scan_s), 1)
                sub[f"matches_{n // 1000}k"] = int(count.item())
            rec[kind] = sub
            del a
        for n in inputs:
            k = f"throughput_Bps_{n // 1000}k"
            rec[f"ratio_{n // 1000}k"] = round(rec["pfac_goto_only"][k] / rec["dfa"][k], 3)
        rows.append(rec)
        log(rec)
    return {"workload": f"build: {BUILD_DESC}", "unit": "B/s", "rows": rows}


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="dna256m", choices=sorted(WORKLOAD_DESC) + ["batched", "served", "build"])
    p.add_argument("--no-batched", action="store_true", help="skip the batched sub-benchmark")
    p.add_argument("--no-served", action="store_true", help="skip the served sub-benchmark")
    p.add_argument("--no-protein", action="store_true", help="skip the 1 GiB protein sub-benchmark")
    p.add_argument("--no-build", action="store_true", help="skip the build-time sub-benchmark")
    p.add_argument("--no-e1", action="store_true", help="skip the 0%%-planted timing check")
    p.add_argument("--slots", type=int, default=SERVE_SLOTS, help="requests a server holds on the device at once")
    p.add_argument("--max-large", type=int, default=0,
                   help="served: requests of 4 MiB or more on the device at once (0: no limit)")
    p.add_argument("--chunk", type=int, default=0)
    p.add_argument("--placement", type=int, default=0)
    p.add_argument("--cpu-sample-mib", type=int, default=256)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-pfac", action="store_true")
    p.add_argument("--no-dfa", action="store_true", help="skip the DFA timing beside a gated headline")
    p.add_argument("--algo", default="auto", choices=sorted(ALGOS),
                   help="headline matcher (auto: the one ac_scan picks by default)")
    p.add_argument("--walkers", type=int, default=0)
    p.add_argument("--calib-copy", action="store_true",
                   help="also run one plain device copy of the text's size (the reference "
                        "kernel for scaling FETCH_SIZE / WRITE_SIZE counter readings)")
    args = p.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the scan has no multi-GPU path in this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1403_1305_amd import ac
    from synth import plain_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if args.workload == "batched":
        b = bench_batched(args, torch, ac, stream)
        rec = {"metric": "scanned text GB/s (% of HBM peak), batched vs plain", "value": b["value"],
               "unit": "GB/s", "n_gpus": 1, "steps": max(3, args.steps // 2), "warmup": args.warmup,
               "ms_per_step": b["graph_ms"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "u8", "data": "synthetic",
               "config": {"workload": b["workload"], "n_texts": b["n_texts"], "n_bytes": b["text_bytes"],
                          "automata": b["automata"], "kernel": "batch_scan"},
               "pct_hbm_peak": round(100 * b["value"] / HBM_PEAK_GBS, 2), "roofline": b["roofline"],
               "cpu_baseline": None, "batched": b}
        print(json.dumps(rec), flush=True)
        return

    if args.workload == "build":
        v = bench_build(args, torch, ac, stream)
        last = v["rows"][-1]
        rec = {"metric": "total-time throughput, eq. (1), build + scan (failure-less PFAC vs full DFA)",
               "value": last["pfac_goto_only"]["throughput_Bps_100k"], "unit": "B/s", "n_gpus": 1,
               "steps": 5, "warmup": 1, "ms_per_step": round(last["pfac_goto_only"]["build_s"] * 1e3, 2),
               "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u8",
               "data": "synthetic", "config": {"workload": v["workload"], "patterns": last["patterns"],
                                               "n_bytes": 100_000, "kernel": "pfac_scan"},
               "roofline": None, "cpu_baseline": None, "build": v}
        print(json.dumps(rec), flush=True)
        return

    if args.workload == "served":
        v = bench_served(args, torch, ac, stream)
        p80 = v["poisson"][-1]
        rec = {"metric": "served aggregate GB/s (saturated) with p50/p99 latency under Poisson load",
               "value": v["saturated"]["value"], "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
               "ms_per_step": v["saturated"]["makespan_ms"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "u8", "data": "synthetic",
               "config": {"workload": v["workload"], "requests": v["requests"], "n_bytes": v["text_bytes"],
                          "automata": v["automata"], "kernel": "dfa_scan (served)"},
               "p50_ms": p80["p50_ms"], "p99_ms": p80["p99_ms"], "roofline": None, "cpu_baseline": None,
               "served": v}
        print(json.dumps(rec), flush=True)
        return

    log("generate", args.workload)
    w = plain_workload(args.workload)
    n = len(w.text)
    d, o = ac.patterns_csr(w.patterns)
    t0 = time.perf_counter()
    auto = ac.ac_build(d, o)
    build_wall_ms = (time.perf_counter() - t0) * 1e3
    info = ac.ac_info(auto)
    log("built", info)

    copies = [torch.from_numpy(w.text).to("cuda") for _ in range(3)]
    cap = 1 << 24
    outs = torch.empty(cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    algo = resolved_algo(ac, auto, ALGOS[args.algo])
    kind = ALGO_NAMES[algo]
    if kind == "gated" and info["has_gate"] == 2:
        kind = "qgated"  # the hashed gate's kernel
    # append mode into a counter of the step's own, zeroed before the timed
    # region: a step is the scan kernel alone (the launch rocprofv3 times),
    # which writes the whole match list from its start and counts it
    opts = ac._scan_opts(algo, args.chunk, 0, args.placement, args.walkers, append=1)
    log("headline matcher", kind)

    def zero(i):
        count.zero_()

    step_counts = torch.zeros(max(1, args.steps), dtype=torch.int64, device="cuda")

    def step(i):
        t = copies[i % 3]
        ac.ac_scan(auto, t, n, outs, cap, step_counts[i:i + 1], opts, stream)

    for i in range(args.warmup):
        zero(i)
        ac.ac_scan(auto, copies[i % 3], n, outs, cap, count, opts, stream)
    torch.cuda.synchronize()
    log("timed", kind)
    wall, ms = time_steps(step, args.steps, stream, torch)
    per_step = step_counts.cpu().numpy()
    matches = int(per_step[-1])
    assert (per_step == matches).all(), "every timed step must report the same match count"
    count.copy_(step_counts[-1:])
    # the timed list against the oracle's digest of this workload
    golden_ok = None
    gpath = os.path.join(ROOT, "tests", "golden", args.workload + ".json")
    if os.path.exists(gpath) and matches <= cap:
        import hashlib
        g = json.load(open(gpath))
        got = np.sort(ac.keys_to_numpy(outs[:matches]))
        golden_ok = bool(got.size == g["count"] and
                         hashlib.sha256(np.ascontiguousarray(got, dtype="<u8").tobytes()).hexdigest() == g["sha256"])
        del got
    kernel_ms = float(np.mean(ms))
    value = n * args.steps / wall / 1e9
    algo_bytes = n + 8 * matches
    achieved = algo_bytes / (kernel_ms * 1e-3) / 1e9

    kernel_ms_median = float(np.median(ms))

    # canonical order, timed separately
    keys = outs[:min(matches, cap)].clone()
    sort_ms = None
    if keys.numel() > 1:
        tmp = torch.empty(ac.ac_sort_scratch_bytes(keys.numel()), dtype=torch.uint8, device="cuda")
        _, sms = time_steps(lambda i: ac.ac_sort_matches(keys, keys.numel(), tmp, tmp.numel(), stream),
                            3, stream, torch)
        sort_ms = round(float(np.median(sms)), 4)

    # the chunked full-DFA walk over the same text, when it is not the headline
    dfa = None
    if kind != "dfa" and not args.no_dfa:
        dopts = ac._scan_opts(ac.AC_ALGO_DFA, args.chunk, 0, args.placement, args.walkers, append=1)
        dstep = lambda i: ac.ac_scan(auto, copies[i % 3], n, outs, cap, count, dopts, stream)
        for i in range(2):
            zero(i)
            dstep(i)
        log("timed dfa")
        dwall, dms = time_steps(dstep, max(5, args.steps // 2), stream, torch, pre=zero)
        dfa = {"value": round(n * len(dms) / dwall / 1e9, 3), "unit": "GB/s",
               "kernel_ms": round(float(np.mean(dms)), 4), "kernel_ms_median": round(float(np.median(dms)), 4),
               "matches": int(count.item()), "traffic": profiled_traffic(args.workload, "dfa")}

    pfac = None
    if not args.no_pfac:
        popts = ac._scan_opts(ac.AC_ALGO_PFAC, 0, 0, 0, append=1)
        pstep = lambda i: ac.ac_scan(auto, copies[i % 3], n, outs, cap, count, popts, stream)
        for i in range(2):
            zero(i)
            pstep(i)
        log("timed pfac")
        pwall, pms = time_steps(pstep, max(3, args.steps // 4), stream, torch, pre=zero)
        pfac = {"value": round(n * len(pms) / pwall / 1e9, 3), "unit": "GB/s",
                "kernel_ms": round(float(np.mean(pms)), 4), "matches": int(count.item()),
                "lookups_per_byte": pfac_lookups_per_byte(auto, w.text[:1 << 16]),
                "lookups_per_byte_sample": "every start of the first 64 KiB, on the host goto table"}

    # measured streaming-read ceiling: the library's read kernel (the scans'
    # 16-byte non-temporal loads, nothing else) over each text copy
    fold = torch.zeros(1, dtype=torch.int64, device="cuda")
    def read_step(i):
        ac.ac_hbm_read(copies[i % 3], n, fold, 0, stream)
    for i in range(2):
        read_step(i)
    _, rms = time_steps(read_step, 10, stream, torch)
    read_gbs = n / (float(np.median(rms)) * 1e-3) / 1e9

    # planted patterns must not change the scan time (the same text, 0% planted)
    e1 = None
    if args.workload == "dna256m" and not args.no_e1:
        w0 = plain_workload(args.workload, planted=0.0)
        d0, o0 = ac.patterns_csr(w0.patterns)
        a0 = ac.ac_build(d0, o0)
        for i in range(2):
            zero(i)
            ac.ac_scan(a0, copies[i % 3], n, outs, cap, count, opts, stream)
        _, ms0 = time_steps(lambda i: ac.ac_scan(a0, copies[i % 3], n, outs, cap, count, opts, stream),
                            10, stream, torch, pre=zero)
        e1 = {"planted": 0.0, "kernel_ms_median": round(float(np.median(ms0)), 4),
              "matches": int(count.item()), "planted_10pct_kernel_ms_median": round(kernel_ms_median, 4),
              "ratio": round(float(np.median(ms0)) / kernel_ms_median, 3)}
        del a0
        # the same machine over an unrelated text of the same size: only the
        # number of matches differs from the timed steps
        from synth import dna_text
        other = torch.from_numpy(dna_text(n, 1000 + w.cfg + 17)).to("cuda")
        others = [other, other.clone(), other.clone()]
        del other
        for i in range(2):
            zero(i)
            ac.ac_scan(auto, others[i % 3], n, outs, cap, count, opts, stream)
        _, ms1 = time_steps(lambda i: ac.ac_scan(auto, others[i % 3], n, outs, cap, count, opts, stream),
                            10, stream, torch, pre=zero)
        e1["same_machine_unrelated_text"] = {
            "kernel_ms_median": round(float(np.median(ms1)), 4), "matches": int(count.item()),
            "ratio": round(float(np.median(ms1)) / kernel_ms_median, 3)}
        del others
        # the timed text again, after the two runs above (drift of the device's clocks)
        _, ms2 = time_steps(lambda i: ac.ac_scan(auto, copies[i % 3], n, outs, cap, count, opts, stream),
                            10, stream, torch, pre=zero)
        e1["timed_text_again_kernel_ms_median"] = round(float(np.median(ms2)), 4)

    if args.calib_copy:
        # a kernel of known traffic (n bytes read, n written) for scaling the
        # HBM byte counters of a profiled run
        dst = torch.empty_like(copies[0])
        ac.ac_hbm_copy(dst, copies[1], n, 0, stream)
        torch.cuda.synchronize()

    cpu = cpu_all = None
    if not args.no_cpu:
        cpu, (ac_cpu, sample, count) = cpu_baseline(w, args.cpu_sample_mib << 20)
        log("cpu baseline, all cores")
        cpu_all = cpu_all_cores(ac_cpu, sample, count, max(len(p) for p in w.patterns))
        del ac_cpu, sample
    del copies, outs
    protein = None
    if args.workload != "protein1g" and not args.no_protein:
        torch.cuda.empty_cache()
        protein = bench_protein(args, torch, ac, stream)
        torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        batched = bench_batched(args, torch, ac, stream)
    build = None
    if not args.no_build:
        torch.cuda.empty_cache()
        build = bench_build(args, torch, ac, stream)
    served = None
    if not args.no_served:
        torch.cuda.empty_cache()
        served = bench_served(args, torch, ac, stream)

    rec = {
        "metric": "scanned text GB/s (% of HBM peak)",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "n_bytes": n, "n_patterns": len(w.patterns), "states": info["n_states"],
                   "placement": info["placement"], "hot_states": info["hot_states"],
                   "chunk": args.chunk or "auto", "kernel": f"{kind}_scan",
                   "gate_pass": round(info["gate_pass"], 5)},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "matches": matches,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(args.workload, kind)},
        "exact_vs_oracle_digest": golden_ok,
        "kernel_ms": round(kernel_ms, 4),
        "kernel_ms_median": round(kernel_ms_median, 4),
        "hbm_read_ceiling": {"value": round(read_gbs, 1), "unit": "GB/s",
                             "how": "median of 10 ac_hbm_read launches over the same text copies",
                             "scan_frac": round(value / read_gbs, 4)},
        "e1_planted0": e1,
        "build_ms": round(info["build_ms"], 2),
        "build_upload_ms": round(build_wall_ms, 2),
        "sort_ms": sort_ms,
        "dfa": dfa,
        "pfac": pfac,
        "cpu_baseline": cpu,
        "cpu_all_cores": cpu_all,
        "protein1g": protein,
        "batched": batched,
        "served": served,
        "build": build,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
