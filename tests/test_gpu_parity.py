"""GPU parity: every scan's sorted match list equals the CPU oracle's, bit for bit.

All calls go through the C ABI (libac.so via its ctypes binding). Inputs are
seeded (synth); expected values come from the oracle at run time or from
tests/golden/*.json, which tests/golden/make_golden.py writes with the oracle.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from synth import DNA, PROTEIN, dna_text, plain_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PLACEMENTS = [ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_FULL, ac.AC_PLACE_LDS_HOT]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def build(patterns, placement=ac.AC_PLACE_AUTO, hot_states=0):
    d, o = ac.patterns_csr(patterns)
    return ac.ac_build(d, o, opts=ac._opts(placement=placement, hot_states=hot_states))


def to_device(text) -> "torch.Tensor":
    a = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    t = torch.empty(max(1, len(a)), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(np.array(a, dtype=np.uint8, copy=True)))
    return t[: len(a)]


def gpu_keys(auto, text, algo=ac.AC_ALGO_DFA, chunk=0, placement=0, capacity=None,
             walkers=0, block_bytes=0) -> np.ndarray:
    d = to_device(text) if not isinstance(text, torch.Tensor) else text
    keys = ac.scan_text(auto, d, capacity=capacity,
                        opts=ac._scan_opts(algo, chunk, 0, placement, walkers, block_bytes))
    return np.sort(ac.keys_to_numpy(keys))


def placements_for(auto):
    info = ac.ac_info(auto)
    out = [ac.AC_PLACE_GLOBAL]
    if 256 + info["table_bytes"] + 4 * 528 <= 160 * 1024:
        out.append(ac.AC_PLACE_LDS_FULL)
    if info["hot_states"]:
        out.append(ac.AC_PLACE_LDS_HOT)
    return out


# ---------------------------------------------------------------- worked examples

@pytest.mark.parametrize("name", ["fig1_abede.json", "fig6_ushers.json"])
@pytest.mark.parametrize("placement", [ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_FULL, ac.AC_PLACE_LDS_HOT])
@pytest.mark.parametrize("algo", [ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC])
def test_worked_example(name, placement, algo):
    g = json.load(open(os.path.join(GOLDEN, name)))
    pats = [p.encode() for p in g["patterns"]]
    text = g["text"].encode()
    expect = np.array(sorted((e << 32) | k for e, k in g["matches"]), dtype=np.uint64)
    a = build(pats, placement=placement)
    assert np.array_equal(gpu_keys(a, text, algo=algo), expect)
    # embedded in a longer text, at every alignment to a 16-byte block
    for lead in range(0, 40, 3):
        t = b"Z" * lead + text + b"Q" * 7
        assert np.array_equal(gpu_keys(a, t, algo=algo, chunk=16), oracle.oracle_match(t, pats))


# ---------------------------------------------------------------- small workload

@pytest.fixture(scope="module")
def small():
    w = plain_workload("dna1m")
    return w, oracle.oracle_match(w.text, w.patterns)


@pytest.mark.parametrize("algo", [ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC])
@pytest.mark.parametrize("placement", [ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_FULL,
                                       ac.AC_PLACE_LDS_HOT])
def test_small_dna(small, algo, placement):
    w, expect = small
    note("small dna1m", algo, placement)
    a = build(w.patterns, placement=placement, hot_states=300 if placement == ac.AC_PLACE_LDS_HOT else 0)
    got = gpu_keys(a, w.text, algo=algo)
    assert got.size == expect.size and np.array_equal(got, expect)


@pytest.mark.parametrize("walkers", [1, 2, 3, 4])
@pytest.mark.parametrize("chunk", [16, 32, 48, 64, 80, 1024, 4096, 1 << 20])
def test_small_dna_chunk_lengths(small, chunk, walkers):
    w, expect = small
    a = build(w.patterns)
    for bb in (64, 128):
        assert np.array_equal(gpu_keys(a, w.text, chunk=chunk, walkers=walkers, block_bytes=bb),
                              expect), bb


def test_determinism(small):
    w, expect = small
    a = build(w.patterns)
    d = to_device(w.text)
    r1, r2 = gpu_keys(a, d), gpu_keys(a, d)
    assert np.array_equal(r1, r2) and np.array_equal(r1, expect)


# ---------------------------------------------------------------- chunk boundaries

def boundary_case(chunk: int, m: int, n: int, seed: int):
    """Patterns copied from the text so that occurrences end at every offset
    kC - j, j in [0, m], around several chunk boundaries kC."""
    text = dna_text(n, seed)
    rng = np.random.default_rng(seed)
    pats = []
    for k in range(1, min(6, n // chunk)):
        for j in range(0, m + 1):
            e = k * chunk - j
            ln = int(rng.integers(1, m + 1))
            if e - ln + 1 >= 0 and e < n:
                pats.append(text[e - ln + 1:e + 1].tobytes())
    pats += [dna_text(int(rng.integers(1, m + 1)), seed * 7 + i).tobytes() for i in range(10)]
    return text, pats


@pytest.mark.parametrize("chunk", [16, 32, 48, 64, 112, 256])
@pytest.mark.parametrize("m", [1, 15, 16, 17, 33])
def test_chunk_boundaries(chunk, m):
    text, pats = boundary_case(chunk, m, 6 * chunk + 37, seed=chunk * 100 + m)
    expect = oracle.oracle_match(text, pats)
    for placement in (ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_HOT):
        a = build(pats, placement=placement, hot_states=7 if placement == ac.AC_PLACE_LDS_HOT else 0)
        for walkers in (1, 2, 3, 4):
            for bb in (64, 128):
                assert np.array_equal(gpu_keys(a, text, chunk=chunk, walkers=walkers, block_bytes=bb),
                                      expect), (chunk, m, placement, walkers, bb)
    a = build(pats)
    assert np.array_equal(gpu_keys(a, text, algo=ac.AC_ALGO_PFAC), expect)


@pytest.mark.parametrize("n", [0, 1, 2, 15, 16, 17, 31, 33, 47, 100, 1023, 1025, 4099])
def test_ragged_and_tiny_texts(n):
    text = (b"ACGTTGCAACGT" * 400)[:n]
    pats = [b"A", b"ACG", b"GTTGCAACGTACGTTG", b"T" * 20, b"CAACGTACGTTGCAACGTAC"]
    expect = oracle.oracle_match(text, pats)
    for placement in (ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_FULL, ac.AC_PLACE_LDS_HOT):
        a = build(pats, placement=placement)
        for algo in (ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC):
            for chunk in (0, 16, 32):
                for walkers in ((1, 2, 3, 4) if algo == ac.AC_ALGO_DFA else (0,)):
                    if algo == ac.AC_ALGO_PFAC and chunk:
                        continue
                    for bb in ((64, 128) if algo == ac.AC_ALGO_DFA else (0,)):
                        assert np.array_equal(gpu_keys(a, text, algo=algo, chunk=chunk, walkers=walkers,
                                                       block_bytes=bb),
                                              expect), (n, placement, algo, chunk, walkers, bb)


def test_bytes_outside_the_alphabet():
    rng = np.random.default_rng(4)
    text = dna_text(50_000, 3)
    holes = rng.integers(0, len(text), size=2000)
    text[holes] = rng.integers(0, 256, size=2000).astype(np.uint8)
    pats = [text[i:i + int(rng.integers(3, 12))].tobytes() for i in rng.integers(0, 49_000, 200)]
    pats += [b"ACGT", b"NNN", b"\x00A", b"GATTACA"]
    expect = oracle.oracle_match(text, pats)
    a = build(pats)
    for placement in placements_for(a):
        for algo in (ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC):
            assert np.array_equal(gpu_keys(a, text, algo=algo, placement=placement), expect)


def test_nested_duplicate_and_dense_outputs():
    pats = [b"A", b"AA", b"AAA", b"A", b"AAAA" * 4, b"C", b"AC", b"CA"]
    text = (b"A" * 37 + b"C" + b"A" * 50 + b"CA") * 30
    expect = oracle.oracle_match(text, pats)
    a = build(pats)
    for placement in placements_for(a):
        for algo in (ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC):
            for chunk in (0, 16, 48):
                if algo == ac.AC_ALGO_PFAC and chunk:
                    continue
                assert np.array_equal(gpu_keys(a, text, algo=algo, chunk=chunk, placement=placement),
                                      expect)


def test_protein_small():
    w = plain_workload("protein1g", n=1 << 22)
    pats = w.patterns[:5000]
    expect = oracle.oracle_match(w.text, pats)
    a = build(pats)
    assert ac.ac_info(a)["class_hashed"] == 0
    for placement in placements_for(a):
        note("protein small", placement)
        assert np.array_equal(gpu_keys(a, w.text, placement=placement), expect)
    assert np.array_equal(gpu_keys(a, w.text, algo=ac.AC_ALGO_PFAC), expect)


# ---------------------------------------------------------------- errors and overflow

def test_overflow_reports_true_count(small):
    w, expect = small
    a = build(w.patterns)
    d = to_device(w.text)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    for cap in (0, 1, 5):
        with pytest.raises(ac.AcError) as e:
            ac.ac_scan_sync(a, d, d.numel(), out, cap, count)
        assert e.value.status == ac.AC_ERR_OVERFLOW
        assert int(count.item()) == expect.size
        if cap:
            got = ac.keys_to_numpy(out[:cap])
            assert set(got.tolist()) <= set(expect.tolist())


def test_misaligned_text_rejected(small):
    w, _ = small
    a = build(w.patterns)
    d = to_device(w.text)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(ac.AcError) as e:
        ac.ac_scan(a, d[1:], d.numel() - 1, None, 0, count)
    assert e.value.status == ac.AC_ERR_INVALID


# ---------------------------------------------------------------- sort

@pytest.mark.parametrize("n", [0, 1, 2, 4095, 4096, 4097, 100_003])
def test_sort_matches(n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64)
    keys[: n // 3] = keys[n // 3: 2 * (n // 3)]  # duplicates
    t = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    ac.sort_keys(t)
    torch.cuda.synchronize()
    assert np.array_equal(ac.keys_to_numpy(t), np.sort(keys))


# ---------------------------------------------------------------- full-size workloads

def digest(keys: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(keys, dtype="<u8").tobytes()).hexdigest()


def check_full(name, algo=ac.AC_ALGO_DFA, device_sort=False):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))
    note("full", name, "generate")
    w = plain_workload(name)
    assert len(w.text) == g["n"]
    a = build(w.patterns)
    d = to_device(w.text)
    note("full", name, "scan", ac.ac_info(a)["placement"], algo)
    keys = ac.scan_text(a, d, capacity=g["count"] + 16, opts=ac._scan_opts(algo))
    if device_sort:
        ac.sort_keys(keys)
        torch.cuda.synchronize()
        got = ac.keys_to_numpy(keys)
    else:
        got = np.sort(ac.keys_to_numpy(keys))
    assert got.size == g["count"]
    assert [int(k) for k in got[:64]] == g["first"]
    assert [int(k) for k in got[-64:]] == g["last"]
    assert digest(got) == g["sha256"]
    # planted occurrences are all present
    have = set(got.tolist()) if got.size < 5_000_000 else None
    if have is not None:
        for k, off in enumerate(w.planted_offsets):
            if off >= 0:
                assert ((int(off) + len(w.patterns[k]) - 1) << 32 | k) in have


def test_full_dna256m_dfa():
    check_full("dna256m", device_sort=True)


def test_full_dna256m_pfac():
    check_full("dna256m", algo=ac.AC_ALGO_PFAC)


def test_full_dna256m_gated():
    check_full("dna256m", algo=ac.AC_ALGO_GATED)


def test_full_protein1g_dfa():
    check_full("protein1g", device_sort=True)


def test_full_protein1g_gated():
    check_full("protein1g", algo=ac.AC_ALGO_GATED, device_sort=True)


# ---------------------------------------------------------------- streaming (carried state)

def stream_scan(auto, text: np.ndarray, cuts, opts=None):
    """Scan `text` in the pieces between `cuts`, carrying the machine state;
    returns the sorted keys and the final state token."""
    total = len(text)
    out = torch.empty(max(16, total // 8 + 64), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    states = torch.zeros(2, dtype=torch.int32, device="cuda")
    bounds = [0] + sorted(cuts) + [total]
    for i in range(len(bounds) - 1):
        lo, hi = bounds[i], bounds[i + 1]
        piece = to_device(text[lo:hi])
        s_in = None if i == 0 else states[(i - 1) % 2:(i - 1) % 2 + 1]
        s_out = states[i % 2:i % 2 + 1]
        ac.ac_scan_stream(auto, piece, hi - lo, lo, s_in, s_out, out, out.numel(), count,
                          append=i > 0, opts=opts)
    torch.cuda.synchronize()
    n = int(count.item())
    assert n <= out.numel()
    last = (len(bounds) - 2) % 2
    return np.sort(ac.keys_to_numpy(out[:n])), int(states[last].item())


@pytest.mark.parametrize("placement", [ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_HOT])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_stream_pieces(placement, seed):
    w = plain_workload("dna1m", n=1 << 17)
    rng = np.random.default_rng(seed)
    text = w.text.copy()
    pats = list(w.patterns) + [b"A" * 12, b"ACGTACGTACGTAC"]
    # occurrences straddling the cuts: plant some patterns right across them
    cuts = sorted(set(int(c) for c in rng.integers(1, len(text), size=40)))
    cuts += [cuts[0] + 1, cuts[0] + 2, cuts[-1]]  # tiny and empty pieces
    for c in cuts[:10]:
        p = pats[int(rng.integers(0, len(pats)))]
        lo = max(0, c - len(p) // 2)
        text[lo:lo + len(p)] = np.frombuffer(p, dtype=np.uint8)[: len(text) - lo]
    expect = oracle.oracle_match(text, pats)
    a = build(pats, placement=placement, hot_states=200 if placement == ac.AC_PLACE_LDS_HOT else 0)
    whole, st_whole = stream_scan(a, text, [])
    assert np.array_equal(whole, expect)
    for chunk in (0, 64, 48):
        got, st = stream_scan(a, text, cuts, opts=ac._scan_opts(0, chunk, 0, 0, 0))
        assert np.array_equal(got, expect), chunk
        assert st == st_whole


def test_stream_rejects_pfac_and_aliasing():
    a = build([b"AB"])
    d = to_device(b"ABAB" * 8)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.zeros(64, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ac.AcError):
        ac.ac_scan_stream(a, d, 32, 0, None, st, out, 64, count, opts=ac._scan_opts(ac.AC_ALGO_PFAC))
    with pytest.raises(ac.AcError):
        ac.ac_scan_stream(a, d, 32, 0, st, st, out, 64, count)


# ---------------------------------------------------------------- failure-less build

@pytest.mark.parametrize("placement", [ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_FULL,
                                       ac.AC_PLACE_LDS_HOT])
def test_goto_only_build_pfac(small, placement):
    """A machine built without failure function and DFA scans with PFAC to the
    oracle's list; DFA scans, batches and servers refuse it."""
    w, expect = small
    d, o = ac.patterns_csr(w.patterns)
    a = ac.ac_build(d, o, opts=ac._opts(placement=placement, flags=ac.AC_BUILD_GOTO_ONLY,
                                        hot_states=300 if placement == ac.AC_PLACE_LDS_HOT else 0))
    assert ac.ac_info(a)["goto_only"] == 1
    got = gpu_keys(a, w.text, algo=ac.AC_ALGO_PFAC)
    assert np.array_equal(got, expect)
    with pytest.raises(ac.AcError):
        gpu_keys(a, w.text)  # DFA scan
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a], np.zeros(1, np.uint64), np.array([64], np.uint64), np.zeros(1, np.uint32))
    with pytest.raises(ac.AcError):
        ac.Server([a])


def test_scan_captured_in_a_graph(small):
    """A caller can capture ac_scan (counter reset + scan, both kernels) into a
    hipGraph and replay it; every replay, with eager work and host
    synchronisation between replays, gives the oracle's list."""
    w, expect = small
    a = build(w.patterns)
    d = to_device(w.text)
    n = len(w.text)
    cap = 1 << 16
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    opts = ac._scan_opts(ac.AC_ALGO_DFA)
    s = torch.cuda.Stream()
    ac.ac_scan(a, d, n, out, cap, cnt, opts, s)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ac.ac_scan(a, d, n, out, cap, cnt, opts, s)
    other = to_device(dna_text(1 << 15, 9))
    for i in range(4):
        out.fill_(-1)
        cnt.fill_(123456)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(cnt.item()) == expect.size, i
        assert np.array_equal(np.sort(ac.keys_to_numpy(out[:expect.size])), expect), i
        ac.scan_text(a, other)  # eager work between replays
        torch.cuda.synchronize()


# ---------------------------------------------------------------- append mode

@pytest.mark.parametrize("algo,alphabet", [(ac.AC_ALGO_DFA, "dna"), (ac.AC_ALGO_PFAC, "dna"),
                                           (ac.AC_ALGO_GATED, "dna"), (ac.AC_ALGO_GATED, "protein")])
def test_append_mode_fills_one_list(algo, alphabet):
    """With append set, *d_count is kept: two scans of two texts leave both
    lists, one after the other, and the sum of their counts."""
    name = "dna1m" if alphabet == "dna" else "protein1g"
    w = plain_workload(name, n=1 << 20)
    pats = [p for p in w.patterns if len(p) >= 6][:2000]
    a = build(pats)
    t1, t2 = w.text[: 300_000], w.text[300_000: 700_017]
    e1, e2 = oracle.oracle_match(t1, pats), oracle.oracle_match(t2, pats)
    out = torch.full((e1.size + e2.size + 64,), -1, dtype=torch.int64, device="cuda")
    cnt = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    opts = ac._scan_opts(algo, append=1)
    cnt.zero_()
    ac.ac_scan(a, to_device(t1), t1.size, out, out.numel(), cnt, opts)
    torch.cuda.synchronize()
    assert int(cnt.item()) == e1.size
    ac.ac_scan(a, to_device(t2), t2.size, out, out.numel(), cnt, opts)
    torch.cuda.synchronize()
    assert int(cnt.item()) == e1.size + e2.size
    got = ac.keys_to_numpy(out[: e1.size + e2.size])
    assert np.array_equal(np.sort(got), np.sort(np.concatenate([e1, e2])))
    with pytest.raises(ac.AcError):
        ac.ac_scan(a, to_device(t1), t1.size, out, out.numel(), cnt, ac._scan_opts(algo, append=2))
