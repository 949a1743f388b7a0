"""GPU tests of the served form (ac_serve_*): continuous batching over resident
automata. Each request's match list must equal the oracle's and be the same
whether the request runs alone or in a mix that overlaps on the device.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from synth import DNA, PROTEIN, dna_text, protein_text

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")

PIECE = 4096  # small pieces, so that most requests carry state across several


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def build(patterns, placement=ac.AC_PLACE_AUTO):
    d, o = ac.patterns_csr(patterns)
    return ac.ac_build(d, o, opts=ac._opts(placement=placement))


def rand_patterns(rng, alphabet: bytes, count: int, lo: int, hi: int) -> list[bytes]:
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return [a[rng.integers(0, len(a), int(L))].tobytes() for L in rng.integers(lo, hi + 1, count)]


@pytest.fixture(scope="module")
def setup():
    """Four automata (two DNA, two protein, one with an LDS image and one
    global) and requests of mixed sizes, alphabets and memory kinds."""
    rng = np.random.default_rng(41)
    sets = [rand_patterns(rng, DNA, 100, 4, 12), rand_patterns(rng, DNA, 1500, 8, 32),
            rand_patterns(rng, PROTEIN, 50, 2, 6), rand_patterns(rng, PROTEIN, 800, 3, 12)]
    places = [ac.AC_PLACE_AUTO, ac.AC_PLACE_LDS_HOT, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_AUTO]
    autos = [build(s, p) for s, p in zip(sets, places)]
    sizes = [0, 1, 15, 16, 17, PIECE - 1, PIECE, PIECE + 1, 3 * PIECE + 5]
    sizes += [int(x) for x in np.exp(rng.uniform(np.log(16), np.log(1 << 18), 31))]
    reqs = []
    for i, n in enumerate(sizes):
        auto = int(rng.integers(0, 4))
        gen = dna_text if auto < 2 else protein_text
        text = gen(n, 500 + i) if n else np.zeros(0, np.uint8)
        reqs.append((auto, text, bool(i % 2)))  # odd requests: text already on the device
    orc = [oracle.OracleAC(s) for s in sets]
    expect = [orc[a].scan(t) for a, t, _ in reqs]
    return sets, autos, reqs, expect


def device_copy(text: np.ndarray) -> torch.Tensor:
    t = torch.empty(max(16, text.size), dtype=torch.uint8, device="cuda")
    if text.size:
        t[: text.size].copy_(torch.from_numpy(np.ascontiguousarray(text)))
    torch.cuda.synchronize()
    return t


def submit_all(srv, reqs, together=True):
    """Stage every text first, then submit them all; with `together` they are
    given one arrival time 20 ms ahead, so they reach the scheduler at once."""
    keep = [device_copy(t) if on_dev else (np.ascontiguousarray(t) if t.size else np.zeros(16, np.uint8))
            for _, t, on_dev in reqs]
    at = srv.now_ns() + 20_000_000 if together else 0
    tickets = [srv.submit(a, k, n=t.size, on_device=on_dev, arrival_ns=at)
               for (a, t, on_dev), k in zip(reqs, keep)]
    return keep, tickets


WAIT_MS = 60_000  # a request not done by then fails the test instead of hanging it


def collect(srv, tickets):
    out = []
    for t in tickets:
        r = srv.wait(t, WAIT_MS)
        assert r.status == 0
        out.append((np.sort(srv.keys(r)), r.pieces, r.rescans, r))
        srv.release(t)
    return out


def test_mix_equals_alone_and_oracle(setup):
    """40 requests of mixed sizes, half from host memory, all arriving at one
    time in 4 KiB pieces over 8 slots: every list equals the oracle's, and the
    same request run alone gives the same list. (This case once stalled: a
    request arriving between the scheduler's two clock readings of one pass
    was left for a wake-up that never came; one reading per pass since.)"""
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos, hbm_budget=64 << 20, max_inflight=8, piece_bytes=PIECE)
    keep, tickets = submit_all(srv, reqs)
    mix = collect(srv, tickets)
    st = srv.stats()
    note("mix stats", st)
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["queued"] == 0
    assert st["running_peak"] > 1  # requests overlapped on the device
    for i, ((keys, pieces, _, r), e) in enumerate(zip(mix, expect)):
        assert np.array_equal(keys, e), i
        gated = ac.ac_info(autos[reqs[i][0]])["gate_pass"] <= 0.05
        per_request = 1 if gated else (reqs[i][1].size + PIECE - 1) // PIECE
        assert pieces == per_request or reqs[i][1].size == 0, (i, pieces)
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_done_ns
    # each request alone, on the same server
    for i, (a, text, on_dev) in enumerate(reqs):
        keep, (t,) = submit_all(srv, [(a, text, on_dev)])
        (alone,) = collect(srv, [t])
        assert np.array_equal(alone[0], mix[i][0]), i
    srv.close()


def test_mix_equals_plain_scans(setup):
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos, piece_bytes=1 << 20)
    keep, tickets = submit_all(srv, reqs)
    mix = collect(srv, tickets)
    for i, (a, text, _) in enumerate(reqs):
        if text.size == 0:
            assert mix[i][0].size == 0
            continue
        plain = np.sort(ac.keys_to_numpy(ac.scan_text(autos[a], device_copy(text)[: text.size])))
        assert np.array_equal(mix[i][0], plain), i
    srv.close()


def test_small_budget_admits_by_memory(setup):
    """A budget that holds only a few requests at a time: admission waits for
    memory, every result is still exact, and the pool never exceeds it."""
    sets, autos, reqs, expect = setup
    budget = 1 << 20
    srv = ac.Server(autos, hbm_budget=budget, max_inflight=16, piece_bytes=PIECE)
    host_reqs = [(a, t, False) for a, t, _ in reqs]  # host texts take pool memory too
    keep, tickets = submit_all(srv, host_reqs)
    got = collect(srv, tickets)
    for i, e in enumerate(expect):
        assert np.array_equal(got[i][0], e), i
    st = srv.stats()
    assert st["pool_peak"] <= budget and st["pool_used"] == 0
    with pytest.raises(ac.AcError):
        srv.submit(0, np.zeros(2 << 20, np.uint8))  # alone larger than the budget
    srv.close()


def test_low_match_estimate_rescans_exactly(setup):
    """A match-rate guess far too low: requests overflow their lists and are
    scanned again into exact ones."""
    sets, autos, reqs, expect = setup
    # largest first, so the first requests admitted overflow before any
    # finished request can teach the server a better rate
    order = sorted(range(len(reqs)), key=lambda i: -reqs[i][1].size)
    srv = ac.Server(autos, piece_bytes=PIECE, match_ppm=1, max_inflight=4)
    keep, tickets = submit_all(srv, [reqs[i] for i in order])
    got = collect(srv, tickets)
    for g, i in zip(got, order):
        assert np.array_equal(g[0], expect[i]), i
    assert srv.stats()["rescans"] > 0 and sum(g[2] for g in got) > 0
    srv.close()


def test_invalid_requests(setup):
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos[:1])
    with pytest.raises(ac.AcError):
        srv.submit(1, np.zeros(64, np.uint8))  # no such automaton
    d = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ac.AcError):
        srv.submit(0, d[1:], n=32, on_device=True)  # misaligned device text
    with pytest.raises(ac.AcError):
        srv.wait(12345)
    with pytest.raises(ac.AcError):
        srv.release(12345)
    srv.close()


def test_close_with_unreleased_results(setup):
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos, piece_bytes=PIECE)
    keep, tickets = submit_all(srv, reqs[:10])
    for t in tickets:
        srv.wait(t, WAIT_MS)
    srv.close()  # frees the unreleased lists


def test_scheduled_arrivals(setup):
    """Requests given arrival times on the server's clock are not admitted
    before them, whatever order they were submitted in."""
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos, piece_bytes=PIECE)
    t0 = srv.now_ns() + 30_000_000  # 30 ms from now
    picks = [i for i, r in enumerate(reqs) if r[1].size][:12]
    keep, tickets = [], []
    for j, i in enumerate(reversed(picks)):  # submitted in reverse of their arrivals
        a, text, _ = reqs[i]
        d = device_copy(text)
        keep.append(d)
        tickets.append(srv.submit(a, d, n=text.size, on_device=True, arrival_ns=t0 + 1_000_000 * (len(picks) - j)))
    for j, (t, i) in enumerate(zip(tickets, reversed(picks))):
        r = srv.wait(t, WAIT_MS)
        assert r.t_submit_ns == t0 + 1_000_000 * (len(picks) - j)
        assert r.t_admit_ns >= r.t_submit_ns and r.t_done_ns >= r.t_admit_ns
        assert np.array_equal(np.sort(srv.keys(r)), expect[i])
        srv.release(t)
    srv.close()


def test_add_automaton_and_latency_stats(setup):
    """An automaton added to a running server serves requests; the stats
    report latency percentiles and throughput over the finished requests."""
    sets, autos, reqs, expect = setup
    srv = ac.Server(autos[:1], piece_bytes=PIECE)
    j = srv.add(autos[3])
    assert j == 1
    picks = [i for i, (a, t, _) in enumerate(reqs) if a in (0, 3) and t.size][:10]
    keep, tickets = submit_all(srv, [((0 if reqs[i][0] == 0 else 1), reqs[i][1], reqs[i][2]) for i in picks])
    got = collect(srv, tickets)
    for g, i in zip(got, picks):
        assert np.array_equal(g[0], expect[i]), i
    st = srv.stats()
    assert st["completed"] == len(picks) and st["bytes_done"] == sum(reqs[i][1].size for i in picks)
    assert 0 < st["p50_ms"] <= st["p99_ms"] and st["gbps"] > 0
    srv.close()


def test_list_larger_than_budget_fails_cleanly():
    """A request whose match list can never fit the budget ends with
    AC_ERR_TOO_LARGE instead of waiting forever; the server stays usable."""
    a = build([b"A"])  # a match at every 'A'
    srv = ac.Server([a], hbm_budget=1 << 20, piece_bytes=1 << 16)
    big = torch.full((600_000,), ord("A"), dtype=torch.uint8, device="cuda")  # 4.8 MB of keys
    t = srv.submit(0, big, on_device=True)
    with pytest.raises(ac.AcError) as e:
        srv.wait(t, WAIT_MS)
    assert e.value.status == ac.AC_ERR_TOO_LARGE
    srv.release(t)
    small = torch.full((1000,), ord("A"), dtype=torch.uint8, device="cuda")
    t = srv.submit(0, small, on_device=True)
    r = srv.wait(t, WAIT_MS)
    assert r.n_matches == 1000
    srv.release(t)
    assert srv.stats()["pool_used"] == 0
    srv.close()


def test_close_while_waiting_for_memory():
    """Results never released fill the pool; closing the server ends the
    requests still waiting instead of hanging."""
    a = build([b"A"])
    srv = ac.Server([a], hbm_budget=1 << 20, piece_bytes=1 << 16, match_ppm=1_000_000)
    x = torch.full((40_000,), ord("A"), dtype=torch.uint8, device="cuda")  # ~320 KB list each
    tickets = [srv.submit(0, x, on_device=True) for _ in range(6)]
    srv.wait(tickets[0], WAIT_MS)  # held, never released
    srv.close()


def test_grouped_short_requests():
    """Short requests against automata with the class gate that the scheduler
    issues in one pass share a launch (up to 16 per launch, 64 tiles per
    task): 48 requests arriving together over 16 slots, from 1 byte to just
    over the 4 MiB grouping limit (multi-task requests, and one that runs
    alone), against a sparse and a dense pattern set (the two match
    stagings), half of them from host memory, with at most one request of
    4 MiB or more on the device at a time. Every list equals the oracle's,
    and so does a request run alone afterwards."""
    rng = np.random.default_rng(77)
    sets = [rand_patterns(rng, DNA, 2000, 14, 28), rand_patterns(rng, DNA, 400, 6, 9)]
    autos = [build(s) for s in sets]
    for a in autos:
        assert ac.ac_info(a)["has_gate"] == 1 and ac.ac_info(a)["gate_pass"] <= 0.05
    assert ac.ac_info(autos[0])["match_rate"] < 4e-3 < ac.ac_info(autos[1])["match_rate"]
    sizes = [1, 9, 10, 17, 1008, 1009, 2016, 64 * 1008, 64 * 1008 + 1, 3 * 64 * 1008 + 5, (4 << 20), (4 << 20) + 16]
    sizes += [int(x) for x in np.exp(rng.uniform(np.log(16), np.log(1 << 21), 36))]
    reqs = []
    for i, n in enumerate(sizes):
        a = i % 2
        text = dna_text(n, 800 + i)
        for _ in range(min(20, n // 64)):  # planted occurrences of the long patterns too
            p = np.frombuffer(sets[a][int(rng.integers(len(sets[a])))], np.uint8)
            at = int(rng.integers(0, n - len(p)))
            text[at:at + len(p)] = p
        reqs.append((a, text, bool(i % 3)))
    orc = [oracle.OracleAC(s) for s in sets]
    expect = [orc[a].scan(t) for a, t, _ in reqs]
    srv = ac.Server(autos, hbm_budget=512 << 20, max_inflight=16, max_large=1)
    keep, tickets = submit_all(srv, reqs)
    got = collect(srv, tickets)
    for i, ((keys, pieces, _, _), e) in enumerate(zip(got, expect)):
        note("grouped", i, reqs[i][1].size, e.size)
        assert np.array_equal(keys, e), i
        assert pieces == 1, i
    assert srv.stats()["failed"] == 0
    keep, (t,) = submit_all(srv, [reqs[5]])
    (alone,) = collect(srv, [t])
    assert np.array_equal(alone[0], expect[5])
    srv.close()
