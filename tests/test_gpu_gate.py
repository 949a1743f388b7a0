"""GPU parity of the gated failure-less scan (AC_ALGO_GATED): the walks taken
only from the start positions whose next 10 bytes can begin a pattern must
report exactly the oracle's matches, whatever the text length, its alignment
to the kernel's 16-byte lanes and 1 KiB wave steps, bytes outside the
alphabet, short or nested patterns, and match-dense texts."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from synth import DNA, dna_text, plain_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def build(patterns, flags=0):
    d, o = ac.patterns_csr(patterns)
    a = ac.ac_build(d, o, opts=ac._opts(flags=flags))
    assert ac.ac_info(a)["has_gate"] == 1
    return a


def gated(auto, text: np.ndarray, capacity=None) -> np.ndarray:
    t = torch.empty(max(16, text.size), dtype=torch.uint8, device="cuda")
    if text.size:
        t[: text.size].copy_(torch.from_numpy(np.ascontiguousarray(text)))
    keys = ac.scan_text(auto, t[: text.size], capacity=capacity, opts=ac._scan_opts(ac.AC_ALGO_GATED))
    return np.sort(ac.keys_to_numpy(keys))


def rand_patterns(rng, count, lo, hi):
    a = np.frombuffer(DNA, np.uint8)
    return [a[rng.integers(0, 4, int(L))].tobytes() for L in rng.integers(lo, hi + 1, count)]


def test_small_workload():
    w = plain_workload("dna1m")
    a = build(w.patterns)
    assert np.array_equal(gated(a, w.text), oracle.oracle_match(w.text, w.patterns))


@pytest.mark.parametrize("n", [0, 1, 5, 9, 10, 11, 15, 16, 17, 31, 33, 1023, 1024, 1025, 1034, 4095,
                               16 * 1024 + 7, 64 * 1024 + 9, 1_000_003])
def test_lengths_and_tails(n):
    """Short patterns (1-12 bytes, nested and duplicated) on texts of every
    length class: shorter than a window, ragged tails, whole and partial wave
    steps, several workgroups."""
    rng = np.random.default_rng(n + 7)
    pats = rand_patterns(rng, 60, 1, 12) + [b"A", b"AC", b"ACG", b"ACGTACGTACGT", b"ACGTACGTACGT"]
    a = build(pats)
    text = dna_text(n, 900 + n % 1000)
    # plant a few occurrences, also at the very start and end
    for p in pats[-4:]:
        if n >= len(p):
            text[:len(p)] = np.frombuffer(p, np.uint8)
            text[n - len(p):] = np.frombuffer(p, np.uint8)
    note("gated lengths", n)
    assert np.array_equal(gated(a, text), oracle.oracle_match(text, pats))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bytes_outside_the_alphabet(seed):
    """'N', lower case letters (which share a class field with their upper
    case) and other bytes end every occurrence that would cross them."""
    rng = np.random.default_rng(seed)
    pats = rand_patterns(rng, 200, 3, 24)
    text = dna_text(300_000, 40 + seed)
    for p in pats[:40]:
        o = int(rng.integers(0, text.size - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, np.uint8)
    noise = rng.integers(0, text.size, 3000)
    text[noise] = np.frombuffer(b"NacgtX\x00\xff", np.uint8)[rng.integers(0, 8, noise.size)]
    a = build(pats)
    assert np.array_equal(gated(a, text), oracle.oracle_match(text, pats))


def test_every_position_a_candidate():
    """A text of one letter against patterns of that letter: every start is
    walked, the start queues fill on every wave step."""
    pats = [b"A" * k for k in (1, 3, 10, 11, 17)] + [b"CGT"]  # four letters: a 2-bit class field
    text = np.full(70_000, ord("A"), np.uint8)
    text[33_333] = ord("C")
    a = build(pats)
    got = gated(a, text)
    assert got.size > 5 * 60_000
    assert np.array_equal(got, oracle.oracle_match(text, pats))


def test_overflow_reports_true_count():
    w = plain_workload("dna1m", n=1 << 18)
    a = build(w.patterns)
    expect = oracle.oracle_match(w.text, w.patterns)
    d = torch.from_numpy(w.text).to("cuda")
    for cap in (0, 1, 5):
        out = torch.empty(max(1, cap), dtype=torch.int64, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ac.ac_scan(a, d, d.numel(), out, cap, cnt, ac._scan_opts(ac.AC_ALGO_GATED))
        assert int(cnt.item()) == expect.size
        got = ac.keys_to_numpy(out[:min(cap, expect.size)])
        assert set(got.tolist()) <= set(expect.tolist())


def test_auto_picks_the_gate_and_goto_only_builds_scan():
    w = plain_workload("dna256m", n=1 << 22)
    a = build(w.patterns)
    assert ac.ac_info(a)["gate_pass"] < 0.05
    expect = oracle.oracle_match(w.text, w.patterns)
    t = torch.from_numpy(w.text).to("cuda")
    assert np.array_equal(np.sort(ac.keys_to_numpy(ac.scan_text(a, t))), expect)  # AUTO
    g = build(w.patterns, flags=ac.AC_BUILD_GOTO_ONLY)
    assert np.array_equal(gated(g, w.text), expect)
    with pytest.raises(ac.AcError):
        d, o = ac.patterns_csr(w.patterns)
        n = ac.ac_build(d, o, opts=ac._opts(flags=ac.AC_BUILD_NO_GATE))
        ac.scan_text(n, t, opts=ac._scan_opts(ac.AC_ALGO_GATED))


def overflow_case(a, text, expect, cap):
    """Scan into a list of cap keys: the true count, and cap distinct valid keys."""
    d = torch.from_numpy(text).to("cuda")
    out = torch.empty(max(1, cap), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan(a, d, d.numel(), out, cap, cnt, ac._scan_opts(ac.AC_ALGO_GATED))
    assert int(cnt.item()) == expect.size
    got = ac.keys_to_numpy(out[:min(cap, expect.size)]).tolist()
    assert len(set(got)) == len(got) and set(got) <= set(expect.tolist())


@pytest.mark.parametrize("dense", [False, True])
def test_both_match_stagings(dense):
    """Pattern sets on either side of the expected match rate (4e-3 per byte)
    above which the scan stages matches in registers rather than in the LDS
    queue: parity on 3 MB of text (thousands of wavefront flushes when
    dense), then a list a third of the size needed."""
    rng = np.random.default_rng(41 + dense)
    pats = rand_patterns(rng, 400, 6, 9) if dense else rand_patterns(rng, 400, 14, 24)
    pats += pats[:3]  # duplicates: states with several patterns
    a = build(pats)
    assert (ac.ac_info(a)["match_rate"] > 4e-3) == dense
    text = dna_text(3_000_017, 77 + dense)
    for p in pats[::40]:  # planted occurrences of the long ones too
        at = int(rng.integers(0, text.size - len(p)))
        text[at:at + len(p)] = np.frombuffer(p, np.uint8)
    expect = oracle.oracle_match(text, pats)
    note("gated stagings", dense, expect.size)
    assert np.array_equal(gated(a, text), expect)
    for cap in (0, 1, 5, expect.size // 3):
        overflow_case(a, text, expect, cap)


@pytest.mark.parametrize("n8,n_long,seed", [(200, 2000, 0), (400, 6000, 1)])
def test_many_short_patterns(n8, n_long, seed):
    """Sets with many 8-byte patterns: each extends to 256 strings of 12
    classes, so 79% (first set) and 96% (second) of the second gate level's
    bits are set and most starts the first level passes are walked.
    The first set's expected match rate is below 4e-3 per byte (LDS
    staging), the second's above (register staging); both lists equal the
    oracle's, ragged tail included."""
    rng = np.random.default_rng(500 + seed)
    pats = rand_patterns(rng, n8, 8, 8) + rand_patterns(rng, n_long, 12, 32)
    a = build(pats)
    bits = np.unpackbits(ac.ac_get_table(a, ac.AC_TABLE_GATE2_BITS).view(np.uint8))
    assert bits.mean() > 0.5
    assert (ac.ac_info(a)["match_rate"] > 4e-3) == bool(seed)
    text = dna_text((3 << 20) + 12345 + seed, 600 + seed)
    expect = oracle.oracle_match(text, pats)
    assert expect.size > 5000
    note("many short patterns", n8, n_long, text.size, expect.size)
    assert np.array_equal(gated(a, text), expect)

