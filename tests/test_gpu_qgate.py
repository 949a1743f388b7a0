"""GPU parity of the gated failure-less scan with the hashed gate (protein-
shaped and other alphabets, every pattern at least 6 bytes): walks taken only
from the start positions whose 6-byte window passes the blocked Bloom filter
and is found in the window table must report exactly the oracle's matches,
whatever the text length, its alignment to the kernel's 16-byte lanes and
1 KiB wave steps, bytes outside the alphabet, shared or nested windows and
match-dense texts."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from synth import PROTEIN, plain_workload, protein_text

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
    assert ac.ac_info(a)["has_gate"] == 2
    return a


def gated(auto, text: np.ndarray, capacity=None) -> np.ndarray:
    t = torch.empty(max(16, text.size), dtype=torch.uint8, device="cuda")
    if text.size:
        t[: text.size].copy_(torch.from_numpy(np.ascontiguousarray(text)))
    keys = ac.scan_text(auto, t[: text.size], capacity=capacity, opts=ac._scan_opts(ac.AC_ALGO_GATED))
    return np.sort(ac.keys_to_numpy(keys))


def rand_patterns(rng, count, lo, hi):
    a = np.frombuffer(PROTEIN, np.uint8)
    return [a[rng.integers(0, a.size, int(L))].tobytes() for L in rng.integers(lo, hi + 1, count)]


def test_protein_workload_slice():
    """The 50,000-pattern protein set on 4 MiB of its text."""
    w = plain_workload("protein1g", n=1 << 22)
    a = build(w.patterns)
    note("qgate protein slice")
    assert np.array_equal(gated(a, w.text), oracle.oracle_match(w.text, w.patterns))


@pytest.mark.parametrize("n", [0, 1, 5, 6, 7, 15, 16, 17, 21, 22, 1007, 1008, 1013, 1024, 1025, 4095,
                               16 * 1024 + 7, 64 * 1024 + 9, 1_000_003])
def test_lengths_and_tails(n):
    """Patterns of 6-14 bytes (nested, duplicated, sharing windows) on texts
    of every length class: shorter than a window, ragged tails, whole and
    partial wave steps, several workgroups; occurrences planted at the very
    start and end."""
    rng = np.random.default_rng(n + 11)
    pats = rand_patterns(rng, 80, 6, 14)
    base = pats[0][:6]
    pats += [base, base + b"K", base + b"KL", base + b"KLM", b"AAAAAA", b"AAAAAAA"]
    a = build(pats)
    text = protein_text(n, 700 + n % 1000)
    for p in pats[-6:-2] + [pats[1]]:
        if n >= len(p):
            text[:len(p)] = np.frombuffer(p, np.uint8)
            text[n - len(p):] = np.frombuffer(p, np.uint8)
    note("qgate lengths", n)
    assert np.array_equal(gated(a, text), oracle.oracle_match(text, pats))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_arbitrary_bytes(seed):
    """Patterns and text over all 256 byte values (zero bytes, 0xff, lower
    case): the filter hashes raw bytes. With every byte value in some pattern
    the byte map has 256 columns and no entry is free to mark a byte in no
    pattern, so 0xff must still be matched (by the DFA and PFAC kernels
    too)."""
    rng = np.random.default_rng(seed)
    pats = [rng.integers(0, 256, int(L), dtype=np.uint8).tobytes() for L in rng.integers(6, 20, 300)]
    pats += rand_patterns(rng, 200, 6, 12)
    text = protein_text(300_000, 50 + seed)
    for p in pats[::3]:
        o = int(rng.integers(0, text.size - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, np.uint8)
    noise = rng.integers(0, text.size, 5000)
    text[noise] = rng.integers(0, 256, noise.size, dtype=np.uint8)
    assert len(set(b"".join(pats))) == 256
    a = build(pats)
    expect = oracle.oracle_match(text, pats)
    assert any((int(k) & 0xFFFFFFFF) in {i for i, p in enumerate(pats) if 255 in p} for k in expect)
    assert np.array_equal(gated(a, text), expect)
    t = torch.from_numpy(text).to("cuda")
    for algo in (ac.AC_ALGO_DFA, ac.AC_ALGO_PFAC):
        keys = ac.scan_text(a, t, opts=ac._scan_opts(algo))
        assert np.array_equal(np.sort(ac.keys_to_numpy(keys)), expect), algo


def test_every_position_a_candidate():
    """A text of one letter against patterns of it: every start passes and is
    walked, the start queues fill on every wave step."""
    pats = [b"A" * k for k in (6, 7, 10, 17)] + [b"ACDEFG"]
    text = np.full(70_000, ord("A"), np.uint8)
    text[33_333] = ord("C")
    a = build(pats)
    got = gated(a, text)
    assert got.size > 3 * 60_000
    assert np.array_equal(got, oracle.oracle_match(text, pats))


def test_windows_that_differ_in_one_byte():
    """Windows equal but for one byte (any of the six) must not be taken for
    one another by the table lookup."""
    rng = np.random.default_rng(5)
    base = bytearray(b"MKVLAT")
    pats = [bytes(base) + b"GG"]
    for i in range(6):
        for c in b"CDEW":
            v = bytearray(base)
            v[i] = c
            pats.append(bytes(v) + bytes([PROTEIN[int(rng.integers(0, 20))]]))
    text = protein_text(200_000, 9)
    for p in pats:
        for _ in range(3):
            o = int(rng.integers(0, text.size - len(p)))
            text[o:o + len(p)] = np.frombuffer(p, np.uint8)
            # and the window alone, not followed by the pattern's last byte
            o = int(rng.integers(0, text.size - 7))
            text[o:o + 6] = np.frombuffer(p[:6], np.uint8)
            text[o + 6] = ord("Y") if p[6] != ord("Y") else ord("W")
    a = build(pats)
    assert np.array_equal(gated(a, text), oracle.oracle_match(text, pats))


def test_overflow_reports_true_count():
    w = plain_workload("protein1g", n=1 << 18)
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
    w = plain_workload("protein1g", n=1 << 21)
    a = build(w.patterns)
    assert ac.ac_info(a)["gate_pass"] < 0.05
    expect = oracle.oracle_match(w.text, w.patterns)
    t = torch.from_numpy(w.text).to("cuda")
    assert np.array_equal(np.sort(ac.keys_to_numpy(ac.scan_text(a, t))), expect)  # AUTO
    dfa = ac.scan_text(a, t, opts=ac._scan_opts(ac.AC_ALGO_DFA))
    assert np.array_equal(np.sort(ac.keys_to_numpy(dfa)), expect)
    g = build(w.patterns, flags=ac.AC_BUILD_GOTO_ONLY)
    assert np.array_equal(gated(g, w.text), expect)
    d, o = ac.patterns_csr(w.patterns)
    n = ac.ac_build(d, o, opts=ac._opts(flags=ac.AC_BUILD_NO_GATE))
    with pytest.raises(ac.AcError):
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
    queue. The dense set uses five letters (no 2-bit class field tells five
    apart, so the hashed gate applies) and 6-8 byte patterns: parity on 3 MB
    of text over those letters, then a list a third of the size needed."""
    rng = np.random.default_rng(51 + dense)
    if dense:
        five = np.frombuffer(b"ACDEF", np.uint8)
        pats = [five[rng.integers(0, 5, int(L))].tobytes() for L in rng.integers(6, 9, 400)]
        text = five[rng.integers(0, 5, 3_000_017)]
    else:
        pats = rand_patterns(rng, 400, 8, 16)
        text = protein_text(3_000_017, 88)
    pats += pats[:3]  # duplicates: states with several patterns
    a = build(pats)
    assert (ac.ac_info(a)["match_rate"] > 4e-3) == dense
    for p in pats[::40]:
        at = int(rng.integers(0, text.size - len(p)))
        text[at:at + len(p)] = np.frombuffer(p, np.uint8)
    expect = oracle.oracle_match(text, pats)
    note("qgate stagings", dense, expect.size)
    assert np.array_equal(gated(a, text), expect)
    for cap in (0, 1, 5, expect.size // 3):
        overflow_case(a, text, expect, cap)
