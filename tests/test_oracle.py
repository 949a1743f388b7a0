"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
  * the paper's worked examples (Sec. II.A Fig. 1, Sec. II.B Figs. 2-4,
    Sec. IV.A Fig. 6), stored as cited fixtures under tests/golden/;
  * the definition of the match set written out as brute force, on random
    tiny inputs (hypothesis);
  * closed forms: every k-mer as a pattern set, a run of one letter, a
    pattern with a byte the text lacks, and a library routine
    (bytes.find) for a single pattern;
  * invariants: planted occurrences, id permutation, pattern-set partition
    (the paper's pattern-focused split, Sec. IV.A), failure-less walk ==
    failure-link scan;
  * planted mistakes: mutated copies of the oracle source must fail the pins.
"""
from __future__ import annotations

import itertools
import json
import os
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle.naive import naive_match
from synth import dna_text, plain_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def keys(pairs):
    return np.array(sorted((e << 32) | k for e, k in pairs), dtype=np.uint64)


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- worked examples

def check_worked_example(g, lib=None):
    pats = [p.encode() for p in g["patterns"]]
    text = g["text"].encode()
    ac = oracle.OracleAC(pats, lib=lib)
    expect = keys(g["matches"])
    ok = True
    ok &= ac.n_states == g["ac_states"]
    ok &= np.array_equal(ac.scan(text), expect)
    ok &= ac.trace(text) == g["ac_trace"]
    for s, f in g["ac_fail"].items():
        ok &= ac.fail(int(s)) == f
    for p, states in g["pfac_walks"].items():
        ok &= ac.pfac_walk(text, int(p)) == states
    ok &= np.array_equal(ac.pfac_scan(text), expect)
    return bool(ok)


@pytest.mark.parametrize("name", ["fig1_abede.json", "fig6_ushers.json"])
def test_worked_example(name):
    g = load_golden(name)
    assert check_worked_example(g)
    # the fixture itself agrees with the definition of the match set
    pats = [p.encode() for p in g["patterns"]]
    assert np.array_equal(naive_match(g["text"].encode(), pats), keys(g["matches"]))


def test_fig1_failure_step_details():
    """Fig. 1 walk-through: from state 2 (AB) there is no edge on E, the
    failure link goes to 4 (B), which has an edge on E to 5."""
    ac = oracle.OracleAC([b"AB", b"ABG", b"BEDE", b"EF"])
    assert ac.goto(2, ord("E")) == -1
    assert ac.fail(2) == 4
    assert ac.goto(4, ord("E")) == 5
    assert ac.m_max == 4


# ---------------------------------------------------------------- brute force

alphabets = st.sampled_from([b"ab", b"abc", b"ACGT", b"\x00\xff"])


@st.composite
def small_case(draw):
    alpha = draw(alphabets)
    letter = st.sampled_from(list(alpha))
    text = bytes(draw(st.lists(letter, min_size=0, max_size=300)))
    pats = draw(st.lists(st.lists(letter, min_size=1, max_size=10).map(bytes),
                         min_size=1, max_size=24))
    # sometimes copy substrings of the text, or repeat a pattern
    if text and draw(st.booleans()):
        i = draw(st.integers(0, len(text) - 1))
        j = draw(st.integers(i + 1, min(len(text), i + 10)))
        pats.append(text[i:j])
    if draw(st.booleans()):
        pats.append(pats[0])
    return text, pats


@settings(max_examples=2000, deadline=None)
@given(small_case())
def test_bruteforce_agrees(case):
    text, pats = case
    ac = oracle.OracleAC(pats)
    expect = naive_match(text, pats)
    assert np.array_equal(ac.scan(text), expect)
    assert np.array_equal(ac.pfac_scan(text), expect)


def test_nested_prefix_suffix_and_duplicates():
    pats = [b"a", b"aa", b"aaa", b"ba", b"aab", b"b", b"aa", b"abab"]
    text = b"aaabababaaab" * 5
    ac = oracle.OracleAC(pats)
    assert np.array_equal(ac.scan(text), naive_match(text, pats))


# ---------------------------------------------------------------- closed forms

def base4(s: bytes) -> int:
    v = 0
    for ch in s:
        v = 4 * v + b"ACGT".index(ch)
    return v


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_all_kmers(k):
    """Every k-mer over ACGT as the pattern set (id = base-4 code, A<C<G<T):
    exactly one match at each end position e >= k-1, whose id is the code of
    the k bytes ending at e."""
    pats = [bytes(t) for t in itertools.product(b"ACGT", repeat=k)]
    assert all(base4(p) == i for i, p in enumerate(pats))
    text = dna_text(3000, 7).tobytes()
    got = oracle.oracle_match(text, pats)
    e, ids = oracle.split_keys(got)
    assert len(got) == len(text) - k + 1
    assert np.array_equal(e, np.arange(k - 1, len(text)))
    assert all(ids[i] == base4(text[i:i + k]) for i in range(0, len(text) - k + 1, 7))


@pytest.mark.parametrize("pattern", [b"ACA", b"AAAA", b"GATTACA", b"T"])
def test_single_pattern_vs_find(pattern):
    text = (dna_text(20000, 11).tobytes() + b"AAAAAAAACACACAGATTACAGATTACA") * 2
    ends = []
    i = text.find(pattern)
    while i >= 0:
        ends.append(i + len(pattern) - 1)
        i = text.find(pattern, i + 1)
    got = oracle.oracle_match(text, [pattern])
    assert np.array_equal(got, keys((e, 0) for e in ends))


@pytest.mark.parametrize("n,k", [(1, 1), (10, 3), (1000, 17), (5, 6)])
def test_run_of_one_letter(n, k):
    got = oracle.oracle_match(b"A" * n, [b"A" * k])
    assert np.array_equal(got, keys((e, 0) for e in range(k - 1, n)))


def test_absent_byte_and_empty_text():
    assert oracle.oracle_match(b"ACGT" * 100, [b"ACGN", b"N"]).size == 0
    assert oracle.oracle_match(b"", [b"A"]).size == 0


def test_rejects_empty_pattern():
    with pytest.raises(ValueError):
        oracle.OracleAC([b"A", b""])
    with pytest.raises(ValueError):
        oracle.OracleAC([])


# ---------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def small_workload():
    return plain_workload("dna1m")


def test_planted_occurrences_found(small_workload):
    w = small_workload
    got = set(oracle.oracle_match(w.text, w.patterns).tolist())
    for k, off in enumerate(w.planted_offsets):
        if off >= 0:
            assert ((int(off) + len(w.patterns[k]) - 1) << 32 | k) in got


def test_id_permutation(small_workload):
    w = small_workload
    text = w.text[: 1 << 16]
    base = oracle.oracle_match(text, w.patterns)
    perm = np.random.default_rng(3).permutation(len(w.patterns))
    got = oracle.oracle_match(text, [w.patterns[i] for i in perm])
    e, ids = oracle.split_keys(got)
    remapped = np.sort((e.astype(np.uint64) << np.uint64(32)) | perm[ids].astype(np.uint64))
    assert np.array_equal(remapped, base)


def test_partition_union(small_workload):
    """Splitting the pattern set into parts and scanning each part gives the
    same matches (with ids mapped back) as the whole set."""
    w = small_workload
    text = w.text[: 1 << 17]
    whole = oracle.oracle_match(text, w.patterns)
    parts = np.array_split(np.random.default_rng(5).permutation(len(w.patterns)), 3)
    acc = []
    for part in parts:
        got = oracle.oracle_match(text, [w.patterns[i] for i in part])
        e, ids = oracle.split_keys(got)
        acc.append((e.astype(np.uint64) << np.uint64(32)) | part[ids].astype(np.uint64))
    assert np.array_equal(np.sort(np.concatenate(acc)), whole)


def test_failure_less_equals_failure_links(small_workload):
    w = small_workload
    ac = oracle.OracleAC(w.patterns)
    assert np.array_equal(ac.pfac_scan(w.text), ac.scan(w.text))


def test_window_matches(small_workload):
    w = small_workload
    ac = oracle.OracleAC(w.patterns)
    full = ac.scan(w.text)
    e, _ = oracle.split_keys(full)
    rng = np.random.default_rng(9)
    for _ in range(20):
        lo = int(rng.integers(0, len(w.text)))
        hi = min(len(w.text), lo + int(rng.integers(1, 50000)))
        sel = full[(e >= lo) & (e < hi)]
        assert np.array_equal(oracle.window_matches(ac, w.text, lo, hi), sel)


# ---------------------------------------------------------------- planted mistakes

MUTANTS = {
    "no_output_union": ("if (s != 0) {\n            ivec *f = &m->out[m->fail[s]];",
                        "if (0) {\n            ivec *f = &m->out[m->fail[s]];"),
    "single_failure_hop_in_build": ("while (r != 0 && m->go[(size_t)r * 256 + a] == NO_EDGE) r = m->fail[r];",
                                    "if (r != 0 && m->go[(size_t)r * 256 + a] == NO_EDGE) r = m->fail[r];"),
    "failures_to_root": ("m->fail[t] = (g != NO_EDGE && g != t) ? g : 0;", "m->fail[t] = 0;"),
    "single_failure_hop_in_scan": ("while (s != 0 && m->go[(size_t)s * 256 + a] == NO_EDGE) s = m->fail[s];",
                                   "if (s != 0 && m->go[(size_t)s * 256 + a] == NO_EDGE) s = m->fail[s];"),
    "end_off_by_one": ("kvec_push(&out, (i << 32)", "kvec_push(&out, ((i + 1) << 32)"),
    "pfac_emits_failure_outputs": ("for (int32_t i = 0; i < m->own[s].n; i++)\n                if (kvec_push(out, (j << 32) | (uint32_t)m->own[s].v[i]))",
                                   "for (int32_t i = 0; i < m->out[s].n; i++)\n                if (kvec_push(out, (j << 32) | (uint32_t)m->out[s].v[i]))"),
    "pfac_no_stop": ("if (t == NO_EDGE) break;\n        s = t;", "if (t == NO_EDGE) t = 0;\n        s = t;"),
    "wrong_id": ("ivec_push(&m->own[s], (int32_t)k)", "ivec_push(&m->own[s], (int32_t)(n - 1 - k))"),
}


def pin_suite(lib) -> bool:
    """The pins above, condensed; True iff all hold for the library ``lib``."""
    for name in ("fig1_abede.json", "fig6_ushers.json"):
        if not check_worked_example(load_golden(name), lib):
            return False
    rnd = random.Random(1)
    for _ in range(300):
        alpha = rnd.choice([b"ab", b"abc", b"ACGT"])
        text = bytes(rnd.choice(alpha) for _ in range(rnd.randint(0, 120)))
        pats = [bytes(rnd.choice(alpha) for _ in range(rnd.randint(1, 6)))
                for _ in range(rnd.randint(1, 12))]
        ac = oracle.OracleAC(pats, lib=lib)
        expect = naive_match(text, pats)
        if not (np.array_equal(ac.scan(text), expect) and np.array_equal(ac.pfac_scan(text), expect)):
            return False
    return True


def test_pin_suite_passes_on_oracle():
    assert pin_suite(oracle._load())


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, tmp_path):
    src = open(oracle._SRC).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, "mutation target drifted: " + mutant
    path = tmp_path / (mutant + ".c")
    path.write_text(src.replace(old, new))
    lib = oracle.load_library(oracle.compile_source(str(path), str(tmp_path / (mutant + ".so"))))
    assert not pin_suite(lib)
