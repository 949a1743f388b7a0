"""Host-side tests of libac.so (no GPU): exported symbols, argument checks,
and the tables ac_build_host produces, walked in Python against the oracle."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from synth import DNA, PROTEIN, plain_workload

ac = pytest.importorskip("paper_1403_1305_amd.ac")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions() -> set[str]:
    src = open(os.path.join(ROOT, "include", "ac.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(ac_[a-z_]+)\s*\(", src))


def test_library_exports_every_declared_function():
    lib = ac.load_library()
    declared = header_functions()
    assert {"ac_build", "ac_scan", "ac_free", "ac_info", "ac_scan_sync", "ac_last_error"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(ac.SIGNATURES), "binding and header disagree"


def build_host(patterns, **kw):
    d, o = ac.patterns_csr(patterns)
    return ac.ac_build_host(d, o, opts=ac._opts(**kw) if kw else None)


def test_invalid_arguments():
    with pytest.raises(ac.AcError) as e:
        build_host([b"A", b""])
    assert e.value.status == ac.AC_ERR_INVALID
    with pytest.raises(ac.AcError) as e:
        ac.ac_build_host(np.zeros(1, np.uint8), np.zeros(1, np.uint64))
    assert e.value.status == ac.AC_ERR_INVALID
    with pytest.raises(ac.AcError) as e:
        ac.ac_build_host(np.frombuffer(b"AB", np.uint8), np.array([0, 2, 1], np.uint64))
    assert e.value.status == ac.AC_ERR_INVALID
    # a scan on a host-only automaton is rejected before any device work
    a = build_host([b"AB"])
    with pytest.raises(ac.AcError) as e:
        ac.ac_scan(a, 0, 0, 0, 0, 1 << 20)
    assert e.value.status == ac.AC_ERR_INVALID
    lib = ac.load_library()
    assert lib.ac_scan(None, None, 0, None, 0, None, None, None) == ac.AC_ERR_INVALID
    assert lib.ac_info(None, None) == ac.AC_ERR_INVALID
    lib.ac_free(None)
    with pytest.raises(ac.AcError):
        build_host([b"AB"], placement=ac.AC_PLACE_LDS_FULL, lds_bytes=270)


class Tables:
    def __init__(self, a):
        self.info = ac.ac_info(a)
        self.C = self.info["n_cols"]
        self.S = self.info["n_states"]
        dfa = ac.ac_get_table(a, ac.AC_TABLE_DFA)
        self.dfa = dfa.reshape(self.S, self.C) if dfa.size else None  # None: goto-only build
        self.go = ac.ac_get_table(a, ac.AC_TABLE_GO).reshape(self.S, self.C)
        self.out_off = ac.ac_get_table(a, ac.AC_TABLE_OUT_OFF)
        self.out_ids = ac.ac_get_table(a, ac.AC_TABLE_OUT_IDS)
        self.own_off = ac.ac_get_table(a, ac.AC_TABLE_OWN_OFF)
        self.own_ids = ac.ac_get_table(a, ac.AC_TABLE_OWN_IDS)
        self.cmap = ac.ac_get_table(a, ac.AC_TABLE_CMAP)
        H = self.info["hot_states"]
        hot = ac.ac_get_table(a, ac.AC_TABLE_HOT_DFA)
        self.hot = hot[: H * self.C].reshape(H, self.C) if hot.size else None
        self.hot_go = ac.ac_get_table(a, ac.AC_TABLE_HOT_GO)[: H * self.C].reshape(H, self.C)

    def dfa_walk(self, text: bytes) -> np.ndarray:
        s, res = 0, []
        for i, b in enumerate(text):
            c = self.cmap[b]
            e = 0 if c == 255 else int(self.dfa[s, c])
            s = e & 0x7FFFFFFF
            if e >> 31:
                res += [(i << 32) | int(k) for k in self.out_ids[self.out_off[s]:self.out_off[s + 1]]]
        return np.array(sorted(res), dtype=np.uint64)

    def go_walks(self, text: bytes) -> np.ndarray:
        res = []
        for p in range(len(text)):
            s = 0
            for j in range(p, len(text)):
                c = self.cmap[text[j]]
                if c == 255:
                    break
                e = int(self.go[s, c])
                if e == 0:
                    break
                s = e & 0x7FFFFFFF
                res += [(j << 32) | int(k) for k in self.own_ids[self.own_off[s]:self.own_off[s + 1]]]
        return np.array(sorted(res), dtype=np.uint64)


def check_invariants(t: Tables, patterns):
    S, C = t.S, t.C
    assert (t.dfa & 0x7FFFFFFF).max() < S and (t.go & 0x7FFFFFFF).max() < S
    accept = np.diff(t.out_off.astype(np.int64)) > 0
    assert np.array_equal((t.dfa >> 31).astype(bool), accept[t.dfa & 0x7FFFFFFF])
    own = np.diff(t.own_off.astype(np.int64)) > 0
    nz = t.go != 0
    assert np.array_equal((t.go[nz] >> 31).astype(bool), own[t.go[nz] & 0x7FFFFFFF])
    assert not accept[0] and (t.go & 0x7FFFFFFF != 0).sum() == S - 1  # a tree: S-1 edges
    assert sorted(t.own_ids.tolist()) == list(range(len(patterns)))
    for s in range(S):  # output sets ascending, own ids inside them
        o = t.out_ids[t.out_off[s]:t.out_off[s + 1]]
        assert np.all(np.diff(o.astype(np.int64)) > 0)
        assert set(t.own_ids[t.own_off[s]:t.own_off[s + 1]]) <= set(o.tolist())
    alphabet = set(b"".join(patterns))
    for b in range(256):
        assert (t.cmap[b] != 255) == (b in alphabet)
        if b in alphabet:
            assert t.cmap[b] < C
    # ids come in ranges: image rows, final states with own patterns, other
    # final states, the rest (the root alone in front when there is no image)
    H = t.info["hot_states"]
    lo = H if H else 1
    A, T = int(accept.sum()), int(own.sum())
    assert np.array_equal(np.nonzero(own)[0], np.arange(lo, lo + T))
    assert np.array_equal(np.nonzero(accept)[0], np.arange(lo, lo + A))
    if H:
        assert np.array_equal(t.hot.astype(np.uint32), t.dfa[:H] & 0x7FFFFFFF)
        assert np.array_equal(t.hot_go.astype(np.uint32), t.go[:H] & 0x7FFFFFFF)
        assert not accept[:H].any()  # final states are never in the image


@pytest.mark.parametrize("placement", [ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_HOT])
@pytest.mark.parametrize("fixture", [([b"AB", b"ABG", b"BEDE", b"EF"], b"xxABEDEFABG"),
                                     ([b"HE", b"HIS", b"SHE", b"HERS"], b"USHERSHISHE")])
def test_worked_examples_tables(fixture, placement):
    pats, text = fixture
    t = Tables(build_host(pats, placement=placement))
    check_invariants(t, pats)
    expect = oracle.oracle_match(text, pats)
    assert np.array_equal(t.dfa_walk(text), expect)
    assert np.array_equal(t.go_walks(text), expect)


@st.composite
def case(draw):
    alpha = draw(st.sampled_from([b"ab", b"ACGT", b"xyz!", bytes(range(0, 256, 7))]))
    letter = st.sampled_from(list(alpha))
    pats = draw(st.lists(st.lists(letter, min_size=1, max_size=9).map(bytes), min_size=1,
                         max_size=20))
    text = bytes(draw(st.lists(st.sampled_from(list(alpha) + [0x00, 0x41]), max_size=200)))
    hot = draw(st.sampled_from([0, 1, 3, 40]))
    return pats, text, hot


@settings(max_examples=400, deadline=None)
@given(case())
def test_tables_walk_like_the_oracle(c):
    pats, text, hot = c
    kw = dict(placement=ac.AC_PLACE_LDS_HOT, hot_states=hot) if hot else {}
    t = Tables(build_host(pats, **kw))
    check_invariants(t, pats)
    expect = oracle.oracle_match(text, pats)
    assert np.array_equal(t.dfa_walk(text), expect)
    assert np.array_equal(t.go_walks(text), expect)


def test_dna_classes_are_hashed():
    t = Tables(build_host([b"ACGT", b"TTGA"]))
    assert t.info["class_hashed"] == 1 and t.C == 4 and t.info["class_shift"] == 1
    assert [t.cmap[b] for b in b"ACGT"] == [0, 1, 3, 2]


def test_protein_classes_are_ranked():
    t = Tables(build_host([PROTEIN]))
    assert t.info["class_hashed"] == 0 and t.C == 20 and t.info["sigma"] == 20
    assert [t.cmap[b] for b in sorted(PROTEIN)] == list(range(20))


def test_small_workload_tables():
    w = plain_workload("dna1m", n=1 << 14)
    a = build_host(w.patterns)
    t = Tables(a)
    check_invariants(t, w.patterns)
    assert t.info["placement"] == ac.AC_PLACE_LDS_FULL  # ~900 states x 4 columns fits LDS
    text = w.text[:3000].tobytes()
    assert np.array_equal(t.dfa_walk(text), oracle.oracle_match(text, w.patterns))
    assert t.info["n_states"] == oracle.OracleAC(w.patterns).n_states


def test_hot_image_for_large_dna_set():
    """A 10,000-pattern DNA set does not fit LDS as a 32-bit table: the build
    plans a 16-bit image of the shallowest non-final states."""
    w = plain_workload("dna256m", n=1 << 16)
    t = Tables(build_host(w.patterns))
    assert t.info["placement"] == ac.AC_PLACE_LDS_HOT
    assert 10_000 < t.info["hot_states"] <= ((160 - 9) * 1024 - 256) // 8
    check_invariants(t, w.patterns)
    text = w.text[:2000].tobytes()
    assert np.array_equal(t.dfa_walk(text), oracle.oracle_match(text, w.patterns))


def test_pair_rows_compose_two_steps():
    """The two-byte rows (built on request) of the states outside the image
    are the DFA applied twice, flagged where the state in between has a
    non-empty output set; machines without four hashed columns or without an
    image get none."""
    w = plain_workload("dna256m", n=1 << 16)
    pats = w.patterns[:3000]
    assert ac.ac_info(build_host(pats, placement=ac.AC_PLACE_LDS_HOT))["pair_states"] == 0  # not asked for
    a = build_host(pats, placement=ac.AC_PLACE_LDS_HOT, lds_bytes=2048 * 8 + 256, flags=ac.AC_BUILD_PAIR_ROWS)
    info = ac.ac_info(a)
    S, H, C = info["n_states"], info["hot_states"], info["n_cols"]
    assert C == 4 and H == 2048 and info["pair_states"] == S - H
    dfa = ac.ac_get_table(a, ac.AC_TABLE_DFA).reshape(S, C).astype(np.int64)
    pair = ac.ac_get_table(a, ac.AC_TABLE_PAIR).reshape(S - H, 16).astype(np.int64)
    final = np.diff(ac.ac_get_table(a, ac.AC_TABLE_OUT_OFF).astype(np.int64)) > 0
    mask = (1 << 31) - 1
    cold = np.arange(H, S)
    for c1 in range(4):
        mid = dfa[cold, c1] & mask
        for c2 in range(4):
            got = pair[:, c1 | c2 << 2]
            assert np.array_equal(got & mask, dfa[mid, c2] & mask)
            assert np.array_equal((got >> 31) & 1, final[mid].astype(np.int64))
    # a final state in between does occur among the rows checked
    assert any(final[dfa[cold, c] & mask].any() for c in range(4))
    flag = ac.AC_BUILD_PAIR_ROWS
    assert ac.ac_info(build_host([b"ACGT", b"GATTACA"], flags=flag))["pair_states"] == 0  # whole table in LDS
    prot = plain_workload("protein1g", n=1 << 12).patterns[:500]
    assert ac.ac_info(build_host(prot, placement=ac.AC_PLACE_LDS_HOT, flags=flag))["pair_states"] == 0


def test_large_protein_set_builds():
    """50,000 protein patterns: more final states than 16-bit ids can hold
    beside an image, so the build must fall back cleanly (no image)."""
    w = plain_workload("protein1g", n=1 << 16)
    t = Tables(build_host(w.patterns))
    info = t.info
    assert info["n_cols"] == 20 and info["n_states"] > 100_000
    accept = np.diff(t.out_off.astype(np.int64)) > 0
    lo = info["hot_states"] if info["hot_states"] else 1
    assert np.array_equal(np.nonzero(accept)[0], np.arange(lo, lo + int(accept.sum())))
    text = w.text[:1500].tobytes()
    assert np.array_equal(t.dfa_walk(text), oracle.oracle_match(text, w.patterns))
    # forcing the hot placement keeps whatever image fits
    t2 = Tables(build_host(w.patterns, placement=ac.AC_PLACE_LDS_HOT))
    assert np.array_equal(t2.dfa_walk(text), oracle.oracle_match(text, w.patterns))


def test_small_machine_image_is_complete():
    """A machine whose non-final states all fit the LDS image keeps that
    image (every non-final state hot) when LDS_HOT is asked for."""
    for pats in ([b"AB", b"ABG", b"BEDE", b"EF"], [b"ACG", b"T"],
                 [bytes(p) for p in plain_workload("dna1m", n=1 << 12).patterns[:7]]):
        t = Tables(build_host(pats, placement=ac.AC_PLACE_LDS_HOT))
        accept = np.diff(t.out_off.astype(np.int64)) > 0
        assert t.info["hot_states"] == int((~accept).sum()), pats
        assert t.info["placement"] == ac.AC_PLACE_LDS_HOT
        check_invariants(t, pats)


@settings(max_examples=200, deadline=None)
@given(case())
def test_goto_only_build_walks_like_the_oracle(c):
    """AC_BUILD_GOTO_ONLY keeps the goto function and the patterns ending at
    each state (no failure function, no DFA): per-start-position walks over
    it find exactly the oracle's matches, over the same trie as the full build."""
    pats, text, hot = c
    kw = dict(placement=ac.AC_PLACE_LDS_HOT, hot_states=hot) if hot else {}
    t = Tables(build_host(pats, flags=ac.AC_BUILD_GOTO_ONLY, **kw))
    assert t.dfa is None and t.info["goto_only"] == 1 and t.info["table_bytes"] == 0
    assert t.info["n_states"] == ac.ac_info(build_host(pats))["n_states"]
    assert np.array_equal(t.out_off, t.own_off) and np.array_equal(t.out_ids, t.own_ids)
    assert np.array_equal(t.go_walks(text), oracle.oracle_match(text, pats))
    H = t.info["hot_states"]
    if H:
        assert np.array_equal(t.hot_go.astype(np.uint32), t.go[:H] & 0x7FFFFFFF)
        own = np.diff(t.own_off.astype(np.int64)) > 0
        assert not own[:H].any()


def test_goto_only_rejects_dfa_uses():
    with pytest.raises(ac.AcError):
        build_host([b"AB"], flags=8)  # unknown flag


@pytest.mark.parametrize("flags", [0, ac.AC_BUILD_GOTO_ONLY])
def test_threaded_build_is_identical(flags):
    """The construction runs level by level on several threads; every table
    must come out bit-identical to a one-thread build."""
    w = plain_workload("dna256m", n=1 << 16)
    pats = w.patterns[:6000]
    one = build_host(pats, threads=1, flags=flags)
    many = build_host(pats, threads=7, flags=flags)
    for t in (ac.AC_TABLE_DFA, ac.AC_TABLE_GO, ac.AC_TABLE_OUT_OFF, ac.AC_TABLE_OUT_IDS, ac.AC_TABLE_OWN_OFF,
              ac.AC_TABLE_OWN_IDS, ac.AC_TABLE_HOT_DFA, ac.AC_TABLE_HOT_GO, ac.AC_TABLE_CMAP):
        assert np.array_equal(ac.ac_get_table(one, t), ac.ac_get_table(many, t)), t


# ---------------------------------------------------------------- start-position gate

def class_string(p: bytes, shift: int) -> np.ndarray:
    return (np.frombuffer(p, np.uint8) >> shift) & 3


def gate_patterns(seed: int) -> list[bytes]:
    """DNA patterns of lengths 1-16, with duplicates and nested prefixes, so
    that short patterns (all extensions of their class string) take part."""
    rng = np.random.default_rng(seed)
    a = np.frombuffer(DNA, np.uint8)
    pats = [a[rng.integers(0, 4, int(L))].tobytes() for L in rng.integers(1, 17, 120)]
    pats += [pats[3], pats[7][:2], pats[11] + b"ACGT", b"ACGTACGTAC", b"ACGTACGTA"]
    return pats


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gate_tables_match_their_definition(seed):
    """Bit x of the gate is set exactly when some pattern can begin with a
    10-byte window of classes x: its first 10 classes are x's, or it is
    shorter and x begins with its classes (brute force over the patterns).
    The node entry is the deepest goto state of x's class string, and its
    path list holds the patterns that are prefixes of that string."""
    pats = gate_patterns(seed)
    a = build_host(pats)
    info = ac.ac_info(a)
    assert info["has_gate"] == 1 and info["class_hashed"] == 1 and info["n_cols"] == 4
    sh = info["class_shift"]
    Q = 10
    expect = np.zeros(1 << (2 * Q), bool)
    cls = [class_string(p, sh) for p in pats]
    for c in cls:
        L = min(len(c), Q)
        base = int(sum(int(c[i]) << (2 * i) for i in range(L)))
        if L == Q:
            expect[base] = True
        else:
            expect[base + (np.arange(1 << (2 * (Q - L)), dtype=np.int64) << (2 * L))] = True
    bits = ac.ac_get_table(a, ac.AC_TABLE_GATE_BITS)
    got = np.unpackbits(bits.view(np.uint8), bitorder="little").astype(bool)
    assert np.array_equal(got, expect)
    assert info["gate_pass"] == pytest.approx(expect.mean())

    node = ac.ac_get_table(a, ac.AC_TABLE_GATE_NODE)
    path_off = ac.ac_get_table(a, ac.AC_TABLE_PATH_OFF)
    path_ids = ac.ac_get_table(a, ac.AC_TABLE_PATH_IDS)
    path_one = ac.ac_get_table(a, ac.AC_TABLE_PATH_ONE)
    go = ac.ac_get_table(a, ac.AC_TABLE_GO).reshape(-1, 4)
    rng = np.random.default_rng(seed + 100)
    codes = np.concatenate([rng.integers(0, 1 << 20, 600), np.nonzero(expect)[0][::61]])
    for x in codes.tolist():
        w = [(x >> (2 * i)) & 3 for i in range(Q)]
        # deepest prefix of w shared with some pattern, and the patterns that are prefixes of w
        depth = max(next((i for i in range(min(len(c), Q)) if c[i] != w[i]), min(len(c), Q)) for c in cls)
        prefix_ids = sorted(k for k, c in enumerate(cls) if len(c) <= depth and list(c) == w[:len(c)])
        e = int(node[x])
        assert (e >> 26) & 31 == depth, x
        assert bool(e >> 31) == bool(prefix_ids), x
        s = 0
        for i in range(depth):  # the entry's state is that prefix's goto state
            s = int(go[s, w[i]]) & 0x7FFFFFFF
        assert e & ((1 << 26) - 1) == s, x
        assert path_ids[path_off[s]:path_off[s + 1]].tolist() == prefix_ids, x
        # the single-pattern shortcut: that pattern and its length, else none
        one = int(path_one[s])
        if len(prefix_ids) == 1:
            assert one == prefix_ids[0] | len(pats[prefix_ids[0]]) << 28, x
        else:
            assert one == 0xFFFFFFFF, x


@pytest.mark.parametrize("seed", [1, 4])
def test_second_gate_level_passes_every_pattern_start(seed):
    """The second level may pass strings no pattern begins with (it is a
    hashed bitmap), but never stops one that some pattern does: the 12 classes
    a pattern begins with, or any extension of a shorter pattern."""
    rng = np.random.default_rng(seed)
    a8 = np.frombuffer(DNA, np.uint8)
    pats = [a8[rng.integers(0, 4, int(L))].tobytes() for L in rng.integers(9, 30, 400)]
    a = build_host(pats)
    sh = ac.ac_info(a)["class_shift"]
    bits = np.unpackbits(ac.ac_get_table(a, ac.AC_TABLE_GATE2_BITS).view(np.uint8), bitorder="little").astype(bool)
    assert bits.size == 1 << 16 and 0.0 < bits.mean() < 0.2

    def h(y):
        return ((y * 0x9E3779B1) & 0xFFFFFFFF) >> 16

    def h2(y):
        return ((y * 0x85EBCA77) & 0xFFFFFFFF) >> 16

    for p in pats:
        c = class_string(p, sh)
        L = min(len(c), 12)
        base = sum(int(c[i]) << (2 * i) for i in range(L))
        for e in range(1 << (2 * (12 - L))):
            y = base | (e << (2 * L))
            assert bits[h(y)] and bits[h2(y)], (p, e)
    # and strings no pattern begins with mostly fail: both bits set by chance
    rng2 = np.random.default_rng(seed + 50)
    ys = rng2.integers(0, 1 << 24, 20000)
    chance = np.mean([bits[h(int(y))] and bits[h2(int(y))] for y in ys])
    assert chance < bits.mean() ** 2 * 1.5 + 0.01
    # three 3-byte patterns extend to 3 x 4^9 strings, more than 8 per bit: the level passes all
    everything = build_host([b"ACG", b"TTA", b"GGC"] + pats[:5])
    assert ac.ac_get_table(everything, ac.AC_TABLE_GATE2_BITS).min() == 0xFFFFFFFF


def test_gate_only_where_it_applies():
    assert ac.ac_info(build_host([b"ACGTACGTACGT"]))["has_gate"] == 1
    assert ac.ac_info(build_host([b"ACGTACGTACGT"], flags=ac.AC_BUILD_NO_GATE))["has_gate"] == 0
    assert ac.ac_info(build_host([b"ACGTACGTACGT"], flags=ac.AC_BUILD_GOTO_ONLY))["has_gate"] == 1
    # other alphabets: the hashed gate, when every pattern has 6 bytes or more
    prot = ac.ac_info(build_host([PROTEIN[:8], PROTEIN[5:]]))
    assert prot["has_gate"] == 2 and prot["gate_pass"] < 0.01
    short = ac.ac_info(build_host([PROTEIN[:5], PROTEIN[5:]]))
    assert short["has_gate"] == 0 and short["gate_pass"] == 1.0
    assert ac.ac_info(build_host([PROTEIN[:8]], flags=ac.AC_BUILD_NO_GATE))["has_gate"] == 0
    assert ac.ac_info(build_host([PROTEIN[:8]], flags=ac.AC_BUILD_GOTO_ONLY))["has_gate"] == 2
    # a 3-letter alphabet in a 2-bit field: the fourth class has no letter
    three = ac.ac_info(build_host([b"ACGACG", b"GGA"]))
    assert three["n_cols"] == 4 and three["has_gate"] == 1
    # the headline pattern set passes about 1% of windows
    w = plain_workload("dna256m", n=1 << 20)
    info = ac.ac_info(build_host(w.patterns))
    assert info["has_gate"] == 1 and 0.005 < info["gate_pass"] < 0.02


@pytest.mark.parametrize("kind", ["class", "hashed", "none"])
def test_own_one_names_the_single_pattern_of_a_state(kind):
    """own_one[s] is the id of the one pattern whose bytes lead from the root
    to s, and 0xffffffff where none or several do (duplicates), computed here
    by walking each pattern on the goto function; without a gate the table is
    empty."""
    rng = np.random.default_rng(9)
    if kind == "class":
        pats = gate_patterns(5)
    else:
        a20 = np.frombuffer(PROTEIN, np.uint8)
        pats = [a20[rng.integers(0, 20, int(L))].tobytes() for L in rng.integers(6, 14, 150)]
        pats += [pats[4], pats[9] + b"AC"]
    a = build_host(pats, flags=ac.AC_BUILD_NO_GATE) if kind == "none" else build_host(pats)
    info = ac.ac_info(a)
    one = ac.ac_get_table(a, ac.AC_TABLE_OWN_ONE)
    if kind == "none":
        assert info["has_gate"] == 0 and ac.ac_get_table(a, ac.AC_TABLE_OWN_ONE).size <= 1
        return
    assert info["has_gate"] == (1 if kind == "class" else 2)
    go = ac.ac_get_table(a, ac.AC_TABLE_GO).reshape(-1, info["n_cols"])
    cmap = ac.ac_get_table(a, ac.AC_TABLE_CMAP)
    ends: dict[int, list[int]] = {}
    for k, p in enumerate(pats):
        s = 0
        for b in p:
            s = int(go[s, cmap[b]]) & 0x7FFFFFFF
        ends.setdefault(s, []).append(k)
    assert one.size == info["n_states"]
    expect = np.full(info["n_states"], 0xFFFFFFFF, np.uint32)
    for s, ids in ends.items():
        if len(ids) == 1:
            expect[s] = ids[0]
    assert np.array_equal(one, expect)
    assert any(len(ids) > 1 for ids in ends.values())  # the duplicates took the list path


def qgate_window(b: bytes) -> tuple[int, int]:
    """X and Y of the hashed gate's window: bytes 0..2 and 3..5, little endian."""
    return b[0] | b[1] << 8 | b[2] << 16, b[3] | b[4] << 8 | b[5] << 16


@pytest.mark.parametrize("seed", [1, 2])
def test_hashed_gate_tables_match_their_definition(seed):
    """For every pattern's first 6 bytes (X, Y): both bits of the blocked
    Bloom filter are set, and one of the window's two table slots holds an
    entry with the window, the goto state its 6 bytes lead to from the root
    and whether patterns end there. Every entry is some pattern's window, and
    random windows pass the filter about as often as gate_pass says."""
    w = plain_workload("protein1g", n=1 << 16)
    rng = np.random.default_rng(seed)
    pats = [w.patterns[int(k)] for k in rng.choice(len(w.patterns), 3000, replace=False)]
    pats += [pats[0][:6], bytes([0, 255, 7, 128, 1, 2, 3])]  # a 6-byte pattern; bytes outside the alphabet
    a = build_host(pats)
    info = ac.ac_info(a)
    assert info["has_gate"] == 2 and info["n_cols"] > 4
    t = Tables(a)
    bits = ac.ac_get_table(a, ac.AC_TABLE_QGATE_BITS)
    tab = ac.ac_get_table(a, ac.AC_TABLE_QGATE_TAB).reshape(-1, 4)
    assert bits.size == 1 << 15 and tab.shape[0] & (tab.shape[0] - 1) == 0
    slots = tab.shape[0]
    log2 = slots.bit_length() - 1
    M = 0xFFFFFFFF

    def h(x, y):
        return (x * 0x9E3779 + y * 0x85EBCB) & M

    windows = {}
    for p in pats:
        x, y = qgate_window(p[:6])
        s = 0
        for b in p[:6]:
            s = int(t.go[s, t.cmap[b]]) & 0x7FFFFFFF
        windows[(x, y)] = s
        hh = h(x, y)
        word = int(bits[hh >> 17])
        assert (word >> ((hh >> 12) & 31)) & 1 and (word >> (hh & 31)) & 1, p
        sa = (((x * 0xC2B2AF) & M) ^ ((y * 0x27D4EB) & M)) >> (32 - log2)
        sb = (((x * 0x165667) & M) ^ ((y * 0xD3A2E5) & M)) >> (32 - log2)
        key = [x | (y & 255) << 24, (y >> 8) | 1 << 31]
        e = [tab[c] for c in (sa, sb) if [int(tab[c][0]), int(tab[c][1]) & ~(1 << 30)] == key]
        assert len(e) == 1 or (sa == sb and len(e) == 2), p
        e = e[0]
        assert int(e[2]) == s and (int(e[1]) >> 30) & 1 == int(t.own_off[s + 1] > t.own_off[s]), p
        kids = sum(1 << c for c in range(t.C) if t.go[s, c]) if t.C <= 32 else 0xFFFFFFFF
        assert int(e[3]) == kids, p
    used = tab[(tab[:, 1] >> 31) == 1]
    assert len(used) == len(windows) and 5 * len(windows) <= 2 * slots
    assert not tab[(tab[:, 1] >> 31) == 0].any()
    for e in used:
        assert int(e[1]) & 0x3FFF0000 == 0
        key = (int(e[0]) & 0xFFFFFF, int(e[0]) >> 24 | (int(e[1]) & 0xFFFF) << 8)
        assert windows[key] == int(e[2])
    # random windows with the patterns' byte frequencies: pass rate near gate_pass
    allb = np.frombuffer(b"".join(pats), np.uint8)
    sample = rng.choice(allb, size=(20000, 6))
    x = sample[:, 0].astype(np.int64) | sample[:, 1].astype(np.int64) << 8 | sample[:, 2].astype(np.int64) << 16
    y = sample[:, 3].astype(np.int64) | sample[:, 4].astype(np.int64) << 8 | sample[:, 5].astype(np.int64) << 16
    hh = (x * 0x9E3779 + y * 0x85EBCB) & M
    word = bits[hh >> 17].astype(np.int64)
    passed = ((word >> ((hh >> 12) & 31)) & (word >> (hh & 31)) & 1).mean()
    assert abs(passed - info["gate_pass"]) < 0.01 + 0.3 * info["gate_pass"], (passed, info["gate_pass"])


def test_hashed_gate_for_the_protein_set():
    """The 50,000-pattern protein set gets the hashed gate, expected to pass
    a few percent of start positions (below AC_ALGO_AUTO's 1 in 20)."""
    w = plain_workload("protein1g", n=1 << 16)
    info = ac.ac_info(build_host(w.patterns))
    assert info["has_gate"] == 2 and 0.02 < info["gate_pass"] < 0.05


@pytest.mark.parametrize("kind", ["dna", "protein"])
def test_match_rate_is_the_expected_matches_per_byte(kind):
    """ac_info_t.match_rate: for text drawn byte by byte with the patterns' own
    byte frequencies, the expected number of occurrences starting at a
    position is the sum over the patterns of the product of their bytes'
    frequencies (linearity of expectation), computed here from the pattern
    list; an automaton without a gate reports 0."""
    rng = np.random.default_rng(21)
    alphabet = np.frombuffer(DNA if kind == "dna" else PROTEIN, np.uint8)
    probs = None if kind == "dna" else np.linspace(1.0, 3.0, len(alphabet)) / np.linspace(1.0, 3.0, len(alphabet)).sum()
    pats = [rng.choice(alphabet, size=int(L), p=probs).tobytes() for L in rng.integers(6, 14, 300)]
    info = ac.ac_info(build_host(pats))
    assert info["has_gate"] == (1 if kind == "dna" else 2)
    allb = np.frombuffer(b"".join(pats), np.uint8)
    f = np.bincount(allb, minlength=256) / len(allb)
    expect = sum(float(np.prod(f[np.frombuffer(p, np.uint8)])) for p in pats)
    assert info["match_rate"] == pytest.approx(expect, rel=1e-9)
    assert ac.ac_info(build_host(pats, flags=ac.AC_BUILD_NO_GATE))["match_rate"] == 0.0
