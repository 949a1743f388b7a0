"""GPU parity of the batched form: many texts of uneven length against several
resident automata in one persistent launch (ac_batch_*).

Expected lists come from the oracle, one text at a time, shifted to the
text's offset in the batch buffer. The batch must also equal per-text plain
scans (ac_scan) of the same texts, and its hipGraph replays the eager launch.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from synth import DNA, PROTEIN, batched_workload, dna_text, protein_text

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def build(patterns, placement=ac.AC_PLACE_LDS_HOT):
    d, o = ac.patterns_csr(patterns)
    return ac.ac_build(d, o, opts=ac._opts(placement=placement))


def small_batch(seed: int, n_texts: int = 48, len_hi_log2: int = 15, n_sets: int = 4,
                set_lo: int = 20, set_hi: int = 600):
    texts, sets, text_set = batched_workload(n_texts=n_texts, n_sets=n_sets, len_lo_log2=0,
                                             len_hi_log2=len_hi_log2, set_lo=set_lo, set_hi=set_hi,
                                             pat_lo=4, pat_hi=24, seed=seed)
    # empty and ragged texts, and one that is mostly a repeated pattern
    rng = np.random.default_rng(seed)
    for n in (0, 1, 15, 16, 17, 127, 129, 0):
        texts.append(dna_text(n, int(rng.integers(1 << 30))) if n else np.zeros(0, np.uint8))
        text_set = np.append(text_set, np.uint32(rng.integers(n_sets)))
    p = np.frombuffer(sets[0][0], dtype=np.uint8)
    texts.append(np.tile(p, 300))
    text_set = np.append(text_set, np.uint32(0))
    return texts, sets, text_set.astype(np.uint32)


def expected(texts, sets, text_set, offs) -> np.ndarray:
    orc = [oracle.OracleAC(s) for s in sets]
    parts = [np.zeros(0, np.uint64)]
    for t, txt in enumerate(texts):
        k = orc[int(text_set[t])].scan(txt)
        parts.append(k + (np.uint64(int(offs[t])) << np.uint64(32)))
    return np.sort(np.concatenate(parts))


class BatchRun:
    """Device buffers of a packed batch plus its plan."""

    def __init__(self, autos, texts, text_set, tune=None, cap=None):
        buf, self.offs, self.lens = ac.pack_texts(texts)
        self.d_text = torch.from_numpy(buf).to("cuda")
        self.batch = ac.ac_batch_create(autos, self.offs, self.lens, text_set, tune=tune)
        self.info = ac.ac_batch_info(self.batch)
        self.cap = cap if cap is not None else max(4096, 2 * len(buf))
        self.out = torch.empty(self.cap, dtype=torch.int64, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int64, device="cuda")

    def scan(self, use_graph=False) -> np.ndarray:
        ac.ac_batch_scan(self.batch, self.d_text, self.out, self.cap, self.count, use_graph)
        torch.cuda.synchronize()
        n = int(self.count.item())
        assert n <= self.cap, (n, self.cap)
        return np.sort(ac.keys_to_numpy(self.out[:n]))


def tune(placement=0, walkers=0, chunk=0, algo=ac.AC_ALGO_AUTO):
    t = ac.ac_batch_tune()
    t.placement, t.walkers, t.chunk, t.algo = placement, walkers, chunk, algo
    return t


@pytest.fixture(scope="module")
def dna_batch():
    texts, sets, text_set = small_batch(seed=11)
    autos = [build(s) for s in sets]
    buf, offs, _ = ac.pack_texts(texts)
    return texts, sets, text_set, autos, expected(texts, sets, text_set, offs)


@pytest.mark.parametrize("placement", [ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_LDS_HOT])
@pytest.mark.parametrize("walkers", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("chunk", [0, 128, 1024])
def test_batch_matches_oracle(dna_batch, placement, walkers, chunk):
    texts, sets, text_set, autos, expect = dna_batch
    note("batch", placement, walkers, chunk, "texts", len(texts))
    r = BatchRun(autos, texts, text_set, tune=tune(placement, walkers, chunk, ac.AC_ALGO_DFA))
    assert r.info["algo"] == ac.AC_ALGO_DFA
    if placement != ac.AC_PLACE_AUTO:
        assert r.info["placement"] == placement
    got = r.scan()
    assert got.size == expect.size and np.array_equal(got, expect)


@pytest.mark.parametrize("chunk", [0, 1, 1008, 3 * 1008, 50 * 1008])
def test_gated_batch_matches_oracle(dna_batch, chunk):
    """The gated plan: tasks of whole 1,008-byte tiles (one tile, three,
    fifty, or the plan's own size), texts of every length class (empty,
    shorter than a window, ragged, a repeated pattern), short patterns."""
    texts, sets, text_set, autos, expect = dna_batch
    note("gated batch", chunk)
    r = BatchRun(autos, texts, text_set, tune=tune(chunk=chunk, algo=ac.AC_ALGO_GATED))
    assert r.info["algo"] == ac.AC_ALGO_GATED and r.info["threads"] == 1024
    assert np.array_equal(r.scan(), expect)
    assert np.array_equal(r.scan(use_graph=True), expect)


def test_gated_batch_reloads_and_long_texts():
    """Nine automata interleaved, texts up to 1 MiB cut into many tasks:
    workgroups cross automaton boundaries and reload their bitmaps."""
    texts, sets, text_set = small_batch(seed=21, n_texts=120, len_hi_log2=20, n_sets=9,
                                        set_lo=5, set_hi=3000)
    autos = [build(s) for s in sets]
    buf, offs, _ = ac.pack_texts(texts)
    expect = expected(texts, sets, text_set, offs)
    for chunk in (0, 4 * 1008):
        r = BatchRun(autos, texts, text_set, tune=tune(chunk=chunk, algo=ac.AC_ALGO_GATED))
        assert r.info["n_tasks"] >= len(sets)
        assert np.array_equal(r.scan(), expect), chunk


def test_gated_batch_sparse_sets_stage_in_lds():
    """Pattern sets whose expected match rate is below 4e-3 per byte: the
    gated batch stages matches in the LDS queue instead of registers. Texts
    carry planted occurrences so that every queue still flushes."""
    texts, sets, text_set = batched_workload(n_texts=60, n_sets=5, len_lo_log2=0, len_hi_log2=18,
                                             set_lo=50, set_hi=2000, pat_lo=14, pat_hi=24, seed=33)
    rng = np.random.default_rng(33)
    for t, txt in enumerate(texts):
        pats = sets[int(text_set[t])]
        for _ in range(min(40, len(txt) // 64)):
            p = np.frombuffer(pats[int(rng.integers(len(pats)))], np.uint8)
            if len(txt) > len(p):
                at = int(rng.integers(0, len(txt) - len(p)))
                txt[at:at + len(p)] = p
    autos = [build(s) for s in sets]
    assert all(ac.ac_info(a)["match_rate"] < 4e-3 for a in autos)
    buf, offs, _ = ac.pack_texts(texts)
    expect = expected(texts, sets, text_set, offs)
    assert expect.size > 500
    r = BatchRun(autos, texts, text_set, tune=tune(chunk=2 * 1008, algo=ac.AC_ALGO_GATED))
    assert r.info["algo"] == ac.AC_ALGO_GATED
    assert np.array_equal(r.scan(), expect)


def test_batch_equals_plain_scans(dna_batch):
    texts, sets, text_set, autos, expect = dna_batch
    r = BatchRun(autos, texts, text_set)
    got = r.scan()
    plain = []
    for t, txt in enumerate(texts):
        if len(txt) == 0:
            continue
        d = torch.from_numpy(np.ascontiguousarray(txt)).to("cuda")
        k = ac.keys_to_numpy(ac.scan_text(autos[int(text_set[t])], d))
        plain.append(k + (np.uint64(int(r.offs[t])) << np.uint64(32)))
    assert np.array_equal(got, np.sort(np.concatenate(plain)))


def test_batch_graph_replays(dna_batch):
    """Captured submission: every replay, with other device work and host
    synchronisation between replays, equals the eager launch."""
    texts, sets, text_set, autos, expect = dna_batch
    r = BatchRun(autos, texts, text_set)
    eager = r.scan(use_graph=False)
    assert np.array_equal(eager, expect)
    other = torch.from_numpy(dna_text(1 << 16, 5)).to("cuda")
    for i in range(4):
        r.out.fill_(-1)
        got = r.scan(use_graph=True)
        assert np.array_equal(got, eager), i
        ac.scan_text(autos[0], other)  # eager work between replays
        torch.cuda.synchronize()
    # new buffers: the graph is captured again for them
    r.out = torch.empty(r.cap, dtype=torch.int64, device="cuda")
    r.count = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert np.array_equal(r.scan(use_graph=True), eager)


def test_batch_mixed_sizes_and_reloads():
    """Many automata, texts interleaved between them, tiny tasks: work-groups
    cross automaton boundaries and reload the LDS image."""
    texts, sets, text_set = small_batch(seed=12, n_texts=200, len_hi_log2=12, n_sets=9,
                                        set_lo=5, set_hi=3000)
    autos = [build(s) for s in sets]
    buf, offs, _ = ac.pack_texts(texts)
    expect = expected(texts, sets, text_set, offs)
    for w in (1, 2, 3, 4):
        r = BatchRun(autos, texts, text_set, tune=tune(ac.AC_PLACE_LDS_HOT, w, 16, ac.AC_ALGO_DFA))
        assert r.info["n_tasks"] >= len(sets)
        assert np.array_equal(r.scan(), expect), w


def test_batch_protein():
    rng = np.random.default_rng(3)
    sets = []
    for i, n in enumerate((40, 400, 4000)):
        t = protein_text(1 << 16, 50 + i)
        sets.append([t[o:o + L].tobytes() for o, L in
                     zip(rng.integers(0, (1 << 16) - 30, n), rng.integers(3, 20, n))])
    texts = [protein_text(int(n), 70 + i) for i, n in enumerate(rng.integers(0, 40000, 30))]
    text_set = rng.integers(0, 3, len(texts)).astype(np.uint32)
    autos = [build(s) for s in sets]
    buf, offs, _ = ac.pack_texts(texts)
    expect = expected(texts, sets, text_set, offs)
    for placement in (ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL):
        r = BatchRun(autos, texts, text_set, tune=tune(placement))
        assert np.array_equal(r.scan(), expect), placement


def test_batch_overflow_reports_true_count(dna_batch):
    texts, sets, text_set, autos, expect = dna_batch
    r = BatchRun(autos, texts, text_set, cap=max(1, expect.size // 3))
    ac.ac_batch_scan(r.batch, r.d_text, r.out, r.cap, r.count)
    torch.cuda.synchronize()
    assert int(r.count.item()) == expect.size
    kept = np.sort(ac.keys_to_numpy(r.out[:r.cap]))
    assert np.isin(kept, expect).all()


def test_batch_empty_and_all_empty():
    a = build([b"ACG", b"T"])
    r = BatchRun([a], [np.zeros(0, np.uint8)] * 5, np.zeros(5, np.uint32))
    assert r.info["n_items"] == 0 and r.scan().size == 0
    r = BatchRun([a], [], np.zeros(0, np.uint32))
    assert r.scan().size == 0


def test_batch_rejects_bad_plans():
    a = build([b"ACG", b"T"])
    p = build([b"ACDEFGHIKLMNPQRSTVWY"[:10]])  # another class scheme
    g = build([b"ACGT" * 3], placement=ac.AC_PLACE_GLOBAL)
    off = np.array([0, 16], np.uint64)
    ln = np.array([10, 10], np.uint64)
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a], np.array([0, 8], np.uint64), ln, np.zeros(2, np.uint32))
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a], off, ln, np.array([0, 1], np.uint32))
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a, p], off, ln, np.array([0, 1], np.uint32))
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a, g], off, ln, np.array([0, 1], np.uint32), tune=tune(ac.AC_PLACE_LDS_HOT))
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a], np.array([(1 << 32) - 16], np.uint64), np.array([32], np.uint64),
                           np.zeros(1, np.uint32))
    # the gated plan needs the class gate in every automaton
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([p], off, ln, np.zeros(2, np.uint32), tune=tune(algo=ac.AC_ALGO_GATED))
    with pytest.raises(ac.AcError):
        ac.ac_batch_create([a], off, ln, np.zeros(2, np.uint32), tune=tune(algo=7))
    # a plan without images falls back to the global table
    b = ac.ac_batch_create([a, g], off, ln, np.array([0, 1], np.uint32))
    assert ac.ac_batch_info(b)["placement"] == ac.AC_PLACE_GLOBAL
    assert ac.ac_batch_info(b)["algo"] == ac.AC_ALGO_DFA
    d = torch.zeros(64, dtype=torch.uint8, device="cuda")
    out = torch.empty(16, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(ac.AcError):
        ac.ac_batch_scan(b, d[1:], out, 16, cnt)


def packed(texts):
    """Each text padded to a multiple of 16 with a byte outside every pattern,
    so that the texts lie back to back with aligned starts."""
    padded = [np.concatenate([t, np.full((-t.size) % 16, ord("N"), np.uint8)]) for t in texts]
    off = np.concatenate([[0], np.cumsum([p.size for p in padded])]).astype(np.uint64)
    buf = np.concatenate(padded) if padded else np.zeros(16, np.uint8)
    return padded, off, buf


def one_shot(fn, autos, buf, off, text_set, cap, with_text=True):
    d = torch.from_numpy(buf).to("cuda")
    d_off = torch.from_numpy(off.astype(np.int64)).to("cuda")
    d_auto = torch.from_numpy(np.asarray(text_set, dtype=np.int32)).to("cuda")
    out = torch.empty(max(1, cap), dtype=torch.int64, device="cuda")
    mt = torch.full((max(1, cap),), -1, dtype=torch.int32, device="cuda") if with_text else None
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    fn(autos, d, d_off, d_auto, out, cap, cnt, d_match_text=mt)
    n = int(cnt.item())
    keys = ac.keys_to_numpy(out[:min(n, cap)])
    texts = mt[:min(n, cap)].cpu().numpy() if with_text else None
    return n, keys, texts


def test_one_shot_scan_batch(dna_batch):
    """ac_scan_batch over texts packed back to back, descriptors on the
    device, equals the oracle text by text; each key's text index is the text
    its end position lies in."""
    texts, sets, text_set, autos, _ = dna_batch
    padded, off, buf = packed(texts)
    expect = expected(padded, sets, text_set, off[:-1])
    cap = max(4096, 2 * buf.size)
    n, keys, mt = one_shot(ac.ac_scan_batch, autos, buf, off, text_set, cap)
    assert n == expect.size
    assert np.array_equal(np.sort(keys), expect)
    pos = (keys >> np.uint64(32)).astype(np.int64)
    t = np.searchsorted(off.astype(np.int64), pos, side="right") - 1
    assert np.array_equal(mt, t.astype(np.int32))


def test_one_shot_rejects_bad_descriptors(dna_batch):
    texts, sets, text_set, autos, _ = dna_batch
    padded, off, buf = packed(texts[:6])
    ts = np.asarray(text_set[:6], dtype=np.int32)
    bad_auto = ts.copy()
    bad_auto[2] = len(autos)
    with pytest.raises(ac.AcError) as e:
        one_shot(ac.ac_scan_batch, autos, buf, off, bad_auto, 1024)
    assert e.value.status == ac.AC_ERR_INVALID
    bad_off = off.copy()
    bad_off[3] = bad_off[3] + 1  # an unaligned start
    with pytest.raises(ac.AcError) as e:
        one_shot(ac.ac_scan_batch, autos, buf, bad_off, ts, 1024)
    assert e.value.status == ac.AC_ERR_INVALID
    # the same call with valid descriptors still works afterwards
    n, keys, _ = one_shot(ac.ac_scan_batch, autos, buf, off, ts, 1 << 16)
    assert np.array_equal(np.sort(keys), expected(padded, sets, ts, off[:-1]))