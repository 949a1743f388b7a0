"""Two-byte lookups from the states outside the LDS image (4-column DNA
machines built with AC_BUILD_PAIR_ROWS): every scan with them equals the
one-byte scan and the oracle,
over image sizes that leave most steps outside the image, dense and sparse
final states, every walker count, short and long chunks, ragged lengths,
bytes outside the alphabet and texts scanned in pieces."""
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


def build(patterns, rows: int):
    """LDS_HOT machine whose image holds `rows` rows (0 = as many as fit)."""
    d, o = ac.patterns_csr(patterns)
    lds = rows * 8 + 256 if rows else 0
    a = ac.ac_build(d, o, opts=ac._opts(placement=ac.AC_PLACE_LDS_HOT, lds_bytes=lds,
                                        flags=ac.AC_BUILD_PAIR_ROWS))
    info = ac.ac_info(a)
    assert info["placement"] == ac.AC_PLACE_LDS_HOT and info["pair_states"] > 0, info
    return a


def to_device(a: np.ndarray):
    t = torch.empty(max(1, len(a)), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)))
    return t[: len(a)]


def keys(auto, d_text, pair: int, walkers=0, block_bytes=0, chunk=0, capacity=None):
    opts = ac._scan_opts(ac.AC_ALGO_DFA, chunk, 0, 0, walkers, block_bytes, pair)
    return np.sort(ac.keys_to_numpy(ac.scan_text(auto, d_text, capacity=capacity, opts=opts)))


def random_patterns(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(DNA, np.uint8)
    return [letters[rng.integers(0, 4, size=int(m))].tobytes() for m in rng.integers(lo, hi + 1, size=n)]


@pytest.fixture(scope="module")
def planted():
    """10,000 patterns of length 20-32 (10% planted) in 2 MiB of DNA."""
    w = plain_workload("dna256m", n=2 << 20)
    return w.patterns, w.text


@pytest.mark.parametrize("rows", [256, 2048, 0])
def test_planted_set_against_one_byte_steps_and_oracle(planted, rows):
    pats, text = planted
    a = build(pats, rows)
    d = to_device(text)
    base = keys(a, d, ac.AC_PAIR_OFF)
    assert base.size > 100
    for walkers, bb in ((1, 128), (1, 64), (2, 128), (2, 64), (3, 0), (4, 0)):
        note("rows", rows, "walkers", walkers, "block", bb)
        got = keys(a, d, ac.AC_PAIR_AUTO, walkers=walkers, block_bytes=bb)
        assert np.array_equal(got, base), (rows, walkers, bb)
    sample = text[:1 << 16]
    want = oracle.OracleAC(pats).scan(sample.tobytes())
    assert np.array_equal(keys(a, to_device(sample), ac.AC_PAIR_AUTO), want)


@pytest.mark.parametrize("seed", [1, 2])
def test_dense_finals_mostly_outside_the_image(seed):
    """Short patterns put final states at odd and even positions of most
    16-byte groups; a 64-row image leaves most steps to the pair rows."""
    pats = random_patterns(400, 3, 12, seed)
    a = build(pats, 64)
    text = dna_text(300_001, 77 + seed)
    want = oracle.OracleAC(pats).scan(text.tobytes())
    assert want.size > 10_000
    d = to_device(text)
    for walkers in (1, 2, 3, 4):
        for chunk in (16, 48, 0):
            got = keys(a, d, ac.AC_PAIR_AUTO, walkers=walkers, chunk=chunk, capacity=want.size + 64)
            assert np.array_equal(got, want), (walkers, chunk)


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 33, 47, 1023, 4097, 100_003])
def test_ragged_lengths(n):
    pats = random_patterns(300, 2, 9, 5)
    a = build(pats, 128)
    text = dna_text(n, 900 + n)
    want = oracle.OracleAC(pats).scan(text.tobytes())
    assert np.array_equal(keys(a, to_device(text), ac.AC_PAIR_AUTO, capacity=want.size + 16), want)


def test_bytes_outside_the_alphabet():
    """Groups holding other bytes take the byte-by-byte path; the rest pair."""
    pats = random_patterns(300, 3, 10, 9)
    a = build(pats, 128)
    text = dna_text(200_000, 31).copy()
    rng = np.random.default_rng(4)
    text[rng.integers(0, text.size, size=300)] = ord("N")
    want = oracle.OracleAC(pats).scan(text.tobytes())
    assert np.array_equal(keys(a, to_device(text), ac.AC_PAIR_AUTO, capacity=want.size + 16), want)


def test_pieces_carry_the_state():
    pats = random_patterns(500, 4, 24, 11)
    a = build(pats, 256)
    text = dna_text(400_000, 12)
    want = oracle.OracleAC(pats).scan(text.tobytes())
    cuts = [1, 17, 4096, 4111, 65_537, 200_000, 399_999]
    out = torch.empty(want.size + 64, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    states = torch.zeros(2, dtype=torch.int32, device="cuda")
    bounds = [0] + cuts + [text.size]
    for i in range(len(bounds) - 1):
        lo, hi = bounds[i], bounds[i + 1]
        s_in = None if i == 0 else states[(i - 1) % 2:(i - 1) % 2 + 1]
        ac.ac_scan_stream(a, to_device(text[lo:hi]), hi - lo, lo, s_in, states[i % 2:i % 2 + 1], out, out.numel(),
                          count, append=i > 0, opts=ac._scan_opts(pair_steps=ac.AC_PAIR_AUTO))
    torch.cuda.synchronize()
    n = int(count.item())
    assert np.array_equal(np.sort(ac.keys_to_numpy(out[:n])), want)


def test_unknown_pair_option_rejected():
    a = build(random_patterns(300, 3, 9, 2), 128)
    d = to_device(dna_text(1000, 1))
    with pytest.raises(ac.AcError):
        keys(a, d, 2)
