"""Hashed byte classes of every width with the LDS image: 2, 4 and 8
columns, images from a handful of rows (almost every step outside the
image) to as many as fit, every walker count, bytes outside the alphabet,
and texts in pieces, all against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")

# alphabet -> (columns, hashed) the build gives it
ALPHABETS = {b"AB": 2, b"ACG": 4, b"ACGTN": 8, b"abcdefgh": 8}


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def random_patterns(alpha: bytes, n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(alpha, np.uint8)
    return [letters[rng.integers(0, len(letters), size=int(m))].tobytes() for m in rng.integers(lo, hi + 1, size=n)]


def random_text(alpha: bytes, n, seed, foreign=0, plant=()):
    """Uniform letters of `alpha`, `foreign` bytes outside it, and one
    occurrence of each pattern in `plant` at a random place."""
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(alpha, np.uint8)
    t = letters[rng.integers(0, len(letters), size=n)].copy()
    for p in plant:
        at = int(rng.integers(0, n - len(p)))
        t[at:at + len(p)] = np.frombuffer(p, np.uint8)
    if foreign:
        t[rng.integers(0, n, size=foreign)] = ord("#")
    return t


def to_device(a: np.ndarray):
    t = torch.empty(max(1, len(a)), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)))
    return t[: len(a)]


def build(patterns, rows):
    d, o = ac.patterns_csr(patterns)
    lds = rows * 8 * 8 + 256 if rows else 0  # room for `rows` rows of up to 8 columns
    a = ac.ac_build(d, o, opts=ac._opts(placement=ac.AC_PLACE_LDS_HOT, lds_bytes=lds))
    return a, ac.ac_info(a)


@pytest.mark.parametrize("lens", [(3, 14), (12, 24)])  # dense finals, or sparse finals and a fuller image
@pytest.mark.parametrize("rows", [128, 0])
@pytest.mark.parametrize("alpha", list(ALPHABETS))
def test_hashed_image_scans(alpha, rows, lens):
    pats = random_patterns(alpha, 800, lens[0], lens[1], len(alpha))
    a, info = build(pats, rows)
    assert info["class_hashed"] == 1 and info["n_cols"] == ALPHABETS[alpha]
    assert info["placement"] == ac.AC_PLACE_LDS_HOT and info["hot_states"] > 0
    text = random_text(alpha, 250_003, 7 + len(alpha), foreign=40, plant=pats[:200])
    want = oracle.OracleAC(pats).scan(text.tobytes())
    assert want.size >= 150
    d = to_device(text)
    for walkers in (1, 2, 3, 4):
        for chunk in (16, 0):
            note(alpha, rows, walkers, chunk)
            opts = ac._scan_opts(ac.AC_ALGO_DFA, chunk, 0, ac.AC_PLACE_LDS_HOT, walkers)
            got = np.sort(ac.keys_to_numpy(ac.scan_text(a, d, capacity=want.size + 64, opts=opts)))
            assert np.array_equal(got, want), (alpha, rows, walkers, chunk)


@pytest.mark.parametrize("alpha", [b"AB", b"ACGTN"])
def test_hashed_image_pieces(alpha):
    pats = random_patterns(alpha, 500, 2, 20, 3)
    a, _ = build(pats, 64)
    text = random_text(alpha, 200_000, 4)
    want = oracle.OracleAC(pats).scan(text.tobytes())
    out = torch.empty(want.size + 64, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    states = torch.zeros(2, dtype=torch.int32, device="cuda")
    bounds = [0, 1, 33, 4096, 50_001, 150_000, 200_000]
    for i in range(len(bounds) - 1):
        lo, hi = bounds[i], bounds[i + 1]
        s_in = None if i == 0 else states[(i - 1) % 2:(i - 1) % 2 + 1]
        ac.ac_scan_stream(a, to_device(text[lo:hi]), hi - lo, lo, s_in, states[i % 2:i % 2 + 1], out,
                          out.numel(), count, append=i > 0)
    torch.cuda.synchronize()
    n = int(count.item())
    assert np.array_equal(np.sort(ac.keys_to_numpy(out[:n])), want)
