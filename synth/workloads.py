"""Seeded synthetic workloads: texts and pattern sets.

This module only draws random bytes. It holds none of the string-matching
arithmetic, so both the CPU oracle's tests and the GPU library's tests and
benchmark can use it without sharing any matching code.

The paper (Sec. V) evaluates on bio-computing pattern sets and input strings
that it does not name or publish. The workloads below stand in for them:
DNA-shaped text (i.i.d. uniform over ACGT) and protein-shaped text (20 amino
acid letters with a skewed, rank-power frequency law), with pattern sets
whose patterns are either copied from the text at random offsets ("planted")
or drawn from the text's letter distribution ("random").

Generator: ``numpy.random.default_rng`` (PCG64). Text seed ``1000 + cfg`` and
pattern seed ``2000 + cfg``, where ``cfg`` is the 1-based workload number.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DNA = b"ACGT"
# Amino-acid alphabet; the r-th letter (1-based) gets probability ~ r**-0.8.
PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"
PROTEIN_EXPONENT = 0.8

# Protein text is drawn through a 2**16-entry inverse-CDF table indexed by a
# uniform uint16, so each letter's probability is its exact value rounded to a
# multiple of 2**-16.
_LUT_BITS = 16
_BLOCK = 1 << 24  # bytes drawn per generator call (fixed so streams are reproducible)


def protein_probs() -> np.ndarray:
    r = np.arange(1, len(PROTEIN) + 1, dtype=np.float64)
    w = r ** (-PROTEIN_EXPONENT)
    return w / w.sum()


def _protein_lut() -> np.ndarray:
    """uint16 -> letter table realising protein_probs() at 2**-16 resolution."""
    p = protein_probs()
    size = 1 << _LUT_BITS
    counts = np.floor(p * size).astype(np.int64)
    # hand the rounding remainder to the most frequent letters, one each
    rem = size - counts.sum()
    counts[np.argsort(-(p * size - counts))[:rem]] += 1
    assert counts.sum() == size and (counts > 0).all()
    return np.repeat(np.frombuffer(PROTEIN, dtype=np.uint8), counts)


def dna_text(n: int, seed: int) -> np.ndarray:
    """n bytes i.i.d. uniform over ACGT."""
    rng = np.random.default_rng(seed)
    lut = np.frombuffer(DNA, dtype=np.uint8)
    out = np.empty(n, dtype=np.uint8)
    for lo in range(0, n, _BLOCK):
        hi = min(n, lo + _BLOCK)
        out[lo:hi] = lut[rng.integers(0, 4, size=hi - lo, dtype=np.uint8)]
    return out


def protein_text(n: int, seed: int) -> np.ndarray:
    """n bytes over the 20-letter alphabet with rank-power letter frequencies."""
    rng = np.random.default_rng(seed)
    lut = _protein_lut()
    out = np.empty(n, dtype=np.uint8)
    for lo in range(0, n, _BLOCK):
        hi = min(n, lo + _BLOCK)
        out[lo:hi] = lut[rng.integers(0, 1 << _LUT_BITS, size=hi - lo, dtype=np.uint16)]
    return out


def _letters(rng: np.random.Generator, alphabet: bytes, count: int) -> np.ndarray:
    if alphabet == DNA:
        return np.frombuffer(DNA, dtype=np.uint8)[rng.integers(0, 4, size=count, dtype=np.uint8)]
    if alphabet == PROTEIN:
        return _protein_lut()[rng.integers(0, 1 << _LUT_BITS, size=count, dtype=np.uint16)]
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return a[rng.integers(0, len(a), size=count)]


def pattern_set(text: np.ndarray, n: int, lo: int, hi: int, planted_frac: float,
                alphabet: bytes, seed: int) -> tuple[list[bytes], np.ndarray]:
    """n patterns with lengths uniform in [lo, hi].

    The first round(planted_frac * n) ids of a seeded permutation are planted:
    copied from ``text`` at an offset uniform in [0, len(text) - length].
    The others are i.i.d. letters of ``alphabet`` (with the text's letter law).
    Returns (patterns, offsets) where offsets[k] is the planted offset or -1.
    """
    rng = np.random.default_rng(seed)
    lengths = rng.integers(lo, hi + 1, size=n)
    order = rng.permutation(n)
    n_planted = int(round(planted_frac * n))
    planted = np.zeros(n, dtype=bool)
    planted[order[:n_planted]] = True
    offsets = np.full(n, -1, dtype=np.int64)
    N = len(text)
    for k in np.nonzero(planted)[0]:
        offsets[k] = rng.integers(0, N - lengths[k] + 1)
    rand_ids = np.nonzero(~planted)[0]
    pool = _letters(rng, alphabet, int(lengths[rand_ids].sum()))
    pats: list[bytes] = [b""] * n
    pos = 0
    for k in rand_ids:
        ln = int(lengths[k])
        pats[k] = pool[pos:pos + ln].tobytes()
        pos += ln
    for k in np.nonzero(planted)[0]:
        o = int(offsets[k])
        pats[k] = text[o:o + int(lengths[k])].tobytes()
    return pats, offsets


def patterns_to_csr(patterns: list[bytes]) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated bytes (uint8) and offsets (uint64, len n+1)."""
    off = np.zeros(len(patterns) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(p) for p in patterns], dtype=np.uint64)
    data = np.frombuffer(b"".join(patterns), dtype=np.uint8).copy()
    if data.size == 0:
        data = np.zeros(1, dtype=np.uint8)
    return data, off


@dataclass
class PlainWorkload:
    name: str
    cfg: int
    text: np.ndarray
    patterns: list[bytes]
    planted_offsets: np.ndarray
    alphabet: bytes
    meta: dict = field(default_factory=dict)


# Plain single-text scans (workloads 1-3).
PLAIN = {
    "dna1m":     dict(cfg=1, n=1 << 20, alphabet=DNA, count=100, lo=8, hi=16, planted=0.5),
    "dna256m":   dict(cfg=2, n=1 << 28, alphabet=DNA, count=10_000, lo=20, hi=32, planted=0.1),
    "protein1g": dict(cfg=3, n=1 << 30, alphabet=PROTEIN, count=50_000, lo=6, hi=20, planted=0.2),
}


def plain_workload(name: str, n: int | None = None, planted: float | None = None) -> PlainWorkload:
    """Workload ``name`` from PLAIN; ``n`` / ``planted`` override the text size
    and planted fraction (used for smaller parity cases and the E1 check)."""
    spec = dict(PLAIN[name])
    if n is not None:
        spec["n"] = n
    if planted is not None:
        spec["planted"] = planted
    cfg = spec["cfg"]
    gen = dna_text if spec["alphabet"] == DNA else protein_text
    text = gen(spec["n"], 1000 + cfg)
    pats, offs = pattern_set(text, spec["count"], spec["lo"], spec["hi"], spec["planted"],
                             spec["alphabet"], 2000 + cfg)
    return PlainWorkload(name, cfg, text, pats, offs, spec["alphabet"], spec)


# Batched workload (4): many texts of uneven length against several pattern sets.
def batched_workload(n_texts: int = 4096, n_sets: int = 16, len_lo_log2: int = 10,
                     len_hi_log2: int = 22, set_lo: int = 100, set_hi: int = 20_000,
                     pat_lo: int = 8, pat_hi: int = 32, seed: int = 4):
    """Returns (texts: list[np.ndarray], sets: list[list[bytes]], text_set: np.ndarray).

    Text lengths are log-uniform in [2**len_lo_log2, 2**len_hi_log2]; set sizes
    log-uniform in [set_lo, set_hi]; nothing is planted; every text names one
    set, uniformly at random.
    """
    rng = np.random.default_rng(1000 + seed)
    u = rng.random(n_texts)
    lens = np.floor(2.0 ** (len_lo_log2 + (len_hi_log2 - len_lo_log2) * u)).astype(np.int64)
    texts = [np.frombuffer(DNA, dtype=np.uint8)[rng.integers(0, 4, size=int(L), dtype=np.uint8)]
             for L in lens]
    text_set = rng.integers(0, n_sets, size=n_texts).astype(np.uint32)
    prng = np.random.default_rng(2000 + seed)
    sizes = np.floor(np.exp(np.log(set_lo) + (np.log(set_hi) - np.log(set_lo)) * prng.random(n_sets)))
    sets = []
    for sz in sizes.astype(np.int64):
        lengths = prng.integers(pat_lo, pat_hi + 1, size=int(sz))
        pool = _letters(prng, DNA, int(lengths.sum()))
        ends = np.cumsum(lengths)
        sets.append([pool[e - l:e].tobytes() for e, l in zip(ends, lengths)])
    return texts, sets, text_set


@dataclass
class ServedWorkload:
    """Requests for the served form. Request i scans bytes
    [offset[i], offset[i] + length[i]) of the text of its alphabet
    (``texts[alpha[i]]``, 0 = DNA, 1 = protein) with automaton ``automaton[i]``;
    sets[j] is automaton j's pattern set and set_alpha[j] its alphabet."""
    texts: list[np.ndarray]
    sets: list[list[bytes]]
    set_alpha: np.ndarray
    alpha: np.ndarray
    automaton: np.ndarray
    offset: np.ndarray
    length: np.ndarray


def served_workload(n_requests: int = 512, text_bytes: int = 1 << 26, len_lo_log2: int = 10,
                    len_hi_log2: int = 26, n_sets: int = 8, set_lo: int = 1000, set_hi: int = 50_000,
                    seed: int = 5) -> ServedWorkload:
    """Request lengths log-uniform in [2**len_lo_log2, 2**len_hi_log2], half DNA
    and half protein-shaped; ``n_sets`` pattern sets with sizes log-spaced in
    [set_lo, set_hi], alternately DNA (lengths 8-32, uniform letters) and
    protein (lengths 6-20, the skewed letter law); each request names a set of
    its own alphabet uniformly at random. Request texts are windows, at
    16-byte aligned random offsets, of one text per alphabet of ``text_bytes``
    bytes (at least the longest request)."""
    rng = np.random.default_rng(3000 + seed)
    texts = [dna_text(text_bytes, 3100 + seed), protein_text(text_bytes, 3200 + seed)]
    sizes = np.round(np.geomspace(set_lo, set_hi, n_sets)).astype(np.int64)
    set_alpha = np.arange(n_sets) % 2
    sets = []
    for j, sz in enumerate(sizes):
        alphabet, lo, hi = (DNA, 8, 32) if set_alpha[j] == 0 else (PROTEIN, 6, 20)
        lengths = rng.integers(lo, hi + 1, size=int(sz))
        pool = _letters(rng, alphabet, int(lengths.sum()))
        ends = np.cumsum(lengths)
        sets.append([pool[e - L:e].tobytes() for e, L in zip(ends, lengths)])
    u = rng.random(n_requests)
    length = np.floor(2.0 ** (len_lo_log2 + (len_hi_log2 - len_lo_log2) * u)).astype(np.int64)
    length = np.minimum(length, text_bytes)
    alpha = rng.integers(0, 2, size=n_requests)
    automaton = np.empty(n_requests, dtype=np.int64)
    for i in range(n_requests):
        own = np.nonzero(set_alpha == alpha[i])[0]
        automaton[i] = own[rng.integers(0, len(own))]
    offset = (rng.integers(0, text_bytes - length + 1) // 16) * 16
    return ServedWorkload(texts, sets, set_alpha, alpha, automaton, offset.astype(np.int64), length)


def random_pattern_csr(n: int, lo: int, hi: int, alphabet: bytes, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """n random patterns with lengths uniform in [lo, hi], i.i.d. letters of
    ``alphabet`` (its letter law), as concatenated bytes and n + 1 offsets:
    the large pattern sets of the build-time measurements."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(lo, hi + 1, size=n)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    return _letters(rng, alphabet, int(off[-1])), off
