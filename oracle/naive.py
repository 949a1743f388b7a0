"""Brute-force matcher -- TEST INFRASTRUCTURE ONLY.

The match set written out as its definition: pattern k (a non-empty byte
string, id = its index) ends at text position e exactly when the |P_k| bytes
ending at e equal P_k. Every (position, pattern) pair is compared, so this is
only for tiny inputs. It shares nothing with ac_oracle.c and pins it.
"""
from __future__ import annotations

import numpy as np


def naive_match(text: bytes, patterns) -> np.ndarray:
    """Sorted uint64 keys (e << 32) | k of every occurrence."""
    text = bytes(text)
    keys = []
    for e in range(len(text)):
        for k, p in enumerate(patterns):
            p = bytes(p)
            if len(p) == 0:
                raise ValueError("empty pattern")
            if len(p) <= e + 1 and text[e - len(p) + 1:e + 1] == p:
                keys.append((e << 32) | k)
    return np.array(sorted(keys), dtype=np.uint64)
