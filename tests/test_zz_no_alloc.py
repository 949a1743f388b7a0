"""ac_scan_batch_noalloc (the entry point for callers that cannot allocate
device memory) against ac_scan_batch: on two calls in a row, the second with a
smaller batch, its keys, per-key text indices and count equal those of the
allocating form bit for bit (the second call also shows that what the first
left in the library's scratch array does not leak into it)."""
from __future__ import annotations

import numpy as np
import pytest

from synth import batched_workload, protein_text

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def packed(texts):
    padded = [np.concatenate([t, np.full((-t.size) % 16, ord("N"), np.uint8)]) for t in texts]
    off = np.concatenate([[0], np.cumsum([p.size for p in padded])]).astype(np.int64)
    buf = np.concatenate(padded) if padded else np.zeros(16, np.uint8)
    return off, buf


def run(fn, autos, off, buf, text_set, cap):
    d = torch.from_numpy(buf).to("cuda")
    d_off = torch.from_numpy(off).to("cuda")
    d_auto = torch.from_numpy(np.asarray(text_set, dtype=np.int32)).to("cuda")
    out = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    mt = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")  # the call must zero it
    fn(autos, d, d_off, d_auto, out, cap, cnt, d_match_text=mt)
    n = int(cnt.item())
    keys = ac.keys_to_numpy(out[:min(n, cap)])
    order = np.argsort(keys, kind="stable")
    return n, keys[order], mt[:min(n, cap)].cpu().numpy()[order]


@pytest.mark.parametrize("placement", [ac.AC_PLACE_LDS_HOT, ac.AC_PLACE_GLOBAL])
def test_noalloc_equals_scan_batch(placement):
    texts, sets, text_set = batched_workload(n_texts=300, n_sets=5, len_lo_log2=0, len_hi_log2=16,
                                             set_lo=30, set_hi=3000, pat_lo=6, pat_hi=20, seed=11)
    autos = []
    for s in sets:
        d, o = ac.patterns_csr(s)
        autos.append(ac.ac_build(d, o, opts=ac._opts(placement=ac.AC_PLACE_LDS_HOT)))
    tune = ac.ac_batch_tune(placement, 0, 0, 0)
    # the first call: the whole batch; the second: a smaller one (fewer texts,
    # fewer automata named, fewer items)
    for k, (n_texts, cap) in enumerate([(300, 1 << 20), (37, 1 << 16)]):
        off, buf = packed(texts[:n_texts])
        ts = text_set[:n_texts]
        a = run(lambda *x, **y: ac.ac_scan_batch(*x, tune=tune, **y), autos, off, buf, ts, cap)
        b = run(lambda *x, **y: ac.ac_scan_batch_noalloc(*x, tune=tune, **y), autos, off, buf, ts, cap)
        assert a[0] == b[0] and a[0] > 0, (k, a[0], b[0])
        assert np.array_equal(a[1], b[1]), k
        assert np.array_equal(a[2], b[2]), k


def test_noalloc_limits_and_errors():
    d, o = ac.patterns_csr([b"ACGTAC", b"GGA"])
    autos = [ac.ac_build(d, o)]
    big = np.zeros(65_537, dtype=np.int32)
    off = np.zeros(65_538, dtype=np.int64)
    with pytest.raises(ac.AcError) as e:
        run(ac.ac_scan_batch_noalloc, autos, off, np.zeros(16, np.uint8), big, 16)
    assert e.value.status == ac.AC_ERR_TOO_LARGE
    # a rejected plan (automaton index out of range) is reported, and the next call works
    off2, buf2 = packed([np.frombuffer(b"ACGTACGTAC" * 20, np.uint8)] * 3)
    with pytest.raises(ac.AcError) as e:
        run(ac.ac_scan_batch_noalloc, autos, off2, buf2, [0, 1, 0], 64)
    assert e.value.status == ac.AC_ERR_INVALID
    n, keys, mt = run(ac.ac_scan_batch_noalloc, autos, off2, buf2, [0, 0, 0], 1024)
    m, keys2, mt2 = run(ac.ac_scan_batch, autos, off2, buf2, [0, 0, 0], 1024)
    assert n == m > 0 and np.array_equal(keys, keys2) and np.array_equal(mt, mt2)
    assert set(mt.tolist()) == {0, 1, 2}
