"""Full-size parity of the batched and served forms, in the launch
configurations bench.py times: every text's (request's) list against plain
scans of the same text, and sampled texts against the oracle one by one.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from synth import batched_workload, served_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")
autotune = pytest.importorskip("paper_1403_1305_amd.autotune")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def sample_indices(lengths: np.ndarray, k: int, max_len: int) -> list[int]:
    """k indices spread over the length order, each at most max_len long."""
    order = [int(i) for i in np.argsort(lengths, kind="stable") if lengths[i] <= max_len]
    step = max(1, len(order) // k)
    return order[::step][:k]


def test_full_batched_configuration():
    note("generate batched workload (4,096 texts)")
    texts, sets, text_set = batched_workload()
    autos = []
    for s in sets:
        d, o = ac.patterns_csr(s)
        autos.append(ac.ac_build(d, o, opts=ac._opts(placement=ac.AC_PLACE_LDS_HOT)))
    buf, offs, lens = ac.pack_texts(texts)
    d_text = torch.from_numpy(buf).to("cuda")
    del buf
    cap = 1 << 25
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    note("tune and scan")
    batch, tune, report = autotune.tune_batch(autos, d_text, offs, lens, text_set, out, cap, count,
                                              use_cache=False)
    ac.ac_batch_scan(batch, d_text, out, cap, count, True)
    torch.cuda.synchronize()
    n = int(count.item())
    assert 0 < n <= cap
    keys = np.sort(ac.keys_to_numpy(out[:n]))

    note("per-text plain scans")
    plain = []
    for t in range(len(texts)):
        if lens[t] == 0:
            continue
        o, m = int(offs[t]), int(lens[t])
        k = ac.keys_to_numpy(ac.scan_text(autos[int(text_set[t])], d_text[o:o + m]))
        plain.append(k + (np.uint64(o) << np.uint64(32)))
    assert np.array_equal(keys, np.sort(np.concatenate(plain)))

    note("oracle samples")
    pos = (keys >> np.uint64(32)).astype(np.int64)
    orc = {}
    for t in sample_indices(lens, 12, 1 << 20):
        a = int(text_set[t])
        if a not in orc:
            orc[a] = oracle.OracleAC(sets[a])
        o, m = int(offs[t]), int(lens[t])
        lo, hi = np.searchsorted(pos, o), np.searchsorted(pos, o + m)
        got = keys[lo:hi] - (np.uint64(o) << np.uint64(32))
        assert np.array_equal(got, orc[a].scan(texts[t])), (t, m, a)


def test_full_served_configuration():
    note("generate served workload (512 requests)")
    w = served_workload()
    R = len(w.length)
    d_texts = [torch.from_numpy(t).to("cuda") for t in w.texts]
    autos = []
    for s in w.sets:
        d, o = ac.patterns_csr(s)
        autos.append(ac.ac_build(d, o))
    views = [d_texts[int(w.alpha[i])][int(w.offset[i]):int(w.offset[i] + w.length[i])] for i in range(R)]

    note("serial plain counts")
    cap = 1 << 26
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    counts = torch.zeros(R, dtype=torch.int64, device="cuda")
    for i in range(R):
        ac.ac_scan(autos[int(w.automaton[i])], views[i], int(w.length[i]), out, cap, counts[i:i + 1])
    torch.cuda.synchronize()
    plain_counts = counts.cpu().numpy()
    del out

    note("served, all requests arriving together")
    srv = ac.Server(autos, hbm_budget=4 << 30, max_inflight=8)
    at = srv.now_ns() + 50_000_000
    tickets = [srv.submit(int(w.automaton[i]), views[i], n=int(w.length[i]), on_device=True, arrival_ns=at)
               for i in range(R)]
    sample = set(sample_indices(w.length, 16, 1 << 20))
    served_keys = {}
    dfa = ac._scan_opts(ac.AC_ALGO_DFA)
    for i, t in enumerate(tickets):
        r = srv.wait(t, 60_000)  # fails the test instead of hanging it
        assert r.n_matches == plain_counts[i], i
        # every request's whole list, sorted on the device, against a plain
        # DFA scan of its text alone
        got = torch.sort(srv.keys_tensor(r))[0]
        plain = torch.sort(ac.scan_text(autos[int(w.automaton[i])], views[i], opts=dfa))[0]
        assert torch.equal(got, plain), i
        if i in sample:
            served_keys[i] = np.sort(srv.keys(r))
        srv.release(t)
    assert srv.stats()["running_peak"] > 1
    srv.close()

    note("oracle samples")
    orc = {}
    for i in sorted(sample):
        a = int(w.automaton[i])
        if a not in orc:
            orc[a] = oracle.OracleAC(w.sets[a])
        text = w.texts[int(w.alpha[i])][int(w.offset[i]):int(w.offset[i] + w.length[i])]
        assert np.array_equal(served_keys[i], orc[a].scan(text)), (i, a)
