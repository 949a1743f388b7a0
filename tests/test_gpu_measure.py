"""The streaming kernels that price the scans: the read kernel's XOR fold
equals the fold of the bytes computed on the host, and the copy kernel
reproduces its source, at sizes with ragged 16-byte and 4-byte tails and at
grids smaller and larger than the buffer needs."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ac = pytest.importorskip("paper_1403_1305_amd.ac")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ac.load_library()


def host_fold(b: np.ndarray) -> int:
    pad = np.zeros((-b.size) % 4, np.uint8)
    w = np.concatenate([b, pad]).view("<u4")
    return int(np.bitwise_xor.reduce(w)) if w.size else 0


@pytest.mark.parametrize("n", [0, 1, 3, 15, 16, 17, 4096 + 5, 3 * (1 << 20) + 7, 64 << 20])
@pytest.mark.parametrize("blocks", [0, 1, 3])
def test_read_fold_and_copy(n, blocks):
    rng = np.random.default_rng(n + blocks)
    b = rng.integers(0, 256, size=n, dtype=np.uint8)
    d = torch.from_numpy(b).to("cuda") if n else torch.zeros(16, dtype=torch.uint8, device="cuda")
    fold = torch.full((1,), 0x5A5A, dtype=torch.int64, device="cuda")
    ac.ac_hbm_read(d, n, fold, blocks)
    assert int(fold.item()) == 0x5A5A ^ host_fold(b)
    dst = torch.full((max(n, 16) + 32,), 0xEE, dtype=torch.uint8, device="cuda")
    ac.ac_hbm_copy(dst, d, n, blocks)
    out = dst.cpu().numpy()
    assert np.array_equal(out[:n], b)
    assert (out[n:] == 0xEE).all()  # nothing past the end is written


def test_errors():
    d = torch.zeros(64, dtype=torch.uint8, device="cuda")
    fold = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(ac.AcError) as e:
        ac.ac_hbm_read(d[1:], 32, fold)
    assert e.value.status == ac.AC_ERR_INVALID
    with pytest.raises(ac.AcError) as e:
        ac.ac_hbm_copy(d[16:], d, 32)
    assert e.value.status == ac.AC_ERR_INVALID
    with pytest.raises(ac.AcError) as e:
        ac.ac_hbm_copy(d, d[3:], 16)
    assert e.value.status == ac.AC_ERR_INVALID
