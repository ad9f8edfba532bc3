"""The random-gather measurement probe reads what it should: its per-item xors
equal a NumPy re-computation of the same published hash sequence."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M32 = 0xFFFFFFFF


def _mix32(v):
    """lowbias32 (C. Wellons) on uint64 arrays holding 32-bit values."""
    v = v & M32
    v ^= v >> 16
    v = (v * 0x7FEB352D) & M32
    v ^= v >> 15
    v = (v * 0x846CA68B) & M32
    v ^= v >> 16
    return v


def _expected(words, n, loads, seed):
    """words: uint32 [n_words][4] view of the table."""
    gw = words.shape[0] // 8
    out = np.zeros((8, n), np.uint64)
    s = np.arange(n, dtype=np.uint64)
    for g in range(8):
        h = _mix32(s ^ _mix32(np.uint64((seed + g) & M32)))
        acc = np.zeros(n, np.uint64)
        for j in range(loads):
            r = _mix32((h + np.uint64((j * 0x9E3779B9) & M32)) & M32)
            idx = (r * np.uint64(gw)) >> np.uint64(32)
            q = words[g * gw + idx.astype(np.int64)].astype(np.uint64)
            acc ^= q[:, 0] ^ q[:, 1] ^ q[:, 2] ^ q[:, 3]
        out[g] = acc
    return out.astype(np.uint32)


@pytest.mark.parametrize("n_words,n,loads", [(8 * 1000 + 5, 3001, 8), (64, 257, 4), (8, 1, 12)])
def test_probe_gather_reads_the_hashed_offsets(n_words, n, loads):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_03184_amd import ops as O
    rng = np.random.default_rng(11)
    words = rng.integers(0, 2**32, size=(n_words, 4), dtype=np.uint64).astype(np.uint32)
    table = torch.from_numpy(words.view(np.int32)).cuda()
    out = O.probe_gather(table, n, loads, seed=7)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, _expected(words, n, loads, 7))
