"""Host check of the candidate-scan rule the per-sequence kernels use: the
first maximum over predecessors in index order (strict '>' from -inf, the
winner's own value kept) equals two or four interleaved first-maximum chains
merged so that the larger value wins and equal values (-0 == +0) go to the
lower index.  Written out in plain Python over float32 values; padding
states beyond K carry -inf and must never win."""
import numpy as np
import pytest


def _scan(x):
    best, arg = np.float32(-np.inf), 0
    for i, v in enumerate(x):
        if v > best:
            best, arg = v, i
    return best, arg


def _chains(x, n_chains, kmax):
    xs = np.full(kmax, -np.inf, np.float32)
    xs[:len(x)] = x
    parts = []
    for c in range(n_chains):
        best, arg = np.float32(-np.inf), 0
        for i in range(c, kmax, n_chains):
            if xs[i] > best:
                best, arg = xs[i], i
        parts.append((best, arg))
    best, arg = parts[0]
    for b, a in parts[1:]:
        if b > best or (b == best and a < arg):
            best, arg = b, a
    return best, arg


@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("n_chains", [2, 4])
def test_interleaved_chains_equal_index_order_scan(seed, n_chains):
    r = np.random.default_rng(seed)
    K = int(r.integers(1, 130))
    kind = seed % 4
    if kind == 0:
        x = r.standard_normal(K).astype(np.float32)
    elif kind == 1:   # many exact ties
        x = r.integers(-3, 1, size=K).astype(np.float32)
    elif kind == 2:   # signed zeros and -inf mixed in
        x = r.choice(np.array([-0.0, 0.0, -1.0, -np.inf], np.float32), size=K)
    else:             # all -inf but a few NaN (never chosen by '>')
        x = np.full(K, -np.inf, np.float32)
        x[r.integers(0, K, size=max(1, K // 8))] = np.nan
    kmax = 128 if K <= 128 else 256
    b0, a0 = _scan(x)
    b1, a1 = _chains(x, n_chains, kmax)
    assert a0 == a1
    assert np.float32(b0).tobytes() == np.float32(b1).tobytes()


def test_signed_zero_keeps_first_index_and_its_sign():
    x = np.array([-1.0, -0.0, 0.0, -0.0], np.float32)
    for n in (2, 4):
        b, a = _chains(x, n, 128)
        assert a == 1 and np.signbit(b)
