"""Host checks of the wavefront sort of the orderings (Sec. 3.3 orderings of a
cell along 13 axes): the mirrored bitonic network over 64 E words, word i in
lane i % 64 and slot i / 64, and the sort words (order-preserving image of
the FP32 projection with the cell index in its low bits).

The network, as the kernel runs it: for each merge size kk = 2, 4, ..., 64 E,
first pair i with i ^ (kk - 1), then i with i ^ j for j = kk/4, ..., 1; every
comparator keeps the smaller word at the lower index.  Emulated here with
numpy on whole arrays, lane by lane as the kernel's exchanges move words."""
import numpy as np
import pytest


def network(E):
    kk = 2
    while kk <= 64 * E:
        yield kk - 1, kk >> 1
        j = kk >> 2
        while j >= 1:
            yield j, j
            j >>= 1
        kk <<= 1


def run_network(words, E):
    v = words.reshape(E, 64).copy()
    lanes = np.arange(64)
    for m, hb in network(E):
        new = np.empty_like(v)
        for e in range(E):
            partner = v[e ^ (m >> 6)][lanes ^ (m & 63)]
            low = ((e * 64 + lanes) & hb) == 0
            new[e] = np.where(low, np.minimum(v[e], partner), np.maximum(v[e], partner))
        v = new
    return v.reshape(-1)


def float_key(f):
    b = np.asarray(f, dtype=np.float32).view(np.uint32)
    return np.where(b & 0x80000000, ~b, b | 0x80000000).astype(np.uint32)


def key_float(k):
    k = np.asarray(k, dtype=np.uint32)
    return np.where(k & 0x80000000, k & 0x7fffffff, ~k).astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("E", [1, 2, 4])
def test_network_sorts(E):
    rng = np.random.default_rng(E)
    assert len(list(network(E))) == {1: 21, 2: 28, 4: 36}[E]
    for t in range(200):
        hi = 5 if t % 3 == 0 else 1 << 30          # many ties, or few
        x = rng.integers(0, hi, 64 * E, dtype=np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(run_network(x, E), np.sort(x))


@pytest.mark.parametrize("E", [1, 2, 4])
def test_sort_words_round_keys_down_and_keep_cell_order_of_ties(E):
    rng = np.random.default_rng(10 + E)
    idx = np.uint32(64 * E - 1)
    n = 64 * E - 7                                  # a ragged cell: the rest are padding words
    f = rng.normal(0.0, 0.05, n).astype(np.float32)
    f[5] = f[9] = f[3]                              # equal projections
    f[11] = 0.0
    f[12] = -0.0
    words = np.full(64 * E, 0xffffffff, dtype=np.uint32)
    words[:n] = (float_key(f) & ~idx) | np.arange(n, dtype=np.uint32)
    out = run_network(words, E)[:n]
    order = (out & idx).astype(np.int64)
    keys = key_float(out & ~idx)
    assert sorted(order.tolist()) == list(range(n))             # a permutation of the cell
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)         # monotone stored keys
    exact = f[order].astype(np.float64)
    assert np.all(keys <= exact)                                 # rounded down ...
    # ... by < 2^-15 of the key, or (at zero) by at most 2^8 of the smallest subnormal
    assert np.all(exact - keys <= 2.0 ** -15 * np.abs(exact) + 2.0 ** -141)
    ties = [k for k in order if f[k] == f[3]]
    assert ties == sorted(ties)                                  # equal keys keep the cell order
    # the order agrees with the exact projections up to that rounding
    assert np.all(np.diff(exact) >= -2.0 ** -14 * np.maximum(np.abs(exact[:-1]), np.abs(exact[1:])))
