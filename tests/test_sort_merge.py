"""Host checks of the ordering of cells larger than one wavefront sorts (Sec.
3.3: a parent's ordering made from the sorted orderings of its parts by O(n)
merges).  The work-group kernel, as it runs: words (order-preserving image of
the FP32 projection) << 32 | cell index, padded with all-ones words to whole
runs of 256; a bitonic network inside each run (stages of span <= 256, the
comparator of i and i ^ j ascending where i & k & 255 == 0, so that the
last stage leaves every run ascending); then merges of runs of
w into runs of 2w, each word placed at its index in its run plus the number of
words of the partner run below it (strictly below for the first run, at most
equal for the second).  Emulated word by word with numpy; the result must be
the lexicographic order of (projection image, cell index), the order that
ranking every word against all others gives."""
import numpy as np
import pytest

RUN = 256
CAP = 4096


def key_image(f):
    b = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return np.where(b & 0x80000000, (~b) & 0xFFFFFFFF, b | 0x80000000)


def merge_sort_emulated(f):
    count = len(f)
    np_ = (count + RUN - 1) // RUN * RUN
    assert np_ <= CAP
    buf = np.full(np_, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    buf[:count] = (key_image(f) << np.uint64(32)) | np.arange(count, dtype=np.uint64)
    k = 2
    while k <= RUN:
        j = k >> 1
        while j > 0:
            i = np.arange(np_)
            l = i ^ j
            m = l > i
            i, l = i[m], l[m]
            a, b = buf[i].copy(), buf[l].copy()
            swap = (a > b) == ((i & k & (RUN - 1)) == 0)
            buf[i[swap]], buf[l[swap]] = b[swap], a[swap]
            j >>= 1
        k <<= 1
    w = RUN
    while w < np_:
        out = np.empty_like(buf)
        written = np.zeros(np_, dtype=bool)
        for i in range(np_):
            pair = i // (2 * w) * (2 * w)
            la = min(w, np_ - pair)
            lb = min(w, np_ - pair - la)
            x = buf[i]
            if i < pair + la:
                part = buf[pair + la:pair + la + lb]
                place = (i - pair) + int(np.searchsorted(part, x, side="left"))
            else:
                part = buf[pair:pair + la]
                place = (i - pair - la) + int(np.searchsorted(part, x, side="right"))
            assert 0 <= place < la + lb or (lb == 0 and place < la)
            assert not written[pair + place]
            written[pair + place] = True
            out[pair + place] = x
        assert written.all()
        buf = out
        w <<= 1
    return buf[:count]


@pytest.mark.parametrize("count", [257, 300, 511, 512, 513, 769, 1000, 1300, 2049, 4096])
def test_merge_order_is_the_lexicographic_order(count):
    rng = np.random.default_rng(count)
    f = rng.normal(size=count).astype(np.float32)
    # ties: a block of equal projections and both zeros
    f[: count // 5] = f[0]
    f[count // 5] = 0.0
    f[count // 5 + 1] = -0.0
    got = merge_sort_emulated(f)
    keys = key_image(f)
    want = np.lexsort((np.arange(count), keys))
    assert np.array_equal((got & np.uint64(0xFFFFFFFF)).astype(np.int64), want)
    assert np.all(np.diff((got >> np.uint64(32)).astype(np.int64)) >= 0)
