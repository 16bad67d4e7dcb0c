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


# ---------------------------------------------------------------- shift and merge
# The construction the work-group kernel uses for cells whose particles do not
# crowd one sub-cell (Sec. 3.3, Fig. HierarchySorting): sub-cells of depth D
# (the shallowest with at most 64 particles each; 3 when only that holds at
# most 256) are ordered directly with keys in their own frames; then per level
# every run is shifted into its parent's frame and the eight siblings are
# merged pairwise in three rounds, a word's place being its index in its run
# plus the number of partner words with a smaller key (at most equal for the
# second run).  FP32 throughout, as the kernel.

SUB = 3


def sub_morton(ix, iy, iz):
    m = np.zeros_like(ix)
    for b in range(SUB - 1, -1, -1):
        m = (m << 3) | (((ix >> b) & 1) << 2) | (((iy >> b) & 1) << 1) | ((iz >> b) & 1)
    return m


def sub_corner(m, L):
    c = np.zeros((len(m), 3), dtype=np.int64)
    for b in range(SUB - 1, SUB - L - 1, -1):
        tri = (m >> (3 * b)) & 7
        c[:, 0] |= ((tri >> 2) & 1) << b
        c[:, 1] |= ((tri >> 1) & 1) << b
        c[:, 2] |= (tri & 1) << b
    return c


def f32(a):
    return np.asarray(a, dtype=np.float32)


def proj(u, v):
    # su[0] * v0 + su[1] * v1 + su[2] * v2 in FP32, left to right (no fusing: the
    # kernel's compiler may fuse, which the tolerance below covers)
    return f32(f32(f32(u[0] * v[:, 0]) + f32(u[1] * v[:, 1])) + f32(u[2] * v[:, 2]))


def shift_merge_emulated(x, edge, u):
    n = len(x)
    es = f32(edge / 2 ** SUB)
    i3 = np.clip((f32(x) / es).astype(np.int64), 0, 2 ** SUB - 1)
    m = sub_morton(i3[:, 0], i3[:, 1], i3[:, 2])
    cnt = np.bincount(m, minlength=8 ** SUB)
    runmax = {3: cnt.max(), 2: cnt.reshape(-1, 8).sum(1).max(), 1: cnt.reshape(-1, 64).sum(1).max()}
    D = next((L for L in (1, 2, 3) if runmax[L] <= 64), 3 if runmax[3] <= 256 else 0)
    if D == 0:
        return None, 0
    off = np.concatenate([[0], np.cumsum(cnt)])
    gsh = 3 * (SUB - D)
    key = proj(u, f32(f32(x) - f32(f32(sub_corner(m, D)) * es)))
    # grouped by depth-D sub-cell, each ordered by (key image, index): the
    # rank of every word in its run
    order = np.lexsort((np.arange(n), key_image(key), m >> gsh))
    idx = order.copy()
    keys = key[order].astype(np.float32)
    for L in range(D, 0, -1):
        csh = 3 * (SUB - L)
        sh = proj(u, f32(f32(sub_corner(m[idx], L) - sub_corner(m[idx], L - 1)) * es))
        keys = f32(keys + sh)
        for q in range(3):
            span = 1 << (csh + q)
            out_k = np.empty_like(keys)
            out_i = np.empty_like(idx)
            filled = np.zeros(n, dtype=bool)
            for g0 in range(0, 8 ** SUB // span, 2):
                a0, a1 = off[g0 * span], off[(g0 + 1) * span]
                b0, b1 = a1, off[(g0 + 2) * span]
                A, B = key_image(keys[a0:a1]), key_image(keys[b0:b1])
                pa = a0 + np.arange(a1 - a0) + np.searchsorted(B, A, side="left")
                pb = a0 + np.arange(b1 - b0) + np.searchsorted(A, B, side="right")
                for p, lo, hi in ((pa, a0, a1), (pb, b0, b1)):
                    assert not filled[p].any()
                    filled[p] = True
                    out_k[p] = keys[lo:hi]
                    out_i[p] = idx[lo:hi]
            assert filled.all()
            keys, idx = out_k, out_i
    return list(zip(keys, idx)), D


@pytest.mark.parametrize("n,clump,seed", [(300, 0.0, 1), (700, 0.0, 2), (2000, 0.0, 3), (1500, 0.6, 4),
                                          (4096, 0.3, 5)])
def test_shift_merge_orders_the_cell(n, clump, seed):
    """A permutation, keys non-decreasing along it, and every key within a few
    units of rounding of the cell's size of the projection in the cell's frame
    (the staging's margin, 1e-5 of the edge, covers them)."""
    rng = np.random.default_rng(seed)
    edge = f32([0.25, 0.2, 0.3])
    x = rng.random((n, 3)) * edge
    k = int(clump * n)
    x[:k] = edge * (0.3 + 0.05 * rng.random((k, 3)))   # a dense clump
    x = f32(np.clip(x, 0, edge * (1 - 1e-7)))
    for s in range(13):
        d = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)][s + 13]
        u = f32(np.array(d) / np.linalg.norm(d))
        got, D = shift_merge_emulated(x, edge, u)
        if got is None:
            continue
        order = np.array([w[1] for w in got])
        keys = np.array([w[0] for w in got], dtype=np.float32)
        assert np.array_equal(np.sort(order), np.arange(n))
        assert np.all(np.diff(keys.astype(np.float64)) >= 0)
        exact = np.asarray(x[order], np.float64) @ np.asarray(u, np.float64)
        assert np.max(np.abs(keys - exact)) <= 2e-6 * float(edge.max()), (s, D)


def test_shift_merge_depth_choice():
    # uniform cells take the shallowest depth with at most 64 per sub-cell;
    # a cell crowding > 256 into one depth-3 sub-cell is left to the runs of 256
    edge = f32([1.0, 1.0, 1.0])
    rng = np.random.default_rng(9)
    u = f32([1.0, 0.0, 0.0])
    _, D = shift_merge_emulated(f32(rng.random((400, 3))), edge, u)
    assert D == 1
    _, D = shift_merge_emulated(f32(rng.random((3000, 3))), edge, u)
    assert D == 3
    x = f32(rng.random((600, 3)))
    x[:300] = 0.01
    got, D = shift_merge_emulated(x, edge, u)
    assert got is None and D == 0
