"""CPU model of the clustering BVH builder's rounds and layout (host logic only).

The GPU builder (agglomerative clustering over the Morton order, then a
depth-first layout) is restated here step by step in numpy: nearest neighbours
by union surface area within R places, ties broken by the total order on pairs
(nearer pairs, then pairs whose smaller member is even, then smaller member),
mutual pairs merging, in-order compaction, and the preorder / first-leaf walk.
The tests check the properties the GPU code relies on: every round merges,
identical boxes pair up into a balanced tree, the layout gives each node a
contiguous leaf range, and chains of nested boxes are as deep as the fallback
test expects."""
import numpy as np
import pytest

from mrs_inputs import scenes as S

LEAF = 1 << 31


def _half_area(lo, hi):
    d = hi - lo
    return d[..., 0] * d[..., 1] + d[..., 1] * d[..., 2] + d[..., 2] * d[..., 0]


def _morton_order(tri):
    c = tri.mean(1)
    lo, hi = c.min(0), c.max(0)
    q = np.clip(((c - lo) / np.maximum(hi - lo, 1e-30) * 1024).astype(np.int64), 0, 1023)

    def spread(v):
        v = v.astype(np.uint64)
        for mul, mask in ((0x00010001, 0xFF0000FF), (0x00000101, 0x0F00F00F),
                          (0x00000011, 0xC30C30C3), (0x00000005, 0x49249249)):
            v = (v * np.uint64(mul)) & np.uint64(mask)
        return v
    code = (spread(q[:, 0]) << np.uint64(2)) | (spread(q[:, 1]) << np.uint64(1)) | spread(q[:, 2])
    key = (code << np.uint64(32)) | np.arange(len(tri), dtype=np.uint64)
    return np.argsort(key, kind="stable")


def _pair_key_less(c, j, b):
    """Pair {c, j} before {c, b} (arrays); b < 0 is no pair."""
    dj, db = np.abs(c - j), np.abs(c - b)
    j0, b0 = np.minimum(c, j), np.minimum(c, b)
    return ((b < 0) | (dj < db) | ((dj == db) & ((j0 & 1) == 0) & ((b0 & 1) == 1))
            | ((dj == db) & ((j0 & 1) == (b0 & 1)) & (j0 < b0)))


def cluster(tri, radius=12):
    """Returns (children [n-1, 2] in temporary ids, root, rounds, merges per round)."""
    n = len(tri)
    order = _morton_order(tri)
    t3 = tri[order]
    ref = (LEAF | np.arange(n)).astype(np.int64)
    lo, hi = t3.min(1).astype(np.float32), t3.max(1).astype(np.float32)
    children = np.zeros((n - 1, 2), np.int64)
    count, per_round = 0, []
    while len(ref) > 1:
        m = len(ref)
        idx = np.arange(m)
        best = np.full(m, np.inf, np.float32)
        bj = np.full(m, -1)
        for off in range(-radius, radius + 1):
            if off == 0:
                continue
            j = idx + off
            ok = (j >= 0) & (j < m)
            jj = np.clip(j, 0, m - 1)
            a = _half_area(np.minimum(lo, lo[jj]), np.maximum(hi, hi[jj])).astype(np.float32)
            better = ok & ((a < best) | ((a == best) & _pair_key_less(idx, jj, bj)))
            best, bj = np.where(better, a, best), np.where(better, jj, bj)
        mutual = bj[bj] == idx
        first = idx[mutual & (idx < bj)]
        for c in first:
            j = bj[c]
            children[count] = (ref[c], ref[j])
            ref[c] = count
            lo[c], hi[c] = np.minimum(lo[c], lo[j]), np.maximum(hi[c], hi[j])
            count += 1
        keep = ~(mutual & (idx > bj))
        per_round.append(len(first))
        ref, lo, hi = ref[keep], lo[keep], hi[keep]
    return children, int(ref[0]), len(per_round), per_round


def layout(children, root, n):
    """Preorder number of every internal node, first leaf of every node, depth."""
    nint = n - 1
    parent = {}
    for t in range(nint):
        for side in range(2):
            parent[int(children[t, side])] = (t, side)
    size = {}

    def leaves(r):
        if r & LEAF:
            return 1
        if r not in size:
            size[r] = leaves(int(children[r, 0])) + leaves(int(children[r, 1]))
        return size[r]
    leaves(root)
    pre, first, depth = {}, {}, 0
    for node in list(range(nint)) + [LEAF | k for k in range(n)]:
        p_, f_, d, x = 0, 0, 0, node
        while x in parent:
            t, side = parent[x]
            left = leaves(int(children[t, 0]))
            p_ += left if side else 1
            f_ += left if side else 0
            x, d = t, d + 1
        pre[node], first[node] = p_, f_
        depth = max(depth, d)
    return pre, first, size, depth


@pytest.mark.parametrize("maker", [lambda: S.random_soup(2, 40), lambda: S.cornell(1),
                                   lambda: S.random_soup(5, 1500)])
def test_every_round_merges_and_layout_is_contiguous(maker):
    tri = maker().vertices.astype(np.float32)
    n = len(tri)
    children, root, rounds, per_round = cluster(tri)
    assert min(per_round) >= 1 and sum(per_round) == n - 1
    pre, first, size, _ = layout(children, root, n)
    assert sorted(pre[t] for t in range(n - 1)) == list(range(n - 1)) and pre[root] == 0
    assert sorted(first[LEAF | k] for k in range(n)) == list(range(n))
    for t in range(n - 1):  # the left range is followed by the right range
        a, b = (int(c) for c in children[t])
        la = 1 if a & LEAF else size[a]
        assert first[a] == first[t] and first[b] == first[t] + la


def test_identical_boxes_make_a_balanced_tree():
    tri = np.tile(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), (1000, 1, 1))
    children, root, rounds, per_round = cluster(tri)
    _, _, _, depth = layout(children, root, len(tri))
    assert depth == 10 and rounds == 10  # ceil(log2 1000)


def test_nested_boxes_chain_one_merge_per_round():
    base = np.array([[-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 1.0, 0.0]])
    tri = np.array([base * 1.5 ** k + np.array([0.0, 0.0, 0.01 * k]) for k in range(100)],
                   np.float32)
    children, root, rounds, per_round = cluster(tri)
    _, _, _, depth = layout(children, root, len(tri))
    assert rounds == 99 and depth == 99 and max(per_round) == 1  # > 64: the GPU falls back
