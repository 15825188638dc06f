"""Tree walks of the thesis's query algorithms over an oracle tree, with naive bit counting.

Test-side helper: given the level bits and cumulative histogram the oracle built, answer
access / rank / select the way the query sections of the thesis traverse the level-wise
tree (Section 5.2 top-down access, Section 5.3 top-down rank, Section 5.4 bottom-up
select), counting bits one by one instead of using a rank/select directory. If the oracle's
levels, cumulative histogram or codes were wrong, these walks would not reproduce the
definitions, so they pin the oracle's structure to the sequence.

The walks also return the intermediate values the worked example of the thesis prints.
"""
from __future__ import annotations


def pow2_below(x: int) -> int:
    p = 1
    while p * 2 < x:
        p *= 2
    return p


def _bits(t, l):
    return [t.bit(l, j) for j in range(t.level_n[l])]


def rank_bit(t, l, b, x):
    row = _bits(t, l)
    return sum(1 for j in range(x) if row[j] == b)


def select_bit(t, l, b, k):
    row = _bits(t, l)
    seen = 0
    for j, v in enumerate(row):
        if v == b:
            seen += 1
            if seen == k:
                return j
    raise ValueError("select beyond count")


def walk_access(t, i):
    """Top-down: at each node read the bit of the element, move to the child it names."""
    start, end = 0, t.sigma
    trace = []
    if t.L == 0:
        return 0, trace
    for l in range(t.L):
        base = int(t.cum_hist[start])
        width = end - start
        if width <= 2:
            bit = t.bit(l, base + i) if width > 1 else 0
            trace.append(("leaf", l, bit, i))
            return (start + 1 if (width > 1 and bit) else start), trace
        bit = t.bit(l, base + i)
        z_node = rank_bit(t, l, 0, base)
        z_pos = rank_bit(t, l, 0, base + i)
        half = pow2_below(width)
        if bit == 0:
            i = z_pos - z_node
            end = start + half
        else:
            i = i - (z_pos - z_node)
            start = start + half
        trace.append(("step", l, bit, i))
    return start, trace


def walk_rank(t, c, i):
    """Top-down along the path of c, counting the bits of c's side before the position."""
    start, end = 0, t.sigma
    trace = []
    if t.L == 0:
        return i, trace
    for l in range(t.L):
        if end - start <= 1:
            break
        base = int(t.cum_hist[start])
        z_node = rank_bit(t, l, 0, base)
        z_pos = rank_bit(t, l, 0, base + i)
        split = start + pow2_below(end - start)
        if c < split:
            i = z_pos - z_node
            end = split
        else:
            i = i - (z_pos - z_node)
            start = split
        trace.append((l, i))
    return i, trace


def walk_select(t, c, k):
    """Bottom-up: from c's leaf, map the k-th occurrence to its position in each parent."""
    if t.L == 0:
        return k - 1, []
    # nodes on the root-to-leaf path of c: (level, start symbol, side of c)
    path = []
    start, end = 0, t.sigma
    l = 0
    while end - start > 1:
        split = start + pow2_below(end - start)
        side = 1 if c >= split else 0
        path.append((l, start, side))
        if side:
            start = split
        else:
            end = split
        l += 1
    trace = []
    r = k  # 1-based occurrence within the current node
    for (l, s, side) in reversed(path):
        base = int(t.cum_hist[s])
        before = rank_bit(t, l, side, base)
        pos = select_bit(t, l, side, before + r)
        trace.append((l, side, r, pos - base))
        r = pos - base + 1
    return r - 1, trace
