"""Independent structural checker for block trees (used on oracle and GPU output).

Given only what a block tree stores -- per level the marked bits and the
(block, offset) pointers of unmarked blocks, plus the leaf bytes -- it rebuilds
block starts from the marks, reconstructs the text bottom-up through the
pointers, and checks the invariants that the definition of Section 4 implies:

  I1  the reconstruction equals T (access(i) = T[i] for every i)
  I2  each pointer's source equals its block and is the leftmost occurrence
  I3  the target block is marked; when the source spills over, the next block
      is consecutive and marked
  I4  the source ends at or before the block's own start
  I6  every leftmost consecutive pair is marked, and every marked block with a
      consecutive neighbour lies in a leftmost pair
  I7  block 0 of every non-leaf level is marked
It shares no code with the oracle or the GPU library.
"""
import numpy as np


class Shape:
    """Minimal tree view: levels = [(b, marked, ptr_block, ptr_off)], leaves."""

    def __init__(self, n, tau, leaf_len, b1, levels, leaves, exact_split=True):
        self.n, self.tau, self.leaf_len, self.b1 = n, tau, leaf_len, b1
        self.levels = levels
        self.leaves = bytes(leaves)
        self.exact_split = exact_split


def from_oracle(t, exact_split=True):
    lv = [(L.b, L.marked, L.ptr_block, L.ptr_off) for L in t.levels]
    return Shape(t.n, t.tau, t.leaf_len, t.b1, lv, t.leaves.tobytes(), exact_split)


def block_layout(s):
    """Per level: (starts, lengths) implied by the marks."""
    n = s.n
    st = np.arange(0, n, s.b1, dtype=np.int64) if n else np.zeros(0, np.int64)
    ln = np.minimum(s.b1, n - st)
    out = []
    b = s.b1
    for li, (lb, marked, _, _) in enumerate(s.levels):
        assert lb == b, "level %d block length %d, expected %d" % (li + 1, lb, b)
        assert len(marked) == len(st), "level %d has %d marks for %d blocks" % (li + 1, len(marked), len(st))
        out.append((st, ln))
        if li == len(s.levels) - 1:
            break
        nb = b // s.tau if s.exact_split else -(-b // s.tau)
        m = np.asarray(marked).astype(bool)
        ms, ml = st[m], ln[m]
        cnt = (ml + nb - 1) // nb
        par = np.repeat(np.arange(ms.size), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        k = np.arange(par.size) - first
        st = ms[par] + k * nb
        ln = np.minimum(nb, ms[par] + ml[par] - st)
        b = nb
    return out


def check(s, T, check_leftmost=True, max_leftmost=None):
    """Run every invariant; raise AssertionError on the first violation."""
    T = bytes(T)
    n = len(T)
    assert s.n == n
    lay = block_layout(s)
    h = len(s.levels)
    # leaves
    st, ln = lay[-1]
    assert int(ln.sum()) == len(s.leaves), "leaf bytes %d vs blocks %d" % (len(s.leaves), int(ln.sum()))
    R = np.full(n, -1, np.int32)
    lv = np.frombuffer(s.leaves, np.uint8)
    o = 0
    for a, l in zip(st.tolist(), ln.tolist()):
        R[a:a + l] = lv[o:o + l]
        o += l
    Tb = T
    for li in range(h - 2, -1, -1):
        b, marked, pb, po = s.levels[li]
        st, ln = lay[li]
        c = len(st)
        marked = np.asarray(marked).astype(bool)
        if c:
            assert marked[0], "I7: level %d block 0 not marked" % (li + 1)
        adj = np.zeros(c, bool)
        if c > 1:
            adj[:-1] = st[1:] == st[:-1] + ln[:-1]
        um = np.flatnonzero(~marked)
        assert len(um) == len(pb) == len(po), "level %d: %d unmarked, %d pointers" % (li + 1, len(um), len(pb))
        checked = 0
        for k, j in enumerate(um.tolist()):
            t, off = int(pb[k]), int(po[k])
            assert 0 <= t < c and marked[t], "I3: level %d block %d -> unmarked/absent %d" % (li + 1, j, t)
            assert 0 <= off < ln[t], "I3: offset %d outside block %d" % (off, t)
            p, L, a = int(st[t]) + off, int(ln[j]), int(st[j])
            if off + L > ln[t]:
                assert t + 1 < c and adj[t] and marked[t + 1], "I3: spill past block %d" % t
                assert off + L <= ln[t] + ln[t + 1], "I3: source exceeds the pair"
            assert p + L <= a, "I4: source [%d,%d) overlaps block at %d" % (p, p + L, a)
            src = R[p:p + L]
            assert (src >= 0).all(), "source not yet reconstructed at level %d" % (li + 1)
            R[a:a + L] = src
            if check_leftmost and (max_leftmost is None or checked < max_leftmost):
                X = Tb[a:a + L]
                assert Tb[p:p + L] == X, "I2: source differs from block %d" % j
                assert Tb.find(X, 0, p + L) == p, "I2: block %d has an earlier occurrence" % j
                checked += 1
        if check_leftmost and c <= 200000:
            for j in range(c - 1):
                if not adj[j]:
                    continue
                a, L = int(st[j]), int(ln[j] + ln[j + 1])
                lm = Tb.find(Tb[a:a + L], 0, a + L) == a
                if lm:
                    assert marked[j] and marked[j + 1], "I6: leftmost pair %d unmarked" % j
            for j in range(c):
                if not marked[j]:
                    continue
                left = j > 0 and adj[j - 1]
                if not left and not adj[j]:
                    continue
                ok = False
                for i in (j - 1, j):
                    if 0 <= i and i + 1 < c and adj[i]:
                        a, L = int(st[i]), int(ln[i] + ln[i + 1])
                        if Tb.find(Tb[a:a + L], 0, a + L) == a:
                            ok = True
                assert ok, "I6: marked block %d of level %d is in no leftmost pair" % (j, li + 1)
    assert (R >= 0).all(), "I1: positions not covered by the tree"
    assert bytes(R.astype(np.uint8)) == T, "I1: reconstruction differs from T"
    return True


def level_sizes(s):
    return [len(m) for (_, m, _, _) in s.levels]
