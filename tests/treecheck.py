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


def _runs(st, ln):
    """Maximal runs of consecutive blocks, as (start, end) pairs."""
    out = []
    for a, l in zip(st.tolist(), ln.tolist()):
        if out and out[-1][1] == a:
            out[-1][1] = a + l
        else:
            out.append([a, a + l])
    return out


def _leftmost_on_level(Tb, runs, a, L):
    """Smallest p with T[p..p+L) == T[a..a+L) inside one run (a itself qualifies)."""
    X = Tb[a:a + L]
    for rs, re in runs:
        if rs > a:
            break
        p = Tb.find(X, rs, min(re, a + L))
        if p >= 0:
            return p
    raise AssertionError("block at %d not found on its own level" % a)


def check_pruned(s, T):
    """Invariants of a pruned tree (Section 4.1, optional pruning), checked
    without replaying the pruning sweep.

    The tree the marking rule defines ("unpruned") is rebuilt level by level
    from the definition alone.  A pruned tree keeps that block layout on every
    level except for the children of pruned blocks.  Per level, with every
    pointer that existed when the level was judged -- the final ones plus those
    of blocks removed later with a pruned parent, each aimed at its block's
    leftmost occurrence among the level's runs -- it asserts:
      Q1  marks only go away: a marked block is marked by the definition
      Q2  a pruned block (marked by the definition, unmarked or gone) is
          untargeted, has no marked child, and its leftmost occurrence ends at
          or before its start and lies in one block or a consecutive pair; a
          stored pointer is that occurrence
      Q3  a block that stays marked fails one of those conditions
    plus I1, I3, I4 and I7 of check() (the pruned tree still spells T)."""
    T = bytes(T)
    h = len(s.levels)
    n = len(T)

    def nb_of(b):
        return b // s.tau if s.exact_split else -(-b // s.tau)

    def children(st, ln, sel, b):
        nb = nb_of(b)
        ms, ml = st[sel], ln[sel]
        cnt = (ml + nb - 1) // nb
        par = np.repeat(np.arange(ms.size), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        cst = ms[par] + (np.arange(par.size) - first) * nb
        return cst, np.minimum(nb, ms[par] + ml[par] - cst), cnt

    # unpruned layouts and definition marks, top-down
    U = []
    st = np.arange(0, n, s.b1, dtype=np.int64) if n else np.zeros(0, np.int64)
    ln = np.minimum(s.b1, n - st)
    for li in range(h):
        c = len(st)
        dm = np.zeros(c, bool)
        if li < h - 1:
            adj = np.zeros(c, bool)
            if c > 1:
                adj[:-1] = st[1:] == st[:-1] + ln[:-1]
            for j in range(c):
                if adj[j]:
                    a, L = int(st[j]), int(ln[j] + ln[j + 1])
                    if T.find(T[a:a + L], 0, a + L) == a:
                        dm[j] = dm[j + 1] = True
                if not (j > 0 and adj[j - 1]) and not adj[j]:
                    dm[j] = True
        U.append((st, ln, dm))
        if li < h - 1:
            st, ln, _ = children(st, ln, dm, s.levels[li][0])
    # which unpruned blocks are present in the pruned tree, and their marks
    # when their level was judged (a block removed later was unmarked then)
    present = np.ones(len(U[0][0]), bool)
    pres_all, jm_all = [], []
    for li in range(h):
        st, ln, dm = U[li]
        fm = np.asarray(s.levels[li][1]).astype(bool)
        assert int(present.sum()) == len(fm), "level %d: %d blocks, %d expected" % (
            li + 1, len(fm), int(present.sum()))
        jm = np.zeros(len(st), bool)
        jm[present] = fm
        assert not (jm & ~dm).any(), "Q1: level %d marks a block the definition leaves unmarked" % (li + 1)
        pres_all.append(present)
        jm_all.append(jm)
        if li < h - 1:
            _, _, cnt = children(st, ln, dm, s.levels[li][0])
            present = np.repeat(jm[dm], cnt)
    for li in range(h - 1):
        st, ln, dm = U[li]
        jm, present = jm_all[li], pres_all[li]
        c = len(st)
        runs = _runs(st, ln)
        lm = np.array([_leftmost_on_level(T, runs, int(st[j]), int(ln[j])) for j in range(c)], np.int64)
        tb = np.searchsorted(st, lm, side="right") - 1
        spill = lm + ln > st[tb] + ln[tb] if c else np.zeros(0, bool)
        tgt = np.zeros(c, bool)
        for j in np.flatnonzero(~jm).tolist():
            tgt[tb[j]] = True
            if spill[j]:
                tgt[tb[j] + 1] = True
        _, _, cnt = children(st, ln, dm, s.levels[li][0])
        cf = np.zeros(c + 1, np.int64)
        cf[1:][dm] = cnt
        cf = np.cumsum(cf)
        below = jm_all[li + 1] if li + 1 < h - 1 else np.zeros(int(cf[-1]), bool)
        for j in np.flatnonzero(dm).tolist():
            inner = bool(below[cf[j]:cf[j + 1]].any())
            t = int(tb[j])
            # the occurrence fits one block or a consecutive pair
            fits = not spill[j] or (t + 1 < c and st[t + 1] == st[t] + ln[t] and
                                    lm[j] + ln[j] <= st[t + 1] + ln[t + 1])
            early = lm[j] + ln[j] <= st[j] and fits
            if jm[j]:
                assert tgt[j] or inner or not early, \
                    "Q3: level %d block at %d stays marked but could be pruned" % (li + 1, int(st[j]))
            else:
                why = "targeted" if tgt[j] else "has a marked child" if inner else "has no earlier occurrence"
                assert not tgt[j] and not inner and early, \
                    "Q2: level %d block at %d is pruned but %s" % (li + 1, int(st[j]), why)
        # stored pointers of the present unmarked blocks
        rank = np.full(c, -1, np.int64)
        rank[present] = np.arange(int(present.sum()))
        _, _, pb, po = s.levels[li]
        k = 0
        for j in np.flatnonzero(present & ~jm).tolist():
            t = int(tb[j])
            want = (int(rank[t]), int(lm[j] - st[t]))
            assert k < len(pb) and (int(pb[k]), int(po[k])) == want, \
                "Q2: level %d block at %d: pointer %s, expected %s" % (
                    li + 1, int(st[j]), (int(pb[k]), int(po[k])) if k < len(pb) else None, want)
            k += 1
        assert k == len(pb), "level %d: %d pointers stored, %d expected" % (li + 1, len(pb), k)
    check(s, T, check_leftmost=False)
    return True
