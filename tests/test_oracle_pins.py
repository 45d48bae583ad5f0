"""Pins for the CPU oracle: the paper's worked example, brute force on tiny
inputs, closed forms, invariants and the per-level block bound.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth
from tests import treecheck

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_fig1():
    spec = {}
    rows = {"unpruned": [], "pruned": []}
    leaves = {}
    with open(os.path.join(GOLDEN, "fig1_abrainadrain.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] in ("text", "tau", "leaf", "b1"):
                spec[tok[0]] = tok[1]
            elif tok[1] == "leaves":
                leaves[tok[0]] = tok[2].encode()
            else:
                kind = tok[0]
                b = int(tok[4])
                i = tok.index("marked")
                j = tok.index("ptr")
                marked = [int(x) for x in tok[i + 1:j]]
                ptr = [tuple(int(v) for v in p.split(":")) for p in tok[j + 1:]]
                rows[kind].append((b, marked, ptr))
    return spec, rows, leaves


def test_fig1_worked_example():
    """Section 4, Figure 1 (unpruned reading; see the fixture's header)."""
    spec, rows, leaves = _load_fig1()
    t = oracle.build_tree(spec["text"].encode(), int(spec["tau"]), int(spec["leaf"]),
                          b1=int(spec["b1"]), exact_split=False)
    assert t.h == 3
    for (b, marked, ptr), L in zip(rows["unpruned"], t.levels):
        assert L.b == b
        assert L.marked.tolist() == marked
        assert list(zip(L.ptr_block.tolist(), L.ptr_off.tolist())) == ptr
    assert t.leaves.tobytes() == leaves["unpruned"]
    treecheck.check(treecheck.from_oracle(t, exact_split=False), spec["text"].encode())


def _brute_equal(T, tau, leaf, b1, exact):
    t = oracle.build_tree(T, tau, leaf, b1=b1, exact_split=exact)
    lv, leaves = brute.build(T, tau, leaf, b1, exact_split=exact)
    assert len(lv) == t.h
    for a, L in zip(lv, t.levels):
        assert a["b"] == L.b and a["c"] == L.c
        assert a["marked"] == L.marked.tolist() or L is t.levels[-1]
        assert a["ptr"] == list(zip(L.ptr_block.tolist(), L.ptr_off.tolist()))
    assert leaves == t.leaves.tobytes()


@pytest.mark.parametrize("sigma,nmax", [(2, 11), (3, 7)])
def test_brute_force_exhaustive(sigma, nmax):
    """Every text over a tiny alphabet: C oracle (memmem) == dictionary brute
    force, for tau in {2,3}, leaf in {1,2} and every admissible b1 = leaf*tau^k."""
    alph = b"ab" if sigma == 2 else b"abc"
    cases = 0
    for n in range(1, nmax + 1):
        for word in itertools.product(alph, repeat=n):
            T = bytes(word)
            for tau in (2, 3):
                for leaf in (1, 2):
                    b1 = leaf
                    while True:
                        _brute_equal(T, tau, leaf, b1, True)
                        cases += 1
                        if b1 >= n:
                            break
                        b1 *= tau
    assert cases > 10000


def test_brute_force_general_split():
    """General ceil(b/tau) split (Figure 1 style) on random small texts."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(1, 30))
        T = bytes(rng.integers(97, 97 + int(rng.integers(1, 4)), n).astype(np.uint8))
        tau = int(rng.integers(2, 5))
        b1 = int(rng.integers(1, n + 1))
        leaf = int(rng.integers(1, 3))
        if b1 < leaf:
            b1 = leaf
        _brute_equal(T, tau, leaf, b1, False)


def test_search_modes_agree():
    """memmem over T == literal double loop == search restricted to level runs
    (the 'leftmost on this level' reading of Section 4)."""
    texts = [synth.cfg1_text(1 << 14), synth.random_text(3000, 4, 5),
             synth.periodic_text(2048, 7, 1), bytes(b"ab" * 700),
             synth.markov_versions(1 << 14, 1024, 16, 5e-3, 16, 9)]
    for T in texts:
        T = bytes(T)
        for tau, leaf in ((2, 4), (3, 2), (4, 16)):
            a = oracle.build_tree(T, tau, leaf, search=oracle.SEARCH_MEMMEM)
            b = oracle.build_tree(T, tau, leaf, search=oracle.SEARCH_RUNS)
            assert a.canonical == b.canonical
            if len(T) <= 4096:
                c = oracle.build_tree(T, tau, leaf, search=oracle.SEARCH_NAIVE)
                assert a.canonical == c.canonical


def test_unary_text():
    """T = a^n (n >= 3*b1): blocks 0 and 1 are marked, every other block points
    at (0, 0); every later level has 2*tau blocks; 2*tau leaves."""
    for tau, leaf, n in ((2, 1, 200), (3, 2, 500), (4, 4, 1000)):
        b1 = leaf
        while b1 * tau * 3 <= n:
            b1 *= tau
        T = b"a" * n
        t = oracle.build_tree(T, tau, leaf, b1=b1)
        for li, L in enumerate(t.levels[:-1]):
            assert L.marked[:2].tolist() == [1, 1] and not L.marked[2:].any()
            assert (L.ptr_block == 0).all() and (L.ptr_off == 0).all()
            if li > 0:
                assert L.c == 2 * tau
        assert t.levels[-1].c == 2 * tau
        treecheck.check(treecheck.from_oracle(t), T)


def test_all_distinct_text():
    """A permutation of the byte values: every block on every level is marked."""
    rng = np.random.default_rng(3)
    for n in (256, 200, 77):
        T = bytes(rng.permutation(256)[:n].astype(np.uint8))
        for tau, leaf in ((2, 1), (3, 2), (4, 4)):
            t = oracle.build_tree(T, tau, leaf)
            for L in t.levels[:-1]:
                assert L.u == 0 and L.marked.all()
                assert L.c == -(-n // L.b)
            assert t.leaves.tobytes() == T


def test_period_two_text():
    """(ab)^m with tau = 3 and leaf = 1 (odd block lengths): blocks 0 and 1 are
    marked; even blocks j >= 2 point at (0, 0) and odd blocks j >= 3 at (0, 1)."""
    for m in (60, 121):
        T = b"ab" * m
        n = len(T)
        b1 = 1
        while b1 * 3 * 3 <= n:
            b1 *= 3
        t = oracle.build_tree(T, 3, 1, b1=b1)
        for L in t.levels[:-1]:
            assert L.marked[:2].tolist() == [1, 1] and not L.marked[2:].any()
            js = np.arange(2, L.c)
            assert L.ptr_block.tolist() == [0] * (L.c - 2)
            assert L.ptr_off.tolist() == [int(j % 2) for j in js]
        treecheck.check(treecheck.from_oracle(t), T)


@pytest.mark.parametrize("name", ["cfg1_16k", "markov", "random", "periodic"])
def test_invariants(name):
    T = {
        "cfg1_16k": lambda: synth.cfg1_text(1 << 14),
        "markov": lambda: synth.markov_versions(50000, 4096, 12, 2e-3, 32, 21),
        "random": lambda: synth.random_text(20000, 4, 8),
        "periodic": lambda: synth.periodic_text(30001, 97, 2),
    }[name]()
    T = bytes(T)
    for tau, leaf, s in ((2, 16, 1), (4, 16, 1), (3, 5, 1), (2, 8, 64)):
        t = oracle.build_tree(T, tau, leaf, s_hint=s)
        treecheck.check(treecheck.from_oracle(t), T)


def test_blocks_per_level_bound():
    """Section 4, lemma on blocks per level: c_l <= 3*z*tau for l >= 2, with z
    from a brute-force LZ77 parse."""
    rng = np.random.default_rng(5)
    texts = [synth.cfg1_text(1500, seed=3), bytes(b"abcab" * 100), synth.random_text(700, 2, 4)]
    for _ in range(20):
        texts.append(synth.markov_versions(int(rng.integers(50, 900)), 40, 8, 0.02, 4,
                                           int(rng.integers(1 << 30))))
    for T in texts:
        T = bytes(T)
        z = brute.lz77_z(T)
        for tau, leaf in ((2, 1), (3, 2), (4, 1)):
            t = oracle.build_tree(T, tau, leaf)
            for L in t.levels[1:]:
                assert L.c <= 3 * z * tau


def test_plan():
    """Level plan: b1 = leaf*tau^k with the largest k such that b1 <= n/s."""
    assert oracle.plan(1 << 20, 2, 16) == (1 << 20, 17)
    assert oracle.plan(1 << 28, 4, 16) == (1 << 28, 13)
    assert oracle.plan(1 << 31, 2, 16) == (1 << 31, 28)
    assert oracle.plan(1 << 20, 2, 16, s_hint=10000) == (64, 3)
    assert oracle.plan(10, 2, 16) == (16, 1)
    assert oracle.plan(0, 2, 16) == (16, 1)
    assert oracle.plan(100, 3, 2, root_block_len=54) == (54, 4)
    with pytest.raises(ValueError):
        oracle.plan(100, 3, 2, root_block_len=50)
    with pytest.raises(ValueError):
        oracle.plan(100, 1, 2)


def test_empty_and_tiny():
    t = oracle.build_tree(b"", 2, 16)
    assert t.h == 1 and t.levels[0].c == 0 and t.leaves.size == 0
    t = oracle.build_tree(b"x", 2, 1)
    assert t.h == 1 and t.leaves.tobytes() == b"x"


# ---- Karp-Rabin fingerprints (Section 2, phi; Section 5.3, the two update rules)

P = oracle.P61


def test_prefix_fp_definition():
    """P[e] - P[s]*x^(e-s) equals the defining sum of T[i]*x^(e-1-i) over the
    window, evaluated with Python integers."""
    rng = np.random.default_rng(1)
    for n in (1, 2, 17, 300):
        T = rng.integers(0, 256, n).astype(np.uint8)
        x = int(rng.integers(256, P - 1))
        Pa = oracle.prefix_fp(T, x)
        for _ in range(30):
            s = int(rng.integers(0, n))
            e = int(rng.integers(s, n + 1))
            want = sum(int(T[i]) * pow(x, e - 1 - i, P) for i in range(s, e)) % P
            got = (int(Pa[e]) - int(Pa[s]) * pow(x, e - s, P)) % P
            assert got == want
            assert oracle.window_fp(T, s, e - s, x) == want


def test_prefix_fp_geometric_closed_form():
    """A constant text c^n has P[n] = c*(x^n - 1)/(x - 1) mod p."""
    for c, n, x in ((1, 1000, 3), (200, 4097, 123456789012345), (255, 1, P - 2)):
        T = np.full(n, c, np.uint8)
        want = c * (pow(x, n, P) - 1) * pow(x - 1, P - 2, P) % P
        assert int(oracle.prefix_fp(T, x)[n]) == want


def test_rolling_identities():
    """The one-step roll (Section 5.3, conventional relation) and the 16-step
    jump used by the SIMD kernel (Section 5.3, first equation)."""
    rng = np.random.default_rng(2)
    T = rng.integers(0, 256, 500).astype(np.uint8)
    x = 0x1234567890ABCDE % P
    for L in (1, 5, 16, 40):
        for s in range(1, 500 - L - 16):
            e = s + L - 1
            f = oracle.window_fp(T, s, L, x)
            prev = oracle.window_fp(T, s - 1, L, x)
            assert f == (prev * x - int(T[s - 1]) * pow(x, L, P) + int(T[e])) % P
            if s >= 16 and L >= 16:
                back = oracle.window_fp(T, s - 16, L, x)
                head = oracle.window_fp(T, s - 16, 16, x)
                tail = oracle.window_fp(T, e - 15, 16, x)
                assert f == (back * pow(x, 16, P) - head * pow(x, L, P) + tail) % P
            if s > 60:
                break


# ---- counted-prefix queries (Section 1)

def test_rank_select_access_against_numpy():
    rng = np.random.default_rng(4)
    T = synth.cfg1_text(1 << 15)
    n = T.size
    pos = rng.integers(0, n + 1, 5000).astype(np.uint64)
    cs = rng.choice(np.frombuffer(b"ACGTZ", np.uint8), 5000)
    got = oracle.rank(T, cs, pos)
    for c in np.unique(cs):
        cum = np.concatenate([[0], np.cumsum(T == c)])
        sel = cs == c
        assert (got[sel] == cum[pos[sel].astype(np.int64)]).all()
    ks = rng.integers(0, 9000, 5000).astype(np.uint64)
    got = oracle.select(T, cs, ks)
    for c in np.unique(cs):
        where = np.flatnonzero(T == c)
        sel = np.flatnonzero(cs == c)
        for q in sel:
            k = int(ks[q])
            want = int(where[k - 1]) if 1 <= k <= where.size else 2**64 - 1
            assert int(got[q]) == want
    ap = rng.integers(0, n, 1000).astype(np.uint64)
    assert (oracle.access(T, ap) == T[ap.astype(np.int64)]).all()


# ---- optional pruning (Section 4.1)

def test_fig1_pruned_worked_example():
    """Section 4, Figure 1 as drawn: the pruned tree (the block "ra" at 8 is a
    pointer to block 1; 8 leaves)."""
    spec, rows, leaves = _load_fig1()
    T = spec["text"].encode()
    t = oracle.build_tree(T, int(spec["tau"]), int(spec["leaf"]), b1=int(spec["b1"]),
                          exact_split=False, prune=True)
    assert t.h == 3
    for (b, marked, ptr), L in zip(rows["pruned"], t.levels):
        assert L.b == b
        assert L.marked.tolist() == marked
        assert list(zip(L.ptr_block.tolist(), L.ptr_off.tolist())) == ptr
    assert t.leaves.tobytes() == leaves["pruned"]
    assert t.levels[-1].c == len(leaves["pruned"])
    treecheck.check_pruned(treecheck.from_oracle(t, exact_split=False), T)


def test_pruned_checker_rejects_unpruned_fig1():
    """The pruned-tree checker is not vacuous: the unpruned Figure 1 tree keeps
    a block that could be pruned."""
    spec, _, _ = _load_fig1()
    T = spec["text"].encode()
    t = oracle.build_tree(T, int(spec["tau"]), int(spec["leaf"]), b1=int(spec["b1"]), exact_split=False)
    with pytest.raises(AssertionError, match="Q3"):
        treecheck.check_pruned(treecheck.from_oracle(t, exact_split=False), T)


@pytest.mark.parametrize("sigma,nmax", [(2, 10), (3, 6)])
def test_pruned_exhaustive(sigma, nmax):
    """Every text over a tiny alphabet, tau in {2,3}, leaf in {1,2}, every b1:
    the pruned oracle tree satisfies the pruning characterisation (Q1-Q3) and
    still spells T."""
    alph = b"ab" if sigma == 2 else b"abc"
    cases = pruned = 0
    for n in range(1, nmax + 1):
        for word in itertools.product(alph, repeat=n):
            T = bytes(word)
            for tau in (2, 3):
                for leaf in (1, 2):
                    b1 = leaf
                    while True:
                        t = oracle.build_tree(T, tau, leaf, b1=b1, prune=True)
                        treecheck.check_pruned(treecheck.from_oracle(t), T)
                        u = oracle.build_tree(T, tau, leaf, b1=b1)
                        pruned += u.canonical != t.canonical
                        cases += 1
                        if b1 >= n:
                            break
                        b1 *= tau
    assert cases > 3000 and pruned > 100


def test_pruned_general_split_random():
    """ceil(b/tau) splits (Figure 1 style).  Such a split can leave a short
    block between full ones, so that an occurrence spans three blocks and the
    unpruned tree itself is not well formed; those draws are skipped."""
    rng = np.random.default_rng(12)
    done = 0
    for _ in range(400):
        n = int(rng.integers(1, 40))
        T = bytes(rng.integers(97, 97 + int(rng.integers(1, 4)), n).astype(np.uint8))
        tau = int(rng.integers(2, 5))
        leaf = int(rng.integers(1, 3))
        b1 = max(leaf, int(rng.integers(1, n + 1)))
        try:
            oracle.build_tree(T, tau, leaf, b1=b1, exact_split=False)
        except AssertionError:
            continue
        t = oracle.build_tree(T, tau, leaf, b1=b1, exact_split=False, prune=True)
        treecheck.check_pruned(treecheck.from_oracle(t, exact_split=False), T)
        done += 1
    assert done > 200


def test_pruned_unary_closed_form():
    """T = a^n: every pointer targets block 0 alone, so each level keeps only
    block 0 marked; levels below the first have tau blocks; tau*leaf leaf bytes."""
    for tau, leaf, n in ((2, 1, 200), (3, 2, 500), (4, 4, 1000), (2, 3, 97)):
        b1 = leaf
        while b1 * tau * 3 <= n:
            b1 *= tau
        T = b"a" * n
        t = oracle.build_tree(T, tau, leaf, b1=b1, prune=True)
        for li, L in enumerate(t.levels[:-1]):
            assert L.marked.tolist() == [1] + [0] * (L.c - 1)
            assert (L.ptr_block == 0).all() and (L.ptr_off == 0).all()
            assert L.c == (-(-n // b1) if li == 0 else tau)
        assert t.levels[-1].c == tau and t.leaves.tobytes() == b"a" * (tau * leaf)
        treecheck.check_pruned(treecheck.from_oracle(t), T)


def test_pruning_keeps_trees_without_earlier_copies():
    """All-distinct text: no block has an earlier occurrence.  (ab)^m with odd
    block lengths: block 1's only earlier copy overlaps it, and it is targeted.
    Pruning leaves both trees as they are."""
    rng = np.random.default_rng(3)
    T = bytes(rng.permutation(256)[:200].astype(np.uint8))
    for tau, leaf in ((2, 1), (3, 2)):
        assert oracle.build_tree(T, tau, leaf, prune=True).canonical == oracle.build_tree(T, tau, leaf).canonical
    T = b"ab" * 121
    b1 = 1
    while b1 * 9 <= len(T):
        b1 *= 3
    assert oracle.build_tree(T, 3, 1, b1=b1, prune=True).canonical == oracle.build_tree(T, 3, 1, b1=b1).canonical


@pytest.mark.parametrize("name", ["cfg1_8k", "markov", "random", "periodic"])
def test_pruned_invariants(name):
    T = {
        "cfg1_8k": lambda: synth.cfg1_text(1 << 13),
        "markov": lambda: synth.markov_versions(20000, 2048, 8, 2e-3, 32, 21),
        "random": lambda: synth.random_text(6000, 2, 8),
        "periodic": lambda: synth.periodic_text(9001, 97, 2),
    }[name]()
    T = bytes(T)
    for tau, leaf, s in ((2, 4, 1), (4, 4, 1), (3, 5, 1), (2, 8, 16)):
        t = oracle.build_tree(T, tau, leaf, s_hint=s, prune=True)
        u = oracle.build_tree(T, tau, leaf, s_hint=s)
        assert sum(L.c for L in t.levels) <= sum(L.c for L in u.levels)
        treecheck.check_pruned(treecheck.from_oracle(t), T)


def test_pruned_random_small():
    """Random texts of 8..200 bytes over 2-3 letters.  These reach the case the
    exhaustive tiny texts miss: a child kept marked because a pointer targets
    it through an occurrence that crosses its parent's right end, which must
    keep the parent marked too."""
    rng = np.random.default_rng(1)
    for _ in range(150):
        n = int(rng.integers(8, 200))
        T = bytes(rng.integers(97, 97 + int(rng.integers(2, 4)), n).astype(np.uint8))
        for tau, leaf in ((2, 1), (3, 1), (2, 2)):
            t = oracle.build_tree(T, tau, leaf, prune=True)
            treecheck.check_pruned(treecheck.from_oracle(t), T)


def _decode_canonical(buf):
    """Read canonical tree bytes field by field, following the layout the C ABI
    documents for bt_serialize (little-endian):
      "BTv1", u64 n, u32 tau, u32 leaf_len, u64 b1, u32 h, u32 0,
      per level l < h: u64 b, u64 c, ceil(c/64) u64 mark words (bit j%64 of word
        j/64 is block j, pad bits zero), u64 u, u64 ptr_block[u], u64 ptr_off[u];
      level h: u64 b, u64 c, u64 leaf byte count, the leaf bytes, zeros to a
        multiple of 8."""
    import struct
    at = 0

    def take(fmt):
        nonlocal at
        v = struct.unpack_from("<" + fmt, buf, at)
        at += struct.calcsize("<" + fmt)
        return v

    assert buf[:4] == b"BTv1"
    at = 4
    n, tau, leaf, b1, h, zero = take("QIIQII")
    assert zero == 0
    levels = []
    for _ in range(h - 1):
        b, c = take("QQ")
        words = take("%dQ" % ((c + 63) // 64)) if c else ()
        marked = [(words[j // 64] >> (j % 64)) & 1 for j in range(c)]
        used = c - 64 * (len(words) - 1)          # bits used in the last word
        if words and used < 64:
            assert words[-1] >> used == 0, "pad bits set"
        (u,) = take("Q")
        pb = list(take("%dQ" % u)) if u else []
        po = list(take("%dQ" % u)) if u else []
        levels.append((b, c, marked, pb, po))
    b, c, nb = take("QQQ")
    leaves = bytes(buf[at:at + nb])
    at += nb
    pad = (8 - nb % 8) % 8
    assert buf[at:at + pad] == b"\0" * pad
    at += pad
    assert at == len(buf), "trailing bytes"
    return (n, tau, leaf, b1, h), levels, (b, c), leaves


def test_canonical_layout_fig1():
    """The canonical bytes of Figure 1's trees (Section 4), decoded field by field
    against the documented layout, hold exactly the fixture's rows; the total
    size is the sum of the documented field sizes."""
    spec, rows, leaves = _load_fig1()
    T = spec["text"].encode()
    for kind, prune in (("unpruned", False), ("pruned", True)):
        t = oracle.build_tree(T, int(spec["tau"]), int(spec["leaf"]), b1=int(spec["b1"]),
                              exact_split=False, prune=prune)
        head, levels, last, lv = _decode_canonical(t.canonical)
        assert head == (12, 3, 1, 6, 3)
        assert len(levels) == 2
        for (b, c, marked, pb, po), (rb, rmarked, rptr) in zip(levels, rows[kind]):
            assert b == rb and c == len(rmarked) and marked == rmarked
            assert list(zip(pb, po)) == rptr
        assert last == (1, len(leaves[kind])) and lv == leaves[kind]
        # header 36, level 1: b c word u = 32, level 2: 24 + 8 + 8 + 16 u
        size = 36 + 32 + (32 + 16 * len(rows[kind][1][2])) + 24 + len(lv) + (8 - len(lv) % 8) % 8
        assert len(t.canonical) == size


def test_canonical_layout_multiword():
    """A tree with more than 64 blocks on a level: mark words split at bit 64,
    pointer arrays in block order, pad bits zero."""
    T = synth.cfg1_text(1 << 14)
    t = oracle.build_tree(T, 2, 16, s_hint=100)
    head, levels, last, lv = _decode_canonical(t.canonical)
    assert head == (t.n, 2, 16, t.b1, t.h)
    assert any(c > 64 for _, c, _, _, _ in levels)
    for (b, c, marked, pb, po), L in zip(levels, t.levels):
        assert (b, c) == (L.b, L.c) and marked == L.marked.tolist()
        assert pb == L.ptr_block.tolist() and po == L.ptr_off.tolist()
    assert lv == t.leaves.tobytes()


@pytest.mark.parametrize("s_hint", [1, 64])
def test_literal_double_loop_16k(s_hint):
    """The literal double loop (no library search) on the first 16 KiB of the
    1 MiB DNA text gives the same tree as memmem."""
    T = synth.cfg1_text()[:1 << 14]
    a = oracle.build_tree(T, 2, 16, s_hint=s_hint, search=oracle.SEARCH_NAIVE)
    b = oracle.build_tree(T, 2, 16, s_hint=s_hint, search=oracle.SEARCH_MEMMEM)
    assert a.canonical == b.canonical
