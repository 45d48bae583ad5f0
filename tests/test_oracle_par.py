"""Pins for the threaded oracle construction (``oracle.build_tree_par``: the
paper's two-phase method over a domain decomposition, Section 4.1, Section 5.2,
Section 5.4): it must give the same canonical bytes as the plain definition
(``oracle.build_tree``, leftmost occurrences by direct search) on every input the
definition can finish, for any thread count, Karp-Rabin base, and with
fingerprints cut to a few bits so that collisions are everywhere.  CPU only.

The full-size expected trees in tests/golden/fullsize_trees.json are written by
tests/golden/make_fullsize.py with this construction."""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth

Q = 2**64 - 2**32 + 1


def _same(T, tau, leaf, b1=None, s_hint=1, **kw):
    want = oracle.build_tree(T, tau, leaf, b1=b1, s_hint=s_hint).canonical
    got = oracle.build_tree_par(T, tau, leaf, b1=b1, s_hint=s_hint, levels=False, **kw).canonical
    assert got == want, (len(T), tau, leaf, b1, s_hint, kw)


def test_window_fingerprint_definition():
    """phi(i, L) = sum_k T[i+k] r^(L-1-k) mod q (Section 2), against Python
    integers, for windows crossing many bytes and bases near q."""
    rng = np.random.default_rng(1)
    T = rng.integers(0, 256, 5000).astype(np.uint8)
    for base in (2, 33, oracle.PAR_BASE, Q - 1, Q - 2, 2**63 + 12345):
        for i, L in ((0, 1), (3, 17), (100, 999), (0, 5000), (4999, 1)):
            want = 0
            for k in range(L):
                want = (want * (base % Q) + int(T[i + k])) % Q
            assert oracle.par_window_fp(T, i, L, base) == want


@pytest.mark.parametrize("sigma,nmax", [(2, 10), (3, 6)])
def test_exhaustive_tiny_texts(sigma, nmax):
    """Every text over a tiny alphabet, tau in {2,3}, leaf in {1,2}, every b1:
    one thread with full fingerprints, and three threads with 3-bit
    fingerprints (every window collides with some key)."""
    alph = b"ab" if sigma == 2 else b"abc"
    cases = 0
    for n in range(1, nmax + 1):
        for word in itertools.product(alph, repeat=n):
            T = bytes(word)
            for tau in (2, 3):
                for leaf in (1, 2):
                    b1 = leaf
                    while True:
                        want = oracle.build_tree(T, tau, leaf, b1=b1).canonical
                        a = oracle.build_tree_par(T, tau, leaf, b1=b1, threads=1, levels=False)
                        b = oracle.build_tree_par(T, tau, leaf, b1=b1, threads=3, fp_bits=3,
                                                  levels=False)
                        assert a.canonical == want and b.canonical == want, (T, tau, leaf, b1)
                        cases += 1
                        if b1 >= n:
                            break
                        b1 *= tau
    assert cases > 3000


def test_closed_forms_and_edges():
    """Unary, all-distinct and period-2 texts (pinned in closed form for the
    plain definition), empty and sub-leaf texts, ragged tails."""
    texts = [b"a" * 1000, bytes(range(256)), b"ab" * 300, b"", b"x", b"xyz",
             synth.random_text(4097, 4, 2).tobytes(), synth.periodic_text(3001, 5, 3).tobytes()]
    for T in texts:
        for tau, leaf in ((2, 1), (3, 2), (4, 4), (2, 16)):
            _same(T, tau, leaf)
            _same(T, tau, leaf, threads=5, fp_bits=5)


@pytest.mark.parametrize("mode", ["A", "B"])
def test_dna_1mib(mode):
    """The 1 MiB DNA text, one root block (mode A) and s near z (mode B)."""
    T = synth.cfg1_text()
    s_hint = 1 if mode == "A" else 10000
    _same(T, 2, 16, s_hint=s_hint)
    _same(T, 2, 16, s_hint=s_hint, threads=2, base=12345)


def test_versioned_prefix():
    """The first 4 MiB of the 256 MiB versioned text (sigma 96, tau 4, leaf 16):
    ten levels, the same recipe as the full-size workload."""
    T = synth.cfg2_text()[:1 << 22]
    _same(T, 4, 16)


def test_haplotype_recipe():
    """The 2 GiB haplotype recipe scaled to 2 MiB (a 64 KiB reference, 32
    haplotypes, 0.1% SNPs, 0.01% indels of length 1-20), for the tau and leaf
    values of the full-size sweep."""
    T = synth.dna_copies(1 << 21, 64 << 10, 32, 1e-3, 1e-4, 20, 0x5EED0003)
    for tau, leaf in ((4, 16), (2, 8), (8, 32), (16, 16)):
        _same(T, tau, leaf)


def test_batch_texts():
    """Texts of the 4096-text batch: the shortest ones, and some of median size."""
    lens = np.array(synth.batch_lengths_of())
    order = np.argsort(lens, kind="stable")
    pick = list(order[:6]) + list(order[len(order) // 2:len(order) // 2 + 3])
    for i in pick:
        T = synth.batch_text(int(i))
        _same(T, 4, 16)
        _same(T, 4, 16, threads=4, fp_bits=10)


def test_forced_collisions():
    """Fingerprints cut to 6-16 bits on repetitive texts with many keys: every
    collision must be rejected by byte comparison."""
    texts = [synth.cfg1_text(1 << 16), synth.markov_versions(1 << 16, 2048, 32, 5e-3, 16, 4)]
    for T in texts:
        for bits in (6, 10, 16):
            _same(T, 2, 4, fp_bits=bits, threads=3)
            _same(T, 4, 16, fp_bits=bits, threads=8)


def test_thread_counts():
    """1 to 16 threads, more threads than windows included."""
    T = synth.cfg1_text(1 << 17)
    want = oracle.build_tree(T, 2, 16).canonical
    for k in (1, 2, 3, 7, 8, 16):
        assert oracle.build_tree_par(T, 2, 16, threads=k, levels=False).canonical == want
    tiny = b"abracadabra"
    want = oracle.build_tree(tiny, 2, 1).canonical
    assert oracle.build_tree_par(tiny, 2, 1, threads=64, levels=False).canonical == want


def test_level_arrays():
    """Level arrays (not only the canonical bytes) equal the definition's."""
    T = synth.cfg1_text(1 << 16)
    a = oracle.build_tree(T, 2, 8)
    b = oracle.build_tree_par(T, 2, 8, threads=3)
    assert a.h == b.h
    for x, y in zip(a.levels, b.levels):
        assert np.array_equal(x.start, y.start) and np.array_equal(x.marked, y.marked)
        assert np.array_equal(x.ptr_block, y.ptr_block) and np.array_equal(x.ptr_off, y.ptr_off)
    assert np.array_equal(a.leaves, b.leaves)


def test_invalid_parameters():
    with pytest.raises(ValueError):
        oracle.build_tree_par(b"abc", 1, 1)
    with pytest.raises(ValueError):
        oracle.build_tree_par(b"abcdef", 2, 2, b1=6)          # not leaf * tau^k
    with pytest.raises(ValueError):
        oracle.build_tree_par(b"abc", 2, 1, threads=0)


@pytest.mark.skipif(os.environ.get("BT_LARGE_PINS") != "1",
                    reason="8 MiB plain-definition builds take minutes; set BT_LARGE_PINS=1")
def test_large_prefixes():
    """8 MiB: the versioned text's prefix, and the haplotype recipe with a
    256 KiB reference (32 haplotypes)."""
    _same(synth.cfg2_text()[:1 << 23], 4, 16)
    T = synth.dna_copies(1 << 23, 256 << 10, 32, 1e-3, 1e-4, 20, 77)
    _same(T, 4, 16)
    _same(T, 2, 8)
