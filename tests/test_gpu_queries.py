"""Batched access/rank/select against counted prefixes (the query definitions
of Section 1), on single and batched trees, including the edges i = 0, i = n,
k = count, k = count + 1, out-of-range positions and absent symbols."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu
U64MAX = 2**64 - 1


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    import paper_2512_23314_amd as bt
    c = bt.Context(0)
    yield c
    c.close()


def _dev_u64(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64)).to("cuda:0").view(torch.uint64)


def _check_queries(tree, T, seed, m=20000):
    T = np.asarray(T, np.uint8)
    n = T.size
    rng = np.random.default_rng(seed)
    alph = np.unique(T) if n else np.zeros(0, np.uint8)
    extra = np.array([0, 255, 200], np.uint8)
    cand = np.concatenate([alph, extra])
    cs = rng.choice(cand, m).astype(np.uint8)
    pos = rng.integers(0, n + 1, m).astype(np.uint64)
    pos[:4] = [0, n, n + 1, n + 7]
    counts = {int(c): int((T == c).sum()) for c in cand}
    ks = np.array([rng.integers(0, counts[int(c)] + 3) for c in cs], np.uint64)
    for q in range(min(len(alph), 8)):
        cs[4 + 2 * q] = alph[q]
        ks[4 + 2 * q] = counts[int(alph[q])]
        cs[5 + 2 * q] = alph[q]
        ks[5 + 2 * q] = counts[int(alph[q])] + 1
    dc = to_device(cs)
    got_r = tree.rank(dc, _dev_u64(pos)).cpu().numpy()
    want_r = oracle.rank(T, cs, pos)
    bad = np.flatnonzero(got_r != want_r)
    assert bad.size == 0, "rank differs at %s: got %s want %s" % (
        bad[:5].tolist(), got_r[bad[:5]].tolist(), want_r[bad[:5]].tolist())
    got_s = tree.select(dc, _dev_u64(ks)).cpu().numpy()
    want_s = oracle.select(T, cs, ks)
    bad = np.flatnonzero(got_s != want_s)
    assert bad.size == 0, "select differs at %s: got %s want %s (c=%s k=%s)" % (
        bad[:5].tolist(), got_s[bad[:5]].tolist(), want_s[bad[:5]].tolist(),
        cs[bad[:5]].tolist(), ks[bad[:5]].tolist())
    if n:
        ap = rng.integers(0, n, m).astype(np.uint64)
        assert np.array_equal(tree.access(_dev_u64(ap)).cpu().numpy(), oracle.access(T, ap))


TEXTS = [
    ("cfg1_64k", lambda: synth.cfg1_text(1 << 16), 2, 16),
    ("markov", lambda: synth.markov_versions(200003, 8192, 25, 2e-3, 32, 3), 4, 16),
    ("random", lambda: synth.random_text(50001, 4, 9), 3, 4),
    ("periodic", lambda: synth.periodic_text(40000, 13, 5), 2, 8),
    ("unary", lambda: np.full(30000, 66, np.uint8), 2, 16),
    ("bytes256", lambda: synth.random_text(70000, 256, 2), 4, 8),
    ("short", lambda: synth.random_text(10, 4, 2), 2, 16),
]


@pytest.mark.parametrize("name,gen,tau,leaf", TEXTS, ids=[t[0] for t in TEXTS])
def test_queries_single(ctx, name, gen, tau, leaf):
    T = gen()
    tree = ctx.build(to_device(T), tau=tau, leaf_len=leaf, rank_select=True)
    _check_queries(tree, T, len(T))


def test_queries_mode_b(ctx):
    T = synth.cfg1_text(1 << 17)
    tree = ctx.build(to_device(T), tau=2, leaf_len=16, s_hint=2000, rank_select=True)
    _check_queries(tree, T, 11)


def test_queries_batch(ctx):
    texts = [synth.cfg1_text(n, seed=n) if n else np.zeros(0, np.uint8)
             for n in (0, 1, 100, 4096, 30000, 70001)]
    texts.append(synth.random_text(5000, 256, 1))
    offs = [0]
    for T in texts:
        offs.append(offs[-1] + len(T))
    concat = np.concatenate(texts)
    trees = ctx.build_batch(to_device(concat), offs, tau=4, leaf_len=8, rank_select=True)
    for k, (T, tr) in enumerate(zip(texts, trees)):
        _check_queries(tr, T, 100 + k, m=3000)


def test_rank_needs_support(ctx):
    import paper_2512_23314_amd as bt
    T = synth.random_text(1000, 4, 1)
    tree = ctx.build(to_device(T), tau=2, leaf_len=16)
    with pytest.raises(bt.BtError):
        tree.rank(to_device(np.array([65], np.uint8)), _dev_u64([3]))


def _dense_support_bytes(tree, S):
    """What 32-bit counters for every block and every pointer would take (the
    uncompacted form), plus the same block starts."""
    tot = 0
    for l in range(1, tree.height + 1):
        _, c, u = tree.level_info(l)
        tot += 4 * S * (c + u) + 8 * c
    return tot


@pytest.mark.parametrize("tau,leaf", [(4, 16), (2, 8), (8, 4)])
def test_queries_counter_widths(ctx, tau, leaf):
    """A 3 MiB versioned text (sigma 96): its levels span 32-bit absolute
    counters (long blocks), 16-bit and 8-bit relative ones, and 8/16/32-bit
    pointer counts; queries walk up the parents through all of them.  The
    support takes well under half of the 32-bit form."""
    T = synth.cfg2_text()[: 3 << 20].copy()
    tree = ctx.build(to_device(T), sigma=96, tau=tau, leaf_len=leaf, rank_select=True)
    _check_queries(tree, T, tau * 100 + leaf, m=40000)
    S = int(np.unique(T).size)
    rb = tree.rank_bytes()
    assert 0 < rb <= 0.5 * _dense_support_bytes(tree, S), (rb, _dense_support_bytes(tree, S))
    plain = ctx.build(to_device(T), sigma=96, tau=tau, leaf_len=leaf)
    assert plain.rank_bytes() == 0
    assert plain.serialize() == tree.serialize()
