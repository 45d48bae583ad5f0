"""The 256 MiB versioned-text workload (sigma 96, tau 4, leaf 16, one root
block), built exactly as the benchmark builds it.  The oracle cannot build a
tree of this size, so the full tree is checked through properties that hold at
any size, plus exact oracle answers on samples:
  - access over every position reconstructs the text;
  - every pointer targets a marked block (and a marked consecutive successor
    when its source spills over), and its source ends before its block;
  - level sizes follow from the marks;
  - sampled pointers: the source equals the block and is its leftmost
    occurrence (direct search in the text);
  - sampled consecutive pairs: marked when and only when leftmost;
and the tree of the text's first 4 MiB equals the oracle's tree exactly."""
import numpy as np
import pytest

import oracle
import synth
from tests import treecheck
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu
TAU, LEAF, SIGMA = 4, 16, 96


@pytest.fixture(scope="module")
def built():
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    T = synth.cfg2_text()
    ctx = bt.Context(0)
    d = torch.from_numpy(T).to("cuda:0")
    tree = ctx.build(d, sigma=SIGMA, tau=TAU, leaf_len=LEAF)
    yield T, d, ctx, tree
    tree.free()
    ctx.close()


def test_access_reconstructs_all(built):
    torch = torch_cuda()
    T, d, ctx, tree = built
    n = T.size
    step = 1 << 24
    for a in range(0, n, step):
        pos = torch.arange(a, min(n, a + step), device="cuda:0", dtype=torch.int64).to(torch.uint64)
        got = tree.access(pos)
        assert bool((got == d[a:a + step]).all()), "access differs in [%d, %d)" % (a, a + step)


def test_structure_and_sampled_leftmost(built):
    T, d, ctx, tree = built
    s = treecheck.Shape(tree.n, TAU, LEAF, tree.b1,
                        [tree.level(l) for l in range(1, tree.height)] +
                        [(tree.level_info(tree.height)[0],
                          np.zeros(tree.level_info(tree.height)[1], np.uint8), None, None)],
                        b"")
    lay = treecheck.block_layout(s)
    Tb = T.tobytes()
    rng = np.random.default_rng(7)
    checked_ptr = checked_pair = 0
    for li in range(tree.height - 1):
        b, marked, pb, po = s.levels[li]
        st, ln = lay[li]
        c = st.size
        m = marked.astype(bool)
        assert m[0]
        adj = np.zeros(c, bool)
        adj[:-1] = st[1:] == st[:-1] + ln[:-1]
        um = np.flatnonzero(~m)
        assert um.size == pb.size
        if um.size:
            t = pb.astype(np.int64)
            off = po.astype(np.int64)
            assert (t < c).all() and m[t].all(), "a pointer targets an unmarked block"
            assert (off < ln[t]).all()
            L = ln[um]
            spill = off + L > ln[t]
            if spill.any():
                ts = t[spill]
                assert (ts + 1 < c).all() and adj[ts].all() and m[ts + 1].all()
            src = st[t] + off
            assert (src + L <= st[um]).all(), "a source overlaps its block"
            for k in rng.choice(um.size, min(12, um.size), replace=False):
                j, p, l = int(um[k]), int(src[k]), int(L[k])
                a = int(st[j])
                assert Tb[p:p + l] == Tb[a:a + l]
                assert Tb.find(Tb[a:a + l], 0, p + l) == p
                checked_ptr += 1
        pairs = np.flatnonzero(adj)
        for j in rng.choice(pairs, min(8, pairs.size), replace=False) if pairs.size else []:
            a, l = int(st[j]), int(ln[j] + ln[j + 1])
            if Tb.find(Tb[a:a + l], 0, a + l) == a:
                assert m[j] and m[j + 1]
            checked_pair += 1
    assert checked_ptr > 20 and checked_pair > 20


def test_prefix_4mib_matches_oracle(built):
    import paper_2512_23314_amd as bt
    T, d, ctx, tree = built
    S = T[:4 << 20]
    ora = oracle.build_tree(S, TAU, LEAF)
    got = ctx.build(d[:4 << 20], sigma=SIGMA, tau=TAU, leaf_len=LEAF)
    assert got.serialize() == ora.canonical
