"""GPU parity: the HIP pipeline (through the C ABI) against the CPU oracle,
element by element, on seeded synthetic texts that span several tiles and end
in ragged tails; plus edge cases and hash-independence."""
import numpy as np
import pytest

import oracle
import synth
from tests import hashref, treecheck
from tests.gpu_util import assert_same_tree, shape_of, to_device, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    import paper_2512_23314_amd as bt
    c = bt.Context(0)
    yield c
    c.close()


def _build(ctx, T, tau, leaf, sigma=256, **kw):
    d = to_device(T)
    return ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, **kw)


# ---- step a2: prefix fingerprints

# sizes around a thread's 64 bytes, a row of the output pass (8 KiB), a 32 KiB
# tile, and enough tiles for the look-back to cross more than one window of 64
@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 4095, 4096, 4097, 12289, 16383, 16384, 16385,
                               32767, 32768, 32769, 65536 * 3 + 7, (1 << 20) + 13, (5 << 20) + 1])
def test_prefix_fingerprints(ctx, n):
    rng = np.random.default_rng(n + 1)
    T = rng.integers(0, 256, n).astype(np.uint8)
    x = int(rng.integers(256, oracle.P61 - 1))
    got = ctx.prefix_fingerprints(to_device(T), x).cpu().numpy()
    assert np.array_equal(got, oracle.prefix_fp(T, x))


def test_prefix_fingerprints_unaligned_view(ctx):
    torch = torch_cuda()
    T = np.random.default_rng(3).integers(0, 256, 50001).astype(np.uint8)
    d = to_device(T)
    for off in (1, 3, 8, 13):
        x = 1234567 + off
        got = ctx.prefix_fingerprints(d[off:], x).cpu().numpy()
        assert np.array_equal(got, oracle.prefix_fp(T[off:], x))
    del torch


def test_prefix_fingerprints_misaligned_output(ctx):
    """An output view 8 bytes off a 16-byte boundary takes single-word stores."""
    torch = torch_cuda()
    T = np.random.default_rng(5).integers(0, 256, 40003).astype(np.uint8)
    buf = torch.zeros(len(T) + 2, dtype=torch.uint64, device="cuda:0")
    got = ctx.prefix_fingerprints(to_device(T), 987654321, out=buf[1:]).cpu().numpy()
    assert np.array_equal(got, oracle.prefix_fp(T, 987654321))
    assert int(buf[0]) == 0


# both prefix arrays in one pass (the builds' form): dense or sampled
# fingerprints, and the 32-bit hashes against their recurrence (sampled too
# in the memory-lean form, sampled=2)
@pytest.mark.parametrize("sampled", [0, 1, 2], ids=["dense", "sampled", "both_sampled"])
@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 63, 64, 65, 4095, 8191, 8192, 16385, 32767, 32768,
                               32769, 65536 * 3 + 7, (5 << 20) + 1])
def test_prefix_scan(ctx, n, sampled):
    rng = np.random.default_rng(n + 7)
    T = rng.integers(0, 256, n).astype(np.uint8)
    x = int(rng.integers(256, oracle.P61 - 1))
    x32 = int(rng.integers(0, 1 << 31)) * 2 + 1
    P, H = ctx.prefix_scan(to_device(T), x, x32, sampled=sampled)
    want = oracle.prefix_fp(T, x)
    assert np.array_equal(P.cpu().numpy(), want[::16] if sampled else want)
    h = hashref.h32(T, x32)
    assert np.array_equal(H.cpu().numpy().view(np.uint32), h[::16] if sampled == 2 else h)


def test_prefix_scan_unaligned_views(ctx):
    T = np.random.default_rng(8).integers(0, 256, 70001).astype(np.uint8)
    d = to_device(T)
    for off in (1, 3, 8, 13):
        for sampled in (0, 1, 2):
            P, H = ctx.prefix_scan(d[off:], 1234567 + off, 0x9E3779B1, sampled=sampled)
            want = oracle.prefix_fp(T[off:], 1234567 + off)
            assert np.array_equal(P.cpu().numpy(), want[::16] if sampled else want)
            h = hashref.h32(T[off:], 0x9E3779B1)
            assert np.array_equal(H.cpu().numpy().view(np.uint32), h[::16] if sampled == 2 else h)


# ---- whole builds against the oracle

CASES = [
    ("cfg1_16k", lambda: synth.cfg1_text(1 << 14), [(2, 16, 1), (2, 16, 64), (4, 4, 1)]),
    ("random4_ragged", lambda: synth.random_text(100003, 4, 7), [(2, 16, 1), (3, 4, 1), (4, 1, 1)]),
    ("markov_versions", lambda: synth.markov_versions(300007, 8192, 40, 2e-3, 32, 17),
     [(4, 16, 1), (2, 8, 1), (4, 16, 256)]),
    ("periodic", lambda: synth.periodic_text(70001, 89, 3), [(2, 16, 1), (3, 2, 1)]),
    ("unary", lambda: np.full(50000, 65, np.uint8), [(2, 16, 1), (4, 3, 1)]),
    ("dna_copies_tiny", lambda: synth.dna_copies(5000, 300, 20, 0.01, 0.002, 4, 9), [(2, 1, 1), (3, 2, 1)]),
]


@pytest.mark.parametrize("name,gen,params", CASES, ids=[c[0] for c in CASES])
def test_build_matches_oracle(ctx, name, gen, params):
    T = gen()
    for tau, leaf, s in params:
        ora = oracle.build_tree(T, tau, leaf, s_hint=s)
        tree = _build(ctx, T, tau, leaf, s_hint=s)
        assert_same_tree(tree, ora)
        if len(T) <= 100003:
            treecheck.check(shape_of(tree, tau, leaf), bytes(T), max_leftmost=2000)


def test_cfg1_full_mode_a_and_b(ctx):
    """1 MiB DNA copies, tau=2, leaf=16: one root block (mode A) and s close to
    the text's phrase count (mode B)."""
    T = synth.cfg1_text()
    for s in (1, 10000):
        ora = oracle.build_tree(T, 2, 16, s_hint=s)
        tree = _build(ctx, T, 2, 16, s_hint=s)
        assert_same_tree(tree, ora)


def test_hash_independence_and_weak_hash(ctx):
    """Two seeds and 12-bit fingerprints (forced collisions) give the same bytes."""
    import paper_2512_23314_amd as bt
    for T in (synth.cfg1_text(1 << 13), synth.markov_versions(20000, 2000, 10, 5e-3, 16, 5),
              synth.random_text(9000, 2, 4)):
        ref = oracle.build_tree(T, 2, 4).canonical
        for seed in (1, 0xDEADBEEF):
            assert _build(ctx, T, 2, 4, hash_seed=seed).serialize() == ref
        assert _build(ctx, T, 2, 4, debug_flags=bt.BT_DBG_WEAK_HASH).serialize() == ref
        # the unqueued 61-bit scan (taken only past the queue's packing limits)
        assert _build(ctx, T, 2, 4, debug_flags=bt.BT_DBG_NO_QUEUE).serialize() == ref
        assert _build(ctx, T, 2, 4,
                      debug_flags=bt.BT_DBG_NO_QUEUE | bt.BT_DBG_WEAK_HASH).serialize() == ref
        # the hash pre-filter where the byte scan would be taken, and the byte
        # scan with forced collisions
        assert _build(ctx, T, 2, 4, debug_flags=bt.BT_DBG_NO_BYTE_SCAN).serialize() == ref
        assert _build(ctx, T, 2, 16, debug_flags=bt.BT_DBG_WEAK_HASH).serialize() == \
            oracle.build_tree(T, 2, 16).canonical


@pytest.mark.parametrize("n,tau,leaf", [(0, 2, 16), (1, 2, 16), (15, 2, 16), (16, 2, 16),
                                        (17, 2, 16), (33, 2, 16), (2, 2, 1), (100, 3, 7)])
def test_edge_sizes(ctx, n, tau, leaf):
    T = synth.random_text(n, 3, n + 5)
    ora = oracle.build_tree(T, tau, leaf)
    if n == 0:
        import paper_2512_23314_amd as bt
        torch = torch_cuda()
        d = torch.zeros(1, dtype=torch.uint8, device="cuda:0")[:0]
        tree = ctx.build(d, tau=tau, leaf_len=leaf)
    else:
        tree = _build(ctx, T, tau, leaf)
    assert_same_tree(tree, ora)


def test_build_from_unaligned_views(ctx):
    """Texts that start 1..3 bytes past a 4-byte boundary: the byte scan reads
    aligned words around each lane's windows."""
    T = synth.markov_versions(200003, 8192, 20, 2e-3, 32, 23)
    d = to_device(T)
    for off in (1, 2, 3, 5):
        for tau, leaf in ((4, 16), (2, 8)):
            tree = ctx.build(d[off:], tau=tau, leaf_len=leaf)
            assert tree.serialize() == oracle.build_tree(T[off:], tau, leaf).canonical


def test_root_block_len_override(ctx):
    T = synth.cfg1_text(1 << 15)
    ora = oracle.build_tree(T, 2, 16, b1=1024)
    tree = _build(ctx, T, 2, 16, root_block_len=1024)
    assert_same_tree(tree, ora)


def test_invalid_params(ctx):
    import paper_2512_23314_amd as bt
    d = to_device(synth.random_text(1000, 4, 1))
    for kw in (dict(tau=1, leaf_len=16), dict(tau=2, leaf_len=0), dict(tau=2, leaf_len=16, root_block_len=100),
               dict(tau=2, leaf_len=16, sigma=0), dict(tau=2, leaf_len=16, sigma=300)):
        with pytest.raises(bt.BtError) as e:
            ctx.build(d, **kw)
        assert e.value.code == bt.BT_E_INVAL
    # more distinct bytes than sigma
    with pytest.raises(bt.BtError) as e:
        ctx.build(d, sigma=3, tau=2, leaf_len=16)
    assert e.value.code == bt.BT_E_INVAL


def test_access_reconstructs_text(ctx):
    torch = torch_cuda()
    for T, tau, leaf in ((synth.cfg1_text(1 << 16), 2, 16), (synth.random_text(77777, 4, 2), 3, 5),
                         (synth.markov_versions(120001, 4096, 30, 2e-3, 16, 8), 4, 16)):
        d = to_device(T)
        tree = ctx.build(d, tau=tau, leaf_len=leaf)
        pos = torch.arange(len(T), dtype=torch.int64, device="cuda:0").to(torch.uint64)
        got = tree.access(pos).cpu().numpy()
        assert np.array_equal(got, np.asarray(T, np.uint8))
