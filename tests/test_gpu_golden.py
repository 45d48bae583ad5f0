"""Full-size parity: the GPU's trees of the full-size workloads against the trees
the threaded oracle construction built on the host (the paper's two-phase
method, pinned to the plain definition in tests/test_oracle_par.py).  The
expected values are SHA-256 digests of the canonical tree bytes, written by
tests/golden/make_fullsize.py into tests/golden/fullsize_trees.json and
tests/golden/batch4096_trees.txt.  Each test first checks that the regenerated
input has the recorded SHA-256, then that every tree is byte-for-byte the
oracle's, in the launch configuration the benchmark times."""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
with open(os.path.join(GOLDEN, "fullsize_trees.json")) as _f:
    GOLD = json.load(_f)["entries"]

DNA2G = sorted(k for k in GOLD if k.startswith("dna2g"))


def _entry(name):
    if name not in GOLD:
        pytest.skip("no expected tree recorded for %s" % name)
    return GOLD[name]


def _sha(b):
    return hashlib.sha256(b).hexdigest()


def _check_single(T, e, sigma, **kw):
    import paper_2512_23314_amd as bt
    assert T.size == e["n"]
    assert _sha(T.tobytes()) == e["input_sha256"], "regenerated input differs from the recorded one"
    ctx = bt.Context(0)
    try:
        d = to_device(T)
        tree = ctx.build(d, sigma=sigma, tau=e["tau"], leaf_len=e["leaf_len"], s_hint=e["s_hint"], **kw)
        try:
            assert tree.b1 == e["b1"] and tree.height == e["h"]
            got = [list(tree.level_info(l)) for l in range(1, tree.height + 1)]
            assert got == e["levels_b_c_u"], "level sizes differ from the oracle's"
            can = tree.serialize()
            assert len(can) == e["canonical_bytes"]
            assert _sha(can) == e["canonical_sha256"], "tree bytes differ from the oracle's"
        finally:
            tree.free()
        del d
    finally:
        ctx.close()


def test_versioned256m():
    """256 MiB versioned text (sigma 96, tau 4, leaf 16, one root block): the
    benchmark's build, and the same tree with rank/select support (bt_build's
    configuration) and with sampled prefix fingerprints."""
    torch_cuda()
    e = _entry("versioned256m")
    T = synth.cfg2_text()
    _check_single(T, e, 96)
    _check_single(T, e, 96, rank_select=True)
    _check_single(T, e, 96, lean=True)


@pytest.mark.parametrize("name", DNA2G or ["dna2g_t4_l16"])
def test_dna2g(name):
    """2 GiB haplotype collection (sigma 4) at each recorded (tau, leaf) point
    of the sweep."""
    torch_cuda()
    e = _entry(name)
    T = _dna2g()
    _check_single(T, e, 4)
    if name == "dna2g_t4_l16":
        _check_single(T, e, 4, lean=True)


_DNA = {}


def _dna2g():
    if "T" not in _DNA:
        _DNA["T"] = synth.cfg3_text()
    return _DNA["T"]


def test_batch4096():
    """All 4096 texts of the batch (about 3.9 GiB) in one bt_build_batch call:
    every tree equals the oracle's."""
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    e = _entry("batch4096")
    want = {}
    with open(os.path.join(GOLDEN, e["per_text"])) as f:
        for line in f:
            if line.startswith("#"):
                continue
            i, n, h = line.split()
            want[int(i)] = (int(n), h)
    texts = synth.batch_texts()
    assert len(texts) == e["texts"] == len(want)
    insha = [_sha(t.tobytes()) for t in texts]
    assert _sha("".join(insha).encode()) == e["input_digest"], "regenerated inputs differ"
    offs = np.zeros(len(texts) + 1, np.uint64)
    offs[1:] = np.cumsum([t.size for t in texts])
    d = torch.from_numpy(np.concatenate(texts)).to("cuda:0")
    del texts
    ctx = bt.Context(0)
    try:
        trees = ctx.build_batch(d, offs, sigma=4, tau=4, leaf_len=16)
        got, bad = [], []
        for i, tr in enumerate(trees):
            h = _sha(tr.serialize())
            got.append(h)
            if h[:16] != want[i][1]:
                bad.append(i)
            tr.free()
        assert not bad, "%d trees differ from the oracle's, first %s" % (len(bad), bad[:10])
        assert _sha("".join(got).encode()) == e["tree_digest"]
    finally:
        ctx.close()
