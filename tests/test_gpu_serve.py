"""Serving: requests arriving while others build are admitted as slots and
memory free up, their builds overlap, and every tree and query answer is
identical to the same request served alone (exact; the output is integers)."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import to_device, torch_cuda

pytestmark = pytest.mark.gpu


def _requests(seed, count):
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.exp(rng.normal(np.log(20000), 1.5, count)), 1, 400000).astype(int)
    return [synth.dna_copies(int(n), max(1, int(n) // 16), 16, 1e-3, 1e-4, 8, int(rng.integers(1 << 30)))
            for n in sizes]


def test_mixed_equals_alone():
    torch = torch_cuda()
    import paper_2512_23314_amd as bt
    from paper_2512_23314_amd.serve import Server
    texts = _requests(1, 40)
    srv = Server(budget=2 << 30, slots=2, max_batch=8, tau=4, leaf_len=16, sigma=4)
    futs = []
    qfuts = []
    rng = np.random.default_rng(2)
    for k, T in enumerate(texts):
        futs.append(srv.submit_build(T))
        time.sleep(float(rng.exponential(0.002)))
        # query earlier finished trees while later ones build
        if k >= 5 and futs[k - 5].done():
            rid = futs[k - 5].result()
            Tq = texts[k - 5]
            pos = torch.arange(len(Tq), device="cuda:0", dtype=torch.int64).to(torch.uint64)
            qfuts.append((Tq, srv.submit_queries(rid, "access", pos)))
    rids = [f.result(timeout=120) for f in futs]
    for Tq, qf in qfuts:
        assert np.array_equal(qf.result(timeout=60).cpu().numpy(), Tq)
    st = srv.stats()
    alone = bt.Context(0)
    for T, rid in zip(texts, rids):
        mixed = srv.tree(rid).serialize()
        solo = alone.build(to_device(T) if len(T) else torch.zeros(0, dtype=torch.uint8, device="cuda:0"),
                           sigma=4, tau=4, leaf_len=16, rank_select=True).serialize()
        assert mixed == solo
        if len(T) <= 50000:
            assert mixed == oracle.build_tree(T, 4, 16).canonical
    # rank/select in the mix equal counted prefixes
    T = texts[3]
    if len(T):
        cs = to_device(np.frombuffer(b"ACGT" * 50, np.uint8))
        ks = torch.arange(1, 201, device="cuda:0", dtype=torch.int64).to(torch.uint64)
        got = srv.submit_queries(rids[3], "select", cs, ks).result(timeout=60).cpu().numpy()
        want = oracle.select(T, np.frombuffer(b"ACGT" * 50, np.uint8), np.arange(1, 201, dtype=np.uint64))
        assert np.array_equal(got, want)
    srv.close()
    alone.close()
    assert st["builds"] == len(texts)
    assert st["batches"] < len(texts), "requests were never batched"


def test_admission_respects_budget():
    torch_cuda()
    from paper_2512_23314_amd.serve import Server, build_footprint
    texts = _requests(3, 12)
    big = max(len(T) + build_footprint(len(T), 4, 16, 4, True) for T in texts)
    srv = Server(budget=big + (1 << 20), slots=3, max_batch=4, tau=4, leaf_len=16, sigma=4)
    futs = [srv.submit_build(T) for T in texts]
    rids = [f.result(timeout=120) for f in futs]
    st = srv.stats()
    # a tree with a queued query is released only after the query ran
    import torch
    pos = torch.zeros(4, dtype=torch.int64, device="cuda:0").to(torch.uint64)
    qf = [srv.submit_queries(rid, "access", pos) for rid in rids if srv.tree(rid).n]
    # resident trees stay charged; release them and check the accounting empties
    for rid in rids:
        srv.release(rid)
    for f in qf:
        f.result(timeout=60)
    assert srv.used == 0
    srv.close()
    assert st["max_admitted_bytes"] <= srv.budget


def test_device_bytes_within_budget():
    """The device bytes the server really holds stay within its budget.  Every
    context takes its memory from torch's caching allocator, so torch's exact
    peak of allocated bytes over the run (the texts, uploaded by the client
    beforehand, excluded) bounds the library's bytes, its pools' cached blocks
    and the batches' text copies.  The budget is tight: a few requests at a
    time, so slots wait, and trim their pools when the cached blocks would not
    fit."""
    torch = torch_cuda()
    from paper_2512_23314_amd.serve import Server, build_footprint
    texts = _requests(5, 40)
    dev = [torch.from_numpy(T).to("cuda:0") for T in texts]
    torch.cuda.synchronize()
    biggest = max(len(T) + build_footprint(len(T), 4, 16, 4, True) for T in texts)
    budget = 3 * biggest
    base = torch.cuda.memory_allocated(0)
    torch.cuda.reset_peak_memory_stats(0)
    srv = Server(budget=budget, slots=3, max_batch=6, tau=4, leaf_len=16, sigma=4)
    rids = [f.result(timeout=120) for f in [srv.submit_build(d) for d in dev]]
    held = srv.used
    peak = torch.cuda.max_memory_allocated(0) - base
    st = srv.stats()
    for T, rid in zip(texts, rids):
        assert srv.tree(rid).n == len(T)
    for rid in rids:
        srv.release(rid)
    srv.close()
    assert peak <= budget, "device bytes %d over the budget %d" % (peak, budget)
    assert st["max_admitted_bytes"] <= budget
    assert 0 < held <= budget
    assert st["measured"]
