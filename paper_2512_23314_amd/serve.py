"""Serving loop: continuous batching of block-tree builds plus batched queries
against resident trees, on one GPU.

Requests arrive at any time (``submit_build``, ``submit_queries``).  Builds are
admitted by device-memory footprint: a build slot (a worker thread with its own
library context on its own HIP stream) takes every queued build request that
fits the free memory budget, up to ``max_batch`` texts, and builds them with one
``bt_build_batch`` call.  Requests that arrive while slots are busy wait for the
next free slot; several slots build at once, so their kernels overlap on the
device.  Finished trees stay resident (their bytes stay charged to the budget)
until ``release``.  Query batches run on their own slot and stream.

Memory.  Every context takes its device memory from PyTorch's caching
allocator, so the library's bytes are torch's allocated bytes.  A request is
charged its text, its copy in the batch, a fixed 16 MiB (a build's filters and
smallest tables), and the library's measured peak per text byte beyond that
(the most that any finished batch needed: bt_ctx_memory's peak less 16 MiB,
over the batch's text bytes; before the first measurement, an upper bound
computed from the sizes of the build's arrays).  The budget covers the resident
trees, the charges of the builds in flight and the blocks the slots' pools keep
cached; a slot trims its pool after a batch when that sum would exceed the
budget, and a waiting slot trims its pool when its cached blocks keep the next
request out.

Every build is the library's exact construction, so a tree built in a mix is
byte-identical to the same text built alone (tests/test_gpu_serve.py).
"""
import collections
import threading
import time
from concurrent.futures import Future

import numpy as np

from . import Context, BtError


def build_footprint(n, tau=4, leaf_len=16, sigma=256, rank_select=False):
    """Upper bound on the device bytes a build of an n-byte text needs while it
    runs: the text (n), its prefix fingerprints (8(n+1)) and 32-bit prefix
    hashes (4(n+1)); about 320 bytes per
    block of the largest scanned level (block, run, key, table at load 1/2 or
    less, verification, pointer and split arrays; that level has at most
    n / (tau * leaf_len) + 2 blocks); the leaf bytes; with rank/select support,
    4 bytes per symbol for every block and pointer of every level (at most
    2n / leaf_len + 2 of each) and the sampled count table; 16 MiB for small
    buffers."""
    blocks = n // max(tau * leaf_len, 1) + 2
    foot = 13 * n + 12 + 320 * blocks + 2 * n + (16 << 20)
    if rank_select:
        foot += 8 * sigma * (2 * n // max(leaf_len, 1) + 2) + 16 * sigma * (n // 1024 + 2)
    return foot


_FIXED = 16 << 20  # per-request charge beyond the per-byte rate


class _BuildReq:
    __slots__ = ("rid", "text", "t_arrive", "future", "foot")

    def __init__(self, rid, text, foot):
        self.rid, self.text, self.foot = rid, text, foot
        self.t_arrive = time.perf_counter()
        self.future = Future()


class Server:
    """See the module docstring.  ``budget`` is the device memory (bytes) that
    admitted builds plus resident trees may use."""

    def __init__(self, budget=64 << 30, slots=2, max_batch=256, tau=4, leaf_len=16, sigma=256,
                 rank_select=True, device=0):
        import torch
        self.torch = torch
        self.budget = budget
        self.used = 0            # resident trees + charges of the builds in flight
        self.cached = {}         # slot -> pooled bytes its context keeps for reuse
        self.peak_per_byte = 0.0  # measured library peak beyond _FIXED, per text byte
        self.measured = False
        self.trims = 0
        self.params = dict(tau=tau, leaf_len=leaf_len, sigma=sigma, rank_select=rank_select)
        self.max_batch = max_batch
        self.device = device
        self.lock = threading.Condition()
        self.pending = collections.deque()
        self.trees = {}          # rid -> (tree, bytes)
        self.next_id = 0
        self.stop = False
        self.build_lat = []      # seconds, arrival -> resident
        self.query_lat = []
        self.built_bytes = 0
        self.batches = 0
        self.max_inflight = 0
        self.inflight = 0
        self.max_used = 0
        self.qqueue = collections.deque()
        self.pins = collections.Counter()   # queued or running queries per tree
        self.doomed = set()                 # released while pinned
        self.workers = [threading.Thread(target=self._build_worker, daemon=True) for _ in range(slots)]
        self.qworker = threading.Thread(target=self._query_worker, daemon=True)
        for w in self.workers:
            w.start()
        self.qworker.start()

    # ---- client side
    def footprint(self, n):
        """Device bytes a build of an n-byte text is charged: the text on the
        device and its copy in the batch, plus the library's peak (16 MiB and
        the measured rate per text byte, or the computed bound before any build
        finished)."""
        if self.measured:
            return 2 * n + int(self.peak_per_byte * n) + _FIXED
        return n + build_footprint(n, self.params["tau"], self.params["leaf_len"],
                                   self.params["sigma"], self.params["rank_select"])

    def submit_build(self, text):
        """text: uint8 numpy array (host) or uint8 CUDA tensor.  Returns a Future
        resolving to the request id once the tree is resident."""
        n = int(text.size if isinstance(text, np.ndarray) else text.numel())
        foot = self.footprint(n)
        if foot > self.budget:
            raise BtError(-1, "request of %d bytes exceeds the memory budget" % n)
        with self.lock:
            rid = self.next_id
            self.next_id += 1
            req = _BuildReq(rid, text, foot)
            self.pending.append(req)
            self.lock.notify_all()
        return req.future

    def submit_queries(self, rid, kind, a, b=None):
        """kind: 'access' (a = positions), 'rank' (a = symbols, b = positions) or
        'select' (a = symbols, b = ranks); device tensors.  Returns a Future of
        the result tensor."""
        fut = Future()
        with self.lock:
            if rid not in self.trees or rid in self.doomed:
                raise KeyError("no resident tree %d" % rid)
            self.pins[rid] += 1  # the tree stays resident until its queries ran
            self.qqueue.append((rid, kind, a, b, fut, time.perf_counter()))
            self.lock.notify_all()
        return fut

    def tree(self, rid):
        return self.trees[rid][0]

    def release(self, rid):
        """Free a resident tree (deferred until its queued queries have run)."""
        with self.lock:
            if self.pins[rid]:
                self.doomed.add(rid)
                return
            self._free(rid)

    def _free(self, rid):
        tree, nbytes = self.trees.pop(rid)
        tree.free()
        self.used -= nbytes
        self.doomed.discard(rid)
        self.lock.notify_all()

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify_all()
        for w in self.workers:
            w.join()
        self.qworker.join()
        with self.lock:
            for rid in list(self.trees):
                self.trees[rid][0].free()
            self.trees.clear()

    # ---- workers
    def _take_batch(self):
        """Under the lock: the queued requests (in arrival order) that fit the
        free budget, at most max_batch of them."""
        batch, need = [], 0
        cached = sum(self.cached.values())
        while self.pending and len(batch) < self.max_batch:
            r = self.pending[0]
            if self.used + cached + need + r.foot > self.budget:
                break
            batch.append(self.pending.popleft())
            need += r.foot
        return batch, need

    def _build_worker(self):
        torch = self.torch
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(self.device)
        ctx = Context(self.device, stream)
        slot = threading.get_ident()
        while True:
            trim = False
            with self.lock:
                while not self.stop and not (self.pending and self._fits_head()):
                    # the head request waits while this slot keeps cached blocks:
                    # give them back
                    if self.pending and self.cached.get(slot, 0):
                        trim = True
                        break
                    self.lock.wait(0.05)
                if trim:
                    batch = None
                elif self.stop and not self.pending:
                    break
                else:
                    batch, need = self._take_batch()
                    if not batch:
                        continue
                if batch:
                    self.used += need
                    self.max_used = max(self.max_used, self.used)
                    self.inflight += 1
                    self.max_inflight = max(self.max_inflight, self.inflight)
            if trim:
                ctx.trim()
                m = ctx.memory()
                with self.lock:
                    self.cached[slot] = m["held"] - m["in_use"]
                    self.trims += 1
                    self.lock.notify_all()
                continue
            try:
                with torch.cuda.stream(stream):
                    parts = [r.text if not isinstance(r.text, np.ndarray)
                             else torch.from_numpy(r.text).to(f"cuda:{self.device}", non_blocking=False)
                             for r in batch]
                    offs = [0]
                    for p in parts:
                        offs.append(offs[-1] + int(p.numel()))
                    concat = torch.cat([p.reshape(-1) for p in parts]) if parts else None
                    stream.synchronize()
                    base = ctx.memory()["in_use"]
                    ctx.reset_peak()
                    trees = ctx.build_batch(concat, offs, **self.params)
                    del concat, parts
                t_done = time.perf_counter()
                mem = ctx.memory()
                nbytes = offs[-1]
                with self.lock:
                    if nbytes:
                        over = max(0, mem["peak"] - base - _FIXED)
                        self.peak_per_byte = max(self.peak_per_byte, over / nbytes)
                        self.measured = True
                    self.batches += 1
                    for r, tr in zip(batch, trees):
                        nb = tr.device_bytes()
                        self.trees[r.rid] = (tr, nb)
                        self.used += nb
                        self.build_lat.append(t_done - r.t_arrive)
                        self.built_bytes += int(r.text.size if isinstance(r.text, np.ndarray) else r.text.numel())
                    self.used -= need
                    self.inflight -= 1
                    # this slot's cached blocks count against the budget: give
                    # them back when the sum would not fit
                    self.cached[slot] = mem["held"] - mem["in_use"]
                    trim = self.used + sum(self.cached.values()) > self.budget
                if trim:
                    ctx.trim()
                    m2 = ctx.memory()
                    with self.lock:
                        self.cached[slot] = m2["held"] - m2["in_use"]
                        self.trims += 1
                with self.lock:
                    self.lock.notify_all()
                for r in batch:
                    r.future.set_result(r.rid)
            except Exception as e:  # report to every request of the batch
                with self.lock:
                    self.used -= need
                    self.inflight -= 1
                    self.lock.notify_all()
                for r in batch:
                    r.future.set_exception(e)
        ctx.close()

    def _fits_head(self):
        return self.used + sum(self.cached.values()) + self.pending[0].foot <= self.budget

    def _query_worker(self):
        torch = self.torch
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(self.device)
        ctx = Context(self.device, stream)
        while True:
            with self.lock:
                while not self.stop and not self.qqueue:
                    self.lock.wait(0.05)
                if self.stop and not self.qqueue:
                    break
                rid, kind, a, b, fut, t0 = self.qqueue.popleft()
                tree = self.trees.get(rid, (None, 0))[0]
            out, err = None, None
            try:
                if tree is None:
                    raise KeyError("no resident tree %d" % rid)
                with torch.cuda.stream(stream):
                    if kind == "access":
                        out = tree.access(a, ctx=ctx)
                    elif kind == "rank":
                        out = tree.rank(a, b, ctx=ctx)
                    else:
                        out = tree.select(a, b, ctx=ctx)
            except Exception as e:
                err = e
            with self.lock:
                if err is None:
                    self.query_lat.append(time.perf_counter() - t0)
                self.pins[rid] -= 1
                if self.pins[rid] <= 0:
                    del self.pins[rid]
                    if rid in self.doomed:
                        self._free(rid)
            if err is None:
                fut.set_result(out)
            else:
                fut.set_exception(err)
        ctx.close()

    def stats(self):
        def pct(v, q):
            return float(np.percentile(v, q)) if v else None
        return {"builds": len(self.build_lat), "batches": self.batches,
                "build_p50_ms": pct(self.build_lat, 50) and pct(self.build_lat, 50) * 1e3,
                "build_p99_ms": pct(self.build_lat, 99) and pct(self.build_lat, 99) * 1e3,
                "query_batches": len(self.query_lat),
                "query_p50_ms": pct(self.query_lat, 50) and pct(self.query_lat, 50) * 1e3,
                "query_p99_ms": pct(self.query_lat, 99) and pct(self.query_lat, 99) * 1e3,
                "built_bytes": self.built_bytes, "max_concurrent_builds": self.max_inflight,
                "max_admitted_bytes": self.max_used, "peak_per_byte": self.peak_per_byte,
                "measured": self.measured,
                "trims": self.trims}
