"""Python binding of libbt (include/bt.h): block-tree construction and queries on
an MI355X GPU.

This module only marshals arguments: every step of construction and every query
runs in the HIP kernels of ``libbt.so``.  PyTorch supplies device memory (CUDA
tensors on ROCm) and the current stream.  If ``libbt.so`` is missing, importing
the binding raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbt.so")

BT_OK, BT_E_INVAL, BT_E_NOMEM, BT_E_DEVICE, BT_E_INTERNAL = 0, -1, -2, -3, -4
BT_DBG_WEAK_HASH = 1
BT_DBG_NO_QUEUE = 2
BT_DBG_NO_BYTE_SCAN = 4
BT_DBG_SORT_PHASES = 8
BT_DBG_SHARED_FILTERS = 16
BT_WITH_RANK_SELECT = 1
BT_PRUNE = 2
BT_LEAN = 4

_lib = None


class BtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "error"), code, msg))
        self.code = code


_ERRNAMES = {BT_E_INVAL: "BT_E_INVAL", BT_E_NOMEM: "BT_E_NOMEM", BT_E_DEVICE: "BT_E_DEVICE",
             BT_E_INTERNAL: "BT_E_INTERNAL"}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class bt_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class Allocator:
    """A bt_allocator made of two Python callables: alloc(nbytes) -> device
    address (int) or None, free(address).  The callbacks stay referenced for the
    life of the process (the library may call them until the last tree of a
    context is freed)."""

    _keep = []

    def __init__(self, alloc, free):
        def _a(user, nbytes, stream):
            try:
                return alloc(int(nbytes))
            except Exception:  # reported by the library as BT_E_NOMEM
                return None

        def _f(user, ptr, stream):
            try:
                free(int(ptr))
            except Exception:
                pass

        self.c = bt_allocator(ALLOC_FN(_a), FREE_FN(_f), None)
        Allocator._keep.append(self)


_torch_allocators = {}


def torch_allocator(device, stream):
    """Device memory from PyTorch's caching allocator on `stream` (a
    torch.cuda.Stream): the library's blocks count in torch's statistics and go
    back to torch's cache when the context trims or is destroyed.  One per
    (device, stream)."""
    torch = _torch()
    key = (device, stream.cuda_stream)
    if key not in _torch_allocators:
        _torch_allocators[key] = Allocator(
            lambda n: torch.cuda.caching_allocator_alloc(n, device, stream),
            torch.cuda.caching_allocator_delete)
    return _torch_allocators[key]


class bt_tuning(ctypes.Structure):
    _fields_ = [("table_load_log2", ctypes.c_uint32), ("text_filter_bits_log2", ctypes.c_uint32),
                ("span_chunks", ctypes.c_uint32), ("filter2_max_log2", ctypes.c_uint32)]


DEFAULT_TUNING = {"table_load_log2": 1, "text_filter_bits_log2": 5, "span_chunks": 0,
                  "filter2_max_log2": 24}


class bt_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_uint32), ("leaf_len", ctypes.c_uint32),
                ("root_block_len", ctypes.c_uint64), ("s_hint", ctypes.c_uint64),
                ("hash_seed", ctypes.c_uint64), ("debug_flags", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


# name -> (restype, argtypes); the exported surface of include/bt.h
_vp, _u64, _u32, _i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
_pu64, _pu32, _pd = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "bt_ctx_create": (_i32, [_i32, _vp, ctypes.POINTER(_vp)]),
    "bt_ctx_create_ex": (_i32, [_i32, _vp, ctypes.POINTER(bt_allocator), ctypes.POINTER(_vp)]),
    "bt_ctx_destroy": (None, [_vp]),
    "bt_ctx_last_error": (ctypes.c_char_p, [_vp]),
    "bt_ctx_trim": (_i32, [_vp]),
    "bt_ctx_profile": (_i32, [_vp, _i32]),
    "bt_ctx_kernel_stats": (_i32, [_vp, ctypes.c_char_p, _pu64, _pd, _pd, _pd]),
    "bt_ctx_reset_stats": (_i32, [_vp]),
    "bt_ctx_launch_count": (_i32, [_vp, _pu64]),
    "bt_ctx_phase_count": (_i32, [_vp, _pu64]),
    "bt_ctx_set_tuning": (_i32, [_vp, ctypes.POINTER(bt_tuning)]),
    "bt_ctx_get_tuning": (_i32, [_vp, ctypes.POINTER(bt_tuning)]),
    "bt_ctx_phase_record": (_i32, [_vp, _u64, _vp]),
    "bt_ctx_launch_record": (_i32, [_vp, _u64, ctypes.c_char_p, _u64, _pu64, _pd, _pd, _pd]),
    "bt_ctx_memory": (_i32, [_vp, _pu64, _pu64, _pu64]),
    "bt_ctx_reset_peak": (_i32, [_vp]),
    "bt_prefix_fingerprints": (_i32, [_vp, _vp, _u64, _u64, _vp]),
    "bt_prefix_scan": (_i32, [_vp, _vp, _u64, _u64, _u32, _i32, _vp, _vp]),
    "bt_prefix_scan_noalloc": (_i32, [_vp, _vp, _u64, _u64, _u32, _i32, _vp, _vp]),
    "bt_build": (_i32, [_vp, _vp, _u64, _u32, _u32, _u32, ctypes.POINTER(_vp)]),
    "bt_build_ex": (_i32, [_vp, _vp, _u64, _u32, ctypes.POINTER(bt_params), ctypes.POINTER(_vp)]),
    "bt_build_batch": (_i32, [_vp, _vp, _vp, _u32, _u32, ctypes.POINTER(bt_params), _vp]),
    "bt_tree_info": (_i32, [_vp, _pu64, _pu32, _pu64]),
    "bt_level_info": (_i32, [_vp, _u32, _pu64, _pu64, _pu64]),
    "bt_level_copy": (_i32, [_vp, _u32, _vp, _vp, _vp]),
    "bt_level_copy_async": (_i32, [_vp, _u32, _vp, _vp, _vp, _vp]),
    "bt_leaves_size": (_i32, [_vp, _pu64]),
    "bt_leaves_copy": (_i32, [_vp, _vp]),
    "bt_serialize": (_i32, [_vp, _vp, _u64, _pu64]),
    "bt_access": (_i32, [_vp, _vp, _vp, _u64, _vp]),
    "bt_rank": (_i32, [_vp, _vp, _vp, _vp, _u64, _vp]),
    "bt_select": (_i32, [_vp, _vp, _vp, _vp, _u64, _vp]),
    "bt_tree_device_bytes": (_i32, [_vp, _pu64]),
    "bt_tree_rank_bytes": (_i32, [_vp, _pu64]),
    "bt_trees_free": (_i32, [_vp, _u64]),
    "bt_tree_free": (None, [_vp]),
    "bt_strerror": (ctypes.c_char_p, [_i32]),
}


def lib():
    """Load libbt.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbt.so not built: run __graft_entry__.build() or "
                              "python paper_2512_23314_amd/_build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A bt_ctx bound to one device and the torch current stream at creation.
    allocator: "torch" (default: PyTorch's caching allocator supplies the
    library's device memory), None (the library's own hipMalloc), or an
    Allocator."""

    def __init__(self, device=0, stream=None, allocator="torch"):
        torch = _torch()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        if allocator == "torch":
            allocator = torch_allocator(device, stream)
        self.allocator = allocator
        h = ctypes.c_void_p()
        if allocator is None:
            rc = lib().bt_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        else:
            rc = lib().bt_ctx_create_ex(device, ctypes.c_void_p(stream.cuda_stream),
                                        ctypes.byref(allocator.c), ctypes.byref(h))
        if rc != 0:
            raise BtError(rc, "bt_ctx_create failed")
        self.h = h
        self._tcache = None    # tuning cache (autotune.py), loaded on the first build
        self._applied = None   # the cached tuning last applied

    def close(self):
        if self.h:
            lib().bt_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise BtError(rc, lib().bt_ctx_last_error(self.h).decode())

    # ---- profiling
    def profile(self, on=True):
        self._check(lib().bt_ctx_profile(self.h, 1 if on else 0))

    def reset_stats(self):
        self._check(lib().bt_ctx_reset_stats(self.h))

    def kernel_stats(self, name):
        n = ctypes.c_uint64()
        ms, by, un = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().bt_ctx_kernel_stats(self.h, name.encode(), ctypes.byref(n),
                                              ctypes.byref(ms), ctypes.byref(by), ctypes.byref(un)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value, "units": un.value}

    def launches(self):
        """Per-launch records since reset_stats(): (name, window length, units,
        ms, algorithmic bytes), in launch order."""
        n = ctypes.c_uint64()
        self._check(lib().bt_ctx_launch_count(self.h, ctypes.byref(n)))
        out = []
        name = ctypes.create_string_buffer(64)
        wl = ctypes.c_uint64()
        un, ms, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        for k in range(n.value):
            self._check(lib().bt_ctx_launch_record(self.h, k, name, 64, ctypes.byref(wl), ctypes.byref(un),
                                                   ctypes.byref(ms), ctypes.byref(by)))
            out.append((name.value.decode(), wl.value, un.value, ms.value, by.value))
        return out

    def set_tuning(self, **kw):
        """Set launch and sizing choices (bt_ctx_set_tuning); unnamed ones keep
        their current values.  Returns the previous tuning as a dict."""
        cur = bt_tuning()
        self._check(lib().bt_ctx_get_tuning(self.h, ctypes.byref(cur)))
        prev = {k: getattr(cur, k) for k, _ in bt_tuning._fields_}
        new = bt_tuning(**dict(prev, **kw))
        self._check(lib().bt_ctx_set_tuning(self.h, ctypes.byref(new)))
        return prev

    def tuning(self):
        cur = bt_tuning()
        self._check(lib().bt_ctx_get_tuning(self.h, ctypes.byref(cur)))
        return {k: getattr(cur, k) for k, _ in bt_tuning._fields_}

    PHASE_FIELDS = ("step", "b", "phase", "blocks", "keys", "windows", "candidates", "verified",
                    "collisions")

    def phases(self):
        """Per-phase device counters of the profiled builds since reset_stats(),
        as dicts with the fields PHASE_FIELDS (see bt_ctx_phase_record)."""
        n = ctypes.c_uint64()
        self._check(lib().bt_ctx_phase_count(self.h, ctypes.byref(n)))
        out = []
        rec = np.zeros(9, np.uint64)
        for k in range(n.value):
            self._check(lib().bt_ctx_phase_record(self.h, k, rec.ctypes.data_as(ctypes.c_void_p)))
            out.append(dict(zip(self.PHASE_FIELDS, (int(v) for v in rec))))
        return out

    def trim(self):
        self._check(lib().bt_ctx_trim(self.h))

    def memory(self):
        """Pool bytes: in use, peak since reset_peak(), held (cached included)."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._check(lib().bt_ctx_memory(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"in_use": a.value, "peak": b.value, "held": c.value}

    def reset_peak(self):
        self._check(lib().bt_ctx_reset_peak(self.h))

    # ---- step a2
    def prefix_fingerprints(self, text, x, out=None):
        torch = _torch()
        n = text.numel()
        if out is None:
            out = torch.empty(n + 1, dtype=torch.uint64, device=text.device)
        self._check(lib().bt_prefix_fingerprints(self.h, _ptr(text), n, x, _ptr(out)))
        return out

    def prefix_scan(self, text, x, x32, sampled=False):
        """Fingerprints (dense, or P[16 q] when sampled) and 32-bit hashes of one
        pass; returns (P, H): uint64, and int32 holding the uint32 values.
        sampled=2 samples H too (H[16 q], the memory-lean build's form)."""
        torch = _torch()
        n = text.numel()
        sampled = int(sampled)
        P = torch.empty(n // 16 + 1 if sampled else n + 1, dtype=torch.uint64, device=text.device)
        H = torch.empty(n // 16 + 1 if sampled == 2 else n + 1, dtype=torch.int32,
                        device=text.device)  # uint32 bits
        self._check(lib().bt_prefix_scan(self.h, _ptr(text), n, x, x32, sampled, _ptr(P), _ptr(H)))
        return P, H

    def prefix_scan_noalloc(self, text, x, x32, sampled=False, P=None, H=None):
        """prefix_scan through bt_prefix_scan_noalloc (the library allocates
        nothing; P and H may be given to reuse caller buffers)."""
        torch = _torch()
        n = text.numel()
        sampled = int(sampled)
        if P is None:
            P = torch.empty(n // 16 + 1 if sampled else n + 1, dtype=torch.uint64, device=text.device)
        if H is None:
            H = torch.empty(n // 16 + 1 if sampled == 2 else n + 1, dtype=torch.int32,
                            device=text.device)  # uint32 bits
        self._check(lib().bt_prefix_scan_noalloc(self.h, _ptr(text), n, x, x32, sampled,
                                                 _ptr(P), _ptr(H)))
        return P, H

    # ---- builds
    @staticmethod
    def params(tau, leaf_len, s_hint=1, root_block_len=0, hash_seed=0x0B10C7EE, debug_flags=0,
               rank_select=False, prune=False, lean=False):
        return bt_params(tau, leaf_len, root_block_len, s_hint, hash_seed, debug_flags,
                         (BT_WITH_RANK_SELECT if rank_select else 0) | (BT_PRUNE if prune else 0) |
                         (BT_LEAN if lean else 0))

    def _apply_tuning(self, ntexts, nbytes):
        """Apply the autotuner's settings for this shape class, if the cache has them."""
        from . import autotune
        if self._tcache is None:
            self._tcache = autotune.load_cache()
            self._arch = autotune.arch_name(self.device) if self._tcache else ""
        t = autotune.lookup(self._tcache, self._arch, autotune.shape_class(ntexts, nbytes))
        if t and t != self._applied:
            self.set_tuning(**t)
            self._applied = t

    def build(self, text, sigma=256, tau=2, leaf_len=16, tuned=True, **kw):
        """Build the tree of a uint8 CUDA tensor; returns a Tree.  tuned: apply
        the autotuner's settings for single texts of this size first (no tree
        depends on them)."""
        if tuned:
            self._apply_tuning(1, text.numel())
        p = self.params(tau, leaf_len, **kw)
        h = ctypes.c_void_p()
        self._check(lib().bt_build_ex(self.h, _ptr(text), text.numel(), sigma, ctypes.byref(p),
                                      ctypes.byref(h)))
        return Tree(self, h)

    def build_batch(self, concat, offsets, sigma=256, tau=2, leaf_len=16, tuned=True, **kw):
        """Build one tree per text concat[offsets[i]:offsets[i+1]] (tuned: as in build)."""
        p = self.params(tau, leaf_len, **kw)
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        num = offs.size - 1
        if tuned:
            self._apply_tuning(num, int(offs[-1] - offs[0]) if num > 0 else 0)
        outs = (ctypes.c_void_p * max(num, 1))()
        self._check(lib().bt_build_batch(self.h, _ptr(concat), offs.ctypes.data_as(ctypes.c_void_p),
                                         num, sigma, ctypes.byref(p), outs))
        return [Tree(self, ctypes.c_void_p(outs[i])) for i in range(num)]


def free_trees(trees):
    """Free many trees with one call (bt_trees_free).  A tree's n, height and b1
    stay readable only if they were read before."""
    hs = [t.h for t in trees if t.h]
    if hs:
        arr = (ctypes.c_void_p * len(hs))(*[h.value for h in hs])
        lib().bt_trees_free(arr, len(hs))
    for t in trees:
        t.h = None


class Tree:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.h = handle
        self._info = None

    def _tree_info(self):
        if self._info is None:
            if not self.h:
                raise BtError(BT_E_INVAL, "tree freed (by free_trees) before its size was read")
            n, hh, b1 = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64()
            self._check_rc(lib().bt_tree_info(self.h, ctypes.byref(n), ctypes.byref(hh), ctypes.byref(b1)))
            self._info = (n.value, hh.value, b1.value)
        return self._info

    @staticmethod
    def _check_rc(rc):
        if rc != 0:
            raise BtError(rc, "bt_tree_info")

    @property
    def n(self):
        return self._tree_info()[0]

    @property
    def height(self):
        return self._tree_info()[1]

    @property
    def b1(self):
        return self._tree_info()[2]

    def free(self):
        """Free the tree's device memory; its n, height and b1 stay readable."""
        if self.h:
            self._tree_info()
            lib().bt_tree_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def level_info(self, level):
        b, c, u = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().bt_level_info(self.h, level, ctypes.byref(b), ctypes.byref(c), ctypes.byref(u))
        if rc != 0:
            raise BtError(rc, "bad level")
        return b.value, c.value, u.value

    def level(self, level):
        """(b, marked uint8[c], ptr_block uint64[u], ptr_off uint64[u]) for level < h."""
        b, c, u = self.level_info(level)
        words = np.zeros((c + 63) // 64, np.uint64)
        pb = np.zeros(u, np.uint64)
        po = np.zeros(u, np.uint64)
        rc = lib().bt_level_copy(self.h, level, words.ctypes.data_as(ctypes.c_void_p),
                                 pb.ctypes.data_as(ctypes.c_void_p), po.ctypes.data_as(ctypes.c_void_p))
        if rc != 0:
            raise BtError(rc, "bt_level_copy")
        bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:c]
        return b, bits.astype(np.uint8), pb, po

    def leaves(self):
        nb = ctypes.c_uint64()
        lib().bt_leaves_size(self.h, ctypes.byref(nb))
        out = np.zeros(nb.value, np.uint8)
        rc = lib().bt_leaves_copy(self.h, out.ctypes.data_as(ctypes.c_void_p))
        if rc != 0:
            raise BtError(rc, "bt_leaves_copy")
        return out

    def serialize(self):
        w = ctypes.c_uint64()
        rc = lib().bt_serialize(self.h, None, 0, ctypes.byref(w))
        if rc != 0:
            raise BtError(rc, "bt_serialize")
        buf = np.zeros(w.value, np.uint8)
        rc = lib().bt_serialize(self.h, buf.ctypes.data_as(ctypes.c_void_p), w.value, ctypes.byref(w))
        if rc != 0:
            raise BtError(rc, "bt_serialize")
        return buf.tobytes()

    def device_bytes(self):
        b = ctypes.c_uint64()
        lib().bt_tree_device_bytes(self.h, ctypes.byref(b))
        return b.value

    def rank_bytes(self):
        """Device bytes of the rank/select support (0 when built without it)."""
        b = ctypes.c_uint64()
        lib().bt_tree_rank_bytes(self.h, ctypes.byref(b))
        return b.value

    # ---- queries (device tensors in, device tensors out)
    # ctx: the context whose stream runs the query (default: the building one)
    def access(self, pos, out=None, ctx=None):
        torch = _torch()
        ctx = ctx or self.ctx
        if out is None:
            out = torch.empty(pos.numel(), dtype=torch.uint8, device=pos.device)
        ctx._check(lib().bt_access(ctx.h, self.h, _ptr(pos), pos.numel(), _ptr(out)))
        return out

    def rank(self, cs, pos, out=None, ctx=None):
        torch = _torch()
        ctx = ctx or self.ctx
        if out is None:
            out = torch.empty(pos.numel(), dtype=torch.uint64, device=pos.device)
        ctx._check(lib().bt_rank(ctx.h, self.h, _ptr(cs), _ptr(pos), pos.numel(), _ptr(out)))
        return out

    def select(self, cs, ks, out=None, ctx=None):
        torch = _torch()
        ctx = ctx or self.ctx
        if out is None:
            out = torch.empty(ks.numel(), dtype=torch.uint64, device=ks.device)
        ctx._check(lib().bt_select(ctx.h, self.h, _ptr(cs), _ptr(ks), ks.numel(), _ptr(out)))
        return out
