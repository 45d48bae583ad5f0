"""Block-tree oracle: plain CPU construction from the definition, for tests.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It shares no code with
the GPU library and never imports it.

``liboracle.so`` is built from ``bt_oracle.c`` (the plain definition, with
leftmost occurrences by direct search) and ``bt_par.c`` (the paper's own
two-phase method on host threads, for full-size texts) by :func:`build` (gcc).
The pure-Python brute force in :mod:`oracle.brute` is a third, independent
formulation used to pin the C code on tiny inputs.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("bt_oracle.c", "bt_par.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

P61 = (1 << 61) - 1


def build():
    """Compile the oracle with gcc (-O2, no vectorisation tricks needed)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", _LIB + ".tmp"] + _SRCS
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        vp, pu64, pu32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)
        L.ora_plan.argtypes = [u64, u32, u32, u64, u64, pu64, pu32]
        L.ora_plan.restype = i32
        L.ora_build.argtypes = [vp, u64, u32, u32, u64, i32, i32, ctypes.POINTER(i32)]
        L.ora_build.restype = vp
        L.ora_prune.argtypes = [vp, vp]
        L.ora_prune.restype = i32
        L.ora_free.argtypes = [vp]
        L.ora_tree_info.argtypes = [vp, pu64, pu32, pu64, pu64]
        L.ora_level_info.argtypes = [vp, u32, pu64, pu64, pu64]
        L.ora_level_info.restype = i32
        L.ora_level_copy.argtypes = [vp, u32, vp, vp, vp, vp, vp]
        L.ora_leaves.argtypes = [vp, vp]
        L.ora_serialize.argtypes = [vp, vp, u64, pu64]
        L.ora_serialize.restype = i32
        L.ora_prefix_fp.argtypes = [vp, u64, u64, vp]
        L.ora_prefix_fp.restype = i32
        L.ora_window_fp.argtypes = [vp, u64, u64, u64]
        L.ora_window_fp.restype = u64
        L.ora_build_par.argtypes = [vp, u64, u32, u32, u64, i32, u64, u32, vp, ctypes.POINTER(i32)]
        L.ora_build_par.restype = vp
        L.ora_par_window_fp.argtypes = [vp, u64, u64, u64]
        L.ora_par_window_fp.restype = u64
        L.ora_access.argtypes = [vp, u64, vp, u64, vp]
        L.ora_access.restype = i32
        L.ora_rank.argtypes = [vp, u64, vp, vp, u64, vp]
        L.ora_rank.restype = i32
        L.ora_select.argtypes = [vp, u64, vp, vp, u64, vp]
        L.ora_select.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _text(T):
    if isinstance(T, (bytes, bytearray)):
        T = np.frombuffer(bytes(T), dtype=np.uint8)
    return np.ascontiguousarray(T, dtype=np.uint8)


def plan(n, tau, leaf_len, s_hint=1, root_block_len=0):
    """(b1, h) for a text of length n (level plan; see include/bt.h)."""
    b1, h = ctypes.c_uint64(), ctypes.c_uint32()
    rc = lib().ora_plan(n, tau, leaf_len, s_hint, root_block_len, ctypes.byref(b1), ctypes.byref(h))
    if rc != 0:
        raise ValueError("invalid plan parameters")
    return b1.value, h.value


class Level:
    def __init__(self, b, c, u, marked, start, length, ptr_block, ptr_off):
        self.b, self.c, self.u = b, c, u
        self.marked, self.start, self.length = marked, start, length
        self.ptr_block, self.ptr_off = ptr_block, ptr_off


class Tree:
    """A built oracle tree, copied out into numpy arrays."""

    def __init__(self, n, tau, leaf_len, b1, levels, leaves, canonical):
        self.n, self.tau, self.leaf_len, self.b1 = n, tau, leaf_len, b1
        self.levels = levels
        self.h = len(levels)
        self.leaves = leaves
        self.canonical = canonical


SEARCH_MEMMEM, SEARCH_NAIVE, SEARCH_RUNS = 0, 1, 2


def _collect(L, h, n, tau, leaf_len, levels=True):
    """Copy a built oracle tree out of the C library (and free nothing)."""
    nn, hh, bb1, lb = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    L.ora_tree_info(h, ctypes.byref(nn), ctypes.byref(hh), ctypes.byref(bb1), ctypes.byref(lb))
    out = []
    for lv in range(1, hh.value + 1):
        b, c, u = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        L.ora_level_info(h, lv, ctypes.byref(b), ctypes.byref(c), ctypes.byref(u))
        if not levels:
            out.append(Level(b.value, c.value, u.value, None, None, None, None, None))
            continue
        c_, u_ = c.value, u.value
        marked = np.zeros(c_, np.uint8)
        st = np.zeros(c_, np.uint64)
        ln = np.zeros(c_, np.uint64)
        pb = np.zeros(u_, np.uint64)
        po = np.zeros(u_, np.uint64)
        L.ora_level_copy(h, lv, _ptr(marked), _ptr(st), _ptr(ln), _ptr(pb), _ptr(po))
        out.append(Level(b.value, c_, u_, marked, st, ln, pb, po))
    leaves = np.zeros(lb.value, np.uint8)
    L.ora_leaves(h, _ptr(leaves))
    w = ctypes.c_uint64()
    L.ora_serialize(h, None, 0, ctypes.byref(w))
    buf = np.zeros(w.value, np.uint8)
    L.ora_serialize(h, _ptr(buf), w.value, ctypes.byref(w))
    return Tree(n, tau, leaf_len, bb1.value, out, leaves, buf.tobytes())


def build_tree(T, tau, leaf_len, b1=None, s_hint=1, exact_split=True, search=SEARCH_MEMMEM,
               prune=False):
    """Build the block tree of T by the definition.  Raises on a lemma breach.
    prune: also run the optional pruning phase (Section 4.1) on the result."""
    T = _text(T)
    n = T.size
    if b1 is None:
        b1, _ = plan(n, tau, leaf_len, s_hint)
    L = lib()
    err = ctypes.c_int()
    h = L.ora_build(_ptr(T), n, tau, leaf_len, b1, int(exact_split), search, ctypes.byref(err))
    if not h:
        raise ValueError("oracle build failed: %d" % err.value)
    try:
        if err.value != 0:
            raise AssertionError("oracle: a pointer target is not a marked block or pair (%d)" % err.value)
        if prune:
            rc = L.ora_prune(h, _ptr(T))
            if rc != 0:
                raise AssertionError("oracle: pruning failed (%d)" % rc)
        return _collect(L, h, n, tau, leaf_len)
    finally:
        L.ora_free(h)


# Karp-Rabin base of the threaded construction (any value in [2, q) gives the
# same tree; tests vary it).
PAR_BASE = 0x3C6EF372FE94F82B


def default_threads():
    """Host threads for the threaded construction: the CPUs this process may use."""
    try:
        return max(1, min(256, len(os.sched_getaffinity(0))))
    except (AttributeError, OSError):
        return max(1, min(256, os.cpu_count() or 1))


def build_tree_par(T, tau, leaf_len, b1=None, s_hint=1, threads=None, base=PAR_BASE, fp_bits=64,
                   levels=True, prune=False, stats=None):
    """Build the block tree of T with the paper's two-phase method on host
    threads (``bt_par.c``): Karp-Rabin fingerprints mod 2^64-2^32+1 with base
    ``base``, every accepted occurrence confirmed by comparing bytes, the level's
    windows split into ``threads`` partitions.  ``fp_bits`` < 64 keeps only the
    low bits of every fingerprint, which forces collisions.  Exact splits only
    (b1 = leaf_len * tau^k).  levels=False skips copying the per-level arrays
    (the canonical bytes are always produced).  stats: None, or a list that
    receives one (phase-1 keys, phase-1 ms, phase-2 keys, phase-2 ms) tuple per
    level."""
    T = _text(T)
    n = T.size
    if b1 is None:
        b1, _ = plan(n, tau, leaf_len, s_hint)
    if threads is None:
        threads = default_threads()
    L = lib()
    err = ctypes.c_int()
    st = np.zeros(4 * 70, np.float64)
    h = L.ora_build_par(_ptr(T), n, tau, leaf_len, b1, int(threads), int(base), int(fp_bits),
                        _ptr(st), ctypes.byref(err))
    if not h:
        raise ValueError("threaded oracle build failed: %d" % err.value)
    try:
        if err.value != 0:
            raise AssertionError("threaded oracle: a key or pointer breaks the level lemma (%d)"
                                 % err.value)
        if prune:
            rc = L.ora_prune(h, _ptr(T))
            if rc != 0:
                raise AssertionError("oracle: pruning failed (%d)" % rc)
        tree = _collect(L, h, n, tau, leaf_len, levels)
        if stats is not None:
            stats.extend(tuple(st[4 * i:4 * i + 4]) for i in range(tree.h - 1))
        return tree
    finally:
        L.ora_free(h)


def par_window_fp(T, s, L, base=PAR_BASE):
    """phi of T[s..s+L) mod 2^64-2^32+1 with the threaded construction's arithmetic."""
    T = _text(T)
    return int(lib().ora_par_window_fp(_ptr(T), s, L, base))


def prefix_fp(T, x):
    """P[0..n] with P[i+1] = (P[i]*x + T[i]) mod 2^61-1."""
    T = _text(T)
    P = np.zeros(T.size + 1, np.uint64)
    if lib().ora_prefix_fp(_ptr(T), T.size, x, _ptr(P)) != 0:
        raise ValueError("base must be below 2^61-1")
    return P


def window_fp(T, s, L, x):
    T = _text(T)
    return int(lib().ora_window_fp(_ptr(T), s, L, x))


def access(T, pos):
    T = _text(T)
    pos = np.ascontiguousarray(pos, np.uint64)
    out = np.zeros(pos.size, np.uint8)
    lib().ora_access(_ptr(T), T.size, _ptr(pos), pos.size, _ptr(out))
    return out


def rank(T, cs, pos):
    T = _text(T)
    cs = np.ascontiguousarray(cs, np.uint8)
    pos = np.ascontiguousarray(pos, np.uint64)
    out = np.zeros(pos.size, np.uint64)
    lib().ora_rank(_ptr(T), T.size, _ptr(cs), _ptr(pos), pos.size, _ptr(out))
    return out


def select(T, cs, ks):
    T = _text(T)
    cs = np.ascontiguousarray(cs, np.uint8)
    ks = np.ascontiguousarray(ks, np.uint64)
    out = np.zeros(ks.size, np.uint64)
    lib().ora_select(_ptr(T), T.size, _ptr(cs), _ptr(ks), ks.size, _ptr(out))
    return out


def leftmost(T, st, L):
    """Leftmost occurrence of T[st..st+L) in T (direct search via bytes.find)."""
    Tb = T if isinstance(T, (bytes, bytearray)) else _text(T).tobytes()
    return Tb.find(Tb[st:st + L], 0, st + L)
