"""Helpers for GPU tests: device setup and conversion of library trees into the
structures the oracle and the structural checker use."""
import numpy as np
import pytest

from tests import treecheck


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_device(T):
    torch = torch_cuda()
    a = np.ascontiguousarray(np.frombuffer(bytes(T), np.uint8) if isinstance(T, (bytes, bytearray)) else T,
                             dtype=np.uint8)
    return torch.from_numpy(a.copy()).to("cuda:0")


def shape_of(tree, tau, leaf_len):
    """treecheck.Shape of a library tree."""
    lv = []
    for l in range(1, tree.height):
        b, marked, pb, po = tree.level(l)
        lv.append((b, marked, pb, po))
    b, c, _ = tree.level_info(tree.height)
    lv.append((b, np.zeros(c, np.uint8), np.zeros(0, np.uint64), np.zeros(0, np.uint64)))
    return treecheck.Shape(tree.n, tau, leaf_len, tree.b1, lv, tree.leaves().tobytes())


def assert_same_tree(gpu_tree, ora_tree):
    """Level by level, then the canonical bytes."""
    assert gpu_tree.n == ora_tree.n
    assert gpu_tree.b1 == ora_tree.b1, (gpu_tree.b1, ora_tree.b1)
    assert gpu_tree.height == ora_tree.h, (gpu_tree.height, ora_tree.h)
    for l in range(1, ora_tree.h):
        L = ora_tree.levels[l - 1]
        b, marked, pb, po = gpu_tree.level(l)
        assert b == L.b
        assert marked.size == L.c, "level %d: %d blocks vs %d" % (l, marked.size, L.c)
        bad = np.flatnonzero(marked != L.marked)
        assert bad.size == 0, "level %d: marks differ at blocks %s" % (l, bad[:10].tolist())
        assert pb.size == L.u
        assert np.array_equal(pb, L.ptr_block), "level %d: pointer blocks differ" % l
        assert np.array_equal(po, L.ptr_off), "level %d: pointer offsets differ" % l
    b, c, _ = gpu_tree.level_info(ora_tree.h)
    assert c == ora_tree.levels[-1].c
    assert gpu_tree.leaves().tobytes() == ora_tree.leaves.tobytes()
    assert gpu_tree.serialize() == ora_tree.canonical
