"""The closed form of tests/hashref.py against the recurrence it stands for."""
import numpy as np
import pytest

from tests import hashref


@pytest.mark.parametrize("n", [0, 1, 2, 17, 300, 5000])
def test_h32_closed_form_matches_recurrence(n):
    rng = np.random.default_rng(n)
    T = rng.integers(0, 256, n).astype(np.uint8)
    for x in (1, 3, 0x9E3779B1, 0xFFFFFFFF, int(rng.integers(0, 1 << 31)) * 2 + 1):
        assert np.array_equal(hashref.h32(T, x), hashref.h32_loop(T, x))


def test_h32_known_values():
    # "ab" with x = 257: H = [0, 97, 97 * 257 + 98]
    assert hashref.h32(np.frombuffer(b"ab", np.uint8), 257).tolist() == [0, 97, 97 * 257 + 98]
    assert hashref.h32_loop(b"\xff" * 3, 0xFFFFFFFF).tolist() == [0, 255, 0, 255]
