"""Reference values of the probe scan's 32-bit pre-filter hashes (test
infrastructure, not the oracle: the hashes are a filter of the GPU path, not
part of the method).  H[0] = 0, H[i+1] = H[i] * x + T[i] (mod 2^32)."""
import numpy as np


def h32_loop(T, x):
    """The recurrence itself, one step per byte (small inputs)."""
    H = [0]
    for b in bytes(T):
        H.append((H[-1] * x + b) & 0xFFFFFFFF)
    return np.array(H, dtype=np.uint32)


def h32(T, x):
    """Vectorised for odd x: with y = x^-1 mod 2^32,
    H[i] = x^(i-1) * sum_{j<i} T[j] y^j (numpy uint32 arithmetic wraps mod 2^32)."""
    assert x & 1, "the closed form needs an odd base"
    T = np.asarray(T, dtype=np.uint8)
    n = len(T)
    H = np.zeros(n + 1, np.uint32)
    if n == 0:
        return H
    y = pow(int(x), -1, 1 << 32)

    def powers(b):
        p = np.empty(n, np.uint32)
        p[0] = 1
        if n > 1:
            p[1:] = np.cumprod(np.full(n - 1, b, np.uint32), dtype=np.uint32)
        return p

    with np.errstate(over="ignore"):
        S = np.cumsum(T.astype(np.uint32) * powers(y), dtype=np.uint32)
        H[1:] = powers(x) * S
    return H
