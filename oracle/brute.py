"""Brute-force block tree in pure Python, for tiny texts only.

TEST INFRASTRUCTURE ONLY.  A second formulation of the block-tree definition
(Section 4) that finds leftmost occurrences through a dictionary of every
substring's first position, built by walking the text left to right, instead
of by string search.  It pins the C oracle on exhaustive tiny inputs.

Also: the LZ77 factor count z (Section 2.1) by a quadratic greedy parse, used
for the per-level block bound 3*z*tau (Section 4, the lemma on blocks per level).
"""


def first_occurrences(T):
    """dict: substring -> smallest start, for every substring of T."""
    first = {}
    n = len(T)
    for p in range(n):
        for e in range(p + 1, n + 1):
            s = T[p:e]
            if s not in first:
                first[s] = p
    return first


def build(T, tau, leaf_len, b1, exact_split=True):
    """Return a list of levels (dicts) and the leaf bytes, following the
    definition literally.  Blocks are (start, length) tuples."""
    T = bytes(T)
    n = len(T)
    first = first_occurrences(T)
    blocks = [(s, min(b1, n - s)) for s in range(0, n, b1)]
    b = b1
    levels = []
    while True:
        if b <= leaf_len:
            leaves = b"".join(T[s:s + l] for s, l in blocks)
            levels.append(dict(b=b, c=len(blocks), marked=[0] * len(blocks), ptr=[]))
            return levels, leaves
        c = len(blocks)
        adj = [j + 1 < c and blocks[j + 1][0] == blocks[j][0] + blocks[j][1] for j in range(c)]
        marked = [0] * c
        for j in range(c):
            if adj[j]:
                s = blocks[j][0]
                X = T[s:s + blocks[j][1] + blocks[j + 1][1]]
                if first[X] == s:
                    marked[j] = marked[j + 1] = 1
        for j in range(c):
            if not (j > 0 and adj[j - 1]) and not adj[j]:
                marked[j] = 1
        ptr = []
        for j in range(c):
            if marked[j]:
                continue
            s, l = blocks[j]
            p = first[T[s:s + l]]
            t = max(k for k in range(c) if blocks[k][0] <= p)
            ptr.append((t, p - blocks[t][0]))
        levels.append(dict(b=b, c=c, marked=marked, ptr=ptr))
        nb = b // tau if exact_split else -(-b // tau)
        nxt = []
        for j in range(c):
            if marked[j]:
                s, l = blocks[j]
                for off in range(0, l, nb):
                    nxt.append((s + off, min(nb, l - off)))
        blocks, b = nxt, nb


def lz77_z(T):
    """Number of phrases of the greedy LZ77 parse where a phrase is the longest
    prefix of the rest with an earlier (possibly overlapping) occurrence, or a
    single new character when there is none."""
    T = bytes(T)
    n = len(T)
    i = z = 0
    while i < n:
        best = 0
        for j in range(i):
            k = 0
            while i + k < n and T[j + k] == T[i + k]:
                k += 1
            best = max(best, k)
        i += max(best, 1)
        z += 1
    return z
