"""Text generators (see the package docstring).  All functions are pure
functions of their arguments and seed."""
import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
# newline plus the 95 printable ASCII characters 0x20..0x7e
PRINTABLE96 = np.concatenate([np.array([10], np.uint8), np.arange(0x20, 0x7F, dtype=np.uint8)])

# per-configuration base seeds
CFG_SEEDS = {k: 0x5EED0000 + k for k in range(1, 6)}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _mutate(src, rng, sub_rate, indel_rate, indel_max, draw):
    """Copy src applying substitutions (a different symbol at a random position)
    and insertions/deletions (50:50, length U[1, indel_max]).  ``draw(k)`` returns
    k fresh symbols; substitutions pick a different symbol of the same alphabet
    by rotating its index."""
    m = src.size
    out = src.copy()
    k = rng.binomial(m, sub_rate) if m else 0
    if k:
        pos = rng.integers(0, m, k)
        out[pos] = draw(k, exclude=out[pos])
    k = rng.binomial(m, indel_rate) if m else 0
    if not k:
        return out
    pos = np.sort(rng.integers(0, m, k))
    lens = rng.integers(1, indel_max + 1, k)
    ins = rng.random(k) < 0.5
    pieces, prev = [], 0
    for p, l, is_ins in zip(pos.tolist(), lens.tolist(), ins.tolist()):
        if p < prev:
            continue
        pieces.append(out[prev:p])
        if is_ins:
            pieces.append(draw(l))
            prev = p
        else:
            prev = min(m, p + l)
    pieces.append(out[prev:])
    return np.concatenate(pieces)


def _alphabet_draw(rng, alphabet):
    sigma = alphabet.size
    index = np.full(256, -1, np.int64)
    index[alphabet] = np.arange(sigma)

    def draw(k, exclude=None):
        if exclude is None:
            return alphabet[rng.integers(0, sigma, k)]
        shift = rng.integers(1, sigma, k)
        return alphabet[(index[exclude] + shift) % sigma]

    return draw


def dna_copies(total_len, base_len, copies, sub_rate, indel_rate, indel_max, seed,
               alphabet=ACGT):
    """A uniform random base over ``alphabet``; ``copies`` independently mutated
    copies of it, concatenated, then cut (or extended with further copies) to
    exactly ``total_len`` bytes."""
    rng = _rng(seed)
    draw = _alphabet_draw(rng, alphabet)
    base = draw(base_len)
    parts, have, i = [], 0, 0
    while have < total_len:
        c = _mutate(base, rng, sub_rate, indel_rate, indel_max, draw)
        parts.append(c)
        have += c.size
        i += 1
        if i >= copies and have >= total_len:
            break
    return np.concatenate(parts)[:total_len] if parts else np.zeros(0, np.uint8)


def _markov_table(rng, sigma, zipf_s=1.5):
    """Order-2 chain: each context (a, b) ranks the symbols by a random
    permutation; rank r has probability proportional to (r+1)^-zipf_s."""
    perms = np.argsort(rng.random((sigma * sigma, sigma)), axis=1).astype(np.int64)
    w = 1.0 / np.arange(1, sigma + 1) ** zipf_s
    cdf = np.cumsum(w / w.sum())
    cdf[-1] = 1.0
    return perms, cdf


def _markov_run(rng, perms, cdf, sigma, length, a=0, b=0):
    ranks = np.searchsorted(cdf, rng.random(length), side="right").tolist()
    P = perms.tolist()
    out = [0] * length
    for k in range(length):
        s = P[a * sigma + b][ranks[k]]
        out[k] = s
        a, b = b, s
    return np.array(out, np.int64)


def markov_versions(total_len, base_len, versions, edit_rate, run_max, seed,
                    alphabet=PRINTABLE96):
    """Successive versions of a document.  Version 0 is an order-2 Markov chain
    sample of ``base_len`` symbols; version v+1 applies round(edit_rate*len)
    edit operations to version v, each a substitution, insertion or deletion
    (uniform) of a run of U[1, run_max] symbols; new symbols are slices of an
    independent chain sample.  Versions are concatenated and cut (or extended
    with further versions) to exactly ``total_len`` bytes."""
    rng = _rng(seed)
    sigma = alphabet.size
    perms, cdf = _markov_table(rng, sigma)
    cur = _markov_run(rng, perms, cdf, sigma, base_len)
    pool = _markov_run(rng, perms, cdf, sigma, max(4096, 64 * run_max))
    parts, have, v = [], 0, 0
    while have < total_len:
        parts.append(cur)
        have += cur.size
        v += 1
        if v >= versions and have >= total_len:
            break
        m = cur.size
        k = int(round(edit_rate * m))
        if k and m:
            pos = np.sort(rng.integers(0, m, k))
            lens = rng.integers(1, run_max + 1, k)
            ops = rng.integers(0, 3, k)
            srcs = rng.integers(0, pool.size - run_max, k)
            pieces, prev = [], 0
            for p, l, op, s in zip(pos.tolist(), lens.tolist(), ops.tolist(), srcs.tolist()):
                if p < prev:
                    continue
                pieces.append(cur[prev:p])
                if op == 0:      # substitute a run
                    pieces.append(pool[s:s + min(l, m - p)])
                    prev = min(m, p + l)
                elif op == 1:    # insert a run
                    pieces.append(pool[s:s + l])
                    prev = p
                else:            # delete a run
                    prev = min(m, p + l)
            pieces.append(cur[prev:])
            cur = np.concatenate(pieces)
    if not parts:
        return np.zeros(0, np.uint8)
    seq = np.concatenate(parts)[:total_len]
    return alphabet[seq]


def cfg1_text(n=1 << 20, seed=CFG_SEEDS[1]):
    """1 MiB DNA-like text: a 64 KiB base copied 16 times, 0.1% substitutions and
    0.01% indels of length 1-8 per copy."""
    return dna_copies(n, 64 << 10, 16, 1e-3, 1e-4, 8, seed)


def cfg2_text(n=1 << 28, base_len=256 << 10, versions=1024, seed=CFG_SEEDS[2]):
    """256 MiB versioned text, sigma=96: 256 KiB order-2 Markov base, 1024
    versions each with 0.05% edit operations (runs of 1-64)."""
    return markov_versions(n, base_len, versions, 5e-4, 64, seed)


def cfg3_text(n=1 << 31, ref_len=8 << 20, haplotypes=256, seed=CFG_SEEDS[3]):
    """2 GiB DNA collection: 256 haplotypes of an 8 MiB random reference with
    0.1% SNPs and 0.01% indels of length 1-20."""
    return dna_copies(n, ref_len, haplotypes, 1e-3, 1e-4, 20, seed)


def batch_lengths(count=4096, median=1 << 18, sigma_ln=1.665, lo=1 << 12, hi=1 << 26,
                  seed=CFG_SEEDS[4]):
    rng = _rng(seed)
    x = np.exp(rng.normal(np.log(median), sigma_ln, count))
    return np.clip(np.round(x), lo, hi).astype(np.int64)


def _batch_params(count, seed, **kw):
    lens = batch_lengths(count, seed=seed, **kw)
    rng = _rng(seed + 1)
    rates = rng.uniform(1e-4, 1e-2, count)
    seeds = rng.integers(0, 2**62, count)
    return lens.tolist(), rates.tolist(), seeds.tolist()


def batch_texts(count=4096, seed=CFG_SEEDS[4], **kw):
    """Independent texts of lognormal lengths, each generated like the 1 MiB DNA
    text (base = len/16, 16 copies) with its own seed and a substitution rate
    drawn from U[0.01%, 1%] (indel rate a tenth of it)."""
    out = []
    for n, r, s in zip(*_batch_params(count, seed, **kw)):
        out.append(dna_copies(n, max(1, n // 16), 16, r, r / 10, 8, int(s)))
    return out


def batch_text(i, count=4096, seed=CFG_SEEDS[4], **kw):
    """Text i of batch_texts(count, seed, ...), generated alone."""
    lens, rates, seeds = _batch_params(count, seed, **kw)
    n, r, s = lens[i], rates[i], seeds[i]
    return dna_copies(n, max(1, n // 16), 16, r, r / 10, 8, int(s))


def batch_lengths_of(count=4096, seed=CFG_SEEDS[4], **kw):
    """The lengths of batch_texts(count, seed, ...), without generating them."""
    return _batch_params(count, seed, **kw)[0]


def serving_sizes(count, median=1 << 18, sigma_ln=2.0, lo=1 << 10, hi=1 << 28, seed=CFG_SEEDS[5]):
    rng = _rng(seed)
    x = np.exp(rng.normal(np.log(median), sigma_ln, count))
    return np.clip(np.round(x), lo, hi).astype(np.int64)


def random_text(n, sigma, seed):
    """Uniform i.i.d. bytes over the first sigma byte values (or ACGT for 4)."""
    rng = _rng(seed)
    if sigma == 4:
        return ACGT[rng.integers(0, 4, n)]
    return rng.integers(0, sigma, n).astype(np.uint8)


def periodic_text(n, period, seed):
    """A random word of length ``period`` repeated to length n."""
    rng = _rng(seed)
    w = rng.integers(0, 256, period).astype(np.uint8)
    return np.resize(w, n)
