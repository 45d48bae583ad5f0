"""Seeded synthetic repetitive texts shaped like the paper's inputs.

The paper measures on the Pizza&Chili repetitive corpus (DNA collections and
versioned documents, Section 6, Table 1), which is not available here.  These
generators stand in for it with the same structure: near-identical copies of a
base sequence (DNA-like, alphabet ACGT) and successive edited versions of a
document drawn from an order-2 Markov chain (96 printable symbols).

This module holds no part of the block-tree method; it only produces bytes.
Randomness: numpy's PCG64 generator, seeded per text.
"""
from .texts import (  # noqa: F401
    ACGT,
    PRINTABLE96,
    CFG_SEEDS,
    dna_copies,
    markov_versions,
    cfg1_text,
    cfg2_text,
    cfg3_text,
    batch_lengths,
    batch_texts,
    batch_text,
    batch_lengths_of,
    serving_sizes,
    random_text,
    periodic_text,
)
