"""Write the full-size expected trees: SHA-256 of the canonical tree bytes of
each full-size workload, built by the threaded oracle construction
(``oracle.build_tree_par``, the paper's two-phase method on host threads).

Only ``oracle`` and ``synth`` are used; nothing here touches the GPU library.
Outputs (merged into what is already there, so runs can be split):
  fullsize_trees.json   one entry per single-text workload, plus the batch's
                        summary (input digest, digest over its trees)
  batch4096_trees.txt   one line per batch text: index, length, the first 16
                        hex digits of its tree's SHA-256

Usage: python tests/golden/make_fullsize.py [--only NAME ...] [--threads K]
Names: versioned256m, versioned256m_s (about 2^19 root blocks), dna1m and
dna1m_s (s about 10^4), dna2g_t<tau>_l<leaf> (tau in 2,4,8,16; leaf in 8,16,32),
batch4096.
"""
import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

JSON_PATH = os.path.join(HERE, "fullsize_trees.json")
BATCH_PATH = os.path.join(HERE, "batch4096_trees.txt")

DNA2G_SWEEP = [(tau, leaf) for tau in (4, 2, 8, 16) for leaf in (16, 8, 32)]


def _cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _load():
    if os.path.exists(JSON_PATH):
        with open(JSON_PATH) as f:
            return json.load(f)
    return {"about": "SHA-256 of canonical block-tree bytes built by the threaded oracle "
                     "construction; inputs from synth (seeded)", "entries": {}}


def _save(name, entry):
    """Merge one entry into the file as it is now on disk."""
    doc = _load()
    doc["entries"][name] = entry
    tmp = JSON_PATH + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, JSON_PATH)


def single(name, T, tau, leaf, threads, recipe, s_hint=1):
    t0 = time.time()
    tree = oracle.build_tree_par(T, tau, leaf, s_hint=s_hint, threads=threads, levels=False)
    dt = time.time() - t0
    return {
        "recipe": recipe,
        "n": int(T.size),
        "input_sha256": hashlib.sha256(T.tobytes()).hexdigest(),
        "tau": tau, "leaf_len": leaf, "s_hint": s_hint, "b1": int(tree.b1), "h": int(tree.h),
        "levels_b_c_u": [[int(L.b), int(L.c), int(L.u)] for L in tree.levels],
        "canonical_bytes": len(tree.canonical),
        "canonical_sha256": hashlib.sha256(tree.canonical).hexdigest(),
        "oracle_seconds": round(dt, 2), "oracle_threads": threads, "host_cpu": _cpu(),
    }


def batch(threads):
    lens = synth.batch_lengths_of()
    count = len(lens)
    order = sorted(range(count), key=lambda i: -lens[i])
    sha = [None] * count
    insha = [None] * count

    def one(i):
        T = synth.batch_text(i)
        tree = oracle.build_tree_par(T, 4, 16, threads=1, levels=False)
        return i, hashlib.sha256(T.tobytes()).hexdigest(), hashlib.sha256(tree.canonical).hexdigest()

    t0 = time.time()
    done = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        for i, a, b in ex.map(one, order):
            insha[i], sha[i] = a, b
            done += 1
            if done % 256 == 0:
                print("  batch4096: %d/%d texts, %.0f s" % (done, count, time.time() - t0), flush=True)
    dt = time.time() - t0
    with open(BATCH_PATH, "w") as f:
        f.write("# batch4096: index length sha256(canonical tree)[:16]; tau 4, leaf 16, s_hint 1\n")
        for i in range(count):
            f.write("%d %d %s\n" % (i, lens[i], sha[i][:16]))
    return {
        "recipe": "synth.batch_texts(): 4096 DNA copies texts, lognormal lengths",
        "texts": count, "n": int(sum(lens)),
        "input_digest": hashlib.sha256("".join(insha).encode()).hexdigest(),
        "tree_digest": hashlib.sha256("".join(sha).encode()).hexdigest(),
        "tau": 4, "leaf_len": 16, "s_hint": 1,
        "oracle_seconds": round(dt, 2), "oracle_threads": threads, "host_cpu": _cpu(),
        "per_text": os.path.basename(BATCH_PATH),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    a = ap.parse_args()
    names = ["versioned256m", "dna2g_t4_l16", "batch4096", "dna1m", "dna1m_s", "versioned256m_s"] + \
        ["dna2g_t%d_l%d" % p for p in DNA2G_SWEEP if p != (4, 16)]
    if a.only:
        names = [x for x in names if x in a.only]
    oracle.build()
    dna = None
    for name in names:
        print("%s ..." % name, flush=True)
        if name == "versioned256m":
            T = synth.cfg2_text()
            e = single(name, T, 4, 16, a.threads, "synth.cfg2_text(): 256 MiB versioned text, sigma 96")
        elif name == "versioned256m_s":
            T = synth.cfg2_text()
            e = single(name, T, 4, 16, a.threads, "synth.cfg2_text(): 256 MiB versioned text, sigma 96",
                       s_hint=1 << 19)
        elif name in ("dna1m", "dna1m_s"):
            T = synth.cfg1_text()
            e = single(name, T, 2, 16, a.threads, "synth.cfg1_text(): 1 MiB DNA, 16 copies of 64 KiB",
                       s_hint=1 if name == "dna1m" else 10000)
        elif name.startswith("dna2g"):
            if dna is None:
                dna = synth.cfg3_text()
            tau, leaf = (int(v[1:]) for v in name.split("_")[1:])
            e = single(name, dna, tau, leaf, a.threads,
                       "synth.cfg3_text(): 2 GiB, 256 haplotypes of an 8 MiB reference")
        elif name == "batch4096":
            e = batch(a.threads)
        else:
            raise SystemExit("unknown workload " + name)
        _save(name, e)
        print("%s: %s in %.0f s" % (name, e.get("canonical_sha256", e.get("tree_digest")),
                                    e["oracle_seconds"]), flush=True)


if __name__ == "__main__":
    main()
