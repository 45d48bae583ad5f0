"""Autotuner for the build's launch and sizing choices (bt_tuning).

None of the choices changes a tree; they trade memory for speed, and the best
values depend on the GPU and on the shape of the work.  For each shape class
the tuner builds a synthetic sample of that class, times candidate settings
(HIP-synchronised wall time, median of several builds) by coordinate descent
from the library's defaults, and keeps the fastest in a JSON cache keyed by GPU
architecture and shape class.  Contexts look the class of each build up in the
cache (``Context.build`` / ``Context.build_batch``) and apply its settings.

Shape classes:
  single-small   one text below 8 MiB
  single-large   one text of 8 MiB or more
  batch          several texts built together

  python -m paper_2512_23314_amd.autotune [--out FILE] [--reps K]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning.json")

# candidate values per setting and class, tried one setting at a time
CANDIDATES = {
    "single-small": {"table_load_log2": [1, 2], "filter2_max_log2": [20, 22, 24]},
    "single-large": {"table_load_log2": [1, 2], "filter2_max_log2": [22, 24, 26]},
    "batch": {"table_load_log2": [1, 2], "text_filter_bits_log2": [4, 5, 6],
              "span_chunks": [0, 32, 64, 128, 256]},
}


def cache_path():
    return os.environ.get("BT_TUNING_CACHE", DEFAULT_CACHE)


def arch_name(device=0):
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def shape_class(ntexts, nbytes):
    if ntexts > 1:
        return "batch"
    return "single-large" if nbytes >= (8 << 20) else "single-small"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(cache, arch, cls):
    """The tuned settings of (arch, cls), or None."""
    return cache.get(arch, {}).get(cls, {}).get("tuning")


def _samples():
    import numpy as np
    import torch
    import synth
    dev = "cuda:0"
    small = torch.from_numpy(synth.cfg1_text()).to(dev)
    large = torch.from_numpy(synth.cfg2_text()[:64 << 20]).to(dev)
    texts = synth.batch_texts()
    offs = np.zeros(len(texts) + 1, np.uint64)
    offs[1:] = np.cumsum([t.size for t in texts])
    batch = torch.from_numpy(np.concatenate(texts)).to(dev)
    return {
        "single-small": (lambda ctx: ctx.build(small, sigma=4, tau=2, leaf_len=16, tuned=False),
                         "1 MiB DNA text, tau 2, leaf 16"),
        "single-large": (lambda ctx: ctx.build(large, sigma=96, tau=4, leaf_len=16, tuned=False),
                         "first 64 MiB of the versioned text, tau 4, leaf 16"),
        "batch": (lambda ctx: ctx.build_batch(batch, offs, sigma=4, tau=4, leaf_len=16, tuned=False),
                  "the 4096-text batch (%.0f MiB), tau 4, leaf 16" % (int(offs[-1]) / 2**20)),
    }


def _time(ctx, fn, reps):
    import torch

    def free(r):
        for t in (r if isinstance(r, list) else [r]):
            t.free()
    free(fn(ctx))  # warm-up: the pool's blocks for this setting
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn(ctx)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        free(r)
    ts.sort()
    return ts[len(ts) // 2]


def tune(reps=5, classes=None, log=print):
    """Coordinate descent per class; returns {cls: {"tuning", "ms", "default_ms", "sample"}}."""
    from . import Context, DEFAULT_TUNING
    ctx = Context(0)
    out = {}
    samples = _samples()
    for cls, cands in CANDIDATES.items():
        if classes and cls not in classes:
            continue
        fn, desc = samples[cls]
        best = dict(DEFAULT_TUNING)
        ctx.set_tuning(**best)
        base = best_t = _time(ctx, fn, reps)
        log("%s: defaults %.2f ms" % (cls, base * 1e3))
        for name, values in cands.items():
            for v in values:
                if v == best[name]:
                    continue
                trial = dict(best, **{name: v})
                ctx.set_tuning(**trial)
                t = _time(ctx, fn, reps)
                log("  %s=%s: %.2f ms" % (name, v, t * 1e3))
                if t < best_t * 0.98:  # keep a change only for a clear gain
                    best, best_t = trial, t
            ctx.set_tuning(**best)
        ctx.trim()
        out[cls] = {"tuning": best, "ms": round(best_t * 1e3, 3), "default_ms": round(base * 1e3, 3),
                    "sample": desc, "reps": reps}
        log("%s: best %s, %.2f ms (defaults %.2f ms)" % (cls, best, best_t * 1e3, base * 1e3))
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=cache_path())
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--classes", nargs="*")
    a = ap.parse_args()
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    res = tune(a.reps, a.classes)
    cache = load_cache(a.out)
    cache.setdefault(arch_name(), {}).update(res)
    with open(a.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", a.out)


if __name__ == "__main__":
    main()
