"""Benchmark: block-tree construction throughput on one MI355X.

Default workload (the largest configuration that fits one GPU): 4096
independent DNA texts of lognormal length, about 3.9 GiB in total (tau = 4,
leaf_len = 16, one root block per text), built by one bt_build_batch call.  One
step = one complete batched build (prefix fingerprints, every level's two
phases, marks, pointers, split, leaves) with the texts already resident in HBM.
The plain per-text loop (bt_build_ex per text) is timed beside it.  Two legs
follow, each with its own roofline and parity check: the 2 GiB haplotype
collection (tau 4, leaf 16) and the 256 MiB versioned text (tau 4, leaf 16),
the latter with its pruned, memory-lean and sort-phase builds.  Prints one
JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Parity first: every tree a reported number rests on is serialized and its
SHA-256 compared with the expected tree in tests/golden/ (written by the
threaded oracle construction, tests/golden/make_fullsize.py).  A mismatch ends
the run with an error and no JSON line.

The roofline object covers the probe-scan kernel (the sliding-window probe,
the dominant kernel): its algorithmic bytes over its HIP-event time on the
library's stream.  Per window it reads two prefix values (4-byte 32-bit
pre-filter hashes, or 8-byte 61-bit fingerprints where it does not
pre-filter); a wave's tile of 1024 consecutive windows must fetch the union of
[i0, i0 + 1024) and [i0 + L, i0 + L + 1024), so a window costs
4 (1 + min(L, 1024) / 1024) bytes (twice that without the pre-filter).

The cpu_baseline object times the threaded oracle construction (the paper's
two-phase method, Section 4.1 over a domain decomposition, Section 5.2) on the
host's cores, on a bounded sample of the same workload, and on one core.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
METRIC = "block-tree build MB/s and KR-scan GB/s (% HBM peak) on 1 MI355X vs CPU oracle"
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")

WORKLOADS = {
    # name: (generator, sigma, tau, leaf_len, s_hint, expected-tree entry, description)
    "batch4096": ("cfg4", 4, 4, 16, 1, "batch4096",
                  "4096 DNA texts, lognormal lengths (median 256 KiB, 4 KiB-64 MiB, ~3.9 GiB), "
                  "each 16 mutated copies of a base: one batched build vs a loop of single builds"),
    "dna2g": ("cfg3", 4, 4, 16, 1, "dna2g_t4_l16",
              "2 GiB DNA collection, sigma 4: 256 haplotypes of an 8 MiB reference, 0.1% SNPs, "
              "0.01% indels of length 1-20"),
    "dna2g_sweep": ("cfg3sweep", 4, 0, 0, 1, None,
                    "the 2 GiB DNA collection built at every tau in {2,4,8,16} x leaf_len in "
                    "{8,16,32}, one root block"),
    "versioned256m": ("cfg2", 96, 4, 16, 1, "versioned256m",
                      "256 MiB versioned text, sigma 96: 1024 versions of a 256 KiB order-2 "
                      "Markov document, 0.05% edit runs per version"),
    "versioned256m_s": ("cfg2", 96, 4, 16, 1 << 19, "versioned256m_s",
                        "same text, about 2^19 root blocks (b1 = 256)"),
    "dna1m": ("cfg1", 4, 2, 16, 1, "dna1m", "1 MiB DNA: 16 mutated copies of a 64 KiB base"),
    "dna1m_s": ("cfg1", 4, 2, 16, 10000, "dna1m_s", "1 MiB DNA, s about 10^4 (b1 = 64)"),
    "serve": ("cfg5", 4, 4, 16, 1, None,
              "serving: Poisson build requests (lognormal sizes, median 256 KiB, 1 KiB-256 MiB, "
              "DNA texts) at 0.8x measured capacity, interleaved 1M-query batches"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_text(gen):
    import synth
    return {"cfg1": synth.cfg1_text, "cfg2": synth.cfg2_text, "cfg3": synth.cfg3_text}[gen]()


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def host_threads():
    """CPUs this process may use, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# ---------------------------------------------------------------- parity

class ParityError(RuntimeError):
    pass


def golden_entry(name):
    with open(os.path.join(GOLDEN_DIR, "fullsize_trees.json")) as f:
        entries = json.load(f)["entries"]
    if name not in entries:
        raise ParityError("no expected tree recorded for %s (tests/golden/make_fullsize.py)" % name)
    return entries[name]


def _sha(b):
    return hashlib.sha256(b).hexdigest()


def check_single(tree, name, T):
    """The GPU tree's canonical bytes against the expected tree of `name`."""
    e = golden_entry(name)
    if _sha(T.tobytes()) != e["input_sha256"]:
        raise ParityError("%s: the generated input differs from the recorded one" % name)
    got = _sha(tree.serialize())
    if got != e["canonical_sha256"]:
        raise ParityError("%s: GPU tree %s differs from the expected tree %s" % (
            name, got[:16], e["canonical_sha256"][:16]))
    return {"expected_tree": "tests/golden/fullsize_trees.json:" + name, "sha256": got,
            "match": True}


def check_batch(trees, name, insha_digest):
    e = golden_entry(name)
    if insha_digest != e["input_digest"]:
        raise ParityError("%s: the generated inputs differ from the recorded ones" % name)
    want = {}
    with open(os.path.join(GOLDEN_DIR, e["per_text"])) as f:
        for line in f:
            if not line.startswith("#"):
                i, _, h = line.split()
                want[int(i)] = h
    got, bad = [], []
    for i, tr in enumerate(trees):
        h = _sha(tr.serialize())
        got.append(h)
        if want.get(i) != h[:16]:
            bad.append(i)
    digest = _sha("".join(got).encode())
    if bad or digest != e["tree_digest"]:
        raise ParityError("%s: %d of %d trees differ from the expected ones (first %s)" % (
            name, len(bad), len(trees), bad[:8]))
    return {"expected_tree": "tests/golden/fullsize_trees.json:" + name, "trees": len(trees),
            "tree_digest": digest, "match": True}


# ---------------------------------------------------------------- roofline

def traffic_record(kernel, workload):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on this workload and on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != workload:
        return None
    if "sources" not in rec or _sources_sha(rec["sources"]) != rec.get("source_sha256"):
        return None
    return rec


# the files the probe scan is compiled from, and the host code that sizes its
# launches; a change to any of them retires the traffic record
PROBE_SOURCES = ["level.hip", "probe_text.hip", "probe.hpp", "common.hpp", "window.hpp",
                 "lean.hpp", "internal.hpp", "bt_host.cpp"]


def _sources_sha(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2512_23314_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def roofline(ctx, steps, workload):
    ps = ctx.kernel_stats("probe_scan")
    achieved = ps["bytes"] / ps["ms"] / 1e6 if ps["ms"] > 0 else 0.0
    tr = traffic_record("probe_scan", workload)
    traffic = tr.get("bytes_per_launch") if (tr is not None and ps["launches"]) else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "probe_scan",
            "launches_per_step": ps["launches"] // max(steps, 1),
            "bytes_per_launch": round(ps["bytes"] / max(ps["launches"], 1)),
            "avg_launch_ms": round(ps["ms"] / max(ps["launches"], 1), 5)}


def kernel_table(ctx, steps):
    """Per-kernel figures of the timed steps (HIP events on the library stream)."""
    out = {}
    for k in ("probe_scan", "byte_scan", "prefix_fp", "verify"):
        s = ctx.kernel_stats(k)
        if s["launches"]:
            out[k] = {"launches_per_step": s["launches"] // max(steps, 1),
                      "ms_per_step": round(s["ms"] / max(steps, 1), 4),
                      "algorithmic_GBps": round(s["bytes"] / max(s["ms"], 1e-9) / 1e6, 1)}
    return out


def probe_launches(ctx, steps):
    """The probe-scan launches of the last timed step: [L, windows, us, bytes]."""
    rows = [r for r in ctx.launches() if r[0] == "probe_scan"]
    per = len(rows) // max(steps, 1)
    return [[int(L), int(u), round(ms * 1e3, 1), int(by)] for _, L, u, ms, by in rows[-per:]] if per else []


def phase_totals(ctx, steps, path=None, workload=None):
    """Per-step sums of the phase counters of the timed steps (and the last
    step's phases as JSON lines to `path`)."""
    ph = ctx.phases()
    if not ph:
        return None
    per = len(ph) // max(steps, 1)
    if path:
        with open(path, "w") as f:
            for r in ph[-per:]:
                f.write(json.dumps(dict(r, workload=workload)) + "\n")
    keys = ("keys", "windows", "candidates", "verified", "collisions")
    return {k: sum(r[k] for r in ph) // max(steps, 1) for k in keys}


def base_line(workload, value, ms, steps, warmup, config):
    return {"metric": METRIC, "value": round(value, 2), "unit": "MB/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": dict({"workload": workload}, **config)}


# ---------------------------------------------------------------- CPU baseline

def cpu_baseline_batch(sample_mib, cores):
    """The threaded oracle construction on the first texts of the batch (in
    index order) up to sample_mib MiB: texts spread over `cores` host threads,
    one text per thread at a time; and the first texts up to 1/16 of that on
    one thread."""
    import concurrent.futures as cf
    import oracle
    import synth
    lens = synth.batch_lengths_of()
    pick, tot = [], 0
    for i, n in enumerate(lens):
        if tot >= (sample_mib << 20):
            break
        pick.append(i)
        tot += n
    texts = [synth.batch_text(i) for i in pick]

    def one(T):
        oracle.build_tree_par(T, 4, 16, threads=1, levels=False)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, sorted(texts, key=lambda t: -t.size)))
    dt = time.perf_counter() - t0
    small, stot = [], 0
    for T in texts:
        if stot >= tot // 16:
            break
        small.append(T)
        stot += T.size
    t1 = time.perf_counter()
    for T in small:
        one(T)
    dt1 = time.perf_counter() - t1
    return {"value": round(tot / dt / 1e6, 3), "unit": "MB/s", "cores": cores, "kind": "oracle",
            "sample": "texts 0..%d of the batch (%d texts, %.1f MiB), tau 4, leaf 16: the threaded "
                      "oracle construction, one text per host thread, %d threads, %.1f s"
                      % (pick[-1], len(pick), tot / 2**20, cores, dt),
            "one_core": {"value": round(stot / dt1 / 1e6, 3), "unit": "MB/s",
                         "sample": "the first %d of those texts (%.1f MiB), one thread, %.1f s"
                                   % (len(small), stot / 2**20, dt1)},
            "host_cpu": host_cpu(), "host_cpus_visible": os.cpu_count()}


def cpu_baseline_single(T, tau, leaf, s_hint, cores, sample_bytes):
    """The threaded oracle construction on the first sample_bytes of T (all of
    it when it is shorter) on `cores` threads."""
    import oracle
    S = T[:sample_bytes]
    t0 = time.perf_counter()
    oracle.build_tree_par(S, tau, leaf, s_hint=s_hint, threads=cores, levels=False)
    dt = time.perf_counter() - t0
    what = "the whole text" if S.size == T.size else "the first %d MiB of the text" % (S.size >> 20)
    return {"value": round(S.size / dt / 1e6, 3), "unit": "MB/s", "cores": cores, "kind": "oracle",
            "sample": "%s, tau %d, leaf %d, s_hint %d: the threaded oracle construction on %d "
                      "threads, %.1f s" % (what, tau, leaf, s_hint, cores, dt),
            "host_cpu": host_cpu(), "host_cpus_visible": os.cpu_count()}


# ---------------------------------------------------------------- workloads

def bench_batch(args, sigma, tau, leaf, golden, desc):
    """Batched build of the 4096 texts (the headline), the plain per-text loop
    over the same device buffer, parity of every tree, then the legs."""
    import numpy as np
    import torch
    import paper_2512_23314_amd as bt
    import synth
    t0 = time.time()
    texts = synth.batch_texts()
    offs = np.zeros(len(texts) + 1, np.uint64)
    offs[1:] = np.cumsum([len(t) for t in texts])
    insha = _sha("".join(_sha(t.tobytes()) for t in texts).encode())
    concat = np.concatenate(texts)
    del texts
    n = int(offs[-1])
    log("generated %d texts, %d bytes in %.1f s" % (len(offs) - 1, n, time.time() - t0))
    d = torch.from_numpy(concat).to("cuda:0")
    del concat
    torch.cuda.synchronize()
    ctx = bt.Context(0)

    def batched():
        return ctx.build_batch(d, offs, sigma=sigma, tau=tau, leaf_len=leaf)

    for _ in range(args.warmup):
        bt.free_trees(batched())
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        trees = batched()
        if k + 1 < args.steps:
            bt.free_trees(trees)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    ctx.profile(False)
    rf = roofline(ctx, args.steps, "batch4096")
    kt = kernel_table(ctx, args.steps)
    pl = probe_launches(ctx, args.steps)
    pt = phase_totals(ctx, args.steps, args.phase_log, "batch4096")
    if args.launch_log:
        with open(args.launch_log, "w") as f:
            json.dump({"workload": "batch4096", "probe_scan": pl}, f)
    parity = check_batch(trees, golden, insha)
    bt.free_trees(trees)
    log("batched %.1f ms (%.0f MB/s); parity: %d trees equal the expected ones" % (
        dt * 1e3, n / 1e6 / dt, parity["trees"]))
    plain = None
    if not args.no_plain:
        def loop():
            for k in range(len(offs) - 1):
                a, b = int(offs[k]), int(offs[k + 1])
                ctx.build(d[a:b], sigma=sigma, tau=tau, leaf_len=leaf).free()
        loop()  # the plain path's allocations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loop()
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        plain = {"batched_mb_s": round(n / 1e6 / dt, 2), "plain_loop_mb_s": round(n / 1e6 / dtp, 2),
                 "speedup": round(dtp / dt, 2), "plain_loop_ms": round(dtp * 1e3, 1)}
        log("plain loop %.1f ms (%.0f MB/s)" % (dtp * 1e3, n / 1e6 / dtp))
    lean = None
    if not args.no_legs:
        lean = batch_lean_leg(ctx, d, offs, n, sigma, tau, leaf, golden, insha)
        log("lean batch: %s" % lean)
    ctx.close()
    del d
    torch.cuda.empty_cache()
    out = base_line("batch4096", n / 1e6 / dt, dt * 1e3, args.steps, args.warmup,
                    {"description": desc, "n": n, "texts": len(offs) - 1, "sigma": sigma,
                     "tau": tau, "leaf_len": leaf, "s_hint": 1})
    out["roofline"] = rf
    out["cpu_baseline"] = None
    out["parity"] = parity
    if plain is not None:
        out["batched_vs_plain"] = plain
    if lean is not None:
        out["lean_build"] = lean
    out["kernels"] = kt
    out["probe_scan_launches"] = {"columns": ["L", "windows", "us", "algorithmic_bytes"], "rows": pl}
    out["phase_counters_per_step"] = pt
    return out


def bench_sweep(args, desc):
    """Every (tau, leaf) point of the 2 GiB DNA collection's sweep: each point's
    tree is checked against its expected tree, then timed (1 warm-up, then
    min(steps, 3) builds)."""
    import torch
    import paper_2512_23314_amd as bt
    import synth
    T = synth.cfg3_text()
    n = int(T.size)
    d = torch.from_numpy(T).to("cuda:0")
    torch.cuda.synchronize()
    ctx = bt.Context(0)
    steps = max(1, min(args.steps, 3))
    rows, tot_ms = [], 0.0
    for tau in (2, 4, 8, 16):
        for leaf in (8, 16, 32):
            name = "dna2g_t%d_l%d" % (tau, leaf)
            tree = ctx.build(d, sigma=4, tau=tau, leaf_len=leaf)
            parity = check_single(tree, name, T)
            h = tree.height
            tree.free()
            ctx.reset_stats()
            ctx.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.build(d, sigma=4, tau=tau, leaf_len=leaf).free()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            ctx.profile(False)
            rf = roofline(ctx, steps, name)
            tot_ms += ms
            rows.append({"tau": tau, "leaf_len": leaf, "levels": h, "ms_per_build": round(ms, 3),
                         "mb_s": round(n / 1e6 / (ms / 1e3), 1), "probe_scan_frac": rf["frac"],
                         "probe_scan_ms": round(rf["avg_launch_ms"] * rf["launches_per_step"], 3),
                         "tree_sha256": parity["sha256"][:16]})
            log("%s: %.1f ms, %.0f MB/s, %d levels, probe scan %.3f of peak" % (
                name, ms, n / 1e6 / (ms / 1e3), h, rf["frac"]))
    ctx.close()
    out = base_line("dna2g_sweep", 12 * n / 1e6 / (tot_ms / 1e3), tot_ms / 12, steps, 1,
                    {"description": desc, "n": n, "sigma": 4, "points": 12})
    out["roofline"] = None
    out["cpu_baseline"] = None
    out["parity"] = {"expected_trees": "tests/golden/fullsize_trees.json:dna2g_t*_l*", "match": True}
    out["sweep"] = rows
    return out


def bench_single(args, workload, steps, warmup, sublegs=False):
    import torch
    import paper_2512_23314_amd as bt
    gen, sigma, tau, leaf, s_hint, golden, desc = WORKLOADS[workload]
    t0 = time.time()
    T = make_text(gen)
    log("generated %s (%d bytes) in %.1f s" % (workload, T.size, time.time() - t0))
    n = int(T.size)
    d = torch.from_numpy(T).to("cuda:0")
    torch.cuda.synchronize()
    ctx = bt.Context(0)

    def step(prune=args.prune, lean=args.lean, keep=False):
        tree = ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint, prune=prune, lean=lean)
        if keep:
            return tree
        h = tree.height
        tree.free()
        return h

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(steps):
        tree = step(keep=True)
        if k + 1 < steps:
            tree.free()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(False)
    ms = dt / max(steps, 1) * 1e3
    h = tree.height
    rf = roofline(ctx, steps, workload)
    kt = kernel_table(ctx, steps)
    pl = probe_launches(ctx, steps)
    pt = phase_totals(ctx, steps, args.phase_log if workload == args.workload else None, workload)
    if args.launch_log and workload == args.workload:
        with open(args.launch_log, "w") as f:
            json.dump({"workload": workload, "probe_scan": pl}, f)
    parity = None
    if not args.prune:  # the expected trees are unpruned; lean builds give the same tree
        parity = check_single(tree, golden, T)
    tree.free()
    for k, s in kt.items():
        log("%-10s %s" % (k, s))
    out = base_line(workload, n / 1e6 / (ms / 1e3), ms, steps, warmup,
                    {"description": desc, "n": n, "sigma": sigma, "tau": tau, "leaf_len": leaf,
                     "s_hint": s_hint, "levels": h, "prune": bool(args.prune),
                     "lean": bool(args.lean)})
    out["roofline"] = rf
    out["parity"] = parity
    out["kernels"] = kt
    out["probe_scan_launches"] = {"columns": ["L", "windows", "us", "algorithmic_bytes"], "rows": pl}
    out["phase_counters_per_step"] = pt
    if sublegs:
        if not args.prune:
            out["pruned_build"] = pruned_leg(ctx, d, n, sigma, tau, leaf, s_hint, step)
            log("pruned build: %s" % out["pruned_build"])
        if not args.lean:
            out["lean_build"] = lean_leg(ctx, d, n, sigma, tau, leaf, s_hint, step)
            log("lean build: %s" % out["lean_build"])
        out["sort_phase_build"] = sort_leg(ctx, d, n, sigma, tau, leaf, s_hint, ms)
        log("sort-phase build: %s" % out["sort_phase_build"])
        out["rank_select_build"] = rank_leg(ctx, d, T, sigma, tau, leaf, s_hint, ms, golden)
        log("rank/select build: %s" % out["rank_select_build"])
    ctx.close()
    del d
    torch.cuda.empty_cache()
    return out, T


# ---------------------------------------------------------------- profile summaries
# These turn rocprofv3 output (CSV) into the short text summaries kept under
# profiles/; they read files only and never touch a GPU.

def _find_csv(d, suffix):
    for root, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, d))


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short_name(name):
    """'void bt::k_probe_scan<2, false, false>(bt::PhaseArgs, ...)' -> 'k_probe_scan<2, false, false>'"""
    s = name[5:] if name.startswith("void ") else name
    s = s.replace("(anonymous namespace)::", "")
    depth, cut = 0, len(s)
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    s = s[:cut]
    return s[4:] if s.startswith("bt::") else s


def _bench_line(path):
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    raise ValueError("no bench JSON line in %s" % path)


def summarize_stats(stats_dir, bench_json, cmd, out, top=20):
    rows = _csv_rows(_find_csv(stats_dir, "kernel_stats.csv"))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    b = _bench_line(bench_json)
    probe = [r for r in rows if any(k in r["Name"] for k in PROBE_KERNELS)]
    calls = sum(int(r["Calls"]) for r in probe)
    pns = sum(float(r["TotalDurationNs"]) for r in probe)
    rf = b["roofline"]
    lines = ["# Kernel time, %s build" % b["config"]["workload"], "",
             "Command (repository root, one MI355X):", "", "    " + cmd, "",
             "Bench line of the same run: %.2f %s, %.3f ms per step, probe_scan average "
             "launch %.4f ms (HIP events on the library stream), %d launches per step." % (
                 b["value"], b["unit"], b["ms_per_step"], rf["avg_launch_ms"], rf["launches_per_step"]),
             "",
             "rocprofv3: the probe scan (k_probe_scan and k_probe_text, all instantiations) %d "
             "calls, average %.4f ms "
             "(ratio to the HIP-event average %.3f); warmup and timed steps launch the same "
             "kernels, so the averages compare." % (calls, pns / max(calls, 1) / 1e6,
                                                     pns / max(calls, 1) / 1e6 / rf["avg_launch_ms"]),
             "", "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append("| %s | %s | %.3f | %.1f | %.1f |" % (
            _short_name(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / total))
    lines.append("| (all kernels) | %d | %.3f | | 100 |" % (sum(int(r["Calls"]) for r in rows), total / 1e6))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out)


# the probe scan's kernels: the shared-filter scan and the per-text scan of batches
PROBE_KERNELS = ("k_probe_scan<", "k_probe_text<")


def _counter_per_launch(d, needles):
    needles = (needles,) if isinstance(needles, str) else needles
    rows = [r for r in _csv_rows(_find_csv(d, "counter_collection.csv"))
            if any(nd in r["Kernel_Name"] for nd in needles)]
    if not rows:
        raise ValueError("no %s dispatches in %s" % (needles, d))
    return sum(float(r["Counter_Value"]) for r in rows) / len(rows), len(rows)


def summarize_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib, bench_json, cmds,
                      out_md, out_json, kernel="probe_scan", sources=None):
    sources = sources or PROBE_SOURCES
    copy_bytes = copy_mib << 20
    cf, _ = _counter_per_launch(cfetch_dir, "copyBuffer")
    cw, _ = _counter_per_launch(cwrite_dir, "copyBuffer")
    # a copy of B bytes reads B and writes B: scale each counter (KiB) to that
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    kf, n = _counter_per_launch(fetch_dir, PROBE_KERNELS)
    kw, _ = _counter_per_launch(write_dir, PROBE_KERNELS)
    fetch, write = kf * 1024.0 * ff, kw * 1024.0 * fw
    b = _bench_line(bench_json)
    algo = b["roofline"].get("bytes_per_launch")
    rec = {"kernel": kernel, "sources": sources, "source_sha256": _sources_sha(sources),
           "workload": b["config"]["workload"], "launches": n,
           "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "bytes_per_launch": round(fetch + write), "algorithmic_bytes_per_launch": algo,
           "fetch_scale": ff, "write_scale": fw}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    lines = ["# HBM traffic of %s, %s build" % (kernel, b["config"]["workload"]), "",
             "Commands (repository root, one MI355X, each its own run):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["",
              "Calibration: a device copy of %d MiB reads FETCH_SIZE %.1f KiB and WRITE_SIZE "
              "%.1f KiB per dispatch, so the scale factors are %.4f (fetch) and %.4f (write)." % (
                  copy_mib, cf, cw, ff, fw), "",
              "| per launch (average of %d) | bytes |" % n, "|---|---:|",
              "| FETCH_SIZE, scaled | %.4g |" % fetch, "| WRITE_SIZE, scaled | %.4g |" % write,
              "| traffic (fetch + write) | %.4g |" % (fetch + write)]
    if algo:
        lines += ["| algorithmic (the two prefix values per window: 8 B pre-filtered, 16 B "
                  "otherwise) | %.4g |" % algo,
                  "| traffic / algorithmic | %.3f |" % ((fetch + write) / algo)]
    lines += ["", "Source hash (SHA-256 of %s, in that order): %s" % (", ".join(sources),
                                                                     rec["source_sha256"])]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md, out_json)


def summarize_calibration(copy_fetch, copy_write, read_fetch, gather_fetch, mib, cmds, out_md):
    """The FETCH_SIZE scale factor from three access patterns of known size: a
    copy (stream in, stream out), a streaming read, and random 8-byte gathers
    (a cache line fetched per row)."""
    mib = int(mib)
    nb = mib << 20
    cf, _ = _counter_per_launch(copy_fetch, "copyBuffer")
    cw, _ = _counter_per_launch(copy_write, "copyBuffer")

    def largest(d):
        # the run's main dispatch: the fills that make its inputs only write, and
        # a reduction's second pass is small, so it is the one that fetches most
        per = {}
        for r in _csv_rows(_find_csv(d, "counter_collection.csv")):
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        if not per:
            raise ValueError("no dispatches in %s" % d)
        return max(per.values())
    rf = largest(read_fetch)
    gf = largest(gather_fetch)
    rows = 1 << 24
    lines = ["# FETCH_SIZE and WRITE_SIZE calibration on MI355X", "",
             "Commands (repository root, one MI355X, each its own run):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["", "| kernel | known bytes | counter, KiB per dispatch | known / counter |",
              "|---|---:|---:|---:|",
              "| copy of %d MiB, FETCH_SIZE | %d read | %.1f | %.4f |" % (mib, nb, cf, nb / (cf * 1024.0)),
              "| copy of %d MiB, WRITE_SIZE | %d written | %.1f | %.4f |" % (mib, nb, cw, nb / (cw * 1024.0)),
              "| streaming read of %d MiB, FETCH_SIZE | %d read | %.1f | %.4f |" % (
                  mib, nb, rf, nb / (rf * 1024.0)),
              "", "Random gathers: 2^24 rows of 8 bytes from an array far larger than the caches "
              "(its size is in the command); the indices (8 B each) stream in.  FETCH_SIZE %.1f KiB "
              "per dispatch; with the copy's fetch factor that is %.1f bytes per row beyond the "
              "indices (a row costs one cache line from HBM)." % (
                  gf, (gf * 1024.0 * nb / (cf * 1024.0) - rows * 8) / rows)]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def summarize_sweep(bench_json, cmd, out_md):
    """Markdown table of a --workload dna2g_sweep line."""
    b = _bench_line(bench_json)
    lines = ["# 2 GiB DNA collection: the tau x leaf_len sweep", "",
             "Command (repository root, one MI355X):", "", "    " + cmd, "",
             "Each point's tree was first compared with its expected tree "
             "(tests/golden/fullsize_trees.json, written by the threaded oracle construction): "
             "all twelve equal.  Then 1 warm-up and %d timed builds per point, text resident in HBM; "
             "probe-scan fraction = algorithmic bytes (same-tile rule) over HIP-event time, against "
             "8 TB/s." % b["steps"], "",
             "| tau | leaf | levels | ms per build | MB/s | probe scan ms | probe scan frac | "
             "tree SHA-256 (first 16) |", "|---:|---:|---:|---:|---:|---:|---:|---|"]
    for r in b["sweep"]:
        lines.append("| %d | %d | %d | %.1f | %.0f | %.1f | %.3f | %s |" % (
            r["tau"], r["leaf_len"], r["levels"], r["ms_per_build"], r["mb_s"], r["probe_scan_ms"],
            r["probe_scan_frac"], r["tree_sha256"]))
    lines += ["", "All twelve builds: %.0f MB/s (%.1f ms per build on average)." % (
        b["value"], b["ms_per_step"])]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def summarize_phases(jsonl, cmd, out_md):
    """Markdown table of the per-phase device counters that --phase-log wrote
    (one build; phases with keys only)."""
    rows = [json.loads(line) for line in open(jsonl) if line.strip()]
    wl = rows[0].get("workload", "?") if rows else "?"
    lines = ["# Per-phase device counters, one %s build" % wl, "",
             "Command (repository root, one MI355X):", "", "    " + cmd, "",
             "From bt_ctx_phase_record (the JSON lines are in %s beside this file).  keys: keys "
             "inserted (those the level above proved copies stay out); candidates: windows that "
             "passed the filters and probed the table; verified: keys whose leftmost hit is not "
             "their own start, compared byte by byte; collisions: verifications that failed, "
             "resolved by the exact retry walk." % os.path.basename(jsonl), "",
             "| b | phase | blocks | keys | windows | candidates | candidates / window | "
             "candidates / key | verified | collisions |",
             "|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        if not r["keys"]:
            continue
        lines.append("| %d | %d | %d | %d | %d | %d | %.4f | %.2f | %d | %d |" % (
            r["b"], r["phase"], r["blocks"], r["keys"], r["windows"], r["candidates"],
            r["candidates"] / max(r["windows"], 1), r["candidates"] / max(r["keys"], 1),
            r["verified"], r["collisions"]))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def bench_serve(args, sigma, tau, leaf, desc, seconds=10.0):
    """Open-loop serving: Poisson build arrivals at 0.8x the capacity measured by a
    closed-loop burst, 1M-query batches (a third each of access, rank, select)
    against random resident trees."""
    import numpy as np
    import torch
    import synth
    from paper_2512_23314_amd.serve import Server
    rng = np.random.default_rng(synth.CFG_SEEDS[5])
    sizes = synth.serving_sizes(384)
    t0 = time.time()
    pool = [synth.dna_copies(int(s), max(1, int(s) // 16), 16, 1e-3, 1e-4, 8, int(rng.integers(1 << 30)))
            for s in sizes]
    log("generated %d request texts (%.0f MiB) in %.1f s" % (
        len(pool), sum(len(p) for p in pool) / 2**20, time.time() - t0))
    dpool = [torch.from_numpy(p).to("cuda:0") for p in pool]
    torch.cuda.synchronize()
    mean = float(np.mean([len(p) for p in pool]))

    def run(srv, arrivals, query_every):
        """arrivals: list of (time, pool index).  Returns wall seconds."""
        futs, rids, seen = [], [], []
        qfuts = []
        t_start = time.perf_counter()
        next_q = query_every
        for ta, k in arrivals:
            now = time.perf_counter() - t_start
            if ta > now:
                time.sleep(ta - now)
            futs.append(srv.submit_build(dpool[k]))
            now = time.perf_counter() - t_start
            if query_every and now >= next_q:
                if rids:
                    rid = rids[int(rng.integers(len(rids)))]
                    n = srv.tree(rid).n
                    m = 1 << 20
                    third = m // 3
                    pos = torch.randint(0, max(n, 1), (m,), device="cuda:0").to(torch.uint64)
                    cs = torch.from_numpy(np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, m)]).to("cuda:0")
                    ks = torch.randint(1, max(2, n // 8), (m,), device="cuda:0").to(torch.uint64)
                    qfuts.append(srv.submit_queries(rid, "access", pos[:third]))
                    qfuts.append(srv.submit_queries(rid, "rank", cs[third:2 * third], pos[third:2 * third]))
                    qfuts.append(srv.submit_queries(rid, "select", cs[2 * third:], ks[2 * third:]))
                next_q += query_every
            # keep the resident set bounded (oldest finished trees first)
            for f in futs[len(seen):]:
                if not f.done():
                    break
                seen.append(int(f.result()))
                rids.append(seen[-1])
            while len(rids) > 128:
                srv.release(rids.pop(0))
        for f in futs:
            f.result()
        for q in qfuts:
            q.result()
        return time.perf_counter() - t_start

    # capacity: closed-loop burst
    srv = Server(budget=96 << 30, slots=3, max_batch=256, tau=tau, leaf_len=leaf, sigma=sigma)
    burst = [(0.0, k) for k in range(len(pool))]
    dt = run(srv, burst, 0)
    cap = sum(len(p) for p in pool) / dt
    srv.close()
    lam = 0.8 * cap / mean
    log("capacity %.0f MB/s (burst of %d requests in %.2f s); Poisson rate %.1f req/s" % (
        cap / 1e6, len(pool), dt, lam))
    t, arrivals = 0.0, []
    while t < seconds:
        t += float(rng.exponential(1.0 / lam))
        arrivals.append((t, int(rng.integers(len(pool)))))
    srv = Server(budget=96 << 30, slots=3, max_batch=256, tau=tau, leaf_len=leaf, sigma=sigma)
    wall = run(srv, arrivals, 0.1)
    st = srv.stats()
    srv.close()
    served = st["built_bytes"] / wall
    log("served %s" % st)
    out = {
        "metric": METRIC,
        "value": round(served / 1e6, 2), "unit": "MB/s", "n_gpus": 1, "steps": len(arrivals),
        "warmup": len(pool), "ms_per_step": round(wall / max(len(arrivals), 1) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serve", "description": desc, "requests": len(arrivals),
                   "rate_per_s": round(lam, 2), "seconds": round(wall, 2), "tau": tau,
                   "leaf_len": leaf, "sigma": sigma},
        "serving": {"build_p50_ms": st["build_p50_ms"], "build_p99_ms": st["build_p99_ms"],
                    "query_batch_p50_ms": st["query_p50_ms"], "query_batch_p99_ms": st["query_p99_ms"],
                    "query_batches": st["query_batches"], "build_batches": st["batches"],
                    "capacity_mb_s": round(cap / 1e6, 2)},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def pruned_leg(ctx, d, n, sigma, tau, leaf, s_hint, step, steps=3):
    """The same build with the optional pruning phase: rate and marked blocks."""
    import torch
    step(prune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(prune=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    marked = {}
    for pr in (False, True):
        tree = ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint, prune=pr)
        marked[pr] = int(sum(int(tree.level(l)[1].sum()) for l in range(1, tree.height)))
        leaves = int(tree.level_info(tree.height)[1])
        marked[pr] = (marked[pr], leaves)
        tree.free()
    return {"value": round(n / 1e6 / (ms / 1e3), 2), "unit": "MB/s", "ms_per_step": round(ms, 3),
            "steps": steps, "marked_blocks": marked[True][0], "marked_blocks_unpruned": marked[False][0],
            "leaf_blocks": marked[True][1], "leaf_blocks_unpruned": marked[False][1]}


def peak_build_bytes(ctx, d, sigma, tau, leaf, s_hint, lean):
    """Most device memory the pool hands out during one build (scratch plus the
    finished tree's storage), over what it held before."""
    import torch
    torch.cuda.synchronize()
    base = ctx.memory()["in_use"]
    ctx.reset_peak()
    tree = ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint, lean=lean)
    peak = ctx.memory()["peak"] - base
    tree.free()
    return peak


def batch_lean_leg(ctx, d, offs, n, sigma, tau, leaf, golden, insha, steps=2):
    """The batch built memory-lean (prefix fingerprints and 32-bit hashes kept
    one in 16): parity of every tree, rate, and peak pool bytes of one build
    against the dense build's."""
    import torch
    import paper_2512_23314_amd as bt

    def build(lean):
        return ctx.build_batch(d, offs, sigma=sigma, tau=tau, leaf_len=leaf, lean=lean)

    def peak(lean):
        torch.cuda.synchronize()
        base = ctx.memory()["in_use"]
        ctx.reset_peak()
        trees = build(lean)
        p = ctx.memory()["peak"] - base
        bt.free_trees(trees)
        return p
    trees = build(True)
    parity = check_batch(trees, golden, insha)
    bt.free_trees(trees)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.free_trees(build(True))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    dense, lean = peak(False), peak(True)
    return {"value": round(n / 1e6 / (ms / 1e3), 2), "unit": "MB/s", "ms_per_step": round(ms, 3),
            "steps": steps, "parity_trees": parity["trees"], "peak_build_bytes": lean,
            "peak_build_bytes_dense": dense, "peak_bytes_per_text_byte": round(lean / n, 3),
            "peak_bytes_per_text_byte_dense": round(dense / n, 3)}


def lean_leg(ctx, d, n, sigma, tau, leaf, s_hint, step, steps=3):
    """The same build with sampled prefix fingerprints: rate and peak memory."""
    import torch
    step(prune=False, lean=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(prune=False, lean=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    dense = peak_build_bytes(ctx, d, sigma, tau, leaf, s_hint, False)
    lean = peak_build_bytes(ctx, d, sigma, tau, leaf, s_hint, True)
    return {"value": round(n / 1e6 / (ms / 1e3), 2), "unit": "MB/s", "ms_per_step": round(ms, 3),
            "steps": steps, "peak_build_bytes": lean, "peak_build_bytes_dense": dense,
            "peak_bytes_per_text_byte": round(lean / n, 3),
            "peak_bytes_per_text_byte_dense": round(dense / n, 3)}


def rank_leg(ctx, d, T, sigma, tau, leaf, s_hint, plain_ms, golden, steps=3):
    """Builds with the rank/select support (bt_build's configuration): the same
    tree (checked against the expected one), rate, the support's device bytes
    per text byte, and what 32-bit counters for every block and pointer would
    take on the same tree."""
    import numpy as np
    import torch
    n = int(T.size)

    def one():
        return ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint, rank_select=True)
    tree = one()
    parity = check_single(tree, golden, T)
    counts = [tree.level_info(l) for l in range(1, tree.height + 1)]
    rb = tree.rank_bytes()
    tree.free()
    S = int(np.count_nonzero(np.bincount(T, minlength=256)))  # the support's alphabet
    dense = sum(4 * S * (c + u) + 8 * c for _, c, u in counts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one().free()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return {"value": round(n / 1e6 / (ms / 1e3), 2), "unit": "MB/s", "ms_per_step": round(ms, 3),
            "steps": steps, "support_ms": round(ms - plain_ms, 3), "symbols": S,
            "support_bytes": rb, "support_bytes_per_text_byte": round(rb / n, 3),
            "support_bytes_32bit_form": dense,
            "support_bytes_per_text_byte_32bit_form": round(dense / n, 3), "parity": parity}


def sort_leg(ctx, d, n, sigma, tau, leaf, s_hint, hash_ms, steps=2):
    """The same build with the sort-based phases of Section 5.1 in place of the
    hash-table scan (same tree): rate, and its sort time per build."""
    import torch
    import paper_2512_23314_amd as bt

    def one():
        ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint,
                  debug_flags=bt.BT_DBG_SORT_PHASES).free()
    one()
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ctx.profile(False)
    st = ctx.kernel_stats("sort_phase")
    return {"value": round(n / 1e6 / (ms / 1e3), 2), "unit": "MB/s", "ms_per_step": round(ms, 3),
            "steps": steps, "sort_ms_per_step": round(st["ms"] / steps, 3),
            "slowdown_vs_hashing": round(ms / hash_ms, 2)}


def summarize_launches(launch_json, pmc_dirs, calib, cmds, out_md):
    """Per-launch table of the probe scan for one build: the bench's launch log
    (window length, windows, HIP-event time, algorithmic bytes) joined in
    dispatch order with per-dispatch rocprofv3 counters from --pmc runs of the
    same command.  calib: (copy MiB, fetch dir, write dir) of the copy
    calibration, or None."""
    import collections
    with open(launch_json) as f:
        rec = json.load(f)
    rows = rec["probe_scan"]
    per = collections.OrderedDict()
    for d in pmc_dirs:
        for r in _csv_rows(_find_csv(d, "counter_collection.csv")):
            if not any(k in r["Kernel_Name"] for k in PROBE_KERNELS):
                continue
            key = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
            per.setdefault(r["Counter_Name"], collections.OrderedDict())[key] = float(r["Counter_Value"])
    counters = {k: [v[x] for x in sorted(v)] for k, v in per.items()}
    ff = fw = None
    if calib:
        mib, cfd, cwd = calib
        cf, _ = _counter_per_launch(cfd, "copyBuffer")
        cw, _ = _counter_per_launch(cwd, "copyBuffer")
        ff, fw = (mib << 20) / (cf * 1024.0), (mib << 20) / (cw * 1024.0)
    names = sorted(counters)
    lines = ["# Probe-scan launches, one %s build" % rec["workload"], "",
             "Commands (repository root, one MI355X, each its own run):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["", "Window length L, windows, HIP-event time and algorithmic bytes come from the "
              "library's launch log (bt_ctx_launch_record); the counters are rocprofv3 --pmc values "
              "per dispatch, joined in dispatch order."]
    if ff:
        lines += ["FETCH_SIZE and WRITE_SIZE are scaled to bytes with the copy calibration "
                  "(x%.4f and x%.4f)." % (ff, fw)]
    head = ["#", "L", "windows", "us", "algorithmic GB/s"] + names
    lines += ["", "| " + " | ".join(head) + " |", "|" + "---:|" * len(head)]
    for k, (L, w, us, by) in enumerate(rows):
        cells = [str(k), str(L), str(w), "%.1f" % us, "%.0f" % (by / us / 1e3 if us else 0)]
        for nm in names:
            v = counters[nm][k] if k < len(counters[nm]) else float("nan")
            if nm == "FETCH_SIZE" and ff:
                cells.append("%.3g B" % (v * 1024 * ff))
            elif nm == "WRITE_SIZE" and fw:
                cells.append("%.3g B" % (v * 1024 * fw))
            else:
                cells.append("%.4g" % v)
        lines.append("| " + " | ".join(cells) + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out_md)


def leg_view(line):
    """A leg's own figures, without the fields the main line already states."""
    drop = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "dtype", "data")
    return {k: v for k, v in line.items() if k not in drop}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch4096", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="batch4096: skip the 2 GiB and 256 MiB legs; versioned256m: skip the "
                         "pruned, lean and sort-phase builds")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch4096: skip the plain per-text loop")
    ap.add_argument("--prune", action="store_true",
                    help="single-text workloads: time builds with the optional pruning phase")
    ap.add_argument("--lean", action="store_true",
                    help="single-text workloads: time memory-lean builds (sampled fingerprints)")
    ap.add_argument("--cpu-sample-mib", type=int, default=512,
                    help="bytes of the workload the CPU baseline builds")
    ap.add_argument("--launch-log", metavar="FILE",
                    help="write the probe-scan launches of the last timed step as JSON")
    ap.add_argument("--phase-log", metavar="FILE",
                    help="write the per-phase device counters of the last timed step as JSON lines")
    ap.add_argument("--calibrate-read", type=int, default=0, metavar="MIB",
                    help="run a streaming read of MIB MiB three times (traffic calibration)")
    ap.add_argument("--calibrate-gather", type=int, default=0, metavar="MIB",
                    help="gather 2^24 random 8-byte rows from MIB MiB three times (traffic calibration)")
    ap.add_argument("--summarize-sweep", metavar="BENCH_JSON",
                    help="markdown table of a --workload dna2g_sweep run's JSON line")
    ap.add_argument("--summarize-phases", metavar="JSONL",
                    help="markdown table of the per-phase counters that --phase-log wrote")
    ap.add_argument("--summarize-calibration", nargs=5,
                    metavar=("COPY_FETCH", "COPY_WRITE", "READ_FETCH", "GATHER_FETCH", "MIB"),
                    help="counter directories of the copy, read and gather runs, and their MiB")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (the "
                         "known-size reference for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="write a markdown summary of a rocprofv3 --stats run (no GPU)")
    ap.add_argument("--summarize-traffic", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the probe_scan traffic record from four --pmc runs (no GPU)")
    ap.add_argument("--summarize-launches", nargs="+", metavar="PATH",
                    help="LAUNCH_JSON PMC_DIR...: the per-launch probe-scan table (no GPU)")
    ap.add_argument("--calib-dirs", nargs=2, metavar=("COPY_FETCH_DIR", "COPY_WRITE_DIR"))
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--bench-json", help="stdout of the profiled bench run")
    ap.add_argument("--profile-cmd", action="append", default=[],
                    help="the command(s) that produced the profile, quoted in the summary")
    ap.add_argument("--out", nargs="+", help="output file(s) of a summary")
    args = ap.parse_args()
    if args.summarize_stats:
        return summarize_stats(args.summarize_stats, args.bench_json, " ".join(args.profile_cmd),
                               args.out[0])
    if args.summarize_traffic:
        return summarize_traffic(*args.summarize_traffic, args.copy_mib, args.bench_json,
                                 args.profile_cmd, args.out[0], args.out[1])
    if args.summarize_sweep:
        return summarize_sweep(args.summarize_sweep, args.profile_cmd[0], args.out[0])
    if args.summarize_phases:
        return summarize_phases(args.summarize_phases, args.profile_cmd[0], args.out[0])
    if args.summarize_calibration:
        return summarize_calibration(*args.summarize_calibration, args.profile_cmd, args.out[0])
    if args.summarize_launches:
        calib = (args.copy_mib,) + tuple(args.calib_dirs) if args.calib_dirs else None
        return summarize_launches(args.summarize_launches[0], args.summarize_launches[1:], calib,
                                  args.profile_cmd, args.out[0])
    if args.calibrate_copy:
        import torch
        nb = args.calibrate_copy << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nb, "launches": 3}))
        return
    if args.calibrate_read:
        # a streaming read: the sum of MIB MiB of 64-bit words
        import torch
        nb = args.calibrate_read << 20
        src = torch.ones(nb // 8, dtype=torch.int64, device="cuda:0")
        for _ in range(3):
            src.sum()
        torch.cuda.synchronize()
        print(json.dumps({"calibration_read_bytes": nb, "launches": 3}))
        return
    if args.calibrate_gather:
        # random 8-byte gathers: 2^24 rows of 8 bytes from an array of MIB MiB
        # (far beyond the caches), indices read as a stream, rows written as one
        import torch
        nb = args.calibrate_gather << 20
        src = torch.ones(nb // 8, dtype=torch.int64, device="cuda:0")
        g = torch.Generator(device="cuda:0")
        g.manual_seed(7)
        idx = torch.randint(0, nb // 8, (1 << 24,), device="cuda:0", generator=g)
        for _ in range(3):
            torch.index_select(src, 0, idx)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_gather_rows": 1 << 24, "row_bytes": 8, "array_bytes": nb,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is a design note, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    gen, sigma, tau, leaf, s_hint, golden, desc = WORKLOADS[args.workload]
    cores = host_threads()
    try:
        if gen == "cfg5":
            return bench_serve(args, sigma, tau, leaf, desc)
        if gen == "cfg3sweep":
            out = bench_sweep(args, desc)
            print(json.dumps(out), flush=True)
            return
        if gen == "cfg4":
            out = bench_batch(args, sigma, tau, leaf, golden, desc)
            if not args.no_legs:
                legs = {}
                for w, steps in (("dna2g", 3), ("versioned256m", 5)):
                    leg, T = bench_single(args, w, steps, 1, sublegs=(w == "versioned256m"))
                    if w == "versioned256m" and not args.no_cpu_baseline:
                        leg["cpu_baseline"] = cpu_baseline_single(T, 4, 16, 1, cores, T.size)
                        log("cpu baseline (256 MiB): %s" % leg["cpu_baseline"])
                    del T
                    legs[w] = leg_view(leg)
                    log("leg %s: %.0f MB/s, probe scan %.3f of peak" % (
                        w, leg["value"], leg["roofline"]["frac"]))
                out["legs"] = legs
            if not args.no_cpu_baseline:
                out["cpu_baseline"] = cpu_baseline_batch(args.cpu_sample_mib, cores)
                log("cpu baseline: %s" % out["cpu_baseline"])
        else:
            out, T = bench_single(args, args.workload, args.steps, args.warmup,
                                  sublegs=(gen == "cfg2" and s_hint == 1 and not args.no_legs))
            out["cpu_baseline"] = None
            if not args.no_cpu_baseline:
                out["cpu_baseline"] = cpu_baseline_single(T, tau, leaf, s_hint, cores,
                                                          args.cpu_sample_mib << 20)
                log("cpu baseline: %s" % out["cpu_baseline"])
    except ParityError as e:
        log("bench.py: parity check failed, no result reported: %s" % e)
        sys.exit(3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
