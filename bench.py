"""Benchmark: block-tree construction throughput on one MI355X.

One step = one complete build (prefix fingerprints, every level's two phases,
marks, pointers, split, leaves) of the 256 MiB versioned text (sigma = 96,
tau = 4, leaf_len = 16, one root block), with the text already resident in
HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

The roofline object covers the probe-scan kernel (the sliding-window
fingerprint probe, the dominant kernel): its algorithmic bytes (the two prefix
values each window reads: 8 bytes of 32-bit pre-filter hashes, or 16 bytes of
61-bit prefix fingerprints where the scan does not pre-filter) over its
HIP-event time on the library's stream.  The cpu_baseline object times the CPU oracle on a bounded
prefix of the same text.  The pruned_build object times the same build with the
optional pruning phase (--prune times that as the main step instead); the
lean_build object times it with sampled prefix fingerprints (--lean) and gives
both builds' peak device memory; the sort_phase_build object times it with the
sort-based phases of Section 5.1 in place of the hash-table scan.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth

WORKLOADS = {
    # name: (generator, sigma, tau, leaf_len, s_hint, description)
    "versioned256m": ("cfg2", 96, 4, 16, 1,
                      "256 MiB versioned text, sigma 96: 1024 versions of a 256 KiB order-2 "
                      "Markov document, 0.05% edit runs per version"),
    "versioned256m_s": ("cfg2", 96, 4, 16, 1 << 19,
                        "same text, about 2^19 root blocks (b1 = 256)"),
    "dna1m": ("cfg1", 4, 2, 16, 1, "1 MiB DNA: 16 mutated copies of a 64 KiB base"),
    "dna1m_s": ("cfg1", 4, 2, 16, 10000, "1 MiB DNA, s about 10^4 (b1 = 64)"),
    "batch4096": ("cfg4", 4, 4, 16, 1,
                  "4096 DNA texts, lognormal lengths (median 256 KiB, 4 KiB-64 MiB, ~3.9 GiB): "
                  "one batched build vs a loop of single builds"),
    "serve": ("cfg5", 4, 4, 16, 1,
              "serving: Poisson build requests (lognormal sizes, median 256 KiB, 1 KiB-256 MiB, "
              "DNA texts) at 0.8x measured capacity, interleaved 1M-query batches"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_text(gen):
    import synth
    return {"cfg1": synth.cfg1_text, "cfg2": synth.cfg2_text}[gen]()


def traffic_record(kernel):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_traffic.json" % kernel)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if "sources" not in rec or _sources_sha(rec["sources"]) != rec.get("source_sha256"):
        return None
    return rec


# the files the probe scan is compiled from; a change to any of them retires
# the traffic record
PROBE_SOURCES = ["level.hip", "common.hpp", "window.hpp", "internal.hpp"]


def _sources_sha(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2512_23314_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


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
    probe = [r for r in rows if "k_probe_scan<" in r["Name"]]
    calls = sum(int(r["Calls"]) for r in probe)
    pns = sum(float(r["TotalDurationNs"]) for r in probe)
    rf = b["roofline"]
    lines = ["# Kernel time, %s build" % b["config"]["workload"], "",
             "Command (repository root, one MI355X):", "", "    " + cmd, "",
             "Bench line of the same run: %.2f %s, %.3f ms per step, probe_scan average "
             "launch %.4f ms (HIP events on the library stream), %d launches per step." % (
                 b["value"], b["unit"], b["ms_per_step"], rf["avg_launch_ms"], rf["launches_per_step"]),
             "",
             "rocprofv3: k_probe_scan (all instantiations) %d calls, average %.4f ms "
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


def _counter_per_launch(d, needle):
    rows = [r for r in _csv_rows(_find_csv(d, "counter_collection.csv")) if needle in r["Kernel_Name"]]
    if not rows:
        raise ValueError("no %s dispatches in %s" % (needle, d))
    return sum(float(r["Counter_Value"]) for r in rows) / len(rows), len(rows)


def summarize_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_mib, bench_json, cmds,
                      out_md, out_json, kernel="probe_scan", sources=None):
    sources = sources or PROBE_SOURCES
    copy_bytes = copy_mib << 20
    cf, _ = _counter_per_launch(cfetch_dir, "copyBuffer")
    cw, _ = _counter_per_launch(cwrite_dir, "copyBuffer")
    # a copy of B bytes reads B and writes B: scale each counter (KiB) to that
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    kf, n = _counter_per_launch(fetch_dir, "k_%s<" % kernel)
    kw, _ = _counter_per_launch(write_dir, "k_%s<" % kernel)
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


def bench_batch(args, sigma, tau, leaf, desc):
    """Batched build of 4096 texts vs a loop of single builds over the same
    device buffer."""
    import numpy as np
    import torch
    import paper_2512_23314_amd as bt
    import synth
    t0 = time.time()
    texts = synth.batch_texts()
    offs = np.zeros(len(texts) + 1, np.uint64)
    offs[1:] = np.cumsum([len(t) for t in texts])
    concat = np.concatenate(texts)
    del texts
    n = int(offs[-1])
    log("generated %d texts, %d bytes in %.1f s" % (len(offs) - 1, n, time.time() - t0))
    d = torch.from_numpy(concat).to("cuda:0")
    del concat
    ctx = bt.Context(0)

    def batched():
        trees = ctx.build_batch(d, offs, sigma=sigma, tau=tau, leaf_len=leaf)
        for tr in trees:
            tr.free()

    def plain():
        for k in range(len(offs) - 1):
            a, b = int(offs[k]), int(offs[k + 1])
            ctx.build(d[a:b], sigma=sigma, tau=tau, leaf_len=leaf).free()

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched()
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    ctx.profile(False)
    ps = ctx.kernel_stats("probe_scan")
    plain()  # warm the plain path's allocations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    log("batched %.1f ms (%.0f MB/s), plain loop %.1f ms (%.0f MB/s)" % (
        dt_b * 1e3, n / 1e6 / dt_b, dt_p * 1e3, n / 1e6 / dt_p))
    achieved = ps["bytes"] / ps["ms"] / 1e6 if ps["ms"] > 0 else 0.0
    out = {
        "metric": "block-tree build MB/s and KR-scan GB/s (% HBM peak) on 1 MI355X vs CPU oracle",
        "value": round(n / 1e6 / dt_b, 2), "unit": "MB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt_b * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batch4096", "description": desc, "n": n, "texts": len(offs) - 1,
                   "sigma": sigma, "tau": tau, "leaf_len": leaf},
        "batched_vs_plain": {"batched_mb_s": round(n / 1e6 / dt_b, 2),
                             "plain_loop_mb_s": round(n / 1e6 / dt_p, 2),
                             "speedup": round(dt_p / dt_b, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "probe_scan"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


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
        "metric": "block-tree build MB/s and KR-scan GB/s (% HBM peak) on 1 MI355X vs CPU oracle",
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


def cpu_baseline(T, sigma, tau, leaf, s_hint, sample_bytes):
    import oracle
    S = T[:sample_bytes]
    t0 = time.perf_counter()
    oracle.build_tree(S, tau, leaf, s_hint=s_hint)
    dt = time.perf_counter() - t0
    return {"value": round(S.size / dt / 1e6, 4), "unit": "MB/s", "cores": 1, "kind": "oracle",
            "sample": "first %d MiB of the same text, same tau/leaf/s, single-threaded oracle "
                      "(leftmost occurrences by memmem), %.1f s" % (S.size >> 20, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="versioned256m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prune", action="store_true",
                    help="time builds with the optional pruning phase (BT_PRUNE)")
    ap.add_argument("--no-pruned-leg", action="store_true",
                    help="skip the short pruned-build measurement beside the main line")
    ap.add_argument("--lean", action="store_true",
                    help="time memory-lean builds (BT_LEAN: sampled prefix fingerprints)")
    ap.add_argument("--no-lean-leg", action="store_true",
                    help="skip the short memory-lean measurement beside the main line")
    ap.add_argument("--no-sort-leg", action="store_true",
                    help="skip the build with the sort-based phases of Section 5.1")
    ap.add_argument("--cpu-sample-mib", type=int, default=8)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (the "
                         "known-size reference for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="write a markdown summary of a rocprofv3 --stats run (no GPU)")
    ap.add_argument("--summarize-traffic", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the probe_scan traffic record from four --pmc runs (no GPU)")
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
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is a design note, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2512_23314_amd as bt

    gen, sigma, tau, leaf, s_hint, desc = WORKLOADS[args.workload]
    if gen == "cfg4":
        return bench_batch(args, sigma, tau, leaf, desc)
    if gen == "cfg5":
        return bench_serve(args, sigma, tau, leaf, desc)
    t0 = time.time()
    T = make_text(gen)
    log("generated %s (%d bytes) in %.1f s" % (args.workload, T.size, time.time() - t0))
    n = int(T.size)
    d = torch.from_numpy(T).to("cuda:0")
    torch.cuda.synchronize()
    ctx = bt.Context(0)

    def step(prune=args.prune, lean=args.lean):
        tree = ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint, prune=prune, lean=lean)
        h = tree.height
        tree.free()
        return h

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(False)
    ms = dt / args.steps * 1e3
    value = n / 1e6 / (ms / 1e3)

    stats = {k: ctx.kernel_stats(k) for k in ("probe_scan", "byte_scan", "prefix_fp", "verify")}
    for k, s in stats.items():
        if s["launches"]:
            log("%-10s launches %5d  total %8.3f ms  avg %.4f ms  units %.3e  GB/s %.1f" % (
                k, s["launches"], s["ms"], s["ms"] / s["launches"], s["units"],
                s["bytes"] / max(s["ms"], 1e-9) / 1e6))
    ps = stats["probe_scan"]
    achieved = ps["bytes"] / ps["ms"] / 1e6 if ps["ms"] > 0 else 0.0
    tr = traffic_record("probe_scan")
    traffic = None
    if tr is not None and ps["launches"]:
        traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "probe_scan", "launches_per_step": ps["launches"] // max(args.steps, 1),
                "bytes_per_launch": round(ps["bytes"] / max(ps["launches"], 1)),
                "avg_launch_ms": round(ps["ms"] / max(ps["launches"], 1), 5)}
    pruned = None
    if not args.prune and not args.no_pruned_leg:
        pruned = pruned_leg(ctx, d, n, sigma, tau, leaf, s_hint, step)
        log("pruned build: %s" % pruned)
    leanr = None
    if not args.lean and not args.no_lean_leg:
        leanr = lean_leg(ctx, d, n, sigma, tau, leaf, s_hint, step)
        log("lean build: %s" % leanr)
    sortr = None
    if not args.no_sort_leg:
        sortr = sort_leg(ctx, d, n, sigma, tau, leaf, s_hint, ms)
        log("sort-phase build: %s" % sortr)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(T, sigma, tau, leaf, s_hint, args.cpu_sample_mib << 20)
        log("cpu baseline: %s" % cpu)
    out = {
        "metric": "block-tree build MB/s and KR-scan GB/s (% HBM peak) on 1 MI355X vs CPU oracle",
        "value": round(value, 2), "unit": "MB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "sigma": sigma,
                   "tau": tau, "leaf_len": leaf, "s_hint": s_hint, "levels": h,
                   "prune": bool(args.prune), "lean": bool(args.lean)},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    # per-kernel figures of the timed steps (HIP events on the library stream;
    # algorithmic bytes as in the roofline: 8 or 16 B per probe-scan window,
    # 1 B per byte-scan window, 13 B per text byte for the prefix scan: 1 read,
    # 8 + 4 written)
    out["kernels"] = {k: {"launches_per_step": s["launches"] // max(args.steps, 1),
                          "ms_per_step": round(s["ms"] / max(args.steps, 1), 4),
                          "algorithmic_GBps": round(s["bytes"] / max(s["ms"], 1e-9) / 1e6, 1)}
                      for k, s in stats.items() if s["launches"]}
    if pruned is not None:
        out["pruned_build"] = pruned
    if leanr is not None:
        out["lean_build"] = leanr
    if sortr is not None:
        out["sort_phase_build"] = sortr
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
