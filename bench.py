"""Benchmark: block-tree construction throughput on one MI355X.

One step = one complete build (prefix fingerprints, every level's two phases,
marks, pointers, split, leaves) of the 256 MiB versioned text (sigma = 96,
tau = 4, leaf_len = 16, one root block), with the text already resident in
HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

The roofline object covers the probe-scan kernel (the sliding-window
fingerprint probe, the dominant kernel): its algorithmic bytes (16 per window:
the two prefix fingerprints each window reads) over its HIP-event time on the
library's stream.  The cpu_baseline object times the CPU oracle on a bounded
prefix of the same text.
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
    src = os.path.join(ROOT, "paper_2512_23314_amd", "csrc", rec.get("source", "level.hip"))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if h != rec.get("source_sha256"):
        return None
    return rec


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
    ap.add_argument("--cpu-sample-mib", type=int, default=8)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (the "
                         "known-size reference for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
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
    t0 = time.time()
    T = make_text(gen)
    log("generated %s (%d bytes) in %.1f s" % (args.workload, T.size, time.time() - t0))
    n = int(T.size)
    d = torch.from_numpy(T).to("cuda:0")
    torch.cuda.synchronize()
    ctx = bt.Context(0)

    def step():
        tree = ctx.build(d, sigma=sigma, tau=tau, leaf_len=leaf, s_hint=s_hint)
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

    stats = {k: ctx.kernel_stats(k) for k in ("probe_scan", "prefix_fp", "verify")}
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
                "avg_launch_ms": round(ps["ms"] / max(ps["launches"], 1), 5)}
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
                   "tau": tau, "leaf_len": leaf, "s_hint": s_hint, "levels": h},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
