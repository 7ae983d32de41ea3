"""Throughput of the exact Tukey-depth hot path on one MI355X.

Workload (default): p = 5, n = 500 observations from a multivariate Student-t
with 3 degrees of freedom, m = 32 queries (16 sample points + 16 from
N(0, I_5)); every query sweeps all C(n', 3) subsets (about 2.07e7).  One step
= one td_depth call over the 32 queries with inputs already in HBM: the whole
path (preparation, subset kernel, exact tier, finalisation).

Prints ONE JSON line: subset sweeps/s of the float32-filtered path with the
bucketed sweep (`value`), queries/s, the rates of the filtered path with the
full bitonic sort and of the plain float64 path with the speedups, the
roofline object of the subset kernel (VALU-bound: algorithmic lane-ops per
launch over its HIP-event duration) and the CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit lane-ops/s, non-packed: 39.3 T
# Sources of the subset kernel: the HBM counters in the committed profile hold
# only while these still hash to the fingerprint recorded there.
KERNEL_SOURCES = ["td_subset.hpp", "td_device.hpp", "td_common.hpp", "td_subset_bucket.hip",
                  "td_subset_bucket64.hip", "td_subset_filt.hip", "td_subset_plain.hip"]
PROFILE = os.path.join(ROOT, "profiles", "subset_kernel_c3_p5_n500.md")


def kernel_fingerprint() -> str:
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1409_3901_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch of the filtered subset kernel (FETCH_SIZE and
    WRITE_SIZE, calibrated against a plain copy) from the committed profile,
    or None when the kernel sources changed since the counters were taken."""
    import re
    try:
        with open(PROFILE) as f:
            txt = f.read()
    except OSError:
        return None
    fp = re.search(r"kernel_sources_sha256: ([0-9a-f]{16})", txt)
    tb = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", txt)
    if not fp or not tb or fp.group(1) != kernel_fingerprint():
        return None
    return float(tb.group(1))


def algorithmic_ops(m: int, p: int) -> float:
    """Lane-ops of one sweep of m points: 2p FMA per point for the projection,
    m*ceil(log2 m) comparisons (the comparison-sort bound for the angular
    sort) and 2 per point for the scan and the minimum."""
    return 2.0 * p * m + m * math.ceil(math.log2(max(m, 2))) + 2.0 * m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain float64 comparison legs (c3 and --c4)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (calibrates HBM counters)")
    ap.add_argument("--precision", default="filtered", choices=["filtered", "bitonic", "plain"],
                    help="kernel timed as `value` (profiling runs): filtered = float32-filtered "
                         "with the bucketed sweep, bitonic = float32-filtered with the full sort, "
                         "plain = plain float64")
    ap.add_argument("--c4", action="store_true",
                    help="batched workload instead: 256 datasets in one graph launch vs "
                         "256*8 plain float64 launches")
    ap.add_argument("--all-configs", action="store_true",
                    help="every workload against its stored oracle counts: mismatches, "
                         "fallback rates and time of the filtered and plain tiers")
    ap.add_argument("--paper-grid", action="store_true",
                    help="the paper's simulation grid (X ~ N(0, I_p), z = alpha 1_p, one query), "
                         "Algorithm 1 (RCom) and Algorithm 3 (ADIA) timed per query beside the "
                         "paper's own timings as context")
    ap.add_argument("--widths", action="store_true",
                    help="point-steps/s of the bucketed kernel for every points-per-lane width at "
                         "p = 5 (one law, queries inside the hull, no pruning)")
    ap.add_argument("--p2", action="store_true",
                    help="p = 2, n = 1024, m = 1024 queries: one sweep per query (Algorithm 2 "
                         "alone), filtered and plain tiers, against stored oracle counts")
    ap.add_argument("--every-point", action="store_true",
                    help="the depth of every observation of a sample (the paper's real-data "
                         "shapes on seeded stand-ins), timed per observation beside the "
                         "paper's own timings as context")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the subset loop would shard by rank ranges of each query, followed by "
              "one MIN all-reduce of the per-query counts); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1409_3901_amd as td
    import workloads

    dev = torch.device("cuda:0")
    if a.copy_probe:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "dispatches": 3}), flush=True)
        return
    if a.c4:
        return bench_c4(a, td, workloads, torch, np, dev)
    if a.paper_grid:
        return bench_paper_grid(td, workloads, torch, np, dev)
    if a.every_point:
        return bench_every_point(td, workloads, torch, np, dev)
    if a.widths:
        return bench_widths(td, torch, np, dev)
    if a.p2:
        return bench_p2(a, td, workloads, torch, np, dev)
    if a.all_configs:
        return bench_all_configs(td, workloads, torch, np, dev)
    X, Z = workloads.c3()
    n, p = X.shape
    m = Z.shape[0]
    n0 = [int(np.sum(np.all(X == Z[q], axis=1))) for q in range(m)]
    sweeps = sum(math.comb(n - n0[q], p - 2) for q in range(m))
    ops = sum(math.comb(n - n0[q], p - 2) * algorithmic_ops(n - n0[q] - (p - 2), p) for q in range(m))
    Xd = torch.from_numpy(X).to(dev)
    Zd = torch.from_numpy(Z).to(dev)
    stream = torch.cuda.current_stream()

    OPTS = {"filtered": dict(precision="filtered"),
            "bitonic": dict(precision="filtered", sweep="bitonic"),
            "plain": dict(precision="plain")}

    def timed(prec):
        # launch shape (chunk, grid) chosen by the library's autotuner for
        # this shape and tier, then cached for the timed calls
        td.autotune(p, n, **OPTS[prec])
        for _ in range(a.warmup):
            td.depth(Xd, Zd, timing=True, **OPTS[prec])
        torch.cuda.synchronize()
        sub_ms = []
        st = None
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        total = 0.0
        out = None
        for _ in range(a.steps):
            torch.cuda.synchronize()
            t0.record(stream)
            out = td.depth(Xd, Zd, timing=True, **OPTS[prec])
            t1.record(stream)
            torch.cuda.synchronize()
            total += t0.elapsed_time(t1)
            st = td.get_stats()
            sub_ms.append(st["subset_ms"])
        return total / a.steps, sum(sub_ms) / len(sub_ms), st, out.cpu().numpy()

    ms, sub_ms, st, counts = timed(a.precision)
    names = {"filtered": "float32-filtered, exact, bucketed sweep",
             "bitonic": "float32-filtered, exact, full bitonic sort", "plain": "plain float64"}
    res = {
        "metric": "subset sweeps/s (%s) at p=5, n=500" % names[a.precision],
        "value": sweeps / (ms / 1e3),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "plain" else "f32",
        "data": "synthetic",
        "config": {"workload": "c3: p=5, n=500 multivariate t(3), m=32 queries "
                               "(16 sample points + 16 N(0,I_5)), all C(n',3) subsets",
                   "p": p, "n": n, "m": m,
                   "precision": "fp64-plain" if a.precision == "plain" else "fp32-filtered+fp64+exact",
                   "sweep": "bitonic" if a.precision != "filtered" else "bucketed"},
        "value_definition": "enumerated subsets (sum over queries of C(n'_q, p-2)) resolved per second; "
                            "subsets the pruning bound settles without a sweep are included, see "
                            "processed_sweeps_per_s",
        "queries_per_s": m / (ms / 1e3),
        "sweeps_per_step": sweeps,
        "fp64_rechecks_per_sweep": st["fp64_rechecks"] / max(1, st["subsets_swept"]),
        "walked_per_sweep": st["walked_sweeps"] / max(1, st["subsets_swept"]),
        "deferred_subsets": st["deferred_subsets"],
        "f64_items": st["f64_items"],
        "exact_predicates": st["exact_predicates"],
        "device_status": st["device_status"],
    }
    gold = os.path.join(ROOT, "tests", "golden", "c3.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)["counts"]
        qs = [int(k) for k in g]
        res["mismatches_vs_oracle"] = int(sum(int(counts[q]) != g[str(q)] for q in qs))
        res["queries_checked"] = len(qs)
    # roofline of the subset kernel: algorithmic ops over its event duration
    # subsets skipped by the pruning bound are not processed: their work is
    # taken out at the largest per-sweep count of any query (a lower bound on
    # the work done)
    res["pruned_subsets"] = st["pruned_subsets"]
    res["processed_sweeps_per_s"] = (sweeps - st["pruned_subsets"]) / (ms / 1e3)
    max_ops = max(algorithmic_ops(n - n0[q] - (p - 2), p) for q in range(m))
    ops_done = ops - st["pruned_subsets"] * max_ops
    achieved = ops_done / (sub_ms / 1e3) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS,
                       "unit": "TOP/s", "frac": achieved / PEAK_VALU_TOPS,
                       "traffic": profiled_traffic() if a.precision == "filtered" else None,
                       "kernel": "subset_kernel<5,8,%d,false>" % {"plain": 0, "bitonic": 1, "filtered": 3}[a.precision],
                       # HIP events around the subset stage: for the bucketed
                       # sweep this includes its float64 pass (the second
                       # launch, subset_kernel<5,8,3,true>, under 1 ms here)
                       "kernel_ms": sub_ms,
                       "ops_per_launch": ops_done,
                       "subsets_processed": sweeps - st["pruned_subsets"]}
    if not a.no_plain and a.precision == "filtered":
        bms, bsub, bst, bcounts = timed("bitonic")
        res["filtered_bitonic"] = {"sweeps_per_s": sweeps / (bms / 1e3), "ms_per_step": bms,
                                   "subset_kernel_ms": bsub,
                                   "mismatches_vs_bucketed": int(np.sum(bcounts != counts))}
        res["speedup_bucketed_vs_bitonic"] = bms / ms
        pms, psub, pst, pcounts = timed("plain")
        res["plain_fp64"] = {"sweeps_per_s": sweeps / (pms / 1e3), "ms_per_step": pms,
                             "subset_kernel_ms": psub,
                             "mismatches_vs_filtered": int(np.sum(pcounts != counts))}
        res["speedup_filtered_vs_plain"] = pms / ms
        # the same full bitonic sort in both: the factor due to the arithmetic
        # alone (float32 filter with certification against plain float64)
        res["speedup_precision_only"] = pms / bms
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(X, Z, a.cpu_seconds)
    print(json.dumps(res), flush=True)


def bench_p2(a, td, workloads, torch, np, dev):
    """p = 2 (one sweep per query, I empty): n = 1024 points, m = 1024
    queries, one td_depth call per step (HIP events around the call, mean over
    the timed steps), filtered and plain tiers, mismatches against the stored
    oracle counts, and the roofline of the subset kernel (algorithmic
    lane-ops of the sweeps over its duration)."""
    X, Z = workloads.p2()
    n, p = X.shape
    m = Z.shape[0]
    n0 = [int(np.sum(np.all(X == Z[q], axis=1))) for q in range(m)]
    ops = sum(algorithmic_ops(n - n0[q], p) for q in range(m))
    g = _stored_counts("p2")
    exp = np.array([g[str(q)] for q in range(m)])
    Xd = torch.from_numpy(X).to(dev)
    Zd = torch.from_numpy(Z).to(dev)
    stream = torch.cuda.current_stream()
    out = {}
    for prec, opts in (("filtered", {}), ("plain", {"precision": "plain"})):
        for _ in range(a.warmup):
            td.depth(Xd, Zd, timing=True, **opts)
        torch.cuda.synchronize()
        tot, sub = 0.0, 0.0
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        for _ in range(a.steps):
            t0.record(stream)
            c = td.depth(Xd, Zd, timing=True, **opts)
            t1.record(stream)
            torch.cuda.synchronize()
            tot += t0.elapsed_time(t1)
            st = td.get_stats()
            sub += st["subset_ms"]
        ms, sub_ms = tot / a.steps, sub / a.steps
        got = c.cpu().numpy()
        achieved = ops / (sub_ms / 1e3) / 1e12
        out[prec] = {"ms_per_step": ms, "queries_per_s": m / (ms / 1e3), "sweeps_per_s": m / (ms / 1e3),
                     "mismatches_vs_oracle": int(np.sum(got != exp)), "queries_checked": m,
                     "deferred_subsets": st["deferred_subsets"], "device_status": st["device_status"],
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                                  "frac": achieved / PEAK_VALU_TOPS, "traffic": None,
                                  "kernel": "subset_kernel<2,16,%d,false>" % (1 if prec == "filtered" else 0),
                                  "kernel_ms": sub_ms, "ops_per_launch": ops}}
    f = out["filtered"]
    print(json.dumps({"metric": "queries/s at p=2, n=1024 (one sweep per query)", "value": f["queries_per_s"],
                      "unit": "queries/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                      "ms_per_step": f["ms_per_step"], "higher_is_better": True, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": "p2: N(0,I_2), n=1024, m=1024 queries (512 sample points, "
                                             "512 N(0,I_2))"},
                      "filtered": f, "plain_fp64": out["plain"],
                      "speedup_filtered_vs_plain": out["plain"]["ms_per_step"] / f["ms_per_step"]}), flush=True)


def bench_c4(a, td, workloads, torch, np, dev):
    """256 datasets of uneven n and p (8 queries each): one td_depth_batched
    call (one captured graph launch; median of 3 timed launches) against one
    plain float64 td_depth call per query (one pass)."""
    def note(msg):
        print("[c4] %s" % msg, file=sys.stderr, flush=True)

    data = workloads.c4()
    note("generated %d datasets" % len(data))
    probs = [(torch.from_numpy(X).to(dev), torch.from_numpy(Z).to(dev)) for X, Z in data]
    sweeps = 0
    for X, Z in data:
        n, p = X.shape
        for q in range(Z.shape[0]):
            n0 = int(np.sum(np.all(X == Z[q], axis=1)))
            sweeps += math.comb(n - n0, p - 2)
    note("%d sweeps" % sweeps)
    # launch shapes tuned per kernel class, at the class's largest n: points
    # per lane k = sort width / 64, except that the bucketed sweep runs 10, 12
    # or 14 for 512 < n <= 896 at p <= 6
    classes = {}
    for X, Z in data:
        n, p = X.shape
        k = max(64, 1 << (n - 1).bit_length()) // 64
        if k == 16 and p <= 6 and n <= 896:
            k = (n + 127) // 128 * 2
        classes[(p, k)] = max(classes.get((p, k), 0), n)
    for (p, k), n in sorted(classes.items()):
        td.autotune(p, n)
    note("autotuned %d classes" % len(classes))
    td.depth_batched(probs)       # captures the graph
    torch.cuda.synchronize()
    note("warm-up launch done")
    runs = []
    outs = None
    for _ in range(3):
        t = time.time()
        outs = td.depth_batched(probs)
        torch.cuda.synchronize()
        runs.append(time.time() - t)
        note("timed graph launch: %.2f s" % runs[-1])
    tb = sorted(runs)[1]   # median of 3
    st = td.get_stats()
    res = {"metric": "c4 batched: sweeps/s of one graph launch (float32-filtered, exact)",
           "value": sweeps / tb, "unit": "sweeps/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "c4: 256 datasets, p in {3,4,5}, n in [50,800], 8 queries each"},
           "sweeps": sweeps, "batched_s": tb, "batched_runs_s": runs,
           "deferred_subsets": st["deferred_subsets"], "device_status": st["device_status"]}
    if not a.no_plain:
        t = time.time()
        plain = []
        for i, (Xd, Zd) in enumerate(probs):
            for q in range(Zd.shape[0]):
                plain.append(td.depth(Xd, Zd[q:q + 1].contiguous(), precision="plain"))
            if i % 32 == 31:
                torch.cuda.synchronize()
                note("plain launches: %d datasets, %.1f s" % (i + 1, time.time() - t))
        torch.cuda.synchronize()
        tp = time.time() - t
        got = np.concatenate([o.cpu().numpy() for o in outs])
        pl = np.concatenate([o.cpu().numpy() for o in plain])
        res.update({"plain_launches": len(pl), "plain_s": tp, "plain_sweeps_per_s": sweeps / tp,
                    "speedup_batched_vs_plain_launches": tp / tb,
                    "mismatches_batched_vs_plain": int(np.sum(got != pl))})
    print(json.dumps(res), flush=True)


def _stored_counts(cfg):
    """Stored oracle counts of a workload (tests/golden, merged over parts)."""
    import glob
    gold = os.path.join(ROOT, "tests", "golden")
    counts = {}
    for path in sorted(glob.glob(os.path.join(gold, cfg + ".json")) +
                       glob.glob(os.path.join(gold, cfg + ".*.json"))):
        with open(path) as f:
            counts.update(json.load(f)["counts"])
    return counts


def bench_all_configs(td, workloads, torch, np, dev):
    """Each workload through the filtered tier (bucketed sweep) and the plain
    float64 tier, against the stored oracle counts (and the vertex check on
    c1 and four c3 queries): mismatches (0 required of the filtered tier; the
    plain tier's are reported), float64 re-checks and
    deferred subsets per sweep, the HIP-event time of the call, and the
    subset kernel's roofline fraction (algorithmic lane-ops of the processed
    subsets over its duration, against the non-packed 32-bit lane-op peak)."""
    out = {}

    def one(name, X, Z, idx, exp, **opts):
        Xd = torch.from_numpy(X).to(dev)
        Zd = torch.from_numpy(np.ascontiguousarray(Z[idx])).to(dev)
        td.depth(Xd, Zd, **opts)
        c = td.depth(Xd, Zd, timing=True, **opts)
        torch.cuda.synchronize()
        st = td.get_stats()
        got = c.cpu().numpy()
        n, p = X.shape
        covered, ops, max_ops = 0, 0.0, 0.0
        for q in idx:
            nq = n - int(np.sum(np.all(X == Z[q], axis=1)))
            per = algorithmic_ops(nq - (p - 2), p)
            covered += math.comb(nq, p - 2)
            ops += math.comb(nq, p - 2) * per
            max_ops = max(max_ops, per)
        ops_done = ops - st["pruned_subsets"] * max_ops
        sweeps = max(st["subsets_swept"] + st["deferred_subsets"] + st["pruned_subsets"], 1)
        return {"queries": len(idx), "mismatches": int(np.sum(got != exp)), "ms": st["total_ms"],
                "sweeps_per_s": covered / (st["total_ms"] / 1e3),
                "roofline_frac": ops_done / (st["subset_ms"] / 1e3) / 1e12 / PEAK_VALU_TOPS,
                "fp64_rechecks_per_sweep": st["fp64_rechecks"] / sweeps,
                "deferred_subsets": st["deferred_subsets"], "exact_predicates": st["exact_predicates"],
                "pruned_subsets": st["pruned_subsets"], "device_status": st["device_status"]}

    for cfg in ("c1", "c2", "c3", "c5"):
        X, Z = workloads.config(cfg)
        g = _stored_counts(cfg)
        idx = sorted(int(k) for k in g)
        exp = np.array([g[str(q)] for q in idx])
        out[cfg] = {"filtered": one(cfg, X, Z, idx, exp),
                    "plain": one(cfg, X, Z, idx, exp, precision="plain")}
        print("[configs] %s done" % cfg, file=sys.stderr, flush=True)
    # c4: the stored subsample (queries of the datasets the oracle affords)
    data = workloads.c4()
    g = _stored_counts("c4")
    probs, exp = [], []
    for d, (X, Z) in enumerate(data):
        qs = [q for q in range(Z.shape[0]) if "%d:%d" % (d, q) in g]
        if qs:
            probs.append((torch.from_numpy(X).to(dev), torch.from_numpy(np.ascontiguousarray(Z[qs])).to(dev)))
            exp.extend(g["%d:%d" % (d, q)] for q in qs)
    outs = td.depth_batched(probs)
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy() for o in outs])
    out["c4_subsample"] = {"filtered_batched": {"queries": len(exp),
                                                "mismatches": int(np.sum(got != np.array(exp)))}}
    # the vertex-form check (Proposition 1, r = p - 1) beside the stored
    # counts, where its O(n^p) work is small: c1, and four c3 queries
    for cfg, qs in (("c1", None), ("c3", [0, 7, 16, 25])):
        X, Z = workloads.config(cfg)
        g = _stored_counts(cfg)
        idx = qs if qs is not None else sorted(int(k) for k in g)
        Xd = torch.from_numpy(X).to(dev)
        Zd = torch.from_numpy(np.ascontiguousarray(Z[idx])).to(dev)
        t = time.perf_counter()
        c = td.depth(Xd, Zd, method="vertex")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = td.get_stats()
        got = c.cpu().numpy()
        out[cfg]["vertex"] = {"queries": len(idx), "mismatches": int(np.sum(got != np.array([g[str(q)] for q in idx]))),
                              "declined": int(np.sum(got == -1)), "s": dt,
                              "hyperplanes_per_s": st["subsets_swept"] / dt}
        print("[configs] %s vertex done" % cfg, file=sys.stderr, flush=True)
    print(json.dumps({"metric": "mismatches against the oracle and fallback rates, every workload",
                      "n_gpus": 1, "data": "synthetic", "configs": out}), flush=True)


# The paper's timings of its first algorithm (Table 2: seconds per query,
# X ~ N(0, I_p), z = 0, Matlab 7.8 on an Intel Core i7-2670QM at 2.2 GHz),
# quoted as context only: other hardware, software and data.
PAPER_TABLE2_S = {
    (3, 40): 0.0268, (3, 80): 0.0481, (3, 160): 0.0899, (3, 320): 0.2531, (3, 640): 0.8073,
    (4, 40): 0.1876, (4, 80): 0.8045, (4, 160): 5.0550, (4, 320): 43.3812, (4, 640): 248.5797,
    (5, 40): 1.9517, (5, 80): 21.1227, (5, 160): 262.3251, (5, 320): 3864.4624,
    (6, 40): 18.4515, (6, 80): 446.0153, (6, 160): 14695.1294,
}


# The paper's timings of its adaptive algorithm (Table 3: ADIA, seconds per
# query, the same design at z = alpha 1_p), quoted as context only.
PAPER_TABLE3_S = {
    (3, 0.0): [0.0193, 0.0634, 0.0503, 0.1297, 0.4372], (3, 0.4): [0.0167, 0.0470, 0.0668, 0.0968, 0.3418],
    (3, 0.8): [0.0065, 0.0131, 0.0180, 0.0460, 0.3248], (3, 1.2): [0.0067, 0.0136, 0.0186, 0.0390, 0.1220],
    (4, 0.0): [0.3416, 0.3211, 1.7991, 6.5374, 60.6911], (4, 0.4): [0.0607, 0.1704, 0.5131, 1.7255, 11.9404],
    (4, 0.8): [0.1070, 0.1172, 0.1140, 0.5171, 1.7526], (4, 1.2): [0.1373, 0.1465, 0.0538, 0.2278, 0.9409],
    (5, 0.0): [0.9466, 6.9212, 68.0360, 404.5147, 13177.5227], (5, 0.4): [0.4048, 1.0052, 8.3791, 43.6717, 609.6461],
    (5, 0.8): [1.2751, 1.1352, 1.6600, 5.3665, 15.8776], (5, 1.2): [0.1923, 0.1001, 0.3339, 0.3162, 1.5744],
    (6, 0.0): [12.3953, 95.3378, 3883.9385, None, None], (6, 0.4): [4.3607, 18.3686, 173.8880, 1504.1087, None],
    (6, 0.8): [0.1638, 0.2295, 62.8009, 158.7744, 1777.3669], (6, 1.2): [1.1149, 3.0121, 1.4400, 4.9680, 19.3288],
}
GRID_N = [40, 80, 160, 320, 640]


def bench_widths(td, torch, np, dev):
    """The first-pass bucketed kernel at every points-per-lane width of p = 5
    (n = 500, 512: 8; 600, 640: 10; 700, 768: 12; 800, 896: 14; 960, 1024:
    16) on one law, X ~ N(0, I_5), with 8 queries drawn inside the hull
    (0.2 N(0, I_5)) and pruning off, so that every class sweeps every subset
    of the same kind of query: subset-stage time (the library's events, best
    of 3) and point-steps/s over the real points.  The per-class rates of the
    batched workload mix in how fast each class's queries settle under the
    pruning bound and how much padding the class carries."""
    rng = np.random.default_rng(11)
    rows = []
    for n in (500, 512, 600, 640, 700, 768, 800, 896, 960, 1024):
        X = rng.standard_normal((n, 5))
        Z = 0.2 * rng.standard_normal((8, 5))
        Xd = torch.tensor(X, device=dev)
        Zd = torch.tensor(Z, device=dev)
        td.autotune(5, n)
        td.depth(Xd, Zd, prune=False)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            td.depth(Xd, Zd, prune=False, timing=True)
            torch.cuda.synchronize()
            st = td.get_stats()
            best = st["subset_ms"] if best is None else min(best, st["subset_ms"])
        k = max(64, 1 << (n - 1).bit_length()) // 64
        if k == 16 and n <= 896:
            k = (n + 127) // 128 * 2
        sub = 8 * math.comb(n, 3)
        rows.append({"n": n, "points_per_lane": k, "subset_ms": best, "sweeps_per_s": sub / (best / 1e3),
                     "point_steps_per_s": sub * (n - 3) / (best / 1e3),
                     "slot_steps_per_s": sub * 64 * k / (best / 1e3),
                     "walked_per_sweep": st["walked_sweeps"] / sub, "deferred_subsets": st["deferred_subsets"],
                     "f64_items": st["f64_items"], "device_status": st["device_status"]})
        print("[widths] n=%d K=%d %.1f ms %.3g point-steps/s" % (n, k, best, rows[-1]["point_steps_per_s"]),
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "point-steps/s by points per lane (p = 5, one law, no pruning)",
                      "unit": "point-steps/s", "n_gpus": 1, "data": "synthetic", "rows": rows}), flush=True)


def bench_paper_grid(td, workloads, torch, np, dev):
    """The paper's simulation design (X ~ N(0, I_p), seeded; one query
    z = alpha 1_p) for p = 3..6, n = 40..640 and alpha in {0, 0.4, 0.8, 1.2}:
    the time of one td_depth call by Algorithm 1 (RCom) and by Algorithm 3
    (ADIA), best of 3, and of one call of the vertex-form check where it is
    small enough (host clock around the call and a synchronisation; the
    ADIA call synchronises between its steps), the two counts (which must
    agree: the rows report it), ADIA's evaluated subsets and candidate points,
    and the paper's seconds for RCom (Table 2, alpha = 0) and ADIA (Table 3)
    as context.  p = 6 stops at n = 320 (n = 640 sweeps 6.9e9 subsets per
    method and alpha)."""
    rows = []
    for p in (3, 4, 5, 6):
        for ni, n in enumerate(GRID_N):
            if p == 6 and n > 320:
                continue
            for alpha in (0.0, 0.4, 0.8, 1.2):
                X, Z = workloads.grid(p, n, alpha)
                Xd = torch.from_numpy(X).to(dev)
                Zd = torch.from_numpy(Z).to(dev)
                row = {"p": p, "n": n, "alpha": alpha, "subsets": math.comb(n, p - 2)}
                for meth in ("rcom", "adia"):
                    td.depth(Xd, Zd, method=meth)
                    torch.cuda.synchronize()
                    best = None
                    for _ in range(3):
                        t = time.perf_counter()
                        c = td.depth(Xd, Zd, method=meth)
                        torch.cuda.synchronize()
                        dt = (time.perf_counter() - t) * 1e3
                        best = dt if best is None else min(best, dt)
                    st = td.get_stats()
                    row[meth + "_ms"] = best
                    row[meth + "_count"] = int(c.cpu()[0])
                    if meth == "adia":
                        row["adia_evaluations"] = st["adia_evaluations"]
                        row["adia_candidates"] = st["adia_candidates"]
                        row["adia_answered_by_rcom"] = st["adia_rcom_queries"]
                row["counts_agree"] = row["rcom_count"] == row["adia_count"]
                # the vertex-form check (Proposition 1 with r = p - 1, the
                # critical-direction route), O(n^p): one timed call where the
                # work is at most 2e11 point-sides
                row["vertex_ms"] = row["vertex_count"] = None
                if (n <= 512 or p <= 4) and math.comb(n, p - 1) * n <= 2e11:
                    t = time.perf_counter()
                    c = td.depth(Xd, Zd, method="vertex")
                    torch.cuda.synchronize()
                    row["vertex_ms"] = (time.perf_counter() - t) * 1e3
                    row["vertex_count"] = int(c.cpu()[0])
                row["paper_rcom_s"] = PAPER_TABLE2_S.get((p, n)) if alpha == 0.0 else None
                row["paper_adia_s"] = PAPER_TABLE3_S[(p, alpha)][ni]
                rows.append(row)
                print("[grid] p=%d n=%d alpha=%.1f rcom %.3f ms adia %.3f ms vertex %s ms (%d / %d / %s)"
                      % (p, n, alpha, row["rcom_ms"], row["adia_ms"], row["vertex_ms"], row["rcom_count"],
                         row["adia_count"], row["vertex_count"]), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "ms per query on the paper's simulation grid, RCom and ADIA (context)",
                      "unit": "ms", "n_gpus": 1, "data": "synthetic",
                      "paper_hardware": "Intel Core i7-2670QM 2.2 GHz, Matlab 7.8 (Tables 2 and 3)",
                      "all_counts_agree": all(r["counts_agree"] for r in rows),
                      "vertex_agrees_with_rcom": all(r["vertex_count"] in (None, r["rcom_count"]) for r in rows),
                      "rows": rows}), flush=True)


# The paper's per-observation timings on its two real data sets (seconds per
# observation; RCom and the mean of ADIA; Matlab 7.8 on an Intel Core
# i7-2670QM at 2.2 GHz), quoted as context only: the data here are seeded
# stand-ins of the same shapes.
# The paper's real-data table, seconds per observation: RCom, then ADIA's
# minimum, mean and maximum over the observations.
PAPER_OBS_S = {
    ("scores", 3, 64): (0.0145, 0.0066, 0.0117, 0.0380),
    ("returns", 3, 200): (0.0908, 0.0146, 0.0387, 0.1287),
    ("returns", 3, 500): (0.4925, 0.0283, 0.1472, 0.5609),
    ("scores", 4, 64): (0.4614, 0.0335, 0.1410, 0.3731),
    ("returns", 4, 200): (8.8961, 0.0620, 0.4624, 3.3255),
    ("returns", 4, 500): (120.0689, 0.1411, 2.4635, 21.9474),
}


def bench_every_point(td, workloads, torch, np, dev):
    """The depth of every observation (Z = X, m = n queries), for the (p, n)
    of the paper's real-data table.  RCom: one call over all observations (the
    library's own HIP events, best of 5), per observation.  ADIA: one call per
    observation (host clock, as the paper times one observation at a time;
    best of 2), reported as minimum, mean and maximum like the paper's table,
    and checked against the RCom counts; and one ADIA call over all
    observations, checked against the per-observation values."""
    rows = []
    for (kind, p, n), (rcom_s, adia_min_s, adia_mean_s, adia_max_s) in PAPER_OBS_S.items():
        X, Z = workloads.observations(kind, p, n)
        Xd = torch.from_numpy(X).to(dev)
        Zd = torch.from_numpy(Z).to(dev)
        td.depth(Xd, Zd)
        best = None
        for _ in range(5):
            c = td.depth(Xd, Zd, timing=True)
            torch.cuda.synchronize()
            ms = td.get_stats()["total_ms"]
            best = ms if best is None else min(best, ms)
        st = td.get_stats()
        counts = c.cpu().numpy()
        n0 = [int(np.sum(np.all(X == Z[q], axis=1))) for q in range(n)]
        covered = sum(math.comb(n - n0[q], p - 2) for q in range(n))
        # ADIA over all observations in one call (the descents of the queries
        # share their device launches)
        adia_all = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            aa = td.depth(Xd, Zd, method="adia")
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            adia_all = dt if adia_all is None else min(adia_all, dt)
        adia_ms = []
        adia_vals = []
        adia_agree = 0
        for q in range(n):
            zq = Zd[q:q + 1]
            t = None
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                a = td.depth(Xd, zq, method="adia")
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) * 1e3
                t = dt if t is None else min(t, dt)
            adia_ms.append(t)
            adia_vals.append(int(a.cpu().numpy()[0]))
            adia_agree += int(adia_vals[-1] == counts[q])
        rows.append({"data": kind, "p": p, "n": n, "gpu_ms_all_observations": best,
                     "gpu_ms_per_observation": best / n, "sweeps_per_s": covered / (best / 1e3),
                     "pruned_subsets": st["pruned_subsets"], "device_status": st["device_status"],
                     "depth_min": int(counts.min()), "depth_max": int(counts.max()),
                     # the deepest observations (the sample's Tukey median among
                     # its own points) and the depth levels of the paper's
                     # figure of sorted depths: observations per depth count
                     "deepest_observations": [int(i) for i in np.nonzero(counts == counts.max())[0]],
                     "observations_per_depth": {int(k): int(v) for k, v in zip(*np.unique(counts, return_counts=True))},
                     "adia_ms_min": min(adia_ms), "adia_ms_mean": sum(adia_ms) / n, "adia_ms_max": max(adia_ms),
                     "adia_equal_to_rcom": "%d of %d" % (adia_agree, n),
                     "adia_ms_all_observations_one_call": adia_all,
                     "adia_one_call_equals_per_observation": bool(np.array_equal(aa.cpu().numpy(), np.array(adia_vals))),
                     "paper_rcom_s_per_observation": rcom_s, "paper_adia_min_s": adia_min_s,
                     "paper_adia_mean_s": adia_mean_s, "paper_adia_max_s": adia_max_s,
                     "paper_rcom_over_gpu": rcom_s * 1e3 / (best / n)})
        print("[every-point] %s p=%d n=%d %.3f ms; adia %.2f/%.2f/%.2f ms, %d of %d equal; adia one call %.2f ms"
              % (kind, p, n, best, min(adia_ms), sum(adia_ms) / n, max(adia_ms), adia_agree, n, adia_all),
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "depth of every observation: ms per observation (context)",
                      "unit": "ms", "n_gpus": 1, "data": "synthetic stand-ins of the paper's real data",
                      "paper_hardware": "Intel Core i7-2670QM 2.2 GHz, Matlab 7.8",
                      "rows": rows}), flush=True)


def cpu_baseline(X, Z, seconds):
    """The oracle, as it stands, on a bounded sample of the same workload: one
    query (a Gaussian one, index 16), subsets of lexicographic rank [0, R)
    with R sized to about `seconds` of work on the host's cores."""
    import oracle
    threads = oracle.default_threads()
    z = Z[16]
    r = 20000
    t = time.time()
    oracle.depth_range(X, z, 0, r, threads=threads)
    dt = max(time.time() - t, 1e-3)
    R = int(min(math.comb(X.shape[0], X.shape[1] - 2), max(r, r * seconds / dt)))
    t = time.time()
    _, swept = oracle.depth_range(X, z, 0, R, threads=threads)
    dt = time.time() - t
    res = {"value": swept / dt, "unit": "sweeps/s", "cores": threads, "kind": "oracle",
           "sample": "c3 query 16, subsets of lexicographic rank [0, %d) of %d (%.1f s)"
                     % (R, math.comb(X.shape[0], X.shape[1] - 2), dt),
           "queries_per_s": (swept / dt) / math.comb(X.shape[0], X.shape[1] - 2)}
    res["per_core"] = [per_core_rate("c3 query 16", X, z, 3.0)]
    import workloads
    _, _, info = workloads.c5(return_premap=True)
    X5 = info["X0"].astype("float64")
    res["per_core"].append(per_core_rate("c5 query 0 (pre-map lattice, same counts)", X5,
                                         info["Z0"][0].astype("float64"), 3.0))
    return res


def per_core_rate(name, X, z, seconds):
    """The oracle on one thread over a bounded rank range of one query."""
    import oracle
    r = 2000
    t = time.time()
    oracle.depth_range(X, z, 0, r, threads=1)
    dt = max(time.time() - t, 1e-3)
    total = math.comb(X.shape[0], X.shape[1] - 2)
    R = int(min(total, max(r, r * seconds / dt)))
    t = time.time()
    _, swept = oracle.depth_range(X, z, 0, R, threads=1)
    dt = time.time() - t
    return {"value": swept / dt, "unit": "sweeps/s", "cores": 1,
            "sample": "%s, subsets of lexicographic rank [0, %d) of %d (%.1f s)" % (name, R, total, dt)}


if __name__ == "__main__":
    main()
