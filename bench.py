#!/usr/bin/env python3
"""Benchmark of the best-hit path on one MI355X.

Workload (default): 10 synthetic protein genomes x 3000 genes from the family
model (60% core, 30% accessory, 10% singletons, 5-30% divergence), k = 6 from
the k rule; a step rebuilds all ten k-mer dictionaries from residues already
in HBM and computes best hits in both directions plus BBH for all 45 genome
pairs in one plan launch.  value = gene pairs compared (sum of |A||B| over the
45 pairs) per second.

Printed: one JSON line with the metric, a roofline entry for the dominant
kernel (HIP events recorded by the library around that kernel on its own
stream) and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gene-pair similarities/sec incl. BH+BBH at 1 GPU; p50/p99 per-genome latency"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--kernel", default="join", help="kernel for the roofline entry (join, bucket, tile_count, "
                                                    "tile_write, bbh)")
    p.add_argument("--cpu-rows", type=int, default=128, help="rows per direction per pair in the CPU-oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--breakdown", action="store_true", help="also time every kernel group (extra launches)")
    p.add_argument("--calibrate-copy", action="store_true", help="only run a copy of known size (counter calibration)")
    p.add_argument("--tune", action="store_true", help="pick tile shapes and join splits with the autotuner first")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                   help="measured HBM traffic per kernel (from rocprofv3 counters), used when its source hash matches")
    return p.parse_args()


def source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_23679_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, pairs, entries, res_bh_nnz, res_bbh, genes) -> float:
    """Bytes the method itself needs per launch, for the kernel's share of the path.

    join: each unordered genome pair reads both genomes' k-mer entries once, a u64 code
    and a u32 multiplicity each (12 bytes per entry).  tile_write: the best-hit output,
    16 bytes per entry (column, two integers, row bookkeeping) plus 8 bytes per row.
    bbh: 16 bytes per BBH pair.  Other kernels move only intermediate data."""
    if kernel == "join":
        return float(sum(12 * (entries[i] + entries[j]) for i, j in pairs))
    if kernel == "tile_write":
        return float(16 * res_bh_nnz + 8 * sum(genes[i] + genes[j] for i, j in pairs))
    if kernel == "bbh":
        return float(16 * res_bbh)
    return 0.0


def cpu_baseline(ds, k, rows_per_dir):
    """The oracle as it stands, on a bounded sample: multiplicity vectors of every genome, then
    best hits of rows_per_dir evenly spaced rows in each direction of every pair."""
    import numpy as np

    import oracle

    threads = oracle.default_threads()
    t0 = time.perf_counter()
    og = [oracle.OracleGenome(g, k) for g in ds.genomes]
    gene_pairs = 0
    for i, j in ds.pairs():
        for q, t in ((og[i], og[j]), (og[j], og[i])):
            rows = np.linspace(0, q.n - 1, min(rows_per_dir, q.n)).astype(np.uint32)
            oracle.bh(q, t, rows=rows, threads=threads)
            gene_pairs += len(rows) * t.n
    dt = time.perf_counter() - t0
    return {"value": gene_pairs / dt, "unit": "gene-pair similarities/s", "cores": threads, "kind": "oracle",
            "sample": f"multiplicity vectors of all {len(og)} genomes plus best hits of {rows_per_dir} evenly "
                      f"spaced rows per direction of each of the {len(ds.pairs())} pairs "
                      f"({gene_pairs} gene pairs, {dt:.1f} s); BBH on the sampled rows is not included",
            "seconds": dt}


def calibrate_copy(mib: int = 1024) -> None:
    """A plain elementwise copy of known size (reads and writes mib MiB once each), for scaling
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "elementwise int32 copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path shards genome pairs "
                                   "across GPUs by design but no multi-GPU run is part of this build",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_23679_amd as pdp
    from paper_2510_23679_amd import binding as B
    from synth import make_config

    torch.cuda.set_device(0)
    ds = make_config(2)
    k = pdp.k_rule(ds.total_residues())
    pairs = ds.pairs()
    gene_pairs = ds.gene_pairs()
    genes = [g.n_genes for g in ds.genomes]

    # residues and offsets resident in HBM before anything is timed
    dev = [pdp.DeviceGenome.of(g) for g in ds.genomes]
    batch = pdp.DictionaryBatch(dev, k)  # all ten dictionaries in one pdp_dict_build_many
    dicts = batch.dicts
    batch.build()
    tasks = pdp.all_pairs_tasks(dicts)
    tuned = None
    prm = pdp.params()
    if args.tune:
        best, tres = pdp.autotune(tasks, reps=3)
        prm = best
        tuned = {"tile_rows": int(best.tile_rows), "lds_budget": int(best.lds_budget), "join_entries": int(best.join_entries),
                 "persistent": bool(best.flags & B.PDP_PARAM_PERSISTENT), "best_ms": round(tres.best_ms, 4),
                 "first_ms": round(tres.first_ms, 4), "candidates": int(tres.tried)}
    runner = pdp.PairRunner(tasks, prm)
    runner.run()  # sizes the scratch and outputs
    for d in dicts:
        d.check_status()
    stream = torch.cuda.current_stream()

    def step():
        batch.build()
        runner.launch()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    code, needed, where = pdp.read_status(runner.status)
    if code != 0:
        raise SystemExit(f"device status {code} after warm-up (needed {needed}, where {where})")

    kernel_id = B.KERNELS[args.kernel]
    runner.plan.timer_start(kernel_id, args.steps)
    dict_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        dict_ev[s][0].record(stream)
        batch.build()
        dict_ev[s][1].record(stream)
        runner.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_n = runner.plan.timer_read()
    runner.plan.timer_stop()
    code, needed, where = pdp.read_status(runner.status)
    if code != 0:
        raise SystemExit(f"device status {code} in the timed region")
    for d in dicts:
        d.check_status()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = gene_pairs / (ms_per_step / 1e3)
    dict_ms = sum(a.elapsed_time(b) for a, b in dict_ev) / args.steps

    res = runner.results()
    entries = [int(d.host()["mv_ptr"][-1]) for d in dicts]
    bh_nnz = int(res.bh[0][-1])
    bbh_n = int(res.bbh[0][-1]) if res.bbh is not None else 0

    breakdown = {"dictionary_build_ms": round(dict_ms, 4)}
    if args.breakdown:
        for name, kid in B.KERNELS.items():
            runner.plan.timer_start(kid, 5)
            for _ in range(5):
                runner.launch()
            ms, n = runner.plan.timer_read()
            runner.plan.timer_stop()
            breakdown[f"{name}_ms"] = round(ms / max(n, 1), 4)
        torch.cuda.synchronize()

    avg_kernel_ms = kern_ms / max(kern_n, 1)
    alg = algorithmic_bytes(args.kernel, pairs, entries, bh_nnz, bbh_n, genes)
    achieved = alg / (avg_kernel_ms / 1e3) / 1e9 if avg_kernel_ms > 0 else 0.0
    traffic = None
    try:
        with open(args.traffic) as f:
            tr = json.load(f)
        if tr.get("source_hash") == source_hash() and args.kernel in tr.get("kernels", {}):
            traffic = tr["kernels"][args.kernel]["hbm_bytes_per_launch"]
    except (OSError, ValueError):
        pass
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": args.kernel,
                "kernel_ms": round(avg_kernel_ms, 5), "algorithmic_bytes": alg, "launches_timed": kern_n}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "gene-pair similarities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "all-pairs BH+BBH: 10 genomes x 3000 genes (family model), 45 genome pairs, "
                               "dictionary build included",
                   "genomes": len(genes), "genes_per_genome": genes[0], "k": k, "genome_pairs": len(pairs),
                   "gene_pairs": gene_pairs, "kmer_entries": int(sum(entries)), "best_hits": bh_nnz, "bbh_pairs": bbh_n},
        "roofline": roofline,
        "params": tuned if tuned is not None else "defaults",
        "breakdown": breakdown,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(ds, k, args.cpu_rows)
        cb["gpu_over_cpu"] = round(value / cb["value"], 1)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
