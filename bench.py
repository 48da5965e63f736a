#!/usr/bin/env python3
"""Benchmark of the best-hit path on one MI355X.

Headline workload (default): 50 synthetic protein genomes x U{3000..5000} genes
from the family model with 5% paralog copies (exact and near ties), k = 7 from
the k rule.  A step rebuilds all fifty k-mer dictionaries from residues already
in HBM and computes best hits in both directions plus BBH for all 1225 genome
pairs in one plan launch.  value = gene pairs compared (sum of |A||B| over the
pairs) per second.  The same JSON line carries the latency half of the metric:
the serving workload (200 resident genomes of 4000 genes, 2000 Poisson arrivals
at 0.8 of the closed-loop capacity, each compared with every resident), with
its p50/p99 per-genome latency and genomes/s.

Printed: one JSON line with the metric, a roofline entry for the dominant
kernel plus the pair path and the whole step (HIP events recorded by the
library around the kernels on their own stream), and the CPU oracle timed on
a bounded sample of the same workload.
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
    p.add_argument("--cpu-rows", type=int, default=None,
                   help="rows per direction per sampled pair in the dense CPU-oracle sample (default: 160 on the "
                        "50-genome workload, 384 amino-acid / 128 nucleotide rows on the 10 x 3000 one)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-latency", action="store_true", help="skip the serving run that gives p50/p99 latency")
    p.add_argument("--breakdown", action="store_true", help="also time every kernel group (extra launches)")
    p.add_argument("--calibrate-copy", action="store_true", help="only run a copy of known size (counter calibration)")
    p.add_argument("--counters-to-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                   default=None,
                   help="no GPU: turn four rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE of this "
                        "benchmark, then of --calibrate-copy) into the workload's entry of --traffic for the current "
                        "sources, in the launch shape given by --workload/--alphabet/--tile-rows/--colmax/--two-pass, "
                        "and print a markdown table")
    p.add_argument("--no-tune", action="store_true",
                   help="library defaults instead of the autotuner's pick of tile height, column maxima and "
                        "join sub-range size")
    p.add_argument("--tune-all", action="store_true",
                   help="the autotuner's whole built-in grid (tile height x sub-range size x persistence x column "
                        "maxima) instead of tile height x column maxima")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                   help="measured HBM traffic per kernel (from rocprofv3 counters), used when its source hash matches")
    p.add_argument("--two-pass", action="store_true", help="join in two passes (count, then write)")
    p.add_argument("--long-path", action="store_true",
                   help="bind every dictionary for long genes, so every task takes the long-gene path (one "
                        "work-group per best-hit row, sums from the index); the roofline entry is then the "
                        "tile_count group, which holds that path's count launch")
    p.add_argument("--join-entries", type=int, default=0, help="index entries per join sub-range (0: default)")
    p.add_argument("--persistent", action="store_true", help="persistent join and tile kernels")
    p.add_argument("--tile-rows", type=int, default=0, help="rows per accumulation tile (0: default; allpairs, serving)")
    p.add_argument("--colmax", action="store_true",
                   help="second genome's best hits from column maxima (Alg. 3): join records for one direction only")
    p.add_argument("--theta", default=None, help="length filter as NUM/DEN (Eq. length_threshold); off by default")
    p.add_argument("--tau", default=None, help="directional filter as NUM/DEN (Eq. directional_jaccard); off by default")
    p.add_argument("--alphabet", choices=("aa", "nt"), default="aa",
                   help="amino-acid genomes (default) or nucleotide genomes (genes 3x as long, k by the rule with "
                        "|alphabet| = 4)")
    p.add_argument("--workload", choices=("large", "allpairs", "batched", "serving"), default="large",
                   help="large: 50 genomes x U{3000..5000} genes with paralog copies, all 1225 pairs in one launch, "
                        "plus the serving run for latency (default); allpairs: 10 genomes x 3000 genes, 45 pairs; "
                        "batched: independent instances in waves, one graph-captured launch per wave, against one "
                        "plan per genome pair; serving: resident dictionaries and a Poisson stream of arriving genomes")
    p.add_argument("--instances", type=int, default=64, help="batched: instances (of the 400-instance workload)")
    p.add_argument("--wave-genomes", type=int, default=256, help="batched: genomes per wave")
    p.add_argument("--per-pair-sample", type=int, default=256, help="batched: pairs timed with one plan each")
    p.add_argument("--residents", type=int, default=200, help="serving: resident genomes")
    p.add_argument("--resident-genes", type=int, default=4000, help="serving: genes per resident")
    p.add_argument("--arrivals", type=int, default=2000, help="serving: arriving genomes (of the 2000-arrival stream)")
    p.add_argument("--load", type=float, default=0.8, help="serving: offered load as a fraction of closed-loop capacity")
    p.add_argument("--light-load", type=float, default=0.5,
                   help="serving: a second pass of the arrivals at this load (0: none), where queueing adds little")
    p.add_argument("--slots", type=int, default=2, help="serving: concurrent request slots")
    p.add_argument("--budget-gb", type=float, default=32.0, help="serving: HBM budget for requests in flight")
    p.add_argument("--serve-no-colmax", action="store_true",
                   help="serving: the residents' best hits from their own rows instead of column maxima")
    p.add_argument("--serve-tile-rows", type=int, default=128, help="serving: rows per accumulation tile")
    p.add_argument("--serve-join-entries", type=int, default=0,
                   help="serving: index entries per join sub-range (0: the library default, 512)")
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


# ------------------------------------------------------------------ algorithmic bytes

def input_bytes(pairs, entries) -> float:
    """Per unordered genome pair (A, B), each genome's k-mer entries read once: a u64 code and a
    u32 multiplicity, 12 bytes per entry (the join's share of the path)."""
    return float(sum(12 * (entries[i] + entries[j]) for i, j in pairs))


def output_bytes(pairs, genes, bh_nnz, bbh_n) -> float:
    """The outputs of the path: 16 bytes per best hit (row bookkeeping, column, num, den), 16 per
    BBH pair and 8 per gene of each pair's genomes (row pointers of both directions)."""
    return float(16 * bh_nnz + 16 * bbh_n + 8 * sum(genes[i] + genes[j] for i, j in pairs))


def build_bytes(residues, entries) -> float:
    """Dictionary build per genome: the residues read, the multiplicity vectors written (12 bytes
    per entry), read again and written out as the inverted index with its join keys (20 bytes)."""
    return float(sum(r + 12 * e + 12 * e + 20 * e for r, e in zip(residues, entries)))


def kernel_bytes(kernel: str, pairs, entries, genes, bh_nnz, bbh_n) -> float:
    if kernel == "join":
        return input_bytes(pairs, entries)
    if kernel == "tile_write":
        return float(16 * bh_nnz + 8 * sum(genes[i] + genes[j] for i, j in pairs))
    if kernel == "bbh":
        return float(16 * bbh_n)
    return 0.0


def say(*a):
    """Progress of the run on stderr (the result is the one JSON line on stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def _frac(nbytes, ms):
    gbs = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return round(gbs, 2), round(gbs / HBM_PEAK_GBS, 5)


# ------------------------------------------------------------------ CPU baseline

def cpu_info() -> dict:
    model, sockets, cores = None, set(), set()
    try:
        phys = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                    sockets.add(val)
                elif key == "core id":
                    cores.add((phys, val))
    except OSError:
        pass
    import oracle

    return {"model": model, "sockets": len(sockets) or None, "physical_cores": len(cores) or None,
            "logical_cpus": os.cpu_count(), "threads_used": oracle.default_threads()}


def _evenly(n, m):
    import numpy as np

    return np.unique(np.linspace(0, n - 1, min(m, n)).astype(np.uint32))


def cpu_baseline(ds, k, rows_per_dir, full_workload: bool):
    """The oracle as it stands, on the host cores.

    dense: the oracle that merges the multiplicity vectors of every gene pair (the paper's
    per-gene-pair similarity, rows handed to a pool of threads as Alg. 2's units of work), on
    ``rows_per_dir`` evenly spaced rows per direction of a seeded sample of pairs (all pairs of
    the 10 x 3000 workload, 32 of the 50-genome one); its rate gives a labelled extrapolation to
    the whole workload.  One whole pair (both directions and BBH) is timed as well, and a
    single-thread rate for comparison with per-thread CPU figures.  sparse: the oracle that
    visits only gene pairs sharing a k-mer, on every pair of the workload (BH both ways + BBH)."""
    import numpy as np

    import oracle

    threads = oracle.default_threads()
    say(f"CPU baseline on {threads} threads")
    t0 = time.perf_counter()
    og = oracle.genomes(ds.genomes, k, threads=threads)
    mv_s = time.perf_counter() - t0
    pairs = ds.pairs()
    if full_workload and len(pairs) > 32:
        rng = np.random.default_rng(2510236790)
        pick = sorted(int(x) for x in rng.choice(len(pairs), 32, replace=False))
    else:
        pick = list(range(len(pairs)))
    gene_pairs = 0
    t0 = time.perf_counter()
    for t in pick:
        i, j = pairs[t]
        for q, tt in ((og[i], og[j]), (og[j], og[i])):
            rows = _evenly(q.n, rows_per_dir)
            oracle.bh(q, tt, rows=rows, threads=threads)
            gene_pairs += len(rows) * tt.n
    dense_s = time.perf_counter() - t0
    rate = gene_pairs / dense_s
    say(f"dense oracle sample: {gene_pairs} gene pairs in {dense_s:.1f} s")
    # one whole pair, both directions and BBH: the two smallest genomes
    small = sorted(range(len(og)), key=lambda x: og[x].n)[:2]
    a, b = og[small[0]], og[small[1]]
    t0 = time.perf_counter()
    ab = oracle.bh(a, b, threads=threads)
    ba = oracle.bh(b, a, threads=threads)
    nbbh = len(oracle.bbh(ab, ba).a)
    pair_s = time.perf_counter() - t0
    # one thread
    rows = _evenly(og[0].n, 48)
    t0 = time.perf_counter()
    oracle.bh(og[0], og[1], rows=rows, threads=1)
    one_s = time.perf_counter() - t0
    one_rate = len(rows) * og[1].n / one_s
    # the sparse oracle on the whole workload
    say("sparse oracle on every pair")
    t0 = time.perf_counter()
    oracle.all_pairs_sparse(og, pairs, threads=threads)
    sparse_s = time.perf_counter() - t0
    total_gp = ds.gene_pairs()
    return {"value": round(rate, 1), "unit": "gene-pair similarities/s", "cores": threads, "kind": "oracle",
            "sample": f"dense oracle (every gene pair's multiplicity vectors merged, rows over a thread pool): "
                      f"{rows_per_dir} evenly spaced rows per direction of {len(pick)} seeded pairs of the "
                      f"{len(pairs)} ({gene_pairs} gene pairs, {dense_s:.1f} s); multiplicity vectors of every "
                      f"genome built first ({mv_s:.1f} s, not in the rate)",
            "seconds": round(dense_s, 2),
            "whole_pair_with_bbh": {"genes": [a.n, b.n], "seconds": round(pair_s, 2), "bbh_pairs": nbbh,
                                    "gene_pairs_per_s": round(2 * a.n * b.n / pair_s, 1)},
            "single_thread_gene_pairs_per_s": round(one_rate, 1),
            "extrapolated_whole_workload_s": {"value": round(total_gp * 2 / rate, 1),
                                              "label": "extrapolation: both directions of every gene pair of the "
                                                       "workload at the sampled dense rate, BBH excluded"},
            "sparse_oracle": {"seconds": round(sparse_s, 2), "gene_pairs_per_s": round(total_gp / sparse_s, 1),
                              "scope": f"all {len(pairs)} pairs, BH both ways + BBH, after the multiplicity vectors"},
            "host": cpu_info()}


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


# kernel groups of the traffic table: the group's kernels by name prefix
TRAFFIC_GROUPS = {"join": ("pdp::k_join_fused",),
                  "tile_count": ("void pdp::k_tile_count",),
                  "join_backup": ("void pdp::k_join_persistent", "void pdp::k_join<", "pdp::k_tile_ranges"),
                  "dictionary_build": ("pdp::k_mv", "void pdp::k_mv", "pdp::k_ix", "void pdp::k_ix")}


def _counter_rows(folder: str, counter: str):
    """{kernel name: [per-dispatch values]} of one counter from a rocprofv3 --pmc csv folder."""
    import csv
    import glob

    out = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def counters_to_traffic(args) -> None:
    """Calibrated HBM bytes per launch of each kernel group from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), scaled by what the same counters read for a copy of 1 GiB read and 1 GiB written."""
    fetch_dir, write_dir, cf_dir, cw_dir = args.counters_to_traffic
    gib_kib = float(1 << 20)
    copy_f = max(_counter_rows(cf_dir, "FETCH_SIZE").items(), key=lambda kv: sum(kv[1]))[1]
    copy_w = max(_counter_rows(cw_dir, "WRITE_SIZE").items(), key=lambda kv: sum(kv[1]))[1]
    ff = gib_kib / (sum(copy_f) / len(copy_f))
    wf = gib_kib / (sum(copy_w) / len(copy_w))
    fetch, write = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")
    groups, lines = {}, []
    for name in sorted(set(fetch) | set(write)):
        grp = next((g for g, pre in TRAFFIC_GROUPS.items() if any(name.startswith(x) for x in pre)), None)
        if grp is None:
            continue
        fk = sum(fetch.get(name, [0.0])) / max(1, len(fetch.get(name, [])))
        wk = sum(write.get(name, [0.0])) / max(1, len(write.get(name, [])))
        b = ff * fk * 1024 + wf * wk * 1024
        g = groups.setdefault(grp, {"hbm_bytes_per_launch": 0.0, "fetch_kib": 0.0, "write_kib": 0.0})
        g["hbm_bytes_per_launch"] += b
        g["fetch_kib"] += fk
        g["write_kib"] += wk
        lines.append((grp, name.split("(")[0], len(fetch.get(name, [])), fk, wk, b))
    for g in groups.values():
        g["hbm_bytes_per_launch"] = int(round(g["hbm_bytes_per_launch"]))
        g["fetch_kib"] = round(g["fetch_kib"], 1)
        g["write_kib"] = round(g["write_kib"], 1)
    large = args.workload == "large"
    nt = args.alphabet == "nt"
    wl_key = ("large" if large else "allpairs") + ("_nt" if nt else "")
    try:
        with open(args.traffic) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        tr = {}
    if tr.get("source_hash") != source_hash():
        tr = {"workloads": {}}  # counters of other sources say nothing about these kernels
    tr["source_hash"] = source_hash()
    tr["calibration"] = {"kernel": "elementwise int32 copy (1 GiB read, 1 GiB written)",
                         "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)}
    # one entry per launch shape of the workload (the autotuner may pick any of them)
    shape = {"tile_rows": int(args.tile_rows or 64), "column_maxima": bool(args.colmax),
             "join_entries": int(args.join_entries or 512), "two_pass": bool(args.two_pass)}
    entries = tr.setdefault("workloads", {}).get(wl_key, [])
    entries = [e for e in (entries if isinstance(entries, list) else [entries]) if e.get("shape") != shape]
    tr["workloads"][wl_key] = entries + [{"shape": shape, "kernels": groups}]
    with open(args.traffic, "w") as f:
        json.dump(tr, f, indent=1)
        f.write("\n")
    print(f"calibration: FETCH_SIZE x 1024 x {ff:.4f}, WRITE_SIZE x 1024 x {wf:.4f}; source hash {tr['source_hash']}")
    print("| kernel group | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes |")
    print("|---|---|---:|---:|---:|---:|")
    for grp, name, n, fk, wk, b in sorted(lines, key=lambda x: -x[5]):
        print(f"| {grp} | `{name}` | {n} | {fk:.0f} | {wk:.0f} | {b / 1e9:.3f} GB |")
    for grp, g in groups.items():
        print(f"| **{grp}** | **bytes per launch (calibrated)** | | | | **{g['hbm_bytes_per_launch'] / 1e9:.3f} GB** |")


def _pool_map(fn, items):
    """Host-side generation in worker processes (forked before anything touches the GPU)."""
    import multiprocessing as mp

    workers = max(1, min(16, os.cpu_count() or 1, len(items)))
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, items, chunksize=1)


def _gen_instance(i):
    from synth import batched_instances

    return next(batched_instances(start=i, count=1))


def _pctl(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def run_batched(args):
    """Workload 4 sample: independent instances, all pairs of each, in waves.  A wave is one
    dictionary build of all its genomes (k per instance) plus one plan launch (tile height, join
    sub-range size and persistence picked by the autotuner on the first wave),
    captured in a HIP graph; its replay is timed with events.  Instance latency = its wave's
    time (every instance of a wave finishes in the same launch).  The same pairs are also
    timed with one plan per genome pair (a sample), the launch pattern batching replaces."""
    import numpy as np

    t0 = time.perf_counter()
    insts = _pool_map(_gen_instance, list(range(args.instances)))
    gen_s = time.perf_counter() - t0

    import torch

    import paper_2510_23679_amd as pdp
    from paper_2510_23679_amd import binding as B

    torch.cuda.set_device(0)
    waves, cur, cur_g = [], [], 0
    for ds in insts:
        if cur and cur_g + len(ds.genomes) > args.wave_genomes:
            waves.append(cur)
            cur, cur_g = [], 0
        cur.append(ds)
        cur_g += len(ds.genomes)
    if cur:
        waves.append(cur)
    stream = torch.cuda.Stream()
    total_gp, total_ms, lat, wave_rows = 0, 0.0, [], []
    pp_gp, pp_ms = 0, 0.0
    rng = np.random.default_rng(4)
    tuned = None
    for w, wave in enumerate(waves):
        with torch.cuda.stream(stream):
            devs, ks, spans = [], [], []
            for ds in wave:
                k = pdp.k_rule(ds.total_residues())
                spans.append((len(devs), len(ds.genomes)))
                for g in ds.genomes:
                    devs.append(pdp.DeviceGenome.of(g))
                    ks.append(k)
            batch = pdp.DictionaryBatch(devs, ks)
            batch.build(stream)
            tasks, gp = [], 0
            for first, n in spans:
                for i in range(n):
                    for j in range(i + 1, n):
                        tasks.append((batch.dicts[first + i], batch.dicts[first + j],
                                      pdp.PDP_TASK_AB | pdp.PDP_TASK_BA | pdp.PDP_TASK_BBH))
                        gp += devs[first + i].n_genes * devs[first + j].n_genes
            if tuned is None and not args.persistent:
                # the first wave picks tile height, join sub-range size and persistence for all waves:
                # the autotuner times every combination at the capacity a sizing run found
                sizing = pdp.PairRunner(tasks, pdp.params())
                sizing.run(stream)
                cap = int(sizing.plan.info.inc_capacity)
                del sizing
                cands = [pdp.params(inc_capacity=cap, tile_rows=tr, join_entries=je, persistent=pe, colmax=cm)
                         for tr in (64, 128) for je in (256, 512, 768, 1024) for pe in (False, True)
                         for cm in (False, True)]
                best, tres = pdp.autotune(tasks, cands, reps=2, stream=stream)
                tuned = {"tile_rows": int(best.tile_rows), "join_entries": int(best.join_entries),
                         "persistent": bool(best.flags & B.PDP_PARAM_PERSISTENT),
                         "column_maxima": bool(best.flags & B.PDP_PARAM_COLMAX), "candidates": int(tres.tried),
                         "best_ms": round(tres.best_ms, 3), "first_ms": round(tres.first_ms, 3)}
            prm = (pdp.params(persistent=True) if args.persistent else
                   pdp.params(tile_rows=tuned["tile_rows"], join_entries=tuned["join_entries"],
                              persistent=tuned["persistent"], colmax=tuned["column_maxima"]))
            runner = pdp.PairRunner(tasks, prm)
            runner.run(stream)
            batch.check_status()
            graph = pdp.Graph.capture(stream)
            with graph:
                batch.build(stream)
                runner.launch(stream)
            graph.launch(stream)
            stream.synchronize()
            reps = 3
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(reps):
                graph.launch(stream)
            ev[1].record(stream)
            stream.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            code = pdp.read_status(runner.status)[0]
            if code != 0:
                raise SystemExit(f"wave {w}: device status {code}")
            two_pass = bool(pdp.status_flags(runner.status) & pdp.PDP_STATUS_TWO_PASS)
            total_gp += gp
            total_ms += ms
            lat += [ms] * len(wave)
            wave_rows.append({"instances": len(wave), "genomes": len(devs), "pairs": len(tasks), "gene_pairs": gp,
                              "ms": round(ms, 3), "join_two_passes": two_pass})
            # one plan per genome pair, launched back to back (sampled)
            pick = rng.choice(len(tasks), min(args.per_pair_sample, len(tasks)), replace=False)
            singles = [pdp.PairRunner([tasks[t]]) for t in pick]
            for r in singles:
                r.run(stream)
            ev[0].record(stream)
            for r in singles:
                r.launch(stream)
            ev[1].record(stream)
            stream.synchronize()
            pp_ms += ev[0].elapsed_time(ev[1])
            pp_gp += sum(tasks[t][0].n_genes * tasks[t][1].n_genes for t in pick)
            del graph, runner, singles, batch, devs
            torch.cuda.empty_cache()
    value = total_gp / (total_ms / 1e3)
    per_pair = pp_gp / (pp_ms / 1e3)
    out = {"metric": "batched all-pairs gene-pair similarities/sec incl. dictionary build, BH+BBH (1 GPU)",
           "value": round(value, 1), "unit": "gene-pair similarities/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"batched instances: first {len(insts)} of the 400-instance workload "
                                  f"(U{{4..30}} genomes x U{{500..5000}} genes each), waves of <= "
                                  f"{args.wave_genomes} genomes", "instances": len(insts), "waves": len(waves),
                      "gene_pairs": total_gp},
           "ms_total": round(total_ms, 3),
           "params": tuned if tuned is not None else {"persistent": True},
           "instance_latency_ms": {"p50": round(_pctl(lat, 50), 3), "p99": round(_pctl(lat, 99), 3)},
           "per_pair_launches": {"value": round(per_pair, 1), "pairs_timed": int(sum(min(args.per_pair_sample, w["pairs"])
                                                                                     for w in wave_rows)),
                                 "note": "one plan per genome pair, launched back to back; pairs sampled per wave"},
           "speedup_vs_per_pair": round(value / per_pair, 2), "waves_detail": wave_rows,
           "host_generation_s": round(gen_s, 1)}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ serving

_SERVING = None


def _gen_arrival(j):
    return _SERVING.arrival(j)


def prepare_serving(args):
    """Resident genomes and the first args.arrivals arriving genomes of the serving workload,
    generated on the host (arrivals in forked workers, before anything touches the GPU)."""
    global _SERVING
    from synth import serving_workload

    t0 = time.perf_counter()
    wl = serving_workload(n_residents=args.residents, resident_genes=args.resident_genes, n_arrivals=2000,
                          rate_per_s=1.0)
    _SERVING = wl
    n = min(args.arrivals, 2000)
    say(f"serving residents generated ({time.perf_counter() - t0:.1f} s); generating {n} arrivals")
    arrivals = _pool_map(_gen_arrival, list(range(n)))
    say(f"serving inputs ready ({time.perf_counter() - t0:.1f} s)")
    return wl, arrivals, time.perf_counter() - t0


def serve_stream(args, wl, arrivals):
    """Resident dictionaries built once; the arrivals are submitted to pdp_server at Poisson
    times at the offered load (a fraction of the closed-loop capacity measured first on the first
    arrivals); latency = completion - submission on the server's clock.  Each request builds its
    dictionary and computes BH both ways + BBH against every resident."""
    import torch

    import paper_2510_23679_amd as pdp

    n = len(arrivals)
    warm = min(16, n)
    k = pdp.k_rule(wl.residents.total_residues())
    devs = [pdp.DeviceGenome.of(g) for g in wl.residents.genomes]
    batch = pdp.DictionaryBatch(devs, k)
    batch.build()
    torch.cuda.synchronize()
    batch.check_status()
    res_genes = sum(d.n_genes for d in batch.dicts)
    srv = pdp.Server(batch.dicts, int(args.budget_gb * (1 << 30)), slots=args.slots,
                     prm=pdp.params(tile_rows=args.serve_tile_rows, colmax=not args.serve_no_colmax,
                                    join_entries=args.serve_join_entries))

    def drain(want, done):
        while len(done) < want:
            for d in srv.poll(64, wait_us=2000):
                done[d.tag] = d
                srv.release(d.tag)

    def open_loop(load, tag0):
        """Every arrival submitted at its Poisson time rescaled to load x capacity; per-request records."""
        lam = load * capacity
        times = wl.arrival_times[:n] / lam  # unit-rate Poisson times rescaled to rate lam
        done = {}
        start = time.perf_counter()
        for j in range(n):
            while time.perf_counter() - start < times[j]:
                for d in srv.poll(64, wait_us=0):
                    done[d.tag] = d
                    srv.release(d.tag)
            srv.submit(arrivals[j], tag0 + j)
        drain(n, done)
        wall = time.perf_counter() - start
        bad = [d.code for d in done.values() if d.code != 0]
        if bad:
            raise SystemExit(f"{len(bad)} requests failed, first code {bad[0]}")
        lat = [(d.done_us - d.submit_us) / 1e3 for d in done.values()]
        svc = [(d.done_us - d.admit_us) / 1e3 for d in done.values()]
        wait = [(d.admit_us - d.submit_us) / 1e3 for d in done.values()]
        phases = {}
        for name in ("h2d_ms", "build_ms", "pairs_ms", "d2h_ms"):
            xs = [getattr(d, name) for d in done.values()]
            phases[name[:-3]] = {"p50_ms": round(_pctl(xs, 50), 3), "p99_ms": round(_pctl(xs, 99), 3)}
        return {"offered_load": load, "offered_rate_per_s": round(lam, 2), "genomes_per_s": round(n / wall, 2),
                "p50_ms": round(_pctl(lat, 50), 3), "p99_ms": round(_pctl(lat, 99), 3), "max_ms": round(max(lat), 3),
                "service_p50_ms": round(_pctl(svc, 50), 3), "service_p99_ms": round(_pctl(svc, 99), 3),
                "admission_wait_p99_ms": round(_pctl(wait, 99), 3), "device_phases": phases,
                "gene_pairs_per_s": round(gp / wall, 1), "attempts_max": int(max(d.attempts for d in done.values())),
                "join_two_passes": sum(1 for d in done.values() if d.flags & pdp.PDP_STATUS_TWO_PASS)}

    gp = sum(int(g.n_genes) * res_genes for g in arrivals)
    try:
        # closed loop: the first arrivals submitted at once (admission under the budget), rate =
        # completions/s; the server keeps nothing of a request after its release, so the same
        # genomes are submitted again below as independent requests
        done = {}
        tw = time.perf_counter()
        for j in range(warm):
            srv.submit(arrivals[j], 10 ** 6 + j)
        drain(warm, done)
        cap_s = time.perf_counter() - tw
        capacity = warm / cap_s
        say(f"serving: closed-loop capacity {capacity:.1f} genomes/s; open loop of {n} arrivals at {args.load}")
        main = open_loop(args.load, 0)
        light = None
        if args.light_load:
            say(f"serving: open loop of {n} arrivals at {args.light_load}")
            light = open_loop(args.light_load, 2 * 10 ** 6)
        stats = srv.stats()
    finally:
        srv.close()
        del srv, batch, devs
        torch.cuda.empty_cache()
    out = dict(main)
    out.update({"arrivals": n, "closed_loop_genomes_per_s": round(capacity, 2), "retries": int(stats.retries),
                "peak_inflight": int(stats.peak_inflight), "peak_used_gb": round(stats.peak_used_bytes / 2 ** 30, 2),
                "workload": f"serving: {len(wl.residents.genomes)} resident genomes x "
                            f"{wl.residents.genomes[0].n_genes} genes (k = {k}), first {n} of 2000 Poisson arrivals "
                            f"(U{{1000..6000}} genes drawn from resident families), offered load {args.load} of the "
                            f"closed-loop capacity, {args.slots} slots, {args.budget_gb} GB budget, "
                            f"{args.serve_tile_rows}-row tiles, column maxima {'off' if args.serve_no_colmax else 'on'}",
                "note": "latency = completion - submission, including planning, admission wait, the host-to-device "
                        "copy of the arriving genome and the copy of its results to host memory"})
    if light is not None:
        out["light_load"] = light
    return out


def run_serving(args):
    wl, arrivals, gen_s = prepare_serving(args)
    import torch

    torch.cuda.set_device(0)
    lat = serve_stream(args, wl, arrivals)
    out = {"metric": "served genomes/sec and p50/p99 per-genome latency (BH+BBH against every resident, 1 GPU)",
           "value": lat["genomes_per_s"], "unit": "genomes/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u32",
           "data": "synthetic", "config": {"workload": lat.pop("workload"), "slots": args.slots,
                                            "budget_gb": args.budget_gb, "offered_load": args.load,
                                            "tile_rows": args.serve_tile_rows,
                                            "join_entries": args.serve_join_entries or 512,
                                            "column_maxima": not args.serve_no_colmax},
           "latency": lat, "host_generation_s": round(gen_s, 1)}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ all pairs

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: genome pairs are independent and "
                                   "would shard across GPUs, but no multi-GPU path is built",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.counters_to_traffic:
        counters_to_traffic(args)
        return
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return

    large = args.workload == "large"
    serving = None
    if large and not args.no_latency:
        serving = prepare_serving(args)  # forks workers: before anything touches the GPU

    import torch

    import paper_2510_23679_amd as pdp
    from paper_2510_23679_amd import binding as B
    from synth import make_config

    torch.cuda.set_device(0)
    nt = args.alphabet == "nt"
    ds = make_config(3 if large else 2, alphabet=args.alphabet)
    say(f"{ds.description}: {len(ds.genomes)} genomes, {ds.total_genes()} genes")
    k = pdp.k_rule(ds.total_residues(), 4 if nt else 20)
    pairs = ds.pairs()
    gene_pairs = ds.gene_pairs()
    genes = [g.n_genes for g in ds.genomes]

    # residues and offsets resident in HBM before anything is timed
    dev = [pdp.DeviceGenome.of(g) for g in ds.genomes]
    # every dictionary in one pdp_dict_build_many
    batch = pdp.DictionaryBatch(dev, k, long_genes=True if args.long_path else None)
    if args.long_path and args.kernel == "join":
        args.kernel = "tile_count"  # no join runs on the long-gene path
    dicts = batch.dicts
    batch.build()
    tasks = pdp.all_pairs_tasks(dicts)
    tuned = None

    def frac(x):
        return tuple(int(v) for v in x.split("/")) if x else None

    prm = pdp.params(theta=frac(args.theta), tau=frac(args.tau), colmax=args.colmax, two_pass=args.two_pass,
                     join_entries=args.join_entries, persistent=args.persistent, tile_rows=args.tile_rows)
    explicit = args.join_entries or args.persistent or args.tile_rows or args.colmax or args.two_pass or args.long_path
    if not args.no_tune and not explicit:
        # the launch shape for this workload, picked by the library's autotuner before anything is timed
        cands = None if args.tune_all else [pdp.params(tile_rows=tr, colmax=cm, join_entries=je, theta=frac(args.theta),
                                                       tau=frac(args.tau))
                                            for tr in (64, 128) for cm in (False, True) for je in (0, 768)]
        best, tres = pdp.autotune(tasks, cands, reps=3, base=prm)
        prm = best
        tuned = {"autotuned": True, "tile_rows": int(best.tile_rows), "join_entries": int(best.join_entries),
                 "persistent": bool(best.flags & B.PDP_PARAM_PERSISTENT),
                 "column_maxima": bool(best.flags & B.PDP_PARAM_COLMAX), "best_ms": round(tres.best_ms, 4),
                 "first_ms": round(tres.first_ms, 4), "candidates": int(tres.tried)}
        say(f"autotuner: {tuned}")
    runner = pdp.PairRunner(tasks, prm)
    runner.run()  # sizes the scratch and outputs
    for d in dicts:
        d.check_status()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        batch.build()
        runner.launch()
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
    two_pass = bool(pdp.status_flags(runner.status) & pdp.PDP_STATUS_TWO_PASS) or bool(prm.flags & B.PDP_PARAM_TWO_PASS)
    for d in dicts:
        d.check_status()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = gene_pairs / (ms_per_step / 1e3)
    say(f"{args.steps} timed steps: {ms_per_step:.3f} ms per step")
    dict_ms = sum(a.elapsed_time(b) for a, b in dict_ev) / args.steps

    res = runner.results()
    entries = [int(d.host()["mv_ptr"][-1]) for d in dicts]
    residues = [int(g.n_residues) for g in ds.genomes]
    bh_nnz = int(res.bh[0][-1])
    bbh_n = int(res.bbh[0][-1]) if res.bbh is not None else 0

    # the whole plan launch (every kernel of the pair path), timed after the timed steps
    reps = 5
    runner.plan.timer_start(B.KERNELS["all"], reps)
    for _ in range(reps):
        runner.launch()
    path_ms, path_n = runner.plan.timer_read()
    runner.plan.timer_stop()
    path_ms /= max(path_n, 1)

    breakdown = {"dictionary_build_ms": round(dict_ms, 4), "pair_path_ms": round(path_ms, 4)}
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
    alg = kernel_bytes(args.kernel, pairs, entries, genes, bh_nnz, bbh_n)
    achieved, kfrac = _frac(alg, avg_kernel_ms)
    path_bytes = input_bytes(pairs, entries) + output_bytes(pairs, genes, bh_nnz, bbh_n)
    step_bytes = path_bytes + build_bytes(residues, entries)
    path_gbs, path_frac = _frac(path_bytes, path_ms)
    step_gbs, step_frac = _frac(step_bytes, ms_per_step)
    traffic, measured = None, None
    wl_key = ("large" if large else "allpairs") + ("_nt" if nt else "")
    shape = {"tile_rows": int(prm.tile_rows or 64), "column_maxima": bool(prm.flags & B.PDP_PARAM_COLMAX),
             "join_entries": int(prm.join_entries or 512), "two_pass": two_pass}
    try:
        with open(args.traffic) as f:
            tr = json.load(f)
        wl_tr = tr.get("workloads", {}).get(wl_key, [])
        wl_tr = next((e for e in (wl_tr if isinstance(wl_tr, list) else [wl_tr]) if e.get("shape") == shape), {})
        kernels = wl_tr.get("kernels", {})
        # counters hold for these kernels in the launch shape they were taken in
        if tr.get("source_hash") == source_hash() and args.kernel in kernels:
            traffic = kernels[args.kernel]["hbm_bytes_per_launch"]
            measured = dict(zip(("achieved", "frac"), _frac(traffic, avg_kernel_ms)))
    except (OSError, ValueError):
        pass
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kfrac,
                "traffic": traffic, "kernel": args.kernel, "kernel_ms": round(avg_kernel_ms, 5),
                "algorithmic_bytes": alg,
                "bytes_scope": "join: 12 bytes per k-mer entry of both genomes of every pair (the input term)",
                "launches_timed": kern_n, "join_layout": "two passes" if two_pass else "one pass",
                "measured": measured,
                "path": {"achieved": path_gbs, "frac": path_frac, "ms": round(path_ms, 4),
                         "algorithmic_bytes": path_bytes,
                         "scope": "every kernel of the plan launch; inputs + outputs (16 B per best hit and per BBH "
                                  "pair, 8 B per gene of each pair)"},
                "step": {"achieved": step_gbs, "frac": step_frac, "ms": round(ms_per_step, 4),
                         "algorithmic_bytes": step_bytes,
                         "scope": "the whole step: the pair path's bytes + the dictionary build's (residues, "
                                  "multiplicity vectors written and read, index written)"}}

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
        "config": {"workload": ("all-pairs BH+BBH: 50 genomes x U{3000..5000} genes (family model with 5% paralog "
                                "copies" if large else "all-pairs BH+BBH: 10 genomes x 3000 genes (family model")
                               + (", nucleotide genes" if nt else "")
                               + f"), {len(pairs)} genome pairs, dictionary build included",
                   "alphabet": "nucleotide" if nt else "amino acid",
                   "genomes": len(genes), "genes_per_genome": genes[0] if not large else [min(genes), max(genes)],
                   "genes": int(sum(genes)), "k": k, "genome_pairs": len(pairs),
                   "gene_pairs": gene_pairs, "kmer_entries": int(sum(entries)), "best_hits": bh_nnz, "bbh_pairs": bbh_n,
                   "filters": {"theta": args.theta, "tau": args.tau},
                   "column_maxima": bool(prm.flags & B.PDP_PARAM_COLMAX),
                   "pair_path": "long-gene path (every dictionary bound for long genes)" if args.long_path
                   else "default"},
        "roofline": roofline,
        "params": tuned if tuned is not None else ("defaults" if not explicit
                                                   else {"join_entries": args.join_entries, "persistent": args.persistent,
                                                         "tile_rows": args.tile_rows, "column_maxima": args.colmax,
                                                         "two_pass": args.two_pass, "long_path": args.long_path}),
        "breakdown": breakdown,
    }
    del runner, res, batch, dicts, dev
    torch.cuda.empty_cache()
    if serving is not None:
        wl, arrivals, gen_s = serving
        lat = serve_stream(args, wl, arrivals)
        lat["host_generation_s"] = round(gen_s, 1)
        out["latency"] = lat
    if not args.no_cpu_baseline:
        cb = cpu_baseline(ds, k, args.cpu_rows or (160 if large else (128 if nt else 384)), large)
        cb["gpu_over_cpu"] = round(value / cb["value"], 1)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
