"""Benchmark of the EBIC evaluation hot path on one MI355X.

One step = one generation's evaluation of the whole population: for every
individual, the trend check over all rows, the row reduction into support
bitmaps and counts, the overlap with a 20-member archive and the FP64
fitness. Inputs (prepared matrix, population, archive) are resident in HBM
before the timed region. Prints one JSON line.

Workload (default): 10,000 x 500 float32 log-normal matrix with 10 planted
trend biclusters, 4,096 individuals of 3-64 columns (10% planted series),
negative trends on, approximate-trend threshold 850 per mille, archive of 20.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=2, help="workload index 1..3")
    ap.add_argument("--mode", choices=["plain"], default="plain")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM "
                         "byte counters of rocprofv3) and exit")
    return ap.parse_args()


def copy_probe(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)


def algorithmic_bytes(R: int, ks: np.ndarray, K: int) -> float:
    """Bytes one evaluation moves in the plain definition: every cell of the
    individual's R x k float32 submatrix once, its CSR entry (offset + k
    indices) and its outputs (support bitmap, count, fitness, K overlaps)."""
    P = ks.size
    return float(4.0 * R * ks.sum() + 4.0 * P + 2.0 * ks.sum() + P * (R / 8.0 + 12 + 4 * K))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the evaluation path "
              "is single-GPU here", file=sys.stderr)
        sys.exit(2)
    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import synth
    from paper_2105_01196_amd import ebic as E

    wi = args.workload
    w = synth.workload(wi)
    case = synth.workload_matrix(wi)
    seqs = synth.workload_population(wi, case)
    ks = np.array([len(s) for s in seqs], dtype=np.int64)
    P, R = len(seqs), case.R
    K = 20
    params = E.make_params(approx_permille=850, negative_trends=1, overlap_permille=750,
                           min_rows=5)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    x = torch.from_numpy(case.X).to(dev)
    m = E.ebic_matrix_prepare(x)
    pop = E.ebic_population_upload(seqs, case.C)
    # archive: the 20 best individuals of a first evaluation
    first = E.ebic_evaluate(m, pop, None, params)
    torch.cuda.synchronize()
    fit = first.fitness.cpu().numpy()[:P]
    top = [int(i) for i in np.argsort(-fit, kind="stable")[:K]]
    arch = E.archive_from_device(first.support, top, seqs)
    out = E.alloc_eval_out(P, m.words, K)

    def step():
        E.ebic_evaluate(m, pop, arch, params, out=out, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev0[s].record(stream)
        step()
        ev1[s].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))
    ms_per_step = wall * 1e3 / args.steps
    value = P / (ms_per_step / 1e3)
    alg = algorithmic_bytes(R, ks, K)
    achieved = alg / (kern_ms / 1e3) / 1e9
    cells = float(R * ks.sum())

    line = {
        "metric": "individual evaluations/s and % peak HBM GB/s (batched vs plain, bit-exact)",
        "value": value,
        "unit": "individual evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": R, "cols": case.C, "population": P,
                   "k_range": [w.k_min, w.k_max], "archive": K, "negative_trends": 1,
                   "approx_permille": 850, "path": args.mode},
        "cells_per_s": cells / (kern_ms / 1e3),
        "kernel_ms": kern_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": None},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(case.X, seqs, args)
    print(json.dumps(line), flush=True)


def cpu_baseline(X, seqs, args):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    p = oracle.make_params(approx_permille=850, negative_trends=1, overlap_permille=750,
                           min_rows=5, k_score_min=3)
    n = min(len(seqs), 1024)
    sample = seqs[:n]
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.evaluate(X, sample, params=p, nthreads=threads)
        reps += 1
        if time.perf_counter() - t0 > 8.0 or reps >= 20:
            break
    dt = time.perf_counter() - t0
    return {"value": reps * n / dt, "unit": "individual evaluations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n} individuals of the same population, {reps} passes, "
                      f"empty archive, {threads} OpenMP threads"}


if __name__ == "__main__":
    main()
