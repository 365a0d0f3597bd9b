"""Benchmark of the EBIC evaluation hot path on one MI355X.

One step = one generation's evaluation of every individual of the batch:
the trend check over all rows, the row reduction into support bitmaps and
counts, the overlap with each population's 20-member archive and the FP64
fitness. Inputs (prepared matrix and its pair table, populations, archives)
are resident in HBM before the timed region. Prints one JSON line.

Workload (default, "batched-10000x500"): 10,000 x 500 float32 log-normal
matrix with 10 planted trend biclusters; 4 independent populations of 1,024
individuals of 3-64 columns (10% planted series) = 4,096 evaluations per
step, all in one launch of the batched evaluator; negative trends on,
approximate-trend threshold 850 per mille. The plain path (one launch per
population) is timed on the same inputs for the batched-vs-plain ratio, and
both outputs are compared bit for bit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batch_kernel.txt")
KERNEL_SOURCES = ["paper_2105_01196_amd/csrc/batched.hip", "paper_2105_01196_amd/csrc/device.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=2, help="matrix workload index 1..3")
    ap.add_argument("--populations", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-path leg")
    ap.add_argument("--legs", action="store_true",
                    help="also time the same step as a graph replay and in the gather form")
    ap.add_argument("--overlap", action="store_true",
                    help="also write each individual's per-member overlap counts (the "
                         "penalty itself never needs this output)")
    ap.add_argument("--serving", type=int, default=0, metavar="JOBS",
                    help="instead of the evaluation step, run the job-server mix: JOBS jobs "
                         "with Poisson arrivals, and print its own JSON line")
    ap.add_argument("--serving-gens", type=int, default=30)
    ap.add_argument("--recovery", type=int, default=None, metavar="WORKLOAD",
                    help="instead of the evaluation step, run the whole method on a planted "
                         "workload (0, 1 or 2) with its parameters and print the clustering "
                         "error of the biclusters found against the planted ones")
    ap.add_argument("--loop", type=int, default=None, metavar="WORKLOAD",
                    help="instead of the evaluation step, run the whole method on a workload "
                         "(1, 2 or 3) with the loop on the host (ebic_run) and on the device "
                         "(ebic_run_device), and print the time per generation of each")
    ap.add_argument("--loop-only", choices=["host", "device"], default=None,
                    help="with --loop: run only that loop (for profiling)")
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, cpi: int, kb: int, wpl: int):
    """HBM bytes per launch of the evaluation kernel from the committed
    rocprofv3 counter summary (one block per workload, each opened by a
    `workload:` line), or None when the kernel source changed since the
    counters were taken or they were taken on another item shape."""
    try:
        blocks, glob, cur = {}, {}, None
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" not in line or line.startswith("#"):
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k == "workload":
                    cur = blocks.setdefault(v, {})
                elif cur is None:
                    glob[k] = v
                else:
                    cur[k] = v
        if glob.get("source_sha256_16") != kernel_source_hash():
            return None
        fields = blocks.get(workload)
        if not fields or (int(fields["chunk_groups_per_item"]), int(fields["loads_in_flight"]),
                          int(fields["words_per_lane"])) != (cpi, kb, wpl):
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus == 1 and args.serving:
        serving(args)
        return
    if args.gpus == 1 and args.recovery is not None:
        recovery(args)
        return
    if args.gpus == 1 and args.loop is not None:
        loop_times(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the evaluation path "
              "is single-GPU here", file=sys.stderr)
        sys.exit(2)
    import torch
    sys.path.insert(0, ROOT)
    import synth
    from paper_2105_01196_amd import ebic as E

    wi = args.workload
    w = synth.workload(wi)
    case = synth.workload_matrix(wi)
    R, C = case.R, case.C
    npop = args.populations
    per = w.population // npop
    pops_seqs = [synth.workload_population(wi, case, P=per, seed=synth.POP_SEED + wi + 10 * j)
                 for j in range(npop)]
    K = 20
    params = E.make_params(approx_permille=850, negative_trends=1, overlap_permille=750,
                           min_rows=5)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    x = torch.from_numpy(case.X).to(dev)
    m = E.ebic_matrix_prepare(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.ebic_pairs_prepare(m)
    torch.cuda.synchronize()
    table_ms = (time.perf_counter() - t0) * 1e3

    pops, archs, plain_outs, jobs = [], [], [], []
    for seqs in pops_seqs:
        pop = E.ebic_population_upload(seqs, C)
        first = E.ebic_evaluate(m, pop, None, params)
        torch.cuda.synchronize()
        fit = first.fitness.cpu().numpy()[:len(seqs)]
        top = [int(i) for i in np.argsort(-fit, kind="stable")[:K]]
        arch = E.archive_from_device(first.support, top, seqs)
        E.set_order(pop, E.longest_first(seqs))
        pops.append(pop)
        archs.append(arch)
        plain_outs.append(E.alloc_eval_out(len(seqs), m.words, K, overlap=args.overlap))
        jobs.append(E.make_job(m, pop, arch, params, overlap=args.overlap))
    # item shape timed on the first (warm-up) run. One kernel per step: a HIP
    # graph of that one node (EBIC_BATCH_GRAPH) adds launch overhead here
    batch = E.Batch(jobs, tune=True)
    P = sum(len(s) for s in pops_seqs)
    ks = np.array([len(s) for seqs in pops_seqs for s in seqs], dtype=np.int64)

    def plain_step():
        for pop, arch, out in zip(pops, archs, plain_outs):
            E.ebic_evaluate(m, pop, arch, params, out=out, stream=stream)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps

    # batched (the measured path). Two HIP events on the launch stream
    # bracket the timed region: the kernel's average duration is their
    # interval over the steps (gaps between launches included). Events
    # around every launch would put markers between the kernels and slow
    # the very steps they time.
    for _ in range(args.warmup):
        batch.run(stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        batch.run(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_batched = (time.perf_counter() - t) * 1e3 / args.steps
    kern = ev0.elapsed_time(ev1) / args.steps
    cpi, kb, wpl = batch.tuning()

    plain = None
    if not args.no_plain:
        for _ in range(args.warmup):
            plain_step()
        ms_plain = timed(plain_step, max(args.steps // 4, 5))
        same = all(torch.equal(o.count, j.out.count) and torch.equal(o.fitness, j.out.fitness)
                   and torch.equal(o.support, j.out.support)
                   and (o.overlap is None or torch.equal(o.overlap, j.out.overlap))
                   for o, j in zip(plain_outs, jobs))
        plain = {"value": P / (ms_plain / 1e3), "ms_per_step": ms_plain,
                 "launches_per_step": npop, "bit_exact_vs_batched": bool(same)}

    legs = None
    if args.legs:
        # the same step replayed from a HIP graph (same item shape), and in
        # the gather form (no pair table); both write the same outputs
        ref = [(j.out.count.clone(), j.out.fitness.clone(), j.out.support.clone()) for j in jobs]
        legs = {}
        for name, kw in (("graph", {"graph": True}), ("gather", {"gather": True})):
            b2 = E.Batch(jobs, **kw)
            if name == "graph":
                b2.set_tuning(cpi, kb, wpl)
            for _ in range(args.warmup):
                b2.run(stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                b2.run(stream)
            e1.record(stream)
            torch.cuda.synchronize()
            same = all(torch.equal(r[0], j.out.count) and torch.equal(r[1], j.out.fitness)
                       and torch.equal(r[2], j.out.support) for r, j in zip(ref, jobs))
            legs[name] = {"ms_per_step": e0.elapsed_time(e1) / args.steps,
                          "tuning": list(b2.tuning()), "bit_exact_vs_batched": bool(same)}
            b2.close()
        legs["direct_ms_per_step"] = kern

    value = P / (ms_batched / 1e3)
    # Algorithmic bytes of the kernel: per individual, one R-bit pair bitmap
    # per step ((k-1) R/8), its CSR entry (4 + 2k), its support bitmap
    # written (R/8), and its count and fitness (12).
    alg = float(((ks - 1) * R / 8.0 + 4 + 2 * ks + R / 8.0 + 12).sum())
    achieved = alg / (kern / 1e3) / 1e9
    traffic = measured_traffic(w.name, cpi, kb, wpl)
    line = {
        "metric": "individual evaluations/s and % peak HBM GB/s (batched vs plain, bit-exact)",
        "value": value,
        "unit": "individual evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": R, "cols": C, "populations": npop,
                   "individuals": P, "k_range": [w.k_min, w.k_max], "archive": K,
                   "negative_trends": 1, "approx_permille": 850, "overlap_output": args.overlap,
                   "path": "batched, pair table, one fused launch per step",
                   "tuned_item": {"chunk_groups_per_item": cpi, "loads_in_flight": kb,
                                  "words_per_lane": wpl}},
        "cells_per_s": float(R * ks.sum()) / (ms_batched / 1e3),
        "kernel_ms": {"batch_kernel": kern},
        "pair_table": {"bytes": int(m.pairs.numel() * 8), "build_ms": table_ms},
        "plain": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / ms_batched) if plain else None,
        "legs": legs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "achieved_kind": "effective: algorithmic bytes over kernel time, every "
                                      "step's pair bitmap counted, also those that early "
                                      "exit skips",
                     "traffic": traffic,
                     "dram_gbps": (traffic / (kern / 1e3) / 1e9) if traffic else None,
                     "dram_frac": (traffic / (kern / 1e3) / 1e9 / HBM_PEAK_GBPS)
                     if traffic else None,
                     "kernel": "batch_kernel",
                     "kernel_timing": "two HIP events on the launch stream around the "
                                      "timed steps, interval / steps",
                     "source_sha256_16": kernel_source_hash()},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(case.X, pops_seqs, K)
    print(json.dumps(line), flush=True)
    batch.close()


def serving(args):
    """Job-server mix: jobs on matrices of 500-50,000 rows x 20-2,000 columns
    (log-uniform, log-normal background, 1-20 planted biclusters each),
    populations of 256-4,096, arriving as a Poisson process whose mean gap is
    a quarter of one median job's time alone. Reports the server's throughput
    and p50/p99 job latency, and the same jobs run one after another."""
    import torch
    sys.path.insert(0, ROOT)
    import synth
    from paper_2105_01196_amd import ebic as E

    specs = synth.serving_jobs(args.serving)
    t0 = time.perf_counter()
    mats = [synth.job_matrix(s).X for s in specs]
    gen_s = time.perf_counter() - t0

    def params(s):
        return E.make_params(approx_permille=850, negative_trends=1, overlap_permille=750,
                             min_rows=5, k_min=3, k_max=min(64, s.C), archive_size=20,
                             n_out=20, population=s.population, generations=args.serving_gens,
                             max_tabu_hits=10 ** 9, tournament=4, max_attempts=1000)

    sizes = [s.R * s.C * s.population for s in specs]
    med = int(np.argsort(sizes)[len(sizes) // 2])
    E.ebic_run(mats[med], params(specs[med]), specs[med].seed)  # warm-up
    t = time.perf_counter()
    E.ebic_run(mats[med], params(specs[med]), specs[med].seed)
    t_one = time.perf_counter() - t
    arrivals = synth.poisson_arrivals(len(specs), t_one / 4)

    srv = E.Server()
    torch.cuda.synchronize()
    start = time.perf_counter()
    ids = []
    for s, X, at in zip(specs, mats, arrivals):
        delay = at - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(X, params(s), s.seed))
    results = [srv.wait(i) for i in ids]
    wall = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    evals = sum(r.evaluations for r in results)

    # the same jobs, one after another, each through ebic_run
    t = time.perf_counter()
    same = True
    for s, X, r in zip(specs, mats, results):
        a = E.ebic_run(X, params(s), s.seed)
        same &= (a.generations == r.generations and np.array_equal(a.trace, r.trace)
                 and all(np.array_equal(x.rows, y.rows) and np.array_equal(x.cols, y.cols)
                         for x, y in zip(a.biclusters, r.biclusters)))
    seq = time.perf_counter() - t
    line = {
        "metric": "job-server individual evaluations/s and p50/p99 job latency",
        "value": evals / wall, "unit": "individual evaluations/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "u32",
        "config": {"workload": "serving-mix", "jobs": len(specs),
                   "rows": [min(s.R for s in specs), max(s.R for s in specs)],
                   "cols": [min(s.C for s in specs), max(s.C for s in specs)],
                   "populations": sorted({s.population for s in specs}),
                   "generations": args.serving_gens, "archive": 20,
                   "mean_gap_s": t_one / 4},
        "wall_s": wall, "p50_latency_s": st["p50_latency_s"],
        "p99_latency_s": st["p99_latency_s"], "mean_latency_s": st["mean_latency_s"],
        "ticks": st["ticks"], "evaluations": evals,
        "tick_phases_s": {"stage": st["stage_s"], "device": st["device_s"],
                          "host_steps": st["host_s"], "setup_beside_ticks": st["setup_s"],
                          "release": st["release_s"], "ticks_total": st["busy_s"]},
        "sequential_runs": {"wall_s": seq, "value": evals / seq},
        "results_identical_alone_and_mixed": bool(same),
        "matrix_generation_s": gen_s,
    }
    print(json.dumps(line), flush=True)


def recovery(args):
    """ebic_run on a planted workload with its own parameters; the
    clustering error (Sec. 2.2, Eq. 1) of the biclusters found against the
    planted ones, reported as D_max/|U| (1 = perfect) beside Eq. (1)'s
    value."""
    sys.path.insert(0, ROOT)
    import synth
    from paper_2105_01196_amd import ebic as E
    wi = args.recovery
    w = synth.workload(wi)
    case = synth.workload_matrix(wi)
    p = E.make_params(approx_permille=850, negative_trends=w.negative_trends,
                      overlap_permille=750, min_rows=5, k_min=w.k_min, k_max=w.k_max,
                      archive_size=w.archive_size, n_out=w.n_out, population=w.population,
                      generations=w.generations, max_tabu_hits=100000, tournament=4,
                      max_attempts=1000)
    E.ebic_run(case.X, p, synth.GA_SEED + wi)  # warm-up (first-use costs)
    t0 = time.perf_counter()
    res = E.ebic_run(case.X, p, synth.GA_SEED + wi)
    wall = time.perf_counter() - t0
    truth = [(t.rows, t.cols) for t in case.truth]
    score, ce = E.ebic_ce_score(res.biclusters, truth, case.R, case.C)
    print(json.dumps({
        "metric": "clustering error of ebic_run vs the planted biclusters (D_max/|U|)",
        "value": score, "unit": "fraction of the union of cells", "higher_is_better": True,
        "eq1_value": ce, "n_gpus": 1, "data": "synthetic",
        "config": {"workload": w.name, "planted": len(truth), "found": len(res.biclusters),
                   "generations": res.generations, "population": w.population,
                   "negative_trends": w.negative_trends},
        "wall_s": wall, "evaluations": res.evaluations,
        "evaluations_per_s": res.evaluations / wall}), flush=True)


def loop_times(args):
    """ebic_run and ebic_run_device on one workload with its loop settings
    (the batched and large workloads with 100 and 20 generations): wall time
    per generation, median of three runs after a warm-up run, and whether the
    two loops gave the same run."""
    sys.path.insert(0, ROOT)
    import synth
    from paper_2105_01196_amd import ebic as E
    wi = args.loop
    w = synth.workload(wi)
    case = synth.workload_matrix(wi)
    gens = {1: w.generations, 2: 100, 3: 20}.get(wi, w.generations)
    p = E.make_params(approx_permille=850, negative_trends=1, overlap_permille=750, min_rows=5,
                      k_min=w.k_min, k_max=w.k_max, archive_size=20, n_out=w.n_out,
                      population=w.population, generations=gens, max_tabu_hits=100000,
                      tournament=4, max_attempts=1000)
    seed = synth.GA_SEED + wi
    out = {"metric": "wall time per generation of the method's loop",
           "unit": "us per generation", "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic",
           "config": {"workload": w.name, "population": w.population, "generations": gens,
                      "archive": 20, "negative_trends": 1}}
    results = {}
    for name, fn in (("host", E.ebic_run), ("device", E.ebic_run_device)):
        if args.loop_only and name != args.loop_only:
            continue
        fn(case.X, p, seed)  # warm-up
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            r = fn(case.X, p, seed)
            ts.append(time.perf_counter() - t)
        results[name] = r
        out[f"{name}_us_per_generation"] = sorted(ts)[1] / r.generations * 1e6
    if len(results) == 2:
        a, b = results["host"], results["device"]
        out["same_run"] = bool(
            (a.generations, a.evaluations, a.tabu_hits, a.stop_reason) ==
            (b.generations, b.evaluations, b.tabu_hits, b.stop_reason)
            and np.array_equal(a.trace, b.trace)
            and all(np.array_equal(x.rows, y.rows) and np.array_equal(x.cols, y.cols)
                    for x, y in zip(a.biclusters, b.biclusters)))
        out["device_vs_host"] = out["host_us_per_generation"] / out["device_us_per_generation"]
    print(json.dumps(out), flush=True)


def cpu_threads():
    """Threads for the oracle leg: the host's CPU share as OpenMP sees it
    (OMP_NUM_THREADS when set, else the CPUs this process may run on)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(int(env), avail)) if env.isdigit() else avail


def cpu_baseline(X, pops_seqs, K):
    """The oracle, as it stands, on the same step the GPU times: every
    individual of every population, each population against an archive of
    its own top K (chosen by the oracle's own first pass, as the GPU leg
    chooses them from its first pass)."""
    import oracle
    threads = cpu_threads()
    p = oracle.make_params(approx_permille=850, negative_trends=1, overlap_permille=750,
                           min_rows=5, k_score_min=3)
    archives = []
    for seqs in pops_seqs:
        first = oracle.evaluate(X, seqs, params=p, nthreads=threads)
        top = [int(i) for i in np.argsort(-first.fitness, kind="stable")[:K]]
        archives.append(oracle.Archive(first.support[top], [list(seqs[i]) for i in top]))
    P = sum(len(s) for s in pops_seqs)
    t0 = time.perf_counter()
    reps = 0
    while True:
        for seqs, arch in zip(pops_seqs, archives):
            oracle.evaluate(X, seqs, archive=arch, params=p, nthreads=threads)
        reps += 1
        if time.perf_counter() - t0 > 3.0 or reps >= 20:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one thread, over the first population's first 128
    one = list(pops_seqs[0])[:128]
    t1 = time.perf_counter()
    oracle.evaluate(X, one, archive=archives[0], params=p, nthreads=1)
    d1 = time.perf_counter() - t1
    return {"value": reps * P / dt, "unit": "individual evaluations/s",
            "cores": threads, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"the timed step itself: {len(pops_seqs)} populations, {P} individuals, "
                      f"each population against its own {K}-member archive, {reps} passes, "
                      f"{threads} OpenMP threads (the process's CPU share; the host reports "
                      f"{os.cpu_count()} CPUs), {dt:.1f} s wall",
            "single_thread": {"value": len(one) / d1, "cores": 1,
                              "sample": f"the first population's first {len(one)} individuals "
                                        f"against its archive, one pass, {d1:.2f} s"}}


if __name__ == "__main__":
    main()
