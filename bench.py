#!/usr/bin/env python3
"""Benchmark of the chunked speculative DFA scan on one MI355X.

Default workload (the 3.2-Gbase genome-scale configuration): 3.2e9 bases of a
first-order Markov source (GC 0.41, 1% N in runs), stored 2-bit packed with a
1-bit N mask, scanned for 64 random 12-mers (Aho-Corasick automaton of 632
states) with per-pattern counts.  A step is one coex_count over the whole
sequence: possible starting states, speculation with ballot convergence, the
scan of every chunk, the join, the fix-up and the per-pattern reduction.  The
sequence is resident in HBM before timing starts.

Prints one JSON line:  metric/value (Gbases/s), ms_per_step, a roofline entry
for the dominant kernel (the speculation + chunk scan kernel, timed with HIP
events on its stream inside the timed region), and a CPU baseline (the oracle,
single thread, over the same sequence, which doubles as the exactness check).

  python bench.py [--steps K] [--warmup W] [--workload genome|mid|small|batched|serving|parity|partitioned]
"""
from __future__ import annotations

import argparse
import types
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1509_01506_amd", "csrc", f) for f in ("coex.hip", "kernels.hpp", "tail.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """The host CPU the baselines ran on: model (as lscpu names it), logical
    CPUs of the machine and CPUs this process may use."""
    model = ""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "usable_cpus": usable}


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the scan kernel from the stored rocprofv3 PMC
    runs, if they were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        e = t.get(workload)
        if not e or e.get("source_sha") != kernel_source_sha():
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def build_workload(name: str):
    import numpy as np
    import paper_1509_01506_amd as coex
    from synth import configs
    if name == "genome":
        packed, mask, kmers = configs.genome()
        n = configs.GENOME_N
        return dict(
            n=n, enc=coex.ENC_2BIT, host=(packed, mask), dfa=coex.Dfa.kmers(kmers), patterns=kmers, chunk=0,
            bytes_per_base=0.375, find=False,
            desc="genome: 3.2e9 Markov bases (GC 0.41, 1% N runs), 2-bit packed + 1-bit N mask; "
                 "64 random 12-mers as one Aho-Corasick automaton; per-pattern counts")
    if name == "partitioned":
        import synth
        packed, mask, _ = configs.genome()
        n = configs.GENOME_N
        kmers = synth.random_kmers(61, 1000, 12)
        part = coex.Partition(kmers)
        return dict(
            n=n, enc=coex.ENC_2BIT, host=(packed, mask), dfa=None, partition=part, patterns=kmers, chunk=0,
            bytes_per_base=0.375, find=False,
            desc="partitioned: the genome workload's 3.2e9 bases; 1,000 random 12-mers (one automaton would pass "
                 "the 4,096-state device tables) split into %d parts of at most 1,023 states, every part "
                 "scanning the whole sequence; per-pattern counts" % part.n_parts)
    if name == "parity":
        packed, mask, _ = configs.genome()
        n = configs.GENOME_N
        delta = np.array([1, 0, 0, 0, 0, 1, 1, 1], np.uint32)
        table = (delta, 0, np.array([0, 0, 1], np.uint32), np.array([0], np.uint32))
        return dict(
            n=n, enc=coex.ENC_2BIT, host=(packed, mask), dfa=coex.Dfa.table(*table, 1), table=table, patterns=None,
            chunk=0, bytes_per_base=0.375, find=False,
            desc="parity: the genome workload's 3.2e9 bases through the two-state parity automaton "
                 "(odd number of A since the last N), which has no synchronising word: no chunk converges, "
                 "every chunk's candidates run to its end and the join composes every chunk's map")
    if name == "mid":
        seq, rx = configs.mid()
        return dict(n=seq.size, enc=coex.ENC_BYTE, host=(seq, None), dfa=coex.Dfa.regex(rx), patterns=rx, chunk=0,
                    bytes_per_base=1.0, find=True,
                    desc="mid: 256 MiB Markov bytes with 1%% N runs; regex %s (60-state search automaton); "
                         "count and end positions" % rx)
    if name == "small":
        seq, kmers = configs.small()
        return dict(n=seq.size, enc=coex.ENC_BYTE, host=(seq, None), dfa=coex.Dfa.kmers(kmers), patterns=kmers,
                    chunk=configs.SMALL_CHUNK, bytes_per_base=1.0, find=True,
                    desc="small: 1 MiB iid bytes; one random 8-mer (9-state automaton); chunk 64 KiB; "
                         "count and end positions")
    if name == "batched":
        import torch
        lengths, buf, offs, (sets, rxs) = configs.batched()
        dfas = [coex.Dfa.kmers(k) for k in sets] + [coex.Dfa.regex(r) for r in rxs]
        return dict(n=int(sum(lengths)), lengths=lengths, buf=buf, offs=offs, dfas=dfas, sets=sets, rxs=rxs,
                    bytes_per_base=1.0,
                    desc="batched: 512 Markov byte sequences (log-normal lengths, sigma 1.5, clipped to [1e4, 5e7], "
                         "%d bases) x 16 automata (8 random k-mer sets, 8 random regexes); per-pair counts; "
                         "one persistent launch replayed as a HIP graph" % int(sum(lengths)))
    if name == "serving":
        sets, rxs = configs.serving_patterns()
        dfas = [coex.Dfa.kmers(k) for k in sets] + [coex.Dfa.regex(r) for r in rxs]
        return dict(n=0, dfas=dfas, sets=sets, rxs=rxs,
                    desc="serving: Poisson arrivals; sizes log-uniform over [1e3, 1e8] bases (Markov bytes, "
                         "1%% N runs); automaton ids uniform over 32 resident automata (16 random k-mer sets, "
                         "16 random regexes, %d-%d states)" % (min(d.info().n_states for d in dfas),
                                                               max(d.info().n_states for d in dfas)))
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(name: str, w, gpu_counts):
    """The oracle (single thread) over the same input: rate and exactness."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    if name == "genome":
        packed, mask = w["host"]
        seq = oracle.twobit_seq(packed, mask, w["n"])
        counts, pos, pat = oracle.count_kmers(w["patterns"], seq, positions=True)
        w["oracle_positions"] = (pos, pat)
    elif name == "partitioned":
        packed, mask = w["host"]
        counts = oracle.count_kmers(w["patterns"], oracle.twobit_seq(packed, mask, w["n"]))[0]
    elif name == "parity":
        packed, mask = w["host"]
        counts = oracle.scan_table(oracle.make_table(*w["table"], 1), oracle.twobit_seq(packed, mask, w["n"]))[0]
    elif name == "mid":
        counts = np.array([oracle.Regex(w["patterns"]).scan(oracle.byte_seq(w["host"][0]))[0]], dtype=np.uint64)
    else:
        counts = oracle.count_kmers(w["patterns"], oracle.byte_seq(w["host"][0]))[0]
    dt = time.perf_counter() - t0
    exact = [int(x) for x in counts] == [int(x) for x in gpu_counts]
    return dict({"value": round(w["n"] / dt / 1e9, 4), "unit": "Gbases/s", "cores": 1, "kind": "oracle",
                 "sample": "the whole workload (%d bases), one thread, %.1f s" % (w["n"], dt)}, **host_cpu()), exact


def paper_method_series(w, gpu_counts, threads_list):
    """The paper's own method on the host (coex_count_host: equal chunks, one
    per thread, PSS, R0 record, converging point, fix-up, join) over the same
    input, for a series of thread counts: the shape of the paper's
    thread-scaling experiment, on this machine's host CPU."""
    import paper_1509_01506_amd as coex
    data, mask = w["host"]
    rates, exact = [], True
    for t in threads_list:
        t0 = time.perf_counter()
        got = coex.count_host(w["dfa"], data, n=w["n"], encoding=w["enc"], nmask=mask, threads=t)
        dt = time.perf_counter() - t0
        rates.append(round(w["n"] / dt / 1e9, 3))
        exact &= [int(x) for x in got] == [int(x) for x in gpu_counts]
        log("paper method on %d host threads: %.2f s" % (t, dt))
    return dict({"kind": "paper_method", "unit": "Gbases/s", "threads": threads_list, "gbases_per_s": rates,
                 "speedup_vs_1": [round(r / rates[0], 2) for r in rates], "exact": bool(exact),
                 "sample": "the whole workload, chunks = threads"}, **host_cpu())


def bench_batched(args, w):
    """Batched workload: the tuned batch replayed as a HIP graph; the plain
    path over the same pairs for comparison; the oracle on a sample."""
    import numpy as np
    import torch
    import paper_1509_01506_amd as coex
    dbuf = torch.from_numpy(w["buf"]).to("cuda")
    seqs = [coex.DeviceSeq(dbuf[o:o + max(n, 1)], n, coex.ENC_BYTE) for o, n in zip(w["offs"], w["lengths"])]
    dset = coex.DfaSet(w["dfas"])
    out = torch.empty(len(seqs) * len(w["dfas"]), dtype=torch.int64, device="cuda")
    tb = coex.Batch(dset, seqs)
    chunk, width = tb.tune(out=out)
    tb.free()
    b = coex.Batch(dset, seqs, chunk=chunk, width=width, graph=True, timed=True)
    log("tuned chunk %d, width cap %d; %s" % (chunk, width, b.info()))
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < args.clock_warmup_s:
        b.run(out=out)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        b.run(out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    graph_ms = []
    ev0.record(stream)
    for _ in range(args.steps):
        b.run(out=out)
        graph_ms.append(b.info().last_ms)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    got = out.view(len(seqs), len(w["dfas"])).cpu().numpy().view(np.uint64)
    info = b.info()
    # the plain path over the same pairs: one coex_count per (sequence, automaton)
    plain_out = torch.empty(max(d.info().n_patterns for d in w["dfas"]), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    ev0.record(stream)
    plain_ok = True
    for si, s in enumerate(seqs):
        for d, dfa in enumerate(w["dfas"]):
            r = coex.count(dfa, s, out=plain_out)
            if si % 97 == 0 and d == 0:
                plain_ok &= int(r.sum().item()) == int(got[si, d])
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1)
    log("plain path over the same %d pairs: %.1f ms (host wall %.1f ms)"
        % (len(seqs) * len(w["dfas"]), plain_ms, (time.perf_counter() - p0) * 1e3))
    n = w["n"]
    value = n / (ms_step * 1e-3) / 1e9
    groups = info.n_groups
    kern_ms = sorted(graph_ms)[len(graph_ms) // 2]
    # algorithmic bytes of one replay: the byte sequences read once and
    # written as 2-bit codes + N mask (0.375 B/base), which every LDS group
    # of automata then reads once
    algo = n * (1.0 + 0.375) + n * 0.375 * groups
    achieved = algo / (kern_ms * 1e-3) / 1e9
    res = {
        "metric": "Gbases/s scanned (exact counts), batched",
        "value": round(value, 2),
        "unit": "Gbases/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": w["desc"], "bases": n, "pairs": len(seqs) * len(w["dfas"]),
                   "chunk": info.chunk, "width_cap": width, "width": info.width, "lds_groups": groups,
                   "parallelism": "single GPU"},
        "base_automaton_steps_per_s": round(n * len(w["dfas"]) / (ms_step * 1e-3) / 1e12, 3),
        "plain": {"ms": round(plain_ms, 2), "gbases_per_s": round(n / (plain_ms * 1e-3) / 1e9, 2),
                  "speedup_of_batched": round(plain_ms / ms_step, 2), "spot_checks_equal": plain_ok},
        "roofline": {"bound": "hbm", "kernel": "k_bscan (graph)", "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None, "kernel_ms": round(kern_ms, 4),
                     "algorithmic_bytes_per_launch": int(algo),
                     "note": "lookup-bound (16 automata per base read): bytes = one conversion pass "
                             "(1 B read + 0.375 B written per base) + 0.375 B/base per LDS group"},
    }
    if not args.no_cpu_baseline:
        import oracle
        host = host_cpu()
        threads = min(16, host["usable_cpus"])
        lengths, buf, offs = w["lengths"], w["buf"], w["offs"]
        regs = [oracle.Regex(r) for r in w["rxs"]]
        nk = len(w["sets"])
        jobs = sorted(((s, d) for s in range(len(lengths)) for d in range(len(w["dfas"]))),
                      key=lambda sd: -lengths[sd[0]])

        def one(sd):
            s, d = sd
            h = oracle.byte_seq(buf[offs[s]:offs[s] + lengths[s]])
            return int(oracle.count_kmers(w["sets"][d], h)[0].sum()) if d < nk else int(regs[d - nk].scan(h)[0])

        t0 = time.perf_counter()
        vals = oracle.pool_map(one, jobs, threads)
        dt = time.perf_counter() - t0
        exact = all(v == int(got[s, d]) for (s, d), v in zip(jobs, vals))
        res["cpu_baseline"] = dict({"value": round(n / dt / 1e9, 4), "unit": "Gbases/s", "cores": threads,
                                    "kind": "oracle",
                                    "sample": "all %d pairs (%d sequences, %d bases, x %d automata) on a pool of %d "
                                              "threads, each pair one sequential scan, %.1f s"
                                              % (len(jobs), len(lengths), n, len(w["dfas"]), threads, dt)}, **host)
        res["exact"] = bool(exact)
        res["exact_pairs_checked"] = len(jobs)
        log("oracle: all %d pairs in %.1f s on %d threads; exact=%s" % (len(jobs), dt, threads, exact))
    print(json.dumps(res), flush=True)


def bench_serving(args, w):
    """Serving workload: the saturated rate of the serving loop (a burst of
    requests) sets the capacity; two Poisson runs at 0.5 and 0.8 of it give
    p50/p99 latency, submit to result (copy included) and device-only."""
    import threading
    import numpy as np
    import torch
    import paper_1509_01506_amd as coex
    from synth import configs
    pool_np = configs.serving_pool()
    pool = torch.from_numpy(pool_np).pin_memory()
    srv = coex.Server(w["dfas"], hbm_budget=8 << 30, copy_piece=args.copy_piece_mib << 20)

    def run(arrivals, sizes, ids, offs):
        tickets = [None] * len(sizes)
        t0 = time.perf_counter()

        def submitter():
            for i, (a, n, d, o) in enumerate(zip(arrivals, sizes, ids, offs)):
                dt = a - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(pool[o:o + n], d)

        th = threading.Thread(target=submitter)
        th.start()
        res = []
        for i in range(len(sizes)):
            while tickets[i] is None:
                time.sleep(0.0002)
            res.append(srv.wait(tickets[i]))
        th.join()
        wall = time.perf_counter() - t0
        return res, wall

    # capacity: a burst of requests submitted at once
    n_burst = 400
    _, sz, ids, offs = configs.serving_requests(n_burst, 1.0)
    run([0.0] * n_burst, sz, ids, offs)  # warm-up
    res, wall = run([0.0] * n_burst, sz, ids, offs)
    cap_bases = sum(sz) / wall
    mean_size = (1e8 - 1e3) / np.log(1e8 / 1e3)
    cap_qps = cap_bases / mean_size
    log("capacity: %d requests, %.3e bases in %.2f s = %.1f Gbases/s = %.1f requests/s at the mean size"
        % (n_burst, sum(sz), wall, cap_bases / 1e9, cap_qps))
    points = {}
    sample_check = []
    for load in (0.5, 0.8):
        qps = load * cap_qps
        n_req = max(2000, int(qps * 3))
        arr, sz, ids, offs = configs.serving_requests(n_req, qps)
        res, wall = run(arr, sz, ids, offs)
        tot = np.array([r[1]["total_ms"] for r in res])
        dev = np.array([r[1]["device_ms"] for r in res])
        l2d = np.array([r[1]["launch_to_done_ms"] for r in res])
        bs = np.array([r[1]["batch_size"] for r in res])
        points[str(load)] = {
            "qps_offered": round(qps, 1), "requests": n_req, "wall_s": round(wall, 2),
            "gbases_per_s": round(sum(sz) / wall / 1e9, 2),
            "p50_ms": round(float(np.percentile(tot, 50)), 3), "p99_ms": round(float(np.percentile(tot, 99)), 3),
            "device_p50_ms": round(float(np.percentile(dev, 50)), 3),
            "device_p99_ms": round(float(np.percentile(dev, 99)), 3),
            "launch_to_result_p50_ms": round(float(np.percentile(l2d, 50)), 3),
            "mean_batch": round(float(bs.mean()), 2)}
        log("load %.1f: %s" % (load, points[str(load)]))
        if load == 0.8:
            trace8 = (arr, sz, ids, offs)
            sample_check = [(int(o), int(n), int(d), r[0]) for o, n, d, r in zip(offs, sz, ids, res)]
    st = srv.stats()
    srv.close()
    # the plain path on the same 0.8 trace: one request at a time, in arrival
    # order, each a host-to-device copy and one coex_count on one stream
    arr, sz, ids, offs = trace8
    dev_buf = torch.empty(int(max(sz)) + 16, dtype=torch.uint8, device="cuda")
    pout = torch.empty(max(d.info().n_patterns for d in w["dfas"]), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    lat, plain_counts = [], []
    t0 = time.perf_counter()
    for a, n, d, o in zip(arr, sz, ids, offs):
        dt = a - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        dev_buf[:n].copy_(pool[o:o + n], non_blocking=True)
        r = coex.count(w["dfas"][d], coex.DeviceSeq(dev_buf, n, coex.ENC_BYTE), out=pout)
        plain_counts.append(int(r.sum().item()))  # synchronises
        lat.append((time.perf_counter() - t0 - a) * 1e3)
    pwall = time.perf_counter() - t0
    lat = np.array(lat)
    plain = {"requests": len(sz), "wall_s": round(pwall, 2), "gbases_per_s": round(sum(sz) / pwall / 1e9, 2),
             "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
             "same_counts_as_served": plain_counts == [c[3] for c in sample_check]}
    log("plain path on the 0.8 trace: %s" % plain)
    del dev_buf
    p8 = points["0.8"]
    result = {
        "metric": "Gbases/s served and p50/p99 latency (exact counts)",
        "value": p8["gbases_per_s"], "unit": "Gbases/s",
        "n_gpus": 1, "steps": 2, "warmup": 1, "ms_per_step": None,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": w["desc"], "capacity_requests_per_s": round(cap_qps, 1),
                   "capacity_gbases_per_s": round(cap_bases / 1e9, 2), "hbm_budget_bytes": 8 << 30,
                   "parallelism": "single GPU"},
        "latency": points, "server": {"batches": st["n_batches"], "requests": st["n_done"],
                                      "max_arena_bytes": st["max_arena_bytes"]},
        "plain_same_trace_0.8": plain,
    }
    if not args.no_cpu_baseline:
        import oracle
        host = host_cpu()
        threads = min(16, host["usable_cpus"])
        regs = [oracle.Regex(r) for r in w["rxs"]]
        nk = len(w["sets"])
        jobs = sorted(sample_check, key=lambda x: -x[1])

        def one(job):
            o, n, d, _ = job
            h = oracle.byte_seq(pool_np[o:o + n])
            return int(oracle.count_kmers(w["sets"][d], h)[0].sum()) if d < nk else int(regs[d - nk].scan(h)[0])

        t0 = time.perf_counter()
        vals = oracle.pool_map(one, jobs, threads)
        dt = time.perf_counter() - t0
        bases = sum(j[1] for j in jobs)
        exact = all(v == j[3] for v, j in zip(vals, jobs))
        result["cpu_baseline"] = dict({"value": round(bases / dt / 1e9, 4), "unit": "Gbases/s", "cores": threads,
                                       "kind": "oracle",
                                       "sample": "every request of the 0.8 run (%d requests, %d bases) on a pool of "
                                                 "%d threads, each request one sequential scan, %.1f s"
                                                 % (len(jobs), bases, threads, dt)}, **host)
        result["exact"] = bool(exact)
        result["exact_requests_checked"] = len(jobs)
        log("oracle: %d requests in %.1f s on %d threads; exact=%s" % (len(jobs), dt, threads, exact))
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="genome", choices=["genome", "mid", "small", "batched", "serving", "parity", "partitioned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--clock-warmup-s", type=float, default=0.5,
                    help="untimed steps for this many seconds before the warm-up steps (sustained clocks)")
    ap.add_argument("--copy-piece-mib", type=int, default=0,
                    help="serving: bytes per host-to-device copy piece in MiB (0 = the library's default)")
    ap.add_argument("--step", type=int, default=0,
                    help="symbols per table lookup in the chunk scan (0 = the planner's choice; 1, 2 or 3)")
    ap.add_argument("--chunk", type=int, default=0, help="bases per chunk (0 = the workload's or the planner's)")
    ap.add_argument("--chains", type=int, default=0, help="chunks walked per lane at once (0 = the planner's choice)")
    ap.add_argument("--lookback", type=int, default=0, help="bases before a chunk that narrow its starting states (0 = planner)")
    ap.add_argument("--width", type=int, default=0, help="lanes per chunk in the speculation (0 = planner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (scale for rocprofv3 byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library scans one GPU's share of a sequence; sharding over "
              "several GPUs (one exchange of boundary states, one reduction of counts) is not part of it",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 1 << 30, "copy_bytes_written_per_launch": 1 << 30}))
        return

    import paper_1509_01506_amd as coex
    t0 = time.perf_counter()
    w = build_workload(args.workload)
    log("workload generated in %.1f s" % (time.perf_counter() - t0))
    if args.workload == "batched":
        return bench_batched(args, w)
    if args.workload == "serving":
        return bench_serving(args, w)
    data, mask = w["host"]
    seq = coex.to_device(data, n=w["n"], encoding=w["enc"], nmask=mask)
    dfa = w["dfa"]
    part = w.get("partition")
    if part is not None:
        sizes = [part.part(i)[0] for i in range(part.n_parts)]
        info = types.SimpleNamespace(n_states=sum(sizes), n_patterns=part.n_patterns)
    else:
        info = dfa.info()
    torch.cuda.synchronize()
    log("resident in HBM; automaton %d states" % info.n_states)

    out = torch.empty(max(1, info.n_patterns), dtype=torch.int64, device="cuda")

    chunk = args.chunk or w["chunk"]

    def step(timed: bool):
        if part is not None:
            part.count(seq, out=out, chunk=chunk, step=args.step, timed=timed, chains=args.chains)
            return
        if w["find"]:
            # counts and end positions from one scan
            coex.count_find(dfa, seq, out=out, chunk=chunk, step=args.step, timed=timed, chains=args.chains,
                            lookback=args.lookback, width=args.width)
            return
        coex.count(dfa, seq, out=out, chunk=chunk, step=args.step, timed=timed, chains=args.chains,
                   lookback=args.lookback, width=args.width)

    # untimed: bring the GPU to its sustained clocks (about half a second of
    # steps), then the W warm-up steps of the contract
    t_warm = time.perf_counter()
    n_clock = 0
    while time.perf_counter() - t_warm < args.clock_warmup_s:
        for _ in range(20):
            step(False)
        torch.cuda.synchronize()
        n_clock += 20
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    coex.profile(reset=True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step(True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    k_ms, k_n = coex.profile(reset=True)
    k_avg_ms = k_ms / max(1, k_n)
    # the kernels' own consistency checks over every step run so far (read
    # after the timed region)
    device_failures = coex.errors()
    gpu_counts = out[: info.n_patterns].cpu().numpy().view(np.uint64)
    positions = None
    if args.workload == "genome":
        # per-pattern end positions of the whole sequence (coex_find: one pass,
        # one host sync, then a sort of the appended keys), timed on its own
        coex.find(dfa, seq)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            pos, pat = coex.find(dfa, seq)
        torch.cuda.synchronize()
        find_ms = (time.perf_counter() - t1) / 5 * 1e3
        positions = {"ms": round(find_ms, 3), "matches": int(pos.numel()),
                     "gbases_per_s": round(w["n"] / (find_ms * 1e-3) / 1e9, 1)}
        log("find: %.3f ms, %d matches" % (find_ms, pos.numel()))
    value = w["n"] / (ms_step * 1e-3) / 1e9
    log("wall %.3f s for %d steps; events %.3f ms/step; scan kernel %.3f ms avg over %d launches"
        % (wall, args.steps, ms_step, k_avg_ms, k_n))

    algo_bytes = w["n"] * w["bytes_per_base"]
    kernel_name = "k_tail"
    if part is not None:
        # the parts run on the partition's own streams (no per-launch events
        # there): every part reads the whole sequence once per step
        k_avg_ms = ms_step / part.n_parts
        kernel_name = "k_tail (all parts: step time / parts)"
    achieved = algo_bytes / (k_avg_ms * 1e-3) / 1e9
    # symbols per lookup of the chunk scan (the planner's default: three for
    # an automaton of at most 1023 states, else two, else one)
    sym = args.step or (3 if part is not None else (1 if info.n_states > 1024 else (3 if info.n_states <= 1023 else 2)))
    # lookups per base: three symbols per lookup walk 512-base blocks as ten
    # 48-base units (16 lookups) and two words (5 three- + 1 one-symbol lookup)
    per_base = {1: 1.0, 2: 0.5, 3: 172.0 / 512.0}[sym]
    lookups_per_clk = w["n"] * per_base / (k_avg_ms * 1e-3) / (256 * 2.4e9)
    traffic = measured_traffic(args.workload)
    res = {
        "metric": "Gbases/s scanned (exact counts)",
        "value": round(value, 2),
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_warmup_steps": n_clock,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "device_check_failures": device_failures,
        "positions": positions,
        "config": {"workload": w["desc"], "bases": w["n"], "automaton_states": info.n_states,
                   **({"parts": part.n_parts} if part is not None else {}),
                   "patterns": info.n_patterns, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": kernel_name, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel_ms": round(k_avg_ms, 4),
                     "algorithmic_bytes_per_launch": int(algo_bytes),
                     "note": "the walk is bound by dependent random LDS reads: %.1f table lookups per clock "
                             "per CU (%d symbols per lookup, 256 CUs at 2.4 GHz)" % (lookups_per_clk, sym)},
    }
    if not args.no_cpu_baseline:
        cb, exact = cpu_baseline(args.workload, w, gpu_counts)
        res["cpu_baseline"] = cb
        res["exact"] = exact
        if positions is not None and "oracle_positions" in w:
            epos, epat = w["oracle_positions"]
            positions["exact"] = bool(pos.cpu().numpy().tolist() == epos.tolist() and
                                      pat.cpu().numpy().astype(np.uint32).tolist() == epat.tolist())
        log("oracle: %s; exact=%s" % (cb["sample"], exact))
        if args.workload == "genome":
            usable = host_cpu()["usable_cpus"]
            series = [t for t in (1, 2, 4, 8, 16, 32, 64) if t < usable] + [usable]
            res["cpu_paper_method"] = paper_method_series(w, gpu_counts, series)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
