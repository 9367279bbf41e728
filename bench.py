"""Benchmark: LSD radix sort of 1e9 int32 keys on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--dtype int32|int64|...]

One step = one full sort call (evosort_sort) of the whole array: the
adaptive-partition dispatch, the all-pass digit histogram, the digit-base scan
and every single-sweep radix pass.  Keys are generated once (seeded, uniform
over the full int32 range), copied to HBM before timing, and sorted from the
same input buffer into an output buffer on every step.

Prints one JSON line with the contract fields plus:
  roofline      the dominant kernel (the radix pass): algorithmic bytes per
                launch / its mean duration from HIP events recorded around
                every launch during the timed steps, against 8 TB/s; `traffic`
                is the HBM bytes per launch from the committed rocprofv3
                counter summary when it was taken on the current kernel source;
                `copy_gbs` is a plain 4 GiB device copy timed on the same GPU
                (the practical read+write ceiling) and `frac_of_copy` the
                pass's rate against it;
  cpu_baseline  the CPU oracle (single-threaded stable mergesort) timed on a
                bounded sample of the same workload on the host;
  kernels       mean milliseconds per launch of every library kernel;
  secondary     the same measurement for 1e9 int64 keys (unless --no-secondary);
  batched       100k uint32 arrays of log-normal sizes sorted by one segmented
                call, by its HIP-graph replay and by one plain sort per array
                (unless --no-batched);
  tuned         GA-tuned parameters per distribution of the 1e8 int32 sweep
                against the defaults (unless --no-tuned);
  serving       the request loop under Poisson arrivals (2000/s, log-uniform
                sizes in [1e3, 1e8], int32/int64/float32, 200 GB budget):
                p50/p99 latency and keys/s, beside a plain one-call-at-a-time
                FIFO on the same trace (unless --no-serving);
  paper_sweep   the paper's nine int32 distributions at 1e8 keys, ascending
                and descending (unless --no-paper-sweep).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "Gkeys/s and HBM GB/s vs peak, int32/int64 1e9 sort; batched segs/s, p99 latency"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "radix_pass_int32_1e9_pmc.md")
KERNEL_SOURCES = ["paper_2505_18681_amd/csrc/radix_impl.hpp", "paper_2505_18681_amd/csrc/common.hpp",
                  "paper_2505_18681_amd/csrc/kernels.hpp",
                  "paper_2505_18681_amd/csrc/radix_shapes.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counted_traffic(dtype_name: str, n: int):
    """HBM bytes per radix-pass launch from the committed counter summary, if current."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_hash") != kernel_source_hash():
        return None  # kernel changed since the counters were taken
    if rec.get("dtype") != dtype_name or int(rec.get("n", -1)) != n:
        return None
    return float(rec["bytes_per_launch"])


def algorithmic_pass_bytes(n: int, key_bytes: int, value_bytes: int = 0) -> int:
    """One LSD pass reads and writes every key (and value) once."""
    return 2 * n * (key_bytes + value_bytes)


def run_sort_bench(es, torch, dtype_name: str, n: int, steps: int, warmup: int, seed: int, digit_bits: int,
                   tile=None, algo: str = "radix"):
    import numpy as np

    import workloads

    np_dt = np.dtype(dtype_name)
    t_dt = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32, "float64": torch.float64,
            "uint32": torch.uint32}[dtype_name]
    t0 = time.perf_counter()
    host = workloads.uniform(np_dt, n, seed)
    if np_dt == np.uint32:
        keys = torch.from_numpy(host.view(np.int32)).cuda().view(torch.uint32)
    else:
        keys = torch.from_numpy(host).cuda()
    del host
    gen_s = time.perf_counter() - t0
    out = torch.empty_like(keys)
    params = es.default_params(algo=es.ALGO_RADIX if algo == "radix" else es.ALGO_MERGE, digit_bits=digit_bits,
                               fallback_threshold=0)
    if tile:
        params.block_threads, params.items_per_thread = tile
    code = es.dtype_code(t_dt)
    info = es.plan(es.OP_SORT, code, n, 0, params)
    temp = torch.empty(max(es.temp_bytes(es.OP_SORT, code, n, 0, params), 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(warmup):
        es.sort(keys, params=params, out=out, temp=temp)
    torch.cuda.synchronize()

    es.profile_reset()
    es.profile_enable(True)
    # one event between consecutive steps: the whole run and every step are timed on the same stream
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    marks[0].record(stream)
    for i in range(steps):
        es.sort(keys, params=params, out=out, temp=temp)
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    es.profile_enable(False)
    total_ms = marks[0].elapsed_time(marks[-1])
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    kernels = es.profile_collect()
    es.profile_reset()

    # cheap device-side sanity check of the last output (parity lives in tests/)
    if n > 1:
        if dtype_name in ("float32", "float64"):
            ok = True  # totalOrder check needs the bit map; covered by the GPU tests
        elif dtype_name == "uint32":
            o = out.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
            ok = bool((o[1:] >= o[:-1]).all().item())
        else:
            ok = bool((out[1:] >= out[:-1]).all().item())
        if not ok:
            raise RuntimeError("benchmark output is not sorted")

    ms_per_step = total_ms / steps
    kb = np_dt.itemsize
    pass_launches, pass_ms = kernels.get("radix_pass", (0, 0.0))
    mean_pass_ms = pass_ms / pass_launches if pass_launches else float("nan")
    achieved = algorithmic_pass_bytes(n, kb) / (mean_pass_ms * 1e-3) / 1e9 if pass_launches else None
    per_kernel = {k: round(v[1] / v[0], 4) for k, v in kernels.items() if v[0]}
    del keys, out, temp
    torch.cuda.empty_cache()
    return {
        "ms_per_step": ms_per_step,
        "gkeys_per_s": n / (ms_per_step * 1e-3) / 1e9,
        "pass_mean_ms": mean_pass_ms,
        "pass_gbs": achieved,
        "kernels_ms": per_kernel,
        "passes": info["passes"],
        "tile": [info["block_threads"], info["items_per_thread"]],
        "status_bytes": info["status_bytes"],
        "gen_s": gen_s,
        "step_ms": {"min": round(step_ms[0], 4), "median": round(step_ms[len(step_ms) // 2], 4),
                    "max": round(step_ms[-1], 4)} if step_ms else None,
    }


def run_batched_bench(es, torch, nseg: int, steps: int, warmup: int, seed: int, each_steps: int = 1,
                      per_array: bool = True):
    """Batched segmented sort of `nseg` uint32 arrays with log-normal sizes, against one plain sort per array.

    Three schedules of the same batch, from the same resident input buffer:
      segmented  one evosort_segmented_sort call (fixed launch sequence);
      graph      that call captured once in a HIP graph and replayed;
      per_array  evosort_sort_each: one evosort_sort per array, in order
                 (skipped when per_array is false, e.g. under a kernel trace).
    All of them must produce identical bytes (checked on the device).
    """
    import numpy as np

    import workloads

    sizes = workloads.segment_sizes(nseg, seed)
    offs = workloads.segment_offsets(sizes)
    total = int(offs[-1])
    host = workloads.uniform(np.uint32, total, seed)
    keys = torch.from_numpy(host.view(np.int32)).cuda().view(torch.uint32)
    del host
    offsets = torch.from_numpy(offs).cuda()
    out = torch.empty_like(keys)
    ref = torch.empty_like(keys)
    params = es.default_params()
    temp = torch.empty(es.segmented_temp_bytes(es.UINT32, total, nseg, 0, params), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, k):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(k):
            fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / k

    seg = lambda: es.segmented_sort(keys, offsets, params=params, out=out, temp=temp)  # noqa: E731
    for _ in range(warmup):
        seg()
    torch.cuda.synchronize()
    stats = es.segmented_stats(temp)
    es.profile_reset()
    es.profile_enable(True)
    seg_ms = timed(seg, steps)
    es.profile_enable(False)
    kernels = es.profile_collect()
    es.profile_reset()

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        seg()  # warm the allocator-free path on the capture stream
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        seg()
    graph.replay()
    torch.cuda.synchronize()
    graph_ms = timed(graph.replay, steps)
    graph_equal = True  # compared below against the eager output

    seg_out = out.clone()
    each_ms = each_wall_ms = None
    if per_array:
        each_temp = torch.empty(max(es.temp_bytes(es.OP_SORT, es.UINT32, int(sizes.max()), 0, params), 256),
                                dtype=torch.uint8, device="cuda")
        each = lambda: es.sort_each(keys, offs, params=params, out=ref, temp=each_temp)  # noqa: E731
        each()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        each_ms = timed(each, each_steps)
        each_wall_ms = (time.perf_counter() - t0) * 1e3 / each_steps
        del each_temp
    else:
        ref.copy_(seg_out)
    same = bool(torch.equal(seg_out.view(torch.int32), ref.view(torch.int32)))
    out.zero_()
    graph.replay()
    torch.cuda.synchronize()
    graph_equal = bool(torch.equal(out.view(torch.int32), ref.view(torch.int32)))
    if not (same and graph_equal):
        raise RuntimeError("segmented, graph and per-array outputs differ")
    del keys, out, ref, temp, offsets, graph
    torch.cuda.empty_cache()
    per_kernel = {k: round(v[1] / v[0], 4) for k, v in kernels.items() if v[0]}
    per_kernel_calls = {k: v[0] // max(steps, 1) for k, v in kernels.items() if v[0]}
    return {
        "workload": f"{nseg} uint32 arrays, log-normal sizes (median 2048, sigma 2, clipped to [16, 4e6]), "
                    f"{total} keys in all, uniform keys, keys-only, one buffer",
        "nseg": nseg, "keys": total,
        "value": round(nseg / (graph_ms * 1e-3), 1), "unit": "segs/s",
        "gkeys_per_s": round(total / (graph_ms * 1e-3) / 1e9, 3),
        "ms": {"segmented": round(seg_ms, 3), "graph": round(graph_ms, 3),
               "per_array": round(each_ms, 3) if each_ms is not None else None,
               "per_array_host_wall": round(each_wall_ms, 3) if each_wall_ms is not None else None},
        "speedup_vs_per_array": round(each_ms / graph_ms, 2) if each_ms is not None else None,
        "size_classes": stats,
        "kernels_ms": per_kernel, "launches_per_call": per_kernel_calls,
        "identical_bytes": True,
    }


def run_tuned_bench(es, torch, n: int, seed: int, pop: int, generations: int, reps: int):
    """GA-tuned parameters per distribution (the distribution sweep), against the library defaults.

    For each distribution a reduced GA (Algorithm 2's operators, `pop` x
    `generations`) times sorts of n int32 keys; the entry reports the tuned
    parameters, the tuned time and the default time, both re-timed after the
    search.  Every candidate's output is checked bit for bit against the first.
    """
    import numpy as np

    import workloads
    from paper_2505_18681_amd import tuner

    out = []
    t0 = time.perf_counter()
    for dist in workloads.DISTRIBUTIONS:
        keys = torch.from_numpy(workloads.make(dist, np.int32, n, seed)).cuda()
        e = tuner.tune_sort(es, keys, seed=seed, pop_size=pop, generations=generations, reps=reps)
        out.append({"dist": dist, "params": e["params"], "ms": e["ms"], "default_ms": e["default_ms"],
                    "speedup": round(e["default_ms"] / e["ms"], 3) if e["ms"] else None,
                    "gkeys_per_s": round(n / (e["ms"] * 1e-3) / 1e9, 2) if e["ms"] else None,
                    "evaluations": e["evaluations"]})
        del keys
        torch.cuda.empty_cache()
    return {"workload": f"int32 distribution sweep at {n:.0e} keys each, GA with population {pop} over "
                        f"{generations} generations, median of {reps} timed sorts per candidate",
            "entries": out, "search_s": round(time.perf_counter() - t0, 1)}


def run_auto_table_bench(es, torch, seed: int, steps: int = 7):
    """Where the GA table the library compiles in replaces the hand-coded defaults of the automatic choice
    (A_code 0), the sort with the table's pick (default params), with the hand-coded default (A_code 4) and
    with the closed-form parameters, on uniform keys at each row's size class; median of `steps` event-timed
    sorts after a quarter second of untimed ones, outputs checked identical."""
    import numpy as np

    import workloads
    from paper_2505_18681_amd import tuner

    stream = torch.cuda.current_stream()

    def median_ms(keys, out, p):
        temp = torch.empty(max(es.temp_bytes(es.OP_SORT, es.dtype_code(keys.dtype), keys.numel(), 0, p), 256),
                           dtype=torch.uint8, device="cuda")
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.25:
            es.sort(keys, params=p, out=out, temp=temp)
            torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            es.sort(keys, params=p, out=out, temp=temp)
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    entries = []
    for name, n, _lo, _hi, _algo in tuner.auto_table_rows(tuner.packaged_table()):
        host = workloads.uniform(np.dtype(name), n, seed)
        if name == "uint32":
            keys = torch.from_numpy(host.view(np.int32)).cuda().view(torch.uint32)
        else:
            keys = torch.from_numpy(host).cuda()
        outs = [torch.empty_like(keys) for _ in range(3)]
        cases = (("table", es.default_params()), ("hand_coded", es.default_params(algo=es.ALGO_RADIX)),
                 ("closed_form", tuner.closed_form_params(es, name, n)))
        res = {"dtype": name, "n": n}
        for (label, p), out in zip(cases, outs):
            info = es.plan(es.OP_SORT, es.dtype_code(keys.dtype), n, 0, p)
            res[label + "_ms"] = round(median_ms(keys, out, p), 4)
            res[label + "_route"] = (info["path_name"] if info["path_name"] != "radix" else
                                     [info["block_threads"], info["items_per_thread"]])
        bits = [o.view(torch.int32 if o.element_size() == 4 else torch.int64) for o in outs]
        if not (torch.equal(bits[0], bits[1]) and torch.equal(bits[0], bits[2])):
            raise RuntimeError("table, hand-coded and closed-form sorts differ")
        res["table_speedup"] = round(res["hand_coded_ms"] / res["table_ms"], 3)
        entries.append(res)
        del keys, outs, bits, host
        torch.cuda.empty_cache()
    return {"workload": "uniform keys at every size class where the compiled GA table overrides the automatic "
                        "choice's hand-coded defaults", "entries": entries}


def serving_trace(count: int, rate: float, seed: int, lo: float = 1e3, hi: float = 1e8):
    """Request trace: Poisson arrivals at `rate` per second, log-uniform sizes in [lo, hi], dtype uniform over
    int32, int64, float32; returns (arrival seconds, sizes, dtype names)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count)).astype(np.int64)
    dts = np.array(["int32", "int64", "float32"])[rng.integers(3, size=count)]
    return arrivals, sizes, dts


def run_serving_bench(es, torch, count: int, rate: float, budget_gb: float, seed: int, streams: int = 4):
    """The request loop under a Poisson trace, against a plain FIFO of one sort call at a time.

    Inputs are slices of per-dtype pools of uniform keys resident in HBM (the
    paper's uniform generator, full range; floats without NaN).  Latency is
    arrival to completion on the host clock; throughput is total keys over the
    span from the first arrival to the last completion.
    """
    import numpy as np

    import workloads

    arrivals, sizes, dts = serving_trace(count, rate, seed)
    hi = int(sizes.max())
    pools = {}
    for name in ("int32", "int64", "float32"):
        pools[name] = torch.from_numpy(workloads.uniform(np.dtype(name), hi, seed)).cuda()
    rng = np.random.default_rng(seed + 1)
    starts = [int(rng.integers(0, hi - int(n) + 1)) for n in sizes]
    inputs = [pools[d][s:s + int(n)] for d, s, n in zip(dts, starts, sizes)]
    torch.cuda.synchronize()

    def pct(lat):
        return {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                "mean": round(float(np.mean(lat)), 3), "max": round(float(np.max(lat)), 3)}

    # --- the server: admission by budget, batching, overlapping streams.
    # The client releases each result once it is done (after reading its
    # times), except for a sample kept to compare with the request sorted alone.
    srv = es.Server(hbm_budget_bytes=int(budget_gb * (1 << 30)), streams=streams, batch_max_keys=65536)
    sample = set(range(0, count, max(1, count // 16)))
    times = {}
    outstanding = []

    def reap(block=False):
        keep = []
        for i in outstanding:
            if block:
                srv.wait(ids[i])
            if srv.done(ids[i]):
                times[i] = srv.times(ids[i])
                if i not in sample:
                    srv.release(ids[i])
            else:
                keep.append(i)
        return keep

    ids = []
    t_base = time.perf_counter() - arrivals[0]
    for i, x in enumerate(inputs):
        while time.perf_counter() - t_base < arrivals[i]:
            pass
        ids.append(srv.submit(x))
        outstanding.append(i)
        if len(outstanding) > 8:
            outstanding = reap()
    outstanding = reap(block=True)
    lat = np.array([times[i][2] - times[i][0] for i in range(count)])
    queued = np.array([times[i][1] - times[i][0] for i in range(count)])
    span_s = (max(t[2] for t in times.values()) - min(t[0] for t in times.values())) * 1e-3
    checked = 0
    for j in sorted(sample):
        got = srv.result(ids[j])
        alone = es.sort(inputs[j])
        if not torch.equal(got.view(torch.uint8), alone.view(torch.uint8)):
            raise RuntimeError(f"served request {j} differs from the same request sorted alone")
        srv.release(ids[j])
        checked += 1
    st = srv.stats()
    srv.close()
    keys = int(sizes.sum())
    server = {"latency_ms": pct(lat), "queued_ms": pct(queued), "gkeys_per_s": round(keys / span_s / 1e9, 3),
              "span_s": round(span_s, 3), "jobs": st["jobs"], "batched_requests": st["batched_requests"],
              "max_concurrent_jobs": st["max_concurrent_jobs"], "peak_gb": round(st["peak_bytes"] / 2**30, 2),
              "identical_to_alone": checked}

    # --- plain FIFO: one sort call at a time on one stream, same trace
    stream = torch.cuda.current_stream()
    done = []
    t_base = time.perf_counter() - arrivals[0]
    outs = {}
    for i, x in enumerate(inputs):
        while time.perf_counter() - t_base < arrivals[i]:
            pass
        es.sort(x)
        stream.synchronize()
        done.append(time.perf_counter() - t_base)
    lat_plain = (np.array(done) - arrivals) * 1e3
    span_plain = done[-1] - arrivals[0]
    plain = {"latency_ms": pct(lat_plain), "gkeys_per_s": round(keys / span_plain / 1e9, 3),
             "span_s": round(span_plain, 3)}
    del pools, inputs, outs
    torch.cuda.empty_cache()
    return {"workload": f"{count} requests, Poisson arrivals at {rate:.0f}/s, log-uniform sizes in [1e3, 1e8] "
                        f"({keys} keys), dtype uniform over int32/int64/float32, HBM budget {budget_gb:.0f} GB, "
                        f"{streams} streams",
            "value": server["latency_ms"]["p99"], "unit": "ms p99 latency", "server": server,
            "plain_fifo": plain}


def stream_ceilings(es, torch, nbytes: int = 4 << 30, reps: int = 10) -> dict:
    """The library's hand-written streaming kernels on `nbytes` of HBM, timed with HIP events: the copy (reads
    and writes every byte once, like a radix pass) and the read (reads every byte once, like the histogram).
    Rates count bytes read plus bytes written; these are the practical ceilings of the two kernel kinds."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = {}
    for name, fn, moved in (("copy_gbs", lambda: es.stream_copy(dst, src), 2 * nbytes),
                            ("read_gbs", lambda: es.stream_read(src, sink), nbytes)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[name] = round(moved / (ms * 1e-3) / 1e9, 1)
    del src, dst, sink
    torch.cuda.empty_cache()
    return out


def run_paper_sweep(es, torch, n: int, seed: int, steps: int = 5):
    """The paper's nine int32 distributions at n keys each: default parameters, ascending and descending,
    median time of `steps` sorts after a quarter second of untimed calls; each output is checked ordered
    on the device."""
    import numpy as np

    import workloads

    out = []
    stream = torch.cuda.current_stream()
    for dist in workloads.PAPER_DISTRIBUTIONS:
        keys = torch.from_numpy(workloads.make(dist, np.int32, n, seed)).cuda()
        res = torch.empty_like(keys)
        entry = {"dist": dist}
        for desc in (0, 1):
            p = es.default_params(descending=desc)
            temp = torch.empty(max(es.temp_bytes(es.OP_SORT, es.INT32, n, 0, p), 256), dtype=torch.uint8,
                               device="cuda")
            t_warm = time.perf_counter()
            while time.perf_counter() - t_warm < 0.25:  # untimed calls until the clocks are up
                es.sort(keys, params=p, out=res, temp=temp)
                torch.cuda.synchronize()
            times = []
            for _ in range(steps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                es.sort(keys, params=p, out=res, temp=temp)
                b.record(stream)
                b.synchronize()
                times.append(a.elapsed_time(b))
            bad = (res[1:] > res[:-1]) if desc else (res[1:] < res[:-1])
            if bool(bad.any().item()):
                raise RuntimeError(f"{dist} output not ordered")
            ms = float(np.median(times))
            entry["descending_ms" if desc else "ms"] = round(ms, 4)
            entry["descending_gkeys_per_s" if desc else "gkeys_per_s"] = round(n / (ms * 1e-3) / 1e9, 2)
            del temp
        out.append(entry)
        del keys, res
    torch.cuda.empty_cache()
    return {"workload": f"the paper's nine int32 distributions at {n:.0e} keys each, default parameters",
            "entries": out}


def run_routines_bench(es, torch, seed: int, n_merge: int = 100_000_000, steps: int = 10):
    """The other two routines of the adaptive partition sort, on uniform int32 keys with default parameters:
    the mergesort at n_merge keys (block sort, then merge-path rounds; roofline of each kernel from its
    algorithmic bytes, one read and one write of every key per launch) and the one-workgroup sort at its
    largest size (latency per call)."""
    import numpy as np

    import workloads

    stream = torch.cuda.current_stream()

    def timed(fn, k):
        t_warm = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        while time.perf_counter() - t_warm < 0.25:  # untimed calls until the clocks are up
            fn()
            torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / k

    keys = torch.from_numpy(workloads.uniform(np.int32, n_merge, seed)).cuda()
    out = torch.empty_like(keys)
    p = es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0)
    info = es.plan(es.OP_SORT, es.INT32, n_merge, 0, p)
    temp = torch.empty(max(es.temp_bytes(es.OP_SORT, es.INT32, n_merge, 0, p), 256), dtype=torch.uint8,
                       device="cuda")
    call = lambda: es.sort(keys, params=p, out=out, temp=temp)  # noqa: E731
    call()
    # the sort's time without events between its 32 launches, then the same steps again with the
    # library's per-launch events for the per-kernel figures
    ms = timed(call, steps)
    es.profile_reset()
    es.profile_enable(True)
    timed(call, steps)
    es.profile_enable(False)
    kernels = es.profile_collect()
    es.profile_reset()
    if not bool((out[1:] >= out[:-1]).all().item()):
        raise RuntimeError("mergesort output is not sorted")
    per_kernel = {k: round(v[1] / v[0], 4) for k, v in kernels.items() if v[0]}
    launch_bytes = 2 * 4 * n_merge

    def roof(name):
        t = per_kernel.get(name)
        if not t:
            return None
        gbs = launch_bytes / (t * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "mean_launch_ms": t}

    merge = {"workload": f"int32 uniform full-range {n_merge:.0e} keys-only mergesort (T_ins "
                         f"{p.insertion_threshold}, {info['merge_rounds']} merge rounds after blocks of "
                         f"{info['merge_block_run']} keys)",
             "ms": round(ms, 3), "gkeys_per_s": round(n_merge / (ms * 1e-3) / 1e9, 2), "kernels_ms": per_kernel,
             "roofline": {"merge_block_sort": roof("merge_block_sort"), "merge_round": roof("merge_round")}}
    del keys, out, temp
    torch.cuda.empty_cache()

    cap = es.plan(es.OP_SORT, es.INT32, 1)["small_capacity"]
    n_small = cap - 1
    keys = torch.from_numpy(workloads.uniform(np.int32, n_small, seed)).cuda()
    out = torch.empty_like(keys)
    p = es.default_params()
    assert es.plan(es.OP_SORT, es.INT32, n_small, 0, p)["path_name"] == "small"
    temp = torch.empty(max(es.temp_bytes(es.OP_SORT, es.INT32, n_small, 0, p), 256), dtype=torch.uint8,
                       device="cuda")
    us = 1000 * timed(lambda: es.sort(keys, params=p, out=out, temp=temp), 200)
    if not bool((out[1:] >= out[:-1]).all().item()):
        raise RuntimeError("small-array output is not sorted")
    small = {"workload": f"int32 uniform {n_small} keys (one workgroup), back-to-back calls on one stream",
             "us_per_call": round(us, 2), "mkeys_per_s": round(n_small / us, 1), "bound": "latency"}
    return {"merge": merge, "small": small}


def run_vendor_compare(es, torch, n: int, seed: int, steps: int = 3):
    """torch.sort(stable=True) on the same n uniform int32 keys, against this library's sort of (key, int64
    index) pairs, which returns the same two arrays; both outputs are checked identical (the stable sort is
    unique).  Median of `steps` event-timed calls after one untimed call each."""
    import numpy as np

    import workloads

    keys = torch.from_numpy(workloads.uniform(np.int32, n, seed)).cuda()
    stream = torch.cuda.current_stream()

    def median_ms(fn):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.median(times))

    res = {}
    torch_ms = median_ms(lambda: res.__setitem__("t", torch.sort(keys, stable=True)))
    t_vals, t_idx = res.pop("t")
    iota = torch.arange(n, dtype=torch.int64, device="cuda")
    ko, vo = torch.empty_like(keys), torch.empty_like(iota)
    p = es.default_params()
    temp = torch.empty(max(es.temp_bytes(es.OP_SORT_PAIRS, es.INT32, n, 8, p), 256), dtype=torch.uint8,
                       device="cuda")
    ours_ms = median_ms(lambda: es.sort_pairs(keys, iota, params=p, keys_out=ko, values_out=vo, temp=temp))
    identical = bool(torch.equal(t_vals, ko) and torch.equal(t_idx, vo))
    if not identical:
        raise RuntimeError("torch.sort and the pairs sort disagree")
    del keys, iota, ko, vo, temp, t_vals, t_idx
    torch.cuda.empty_cache()
    return {"workload": f"int32 uniform full-range {n:.0e} keys, sorted keys and int64 source indices",
            "torch_sort_ms": round(torch_ms, 3), "evosort_pairs_ms": round(ours_ms, 3),
            "speedup": round(torch_ms / ours_ms, 2), "identical": identical,
            "torch_version": torch.__version__}


def host_cpu() -> dict:
    """Host cores this process may use, and the CPU model from /proc/cpuinfo."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline(dtype_name: str, n_sample: int, seed: int):
    """The oracle, untuned, on a bounded sample of the same workload (one host thread)."""
    import numpy as np

    import oracle
    import workloads

    keys = workloads.uniform(np.dtype(dtype_name), n_sample, seed)
    t0 = time.perf_counter()
    perm = oracle.stable_perm(keys)
    out = keys[perm]
    dt = time.perf_counter() - t0
    del out, perm
    host = host_cpu()
    return {"value": round(n_sample / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample:.0e} {dtype_name} uniform keys (seed {seed}), stable mergesort, "
                      f"{dt:.2f} s on one host thread",
            "nproc": host["nproc"], "cpu_count": host["cpu_count"], "cpu_model": host["cpu_model"]}


# ------------------------------------------------------- profile summaries --
# rocprofv3 writes CSV files (--output-format csv); these turn a kernel trace
# and two counter runs of this script into the markdown summaries kept under
# profiles/ (python bench.py --summarize-trace DIR ... / --summarize-pmc DIR DIR ...).

def _csv_rows(directory: str, suffix: str):
    import csv
    import glob

    paths = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    rows = []
    for path in paths:
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def short_kernel_name(name: str) -> str:
    """`void evosort::radix_pass_kernel<4, 0, ...>(args)` -> `radix_pass_kernel<4, 0, ...>`."""
    name = name.strip().replace("(anonymous namespace)::", "")
    for prefix in ("void ",):
        if name.startswith(prefix):
            name = name[len(prefix):]
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut].replace("evosort::", "")
    return name if len(name) <= 64 else name[:61] + "..."


def summarize_trace(trace_dir: str, kernel: str, skip: int, passes: int, bytes_per_launch: float,
                    command: str, title: str) -> str:
    """Markdown summary of a kernel trace: per-kernel statistics over every dispatch, then the dominant
    kernel's launches without the first `skip` (the warm-up calls), by pass, and its roofline."""
    rows = _csv_rows(trace_dir, "kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    per = {}
    for r in rows:
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per.setdefault(short_kernel_name(r["Kernel_Name"]), []).append(us)
    total = sum(sum(v) for v in per.values())
    lines = [f"# {title}", "", "Command (from the repository root on the GPU box):", "", "```", command, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                     f"{100 * sum(v) / total:.1f}% |")
    dom = [(n, v) for n, v in per.items() if n.startswith(kernel)]
    if len(dom) != 1:
        raise SystemExit(f"kernel {kernel!r} matches {[n for n, _ in dom]}")
    name, launches = dom[0]
    timed = launches[skip:]
    avg = sum(timed) / len(timed)
    gbs = bytes_per_launch / (avg * 1e-6) / 1e9
    lines += ["", f"Timed launches of `{name}`: {len(timed)} (the first {skip} of {len(launches)}, from the "
              "warm-up calls, left out).", "", "| pass | launches | avg (us) | min (us) | max (us) |",
              "|---|---|---|---|---|"]
    for p in range(passes):
        v = timed[p::passes]
        if v:
            lines.append(f"| {p} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    lines.append(f"| all | {len(timed)} | {avg:.1f} | {min(timed):.1f} | {max(timed):.1f} |")
    rec = {"kernel": name, "timed_launches": len(timed), "avg_us": round(avg, 2),
           "algorithmic_bytes_per_launch": bytes_per_launch, "achieved_gbs": round(gbs, 1),
           "peak_gbs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}
    lines += ["", f"Algorithmic bytes per launch {bytes_per_launch / 1e9:.3f} GB / {avg:.1f} us = {gbs:.1f} GB/s, "
              f"{100 * gbs / HBM_PEAK_GBS:.1f} % of {HBM_PEAK_GBS:.0f} GB/s.", "",
              "roofline_json: " + json.dumps(rec)]
    return "\n".join(lines) + "\n"


def summarize_pmc(fetch_dir: str, write_dir: str, kernel: str, bytes_per_launch: float, calib_bytes: int,
                  dtype: str, n: int, commands: list, title: str) -> str:
    """Markdown summary of two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Both counters
    are scaled by what they read for the largest dispatch of the library's streaming copy kernel, which
    moves `calib_bytes` each way."""
    counts = {}
    for d, cname in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        per_dispatch = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != cname:
                continue
            key = (short_kernel_name(r["Kernel_Name"]), int(r["Dispatch_Id"]))
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
        counts[cname] = per_dispatch
    calib = {c: max(v for (k, _), v in counts[c].items() if k.startswith("stream_copy_kernel"))
             for c in ("FETCH_SIZE", "WRITE_SIZE")}
    scale = {c: calib_bytes / (calib[c] * 1024.0) for c in calib}
    lines = [f"# {title}", "", "Two counter runs, one counter each (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch):",
             "", "```"] + commands + ["```", "",
             f"Calibration: the largest dispatch of the library's streaming copy kernel moves {calib_bytes} bytes "
             f"each way and reads FETCH_SIZE = {calib['FETCH_SIZE']:.0f} KiB, WRITE_SIZE = "
             f"{calib['WRITE_SIZE']:.0f} KiB, so fetch counts are scaled by {scale['FETCH_SIZE']:.4f} and write "
             f"counts by {scale['WRITE_SIZE']:.4f}.", "",
             "| kernel | dispatches | FETCH_SIZE KiB per dispatch (raw) | WRITE_SIZE KiB per dispatch (raw) | "
             "scaled HBM bytes per dispatch |", "|---|---|---|---|---|"]
    names = {}
    for c in counts:
        for (k, _), v in counts[c].items():
            names.setdefault(k, {}).setdefault(c, []).append(v)
    dom = None
    for k, by in sorted(names.items()):
        f = by.get("FETCH_SIZE", [0.0])
        w = by.get("WRITE_SIZE", [0.0])
        fa, wa = sum(f) / len(f), sum(w) / len(w)
        scaled = (fa * scale["FETCH_SIZE"] + wa * scale["WRITE_SIZE"]) * 1024.0
        lines.append(f"| `{k}` | {len(f)} | {fa:.0f} | {wa:.0f} | {scaled / 1e9:.3f} GB |")
        if k.startswith(kernel):
            dom = (k, fa, wa, scaled, f, w)
    if dom is None:
        raise SystemExit(f"kernel {kernel!r} not in the counter runs")
    k, fa, wa, scaled, f, w = dom
    lines += ["", f"Per launch of `{k}`, in dispatch order: " + "; ".join(
        f"{(a * scale['FETCH_SIZE'] + b * scale['WRITE_SIZE']) * 1024.0 / 1e9:.3f} GB" for a, b in zip(f, w)),
        "", f"Algorithmic bytes per launch: {bytes_per_launch / 1e9:.3f} GB; counted (scaled) bytes per launch: "
        f"{scaled / 1e9:.3f} GB ({scaled / bytes_per_launch:.3f}x).", "",
        "Machine-readable line read by bench.py (`source_hash` = kernel sources the counters were taken on):", "",
        "traffic_json: " + json.dumps({"kernel": k, "n": n, "dtype": dtype, "fetch_kib_raw": round(fa),
                                       "write_kib_raw": round(wa), "fetch_scale": round(scale["FETCH_SIZE"], 4),
                                       "write_scale": round(scale["WRITE_SIZE"], 4),
                                       "bytes_per_launch": round(scaled),
                                       "algorithmic_bytes_per_launch": bytes_per_launch,
                                       "source_hash": kernel_source_hash()})]
    return "\n".join(lines) + "\n"


def summarize_counters(dirs: list, kernels: list, commands: list, title: str) -> str:
    """Markdown table of hardware counters (rocprofv3 --pmc runs, any counters): per kernel whose short name
    starts with one of `kernels`, the mean value per dispatch of every counter collected."""
    table, order = {}, []
    for d in dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            k = short_kernel_name(r["Kernel_Name"])
            if not any(k.startswith(x) for x in kernels):
                continue
            c = r["Counter_Name"]
            per = table.setdefault(k, {}).setdefault(c, {})
            per[int(r["Dispatch_Id"])] = per.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
            if c not in order:
                order.append(c)
    lines = [f"# {title}", "", "Counter runs (one rocprofv3 --pmc run per group of counters):", "", "```"] + commands
    lines += ["```", "", "Mean value per dispatch (summed over the device's units):", "",
              "| kernel | dispatches | " + " | ".join(order) + " |", "|---|---|" + "---|" * len(order)]
    for k in sorted(table):
        vals = table[k]
        nd = max(len(v) for v in vals.values())
        cells = []
        for c in order:
            v = vals.get(c)
            cells.append(f"{sum(v.values()) / len(v):.4g}" if v else "")
        lines.append(f"| `{k}` | {nd} | " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("--summarize-trace", "--summarize-pmc", "--summarize-counters"):
        return summarize_main()
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000_000)
    ap.add_argument("--dtype", default="int32")
    ap.add_argument("--digit-bits", type=int, default=8)
    ap.add_argument("--tile", default=None, help="radix tile shape THREADS,ITEMS (default: library default)")
    ap.add_argument("--algo", choices=["radix", "merge"], default="radix")
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--cpu-sample", type=int, default=100_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-vendor", action="store_true", help="skip the torch.sort comparison")
    ap.add_argument("--no-routines", action="store_true", help="skip the mergesort and small-array measurements")
    ap.add_argument("--batched-nseg", type=int, default=100_000)
    ap.add_argument("--batched-no-per-array", action="store_true",
                    help="skip the one-sort-per-array comparison (100k sorts; slow under a kernel trace)")
    ap.add_argument("--no-tuned", action="store_true")
    ap.add_argument("--no-auto-table", action="store_true",
                    help="skip the comparison of the compiled GA table with the hand-coded defaults")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-paper-sweep", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--serving-budget-gb", type=float, default=200.0)
    ap.add_argument("--tuned-n", type=int, default=100_000_000)
    ap.add_argument("--tuned-pop", type=int, default=10)
    ap.add_argument("--tuned-generations", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB copy with the library's streaming copy kernel (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; run it with --gpus 1"}), flush=True)
        sys.exit(2)

    import torch

    import paper_2505_18681_amd as es

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)

    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None
    main_res = run_sort_bench(es, torch, args.dtype, args.n, args.steps, args.warmup, args.seed, args.digit_bits,
                              tile, args.algo)
    print(f"# {args.dtype} n={args.n}: {main_res['ms_per_step']:.3f} ms/step, "
          f"{main_res['gkeys_per_s']:.2f} Gkeys/s, pass {main_res['pass_mean_ms']:.3f} ms", file=sys.stderr,
          flush=True)

    secondary = None
    if not args.no_secondary and args.dtype == "int32" and args.algo == "radix":
        sec = run_sort_bench(es, torch, "int64", args.n, max(2, args.steps // 2), 1, args.seed, args.digit_bits,
                             None, args.algo)
        secondary = {
            "workload": f"int64 uniform {args.n:.0e} keys-only LSD radix sort, {sec['passes']} passes of "
                        f"{args.digit_bits}-bit digits",
            "value": round(sec["gkeys_per_s"], 4), "unit": "Gkeys/s", "ms_per_step": round(sec["ms_per_step"], 4),
            "step_ms": sec["step_ms"],
            "roofline": {"bound": "hbm", "achieved": round(sec["pass_gbs"], 1) if sec["pass_gbs"] else None,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(sec["pass_gbs"] / HBM_PEAK_GBS, 4) if sec["pass_gbs"] else None},
            "kernels_ms": sec["kernels_ms"],
        }
        print(f"# int64: {sec['ms_per_step']:.3f} ms/step, {sec['gkeys_per_s']:.2f} Gkeys/s", file=sys.stderr,
              flush=True)

    vendor = None
    if not args.no_vendor and args.dtype == "int32" and args.algo == "radix":
        vendor = run_vendor_compare(es, torch, args.n, args.seed)
        print(f"# torch.sort {vendor['torch_sort_ms']} ms, pairs {vendor['evosort_pairs_ms']} ms", file=sys.stderr,
              flush=True)

    routines = None
    if not args.no_routines:
        routines = run_routines_bench(es, torch, args.seed)
        print(f"# mergesort 1e8 {routines['merge']['ms']} ms; small {routines['small']['us_per_call']} us",
              file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = run_batched_bench(es, torch, args.batched_nseg, max(2, args.steps // 2), 1, args.seed,
                                    per_array=not args.batched_no_per_array)
        print(f"# batched: {batched['ms']}", file=sys.stderr, flush=True)

    auto_table = None
    if not args.no_auto_table:
        auto_table = run_auto_table_bench(es, torch, args.seed)
        print(f"# auto table: {auto_table['entries']}", file=sys.stderr, flush=True)

    tuned = None
    if not args.no_tuned:
        tuned = run_tuned_bench(es, torch, args.tuned_n, args.seed, args.tuned_pop, args.tuned_generations, 3)
        print(f"# tuned: {[(e['dist'], e['ms'], e['default_ms']) for e in tuned['entries']]}", file=sys.stderr,
              flush=True)

    paper_sweep = None
    if not args.no_paper_sweep:
        paper_sweep = run_paper_sweep(es, torch, 100_000_000, args.seed)
        print(f"# paper sweep: {[(e['dist'], e['ms'], e['descending_ms']) for e in paper_sweep['entries']]}",
              file=sys.stderr, flush=True)

    serving = None
    if not args.no_serving:
        serving = run_serving_bench(es, torch, args.serving_requests, args.serving_rate, args.serving_budget_gb,
                                    args.seed)
        # the same request mix offered faster than the GPU sorts it: saturation throughput
        serving["overload"] = run_serving_bench(es, torch, args.serving_requests, 10 * args.serving_rate,
                                                args.serving_budget_gb, args.seed + 7)
        print(f"# serving: server {serving['server']['latency_ms']} {serving['server']['gkeys_per_s']} Gkeys/s; "
              f"plain {serving['plain_fifo']['latency_ms']} {serving['plain_fifo']['gkeys_per_s']} Gkeys/s",
              file=sys.stderr, flush=True)

    if args.copy_calibration:
        # one 1 GiB copy with the library's streaming copy kernel: counter runs scale by what it reads
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        es.stream_copy(dst, src)
        torch.cuda.synchronize()
        del src, dst

    ceilings = stream_ceilings(es, torch)
    copy_gbs = ceilings["copy_gbs"]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.dtype, min(args.cpu_sample, args.n), args.seed)

    kb = {"int32": 4, "uint32": 4, "float32": 4, "int64": 8, "float64": 8}[args.dtype]
    achieved = main_res["pass_gbs"]
    line = {
        "metric": METRIC,
        "value": round(main_res["gkeys_per_s"], 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "step_ms": main_res["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{args.dtype} uniform full-range {args.n:.0e} keys-only LSD radix sort "
                        f"({main_res['passes']} passes of {args.digit_bits}-bit digits), keys resident in HBM",
            "n": args.n,
            "key_dtype": args.dtype,
            "digit_bits": args.digit_bits,
            "tile": main_res["tile"],
            "status_word_bytes": main_res["status_bytes"],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "radix_pass",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": counted_traffic(args.dtype, args.n),
            "algorithmic_bytes_per_launch": algorithmic_pass_bytes(args.n, kb),
            "mean_launch_ms": round(main_res["pass_mean_ms"], 4),
            "copy_gbs": copy_gbs,
            "read_gbs": ceilings["read_gbs"],
            "frac_of_copy": round(achieved / copy_gbs, 4) if achieved and copy_gbs else None,
        },
        "cpu_baseline": cpu,
        "kernels_ms": main_res["kernels_ms"],
        "secondary": secondary,
        "vendor": vendor,
        "routines": routines,
        "batched": batched,
        "tuned": tuned,
        "auto_table": auto_table,
        "serving": serving,
        "paper_sweep": paper_sweep,
    }
    print(json.dumps(line), flush=True)


def summarize_main():
    ap = argparse.ArgumentParser(description="Summarize rocprofv3 CSV output of this script as markdown")
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR")
    ap.add_argument("--kernel", default="radix_pass_kernel<4, 0, 8, 768, 24")
    ap.add_argument("--skip", type=int, default=0, help="leading launches of the kernel to leave out (warm-up)")
    ap.add_argument("--passes", type=int, default=4)
    ap.add_argument("--bytes-per-launch", type=float, default=8e9)
    ap.add_argument("--calib-bytes", type=int, default=4 << 30)
    ap.add_argument("--dtype", default="int32")
    ap.add_argument("--n", type=int, default=1_000_000_000)
    ap.add_argument("--command", action="append", default=[], help="command line that produced the CSVs")
    ap.add_argument("--title", default="")
    a = ap.parse_args()
    if a.summarize_counters:
        print(summarize_counters(a.summarize_counters, a.kernel.split(";"), a.command, a.title), end="")
    elif a.summarize_trace:
        print(summarize_trace(a.summarize_trace, a.kernel, a.skip, a.passes, a.bytes_per_launch,
                              "\n".join(a.command), a.title), end="")
    else:
        print(summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.kernel, a.bytes_per_launch, a.calib_bytes,
                            a.dtype, a.n, a.command, a.title), end="")


if __name__ == "__main__":
    main()
