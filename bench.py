"""Benchmark of the IPLS sort on one MI355X.

A step is one complete sort (every distribution level, the sample sorts, fits, and the base case)
of 1e8 fp64 keys, keys only, 256 buckets, base case at <= 4096 keys, FMCD fit on a 1% sample
capped at 4096 keys per bucket (the paper's IPLS samples alpha k - 1, about 1330 keys, at this
size; the cap keeps every sample inside one base-case sort).
Steps cycle through the five distributions of this workload: normal(0,1), lognormal(0,0.5),
exponential(2), an equal-weight mixture of 5 N(mu_i, 1) with mu_i ~ U[-100,100], and integers
uniform in [0, 1e6) cast to fp64.  Inputs are synthetic (seeded), generated on the host and staged
in HBM before the timed region: every step sorts its own pre-staged copy, so no copy is timed.

Prints one JSON line (see the keys below).  The roofline object reports the dominant kernel, the
scatter of the distribution pass, from HIP events recorded around its launches on the sort's
stream during the timed steps; its algorithmic bytes are 2 (w + w_p) per key it moves.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sorted keys/s + HBM GB/s (% peak) per pass, 1e8 fp64; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0
DISTS = ("normal", "lognormal", "exponential", "mixgauss", "uniform_int")
SEEDS = {"normal": 2, "lognormal": 3, "exponential": 4, "mixgauss": 5, "uniform_int": 6}
# the scatter and the helpers it uses (the base case lives in ipls_base.h and does not count)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2208_06902_amd", "csrc", f) for f in ("ipls_kernels.h", "ipls_device.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scatter_traffic.json")
PROFILE_LEVELS = 16  # IPLS_PROFILE_LEVELS
BUCKET_POLICY_LABEL = "256, fewer for a bucket below 32T keys: the smallest power of two >= 8n/T, at least 64"


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per scatter launch from committed rocprofv3 counter runs, if they match this kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def summarize_profiles(ktrace_dir: str, fetch_dir: str, write_dir: str, bench_json: str, out_dir: str) -> None:
    """Write the committed profile summaries from rocprofv3 CSV output of this bench.

    ktrace_dir: `rocprofv3 --kernel-trace --stats -f csv` run of the bench; fetch_dir / write_dir:
    `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs.  The counters are calibrated on the
    bench's own device-to-device copies of one 1e8 fp64 input (800,000,000 bytes each way)."""
    import csv
    import glob
    import re

    def one(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        if not f:
            raise FileNotFoundError(f"{pat} under {d}")
        return f[0]

    def short(name):
        return re.sub(r"\(.*", "", name).replace("void ", "")

    stats = list(csv.DictReader(open(one(ktrace_dir, "*kernel_stats.csv"))))
    bench = json.load(open(bench_json))
    lines = ["# Kernel time of the 1e8 fp64 sort bench (rocprofv3 --kernel-trace --stats)", "",
             "Command (from the repository root, GPU box):", "",
             "    rocprofv3 --kernel-trace --stats -f csv -d <dir> -o bench -- \\",
             "        python3 -u bench.py --steps 5 --warmup 5 --no-cpu-baseline --no-extras", "",
             f"Bench line of the same run: {bench['value']:.4g} keys/s, {bench['ms_per_step']} ms per step; "
             f"k_scatter average launch by HIP events in bench.py: {bench['roofline']['avg_launch_ms']} ms over "
             f"{bench['roofline']['launches']} timed launches.", "",
             "15 sorts (5 warmup, 5 timed, then the timed steps again, untimed, for the counting and base-case "
             "timings; all five distributions).  `__amd_rocclr_copyBuffer` is the bench's "
             "own staging of inputs, outside the timed steps.", "",
             "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in stats[:28]:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    sc = [r for r in stats if "k_scatter" in r["Name"]]
    if sc:
        lines += ["", f"k_scatter average by rocprofv3: {float(sc[0]['AverageNs']) / 1e6:.4f} ms "
                      f"(bench.py HIP events: {bench['roofline']['avg_launch_ms']} ms)."]
    open(os.path.join(out_dir, "sort_1e8_fp64_kernel_stats.md"), "w").write("\n".join(lines) + "\n")

    def counters(d):
        rows = list(csv.DictReader(open(one(d, "*counter_collection.csv"))))
        return [(short(r["Kernel_Name"]), int(r["Grid_Size"]) // int(r["Workgroup_Size"]),
                 float(r["Counter_Value"]) * 1024.0) for r in rows]

    fetch, write = counters(fetch_dir), counters(write_dir)
    copy_bytes = 8.0 * 100_000_000
    cf = [b for k, g, b in fetch if "copyBuffer" in k and b > 0.25 * copy_bytes]
    cw = [b for k, g, b in write if "copyBuffer" in k and b > 0.5 * copy_bytes]
    f_scale = copy_bytes / (sum(cf) / len(cf))
    w_scale = copy_bytes / (sum(cw) / len(cw))
    sf = [b * f_scale for k, g, b in fetch if "k_scatter" in k]
    sw = [b * w_scale for k, g, b in write if "k_scatter" in k]
    n_launch = min(len(sf), len(sw))
    per_launch = (sum(sf[:n_launch]) + sum(sw[:n_launch])) / n_launch
    big = [(f, w) for f, w in zip(sf, sw) if f > 1e8]
    t = {"kernel": "k_scatter", "kernel_sha": kernel_hash(), "bytes_per_launch": round(per_launch),
         "launches": n_launch, "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
         "workload": "bench.py --steps 5 --warmup 5 --no-cpu-baseline --no-extras (15 sorts of 1e8 fp64, all five distributions)",
         "large_launches_bytes": [[round(f), round(w)] for f, w in big[:6]],
         "algorithmic_bytes_large_launch": 1_600_000_000}
    json.dump(t, open(os.path.join(out_dir, "scatter_traffic.json"), "w"), indent=1)
    md = ["# HBM traffic of k_scatter (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, separate runs)", "",
          "Commands (from the repository root, GPU box), one counter per run:", "",
          "    rocprofv3 --pmc FETCH_SIZE -f csv -d <dir> -o bench -- \\",
          "        python3 -u bench.py --steps 5 --warmup 5 --no-cpu-baseline --no-extras",
          "    rocprofv3 --pmc WRITE_SIZE -f csv -d <dir> -o bench -- \\",
          "        python3 -u bench.py --steps 5 --warmup 5 --no-cpu-baseline --no-extras", "",
          "The same command as the kernel trace: 15 sorts, three of each of the five distributions, the launch "
          "mix of the bench's timed steps.", "",
          f"Calibration: the bench's device-to-device copies of one 800,000,000-byte input read as "
          f"FETCH_SIZE x {f_scale:.3f} and WRITE_SIZE x {w_scale:.3f}; every k_scatter value below is scaled "
          f"by those factors.", "",
          "| scatter launch (level) | fetch MB | write MB | algorithmic MB (read + write) |",
          "|---|---:|---:|---:|"]
    for i, (f, w) in enumerate(big[:6]):
        md.append(f"| {i} | {f / 1e6:.1f} | {w / 1e6:.1f} | 1600.0 |")
    alg = bench["roofline"].get("algorithmic_bytes_per_launch")
    md += ["", f"Mean over all {n_launch} scatter launches of the run: {per_launch / 1e6:.1f} MB per launch "
               f"(bench.py reports it as roofline.traffic while the kernel source is unchanged, sha {t['kernel_sha']})."]
    if alg:
        md += ["", f"Algorithmic bytes per launch of the kernel-trace run (same command): {alg / 1e6:.1f} MB; "
                   f"measured / algorithmic = {per_launch / alg:.3f}."]
    open(os.path.join(out_dir, "scatter_traffic.md"), "w").write("\n".join(md) + "\n")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _line(value, ms_per_step, steps, warmup, dtype, config, **extra):
    line = {"metric": METRIC, "value": round(value, 1), "unit": "keys/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
            "roofline": None, "cpu_baseline": None}
    line.update(extra)
    return line


def _ord_i64(t, dtype_code, torch):
    """A monotone int64 image of keys: IEEE totalOrder for fp64 (0) and fp32 (1), unsigned order for
    uint64 (2).  One to one, so equal images mean equal bits."""
    if dtype_code == 1:
        s = t.view(torch.int32)
        return torch.bitwise_xor(s, torch.bitwise_and(s >> 31, 0x7FFFFFFF)).to(torch.int64)
    s = t.view(torch.int64)
    if dtype_code == 2:
        return torch.bitwise_xor(s, torch.tensor(-(2**63), dtype=torch.int64, device=t.device))
    return torch.bitwise_xor(s, torch.bitwise_and(s >> 63, 0x7FFFFFFFFFFFFFFF))


def _sorted_equal(out, inp, dtype_code, torch):
    """Exact check of one keys-only sort: out equals the input's keys in ascending order (the
    sorted sequence of a multiset is unique), compared through the ord image with torch's sort."""
    want = torch.sort(_ord_i64(inp, dtype_code, torch)).values
    return bool(torch.equal(want, _ord_i64(out, dtype_code, torch)))


def _segments_sorted_equal(out, inp, sizes_t, torch):
    """Exact check of a keys-only segmented fp64 sort over every segment: the input's keys sorted
    by (segment, ord) with two stable sorts equal the output."""
    nseg = sizes_t.numel()
    seg = torch.repeat_interleave(torch.arange(nseg, device=inp.device), sizes_t)
    v1, i1 = torch.sort(_ord_i64(inp, 0, torch), stable=True)
    s1 = seg[i1]
    del seg, i1
    _, i2 = torch.sort(s1, stable=True)
    del s1
    want = v1[i2]
    del v1, i2
    ok = bool(torch.equal(want, _ord_i64(out, 0, torch)))
    del want
    torch.cuda.empty_cache()
    return ok


def _u64_sorted(t, torch):
    flip = torch.tensor(-(2**63), dtype=torch.int64, device=t.device)
    v = torch.bitwise_xor(t.view(torch.int64), flip)
    return bool((v[1:] >= v[:-1]).all())


def bench_large_u64(args):
    """Single-array sorts of uint64 keys drawn on the device: 1e9 uniform keys, keys only, or 2e8
    Zipf(1.1) ranks over [1, 2^32] with their uint32 index as payload (stable).  Each step sorts a
    fresh copy of the input (staged before the step); the output of the last step is checked to be
    non-decreasing, and a permutation of the input (against a device sort), with the payload
    pointing at equal keys."""
    import numpy as np
    import torch

    import gen.device as gdev
    import paper_2208_06902_amd as ipls

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    zipf = args.workload == "zipf"
    n = 200_000_000 if zipf else 1_000_000_000
    print(f"# {args.workload}: drawing {n} keys on the device", file=sys.stderr, flush=True)
    src = gdev.zipf_u64(n, 8) if zipf else gdev.u64_uniform(n, 7)
    work = torch.empty_like(src)
    pay0 = torch.arange(n, dtype=torch.int32, device=dev) if zipf else None
    pay = torch.empty_like(pay0) if zipf else None
    params = ipls.default_params(sample_max=args.sample_max, equality=args.equality, inherit=args.inherit)
    stream = torch.cuda.current_stream()
    ipls.profile_enable(1 << ipls.KERNEL_SCATTER)
    ms, stats = [], None
    for step in range(args.warmup + args.steps):
        work.copy_(src)
        if zipf:
            pay.copy_(pay0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if step == args.warmup:
            ipls.profile_enable(1 << ipls.KERNEL_SCATTER)
        a.record(stream)
        stats = ipls.sort_(work.view(torch.uint64), pay, params, stats=True)
        b.record(stream)
        torch.cuda.synchronize()
        if step >= args.warmup:
            ms.append(a.elapsed_time(b))
    sc_n, sc_ms, sc_bytes = ipls.profile_read(ipls.KERNEL_SCATTER)
    ipls.profile_enable(False)
    flip = torch.tensor(-(2**63), dtype=torch.int64, device=dev)
    got = torch.bitwise_xor(work, flip)
    ok = bool((got[1:] >= got[:-1]).all())
    ref = torch.sort(torch.bitwise_xor(src, flip)).values
    ok = ok and torch.equal(ref, got)
    del ref
    if zipf:
        ok = ok and torch.equal(src[pay.long()], work)
    mean_ms = sum(ms) / len(ms)
    sc_gbs = sc_bytes / (sc_ms / 1e3) / 1e9 if sc_ms > 0 else None
    desc = ("plain key+payload sort, 200000000 uint64 Zipf(1.1) ranks over [1, 2^32] with a uint32 index payload, stable"
            if zipf else "plain single-array sort, 1000000000 uniform uint64 keys, keys only")
    line = _line(n / (mean_ms / 1e3), mean_ms, args.steps, args.warmup, "u64",
                 {"workload": desc, "n": n, "num_buckets": 256, "base_case_max": 4096,
                  "bucket_policy": BUCKET_POLICY_LABEL if not args.equality else "256 everywhere",
                  "sample": sample_label(args), "model": "FMCD",
                  "equality_buckets": bool(args.equality), "parallelism": "single GPU"},
                 roofline={"kernel": "k_scatter", "bound": "hbm",
                           "achieved": round(sc_gbs, 1) if sc_gbs else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(sc_gbs / HBM_PEAK_GBS, 4) if sc_gbs else None, "traffic": None,
                           "launches": sc_n},
                 stats={k: int(v) for k, v in stats.items()}, outputs_sorted=ok)
    print(json.dumps(line), flush=True)


def bench_batched(args):
    """Batched form: 100,000 fp64 arrays with lognormal sizes (median 4096, sigma 1.39, clipped to
    [64, 1e7]), each drawn from one of six distributions chosen per array by seed, sorted by one
    segmented sort with autotuned parameters; compared with the default parameters and with one
    plain ipls_sort launch per array (on a bounded leading subset of the arrays)."""
    import numpy as np
    import torch

    import gen
    import gen.device as gdev
    import paper_2208_06902_amd as ipls

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nseg = args.arrays
    sizes = gen.segment_sizes_lognormal(nseg, 10, median=4096, lo=64, hi=10_000_000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(off[-1])
    dists6 = ("uniform01", "normal", "lognormal", "exponential", "mixgauss", "uniform_int")
    which = np.random.default_rng(11).integers(0, 6, nseg)
    print(f"# batched: {nseg} arrays, {total} fp64 keys", file=sys.stderr, flush=True)
    ids = torch.repeat_interleave(torch.from_numpy(which).to(dev), torch.from_numpy(sizes.astype(np.int64)).to(dev))
    pristine = torch.empty(total, dtype=torch.float64, device=dev)
    for d in range(6):
        part = gdev.fp64(dists6[d], total, 20 + d, device=dev)
        torch.where(ids == d, part, pristine, out=pristine)
        del part
    del ids
    offs = torch.from_numpy(off.view(np.int64)).to(dev)
    work = torch.empty_like(pristine)
    stream = torch.cuda.current_stream()

    t = time.perf_counter()
    tuned, rep = ipls.autotune_segmented(pristine, offs)
    tune_s = time.perf_counter() - t
    base = ipls.default_params()

    def run(params, reps):
        ms = []
        for _ in range(reps):
            work.copy_(pristine)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ipls.sort_segmented_(work, offs, params=params)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return ms

    run(tuned, args.warmup)
    tuned_ms = run(tuned, args.steps)
    base_ms = run(base, max(1, args.steps // 2))
    # correctness of every array: the output equals the input sorted by (array, totalOrder) with
    # torch's stable sorts (keys only: the sorted sequence of each array is unique)
    work.copy_(pristine)
    ipls.sort_segmented_(work, offs, params=tuned)
    torch.cuda.synchronize()
    ok = _segments_sorted_equal(work, pristine, torch.from_numpy(sizes.astype(np.int64)).to(dev), torch)
    # plain launches, one per array, on the leading arrays up to args.plain_keys keys
    m = int(np.searchsorted(off, args.plain_keys, side="right")) - 1
    m = max(1, min(m, nseg))
    sub_keys = int(off[m])
    work[:sub_keys].copy_(pristine[:sub_keys])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for i in range(m):
        lo, hi = int(off[i]), int(off[i + 1])
        ipls.sort_(work[lo:hi], None, base)
    b.record(stream)
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b)
    sub_offs = offs[: m + 1].clone()
    work[:sub_keys].copy_(pristine[:sub_keys])
    a.record(stream)
    ipls.sort_segmented_(work[:sub_keys], sub_offs, params=tuned)
    b.record(stream)
    torch.cuda.synchronize()
    sub_batched_ms = a.elapsed_time(b)
    mean_ms = sum(tuned_ms) / len(tuned_ms)
    line = _line(total / (mean_ms / 1e3), mean_ms, args.steps, args.warmup, "f64",
                 {"workload": f"batched segmented sort: {nseg} fp64 arrays, lognormal sizes (median 4096, "
                              f"sigma 1.39, clipped to [64, 1e7]), {total} keys, six distributions chosen per array",
                  "arrays": nseg, "keys": total, "parallelism": "single GPU"},
                 tuned_params={"num_buckets": tuned.num_buckets, "base_case_max": tuned.base_case_max,
                               "tile_keys": tuned.tile_keys or 4096},
                 autotune={"seconds": round(tune_s, 3), **{k: (round(v, 4) if isinstance(v, float) else v)
                                                           for k, v in rep.items()}},
                 default_params_keys_per_s=round(total / (sum(base_ms) / len(base_ms) / 1e3), 1),
                 plain_per_array={"arrays": m, "keys": sub_keys, "plain_keys_per_s": round(sub_keys / (plain_ms / 1e3), 1),
                                  "batched_keys_per_s": round(sub_keys / (sub_batched_ms / 1e3), 1),
                                  "speedup": round(plain_ms / sub_batched_ms, 2)},
                 outputs_sorted=bool(ok), outputs_checked=f"all {nseg} arrays, exact against torch's sort")
    print(json.dumps(line), flush=True)


def run_served(args, validate=True):
    """Served form: Poisson arrivals at args.rate requests/s (seed 9), sizes log-uniform in
    [1e3, 1e8], dtypes 50% fp64 / 30% uint64 / 20% fp32, distributions including lognormal(sigma=2)
    and a 20-component Gaussian mixture, admitted under a 64 GB HBM budget, the learned model
    chosen when its max bucket load is lower.  Inputs are generated on the device into the
    admitted slots.  Measures latency (arrival to completion) percentiles and throughput, then the
    same requests all at once (capacity) and as plain one-at-a-time ipls_sort launches.  With
    validate, the stream is served once more, untimed, and every request's output is compared with
    torch's sort of its regenerated input.  Returns a dict."""
    import numpy as np
    import torch

    import gen.device as gdev
    import paper_2208_06902_amd as ipls

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    count = args.requests
    r = np.random.default_rng(9)
    arrival = np.cumsum(r.exponential(1.0 / args.rate, count))
    sizes = np.round(10 ** r.uniform(3, 8, count)).astype(np.int64)
    u = r.random(count)
    dtypes = np.where(u < 0.5, 0, np.where(u < 0.8, 2, 1))
    dnames = ("lognormal2", "mixgauss20", "normal", "exponential", "uniform01", "lognormal")
    which = r.integers(0, len(dnames), count)
    total = int(sizes.sum())
    params = ipls.default_params(model=args.model, sample_max=args.sample_max)
    budget = args.budget_gb << 30
    arena = torch.empty(budget, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    print(f"# served: {count} requests, {total} keys, budget {args.budget_gb} GB", file=sys.stderr, flush=True)
    tmp = {0: torch.empty(int(sizes.max()), dtype=torch.float64, device=dev),
           1: torch.empty(int(sizes.max()), dtype=torch.float32, device=dev),
           2: torch.empty(int(sizes.max()), dtype=torch.int64, device=dev)}

    srv = ipls.Server(arena, ipls.server_config(params, lanes=args.lanes))

    def serve(arrivals, k, check=False):
        done_t = {}
        bad = []
        before = srv.stats()
        views = {}

        def reap():
            for d in srv.poll(1024):
                i, kv = views.pop(d["req_id"])
                if d["status"] != 0:
                    raise RuntimeError(f"request {i} failed: {d}")
                done_t[i] = d["t_done"]
                if check:
                    n, dt = int(sizes[i]), int(dtypes[i])
                    ref = tmp[dt][:n]
                    gdev.request_keys(dnames[which[i]], n, 50_000 + i, dt, ref, device=dev)
                    if not _sorted_equal(kv, ref, dt, torch):
                        want = torch.sort(_ord_i64(ref, dt, torch)).values
                        got = _ord_i64(kv, dt, torch)
                        diff = torch.nonzero(want != got).flatten()
                        bad.append({"request": i, "n": n, "dtype": dt, "dist": dnames[which[i]],
                                    "batch_size": d["batch_size"], "mismatches": int(diff.numel()),
                                    "first": int(diff[0]) if diff.numel() else None,
                                    "last": int(diff[-1]) if diff.numel() else None,
                                    "sorted": bool((got[1:] >= got[:-1]).all()),
                                    # the input left as it was / the input's keys in another order
                                    "unchanged": bool(torch.equal(got, _ord_i64(ref, dt, torch))),
                                    "permutation": bool(torch.equal(torch.sort(got).values, want)),
                                    "arena_offset": int(kv.data_ptr() - arena.data_ptr())})
                srv.release(d["req_id"])

        t0 = time.monotonic() + 0.02
        for i in range(k):
            while time.monotonic() < t0 + arrivals[i]:
                reap()
            while True:
                got = srv.reserve(int(sizes[i]), int(dtypes[i]), False)
                if got is not None:
                    break
                reap()
                time.sleep(0.0002)
            rid, kv, _ = got
            gdev.request_keys(dnames[which[i]], int(sizes[i]), 50_000 + i, int(dtypes[i]), kv, device=dev)
            srv.submit(rid, stream)
            views[rid] = (i, kv)
        while views:
            reap()
            time.sleep(0.0002)
        after = srv.stats()
        st = {f: after[f] - before[f] for f in ("batches_run", "singles_run", "rejected")}
        st["max_queue_depth"] = after["max_queue_depth"]
        st["peak_bytes_in_use"] = after["peak_bytes_in_use"]
        lat = np.array([done_t[i] - (t0 + arrivals[i]) for i in range(k)]) * 1e3
        span = max(done_t.values()) - t0
        return lat, span, st, bad

    serve(np.zeros(count), min(count, 200))  # warm the lanes' contexts
    lat, span, st, _ = serve(arrival, count)
    lat_sat, span_sat, st_sat, _ = serve(np.zeros(count), count)
    bad = None
    if validate:
        print("# served: validating every request", file=sys.stderr, flush=True)
        _, _, _, bad = serve(np.zeros(count), count, check=True)
    srv.close()
    del arena
    # plain: one request at a time through ipls_sort, same generation
    torch.cuda.synchronize()
    t = time.monotonic()
    for i in range(count):
        n = int(sizes[i])
        b = tmp[int(dtypes[i])][:n]
        gdev.request_keys(dnames[which[i]], n, 50_000 + i, int(dtypes[i]), b, device=dev)
        ipls.sort_(b.view(torch.uint64) if dtypes[i] == 2 else b, None, params)
    torch.cuda.synchronize()
    plain_s = time.monotonic() - t
    del tmp
    torch.cuda.empty_cache()
    return {"requests": count, "keys": total, "span_s": span,
            "achieved_keys_per_s": round(total / span, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "mean": round(float(lat.mean()), 3), "max": round(float(lat.max()), 3)},
            "offered_keys_per_s": round(total / float(arrival[-1]), 1),
            "saturated": {"keys_per_s": round(total / span_sat, 1),
                          "latency_p50_ms": round(float(np.percentile(lat_sat, 50)), 3),
                          "latency_p99_ms": round(float(np.percentile(lat_sat, 99)), 3)},
            "plain_one_at_a_time_keys_per_s": round(total / plain_s, 1),
            "saturated_vs_plain": round(plain_s / span_sat, 2),
            "server": {"batches_run": st["batches_run"], "singles_run": st["singles_run"],
                       "max_queue_depth": st["max_queue_depth"], "rejected_reserves": st["rejected"],
                       "peak_bytes_in_use": st["peak_bytes_in_use"]},
            "outputs_checked": (f"all {count} requests, exact against torch's sort of each regenerated input"
                                if validate else "not checked"),
            "outputs_ok": None if bad is None else not bad,
            "failed_requests": None if bad is None else bad[:10]}


def bench_served(args):
    """The served form's own line (see run_served)."""
    res = run_served(args)
    count = res["requests"]
    line = _line(res["achieved_keys_per_s"], res["span_s"] * 1e3 / count, count, 0, "mixed f64/u64/f32",
                 {"workload": f"served: {count} requests, Poisson {args.rate:g}/s, sizes log-uniform [1e3, 1e8], "
                              f"dtypes 50/30/20 f64/u64/f32, {args.budget_gb} GB budget, learned model when lower "
                              f"max load", "requests": count, "keys": res["keys"], "lanes": args.lanes,
                  "parallelism": "single GPU"},
                 **{k: v for k, v in res.items() if k not in ("requests", "keys", "span_s", "achieved_keys_per_s")},
                 outputs_sorted=bool(res["outputs_ok"]))
    print(json.dumps(line), flush=True)


def sample_label(args) -> str:
    cap = f"capped at {args.sample_max} keys" if args.sample_max else "uncapped"
    return f"1% jittered stratified, {cap}" + (", inherited by children" if args.inherit else "")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="sort: skip the figures beside the headline (defaults, learned model, served)")
    ap.add_argument("--dists", default=",".join(DISTS))
    ap.add_argument("--sample-max", type=int, default=4096)
    ap.add_argument("--tile-keys", type=int, default=0, help="keys per distribution tile (0 = library default)")
    ap.add_argument("--sort-model", type=int, default=0, help="sort: 0 FMCD (default), 1 auto, 2 learned")
    ap.add_argument("--equality", type=int, default=0, help="sort, u64, zipf: 1 = equality buckets for heavy values")
    ap.add_argument("--inherit", type=int, default=0,
                    help="sort, u64, zipf: 1 = children reuse their part of the parent's sample")
    ap.add_argument("--workload", choices=("sort", "u64", "zipf", "batched", "served"), default="sort",
                    help="sort: the 1e8 fp64 single-array sort (default); u64: 1e9 uniform uint64 keys; "
                         "zipf: 2e8 Zipf(1.1) uint64 keys with a uint32 index payload; batched; served")
    ap.add_argument("--arrays", type=int, default=100_000, help="batched: number of arrays")
    ap.add_argument("--plain-keys", type=int, default=50_000_000, help="batched: keys of the per-array subset")
    ap.add_argument("--requests", type=int, default=4000, help="served: number of requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: arrivals per second")
    ap.add_argument("--budget-gb", type=int, default=64, help="served: HBM budget")
    ap.add_argument("--lanes", type=int, default=3, help="served: concurrent lanes")
    ap.add_argument("--model", type=int, default=1, help="served: 0 FMCD, 1 auto (learned model when lower max load)")
    ap.add_argument("--summarize-profiles", nargs=4, metavar=("KTRACE_DIR", "FETCH_DIR", "WRITE_DIR", "BENCH_JSON"),
                    help="write profiles/ summaries from rocprofv3 CSV output and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, out_dir=os.path.join(ROOT, "profiles"))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form is not built",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.workload in ("u64", "zipf"):
        return bench_large_u64(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)

    import numpy as np
    import torch

    import gen
    import paper_2208_06902_amd as ipls

    dists = [d for d in args.dists.split(",") if d]
    n = args.n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"# generating {len(dists)} inputs of {n} keys", file=sys.stderr, flush=True)
    host_inputs = {d: gen.make(d, n, SEEDS.get(d, 1)) for d in dists}
    pristine = {d: torch.from_numpy(host_inputs[d]).to(dev) for d in dists}
    total = args.warmup + args.steps
    order = [dists[i % len(dists)] for i in range(total)]

    params = ipls.default_params(sample_max=args.sample_max, tile_keys=args.tile_keys, model=args.sort_model,
                                 equality=args.equality, inherit=args.inherit)
    stream = torch.cuda.current_stream()

    # warmup: also checks parity of each distribution's output against numpy's sort
    print("# warmup", file=sys.stderr, flush=True)
    stats = {}
    checked = {}
    for i in range(args.warmup):
        d = order[i]
        buf = pristine[d].clone()
        st = ipls.sort_(buf, None, params, stats=True)
        torch.cuda.synchronize()
        stats[d] = st
        if d not in checked:
            out = buf.cpu().numpy()
            checked[d] = bool(np.all(out[1:] >= out[:-1]))
        del buf

    # stage one private copy per timed step, then time the steps back to back
    bufs = [pristine[order[args.warmup + i]].clone() for i in range(args.steps)]
    torch.cuda.synchronize()
    # the timed steps record events around the scatter only (each record costs host time on a
    # launch-bound path); the counting and base-case figures come from extra steps afterwards
    ipls.profile_enable(1 << ipls.KERNEL_SCATTER)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per_step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ipls.sort_(bufs[i], None, params)
        b.record(stream)
        per_step_ms.append((a, b))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sc_n, sc_ms, sc_bytes = ipls.profile_read(ipls.KERNEL_SCATTER)
    sc_lv = [ipls.profile_read_level(ipls.KERNEL_SCATTER, lv) for lv in range(PROFILE_LEVELS)]
    ipls.profile_enable(False)
    gpu_ms = ev0.elapsed_time(ev1)
    # counting and base case: the same steps again (outside the timed region), profiled
    ipls.profile_enable((1 << ipls.KERNEL_CLASSIFY) | (1 << ipls.KERNEL_BASE))
    for i in range(args.steps):
        b2 = pristine[order[args.warmup + i]].clone()
        ipls.sort_(b2, None, params)
        del b2
    torch.cuda.synchronize()
    cl_n, cl_ms, cl_bytes = ipls.profile_read(ipls.KERNEL_CLASSIFY)
    bc_n, bc_ms, bc_bytes = ipls.profile_read(ipls.KERNEL_BASE)
    cl_lv = [ipls.profile_read_level(ipls.KERNEL_CLASSIFY, lv) for lv in range(PROFILE_LEVELS)]
    ipls.profile_enable(False)
    steps_ms = [a.elapsed_time(b) for a, b in per_step_ms]
    ms_per_step = gpu_ms / args.steps
    value = n * args.steps / (gpu_ms / 1e3)

    # output check of the timed steps: ascending, and the same multiset of bit patterns as the input
    def multiset_hash(a):
        u = np.ascontiguousarray(a).view(np.uint64)
        h = (u ^ (u >> np.uint64(31))) * np.uint64(0x9E3779B97F4A7C15)
        return int(np.sum(h, dtype=np.uint64)), int(np.bitwise_xor.reduce(h))

    timed_ok = True
    for i in range(min(args.steps, len(dists))):
        out = bufs[i].cpu().numpy()
        src = host_inputs[order[args.warmup + i]]
        timed_ok &= bool(np.all(out[1:] >= out[:-1])) and multiset_hash(out) == multiset_hash(src)
    del bufs

    by_dist = {}
    for d, ms in zip(order[args.warmup:], steps_ms):
        by_dist.setdefault(d, []).append(ms)

    sc_gbs = sc_bytes / (sc_ms / 1e3) / 1e9 if sc_ms > 0 else None
    traffic = traffic_per_launch()
    roofline = {
        "kernel": "k_scatter (classify, stable wave rank, LDS-staged bucket-ordered write)",
        "bound": "hbm",
        "achieved": round(sc_gbs, 1) if sc_gbs else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(sc_gbs / HBM_PEAK_GBS, 4) if sc_gbs else None,
        "traffic": traffic,
        "launches": sc_n,
        "avg_launch_ms": round(sc_ms / sc_n, 4) if sc_n else None,
        "algorithmic_bytes_per_launch": round(sc_bytes / sc_n) if sc_n else None,
    }
    pass_gbs = (sc_bytes + cl_bytes) / ((sc_ms + cl_ms) / 1e3) / 1e9 if (sc_ms + cl_ms) > 0 else None
    # each level's distribution pass (counting + scatter), per step: the keys it moves, its time and
    # its rate against peak (the timed steps give the scatter, the profiled repeat the counting)
    pass_by_level = []
    for lv in range(PROFILE_LEVELS):
        (sn, sms, sby), (cn, cms, cby) = sc_lv[lv], cl_lv[lv]
        if sn == 0 or cn == 0:
            continue
        ms_lv = (sms + cms) / args.steps
        gb_lv = (sby + cby) / args.steps / 1e9
        pass_by_level.append({"level": lv, "scatter_launches_per_step": round(sn / args.steps, 2),
                              "algorithmic_gb": round(gb_lv, 3), "ms": round(ms_lv, 4),
                              "gbs": round(gb_lv / (ms_lv / 1e3), 1),
                              "frac_of_peak": round(gb_lv / (ms_lv / 1e3) / HBM_PEAK_GBS, 4)})

    cpu_baseline = None
    if not args.no_cpu_baseline:
        import oracle
        d0 = dists[0]
        print(f"# cpu baseline: oracle on one full step ({d0}, {n} keys)", file=sys.stderr, flush=True)
        t = time.perf_counter()
        want, _, _ = oracle.sort(host_inputs[d0], None, oracle.params(sample_max=args.sample_max, model=args.sort_model,
                                                                      equality=args.equality, inherit=args.inherit))
        dt = time.perf_counter() - t
        # parity of the GPU result for this step against the oracle
        g = pristine[d0].clone()
        ipls.sort_(g, None, params)
        torch.cuda.synchronize()
        parity = bool(np.array_equal(g.cpu().numpy().view(np.uint64), want.view(np.uint64)))
        cpu_baseline = {"value": round(n / dt, 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
                        "sample": f"one full step: {n} {d0} fp64 keys sorted by the sequential C oracle "
                                  f"({dt:.1f} s on 1 thread of {cpu_model()}); GPU output bit-identical: {parity}",
                        "host_cpus": os.cpu_count(), "host_cpus_usable": len(os.sched_getaffinity(0))}
        # context: the C++ standard library's sorts on one thread, on the first 1e7 keys of that input
        m = min(n, 10_000_000)
        ctx = oracle.std_sorts_seconds(host_inputs[d0][:m])
        cpu_baseline["context"] = {"sample": f"first {m} keys of the {d0} input, 1 thread, g++ -O2",
                                   **{f"{k}_keys_per_s": round(m / v, 1) for k, v in ctx.items()}}

    extras = {}
    if not args.no_extras:
        extras = sort_extras(args, dists, pristine, n)
    del pristine

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain single-array sort, {n} fp64 keys per step, keys only, cycling "
                               + "/".join(dists), "n": n, "num_buckets": 256, "base_case_max": 4096,
                   "bucket_policy": BUCKET_POLICY_LABEL if args.sort_model == 0 else "256 everywhere",
                   "sample": sample_label(args),
                   "model": ("FMCD", "auto (learned model when lower max load)", "learned",
                             "splitter tree")[args.sort_model],
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        "pass_gbs": round(pass_gbs, 1) if pass_gbs else None,
        "pass_frac_of_peak": round(pass_gbs / HBM_PEAK_GBS, 4) if pass_gbs else None,
        "pass_by_level": pass_by_level,
        "classify_gbs": round(cl_bytes / (cl_ms / 1e3) / 1e9, 1) if cl_ms > 0 else None,
        "base_case_ms_per_step": round(bc_ms / args.steps, 4),
        "scatter_ms_per_step": round(sc_ms / args.steps, 4),
        "classify_ms_per_step": round(cl_ms / args.steps, 4),
        "ms_by_dist": {d: round(sum(v) / len(v), 4) for d, v in by_dist.items()},
        "levels_by_dist": {d: stats[d]["levels"] for d in stats},
        "wall_s_timed": round(wall, 3),
        "outputs_sorted": all(checked.values()) and timed_ok,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


def sort_extras(args, dists, pristine, n):
    """Figures beside the headline, all outside its timed region: the library's default parameters
    on the same inputs, the learned model against FMCD on its two inputs, and the served form."""
    import torch

    import gen.device as gdev
    import paper_2208_06902_amd as ipls

    stream = torch.cuda.current_stream()

    def timed(x, params, reps):
        ms, st, out = [], None, None
        for k in range(reps + 1):
            out = x.clone()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            st = ipls.sort_(out, None, params, stats=True)
            b.record(stream)
            torch.cuda.synchronize()
            if k:
                ms.append(a.elapsed_time(b))
        return sum(ms) / len(ms), st, out

    print("# extras: default parameters", file=sys.stderr, flush=True)
    dflt = ipls.default_params()
    by = {d: timed(pristine[d], dflt, 2)[0] for d in dists}
    out = {"default_params": {"sample": "1% jittered stratified, uncapped (the library's defaults)",
                              "keys_per_s": round(n * len(dists) / (sum(by.values()) / 1e3), 1),
                              "ms_by_dist": {d: round(v, 4) for d, v in by.items()}}}

    print("# extras: learned model", file=sys.stderr, flush=True)
    learned = {}
    for dname, seed in (("lognormal2", 40), ("mixgauss20", 41)):
        x = gdev.fp64(dname, n, seed)
        r = {}
        for tag, model in (("fmcd", 0), ("auto", 1)):
            ms, st, o = timed(x, ipls.default_params(sample_max=args.sample_max, model=model), 3)
            r[tag] = {"ms": round(ms, 4), "keys_per_s": round(n / (ms / 1e3), 1), "levels": st["levels"],
                      "passes": st["passes"], "level1_max_load": st["level1_max_load"],
                      "l2pl_used": st["l2pl_used"], "output_exact": _sorted_equal(o, x, 0, torch)}
            del o
        r["speedup"] = round(r["fmcd"]["ms"] / r["auto"]["ms"], 3)
        learned[dname] = r
        del x
    out["learned"] = {"workload": f"{n} fp64 keys drawn on the device, sample capped at {args.sample_max} keys; "
                                  "auto = two-level model when its max sample load is lower", **learned}
    torch.cuda.empty_cache()

    print("# extras: served", file=sys.stderr, flush=True)
    res = run_served(args)
    out["served"] = {"workload": f"{res['requests']} requests, Poisson {args.rate:g}/s, sizes log-uniform [1e3, 1e8], "
                                 f"dtypes 50/30/20 f64/u64/f32, {args.budget_gb} GB budget, {args.lanes} lanes, "
                                 f"learned model when lower max load", **res}
    return out


if __name__ == "__main__":
    main()
