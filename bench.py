#!/usr/bin/env python3
"""Serial-EMD throughput on one MI355X.

Default workload: the uneven multivariate batch at full size -- 4,096 series
of 2-16 channels x 1e3-6.5e4 samples per channel (log-uniform), each
serialized (D = 0) and decomposed as an EEMD ensemble of 64 white-noise
realizations (noise sigma 0.2 std of the series), up to 6 IMFs with 10 sifts
per IMF.  The batch runs in 16 waves of 256 consecutive series; one step is
one wave (one semd_eemd_batch call), and the timed steps cycle through the
waves.  Inputs and outputs stay resident in HBM.  `value` is input samples
per second; the line also carries realization-samples per second, the
per-kernel times (HIP events around every kernel in the timed region), the
HBM roofline position of the dominant kernel (st_eval_kernel) and the CPU
oracle timed on a seeded random sample of the series.

Other workloads (--workload), each printing one line of the same shape:
  faces     1,024 face-like 112 x 92 images (uint8-valued), one batched
            launch per step, with the plain path (one launch per image)
  series    one 3 x 1000 multivariate series, plain path, latency over repeats
  textures  64 texture images 128 x 128, one launch per image (and batched)
  serving   the serving mix with Poisson arrivals: continuous-batching
            engine against plain per-request decompositions
  dsweep    the transition-length sweep of Sec. 4.1 (D = 1..500) on the
            six-variate pick-up-mask series, fixed and SD stopping rules
  ensembles serial-CEEMDAN, serial-EEMD and serial-EMD of that series at
            D = 50 (the serial-version comparison of Sec. 4.1)

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP64 operations of the method: per sample per sift 4 compares
# (extrema), 2 x 12 (one cubic piece of each envelope) and 3 (mean and
# update); per knot per sift about 10 for its Thomas row plus 1 reciprocal
FLOPS_PER_SAMPLE_SIFT = 30
FLOPS_PER_KNOT = 11
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0

# HBM traffic of the resident kernel on the face workload, read from
# FETCH_SIZE and WRITE_SIZE counter runs and scaled by the same counters on a
# copy of known size; valid only while the kernel sources are the ones it was
# taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "resident_emd_kernel_faces_112x92x1024_traffic.txt")
KERNEL_SOURCES = ["semd_kernels.hip", "semd_device.h", "semd_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_15319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n_images: int, D: int):
    """Bytes per launch from the committed counter summary, or None when it
    is absent, was taken on another workload, or the kernel changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv["source_sha256"] != kernel_source_hash():
            return None
        if int(kv["images"]) != n_images or int(kv["D"]) != D:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# longest serialized signal the automatic path decomposes on chip
ONCHIP_MAX_LENGTH = 16384

STREAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "st_eval_kernel_eemd_uneven_traffic.txt")
STREAM_SOURCES = ["semd_stream.hip", "semd_stream.h", "semd_device.h", "semd_internal.h"]


def stream_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in STREAM_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_15319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_stream_traffic(D: int):
    """HBM bytes per st_eval_kernel launch from the committed counter summary
    of the uneven EEMD workload, or None when it is absent, was taken on
    another D, or the streaming kernels changed since."""
    if not os.path.exists(STREAM_TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(STREAM_TRAFFIC_FILE):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv["source_sha256"] != stream_source_hash() or int(kv["D"]) != D:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mib: int, reps: int) -> int:
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (bytes read = bytes written per copy), and its bandwidth."""
    import torch
    gbps = copy_bandwidth(torch, mib, reps)
    print(json.dumps({"copy_bytes": mib * (1 << 20), "reps": reps,
                      "read_plus_write_GBps": gbps}), flush=True)
    return 0


def copy_bandwidth(torch, mib: int = 1024, reps: int = 10) -> float:
    """Read plus written GB/s of a plain device copy (torch's), timed with
    HIP events: what a streaming kernel reaches in practice, for context
    beside the published peak."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    return 2 * n * 8 / (ms / 1e3) / 1e9


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def base_record(args, metric_value, ms_per_step, dtype="f64"):
    return {
        "metric": "samples decomposed/s/GPU (batched+served vs plain), p50/p99 latency, "
                  "%HBM peak",
        "value": metric_value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
    }


def roofline_alu(flops, kern_ms, kernel, traffic=None):
    achieved = flops / (kern_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic, "kernel": kernel,
            "kernel_ms": kern_ms, "flops_per_launch": flops}


def work_stats(stats, counts):
    st = stats.sum(0).cpu().numpy()
    n_imfs = counts.cpu().numpy()
    return {"sifts": int(st[0]), "knots": int(st[1]), "sample_sifts": int(st[2]),
            "mean_imfs": float(np.maximum(n_imfs, 0).mean())}


def cpu_threads():
    """Host threads for the oracle: all logical CPUs up to 16, the host share
    of one GPU on the measurement machines."""
    return min(16, os.cpu_count() or 1)


def cpu_decompose_rate(items, D, K, S, threads):
    """The oracle over the given items on the host, one item per task."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    oracle.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda it: oracle.decompose(it.X, it.M, it.N, D, K, S), items))
    dt = time.perf_counter() - t0
    samples = sum(it.M * it.N for it in items)
    return samples / dt, dt, samples


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def run_faces(args, semd, torch, workloads):
    dev = torch.device("cuda:0")
    K, S, D = 8, 10, args.D
    path = {"auto": semd.SEMD_PATH_AUTO, "onchip": semd.SEMD_PATH_ONCHIP,
            "stream": semd.SEMD_PATH_STREAM}[args.path]
    items = workloads.config2(args.batch)
    M, N = items[0].M, items[0].N
    MN = M * N
    L = M * N + D * N - D
    n = len(items)

    X = torch.from_numpy(np.stack([it.X for it in items])).to(dev)
    out = torch.empty((n, K + 1, MN), dtype=torch.float64, device=dev)
    counts = torch.zeros(n, dtype=torch.int32, device=dev)
    stats = torch.zeros((n, 3), dtype=torch.int64, device=dev)
    shapes = [[M, N]] * n

    # work statistics of one decomposition of the batch (untimed)
    semd.PreparedBatch([X[i] for i in range(n)], shapes, [out[i] for i in range(n)], counts, D,
                       K, S, stats=stats, path=path).run()
    torch.cuda.synchronize()
    work = work_stats(stats, counts)

    pb = semd.PreparedBatch([X[i] for i in range(n)], shapes, [out[i] for i in range(n)],
                            counts, D, K, S, path=path)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        pb.run()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        pb.run()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = n * MN / (ms_per_step / 1e3)

    # plain path: one launch per image, same images
    npl = min(args.plain_items, n)
    plain = None
    if npl > 0:
        outs1 = [torch.empty((K + 1, MN), dtype=torch.float64, device=dev) for _ in range(npl)]
        cnt1 = torch.empty(npl, dtype=torch.int32, device=dev)
        for i in range(min(4, npl)):
            semd.semd_decompose_ex(X[i], [M, N], D, K, S, outs1[i], cnt1[i:i + 1])
        torch.cuda.synchronize()
        pev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(npl)]
        t1 = time.perf_counter()
        for i, (a, b) in enumerate(pev):
            a.record(stream)
            semd.semd_decompose_ex(X[i], [M, N], D, K, S, outs1[i], cnt1[i:i + 1])
            b.record(stream)
        torch.cuda.synchronize()
        plain_wall = time.perf_counter() - t1
        plain_ms = [a.elapsed_time(b) for a, b in pev]
        plain_value = npl * MN / plain_wall
        same = all(torch.equal(outs1[i], out[i]) for i in range(npl))
        plain = {"value": plain_value, "unit": "samples/s", "images": npl,
                 "image_p50_ms": pct(plain_ms, 50), "image_p99_ms": pct(plain_ms, 99),
                 "batched_over_plain": value / plain_value, "outputs_identical": same}

    # roofline of the dominant kernel: on the on-chip path the batch is one
    # launch of the resident kernel per step (the events bracket that launch
    # and its ~100 KB descriptor upload); on the streaming path the figure
    # covers the whole step's kernel sequence
    kern_ms = float(np.mean(step_ms))
    flops = FLOPS_PER_SAMPLE_SIFT * work["sample_sifts"] + FLOPS_PER_KNOT * work["knots"]
    onchip = args.path == "onchip" or (args.path == "auto" and L <= semd.semd_resident_max_length())
    traffic = measured_traffic(n, D) if onchip else None
    b_io = 8 * MN * n * (K + 2)
    b_stream = b_io + 16 * work["sample_sifts"] + 16 * L * int(round(work["mean_imfs"] * n))

    res = base_record(args, value, ms_per_step)
    res["config"] = {"workload": f"face-like images 112x92 (uint8-valued) x {n}, serialized "
                                 f"column-wise, D={D}, batched Serial-EMD",
                     "batch": n, "M": M, "N": N, "D": D, "L": L, "max_imfs": K,
                     "sift_iters": S, "path": args.path}
    res["latency_ms"] = {"step_p50": pct(step_ms, 50), "step_p99": pct(step_ms, 99)}
    res["plain"] = plain
    res["work"] = work
    res["roofline"] = roofline_alu(flops, kern_ms,
                                   "resident_emd_kernel" if onchip else "streaming step", traffic)
    res["hbm"] = {"algorithmic_io_bytes": b_io,
                  "io_GBps": b_io / (kern_ms / 1e3) / 1e9,
                  "io_frac_of_peak": b_io / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
                  # what a kernel that re-read and re-wrote the candidate through HBM on
                  # every sift would have to sustain to match this rate: a comparison
                  # figure, not a measured bandwidth
                  "hypothetical_stream_GBps": b_stream / (kern_ms / 1e3) / 1e9}
    if not args.no_cpu:
        threads = cpu_threads()
        nproc, model = host_cpu()
        ncpu = min(args.cpu_items, n)
        rate, dt, samples = cpu_decompose_rate(items[:ncpu], D, K, S, threads)
        res["cpu_baseline"] = {"value": rate, "unit": "samples/s", "cores": threads,
                               "kind": "oracle", "host_cpus": nproc, "cpu_model": model,
                               "sample": f"{ncpu} of the {n} images, {samples} input samples, "
                                         f"{dt:.1f} s wall on {threads} threads"}
    return res


def run_series(args, semd, torch, workloads):
    """One 3 x 1000 series per launch (plain path), repeated."""
    dev = torch.device("cuda:0")
    K, S, D = 6, 10, args.D
    it = workloads.config0()
    M, N = it.M, it.N
    X = torch.from_numpy(it.X).to(dev)
    out = torch.empty((K + 1, M * N), dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    st = torch.zeros((1, 3), dtype=torch.int64, device=dev)
    semd.PreparedBatch([X], [[M, N]], [out], cnt, D, K, S, stats=st).run()
    torch.cuda.synchronize()
    work = work_stats(st, cnt)
    reps = max(args.repeats, 1)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        semd.semd_decompose_ex(X, [M, N], D, K, S, out, cnt)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        semd.semd_decompose_ex(X, [M, N], D, K, S, out, cnt)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in ev]
    ms = wall * 1e3 / reps
    res = base_record(args, M * N / (ms / 1e3), ms)
    L = M * N + D * N - D
    res["config"] = {"workload": f"3-channel series x 1000 samples, D={D}, plain path, one "
                                 f"signal per launch", "M": M, "N": N, "D": D, "L": L,
                     "max_imfs": K, "sift_iters": S, "repeats": reps}
    res["latency_ms"] = {"p50": pct(lat, 50), "p99": pct(lat, 99)}
    # the standard (slice-wise) EMD of the same channels, for comparison
    so = torch.empty((K + 1, M * N), dtype=torch.float64, device=dev)
    sn = torch.empty(N, dtype=torch.int32, device=dev)
    semd.semd_decompose_slices(X, [M, N], K, S, so, sn)
    torch.cuda.synchronize()
    sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in sev:
        a.record(stream)
        semd.semd_decompose_slices(X, [M, N], K, S, so, sn)
        b.record(stream)
    torch.cuda.synchronize()
    slat = [a.elapsed_time(b) for a, b in sev]
    res["slices"] = {"p50_ms": pct(slat, 50), "p99_ms": pct(slat, 99),
                     "channels": N, "imfs_per_channel": [int(v) for v in sn.cpu().tolist()]}
    res["work"] = work
    flops = FLOPS_PER_SAMPLE_SIFT * work["sample_sifts"] + FLOPS_PER_KNOT * work["knots"]
    res["roofline"] = roofline_alu(flops, float(np.mean(lat)),
                                   "resident_emd_kernel (1 workgroup)")
    if not args.no_cpu:
        import oracle
        oracle.lib()
        nrep = 50
        t1 = time.perf_counter()
        for _ in range(nrep):
            oracle.decompose(it.X, M, N, D, K, S)
        dt = time.perf_counter() - t1
        res["cpu_baseline"] = {"value": nrep * M * N / dt, "unit": "samples/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{nrep} decompositions of the series, {dt:.2f} s on "
                                         f"one thread ({1e3 * dt / nrep:.2f} ms each)"}
    return res


def run_dsweep(args, semd, torch, workloads):
    """Transition-length sweep of Sec. 4.1: the six-variate pick-up-mask series
    (6 x 1000 samples) decomposed on the plain path for D = 1..500 under the
    fixed sift count (S = 10) and the SD rule (at most 100 sifts per IMF).
    Per D and rule: latency percentiles over the repeats, the work done, the
    oracle's time on one host thread, and how far the first two serial IMFs
    of each variate lie from its slice-wise (standard EMD) IMFs."""
    dev = torch.device("cuda:0")
    it = workloads.config5()
    M, N, K = it.M, it.N, 8
    X = torch.from_numpy(it.X).to(dev)
    rules = [("fixed", 10, 0.0), ("sd", 100, args.sd)]
    Ds = [1, 2, 5, 10, 20, 50, 100, 200, 300, 400, 500]
    reps = max(args.steps, 1)
    stream = torch.cuda.current_stream()
    slices = {}
    for name, S, sd in rules:
        so, sn = semd.semd_decompose_slices(X, [M, N], K, S, sd=sd)
        slices[name] = (so.cpu().numpy(), sn.cpu().numpy())
    cpu_reps = 0 if args.no_cpu else 10
    if cpu_reps:
        import oracle
        oracle.lib()
    rows = []
    for D in Ds:
        for name, S, sd in rules:
            out = torch.empty((K + 1, M * N), dtype=torch.float64, device=dev)
            cnt = torch.empty(1, dtype=torch.int32, device=dev)
            st = torch.zeros((1, 3), dtype=torch.int64, device=dev)
            semd.PreparedBatch([X], [[M, N]], [out], cnt, D, K, S, stats=st, sd=sd).run()
            torch.cuda.synchronize()
            work = work_stats(st, cnt)
            for _ in range(max(args.warmup, 1)):
                semd.semd_decompose_ex(X, [M, N], D, K, S, out, cnt, sd=sd)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for a, b in ev:
                a.record(stream)
                semd.semd_decompose_ex(X, [M, N], D, K, S, out, cnt, sd=sd)
                b.record(stream)
            torch.cuda.synchronize()
            lat = [a.elapsed_time(b) for a, b in ev]
            o = out.cpu().numpy()
            so = slices[name][0]
            diffs = []
            for q in range(2):
                d = [float(np.linalg.norm(o[q, c * M:(c + 1) * M] - so[q, c * M:(c + 1) * M]) /
                           max(np.linalg.norm(so[q, c * M:(c + 1) * M]), 1e-300))
                     for c in range(N)]
                diffs.append(float(np.mean(d)))
            row = {"D": D, "rule": name, "L": M * N + D * N - D, "p50_ms": pct(lat, 50),
                   "p10_ms": pct(lat, 10), "p90_ms": pct(lat, 90), "sifts": work["sifts"],
                   "n_imfs": int(cnt.cpu()[0]), "imf12_rel_diff_vs_slices": diffs}
            if cpu_reps:
                ct = []
                for _ in range(cpu_reps):
                    t1 = time.perf_counter()
                    oracle.decompose(it.X, M, N, D, K, S, sd=sd)
                    ct.append(1e3 * (time.perf_counter() - t1))
                row["cpu_ms"] = pct(ct, 50)
            rows.append(row)
    head = next(r for r in rows if r["D"] == 200 and r["rule"] == "sd")
    ms = head["p50_ms"]
    res = base_record(args, M * N / (ms / 1e3), ms)
    res["config"] = {"workload": "six-variate pick-up-mask series 6 x 1000 (Sec. 4.1), "
                                 "transition-length sweep, plain path; value at D=200 "
                                 "(20 % of the length) under the SD rule",
                     "M": M, "N": N, "max_imfs": K, "D_values": Ds,
                     "rules": {"fixed": "S=10 sifts per IMF",
                               "sd": f"SD < {args.sd}, at most 100 sifts per IMF"},
                     "repeats": reps}
    res["sweep"] = rows
    res["slices"] = {name: [int(v) for v in slices[name][1]] for name, _, _ in rules}
    # the D=200 SD-rule decomposition on the roofline
    out = torch.empty((K + 1, M * N), dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    st = torch.zeros((1, 3), dtype=torch.int64, device=dev)
    semd.PreparedBatch([X], [[M, N]], [out], cnt, 200, K, 100, stats=st, sd=args.sd).run()
    torch.cuda.synchronize()
    work = work_stats(st, cnt)
    res["work"] = work
    flops = FLOPS_PER_SAMPLE_SIFT * work["sample_sifts"] + FLOPS_PER_KNOT * work["knots"]
    res["roofline"] = roofline_alu(flops, ms, "resident_emd_kernel (1 workgroup)")
    res["paper_context"] = {"serial_emd_ms_at_D50": 10.96, "hardware": "i7-6700HQ laptop",
                            "note": "the paper's stopping rule is not stated"}
    if cpu_reps:
        res["cpu_baseline"] = {"value": M * N / (head["cpu_ms"] / 1e3), "unit": "samples/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"median of {cpu_reps} oracle decompositions per "
                                         "sweep row on one thread; value at D=200, SD rule"}
    return res


def run_textures(args, semd, torch, workloads):
    """64 texture images 128 x 128, one launch per image; batched alongside."""
    dev = torch.device("cuda:0")
    K, S, D = 8, 10, args.D
    items = workloads.config1(64, 128)
    n = len(items)
    M, N = items[0].M, items[0].N
    MN = M * N
    X = torch.from_numpy(np.stack([i.X for i in items])).to(dev)
    outs = [torch.empty((K + 1, MN), dtype=torch.float64, device=dev) for _ in range(n)]
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    st = torch.zeros((n, 3), dtype=torch.int64, device=dev)
    semd.PreparedBatch([X[i] for i in range(n)], [[M, N]] * n, outs, cnt, D, K, S,
                       stats=st).run()
    torch.cuda.synchronize()
    work = work_stats(st, cnt)
    stream = torch.cuda.current_stream()
    for i in range(2):
        semd.semd_decompose_ex(X[i], [M, N], D, K, S, outs[i], cnt[i:i + 1])
    torch.cuda.synchronize()
    steps = max(args.steps // 10, 1)
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n)]
        for i, (a, b) in enumerate(ev):
            a.record(stream)
            semd.semd_decompose_ex(X[i], [M, N], D, K, S, outs[i], cnt[i:i + 1])
            b.record(stream)
        torch.cuda.synchronize()
        lat += [a.elapsed_time(b) for a, b in ev]
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / steps
    res = base_record(args, n * MN / (ms / 1e3), ms)
    res["steps"] = steps
    L = M * N + D * N - D
    res["config"] = {"workload": f"texture images 128x128 x {n}, D={D}, plain path (one launch "
                                 f"per image)", "images": n, "M": M, "N": N, "D": D, "L": L,
                     "max_imfs": K, "sift_iters": S}
    res["latency_ms"] = {"image_p50": pct(lat, 50), "image_p99": pct(lat, 99)}
    pb = semd.PreparedBatch([X[i] for i in range(n)], [[M, N]] * n, outs, cnt, D, K, S)
    pb.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        pb.run()
    torch.cuda.synchronize()
    bms = (time.perf_counter() - t1) * 1e3 / steps
    res["batched"] = {"value": n * MN / (bms / 1e3), "ms_per_step": bms,
                      "batched_over_plain": ms / bms}
    res["work"] = work
    flops = FLOPS_PER_SAMPLE_SIFT * work["sample_sifts"] + FLOPS_PER_KNOT * work["knots"]
    if L <= ONCHIP_MAX_LENGTH:
        res["roofline"] = roofline_alu(flops / n, float(np.mean(lat)),
                                       "resident_emd_kernel (1 workgroup per launch)")
    else:
        # beyond the on-chip limit one call is a whole streaming decomposition
        # (many kernels), so no single kernel's roofline describes it
        res["roofline"] = None
        res["path"] = "streaming"
    if not args.no_cpu:
        threads = cpu_threads()
        rate, dt, samples = cpu_decompose_rate(items, D, K, S, threads)
        res["cpu_baseline"] = {"value": rate, "unit": "samples/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"all {n} images, {dt:.1f} s wall on {threads} threads"}
    return res


def host_cpu():
    """(logical CPUs of the host, CPU model name)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_eemd_rate(items, D, K, S, NR, sigmas, seed, ids, threads):
    """The oracle's EEMD of the given series on host threads, one realization
    per task (the oracle's EMD of x + beta w_m; the mean over m is
    negligible next to the decompositions and left out).  Returns input
    samples per second, the wall time and the input samples."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    oracle.lib()
    xs = [oracle.serialize(it.X, it.M, it.N, D) for it in items]

    def one(job):
        i, m = job
        x = xs[i] + sigmas[i] * oracle.noise(seed, ids[i], m, xs[i].size)
        oracle.emd(x, K, S)

    jobs = sorted(((i, m) for i in range(len(items)) for m in range(NR)),
                  key=lambda j: -xs[j[0]].size)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, jobs))
    dt = time.perf_counter() - t0
    samples = sum(it.M * it.N for it in items)
    return samples / dt, dt, samples


def run_eemd(args, semd, torch, workloads):
    """The uneven-series batch at full size: 4,096 series of 2-16 channels x
    1e3-6.5e4 samples, each an EEMD ensemble of 64 noise realizations, in 16
    waves of consecutive series.  One step is one wave (one semd_eemd_batch
    call over its 256 series); the timed steps cycle through the waves, so
    a multiple of 16 steps (the default) weighs every series equally."""
    dev = torch.device("cuda:0")
    K, S, D, NR, seed = 6, 10, args.D, 64, 2106
    n, W = workloads.CONFIG3_SERIES, workloads.CONFIG3_WAVES
    shapes = workloads.config3_shapes(n)
    t_gen = time.perf_counter()
    items = workloads.config3_items(range(n), shapes, threads=cpu_threads())
    gen_s = time.perf_counter() - t_gen
    MNs = [it.M * it.N for it in items]
    # inputs and outputs resident in device memory for the whole run
    Xs = [torch.from_numpy(it.X).to(dev) for it in items]
    out_all = torch.empty(sum((K + 1) * mn for mn in MNs), dtype=torch.float64, device=dev)
    outs, o = [], 0
    for mn in MNs:
        outs.append(out_all[o:o + (K + 1) * mn].view(K + 1, mn))
        o += (K + 1) * mn
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    stats = torch.zeros((n, 3), dtype=torch.int64, device=dev)
    sig = []
    for it, x in zip(items, Xs):
        if D == 0:
            sig.append(0.2 * float(np.std(it.X)))
        else:
            xs = semd.semd_serialize(x, [it.M, it.N], D)
            sig.append(0.2 * float(xs.std(unbiased=False).item()))
    waves = [list(workloads.config3_wave(w, n, W)) for w in range(W)]
    pbs = []
    for idx in waves:
        a, b = idx[0], idx[-1] + 1
        pbs.append(semd.PreparedBatch([Xs[i] for i in idx], [[items[i].M, items[i].N] for i in idx],
                                      [outs[i] for i in idx], cnt[a:b], D, K, S,
                                      stats=stats[a:b], ensemble=NR, seed=seed,
                                      noise_sigmas=[sig[i] for i in idx], item_ids=idx))
    wave_samples = [sum(MNs[i] for i in idx) for idx in waves]
    torch.cuda.synchronize()
    for k in range(args.warmup):
        pbs[k % W].run()
    torch.cuda.synchronize()
    # timed region: HIP events around every kernel (on the library's launch
    # stream, the current torch stream) and torch events around every step
    stream = torch.cuda.current_stream()
    semd.semd_profile_reset()
    semd.semd_profile_enable(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    order = [k % W for k in range(args.steps)]
    host_ms = []
    t0 = time.perf_counter()
    for (a, b), w in zip(ev, order):
        a.record(stream)
        th = time.perf_counter()
        pbs[w].run()
        host_ms.append((time.perf_counter() - th) * 1e3)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    semd.semd_profile_enable(False)
    kern = {}
    for name in ("st_load_kernel", "st_scan_kernel", "st_compact_kernel",
                 "st_solve_kernel", "st_eval_kernel", "resident_emd_kernel"):
        nl, ms = semd.semd_profile_read(name)
        kern[name] = {"launches": nl, "total_ms": ms, "avg_ms": ms / nl if nl else None}
    host_phases = {}
    for name in ("host_alloc", "host_tables", "host_upload", "host_launch", "host_batch_call"):
        nl, ms = semd.semd_profile_read(name)
        host_phases[name] = {"calls": nl, "total_ms": ms}
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    samples = sum(wave_samples[w] for w in order)
    value = samples / wall
    st = stats.cpu().numpy()
    wave_ss = [int(st[idx[0]:idx[-1] + 1, 2].sum()) for idx in waves]
    wave_sifts = [int(st[idx[0]:idx[-1] + 1, 0].sum()) for idx in waves]
    wave_knots = [int(st[idx[0]:idx[-1] + 1, 1].sum()) for idx in waves]
    sample_sifts = sum(wave_ss[w] for w in order)
    # Algorithmic bytes (the streaming path's B_stream, per realization:
    # 8 per input sample read, 8 per output sample written (K+1 slots), 16
    # per sample and sift for h, 16 per sample and IMF end for r).  Every
    # IMF takes at most S sifts, so an item's IMF ends number at least
    # floor(sifts / S).  The dominant kernel, the streaming evaluation,
    # moves all of it but the input read (the load's); items short enough
    # for the on-chip path keep h and r on chip, their floor is the I/O.
    Lmax = semd.semd_resident_max_length()
    Ls = [it.M * it.N + D * (it.N - 1) for it in items]
    eval_b, step_b, h_b = [0] * n, [0] * n, [0] * n
    for i in range(n):
        io_out = 8 * MNs[i] * (K + 1) * NR
        if Ls[i] > Lmax:
            h_b[i] = 16 * int(st[i, 2])
            eval_b[i] = h_b[i] + 16 * Ls[i] * (int(st[i, 0]) // S) + io_out
            step_b[i] = eval_b[i] + 8 * MNs[i] * NR
        else:
            step_b[i] = io_out + 8 * MNs[i] * NR
    timed = [i for w in order for i in waves[w]]
    ev_k = kern["st_eval_kernel"]
    eval_bytes = sum(eval_b[i] for i in timed)
    alg_bytes = sum(step_b[i] for i in timed)
    roof = None
    if ev_k["launches"]:
        per_launch = eval_bytes / ev_k["launches"]
        achieved = per_launch / (ev_k["avg_ms"] / 1e3) / 1e9
        h_only = sum(h_b[i] for i in timed) / ev_k["launches"] / (ev_k["avg_ms"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS,
                "traffic": measured_stream_traffic(D),
                "kernel": "st_eval_kernel", "kernel_avg_ms": ev_k["avg_ms"],
                "launches": ev_k["launches"], "alg_bytes_per_launch": per_launch,
                "frac_h_only": h_only / HBM_PEAK_GBPS,
                "note": "B_stream less the input read, streaming items: 16 B per sample-sift "
                        "(h), 16 B per sample and IMF end (r), 8 B per output sample; "
                        "frac_h_only counts the 16 B per sample-sift alone; copy_GBps: a "
                        "plain 1 GiB device copy measured after the timed region (context)"}
        copy = copy_bandwidth(torch)
        roof["copy_GBps"] = copy
        roof["frac_of_copy"] = achieved / copy
    res = base_record(args, value, ms_per_step)
    res["config"] = {"workload": f"uneven multivariate series, {n} series (2-16 channels x "
                                 f"1e3-6.5e4 samples per channel, log-uniform), D={D}, EEMD with "
                                 f"{NR} realizations each (noise sigma 0.2 std), K={K}, S={S}; "
                                 f"{W} waves of {len(waves[0])} series, one wave per step",
                     "series": n, "waves": W, "input_samples": sum(MNs), "realizations": NR,
                     "max_imfs": K, "sift_iters": S, "D": D,
                     "timed_waves": order, "timed_input_samples": samples}
    res["realization_samples_per_s"] = value * NR
    res["latency_ms"] = {"step_p50": pct(step_ms, 50), "step_p99": pct(step_ms, 99),
                         "host_call_p50": pct(host_ms, 50), "host_call_max": max(host_ms)}
    res["work"] = {"sample_sifts": sample_sifts,
                   "streaming_sample_sifts": sum(h_b[i] for i in timed) // 16,
                   "streaming_knots": sum(int(st[i, 1]) for i in timed if Ls[i] > Lmax),
                   "sifts": sum(wave_sifts[w] for w in order),
                   "knots": sum(wave_knots[w] for w in order),
                   "mean_imfs_max_over_realizations": float(np.maximum(cnt.cpu().numpy(), 0).mean())}
    res["roofline"] = roof
    tot_k = sum(v["total_ms"] for v in kern.values())
    res["kernels"] = {k: dict(v, share=(v["total_ms"] / tot_k if tot_k else None))
                      for k, v in kern.items() if v["launches"]}
    res["hbm"] = {"step_alg_GBps": alg_bytes / wall / 1e9,
                  "step_alg_frac_of_peak": alg_bytes / wall / 1e9 / HBM_PEAK_GBPS,
                  "note": "B_stream per realization (B_io for the on-chip items) over the "
                          "whole timed region (all kernels, launch gaps included)"}
    res["host_phases"] = host_phases
    res["input_generation_s"] = gen_s
    if not args.no_cpu:
        threads = cpu_threads()
        nproc, model = host_cpu()
        rng = np.random.default_rng(2106_15319 + 33)
        pick, tot = [], 0
        for i in rng.permutation(n):
            if tot >= args.cpu_samples:
                break
            pick.append(int(i))
            tot += MNs[i]
        sub = [items[i] for i in pick]
        rate, dt, cs = cpu_eemd_rate(sub, D, K, S, NR, [sig[i] for i in pick], seed, pick,
                                     threads)
        res["cpu_baseline"] = {"value": rate, "unit": "samples/s", "cores": threads,
                               "kind": "oracle", "host_cpus": nproc, "cpu_model": model,
                               "sample": f"{len(pick)} seeded random series of the batch "
                                         f"({cs} input samples) x {NR} realizations, one "
                                         f"realization per task on {threads} threads "
                                         f"(the GPU's host share), {dt:.1f} s wall"}
    return res


def run_ensembles(args, semd, torch, workloads):
    """The serial-version comparison of Sec. 4.1 (its Fig. 6 timing) on the
    six-variate pick-up-mask series, D = 50: serial-EMD, serial-EEMD
    (NR = 100, beta = 0.2 std of the serialized signal) and serial-CEEMDAN
    (NR = 100, eps = 0.2), each one plain call on one signal; the step is
    the CEEMDAN decomposition."""
    dev = torch.device("cuda:0")
    it = workloads.config5()
    M, N, D, K, S, NR, eps, seed = it.M, it.N, 50, 8, 10, 100, 0.2, 2106
    X = torch.from_numpy(it.X).to(dev)
    out = torch.empty((K + 1, M * N), dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    xs = semd.semd_serialize(X, [M, N], D)
    beta = 0.2 * float(xs.std(unbiased=False).item())

    def emd():
        semd.semd_decompose_ex(X, [M, N], D, K, S, out, cnt)

    def eemd():
        semd.semd_eemd_batch([X], [[M, N]], [out], cnt, D, K, S, NR, seed, [beta], [0])

    def ceemdan():
        semd.semd_ceemdan_batch([X], [[M, N]], [out], cnt, D, K, S, NR, seed, [eps], [0])

    def timed(fn, reps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        return lat

    reps = max(min(args.steps, 10), 1)
    lat_c = timed(ceemdan, reps)
    n_c = int(cnt.cpu()[0])
    lat_e = timed(eemd, reps)
    n_e = int(cnt.cpu()[0])
    lat_m = timed(emd, reps)
    ms = pct(lat_c, 50)
    res = base_record(args, M * N / (ms / 1e3), ms)
    res["steps"] = reps
    res["config"] = {"workload": "six-variate pick-up-mask series 6 x 1000 (Sec. 4.1), D=50; "
                                 "serial-CEEMDAN per step (NR=100, eps=0.2), serial-EEMD and "
                                 "serial-EMD beside it", "M": M, "N": N, "D": D,
                     "max_imfs": K, "sift_iters": S, "realizations": NR, "eps": eps,
                     "eemd_beta": beta}
    res["latency_ms"] = {"ceemdan_p50": ms, "ceemdan_p99": pct(lat_c, 99),
                         "eemd_p50": pct(lat_e, 50), "eemd_p99": pct(lat_e, 99),
                         "emd_p50": pct(lat_m, 50), "emd_p99": pct(lat_m, 99)}
    res["modes"] = {"ceemdan": n_c, "eemd_max": n_e}
    res["paper_context"] = {"serial_emd_ms": 10.96, "serial_eemd_ms": 397.92,
                            "serial_ceemdan_ms": 1154.97, "hardware": "i7-6700HQ laptop",
                            "note": "D = 50; the paper's NR and stopping rule are those "
                                    "recommended by the methods' authors, not stated"}
    res["roofline"] = None
    if not args.no_cpu:
        import oracle
        oracle.lib()
        t1 = time.perf_counter()
        oracle.ceemdan(it.X, M, N, D, K, S, NR, eps, seed, 0)
        dt = time.perf_counter() - t1
        res["cpu_baseline"] = {"value": M * N / dt, "unit": "samples/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one oracle CEEMDAN of the series (NR={NR}), {dt:.2f} s "
                                         "on one thread"}
    return res


def run_serving(args, semd, torch, workloads):
    """Poisson arrivals of the serving mix: the continuous-batching engine
    against the plain per-request path.  With --sweep: the saturation rate
    (every request queued at once, engine), then Poisson arrivals at 0.05
    (light load), 0.25, 0.5, 0.75 and 0.9 of it, each point served by both."""
    from paper_2106_15319_amd import serving

    dev = torch.device("cuda:0")
    S, D = 10, 0
    nreq = args.requests
    reqs, kinds = [], []
    for i in range(nreq):
        kind, it = workloads.serving_request(i)
        K = 6 if kind == "series" else 8
        x = torch.from_numpy(it.X).to(dev)
        out = torch.empty((K + 1, it.M * it.N), dtype=torch.float64, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        reqs.append(serving.Request(x, (it.M, it.N), out, cnt, D, K, S))
        kinds.append(kind)
    samples = sum(r.dims[0] * r.dims[1] for r in reqs)
    budget = args.budget_gib << 30
    # warm both paths on the first requests
    serving.serve_plain(reqs[:2], [0.0, 0.0], semd.SEMD_PATH_AUTO)
    serving.serve_engine(reqs[:2], [0.0, 0.0], budget, 256)

    def point(qps, with_plain=True):
        rng = np.random.default_rng(2106_15319 + 4)
        if qps > 0:
            arrivals = np.cumsum(rng.exponential(1.0 / qps, size=nreq)).tolist()
        else:  # saturation: every request queued at the start
            arrivals = [0.0] * nreq
        eng = serving.serve_engine(reqs, arrivals, budget, 256)
        r = {"qps": qps,
             "engine": {"req_per_s": nreq / eng["wall"], "samples_per_s": samples / eng["wall"],
                        "wall_s": eng["wall"], "p50_ms": 1e3 * pct(eng["latency"], 50),
                        "p99_ms": 1e3 * pct(eng["latency"], 99), "steps": eng["steps"],
                        "max_resident": eng["max_resident"]}}
        if with_plain:
            plain = serving.serve_plain(reqs, arrivals, semd.SEMD_PATH_AUTO)
            r["plain"] = {"req_per_s": nreq / plain["wall"],
                          "samples_per_s": samples / plain["wall"], "wall_s": plain["wall"],
                          "p50_ms": 1e3 * pct(plain["latency"], 50),
                          "p99_ms": 1e3 * pct(plain["latency"], 99)}
            r["engine_over_plain_throughput"] = plain["wall"] / eng["wall"]
        return r

    res = base_record(args, 0.0, 0.0)
    res["warmup"] = 0
    mix = {k: kinds.count(k) for k in sorted(set(kinds))}
    if args.sweep:
        sat = point(0.0)
        lam = sat["engine"]["req_per_s"]
        # 0.05: light load, below the plain path's own capacity
        fracs = (0.05, 0.25, 0.5, 0.75, 0.9)
        pts = [point(f * lam) for f in fracs]
        for f, q in zip(fracs, pts):
            q["fraction_of_saturation"] = f
        top = pts[-1]
        res["value"] = top["engine"]["samples_per_s"]
        res["ms_per_step"] = 1e3 * top["engine"]["wall_s"] / max(1, top["engine"]["steps"])
        res["steps"] = top["engine"]["steps"]
        res["config"] = {"workload": f"serving mix (60% textures 64-512 px, 30% series 2-16 x "
                                     f"1e3-65536, 10% 1024x1024), {nreq} requests per point, "
                                     "Poisson arrivals at 0.05/0.25/0.5/0.75/0.9 x the "
                                     "engine's saturation rate; value at 0.9",
                         "requests": nreq,
                         "input_samples": samples, "mix": mix}
        res["saturation"] = sat
        res["sweep"] = pts
        res["latency_ms"] = {"p50": top["engine"]["p50_ms"], "p99": top["engine"]["p99_ms"]}
    else:
        q = point(args.qps)
        res["value"] = q["engine"]["samples_per_s"]
        res["ms_per_step"] = 1e3 * q["engine"]["wall_s"] / max(1, q["engine"]["steps"])
        res["steps"] = q["engine"]["steps"]
        res["config"] = {"workload": f"serving mix (60% textures 64-512 px, 30% series 2-16 x "
                                     f"1e3-65536, 10% 1024x1024), {nreq} requests, "
                                     + (f"Poisson arrivals at {args.qps} req/s" if args.qps > 0
                                        else "all queued at the start"), "requests": nreq,
                         "qps": args.qps, "input_samples": samples, "mix": mix}
        res["latency_ms"] = {"p50": q["engine"]["p50_ms"], "p99": q["engine"]["p99_ms"]}
        res["served"] = q["engine"]
        res["plain"] = q["plain"]
    res["roofline"] = None
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 16 for eemd, one pass over its waves; 20 else)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload",
                    choices=["faces", "series", "textures", "eemd", "serving", "dsweep",
                             "ensembles"],
                    default="eemd")
    ap.add_argument("--sd", type=float, default=0.05, help="dsweep: SD stopping threshold")
    ap.add_argument("--batch", type=int, default=1024, help="faces: images per step")
    ap.add_argument("--D", type=int, default=0, help="transition length")
    ap.add_argument("--plain-items", type=int, default=256,
                    help="faces: images timed on the plain path")
    ap.add_argument("--cpu-items", type=int, default=1024,
                    help="faces: images timed with the oracle")
    ap.add_argument("--cpu-samples", type=int, default=1_200_000,
                    help="eemd: input samples of the oracle's random series sample")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests")
    ap.add_argument("--repeats", type=int, default=1000,
                    help="series: decompositions timed one by one (latency percentiles)")
    ap.add_argument("--qps", type=float, default=40.0,
                    help="serving: arrival rate (0: all requests queued at the start)")
    ap.add_argument("--budget-gib", type=int, default=32, help="serving: engine HBM budget")
    ap.add_argument("--sweep", action="store_true",
                    help="serving: saturation, then 0.25/0.5/0.75/0.9 of it")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--path", choices=["auto", "onchip", "stream"], default="auto",
                    help="faces: execution path of the batched decomposition")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 16 if args.workload == "eemd" else 20
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the independent "
              "signals of a batch would shard across GPUs with no exchange", file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe, max(1, args.steps))

    import torch

    import paper_2106_15319_amd as semd
    import workloads

    assert torch.cuda.is_available(), "bench.py needs the HIP device"
    torch.cuda.set_device(0)
    run = {"faces": run_faces, "series": run_series, "textures": run_textures,
           "eemd": run_eemd, "serving": run_serving, "dsweep": run_dsweep,
           "ensembles": run_ensembles}[args.workload]
    res = run(args, semd, torch, workloads)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
