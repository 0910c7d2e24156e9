"""Benchmark of the RLWE-PIR first-dimension scan on one MI355X.

One step = one pass of the whole online hot path over one batch of queries,
with the database and the queries already resident in HBM: forward NTT of
the queries, their transposition into scan tiles, the database scan, the
answer transposition and the inverse NTT (pir_answer_batch).

Metric: DB-scan GB/s = raw database bytes (R*C*N, one byte per plaintext
coefficient) x queries / wall time, decimal GB.

Default workload (the headline): N=2048, two 28-bit primes, a 4096 x 2048
database (16 GiB raw, 128 GiB NTT form).  The timed steps are batches of
128 queries in one call; beside them the same database answers one query
per call (B=1), and the continuous-batching server runs Poisson arrivals
for p50/p99 latency.  The roofline object covers the batched scan kernel
(int8 matrix-core bound); `batch1_config` holds the batch-1 scan of the
512 x 256 database (256 MiB raw), which is HBM-bound.  Kernel times come
from HIP events the scan launch records itself, on the launch stream,
inside the timed region.  The CPU baseline times the oracle on a bounded
sample of the same workload on this host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "DB-scan GB/s (raw DB bytes×queries/s), batched vs B=1; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0   # dense int8 matrix-core peak of MI355X (TOP/s)
LIMB_MACS = 16            # int8 MACs per modular MAC: 4 x 4 seven-bit limbs

# headline: batched and batch-1 scans and serving on the 16 GiB-raw database
HEADLINE = dict(log2n=11, K=2, R=4096, C=2048, B=128, pool=16, max_batch=128, n_chunks=64,
                rates=[100, 500, 2000])

WORKLOADS = {
    # name: (log2n, K, R, C, B)
    "batch1": (11, 2, 512, 256, 1),
    "batched": (11, 2, 2048, 1024, 32),
    "batched_b1": (11, 2, 2048, 1024, 1),
    "tiny": (10, 1, 16, 16, 1),
}
# serving: device-resident 16 GiB raw database, Poisson arrivals
SERVE = dict(log2n=11, K=2, R=4096, C=2048, max_batch=128, n_chunks=64, pool=16,
             rates=[50, 100, 200, 500, 1000, 2000])
# answer drain with modulus switching: the answers of one batch of 32 queries over
# 1024 columns (32 x 1024 x 2 polynomials), switched to 2^29
DRAIN = dict(log2n=11, K=2, polys=32 * 1024 * 2, bits=29)
# scalar-HE database GEMM mod 2^32: D1 x D0 int8 database (16 GiB, the paper's
# D0 = 65536 words per query), one query and a batch of 32
SCALAR = dict(D1=1 << 18, D0=1 << 16, batches=[1, 16, 32])
# ring packing of the scalar GEMM's answers: D1 LWE ciphertexts per client
# (the 2^18 rows of the 16 GiB scalar database), LWE dimension n = 1280,
# packed into RLWE ciphertexts of N = 4096 under two primes, p = 2^18
PACK = dict(log2n=12, K=2, D1=1 << 18, n=1280, p_log2=18, B=32)
# query expansion of ExpPack (one ciphertext per client expanded into the n = 1280
# special ciphertexts of ring packing, N = 4096, two primes, gadget 2^14 x 4 digits)
# and RGSW folding of D = 2^8 ciphertexts per client (the paper's log2 D_r = 8 rounds)
EXPAND = dict(log2n=12, K=2, n=1280, B=32, base_log=14, n_digits=4, fold_L=8)
# three databases of uneven shape in one batch: (log2n, K, R, C)
MULTIDB = [(12, 2, 1024, 512), (11, 2, 3000, 700), (11, 2, 256, 4096)]


KERNEL_SOURCES = ["paper_2606_11536_amd/csrc/scan.hip", "paper_2606_11536_amd/csrc/device_util.h",
                  "paper_2606_11536_amd/csrc/pir_internal.h"]


def _profile_entry(kernel: str, workload: str):
    """The entry of profiles/traffic.json for (kernel, workload), or None if absent or
    if the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        entries = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["entries"]
    except (OSError, ValueError, KeyError):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    for e in entries:
        if e["kernel"] == kernel and e["workload"] == workload and e["source_sha256"] == h.hexdigest():
            return e
    return None


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter runs (None if stale or absent)."""
    e = _profile_entry(kernel, workload)
    return e.get("bytes_per_launch") if e else None


def measured_mfma(kernel: str, workload: str):
    """Matrix-core busy fraction from the committed counter runs (None if stale or absent)."""
    e = _profile_entry(kernel, workload)
    return e.get("mfma") if e else None


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def scan_alg_bytes(log2n, K, R, C, B) -> int:
    """Algorithmic HBM bytes of one scan launch: NTT-form DB once, B queries, B answers."""
    N = 1 << log2n
    return R * C * N * K * 4 + B * R * 2 * N * K * 4 + B * C * 2 * N * K * 4


def scan_mod_macs(log2n, K, R, C, B) -> int:
    """Modular multiply-adds of one scan: R x C x 2B per (prime, slot)."""
    return R * C * 2 * B * K * (1 << log2n)


def hbm_roofline(kernel, log2n, K, R, C, B, avg_ms, traffic=None) -> dict:
    alg = scan_alg_bytes(log2n, K, R, C, B)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": alg, "avg_launch_ms": round(avg_ms, 5)}


def mfma_roofline(kernel, log2n, K, R, C, B, avg_ms, traffic=None, mfma_busy=None) -> dict:
    """The batched scan against the int8 matrix-core peak: each modular MAC is
    LIMB_MACS int8 MACs (2 ops each) on the matrix cores; beside it the same
    launch's algorithmic HBM rate."""
    macs = scan_mod_macs(log2n, K, R, C, B)
    ops = 2 * LIMB_MACS * macs
    tops = ops / (avg_ms * 1e-3) / 1e12
    alg = scan_alg_bytes(log2n, K, R, C, B)
    gbs = alg / (avg_ms * 1e-3) / 1e9
    return {"bound": "mfma", "kernel": kernel, "achieved": round(tops, 2), "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s (int8)", "frac": round(tops / INT8_PEAK_TOPS, 4), "traffic": traffic,
            "int8_ops_per_launch": ops, "mod_macs_per_launch": macs,
            "ops_what": f"{LIMB_MACS} int8 MACs (4 x 4 seven-bit limbs) per modular MAC, 2 ops per MAC",
            "mfma_busy": mfma_busy,
            "hbm": {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": alg},
            "avg_launch_ms": round(avg_ms, 5)}


def _oracle_sample(log2n, K, R, cs, primes, seed, min_s, max_reps):
    """One process: the oracle's NTT of one query, its scan over ``cs`` database
    columns and their INTT, repeated until ``min_s`` seconds.  Returns
    (seconds in the NTT, seconds in scan + INTT, repetitions)."""
    from oracle import params as op
    from oracle import scan as osc
    N = 1 << log2n
    psis = [op.psi_min(N, q) for q in primes]
    rng = np.random.default_rng(seed)
    query = np.stack([rng.integers(0, q, size=(1, R, 2, N), dtype=np.uint64) for q in primes], axis=3)
    # the oracle scan's work does not depend on values: NTT-form database columns drawn uniform
    d_hat = np.stack([rng.integers(0, q, size=(R, cs, N), dtype=np.uint64) for q in primes])
    t_ntt = t_scan = 0.0
    reps = 0
    while t_ntt + t_scan < min_s and reps < max_reps:
        t0 = time.perf_counter()
        q_hat = osc.query_ntt(query, primes, psis)
        t1 = time.perf_counter()
        y = osc.db_mul(d_hat, q_hat, primes)
        osc.answer_intt(y, primes, psis)
        t2 = time.perf_counter()
        t_ntt += t1 - t0
        t_scan += t2 - t1
        reps += 1
    return t_ntt, t_scan, reps


def _oracle_sample_star(a):
    return _oracle_sample(*a)


def host_description() -> tuple[int, str]:
    """(usable host cores, CPU model name)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(log2n, K, R, C, primes, seed, min_s: float = 10.0) -> dict:
    """Time the oracle on a bounded sample of one query of the workload.

    The sample is the oracle's forward NTT of one query, its scan over a block
    of database columns (all rows, all slots, all primes) and the INTT of those
    answers, repeated until at least ``min_s`` seconds have been measured, on
    one core.  Scan and INTT time scale linearly in the number of columns.
    Beside it, the same sample (a quarter of the columns each) runs in one
    process per usable host core at once, for the all-core rate.
    """
    import multiprocessing as mp
    N = 1 << log2n
    cs = min(C, max(8, (128 * 512 * 2048) // (R * N)))
    t_ntt, t_scan, reps = _oracle_sample(log2n, K, R, cs, primes, seed, min_s, 64)
    per_query = (t_ntt + (C / cs) * t_scan) / reps
    value = R * C * N / per_query / 1e9
    host_cores, model = host_description()
    P = max(1, min(host_cores, 16))
    cs_all = max(1, cs // 4)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(P) as pool:
        res = pool.map(_oracle_sample_star,
                       [(log2n, K, R, cs_all, primes, seed + 1 + p, min_s, reps) for p in range(P)])
    wall = time.perf_counter() - t0
    # the workers ran concurrently: each one's per-query time (NTT plus the
    # scan and INTT scaled to all C columns) is its rate on a loaded host, and
    # the all-core rate is their sum
    value_all = sum(R * C * N / ((tn + (C / cs_all) * ts) / r) / 1e9 for tn, ts, r in res)
    par = sum(tn + ts for tn, ts, _ in res) / wall  # processes busy on average
    return {"value": round(value, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle forward NTT of one query ({R*2*K} polys), its scan over {cs} of "
                       f"{C} columns (all {R} rows, {N} slots, {K} primes) and their INTT, "
                       f"{reps}x in {t_ntt + t_scan:.1f} s on one core; scan+INTT scaled by "
                       f"{C}/{cs}: {per_query*1e3:.1f} ms/query"),
            "queries_per_s": round(1.0 / per_query, 6),
            "host": {"cores": host_cores, "cpu": model},
            "all_cores": {"value": round(value_all, 6), "unit": "GB/s", "cores": P,
                          "sample": (f"the same sample over {cs_all} columns in {P} processes at "
                                     f"once, {wall:.1f} s wall, {par:.1f} processes busy on "
                                     f"average")}}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain device-to-device copy of known size, for scaling HBM byte counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "reps": reps}), flush=True)


SATURATION_WHAT = ("completions per second while requests were waiting for a slot, at the "
                   "highest offered rate that built a backlog (else the highest achieved rate)")


def saturation(results):
    """The server's saturation throughput from a rate sweep (see SATURATION_WHAT)."""
    backlogged = [r["backlogged_qps"] for r in results if r.get("backlogged_qps")]
    if backlogged:
        return max(backlogged)
    return max([r["achieved_qps"] for r in results] or [float("nan")])


def serve_rates(pir, ctx, db, pool, max_batch, n_chunks, rates, args):
    """Poisson arrivals at each rate against a continuous-batching server; the
    pool's queries are submitted round-robin.  Latency runs from a request's
    arrival to its completion event."""
    import collections

    import torch
    if not rates:
        return [], max_batch
    C, K, N = db.C, db.params.K, db.params.N
    dev = torch.device("cuda:0")
    srv = pir.Server(ctx, db, max_batch, n_chunks)
    n_out = srv.info()["max_batch"] + 64
    outs = [torch.empty((C, 2, K, N), dtype=torch.int32, device=dev) for _ in range(n_out)]
    results = []
    for lam in rates:
        n_req = int(max(100, min(lam * args.serve_seconds, args.serve_max_requests)))
        arr = synth.poisson_arrivals(args.seed, float(lam), n_req)
        free = collections.deque(range(n_out))
        waiting, inflight, lat, batch = collections.deque(), {}, [], []
        events = collections.deque()
        i_next, steps = 0, 0
        backlog = []  # (time, completions so far) at every pass with requests left waiting
        t0 = time.perf_counter()
        while len(lat) < n_req:
            now = time.perf_counter() - t0
            while i_next < n_req and arr[i_next] <= now:
                waiting.append((i_next, arr[i_next]))
                i_next += 1
            while waiting and free:
                rid, ta = waiting.popleft()
                o = free.popleft()
                inflight[srv.submit(pool[rid % len(pool)], outs[o])] = (ta, o)
            if waiting:
                backlog.append((now, len(lat)))
            if inflight:
                if len(events) >= 2:
                    events.popleft().synchronize()
                srv.step()
                steps += 1
                batch.append(srv.info()["active"])
                ev = torch.cuda.Event()
                ev.record()
                events.append(ev)
            elif i_next < n_req:
                time.sleep(max(0.0, min(0.002, arr[i_next] - now)))
            for tk in list(inflight):
                if srv.poll(tk):
                    ta, o = inflight.pop(tk)
                    lat.append(time.perf_counter() - t0 - ta)
                    free.append(o)
        wall = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1e3
        qps = n_req / (wall - arr[0])
        # completions per second while requests were left waiting (every slot busy):
        # the server's own rate, without the ramp-up and the final drain
        steady = None
        if len(backlog) >= 2 and backlog[-1][0] - backlog[0][0] > 0.2:
            steady = round((backlog[-1][1] - backlog[0][1]) / (backlog[-1][0] - backlog[0][0]), 2)
        r = {"offered_qps": lam, "requests": n_req, "achieved_qps": round(qps, 2),
             "backlogged_qps": steady,
             "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
             "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
             "mean_active": round(float(np.mean(batch)) if batch else 0.0, 2),
             "max_active": int(max(batch)) if batch else 0, "steps": steps}
        log(f"[serve] {r}")
        results.append(r)
    mb = srv.info()["max_batch"]
    srv.close()
    del outs
    return results, mb


def load_db(pir, ctx, log2n, K, R, C, seed, parallel=True):
    """The seeded synthetic database, lifted, transformed and tiled on the device."""
    N = 1 << log2n
    primes = pir.find_primes(log2n, K, 28)
    t = time.perf_counter()
    raw = (synth.db_bytes_parallel if parallel else synth.db_bytes)(seed, R, C, N)
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    db = ctx.load_db(pir.Params(log2n, primes, 8), raw, R, C)
    load_s = time.perf_counter() - t
    del raw
    log(f"[bench] database N={N} {R}x{C}: generated in {gen_s:.1f} s, loaded (lift+NTT+tiling) "
        f"in {load_s:.2f} s, {db.device_bytes / 2**30:.2f} GiB NTT form")
    return db, primes, load_s


def time_steps(ctx, jobs, steps, warmup, stage_pass=True):
    """Warm up, then time `steps` calls of answer_batch(jobs) with only the scan's
    launch-recorded events on; then a separate pass with every stage timed."""
    import torch
    for _ in range(warmup):
        ctx.answer_batch(jobs)
    torch.cuda.synchronize()
    ctx.profile(True, stages=("scan",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.answer_batch(jobs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    scan_ms, scan_n = ctx.profile_read("scan")
    stage = None
    if stage_pass:
        ctx.profile(True)
        calls = max(1, min(steps, 5))
        for _ in range(calls):
            ctx.answer_batch(jobs)
        # milliseconds per step (a stage may launch more than once per step)
        stage = {st: ctx.profile_read(st) for st in ("ntt", "pack", "scan", "unpack", "intt")}
        stage = {st: round(v[0] / calls, 5) for st, v in stage.items()}
    ctx.profile(False)
    return wall, scan_ms / max(scan_n, 1), stage


def serve(args) -> dict:
    """Continuous batching on the 16 GiB-raw database under Poisson arrivals."""
    import torch

    from paper_2606_11536_amd import pir
    cfg = SERVE
    log2n, K, R, C = cfg["log2n"], cfg["K"], cfg["R"], cfg["C"]
    N = 1 << log2n
    dev = torch.device("cuda:0")
    ctx = pir.Context(0)
    db, primes, load_s = load_db(pir, ctx, log2n, K, R, C, args.seed)
    pool = [torch.from_numpy(synth.uniform_query_parallel(args.seed, b, R, primes, N).view(np.int32))
            .to(dev) for b in range(cfg["pool"])]
    # batch-1 reference on the same database: one query per pir_answer_batch call
    ans1 = torch.empty((1, C, 2, K, N), dtype=torch.int32, device=dev)
    q1 = pool[0].view(1, R, 2, K, N)
    ctx.tune(db, 1)
    wall, _, _ = time_steps(ctx, [(db, 1, q1, ans1)], 5, 1, stage_pass=False)
    b1_ms = wall * 1e3 / 5
    log(f"[serve] batch-1 pass: {b1_ms:.2f} ms/query")
    results, mb = serve_rates(pir, ctx, db, pool, cfg["max_batch"], cfg["n_chunks"], cfg["rates"],
                              args)
    best = saturation(results)
    raw_bytes = R * C * N
    out = {
        "metric": METRIC, "value": round(raw_bytes * best / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": sum(r["steps"] for r in results), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": (f"serving: N={N}, {K} primes < 2^28, p=2^8, device-resident DB "
                                f"R={R} x C={C} ({raw_bytes / 2**30:.0f} GiB raw, "
                                f"{db.device_bytes / 2**30:.0f} GiB NTT form), Poisson arrivals, "
                                f"continuous batching up to {mb} queries, "
                                f"{cfg['n_chunks']} slot ranges per lap, pool of {cfg['pool']} "
                                f"uniform ciphertext-shaped queries"),
                   "N": N, "primes": primes, "R": R, "C": C, "db_load_s": round(load_s, 2)},
        "serving": results,
        "saturation_qps": best,
        "saturation_what": SATURATION_WHAT,
        "batch1_ms_per_query": round(b1_ms, 3),
        "batch1_qps": round(1e3 / b1_ms, 2),
        "speedup_vs_batch1": round(best * b1_ms / 1e3, 2),
    }
    db.free()
    ctx.close()
    return out


def headline(args, cpu) -> dict:
    """Batched (B=128) and batch-1 scans and serving on the 16 GiB-raw database,
    plus the batch-1 scan of the 512 x 256 database for its HBM roofline."""
    import torch

    from paper_2606_11536_amd import pir
    cfg = HEADLINE
    log2n, K, R, C, B = cfg["log2n"], cfg["K"], cfg["R"], cfg["C"], cfg["B"]
    N = 1 << log2n
    dev = torch.device("cuda:0")
    ctx = pir.Context(0)
    db, primes, load_s = load_db(pir, ctx, log2n, K, R, C, args.seed)
    t = time.perf_counter()
    pool = [torch.from_numpy(synth.uniform_query_parallel(args.seed, b, R, primes, N).view(np.int32))
            .to(dev) for b in range(cfg["pool"])]
    log(f"[bench] {len(pool)} ciphertext-shaped queries drawn in {time.perf_counter() - t:.1f} s")
    raw_bytes = R * C * N

    # batched: B queries per call (the pool repeated), every one computed separately
    qb = torch.empty((B, R, 2, K, N), dtype=torch.int32, device=dev)
    for b in range(B):
        qb[b].copy_(pool[b % len(pool)])
    ansb = torch.empty((B, C, 2, K, N), dtype=torch.int32, device=dev)
    tune_b = None if args.no_tune else ctx.tune(db, B)
    log(f"[bench] tuned B={B}: {tune_b}")
    wall, scan_b_ms, stage = time_steps(ctx, [(db, B, qb, ansb)], args.steps, args.warmup)
    ms_b = wall * 1e3 / args.steps
    value = raw_bytes * B * args.steps / wall / 1e9
    kernel_b = ctx.scan_kernel(db, B)
    log(f"[bench] B={B}: {ms_b:.3f} ms/step, scan {scan_b_ms:.3f} ms, {value:.1f} GB/s raw")
    del qb, ansb
    torch.cuda.empty_cache()

    # batch-1 on the same database
    q1 = pool[0].view(1, R, 2, K, N)
    ans1 = torch.empty((1, C, 2, K, N), dtype=torch.int32, device=dev)
    tune_1 = None if args.no_tune else ctx.tune(db, 1)
    n1 = max(10, args.steps)
    wall1, scan_1_ms, stage1 = time_steps(ctx, [(db, 1, q1, ans1)], n1, max(1, args.warmup))
    ms_1 = wall1 * 1e3 / n1
    value_1 = raw_bytes * n1 / wall1 / 1e9
    kernel_1 = ctx.scan_kernel(db, 1)
    log(f"[bench] B=1: {ms_1:.3f} ms/query, scan {scan_1_ms:.3f} ms, {value_1:.1f} GB/s raw")
    del ans1

    # serving: continuous batching under Poisson arrivals
    serving, mb = serve_rates(pir, ctx, db, pool, cfg["max_batch"], cfg["n_chunks"],
                              [] if args.no_serving else cfg["rates"], args)
    sat = saturation(serving)
    del pool
    db_bytes = db.device_bytes
    db.free()
    torch.cuda.empty_cache()

    # the batch-1 scan of the 512 x 256 database: the HBM-bound kernel
    b1c = scan_workload(pir, ctx, "batch1", args)
    ctx.close()

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched scan of a 16 GiB-raw database: N={N}, {K} primes < 2^28, p=2^8, "
                         f"DB R={R} x C={C} ({raw_bytes / 2**30:.0f} GiB raw, "
                         f"{db_bytes / 2**30:.0f} GiB NTT form), B={B} uniform ciphertext-shaped "
                         f"queries per step (NTT, pack, scan, unpack, INTT); B=1 and "
                         f"continuous-batching serving on the same database"),
            "N": N, "primes": primes, "R": R, "C": C, "B": B,
            "raw_db_bytes": raw_bytes, "ntt_db_bytes": db_bytes, "db_load_s": round(load_s, 2),
        },
        "queries_per_s": round(B * 1e3 / ms_b, 2),
        "speedup_vs_batch1": round(value / value_1, 2),
        "batch1": {"value": round(value_1, 3), "unit": "GB/s", "ms_per_query": round(ms_1, 4),
                   "queries_per_s": round(1e3 / ms_1, 2), "steps": n1, "kernel": kernel_1,
                   "stage_ms": stage1, "scan_tuning": tune_1,
                   "roofline": hbm_roofline(kernel_1, log2n, K, R, C, 1, scan_1_ms,
                                            measured_traffic(kernel_1, "headline_b1"))},
        "serving": {"max_batch": mb, "n_chunks": cfg["n_chunks"], "rates": serving,
                    "saturation_qps": sat,
                    "saturation_what": SATURATION_WHAT,
                    "saturation_GBps": round(raw_bytes * sat / 1e9, 3),
                    "speedup_vs_batch1": round(sat * ms_1 / 1e3, 2),
                    "latency_what": "arrival to the completion event of the query's INTT"},
        "latency_ms": ({"p50": serving[0]["p50_ms"], "p99": serving[0]["p99_ms"],
                        "what": f"serving at {serving[0]['offered_qps']} q/s offered"}
                       if serving else None),
        "stage_ms": stage,
        "stage_ms_what": "ms per step, from a separate pass after the timed steps with every stage bracketed by events",
        "scan_tuning": tune_b,
        "roofline": mfma_roofline(kernel_b, log2n, K, R, C, B, scan_b_ms,
                                  measured_traffic(kernel_b, "headline"),
                                  measured_mfma(kernel_b, "headline")),
        "batch1_config": b1c,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    return out


def srv_max(cfg) -> int:
    return cfg["max_batch"]


def drain(args) -> dict:
    """Inverse NTT fused with modulus switching over one batch's answers, against the
    plain inverse NTT of the same residues."""
    import torch

    from paper_2606_11536_amd import pir
    log2n, K, P, bits = DRAIN["log2n"], DRAIN["K"], DRAIN["polys"], DRAIN["bits"]
    N = 1 << log2n
    primes = pir.find_primes(log2n, K, 28)
    params = pir.Params(log2n, primes, 8)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import modswitch as oms
        from oracle import params as op
        psis = [op.psi_min(N, q) for q in op.ntt_primes(N, K)]
        sample = 1024
        rng = np.random.default_rng(args.seed)
        hat = np.stack([rng.integers(0, q, (sample, N), dtype=np.uint64) for q in primes], axis=1)
        t = time.perf_counter()
        oms.intt_switch(hat, op.ntt_primes(N, K), psis, bits)
        sec = time.perf_counter() - t
        cpu = {"value": round(sample * (K + 1) * N * 4 / sec / 1e9, 6), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "sample": f"oracle INTT + switch of {sample} polynomials "
                                           f"({K} primes, N={N}) in {sec:.2f} s on one core"}
    ctx = pir.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(args.seed)
    src = torch.empty((P, K, N), dtype=torch.int32, device="cuda")
    for k, q in enumerate(primes):
        src[:, k].copy_(torch.randint(0, q, (P, N), generator=gen, device="cuda",
                                      dtype=torch.int64).to(torch.int32))
    out = torch.empty((P, N), dtype=torch.int32, device="cuda")
    plain = src.clone()
    for _ in range(args.warmup):
        ctx.intt_modswitch(params, src, out, bits)
    torch.cuda.synchronize()
    ctx.profile(True, stages=("intt",))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.intt_modswitch(params, src, out, bits)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = ctx.profile_read("intt")
    fused_ms = ms / max(n, 1)
    ctx.profile(False)
    # the plain inverse NTT (in place; the values do not affect timing), timed with
    # events on the stream both calls use
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.intt(params, plain)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.steps
    in_b, out_b = P * K * N * 4, P * N * 4
    achieved = (in_b + out_b) / (fused_ms * 1e-3) / 1e9
    res = {
        "metric": "answer drain GB/s (inverse NTT fused with modulus switching to 2^29)",
        "value": round((in_b + out_b) * args.steps / wall / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"answers of one batch of 32 queries x 1024 columns: {P} "
                               f"polynomials, N={N}, {K} primes < 2^28, switched to 2^{bits}",
                   "polys": P, "N": N, "primes": primes, "bits": bits},
        "fused_ms": round(fused_ms, 5), "plain_intt_ms": round(plain_ms, 5),
        "roofline": {"bound": "hbm", "kernel": "k_intt_switch", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_launch": in_b + out_b,
                     "avg_launch_ms": round(fused_ms, 5),
                     "note": "the two inverse NTTs per polynomial are fp64-issue-bound"},
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    ctx.close()
    return res


def scalar(args) -> dict:
    """pir_sdb_mul over a 16 GiB int8 database for one query and for a batch of 32."""
    import torch

    from paper_2606_11536_amd import pir
    D1, D0 = SCALAR["D1"], SCALAR["D0"]
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import scalar as oscl
        rng = np.random.default_rng(args.seed)
        rows = 4096
        dbs = rng.integers(-128, 128, (rows, D0), dtype=np.int64).astype(np.int8)
        qs = rng.integers(0, 1 << 32, (1, D0), dtype=np.uint64).astype(np.uint32)
        t = time.perf_counter()
        reps = 0
        while time.perf_counter() - t < 2.0:
            oscl.db_gemm(dbs, qs)
            reps += 1
        sec = (time.perf_counter() - t) / reps
        cpu = {"value": round(rows * D0 / sec / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "sample": f"oracle GEMM of one query over {rows} rows x {D0} "
                                           f"(int64 numpy product), {reps} runs in 2 s"}
    ctx = pir.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(args.seed)
    raw = torch.randint(-128, 128, (D1, D0), generator=gen, device="cuda", dtype=torch.int8)
    t = time.perf_counter()
    sdb = ctx.load_sdb(raw, D1, D0)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t
    del raw
    torch.cuda.empty_cache()
    runs = []
    for B in SCALAR["batches"]:
        q = torch.randint(-(1 << 31), 1 << 31, (B, D0), generator=gen, device="cuda",
                          dtype=torch.int64).to(torch.int32)
        out = torch.empty((B, D1), dtype=torch.int32, device="cuda")
        for _ in range(args.warmup):
            ctx.sdb_mul(sdb, q, B, out)
        torch.cuda.synchronize()
        ctx.profile(True, stages=("scan",))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.sdb_mul(sdb, q, B, out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, n = ctx.profile_read("scan")
        ctx.profile(False)
        k_ms = ms / max(n, 1)
        alg = D1 * D0 + B * D0 * 4 + B * D1 * 4
        ops = 2 * D1 * D0 * B * 4                     # int8 MACs of the four digit GEMMs, x2
        runs.append({"B": B, "ms_per_step": round(wall * 1e3 / args.steps, 4),
                     "db_GBps": round(D1 * D0 * B * args.steps / wall / 1e9, 2),
                     "queries_per_s": round(B * args.steps / wall, 2),
                     "kernel_ms": round(k_ms, 4),
                     "hbm_frac": round(alg / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "int8_TOPS": round(ops / (k_ms * 1e-3) / 1e12, 1)})
        log(f"[scalar] B={B}: {runs[-1]}")
    one = runs[0]
    res = {
        "metric": "scalar-HE DB GEMM GB/s (int8 DB bytes x queries / s)",
        "value": one["db_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": one["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": f"scalar-HE database GEMM mod 2^32: {D1} x {D0} int8 "
                               f"({D1 * D0 / 2**30:.0f} GiB), uniform uint32 query words",
                   "D1": D1, "D0": D0, "db_load_s": round(load_s, 3)},
        "batches": runs,
        "roofline": {"bound": "hbm", "kernel": "k_sgemm", "achieved": round(
            one["hbm_frac"] * HBM_PEAK_GBS, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": one["hbm_frac"], "traffic": None,
            "alg_bytes_per_launch": D1 * D0 + D0 * 4 + D1 * 4, "avg_launch_ms": one["kernel_ms"]},
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    sdb.free()
    ctx.close()
    return res


def pack(args) -> dict:
    """Ring packing (pir_pack): B clients' D1 LWE ciphertexts each into RLWE ones."""
    import torch

    from paper_2606_11536_amd import pir
    cfg = PACK
    log2n, K, D1, n, plog, B = (cfg[k] for k in ("log2n", "K", "D1", "n", "p_log2", "B"))
    N = 1 << log2n
    Cp = -(-D1 // N)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import pack as opk
        from oracle import params as op
        primes_o = op.ntt_primes(N, K)
        psis = [op.psi_min(N, q) for q in primes_o]
        rows = N                                        # one chunk of one client
        A_s = synth.lwe_matrix(args.seed, rows, n, 1 << plog)
        b_s = synth.lwe_offsets(args.seed, 1, rows, 1 << plog)
        ct_s = synth.uniform_query(args.seed, 0, n, primes_o, N)[None].astype(np.uint64)
        t = time.perf_counter()
        opk.pack(A_s, b_s, ct_s, primes_o, psis, 1 << plog)
        sec = time.perf_counter() - t
        cpu = {"value": round(rows / sec, 2), "unit": "LWE ciphertexts/s", "cores": 1,
               "kind": "oracle",
               "sample": f"oracle packing of one chunk ({rows} LWE ciphertexts, n={n}) of one "
                         f"client through the NTT, in {sec:.2f} s on one core"}
    ctx = pir.Context(0)
    primes = pir.find_primes(log2n, K, 28)
    params = pir.Params(log2n, primes, plog)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device="cuda").manual_seed(args.seed)
    A = torch.randint(0, 1 << plog, (D1, n), generator=gen, device=dev, dtype=torch.int32)
    t = time.perf_counter()
    H = ctx.load_pack(params, A, D1, n)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t
    del A
    torch.cuda.empty_cache()
    sp = torch.empty((B, n, 2, K, N), dtype=torch.int32, device=dev)
    for k, q in enumerate(primes):
        sp[:, :, :, k].copy_(torch.randint(0, q, (B, n, 2, N), generator=gen, device=dev,
                                           dtype=torch.int64).to(torch.int32))
    b = torch.randint(0, 1 << plog, (B, D1), generator=gen, device=dev, dtype=torch.int32)
    out = torch.empty((B, Cp, 2, K, N), dtype=torch.int32, device=dev)
    tune = None if args.no_tune else ctx.tune(H, B)
    for _ in range(args.warmup):
        ctx.pack(H, B, sp, b, out)
    torch.cuda.synchronize()
    ctx.profile(True, stages=("scan",))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.pack(H, B, sp, b, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    scan_ms, scan_n = ctx.profile_read("scan")
    ctx.profile(True)
    calls = max(1, min(args.steps, 5))
    for _ in range(calls):
        ctx.pack(H, B, sp, b, out)
    # milliseconds per step: the NTT stage is the offsets' transform and the
    # special ciphertexts' transform
    stage = {st: ctx.profile_read(st) for st in ("ntt", "pack", "scan", "unpack", "intt")}
    stage = {st: round(v[0] / calls, 5) for st, v in stage.items()}
    ctx.profile(False)
    ms = wall * 1e3 / args.steps
    scan_avg = scan_ms / max(scan_n, 1)
    kernel = ctx.scan_kernel(H, B)
    res = {
        "metric": "ring packing: LWE ciphertexts packed into RLWE ciphertexts per second",
        "value": round(B * D1 / (ms * 1e-3), 1), "unit": "LWE ciphertexts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": (f"ring packing H C + (0|G): D1={D1} LWE ciphertexts per client, "
                                f"n={n}, p=2^{plog}, N={N}, {K} primes < 2^28, {Cp} RLWE "
                                f"ciphertexts per client, B={B} clients (special ciphertexts "
                                f"and offsets uniform)"),
                   "N": N, "primes": primes, "D1": D1, "n": n, "B": B, "chunks": Cp,
                   "hint_load_s": round(load_s, 3)},
        "stage_ms": stage,
        "stage_ms_what": "ms per step, from a separate pass after the timed steps with every stage bracketed by events",
        "scan_tuning": tune,
        "roofline": hbm_roofline(kernel, log2n, K, n, Cp, B, scan_avg,
                                 measured_traffic(kernel, "pack")),
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    H.free()
    ctx.close()
    return res


def expand(args) -> dict:
    """Query expansion (pir_expand) and RGSW folding (pir_fold) of a batch of clients."""
    import torch

    from paper_2606_11536_amd import pir
    cfg = EXPAND
    log2n, K, n, B, bl, nd, L = (cfg[k] for k in ("log2n", "K", "n", "B", "base_log",
                                                   "n_digits", "fold_L"))
    N = 1 << log2n
    levels = max(1, (n - 1).bit_length())
    # key switches per client: every output of every level below n
    n_ks = sum(min(2 << j, n) for j in range(levels))
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import expand as ex
        from oracle import params as op
        qs = op.ntt_primes(N, K)
        psis = [op.psi_min(N, q) for q in qs]
        rng = np.random.default_rng(args.seed)
        ct = np.stack([np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in qs])
                       for _ in range(2)])
        key = np.stack([np.stack([np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in qs])
                                  for _ in range(2)]) for _ in range(nd)])
        reps, t = 0, time.perf_counter()
        while time.perf_counter() - t < 10.0:
            ex.subs(ct, ex.expansion_exponent(N, 0), key, qs, psis, bl)
            reps += 1
        sec = (time.perf_counter() - t) / reps
        cpu = {"value": round(1.0 / (sec * n_ks), 6), "unit": "clients/s", "cores": 1,
               "kind": "oracle",
               "sample": f"oracle key switch (automorphism, {nd} gadget digits, N={N}, {K} "
                         f"primes) x{reps} in {sec * reps:.1f} s on one core, scaled by the "
                         f"{n_ks} key switches of one client's expansion"}
    ctx = pir.Context(0)
    primes = pir.find_primes(log2n, K, 28)
    params = pir.Params(log2n, primes, 8)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device="cuda").manual_seed(args.seed)

    def uniform(shape):
        t = torch.empty(shape + (K, N), dtype=torch.int32, device=dev)
        for k, q in enumerate(primes):
            t[..., k, :].copy_(torch.randint(0, q, shape + (N,), generator=gen, device=dev,
                                             dtype=torch.int64).to(torch.int32))
        return t

    keys = ctx.load_expand_keys(params, uniform((B, levels, nd, 2)), B, levels, bl, nd)
    ct = uniform((B, 2))
    out = torch.empty((B, n, 2, K, N), dtype=torch.int32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        ctx.expand(keys, ct, n, out)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        ctx.expand(keys, ct, n, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    keys.free()
    del out
    torch.cuda.empty_cache()
    D = 1 << L
    cts = uniform((B, D, 2))
    rg = uniform((B, L, 2 * nd, 2))
    fo = torch.empty((B, 2, K, N), dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        ctx.fold(params, cts, D, rg, bl, nd, B, fo)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        ctx.fold(params, cts, D, rg, bl, nd, B, fo)
    e1.record()
    torch.cuda.synchronize()
    fold_ms = e0.elapsed_time(e1) / args.steps
    ctx.close()
    res = {
        "metric": "query expansion: clients expanded per second (n special ciphertexts each)",
        "value": round(B * 1e3 / ms, 2), "unit": "clients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": (f"ExpPack expansion: one RLWE ciphertext per client into n={n} "
                                f"ciphertexts ({levels} levels, {n_ks} key switches per client), "
                                f"N={N}, {K} primes < 2^28, gadget 2^{bl} x {nd} digits, B={B} "
                                f"clients (keys and ciphertexts uniform)"),
                   "N": N, "primes": primes, "n": n, "B": B, "base_log": bl, "n_digits": nd},
        "key_switches_per_s": round(B * n_ks * 1e3 / ms, 1),
        "fold": {"D": D, "rounds": L, "B": B, "ms": round(fold_ms, 4),
                 "clients_per_s": round(B * 1e3 / fold_ms, 2),
                 "external_products_per_s": round(B * (D - 1) * 1e3 / fold_ms, 1)},
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    return res


def multidb(args) -> dict:
    """Three uneven databases, 1..64 queries each, one fused batch, HIP-graph replays."""
    import torch

    from paper_2606_11536_amd import pir
    dev = torch.device("cuda:0")
    ctx = pir.Context(0)
    Bs = [int(b) for b in synth.batch_sizes(args.seed, len(MULTIDB))]
    jobs, desc, raw_total = [], [], 0
    for n, ((log2n, K, R, C), B) in enumerate(zip(MULTIDB, Bs)):
        N = 1 << log2n
        primes = pir.find_primes(log2n, K, 28)
        raw = synth.db_bytes_parallel(args.seed + n, R, C, N)
        db = ctx.load_db(pir.Params(log2n, primes, 8), raw, R, C)
        del raw
        qc = torch.empty((B, R, 2, K, N), dtype=torch.int32, device=dev)
        for b in range(B):
            qc[b] = torch.from_numpy(synth.uniform_query_parallel(args.seed + n, b, R, primes, N)
                                     .view(np.int32)).to(dev)
        ans = torch.empty((B, C, 2, K, N), dtype=torch.int32, device=dev)
        jobs.append((db, B, qc, ans))
        raw_total += R * C * N * B
        desc.append({"N": N, "R": R, "C": C, "B": B, "ntt_db_GiB": round(db.device_bytes / 2**30, 2)})
        log(f"[multidb] db {n}: {desc[-1]}")
    report = ctx.tune_batch(jobs)
    log(f"[multidb] tuned: {report}")
    plan = ctx.plan(jobs)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / args.steps
    # the same batch through pir_answer_batch (host-side launch each time) for comparison
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.answer_batch(jobs)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    plan.close()
    out = {
        "metric": METRIC, "value": round(raw_total / (ms * 1e-3) / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "uneven multi-database batch, HIP-graph replay: " + "; ".join(
            f"N={d['N']} R={d['R']} C={d['C']} B={d['B']}" for d in desc), "databases": desc},
        "queries_per_s": round(sum(Bs) / (ms * 1e-3), 2),
        "eager_ms_per_step": round(eager_ms, 4),
        "scan_tuning": report,
    }
    ctx.close()
    return out


def scan_workload(pir, ctx, name, args) -> dict:
    """One of WORKLOADS through pir_answer_batch on its own database."""
    import torch
    log2n, K, R, C, B = WORKLOADS[name]
    N = 1 << log2n
    dev = torch.device("cuda:0")
    db, primes, load_s = load_db(pir, ctx, log2n, K, R, C, args.seed, parallel=False)
    qc = torch.empty((B, R, 2, K, N), dtype=torch.int32, device=dev)
    for b in range(B):
        qc[b] = torch.from_numpy(synth.uniform_query(args.seed, b, R, primes, N).view(np.int32)).to(dev)
    sb = args.switch_bits
    ans = torch.empty((B, C, 2, N) if sb else (B, C, 2, K, N), dtype=torch.int32, device=dev)
    jobs = [(db, B, qc, ans, sb)]
    tune_report = None
    if not args.no_tune:
        tune_report = ctx.tune(db, B)
        log(f"[bench] tuned scan: {tune_report}")
    wall, scan_avg_ms, stage = time_steps(ctx, jobs, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    raw_bytes = R * C * N
    value = raw_bytes * B * args.steps / wall / 1e9
    log(f"[bench] {name}: timed {args.steps} steps: {ms_per_step:.4f} ms/step")
    lat = []
    for _ in range(args.latency_steps):
        a = time.perf_counter()
        ctx.answer_batch(jobs)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat if lat else [float("nan")])
    kernel = ctx.scan_kernel(db, B)
    roof = (hbm_roofline(kernel, log2n, K, R, C, B, scan_avg_ms, measured_traffic(kernel, name))
            if B == 1 else
            mfma_roofline(kernel, log2n, K, R, C, B, scan_avg_ms, measured_traffic(kernel, name),
                          measured_mfma(kernel, name)))
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"{'batch-1' if B == 1 else 'batched'} scan: N={N}, {K} primes < 2^28, "
                         f"p=2^8, DB R={R} x C={C} ({raw_bytes / 2**20:.0f} MiB raw, "
                         f"{db.device_bytes / 2**30:.2f} GiB NTT form), B={B} uniform "
                         f"ciphertext-shaped queries"
                         + (f", answers switched to 2^{sb}" if sb else "")),
            "N": N, "primes": primes, "R": R, "C": C, "B": B,
            "raw_db_bytes": raw_bytes, "ntt_db_bytes": db.device_bytes,
            "answer_switch_bits": sb,
            "db_load_s": round(load_s, 3),
        },
        "queries_per_s": round(B * args.steps / wall, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "what": "one pir_answer_batch call of B queries, host clock, synchronized"},
        "stage_ms": stage,
        "stage_ms_what": "ms per step, from a separate pass after the timed steps with every stage bracketed by events",
        "scan_tuning": tune_report,
        "roofline": roof,
    }
    db.free()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline",
                    choices=["headline"] + sorted(WORKLOADS) + ["serving", "multidb", "drain",
                                                                "scalar", "pack", "expand"])
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-max-requests", type=int, default=1500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--no-tune", action="store_true", help="use the default scan variant")
    ap.add_argument("--no-serving", action="store_true",
                    help="headline without the serving runs (for short profiled runs)")
    ap.add_argument("--switch-bits", type=int, default=0,
                    help="drain the answers with modulus switching to 2^bits (0: plain INTT)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; run it with --gpus 1"}))
        return 2
    if args.calibrate_copy:
        calibrate_copy()
        return 0
    if args.workload in ("serving", "multidb", "drain", "scalar", "pack", "expand"):
        fn = {"serving": serve, "multidb": multidb, "drain": drain, "scalar": scalar,
              "pack": pack, "expand": expand}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return 0

    if args.workload == "headline":
        log2n, K, R, C = (HEADLINE[k] for k in ("log2n", "K", "R", "C"))
    else:
        log2n, K, R, C, _ = WORKLOADS[args.workload]
    cpu = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the all-core leg forks worker processes
        from oracle import params as op
        log("[bench] timing the CPU oracle on a bounded sample")
        oracle_primes = op.ntt_primes(1 << log2n, K)
        cpu = cpu_baseline(log2n, K, R, C, oracle_primes, args.seed)

    from paper_2606_11536_amd import pir
    if cpu is not None and pir.find_primes(log2n, K, 28) != [int(x) for x in oracle_primes]:
        raise RuntimeError("the oracle's primes differ from the library's")
    if args.workload == "headline":
        out = headline(args, cpu)
    else:
        ctx = pir.Context(0)
        out = scan_workload(pir, ctx, args.workload, args)
        ctx.close()
        if cpu is not None:
            out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
