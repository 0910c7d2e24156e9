"""Benchmark of the RLWE-PIR first-dimension scan on one MI355X.

One step = one pass of the whole online hot path over one batch of queries,
with the database and the queries already resident in HBM:
forward NTT of the queries, their transposition into scan tiles, the
database scan, and the inverse NTT of the answers (pir_answer_batch).

Metric: DB-scan GB/s = raw database bytes (R*C*N, one byte per plaintext
coefficient) x queries / wall time, decimal GB.  The roofline object reports
the scan kernel's algorithmic HBM bytes per launch divided by its average
launch time, measured with HIP events on the launch stream inside the
timed region.  The CPU baseline times the oracle on a bounded sample of the
same workload on this host.

Default workload: N=2048, two 28-bit primes, 512 x 256 database
(256 MiB raw, 2 GiB NTT form), one query per step.
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

WORKLOADS = {
    # name: (log2n, K, R, C, B)
    "batch1": (11, 2, 512, 256, 1),
    "batched": (11, 2, 2048, 1024, 32),
    "batched_b1": (11, 2, 2048, 1024, 1),
    "tiny": (10, 1, 16, 16, 1),
}


KERNEL_SOURCES = ["paper_2606_11536_amd/csrc/scan.hip", "paper_2606_11536_amd/csrc/device_util.h",
                  "paper_2606_11536_amd/csrc/pir_internal.h"]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from profiles/traffic.json, or None if absent or if the
    kernel sources changed since the counters were taken."""
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
            return e["bytes_per_launch"]
    return None


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def scan_alg_bytes(log2n, K, R, C, B) -> int:
    """Algorithmic HBM bytes of one scan launch: NTT-form DB once, B queries, B answers."""
    N = 1 << log2n
    return R * C * N * K * 4 + B * R * 2 * N * K * 4 + B * C * 2 * N * K * 4


def cpu_baseline(log2n, K, R, C, primes, seed, min_s: float = 10.0) -> dict:
    """Time the oracle on a bounded sample of one query of the workload (single core).

    The sample is the oracle's forward NTT of one query, its scan over a block
    of database columns (all rows, all slots, all primes) and the INTT of those
    answers, repeated until at least ``min_s`` seconds have been measured.
    Scan and INTT time scale linearly in the number of columns.
    """
    from oracle import params as op
    from oracle import scan as osc
    N = 1 << log2n
    psis = [op.psi_min(N, q) for q in primes]
    rng = np.random.default_rng(seed)
    cs = min(C, max(8, (128 * 512 * 2048) // (R * N)))
    query = np.stack([rng.integers(0, q, size=(1, R, 2, N), dtype=np.uint64) for q in primes], axis=3)
    # the oracle scan's work does not depend on values: NTT-form database columns drawn uniform
    d_hat = np.stack([rng.integers(0, q, size=(R, cs, N), dtype=np.uint64) for q in primes])
    t_ntt = t_scan = 0.0
    reps = 0
    while t_ntt + t_scan < min_s and reps < 64:
        t0 = time.perf_counter()
        q_hat = osc.query_ntt(query, primes, psis)
        t1 = time.perf_counter()
        y = osc.db_mul(d_hat, q_hat, primes)
        osc.answer_intt(y, primes, psis)
        t2 = time.perf_counter()
        t_ntt += t1 - t0
        t_scan += t2 - t1
        reps += 1
    per_query = (t_ntt + (C / cs) * t_scan) / reps
    value = R * C * N / per_query / 1e9
    return {"value": round(value, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle forward NTT of one query ({R*2*K} polys), its scan over {cs} of "
                       f"{C} columns (all {R} rows, {N} slots, {K} primes) and their INTT, "
                       f"{reps}x in {t_ntt + t_scan:.1f} s; scan+INTT scaled by {C}/{cs}: "
                       f"{per_query*1e3:.1f} ms/query"),
            "queries_per_s": round(1.0 / per_query, 6)}


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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch1", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--no-tune", action="store_true", help="use the default scan variant")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        return 2
    if args.calibrate_copy:
        calibrate_copy()
        return 0

    import torch

    from paper_2606_11536_amd import pir

    log2n, K, R, C, B = WORKLOADS[args.workload]
    N = 1 << log2n
    primes = pir.find_primes(log2n, K, 28)
    params = pir.Params(log2n, primes, 8)
    dev = torch.device("cuda:0")

    log(f"[bench] workload={args.workload} N={N} K={K} R={R} C={C} B={B}")
    t = time.perf_counter()
    raw = synth.db_bytes(args.seed, R, C, N)
    log(f"[bench] database generated in {time.perf_counter() - t:.1f} s")
    ctx = pir.Context(0)
    t = time.perf_counter()
    db = ctx.load_db(params, raw, R, C)
    load_s = time.perf_counter() - t
    del raw
    log(f"[bench] database loaded (lift+NTT+tiling) in {load_s:.2f} s")
    qc = torch.empty((B, R, 2, K, N), dtype=torch.int32, device=dev)
    for b in range(B):
        qc[b] = torch.from_numpy(synth.uniform_query(args.seed, b, R, primes, N).view(np.int32)).to(dev)
    ans = torch.empty((B, C, 2, K, N), dtype=torch.int32, device=dev)
    jobs = [(db, B, qc, ans)]
    tune_report = None
    if not args.no_tune:
        tune_report = ctx.tune(db, B)
        log(f"[bench] tuned scan: {tune_report}")

    for _ in range(args.warmup):
        ctx.answer_batch(jobs)
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.answer_batch(jobs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage = {s: ctx.profile_read(s) for s in ("ntt", "pack", "scan", "intt")}
    ctx.profile(False)
    wall = t1 - t0
    ms_per_step = wall * 1e3 / args.steps
    raw_bytes = R * C * N
    value = raw_bytes * B * args.steps / wall / 1e9
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step")

    lat = []
    for _ in range(args.latency_steps):
        a = time.perf_counter()
        ctx.answer_batch(jobs)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat if lat else [float("nan")])

    scan_ms, scan_n = stage["scan"]
    scan_avg_ms = scan_ms / max(scan_n, 1)
    alg = scan_alg_bytes(log2n, K, R, C, B)
    achieved = alg / (scan_avg_ms * 1e-3) / 1e9
    kernel = "k_scan_b1" if B == 1 else "k_scan_mfma"
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
                         f"ciphertext-shaped queries"),
            "N": N, "primes": primes, "R": R, "C": C, "B": B,
            "raw_db_bytes": raw_bytes, "ntt_db_bytes": db.device_bytes,
            "db_load_s": round(load_s, 3),
        },
        "queries_per_s": round(B * args.steps / wall, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "what": "one pir_answer_batch call of B queries, host clock, synchronized"},
        "stage_ms": {s: round(v[0] / max(v[1], 1), 5) for s, v in stage.items()},
        "scan_tuning": tune_report,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kernel, args.workload),
            "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(scan_avg_ms, 5),
        },
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(log2n, K, R, C, primes, args.seed)
    print(json.dumps(out), flush=True)
    db.free()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
