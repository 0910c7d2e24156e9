"""GPU parity at the full sizes of the serving and multi-database workloads.

Serving: N=2048, two primes, a 4096 x 2048 database (16 GiB raw, 128 GiB
NTT form) behind the continuous-batching server with 128 column slots and 64
slot ranges per lap -- the server bench.py times.  Queries join at staggered
steps so that laps run with up to 48 queries (96 columns) active.

Multi-database: the three uneven databases bench.py times -- (N=4096,
1024 x 512), (N=2048, 3000 x 700), (N=2048, 256 x 4096) -- with the seeded
batch sizes (30, 57, 14), fused into one job list and replayed from a HIP
graph.

The oracle cannot recompute these answers in full, so every answer is checked
three ways (bigcheck.Expected):
* 18 sampled columns (always 0 and C-1), every slot, both primes, exactly;
* two Freivalds draws per prime over the whole answer (a wrong answer passes
  one draw with probability at most 1/q < 2^-27);
* encrypted one-hot queries decrypt, on the sampled columns, to their row.
Each batch cycles through a small pool of distinct queries (encrypted ones
and a uniform ciphertext-shaped one); every submitted query's answer is
computed separately on the GPU and checked against its pool member's
expectation.  Serving also checks one query's answer alone == in the mix.
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from oracle import query as oq

from bigcheck import Expected
from pirtest import empty_dev, ring, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pool(seed, R, rg, n_enc):
    """n_enc encrypted one-hot queries (rows from synth.indices, the last one
    forced to R - 1) and one uniform ciphertext-shaped query."""
    idx = synth.indices(seed, n_enc, R)
    idx[-1] = R - 1

    def enc(b):
        return oq.onehot_query(seed, b, int(idx[b]), R, rg.primes, rg.psis, rg.delta, rg.N)

    with ThreadPoolExecutor(n_enc) as ex:
        cts = list(ex.map(enc, range(n_enc)))
    unif = synth.uniform_query_parallel(seed, 0, R, rg.primes, rg.N).astype(np.uint64)
    pool = np.stack([c for c, _ in cts] + [unif])
    return pool, idx, [s for _, s in cts]


# ---------------------------------------------------------------- serving --
SERVE_SEED, SR, SC, MAXB, NCH = 41, 4096, 2048, 128, 64


@pytest.fixture(scope="module")
def serving():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    rg = ring(11, 2)
    print(f"[serving] generating the {SR}x{SC} database", flush=True)
    raw = synth.db_bytes_parallel(SERVE_SEED, SR, SC, rg.N)
    ctx = pir.Context(0)
    db = ctx.load_db(rg.pir_params(), raw, SR, SC)
    print("[serving] database loaded; oracle expectations", flush=True)
    pool, idx, secrets = _pool(SERVE_SEED, SR, rg, 3)
    exp = Expected(rg, raw, pool, SERVE_SEED)
    yield pir, ctx, db, rg, raw, pool, idx, secrets, exp
    ctx.close()
    torch.cuda.empty_cache()


def _serve(pir, srv, schedule, dev_pool, shape, max_steps=400):
    """schedule: {step: [pool member, ...]}; returns [(member, answer tensor)] in
    submission order once every query has finished."""
    import torch
    subs, tickets = [], {}
    last = max(schedule)
    for step in range(max_steps):
        for m in schedule.get(step, []):
            out = empty_dev(shape)
            tickets[srv.submit(dev_pool[m], out)] = len(subs)
            subs.append((m, out))
        srv.step()
        torch.cuda.synchronize()
        for t in [t for t in tickets if srv.poll(t)]:
            tickets.pop(t)
        if not tickets and step >= last:
            return subs
    raise AssertionError("queries did not finish")


def test_serving_full_size(serving):
    pir, ctx, db, rg, raw, pool, idx, secrets, exp = serving
    srv = pir.Server(ctx, db, MAXB, NCH)
    assert srv.info()["max_batch"] == MAXB
    dev_pool = [to_dev(p) for p in pool]
    shape = (SC, 2, rg.K, rg.N)
    print("[serving] one query alone", flush=True)
    alone = to_host(_serve(pir, srv, {0: [0]}, dev_pool, shape)[0][1])
    exp.check(alone, 0)
    exp.decrypts(alone, secrets[0], raw, int(idx[0]))
    # 48 queries: 16 at step 0, 16 at step 3 and 16 at step 20 (mid-lap), so
    # the laps from step 20 on run with 48 queries in column slots 0..47
    members = list(range(len(pool)))
    schedule = {0: (members * 4)[:16], 3: (members[1:] + members[:1]) * 4, 20: members[::-1] * 4}
    print("[serving] 48 staggered queries", flush=True)
    subs = _serve(pir, srv, schedule, dev_pool, shape)
    assert len(subs) == 48
    first0 = next(n for n, (m, _) in enumerate(subs) if m == 0)
    for n, (m, out) in enumerate(subs):
        a = to_host(out)
        exp.check(a, m)
        if m < len(secrets):
            exp.decrypts(a, secrets[m], raw, int(idx[m]))
        if n == first0:
            assert np.array_equal(a, alone), "answer in the mix differs from the answer alone"
    assert srv.info()["active"] == 0 and srv.info()["queued"] == 0
    srv.close()


# ----------------------------------------------------------- multi-database --
MULTI_SEED = 0
MULTIDB = [(12, 2, 1024, 512), (11, 2, 3000, 700), (11, 2, 256, 4096)]


def test_multidb_graph_full_size():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    Bs = [int(b) for b in synth.batch_sizes(MULTI_SEED, len(MULTIDB))]
    assert Bs == [30, 57, 14]
    ctx = pir.Context(0)
    try:
        jobs, checks = [], []
        for n, ((log2n, K, R, C), B) in enumerate(zip(MULTIDB, Bs)):
            rg = ring(log2n, K)
            print(f"[multidb] database {n}: N={rg.N} {R}x{C}, B={B}", flush=True)
            raw = synth.db_bytes_parallel(MULTI_SEED + n, R, C, rg.N)
            db = ctx.load_db(rg.pir_params(), raw, R, C)
            pool, idx, secrets = _pool(MULTI_SEED + 100 + n, R, rg, 2)
            exp = Expected(rg, raw, pool, MULTI_SEED + n)
            qd = torch.empty((B, R, 2, K, rg.N), dtype=torch.int32, device="cuda")
            dev_pool = [to_dev(p) for p in pool]
            for b in range(B):
                qd[b].copy_(dev_pool[b % len(pool)])
            ans = empty_dev((B, C, 2, K, rg.N))
            jobs.append((db, B, qd, ans))
            checks.append((rg, raw, pool, idx, secrets, exp))
        ctx.tune_batch(jobs)
        plan = ctx.plan(jobs)

        def check_all():
            for (db, B, qd, ans), (rg, raw, pool, idx, secrets, exp) in zip(jobs, checks):
                for b in range(B):
                    m = b % len(pool)
                    a = to_host(ans[b])
                    exp.check(a, m)
                    if m < len(secrets):
                        exp.decrypts(a, secrets[m], raw, int(idx[m]))

        plan.launch()
        torch.cuda.synchronize()
        print("[multidb] checking the first replay", flush=True)
        check_all()
        # eager work between replays, answers overwritten, then a second replay
        for (_, _, _, ans) in jobs:
            ans.fill_(-1)
        ctx.answer_batch([jobs[2][:1] + (1, jobs[2][2][:1], empty_dev((1,) + tuple(jobs[2][3].shape[1:])))])
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        print("[multidb] checking the second replay", flush=True)
        check_all()
        plan.close()
    finally:
        ctx.close()
        torch.cuda.empty_cache()
