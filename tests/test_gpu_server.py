"""GPU tests of the continuous-batching server (pir_server_*).

* a query's answer is the same bytes alone and in a staggered mix where
  others join at different steps, and equals the oracle's;
* more queries than column slots wait in the queue and are admitted as slots
  free; every answer is still exact;
* the HBM budget lowers the admission limit, and a budget too small for one
  query is refused with PIR_ERR_BUDGET.
"""

import numpy as np
import pytest

import synth
from oracle import query as oq
from oracle import scan as osc

from pirtest import empty_dev, onehot_queries, residues, ring, to_dev, to_host

pytestmark = pytest.mark.gpu

LOG2N, K, R, C = 10, 2, 100, 30


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    rg = ring(LOG2N, K)
    raw = synth.db_bytes(31, R, C, rg.N)
    ctx = pir.Context(0)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    rng = np.random.default_rng(77)
    enc, sec = onehot_queries(31, np.array([17]), R, rg)
    queries = np.concatenate([enc, residues(rng, (7, R, 2), rg)])     # [8][R][2][K][N]
    y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(queries, rg.primes, rg.psis),
                   rg.primes)
    expect = osc.answer_intt(y, rg.primes, rg.psis)                    # [8][C][2][K][N]
    yield pir, ctx, db, rg, raw, queries, expect, sec
    ctx.close()


def run(pir, srv, submit_at, queries, rg, max_steps=200):
    """Submit query q at step submit_at[q]; step until all finish; return answers."""
    outs = {q: empty_dev((C, 2, rg.K, rg.N)) for q in submit_at}
    qd = {q: to_dev(queries[q]) for q in submit_at}
    tickets = {}
    for step in range(max_steps):
        for q, s in submit_at.items():
            if s == step:
                tickets[q] = srv.submit(qd[q], outs[q])
        srv.step()
        done = [q for q, t in tickets.items() if srv.poll(t)]
        for q in done:
            tickets.pop(q)
        if len(tickets) == 0 and step >= max(submit_at.values()):
            break
        if done == []:
            import torch
            torch.cuda.synchronize()
    assert not tickets, "queries did not finish"
    return {q: to_host(o) for q, o in outs.items()}


def test_alone_equals_mixed_equals_oracle(env):
    pir, ctx, db, rg, raw, queries, expect, sec = env
    srv = pir.Server(ctx, db, max_batch=4, n_chunks=5)
    alone = run(pir, srv, {0: 0}, queries, rg)[0]
    assert np.array_equal(alone, expect[0])
    m, _ = oq.decrypt_answers(alone, sec[0], rg.primes, rg.psis, rg.delta, rg.p)
    assert np.array_equal(m, raw[17].astype(np.int64))
    mixed = run(pir, srv, {1: 0, 0: 2, 2: 2, 3: 3, 4: 6}, queries, rg)
    assert np.array_equal(mixed[0], alone)
    for q, a in mixed.items():
        assert np.array_equal(a, expect[q]), f"query {q}"
    srv.close()


def test_queue_beyond_slots(env):
    pir, ctx, db, rg, raw, queries, expect, sec = env
    srv = pir.Server(ctx, db, max_batch=3, n_chunks=4)
    got = run(pir, srv, {q: 0 for q in range(8)}, queries, rg)
    for q, a in got.items():
        assert np.array_equal(a, expect[q]), f"query {q}"
    assert srv.info()["active"] == 0 and srv.info()["queued"] == 0
    srv.close()


def test_single_range_and_one_slot(env):
    pir, ctx, db, rg, raw, queries, expect, sec = env
    srv = pir.Server(ctx, db, max_batch=1, n_chunks=1)
    got = run(pir, srv, {5: 0, 6: 0}, queries, rg)
    assert np.array_equal(got[5], expect[5]) and np.array_equal(got[6], expect[6])
    srv.close()


def test_budget_limits_admission(env):
    pir, ctx, db, rg, raw, queries, expect, sec = env
    n_ib = (R + 63) // 64 * 2
    per_cb = rg.K * rg.N * n_ib * 1024            # query limbs of 4 column slots
    ans = C * 2 * rg.K * rg.N * 4                  # answer state of one slot
    scratch = R * 2 * rg.K * rg.N * 4              # NTT scratch of one admission
    need4 = per_cb + 4 * ans + scratch             # a server of 4 slots
    budget = 1 << 30
    tight = pir.Context(0, hbm_budget_bytes=budget)
    try:
        tdb = tight.load_db(rg.pir_params(), raw, R, C)
        mib = 1 << 20
        tight.reserve((budget - tight.device_bytes - need4 - ans // 2) // mib * mib)
        assert budget - tight.device_bytes >= need4
        srv = pir.Server(tight, tdb, max_batch=64, n_chunks=3)
        assert srv.info()["max_batch"] == 4
        got = run(pir, srv, {q: 0 for q in range(6)}, queries, rg)
        for q, a in got.items():
            assert np.array_equal(a, expect[q])
        srv.close()
        with pytest.raises(pir.PirError) as e:
            tight.reserve(budget + (64 << 20))
        assert e.value.status == 4
    finally:
        tight.close()
    none = pir.Context(0, hbm_budget_bytes=budget)
    try:
        ndb = none.load_db(rg.pir_params(), raw, R, C)
        none.reserve((budget - none.device_bytes - scratch) // (1 << 20) * (1 << 20))
        with pytest.raises(pir.PirError) as e:
            pir.Server(none, ndb, max_batch=4, n_chunks=3)
        assert e.value.status == 4
    finally:
        none.close()


def test_ragged_range_count(env):
    # 700 ranges over K N = 2048 slots (2 or 3 slots each; more ranges than
    # sqrt(K N)): every query still meets every slot once, also query 4, which
    # joins mid-lap at step 350 and finishes at step 1049
    pir, ctx, db, rg, raw, queries, expect, sec = env
    srv = pir.Server(ctx, db, max_batch=3, n_chunks=700)
    got = run(pir, srv, {0: 0, 3: 0, 4: 350}, queries, rg, max_steps=1200)
    for q, a in got.items():
        assert np.array_equal(a, expect[q]), f"query {q}"
    srv.close()
