"""GPU parity at full workload sizes (the shapes bench.py times).

Batched workload: N=2048, two primes, 2048 x 1024 database (4 GiB raw,
32 GiB NTT form), B=32 in one call, and B=1 on the same database.  The
oracle cannot recompute 32 GiB of NTT-form products, so every answer is
checked through properties that hold at any size and through sampled
outputs the oracle computes one by one:

* 10 columns (always 0 and C-1) exactly, all slots, both primes, every query;
* two Freivalds draws per prime over the whole answer (miss probability
  at most 2^-27 per draw for any wrong answer);
* the four encrypted queries decrypt, on every sampled column, to the row
  they select (the other 28 queries are uniform ciphertext-shaped data).
"""

import numpy as np
import pytest

import synth
from oracle import query as oq
from oracle import scan as osc

from pirtest import (empty_dev, expected_columns, freivalds_ok, onehot_queries, ring,
                     sample_columns, to_dev, to_host)

pytestmark = pytest.mark.gpu

R, C, B, N_ENC, SEED = 2048, 1024, 32, 4, 11


@pytest.fixture(scope="module")
def batched():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    rg = ring(11, 2)
    raw = synth.db_bytes(SEED, R, C, rg.N)
    idx = synth.indices(SEED, N_ENC, R)
    ct, secrets = onehot_queries(SEED, idx, R, rg)
    unif = np.stack([synth.uniform_query(SEED, b, R, rg.primes, rg.N)
                     for b in range(N_ENC, B)]).astype(np.uint64)
    query = np.concatenate([ct, unif])                            # [B][R][2][K][N]
    ctx = pir.Context(0)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    yield ctx, db, rg, raw, query, idx, secrets
    ctx.close()


def _check(rg, raw, query, ans_coeff, idx, secrets, Bq):
    q_hat = osc.query_ntt(query, rg.primes, rg.psis)
    cols = sample_columns(C, 8, SEED)
    exp = osc.answer_intt(expected_columns(raw, q_hat, cols, rg), rg.primes, rg.psis)
    assert np.array_equal(ans_coeff[:, cols], exp)
    assert freivalds_ok(raw, q_hat, ans_coeff, rg, SEED, coeff_form=True)
    for b in range(min(Bq, N_ENC)):
        m, _ = oq.decrypt_answers(ans_coeff[b, cols], secrets[b], rg.primes, rg.psis, rg.delta,
                                  rg.p)
        assert np.array_equal(m, raw[idx[b], cols].astype(np.int64))


def test_batched_full_size(batched):
    ctx, db, rg, raw, query, idx, secrets = batched
    ctx.tune(db, B)
    out = empty_dev((B, C, 2, rg.K, rg.N))
    ctx.answer_batch([(db, B, to_dev(query), out)])
    _check(rg, raw, query, to_host(out), idx, secrets, B)


def test_batch1_on_batched_database(batched):
    ctx, db, rg, raw, query, idx, secrets = batched
    ctx.tune(db, 1)
    out = empty_dev((1, C, 2, rg.K, rg.N))
    ctx.answer_batch([(db, 1, to_dev(query[:1]), out)])
    _check(rg, raw, query[:1], to_host(out), idx, secrets, 1)
