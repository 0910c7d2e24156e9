"""GPU tests of HIP-graph plans (pir_plan_*): the captured steady state.

A job list over three databases of uneven shape (mixed N, R, C, B) is
captured once; every replay -- with eager work and synchronizations between
replays, and with new query contents written into the same buffers -- must
give exactly the oracle's answers.
"""

import numpy as np
import pytest

import synth
from oracle import scan as osc

from pirtest import empty_dev, residues, ring, to_dev, to_host

pytestmark = pytest.mark.gpu

SPECS = [(12, 2, 40, 20, 3), (11, 2, 75, 23, 1), (11, 2, 16, 70, 6)]


def expected(rg, raw, qc):
    y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(qc, rg.primes, rg.psis),
                   rg.primes)
    return osc.answer_intt(y, rg.primes, rg.psis)


def test_plan_replays_match_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    ctx = pir.Context(0)
    try:
        rng = np.random.default_rng(41)
        jobs, meta = [], []
        for n, (log2n, K, R, C, B) in enumerate(SPECS):
            rg = ring(log2n, K)
            raw = synth.db_bytes(700 + n, R, C, rg.N)
            db = ctx.load_db(rg.pir_params(), raw, R, C)
            qc = residues(rng, (B, R, 2), rg)
            jobs.append((db, B, to_dev(qc), empty_dev((B, C, 2, K, rg.N))))
            meta.append((rg, raw, qc))
        exp = [expected(rg, raw, qc) for rg, raw, qc in meta]
        plan = ctx.plan(jobs)
        # an unrelated eager job run between replays
        rg0, raw0, _ = meta[1]
        side_q = to_dev(residues(rng, (2, 75, 2), rg0))
        side_out = empty_dev((2, 23, 2, 2, rg0.N))
        for rep in range(3):
            for (_, _, _, out) in jobs:
                out.zero_()
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            for (_, _, _, out), e in zip(jobs, exp):
                assert np.array_equal(to_host(out), e), f"replay {rep}"
            ctx.answer_batch([(jobs[1][0], 2, side_q, side_out)])
            torch.cuda.synchronize()
        # new queries in the same buffers
        for n, ((db, B, qd, out), (rg, raw, _)) in enumerate(zip(jobs, meta)):
            qc = residues(rng, (B, db.R, 2), rg)
            qd.copy_(to_dev(qc))
            meta[n] = (rg, raw, qc)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (_, _, _, out), (rg, raw, qc) in zip(jobs, meta):
            assert np.array_equal(to_host(out), expected(rg, raw, qc))
        plan.close()
    finally:
        ctx.close()
