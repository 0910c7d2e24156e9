"""GPU parity at the ABI's size limits.

R = PIR_MAX_R = 32768 rows is the largest contraction the exact int32 limb
sums are specified for (each sum is below 32768 * 127^2 < 2^31), and the
largest inputs of both epilogues: the batch-1 kernel's 64-bit limb sum stays
below 2^53 and the batched kernel's fp64 partial sums below 2^51.  The query
residues are drawn from the top of [0, q) so that every limb is at least 120,
which pushes the sums toward their bound.  Both kernels (B = 1 and B = 3) are
compared word for word with the oracle over the whole answer.  One row more
than the limit is refused before any allocation.
"""

import numpy as np
import pytest

import synth
from oracle import scan as osc

from pirtest import empty_dev, ring, to_dev, to_host

pytestmark = pytest.mark.gpu

R_MAX, C, SEED = 32768, 2, 5


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    c = pir.Context(0)
    yield c
    c.close()


def test_max_rows_both_kernels(ctx):
    rg = ring(10, 1)
    q = rg.primes[0]
    lo = 120 * sum(1 << (7 * a) for a in range(4))   # every 7-bit limb >= 120
    assert lo < q
    raw = synth.db_bytes(SEED, R_MAX, C, rg.N)
    q_hat = np.random.default_rng(SEED).integers(lo, q, size=(3, R_MAX, 2, 1, rg.N),
                                                 dtype=np.uint64)
    exp = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), q_hat, rg.primes)
    db = ctx.load_db(rg.pir_params(), raw, R_MAX, C)
    qd = to_dev(q_hat)
    for B in (1, 3):
        out = empty_dev((B, C, 2, 1, rg.N))
        ctx.db_mul(db, qd[:B], B, out)
        assert np.array_equal(to_host(out), exp[:B]), f"B={B}"


def test_rows_past_the_limit_are_refused(ctx):
    from paper_2606_11536_amd import pir
    rg = ring(10, 1)
    raw = np.zeros((R_MAX + 1, 1, rg.N), dtype=np.uint8)
    with pytest.raises(pir.PirError):
        ctx.load_db(rg.pir_params(), raw, R_MAX + 1, 1)
